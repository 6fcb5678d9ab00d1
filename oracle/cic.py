"""Cloud-in-cell mass assignment and interpolation (Sec. II: the density comes
from interpolating particles onto the mesh; Sec. IV-C: CIC).

Reading R10: for a coordinate X in cell units on a cell-centred mesh
(cell i spans [i, i+1)), i0 = floor(X - 1/2), t = X - 1/2 - i0, and the two
cells i0, i0+1 get weights 1-t, t per axis; the 3-D weight is the product.
Deposit and gather use the same weights.

Exactness: decoded positions are dyadic with at most 9 fractional bits per axis,
so every weight product is an exact dyadic and float64 sums of them are exact
in any order (below 2^53).  The oracle's mesh is therefore exactly the value a
fixed-point integer accumulation produces.

Pins (tests/test_oracle_cic.py): total mass equals the particle count exactly;
a particle at a cell centre fills one cell; a single particle's weights equal
the closed-form products; an integer shift of all particles shifts the mesh;
gather of a linear field reproduces it exactly.
"""

import itertools

import numpy as np


def _corners(X):
    X = np.asarray(X, dtype=np.float64)
    base = X - 0.5
    i0 = np.floor(base).astype(np.int64)
    t = base - i0
    return i0, t


def deposit(X, n: int, periodic: bool = True, mass=None) -> np.ndarray:
    """Mass per cell on an n^3 mesh indexed [ix, iy, iz].

    X: (N, 3) coordinates in cell units.  periodic=False drops contributions
    that fall outside [0, n) (tile boxes, R11)."""
    i0, t = _corners(X)
    w_axis = (1.0 - t, t)
    out = np.zeros(n * n * n, dtype=np.float64)
    mass = np.ones(i0.shape[0]) if mass is None else np.asarray(mass, dtype=np.float64)
    for ox, oy, oz in itertools.product((0, 1), repeat=3):
        ix = i0[:, 0] + ox
        iy = i0[:, 1] + oy
        iz = i0[:, 2] + oz
        w = w_axis[ox][:, 0] * w_axis[oy][:, 1] * w_axis[oz][:, 2] * mass
        if periodic:
            ix, iy, iz = ix % n, iy % n, iz % n
            keep = slice(None)
        else:
            keep = (ix >= 0) & (ix < n) & (iy >= 0) & (iy < n) & (iz >= 0) & (iz < n)
            ix, iy, iz, w = ix[keep], iy[keep], iz[keep], w[keep]
        flat = (ix * n + iy) * n + iz
        out += np.bincount(flat, weights=w, minlength=n ** 3)
    return out.reshape(n, n, n)


def gather(field, X, periodic: bool = True) -> np.ndarray:
    """Interpolate a scalar (n,n,n) or vector (c,n,n,n) field at X (N, 3)."""
    f = np.asarray(field, dtype=np.float64)
    vector = f.ndim == 4
    if not vector:
        f = f[None]
    n = f.shape[1]
    i0, t = _corners(X)
    w_axis = (1.0 - t, t)
    out = np.zeros((f.shape[0], i0.shape[0]), dtype=np.float64)
    for ox, oy, oz in itertools.product((0, 1), repeat=3):
        ix = i0[:, 0] + ox
        iy = i0[:, 1] + oy
        iz = i0[:, 2] + oz
        if periodic:
            ix, iy, iz = ix % n, iy % n, iz % n
        elif ix.size:
            assert ix.min() >= 0 and ix.max() < n and iy.min() >= 0 and iy.max() < n \
                and iz.min() >= 0 and iz.max() < n, "gather outside the mesh"
        w = w_axis[ox][:, 0] * w_axis[oy][:, 1] * w_axis[oz][:, 2]
        out += f[:, ix, iy, iz] * w
    return out if vector else out[0]
