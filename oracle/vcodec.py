"""Cell-mean velocity codec (Sec. III-A, Eq. (3); fast arctangent Eq. (4)).

Test infrastructure: part of the FP64 oracle.

Eq. (3) splits a particle's velocity into the mean velocity of its coarse
cell and a deviation stored in one signed byte per axis through a nonlinear
map; the paper builds that map from an arctangent and evaluates the
arctangent with the approximation of Eq. (4).  Readings (the paper gives the
form of the map only through its reference):

* V1  the cell velocity v_c is the mean of the velocities of the particles
      stored in the cell: summed in FP64 one particle after another in
      storage order, divided by the count, and kept as FP32 (one value per
      axis and coarse cell); an empty cell has v_c = 0.
* V2  deviation dv = v - v_c.  Decode: dv = sigma tan(u pi / 255) for
      u in [-127, 127].  Encode: u = clamp(rint(atan~(dv / sigma) * (255 / pi))),
      atan~ the Eq. (4) approximation; |atan~ - atan| <= 0.0038 rad is below
      half a code's angle pi / 510, so every code decodes and re-encodes to
      itself.  Eq. (4) stays below pi / 2, so the code never leaves the
      range; a component beyond the last code's value sigma tan(127 pi / 255)
      (about 162 sigma) decodes to that value and is counted as saturated.
* V3  sigma is one power of two per box: the smallest one >= the rms of all
      deviation components (1 when they are all zero).
* V4  in a step the kicked velocity v' = v_c + dv + a dt is held in FP32
      until the particles are re-ordered, then re-encoded against the new
      cells' means; the drift uses that FP32 velocity, which keeps the drift
      exact in FP64 (a 24-bit mantissa times powers of two times the 24-bit
      dt).

Pins (tests/test_oracle_vcodec.py): Eq. (4)'s error bound over the whole
line, its symmetry and continuity; every code's round trip; monotone odd
decode table; the deviation bound of a round trip; cell means against a
per-cell brute force; sigma against the rms; the codec's velocity error below
the linear codec's on Zel'dovich velocities.
"""

import numpy as np

from .codec import pow2ceil

ANGLE = np.pi / 255.0          # angle of one code step
CODES_PER_RADIAN = 255.0 / np.pi
CODE_MAX = 127


def fast_atan(x):
    """Eq. (4): arctan from a quadratic on |x| <= 1 and the reflection
    atan(x) = +-pi/2 - atan(1/x) outside."""
    x = np.asarray(x, dtype=np.float64)
    out = np.empty_like(x)
    inner = np.abs(x) <= 1.0
    xi = x[inner]
    out[inner] = (np.pi / 4.0) * xi + 0.273 * xi * (1.0 - np.abs(xi))
    xo = x[~inner]
    r = 1.0 / xo
    out[~inner] = np.sign(xo) * (np.pi / 2.0) - (np.pi / 4.0) * r - 0.273 * r * (1.0 - np.abs(r))
    return out


def deviation_table():
    """tan(u pi / 255) for u = -127 .. 127 (index u + 127)."""
    u = np.arange(-CODE_MAX, CODE_MAX + 1, dtype=np.float64)
    return np.tan(u * ANGLE)


def encode_deviation(dv, sigma: float):
    """Codes (int8) of deviations and the number of components beyond the
    last code's value."""
    dv = np.asarray(dv, dtype=np.float64)
    t = fast_atan(dv / sigma)
    w = np.rint(t * CODES_PER_RADIAN)
    sat = int(np.count_nonzero(np.abs(dv) > sigma * np.tan(CODE_MAX * ANGLE)))
    return np.clip(w, -CODE_MAX, CODE_MAX).astype(np.int8), sat


def decode_deviation(u, sigma: float):
    return sigma * deviation_table()[np.asarray(u, dtype=np.int64) + CODE_MAX]


def cell_means(counts, v):
    """V1: FP32 mean velocity (n_cells, 3) of cell-ordered velocities v (N, 3),
    each cell summed sequentially in storage order."""
    counts = np.asarray(counts, dtype=np.int64)
    v = np.asarray(v, dtype=np.float64)
    off = np.zeros(counts.size + 1, dtype=np.int64)
    np.cumsum(counts, out=off[1:])
    sums = np.zeros((counts.size, 3))
    for j in range(int(counts.max()) if counts.size else 0):
        live = np.nonzero(counts > j)[0]          # cells with a (j+1)-th particle
        sums[live] += v[off[live] + j]
    nz = counts > 0
    mean = np.zeros((counts.size, 3))
    mean[nz] = sums[nz] / counts[nz, None]
    return mean.astype(np.float32)


def deviation_scale(dv) -> float:
    """V3: smallest power of two >= rms of all deviation components."""
    dv = np.asarray(dv, dtype=np.float64)
    if dv.size == 0:
        return 1.0
    rms = float(np.sqrt(np.mean(dv * dv)))
    return pow2ceil(rms) if rms > 0.0 else 1.0


def encode(counts, v):
    """Cell-ordered velocities (N, 3) -> (v_c FP32 (n_cells, 3), u int8 (N, 3),
    sigma, saturated components)."""
    v = np.asarray(v, dtype=np.float64)
    vc = cell_means(counts, v)
    cell = np.repeat(np.arange(np.asarray(counts).size), np.asarray(counts, dtype=np.int64))
    dv = v - vc[cell].astype(np.float64)
    sigma = deviation_scale(dv)
    u, sat = encode_deviation(dv, sigma)
    return vc, u, sigma, sat


def decode(counts, vc, u, sigma: float):
    """Velocities (N, 3) in FP64 from cell means and codes (u given (N, 3))."""
    cell = np.repeat(np.arange(np.asarray(counts).size), np.asarray(counts, dtype=np.int64))
    return np.asarray(vc, dtype=np.float64)[cell] + decode_deviation(u, sigma)
