"""Extended particle-particle (PP) force (Sec. II, optional PP module;
Sec. III-B, pair distances from the compressed integer positions).

Test infrastructure: part of the FP64 oracle.

With the PP module on, pairs of particles a preset number of fine cells apart
or closer attract explicitly, and the fine mesh's short-range kernel is
corrected so that the mesh no longer carries that part.  The paper gives the
range in fine cells and leaves the correction's form to its references.
Readings (P1-P4):

* P1  range: Box.pp_range = n_pp fine cells, r_pp = n_pp h spacings, with
      1 <= n_pp <= r (so r_pp <= H: a particle's PP partners lie in its own
      or the adjacent coarse cells, and every partner closer than r_pp is
      under 256 position quanta away on each axis, so the squared distance
      is an exact small integer).  The split only pays once r_pp spans a few
      fine cells: the mesh smooths the part it keeps on the scale of h.
* P2  split: a second compact S2 split, of diameter r_pp, inside the one of
      diameter a_len (R12).  The pair force is F_pp(r) = F_G(r) - F_l(r; r_pp)
      for 0 < r < r_pp and 0 otherwise (also for coincident particles); the
      fine mesh carries F_l(r; r_pp) - F_l(r; a_len), i.e. the continuum
      kernel -(S_pp^2 - S_a^2) / k^2 with the k -> 0 limit
      -(a_len^2 - r_pp^2) / 30, truncated to |d| <= a as before.  In the
      continuum coarse + fine + PP is exactly Newton's force at every r.
* P3  F_l(r; D), the attraction of two S2 clouds of diameter D (Hockney &
      Eastwood's reference force), with xi = 2 r / D and 4 pi G = 1:
        4 pi D^2 F_l = (224 xi - 224 xi^3 + 70 xi^4 + 48 xi^5 - 21 xi^6) / 35
                                                                  (xi <= 1)
                     = (12 / xi^2 - 224 + 896 xi - 840 xi^2 + 224 xi^3
                        + 70 xi^4 - 48 xi^5 + 7 xi^6) / 35          (1 <= xi <= 2)
        F_l = 1 / (4 pi r^2) beyond (xi >= 2).
* P4  PP accelerations are summed over every other particle (minimum image);
      F_pp vanishing beyond r_pp makes that the pairs of neighbouring coarse
      cells.  They add to the mesh acceleration before the kick and are
      scaled like it (K_n in comoving runs).  The potential-energy
      diagnostic stays the mesh part.

Pins (tests/test_oracle_pp.py): P3 against the numerical radial Fourier
transform of S(k D / 2)^2 / k^2; continuity at xi = 1 and xi = 2; the cell
search against an all-pairs brute force on a small box; Newton's third law;
a pair of particles whose total force (both meshes with the corrected kernel
plus PP) follows 1/(4 pi r^2) inside r_pp, where the mesh alone falls short.
"""

import itertools

import numpy as np

from .geometry import Box


def s2_pair_force(r, D: float):
    """F_l(r; D) of P3 (attraction magnitude, FP64), vectorised."""
    r = np.asarray(r, dtype=np.float64)
    xi = 2.0 * r / D
    out = np.empty_like(r)
    inner = xi <= 1.0
    mid = (xi > 1.0) & (xi < 2.0)
    far = xi >= 2.0
    x = xi[inner]
    out[inner] = (224 * x - 224 * x ** 3 + 70 * x ** 4 + 48 * x ** 5 - 21 * x ** 6) / 35.0
    x = xi[mid]
    out[mid] = (12 / x ** 2 - 224 + 896 * x - 840 * x ** 2 + 224 * x ** 3 + 70 * x ** 4
                - 48 * x ** 5 + 7 * x ** 6) / 35.0
    out[inner | mid] /= 4.0 * np.pi * D * D
    out[far] = 1.0 / (4.0 * np.pi * r[far] ** 2)
    return out


def pair_force(r, r_pp: float):
    """F_pp(r) of P2: Newton minus the S2 pair force, zero at r = 0 and r >= r_pp."""
    r = np.asarray(r, dtype=np.float64)
    out = np.zeros_like(r)
    live = (r > 0.0) & (r < r_pp)
    rl = r[live]
    out[live] = 1.0 / (4.0 * np.pi * rl * rl) - s2_pair_force(rl, r_pp)
    return out


def pp_radius(box: Box) -> float:
    return box.pp_range * box.h


def _pair_terms(box: Box, Qi, Qj):
    """Acceleration on particles at global quanta Qi from partners at Qj (rows
    paired up), minimum image: (P, 3) FP64."""
    L = 256 * box.n_coarse
    dq = np.asarray(Qj, dtype=np.int64) - np.asarray(Qi, dtype=np.int64)
    dq = (dq + L // 2) % L - L // 2
    d = dq.astype(np.float64) * (box.H / 256.0)
    r = np.sqrt(np.sum(d * d, axis=1))
    f = pair_force(r, pp_radius(box))
    w = np.zeros_like(r)
    live = f != 0.0
    w[live] = f[live] / r[live]
    return w[:, None] * d


def _neighbour_cells(box: Box, cx, cy, cz):
    Nc = box.n_coarse
    return [box.canon((cx + dx) % Nc, (cy + dy) % Nc, (cz + dz) % Nc)
            for dx, dy, dz in itertools.product((-1, 0, 1), repeat=3)]


def pp_accel(box: Box, state) -> np.ndarray:
    """PP acceleration (N, 3) in canonical order (P4): the partners of a
    particle are the particles of the 27 coarse cells around its own."""
    Q = state.quanta()
    counts = np.asarray(state.counts, dtype=np.int64)
    offsets = state.offsets()
    cx, cy, cz = box.cell_of_canon(state.cell_canon())
    n = Q.shape[0]
    acc = np.zeros((n, 3))
    idx = np.arange(n, dtype=np.int64)
    for nb in _neighbour_cells(box, cx, cy, cz):
        lens = counts[nb]
        i = np.repeat(idx, lens)
        # partner k of particle i sits at offsets[nb_i] + k
        j = np.repeat(offsets[nb] - np.cumsum(lens) + lens, lens) + np.arange(i.size, dtype=np.int64)
        t = _pair_terms(box, Q[i], Q[j])
        for k in range(3):
            acc[:, k] += np.bincount(i, weights=t[:, k], minlength=n)
    return acc


def pp_accel_cells(box: Box, counts, offsets, m, cells):
    """(storage indices, PP acceleration) of the particles of the given
    canonical cells, decoding only their neighbourhoods from the planes
    (sampled checks of boxes too large for pp_accel)."""
    counts = np.asarray(counts)
    out_idx, out_acc = [], []

    def decode(cs):
        cs = np.asarray(cs, dtype=np.int64)
        lens = np.asarray(counts[cs], dtype=np.int64)
        idx = np.concatenate([np.arange(offsets[c], offsets[c] + k, dtype=np.int64)
                              for c, k in zip(cs, lens)]) if lens.sum() else np.zeros(0, np.int64)
        cx, cy, cz = box.cell_of_canon(np.repeat(cs, lens))
        Q = np.stack([256 * cx + m[0][idx], 256 * cy + m[1][idx], 256 * cz + m[2][idx]], axis=1)
        return idx, Q.astype(np.int64)

    for c in np.asarray(cells, dtype=np.int64):
        ti, Qt = decode([c])
        if ti.size == 0:
            continue
        cx, cy, cz = box.cell_of_canon(np.array([c]))
        _, Qp = decode([int(nb[0]) for nb in _neighbour_cells(box, cx, cy, cz)])
        a = np.zeros((ti.size, 3))
        for k in range(ti.size):
            a[k] = _pair_terms(box, np.broadcast_to(Qt[k], Qp.shape), Qp).sum(axis=0)
        out_idx.append(ti)
        out_acc.append(a)
    if not out_idx:
        return np.zeros(0, np.int64), np.zeros((0, 3))
    return np.concatenate(out_idx), np.concatenate(out_acc)
