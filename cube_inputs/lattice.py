"""A compressed state written directly in the storage format, for full-size
tests.

Every coarse cell holds the 8 particles of a lattice with two particles per
axis per cell (in-cell bytes 64 and 192 on each axis, zero velocity bytes);
inside a few runs of consecutive cells (in storage order) the bytes are
random and each pair of consecutive cells splits its 16 particles at random,
so that counts there range over 0..16.  Nothing here encodes or computes:
the arrays are laid out as the format defines them.
"""

import numpy as np

LATTICE_BYTES = (64, 192)


def lattice_run_state(n_cells, runs, seed, u_amp=20):
    """counts int32 [n_cells], m uint8 [3, 8 n_cells], u int8 [3, 8 n_cells].

    runs: list of (first_cell, n_run_cells) in storage order, n_run_cells even
    and first_cell even.  Returns (counts, m, u)."""
    lo, hi = LATTICE_BYTES
    px = np.array([lo, hi] * 4, dtype=np.uint8)
    py = np.array([lo, lo, hi, hi] * 2, dtype=np.uint8)
    pz = np.array([lo] * 4 + [hi] * 4, dtype=np.uint8)
    counts = np.full(n_cells, 8, dtype=np.int32)
    m = np.empty((3, 8 * n_cells), dtype=np.uint8)
    for k, pat in enumerate((px, py, pz)):
        m[k] = np.tile(pat, n_cells)
    u = np.zeros((3, 8 * n_cells), dtype=np.int8)
    for i, (c0, L) in enumerate(runs):
        assert c0 % 2 == 0 and L % 2 == 0 and c0 + L <= n_cells
        rng = np.random.default_rng(seed + i)
        a = rng.integers(0, 17, size=L // 2)
        counts[c0:c0 + L:2] = a
        counts[c0 + 1:c0 + L:2] = 16 - a
        seg = slice(8 * c0, 8 * (c0 + L))
        m[:, seg] = rng.integers(0, 256, size=(3, 8 * L), dtype=np.uint8)
        u[:, seg] = rng.integers(-u_amp, u_amp + 1, size=(3, 8 * L)).astype(np.int8)
    return counts, m, u
