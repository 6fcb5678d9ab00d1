"""Pins of the power-spectrum diagnostic (Sec. IV-C; reading R20)."""

import numpy as np

from oracle import diag


def test_shell_index_brute_force():
    n = 8
    j = diag.shell_index(n)
    for a in range(n):
        for b in range(n):
            for c in range(n):
                m = [x if x < n // 2 else x - n for x in (a, b, c)]
                r2 = sum(x * x for x in m)
                best = min(range(0, 2 * n), key=lambda s: abs(s - r2 ** 0.5))
                assert j[a, b, c] == best


def test_single_plane_wave_lands_in_one_shell():
    n, m, A = 32, 3, 0.01
    i = np.arange(n)
    delta = A * np.cos(2 * np.pi * m * i / n)[:, None, None] * np.ones((n, n, n))
    kk, P, cnt = diag.power_spectrum_from_delta(delta)
    j = m - 1
    assert np.max(np.delete(P, j)) < 1e-25
    # two modes (+m, -m) with |delta_hat| = A n^3 / 2, P = L^3 |.|^2 / N^2
    expect = 2 * (A * n ** 3 / 2) ** 2 / n ** 3 / cnt[j]
    assert abs(P[j] / expect - 1) < 1e-12
    assert abs(kk[j] - 2 * np.pi * m / n) < 2 * np.pi / n / 2


def test_displaced_lattice_peaks_in_its_shell():
    n, m, A = 32, 3, 0.01
    c = np.arange(n) + 0.5
    z, y, x = np.meshgrid(c, c, c, indexing="ij")
    xs = x + A * np.sin(2 * np.pi * m * x / n)
    pos = np.stack([xs.ravel(), y.ravel(), z.ravel()], 1)
    kk, P, cnt = diag.power_spectrum_from_positions(pos, n)
    assert np.argmax(P) == m - 1
    # an undisplaced lattice has no power at all (particles at cell centres)
    kk0, P0, _ = diag.power_spectrum_from_positions(
        np.stack([x.ravel(), y.ravel(), z.ravel()], 1), n)
    assert np.max(P0) < 1e-25


def test_poisson_particles_give_cic_shot_noise():
    n = 32
    rng = np.random.default_rng(9)
    pos = rng.uniform(0, n, size=(n ** 3, 3))
    kk, P, cnt = diag.power_spectrum_from_positions(pos, n)
    # expected shot noise for CIC with aliasing: prod_i (1 - 2/3 sin^2(k_i/2))
    modes = np.fft.fftfreq(n, d=1.0 / n)
    kx = 2 * np.pi * modes / n
    s = 1 - (2.0 / 3.0) * np.sin(kx / 2) ** 2
    w = s[:, None, None] * s[None, :, None] * s[None, None, :]
    j = diag.shell_index(n)
    for b in range(1, n // 4):
        sel = j == b
        expect = w[sel].mean()
        assert abs(P[b - 1] / expect - 1) < 5.0 / np.sqrt(cnt[b - 1])
