"""Seeded Zel'dovich initial conditions (Sec. IV-A: the initial positions and
velocities come from the Zel'dovich approximation).

Recipe (static background, units of the dynamical time, so the growing mode
grows as e^t and its velocity equals its displacement):

1. Gaussian white noise on the n^3 lattice from ``numpy.random.default_rng(seed)``
   (PCG64), array axes ordered (z, y, x) so x is fastest in memory.
2. Forward real FFT; multiply by k^(n/2) so the density spectrum is P ~ k^n;
   zero the k = 0 mode and every Nyquist plane.
3. Displacement psi_hat = i k delta_hat / k^2 (so that delta = -div psi),
   inverse FFT per component.
4. Rescale psi so that the rms of the 3-D |psi| equals the target.
5. Positions x = q + psi (mod L) with lattice points q = i + 1/2; velocities
   v = psi * exp(-dt/2) (the leapfrog velocity half a step before t = 0).

Particles are returned in lattice order p = ix + n*(iy + n*iz).  The arrays are
float32: both the HIP library and the oracle encode these exact values.
"""

import numpy as np


def _fft_module():
    try:
        import scipy.fft as sfft
        return sfft, {"workers": -1}
    except Exception:  # pragma: no cover - scipy is present in this image
        return np.fft, {}


def zeldovich_ics(n: int, spectral_index: float, rms_disp: float, seed: int,
                  dt: float):
    """Return (pos, vel), each float32 of shape (n^3, 3), lattice order."""
    fft, kw = _fft_module()
    # float64 arithmetic below 512^3, float32 above (memory); deterministic either way
    real_t = np.float64 if n <= 256 else np.float32
    rng = np.random.default_rng(seed)
    noise = rng.standard_normal((n, n, n), dtype=real_t)      # axes (z, y, x)
    dk = fft.rfftn(noise, **kw)
    del noise
    kz = np.fft.fftfreq(n, d=1.0 / n).astype(real_t)          # integer mode numbers
    ky = kz
    kx = np.fft.rfftfreq(n, d=1.0 / n).astype(real_t)
    two_pi_over_l = real_t(2.0 * np.pi / n)
    KZ = kz[:, None, None] * two_pi_over_l
    KY = ky[None, :, None] * two_pi_over_l
    KX = kx[None, None, :] * two_pi_over_l
    k2 = KX * KX + KY * KY + KZ * KZ
    k2[0, 0, 0] = 1.0
    amp = k2 ** real_t(spectral_index / 4.0)                  # |k|^(n/2)
    amp[0, 0, 0] = 0.0
    nyq = n // 2
    if n % 2 == 0:
        amp[nyq, :, :] = 0.0
        amp[:, nyq, :] = 0.0
        amp[:, :, nyq] = 0.0
    dk *= amp
    del amp
    inv_k2 = (1.0 / k2).astype(real_t)
    del k2
    psi = np.empty((3, n, n, n), dtype=real_t)
    for c, K in enumerate((KX, KY, KZ)):
        comp = dk * (1j * K * inv_k2)
        psi[c] = fft.irfftn(comp, s=(n, n, n), **kw)
        del comp
    del dk, inv_k2
    rms = np.sqrt(sum(float(np.sum(psi[c].astype(np.float64) ** 2)) for c in range(3)) / n ** 3)
    psi *= real_t(rms_disp / rms)
    # lattice order p = ix + n*(iy + n*iz): the (z, y, x) arrays flattened in C order
    N = n ** 3
    pos = np.empty((N, 3), dtype=np.float32)
    vel = np.empty((N, 3), dtype=np.float32)
    lattice = np.arange(n, dtype=np.float64) + 0.5
    shape = [(1, 1, n), (1, n, 1), (n, 1, 1)]          # q_x, q_y, q_z broadcasts
    damp = np.exp(-0.5 * dt)
    for c in range(3):
        comp = psi[c].astype(np.float64)
        x = np.mod(comp + lattice.reshape(shape[c]), float(n)).astype(np.float32)
        x[x >= np.float32(n)] = np.float32(0.0)                # mod can round up to L
        pos[:, c] = x.ravel()
        vel[:, c] = (comp * damp).astype(np.float32).ravel()
        del comp, x
    return pos, vel


def plane_wave_ics(n: int, amplitude: float, dt: float, mode: int = 1):
    """A single Zel'dovich plane wave along x: psi = A sin(2 pi mode q_x / L) e_x.

    Returns (q, pos, vel) as float64 arrays of shape (n^3, 3): the lattice
    points, the displaced positions and the half-step-back growing-mode
    velocities.  Used for the dynamics pins (exact solution before shell
    crossing)."""
    idx = np.arange(n, dtype=np.float64) + 0.5
    qz, qy, qx = np.meshgrid(idx, idx, idx, indexing="ij")
    q = np.stack([qx.ravel(), qy.ravel(), qz.ravel()], axis=1)
    psi = np.zeros_like(q)
    psi[:, 0] = amplitude * np.sin(2.0 * np.pi * mode * q[:, 0] / n)
    pos = np.mod(q + psi, float(n))
    vel = psi * np.exp(-0.5 * dt)
    return q, pos, vel


def zeldovich_ics_device(n: int, spectral_index: float, rms_disp: float, seed: int, dt: float,
                         device="cuda"):
    """The recipe of zeldovich_ics (the same seeded white noise, drawn on the
    host) with the transforms on a GPU through torch, for workloads of many
    boxes: float64 up to 256^3, float32 above.  Returns float32 (pos, vel)
    tensors of shape (n^3, 3) on `device`, lattice order.  Rounding differs
    from the host version in the last bits: use one or the other for inputs
    that are compared."""
    import torch
    real_np = np.float64 if n <= 256 else np.float32
    real_t = torch.float64 if n <= 256 else torch.float32
    rng = np.random.default_rng(seed)
    noise = torch.from_numpy(rng.standard_normal((n, n, n), dtype=real_np)).to(device)   # axes (z, y, x)
    dk = torch.fft.rfftn(noise)
    del noise
    kz = torch.fft.fftfreq(n, d=1.0 / n, dtype=real_t, device=device)
    kx = torch.fft.rfftfreq(n, d=1.0 / n, dtype=real_t, device=device)
    s = 2.0 * np.pi / n
    KZ = (kz * s)[:, None, None]
    KY = (kz * s)[None, :, None]
    KX = (kx * s)[None, None, :]
    k2 = KX * KX + KY * KY + KZ * KZ
    k2[0, 0, 0] = 1.0
    amp = k2 ** (spectral_index / 4.0)
    amp[0, 0, 0] = 0.0
    if n % 2 == 0:
        nyq = n // 2
        amp[nyq, :, :] = 0.0
        amp[:, nyq, :] = 0.0
        amp[:, :, nyq] = 0.0
    dk = dk * amp
    del amp
    inv_k2 = 1.0 / k2
    del k2
    psi = torch.empty((3, n, n, n), dtype=real_t, device=device)
    for c, K in enumerate((KX, KY, KZ)):
        psi[c] = torch.fft.irfftn(dk * (1j * K * inv_k2), s=(n, n, n))
    del dk, inv_k2
    rms = torch.sqrt(sum(torch.sum(psi[c].double() ** 2) for c in range(3)) / n ** 3)
    psi *= (rms_disp / rms).to(real_t)
    N = n ** 3
    pos = torch.empty((N, 3), dtype=torch.float32, device=device)
    vel = torch.empty((N, 3), dtype=torch.float32, device=device)
    lattice = torch.arange(n, dtype=torch.float64, device=device) + 0.5
    shape = [(1, 1, n), (1, n, 1), (n, 1, 1)]
    damp = float(np.exp(-0.5 * dt))
    for c in range(3):
        comp = psi[c].double()
        x = torch.remainder(comp + lattice.reshape(shape[c]), float(n)).float()
        x[x >= float(n)] = 0.0
        pos[:, c] = x.reshape(-1)
        vel[:, c] = (comp * damp).float().reshape(-1)
        del comp, x
    return pos, vel
