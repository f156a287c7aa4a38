"""Seeded synthetic interferograms for swept-source off-axis holographic OCT.

This module models the *recording* (the interferometer of Fig. 1 and the
interferogram model I = |E + E_LO|^2 of the setup paragraph), not the
reconstruction: it holds none of the reconstruction's arithmetic, and both the
FP64 oracle and the HIP library consume its output unchanged.

Physics of one sweep of T frames (wavenumber k_t swept linearly, Eq. 1-2):
  * local oscillator: unit plane wave tilted so that its carrier is 1/4 of the
    Nyquist frequency in x and y at the longest wavelength lambda_max, and
    f_c lambda_max / lambda_t at frame t (fixed angle);
  * point scatterers at distance z: E_m = a_m exp(2 i k_t delta_m)
    exp(i pi |r' - r_m|^2 / (lambda_t z)), restricted (per axis) to the sensor
    region where their fringes are sampled without aliasing;  depth delta_m is
    placed on an integer depth bin q_m, lateral position r_m on an integer
    output pixel of the reconstruction grid (pitch lambda_max z / (N d));
  * optional static speckle: circular complex Gaussian field at one depth bin;
  * optional aberration screen exp(-i sum_j c_j Z_j) (own Zernike
    implementation, Cartesian closed forms) and dispersion exp(-i phi_t);
  * photo-counts: gain so the mean is 2048, Gaussian approximation of shot
    noise, 12-bit clip, x16 into uint16.

All randomness comes from numpy.random.Generator(PCG64(seed)).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


@dataclass
class SweepConfig:
    T: int
    N: int
    pitch: float
    z: float
    lam_max: float
    lam_min: float
    n_scatterers: int
    speckle: float = 0.0
    aberration_rms: float = 0.0       # rad, std of the 15 Zernike coefficients
    dispersion_kappa: float = 0.0     # rad, quadratic dispersion amplitude
    k_bend: float = 0.0               # quadratic departure of k(t) from a linear sweep
    name: str = ""


# The five workloads (shapes and sweeps follow the paper's camera: 16-bit
# 1024x1024 frames, 256 frames per sweep, 12 um pixels, 820-870 nm class sweep).
CONFIGS = {
    "tiny": SweepConfig(T=32, N=128, pitch=20e-6, z=0.3, lam_max=870e-9, lam_min=800e-9,
                        n_scatterers=5, name="tiny"),
    "mid": SweepConfig(T=128, N=512, pitch=20e-6, z=0.3, lam_max=875e-9, lam_min=805e-9,
                       n_scatterers=50, speckle=0.02, name="mid"),
    "paper": SweepConfig(T=256, N=1024, pitch=12e-6, z=0.3, lam_max=870e-9, lam_min=800e-9,
                         n_scatterers=200, speckle=0.02, name="paper"),
    "diff": SweepConfig(T=128, N=512, pitch=20e-6, z=0.3, lam_max=875e-9, lam_min=805e-9,
                        n_scatterers=50, speckle=0.02, aberration_rms=0.3,
                        dispersion_kappa=3.0, name="diff"),
}
SEEDS = {"tiny": 1, "mid": 2, "paper": 3, "diff": 4}


@dataclass
class Sweep:
    frames: np.ndarray            # uint16 [T, N, N], (t, y, x)
    lam: np.ndarray               # float64 [T], metres
    pitch: float
    z: float
    cfg: SweepConfig
    scatterers: np.ndarray = field(default_factory=lambda: np.zeros((0, 4)))  # (u, v, q, amp)
    zernike_true: np.ndarray | None = None
    dispersion_true: np.ndarray | None = None


def sweep_wavelengths(T: int, lam_max: float, lam_min: float, bend: float = 0.0) -> np.ndarray:
    """Wavelengths from lam_max down to lam_min inclusive, linear in wavenumber
    (bend = 0) or with the quadratic wavenumber k(u) = k0 + (k1 - k0)(u + bend u (u - 1)),
    u = t / (T - 1), of a sweep that is not linear in k."""
    if T == 1:
        return np.array([lam_max])
    u = np.linspace(0.0, 1.0, T)
    k0, k1 = 2 * np.pi / lam_max, 2 * np.pi / lam_min
    k = k0 + (k1 - k0) * (u + bend * u * (u - 1.0))
    return 2 * np.pi / k


def _zernike_cartesian(x, y):
    """Orthonormal ANSI Zernike j = 0..14 on the unit disk, Cartesian closed forms."""
    r2 = x * x + y * y
    s3, s5, s6, s8, s10 = math.sqrt(3), math.sqrt(5), math.sqrt(6), math.sqrt(8), math.sqrt(10)
    one = np.ones_like(x)
    return np.stack([
        one,
        2 * y,
        2 * x,
        s6 * 2 * x * y,
        s3 * (2 * r2 - 1),
        s6 * (x * x - y * y),
        s8 * (3 * x * x * y - y ** 3),
        s8 * (3 * r2 - 2) * y,
        s8 * (3 * r2 - 2) * x,
        s8 * (x ** 3 - 3 * x * y * y),
        s10 * 4 * (x ** 3 * y - x * y ** 3),
        s10 * (4 * r2 - 3) * 2 * x * y,
        s5 * (6 * r2 * r2 - 6 * r2 + 1),
        s10 * (4 * r2 - 3) * (x * x - y * y),
        s10 * (x ** 4 - 6 * x * x * y * y + y ** 4),
    ])


def make_sweep(cfg: SweepConfig, seed: int, dtype=np.complex64) -> Sweep:
    rng = np.random.Generator(np.random.PCG64(seed))
    T, N, d, z = cfg.T, cfg.N, cfg.pitch, cfg.z
    lam = sweep_wavelengths(T, cfg.lam_max, cfg.lam_min, cfg.k_bend)
    k = 2 * np.pi / lam
    dk = (k[-1] - k[0]) / max(T - 1, 1)
    c = np.arange(N) - N // 2
    xs = c * d                                          # sensor coordinates (m)
    dprime = cfg.lam_max * z / (N * d)                  # output pixel pitch at lam_max

    # scatterers: target output pixel in the +1 order quadrant, integer depth bin
    M = cfg.n_scatterers
    half = max(N // 8 - 4, 1)
    cu = N // 8 + rng.integers(-half, half + 1, size=M)
    cv = N // 8 + rng.integers(-half, half + 1, size=M)
    qm = rng.integers(max(T // 8, 1), max(3 * T // 8, 2) + 1, size=M)
    amp = rng.uniform(0.05, 0.2, size=M)
    phase0 = rng.uniform(0, 2 * np.pi, size=M)
    y0 = (cu - N // 8) * dprime
    x0 = (cv - N // 8) * dprime
    delta = np.pi * qm / (T * abs(dk)) if T > 1 else np.zeros(M)

    if cfg.speckle > 0:
        spk = cfg.speckle * (rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N))) / math.sqrt(2)
        q_spk = int(rng.integers(max(T // 8, 1), max(3 * T // 8, 2) + 1))
        spk_phase0 = rng.uniform(0, 2 * np.pi)
    else:
        spk = None

    if cfg.aberration_rms > 0:
        zc = rng.normal(0.0, cfg.aberration_rms, size=15)
        X, Y = np.meshgrid(c / (N / math.sqrt(2)), c / (N / math.sqrt(2)))
        screen = np.exp(-1j * np.tensordot(zc, _zernike_cartesian(X, Y), axes=(0, 0))).astype(dtype)
    else:
        zc, screen = None, None
    if cfg.dispersion_kappa > 0 and T > 1:
        tn = (np.arange(T) - (T - 1) / 2) / ((T - 1) / 2)
        disp = cfg.dispersion_kappa * tn * tn
    else:
        disp = None

    frames = np.empty((T, N, N), dtype=np.uint16)
    gain = None
    fc = 1.0 / (8 * d)
    for t in range(T):
        lt = lam[t]
        f_t = fc * cfg.lam_max / lt
        ref_x = np.exp(2j * np.pi * f_t * xs)
        E_lo = np.outer(ref_x, ref_x).astype(dtype)          # [y, x]
        # separable point-source fields, windowed where fringes are resolved
        ph_x = np.pi * (xs[:, None] - x0[None, :]) ** 2 / (lt * z)
        ph_y = np.pi * (xs[:, None] - y0[None, :]) ** 2 / (lt * z)
        fr_x = (xs[:, None] - x0[None, :]) * d / (lt * z) - f_t * d
        fr_y = (xs[:, None] - y0[None, :]) * d / (lt * z) - f_t * d
        Ex = np.exp(1j * ph_x) * (np.abs(fr_x) <= 0.45)
        Ey = np.exp(1j * ph_y) * (np.abs(fr_y) <= 0.45)
        coef = amp * np.exp(1j * (phase0 + 2 * k[t] * delta))
        O = ((Ey * coef[None, :]).astype(dtype) @ Ex.T.astype(dtype))
        if spk is not None:
            O = O + (spk * np.exp(1j * (spk_phase0 + 2 * np.pi * q_spk * t / T))).astype(dtype)
        if screen is not None:
            O = O * screen
        if disp is not None:
            O = O * np.complex64(np.exp(-1j * disp[t])).astype(dtype)
        E = E_lo + O
        I = (E.real.astype(np.float64) ** 2 + E.imag.astype(np.float64) ** 2)
        if gain is None:
            gain = 2048.0 / float(np.mean(I))
        pe = gain * I
        counts = np.rint(pe + np.sqrt(pe) * rng.standard_normal((N, N)))
        frames[t] = (np.clip(counts, 0, 4095) * 16).astype(np.uint16)
    scat = np.stack([cu + N // 2, cv + N // 2, qm, amp], axis=1)
    return Sweep(frames=frames, lam=lam, pitch=d, z=z, cfg=cfg, scatterers=scat,
                 zernike_true=zc, dispersion_true=disp)


def make_config(name: str, seed: int | None = None) -> Sweep:
    """One of the named workloads ('tiny', 'mid', 'paper', 'diff') with its default seed."""
    cfg = CONFIGS[name]
    return make_sweep(cfg, SEEDS[name] if seed is None else seed)


def random_frames(T: int, N: int, seed: int, lo: int = 0, hi: int = 65535) -> np.ndarray:
    """Uniform random uint16 frames (for parity tests that need no physics)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.integers(lo, hi + 1, size=(T, N, N), dtype=np.uint16)
