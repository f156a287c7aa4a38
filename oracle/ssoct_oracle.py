"""Plain FP64 CPU oracle of the swept-source holographic OCT reconstruction.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, the smoke check in
``__graft_entry__.py`` and the ``cpu_baseline`` leg of ``bench.py`` import this
module.  The HIP library never calls it, links it or shares code with it.

Method (Charpentier et al., arXiv 2003.08960, flowchart of Fig. 3):

  1. rescale every interferogram by linear interpolation so that the Fresnel
     reconstruction pitch no longer depends on the wavelength  (Eq. 4, Eq. 5)
  2. discrete Fresnel transform of each rescaled frame, with the start
     wavelength lambda_1 used for every frame of the sweep    (Eq. 6)
  3. Fourier transform along the sweep with a rectangular gate of the whole
     stack (one window of T frames)                            (Eq. 7)
  4. envelope |H~| and three orthogonal cuts                   (text after Eq. 7)

Every step below is the plain definition, evaluated in float64/complex128.
Library FFTs serve as the discrete Fourier sums; ``render_columns`` evaluates
the same sums directly, term by term, for sampled outputs and brute-force pins.

Readings of points the paper leaves open:

  * lambda_1 ("start wavelength", the longest of the sweep) is taken as
    lambda_ref = max(lambda).  Then s_t = lambda_t / lambda_ref <= 1 and every
    interpolation sample stays inside the frame.
  * The rescale (Eq. 5) is about the array centre: the sample of output pixel
    (m, n) is taken at source position (N/2 + c_m s_t, N/2 + c_n s_t) with
    centred index c_j = j - N/2; separable bilinear interpolation with
    clamp-to-edge (the clamp never changes a value when s_t <= 1).
  * Eq. 6 expanded: (x - x')^2 = x^2 - 2 x x' + x'^2.  The input chirp is
    exp(-i pi x'^2 / (lambda_1 z)) sampled at x' = c d, i.e.
    exp(-i alpha c^2) with alpha = pi d^2 / (lambda_1 z); the kernel
    exp(+2 pi i x x' / (lambda_1 z)) sampled at x = c_u d' with d' from Eq. 4
    is exp(+2 pi i c_u c_n / N): a centred, positive-exponent, unnormalised
    DFT.  Option ``exact_chirp`` uses alpha_t = pi d^2 s_t / (lambda_1 z).
  * The prefactor (i d^2 / (lambda_1 z)) exp(-i k_1 z) and the output phase
    exp(-i pi x^2 / (lambda_1 z)) of Eq. 6 are unimodular-times-constant; they
    are off by default and applied with ``eq6_phase=True``.
  * Eq. 7 with a rectangular gate over the T frames of one volume is the
    unnormalised DFT V[q] = sum_t h_t exp(-2 pi i q t / T), bins in natural
    order (bins q >= T/2 are negative depths).
  * Optional per-frame dispersion phase exp(i phi_t) multiplies h_t before the
    depth transform; optional aberration exp(i sum_j c_j Z_j) (ANSI/OSA
    Zernike, j = 0..14, orthonormal, rho = r / (N d / sqrt 2)) multiplies the
    rescaled frame.  Neither is in the paper (it names aberration correction
    only as a motivation); they parameterise the sharpness gradient.
  * Cuts are |V| (caption of Fig. 3); ``power=True`` gives |V|^2 (text after
    Eq. 7).
  * Gate and sweep linearity.  The paper's gate g is rectangular and its
    laser is swept linearly in wavenumber (setup paragraph; Eq. 7).  Two
    generalisations are offered: ``gate`` (real weights g_t on h_t before the
    depth transform, an apodised gate) and ``nonuniform_k`` (the depth
    transform evaluated at the uniform depth grid of a sweep whose k_t is
    not linear in t: V[q] = sum_t h_t exp(-2 pi i q kappa_t / T) with
    kappa_t = (k_t - k_0) / dk, dk = (k_{T-1} - k_0) / (T - 1), which is t
    for a k-linear sweep).
  * Angular-spectrum propagation (the alternative the paper contrasts with
    the Fresnel transform; it keeps the sensor pitch for every wavelength, so
    no rescale): h_t = F^-1{ F{I_t} exp(-2 pi i z sqrt(lambda_t^-2 - fx^2 - fy^2)) }
    with F the unnormalised DFT (negative exponent), F^-1 its inverse (1/N^2),
    frequencies fx = k / (N d) for the DFT index k folded to [-N/2, N/2), and
    the evanescent components (negative radicand) set to zero.  The sign is
    the paper's: its fields carry exp(+i omega t) (setup paragraph), so
    propagation by +z carries exp(-i k z), as the prefactor of Eq. 6 does.
    With this sign one z names the same plane for both propagators: at
    z = z_b (where the Fresnel pixel of Eq. 4 equals the sensor pitch) Eq. 6
    with its prefactor and output phase is the paraxial limit of this
    transfer function on the same grid.
"""
from __future__ import annotations

import math

import numpy as np

N_ZERNIKE = 15


# ---------------------------------------------------------------------------
# Geometry helpers (Eq. 3, Eq. 4, validity condition after Eq. 6)
# ---------------------------------------------------------------------------

def centred(N: int) -> np.ndarray:
    """Centred sample index c_j = j - N/2, j = 0..N-1."""
    return np.arange(N, dtype=np.float64) - N // 2


def reference_wavelength(lam) -> float:
    """lambda_1 of Eq. 5-6: the sweep start, the longest wavelength."""
    return float(np.max(np.asarray(lam, dtype=np.float64)))


def scale_factors(lam) -> np.ndarray:
    """s_t = lambda_t / lambda_1: the resampling pitch d_lambda / d (Eq. 5)."""
    lam = np.asarray(lam, dtype=np.float64)
    return lam / reference_wavelength(lam)


def reconstructed_pitch(lam: float, z: float, N: int, pitch: float) -> float:
    """Eq. 4: lateral size of a Fresnel-reconstructed pixel, d' = lambda z / (N d)."""
    return lam * z / (N * pitch)


def boundary_distance(N: int, pitch: float, lam1: float) -> float:
    """z_b = N d^2 / lambda_1: Eq. 6 is used for z >= z_b (text after Eq. 6)."""
    return N * pitch * pitch / lam1


def twice_axial_pitch(lam1: float, lam2: float) -> float:
    """Lambda = lambda_1 lambda_2 / |lambda_2 - lambda_1| (text after Eq. 3)."""
    return lam1 * lam2 / abs(lam2 - lam1)


def axial_range(lam1: float, lam2: float, n_z: int) -> float:
    """Eq. 3: Delta z = (N_z / 2) Lambda."""
    return 0.5 * n_z * twice_axial_pitch(lam1, lam2)


def coherence_length(lam1: float, lam2: float) -> float:
    """Round-trip coherence length mean(lambda)^2 / Delta lambda (text after Eq. 3)."""
    lbar = 0.5 * (lam1 + lam2)
    return lbar * lbar / abs(lam2 - lam1)


def depth_of_bin(q, lam) -> np.ndarray:
    """Depth of depth-DFT bin q for a sweep sampled at wavelengths lam.

    Eq. 1-2: a reflector at path detuning delta makes the phase 2 k delta,
    linear in the sampled wavenumber k_t.  With the mean wavenumber step
    dk = (k_{T-1} - k_0)/(T-1), bin q of the T-point DFT is the tone
    exp(2 pi i q t / T) = exp(2 i dk delta_q t), so delta_q = pi q / (T dk).
    Bins q >= T/2 are negative depths (aliases).
    """
    lam = np.asarray(lam, dtype=np.float64)
    T = lam.size
    k = 2.0 * np.pi / lam
    dk = (k[-1] - k[0]) / (T - 1)
    q = np.asarray(q, dtype=np.float64)
    qs = np.where(q >= T / 2, q - T, q)
    return np.pi * qs / (T * abs(dk))


# ---------------------------------------------------------------------------
# Step 1: chromatic rescale (Eq. 5, "resampled by linear interpolation")
# ---------------------------------------------------------------------------

def interp_positions(N: int, s: float):
    """Source positions P_j = N/2 + c_j s and their bilinear split (j0, j1, f)."""
    P = N // 2 + centred(N) * s
    j0 = np.floor(P).astype(np.int64)
    f = P - j0
    j1 = np.minimum(j0 + 1, N - 1)
    j0 = np.clip(j0, 0, N - 1)
    return j0, j1, f


def rescale(frame, s: float) -> np.ndarray:
    """Eq. 5: I'(x, y) = I(x s, y s) about the array centre, bilinear, FP64."""
    I = np.asarray(frame, dtype=np.float64)
    N = I.shape[0]
    y0, y1, fy = interp_positions(N, s)
    x0, x1, fx = interp_positions(N, s)
    top = I[y0][:, x0] * (1.0 - fx) + I[y0][:, x1] * fx
    bot = I[y1][:, x0] * (1.0 - fx) + I[y1][:, x1] * fx
    return top * (1.0 - fy)[:, None] + bot * fy[:, None]


# ---------------------------------------------------------------------------
# Step 2: chirp, optional aberration, Fresnel transform (Eq. 6)
# ---------------------------------------------------------------------------

def chirp_rates(lam, pitch: float, z: float, exact_chirp: bool = False) -> np.ndarray:
    """alpha_t = pi d^2 s_t^p / (lambda_1 z), p = 0 (paper: lambda_1 for all) or 1."""
    lam1 = reference_wavelength(lam)
    s = scale_factors(lam)
    p = 1.0 if exact_chirp else 0.0
    return np.pi * pitch * pitch * s ** p / (lam1 * z)


def chirp(N: int, alpha: float) -> np.ndarray:
    """Q[m, n] = exp(-i alpha (c_m^2 + c_n^2)): the x'^2 term of Eq. 6."""
    c = centred(N)
    r2 = c[:, None] ** 2 + c[None, :] ** 2
    return np.exp(-1j * alpha * r2)


def zernike_nm(j: int):
    """ANSI/OSA single index j -> (n, m)."""
    n = int(math.ceil((-3.0 + math.sqrt(9.0 + 8.0 * j)) / 2.0))
    m = 2 * j - n * (n + 2)
    return n, m


def zernike(j: int, rho: np.ndarray, theta: np.ndarray) -> np.ndarray:
    """Orthonormal Zernike polynomial Z_j (ANSI/OSA), (1/pi) int Z_j Z_k = delta_jk."""
    n, m = zernike_nm(j)
    am = abs(m)
    R = np.zeros_like(rho)
    for k in range((n - am) // 2 + 1):
        coef = ((-1) ** k * math.factorial(n - k)
                / (math.factorial(k) * math.factorial((n + am) // 2 - k)
                   * math.factorial((n - am) // 2 - k)))
        R = R + coef * rho ** (n - 2 * k)
    norm = math.sqrt((2.0 if m != 0 else 1.0) * (n + 1))
    if m > 0:
        ang = np.cos(am * theta)
    elif m < 0:
        ang = np.sin(am * theta)
    else:
        ang = np.ones_like(theta)
    return norm * R * ang


def pupil_grid(N: int):
    """(rho, theta) of the calculation grid: rho = r / (N d / sqrt 2), theta = atan2(y, x)."""
    c = centred(N)
    y = c[:, None] * np.ones((1, N))
    x = np.ones((N, 1)) * c[None, :]
    rho = np.sqrt(x * x + y * y) / (N / math.sqrt(2.0))
    theta = np.arctan2(y, x)
    return rho, theta


def zernike_stack(N: int) -> np.ndarray:
    """Z_j on the calculation grid, j = 0..14, shape [15, N, N]."""
    rho, theta = pupil_grid(N)
    return np.stack([zernike(j, rho, theta) for j in range(N_ZERNIKE)])


def aberration(N: int, coeffs) -> np.ndarray:
    """A[m, n] = exp(i sum_j c_j Z_j(m, n)); all ones when coeffs is None."""
    if coeffs is None:
        return np.ones((N, N), dtype=np.complex128)
    c = np.asarray(coeffs, dtype=np.float64)
    phase = np.tensordot(c, zernike_stack(N), axes=(0, 0))
    return np.exp(1j * phase)


def fresnel_fft(x: np.ndarray) -> np.ndarray:
    """Centred unnormalised DFT with + exponent over the last two axes.

    h[u, v] = sum_{m,n} x[m, n] exp(+2 pi i (c_u c_m + c_v c_n) / N)
            = N^2 fftshift(ifft2(ifftshift(x))).
    """
    N1, N2 = x.shape[-2:]
    ax = (-2, -1)
    return (N1 * N2) * np.fft.fftshift(np.fft.ifft2(np.fft.ifftshift(x, axes=ax), axes=ax), axes=ax)


def fresnel_fft_adjoint(b: np.ndarray) -> np.ndarray:
    """Adjoint of ``fresnel_fft``: centred unnormalised DFT with - exponent."""
    ax = (-2, -1)
    return np.fft.fftshift(np.fft.fft2(np.fft.ifftshift(b, axes=ax), axes=ax), axes=ax)


def eq6_output_factor(N: int, lam1: float, pitch: float, z: float) -> np.ndarray:
    """(i d^2 / (lambda_1 z)) exp(-i k_1 z) exp(-i pi lambda_1 z (c_u^2 + c_v^2) / (N d)^2).

    The constant prefactor and output-plane quadratic phase of Eq. 6 with the
    output sampled at x = c_u d' (Eq. 4).  The k_1 z argument is reduced in
    whole cycles before the exponential.
    """
    c = centred(N)
    r2 = c[:, None] ** 2 + c[None, :] ** 2
    cyc = z / lam1
    cyc = cyc - np.floor(cyc)
    pref = 1j * pitch * pitch / (lam1 * z) * np.exp(-2j * np.pi * cyc)
    return pref * np.exp(-1j * np.pi * lam1 * z * r2 / (N * pitch) ** 2)


# ---------------------------------------------------------------------------
# Step 3: depth DFT (Eq. 7, rectangular gate of T frames)
# ---------------------------------------------------------------------------

def depth_dft(h: np.ndarray) -> np.ndarray:
    """V[q] = sum_t h_t exp(-2 pi i q t / T), unnormalised, natural order."""
    return np.fft.fft(h, axis=0)


def wavenumber_positions(lam) -> np.ndarray:
    """kappa_t = (k_t - k_0) / dk with k = 2 pi / lambda and dk the mean step
    (k_{T-1} - k_0) / (T - 1): the sweep position in units of the mean
    wavenumber step (equal to t for a sweep linear in k, setup paragraph)."""
    lam = np.asarray(lam, dtype=np.float64)
    T = lam.shape[0]
    if T == 1:
        return np.zeros(1)
    k = 2.0 * np.pi / lam
    dk = (k[-1] - k[0]) / (T - 1)
    return (k - k[0]) / dk


def depth_nudft(h: np.ndarray, kappa) -> np.ndarray:
    """V[q] = sum_t h_t exp(-2 pi i q kappa_t / T): Eq. 7 evaluated at the
    uniform depth grid for sweep positions kappa_t (a matrix product)."""
    T = h.shape[0]
    kappa = np.asarray(kappa, dtype=np.float64)
    cyc = np.mod(np.outer(np.arange(T), kappa), T) / T
    W = np.exp(-2j * np.pi * cyc)
    return np.tensordot(W, h, axes=(1, 0))


def depth_dft_adjoint(G: np.ndarray) -> np.ndarray:
    """beta_t = sum_q G_q exp(+2 pi i q t / T)."""
    return G.shape[0] * np.fft.ifft(G, axis=0)


# ---------------------------------------------------------------------------
# Angular-spectrum propagation (alternative propagator, no rescale)
# ---------------------------------------------------------------------------

def as_transfer(N: int, lam: float, pitch: float, z: float) -> np.ndarray:
    """exp(-2 pi i z sqrt(1/lambda^2 - fx^2 - fy^2)) on the DFT frequency grid, 0 where evanescent.

    Propagation by +z under the exp(+i omega t) convention of the paper's fields."""
    f = np.fft.fftfreq(N, d=pitch)
    rad = 1.0 / lam ** 2 - f[:, None] ** 2 - f[None, :] ** 2
    H = np.zeros((N, N), dtype=np.complex128)
    ok = rad > 0
    cyc = z * np.sqrt(rad[ok])
    H[ok] = np.exp(-2j * np.pi * (cyc - np.floor(cyc)))
    return H


def as_propagate(x, lam: float, pitch: float, z: float) -> np.ndarray:
    """Field x on the sensor grid propagated by z (angular spectrum, same grid)."""
    x = np.asarray(x)
    return np.fft.ifft2(np.fft.fft2(x) * as_transfer(x.shape[-1], lam, pitch, z))


def render_as(frames, lam, pitch, z, disp_phase=None, gate=None, nonuniform_k=False) -> np.ndarray:
    """Complex volume with angular-spectrum propagation of every frame at its own
    wavelength, then the depth transform of Eq. 7 (optionally gated / non-uniform)."""
    frames, lam = _check(frames, lam)
    T, N, _ = frames.shape
    phi = np.zeros(T) if disp_phase is None else np.asarray(disp_phase, dtype=np.float64)
    g = np.ones(T) if gate is None else np.asarray(gate, dtype=np.float64)
    out = np.empty((T, N, N), dtype=np.complex128)
    for t in range(T):
        out[t] = g[t] * np.exp(1j * phi[t]) * as_propagate(frames[t].astype(np.float64), lam[t], pitch, z)
    return depth_nudft(out, wavenumber_positions(lam)) if nonuniform_k else depth_dft(out)


def render_as_columns(frames, lam, pitch, z, pixels, disp_phase=None, gate=None) -> np.ndarray:
    """V[:, u, v] of ``render_as`` for each (u, v) in ``pixels`` (complex128 [T, P]): the forward DFT of
    each frame by the library FFT, times the transfer function, then the inverse DFT evaluated only at
    the sampled pixels as direct sums (integer phase indices reduced modulo N), and the depth sum of
    Eq. 7 term by term."""
    frames, lam = _check(frames, lam)
    T, N, _ = frames.shape
    pix = np.asarray(pixels, dtype=np.int64).reshape(-1, 2)
    k = np.arange(N)
    Eu = np.exp(2j * np.pi * (np.mod(np.outer(pix[:, 0], k), N) / N))   # [P, N] over row frequencies
    Ev = np.exp(2j * np.pi * (np.mod(np.outer(pix[:, 1], k), N) / N))   # [P, N] over column frequencies
    phi = np.zeros(T) if disp_phase is None else np.asarray(disp_phase, dtype=np.float64)
    g = np.ones(T) if gate is None else np.asarray(gate, dtype=np.float64)
    h = np.empty((T, pix.shape[0]), dtype=np.complex128)
    for t in range(T):
        A = np.fft.fft2(frames[t].astype(np.float64)) * as_transfer(N, lam[t], pitch, z)
        h[t] = g[t] * np.exp(1j * phi[t]) * np.sum((Eu @ A) * Ev, axis=1) / (N * N)
    tt = np.arange(T)
    W = np.exp(-2j * np.pi * (np.mod(np.outer(tt, tt), T) / T))        # W[q, t]
    return W @ h


# ---------------------------------------------------------------------------
# Whole chain
# ---------------------------------------------------------------------------

def _check(frames, lam):
    frames = np.asarray(frames)
    lam = np.asarray(lam, dtype=np.float64)
    if frames.ndim != 3 or frames.shape[1] != frames.shape[2]:
        raise ValueError("frames must be [T, N, N]")
    if lam.shape != (frames.shape[0],):
        raise ValueError("lambda must have one entry per frame")
    return frames, lam


def sensor_fields(frames, lam, pitch, z, zernike_coeffs=None, exact_chirp=False):
    """Yield x_t = Q_t A J_t for every frame: the input of the Fresnel transform."""
    frames, lam = _check(frames, lam)
    T, N, _ = frames.shape
    s = scale_factors(lam)
    alpha = chirp_rates(lam, pitch, z, exact_chirp)
    A = aberration(N, zernike_coeffs)
    for t in range(T):
        J = rescale(frames[t], s[t])
        yield t, chirp(N, alpha[t]) * A * J


def render(frames, lam, pitch, z, disp_phase=None, zernike_coeffs=None,
           exact_chirp=False, eq6_phase=False, gate=None, nonuniform_k=False) -> np.ndarray:
    """Complex volume V[q, u, v] (complex128) of one sweep of T frames."""
    frames, lam = _check(frames, lam)
    T, N, _ = frames.shape
    phi = np.zeros(T) if disp_phase is None else np.asarray(disp_phase, dtype=np.float64)
    g = np.ones(T) if gate is None else np.asarray(gate, dtype=np.float64)
    out = np.empty((T, N, N), dtype=np.complex128)
    fac = eq6_output_factor(N, reference_wavelength(lam), pitch, z) if eq6_phase else None
    for t, x in sensor_fields(frames, lam, pitch, z, zernike_coeffs, exact_chirp):
        h = fresnel_fft(x)
        if fac is not None:
            h = h * fac
        out[t] = g[t] * np.exp(1j * phi[t]) * h
    return depth_nudft(out, wavenumber_positions(lam)) if nonuniform_k else depth_dft(out)


def render_columns(frames, lam, pitch, z, pixels, disp_phase=None, zernike_coeffs=None,
                   exact_chirp=False, eq6_phase=False, gate=None, nonuniform_k=False) -> np.ndarray:
    """V[:, u, v] for each (u, v) in ``pixels``, by direct evaluation of the sums.

    Returns complex128 [T, P].  The Fresnel sum of Eq. 6 and the depth sum of
    Eq. 7 are evaluated term by term (integer phase indices reduced modulo N
    and T), without any FFT.
    """
    frames, lam = _check(frames, lam)
    T, N, _ = frames.shape
    pix = np.asarray(pixels, dtype=np.int64).reshape(-1, 2)
    cu = pix[:, 0] - N // 2
    cv = pix[:, 1] - N // 2
    cm = np.arange(N) - N // 2
    Eu = np.exp(2j * np.pi * (np.mod(np.outer(cu, cm), N) / N))   # [P, N] over rows m
    Ev = np.exp(2j * np.pi * (np.mod(np.outer(cv, cm), N) / N))   # [P, N] over cols n
    phi = np.zeros(T) if disp_phase is None else np.asarray(disp_phase, dtype=np.float64)
    if eq6_phase:
        fac = eq6_output_factor(N, reference_wavelength(lam), pitch, z)[pix[:, 0], pix[:, 1]]
    else:
        fac = np.ones(pix.shape[0], dtype=np.complex128)
    h = np.empty((T, pix.shape[0]), dtype=np.complex128)
    for t, x in sensor_fields(frames, lam, pitch, z, zernike_coeffs, exact_chirp):
        xv = x @ Ev.T                                   # [N(m), P]
        h[t] = (1.0 if gate is None else float(gate[t])) * np.exp(1j * phi[t]) * fac * np.sum(Eu * xv.T, axis=1)
    tt = np.arange(T)
    if nonuniform_k:
        W = np.exp(-2j * np.pi * (np.mod(np.outer(tt, wavenumber_positions(lam)), T) / T))
    else:
        W = np.exp(-2j * np.pi * (np.mod(np.outer(tt, tt), T) / T))  # W[q, t]
    return W @ h


def cuts(vol, x0: int, y0: int, q0: int, power: bool = False):
    """Three orthogonal cuts of the envelope (text after Eq. 7, caption of Fig. 3).

    cut_xy[u, v] = M[q0, u, v], cut_xz[q, v] = M[q, y0, v], cut_yz[q, u] = M[q, u, x0]
    with M = |V| (or |V|^2 when ``power``).
    """
    M = np.abs(vol)
    if power:
        M = M * M
    return M[q0, :, :].copy(), M[:, y0, :].copy(), M[:, :, x0].copy()


# ---------------------------------------------------------------------------
# Sharpness loss and its gradient (digital refocusing / aberration correction)
# ---------------------------------------------------------------------------

def sharpness(vol) -> float:
    """L = sum |V|^4 over every voxel."""
    a2 = np.abs(vol) ** 2
    return float(np.sum(a2 * a2))


def forward_linear(x, disp_phase=None):
    """The linear part of the chain: x_t -> V = W' F x (W'[q,t] = e^{-2 pi i qt/T} e^{i phi_t})."""
    T = x.shape[0]
    phi = np.zeros(T) if disp_phase is None else np.asarray(disp_phase, dtype=np.float64)
    h = fresnel_fft(x) * np.exp(1j * phi)[:, None, None]
    return depth_dft(h)


def adjoint_linear(G, disp_phase=None):
    """Adjoint of ``forward_linear``: G -> F^H W'^H G."""
    T = G.shape[0]
    phi = np.zeros(T) if disp_phase is None else np.asarray(disp_phase, dtype=np.float64)
    beta = depth_dft_adjoint(G) * np.exp(-1j * phi)[:, None, None]
    return fresnel_fft_adjoint(beta)


def vjp(frames, lam, pitch, z, G, disp_phase=None, zernike_coeffs=None, exact_chirp=False):
    """Gradients (dL/dz, dL/dc[15], dL/dphi[T]) of any real L with dL = Re sum conj(G) dV.

    G follows PyTorch's convention for complex tensors (G = 2 dL/d conj(V)).
    With gamma_t = F^H (exp(-i phi_t) sum_q exp(+2 pi i q t / T) G_q) and
    u_t = conj(gamma_t) x_t:
        dL/dphi_t = -Im sum u_t
        dL/dc_j   = -sum_t Im sum Z_j u_t
        dL/dz     = -sum_t (alpha_t / z) Im sum (c_m^2 + c_n^2) u_t
    (x_t = Q_t A J_t depends on z only through alpha_t = pi d^2 s_t^p/(lambda_1 z)).
    """
    frames, lam = _check(frames, lam)
    T, N, _ = frames.shape
    phi = np.zeros(T) if disp_phase is None else np.asarray(disp_phase, dtype=np.float64)
    alpha = chirp_rates(lam, pitch, z, exact_chirp)
    Z = zernike_stack(N)
    c = centred(N)
    r2 = c[:, None] ** 2 + c[None, :] ** 2
    beta = depth_dft_adjoint(np.asarray(G, dtype=np.complex128))
    dz = 0.0
    dc = np.zeros(N_ZERNIKE)
    dphi = np.zeros(T)
    for t, x in sensor_fields(frames, lam, pitch, z, zernike_coeffs, exact_chirp):
        gamma = fresnel_fft_adjoint(np.exp(-1j * phi[t]) * beta[t])
        u = np.conj(gamma) * x
        dphi[t] = -np.sum(u).imag
        dc -= np.tensordot(Z, u, axes=((1, 2), (0, 1))).imag
        dz -= alpha[t] / z * np.sum(r2 * u).imag
    return dz, dc, dphi


def sharpness_grad(frames, lam, pitch, z, disp_phase=None, zernike_coeffs=None, exact_chirp=False):
    """(L, dL/dz, dL/dc, dL/dphi) for L = sum |V|^4; the cotangent is G = 4 |V|^2 V."""
    V = render(frames, lam, pitch, z, disp_phase, zernike_coeffs, exact_chirp)
    L = sharpness(V)
    G = 4.0 * np.abs(V) ** 2 * V
    del V
    dz, dc, dphi = vjp(frames, lam, pitch, z, G, disp_phase, zernike_coeffs, exact_chirp)
    return L, dz, dc, dphi
