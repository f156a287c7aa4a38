"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: values the
paper prints, closed forms, exact invariants, brute-force sums on tiny inputs
or synthetic ground truth.  ``test_planted_mistakes`` plants plausible errors
in the oracle (on the CPU) and checks that at least one pin catches each.
"""
import json
import math
import os

import numpy as np
import pytest

from oracle import ssoct_oracle as O
from paper_2003_08960_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_printed_values.json")


def _golden():
    with open(GOLDEN) as f:
        return json.load(f)


# --------------------------------------------------------------------------
# Printed values (text after Eq. 3, caption of Fig. 2)
# --------------------------------------------------------------------------

def check_printed_axial():
    g = _golden()
    e = g["twice_axial_pitch_um"]
    lam1, lam2 = e["lam1_nm"] * 1e-9, e["lam2_nm"] * 1e-9
    assert abs(O.twice_axial_pitch(lam1, lam2) * 1e6 - e["value"]) <= e["printed_digits"]
    e = g["coherence_length_um"]
    assert abs(O.coherence_length(lam1, lam2) * 1e6 - e["value"]) <= e["printed_digits"]
    e = g["axial_range_mm"]
    nz = g["n_z"]["value"]
    for dl, printed in e["cases"]:
        l1 = (e["centre_nm"] + dl / 2) * 1e-9
        l2 = (e["centre_nm"] - dl / 2) * 1e-9
        assert abs(O.axial_range(l1, l2, nz) * 1e3 - printed) <= e["printed_digits"]


def test_printed_axial_values():
    check_printed_axial()


def test_depth_of_bin_matches_eq3():
    """Bin pitch of the depth DFT is Lambda/2 (Eq. 3) when the k step is Delta k / T."""
    lam1, lam2, T = 870e-9, 820e-9, 256
    lam = synth.sweep_wavelengths(T, lam1, lam2)
    pitch = O.depth_of_bin(1, lam)
    # endpoints inclusive: dk = Delta k / (T - 1)  =>  pitch = (Lambda/2)(T-1)/T
    assert pitch * T / (T - 1) == pytest.approx(O.twice_axial_pitch(lam1, lam2) / 2, rel=1e-12)
    assert O.depth_of_bin(T - 1, lam) == pytest.approx(-pitch, rel=1e-12)


def test_eq4_reconstructed_pitch_and_zb():
    assert O.reconstructed_pitch(870e-9, 0.3, 128, 20e-6) == pytest.approx(870e-9 * 0.3 / (128 * 20e-6))
    zb = O.boundary_distance(1024, 12e-6, 870e-9)
    assert zb == pytest.approx(0.16949, rel=1e-4)   # paper camera: z = 0.3 m is above z_b


# --------------------------------------------------------------------------
# Step 1: rescale (Eq. 5)
# --------------------------------------------------------------------------

def check_rescale():
    rng = np.random.default_rng(5)
    N = 32
    I = rng.integers(0, 65536, size=(N, N)).astype(np.uint16)
    # s = 1: every sample falls on its own pixel
    assert np.array_equal(O.rescale(I, 1.0), I.astype(np.float64))
    # a constant frame stays constant
    assert np.allclose(O.rescale(np.full((N, N), 777, np.uint16), 0.9), 777.0, rtol=0, atol=1e-9)
    # a bilinear ramp a + b x + e y is reproduced exactly at the scaled positions
    m, n = np.meshgrid(np.arange(N), np.arange(N), indexing="ij")
    ramp = 100.0 + 3.0 * n + 7.0 * m
    for s in (0.92, 0.8137, 0.5):
        J = O.rescale(ramp, s)
        c = np.arange(N) - N // 2
        X = N // 2 + c * s
        expect = 100.0 + 3.0 * X[None, :] + 7.0 * X[:, None]
        assert np.allclose(J, expect, rtol=0, atol=1e-9)


def test_rescale_pins():
    check_rescale()


# --------------------------------------------------------------------------
# Step 2: Fresnel transform (Eq. 6)
# --------------------------------------------------------------------------

def check_fresnel_closed_forms():
    N = 16
    c = np.arange(N) - N // 2
    # impulse at (m0, n0): h[u, v] = exp(+2 pi i (c_u c_m0 + c_v c_n0) / N)
    x = np.zeros((N, N), complex)
    x[3, 11] = 1.0
    h = O.fresnel_fft(x)
    expect = np.exp(2j * np.pi * (c[:, None] * c[3] + c[None, :] * c[11]) / N)
    assert np.allclose(h, expect, atol=1e-12)
    # plane wave exp(-2 pi i (a c_m + b c_n)/N) focuses to N^2 at (c_u, c_v) = (a, b)
    a, b = 3, -5
    x = np.exp(-2j * np.pi * (a * c[:, None] + b * c[None, :]) / N)
    h = O.fresnel_fft(x)
    k = np.unravel_index(np.argmax(np.abs(h)), h.shape)
    assert (c[k[0]], c[k[1]]) == (a, b)
    assert abs(h[k]) == pytest.approx(N * N)
    h[k] = 0
    assert np.max(np.abs(h)) < 1e-9


def test_fresnel_closed_forms():
    check_fresnel_closed_forms()


def test_fresnel_brute_force():
    """Direct double sum of Eq. 6 (with the centring and + sign) on 8x8 and 16x16."""
    rng = np.random.default_rng(7)
    for N in (8, 16):
        x = rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N))
        h = O.fresnel_fft(x)
        hb = np.zeros((N, N), complex)
        for u in range(N):
            for v in range(N):
                acc = 0j
                for m in range(N):
                    for n in range(N):
                        acc += x[m, n] * complex(np.exp(2j * np.pi * ((u - N // 2) * (m - N // 2)
                                                                      + (v - N // 2) * (n - N // 2)) / N))
                hb[u, v] = acc
        assert np.allclose(h, hb, rtol=0, atol=1e-9 * np.abs(hb).max())


def check_point_source_focus():
    """A spherical wave exp(+i pi |r' - r0|^2 / (lambda z)) focuses at c = r0 / d' (Eq. 4, 6)."""
    N, d, z, lam = 64, 20e-6, 0.1, 800e-9
    dprime = O.reconstructed_pitch(lam, z, N, d)
    c = np.arange(N) - N // 2
    xs = c * d
    for (cy, cx) in ((5, -9), (0, 0), (-13, 7)):
        y0, x0 = cy * dprime, cx * dprime
        field = np.exp(1j * np.pi * ((xs[:, None] - y0) ** 2 + (xs[None, :] - x0) ** 2) / (lam * z))
        frames = np.zeros((1, N, N))
        # drive the oracle through its own chirp by passing the field as the "rescaled" frame
        alpha = O.chirp_rates([lam], d, z)[0]
        h = O.fresnel_fft(O.chirp(N, alpha) * field)
        k = np.unravel_index(np.argmax(np.abs(h)), h.shape)
        assert (c[k[0]], c[k[1]]) == (cy, cx)
        del frames


def test_point_source_focus():
    check_point_source_focus()


def test_pitch_equalisation():
    check_pitch_equalisation()


def check_pitch_equalisation():
    """Eq. 4 + Eq. 5: with the rescale, two points dx apart are dx/d'(lambda_1) pixels apart at
    every wavelength; without it (single-frame sweep, s = 1) they are dx N d/(lambda_t z) apart."""
    N, d, z = 128, 20e-6, 0.3
    lam1, lamt = 870e-9, 800e-9
    dp1 = O.reconstructed_pitch(lam1, z, N, d)
    sep_px = 24.0
    dx = sep_px * dp1
    c = np.arange(N) - N // 2
    xs = c * d
    fc = 1.0 / (8 * d)

    def hologram(lt):
        ref = np.exp(2j * np.pi * fc * lam1 / lt * xs)
        Elo = np.outer(ref, ref)
        E = np.zeros((N, N), complex)
        for x0 in (-dx / 2, dx / 2):
            E += 0.2 * np.exp(1j * np.pi * ((xs[:, None]) ** 2 + (xs[None, :] - x0) ** 2) / (lt * z))
        return np.abs(Elo + E) ** 2

    def centroids(V):
        M = np.abs(V[0]) ** 2
        row = M[N // 2 + N // 8]
        # two peaks around the +1 order; centroid of each
        cols = np.arange(N)
        left = (cols > N // 2) & (cols < N // 2 + N // 8)
        right = (cols >= N // 2 + N // 8) & (cols < N)
        pk = []
        for msk in (left, right):
            w = np.where(msk, row, 0.0)
            i = int(np.argmax(w))
            win = slice(i - 2, i + 3)
            pk.append(np.sum(cols[win] * row[win]) / np.sum(row[win]))
        return pk[1] - pk[0]

    I1 = hologram(lam1)
    It = hologram(lamt)
    frames = np.stack([I1, It])
    V = O.render(frames, [lam1, lamt], d, z, exact_chirp=True)
    # rescaled: bin 0 of the depth transform mixes both frames; transform each frame alone
    V1 = O.render(frames[:1], [lam1], d, z)
    Vt_rescaled = np.fft.ifft(V, axis=0)[1:2] * 2   # frame t back from the 2-point DFT
    Vt_raw = O.render(frames[1:], [lamt], d, z)
    assert centroids(V1) == pytest.approx(sep_px, abs=0.05)
    assert centroids(Vt_rescaled) == pytest.approx(sep_px, abs=0.05)
    assert centroids(Vt_raw) == pytest.approx(dx * N * d / (lamt * z), abs=0.05)


# --------------------------------------------------------------------------
# Step 3: depth DFT (Eq. 7)
# --------------------------------------------------------------------------

def check_depth_tone():
    """A tone exp(+2 i k_t delta) on bin q_m gives exactly T at q_m (sign of Eq. 7)."""
    T, qm = 16, 5
    t = np.arange(T)
    h = np.exp(2j * np.pi * qm * t / T)[:, None, None] * np.ones((1, 2, 2))
    V = O.depth_dft(h)
    expect = np.zeros(T)
    expect[qm] = T
    assert np.allclose(np.abs(V[:, 0, 0]), expect, atol=1e-9)


def test_depth_tone():
    check_depth_tone()


def test_depth_brute_force():
    rng = np.random.default_rng(3)
    T = 7
    h = rng.standard_normal((T, 3, 2)) + 1j * rng.standard_normal((T, 3, 2))
    V = O.depth_dft(h)
    Vb = np.zeros_like(h)
    for q in range(T):
        for t in range(T):
            Vb[q] += h[t] * np.exp(-2j * np.pi * q * t / T)
    assert np.allclose(V, Vb, atol=1e-10)


# --------------------------------------------------------------------------
# Whole chain
# --------------------------------------------------------------------------

def _small_case(T=6, N=16, seed=11):
    rng = np.random.default_rng(seed)
    frames = rng.integers(0, 65536, size=(T, N, N)).astype(np.uint16)
    lam = synth.sweep_wavelengths(T, 870e-9, 800e-9)
    phi = rng.uniform(-2, 2, T)
    zc = rng.normal(0, 0.5, 15)
    return frames, lam, 20e-6, 0.05, phi, zc


def check_parseval():
    frames, lam, d, z, phi, zc = _small_case()
    T, N, _ = frames.shape
    s = O.scale_factors(lam)
    EJ = sum(np.sum(O.rescale(frames[t], s[t]) ** 2) for t in range(T))
    for exact in (False, True):
        V = O.render(frames, lam, d, z, phi, zc, exact_chirp=exact)
        assert np.sum(np.abs(V) ** 2) == pytest.approx(T * N * N * EJ, rel=1e-12)


def test_parseval():
    check_parseval()


def test_render_matches_direct_sums():
    """FFT-based render vs the term-by-term sums of Eq. 6 and Eq. 7 (every pixel, tiny size)."""
    frames, lam, d, z, phi, zc = _small_case(T=5, N=16)
    N = frames.shape[1]
    pix = [(u, v) for u in range(N) for v in range(N)]
    for kw in ({}, {"exact_chirp": True}, {"eq6_phase": True}):
        V = O.render(frames, lam, d, z, phi, zc, **kw)
        Vc = O.render_columns(frames, lam, d, z, pix, phi, zc, **kw)
        assert np.allclose(V.reshape(V.shape[0], -1), Vc, rtol=0, atol=1e-9 * np.abs(Vc).max())


def test_eq6_phase_only_scales_magnitude():
    frames, lam, d, z, phi, zc = _small_case()
    V0 = O.render(frames, lam, d, z, phi, zc)
    V1 = O.render(frames, lam, d, z, phi, zc, eq6_phase=True)
    lam1 = O.reference_wavelength(lam)
    assert np.allclose(np.abs(V1), np.abs(V0) * d * d / (lam1 * z), rtol=1e-10, atol=0)


def check_eq6_as_printed():
    """Eq. 6 exactly as printed, evaluated term by term at the output pixels x = c_u d' (Eq. 4):
    H(x, y) = (i / (lambda_1 z)) exp(-i k_1 z) d^2 sum_{x', y'} I'(x', y')
              exp[-i pi ((x - x')^2 + (y - y')^2) / (lambda_1 z)]
    on the rescaled frames I' (Eq. 5), then the depth sum of Eq. 7; against render(eq6_phase=True).
    The quadratic is not expanded here, so the DFT sign, the centring, the input chirp, the prefactor
    i exp(-i k_1 z) d^2 / (lambda_1 z) and the output phase are all checked in their complex values."""
    frames, lam, d, z, _, _ = _small_case(T=4, N=16, seed=21)
    T, N, _ = frames.shape
    lam1 = float(np.max(lam))
    s = lam / lam1
    dprime = lam1 * z / (N * d)                        # Eq. 4
    c = np.arange(N) - N // 2
    xs = c * d                                         # sensor (calculation-grid) coordinates
    xo = c * dprime                                    # output coordinates
    E = np.exp(-1j * np.pi * (xo[:, None] - xs[None, :]) ** 2 / (lam1 * z))   # [output, sensor]
    pref = 1j / (lam1 * z) * np.exp(-1j * 2 * np.pi * z / lam1) * d * d
    H = np.empty((T, N, N), dtype=np.complex128)
    for t in range(T):
        Ip = O.rescale(frames[t], s[t])                # I'(x', y') at x' = c d
        H[t] = pref * (E @ Ip @ E.T)                   # rows y, columns x
    tt = np.arange(T)
    W = np.exp(-2j * np.pi * np.outer(tt, tt) / T)     # Eq. 7, rectangular gate of the T frames
    V_printed = np.tensordot(W, H, axes=(1, 0))
    V = O.render(frames, lam, d, z, eq6_phase=True)
    assert np.linalg.norm(V - V_printed) <= 1e-10 * np.linalg.norm(V_printed)


def test_eq6_as_printed():
    check_eq6_as_printed()


def check_as_matches_eq6_at_zb():
    """At z = z_b = N d^2 / lambda_1 the Fresnel pixel of Eq. 4 equals the sensor pitch, and the
    sampled Eq. 6 (prefactor and output phase included) is a circular convolution whose transfer
    function is exactly exp(-i k z) exp(i pi lambda z f^2) (a Gauss sum): the paraxial limit of the
    angular-spectrum transfer function.  So, for one wavelength, render(eq6_phase=True) and
    render_as agree pixel by pixel in complex value, up to the non-paraxial phase
    2 pi z lambda^3 f^4 / 8 at most (f^2 <= 1 / (2 d^2)).  This pins the sign of the angular
    spectrum's z to the one of Eq. 6."""
    rng = np.random.default_rng(31)
    T, N, d, lam0 = 3, 16, 1e-3, 870e-9
    frames = rng.integers(0, 65536, size=(T, N, N)).astype(np.uint16)
    lam = np.full(T, lam0)
    zb = O.boundary_distance(N, d, lam0)
    bound = 2 * np.pi * zb * lam0 ** 3 * (1.0 / (2 * d * d)) ** 2 / 8
    assert bound < 1e-5
    Vf = O.render(frames, lam, d, zb, eq6_phase=True)
    Va = O.render_as(frames, lam, d, zb)
    assert np.linalg.norm(Vf - Va) <= 2 * bound * np.linalg.norm(Va)
    # the opposite z is a different plane: the agreement is not an accident of the input
    assert np.linalg.norm(Vf - O.render_as(frames, lam, d, -zb)) > 0.5 * np.linalg.norm(Va)


def test_as_matches_eq6_at_zb():
    check_as_matches_eq6_at_zb()


def test_generator_scatterers_focus():
    """Synthetic ground truth: every scatterer of the tiny workload peaks at its pixel and bin."""
    sw = synth.make_config("tiny")
    for exact in (False, True):
        M = np.abs(O.render(sw.frames, sw.lam, sw.pitch, sw.z, exact_chirp=exact))
        for u, v, q, _ in sw.scatterers:
            u, v, q = int(u), int(v), int(q)
            win = M[q, u - 2:u + 3, v - 2:v + 3]
            assert np.unravel_index(np.argmax(win), win.shape) == (2, 2)
            assert int(np.argmax(M[1:M.shape[0] // 2, u, v])) + 1 == q


def test_cuts_indexing():
    T, N = 5, 8
    q, u, v = np.meshgrid(np.arange(T), np.arange(N), np.arange(N), indexing="ij")
    vol = (1000 * q + 10 * u + v) * np.exp(1j * (q + u - v))
    xy, xz, yz = O.cuts(vol, x0=3, y0=6, q0=2)
    assert np.allclose(xy, 2000 + 10 * u[0] + v[0])
    assert np.allclose(xz, 1000 * q[:, 0, :] + 60 + v[:, 0, :])
    assert np.allclose(yz, 1000 * q[:, :, 0] + 10 * u[:, :, 0] + 3)
    xy2, _, _ = O.cuts(vol, 3, 6, 2, power=True)
    assert np.allclose(xy2, xy ** 2)


# --------------------------------------------------------------------------
# Zernike basis
# --------------------------------------------------------------------------

def test_zernike_closed_forms_and_orthonormality():
    rho = np.linspace(0, 1, 7)
    th = np.linspace(-3, 3, 7)
    assert np.allclose(O.zernike(0, rho, th), 1.0)
    assert np.allclose(O.zernike(4, rho, th), math.sqrt(3) * (2 * rho ** 2 - 1))
    assert np.allclose(O.zernike(12, rho, th), math.sqrt(5) * (6 * rho ** 4 - 6 * rho ** 2 + 1))
    assert np.allclose(O.zernike(3, rho, th), math.sqrt(6) * rho ** 2 * np.sin(2 * th))
    assert np.allclose(O.zernike(9, rho, th), math.sqrt(8) * rho ** 3 * np.cos(3 * th))
    # (1/pi) int_disk Z_j Z_k rho d rho d theta = delta_jk (Gauss-Legendre x uniform angle)
    xr, wr = np.polynomial.legendre.leggauss(24)
    r = 0.5 * (xr + 1)
    wr = 0.5 * wr
    na = 64
    a = 2 * np.pi * np.arange(na) / na
    R, A = np.meshgrid(r, a, indexing="ij")
    W = (wr[:, None] * R) * (2 * np.pi / na) / np.pi
    Z = np.stack([O.zernike(j, R, A) for j in range(15)])
    G = np.einsum("jab,kab,ab->jk", Z, Z, W)
    assert np.allclose(G, np.eye(15), atol=1e-10)


def check_pupil_grid():
    """rho = r / (N d / sqrt 2): exactly 1 at the corner pixel (the circumscribed circle) and 0 at the
    centre; theta = atan2(y, x) with x along columns and y along rows."""
    N = 16
    rho, th = O.pupil_grid(N)
    assert rho[0, 0] == pytest.approx(1.0, abs=1e-15)
    assert rho[N // 2, N // 2] == 0.0
    assert rho[N // 2, N - 1] == pytest.approx((N // 2 - 1) * math.sqrt(2) / N, abs=1e-15)
    assert th[N // 2, N // 2 + 3] == pytest.approx(0.0, abs=1e-15)        # +x: along the row
    assert th[N // 2 + 3, N // 2] == pytest.approx(np.pi / 2, abs=1e-15)  # +y: down the column
    # a tilt Z_2 = 2 rho cos(theta) = 2 sqrt(2) c_n / N (Z_1: c_m) of coefficient k pi / sqrt 2 is the
    # linear phase 2 pi k c / N, which moves the Fresnel DFT (Eq. 6) by exactly -k pixels along v
    # (u for Z_1): the whole volume is circularly shifted, whatever the other coefficients
    frames, lam, d, z, phi, zc = _small_case(T=3, N=16, seed=41)
    V0 = O.render(frames, lam, d, z, phi, zc)
    for j, axis in ((2, 2), (1, 1)):
        for k in (1, 3):
            c = zc.copy()
            c[j] += k * np.pi / math.sqrt(2)
            V = O.render(frames, lam, d, z, phi, c)
            assert np.allclose(V, np.roll(V0, -k, axis=axis), rtol=0, atol=1e-9 * np.abs(V0).max())


def test_pupil_grid():
    check_pupil_grid()


# --------------------------------------------------------------------------
# Adjoint and gradient
# --------------------------------------------------------------------------

def test_dot_product_adjoint():
    rng = np.random.default_rng(1)
    T, N = 6, 16
    x = rng.standard_normal((T, N, N)) + 1j * rng.standard_normal((T, N, N))
    G = rng.standard_normal((T, N, N)) + 1j * rng.standard_normal((T, N, N))
    phi = rng.uniform(-3, 3, T)
    lhs = np.vdot(G, O.forward_linear(x, phi))
    rhs = np.vdot(O.adjoint_linear(G, phi), x)
    assert lhs == pytest.approx(rhs, rel=1e-12)


def _fd_case():
    frames, lam, d, z, phi, zc = _small_case(T=6, N=16, seed=21)
    return frames, lam, d, z, phi, zc


def check_gradient_fd(exact=False):
    frames, lam, d, z, phi, zc = _fd_case()
    L, dz, dc, dphi = O.sharpness_grad(frames, lam, d, z, phi, zc, exact)

    def loss(z_=z, phi_=phi, zc_=zc):
        return O.sharpness(O.render(frames, lam, d, z_, phi_, zc_, exact))

    h = 1e-6 * z
    fd = (loss(z_=z + h) - loss(z_=z - h)) / (2 * h)
    assert dz == pytest.approx(fd, rel=1e-6)
    for j in (1, 4, 7, 12):
        e = np.zeros(15)
        e[j] = 1e-4
        fd = (loss(zc_=zc + e) - loss(zc_=zc - e)) / 2e-4
        assert dc[j] == pytest.approx(fd, rel=1e-5, abs=1e-9 * abs(L))
    for t in (0, 3, 5):
        e = np.zeros(frames.shape[0])
        e[t] = 1e-4
        fd = (loss(phi_=phi + e) - loss(phi_=phi - e)) / 2e-4
        assert dphi[t] == pytest.approx(fd, rel=1e-5, abs=1e-9 * abs(L))
    return L, dz, dc, dphi


def test_gradient_finite_differences():
    check_gradient_fd(False)
    check_gradient_fd(True)


def test_gradient_invariants():
    """Global phase invariance: sum_t dL/dphi_t = 0 and dL/dc_0 = 0 (Z_0 = 1)."""
    frames, lam, d, z, phi, zc = _fd_case()
    L, dz, dc, dphi = O.sharpness_grad(frames, lam, d, z, phi, zc)
    scale = np.max(np.abs(dphi))
    assert abs(np.sum(dphi)) < 1e-9 * scale
    assert abs(dc[0]) < 1e-9 * np.max(np.abs(dc))


# --------------------------------------------------------------------------
# Apodised gate and sweeps that are not linear in k (extensions of Eq. 7)
# --------------------------------------------------------------------------

def chirped_wavelengths(T, lam_max=870e-9, lam_min=800e-9, bend=0.15):
    """A sweep whose wavenumber is a quadratic, not linear, function of t."""
    u = np.linspace(0.0, 1.0, T)
    k0, k1 = 2 * np.pi / lam_max, 2 * np.pi / lam_min
    return 2 * np.pi / (k0 + (k1 - k0) * (u + bend * u * (u - 1.0)))


def check_wavenumber_positions():
    # k = 2 pi (1, 2, 4): mean step 3 pi, so kappa = (0, 2/3, 2) exactly
    kap = O.wavenumber_positions([1.0, 0.5, 0.25])
    assert np.allclose(kap, [0.0, 2.0 / 3.0, 2.0], rtol=0, atol=1e-14)
    lam = synth.sweep_wavelengths(37, 870e-9, 800e-9)          # linear in k
    assert np.allclose(O.wavenumber_positions(lam), np.arange(37), rtol=0, atol=1e-9)


def check_nudft_tone():
    T = 48
    kap = O.wavenumber_positions(chirped_wavelengths(T))
    assert not np.allclose(kap, np.arange(T), atol=0.5)       # really non-uniform
    for qm in (0, 5, 17, 40):
        h = np.exp(2j * np.pi * qm * kap / T)[:, None]
        V = O.depth_nudft(h, kap)
        assert abs(V[qm, 0] - T) < 1e-9 * T
    h = np.random.default_rng(1).standard_normal((T, 3)) + 1j
    assert np.allclose(O.depth_nudft(h, np.arange(T)), np.fft.fft(h, axis=0), atol=1e-10)


def check_chirped_scatterer_focus():
    """Field of a reflector at depth delta: h_t = exp(i 2 k_t delta).  On the uniform depth grid
    delta_q = q pi / (T dk) the non-uniform transform puts exactly T in bin q_m; the plain DFT,
    which assumes k linear in t, spreads it."""
    T = 64
    lam = chirped_wavelengths(T)
    k = 2 * np.pi / lam
    dk = (k[-1] - k[0]) / (T - 1)
    qm = 13
    delta = qm * np.pi / (T * dk)
    h = np.exp(1j * 2 * (k - k[0]) * delta)[:, None]
    V = O.depth_nudft(h, O.wavenumber_positions(lam))
    assert abs(abs(V[qm, 0]) - T) < 1e-8 * T
    assert np.argmax(np.abs(V[:, 0])) == qm
    assert abs(O.depth_dft(h)[qm, 0]) < 0.9 * T


def check_hann_gate():
    """Frames F0 U + a cos(2 pi q_m t / T) P at one wavelength: with the periodic Hann gate
    sin^2(pi t / T) the tone's bin halves and its neighbours take exactly -1/2 of it."""
    T, N, qm = 32, 16, 6
    rng = np.random.default_rng(4)
    U = np.ones((N, N))
    Pm = rng.uniform(0.0, 1.0, (N, N))
    t = np.arange(T)
    frames = 1000.0 * U[None] + 300.0 * np.cos(2 * np.pi * qm * t / T)[:, None, None] * Pm[None]
    lam = np.full(T, 850e-9)
    g = np.sin(np.pi * t / T) ** 2
    Vr = O.render(frames, lam, 20e-6, 0.05)
    Vh = O.render(frames, lam, 20e-6, 0.05, gate=g)
    scale = np.abs(Vr[qm]).max()
    assert np.allclose(Vh[qm], 0.5 * Vr[qm], atol=1e-9 * scale)
    assert np.allclose(Vh[qm + 1], -0.25 * Vr[qm], atol=1e-9 * scale)
    assert np.allclose(Vh[qm - 1], -0.25 * Vr[qm], atol=1e-9 * scale)
    assert np.abs(Vh[qm + 3]).max() < 1e-9 * scale


def test_wavenumber_positions():
    check_wavenumber_positions()


def test_nudft_tone():
    check_nudft_tone()


def test_chirped_scatterer_focus():
    check_chirped_scatterer_focus()


def test_hann_gate():
    check_hann_gate()


def test_render_extensions_reduce_to_the_paper_form():
    """nonuniform_k on a k-linear sweep and a unit gate change nothing; direct sums agree."""
    sw = synth.make_config("tiny")
    V = O.render(sw.frames, sw.lam, sw.pitch, sw.z)
    assert np.allclose(O.render(sw.frames, sw.lam, sw.pitch, sw.z, nonuniform_k=True), V,
                       atol=1e-9 * np.abs(V).max())
    assert np.array_equal(O.render(sw.frames, sw.lam, sw.pitch, sw.z, gate=np.ones(len(sw.lam))), V)
    lam = chirped_wavelengths(len(sw.lam))
    g = np.hanning(len(lam))
    Vn = O.render(sw.frames, lam, sw.pitch, sw.z, gate=g, nonuniform_k=True)
    pix = [(3, 5), (64, 64), (100, 20)]
    cols = O.render_columns(sw.frames, lam, sw.pitch, sw.z, pix, gate=g, nonuniform_k=True)
    for i, (u, v) in enumerate(pix):
        assert np.allclose(cols[:, i], Vn[:, u, v], atol=1e-8 * np.abs(Vn).max())


# --------------------------------------------------------------------------
# Angular-spectrum propagation
# --------------------------------------------------------------------------

def check_as_plane_wave():
    """An on-grid plane wave exp(2 pi i (a m + b n) / N) is an eigenfunction: propagated by +z it
    gains exactly exp(-2 pi i z sqrt(1/lambda^2 - (a/(N d))^2 - (b/(N d))^2)) (the exp(-i k z) of a wave
    travelling +z when fields carry exp(+i omega t), as in the paper), or vanishes if evanescent."""
    N, d, lam, z = 32, 10e-6, 850e-9, 0.01
    m = np.arange(N)
    for a, b in ((0, 0), (3, -5), (-16, 7), (11, 11)):
        x = np.exp(2j * np.pi * (a * m[:, None] + b * m[None, :]) / N)
        fx, fy = a / (N * d), b / (N * d)
        want = np.exp(-2j * np.pi * z * np.sqrt(1 / lam ** 2 - fx ** 2 - fy ** 2))
        assert np.allclose(O.as_propagate(x, lam, d, z), want * x, atol=1e-9)
    dd = 0.3e-6                                           # pitch below lambda / 2: the highest frequencies are evanescent
    x = np.exp(2j * np.pi * (16 * m[:, None]) / N) * np.ones((1, N))   # f = 1/(2 dd) > 1/lambda
    assert np.abs(O.as_propagate(x, lam, dd, z)).max() < 1e-12
    with np.errstate(all="ignore"):
        assert np.abs(O.as_propagate(x, lam, dd, -z)).max() < 1e-12   # dropped, not amplified, going back


def check_as_composition():
    """Propagating by z1 then z2 equals propagating by z1 + z2; z = 0 is the identity."""
    rng = np.random.default_rng(8)
    N, d, lam = 32, 12e-6, 830e-9
    x = rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N))
    assert np.allclose(O.as_propagate(x, lam, d, 0.0), x, atol=1e-12)
    a = O.as_propagate(O.as_propagate(x, lam, d, 0.004), lam, d, 0.011)
    assert np.allclose(a, O.as_propagate(x, lam, d, 0.015), atol=1e-9)
    back = O.as_propagate(O.as_propagate(x, lam, d, 0.02), lam, d, -0.02)
    assert np.allclose(back, x, atol=1e-9)               # no evanescent band at this pitch


def check_as_point_focus():
    """The diverging field exp(-i k r) / r of a point source at distance z (exp(+i omega t)
    convention), sampled on the sensor and band-limited to the grid, propagates back (by -z) to a
    peak at the source pixel."""
    N, d, lam, z = 64, 8e-6, 850e-9, 0.004
    c = (np.arange(N) - N // 2) * d
    r = np.sqrt(c[:, None] ** 2 + (c[None, :] - 5 * d) ** 2 + z ** 2)
    x = np.exp(-2j * np.pi * (r / lam)) / r
    back = np.abs(O.as_propagate(x, lam, d, -z))
    i, j = np.unravel_index(np.argmax(back), back.shape)
    assert (i, j) == (N // 2, N // 2 + 5)


def test_as_plane_wave():
    check_as_plane_wave()


def test_as_composition():
    check_as_composition()


def test_as_point_focus():
    check_as_point_focus()


def test_render_as_parseval_and_depth():
    """With no evanescent band, the angular spectrum is unitary per frame: sum |V|^2 = T sum ||I_t||^2."""
    rng = np.random.default_rng(2)
    T, N = 8, 16
    frames = rng.integers(0, 4096, size=(T, N, N)).astype(np.uint16)
    lam = synth.sweep_wavelengths(T, 870e-9, 800e-9)
    V = O.render_as(frames, lam, 10e-6, 0.02)
    assert abs(np.sum(np.abs(V) ** 2) / (T * np.sum(frames.astype(np.float64) ** 2)) - 1) < 1e-12


def test_render_as_columns_match_render_as():
    """The sampled-pixel evaluation (inverse DFT as direct sums) against the FFT-based render_as, every
    pixel of a tiny sweep, with dispersion and a gate."""
    rng = np.random.default_rng(3)
    T, N = 5, 16
    frames = rng.integers(0, 65536, size=(T, N, N)).astype(np.uint16)
    lam = synth.sweep_wavelengths(T, 870e-9, 800e-9)
    phi, g = rng.uniform(-2, 2, T), np.hanning(T)
    V = O.render_as(frames, lam, 10e-6, 0.003, phi, g)
    pix = [(u, v) for u in range(N) for v in range(N)]
    Vc = O.render_as_columns(frames, lam, 10e-6, 0.003, pix, phi, g)
    assert np.allclose(V.reshape(T, -1), Vc, rtol=0, atol=1e-10 * np.abs(V).max())


# --------------------------------------------------------------------------
# Planted mistakes: each plausible error in the oracle must fail a pin
# --------------------------------------------------------------------------

def _plants():
    yield "depth sign", "depth_dft", lambda orig: (lambda h: np.conj(orig(np.conj(h)))), check_depth_tone
    yield "fresnel sign", "fresnel_fft", lambda orig: (lambda x: np.conj(orig(np.conj(x)))), \
        check_fresnel_closed_forms
    yield "fresnel no centring", "fresnel_fft", \
        lambda orig: (lambda x: x.shape[-1] ** 2 * np.fft.ifft2(x, axes=(-2, -1))), check_fresnel_closed_forms
    yield "rescale inverted", "scale_factors", lambda orig: (lambda lam: 1.0 / orig(lam)), check_pitch_equalisation
    yield "rescale off-centre", "interp_positions", lambda orig: (
        lambda N, s: orig(N, s) if s == 1.0 else _shifted_positions(N, s)), check_rescale
    yield "chirp sign", "chirp", lambda orig: (lambda N, a: np.conj(orig(N, a))), check_point_source_focus
    yield "chirp factor 2", "chirp_rates", lambda orig: (lambda *a, **k: 2 * orig(*a, **k)), \
        check_point_source_focus
    yield "axial range halved", "axial_range", lambda orig: (lambda a, b, n: orig(a, b, n) / 2), \
        check_printed_axial
    yield "kappa from lambda", "wavenumber_positions", lambda orig: (
        lambda lam: (np.asarray(lam, float) - lam[0]) / ((lam[-1] - lam[0]) / (len(lam) - 1))), \
        check_wavenumber_positions
    yield "kappa from lambda (physics)", "wavenumber_positions", lambda orig: (
        lambda lam: (np.asarray(lam, float) - lam[0]) / ((lam[-1] - lam[0]) / (len(lam) - 1))), \
        check_chirped_scatterer_focus
    yield "nudft sign", "depth_nudft", lambda orig: (lambda h, kap: np.conj(orig(np.conj(h), kap))), check_nudft_tone
    yield "gate ignored", "render", lambda orig: (lambda *a, gate=None, **k: orig(*a, **k)), check_hann_gate
    yield "AS conjugate kernel", "as_transfer", lambda orig: (lambda *a: np.conj(orig(*a))), check_as_plane_wave
    yield "AS Fresnel kernel", "as_transfer", lambda orig: (lambda N, lam, d, z: _fresnel_transfer(N, lam, d, z)), \
        check_as_plane_wave
    yield "AS keeps evanescent", "as_transfer", lambda orig: (lambda N, lam, d, z: _no_cutoff_transfer(N, lam, d, z)), \
        check_as_plane_wave
    yield "AS frequencies unfolded", "as_transfer", lambda orig: (lambda N, lam, d, z: _unfolded_transfer(N, lam, d, z)), \
        check_as_plane_wave
    yield "eq6 prefactor without i", "eq6_output_factor", lambda orig: (lambda *a: -1j * orig(*a)), \
        check_eq6_as_printed
    yield "eq6 output phase conjugated", "eq6_output_factor", lambda orig: (
        lambda N, lam1, d, z: orig(N, lam1, d, z) * _quad_phase(N, lam1, d, z) ** 2), check_eq6_as_printed
    yield "eq6 k1 z sign", "eq6_output_factor", lambda orig: (
        lambda N, lam1, d, z: orig(N, lam1, d, z) * np.exp(4j * np.pi * (z / lam1 % 1.0))), check_eq6_as_printed
    yield "eq6 output phase conjugated (AS)", "eq6_output_factor", lambda orig: (
        lambda N, lam1, d, z: orig(N, lam1, d, z) * _quad_phase(N, lam1, d, z) ** 2), check_as_matches_eq6_at_zb
    yield "AS conjugate kernel (Eq. 6)", "as_transfer", lambda orig: (lambda *a: np.conj(orig(*a))), \
        check_as_matches_eq6_at_zb
    yield "pupil radius N/2", "pupil_grid", lambda orig: (lambda N: (lambda r, t: (r * math.sqrt(2), t))(*orig(N))), \
        check_pupil_grid
    yield "pupil axes swapped", "pupil_grid", lambda orig: (lambda N: (lambda r, t: (r, np.pi / 2 - t))(*orig(N))), \
        check_pupil_grid
    yield "gate squared", "render", lambda orig: (
        lambda *a, gate=None, **k: orig(*a, gate=None if gate is None else np.asarray(gate) ** 2, **k)), \
        check_hann_gate


def _quad_phase(N, lam1, d, z):
    """exp(+i pi lambda_1 z (c_u^2 + c_v^2) / (N d)^2): the conjugate of the Eq. 6 output phase."""
    c = np.arange(N) - N // 2
    return np.exp(1j * np.pi * lam1 * z * (c[:, None] ** 2 + c[None, :] ** 2) / (N * d) ** 2)


def _fresnel_transfer(N, lam, d, z):
    f = np.fft.fftfreq(N, d=d)
    return np.exp(-2j * np.pi * z / lam) * np.exp(1j * np.pi * lam * z * (f[:, None] ** 2 + f[None, :] ** 2))


def _no_cutoff_transfer(N, lam, d, z):
    f = np.fft.fftfreq(N, d=d)
    rad = (1.0 / lam ** 2 - f[:, None] ** 2 - f[None, :] ** 2).astype(np.complex128)
    return np.exp(-2j * np.pi * z * np.sqrt(rad))


def _unfolded_transfer(N, lam, d, z):
    f = np.arange(N) / (N * d)
    rad = 1.0 / lam ** 2 - f[:, None] ** 2 - f[None, :] ** 2
    return np.where(rad > 0, np.exp(-2j * np.pi * z * np.sqrt(np.maximum(rad, 0))), 0)


def _shifted_positions(N, s):
    P = np.arange(N) * s
    j0 = np.floor(P).astype(np.int64)
    return j0, np.minimum(j0 + 1, N - 1), P - j0


def check_rescale_chain():
    """Rescale through the whole chain keeps every sample inside the frame (s <= 1)."""
    lam = synth.sweep_wavelengths(4, 870e-9, 800e-9)
    s = O.scale_factors(lam)
    assert np.all(s <= 1.0) and s[0] == 1.0


@pytest.mark.parametrize("name,attr,mutate,pin", list(_plants()), ids=[p[0] for p in _plants()])
def test_planted_mistakes(monkeypatch, name, attr, mutate, pin):
    pin()                                   # passes on the real oracle
    orig = getattr(O, attr)
    monkeypatch.setattr(O, attr, mutate(orig))
    with pytest.raises(AssertionError):
        pin()
