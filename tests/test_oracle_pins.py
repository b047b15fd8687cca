"""Pins of the FP64 oracle against what the paper and the mathematics fix.

None of these tests re-types an oracle formula: each compares the oracle with
an independent computation (brute-force sums, closed forms, invariants that
follow from the model, finite differences, a library optimiser).
"""
import math
import os

import numpy as np
import pytest

import oracle as orc
from paper_2505_14372_amd import synth

HERE = os.path.dirname(os.path.abspath(__file__))


# ---------------------------------------------------------------- helpers

def brute_dft2(x, inverse=False):
    """O(N^4) unitary 2D DFT written as explicit sums."""
    N = x.shape[-1]
    s = 1.0 if inverse else -1.0
    out = np.zeros(x.shape, dtype=np.complex128)
    for uy in range(N):
        for ux in range(N):
            acc = 0j
            for ry in range(N):
                for rx in range(N):
                    acc += x[..., ry, rx] * complex(
                        math.cos(2 * math.pi * (uy * ry + ux * rx) / N),
                        s * math.sin(2 * math.pi * (uy * ry + ux * rx) / N))
            out[..., uy, ux] = acc / N
    return out


def crandn(rng, *shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


# ---------------------------------------------------------------- F

@pytest.mark.parametrize("N", [1, 2, 3, 4, 6, 8, 12])
def test_fft_matches_brute_force(N):
    rng = np.random.default_rng(N)
    x = crandn(rng, 2, N, N)
    assert np.allclose(orc.fft2u(x), brute_dft2(x), atol=1e-12, rtol=0)
    assert np.allclose(orc.ifft2u(x), brute_dft2(x, inverse=True), atol=1e-12, rtol=0)


@pytest.mark.parametrize("N", [64, 192])
def test_fft_parseval_and_inverse(N):
    rng = np.random.default_rng(N)
    x = crandn(rng, N, N)
    X = orc.fft2u(x)
    assert abs(np.linalg.norm(X) / np.linalg.norm(x) - 1) < 1e-13
    assert np.allclose(orc.ifft2u(X), x, atol=1e-12)


def test_freq_and_bins():
    assert list(orc.signed_bins(4)) == [0, 1, -2, -1]
    assert list(orc.signed_bins(5)) == [0, 1, 2, -2, -1]
    assert np.allclose(orc.freq(4), [0, 0.25, -0.5, -0.25])


# ---------------------------------------------------------------- propagator

@pytest.mark.parametrize("N", [64, 128, 192, 256])
def test_bandlimit_two_thirds_is_integer_test(N):
    k = np.arange(N)
    k = np.where(k < N // 2, k, k - N)
    ref = 9 * (k[:, None] ** 2 + k[None, :] ** 2) <= N * N
    assert np.array_equal(orc.bandlimit_mask(N, 2.0 / 3.0), ref)
    assert orc.bandlimit_mask(N, 0).all()


def test_propagator_unitary_semigroup_identity():
    N, dx, lam = 64, 0.2, 0.019688
    H1 = orc.propagator(N, dx, lam, 3.0, 0)
    H2 = orc.propagator(N, dx, lam, 5.5, 0)
    H12 = orc.propagator(N, dx, lam, 8.5, 0)
    assert np.allclose(np.abs(H1), 1, atol=1e-14)
    assert np.allclose(H1 * H2, H12, atol=1e-12)
    assert np.allclose(orc.propagator(N, dx, lam, 0.0, 0), 1)
    # the propagation operator F^-1 H F is norm preserving without the band limit
    rng = np.random.default_rng(0)
    x = crandn(rng, N, N)
    y = orc.ifft2u(H1 * orc.fft2u(x))
    assert abs(np.linalg.norm(y) / np.linalg.norm(x) - 1) < 1e-13
    # with the band limit, masked frequencies are removed and others kept
    Hm = orc.propagator(N, dx, lam, 3.0, 2 / 3)
    assert np.allclose(np.abs(Hm), orc.bandlimit_mask(N, 2 / 3))


def test_propagator_gaussian_beam_closed_form():
    """Fresnel propagation of a Gaussian: psi_z = (pi w0^2 / a) exp(-pi r^2 / a),
    a = pi w0^2 + i lambda z, for psi_0 = exp(-r^2 / w0^2) (continuous Fourier
    optics under the exp(-2 pi i q.r) transform convention; pins sign and scale)."""
    N, dx, lam, z, w0 = 256, 0.2, 0.019688, 300.0, 3.0
    r = (np.arange(N) - N // 2) * dx
    r2 = r[:, None] ** 2 + r[None, :] ** 2
    psi0 = np.exp(-r2 / w0 ** 2)
    psiz = orc.ifft2u(orc.propagator(N, dx, lam, z, 0) * orc.fft2u(psi0))
    a = np.pi * w0 ** 2 + 1j * lam * z
    ref = (np.pi * w0 ** 2 / a) * np.exp(-np.pi * r2 / a)
    assert np.max(np.abs(psiz - ref)) < 1e-10
    # the opposite sign convention is far off
    bad = (np.pi * w0 ** 2 / np.conj(a)) * np.exp(-np.pi * r2 / np.conj(a))
    assert np.max(np.abs(psiz - bad)) > 1e-2


def test_tilted_propagator_moves_the_gaussian_beam():
    """With a beam tilt t the Fresnel step also moves the wave by -dz tan(t):
    the closed-form beam of the untilted case, evaluated at r + dz tan(t)."""
    N, dx, lam, z, w0 = 256, 0.2, 0.019688, 300.0, 3.0
    tilt = (0.004, -0.007)                # radians
    r = (np.arange(N) - N // 2) * dx
    ry, rx = np.meshgrid(r, r, indexing="ij")
    psi0 = np.exp(-(ry ** 2 + rx ** 2) / w0 ** 2)
    H = orc.propagator(N, dx, lam, z, 0, tilt=tilt)
    psiz = orc.ifft2u(H * orc.fft2u(psi0))
    a = np.pi * w0 ** 2 + 1j * lam * z
    dy, dxs = z * np.tan(tilt[0]), z * np.tan(tilt[1])
    ref = (np.pi * w0 ** 2 / a) * np.exp(-np.pi * ((ry + dy) ** 2 + (rx + dxs) ** 2) / a)
    assert np.max(np.abs(psiz - ref)) < 1e-10
    # tilt is a phase: unitarity and the semigroup property still hold
    assert np.allclose(np.abs(H), 1)
    assert np.allclose(orc.propagator(N, dx, lam, 100.0, 0, tilt=tilt) * orc.propagator(N, dx, lam, 200.0, 0, tilt=tilt),
                       H, atol=1e-12)


def test_custom_bandlimit_mask():
    N = 64
    d = orc.propagator(N, 0.2, 0.02, 5.0, 2 / 3)
    assert np.array_equal(orc.propagator(N, 0.2, 0.02, 5.0, 0.3, mask=orc.bandlimit_mask(N, 2 / 3)), d)
    assert np.array_equal(orc.propagator(N, 0.2, 0.02, 5.0, 2 / 3, mask=np.ones((N, N), np.uint8)),
                          orc.propagator(N, 0.2, 0.02, 5.0, 0))
    k = orc.signed_bins(N)
    square = (np.abs(k)[:, None] <= N // 3) & (np.abs(k)[None, :] <= N // 3)
    H = orc.propagator(N, 0.2, 0.02, 5.0, 2 / 3, mask=square)
    assert np.array_equal(H != 0, square)


# ---------------------------------------------------------------- shift

def test_shift_integer_is_roll_and_composes():
    rng = np.random.default_rng(1)
    N = 16
    P = crandn(rng, N, N)
    s = orc.ifft2u(orc.fft2u(P) * orc.shift_ramp(N, np.array([3.0, -2.0])))
    assert np.allclose(s, np.roll(P, (3, -2), axis=(0, 1)), atol=1e-12)
    d1, d2 = np.array([0.3, -0.2]), np.array([-0.45, 0.1])
    assert np.allclose(orc.shift_ramp(N, d1) * orc.shift_ramp(N, d2),
                       orc.shift_ramp(N, d1 + d2), atol=1e-14)
    # shifting a constant (vacuum) wave leaves it unchanged
    c = np.full((N, N), 2 - 1j)
    assert np.allclose(orc.ifft2u(orc.fft2u(c) * orc.shift_ramp(N, d1)), c, atol=1e-12)


def test_split_positions():
    n, d = orc.split_positions(np.array([[3.5, 2.49], [-0.5, 7.0]]))
    assert n.tolist() == [[4, 2], [0, 7]]
    assert np.allclose(d, [[-0.5, 0.49], [-0.5, 0.0]])


# ---------------------------------------------------------------- forward

def _geom(N, S, loss="gaussian", eps=0.0, frac=2 / 3, dz=2.0):
    return orc.Geometry(N=N, dx=0.2, wavelength=0.019688, dz=[dz] * (S - 1), bandlimit=frac,
                        loss=loss, eps=eps, sigma=1.0)


@pytest.mark.parametrize("N", [4, 8])
def test_single_slice_is_strong_phase_object_model(N):
    """S = 1: I = |F(P(r - X) O(r))|^2 summed over modes (Sec. 1/3), by brute force."""
    rng = np.random.default_rng(N)
    P = crandn(rng, 2, N, N)
    O = np.exp(1j * rng.random((1, N + 3, N + 3)))
    X = np.array([[1.3, 2.2], [2.0, 0.6]])
    I = orc.forward(P, O, X, [0, 1], _geom(N, 1))
    u = np.fft.fftfreq(N)
    for b, x in enumerate(X):
        n = np.floor(x + 0.5).astype(int)
        d = x - n
        R = np.exp(-2j * np.pi * (u[:, None] * d[0] + u[None, :] * d[1]))
        ref = 0
        for m in range(2):
            psi0 = brute_dft2(brute_dft2(P[m]) * R, inverse=True)
            ref = ref + np.abs(brute_dft2(psi0 * O[0, n[0]:n[0] + N, n[1]:n[1] + N])) ** 2
        assert np.allclose(I[b], ref, atol=1e-11)


def test_zero_gap_slices_multiply():
    """dz = 0 and no band limit: S slices act as their product (one slice)."""
    rng = np.random.default_rng(3)
    N = 8
    P = crandn(rng, 2, N, N)
    O = np.exp(1j * rng.random((3, 12, 12))) * (0.5 + 0.5 * rng.random((3, 12, 12)))
    X = np.array([[1.2, 3.4]])
    I3 = orc.forward(P, O, X, [0], _geom(N, 3, frac=0, dz=0.0))
    I1 = orc.forward(P, np.prod(O, axis=0, keepdims=True), X, [0], _geom(N, 1, frac=0))
    assert np.allclose(I3, I1, atol=1e-12)


def test_vacuum_and_dose():
    rng = np.random.default_rng(4)
    N, S = 16, 4
    P = crandn(rng, 3, N, N)
    X = np.array([[0.7, 2.3], [3.4, 1.1]])
    vac = np.ones((S, 24, 24), dtype=complex)
    I = orc.forward(P, vac, X, [0, 1], _geom(N, S, frac=0, dz=7.0))
    ref = np.sum(np.abs(orc.fft2u(P)) ** 2, axis=0)
    assert np.allclose(I[0], ref) and np.allclose(I[1], ref)
    phase_obj = np.exp(1j * 2 * rng.random((S, 24, 24)))
    I = orc.forward(P, phase_obj, X, [0, 1], _geom(N, S, frac=0, dz=7.0))
    dose = np.sum(np.abs(P) ** 2)
    assert np.allclose(I.sum(axis=(1, 2)), dose, rtol=1e-12)


def test_no_trailing_propagation_reading():
    """Without a band limit a propagation after the last slice would not change I."""
    rng = np.random.default_rng(5)
    N, S = 16, 3
    geom = _geom(N, S, frac=0, dz=4.0)
    P = crandn(rng, 2, N, N)
    O = np.exp(1j * rng.random((S, 20, 20)))
    X = np.array([2.3, 1.6])
    psi, far, I = orc.forward_position(P, O, X, geom)
    H = orc.propagator(N, 0.2, 0.019688, 4.0, 0)
    I_trail = np.sum(np.abs(H * far) ** 2, axis=0)
    assert np.allclose(I, I_trail, atol=1e-12)


def test_window_out_of_bounds_raises():
    P = np.ones((1, 8, 8), complex)
    O = np.ones((1, 10, 10), complex)
    with pytest.raises(IndexError):
        orc.forward(P, O, np.array([[3.0, 0.0]]), [0], _geom(8, 1))
    with pytest.raises(IndexError):
        orc.forward(P, O, np.array([[-0.6, 0.0]]), [0], _geom(8, 1))


# ---------------------------------------------------------------- loss

def _golden():
    rows = []
    with open(os.path.join(HERE, "golden", "noise_models.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                k, *v = line.split()
                rows.append((k, *map(float, v)))
    return rows


@pytest.mark.parametrize("row", _golden())
def test_noise_model_golden_values(row):
    kind, I, Ie, eps, sigma, ell_ref, w_ref = row
    ell, w = orc.loss_and_weight(np.array([I]), np.array([Ie]), kind, eps, sigma)
    assert abs(ell[0] - ell_ref) < 1e-12 and abs(w[0] - w_ref) < 1e-12


@pytest.mark.parametrize("kind,eps", [("amplitude", 0.0), ("anscombe", 0.0), ("poisson", 0.0),
                                      ("poisson", 0.8), ("gaussian", 0.0)])
def test_noise_model_weight_is_twice_the_derivative(kind, eps):
    rng = np.random.default_rng(6)
    I = 0.5 + 10 * rng.random(50)
    Ie = np.floor(10 * rng.random(50))
    h = 1e-6
    lp, _ = orc.loss_and_weight(I + h, Ie, kind, eps, 1.7)
    lm, _ = orc.loss_and_weight(I - h, Ie, kind, eps, 1.7)
    _, w = orc.loss_and_weight(I, Ie, kind, eps, 1.7)
    if kind in ("amplitude", "anscombe") and eps != 0:
        pytest.skip("eps regularises only the weight")
    assert np.allclose(w, (lp - lm) / h, atol=1e-7)   # w = 2 dl/dI


def test_amplitude_zero_intensity_weight_is_zero():
    ell, w = orc.loss_and_weight(np.array([0.0]), np.array([4.0]), "amplitude", 0.0)
    assert w[0] == 0 and ell[0] == 2.0


@pytest.mark.parametrize("kind", orc.LOSS_KINDS)
def test_zero_loss_and_gradient_on_noise_free_data(kind):
    wl = synth.make_small(N=16, M=2, S=3, scan=2, step=4, seed=11, loss=kind)
    geom = _geom(16, 3, loss=kind)
    idx = list(range(wl.J))
    I = orc.forward(wl.probe, wl.obj, wl.positions, idx, geom)
    r = orc.loss_and_grad(wl.probe, wl.obj, wl.positions, I, idx, geom)
    assert abs(r["loss"]) < 1e-9 * I.sum()
    for k in ("g_object", "g_probe", "g_pos"):
        assert np.max(np.abs(r[k])) < 1e-9 * max(1.0, np.max(np.abs(I)))


def test_poisson_weight_at_truth_with_eps():
    I = np.array([0.5, 3.0, 80.0])
    _, w = orc.loss_and_weight(I, I, "poisson", 0.8)
    assert np.allclose(w, 2 * 0.8 / (I + 0.8))


# ---------------------------------------------------------------- adjoint

def _fd_problem(kind, eps, frac=2 / 3, seed=21, tilt=(0.0, 0.0), mask=None, dz=(3.0, 3.0)):
    rng = np.random.default_rng(seed)
    N, M, S = 8, 2, 3
    P = crandn(rng, M, N, N) * 0.7
    O = np.exp(1j * 0.8 * rng.random((S, 14, 14))) * (0.6 + 0.4 * rng.random((S, 14, 14)))
    X = np.array([[2.3, 3.8], [4.1, 1.7], [3.0, 4.35]])
    pats = 1.0 + 4 * rng.random((3, N, N))
    geom = _geom(N, S, loss=kind, eps=eps, frac=frac, dz=3.0)
    geom.dz = list(dz)
    geom.tilt = tilt
    geom.bandlimit_mask = mask
    return P, O, X, pats, geom


FD_CASES = [("gaussian", 0.0, {}), ("poisson", 0.8, {}), ("amplitude", 0.0, {}), ("anscombe", 0.0, {}),
            ("poisson", 0.8, dict(tilt=(0.02, -0.03), dz=(2.0, 5.0),
                                  mask=np.random.default_rng(0).random((8, 8)) < 0.7))]


@pytest.mark.parametrize("kind,eps,extra", FD_CASES)
def test_gradients_match_central_finite_differences(kind, eps, extra):
    P, O, X, pats, geom = _fd_problem(kind, eps, **extra)
    idx = [0, 1, 2]
    r = orc.loss_and_grad(P, O, X, pats, idx, geom)
    L = lambda P_, O_, X_: orc.total_loss(P_, O_, X_, pats, idx, geom)  # noqa: E731
    rng = np.random.default_rng(99)
    checks = []
    for _ in range(6):      # object entries inside windows
        i, y, x = rng.integers(0, 3), rng.integers(2, 12), rng.integers(2, 12)
        for part in (1, 1j):
            h = 1e-6
            Op, Om = O.copy(), O.copy()
            Op[i, y, x] += h * part
            Om[i, y, x] -= h * part
            fd = (L(P, Op, X) - L(P, Om, X)) / (2 * h)
            an = r["g_object"][i, y, x].real if part == 1 else r["g_object"][i, y, x].imag
            checks.append((fd, an))
    for _ in range(4):      # probe entries
        m, y, x = rng.integers(0, 2), rng.integers(0, 8), rng.integers(0, 8)
        for part in (1, 1j):
            h = 1e-6
            Pp, Pm = P.copy(), P.copy()
            Pp[m, y, x] += h * part
            Pm[m, y, x] -= h * part
            fd = (L(Pp, O, X) - L(Pm, O, X)) / (2 * h)
            an = r["g_probe"][m, y, x].real if part == 1 else r["g_probe"][m, y, x].imag
            checks.append((fd, an))
    for b in range(3):      # positions (|d| <= 0.4 keeps n fixed)
        for a in range(2):
            h = 1e-6
            Xp, Xm = X.copy(), X.copy()
            Xp[b, a] += h
            Xm[b, a] -= h
            fd = (L(P, O, Xp) - L(P, O, Xm)) / (2 * h)
            checks.append((fd, r["g_pos"][b, a]))
    fd = np.array([c[0] for c in checks])
    an = np.array([c[1] for c in checks])
    scale = np.max(np.abs(an))
    assert np.max(np.abs(fd - an)) < 1e-5 * scale, np.max(np.abs(fd - an)) / scale


def test_adjoint_dot_products():
    """<A x, y> = <x, A^H y> for the linear blocks of the model."""
    rng = np.random.default_rng(8)
    N = 12
    x, y = crandn(rng, N, N), crandn(rng, N, N)
    ip = lambda a, b: np.vdot(a, b)  # noqa: E731
    # F
    assert abs(ip(orc.fft2u(x), y) - ip(x, orc.ifft2u(y))) < 1e-10
    # propagation with band limit
    H = orc.propagator(N, 0.2, 0.02, 9.0, 2 / 3)
    Px = orc.ifft2u(H * orc.fft2u(x))
    PHy = orc.ifft2u(np.conj(H) * orc.fft2u(y))
    assert abs(ip(Px, y) - ip(x, PHy)) < 1e-10
    # subpixel shift
    R = orc.shift_ramp(N, np.array([0.3, -0.4]))
    Sx = orc.ifft2u(orc.fft2u(x) * R)
    SHy = orc.ifft2u(orc.fft2u(y) * np.conj(R))
    assert abs(ip(Sx, y) - ip(x, SHy)) < 1e-10
    # gather (window cut-out) and scatter-add
    big = crandn(rng, 20, 20)
    G = big[3:3 + N, 5:5 + N]
    sc = np.zeros((20, 20), complex)
    sc[3:3 + N, 5:5 + N] += y
    assert abs(ip(G, y) - ip(big, sc)) < 1e-10


def test_gradient_invariants():
    P, O, X, pats, geom = _fd_problem("poisson", 0.8)
    idx = [0, 1, 2]
    r = orc.loss_and_grad(P, O, X, pats, idx, geom)
    gO, gP = r["g_object"], r["g_probe"]
    # (i) a global phase of a slice or of a mode does not change I
    for i in range(O.shape[0]):
        assert abs(np.real(np.vdot(gO[i], 1j * O[i]))) < 1e-9 * np.abs(gO).sum()
    for m in range(P.shape[0]):
        assert abs(np.real(np.vdot(gP[m], 1j * P[m]))) < 1e-9 * np.abs(gP).sum()
    # (ii) scaling any slice by a equals scaling every probe mode by a
    probe_scale = np.real(np.vdot(gP, P))
    for i in range(O.shape[0]):
        assert abs(np.real(np.vdot(gO[i], O[i])) - probe_scale) < 1e-9 * abs(probe_scale)
    # (iii) a vacuum object gives no position gradient
    r0 = orc.loss_and_grad(P, np.ones_like(O), X, pats, idx, geom)
    assert np.max(np.abs(r0["g_pos"])) < 1e-9 * np.max(np.abs(r0["g_probe"]))
    # (iv) translating positions and object together translates the object gradient
    O2 = np.zeros((O.shape[0], 17, 16), complex)
    O2[:, 3:, 2:] = O
    r2 = orc.loss_and_grad(P, O2, X + np.array([3.0, 2.0]), pats, idx, geom)
    assert abs(r2["loss"] - r["loss"]) < 1e-10 * abs(r["loss"])
    assert np.allclose(r2["g_probe"], gP, atol=1e-10 * np.abs(gP).max())
    assert np.allclose(r2["g_pos"], r["g_pos"], atol=1e-9 * np.abs(r["g_pos"]).max())
    assert np.allclose(r2["g_object"][:, 3:, 2:], gO, atol=1e-10 * np.abs(gO).max())
    assert np.all(r2["g_object"][:, :3, :] == 0) and np.all(r2["g_object"][:, :, :2] == 0)


def test_object_gradient_zero_outside_windows():
    P, O, X, pats, geom = _fd_problem("gaussian", 0.0)
    r = orc.loss_and_grad(P, O, X, pats, [0], geom)
    n = np.floor(X[0] + 0.5).astype(int)
    mask = np.zeros(O.shape[1:], bool)
    mask[n[0]:n[0] + 8, n[1]:n[1] + 8] = True
    assert np.all(r["g_object"][:, ~mask] == 0)
    # per-position accumulation adds up to the group result
    parts = [orc.loss_and_grad(P, O, X, pats, [b], geom) for b in range(3)]
    full = orc.loss_and_grad(P, O, X, pats, [0, 1, 2], geom)
    assert np.allclose(sum(p["g_object"] for p in parts), full["g_object"], atol=1e-12)
    assert np.allclose(sum(p["g_probe"] for p in parts), full["g_probe"], atol=1e-12)


# ---------------------------------------------------------------- optimiser

def test_sgd_step_exact():
    P, O, X, pats, geom = _fd_problem("gaussian", 0.0)
    st = dict(probe=P, object=O, positions=X)
    opt = dict(kind="sgd", lr_object=0.1, lr_probe=0.01, lr_pos=0.5)
    new, loss = orc.reconstruct_step(st, pats, [2, 0], geom, opt)
    r = orc.loss_and_grad(P, O, X, pats, [2, 0], geom)
    assert new["object"] is not O
    assert np.array_equal(new["object"], O - 0.1 * r["g_object"])
    assert np.array_equal(new["probe"], P - 0.01 * r["g_probe"])
    gX = np.zeros_like(X)
    gX[2] = r["g_pos"][0]
    gX[0] = r["g_pos"][1]
    assert np.array_equal(new["positions"], X - 0.5 * gX)
    assert loss == r["loss"]


def test_adam_matches_torch():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(12)
    theta = crandn(rng, 5, 4)
    t_param = torch.nn.Parameter(torch.tensor(theta.copy()))
    topt = torch.optim.Adam([t_param], lr=0.03, betas=(0.8, 0.95), eps=1e-6)
    m = np.zeros(theta.shape + (2,))
    v = np.zeros_like(m)
    th = theta.copy()
    for t in range(1, 5):
        g = crandn(rng, 5, 4)
        t_param.grad = torch.tensor(g)
        topt.step()
        th, m, v = orc.adam_update(th, g, m, v, t, 0.03, 0.8, 0.95, 1e-6)
    assert np.allclose(th, t_param.detach().numpy(), atol=1e-13, rtol=0)
