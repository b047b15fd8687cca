"""Pins of the oracle's regularizers (Sec. 3.4): central finite differences of
each cost against its gradient, closed forms on special objects, and the
constraints' defining properties."""
import numpy as np
import pytest

import oracle as orc


def crandn(rng, *shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


@pytest.mark.parametrize("key", orc.REG_KEYS)
def test_regularizer_gradient_matches_finite_differences(key):
    rng = np.random.default_rng(hash(key) % 1000)
    O = 1 + 0.3 * crandn(rng, 3, 6, 7)
    P = crandn(rng, 2, 5, 5)
    reg = {key: 0.7, "tv_delta": 0.05}
    _, gO, gP = orc.regularization(O, P, reg)
    h = 1e-6
    for _ in range(12):
        if key in orc.PROBE_REG_KEYS:
            idx = (rng.integers(2), rng.integers(5), rng.integers(5))
            base, g = P, gP
        else:
            idx = (rng.integers(3), rng.integers(6), rng.integers(7))
            base, g = O, gO
        for part in (1, 1j):
            a, b = base.copy(), base.copy()
            a[idx] += h * part
            b[idx] -= h * part
            if key in orc.PROBE_REG_KEYS:
                fd = (orc.regularization(O, a, reg)[0] - orc.regularization(O, b, reg)[0]) / (2 * h)
            else:
                fd = (orc.regularization(a, P, reg)[0] - orc.regularization(b, P, reg)[0]) / (2 * h)
            an = g[idx].real if part == 1 else g[idx].imag
            assert abs(fd - an) < 1e-6 * max(1.0, abs(an)), (key, idx, fd, an)


def test_vacuum_and_closed_forms():
    S, H, W = 3, 8, 9
    vac = np.ones((S, H, W), complex)
    P = np.zeros((1, 4, 4), complex)
    for key in orc.REG_KEYS:
        if key in ("obj_tv", "layers_tv"):
            continue
        c, gO, gP = orc.regularization(vac, P, {key: 1.0})
        assert c == 0 and np.all(gO == 0) and np.all(gP == 0)
    # smoothed TV of a constant object: delta per difference
    d = 0.01
    c, gO, _ = orc.regularization(vac, P, {"obj_tv": 1.0, "tv_delta": d})
    assert abs(c - d * S * ((H - 1) * W + H * (W - 1))) < 1e-12 and np.all(gO == 0)
    c, _, _ = orc.regularization(vac, P, {"layers_tv": 1.0, "tv_delta": d})
    assert abs(c - d * (S - 1) * H * W) < 1e-12
    # Tikhonov of a phase ramp along y: |e^{ia} - 1|^2 = 2 - 2 cos a per difference
    a = 0.3
    y = np.arange(H)[None, :, None]
    ramp = np.exp(1j * a * y) * np.ones((S, H, W))
    c, _, _ = orc.regularization(ramp, P, {"obj_tikhonov": 1.0})
    assert abs(c - S * (H - 1) * W * (2 - 2 * np.cos(a))) < 1e-10
    # layers Tikhonov of a depth ramp
    z = np.arange(S)[:, None, None]
    c, _, _ = orc.regularization(np.exp(1j * a * z) * np.ones((S, H, W)), P, {"layers_tikhonov": 1.0})
    assert abs(c - (S - 1) * H * W * (2 - 2 * np.cos(a))) < 1e-10
    # L2 of the probe is its power
    P = crandn(np.random.default_rng(1), 2, 4, 4)
    assert abs(orc.regularization(vac, P, {"probe_l2": 1.0})[0] - np.sum(np.abs(P) ** 2)) < 1e-12


def test_phase_and_spectrum_l1_closed_forms():
    """Object-phase L1 is the summed |phase| whatever the amplitude; the
    spectral L1 of 1 + c * (one Fourier mode) is |c| sqrt(H W) per slice (the
    unitary DFT puts sqrt(H W) c on that frequency and the free zero frequency
    costs nothing), and a conjugate pair of modes costs twice that."""
    rng = np.random.default_rng(11)
    S, H, W = 2, 6, 10
    ph = rng.uniform(-3.0, 3.0, (S, H, W))
    amp = 0.3 + 2 * rng.random((S, H, W))
    P = np.zeros((1, 4, 4), complex)
    c, gO, _ = orc.regularization(amp * np.exp(1j * ph), P, {"obj_phase_l1": 1.0})
    assert abs(c - np.sum(np.abs(ph))) < 1e-10
    # the gradient is tangential (changes the phase only): Re(conj(g) O) = 0
    assert np.max(np.abs(np.real(np.conj(gO) * amp * np.exp(1j * ph)))) < 1e-12
    y, x = np.mgrid[:H, :W]
    mode = np.exp(2j * np.pi * (2 * y / H + 3 * x / W))
    cc = 0.2 - 0.7j
    O = 1 + cc * np.stack([mode, mode])
    c, _, _ = orc.regularization(O, P, {"obj_spectrum_l1": 1.0})
    assert abs(c - S * abs(cc) * np.sqrt(H * W)) < 1e-10
    O = 3.0 + cc * np.stack([mode + np.conj(mode)] * S)
    c, _, _ = orc.regularization(O, P, {"obj_spectrum_l1": 1.0})
    assert abs(c - 2 * S * abs(cc) * np.sqrt(H * W)) < 1e-10


def test_probe_phase_plate_closed_forms():
    """Phase-plate Tikhonov / TV of a probe whose centred spectrum is
    A exp(i alpha k_y): every step along k_y has phase alpha and weight
    |z|^2 = A^4, every step along k_x phase 0; a global phase leaves it
    unchanged; a uniform phase plate costs nothing (Tikhonov) or A^4 delta per
    step (TV); at a dark frequency next to a lit one the gradient vanishes."""
    N, A, al, d = 7, 1.3, 0.4, 0.05
    k = np.arange(N)[:, None] * np.ones((1, N))
    C = A * np.exp(1j * al * k)
    P = orc.ifft2u(np.fft.ifftshift(C))[None]
    vac = np.ones((1, 8, 8), complex)
    A4 = A ** 4
    c, _, _ = orc.regularization(vac, P, {"probe_phase_tikhonov": 1.0})
    assert abs(c - N * (N - 1) * A4 * al * al) < 1e-10
    c, _, _ = orc.regularization(vac, P, {"probe_phase_tv": 1.0, "tv_delta": d})
    assert abs(c - N * (N - 1) * A4 * (np.sqrt(al * al + d * d) + d)) < 1e-10
    c2, _, _ = orc.regularization(vac, P * np.exp(0.9j), {"probe_phase_tikhonov": 1.0})
    assert abs(c2 - N * (N - 1) * A4 * al * al) < 1e-10
    flat = orc.ifft2u(np.fft.ifftshift(A * np.exp(0.7j) * np.ones((N, N))))[None]
    c, g, gP = orc.regularization(vac, flat, {"probe_phase_tikhonov": 1.0})
    assert abs(c) < 1e-20 and np.max(np.abs(gP)) < 1e-12
    # an aperture: lit frequencies next to exactly dark ones; the gradient is
    # the same whichever tiny values the dark frequencies hold (continuity at z = 0)
    lit = (k - 3) ** 2 + (k.T - 3) ** 2 <= 4
    rng = np.random.default_rng(3)
    spec = np.where(lit, A * np.exp(1j * rng.uniform(-1, 1, (N, N))), 0)
    noise = 1e-13 * (rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N)))
    g0 = orc.regularization(vac, orc.ifft2u(np.fft.ifftshift(spec))[None], {"probe_phase_tikhonov": 1.0})[2]
    g1 = orc.regularization(vac, orc.ifft2u(np.fft.ifftshift(spec + noise * ~lit))[None],
                            {"probe_phase_tikhonov": 1.0})[2]
    assert np.max(np.abs(g1 - g0)) < 1e-9 * np.max(np.abs(g0))


def test_constraints():
    rng = np.random.default_rng(2)
    O = (0.2 + 2 * rng.random((4, 5, 6))) * np.exp(1j * rng.random((4, 5, 6)))
    P = crandn(rng, 2, 8, 8)
    O2, P2 = orc.apply_constraints(O, P, {"amp_min": 0.5, "amp_max": 1.5})
    assert np.all(np.abs(O2) >= 0.5 - 1e-12) and np.all(np.abs(O2) <= 1.5 + 1e-12)
    assert np.allclose(np.angle(O2), np.angle(O))
    inside = (np.abs(O) >= 0.5) & (np.abs(O) <= 1.5)
    assert np.array_equal(O2[inside], O[inside]) and np.array_equal(P2, P)
    # probe support: all-ones mask is the identity, a mask zeroes the spectrum outside
    _, P3 = orc.apply_constraints(O, P, {"probe_support": np.ones((8, 8))})
    assert np.allclose(P3, P)
    m = np.zeros((8, 8))
    m[:3, :3] = 1
    _, P4 = orc.apply_constraints(O, P, {"probe_support": m})
    assert np.allclose(orc.fft2u(P4) * (1 - m), 0) and np.allclose(orc.fft2u(P4) * m, orc.fft2u(P) * m)
    # real-space probe support: zero outside the mask, unchanged inside, after the reciprocal one
    mr = np.zeros((8, 8))
    mr[2:6, 1:7] = 1
    _, P5 = orc.apply_constraints(O, P, {"probe_support_real": mr})
    assert np.array_equal(P5 * (1 - mr), 0 * P5) and np.array_equal(P5 * mr, P * mr)
    _, P6 = orc.apply_constraints(O, P, {"probe_support": m, "probe_support_real": mr})
    assert np.allclose(P6, P4 * mr)
    # layer blur: identical slices unchanged; one bright slice spreads as normalised Gaussian weights
    same = np.repeat(O[:1], 4, axis=0)
    assert np.allclose(orc.apply_constraints(same, P, {"layer_sigma": 1.3})[0], same)
    spike = np.zeros((5, 1, 1), complex)
    spike[2] = 1
    out = orc.apply_constraints(spike, P, {"layer_sigma": 1.0})[0][:, 0, 0]
    g = np.exp(-0.5 * np.arange(-4, 5) ** 2)
    for i in range(5):
        js = range(max(0, i - 3), min(5, i + 4))
        assert abs(out[i] - (np.exp(-0.5 * (i - 2) ** 2) if abs(i - 2) <= 3 else 0)
                   / sum(np.exp(-0.5 * (i - j) ** 2) for j in js)) < 1e-12
    assert g.sum() > 0


def test_reconstruct_step_adds_regularizer_gradient():
    rng = np.random.default_rng(3)
    N = 8
    P = crandn(rng, 1, N, N) * 0.5
    O = np.exp(1j * rng.random((2, 12, 12)))
    X = np.array([[1.2, 2.3], [3.1, 0.8]])
    pats = 1 + 3 * rng.random((2, N, N))
    geom = orc.Geometry(N=N, dz=[2.0], loss="gaussian")
    reg = {"obj_l2": 0.3, "obj_tikhonov": 0.2, "layers_tikhonov": 0.5, "probe_l2": 0.1}
    opt = dict(kind="sgd", lr_object=1e-3, lr_probe=1e-4, lr_pos=0.0, reg=reg)
    new, loss = orc.reconstruct_step(dict(probe=P, object=O, positions=X), pats, [0, 1], geom, opt)
    r = orc.loss_and_grad(P, O, X, pats, [0, 1], geom)
    c, gO, gP = orc.regularization(O, P, reg)
    assert abs(loss - (r["loss"] + c)) < 1e-12
    assert np.allclose(new["object"], O - 1e-3 * (r["g_object"] + gO))
    assert np.allclose(new["probe"], P - 1e-4 * (r["g_probe"] + gP))


def test_object_lowpass_matches_scipy_and_fourier_modes():
    """In-plane low pass: agrees with scipy.ndimage's periodic Gaussian filter
    (the library routine for a sampled, normalised, truncated Gaussian), keeps
    constants and the slice sums, and scales a Fourier mode by the closed-form
    response sum_t w_t cos(2 pi k t / W)."""
    from scipy import ndimage
    rng = np.random.default_rng(5)
    O = crandn(rng, 2, 11, 13)
    for sigma in (0.7, 1.0, 2.3):
        r = int(np.ceil(3 * sigma))
        out = orc.lowpass_object(O, sigma)

        def filt(a):
            a = ndimage.gaussian_filter1d(a, sigma, axis=2, mode="wrap", truncate=r / sigma)
            return ndimage.gaussian_filter1d(a, sigma, axis=1, mode="wrap", truncate=r / sigma)
        ref = filt(O.real) + 1j * filt(O.imag)
        assert np.max(np.abs(out - ref)) < 1e-12
        assert np.allclose(out.sum(axis=(1, 2)), O.sum(axis=(1, 2)), atol=1e-12)
        assert np.allclose(orc.lowpass_object(np.full((1, 5, 7), 2 - 1j), sigma), 2 - 1j)
        H, W, ky, kx = 11, 13, 3, 5
        y, x = np.mgrid[:H, :W]
        mode = np.exp(2j * np.pi * (ky * y / H + kx * x / W))[None]
        t = np.arange(-r, r + 1)
        w = np.exp(-0.5 * (t / sigma) ** 2)
        w /= w.sum()
        lam = np.sum(w * np.cos(2 * np.pi * kx * t / W)) * np.sum(w * np.cos(2 * np.pi * ky * t / H))
        assert np.max(np.abs(orc.lowpass_object(mode, sigma) - lam * mode)) < 1e-12


def test_phase_deramp():
    """Phase deramp: a pure affine phase is removed exactly (sign and axes),
    the result is invariant to any added affine phase, deramping twice
    changes nothing, and amplitudes are untouched."""
    rng = np.random.default_rng(6)
    S, H, W = 3, 9, 14
    y, x = np.mgrid[:H, :W]
    amp = 0.5 + rng.random((S, H, W))
    c = rng.uniform(-1.0, 1.0, (S, 3))
    ramp = np.exp(1j * (c[:, 0, None, None] + c[:, 1, None, None] * y + c[:, 2, None, None] * x))
    pure = orc.deramp_object(1.7 * ramp)
    assert np.max(np.abs(pure - 1.7)) < 1e-12
    O = amp * np.exp(1j * 0.4 * rng.standard_normal((S, H, W)))
    d = orc.deramp_object(O)
    assert np.max(np.abs(orc.deramp_object(O * ramp) - d)) < 1e-10
    assert np.max(np.abs(orc.deramp_object(d) - d)) < 1e-10
    assert np.allclose(np.abs(d), amp)
    # after deramping, the horizontal and vertical pair sums and the slice sum are real and positive
    for di in d:
        for z in (np.sum(di[:, 1:] * np.conj(di[:, :-1])), np.sum(di[1:] * np.conj(di[:-1])), np.sum(di)):
            assert z.real > 0 and abs(z.imag) < 1e-9 * abs(z)


def test_constraint_order():
    """Constraints run as amplitude range, depth blur, low pass, deramp on the
    object; the probe support acts on the probe alone."""
    rng = np.random.default_rng(7)
    O = (0.2 + 2 * rng.random((3, 8, 9))) * np.exp(1j * rng.random((3, 8, 9)))
    P = crandn(rng, 1, 8, 8)
    con = {"amp_min": 0.5, "amp_max": 1.5, "layer_sigma": 0.8, "obj_lowpass_sigma": 0.9, "phase_deramp": 1}
    O2, P2 = orc.apply_constraints(O, P, con)
    a = np.abs(O)
    step = O * np.clip(a, 0.5, 1.5) / a
    step = orc.apply_constraints(step, P, {"layer_sigma": 0.8})[0]
    step = orc.deramp_object(orc.lowpass_object(step, 0.9))
    assert np.max(np.abs(O2 - step)) < 1e-12 and np.array_equal(P2, P)
