"""FP64 CPU oracle for gradient-descent mixed-state multislice ptychography.

TEST INFRASTRUCTURE. This module is the slow, plain reference that the GPU path
is checked against. Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import or run it; the product path
(the HIP library and its Python binding) never does, and it shares no code,
tables or constants with that path.

Everything is complex128 / float64 and follows the paper (arXiv 2505.14372):

* Forward model: Sec. 3 ("Algorithm description"), the unnumbered multislice
  recursion  Psi_0,k = P_k(r - X_j),  Psi_i,k = (Psi_{i-1,k} O_{i-1}) * p(dz_{i-1}),
  followed by the far-field intensity I(k) = sum_k |F(Psi_n,k)|^2.
* Noise models and detector-plane gradients: Sec. 3.1 ("Noise models").
* Gradient convention and stochastic descent over groups: Sec. 3.2
  ("Gradient descent solver"); Adam per Kingma & Ba as cited there.

Readings fixed where the paper is silent:

* F is the unitary 2D DFT (numpy ``norm="ortho"``); detector in FFT order.
* Propagator H(u) = B(u) exp(-i pi lambda dz |q|^2), q = fftfreq(N)/dx in 1/A;
  B is a circular band limit k_y^2 + k_x^2 <= (f N / 2)^2 on signed integer
  bins (inclusive), f = 2/3 by default, f <= 0 disables it, or any mask the
  caller gives. A beam tilt t multiplies H by exp(2 pi i dz q.tan(t)).
* S slices have S-1 gaps, hence S-1 propagations and none after the last slice.
* Positions X_j = (row, col) of the window's top-left corner in object pixels;
  n_j = floor(X_j + 0.5) is the integer window offset and d_j = X_j - n_j in
  [-0.5, 0.5) is applied to the probe as a Fourier shift
  R_j(u) = exp(-2 pi i (u_y d_y + u_x d_x)).
* Poisson loss l = I - Ie - Ie (ln(I + eps) - ln(Ie + eps)) (l = I where Ie = 0),
  whose exact derivative is the paper's Poisson detector gradient.
* Complex gradients are dL/dRe + i dL/dIm (= 2 dL/dconj(z)), the PyTorch
  convention; the paper's conj(dL/dz) differs by the positive factor 2.
* Losses are sums over pixels and over the positions of the group.
* Regularizers (Sec. 3.4): formulas fixed below, next to their code.

Parity status: every function below is pinned by tests under ``tests/``
(brute-force DFT, unitarity, closed-form Gaussian beam, strong-phase-object
reduction, zero loss at the truth, central finite differences, dot-product
tests, invariants, torch.optim.Adam).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional, Sequence

import numpy as np

LOSS_KINDS = ("amplitude", "anscombe", "poisson", "gaussian")


@dataclass
class Geometry:
    """Physical parameters of one reconstruction (Sec. 3)."""
    N: int
    dx: float = 0.2                 # pixel size, Angstrom
    wavelength: float = 0.019688    # Angstrom (300 keV electrons)
    dz: Sequence[float] = field(default_factory=tuple)  # S-1 slice gaps, Angstrom
    bandlimit: float = 2.0 / 3.0    # fraction of Nyquist; <= 0 disables
    loss: str = "poisson"
    eps: float = 0.0
    sigma: float = 1.0
    tilt: Sequence[float] = (0.0, 0.0)   # beam tilt (theta_y, theta_x) in radians
    bandlimit_mask: Optional[np.ndarray] = None   # custom band-limit mask [N][N] (FFT order); overrides bandlimit

    def props(self, S):
        return [propagator(self.N, self.dx, self.wavelength, self.dz[i], self.bandlimit, self.tilt,
                           self.bandlimit_mask) for i in range(S - 1)]


# --------------------------------------------------------------------------
# Transforms and grids
# --------------------------------------------------------------------------

def fft2u(a):
    """Unitary 2D DFT over the last two axes, F[x](u) = N^-1 sum_r x(r) e^{-2 pi i u.r/N}."""
    return np.fft.fft2(a, norm="ortho")


def ifft2u(a):
    """Inverse of fft2u (its adjoint, since F is unitary)."""
    return np.fft.ifft2(a, norm="ortho")


def freq(N):
    """Spatial frequencies in cycles per pixel, FFT order (Nyquist is -0.5 for even N)."""
    return np.fft.fftfreq(N)


def signed_bins(N):
    """Signed integer frequency bins k in FFT order (k = freq * N)."""
    k = np.arange(N)
    return np.where(k < (N + 1) // 2, k, k - N)


def bandlimit_mask(N, frac):
    """Circular anti-aliasing band limit applied at each propagation (Sec. 3).

    B(u) = 1 iff k_y^2 + k_x^2 <= (frac * N / 2)^2 on signed integer bins,
    inclusive; the radius is compared with a relative slack of 1e-9 so that
    a bin lying exactly on the boundary is kept whatever the rounding of frac.
    frac <= 0 turns the limit off.
    """
    if frac <= 0:
        return np.ones((N, N), dtype=bool)
    k = signed_bins(N).astype(np.float64)
    k2 = k[:, None] ** 2 + k[None, :] ** 2
    r = frac * N / 2.0
    return k2 <= r * r * (1.0 + 1e-9)


def propagator(N, dx, wavelength, dz, frac, tilt=(0.0, 0.0), mask=None):
    """Fresnel free-space propagator in Fourier space (Sec. 3, p(dz)), with
    the propagator tilt of Sec. 1 and the customizable band limit of Sec. 3.

    H(u) = B(u) exp(-i pi lambda dz (q_y^2 + q_x^2) + 2 pi i dz (q_y tan t_y + q_x tan t_x)),
    q = u / dx in 1/Angstrom. Convolution with p(dz) in real space is
    multiplication by H after the forward DFT; the tilt term moves the wave by
    -dz tan(t) per gap. B is `mask` when given (any shape, FFT order), else
    the circular limit of `frac`.
    """
    q = freq(N) / dx
    q2 = q[:, None] ** 2 + q[None, :] ** 2
    ramp = q[:, None] * np.tan(tilt[0]) + q[None, :] * np.tan(tilt[1])
    H = np.exp(-1j * np.pi * wavelength * dz * q2 + 2j * np.pi * dz * ramp)
    B = bandlimit_mask(N, frac) if mask is None else (np.asarray(mask) != 0)
    return H * B


def split_positions(X):
    """Integer window offsets n = floor(X + 0.5) and subpixel remainders d = X - n."""
    X = np.asarray(X, dtype=np.float64)
    n = np.floor(X + 0.5)
    return n.astype(np.int64), X - n


def shift_ramp(N, d):
    """Fourier ramp R(u) = exp(-2 pi i (u_y d_y + u_x d_x)): F^-1(F(P) R) is P(r - d)."""
    u = freq(N)
    return np.exp(-2j * np.pi * (u[:, None] * d[0] + u[None, :] * d[1]))


# --------------------------------------------------------------------------
# Forward model (Sec. 3)
# --------------------------------------------------------------------------

def check_window(n, N, H, W):
    if n[0] < 0 or n[1] < 0 or n[0] + N > H or n[1] + N > W:
        raise IndexError(f"window at {tuple(n)} of size {N} leaves the {H}x{W} object")


def forward_position(probe, obj, X, geom: Geometry, props=None):
    """Multislice forward model for one probe position, every mode.

    Returns (psi, far, I): psi[i] is the entry wave of slice i for all modes
    (shape [S][M][N][N]), far the detector-plane waves F(phi_{S-1}) per mode,
    I = sum_m |far_m|^2.
    """
    N = geom.N
    S = obj.shape[0]
    n, d = split_positions(X)
    check_window(n, N, obj.shape[1], obj.shape[2])
    if props is None:
        props = geom.props(S)
    R = shift_ramp(N, d)
    psi = [ifft2u(fft2u(probe) * R)]                      # Psi_0 = P(r - X_j)
    for i in range(S):
        patch = obj[i, n[0]:n[0] + N, n[1]:n[1] + N]
        phi = psi[i] * patch                               # transmission
        if i < S - 1:
            psi.append(ifft2u(props[i] * fft2u(phi)))      # Fresnel step
    far = fft2u(phi)                                       # far field
    I = np.sum(np.abs(far) ** 2, axis=0)                   # incoherent mode sum
    return np.stack(psi), far, I


def forward(probe, obj, positions, batch_idx, geom: Geometry):
    """Intensities [B][N][N] for the positions positions[batch_idx]."""
    probe = np.asarray(probe, dtype=np.complex128)
    obj = np.asarray(obj, dtype=np.complex128)
    S = obj.shape[0]
    props = geom.props(S)
    return np.stack([forward_position(probe, obj, positions[j], geom, props)[2]
                     for j in batch_idx])


# --------------------------------------------------------------------------
# Noise models (Sec. 3.1)
# --------------------------------------------------------------------------

def loss_and_weight(I, Ie, kind, eps=0.0, sigma=1.0):
    """Per-pixel loss l(I, Ie) and detector weight w = 2 dl/dI.

    amplitude / anscombe (c = 0 / 3/8): l = 1/2 (sqrt(I+c) - sqrt(Ie+c))^2 and the
        regularised weight w = 1 - sqrt(Ie+c) / (eps + sqrt(I+c)) (w := 0 where
        eps + sqrt(I+c) = 0, a pixel where every mode's far field vanishes);
    poisson: l = I - Ie - Ie (ln(I+eps) - ln(Ie+eps)), l := I where Ie = 0 (the
        limit Ie ln Ie -> 0 of the Stirling form), w = 2 (1 - Ie / (I + eps)); negative
        or NaN counts give a non-finite loss;
    gaussian: l = (I - Ie)^2 / (2 sigma^2), w = 2 (I - Ie) / sigma^2.

    The gradient of the loss with respect to a detector-plane wave Psi_m is
    then w * Psi_m (PyTorch convention), the paper's detector gradients up to
    a positive factor.
    """
    I = np.asarray(I, dtype=np.float64)
    Ie = np.asarray(Ie, dtype=np.float64)
    if kind in ("amplitude", "anscombe"):
        c = 0.0 if kind == "amplitude" else 3.0 / 8.0
        a = np.sqrt(I + c)
        ae = np.sqrt(Ie + c)
        ell = 0.5 * (a - ae) ** 2
        den = eps + a
        with np.errstate(divide="ignore", invalid="ignore"):
            w = np.where(den > 0, 1.0 - ae / np.where(den > 0, den, 1.0), 0.0)
        return ell, w
    if kind == "poisson":
        with np.errstate(divide="ignore", invalid="ignore"):
            ell = np.where(Ie == 0, I,
                           I - Ie - Ie * (np.log(I + eps) - np.log(Ie + eps)))
            w = 2.0 * (1.0 - np.where(Ie == 0, 0.0, Ie / (I + eps)))
        return ell, w
    if kind == "gaussian":
        return (I - Ie) ** 2 / (2.0 * sigma ** 2), 2.0 * (I - Ie) / sigma ** 2
    raise ValueError(kind)


# --------------------------------------------------------------------------
# Exact adjoint (vector-Jacobian product, Sec. 3.2)
# --------------------------------------------------------------------------

def loss_and_grad(probe, obj, positions, patterns, batch_idx, geom: Geometry):
    """Loss of one group and its exact gradients.

    Returns a dict with
      loss       total loss (sum over positions and pixels),
      loss_pos   per-position losses [B],
      I          modelled intensities [B][N][N],
      g_object   dL/dRe O + i dL/dIm O, shape of obj,
      g_probe    same for the probe modes,
      g_pos      dL/dX per batch entry [B][2].
    """
    probe = np.asarray(probe, dtype=np.complex128)
    obj = np.asarray(obj, dtype=np.complex128)
    N = geom.N
    M = probe.shape[0]
    S = obj.shape[0]
    props = geom.props(S)
    probe_hat = fft2u(probe)
    u = freq(N)
    g_obj = np.zeros_like(obj)
    g_probe_hat = np.zeros_like(probe)
    g_pos = np.zeros((len(batch_idx), 2))
    loss_pos = np.zeros(len(batch_idx))
    Is = np.zeros((len(batch_idx), N, N))
    for b, j in enumerate(batch_idx):
        n, d = split_positions(positions[j])
        psi, far, I = forward_position(probe, obj, positions[j], geom, props)
        Is[b] = I
        ell, w = loss_and_weight(I, patterns[j], geom.loss, geom.eps, geom.sigma)
        loss_pos[b] = ell.sum()
        # gradient with respect to the last exit wave phi_{S-1}, every mode
        g = ifft2u(w * far)
        for i in range(S - 1, -1, -1):
            patch = obj[i, n[0]:n[0] + N, n[1]:n[1] + N]
            # phi_i = psi_i * O_i: both factors receive conj(other) * g
            g_obj[i, n[0]:n[0] + N, n[1]:n[1] + N] += np.sum(np.conj(psi[i]) * g, axis=0)
            h = np.conj(patch) * g                          # gradient wrt psi_i
            if i > 0:
                # psi_i = F^-1 H F phi_{i-1}  ->  adjoint F^-1 conj(H) F
                g = ifft2u(np.conj(props[i - 1]) * fft2u(h))
        # psi_0 = F^-1 (P_hat R): gradient wrt the shifted spectrum A = P_hat R
        h_hat = fft2u(h)
        R = shift_ramp(N, d)
        g_probe_hat += h_hat * np.conj(R)
        # dA/dd_a = A * (-2 pi i u_a); dL/dd_a = Re sum conj(grad_A) dA/dd_a
        A = probe_hat * R
        dAy = A * (-2j * np.pi * u[:, None])
        dAx = A * (-2j * np.pi * u[None, :])
        g_pos[b, 0] = np.real(np.sum(np.conj(h_hat) * dAy))
        g_pos[b, 1] = np.real(np.sum(np.conj(h_hat) * dAx))
    g_probe = ifft2u(g_probe_hat)                           # P_hat = F P
    return dict(loss=float(loss_pos.sum()), loss_pos=loss_pos, I=Is,
                g_object=g_obj, g_probe=g_probe, g_pos=g_pos)


def total_loss(probe, obj, positions, patterns, batch_idx, geom: Geometry):
    """Loss only (used by finite-difference pins)."""
    I = forward(probe, obj, positions, batch_idx, geom)
    ell, _ = loss_and_weight(I, np.asarray(patterns)[list(batch_idx)], geom.loss,
                             geom.eps, geom.sigma)
    return float(ell.sum())


# --------------------------------------------------------------------------
# Optimiser step (Sec. 3.2: SGD and Adam on each variable)
# --------------------------------------------------------------------------

def _as_real(a):
    a = np.asarray(a)
    if np.iscomplexobj(a):
        return np.stack([a.real, a.imag], axis=-1)
    return np.asarray(a, dtype=np.float64)


def _from_real(r, like):
    if np.iscomplexobj(like):
        return r[..., 0] + 1j * r[..., 1]
    return r


def sgd_update(theta, grad, lr):
    """theta <- theta - lr * grad."""
    return theta - lr * grad


def adam_update(theta, grad, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """Adam (Kingma & Ba) on the real components of theta, step t >= 1.

    m <- b1 m + (1-b1) g;  v <- b2 v + (1-b2) g^2;
    theta <- theta - (lr / (1-b1^t)) m / (sqrt(v) / sqrt(1-b2^t) + eps)
    (the bias-corrected form with eps added after the v correction).
    m and v are real arrays shaped like the real view of theta.
    Returns (theta, m, v).
    """
    g = _as_real(grad)
    th = _as_real(theta)
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    bc1 = 1.0 - beta1 ** t
    bc2 = 1.0 - beta2 ** t
    th = th - (lr / bc1) * m / (np.sqrt(v) / np.sqrt(bc2) + eps)
    return _from_real(th, theta), m, v


# --------------------------------------------------------------------------
# Conventional engine: ePIE / 3PIE (Sec. 3.3)
# --------------------------------------------------------------------------
#
# Readings of the section (its slice equations are garbled):
# * the detector update is the generalized-amplitude one the section gives,
#   chi_hat = (sqrt(Ie + c) / (eps + sqrt(I + c)) - 1) Psi_hat for every mode,
#   with c = 3/8 for the Anscombe model and 0 otherwise, for every noise
#   model (for amplitude, Poisson and Gaussian likelihoods the per-pixel
#   minimiser along the gradient is this same modulus projection at eps = 0);
#   chi_hat = 0 where eps + sqrt(I + c) = 0;
# * the wave that multiplies conj(.) in the object update is the entry wave
#   psi_i of slice i, and the update of the entry wave is carried to the exit
#   wave of slice i - 1 by the adjoint propagator F^-1 conj(H) F;
# * the normalisers are per position and slice: max over the window of
#   sum_m |psi_i,m|^2 (mixed-state form) for the object, and max over the
#   window of |O_i|^2 for the wave; a zero maximum gives a zero update;
# * the group is evaluated at the current state (all positions in parallel),
#   the object update is summed over positions and modes, the probe update
#   (the entry-wave update of slice 0, shifted back by -delta_j) is averaged
#   over the positions of the group; positions are not refined.

def epie_update(probe, obj, positions, patterns, batch_idx, geom: Geometry):
    """Summed ePIE updates of one group at the current state.

    Returns dict(loss (noise-model loss of the current state), dO (sum over
    positions and modes, shape of obj), dP (sum over positions, shape of
    probe), a, b ([B][S] object and wave normalisers 1 / max)).
    """
    probe = np.asarray(probe, dtype=np.complex128)
    obj = np.asarray(obj, dtype=np.complex128)
    N = geom.N
    S = obj.shape[0]
    props = geom.props(S)
    c = 0.375 if geom.loss == "anscombe" else 0.0
    dO = np.zeros_like(obj)
    dP_hat = np.zeros_like(probe)
    A = np.zeros((len(batch_idx), S))
    Bn = np.zeros((len(batch_idx), S))
    loss = 0.0
    for b, j in enumerate(batch_idx):
        n, d = split_positions(positions[j])
        psi, far, I = forward_position(probe, obj, positions[j], geom, props)
        Ie = np.asarray(patterns[j], dtype=np.float64)
        loss += float(loss_and_weight(I, Ie, geom.loss, geom.eps, geom.sigma)[0].sum())
        den = geom.eps + np.sqrt(I + c)
        factor = np.where(den > 0, np.sqrt(Ie + c) / np.where(den > 0, den, 1.0) - 1.0, 0.0)
        chi = ifft2u(factor * far)                       # update of the last exit wave
        for i in range(S - 1, -1, -1):
            patch = obj[i, n[0]:n[0] + N, n[1]:n[1] + N]
            mp = np.max(np.sum(np.abs(psi[i]) ** 2, axis=0))
            mo = np.max(np.abs(patch) ** 2)
            A[b, i] = 1.0 / mp if mp > 0 else 0.0
            Bn[b, i] = 1.0 / mo if mo > 0 else 0.0
            dO[i, n[0]:n[0] + N, n[1]:n[1] + N] += A[b, i] * np.sum(np.conj(psi[i]) * chi, axis=0)
            dpsi = Bn[b, i] * np.conj(patch) * chi       # update of the entry wave psi_i
            if i > 0:
                chi = ifft2u(np.conj(props[i - 1]) * fft2u(dpsi))
        dP_hat += fft2u(dpsi) * np.conj(shift_ramp(N, d))
    return dict(loss=loss, dO=dO, dP=ifft2u(dP_hat), a=A, b=Bn)


# --------------------------------------------------------------------------
# Conventional engine: LSQML (Sec. 3.3)
# --------------------------------------------------------------------------
#
# Readings of the section:
# * detector update chi_hat as for ePIE above; no normalisers in the chain:
#   the illumination update direction conj(O_i) chi_i is carried to slice
#   i - 1 by F^-1 conj(H) F;
# * object, per slice i: the direction summed over the group and the modes,
#   D_i = sum_j sum_m chi_i,m conj(psi_i,m) (scattered into object
#   coordinates), normalised by the illumination sum A_i, regularised
#   relative to its maximum (dose-independent):
#   dO_hat_i = D_i / (A_i + delta_O max A_i);
# * the step is computed per group (one per slice), the least-squares fit of
#   dO_hat_i psi to chi over the group:
#   alpha_i = Re <dO_hat_i, D_i> / (<|dO_hat_i|^2, W_i> + gamma) with
#   W_i = sum_j sum_m |psi_i,m|^2 (scattered), so the section's
#   illumination-weighted average of the steps over the group is alpha_i
#   itself: O_i += beta_O alpha_i dO_hat_i;
# * probe, at slice 0: the direction is the entry-wave update conj(O_0) chi_0
#   shifted back by -delta_j, summed over the group, per mode: dP_m;
#   dP_hat_m = dP_m / (B + delta_P max B); the illumination of the probe is the
#   object's transparency T_j = prod_i |O_i|^2 over window j (probe view,
#   integer window offset), so alpha_P = Re sum_m <dP_hat_m, dP_m> /
#   (sum_m <|dP_hat_m|^2, sum_j T_j> + gamma) and P += beta_P alpha_P dP_hat;
# * A (object view, per slice) and B (probe view) are illumination sums over
#   a whole iteration: a step uses the previous iteration's sums and adds its
#   own group's W_i and sum_j T_j to the running sums of the current
#   iteration; in the first iteration, which has no previous sums, the
#   running sums (this group included) are used;
# * positions are not refined; the loss reported is the noise model's at the
#   state before the step.

def lsqml_step(state, illum, patterns, batch_idx, geom: Geometry, beta_object=1.0, beta_probe=1.0,
               delta_object=1e-2, delta_probe=1e-2, gamma=0.0):
    """One LSQML group step.

    illum: dict(obj_prev [S][H][W], obj_cur [S][H][W], probe_prev [N][N],
    probe_cur [N][N], first (bool)); the *_cur sums are updated in place.
    Returns (new_state, loss, info) with info = dict(alpha [S], alpha_probe).
    """
    P = np.asarray(state["probe"], dtype=np.complex128)
    O = np.asarray(state["object"], dtype=np.complex128)
    X = state["positions"]
    N = geom.N
    S = O.shape[0]
    props = geom.props(S)
    c = 0.375 if geom.loss == "anscombe" else 0.0
    D = np.zeros_like(O)
    W = np.zeros(O.shape)
    dP_hat_spec = np.zeros_like(P)
    T_sum = np.zeros((N, N))
    loss = 0.0
    for j in batch_idx:
        n, d = split_positions(X[j])
        win = (slice(n[0], n[0] + N), slice(n[1], n[1] + N))
        psi, far, I = forward_position(P, O, X[j], geom, props)
        Ie = np.asarray(patterns[j], dtype=np.float64)
        loss += float(loss_and_weight(I, Ie, geom.loss, geom.eps, geom.sigma)[0].sum())
        den = geom.eps + np.sqrt(I + c)
        factor = np.where(den > 0, np.sqrt(Ie + c) / np.where(den > 0, den, 1.0) - 1.0, 0.0)
        chi = ifft2u(factor * far)                       # update of the last exit wave
        T = np.ones((N, N))
        for i in range(S):
            T = T * np.abs(O[i][win]) ** 2
        T_sum += T
        for i in range(S - 1, -1, -1):
            D[i][win] += np.sum(chi * np.conj(psi[i]), axis=0)
            W[i][win] += np.sum(np.abs(psi[i]) ** 2, axis=0)
            dpsi = chi * np.conj(O[i][win])              # update of the entry wave psi_i
            if i > 0:
                chi = ifft2u(np.conj(props[i - 1]) * fft2u(dpsi))
        dP_hat_spec += fft2u(dpsi) * np.conj(shift_ramp(N, d))
    illum["obj_cur"] += W
    illum["probe_cur"] += T_sum
    A = illum["obj_cur"] if illum["first"] else illum["obj_prev"]
    Bp = illum["probe_cur"] if illum["first"] else illum["probe_prev"]
    new = dict(state)
    dO_hat = D / (A + delta_object * A.max(axis=(1, 2), keepdims=True))
    alpha = np.zeros(S)
    for i in range(S):
        num = np.real(np.vdot(dO_hat[i], D[i]))
        den = np.sum(np.abs(dO_hat[i]) ** 2 * W[i]) + gamma
        alpha[i] = num / den if den > 0 else 0.0
    new["object"] = O + beta_object * alpha[:, None, None] * dO_hat
    dP = ifft2u(dP_hat_spec)
    dP_hat = dP / (Bp + delta_probe * Bp.max())
    num = np.real(np.vdot(dP_hat, dP))
    den = np.sum(np.abs(dP_hat) ** 2 * T_sum[None]) + gamma
    alpha_p = num / den if den > 0 else 0.0
    new["probe"] = P + beta_probe * alpha_p * dP_hat
    return new, loss, dict(alpha=alpha, alpha_probe=alpha_p)


def reconstruct_step(state, patterns, batch_idx, geom: Geometry, opt):
    """One gradient step on one group (Sec. 2.2 engine loop, Sec. 3.2 solver).

    state: dict with probe, object, positions and, for Adam, m_/v_ moments
    per variable and the step counter t (number of steps already taken).
    opt: dict(kind='sgd'|'adam', lr_object, lr_probe, lr_pos, beta1, beta2, eps,
    reg (cost regularizer weights, added to the loss and gradients),
    con (constraints applied to the updated state)).
    Gradients of positions outside the group are zero; the update is applied
    to every element, as a dense optimiser on the whole variable does.
    kind='epie' takes the ePIE step instead: object += lr_object * dO,
    probe += lr_probe * dP / B (beta_object, beta_probe), positions kept,
    no cost regularizers (they belong to the gradient engine), constraints
    applied.
    Returns (new_state, loss).
    """
    if opt["kind"] == "epie":
        e = epie_update(state["probe"], state["object"], state["positions"], patterns, batch_idx, geom)
        new = dict(state)
        new["object"] = np.asarray(state["object"]) + opt["lr_object"] * e["dO"]
        new["probe"] = np.asarray(state["probe"]) + opt["lr_probe"] / len(batch_idx) * e["dP"]
        if opt.get("con"):
            new["object"], new["probe"] = apply_constraints(new["object"], new["probe"], opt["con"])
        return new, e["loss"]
    r = loss_and_grad(state["probe"], state["object"], state["positions"],
                      patterns, batch_idx, geom)
    g_pos = np.zeros_like(np.asarray(state["positions"], dtype=np.float64))
    for b, j in enumerate(batch_idx):
        g_pos[j] += r["g_pos"][b]
    grads = dict(object=r["g_object"], probe=r["g_probe"], positions=g_pos)
    if opt.get("reg"):
        cost, gO, gP = regularization(state["object"], state["probe"], opt["reg"])
        r["loss"] += cost
        grads["object"] = grads["object"] + gO
        grads["probe"] = grads["probe"] + gP
    lrs = dict(object=opt["lr_object"], probe=opt["lr_probe"], positions=opt["lr_pos"])
    new = dict(state)
    if opt["kind"] == "sgd":
        for k in grads:
            new[k] = sgd_update(np.asarray(state[k]), grads[k], lrs[k])
        if opt.get("con"):
            new["object"], new["probe"] = apply_constraints(new["object"], new["probe"], opt["con"])
        return new, r["loss"]
    t = state.get("t", 0) + 1
    for k in grads:
        m = state.get("m_" + k)
        v = state.get("v_" + k)
        if m is None:
            m = np.zeros_like(_as_real(state[k]))
            v = np.zeros_like(m)
        new[k], new["m_" + k], new["v_" + k] = adam_update(
            np.asarray(state[k]), grads[k], m, v, t, lrs[k],
            opt.get("beta1", 0.9), opt.get("beta2", 0.999), opt.get("eps", 1e-8))
    new["t"] = t
    if opt.get("con"):
        new["object"], new["probe"] = apply_constraints(new["object"], new["probe"], opt["con"])
    return new, r["loss"]


# --------------------------------------------------------------------------
# Regularization (Sec. 3.4)
# --------------------------------------------------------------------------
#
# Readings (the section names the regularizers without formulas):
# cost regularizers are added to the detector loss of every group step with
# weights lambda; "vacuum" is O = 1; finite differences are forward
# differences inside the array (no wrap); TV uses the smoothed magnitude
# phi(z) = sqrt(|z|^2 + delta^2) so that it is differentiable at 0.
#   obj_l2:       sum |O - 1|^2                 probe_l2: sum |P|^2
#   obj_l1:       sum |O - 1|  (gradient 0 where O = 1)
#   obj_tikhonov: sum over slices of |D_y O|^2 + |D_x O|^2 (in-plane)
#   obj_tv:       sum over slices of phi(D_y O) + phi(D_x O)
#   layers_tikhonov: sum |O_{i+1} - O_i|^2      layers_tv: sum phi(O_{i+1} - O_i)
#   obj_phase_l1: sum |arg O|, arg in (-pi, pi] (gradient 0 where arg O = 0)
#   obj_spectrum_l1: sum over slices and over every frequency but the zero
#                 one of |F2(O_i)(k)|, F2 the unitary 2D DFT of the slice: an
#                 L1 norm on the object's spectral amplitudes, which favours a
#                 sparse (periodic) spectrum; the zero frequency is the mean
#                 transmission and is left free (penalising it would pull the
#                 vacuum level towards 0)
#   probe_phase_tikhonov / probe_phase_tv: the phase plate of mode m is the
#                 phase of its spectrum P^_m = F2(P_m), taken centred (zero
#                 frequency in the middle, so that neighbouring entries are
#                 neighbouring frequencies); for each pair of neighbours
#                 (a, b) along either axis, z = a conj(b) = |z| e^{i t} with t
#                 the phase step in (-pi, pi] (no unwrapping needed), and the
#                 cost is |z|^2 t^2 (Tikhonov) or |z|^2 sqrt(t^2 + delta^2)
#                 (TV): the squared or absolute phase step weighted by the
#                 intensities of the two frequencies, so that the phase where
#                 the aperture is dark costs nothing and the gradient, with
#                 respect to z 2 z (t^2 + i t) or z (2 sqrt(t^2 + delta^2) +
#                 i t / sqrt(t^2 + delta^2)), vanishes continuously as z -> 0
#                 (with weights |z| it would keep a magnitude of order 1 and a
#                 direction set by rounding at a dark frequency next to a lit
#                 one: the aperture edge)
# Constraint regularizers are applied to the state after each group step:
#   amplitude range: O <- O * clip(|O|, a_min, a_max) / |O|
#   probe support:   P <- F^-1(mask * F(P)) with a reciprocal-space mask,
#                    then P <- mask_r * P with a real-space mask
#   layer blur:      O_i <- sum_j g(i - j) O_j / sum_j g(i - j), g Gaussian in
#                    depth (sigma in slices), truncated at 3 sigma, real space
#                    (no periodic wrap between the top and bottom slices).

REG_KEYS = ("obj_l2", "probe_l2", "obj_l1", "obj_tikhonov", "obj_tv", "layers_tikhonov", "layers_tv",
            "obj_phase_l1", "obj_spectrum_l1", "probe_phase_tikhonov", "probe_phase_tv")
PROBE_REG_KEYS = ("probe_l2", "probe_phase_tikhonov", "probe_phase_tv")


def _phi(z, delta):
    return np.sqrt(np.abs(z) ** 2 + delta ** 2)


def regularization(obj, probe, reg):
    """Cost of the enabled cost regularizers and its gradients (dR/dRe + i dR/dIm).

    reg: dict of weights (keys REG_KEYS, missing = 0) and `tv_delta`.
    Returns (cost, g_object, g_probe).
    """
    O = np.asarray(obj, dtype=np.complex128)
    P = np.asarray(probe, dtype=np.complex128)
    d = reg.get("tv_delta", 1e-3)
    cost = 0.0
    gO = np.zeros_like(O)
    gP = np.zeros_like(P)
    w = reg.get("obj_l2", 0.0)
    if w:
        cost += w * np.sum(np.abs(O - 1) ** 2)
        gO += w * 2 * (O - 1)
    w = reg.get("probe_l2", 0.0)
    if w:
        cost += w * np.sum(np.abs(P) ** 2)
        gP += w * 2 * P
    w = reg.get("obj_l1", 0.0)
    if w:
        a = np.abs(O - 1)
        cost += w * np.sum(a)
        gO += w * np.where(a > 0, (O - 1) / np.where(a > 0, a, 1), 0)
    for key, axis in (("obj_tikhonov", None), ("layers_tikhonov", 0)):
        w = reg.get(key, 0.0)
        if not w:
            continue
        for ax in ((1, 2) if axis is None else (0,)):
            D = np.diff(O, axis=ax)                       # O[k+1] - O[k]
            cost += w * np.sum(np.abs(D) ** 2)
            g = np.zeros_like(O)
            lo = [slice(None)] * 3
            hi = [slice(None)] * 3
            lo[ax] = slice(0, -1)
            hi[ax] = slice(1, None)
            g[tuple(hi)] += 2 * D
            g[tuple(lo)] -= 2 * D
            gO += w * g
    for key, axis in (("obj_tv", None), ("layers_tv", 0)):
        w = reg.get(key, 0.0)
        if not w:
            continue
        for ax in ((1, 2) if axis is None else (0,)):
            D = np.diff(O, axis=ax)
            cost += w * np.sum(_phi(D, d))
            gd = D / _phi(D, d)
            g = np.zeros_like(O)
            lo = [slice(None)] * 3
            hi = [slice(None)] * 3
            lo[ax] = slice(0, -1)
            hi[ax] = slice(1, None)
            g[tuple(hi)] += gd
            g[tuple(lo)] -= gd
            gO += w * g
    w = reg.get("obj_phase_l1", 0.0)
    if w:
        ph = np.angle(O)
        a2 = np.abs(O) ** 2
        cost += w * np.sum(np.abs(ph))
        # d arg(O) / d(Re, Im) combined as dRe + i dIm is i O / |O|^2
        gO += w * np.where(a2 > 0, np.sign(ph) * 1j * O / np.where(a2 > 0, a2, 1), 0)
    w = reg.get("obj_spectrum_l1", 0.0)
    if w:
        F = fft2u(O)
        a = np.abs(F)
        keep = a > 0
        keep[:, 0, 0] = False
        cost += w * np.sum(a[keep])
        gO += w * ifft2u(np.where(keep, F / np.where(keep, a, 1), 0))
    for key in ("probe_phase_tikhonov", "probe_phase_tv"):
        w = reg.get(key, 0.0)
        if not w:
            continue
        C = np.fft.fftshift(fft2u(P), axes=(-2, -1))
        gC = np.zeros_like(C)
        for ax in (-2, -1):
            n = C.shape[ax]
            hi = [slice(None)] * C.ndim
            lo = [slice(None)] * C.ndim
            hi[ax] = slice(1, n)
            lo[ax] = slice(0, n - 1)
            a, b = C[tuple(hi)], C[tuple(lo)]
            z = a * np.conj(b)
            r2, t = np.abs(z) ** 2, np.angle(z)
            # cost f(|z|) h(t) with f = |z|^2: gradient with respect to z (dRe + i dIm)
            # e^{it} (f'(|z|) h + i f(|z|) h' / |z|) = z (2 h + i h')
            if key == "probe_phase_tikhonov":
                cost += w * np.sum(r2 * t * t)
                G = z * (2 * t * t + 2j * t)
            else:
                q = np.sqrt(t * t + d * d)
                cost += w * np.sum(r2 * q)
                G = z * (2 * q + 1j * t / q)
            gC[tuple(hi)] += w * G * b                         # z = a conj(b)
            gC[tuple(lo)] += w * np.conj(G) * a
        gP += ifft2u(np.fft.ifftshift(gC, axes=(-2, -1)))
    return float(cost), gO, gP


def gaussian_taps(sigma):
    """Offsets t = -r..r, r = ceil(3 sigma), and the normalised weights
    exp(-t^2 / (2 sigma^2)) / sum."""
    r = int(np.ceil(3 * sigma))
    t = np.arange(-r, r + 1)
    w = np.exp(-0.5 * (t / sigma) ** 2)
    return t, w / w.sum()


def lowpass_object(obj, sigma):
    """Object low pass (Sec. 3.4): every slice convolved in the plane with a
    sampled Gaussian (taps above), separably along x then y, with periodic
    boundaries, as a filter applied in reciprocal space would have."""
    t, w = gaussian_taps(sigma)
    out = np.asarray(obj, dtype=np.complex128)
    for axis in (2, 1):
        acc = np.zeros_like(out)
        for tk, wk in zip(t, w):
            acc += wk * np.roll(out, -tk, axis=axis)       # out[.., x + tk] (periodic)
        out = acc
    return out


def deramp_object(obj):
    """Object phase deramp (Sec. 3.4), per slice: the affine phase
    theta_0 + theta_y y + theta_x x is removed, with theta_x the angle of
    sum O(y, x+1) conj(O(y, x)) over horizontally adjacent pairs, theta_y
    likewise for vertical pairs, and theta_0 the angle of the sum of the
    de-ramped slice (amplitude-weighted estimates of the mean phase gradient
    and the mean phase)."""
    O = np.asarray(obj, dtype=np.complex128)
    out = np.empty_like(O)
    H, W = O.shape[1:]
    y = np.arange(H)[:, None]
    x = np.arange(W)[None, :]
    for i, Oi in enumerate(O):
        tx = np.angle(np.sum(Oi[:, 1:] * np.conj(Oi[:, :-1])))
        ty = np.angle(np.sum(Oi[1:, :] * np.conj(Oi[:-1, :])))
        D = Oi * np.exp(-1j * (ty * y + tx * x))
        out[i] = D * np.exp(-1j * np.angle(np.sum(D)))
    return out


def apply_constraints(obj, probe, con):
    """Constraint regularizers after a step (Sec. 3.4), in this order:
    object amplitude range (amp_min, amp_max), Gaussian depth blur
    (layer_sigma, slices), in-plane Gaussian low pass (obj_lowpass_sigma,
    pixels), phase deramp (phase_deramp), probe support (probe_support,
    reciprocal-space mask [N][N] in FFT order, then probe_support_real, a
    real-space mask [N][N])."""
    O = np.array(obj, dtype=np.complex128)
    P = np.array(probe, dtype=np.complex128)
    if "amp_min" in con or "amp_max" in con:
        a = np.abs(O)
        c = np.clip(a, con.get("amp_min", 0.0), con.get("amp_max", np.inf))
        O = np.where(a > 0, O * (c / np.where(a > 0, a, 1)), c)
    s = con.get("layer_sigma", 0.0)
    if s and O.shape[0] > 1:
        S = O.shape[0]
        r = int(np.ceil(3 * s))
        out = np.zeros_like(O)
        for i in range(S):
            num = 0
            den = 0.0
            for j in range(max(0, i - r), min(S, i + r + 1)):
                g = np.exp(-0.5 * ((i - j) / s) ** 2)
                num = num + g * O[j]
                den += g
            out[i] = num / den
        O = out
    s = con.get("obj_lowpass_sigma", 0.0)
    if s:
        O = lowpass_object(O, s)
    if con.get("phase_deramp"):
        O = deramp_object(O)
    if con.get("probe_support") is not None:
        P = ifft2u(fft2u(P) * (np.asarray(con["probe_support"]) != 0))
    if con.get("probe_support_real") is not None:
        P = P * (np.asarray(con["probe_support_real"]) != 0)
    return O, P
