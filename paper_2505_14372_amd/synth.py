"""Seeded synthetic inputs shaped like the paper's workloads.

This module only draws inputs: probe modes, sliced objects, scan positions and
Poisson-count diffraction patterns. It contains none of the multislice model,
loss or adjoint arithmetic, and it is the one module that both the GPU path
and the CPU checker take their inputs from.

Recipe (the paper's benchmark datasets are not available; these stand in for
them with the same sizes and value structure; the benchmark datasets are
described in the Methods section):

* probe: a circular Fourier aperture of radius N/4 bins with a quadratic
  (defocus) phase of ``defocus_edge`` rad at its edge, transformed to real
  space; mode m >= 1 is the first mode shifted by half a pixel along the
  direction 2 pi m / M, the modes are Gram-Schmidt orthogonalised in order and
  scaled so that ||P_m||^2 = w_m * dose;
* object: per slice, uniform noise smoothed by a periodic Gaussian
  (sigma = 2 px), min-max scaled to a phase in [0, phi_max], unit amplitude;
* scan: a raster with origin floor(step/2), pitch ``step`` and optional
  uniform jitter in (-jitter, jitter), positions = window top-left corners;
* patterns: Poisson counts around a bright-field disk (radius N/4 bins) that
  holds ``bf_fraction`` of the dose, with a weak dark field outside it. They
  have the statistics of measured data (many zero counts at high angle) but
  are not simulated from the object, so a loss evaluated on them is far from
  zero; tests that need consistent data simulate it with the CPU checker.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import numpy as np

C64 = np.complex64


def mode_weights(M: int, config_weights: Optional[Sequence[float]] = None):
    if config_weights is not None:
        w = np.asarray(config_weights, dtype=np.float64)
        return w / w.sum()
    if M == 1:
        return np.ones(1)
    rest = 0.6 ** np.arange(1, M)
    return np.concatenate([[0.6], 0.4 * rest / rest.sum()])


def make_probe(N: int, M: int, dose: float, weights=None, defocus_edge: float = 0.5):
    """Mixed-state probe [M][N][N] complex128."""
    k = np.fft.fftfreq(N) * N
    ky, kx = np.meshgrid(k, k, indexing="ij")
    kr2 = ky ** 2 + kx ** 2
    R = N / 4.0
    aperture = (kr2 <= R * R).astype(np.float64)
    chi = defocus_edge * kr2 / (R * R)
    spec = aperture * np.exp(-1j * chi)
    modes = []
    for m in range(M):
        if m == 0:
            s = spec
        else:
            th = 2 * np.pi * m / M
            dy, dx = 0.5 * np.sin(th), 0.5 * np.cos(th)
            s = spec * np.exp(-2j * np.pi * (ky * dy + kx * dx) / N)
        modes.append(np.fft.ifft2(s))
    # Gram-Schmidt in order
    ortho = []
    for p in modes:
        q = p.copy()
        for o in ortho:
            q = q - np.vdot(o, q) / np.vdot(o, o) * o
        ortho.append(q)
    w = mode_weights(M, weights)
    out = np.stack([o / np.sqrt(np.vdot(o, o).real) * np.sqrt(wm * dose)
                    for o, wm in zip(ortho, w)])
    return out


def make_object(S: int, H: int, W: int, phi_max: float, seed: int, sigma_px: float = 2.0):
    """Sliced phase object [S][H][W] complex128 with unit amplitude."""
    rng = np.random.default_rng(seed)
    fy = np.fft.fftfreq(H)[:, None]
    fx = np.fft.fftfreq(W)[None, :]
    g = np.exp(-2 * (np.pi * sigma_px) ** 2 * (fy ** 2 + fx ** 2))
    out = np.empty((S, H, W), dtype=np.complex128)
    for i in range(S):
        noise = rng.random((H, W))
        sm = np.real(np.fft.ifft2(np.fft.fft2(noise) * g))
        sm = (sm - sm.min()) / max(sm.max() - sm.min(), 1e-300)
        out[i] = np.exp(1j * phi_max * sm)
    return out


def make_scan(n_scan: int, step: int, jitter: float, seed: int):
    """Raster scan positions [n_scan^2][2] (row, col) of window top-left corners."""
    rng = np.random.default_rng(seed + 7919)
    iy, ix = np.meshgrid(np.arange(n_scan), np.arange(n_scan), indexing="ij")
    pos = np.stack([iy.ravel(), ix.ravel()], axis=1).astype(np.float64) * step + step // 2
    if jitter > 0:
        pos += rng.uniform(-jitter, jitter, size=pos.shape)
    return pos


def make_patterns(N: int, J: int, dose: float, seed: int, bf_fraction: float = 0.95,
                  pool: int = 0):
    """Poisson-count patterns [J][N][N] float32 in FFT order (DC at [0, 0]).

    With pool > 0 only ``pool`` distinct patterns are drawn and pattern j is a
    copy of pattern j mod pool (used for multi-GiB pattern stacks).
    """
    rng = np.random.default_rng(seed + 104729)
    k = np.fft.fftfreq(N) * N
    kr2 = k[:, None] ** 2 + k[None, :] ** 2
    disk = kr2 <= (N / 4.0) ** 2
    rate = np.where(disk, bf_fraction * dose / disk.sum(),
                    (1 - bf_fraction) * dose / (~disk).sum() * np.exp(-kr2 / (N / 3.0) ** 2) * 4)
    n_draw = J if pool <= 0 else min(pool, J)
    drawn = np.empty((n_draw, N, N), dtype=np.float32)
    for j in range(n_draw):
        modulation = 1.0 + 0.3 * rng.standard_normal((N, N)) * disk
        drawn[j] = rng.poisson(np.maximum(rate * modulation, 0.0)).astype(np.float32)
    if n_draw == J:
        return drawn
    out = np.empty((J, N, N), dtype=np.float32)
    for j in range(J):
        out[j] = drawn[j % n_draw]
    return out


def poisson_counts(I: np.ndarray, seed: int):
    """Poisson-sample a noise-free intensity stack (float32 counts)."""
    rng = np.random.default_rng(seed + 1299709)
    return rng.poisson(np.maximum(np.asarray(I, dtype=np.float64), 0.0)).astype(np.float32)


@dataclass
class Workload:
    """One synthetic reconstruction problem (physical units: Angstrom)."""
    name: str
    N: int
    M: int
    S: int
    H: int
    W: int
    dz: List[float]
    dx: float
    wavelength: float
    loss: str
    eps: float
    batch: int
    probe: np.ndarray = field(repr=False)
    obj: np.ndarray = field(repr=False)
    positions: np.ndarray = field(repr=False)
    patterns: Optional[np.ndarray] = field(repr=False, default=None)
    bandlimit: float = 2.0 / 3.0
    sigma: float = 1.0
    dose: float = 1e4
    seed: int = 0

    @property
    def J(self):
        return self.positions.shape[0]


LAMBDA_300KV = 0.019688

# name: (N, M, S, dz, scan, step, jitter, phi_max, dose, loss, eps, batch, seed, weights)
CONFIGS = {
    "spoa64": (64, 1, 1, 0.0, 16, 4, 0.0, 0.3, 1e4, "amplitude", 0.0, 256, 0, None),
    "ms128_m4_s8": (128, 4, 8, 2.0, 32, 8, 0.5, 0.1, 1e5, "poisson", 0.8, 1024, 1,
                   (0.6, 0.2, 0.12, 0.08)),
    "ms192_m6_s20": (192, 6, 20, 2.0, 64, 11, 0.5, 0.1, 1e5, "poisson", 0.8, 256, 2, None),
    "ms256_m8_s30": (256, 8, 30, 1.0, 128, 8, 0.5, 0.1, 1e6, "poisson", 0.8, 512, 3, None),
}


def make_workload(name: str, with_patterns: bool = True, pattern_pool: int = 0,
                  scan_override: Optional[int] = None) -> Workload:
    """Build one of the named configurations (see CONFIGS)."""
    (N, M, S, dz, scan, step, jit, phi, dose, loss, eps, batch, seed, wts) = CONFIGS[name]
    if scan_override is not None:
        scan = scan_override
    side = N + scan * step
    probe = make_probe(N, M, dose, wts)
    obj = make_object(S, side, side, phi, seed)
    pos = make_scan(scan, step, jit, seed)
    pats = make_patterns(N, pos.shape[0], dose, seed, pool=pattern_pool) if with_patterns else None
    return Workload(name=name, N=N, M=M, S=S, H=side, W=side, dz=[dz] * (S - 1), dx=0.2,
                    wavelength=LAMBDA_300KV, loss=loss, eps=eps, batch=batch, probe=probe,
                    obj=obj, positions=pos, patterns=pats, dose=dose, seed=seed)


def make_small(N: int, M: int, S: int, scan: int, step: int, seed: int, loss: str = "poisson",
               eps: float = 0.0, dz: float = 2.0, phi_max: float = 0.3, amp_noise: float = 0.0,
               jitter: float = 0.5, dose: float = 1e4, bandlimit: float = 2.0 / 3.0) -> Workload:
    """A small problem for parity tests (optionally with object amplitude below 1)."""
    side = N + scan * step
    probe = make_probe(N, M, dose)
    obj = make_object(S, side, side, phi_max, seed)
    if amp_noise > 0:
        rng = np.random.default_rng(seed + 31)
        obj = obj * (1.0 - amp_noise * rng.random(obj.shape))
    pos = make_scan(scan, step, jitter, seed)
    pats = make_patterns(N, pos.shape[0], dose, seed)
    return Workload(name=f"small{N}", N=N, M=M, S=S, H=side, W=side, dz=[dz] * (S - 1), dx=0.2,
                    wavelength=LAMBDA_300KV, loss=loss, eps=eps, batch=pos.shape[0], probe=probe,
                    obj=obj, positions=pos, patterns=pats, bandlimit=bandlimit, dose=dose,
                    seed=seed)
