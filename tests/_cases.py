"""Shared construction of parity cases: seeded inputs from the synthetic
generator, rounded to the GPU's storage types, fed identically to the HIP
path and to the FP64 oracle."""
from __future__ import annotations

import numpy as np

import oracle as orc
from paper_2505_14372_amd import synth


def rel_l2(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


def max_rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


class Case:
    """Inputs of one problem in float32/complex64 and the matching oracle geometry."""

    def __init__(self, wl: synth.Workload, consistent_patterns: bool = False, batch=None, seed: int = 0):
        self.wl = wl
        self.N, self.M, self.S, self.H, self.W = wl.N, wl.M, wl.S, wl.H, wl.W
        self.probe = wl.probe.astype(np.complex64)
        self.obj = wl.obj.astype(np.complex64)
        self.pos = wl.positions.astype(np.float32)
        self.tilt = tuple(getattr(wl, "tilt", (0.0, 0.0)))
        self.mask = getattr(wl, "bandlimit_mask", None)
        self.geom = orc.Geometry(N=wl.N, dx=wl.dx, wavelength=wl.wavelength, dz=list(wl.dz),
                                 bandlimit=wl.bandlimit, loss=wl.loss, eps=wl.eps, sigma=wl.sigma,
                                 tilt=self.tilt, bandlimit_mask=self.mask)
        J = self.pos.shape[0]
        self.batch = np.arange(J, dtype=np.int32) if batch is None else np.asarray(batch, dtype=np.int32)
        if consistent_patterns:
            # noise-free intensities of the true state, Poisson-sampled
            I = orc.forward(self.probe.astype(np.complex128), self.obj.astype(np.complex128),
                            self.pos.astype(np.float64), range(J), self.geom)
            self.pats = synth.poisson_counts(I, seed)
        else:
            self.pats = wl.patterns.astype(np.float32)

    # oracle views (exactly the float32 values the GPU sees, in float64)
    def o_args(self):
        return (self.probe.astype(np.complex128), self.obj.astype(np.complex128), self.pos.astype(np.float64))

    def oracle_forward(self, batch=None):
        P, O, X = self.o_args()
        return orc.forward(P, O, X, self.batch if batch is None else batch, self.geom)

    def oracle_grad(self, batch=None):
        P, O, X = self.o_args()
        return orc.loss_and_grad(P, O, X, self.pats.astype(np.float64), self.batch if batch is None else batch,
                                 self.geom)

    def problem(self, max_batch=None, checkpoint_every=1, **kw):
        from paper_2505_14372_amd import api
        return api.Problem(self.N, self.M, self.S, self.H, self.W, self.pos.shape[0], dz=self.wl.dz,
                           dx=self.wl.dx, wavelength=self.wl.wavelength, bandlimit=self.wl.bandlimit,
                           loss=self.wl.loss, eps=self.wl.eps, sigma=self.wl.sigma, tilt=self.tilt,
                           bandlimit_mask=self.mask, max_batch=max_batch or len(self.batch),
                           checkpoint_every=checkpoint_every, **kw)

    def device(self, dev="cuda"):
        import torch
        return dict(probe=torch.from_numpy(self.probe).to(dev), obj=torch.from_numpy(self.obj).to(dev),
                    pos=torch.from_numpy(self.pos).to(dev), pats=torch.from_numpy(self.pats).to(dev),
                    batch=torch.from_numpy(self.batch).to(dev))
