"""Python binding of libpty: torch tensors in, C ABI calls out.

Every step of the hot path runs in the HIP library; this module only checks
shapes and dtypes, hands device pointers and the current HIP stream to the
C entry points, and raises PtyError on a non-OK status.
"""
from __future__ import annotations

import ctypes as C
import weakref
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np
import torch

from . import _lib
from ._lib import PtyError


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t: Optional[torch.Tensor]):
    return C.c_void_p(t.data_ptr()) if t is not None else C.c_void_p(0)


def _need(t, dtype, shape, name):
    if t is None:
        raise ValueError(f"{name} is required")
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t


@dataclass
class Optimizer:
    """Settings of pty_reconstruct_step: 'sgd', 'adam' (learning rate 0 freezes a
    variable) or 'epie', the conventional ePIE / 3PIE engine with
    lr_object = beta_object and lr_probe = beta_probe (positions fixed)."""
    kind: str = "adam"
    lr_object: float = 1e-3
    lr_probe: float = 1e-3
    lr_pos: float = 0.0
    beta1: float = 0.9
    beta2: float = 0.999
    eps: float = 1e-8

    def c(self):
        if self.kind not in _lib.OPT_KINDS:
            raise ValueError(f"unknown optimiser {self.kind!r}")
        return _lib.Optim(_lib.OPT_KINDS[self.kind], self.lr_object, self.lr_probe,
                          self.lr_pos, self.beta1, self.beta2, self.eps)


class ReconState:
    """Resident reconstruction state (probe, object, positions, Adam moments).
    With device_step the Adam step count lives in a device int64 (read and
    advanced by the kernels), which a recorded step (Problem.record_step) needs."""

    def __init__(self, probe: torch.Tensor, obj: torch.Tensor, positions: torch.Tensor, adam: bool = True,
                 device_step: bool = False):
        self.probe = probe.contiguous()
        self.object = obj.contiguous()
        self.positions = positions.contiguous()
        z = lambda t: torch.zeros(torch.view_as_real(t).shape if t.is_complex() else t.shape,  # noqa: E731
                                  dtype=torch.float32, device=t.device)
        self.m_probe = z(self.probe) if adam else None
        self.v_probe = z(self.probe) if adam else None
        self.m_object = z(self.object) if adam else None
        self.v_object = z(self.object) if adam else None
        self.m_pos = z(self.positions) if adam else None
        self.v_pos = z(self.positions) if adam else None
        self.step = 0
        self.step_dev = torch.zeros(1, dtype=torch.int64, device=probe.device) if device_step else None

    def c(self):
        return _lib.State(_ptr(self.probe), _ptr(self.object), _ptr(self.positions), _ptr(self.m_probe),
                          _ptr(self.v_probe), _ptr(self.m_object), _ptr(self.v_object), _ptr(self.m_pos),
                          _ptr(self.v_pos), self.step, _ptr(self.step_dev))

    def steps_done(self) -> int:
        """Completed Adam steps (reads the device count when there is one)."""
        return int(self.step_dev.item()) if self.step_dev is not None else self.step

    def nbytes(self):
        return sum(t.numel() * t.element_size() for t in (self.probe, self.object, self.positions, self.m_probe,
                                                          self.v_probe, self.m_object, self.v_object, self.m_pos,
                                                          self.v_pos) if t is not None)


def _geometry(N, M, S, H, W, J, dx, wavelength, dz, bandlimit, loss, eps, sigma, tilt=(0.0, 0.0),
              bandlimit_mask=None):
    dz = list(dz) if dz is not None else []
    if len(dz) != max(S - 1, 0):
        raise ValueError(f"need {S - 1} slice gaps, got {len(dz)}")
    arr = (C.c_double * max(len(dz), 1))(*dz) if dz else None
    mask = None
    if bandlimit_mask is not None:
        m = np.ascontiguousarray(np.asarray(bandlimit_mask) != 0, dtype=np.uint8)
        if m.shape != (N, N):
            raise ValueError(f"bandlimit_mask must be {N}x{N}")
        mask = (C.c_uint8 * (N * N)).from_buffer_copy(m.tobytes())
    g = _lib.Geometry(N, M, S, H, W, J, dx, wavelength, C.cast(arr, C.POINTER(C.c_double)) if arr else None,
                      bandlimit, _lib.LOSS_IDS[loss], eps, sigma, float(tilt[0]), float(tilt[1]),
                      C.cast(mask, C.POINTER(C.c_uint8)) if mask is not None else None)
    return g, (arr, mask)


def workspace_bytes(N, M, S, H, W, J, max_batch, checkpoint_every=1, dx=0.2, wavelength=0.019688,
                    dz=None, bandlimit=2 / 3, loss="poisson", eps=0.0, sigma=1.0, checkpoint_half=False,
                    lsqml=False):
    lib = _lib.load()
    g, _keep = _geometry(N, M, S, H, W, J, dx, wavelength, dz if dz is not None else [1.0] * (S - 1),
                         bandlimit, loss, eps, sigma)
    out = C.c_size_t()
    opt = _lib.Options(max_batch, checkpoint_every, 0, 1 if checkpoint_half else 0, 1 if lsqml else 0)
    st = lib.pty_workspace_bytes_ex(C.byref(g), C.byref(opt), C.byref(out))
    if st:
        raise PtyError(st, "pty_workspace_bytes")
    return out.value


class Problem:
    """One reconstruction geometry bound to a libpty context (pty_create)."""

    def __init__(self, N: int, M: int, S: int, H: int, W: int, J: int, dz: Sequence[float] = (),
                 dx: float = 0.2, wavelength: float = 0.019688, bandlimit: float = 2 / 3,
                 loss: str = "poisson", eps: float = 0.0, sigma: float = 1.0, max_batch: int = 256,
                 checkpoint_every: int = 1, hbm_budget: int = 0, checkpoint_half: bool = False,
                 tilt=(0.0, 0.0), bandlimit_mask=None, lsqml: bool = False):
        self.lib = _lib.load()
        self._graphs = []
        self.N, self.M, self.S, self.H, self.W, self.J = N, M, S, H, W, J
        self.loss_kind = loss
        self.max_batch = max_batch
        g, self._dz_keep = _geometry(N, M, S, H, W, J, dx, wavelength, dz, bandlimit, loss, eps, sigma, tilt,
                                     bandlimit_mask)
        self._g = g
        ctx = C.c_void_p()
        opt = _lib.Options(max_batch, checkpoint_every, hbm_budget, 1 if checkpoint_half else 0, 1 if lsqml else 0)
        st = self.lib.pty_create_ex(C.byref(g), C.byref(opt), C.byref(ctx))
        if st:
            raise PtyError(st, "pty_create")
        self.ctx = ctx
        self.checkpoint_every = self.lib.pty_checkpoint_every(ctx)
        self.checkpoint_half = bool(self.lib.pty_checkpoint_half(ctx))
        self.tape_id = 0          # incremented by every forward_save (identifies the tape)

    def close(self):
        # recorded steps replay into this context's buffers: release them first
        for ref in getattr(self, "_graphs", []):
            g = ref()
            if g is not None:
                g.close()
        self._graphs = []
        if getattr(self, "ctx", None):
            self.lib.pty_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_regularizers(self, obj_l2=0.0, probe_l2=0.0, obj_l1=0.0, obj_tikhonov=0.0, obj_tv=0.0,
                         layers_tikhonov=0.0, layers_tv=0.0, tv_delta=1e-3, amp_range=None, probe_support=None,
                         layer_sigma=0.0, obj_lowpass_sigma=0.0, phase_deramp=False, obj_phase_l1=0.0,
                         obj_spectrum_l1=0.0, probe_phase_tikhonov=0.0, probe_phase_tv=0.0,
                         probe_support_real=None):
        """Cost and constraint regularizers applied by reconstruct_step (see include/pty.h)."""
        def mask_of(a, name):
            if a is None:
                return None
            m = np.ascontiguousarray(np.asarray(a) != 0, dtype=np.uint8)
            if m.shape != (self.N, self.N):
                raise ValueError(f"{name} must be {self.N}x{self.N}")
            return (C.c_uint8 * (self.N * self.N)).from_buffer_copy(m.tobytes())

        mask = mask_of(probe_support, "probe_support")
        mask_r = mask_of(probe_support_real, "probe_support_real")
        as_ptr = lambda m: C.cast(m, C.POINTER(C.c_uint8)) if m is not None else None  # noqa: E731
        lo, hi = amp_range if amp_range is not None else (0.0, 0.0)
        r = _lib.Regularizers(obj_l2, probe_l2, obj_l1, obj_tikhonov, obj_tv, layers_tikhonov, layers_tv, tv_delta,
                              1 if amp_range is not None else 0, lo, hi, as_ptr(mask), layer_sigma,
                              obj_lowpass_sigma, 1 if phase_deramp else 0, obj_phase_l1, obj_spectrum_l1,
                              probe_phase_tikhonov, probe_phase_tv, as_ptr(mask_r))
        st = self.lib.pty_set_regularizers(self.ctx, C.byref(r))
        if st:
            self._err(st, "pty_set_regularizers")

    def set_strategy(self, strategy: str):
        """'auto', 'two_pass' or 'resident' (LDS-resident chains, N = 64 and 128)."""
        st = self.lib.pty_set_strategy(self.ctx, _lib.STRATEGIES[strategy])
        if st:
            self._err(st, "pty_set_strategy")

    def set_reduction(self, mode: str):
        """Object-gradient accumulation: 'atomic' (default) or 'ordered' (bit-reproducible)."""
        st = self.lib.pty_set_reduction(self.ctx, _lib.REDUCTIONS[mode])
        if st:
            self._err(st, "pty_set_reduction")

    def set_chunk(self, positions: int):
        """Positions per launch in loss_and_grad / reconstruct_step (0: the whole group)."""
        st = self.lib.pty_set_chunk(self.ctx, int(positions))
        if st:
            self._err(st, "pty_set_chunk")

    def set_streams(self, n: int):
        """Run the chunks of a chunked schedule (set_chunk) concurrently on n
        internal streams of the context (1: one after the other)."""
        st = self.lib.pty_set_streams(self.ctx, int(n))
        if st:
            self._err(st, "pty_set_streams")

    def _err(self, st, what):
        msg = self.lib.pty_last_error(self.ctx).decode() if self.ctx else ""
        raise PtyError(st, f"{what}: {msg}")

    def _check_inputs(self, probe, obj, positions, batch_idx, patterns=None):
        _need(probe, torch.complex64, (self.M, self.N, self.N), "probe")
        _need(obj, torch.complex64, (self.S, self.H, self.W), "object")
        _need(positions, torch.float32, (self.J, 2), "positions")
        _need(batch_idx, torch.int32, None, "batch_idx")
        if batch_idx.dim() != 1:
            raise ValueError("batch_idx must be 1-D")
        if patterns is not None:
            _need(patterns, torch.float32, (self.J, self.N, self.N), "patterns")
        return batch_idx.numel()

    def forward(self, probe, obj, positions, batch_idx, patterns=None, intensities=True):
        """Intensities [B][N][N] (and the group loss if patterns are given)."""
        B = self._check_inputs(probe, obj, positions, batch_idx, patterns)
        I = torch.empty((B, self.N, self.N), dtype=torch.float32, device=probe.device) if intensities else None
        loss = torch.zeros(1, dtype=torch.float64, device=probe.device) if patterns is not None else None
        st = self.lib.pty_forward(self.ctx, _stream(), _ptr(probe), _ptr(obj), _ptr(positions), _ptr(batch_idx), B,
                                  _ptr(patterns), _ptr(I), _ptr(loss))
        if st:
            self._err(st, "pty_forward")
        return I, loss

    def loss_and_grad(self, probe, obj, positions, patterns, batch_idx, g_object=None, g_probe=None, g_pos=None,
                      accumulate=False, want=("object", "probe", "pos"), dense_pos=False, loss=None):
        """Group loss and gradients (dL/dRe + i dL/dIm) of object, probe and positions
        (per batch entry [B][2], or per position [J][2] with dense_pos); `loss`
        is an optional float64 device tensor of one element written with the loss."""
        B = self._check_inputs(probe, obj, positions, batch_idx, patterns)
        dev = probe.device
        if "object" in want and g_object is None:
            g_object = torch.empty_like(obj)
        if "probe" in want and g_probe is None:
            g_probe = torch.empty_like(probe)
        if "pos" in want and g_pos is None:
            g_pos = torch.empty((self.J if dense_pos else B, 2), dtype=torch.float32, device=dev)
        if loss is None:
            loss = torch.zeros(1, dtype=torch.float64, device=dev)
        flags = (_lib.PTY_ACCUMULATE if accumulate else 0) | (_lib.PTY_POS_DENSE if dense_pos else 0)
        st = self.lib.pty_loss_and_grad(self.ctx, _stream(), _ptr(probe), _ptr(obj), _ptr(positions),
                                        _ptr(patterns), _ptr(batch_idx), B, _ptr(loss), _ptr(g_object),
                                        _ptr(g_probe), _ptr(g_pos), flags)
        if st:
            self._err(st, "pty_loss_and_grad")
        return loss, g_object, g_probe, g_pos

    def forward_save(self, probe, obj, positions, patterns, batch_idx, intensities=False):
        B = self._check_inputs(probe, obj, positions, batch_idx, patterns)
        I = torch.empty((B, self.N, self.N), dtype=torch.float32, device=probe.device) if intensities else None
        loss = torch.zeros(1, dtype=torch.float64, device=probe.device)
        st = self.lib.pty_forward_save(self.ctx, _stream(), _ptr(probe), _ptr(obj), _ptr(positions), _ptr(patterns),
                                       _ptr(batch_idx), B, _ptr(I), _ptr(loss))
        if st:
            self._err(st, "pty_forward_save")
        self.tape_id += 1
        return loss, I

    def backward(self, grad_scale, g_object=None, g_probe=None, g_pos=None, accumulate=False, dense_pos=False):
        """Adjoint from the tape of forward_save, every gradient scaled by
        grad_scale: a Python number, or a one-element float64 device tensor
        that the kernels read on the device (no host synchronisation)."""
        flags = (_lib.PTY_ACCUMULATE if accumulate else 0) | (_lib.PTY_POS_DENSE if dense_pos else 0)
        if isinstance(grad_scale, torch.Tensor):
            _need(grad_scale, torch.float64, None, "grad_scale")
            if grad_scale.numel() != 1:
                raise ValueError("grad_scale must hold one value")
            st = self.lib.pty_backward_dev(self.ctx, _stream(), _ptr(grad_scale), _ptr(g_object), _ptr(g_probe),
                                           _ptr(g_pos), flags)
        else:
            st = self.lib.pty_backward(self.ctx, _stream(), float(grad_scale), _ptr(g_object), _ptr(g_probe),
                                       _ptr(g_pos), flags)
        if st:
            self._err(st, "pty_backward")

    def reconstruct_step(self, state: ReconState, patterns, batch_idx, opt: Optimizer, loss=None):
        B = self._check_inputs(state.probe, state.object, state.positions, batch_idx, patterns)
        if loss is None:
            loss = torch.zeros(1, dtype=torch.float64, device=state.probe.device)
        cs = state.c()
        co = opt.c()
        st = self.lib.pty_reconstruct_step(self.ctx, _stream(), C.byref(cs), _ptr(patterns), _ptr(batch_idx), B,
                                           C.byref(co), _ptr(loss))
        if st:
            self._err(st, "pty_reconstruct_step")
        state.step = cs.step
        return loss

    def record_step(self, state: ReconState, patterns, batch_idx, opt: Optimizer, loss=None) -> "StepGraph":
        """Record one reconstruct_step as a HIP graph (pty_step_graph_create)
        for replays: StepGraph.replay() runs the whole step again on the same
        buffers, reading their current contents (write the next minibatch's
        indices into batch_idx in place between replays). Adam needs a state
        made with device_step=True. Recording runs nothing; it uses a side
        stream, since the default stream cannot record."""
        B = self._check_inputs(state.probe, state.object, state.positions, batch_idx, patterns)
        if loss is None:
            loss = torch.zeros(1, dtype=torch.float64, device=state.probe.device)
        cs = state.c()
        co = opt.c()
        out = C.c_void_p()
        side = torch.cuda.Stream(device=state.probe.device)
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            st = self.lib.pty_step_graph_create(self.ctx, _stream(), C.byref(cs), _ptr(patterns), _ptr(batch_idx),
                                                B, C.byref(co), _ptr(loss), C.byref(out))
        torch.cuda.current_stream().wait_stream(side)
        if st:
            self._err(st, "pty_step_graph_create")
        return StepGraph(self, out, (state, patterns, batch_idx, loss))

    def lsqml_step(self, state: ReconState, illum: "IllumSums", patterns, batch_idx, beta_object=0.1,
                   beta_probe=0.1, delta_object=1e-2, delta_probe=1e-2, gamma=0.0, loss=None):
        """One LSQML group step (pty_lsqml_step); needs Problem(..., lsqml=True).
        Every slice takes its full least-squares correction and also passes it
        on to the slices before it, so with many slices full steps (beta = 1)
        overshoot; the default scale is 0.1."""
        B = self._check_inputs(state.probe, state.object, state.positions, batch_idx, patterns)
        for t, shape, name in ((illum.obj_cur, (self.S, self.H, self.W), "obj_cur"),
                               (illum.obj_prev, (self.S, self.H, self.W), "obj_prev"),
                               (illum.probe_cur, (self.N, self.N), "probe_cur"),
                               (illum.probe_prev, (self.N, self.N), "probe_prev")):
            if t is not None or name.endswith("cur"):
                _need(t, torch.float32, shape, name)
                if not t.is_contiguous():
                    raise ValueError(f"{name} must be contiguous")
        if loss is None:
            loss = torch.zeros(1, dtype=torch.float64, device=state.probe.device)
        cs = state.c()
        co = _lib.Lsqml(beta_object, beta_probe, delta_object, delta_probe, gamma)
        ci = illum.c()
        st = self.lib.pty_lsqml_step(self.ctx, _stream(), C.byref(cs), C.byref(ci), _ptr(patterns), _ptr(batch_idx),
                                     B, C.byref(co), _ptr(loss))
        if st:
            self._err(st, "pty_lsqml_step")
        return loss

    def check(self):
        """Synchronise and raise on a device-side flag (window out of bounds, non-finite loss)."""
        st = self.lib.pty_check(self.ctx, _stream())
        if st:
            self._err(st, "pty_check")


class StepGraph:
    """A recorded reconstruct_step (Problem.record_step). replay() enqueues
    the whole step on the current stream; close() (or closing the Problem)
    releases it."""

    def __init__(self, prob: Problem, handle: C.c_void_p, keep):
        self.prob = prob
        self.handle = handle
        self._keep = keep          # the recorded buffers stay alive with the graph
        prob._graphs.append(weakref.ref(self))

    def replay(self):
        if not self.handle or not self.prob.ctx:
            raise RuntimeError("the recorded step or its problem is closed")
        st = self.prob.lib.pty_step_graph_launch(self.handle, _stream())
        if st:
            self.prob._err(st, "pty_step_graph_launch")

    def close(self):
        if getattr(self, "handle", None):
            self.prob.lib.pty_step_graph_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class IllumSums:
    """Illumination sums of the LSQML engine over an iteration (object view
    [S][H][W], probe view [N][N]): the running sums of the current iteration
    and, after the first, those of the previous one."""

    def __init__(self, S: int, H: int, W: int, N: int, device="cuda"):
        f = dict(dtype=torch.float32, device=device)
        self.obj_cur = torch.zeros((S, H, W), **f)
        self.probe_cur = torch.zeros((N, N), **f)
        self.obj_prev = None
        self.probe_prev = None

    def end_iteration(self):
        """The running sums become the previous iteration's; new running sums start at zero."""
        self.obj_prev, self.probe_prev = self.obj_cur, self.probe_cur
        self.obj_cur = torch.zeros_like(self.obj_prev)
        self.probe_cur = torch.zeros_like(self.probe_prev)

    def c(self):
        return _lib.Illum(_ptr(self.obj_prev), _ptr(self.obj_cur), _ptr(self.probe_prev), _ptr(self.probe_cur))


class Group:
    """Shared-launch workspace for reconstructions with one window size (pty_group_*)."""

    def __init__(self, N: int, max_items: int, max_tiles: int, max_ckpt_tiles: int):
        self.lib = _lib.load()
        self.N = N
        g = C.c_void_p()
        st = self.lib.pty_group_create(N, max_items, max_tiles, max_ckpt_tiles, C.byref(g))
        if st:
            raise PtyError(st, "pty_group_create")
        self.grp = g

    @staticmethod
    def workspace_bytes(N, max_items, max_tiles, max_ckpt_tiles):
        lib = _lib.load()
        out = C.c_size_t()
        st = lib.pty_group_workspace_bytes(N, max_items, max_tiles, max_ckpt_tiles, C.byref(out))
        if st:
            raise PtyError(st, "pty_group_workspace_bytes")
        return out.value

    def step(self, entries):
        """entries: list of (Problem, ReconState, patterns, batch_idx, Optimizer, loss_tensor)."""
        n = len(entries)
        items = (_lib.GroupItem * n)()
        keep = []
        for q, (prob, state, pats, bidx, opt, loss) in enumerate(entries):
            cs, co = state.c(), opt.c()
            keep.append((cs, co))
            items[q] = _lib.GroupItem(prob.ctx, C.pointer(cs), _ptr(pats), _ptr(bidx), bidx.numel(), C.pointer(co),
                                      _ptr(loss))
        st = self.lib.pty_group_reconstruct_step(self.grp, _stream(), items, n)
        if st:
            raise PtyError(st, "pty_group_reconstruct_step: " + self.lib.pty_group_last_error(self.grp).decode())
        for (prob, state, *_), (cs, _co) in zip(entries, keep):
            state.step = cs.step

    def close(self):
        if getattr(self, "grp", None):
            self.lib.pty_group_destroy(self.grp)
            self.grp = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
