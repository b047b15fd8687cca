"""ctypes declarations of the libpty C ABI (include/pty.h).

Loading fails loudly when the in-tree library is missing: there is no other
implementation of these entry points in this package.
"""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpty.so")

PTY_OK, PTY_EINVAL, PTY_EBOUNDS, PTY_EUNSUPPORTED, PTY_ENOMEM, PTY_EHIP, PTY_ENONFINITE, PTY_ESTATE = range(8)
STATUS_NAMES = {0: "PTY_OK", 1: "PTY_EINVAL", 2: "PTY_EBOUNDS", 3: "PTY_EUNSUPPORTED", 4: "PTY_ENOMEM",
                5: "PTY_EHIP", 6: "PTY_ENONFINITE", 7: "PTY_ESTATE"}
LOSS_IDS = {"amplitude": 0, "anscombe": 1, "poisson": 2, "gaussian": 3}
OPT_SGD, OPT_ADAM, OPT_EPIE = 0, 1, 2
OPT_KINDS = {"sgd": OPT_SGD, "adam": OPT_ADAM, "epie": OPT_EPIE}
STRATEGIES = {"auto": 0, "two_pass": 1, "resident": 2}
REDUCTIONS = {"atomic": 0, "ordered": 1}
PTY_ACCUMULATE = 1
PTY_POS_DENSE = 2

# every exported symbol of include/pty.h
EXPORTS = (
    "pty_create", "pty_create_ex", "pty_workspace_bytes", "pty_workspace_bytes_ex", "pty_checkpoint_every",
    "pty_checkpoint_half", "pty_set_chunk", "pty_forward", "pty_loss_and_grad",
    "pty_forward_save", "pty_backward", "pty_reconstruct_step", "pty_check", "pty_last_error",
    "pty_destroy", "pty_group_create", "pty_group_workspace_bytes", "pty_group_reconstruct_step",
    "pty_group_last_error", "pty_group_destroy", "pty_profile_enable", "pty_profile_select", "pty_profile_collect",
    "pty_set_regularizers", "pty_set_strategy", "pty_set_reduction", "pty_lsqml_step", "pty_set_streams",
    "pty_backward_dev", "pty_forward_static", "pty_step_graph_create", "pty_step_graph_launch",
    "pty_step_graph_destroy",
)
# bytes of the static device array behind pty_forward_static (PTY_STATIC_SCRATCH_BYTES)
STATIC_SCRATCH_BYTES = 32 << 20


class Geometry(C.Structure):
    _fields_ = [
        ("N", C.c_int32), ("n_modes", C.c_int32), ("n_slices", C.c_int32),
        ("obj_h", C.c_int32), ("obj_w", C.c_int32), ("n_positions", C.c_int32),
        ("dx", C.c_double), ("wavelength", C.c_double), ("dz", C.POINTER(C.c_double)),
        ("bandlimit", C.c_double), ("loss", C.c_int32), ("eps", C.c_double), ("sigma", C.c_double),
        ("tilt_y", C.c_double), ("tilt_x", C.c_double), ("bandlimit_mask", C.POINTER(C.c_uint8)),
    ]


class Options(C.Structure):
    _fields_ = [("max_batch", C.c_int32), ("checkpoint_every", C.c_int32), ("hbm_budget", C.c_size_t),
                ("checkpoint_half", C.c_int32), ("lsqml", C.c_int32)]


class Regularizers(C.Structure):
    _fields_ = [("obj_l2", C.c_double), ("probe_l2", C.c_double), ("obj_l1", C.c_double),
                ("obj_tikhonov", C.c_double), ("obj_tv", C.c_double), ("layers_tikhonov", C.c_double),
                ("layers_tv", C.c_double), ("tv_delta", C.c_double), ("amp_clamp", C.c_int32),
                ("amp_min", C.c_double), ("amp_max", C.c_double), ("probe_support", C.POINTER(C.c_uint8)),
                ("layer_sigma", C.c_double), ("obj_lowpass_sigma", C.c_double), ("phase_deramp", C.c_int32),
                ("obj_phase_l1", C.c_double), ("obj_spectrum_l1", C.c_double),
                ("probe_phase_tikhonov", C.c_double), ("probe_phase_tv", C.c_double),
                ("probe_support_real", C.POINTER(C.c_uint8))]


class Illum(C.Structure):
    _fields_ = [("obj_prev", C.c_void_p), ("obj_cur", C.c_void_p), ("probe_prev", C.c_void_p),
                ("probe_cur", C.c_void_p)]


class Lsqml(C.Structure):
    _fields_ = [("beta_object", C.c_double), ("beta_probe", C.c_double), ("delta_object", C.c_double),
                ("delta_probe", C.c_double), ("gamma", C.c_double)]


class State(C.Structure):
    _fields_ = [
        ("probe", C.c_void_p), ("object", C.c_void_p), ("positions", C.c_void_p),
        ("m_probe", C.c_void_p), ("v_probe", C.c_void_p),
        ("m_object", C.c_void_p), ("v_object", C.c_void_p),
        ("m_pos", C.c_void_p), ("v_pos", C.c_void_p),
        ("step", C.c_int64), ("step_dev", C.c_void_p),
    ]


class Optim(C.Structure):
    _fields_ = [
        ("kind", C.c_int32), ("lr_object", C.c_double), ("lr_probe", C.c_double), ("lr_pos", C.c_double),
        ("beta1", C.c_double), ("beta2", C.c_double), ("eps", C.c_double),
    ]


class GroupItem(C.Structure):
    _fields_ = [
        ("ctx", C.c_void_p), ("state", C.POINTER(State)), ("patterns", C.c_void_p),
        ("batch_idx", C.c_void_p), ("batch", C.c_int32), ("opt", C.POINTER(Optim)), ("loss", C.c_void_p),
    ]


_lib = None


def load():
    """Load libpty.so (built in-tree by build_lib); raise if it is absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built: run `python -m paper_2505_14372_amd.build_lib`")
    lib = C.CDLL(LIB_PATH)
    vp, i32, i64, f64, u32, sz = C.c_void_p, C.c_int32, C.c_int64, C.c_double, C.c_uint32, C.c_size_t
    sig = {
        "pty_create": ([C.POINTER(Geometry), i32, i32, sz, C.POINTER(vp)], i32),
        "pty_workspace_bytes": ([C.POINTER(Geometry), i32, i32, C.POINTER(sz)], i32),
        "pty_create_ex": ([C.POINTER(Geometry), C.POINTER(Options), C.POINTER(vp)], i32),
        "pty_workspace_bytes_ex": ([C.POINTER(Geometry), C.POINTER(Options), C.POINTER(sz)], i32),
        "pty_checkpoint_half": ([vp], i32),
        "pty_checkpoint_every": ([vp], i32),
        "pty_set_chunk": ([vp, i32], i32),
        "pty_set_streams": ([vp, i32], i32),
        "pty_forward": ([vp, vp, vp, vp, vp, vp, i32, vp, vp, vp], i32),
        "pty_forward_static": ([vp, vp, vp, vp, vp, vp, i32, vp, vp, vp], i32),
        "pty_loss_and_grad": ([vp, vp, vp, vp, vp, vp, vp, i32, vp, vp, vp, vp, u32], i32),
        "pty_forward_save": ([vp, vp, vp, vp, vp, vp, vp, i32, vp, vp], i32),
        "pty_backward": ([vp, vp, f64, vp, vp, vp, u32], i32),
        "pty_backward_dev": ([vp, vp, vp, vp, vp, vp, u32], i32),
        "pty_reconstruct_step": ([vp, vp, C.POINTER(State), vp, vp, i32, C.POINTER(Optim), vp], i32),
        "pty_check": ([vp, vp], i32),
        "pty_last_error": ([vp], C.c_char_p),
        "pty_destroy": ([vp], None),
        "pty_group_create": ([i32, i32, i32, i64, C.POINTER(vp)], i32),
        "pty_group_workspace_bytes": ([i32, i32, i32, i64, C.POINTER(sz)], i32),
        "pty_group_reconstruct_step": ([vp, vp, C.POINTER(GroupItem), i32], i32),
        "pty_group_last_error": ([vp], C.c_char_p),
        "pty_group_destroy": ([vp], None),
        "pty_profile_enable": ([i32], None),
        "pty_profile_select": ([C.c_char_p], i32),
        "pty_set_regularizers": ([vp, C.POINTER(Regularizers)], i32),
        "pty_set_strategy": ([vp, i32], i32),
        "pty_set_reduction": ([vp, i32], i32),
        "pty_lsqml_step": ([vp, vp, C.POINTER(State), C.POINTER(Illum), vp, vp, i32, C.POINTER(Lsqml), vp], i32),
        "pty_profile_collect": ([C.c_char_p, sz, C.POINTER(f64), C.POINTER(i64), i32], i32),
        "pty_step_graph_create": ([vp, vp, C.POINTER(State), vp, vp, i32, C.POINTER(Optim), vp, C.POINTER(vp)], i32),
        "pty_step_graph_launch": ([vp, vp], i32),
        "pty_step_graph_destroy": ([vp], None),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


class PtyError(RuntimeError):
    def __init__(self, status, msg=""):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status
