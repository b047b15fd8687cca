"""Host-side checks of the C ABI: the library loads, exports every declared
entry point, and validates arguments before touching the device."""
import ctypes as C
import os
import re
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pty.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pty_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_2505_14372_amd import _lib
    return _lib.load()


def test_header_declares_the_calls():
    fns = _declared_functions()
    for need in ("pty_forward", "pty_loss_and_grad", "pty_reconstruct_step", "pty_create", "pty_destroy"):
        assert need in fns


def test_every_declared_symbol_is_exported(lib):
    from paper_2505_14372_amd import _lib
    fns = _declared_functions()
    assert set(fns) == set(_lib.EXPORTS)
    out = subprocess.run(["nm", "-D", "--defined-only", _lib.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r" T (pty_\w+)", out))
    missing = [f for f in fns if f not in exported]
    assert not missing, missing
    for f in fns:
        getattr(lib, f)


def test_workspace_sizes_follow_the_layout(lib):
    from paper_2505_14372_amd import api
    N, M, S, H, W, J, B = 256, 8, 30, 1280, 1280, 16384, 512
    tile = N * N * 8
    b1 = api.workspace_bytes(N, M, S, H, W, J, B, checkpoint_every=1)
    b0 = api.workspace_bytes(N, M, S, H, W, J, 0)
    # store-all: B*M work tiles + B*M*S checkpoints + B tiles of ordered-reduction scratch
    assert b1 - b0 >= B * M * (1 + S) * tile + B * tile
    assert b1 - b0 < B * M * (1 + S) * tile + B * tile + 64 * 2 ** 20
    # every 6th slice stored: ceil(30/6) = 5 checkpoints, 5 segment slots, a second work buffer
    b6 = api.workspace_bytes(N, M, S, H, W, J, B, checkpoint_every=6)
    assert b6 - b0 >= B * M * (2 + 5 + 5) * tile
    assert b6 < b1
    # the LSQML scratch: an illumination scatter of the object's size, a transparency map
    # of one slice's size, plus small sums
    bl = api.workspace_bytes(N, M, S, H, W, J, B, checkpoint_every=1, lsqml=True)
    # ... and, for the ordered reduction, one float per pixel and position of the group
    lsq = (S + 1) * H * W * 4 + B * N * N * 4
    assert lsq <= bl - b1 < lsq + 40 * N * N * 4 + 2 ** 20


def test_invalid_arguments_are_rejected_on_the_host(lib):
    from paper_2505_14372_amd import _lib, api
    with pytest.raises(_lib.PtyError) as e:
        api.Problem(100, 1, 1, 128, 128, 4)
    assert e.value.status == _lib.PTY_EUNSUPPORTED
    with pytest.raises(_lib.PtyError) as e:
        api.Problem(64, 1, 1, 32, 128, 4)          # object smaller than the window
    assert e.value.status == _lib.PTY_EINVAL
    with pytest.raises(ValueError):
        api.Problem(64, 1, 3, 128, 128, 4, dz=[1.0])  # wrong number of gaps
    g = _lib.Geometry(64, 1, 2, 128, 128, 4, 0.2, 0.02, None, 2 / 3, 2, 0.0, 1.0)
    ctx = C.c_void_p()
    assert lib.pty_create(C.byref(g), 8, 1, 0, C.byref(ctx)) == _lib.PTY_EINVAL  # dz missing
    assert lib.pty_create(None, 8, 1, 0, C.byref(ctx)) == _lib.PTY_EINVAL
    # one grid dimension holds a launch's positions: at most 65535 per group
    g3 = _lib.Geometry(64, 1, 1, 128, 128, 4, 0.2, 0.02, None, 2 / 3, 2, 0.0, 1.0)
    assert lib.pty_create(C.byref(g3), 65536, 1, 0, C.byref(ctx)) == _lib.PTY_EINVAL
    assert lib.pty_group_create(64, 65536, 1, 1, C.byref(ctx)) == _lib.PTY_EINVAL
    assert lib.pty_backward(None, None, 1.0, None, None, None, 0) == _lib.PTY_EINVAL
    assert lib.pty_group_create(100, 1, 1, 1, C.byref(ctx)) == _lib.PTY_EUNSUPPORTED
    assert lib.pty_group_reconstruct_step(None, None, None, 0) == _lib.PTY_EINVAL
    assert lib.pty_last_error(None) == b"NULL context"
    assert lib.pty_set_reduction(None, 1) == _lib.PTY_EINVAL
    assert lib.pty_set_strategy(None, 1) == _lib.PTY_EINVAL
    assert lib.pty_set_chunk(None, 4) == _lib.PTY_EINVAL


def test_profile_class_selection(lib):
    """pty_profile_select names kernel classes (host only: no event is recorded
    while timing is off)."""
    assert lib.pty_profile_select(b"row_adj") == 1
    assert lib.pty_profile_select(b"row_adj,col_prop\nrow_adj") == 2
    assert lib.pty_profile_select(b"no_such_kernel") == -1
    assert lib.pty_profile_select(b"row_fwd,no_such_kernel") == -1
    n_all = lib.pty_profile_select(None)
    assert n_all >= 19 and lib.pty_profile_select(b"") == n_all


@pytest.mark.parametrize("prog", ["line_fft_check", "resident_check"])
def test_host_fft_emulation(tmp_path, prog):
    """The cross-lane line FFT of the kernels (and the in-place 2D transform of
    the LDS-resident tile), emulated lane by lane on the host, match a
    double-precision DFT for every supported N."""
    from paper_2505_14372_amd import build_lib
    exe = tmp_path / prog
    src = os.path.join(ROOT, "tests", "host", prog + ".cpp")
    r = subprocess.run([build_lib.hipcc(), "-std=c++17", "-O1", "-I", build_lib.CSRC, "-I", build_lib.INCLUDE,
                        src, "-o", str(exe)], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    r = subprocess.run([str(exe)], capture_output=True, text=True)
    print(r.stdout)
    assert r.returncode == 0, r.stdout
