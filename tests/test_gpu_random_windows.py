"""Window placement on random positions near and beyond the object's edges,
including exact half-pixel positions: the GPU flags a window out of bounds
exactly when the oracle's rule (n = floor(X + 0.5) in double from the float32
position, the N x N window inside the object) rejects it, and its
intensities match the oracle's for every accepted one."""
import os

import numpy as np
import pytest

import oracle as orc
from paper_2505_14372_amd import synth

from _cases import Case, rel_l2

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.mark.parametrize("N", [64, 128, 192, 256])
def test_window_bounds_follow_the_oracle(N):
    from paper_2505_14372_amd import _lib
    n_pos = int(os.environ.get("PTY_RANDOM_WINDOWS", "48"))
    rng = np.random.default_rng(9500 + N)
    wl = synth.make_small(N=N, M=1, S=2, scan=2, step=5, seed=9600 + N, loss="gaussian")
    H, W = wl.H, wl.W
    hi_y, hi_x = H - N, W - N
    # positions around both edges of each axis: continuous, exact halves and one ulp around them
    def coord(hi):
        base = float(rng.choice([0.0, hi]))
        kind = rng.integers(0, 3)
        if kind == 0:
            return base + rng.uniform(-1.5, 1.5)
        half = base + float(rng.choice([-0.5, 0.5]))
        if kind == 1:
            return half
        return float(np.nextafter(np.float32(half), np.float32(rng.choice([-np.inf, np.inf]))))
    X = np.array([[coord(hi_y), coord(hi_x)] for _ in range(n_pos)], dtype=np.float32)
    wl.positions = X.astype(np.float64)
    wl.patterns = np.zeros((n_pos, N, N), np.float32)
    c = Case(wl)
    d = c.device()
    prob = c.problem(max_batch=1)
    n_ok = 0
    for j in range(n_pos):
        n, _ = orc.split_positions(X[j].astype(np.float64))
        inside = n[0] >= 0 and n[1] >= 0 and n[0] + N <= H and n[1] + N <= W
        I, _ = prob.forward(d["probe"], d["obj"], d["pos"], torch.tensor([j], dtype=torch.int32, device="cuda"))
        st = prob.lib.pty_check(prob.ctx, None)
        assert st == (_lib.PTY_OK if inside else _lib.PTY_EBOUNDS), (j, X[j], n, st)
        if inside:
            n_ok += 1
            ref = c.oracle_forward([j])
            assert rel_l2(I.cpu().numpy(), ref) < 1e-4, (j, X[j])
    print(f"N={N}: {n_ok} of {n_pos} windows inside")
    assert 0 < n_ok < n_pos
