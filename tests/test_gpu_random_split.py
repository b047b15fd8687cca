"""The library's entry points agree with each other on seeded random
configurations (ordered reduction, so every run is deterministic):
forward_save + backward gives the bits of loss_and_grad, a device-side
gradient scale of 2 doubles them exactly, and pty_forward and
pty_forward_static give the intensities and loss of forward_save."""
import ctypes as C
import os

import numpy as np
import pytest

from paper_2505_14372_amd import synth

from _cases import Case

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.mark.parametrize("seed", range(int(os.environ.get("PTY_RANDOM_SPLIT", "4"))))
def test_entry_points_agree(seed):
    rng = np.random.default_rng(8000 + seed)
    N = int(rng.choice([64, 128, 192, 256]))
    M, S = int(rng.integers(1, 4)), int(rng.integers(1, 5))
    loss = str(rng.choice(["amplitude", "anscombe", "poisson", "gaussian"]))
    eps = float(rng.choice([0.0, 0.3, 0.8])) if loss != "gaussian" else 0.0
    scan, step = (int(rng.integers(2, 4)) if N < 256 else 2), int(rng.integers(3, 9))
    wl = synth.make_small(N=N, M=M, S=S, scan=scan, step=step, seed=8100 + seed, loss=loss, eps=eps,
                          amp_noise=float(rng.choice([0.0, 0.2])), dose=1e5,
                          bandlimit=float(rng.choice([2.0 / 3.0, 0.5, 0.0])))
    J = wl.positions.shape[0]
    batch = rng.permutation(J)[: int(rng.integers(1, J + 1))].astype(np.int32)
    c = Case(wl, batch=batch)
    ck = int(rng.choice([1, 1, 2, 3]))
    chunk = int(rng.choice([0, 0, 2]))
    print(f"seed {seed}: N={N} M={M} S={S} {loss} eps={eps} B={len(batch)} ck={ck} chunk={chunk}", flush=True)
    d = c.device()
    prob = c.problem(checkpoint_every=ck)
    prob.set_reduction("ordered")
    prob.set_chunk(chunk)
    L1, gO1, gP1, gX1 = prob.loss_and_grad(d["probe"], d["obj"], d["pos"], d["pats"], d["batch"])
    L2, I2 = prob.forward_save(d["probe"], d["obj"], d["pos"], d["pats"], d["batch"], intensities=True)
    gO2, gP2 = torch.empty_like(gO1), torch.empty_like(gP1)
    gX2 = torch.empty_like(gX1)
    prob.backward(1.0, g_object=gO2, g_probe=gP2, g_pos=gX2)
    prob.check()
    assert L1.item() == L2.item()
    for a, b in ((gO1, gO2), (gP1, gP2), (gX1, gX2)):
        assert torch.equal(a, b)
    # the same tape again with a device-side scale of 2: exactly twice the gradients
    L3, _ = prob.forward_save(d["probe"], d["obj"], d["pos"], d["pats"], d["batch"])
    two = torch.full((1,), 2.0, dtype=torch.float64, device="cuda")
    prob.backward(two, g_object=gO2, g_probe=gP2, g_pos=gX2)
    prob.check()
    for a, b in ((gO1, gO2), (gP1, gP2), (gX1, gX2)):
        assert torch.equal(2 * a, b)
    # forward alone and the allocation-free forward give the same intensities and loss
    I4, L4 = prob.forward(d["probe"], d["obj"], d["pos"], d["batch"], patterns=d["pats"])
    prob.check()
    assert torch.equal(I2, I4) and L4.item() == L2.item()
    from paper_2505_14372_amd import _lib
    lib = _lib.load()
    ptr = lambda t: C.c_void_p(t.data_ptr())  # noqa: E731
    I5 = torch.full_like(I2, -1.0)
    L5 = torch.full((1,), -1.0, dtype=torch.float64, device="cuda")
    st = lib.pty_forward_static(prob.ctx, C.c_void_p(torch.cuda.current_stream().cuda_stream), ptr(d["probe"]),
                                ptr(d["obj"]), ptr(d["pos"]), ptr(d["batch"]), len(batch), ptr(d["pats"]), ptr(I5),
                                ptr(L5))
    if st == _lib.PTY_OK:
        prob.check()
        assert torch.equal(I2, I5) and L5.item() == L2.item()
    else:
        # only a batch beyond the static array's size is refused
        assert st == _lib.PTY_EINVAL and b"static scratch" in lib.pty_last_error(prob.ctx)
