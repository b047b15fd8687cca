"""Parity at the full size of the headline workload (probe 256 x 256, 8 modes,
30 slices of 1 A, object 1280 x 1280 x 30, a group of 512 positions), in the
launch configuration the benchmark times. The oracle computes sampled
positions one by one; whole-group quantities are checked through properties
that hold at any size (additivity over sub-groups, the loss of the returned
intensities)."""
import numpy as np
import pytest

import oracle as orc
from paper_2505_14372_amd import synth

from _cases import Case, rel_l2

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

B = 512


@pytest.fixture(scope="module")
def full():
    wl = synth.make_workload("ms256_m8_s30", pattern_pool=64)
    rng = np.random.default_rng(3)
    batch = np.sort(rng.choice(wl.J, size=B, replace=False)).astype(np.int32)
    c = Case(wl, batch=batch)
    return c


def _np(t):
    return t.detach().cpu().numpy()


def test_full_size_forward_and_gradient_sampled(full):
    c = full
    print(f"full-size case N={c.N} M={c.M} S={c.S} B={B} H={c.H}", flush=True)
    d = c.device()
    prob = c.problem(max_batch=B)
    I, loss_f = prob.forward(d["probe"], d["obj"], d["pos"], d["batch"], patterns=d["pats"])
    loss, gO, gP, gX = prob.loss_and_grad(d["probe"], d["obj"], d["pos"], d["pats"], d["batch"])
    prob.check()
    I, gX = _np(I), _np(gX)
    # the loss equals the noise model summed over the returned intensities
    Ie = c.pats[c.batch].astype(np.float64)
    ell, _ = orc.loss_and_weight(I.astype(np.float64), Ie, c.geom.loss, c.geom.eps)
    assert abs(loss.item() - ell.sum()) < 1e-4 * abs(ell.sum())
    assert abs(loss.item() - loss_f.item()) < 1e-6 * abs(loss.item())
    # sampled positions against the oracle, one by one
    for b in (0, 257, B - 1):
        ref = c.oracle_grad(batch=[int(c.batch[b])])
        assert rel_l2(I[b], ref["I"][0]) < 1e-4
        assert rel_l2(gX[b], ref["g_pos"][0]) < 1e-3
        print(b, rel_l2(I[b], ref["I"][0]), rel_l2(gX[b], ref["g_pos"][0]), flush=True)
    # additivity over two halves of the group
    h = B // 2
    halves = [d["batch"][:h].contiguous(), d["batch"][h:].contiguous()]
    parts = [prob.loss_and_grad(d["probe"], d["obj"], d["pos"], d["pats"], x) for x in halves]
    assert abs(parts[0][0].item() + parts[1][0].item() - loss.item()) < 1e-6 * abs(loss.item())
    assert rel_l2(_np(parts[0][1] + parts[1][1]), _np(gO)) < 1e-5
    assert rel_l2(_np(parts[0][2] + parts[1][2]), _np(gP)) < 1e-5


def test_full_size_two_position_gradients(full):
    """Object and probe gradients of a two-position group at full size against the oracle."""
    c = full
    sub = Case(c.wl, batch=c.batch[[10, 11]])
    ref = sub.oracle_grad()
    d = sub.device()
    prob = sub.problem(max_batch=2)
    loss, gO, gP, gX = prob.loss_and_grad(d["probe"], d["obj"], d["pos"], d["pats"], d["batch"])
    prob.check()
    assert abs(loss.item() - ref["loss"]) < 1e-4 * abs(ref["loss"])
    assert rel_l2(_np(gO), ref["g_object"]) < 1e-3
    assert rel_l2(_np(gP), ref["g_probe"]) < 1e-3
    assert rel_l2(_np(gX), ref["g_pos"]) < 1e-3


def test_full_size_half_checkpoints(full):
    """Half-precision entry-wave checkpoints at full size: a two-position group
    against the oracle, and the whole group against the float32 checkpoints."""
    c = full
    sub = Case(c.wl, batch=c.batch[[10, 11]])
    ref = sub.oracle_grad()
    d = sub.device()
    prob = sub.problem(max_batch=2, checkpoint_half=True)
    loss, gO, gP, gX = prob.loss_and_grad(d["probe"], d["obj"], d["pos"], d["pats"], d["batch"])
    prob.check()
    assert abs(loss.item() - ref["loss"]) < 1e-4 * abs(ref["loss"])
    assert rel_l2(_np(gO), ref["g_object"]) < 1e-3
    assert rel_l2(_np(gP), ref["g_probe"]) < 1e-3
    assert rel_l2(_np(gX), ref["g_pos"]) < 1e-3
    d = c.device()
    full32 = c.problem(max_batch=B)
    full16 = c.problem(max_batch=B, checkpoint_half=True)
    a = full32.loss_and_grad(d["probe"], d["obj"], d["pos"], d["pats"], d["batch"])
    del full32
    b = full16.loss_and_grad(d["probe"], d["obj"], d["pos"], d["pats"], d["batch"])
    full16.check()
    assert a[0].item() == b[0].item()
    for x, y in zip(a[1:], b[1:]):
        print(rel_l2(_np(y), _np(x)))
        assert rel_l2(_np(y), _np(x)) < 1e-3


def test_full_size_ordered_reduction_is_bitwise_repeatable(full):
    """The ordered object-gradient reduction at full size: two calls give the
    same bits, and the result equals the atomic reduction's to rounding."""
    c = full
    d = c.device()
    prob = c.problem(max_batch=B)
    _, gO_at, gP_at, _ = prob.loss_and_grad(d["probe"], d["obj"], d["pos"], d["pats"], d["batch"])
    prob.set_reduction("ordered")
    runs = [prob.loss_and_grad(d["probe"], d["obj"], d["pos"], d["pats"], d["batch"]) for _ in range(2)]
    prob.check()
    (l1, gO1, gP1, gX1), (l2, gO2, gP2, gX2) = runs
    assert l1.item() == l2.item()
    assert torch.equal(gO1, gO2) and torch.equal(gP1, gP2) and torch.equal(gX1, gX2)
    print(rel_l2(_np(gO1), _np(gO_at)), rel_l2(_np(gP1), _np(gP_at)), flush=True)
    assert rel_l2(_np(gO1), _np(gO_at)) < 1e-5
    assert rel_l2(_np(gP1), _np(gP_at)) < 1e-5
