"""Parity at the full size of the headline workload (probe 256 x 256, 8 modes,
30 slices of 1 A, object 1280 x 1280 x 30, a group of 512 positions), in the
launch configuration the benchmark times. The oracle computes sampled
positions one by one, and the whole group's object gradient on a region of
the object from exactly the positions whose windows cover it; whole-group
quantities are also checked through properties that hold at any size
(additivity over sub-groups, the loss of the returned intensities)."""
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import oracle as orc
from paper_2505_14372_amd import synth

from _cases import Case, max_rel, rel_l2

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


class _Patterns:
    """Patterns of a few positions in float64, indexed like the full stack."""

    def __init__(self, pats, idx):
        self.d = {int(j): pats[int(j)].astype(np.float64) for j in idx}

    def __getitem__(self, j):
        return self.d[int(j)]


REGION = 16


@pytest.fixture(scope="module")
def region_ref(full):
    """Oracle object gradient of the whole group on a REGION x REGION pixel
    column through all slices in the middle of the object, summed over exactly
    the group's positions whose windows cover it (every other position adds
    nothing there), on a thread pool over the host cores."""
    c = full
    R = REGION
    y0, x0 = c.H // 2 - R // 2, c.W // 2 - R // 2
    n = np.floor(c.pos[c.batch].astype(np.float64) + 0.5).astype(np.int64)
    cover = [int(c.batch[b]) for b in range(B)
             if n[b, 0] < y0 + R and n[b, 0] + c.N > y0 and n[b, 1] < x0 + R and n[b, 1] + c.N > x0]
    print(f"region {R}x{R} at ({y0}, {x0}): {len(cover)} covering positions", flush=True)
    assert 10 <= len(cover) < B
    P, O, X = c.o_args()
    pats = _Patterns(c.pats, cover)
    workers = max(1, min(16, len(os.sched_getaffinity(0))))
    parts = [cover[k::workers] for k in range(workers) if cover[k::workers]]

    def run(part):
        return orc.loss_and_grad(P, O, X, pats, part, c.geom)["g_object"][:, y0:y0 + R, x0:x0 + R].copy()

    with ThreadPoolExecutor(max_workers=len(parts)) as ex:
        ref = sum(ex.map(run, parts))
    return (y0, x0), ref


@pytest.mark.parametrize("reduction", ["atomic", "ordered"])
def test_full_size_object_gradient_region(full, region_ref, reduction):
    """The 512-position group's object gradient, element by element against the
    oracle on a region of the object, under both reductions."""
    c = full
    (y0, x0), ref = region_ref
    R = REGION
    d = c.device()
    prob = c.problem(max_batch=B)
    prob.set_reduction(reduction)
    print(f"full-size object-gradient region, {reduction} reduction", flush=True)
    loss, gO, gP, gX = prob.loss_and_grad(d["probe"], d["obj"], d["pos"], d["pats"], d["batch"])
    prob.check()
    got = _np(gO[:, y0:y0 + R, x0:x0 + R]).astype(np.complex128)
    e2, einf = rel_l2(got, ref), max_rel(got, ref)
    print(f"{reduction}: rel L2 {e2:.2e}, max {einf:.2e}", flush=True)
    assert e2 < 1e-3 and einf < 1e-3
