"""Recorded steps (pty_step_graph_*): one reconstruct_step recorded as a HIP
graph and replayed, checked replay by replay against the same step called
directly, with ordinary eager work and synchronisations between replays."""
import numpy as np
import pytest

from paper_2505_14372_amd import synth

from _cases import Case

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

FIELDS = ("probe", "object", "positions", "m_probe", "v_probe", "m_object", "v_object", "m_pos", "v_pos")


def _np(t):
    return (torch.view_as_real(t) if t.is_complex() else t).detach().cpu().numpy()


def _states(c, d, adam, device_step=True):
    from paper_2505_14372_amd import api
    return [api.ReconState(d["probe"].clone(), d["obj"].clone(), d["pos"].clone(), adam=adam,
                           device_step=device_step) for _ in range(2)]


def _batches(J, B, n, seed):
    rng = np.random.default_rng(seed)
    return [torch.from_numpy(np.sort(rng.permutation(J)[:B]).astype(np.int32)).cuda() for _ in range(n)]


@pytest.mark.parametrize("kind", ["adam", "sgd"])
def test_replays_equal_direct_steps_bit_for_bit(kind):
    """Ordered reduction (deterministic): after every replay the recorded
    state equals, bit for bit, a twin state stepped by direct calls with the
    same minibatches; the losses agree too and the device step count advances."""
    from paper_2505_14372_amd import api
    c = Case(synth.make_small(N=64, M=2, S=3, scan=4, step=4, seed=41, loss="poisson", eps=0.8, amp_noise=0.2))
    d = c.device()
    J, B = c.pos.shape[0], 9
    prob = c.problem(max_batch=B)
    prob.set_reduction("ordered")
    opt = (api.Optimizer(kind="adam", lr_object=1e-3, lr_probe=1e-3, lr_pos=1e-2) if kind == "adam" else
           api.Optimizer(kind="sgd", lr_object=1e-5, lr_probe=1e-4, lr_pos=1e-5))
    direct, rec = _states(c, d, adam=kind == "adam")
    g_batch = torch.empty(B, dtype=torch.int32, device="cuda")
    g_loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    batches = _batches(J, B, 5, seed=41)
    g_batch.copy_(batches[0])
    graph = prob.record_step(rec, d["pats"], g_batch, opt, g_loss)
    torch.cuda.synchronize()
    # recording runs nothing
    assert np.array_equal(_np(rec.object), _np(direct.object)) and rec.steps_done() == 0
    for r, b in enumerate(batches):
        loss = prob.reconstruct_step(direct, d["pats"], b, opt)
        g_batch.copy_(b)
        graph.replay()
        prob.check()
        # eager work of the program between replays
        _ = (direct.object.abs().sum() + rec.object.abs().sum()).item()
        for f in FIELDS:
            a, g = getattr(direct, f), getattr(rec, f)
            if a is None:
                continue
            assert np.array_equal(_np(a), _np(g)), (kind, r, f)
        assert loss.item() == g_loss.item(), (r, loss.item(), g_loss.item())
        if kind == "adam":
            assert rec.steps_done() == direct.steps_done() == r + 1
    graph.close()
    prob.close()


def test_replays_with_concurrent_chunks_match_direct_steps():
    """Atomic reduction with the group split in chunks on two internal streams
    (event fork and join inside the recording): every replay matches the
    direct step to float rounding."""
    from paper_2505_14372_amd import api
    c = Case(synth.make_small(N=128, M=2, S=3, scan=3, step=8, seed=42, loss="gaussian", amp_noise=0.2))
    d = c.device()
    J, B = c.pos.shape[0], 8
    prob = c.problem(max_batch=B)
    prob.set_chunk(3)
    prob.set_streams(2)
    opt = api.Optimizer(kind="adam", lr_object=1e-3, lr_probe=1e-3, lr_pos=1e-2)
    direct, rec = _states(c, d, adam=True)
    g_batch = torch.empty(B, dtype=torch.int32, device="cuda")
    batches = _batches(J, B, 3, seed=42)
    g_batch.copy_(batches[0])
    graph = prob.record_step(rec, d["pats"], g_batch, opt)
    for r, b in enumerate(batches):
        prob.reconstruct_step(direct, d["pats"], b, opt)
        g_batch.copy_(b)
        graph.replay()
        prob.check()
        for f in ("object", "probe", "positions"):
            a, g = _np(getattr(direct, f)), _np(getattr(rec, f))
            err = np.max(np.abs(a - g)) / np.max(np.abs(a))
            assert err < 1e-5, (r, f, err)
    graph.close()
    prob.close()


def test_device_step_count_matches_host_count():
    """Adam with the step count on the device forms the same bias corrections
    as with the host count: the two states agree after three steps."""
    from paper_2505_14372_amd import api
    c = Case(synth.make_small(N=64, M=1, S=2, scan=3, step=4, seed=43, loss="amplitude", amp_noise=0.2))
    d = c.device()
    prob = c.problem(max_batch=9)
    prob.set_reduction("ordered")
    opt = api.Optimizer(kind="adam", lr_object=1e-3, lr_probe=1e-3, lr_pos=1e-2)
    host = api.ReconState(d["probe"].clone(), d["obj"].clone(), d["pos"].clone(), adam=True)
    dev = api.ReconState(d["probe"].clone(), d["obj"].clone(), d["pos"].clone(), adam=True, device_step=True)
    for b in _batches(c.pos.shape[0], 9, 3, seed=43):
        prob.reconstruct_step(host, d["pats"], b, opt)
        prob.reconstruct_step(dev, d["pats"], b, opt)
    prob.check()
    assert host.steps_done() == dev.steps_done() == 3
    for f in FIELDS:
        a, g = _np(getattr(host, f)), _np(getattr(dev, f))
        err = np.max(np.abs(a - g)) / max(np.max(np.abs(a)), 1e-30)
        print(f, "bit-equal" if np.array_equal(a, g) else f"max rel {err:.1e}")
        assert err < 1e-6, (f, err)
    prob.close()


def test_recording_refusals():
    """Adam without a device step count, the object-spectrum L1 regularizer
    and enabled launch timing are refused before anything is recorded."""
    from paper_2505_14372_amd import _lib, api
    c = Case(synth.make_small(N=64, M=1, S=1, scan=2, step=4, seed=44, loss="gaussian"))
    d = c.device()
    prob = c.problem(max_batch=4)
    b = torch.arange(4, dtype=torch.int32, device="cuda")
    adam = api.Optimizer(kind="adam", lr_object=1e-3, lr_probe=1e-3, lr_pos=1e-2)
    host_state = api.ReconState(d["probe"].clone(), d["obj"].clone(), d["pos"].clone(), adam=True)
    with pytest.raises(_lib.PtyError, match="step_dev"):
        prob.record_step(host_state, d["pats"], b, adam)
    st = api.ReconState(d["probe"].clone(), d["obj"].clone(), d["pos"].clone(), adam=True, device_step=True)
    prob.set_regularizers(obj_spectrum_l1=0.1)
    with pytest.raises(_lib.PtyError, match="spectrum"):
        prob.record_step(st, d["pats"], b, adam)
    prob.set_regularizers()
    lib = _lib.load()
    lib.pty_profile_enable(1)
    try:
        with pytest.raises(_lib.PtyError, match="timing"):
            prob.record_step(st, d["pats"], b, adam)
    finally:
        lib.pty_profile_enable(0)
        lib.pty_profile_collect(None, 0, None, None, 0)
    # a valid recording after the refusals, and the state untouched by all of them
    g = prob.record_step(st, d["pats"], b, adam)
    g.replay()
    prob.check()
    assert st.steps_done() == 1
    g.close()
    prob.close()
