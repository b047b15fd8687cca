"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Tolerances (relative L2 over the whole array, GPU FP32 vs oracle FP64):
intensities and loss 1e-4, gradients 1e-3 (the bars of the hot-path
contract; observed errors are ~1e-6).
"""
import numpy as np
import pytest

import oracle as orc
from paper_2505_14372_amd import synth

from _cases import Case, max_rel, rel_l2

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

TOL_I = 1e-4
TOL_G = 1e-3


def _widen(wl, extra, seed, shift=0.0):
    """Append `extra` weak-phase columns to every object slice (H != W) and move
    the windows right by `shift` pixels; returns the workload."""
    rng = np.random.default_rng(seed)
    pad = np.exp(1j * 0.2 * rng.random((wl.S, wl.H, extra)))
    wl.obj = np.concatenate([wl.obj, pad], axis=2)
    wl.W = wl.obj.shape[2]
    wl.positions = wl.positions + np.array([0.0, shift])
    return wl


def _case(name):
    if name == "n64_spoa_amp":       # config 0 in miniature: one slice, one mode, amplitude, eps = 0
        return Case(synth.make_small(N=64, M=1, S=1, scan=5, step=4, seed=0, loss="amplitude", eps=0.0,
                                     phi_max=0.3, jitter=0.0), consistent_patterns=True, seed=0)
    if name == "n64_ms_poisson":
        return Case(synth.make_small(N=64, M=3, S=4, scan=4, step=4, seed=1, loss="poisson", eps=0.8,
                                     amp_noise=0.2))
    if name == "n128_ms_poisson":
        return Case(synth.make_small(N=128, M=2, S=3, scan=3, step=8, seed=2, loss="poisson", eps=0.8,
                                     phi_max=0.1, dose=1e5))
    if name == "n192_ms_anscombe":
        return Case(synth.make_small(N=192, M=2, S=3, scan=3, step=11, seed=3, loss="anscombe", eps=0.0,
                                     phi_max=0.1, dose=1e5))
    if name == "n256_ms_gaussian":
        return Case(synth.make_small(N=256, M=2, S=3, scan=3, step=8, seed=4, loss="gaussian", eps=0.0,
                                     phi_max=0.1, dose=1e3, dz=1.0))
    if name == "n128_tilt_mask_dz":     # propagator tilt, a square band-limit mask, non-uniform gaps
        wl = synth.make_small(N=128, M=2, S=4, scan=3, step=8, seed=6, loss="poisson", eps=0.8, phi_max=0.2,
                              dose=1e5)
        wl.dz = [1.0, 3.5, 2.0]
        wl.tilt = (0.003, -0.005)
        k = np.fft.fftfreq(128) * 128
        wl.bandlimit_mask = (np.abs(k)[:, None] <= 40) & (np.abs(k)[None, :] <= 40)
        return Case(wl)
    if name == "n64_offset_mask":      # a band-limit mask whose rows are not centred intervals
        wl = synth.make_small(N=64, M=2, S=3, scan=3, step=5, seed=7, loss="poisson", eps=0.8, phi_max=0.2,
                              dose=1e5)
        k = np.fft.fftfreq(64) * 64
        wl.bandlimit_mask = ((k[None, :] >= -10) & (k[None, :] <= 20) & (np.abs(k)[:, None] <= 18)) | \
            ((np.abs(k)[None, :] <= 3) & (np.abs(k)[:, None] <= 25))
        return Case(wl)
    if name == "n64_wide_object":      # H != W: catches swapped object axes
        wl = synth.make_small(N=64, M=2, S=3, scan=3, step=5, seed=8, loss="poisson", eps=0.8, phi_max=0.2,
                              dose=1e5)
        return Case(_widen(wl, 37, seed=8, shift=29.0))
    if name == "n64_amp_eps_nobl":
        return Case(synth.make_small(N=64, M=2, S=3, scan=3, step=5, seed=5, loss="amplitude", eps=0.5,
                                     bandlimit=0.0, amp_noise=0.1))
    raise KeyError(name)


CASES = ["n64_spoa_amp", "n64_ms_poisson", "n128_ms_poisson", "n192_ms_anscombe", "n256_ms_gaussian",
         "n64_amp_eps_nobl", "n128_tilt_mask_dz", "n64_offset_mask", "n64_wide_object"]


@pytest.fixture(scope="module")
def cache():
    return {}


def _get(cache, name):
    if name not in cache:
        c = _case(name)
        cache[name] = (c, c.oracle_grad())
    return cache[name]


def _real_components(a):
    """Real components of an array (complex entries split into (re, im) pairs)."""
    a = np.asarray(a)
    if np.iscomplexobj(a):
        return np.stack([a.real, a.imag], axis=-1)
    return a.astype(np.float64)


def _np(t):
    return t.detach().cpu().numpy()


@pytest.mark.parametrize("name", CASES)
def test_forward_parity(cache, name):
    c, ref = _get(cache, name)
    print(f"case {name} N={c.N} M={c.M} S={c.S} B={len(c.batch)}", flush=True)
    d = c.device()
    prob = c.problem()
    I, loss = prob.forward(d["probe"], d["obj"], d["pos"], d["batch"], patterns=d["pats"])
    prob.check()
    assert rel_l2(_np(I), ref["I"]) < TOL_I, rel_l2(_np(I), ref["I"])
    # element by element: no pixel off by more than TOL_I of the largest intensity
    assert max_rel(_np(I), ref["I"]) < TOL_I, max_rel(_np(I), ref["I"])
    assert abs(loss.item() - ref["loss"]) < TOL_I * abs(ref["loss"])


@pytest.mark.parametrize("name", CASES)
def test_gradient_parity(cache, name):
    c, ref = _get(cache, name)
    print(f"case {name} N={c.N} M={c.M} S={c.S} B={len(c.batch)}", flush=True)
    d = c.device()
    prob = c.problem()
    loss, gO, gP, gX = prob.loss_and_grad(d["probe"], d["obj"], d["pos"], d["pats"], d["batch"])
    prob.check()
    assert abs(loss.item() - ref["loss"]) < TOL_I * abs(ref["loss"])
    errs = dict(obj=rel_l2(_np(gO), ref["g_object"]), probe=rel_l2(_np(gP), ref["g_probe"]),
                pos=rel_l2(_np(gX), ref["g_pos"]))
    print(errs)
    assert all(e < TOL_G for e in errs.values()), errs
    # element by element, against the largest entry of each gradient
    emax = dict(obj=max_rel(_np(gO), ref["g_object"]), probe=max_rel(_np(gP), ref["g_probe"]),
                pos=max_rel(_np(gX), ref["g_pos"]))
    print(emax)
    assert all(e < TOL_G for e in emax.values()), emax
    # object gradient vanishes outside every window
    n = np.floor(c.pos.astype(np.float64)[c.batch] + 0.5).astype(int)
    cover = np.zeros((c.H, c.W), bool)
    for y, x in n:
        cover[y:y + c.N, x:x + c.N] = True
    assert np.all(_np(gO)[:, ~cover] == 0)


def test_ragged_batch_and_duplicates(cache):
    """A batch with a repeated position and an odd count: the sum over entries."""
    c, _ = _get(cache, "n64_ms_poisson")
    c2 = Case(c.wl, batch=[3, 0, 7, 3, 12])
    ref = c2.oracle_grad()
    d = c2.device()
    prob = c2.problem()
    loss, gO, gP, gX = prob.loss_and_grad(d["probe"], d["obj"], d["pos"], d["pats"], d["batch"])
    prob.check()
    assert abs(loss.item() - ref["loss"]) < TOL_I * abs(ref["loss"])
    assert rel_l2(_np(gO), ref["g_object"]) < TOL_G
    assert rel_l2(_np(gP), ref["g_probe"]) < TOL_G
    assert rel_l2(_np(gX), ref["g_pos"]) < TOL_G


@pytest.mark.parametrize("N", [64, 256])
def test_edge_positions_match_oracle(N):
    """Windows on the object's first and last rows and columns, and positions
    on the rounding boundaries (delta = -0.5 exactly, delta close to +0.5):
    intensities and all gradients against the oracle."""
    wl = synth.make_small(N=N, M=2, S=2, scan=2, step=6, seed=60 + N, loss="poisson", eps=0.5)
    hi = float(wl.H - N)
    wl.positions = np.array([[0.0, 0.0], [hi, hi], [hi - 0.5, 0.25], [0.499, hi - 0.5], [-0.499, 1.0],
                             [3.5, hi - 0.499]], dtype=np.float64)
    wl.patterns = synth.make_patterns(N, len(wl.positions), 1e4, 7)
    c = Case(wl)
    ref = c.oracle_grad()
    d = c.device()
    prob = c.problem()
    I, _ = prob.forward(d["probe"], d["obj"], d["pos"], d["batch"])
    loss, gO, gP, gX = prob.loss_and_grad(d["probe"], d["obj"], d["pos"], d["pats"], d["batch"])
    prob.check()
    assert rel_l2(_np(I), ref["I"]) < TOL_I
    assert abs(loss.item() - ref["loss"]) < TOL_I * abs(ref["loss"])
    errs = dict(obj=rel_l2(_np(gO), ref["g_object"]), probe=rel_l2(_np(gP), ref["g_probe"]),
                pos=rel_l2(_np(gX), ref["g_pos"]))
    assert all(e < TOL_G for e in errs.values()), errs


@pytest.mark.parametrize("N", [64, 256])
def test_stale_workspace_is_never_read(N):
    """Columns outside the propagator's support are never read (at N = 256 the
    passes write the dead columns of the 128-byte lines that also hold live
    ones, and no consumer uses them): after a call whose detector weights are
    NaN everywhere (every work tile and checkpoint full of NaN), the next call
    on the same context still matches the oracle, so no consumer picked up a
    column it was not given."""
    from paper_2505_14372_amd._lib import PTY_ENONFINITE, PtyError
    c = Case(synth.make_small(N=N, M=2, S=3, scan=2, step=6, seed=70 + N, loss="gaussian", amp_noise=0.2))
    ref = c.oracle_grad()
    d = c.device()
    prob = c.problem()
    bad = torch.full_like(d["pats"], float("nan"))
    prob.loss_and_grad(d["probe"], d["obj"], d["pos"], bad, d["batch"])
    with pytest.raises(PtyError) as e:
        prob.check()
    assert e.value.status == PTY_ENONFINITE
    loss, gO, gP, gX = prob.loss_and_grad(d["probe"], d["obj"], d["pos"], d["pats"], d["batch"])
    prob.check()
    assert abs(loss.item() - ref["loss"]) < TOL_I * abs(ref["loss"])
    errs = dict(obj=rel_l2(_np(gO), ref["g_object"]), probe=rel_l2(_np(gP), ref["g_probe"]),
                pos=rel_l2(_np(gX), ref["g_pos"]))
    assert all(e_ < TOL_G for e_ in errs.values()), errs


def test_empty_and_oversized_batches_are_rejected():
    from paper_2505_14372_amd._lib import PTY_EINVAL, PtyError
    c = Case(synth.make_small(N=64, M=1, S=1, scan=2, step=4, seed=14, loss="gaussian"))
    d = c.device()
    prob = c.problem(max_batch=3)
    for b in (torch.zeros(0, dtype=torch.int32, device="cuda"), torch.arange(4, dtype=torch.int32, device="cuda")):
        with pytest.raises(PtyError) as e:
            prob.loss_and_grad(d["probe"], d["obj"], d["pos"], d["pats"], b)
        assert e.value.status == PTY_EINVAL
    # out-of-range position indices are a device-side bounds error, not a fault
    bad = torch.tensor([0, 99, 1], dtype=torch.int32, device="cuda")
    prob.forward(d["probe"], d["obj"], d["pos"], bad)
    from paper_2505_14372_amd._lib import PTY_EBOUNDS
    with pytest.raises(PtyError) as e:
        prob.check()
    assert e.value.status == PTY_EBOUNDS
    # unknown strategy / reduction modes are refused on a live context
    assert prob.lib.pty_set_reduction(prob.ctx, 2) == PTY_EINVAL
    assert prob.lib.pty_last_error(prob.ctx) == b"unknown reduction mode"
    assert prob.lib.pty_set_strategy(prob.ctx, 9) == PTY_EINVAL
    assert prob.lib.pty_last_error(prob.ctx) == b"unknown strategy"
    assert prob.lib.pty_set_chunk(prob.ctx, -1) == PTY_EINVAL
    assert b"chunk" in prob.lib.pty_last_error(prob.ctx)


@pytest.mark.parametrize("k", [2, 3, 7])
def test_checkpoint_recompute_matches_store_all(k):
    c = Case(synth.make_small(N=64, M=2, S=7, scan=3, step=4, seed=8, loss="poisson", eps=0.8, amp_noise=0.2))
    ref = c.oracle_grad()
    d = c.device()
    full = c.problem(checkpoint_every=1)
    part = c.problem(checkpoint_every=k)
    assert part.checkpoint_every == k
    # the same forward kernels on both sides, so the loss agrees bit for bit
    full.set_strategy("two_pass")
    part.set_strategy("two_pass")
    a = full.loss_and_grad(d["probe"], d["obj"], d["pos"], d["pats"], d["batch"])
    b = part.loss_and_grad(d["probe"], d["obj"], d["pos"], d["pats"], d["batch"])
    part.check()
    assert a[0].item() == b[0].item()
    for x, y in zip(a[1:], b[1:]):
        assert rel_l2(_np(y), _np(x)) < 1e-6
    assert rel_l2(_np(b[1]), ref["g_object"]) < TOL_G


@pytest.mark.parametrize("k", [2, 3, 7])
def test_spectral_recompute_is_bitwise_store_all(k):
    """With float checkpoints a recomputed segment runs the forward's own row
    and column passes on the same row spectra, so under the ordered reduction
    the loss and every gradient equal the store-all result bit for bit."""
    c = Case(synth.make_small(N=64, M=2, S=7, scan=3, step=4, seed=8, loss="poisson", eps=0.8, amp_noise=0.2))
    d = c.device()
    out = []
    for kk in (1, k):
        prob = c.problem(checkpoint_every=kk)
        prob.set_strategy("two_pass")
        prob.set_reduction("ordered")
        out.append(prob.loss_and_grad(d["probe"], d["obj"], d["pos"], d["pats"], d["batch"]))
        prob.check()
    assert out[0][0].item() == out[1][0].item()
    for name, x, y in zip(("object", "probe", "positions"), out[0][1:], out[1][1:]):
        assert torch.equal(x, y), name


@pytest.mark.parametrize("k,reduction", [(1, "atomic"), (7, "ordered")])
def test_many_modes_and_slices_match_oracle(k, reduction):
    """Beyond the benchmark's 8 modes and 30 slices: 12 modes, 40 slices with
    unequal gaps, stored or recomputed every 7th slice, against the oracle."""
    wl = synth.make_small(N=64, M=12, S=40, scan=3, step=4, seed=41, loss="poisson", eps=0.8, amp_noise=0.1,
                          phi_max=0.05)
    wl.dz = [float(x) for x in np.random.default_rng(41).uniform(0.5, 3.0, wl.S - 1)]
    c = Case(wl)
    ref = c.oracle_grad()
    d = c.device()
    prob = c.problem(checkpoint_every=k)
    prob.set_reduction(reduction)
    loss, gO, gP, gX = prob.loss_and_grad(d["probe"], d["obj"], d["pos"], d["pats"], d["batch"])
    prob.check()
    assert abs(loss.item() - ref["loss"]) < TOL_I * abs(ref["loss"])
    for name, got, want in (("object", gO, ref["g_object"]), ("probe", gP, ref["g_probe"]),
                            ("positions", gX, ref["g_pos"])):
        g = _np(got)
        print(f"{name}: rel L2 {rel_l2(g, want):.2e}, max {max_rel(g, want):.2e}")
        assert rel_l2(g, want) < TOL_G and max_rel(g, want) < TOL_G, name


def test_layer_blur_refused_beyond_its_slice_limit():
    """The depth blur's Gaussian runs over at most 64 slices; a deeper object
    is refused when the constraint is set, and the other constraints still are
    accepted."""
    from paper_2505_14372_amd._lib import PTY_EINVAL, PtyError
    wl = synth.make_small(N=64, M=1, S=65, scan=2, step=4, seed=42, phi_max=0.02)
    prob = Case(wl).problem()
    with pytest.raises(PtyError) as e:
        prob.set_regularizers(layer_sigma=0.7)
    assert e.value.status == PTY_EINVAL
    prob.set_regularizers(obj_lowpass_sigma=1.0)


def test_checkpoint_auto_by_budget():
    c = Case(synth.make_small(N=64, M=2, S=8, scan=2, step=4, seed=9, loss="poisson", eps=0.8))
    from paper_2505_14372_amd import api
    B = len(c.batch)
    full = api.workspace_bytes(c.N, c.M, c.S, c.H, c.W, len(c.pos), B, 1)
    prob = c.problem(checkpoint_every=0, hbm_budget=int(full * 0.85))
    assert prob.checkpoint_every > 1
    assert api.workspace_bytes(c.N, c.M, c.S, c.H, c.W, len(c.pos), B, prob.checkpoint_every) <= full * 0.85
    ref = c.oracle_grad()
    d = c.device()
    loss, gO, gP, gX = prob.loss_and_grad(d["probe"], d["obj"], d["pos"], d["pats"], d["batch"])
    assert rel_l2(_np(gO), ref["g_object"]) < TOL_G


def test_forward_save_backward_scale_and_accumulate(cache):
    c, ref = _get(cache, "n64_ms_poisson")
    d = c.device()
    prob = c.problem()
    loss, _ = prob.forward_save(d["probe"], d["obj"], d["pos"], d["pats"], d["batch"])
    gO = torch.zeros_like(d["obj"])
    gP = torch.zeros_like(d["probe"])
    gX = torch.zeros((len(c.batch), 2), dtype=torch.float32, device="cuda")
    prob.backward(2.5, gO, gP, gX)
    assert rel_l2(_np(gO), 2.5 * ref["g_object"]) < TOL_G
    assert rel_l2(_np(gP), 2.5 * ref["g_probe"]) < TOL_G
    assert rel_l2(_np(gX), 2.5 * ref["g_pos"]) < TOL_G
    # accumulate: add a second gradient of scale 1
    prob.loss_and_grad(d["probe"], d["obj"], d["pos"], d["pats"], d["batch"], g_object=gO, g_probe=gP, g_pos=gX,
                       accumulate=True)
    assert rel_l2(_np(gO), 3.5 * ref["g_object"]) < TOL_G
    assert rel_l2(_np(gX), 3.5 * ref["g_pos"]) < TOL_G
    # backward without a tape is refused
    from paper_2505_14372_amd._lib import PTY_ESTATE, PtyError
    with pytest.raises(PtyError) as e:
        prob.backward(1.0, gO, gP, gX)
    assert e.value.status == PTY_ESTATE


def test_gradient_subsets_and_dense_positions():
    """NULL gradient outputs skip that gradient and leave the others intact;
    per-position (dense) position gradients add up the entries of a batch that
    visits a position twice."""
    c = Case(synth.make_small(N=64, M=2, S=3, scan=3, step=4, seed=43, loss="amplitude", eps=0.3),
             batch=[4, 0, 4, 7, 2])
    ref = c.oracle_grad()
    d = c.device()
    prob = c.problem()
    loss, gO, gP, gX = prob.loss_and_grad(d["probe"], d["obj"], d["pos"], d["pats"], d["batch"], want=("probe",))
    prob.check()
    assert gO is None and gX is None
    assert abs(loss.item() - ref["loss"]) < TOL_I * abs(ref["loss"])
    assert rel_l2(_np(gP), ref["g_probe"]) < TOL_G
    loss, gO, gP, gX = prob.loss_and_grad(d["probe"], d["obj"], d["pos"], d["pats"], d["batch"],
                                          want=("object", "pos"), dense_pos=True)
    prob.check()
    assert gP is None and gX.shape == (c.pos.shape[0], 2)
    assert rel_l2(_np(gO), ref["g_object"]) < TOL_G
    want = np.zeros((c.pos.shape[0], 2))
    np.add.at(want, c.batch, ref["g_pos"])
    assert rel_l2(_np(gX), want) < TOL_G
    assert np.all(_np(gX)[np.setdiff1d(np.arange(c.pos.shape[0]), c.batch)] == 0)
    # loss only
    loss, gO, gP, gX = prob.loss_and_grad(d["probe"], d["obj"], d["pos"], d["pats"], d["batch"], want=())
    prob.check()
    assert gO is None and gP is None and gX is None
    assert abs(loss.item() - ref["loss"]) < TOL_I * abs(ref["loss"])


def _oracle_state(c):
    P, O, X = c.o_args()
    return dict(probe=P, object=O, positions=X)


def _run_steps(c, opt_kind, n_steps, batches):
    from paper_2505_14372_amd import api
    d = c.device()
    prob = c.problem(max_batch=max(len(b) for b in batches))
    st = api.ReconState(d["probe"].clone(), d["obj"].clone(), d["pos"].clone(), adam=(opt_kind == "adam"))
    # SGD rates large enough that each update sits well above the float32 rounding of the state
    lr = dict(object=2e-2, probe=1e-3, pos=1e-2) if opt_kind == "adam" else dict(object=1e-4, probe=1e-4, pos=1e-4)
    opt = api.Optimizer(kind=opt_kind, lr_object=lr["object"], lr_probe=lr["probe"], lr_pos=lr["pos"])
    ost = _oracle_state(c)
    oopt = dict(kind=opt_kind, lr_object=lr["object"], lr_probe=lr["probe"], lr_pos=lr["pos"])
    losses = []
    for s in range(n_steps):
        b = batches[s % len(batches)]
        loss = prob.reconstruct_step(st, d["pats"], torch.tensor(b, dtype=torch.int32, device="cuda"), opt)
        prob.check()
        ost, oloss = orc.reconstruct_step(ost, c.pats.astype(np.float64), b, c.geom, oopt)
        losses.append((loss.item(), oloss))
    return st, ost, losses, lr


def test_reconstruct_step_sgd():
    c = Case(synth.make_small(N=64, M=2, S=3, scan=3, step=4, seed=10, loss="poisson", eps=0.8, amp_noise=0.1))
    st, ost, losses, lr = _run_steps(c, "sgd", 3, [[0, 4, 8], [1, 2, 3, 5]])
    for g, o in losses:
        assert abs(g - o) < TOL_I * abs(o)
    P0, O0, X0 = c.o_args()
    # compare the accumulated updates (state - initial state)
    assert rel_l2(_np(st.object).astype(np.complex128) - O0, ost["object"] - O0) < TOL_G
    assert rel_l2(_np(st.probe).astype(np.complex128) - P0, ost["probe"] - P0) < TOL_G
    assert rel_l2(_np(st.positions) - X0, ost["positions"] - X0) < TOL_G


def test_reconstruct_step_adam():
    c = Case(synth.make_small(N=64, M=2, S=3, scan=3, step=4, seed=11, loss="poisson", eps=0.8, amp_noise=0.1))
    st, ost, losses, lr = _run_steps(c, "adam", 3, [[0, 4, 8], [1, 2, 3, 5]])
    assert st.step == 3 and ost["t"] == 3
    for g, o in losses:
        assert abs(g - o) < TOL_I * abs(o)
    P0, O0, X0 = c.o_args()
    for key, got, init in (("object", _np(st.object), O0), ("probe", _np(st.probe), P0),
                           ("positions", _np(st.positions), X0)):
        du_g = got.astype(np.complex128 if np.iscomplexobj(init) else np.float64) - init
        du_o = ost[key] - init
        # Adam's first steps move each component by about lr * sign(g): components whose
        # gradient is tiny may legitimately differ in sign between FP32 and FP64.
        err = np.abs(du_g - du_o)
        assert np.max(err) <= 3 * lr[key.replace("positions", "pos")] * (1 + 1e-3) + 1e-6
        assert rel_l2(du_g, du_o) < 2e-2, (key, rel_l2(du_g, du_o))


def test_adam_update_matches_oracle_on_the_gpu_gradient():
    """The optimiser alone, to tight bounds: at each of three Adam steps the
    gradient the GPU computes at its current state (ordered reduction, so the
    step's own gradient has the same bits) is fed with the GPU's moments to the
    oracle's Adam in FP64; the GPU state after reconstruct_step must agree
    element by element to 1e-5 of each component's update (plus one float32
    rounding of the state) and the moments to the float rounding bound of
    their update."""
    from paper_2505_14372_amd import api
    c = Case(synth.make_small(N=64, M=2, S=3, scan=3, step=4, seed=11, loss="poisson", eps=0.8, amp_noise=0.1))
    d = c.device()
    prob = c.problem()
    prob.set_reduction("ordered")
    st = api.ReconState(d["probe"].clone(), d["obj"].clone(), d["pos"].clone(), adam=True)
    lr = dict(object=2e-2, probe=1e-3, positions=1e-2)
    opt = api.Optimizer(kind="adam", lr_object=lr["object"], lr_probe=lr["probe"], lr_pos=lr["positions"])
    batches = [[0, 4, 8], [1, 2, 3, 5], [6, 7, 0]]
    f64 = lambda t: _np(t).astype(np.complex128 if t.is_complex() else np.float64)  # noqa: E731
    for k, b in enumerate(batches):
        bt = torch.tensor(b, dtype=torch.int32, device="cuda")
        _, gO, gP, gX = prob.loss_and_grad(st.probe, st.object, st.positions, d["pats"], bt, dense_pos=True)
        before = {key: (f64(getattr(st, key)), _np(getattr(st, "m_" + mk)).astype(np.float64),
                        _np(getattr(st, "v_" + mk)).astype(np.float64))
                  for key, mk in (("object", "object"), ("probe", "probe"), ("positions", "pos"))}
        grads = dict(object=f64(gO), probe=f64(gP), positions=f64(gX))
        prob.reconstruct_step(st, d["pats"], bt, opt)
        prob.check()
        assert st.step == k + 1
        for key, mk in (("object", "object"), ("probe", "probe"), ("positions", "pos")):
            th0, m0, v0 = before[key]
            th_o, m_o, v_o = orc.adam_update(th0, grads[key], m0, v0, k + 1, lr[key])
            th_g = f64(getattr(st, key))
            m_g = _np(getattr(st, "m_" + mk)).astype(np.float64)
            v_g = _np(getattr(st, "v_" + mk)).astype(np.float64)
            # compare per real component; the oracle's state rounded to float32 as the GPU stores it
            th_o32 = _real_components(th_o).astype(np.float32)
            got, want, init = _real_components(th_g), th_o32.astype(np.float64), _real_components(th0)
            ulp = np.spacing(np.abs(th_o32)).astype(np.float64)
            du = np.abs(_real_components(th_o) - init)
            bad = np.abs(got - want) > 1e-5 * du + ulp
            assert not bad.any(), (k, key, int(bad.sum()), float(np.max(np.abs(got - want))))
            # the moments to the rounding of their float update: every operation of
            # b m + (1 - b) g (and of the constants) errs by at most the unit
            # roundoff u = 2^-24 of the magnitudes it adds, so |error| <= 4 u
            # (|b1 m0| + |c1 g|) however much the two terms cancel
            u = 2.0 ** -24
            g_re = _real_components(grads[key])
            m_tol = 4 * u * (0.9 * np.abs(m0) + 0.1 * np.abs(g_re)) + 1e-30
            v_tol = 4 * u * (0.999 * np.abs(v0) + 0.001 * g_re * g_re) + 1e-37
            assert np.all(np.abs(m_g - m_o) <= m_tol), (k, key, "m", float(np.max(np.abs(m_g - m_o) / m_tol)))
            assert np.all(np.abs(v_g - v_o) <= v_tol), (k, key, "v", float(np.max(np.abs(v_g - v_o) / v_tol)))
            moved = float(np.max(du))
            print(f"step {k + 1} {key}: max update {moved:.3e}, max diff {float(np.max(np.abs(got - want))):.3e}")
            assert moved > 0.5 * lr[key]


@pytest.mark.parametrize("N", [192, 256])
@pytest.mark.parametrize("kind", ["adam", "sgd"])
def test_group_step_large_windows(N, kind):
    """Grouped steps at N = 192 and 256 (the 24-values-per-lane adjoint row pass
    that re-reads the object row, and the 16 x 16 line split): two
    reconstructions with different modes, slices, object sizes and losses in
    shared launches give, under the ordered reduction, the bits of their single
    steps; an SGD step also matches the oracle's step."""
    from paper_2505_14372_amd import api
    step_px = 11 if N == 192 else 8
    cases = [Case(synth.make_small(N=N, M=2, S=3, scan=2, step=step_px, seed=90 + N, loss="poisson", eps=0.8,
                                   phi_max=0.1, dose=1e5)),
             Case(synth.make_small(N=N, M=1, S=2, scan=3, step=step_px - 3, seed=91 + N, loss="amplitude",
                                   eps=0.3, phi_max=0.1, dose=1e5))]
    batches = [[0, 3, 1], [4, 0, 8, 2, 6]]
    if kind == "adam":
        opt = api.Optimizer(kind="adam", lr_object=1e-2, lr_probe=1e-3, lr_pos=1e-2)
    else:
        opt = api.Optimizer(kind="sgd", lr_object=1e-4, lr_probe=1e-6, lr_pos=1e-5)
    runs = []
    for q, c in enumerate(cases):
        d = c.device()
        ps, pg = c.problem(max_batch=16), c.problem(max_batch=16)
        ps.set_reduction("ordered")
        pg.set_reduction("ordered")
        single = api.ReconState(d["probe"].clone(), d["obj"].clone(), d["pos"].clone(), adam=kind == "adam")
        grouped = api.ReconState(d["probe"].clone(), d["obj"].clone(), d["pos"].clone(), adam=kind == "adam")
        runs.append((c, ps, pg, d, single, grouped, torch.tensor(batches[q], dtype=torch.int32, device="cuda")))
    print(f"grouped N={N} {kind}: " + ", ".join(f"M={c.M} S={c.S} H={c.H} B={len(b)}" for c, *_, b in runs),
          flush=True)
    grp = api.Group(N, max_items=16, max_tiles=32, max_ckpt_tiles=64)
    n_steps = 2 if kind == "adam" else 1
    for _ in range(n_steps):
        entries = []
        for c, ps, pg, d, single, grouped, b in runs:
            ps.reconstruct_step(single, d["pats"], b, opt)
            entries.append((pg, grouped, d["pats"], b, opt, torch.zeros(1, dtype=torch.float64, device="cuda")))
        grp.step(entries)
    torch.cuda.synchronize()
    for c, ps, pg, d, single, grouped, b in runs:
        assert torch.equal(grouped.object, single.object)
        assert torch.equal(grouped.probe, single.probe)
        assert torch.equal(grouped.positions, single.positions)
        if kind == "sgd":
            P0, O0, X0 = c.o_args()
            ost, _ = orc.reconstruct_step(dict(probe=P0, object=O0, positions=X0), c.pats.astype(np.float64),
                                          list(_np(b)), c.geom, dict(kind="sgd", lr_object=opt.lr_object,
                                                                      lr_probe=opt.lr_probe, lr_pos=opt.lr_pos))
            for got, init, want in ((grouped.object, O0, ost["object"]), (grouped.probe, P0, ost["probe"]),
                                    (grouped.positions, X0, ost["positions"])):
                du_g = _np(got).astype(np.complex128 if np.iscomplexobj(init) else np.float64) - init
                # the state is stored in float32, so each component of the update is
                # resolved to one float32 spacing of the new value: the bar is the
                # gradient tolerance on the update plus that resolution
                res = np.linalg.norm(np.spacing(_real_components(want).astype(np.float32)).astype(np.float64))
                err = np.linalg.norm(_real_components(du_g) - _real_components(want - init))
                assert err <= TOL_G * np.linalg.norm(_real_components(want - init)) + res, \
                    (rel_l2(du_g, want - init), err, res)


def test_bounds_flag_skips_the_window():
    c = Case(synth.make_small(N=64, M=1, S=2, scan=2, step=4, seed=12, loss="gaussian"))
    c.pos[1] = [c.H - 40.0, 3.0]      # window leaves the object
    d = c.device()
    prob = c.problem()
    I, _ = prob.forward(d["probe"], d["obj"], d["pos"], d["batch"])
    from paper_2505_14372_amd._lib import PTY_EBOUNDS, PtyError
    with pytest.raises(PtyError) as e:
        prob.check()
    assert e.value.status == PTY_EBOUNDS
    prob.check()      # the flag is cleared
    ok = [0, 2, 3]
    ref = c.oracle_forward(batch=ok)
    assert rel_l2(_np(I)[ok], ref) < TOL_I
    assert np.all(_np(I)[1] == 0)


def test_nonfinite_flag():
    c = Case(synth.make_small(N=64, M=1, S=1, scan=2, step=4, seed=13, loss="poisson", eps=0.8))
    c.pats[2, 5, 5] = np.nan
    d = c.device()
    prob = c.problem()
    prob.loss_and_grad(d["probe"], d["obj"], d["pos"], d["pats"], d["batch"])
    from paper_2505_14372_amd._lib import PTY_ENONFINITE, PtyError
    with pytest.raises(PtyError) as e:
        prob.check()
    assert e.value.status == PTY_ENONFINITE


@pytest.mark.parametrize("name", ["n64_ms_poisson", "n128_tilt_mask_dz", "n192_ms_anscombe", "n256_ms_gaussian",
                                  "n64_wide_object"])
def test_ordered_reduction_is_bitwise_repeatable(cache, name):
    """The ordered object-gradient reduction matches the oracle, agrees with the
    atomic one to rounding, and gives identical bits on a repeated call."""
    c, ref = _get(cache, name)
    print(f"case {name} N={c.N} M={c.M} S={c.S} B={len(c.batch)}", flush=True)
    d = c.device()
    prob = c.problem()
    _, gO_at, _, _ = prob.loss_and_grad(d["probe"], d["obj"], d["pos"], d["pats"], d["batch"])
    prob.set_reduction("ordered")
    runs = [prob.loss_and_grad(d["probe"], d["obj"], d["pos"], d["pats"], d["batch"]) for _ in range(2)]
    prob.check()
    (l1, gO1, gP1, gX1), (l2, gO2, gP2, gX2) = runs
    assert l1.item() == l2.item()
    assert torch.equal(gO1, gO2) and torch.equal(gP1, gP2) and torch.equal(gX1, gX2)
    errs = dict(obj=rel_l2(_np(gO1), ref["g_object"]), probe=rel_l2(_np(gP1), ref["g_probe"]),
                pos=rel_l2(_np(gX1), ref["g_pos"]))
    print(errs)
    assert all(e < TOL_G for e in errs.values()), errs
    assert rel_l2(_np(gO1), _np(gO_at)) < 1e-5


def test_ordered_reduction_overrides_the_resident_strategy(cache):
    """RESIDENT with the ordered reduction runs the two-pass kernels: repeatable
    bits, equal to TWO_PASS with the ordered reduction."""
    c, ref = _get(cache, "n128_ms_poisson")
    d = c.device()
    out = {}
    for strat in ("resident", "two_pass"):
        prob = c.problem()
        prob.set_strategy(strat)
        prob.set_reduction("ordered")
        out[strat] = [prob.loss_and_grad(d["probe"], d["obj"], d["pos"], d["pats"], d["batch"])[1]
                      for _ in range(2)]
        prob.check()
    assert torch.equal(out["resident"][0], out["resident"][1])
    assert torch.equal(out["resident"][0], out["two_pass"][0])
    assert rel_l2(_np(out["resident"][0]), ref["g_object"]) < TOL_G


@pytest.mark.parametrize("k,chunk", [(1, 4), (2, 0), (3, 5)])
def test_ordered_reduction_with_chunks_and_recompute(cache, k, chunk):
    """Chunked schedules and recomputed entry waves under the ordered reduction:
    oracle parity, and identical bits on a repeated call."""
    c, ref = _get(cache, "n64_ms_poisson")
    d = c.device()
    prob = c.problem(checkpoint_every=k)
    prob.set_strategy("two_pass")
    prob.set_reduction("ordered")
    prob.set_chunk(chunk)
    runs = [prob.loss_and_grad(d["probe"], d["obj"], d["pos"], d["pats"], d["batch"]) for _ in range(2)]
    prob.check()
    assert torch.equal(runs[0][1], runs[1][1])
    assert rel_l2(_np(runs[0][1]), ref["g_object"]) < TOL_G
    assert abs(runs[0][0].item() - ref["loss"]) < TOL_I * abs(ref["loss"])


@pytest.mark.parametrize("kind", ["sgd", "adam"])
def test_group_step_matches_single_steps(kind):
    """Two reconstructions of one window size (different M, S, object size and
    loss) stepped in shared launches equal their separate steps."""
    from paper_2505_14372_amd import api
    cases = [Case(synth.make_small(N=64, M=2, S=3, scan=3, step=4, seed=20, loss="poisson", eps=0.8)),
             Case(synth.make_small(N=64, M=1, S=5, scan=4, step=5, seed=21, loss="amplitude", eps=0.3))]
    batches = [[0, 2, 4, 8], [1, 3, 5, 6, 9, 15]]
    if kind == "adam":
        opt = api.Optimizer(kind="adam", lr_object=1e-2, lr_probe=1e-3, lr_pos=1e-2)
    else:
        opt = api.Optimizer(kind="sgd", lr_object=1e-4, lr_probe=1e-6, lr_pos=1e-5)
    singles, grouped, probs = [], [], []
    for c in cases:
        d = c.device()
        singles.append(api.ReconState(d["probe"].clone(), d["obj"].clone(), d["pos"].clone(), adam=kind == "adam"))
        grouped.append(api.ReconState(d["probe"].clone(), d["obj"].clone(), d["pos"].clone(), adam=kind == "adam"))
        probs.append((c.problem(max_batch=16), c.problem(max_batch=0), d))
    grp = api.Group(64, max_items=64, max_tiles=128, max_ckpt_tiles=512)
    losses = []
    for step in range(2):
        entries = []
        for q, c in enumerate(cases):
            p_single, p_group, d = probs[q]
            b = torch.tensor(batches[q], dtype=torch.int32, device="cuda")
            ls = p_single.reconstruct_step(singles[q], d["pats"], b, opt)
            lg = torch.zeros(1, dtype=torch.float64, device="cuda")
            entries.append((p_group, grouped[q], d["pats"], b, opt, lg))
            losses.append((ls, lg))
        grp.step(entries)
    torch.cuda.synchronize()
    for ls, lg in losses:
        assert abs(ls.item() - lg.item()) <= 1e-6 * abs(ls.item())
    for q in range(2):
        if kind == "adam":
            assert grouped[q].step == singles[q].step == 2
        for a, b in ((grouped[q].object, singles[q].object), (grouped[q].probe, singles[q].probe),
                     (grouped[q].positions, singles[q].positions)):
            if kind == "sgd":
                assert max_rel(_np(a), _np(b)) < 1e-5
            else:
                assert rel_l2(_np(a), _np(b)) < 1e-4


def test_group_step_at_the_request_limit():
    """Sixteen reconstructions (the request-table limit) of mixed modes, slices
    and object sizes in one grouped step give, under the ordered reduction, the
    bits of their single steps; a seventeenth is refused on the host."""
    from paper_2505_14372_amd import api
    from paper_2505_14372_amd._lib import PTY_EINVAL, PtyError
    opt = api.Optimizer(kind="adam", lr_object=1e-2, lr_probe=1e-3, lr_pos=1e-2)
    runs = []
    for q in range(17):
        c = Case(synth.make_small(N=64, M=1 + q % 3, S=1 + q % 4, scan=2 + q % 2, step=4 + q % 3, seed=70 + q,
                                  loss=("poisson", "amplitude", "gaussian")[q % 3], eps=0.5))
        d = c.device()
        ps, pg = c.problem(max_batch=16), c.problem(max_batch=16)
        ps.set_reduction("ordered")
        pg.set_reduction("ordered")
        b = torch.arange(len(c.batch), dtype=torch.int32, device="cuda")
        single = api.ReconState(d["probe"].clone(), d["obj"].clone(), d["pos"].clone(), adam=True)
        grouped = api.ReconState(d["probe"].clone(), d["obj"].clone(), d["pos"].clone(), adam=True)
        runs.append((ps, pg, d, b, single, grouped))
    grp = api.Group(64, max_items=256, max_tiles=1024, max_ckpt_tiles=4096)
    entries = [(pg, grouped, d["pats"], b, opt, torch.zeros(1, dtype=torch.float64, device="cuda"))
               for ps, pg, d, b, single, grouped in runs]
    with pytest.raises(PtyError) as e:
        grp.step(entries)
    assert e.value.status == PTY_EINVAL
    grp.step(entries[:16])
    for ps, pg, d, b, single, grouped in runs[:16]:
        ps.reconstruct_step(single, d["pats"], b, opt)
    torch.cuda.synchronize()
    for ps, pg, d, b, single, grouped in runs[:16]:
        assert torch.equal(grouped.object, single.object)
        assert torch.equal(grouped.probe, single.probe)
        assert torch.equal(grouped.positions, single.positions)


def test_ordered_group_step_gives_the_single_step_bits():
    """Under the ordered reduction a reconstruction's object, probe and
    positions after Adam steps have the same bits alone and in grouped steps."""
    from paper_2505_14372_amd import api
    cases = [Case(synth.make_small(N=64, M=2, S=3, scan=3, step=4, seed=20, loss="poisson", eps=0.8)),
             Case(synth.make_small(N=64, M=1, S=5, scan=4, step=5, seed=21, loss="amplitude", eps=0.3))]
    batches = [[0, 2, 4, 8], [1, 3, 5, 6, 9, 15]]
    opt = api.Optimizer(kind="adam", lr_object=1e-2, lr_probe=1e-3, lr_pos=1e-2)
    singles, grouped, probs = [], [], []
    for c in cases:
        d = c.device()
        singles.append(api.ReconState(d["probe"].clone(), d["obj"].clone(), d["pos"].clone(), adam=True))
        grouped.append(api.ReconState(d["probe"].clone(), d["obj"].clone(), d["pos"].clone(), adam=True))
        ps, pg = c.problem(max_batch=16), c.problem(max_batch=16)
        ps.set_reduction("ordered")
        pg.set_reduction("ordered")
        probs.append((ps, pg, d))
    grp = api.Group(64, max_items=64, max_tiles=128, max_ckpt_tiles=512)
    for step in range(2):
        entries = []
        for q, c in enumerate(cases):
            ps, pg, d = probs[q]
            b = torch.tensor(batches[q], dtype=torch.int32, device="cuda")
            ps.reconstruct_step(singles[q], d["pats"], b, opt)
            entries.append((pg, grouped[q], d["pats"], b, opt, torch.zeros(1, dtype=torch.float64, device="cuda")))
        grp.step(entries)
    torch.cuda.synchronize()
    for q in range(2):
        assert torch.equal(grouped[q].object, singles[q].object)
        assert torch.equal(grouped[q].probe, singles[q].probe)
        assert torch.equal(grouped[q].positions, singles[q].positions)


@pytest.mark.parametrize("name,k", [("n64_ms_poisson", 1), ("n128_ms_poisson", 1), ("n256_ms_gaussian", 1),
                                    ("n64_ms_poisson", 2)])
def test_half_checkpoints_parity(cache, name, k):
    """Entry waves stored as IEEE halves (with and without recompute): loss and
    intensities are unchanged, gradients stay within the 1e-3 bar."""
    c, ref = _get(cache, name)
    d = c.device()
    prob = c.problem(checkpoint_every=k, checkpoint_half=True)
    assert prob.checkpoint_half
    loss, gO, gP, gX = prob.loss_and_grad(d["probe"], d["obj"], d["pos"], d["pats"], d["batch"])
    prob.check()
    assert abs(loss.item() - ref["loss"]) < TOL_I * abs(ref["loss"])
    errs = dict(obj=rel_l2(_np(gO), ref["g_object"]), probe=rel_l2(_np(gP), ref["g_probe"]),
                pos=rel_l2(_np(gX), ref["g_pos"]))
    print(errs)
    assert all(e < TOL_G for e in errs.values()), errs


def test_regularized_step_matches_oracle():
    """reconstruct_step with every cost regularizer and every constraint (Sec. 3.4)."""
    from paper_2505_14372_amd import api
    # a non-square object (76 x 97) so that the in-plane stencils cannot swap their axes unnoticed
    c = Case(_widen(synth.make_small(N=64, M=2, S=4, scan=3, step=4, seed=30, loss="poisson", eps=0.8,
                                     amp_noise=0.3), 21, seed=30, shift=11.0))
    d = c.device()
    prob = c.problem(max_batch=9)
    k = np.fft.fftfreq(64) * 64
    support = (k[:, None] ** 2 + k[None, :] ** 2) <= 20 ** 2
    reg = dict(obj_l2=3.0, probe_l2=0.02, obj_l1=2.0, obj_tikhonov=5.0, obj_tv=4.0, layers_tikhonov=6.0,
               layers_tv=3.0, tv_delta=0.05)
    con = dict(amp_min=0.75, amp_max=0.98, probe_support=support, layer_sigma=0.8)
    prob.set_regularizers(**reg, amp_range=(con["amp_min"], con["amp_max"]), probe_support=support,
                          layer_sigma=con["layer_sigma"])
    st = api.ReconState(d["probe"].clone(), d["obj"].clone(), d["pos"].clone(), adam=False)
    lr = dict(object=2e-4, probe=1e-4, pos=1e-4)
    opt = api.Optimizer(kind="sgd", lr_object=lr["object"], lr_probe=lr["probe"], lr_pos=lr["pos"])
    P0, O0, X0 = c.o_args()
    ost = dict(probe=P0, object=O0, positions=X0)
    oopt = dict(kind="sgd", lr_object=lr["object"], lr_probe=lr["probe"], lr_pos=lr["pos"], reg=reg, con=con)
    for b in ([0, 3, 5, 8], [1, 2, 4, 6, 7]):
        loss = prob.reconstruct_step(st, d["pats"], torch.tensor(b, dtype=torch.int32, device="cuda"), opt)
        prob.check()
        ost, oloss = orc.reconstruct_step(ost, c.pats.astype(np.float64), b, c.geom, oopt)
        assert abs(loss.item() - oloss) < 1e-4 * abs(oloss), (loss.item(), oloss)
    for key, got in (("object", st.object), ("probe", st.probe), ("positions", st.positions)):
        g = _np(got).astype(np.complex128 if key != "positions" else np.float64)
        assert rel_l2(g, ost[key]) < 1e-5, (key, rel_l2(g, ost[key]))
    # the constraints hold on the GPU state
    a = np.abs(_np(st.object))
    assert a.min() >= 0.75 - 1e-5 and a.max() <= 0.98 + 1e-5
    spec = np.fft.fft2(_np(st.probe))
    assert np.max(np.abs(spec[:, ~support])) < 1e-4 * np.max(np.abs(spec))


def test_phase_regularizers_match_oracle():
    """reconstruct_step with the object-phase L1, the probe phase-plate
    Tikhonov and TV costs and the real-space probe support (Sec. 3.4): the
    group loss (detector plus costs) to 1e-4 and the SGD updates of object and
    probe to the gradient bar (plus the float32 resolution of the state)."""
    from paper_2505_14372_amd import api
    c = Case(synth.make_small(N=64, M=2, S=3, scan=3, step=4, seed=33, loss="poisson", eps=0.8, amp_noise=0.2))
    d = c.device()
    prob = c.problem(max_batch=9)
    yy, xx = np.mgrid[:64, :64]
    mask_r = ((yy - 32) ** 2 + (xx - 32) ** 2 <= 26 ** 2) | ((yy < 20) & (xx < 20))
    reg = dict(obj_phase_l1=4.0, probe_phase_tikhonov=0.3, probe_phase_tv=0.2, tv_delta=0.05)
    con = dict(probe_support_real=mask_r)
    prob.set_regularizers(**reg, probe_support_real=mask_r)
    st = api.ReconState(d["probe"].clone(), d["obj"].clone(), d["pos"].clone(), adam=False)
    lr = dict(object=2e-3, probe=2e-4, pos=0.0)
    opt = api.Optimizer(kind="sgd", lr_object=lr["object"], lr_probe=lr["probe"], lr_pos=lr["pos"])
    P0, O0, X0 = c.o_args()
    ost = dict(probe=P0, object=O0, positions=X0)
    oopt = dict(kind="sgd", lr_object=lr["object"], lr_probe=lr["probe"], lr_pos=lr["pos"], reg=reg, con=con)
    b = [0, 2, 4, 5, 8]
    loss = prob.reconstruct_step(st, d["pats"], torch.tensor(b, dtype=torch.int32, device="cuda"), opt)
    prob.check()
    ost, oloss = orc.reconstruct_step(ost, c.pats.astype(np.float64), b, c.geom, oopt)
    creg, _, _ = orc.regularization(O0, P0, reg)
    print(f"loss {loss.item():.6e} oracle {oloss:.6e} (costs {creg:.4e})")
    assert creg > 1e-3 * abs(oloss)
    assert abs(loss.item() - oloss) < 1e-4 * abs(oloss), (loss.item(), oloss)
    for key, got, init in (("object", st.object, O0), ("probe", st.probe, P0)):
        want = ost[key]
        du_g = _np(got).astype(np.complex128) - init
        res = np.linalg.norm(np.spacing(_real_components(want).astype(np.float32)).astype(np.float64))
        err = np.linalg.norm(_real_components(du_g) - _real_components(want - init))
        print(key, rel_l2(du_g, want - init), err, res)
        assert err <= TOL_G * np.linalg.norm(_real_components(want - init)) + res, (key, err, res)
    # the real-space support holds exactly on the GPU state
    assert np.all(_np(st.probe)[:, ~mask_r] == 0)


def test_tiny_object_pixels_keep_finite_gradients_and_phases():
    """Object pixels of amplitude 1e-20 and 1e-24, where |O|^2 underflows in
    float: the object-phase L1 and L1 gradients (w i O / |O|^2 and
    w (O - 1) / |O - 1|, Sec. 3.4) stay finite and match the oracle's FP64
    values, and the amplitude clamp keeps each pixel's phase."""
    from paper_2505_14372_amd import api
    wl = synth.make_small(N=64, M=1, S=2, scan=2, step=4, seed=35, loss="gaussian", amp_noise=0.2)
    c = Case(wl)
    rng = np.random.default_rng(35)
    ys, xs = rng.integers(0, c.H, 12), rng.integers(0, c.W, 12)
    amp = np.where(np.arange(12) % 2 == 0, 1e-20, 1e-24)
    ph = rng.uniform(-3.0, 3.0, 12)
    c.obj[0, ys, xs] = (amp * np.exp(1j * ph)).astype(np.complex64)
    d = c.device()
    P0, O0, X0 = c.o_args()
    b = [0, 1, 2, 3]
    bt = torch.tensor(b, dtype=torch.int32, device="cuda")
    # (1) the phase L1 and L1 gradients at the tiny pixels: one SGD step
    prob = c.problem(max_batch=4)
    reg = dict(obj_phase_l1=0.5, obj_l1=0.25)
    prob.set_regularizers(**reg)
    st = api.ReconState(d["probe"].clone(), d["obj"].clone(), d["pos"].clone(), adam=False)
    lr = 1e-3
    prob.reconstruct_step(st, d["pats"], bt, api.Optimizer(kind="sgd", lr_object=lr, lr_probe=0.0, lr_pos=0.0))
    prob.check()
    ost, _ = orc.reconstruct_step(dict(probe=P0, object=O0, positions=X0), c.pats.astype(np.float64), b, c.geom,
                                  dict(kind="sgd", lr_object=lr, lr_probe=0.0, lr_pos=0.0, reg=reg))
    got = _np(st.object).astype(np.complex128)
    want = ost["object"]
    assert np.all(np.isfinite(got))
    tiny = got[0, ys, xs], want[0, ys, xs]
    print("tiny pixels after the step", np.abs(tiny[0]).max(), max_rel(tiny[0], tiny[1]))
    assert np.abs(tiny[1]).min() > 1e14          # the phase-L1 step w lr / |O| dominates there
    assert max_rel(tiny[0], tiny[1]) < 1e-5
    rest = np.ones(got.shape, bool)
    rest[0, ys, xs] = False
    du_g, du_w = got[rest] - O0[rest], want[rest] - O0[rest]
    res = np.linalg.norm(np.spacing(_real_components(want[rest]).astype(np.float32)).astype(np.float64))
    assert np.linalg.norm(_real_components(du_g - du_w)) <= TOL_G * np.linalg.norm(_real_components(du_w)) + res
    prob.close()
    # (2) the amplitude clamp alone (no update): the tiny pixels become amp_min with their phase
    prob = c.problem(max_batch=4)
    prob.set_regularizers(amp_range=(0.5, 2.0))
    st = api.ReconState(d["probe"].clone(), d["obj"].clone(), d["pos"].clone(), adam=False)
    prob.reconstruct_step(st, d["pats"], bt, api.Optimizer(kind="sgd", lr_object=0.0, lr_probe=0.0, lr_pos=0.0))
    prob.check()
    ost, _ = orc.reconstruct_step(dict(probe=P0, object=O0, positions=X0), c.pats.astype(np.float64), b, c.geom,
                                  dict(kind="sgd", lr_object=0.0, lr_probe=0.0, lr_pos=0.0,
                                       con=dict(amp_min=0.5, amp_max=2.0)))
    got = _np(st.object).astype(np.complex128)
    assert max_rel(got, ost["object"]) < 1e-6
    assert np.allclose(got[0, ys, xs], 0.5 * np.exp(1j * np.angle(c.obj[0, ys, xs].astype(np.complex128))),
                       rtol=0, atol=1e-6)
    prob.close()


def test_object_spectrum_l1_matches_oracle():
    """reconstruct_step with the object spectral L1 (Sec. 3.4) on a non-square
    object whose sides (76 x 97) are not powers of two: loss to 1e-4 and the
    SGD update of the object to the gradient bar."""
    from paper_2505_14372_amd import api
    c = Case(_widen(synth.make_small(N=64, M=1, S=2, scan=3, step=4, seed=34, loss="amplitude", amp_noise=0.2),
                    21, seed=34, shift=11.0))
    d = c.device()
    prob = c.problem(max_batch=9)
    reg = dict(obj_spectrum_l1=0.5)
    prob.set_regularizers(**reg)
    st = api.ReconState(d["probe"].clone(), d["obj"].clone(), d["pos"].clone(), adam=False)
    lr = dict(object=2e-3, probe=0.0, pos=0.0)
    opt = api.Optimizer(kind="sgd", lr_object=lr["object"], lr_probe=0.0, lr_pos=0.0)
    P0, O0, X0 = c.o_args()
    oopt = dict(kind="sgd", lr_object=lr["object"], lr_probe=0.0, lr_pos=0.0, reg=reg)
    b = [0, 1, 4, 7]
    loss = prob.reconstruct_step(st, d["pats"], torch.tensor(b, dtype=torch.int32, device="cuda"), opt)
    prob.check()
    ost, oloss = orc.reconstruct_step(dict(probe=P0, object=O0, positions=X0), c.pats.astype(np.float64), b,
                                      c.geom, oopt)
    creg, gR, _ = orc.regularization(O0, P0, reg)
    print(f"loss {loss.item():.6e} oracle {oloss:.6e} (cost {creg:.4e})")
    assert creg > 1e-2 * abs(oloss)
    assert abs(loss.item() - oloss) < 1e-4 * abs(oloss), (loss.item(), oloss)
    want = ost["object"]
    du_g = _np(st.object).astype(np.complex128) - O0
    res = np.linalg.norm(np.spacing(_real_components(want).astype(np.float32)).astype(np.float64))
    err = np.linalg.norm(_real_components(du_g) - _real_components(want - O0))
    print(rel_l2(du_g, want - O0), err, res)
    assert err <= TOL_G * np.linalg.norm(_real_components(want - O0)) + res, (err, res)


def test_lowpass_and_deramp_constraints_match_oracle():
    """reconstruct_step with the object low pass and the phase deramp (Sec. 3.4)
    on an odd-sized object that carries an affine phase ramp per slice."""
    from paper_2505_14372_amd import api
    wl = _widen(synth.make_small(N=64, M=2, S=3, scan=5, step=5, seed=31, loss="amplitude", amp_noise=0.2),
                14, seed=31, shift=6.0)
    S, H, W = wl.obj.shape
    y, x = np.mgrid[:H, :W]
    wl.obj = wl.obj * np.exp(1j * (0.3 + 0.02 * np.arange(1, S + 1)[:, None, None] * y
                                  - 0.03 * np.arange(1, S + 1)[:, None, None] * x))
    c = Case(wl)
    d = c.device()
    prob = c.problem(max_batch=len(c.batch))
    con = dict(layer_sigma=0.7, obj_lowpass_sigma=1.5, phase_deramp=1)
    prob.set_regularizers(layer_sigma=0.7, obj_lowpass_sigma=1.5, phase_deramp=True)
    st = api.ReconState(d["probe"].clone(), d["obj"].clone(), d["pos"].clone(), adam=False)
    opt = api.Optimizer(kind="sgd", lr_object=1e-4, lr_probe=1e-5, lr_pos=0.0)
    P0, O0, X0 = c.o_args()
    ost = dict(probe=P0, object=O0, positions=X0)
    oopt = dict(kind="sgd", lr_object=1e-4, lr_probe=1e-5, lr_pos=0.0, con=con)
    for b in ([0, 7, 12, 20], list(range(1, 25, 2))):
        loss = prob.reconstruct_step(st, d["pats"], torch.tensor(b, dtype=torch.int32, device="cuda"), opt)
        prob.check()
        ost, oloss = orc.reconstruct_step(ost, c.pats.astype(np.float64), b, c.geom, oopt)
        assert abs(loss.item() - oloss) < 1e-4 * abs(oloss), (loss.item(), oloss)
        for key, got in (("object", st.object), ("probe", st.probe)):
            e = rel_l2(_np(got).astype(np.complex128), ost[key])
            assert e < 1e-5, (key, e)
    # the ramp is gone: the pair sums of every slice are real and positive
    Og = _np(st.object).astype(np.complex128)
    for Oi in Og:
        z = np.sum(Oi[:, 1:] * np.conj(Oi[:, :-1]))
        assert abs(np.angle(z)) < 1e-5


@pytest.mark.parametrize("strategy", ["two_pass", "resident"])
@pytest.mark.parametrize("name", ["n64_spoa_amp", "n64_ms_poisson", "n128_ms_poisson", "n128_tilt_mask_dz"])
def test_both_strategies_match_oracle(cache, name, strategy):
    """N = 64, 128: the two-pass kernels and the LDS-resident chains both match
    the oracle (intensities, loss, gradients), also with half checkpoints."""
    c, ref = _get(cache, name)
    d = c.device()
    for half in (False, True):
        prob = c.problem(checkpoint_half=half)
        prob.set_strategy(strategy)
        I, lf = prob.forward(d["probe"], d["obj"], d["pos"], d["batch"], patterns=d["pats"])
        loss, gO, gP, gX = prob.loss_and_grad(d["probe"], d["obj"], d["pos"], d["pats"], d["batch"])
        prob.check()
        assert rel_l2(_np(I), ref["I"]) < TOL_I
        assert abs(loss.item() - ref["loss"]) < TOL_I * abs(ref["loss"])
        errs = dict(obj=rel_l2(_np(gO), ref["g_object"]), probe=rel_l2(_np(gP), ref["g_probe"]),
                    pos=rel_l2(_np(gX), ref["g_pos"]))
        print(strategy, half, errs)
        assert all(e < TOL_G for e in errs.values()), errs


@pytest.mark.parametrize("N,loss,eps,ck_every,red", [(64, "amplitude", 0.0, 1, "atomic"),
                                                     (64, "poisson", 0.8, 2, "atomic"),
                                                     (128, "anscombe", 0.1, 1, "atomic"),
                                                     (192, "amplitude", 0.0, 3, "atomic"),
                                                     (128, "poisson", 0.8, 1, "ordered")])
def test_epie_step_matches_oracle(N, loss, eps, ck_every, red):
    """The ePIE / 3PIE engine (Sec. 3.3): the summed object update and the
    averaged probe update of two consecutive group steps, and the state after
    them, against the oracle (objects with amplitude below 1, so the wave
    normalisers differ from 1; recomputed segments when ck_every > 1)."""
    from paper_2505_14372_amd import api
    c = Case(_widen(synth.make_small(N=N, M=2, S=4, scan=3, step=5, seed=40 + N, loss=loss, eps=eps,
                                     amp_noise=0.3), 9, seed=40 + N, shift=4.0))
    d = c.device()
    prob = c.problem(max_batch=len(c.batch), checkpoint_every=ck_every)
    prob.set_reduction(red)
    st = api.ReconState(d["probe"].clone(), d["obj"].clone(), d["pos"].clone(), adam=False)
    beta_o, beta_p = 0.8, 0.5
    opt = api.Optimizer(kind="epie", lr_object=beta_o, lr_probe=beta_p, lr_pos=1.0)
    P0, O0, X0 = c.o_args()
    ost = dict(probe=P0, object=O0, positions=X0)
    oopt = dict(kind="epie", lr_object=beta_o, lr_probe=beta_p, lr_pos=1.0)
    for b in ([0, 4, 8], [1, 2, 3, 5, 6, 7]):
        O_before = _np(st.object).astype(np.complex128)
        P_before = _np(st.probe).astype(np.complex128)
        e = orc.epie_update(ost["probe"], ost["object"], ost["positions"], c.pats.astype(np.float64), b, c.geom)
        loss_g = prob.reconstruct_step(st, d["pats"], torch.tensor(b, dtype=torch.int32, device="cuda"), opt)
        prob.check()
        assert abs(loss_g.item() - e["loss"]) < TOL_I * abs(e["loss"]), (loss_g.item(), e["loss"])
        dO = (_np(st.object).astype(np.complex128) - O_before) / beta_o
        dP = (_np(st.probe).astype(np.complex128) - P_before) * len(b) / beta_p
        errs = dict(dO=rel_l2(dO, e["dO"]), dP=rel_l2(dP, e["dP"]))
        print(N, loss, errs)
        assert all(v < TOL_G for v in errs.values()), errs
        ost, _ = orc.reconstruct_step(ost, c.pats.astype(np.float64), b, c.geom, oopt)
    assert rel_l2(_np(st.object).astype(np.complex128), ost["object"]) < 1e-5
    assert rel_l2(_np(st.probe).astype(np.complex128), ost["probe"]) < 1e-5
    assert np.array_equal(_np(st.positions), c.pos)


@pytest.mark.parametrize("N,loss,eps,ck_every,chunk,red", [(64, "amplitude", 0.0, 1, 0, "atomic"),
                                                           (64, "poisson", 0.5, 2, 4, "atomic"),
                                                           (128, "anscombe", 0.1, 1, 0, "atomic"),
                                                           (192, "amplitude", 0.0, 3, 0, "atomic"),
                                                           (64, "poisson", 0.5, 1, 4, "ordered")])
def test_lsqml_step_matches_oracle(N, loss, eps, ck_every, chunk, red):
    """The LSQML engine (Sec. 3.3) over two iterations: the object and probe
    steps and the illumination sums of every group step against the oracle,
    each step started from the GPU state and sums (first iteration with the
    running sums, then with the previous iteration's)."""
    from paper_2505_14372_amd import api
    c = Case(_widen(synth.make_small(N=N, M=2, S=3, scan=3, step=5, seed=50 + N, loss=loss, eps=eps,
                                     amp_noise=0.3), 9, seed=50 + N, shift=4.0))
    d = c.device()
    prob = c.problem(max_batch=len(c.batch), checkpoint_every=ck_every, lsqml=True)
    prob.set_chunk(chunk)
    prob.set_reduction(red)
    st = api.ReconState(d["probe"].clone(), d["obj"].clone(), d["pos"].clone(), adam=False)
    il = api.IllumSums(c.S, c.H, c.W, c.N)
    kw = dict(beta_object=0.9, beta_probe=0.7, delta_object=1e-2, delta_probe=1e-2, gamma=1e-3)
    pats = c.pats.astype(np.float64)
    for it in range(2):
        for b in ([0, 4, 8], [1, 2, 3, 5, 6, 7]):
            P0 = _np(st.probe).astype(np.complex128)
            O0 = _np(st.object).astype(np.complex128)
            oil = dict(obj_cur=_np(il.obj_cur).astype(np.float64), probe_cur=_np(il.probe_cur).astype(np.float64),
                       obj_prev=None if il.obj_prev is None else _np(il.obj_prev).astype(np.float64),
                       probe_prev=None if il.probe_prev is None else _np(il.probe_prev).astype(np.float64),
                       first=il.obj_prev is None)
            onew, oloss, info = orc.lsqml_step(dict(probe=P0, object=O0, positions=c.pos.astype(np.float64)), oil,
                                               pats, b, c.geom, **kw)
            loss_g = prob.lsqml_step(st, il, d["pats"], torch.tensor(b, dtype=torch.int32, device="cuda"), **kw)
            prob.check()
            assert abs(loss_g.item() - oloss) < TOL_I * abs(oloss), (loss_g.item(), oloss)
            errs = dict(dO=rel_l2(_np(st.object).astype(np.complex128) - O0, onew["object"] - O0),
                        dP=rel_l2(_np(st.probe).astype(np.complex128) - P0, onew["probe"] - P0),
                        obj_cur=rel_l2(_np(il.obj_cur), oil["obj_cur"]),
                        probe_cur=rel_l2(_np(il.probe_cur), oil["probe_cur"]))
            print(N, it, errs, info["alpha"], info["alpha_probe"])
            assert all(v < TOL_G for v in errs.values()), errs
        il.end_iteration()
    assert np.array_equal(_np(st.positions), c.pos)


def test_ordered_lsqml_step_is_bitwise_repeatable():
    """Under the ordered reduction an LSQML step from the same state and sums
    (object direction, illumination scatter, steps) gives identical bits."""
    from paper_2505_14372_amd import api
    c = Case(synth.make_small(N=64, M=2, S=3, scan=4, step=4, seed=61, loss="poisson", eps=0.5, amp_noise=0.3))
    d = c.device()
    prob = c.problem(max_batch=len(c.batch), lsqml=True)
    prob.set_reduction("ordered")
    b = torch.tensor([0, 1, 2, 4, 5, 6, 8, 9, 10, 12, 13, 15], dtype=torch.int32, device="cuda")
    kw = dict(beta_object=0.5, beta_probe=0.5, delta_object=1e-2, delta_probe=1e-2)
    outs = []
    for _ in range(2):
        st = api.ReconState(d["probe"].clone(), d["obj"].clone(), d["pos"].clone(), adam=False)
        il = api.IllumSums(c.S, c.H, c.W, c.N)
        loss = prob.lsqml_step(st, il, d["pats"], b, **kw)
        prob.check()
        outs.append((loss.item(), st.object.clone(), st.probe.clone(), il.obj_cur.clone(), il.probe_cur.clone()))
    (l0, *a0), (l1, *a1) = outs
    assert l0 == l1
    assert all(torch.equal(x, y) for x, y in zip(a0, a1))


def test_lsqml_needs_its_scratch():
    from paper_2505_14372_amd import _lib, api
    c = Case(synth.make_small(N=64, M=1, S=1, scan=2, step=4, seed=3, loss="amplitude"))
    d = c.device()
    prob = c.problem(max_batch=4)
    st = api.ReconState(d["probe"].clone(), d["obj"].clone(), d["pos"].clone(), adam=False)
    il = api.IllumSums(c.S, c.H, c.W, c.N)
    with pytest.raises(_lib.PtyError) as e:
        prob.lsqml_step(st, il, d["pats"], d["batch"])
    assert e.value.status == _lib.PTY_ESTATE


@pytest.mark.parametrize("engine", ["epie", "lsqml"])
def test_conventional_engines_under_resident_strategy_and_chunks(engine):
    """The conventional engines always run on the two-pass kernels: asking for
    the LDS-resident chains and a chunked schedule changes nothing."""
    from paper_2505_14372_amd import api
    c = Case(synth.make_small(N=64, M=2, S=3, scan=3, step=5, seed=80, loss="amplitude", amp_noise=0.3))
    d = c.device()
    prob = c.problem(max_batch=len(c.batch), lsqml=engine == "lsqml")
    prob.set_strategy("resident")
    prob.set_chunk(4)
    st = api.ReconState(d["probe"].clone(), d["obj"].clone(), d["pos"].clone(), adam=False)
    b = [0, 2, 3, 5, 6, 8]
    P0, O0, X0 = c.o_args()
    pats = c.pats.astype(np.float64)
    bt = torch.tensor(b, dtype=torch.int32, device="cuda")
    if engine == "epie":
        prob.reconstruct_step(st, d["pats"], bt, api.Optimizer(kind="epie", lr_object=0.8, lr_probe=0.5))
        ref, _ = orc.reconstruct_step(dict(probe=P0, object=O0, positions=X0), pats, b, c.geom,
                                      dict(kind="epie", lr_object=0.8, lr_probe=0.5, lr_pos=0.0))
    else:
        il = api.IllumSums(c.S, c.H, c.W, c.N)
        kw = dict(beta_object=0.5, beta_probe=0.5, delta_object=1e-2, delta_probe=1e-2, gamma=0.0)
        prob.lsqml_step(st, il, d["pats"], bt, **kw)
        oil = dict(obj_prev=None, probe_prev=None, obj_cur=np.zeros((c.S, c.H, c.W)), probe_cur=np.zeros((c.N, c.N)),
                   first=True)
        ref, _, _ = orc.lsqml_step(dict(probe=P0, object=O0, positions=X0), oil, pats, b, c.geom, **kw)
    prob.check()
    dO = _np(st.object).astype(np.complex128) - O0
    dP = _np(st.probe).astype(np.complex128) - P0
    assert rel_l2(dO, ref["object"] - O0) < TOL_G
    assert rel_l2(dP, ref["probe"] - P0) < TOL_G


def test_final_pass_chains_match_the_oracle_and_the_stored_path():
    """N = 256 with 4 modes: the final column pass runs as chains that keep the
    probe-gradient sums in registers. Loss and gradients against the oracle;
    against a chunked call, which stores h_hat and sums it in k_probe_grad in
    the same order, the position gradient is bit for bit equal and the probe
    gradient equal to float rounding (the two kernels may fuse the products of
    a term into multiply-adds differently); a window outside the object inside
    a chain adds a zero term on both paths."""
    wl = synth.make_small(N=256, M=4, S=2, scan=6, step=4, seed=90, loss="poisson", eps=0.8, amp_noise=0.2)
    c = Case(wl)
    assert len(c.batch) >= 2 * 16
    ref = c.oracle_grad()
    d = c.device()
    outs = {}
    for chunk in (0, 7):
        prob = c.problem()
        prob.set_reduction("ordered")
        prob.set_chunk(chunk)
        outs[chunk] = prob.loss_and_grad(d["probe"], d["obj"], d["pos"], d["pats"], d["batch"])
        prob.check()
        prob.close()
    loss, gO, gP, gX = outs[0]
    assert abs(loss.item() - ref["loss"]) < TOL_I * abs(ref["loss"])
    for name, got, want in (("object", gO, ref["g_object"]), ("probe", gP, ref["g_probe"]),
                            ("positions", gX, ref["g_pos"])):
        e2, einf = rel_l2(_np(got), want), max_rel(_np(got), want)
        print(f"{name}: rel L2 {e2:.2e}, max {einf:.2e}")
        assert e2 < TOL_G and einf < TOL_G, (name, e2, einf)
    assert max_rel(_np(outs[0][2]), _np(outs[7][2])) < 1e-6 and torch.equal(outs[0][3], outs[7][3])
    # one window far outside the object, in the middle of a chain
    pos = d["pos"].clone()
    pos[20] = torch.tensor([-50.0, -50.0], device="cuda")
    got = {}
    for chunk in (0, 7):
        prob = c.problem()
        prob.set_reduction("ordered")
        prob.set_chunk(chunk)
        got[chunk] = prob.loss_and_grad(d["probe"], d["obj"], pos, d["pats"], d["batch"])
        with pytest.raises(Exception, match="window left the object"):
            prob.check()
        prob.close()
    assert max_rel(_np(got[0][2]), _np(got[7][2])) < 1e-6 and torch.equal(got[0][3], got[7][3])
    # the excluded window contributes nothing: the same gradients as without it
    keep = torch.tensor([j for j in c.batch if j != 20], dtype=torch.int32, device="cuda")
    prob = c.problem()
    prob.set_reduction("ordered")
    _, _, gP_keep, _ = prob.loss_and_grad(d["probe"], d["obj"], pos, d["pats"], keep)
    prob.check()
    assert max_rel(_np(got[0][2]), _np(gP_keep)) < 1e-6
