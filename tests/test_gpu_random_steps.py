"""Parity of whole reconstruction steps on seeded random configurations:
window size, modes, slices, noise model, object shape, engine (SGD or ePIE),
a random subset of the cost regularizers and constraints (Sec. 3.4) with
random weights, reduction and checkpoint schedule are drawn per case; two
group steps run on the GPU and in the FP64 oracle from the same state, and
the losses and the state updates are compared. (Adam's arithmetic has its own
tight test; its sign-like update on near-zero gradients makes an
update-to-update comparison meaningless on random data.)"""
import os

import numpy as np
import pytest

import oracle as orc
from paper_2505_14372_amd import synth

from _cases import Case, rel_l2

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

TOL_I, TOL_G = 1e-4, 1e-3


def _real(a):
    a = np.asarray(a)
    return np.stack([a.real, a.imag], -1) if np.iscomplexobj(a) else a


def _disk(N, r):
    k = np.fft.fftfreq(N) * N
    return (k[:, None] ** 2 + k[None, :] ** 2) <= r * r


def _draw(seed):
    rng = np.random.default_rng(5000 + seed)
    N = int(rng.choice([64, 64, 128, 128, 192, 256]))
    M = int(rng.integers(1, 4))
    S = int(rng.integers(1, 5))
    loss = str(rng.choice(["amplitude", "anscombe", "poisson", "gaussian"]))
    eps = float(rng.choice([0.3, 0.8])) if loss != "gaussian" else 0.0
    scan, step = (int(rng.integers(2, 4)) if N < 256 else 2), int(rng.integers(3, 9))
    wl = synth.make_small(N=N, M=M, S=S, scan=scan, step=step, seed=6000 + seed, loss=loss, eps=eps,
                          phi_max=float(rng.uniform(0.05, 0.3)), amp_noise=float(rng.choice([0.1, 0.3])),
                          dose=1e5)
    extra = int(rng.integers(0, 24))
    if extra:
        pad = np.exp(1j * 0.2 * rng.random((wl.S, wl.H, extra)))
        wl.obj = np.concatenate([wl.obj, pad], axis=2)
        wl.W = wl.obj.shape[2]
    kind = str(rng.choice(["sgd", "sgd", "epie"]))
    reg, con, api_kw = {}, {}, {}
    ranges = dict(obj_l2=(0.1, 5.0), probe_l2=(1e-3, 0.05), obj_l1=(0.1, 3.0), obj_tikhonov=(0.5, 6.0),
                  obj_tv=(0.5, 5.0), layers_tikhonov=(0.5, 6.0), layers_tv=(0.5, 5.0), obj_phase_l1=(0.5, 4.0),
                  obj_spectrum_l1=(0.05, 0.5), probe_phase_tikhonov=(0.05, 0.3), probe_phase_tv=(0.05, 0.3))
    for key, (lo, hi) in ranges.items():
        if rng.random() < 0.3 and not (key.startswith("layers") and S == 1):
            reg[key] = float(rng.uniform(lo, hi))
    if any(k in reg for k in ("obj_tv", "layers_tv", "probe_phase_tv")):
        reg["tv_delta"] = float(rng.uniform(0.01, 0.1))
    if rng.random() < 0.25:
        con["amp_min"], con["amp_max"] = float(rng.uniform(0.5, 0.9)), float(rng.uniform(0.95, 1.2))
        api_kw["amp_range"] = (con["amp_min"], con["amp_max"])
    if rng.random() < 0.25:
        con["probe_support"] = api_kw["probe_support"] = _disk(N, float(rng.uniform(N / 4, N / 2.5)))
    if rng.random() < 0.2:
        yy, xx = np.mgrid[:N, :N]
        r = float(rng.uniform(N / 3, N / 2))
        con["probe_support_real"] = api_kw["probe_support_real"] = (yy - N / 2) ** 2 + (xx - N / 2) ** 2 <= r * r
    if S > 1 and rng.random() < 0.2:
        con["layer_sigma"] = api_kw["layer_sigma"] = float(rng.uniform(0.3, 1.0))
    if rng.random() < 0.2:
        con["obj_lowpass_sigma"] = api_kw["obj_lowpass_sigma"] = float(rng.uniform(0.3, 1.0))
    if rng.random() < 0.2:
        con["phase_deramp"] = api_kw["phase_deramp"] = True
    # SGD: relative step sizes (the learning rates follow from the gradients at
    # the start, see _sgd_rates); ePIE: its step fractions
    lr = (dict(rel=float(rng.uniform(3e-4, 3e-3))) if kind == "sgd" else
          dict(lr_object=float(rng.uniform(0.3, 1.0)), lr_probe=float(rng.uniform(0.3, 1.0)), lr_pos=0.0))
    reduction = str(rng.choice(["atomic", "ordered"]))
    sched = dict(checkpoint_every=int(rng.choice([1, 1, 2])), checkpoint_half=bool(rng.random() < 0.2))
    J = wl.positions.shape[0]
    perm = rng.permutation(J)
    half = max(1, J // 2)
    batches = [np.sort(perm[:half]).astype(np.int32), np.sort(perm[half:] if J > 1 else perm).astype(np.int32)]
    return Case(wl), kind, reg, con, api_kw, lr, reduction, sched, batches


def _sgd_rates(c, b, reg, rel):
    """Learning rates that move the object and the probe by `rel` of their
    norms, and the positions by `rel` pixels, on the first group (so that no
    noise model, dose or regularizer weight drives the step far from the
    linear regime, where float32 and FP64 trajectories part ways)."""
    P0, O0, X0 = c.o_args()
    r = orc.loss_and_grad(P0, O0, X0, c.pats.astype(np.float64), list(b), c.geom)
    _, gO, gP = orc.regularization(O0, P0, reg) if reg else (0.0, 0.0, 0.0)
    nO = np.linalg.norm(r["g_object"] + gO)
    nP = np.linalg.norm(r["g_probe"] + gP)
    nX = np.linalg.norm(r["g_pos"])
    return dict(lr_object=rel * np.linalg.norm(O0) / nO if nO > 0 else 0.0,
                lr_probe=rel * np.linalg.norm(P0) / nP if nP > 0 else 0.0,
                lr_pos=rel / nX if nX > 0 else 0.0)


@pytest.mark.parametrize("seed", range(int(os.environ.get("PTY_RANDOM_STEPS", "12"))))
def test_random_step_matches_oracle(seed):
    from paper_2505_14372_amd import api
    c, kind, reg, con, api_kw, lr, reduction, sched, batches = _draw(seed)
    print(f"seed {seed}: N={c.N} M={c.M} S={c.S} H={c.H} W={c.W} loss={c.geom.loss} eps={c.geom.eps} {kind} "
          f"{reduction} {sched} reg={sorted(reg)} con={sorted(con)}", flush=True)
    d = c.device()
    prob = c.problem(max_batch=max(len(b) for b in batches), checkpoint_every=sched["checkpoint_every"],
                     checkpoint_half=sched["checkpoint_half"])
    prob.set_reduction(reduction)
    prob.set_regularizers(**{k: v for k, v in reg.items()}, **api_kw)
    st = api.ReconState(d["probe"].clone(), d["obj"].clone(), d["pos"].clone(), adam=False)
    if kind == "sgd":
        lr = _sgd_rates(c, batches[0], reg, lr["rel"])
    opt = api.Optimizer(kind=kind, **lr)
    P0, O0, X0 = c.o_args()
    ost = dict(probe=P0, object=O0, positions=X0)
    oopt = dict(kind=kind, **lr, reg=reg, con=con)
    for b in batches:
        loss = prob.reconstruct_step(st, d["pats"], torch.from_numpy(b).cuda(), opt)
        prob.check()
        ost, oloss = orc.reconstruct_step(ost, c.pats.astype(np.float64), list(b), c.geom, oopt)
        print(f"  loss {loss.item():.8e} oracle {oloss:.8e}")
        assert abs(loss.item() - oloss) < TOL_I * abs(oloss), (loss.item(), oloss)
    for key, got, init in (("object", st.object, O0), ("probe", st.probe, P0), ("positions", st.positions, X0)):
        g = got.detach().cpu()
        g = (torch.view_as_real(g) if g.is_complex() else g).numpy().astype(np.float64)
        want = _real(ost[key])
        du_g, du_w = g - _real(init), want - _real(init)
        res = np.linalg.norm(np.spacing(want.astype(np.float32)).astype(np.float64))
        if key == "probe" and "probe_support" in con:
            # the reciprocal-space support is a float32 forward and inverse 2D
            # transform of the whole probe: rounding of order u sqrt(log2 N^2)
            # of its norm each, far above one ulp per element
            res += 8 * np.finfo(np.float32).eps * np.sqrt(np.log2(c.N * c.N)) * np.linalg.norm(want)
        err = np.linalg.norm(du_g - du_w)
        scale = np.linalg.norm(du_w)
        print(f"  {key}: |du| {scale:.3e}, error {err:.3e} (float32 resolution {res:.1e})")
        assert err <= TOL_G * scale + res, (key, err, scale, res)
