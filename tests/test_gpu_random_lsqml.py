"""Parity of the LSQML engine (Sec. 3.3) on seeded random configurations:
window size, modes, slices, noise model, object shape, checkpoint interval,
chunk size, reduction and the step parameters are drawn per case; every group
step of two iterations starts the oracle from the GPU's state and sums and
compares the object and probe steps and the illumination sums."""
import os

import numpy as np
import pytest

import oracle as orc
from paper_2505_14372_amd import synth

from _cases import Case, rel_l2

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

TOL_I, TOL_G = 1e-4, 1e-3


def _np(t):
    return t.detach().cpu().numpy()


@pytest.mark.parametrize("seed", range(int(os.environ.get("PTY_RANDOM_LSQML", "4"))))
def test_random_lsqml_steps_match_oracle(seed):
    from paper_2505_14372_amd import api
    rng = np.random.default_rng(7000 + seed)
    N = int(rng.choice([64, 64, 128, 192, 256]))
    M, S = int(rng.integers(1, 4)), int(rng.integers(1, 5))
    loss = str(rng.choice(["amplitude", "anscombe", "poisson", "gaussian"]))
    eps = float(rng.choice([0.3, 0.8])) if loss != "gaussian" else 0.0
    scan, step = (int(rng.integers(2, 4)) if N < 256 else 2), int(rng.integers(3, 9))
    wl = synth.make_small(N=N, M=M, S=S, scan=scan, step=step, seed=7100 + seed, loss=loss, eps=eps,
                          amp_noise=float(rng.choice([0.1, 0.3])), dose=1e5)
    extra = int(rng.integers(0, 16))
    if extra:
        wl.obj = np.concatenate([wl.obj, np.exp(1j * 0.2 * rng.random((wl.S, wl.H, extra)))], axis=2)
        wl.W = wl.obj.shape[2]
    c = Case(wl)
    J = c.pos.shape[0]
    perm = rng.permutation(J)
    half = max(1, J // 2)
    groups = [sorted(perm[:half].tolist()), sorted(perm[half:].tolist() if J > 1 else perm.tolist())]
    kw = dict(beta_object=float(rng.uniform(0.05, 0.9)), beta_probe=float(rng.uniform(0.05, 0.9)),
              delta_object=float(rng.choice([1e-3, 1e-2, 1e-1])), delta_probe=float(rng.choice([1e-3, 1e-2, 1e-1])),
              gamma=float(rng.choice([0.0, 1e-3])))
    ck = int(rng.choice([1, 1, 2]))
    chunk = int(rng.choice([0, 0, 2]))
    red = str(rng.choice(["atomic", "ordered"]))
    print(f"seed {seed}: N={N} M={M} S={S} H={c.H} W={c.W} J={J} {loss} eps={eps} ck={ck} chunk={chunk} {red} {kw}",
          flush=True)
    d = c.device()
    prob = c.problem(max_batch=max(len(g) for g in groups), checkpoint_every=ck, lsqml=True)
    prob.set_chunk(chunk)
    prob.set_reduction(red)
    st = api.ReconState(d["probe"].clone(), d["obj"].clone(), d["pos"].clone(), adam=False)
    il = api.IllumSums(c.S, c.H, c.W, c.N)
    pats = c.pats.astype(np.float64)
    for it in range(2):
        for b in groups:
            P0, O0 = _np(st.probe).astype(np.complex128), _np(st.object).astype(np.complex128)
            oil = dict(obj_cur=_np(il.obj_cur).astype(np.float64), probe_cur=_np(il.probe_cur).astype(np.float64),
                       obj_prev=None if il.obj_prev is None else _np(il.obj_prev).astype(np.float64),
                       probe_prev=None if il.probe_prev is None else _np(il.probe_prev).astype(np.float64),
                       first=il.obj_prev is None)
            onew, oloss, _ = orc.lsqml_step(dict(probe=P0, object=O0, positions=c.pos.astype(np.float64)), oil, pats,
                                            b, c.geom, **kw)
            loss_g = prob.lsqml_step(st, il, d["pats"], torch.tensor(b, dtype=torch.int32, device="cuda"), **kw)
            prob.check()
            assert abs(loss_g.item() - oloss) < TOL_I * abs(oloss), (loss_g.item(), oloss)
            dO_g, dO_w = _np(st.object).astype(np.complex128) - O0, onew["object"] - O0
            dP_g, dP_w = _np(st.probe).astype(np.complex128) - P0, onew["probe"] - P0
            resO = np.linalg.norm(np.spacing(np.abs(onew["object"]).astype(np.float32)).astype(np.float64))
            resP = np.linalg.norm(np.spacing(np.abs(onew["probe"]).astype(np.float32)).astype(np.float64))
            errs = dict(dO=np.linalg.norm(dO_g - dO_w) / (np.linalg.norm(dO_w) + resO / TOL_G),
                        dP=np.linalg.norm(dP_g - dP_w) / (np.linalg.norm(dP_w) + resP / TOL_G),
                        obj_cur=rel_l2(_np(il.obj_cur), oil["obj_cur"]),
                        probe_cur=rel_l2(_np(il.probe_cur), oil["probe_cur"]))
            print("  ", it, {k: f"{v:.1e}" for k, v in errs.items()})
            assert all(v < TOL_G for v in errs.values()), errs
        il.end_iteration()
