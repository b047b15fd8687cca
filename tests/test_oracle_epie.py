"""Pins of the oracle's ePIE / 3PIE engine (Sec. 3.3).

* single slice, single mode: the textbook ePIE updates (modulus projection,
  conj(P) / max |P|^2 and conj(O) / max |O|^2 steps) written out here;
* any slice count: the update chain is the finite-difference-pinned adjoint
  of the amplitude loss with the per-slice normalisers applied, so every
  slice's object update and the probe update equal minus the single-position
  gradients times the product of normalisers they pass through;
* noise-free data of the current state is a fixed point;
* group updates are the sums of single-position updates.
"""
import numpy as np
import pytest

import oracle as orc


def crandn(rng, *shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def _problem(rng, N=8, M=1, S=1, J=1, side=12, amp=0.3):
    P = crandn(rng, M, N, N) * 0.5
    O = (1.0 - amp * rng.random((S, side, side))) * np.exp(1j * rng.random((S, side, side)))
    X = rng.uniform(0.6, side - N - 0.6, (J, 2))
    return P, O, X


def test_single_slice_is_textbook_epie():
    rng = np.random.default_rng(0)
    N = 8
    P, O, _ = _problem(rng, N=N)
    X = np.array([[2.0, 3.0]])                       # integer position: no subpixel shift
    pats = 5 * rng.random((1, N, N))
    geom = orc.Geometry(N=N, dz=[], loss="amplitude", eps=0.0)
    beta_o, beta_p = 0.7, 0.4
    new, _ = orc.reconstruct_step(dict(probe=P, object=O, positions=X), pats, [0], geom,
                                  dict(kind="epie", lr_object=beta_o, lr_probe=beta_p, lr_pos=0.0))
    # textbook ePIE (one position, simultaneous update)
    patch = O[0, 2:2 + N, 3:3 + N]
    psi = P[0] * patch
    Psi = np.fft.fft2(psi, norm="ortho")
    Psi_new = np.sqrt(pats[0]) * Psi / np.abs(Psi)
    dpsi = np.fft.ifft2(Psi_new, norm="ortho") - psi
    O_ref = O.copy()
    O_ref[0, 2:2 + N, 3:3 + N] += beta_o * np.conj(P[0]) / np.max(np.abs(P[0]) ** 2) * dpsi
    P_ref = P + beta_p * np.conj(patch) / np.max(np.abs(patch) ** 2) * dpsi
    assert np.max(np.abs(new["object"] - O_ref)) < 1e-12
    assert np.max(np.abs(new["probe"] - P_ref)) < 1e-12
    assert np.array_equal(new["positions"], X)


@pytest.mark.parametrize("loss,eps", [("amplitude", 0.0), ("anscombe", 0.3)])
def test_update_chain_is_normalised_adjoint(loss, eps):
    rng = np.random.default_rng(1)
    N, M, S = 8, 2, 3
    P, O, X = _problem(rng, N=N, M=M, S=S, J=1, side=13)
    pats = 4 * rng.random((1, N, N))
    geom = orc.Geometry(N=N, dz=[1.5, 2.5], loss=loss, eps=eps, bandlimit=0.0)
    e = orc.epie_update(P, O, X, pats, [0], geom)
    g = orc.loss_and_grad(P, O, X, pats, [0], geom)
    psi, _, _ = orc.forward_position(P, O, X[0], geom)
    n, _ = orc.split_positions(X[0])
    a = np.zeros(S)
    b = np.zeros(S)
    for i in range(S):
        a[i] = 1 / np.max(np.sum(np.abs(psi[i]) ** 2, axis=0))
        b[i] = 1 / np.max(np.abs(O[i, n[0]:n[0] + N, n[1]:n[1] + N]) ** 2)
    assert np.allclose(e["a"][0], a, rtol=1e-14) and np.allclose(e["b"][0], b, rtol=1e-14)
    for i in range(S):
        ref = -a[i] * np.prod(b[i + 1:]) * g["g_object"][i]
        assert np.max(np.abs(e["dO"][i] - ref)) < 1e-12 * np.max(np.abs(ref))
    refP = -np.prod(b) * g["g_probe"]
    assert np.max(np.abs(e["dP"] - refP)) < 1e-12 * np.max(np.abs(refP))


def test_noise_free_data_is_a_fixed_point():
    rng = np.random.default_rng(2)
    N, M, S, J = 8, 2, 3, 4
    P, O, X = _problem(rng, N=N, M=M, S=S, J=J, side=14)
    geom = orc.Geometry(N=N, dz=[2.0, 2.0], loss="amplitude", eps=0.0)
    pats = orc.forward(P, O, X, range(J), geom)
    new, loss = orc.reconstruct_step(dict(probe=P, object=O, positions=X), pats, list(range(J)), geom,
                                     dict(kind="epie", lr_object=1.0, lr_probe=1.0, lr_pos=0.0))
    assert loss < 1e-20
    assert np.max(np.abs(new["object"] - O)) < 1e-12
    assert np.max(np.abs(new["probe"] - P)) < 1e-12


def test_group_update_sums_positions_and_averages_probe():
    rng = np.random.default_rng(3)
    N, M, S, J = 8, 2, 2, 3
    P, O, X = _problem(rng, N=N, M=M, S=S, J=J, side=14)
    pats = 3 * rng.random((J, N, N))
    geom = orc.Geometry(N=N, dz=[2.0], loss="poisson", eps=0.5)
    e = orc.epie_update(P, O, X, pats, [0, 1, 2], geom)
    parts = [orc.epie_update(P, O, X, pats, [j], geom) for j in range(J)]
    assert np.allclose(e["dO"], sum(p["dO"] for p in parts), atol=1e-13)
    assert np.allclose(e["dP"], sum(p["dP"] for p in parts), atol=1e-13)
    assert abs(e["loss"] - orc.total_loss(P, O, X, pats, [0, 1, 2], geom)) < 1e-10 * abs(e["loss"])
    new, _ = orc.reconstruct_step(dict(probe=P, object=O, positions=X), pats, [0, 1, 2], geom,
                                  dict(kind="epie", lr_object=0.5, lr_probe=0.3, lr_pos=0.0))
    assert np.allclose(new["object"], O + 0.5 * e["dO"], atol=1e-14)
    assert np.allclose(new["probe"], P + 0.3 / 3 * e["dP"], atol=1e-14)


def test_epie_iterations_reduce_the_amplitude_loss():
    """Single slice, noise-free data from a known object: ePIE sweeps from a
    perturbed object lower the loss."""
    rng = np.random.default_rng(4)
    N, J = 8, 9
    P = crandn(rng, 1, N, N) * 0.5
    O_true = np.exp(0.5j * rng.random((1, 16, 16)))
    iy, ix = np.mgrid[:3, :3]
    X = np.stack([iy.ravel(), ix.ravel()], 1) * 3.0 + 1.0
    geom = orc.Geometry(N=N, dz=[], loss="amplitude", eps=0.0)
    pats = orc.forward(P, O_true, X, range(J), geom)
    state = dict(probe=P, object=np.ones_like(O_true), positions=X)
    losses = []
    for it in range(6):
        for j in rng.permutation(J):
            state, loss = orc.reconstruct_step(state, pats, [int(j)], geom,
                                               dict(kind="epie", lr_object=1.0, lr_probe=0.0, lr_pos=0.0))
        losses.append(orc.total_loss(P, state["object"], X, pats, range(J), geom))
    assert losses[-1] < 0.2 * losses[0] and all(b <= a * 1.0001 for a, b in zip(losses, losses[1:]))
