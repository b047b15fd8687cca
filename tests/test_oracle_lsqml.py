"""Pins of the oracle's LSQML engine (Sec. 3.3).

* one position, one slice, one mode: a full object step (or a full probe
  step) turns the exit wave into the modulus-projected wave, so the model
  then reproduces the measured pattern exactly;
* the per-group step is the least-squares optimum along the object
  direction (perturbing it raises the exit-wave residual);
* noise-free data of the current state is a fixed point;
* a global phase on the probe leaves the object step unchanged and rotates
  the probe step (catches dropped conjugates);
* the previous-iteration illumination sums are used when present, the
  running sums in the first iteration, and the running sums accumulate.
"""
import numpy as np

import oracle as orc


def crandn(rng, *shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def _illum(S, H, W, N, first=True):
    return dict(obj_prev=np.zeros((S, H, W)), obj_cur=np.zeros((S, H, W)), probe_prev=np.zeros((N, N)),
                probe_cur=np.zeros((N, N)), first=first)


def _single(rng, N=8, side=12):
    P = crandn(rng, 1, N, N) * 0.5
    O = (0.5 + 0.5 * rng.random((1, side, side))) * np.exp(1j * rng.random((1, side, side)))
    X = np.array([[2.0, 3.0]])
    return P, O, X


def test_full_object_step_reproduces_the_pattern():
    rng = np.random.default_rng(0)
    N = 8
    P, O, X = _single(rng, N)
    geom = orc.Geometry(N=N, dz=[], loss="amplitude", eps=0.0)
    pats = 5 * rng.random((1, N, N))
    new, loss, info = orc.lsqml_step(dict(probe=P, object=O, positions=X), _illum(1, 12, 12, N), pats, [0], geom,
                                     beta_object=1.0, beta_probe=0.0, delta_object=1e-300, delta_probe=1e-300)
    assert abs(info["alpha"][0] - 1.0) < 1e-12
    I = orc.forward(new["probe"], new["object"], X, [0], geom)
    assert np.max(np.abs(I - pats)) < 1e-10 * pats.max()
    assert np.array_equal(new["probe"], P)
    assert loss > 0


def test_full_probe_step_reproduces_the_pattern():
    rng = np.random.default_rng(1)
    N = 8
    P, O, X = _single(rng, N)
    geom = orc.Geometry(N=N, dz=[], loss="amplitude", eps=0.0)
    pats = 5 * rng.random((1, N, N))
    new, _, info = orc.lsqml_step(dict(probe=P, object=O, positions=X), _illum(1, 12, 12, N), pats, [0], geom,
                                  beta_object=0.0, beta_probe=1.0, delta_object=1e-300, delta_probe=1e-300)
    assert abs(info["alpha_probe"] - 1.0) < 1e-12
    I = orc.forward(new["probe"], new["object"], X, [0], geom)
    assert np.max(np.abs(I - pats)) < 1e-10 * pats.max()
    assert np.array_equal(new["object"], O)


def test_object_step_is_least_squares_optimal():
    rng = np.random.default_rng(2)
    N, J, side = 8, 4, 14
    P = crandn(rng, 1, N, N) * 0.5
    O = (0.5 + 0.5 * rng.random((1, side, side))) * np.exp(1j * rng.random((1, side, side)))
    X = np.array([[1.0, 2.0], [4.0, 1.0], [3.0, 5.0], [6.0, 6.0]])
    geom = orc.Geometry(N=N, dz=[], loss="amplitude", eps=0.0)
    pats = 4 * rng.random((J, N, N))
    new, _, info = orc.lsqml_step(dict(probe=P, object=O, positions=X), _illum(1, side, side, N), pats,
                                  list(range(J)), geom, beta_object=1.0, beta_probe=0.0)
    a = info["alpha"][0]
    dO = (new["object"] - O) / a

    def residual(step):
        r = 0.0
        for j in range(J):
            psi, far, I = orc.forward_position(P, O, X[j], geom)
            target = orc.ifft2u(np.sqrt(pats[j]) * far / np.sqrt(I))      # modulus-projected exit wave
            n, _ = orc.split_positions(X[j])
            On = (O + step * dO)[0, n[0]:n[0] + N, n[1]:n[1] + N]
            r += np.sum(np.abs(psi[0] * On - target) ** 2)
        return r
    r0 = residual(a)
    assert r0 < residual(a * 1.01) and r0 < residual(a * 0.99)
    assert 0.0 < a < 10.0


def test_noise_free_data_is_a_fixed_point():
    rng = np.random.default_rng(3)
    N, M, S, J, side = 8, 2, 3, 4, 14
    P = crandn(rng, M, N, N) * 0.5
    O = (0.6 + 0.4 * rng.random((S, side, side))) * np.exp(1j * rng.random((S, side, side)))
    X = rng.uniform(0.6, side - N - 0.6, (J, 2))
    geom = orc.Geometry(N=N, dz=[2.0, 1.0], loss="amplitude", eps=0.0)
    pats = orc.forward(P, O, X, range(J), geom)
    new, loss, _ = orc.lsqml_step(dict(probe=P, object=O, positions=X), _illum(S, side, side, N), pats,
                                  list(range(J)), geom)
    assert loss < 1e-20
    assert np.max(np.abs(new["object"] - O)) < 1e-12 and np.max(np.abs(new["probe"] - P)) < 1e-12


def test_probe_phase_and_illumination_bookkeeping():
    rng = np.random.default_rng(4)
    N, M, S, J, side = 8, 2, 2, 3, 14
    P = crandn(rng, M, N, N) * 0.5
    O = (0.6 + 0.4 * rng.random((S, side, side))) * np.exp(1j * rng.random((S, side, side)))
    X = rng.uniform(0.6, side - N - 0.6, (J, 2))
    geom = orc.Geometry(N=N, dz=[1.5], loss="poisson", eps=0.4)
    pats = 3 * rng.random((J, N, N))
    st = dict(probe=P, object=O, positions=X)
    il = _illum(S, side, side, N)
    new, _, _ = orc.lsqml_step(st, il, pats, [0, 1, 2], geom, beta_object=0.7, beta_probe=0.6)
    rot = np.exp(0.9j)
    il2 = _illum(S, side, side, N)
    new_r, _, _ = orc.lsqml_step(dict(probe=rot * P, object=O, positions=X), il2, pats, [0, 1, 2], geom,
                                 beta_object=0.7, beta_probe=0.6)
    assert np.max(np.abs(new_r["object"] - new["object"])) < 1e-12
    assert np.max(np.abs(new_r["probe"] - rot * new["probe"])) < 1e-12
    # first iteration uses the running sums; later ones the previous sums: the same sums give the same step
    il3 = _illum(S, side, side, N, first=False)
    il3["obj_prev"] = il["obj_cur"].copy()
    il3["probe_prev"] = il["probe_cur"].copy()
    new3, _, _ = orc.lsqml_step(st, il3, pats, [0, 1, 2], geom, beta_object=0.7, beta_probe=0.6)
    assert np.max(np.abs(new3["object"] - new["object"])) < 1e-12
    assert np.max(np.abs(new3["probe"] - new["probe"])) < 1e-12
    assert np.allclose(il3["obj_cur"], il["obj_cur"]) and np.allclose(il3["probe_cur"], il["probe_cur"])
    # the running sums accumulate the illumination: sum_j sum_m |psi_i|^2 and sum_j prod_i |O_i|^2
    W = np.zeros((S, side, side))
    T = np.zeros((N, N))
    for j in range(J):
        psi, _, _ = orc.forward_position(P, O, X[j], geom)
        n, _ = orc.split_positions(X[j])
        W[:, n[0]:n[0] + N, n[1]:n[1] + N] += np.sum(np.abs(psi) ** 2, axis=1)
        T += np.prod(np.abs(O[:, n[0]:n[0] + N, n[1]:n[1] + N]) ** 2, axis=0)
    assert np.allclose(il["obj_cur"], W) and np.allclose(il["probe_cur"], T)
