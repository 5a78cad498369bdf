"""Pins of the oracle's reverse-mode rollout gradients.

* Central finite differences (h = 1e-6, binary64) of the oracle's objective,
  on 64-rollout subsets, for the distillation loss w.r.t. network parameters
  (discrete actions) and the mean return w.r.t. continuous action sequences.
  Coordinates whose perturbation changes the ReLU sign pattern of any
  rollout straddle a kink and are excluded (and counted).
* Closed form for an affine generator (ReLUs held active): the return is
  quadratic in the actions, and its gradient follows from the linear state
  recursion with matrix powers.
"""
import numpy as np
import pytest

import oracle
import workloads
from workloads import Model

H_FD = 1e-6


def _with_params(model, flat):
    layers, off = [], 0
    for W, b in model.trans:
        n = W.size
        layers.append((flat[off:off + n].reshape(W.shape), flat[off + n:off + n + b.size]))
        off += n + b.size
    return Model(**{**model.__dict__, "trans": layers})


def _flat(layers):
    return np.concatenate([np.concatenate([np.asarray(W, np.float64).ravel(), np.asarray(b, np.float64)])
                           for W, b in layers])


def distill_case(B=64, H=20, seed=5):
    w = workloads.small(seed=seed)
    rng = np.random.default_rng(seed)
    S0 = rng.standard_normal((B, 4))
    A = rng.integers(0, 5, (B, H)).astype(np.int32)
    teacher = workloads.small(seed=seed + 1).model
    T = oracle.teacher_targets(teacher, S0, A, H, seed=77)
    return w.model, S0, A, T


def cont_model(seed=7):
    rng = np.random.default_rng(seed)
    return workloads.make_model(rng, d_s=4, n_actions=0, d_a=4, d_w=4, d_o=2, d_wz=2, width=64, n_hidden=2)


def test_distillation_gradient_matches_finite_differences():
    m, S0, A, T = distill_case()
    H = A.shape[1]
    loss, grads, _ = oracle.rollout_grad(m, S0, A, H, oracle.DISTILL, targets=T, seed=77)
    assert loss == pytest.approx(oracle.rollout_objective(m, S0, A, H, oracle.DISTILL, targets=T, seed=77),
                                 rel=1e-14)
    flat0 = _flat(m.trans)
    g = _flat(grads)
    rng = np.random.default_rng(0)
    coords = rng.choice(flat0.size, 120, replace=False)
    checked, kinks, worst = 0, 0, 0.0
    for q in coords:
        vals, pats = [], []
        for sgn in (+1, -1):
            f = flat0.copy()
            f[q] += sgn * H_FD
            v, pat = oracle.rollout_objective(_with_params(m, f), S0, A, H, oracle.DISTILL, targets=T, seed=77,
                                              patterns=True)
            vals.append(v)
            pats.append(pat)
        if not np.array_equal(pats[0], pats[1]):
            kinks += 1
            continue
        fd = (vals[0] - vals[1]) / (2 * H_FD)
        worst = max(worst, abs(fd - g[q]))
        checked += 1
    print(f"distillation FD: {checked} coordinates, {kinks} straddle a kink, max abs err {worst:.2e} "
          f"(gradient scale {np.max(np.abs(g)):.2e})")
    assert checked >= 100
    assert worst <= 1e-6 * max(1.0, np.max(np.abs(g)))


def test_return_action_gradient_matches_finite_differences():
    m = cont_model()
    rng = np.random.default_rng(1)
    P, H = 64, 20
    S0 = rng.standard_normal((P, 4))
    A = rng.uniform(-1, 1, (1, H, 4))
    goal = np.array([1.0, 1.0, 0.0, 0.0])
    J, _, gA = oracle.rollout_grad(m, S0, A, H, oracle.RETURN, gamma=0.95, goal=goal, particles=P, seed=9,
                                   want_params=False, want_actions=True)
    kinks, worst = 0, 0.0
    for idx in np.ndindex(A.shape):
        vals, pats = [], []
        for sgn in (+1, -1):
            Ap = A.copy()
            Ap[idx] += sgn * H_FD
            v, pat = oracle.rollout_objective(m, S0, Ap, H, oracle.RETURN, gamma=0.95, goal=goal, particles=P,
                                              seed=9, patterns=True)
            vals.append(v)
            pats.append(pat)
        if not np.array_equal(pats[0], pats[1]):
            kinks += 1
            continue
        worst = max(worst, abs((vals[0] - vals[1]) / (2 * H_FD) - gA[idx]))
    print(f"action FD: {A.size} coordinates, {kinks} straddle a kink, max abs err {worst:.2e} "
          f"(gradient scale {np.max(np.abs(gA)):.2e})")
    assert kinks < A.size // 4
    assert worst <= 1e-6 * max(1.0, np.max(np.abs(gA)))


def test_return_parameter_gradient_matches_finite_differences():
    m = cont_model(seed=3)
    rng = np.random.default_rng(2)
    P, H = 64, 12
    S0 = rng.standard_normal((P, 4))
    A = rng.uniform(-1, 1, (1, H, 4))
    goal = np.array([1.0, 1.0, 0.0, 0.0])
    _, grads, _ = oracle.rollout_grad(m, S0, A, H, oracle.RETURN, gamma=0.9, goal=goal, particles=P, seed=4)
    g = _flat(grads)
    flat0 = _flat(m.trans)
    worst, checked = 0.0, 0
    for q in np.random.default_rng(3).choice(flat0.size, 60, replace=False):
        vals, pats = [], []
        for sgn in (+1, -1):
            f = flat0.copy()
            f[q] += sgn * H_FD
            v, pat = oracle.rollout_objective(_with_params(m, f), S0, A, H, oracle.RETURN, gamma=0.9, goal=goal,
                                              particles=P, seed=4, patterns=True)
            vals.append(v)
            pats.append(pat)
        if np.array_equal(pats[0], pats[1]):
            worst = max(worst, abs((vals[0] - vals[1]) / (2 * H_FD) - g[q]))
            checked += 1
    assert checked >= 50
    assert worst <= 1e-6 * max(1.0, np.max(np.abs(g)))


def test_action_gradient_closed_form_for_affine_generator():
    # s_{t+1} = F s_t + B a_t + C w_t + c  =>  dG/da_t = sum_{u >= t} gamma^u (-2) (s_{u+1} - g)^T F^{u-t} B
    from test_oracle_pins import affine_model, split_transition
    rng = np.random.default_rng(21)
    m = affine_model(rng, d_s=4, n_actions=0, d_a=3, d_w=4, d_o=2, in_scale=0.08, out_scale=0.05)
    F, Bm, C, c = split_transition(m)
    P, H, gamma = 32, 9, 0.9
    S0 = rng.standard_normal((P, 4))
    A = rng.uniform(-1, 1, (1, H, 3))
    noise = rng.standard_normal((P, H, 4))
    goal = np.array([1.0, -1.0, 0.5, 0.0])
    _, _, gA = oracle.rollout_grad(m, S0, A, H, oracle.RETURN, gamma=gamma, goal=goal, particles=P, noise=noise,
                                   want_params=False, want_actions=True)
    ref = np.zeros((H, 3))
    for b in range(P):
        s = S0[b].copy()
        traj = []
        for t in range(H):
            s = F @ s + Bm @ A[0, t] + C @ noise[b, t] + c
            traj.append(s.copy())
        for t in range(H):
            acc = np.zeros(3)
            Fp = np.eye(4)
            for u in range(t, H):
                acc += gamma ** u * (-2.0) * (traj[u] - goal) @ Fp @ Bm
                Fp = F @ Fp
            ref[t] += acc / P
    np.testing.assert_allclose(gA[0], ref, rtol=1e-8, atol=1e-10)


def test_gradient_objective_consistency_and_checks():
    m, S0, A, T = distill_case(B=8, H=5)
    with pytest.raises(oracle.OracleError):
        oracle.rollout_grad(m, S0, A, 5, oracle.DISTILL, targets=None)
    l1, _, _ = oracle.rollout_grad(m, S0, A, 5, oracle.DISTILL, targets=T, seed=77, want_params=False)
    assert l1 == pytest.approx(oracle.rollout_objective(m, S0, A, 5, oracle.DISTILL, targets=T, seed=77), rel=1e-14)
