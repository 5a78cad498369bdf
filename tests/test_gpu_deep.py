"""Rollouts of a transition network at the depth and width of the paper's
distilled samplers (four hidden layers of 1024, bfloat16; Sec. 5), run by the
split rollout kernel: a block of waves shares each layer of two 32-particle
tiles.

* Integer-exact network (small-integer weights, biases, states and explicit
  noise, discount 1/2): Q, the returns and the rollout states equal the
  oracle's bit for bit, for a whole group of tiles (N = 64) and a ragged one
  (N = 100: the second group holds one full and one partly filled tile); Q
  too where 1/N is exact.
* The small workload's counts (K = 32, N = 128, H = 10): Q against the oracle
  in binary64 and in bfloat16 emulation, unweighted and with belief weights.
* The large counts (K = 256, N = 4,096, H = 20): sampled rollouts against the
  bfloat16 emulation; Q is the mean of the returns.
* An observation network of the same depth and width (the split
  observation kernel): the per-step observations of the integer-exact
  rollouts bit for bit; observations of belief rows and of rollouts against
  the bfloat16 emulation; at the large counts sampled rows against the
  oracle's observation of the device's own rollout states with the Philox
  noise of their counters.
* Binary32, and likelihood networks of this shape, are refused; an
  out-of-range action sets the status word.
"""
import numpy as np
import pytest
import torch

import oracle
import workloads
from test_gpu_wide import integer_mlp

pytestmark = pytest.mark.gpu

# Bounds calibrated like the width-1024 ones: twice the largest error seen,
# rounded up to a power of two.  Small counts, 10 seeds (6..15): Q vs
# binary64 6.5e-3, Q vs bfloat16 emulation 1.23e-4.  Large counts, 4 seeds
# (8..11) x 32 sampled rollouts: 5.6e-3 against the emulation (medians
# 2e-6..1.4e-4; the tail is a bfloat16 rounding of an activation that falls
# the other way under the two summation orders, carried through later steps).
BOUND_Q_FP64 = 2.0 ** -6
BOUND_Q_EMUL = 2.0 ** -11
BOUND_ROLLOUT_EMUL = 2.0 ** -6
# Observations through the four-layer observation network against the
# bfloat16 emulation, relative to their scale, calibrated the same way:
# largest seen over seeds 6..11 (K 8, N 96, H 5, rollout and belief rows)
# 4.0e-3; at the large counts (2 seeds x 64 sampled rows) 5.8e-4.
BOUND_OBS_EMUL = 2.0 ** -6


@pytest.fixture(scope="module")
def V():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2606_19729_amd as lib
    return lib


def dev(a, dtype=torch.float32):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def deep_integer_workload(seed, N, with_obs=False):
    rng = np.random.default_rng(seed)
    model = workloads.Model(d_s=4, n_actions=5, d_a=0, d_w=4, d_o=2, d_wz=2,
                            trans=integer_mlp(rng, [4 + 5 + 4] + [1024] * 4 + [4]), obs=[], lik=[])
    if with_obs:
        model.obs = integer_mlp(np.random.default_rng(seed + 1), [4 + 5 + 2] + [1024] * 4 + [2])
    K, H = 6, 4
    S = rng.integers(-3, 4, (N, 4)).astype(np.float32)
    C = rng.integers(0, 5, (K, H)).astype(np.int32)
    noise = rng.integers(-2, 3, (K, N, H, 4)).astype(np.float32)
    goal = rng.integers(-2, 3, 4).astype(np.float32)
    return model, S, C, noise, goal


@pytest.mark.parametrize("N", [64, 100])
def test_integer_exact_deep_network_matches_bitwise(V, N):
    model, S, C, noise, goal = deep_integer_workload(40 + N, N)
    print(f"integer-exact deep plan N={N}", flush=True)
    vm = V.Model(model, compute="bf16")
    q, G, traj = V.plan(vm, dev(S), dev(C, torch.int32), 0.5, goal, noise=dev(noise), return_G=True,
                        return_traj=True)
    torch.cuda.synchronize()
    q_ref, G_ref = oracle.plan(model, S, C, 0.5, goal, noise=noise, return_G=True)
    t_ref, _ = oracle.plan_steps(model, S, C, noise=noise, want_obs=False)
    assert np.max(np.abs(G_ref)) > 1.0 and np.max(np.abs(t_ref)) >= 1.0  # the pin is not vacuous
    assert np.array_equal(G.cpu().numpy().astype(np.float64), G_ref)
    assert np.array_equal(traj.cpu().numpy().astype(np.float64), t_ref)
    # Q = (integer sum) x binary32(1/N): exact for N = 64, one rounding otherwise
    q = q.cpu().numpy().astype(np.float64)
    if N & (N - 1) == 0:
        assert np.array_equal(q, q_ref)
    else:
        assert np.max(np.abs(q - q_ref) / np.abs(q_ref)) <= 2.0 ** -22


def test_deep_model_refusals(V):
    w = workloads.deep(N=8, K=1, H=1, with_obs=True)
    with pytest.raises(V.VoilaError) as e:
        V.Model(w.model, compute="f32")
    assert e.value.status == V.VOILA_ERR_UNSUPPORTED
    # a likelihood network of the same depth is not compiled
    rng = np.random.default_rng(0)
    with_lik = workloads.Model(**{**w.model.__dict__, "lik": workloads.random_mlp(rng, [4 + 5 + 2] + [1024] * 4 + [1])})
    with pytest.raises(V.VoilaError) as e:
        V.Model(with_lik, compute="bf16")
    assert e.value.status == V.VOILA_ERR_UNSUPPORTED
    # the model has no likelihood network: no update
    vm = V.Model(w.model, compute="bf16")
    with pytest.raises(V.VoilaError):
        V.update(vm, dev(w.states), 2, [0.0, 0.0], seed=1, U=1)


@pytest.mark.parametrize("N", [64, 100])
def test_integer_exact_deep_observations_match_bitwise(V, N):
    model, S, C, noise, goal = deep_integer_workload(60 + N, N, with_obs=True)
    print(f"integer-exact deep plan + per-step observations N={N}", flush=True)
    obs_noise = np.random.default_rng(N).integers(-2, 3, (C.shape[0], N, C.shape[1], 2)).astype(np.float32)
    vm = V.Model(model, compute="bf16")
    Cd = dev(C, torch.int32)
    _, traj = V.plan(vm, dev(S), Cd, 0.5, goal, noise=dev(noise), return_traj=True)
    obs = V.plan_observe(vm, traj, Cd, noise=dev(obs_noise))
    # observations of belief rows under one action
    o1 = V.observe(vm, dev(S), 3, noise=dev(obs_noise[0, :, 0]))
    torch.cuda.synchronize()
    t_ref, o_ref = oracle.plan_steps(model, S, C, noise=noise, obs_noise=obs_noise)
    assert np.max(np.abs(o_ref)) >= 1.0
    assert np.array_equal(traj.cpu().numpy().astype(np.float64), t_ref)
    assert np.array_equal(obs.cpu().numpy().astype(np.float64), o_ref)
    o1_ref = oracle.observe(model, S, np.full(N, 3, np.int32), noise=obs_noise[0, :, 0])
    assert np.array_equal(o1.cpu().numpy().astype(np.float64), o1_ref)


def test_deep_observations_within_bounds(V):
    w = workloads.deep(seed=6, N=96, K=8, H=5, with_obs=True)
    print("deep bf16 observations seed 6 (K=8 N=96 H=5)", flush=True)
    vm = V.Model(w.model, compute="bf16")
    Cd = dev(w.cands, torch.int32)
    _, traj = V.plan(vm, dev(w.states), Cd, w.gamma, w.goal, seed=w.plan_seed, return_traj=True)
    obs = V.plan_observe(vm, traj, Cd, seed=w.plan_seed)
    nz = np.random.default_rng(5).standard_normal((w.N, 2)).astype(np.float32)
    o1 = V.observe(vm, dev(w.states), w.update_action, noise=dev(nz))
    torch.cuda.synchronize()
    # the oracle observes the device's rollout states (the states' own error is
    # the rollouts' bound), with the counter noise of every row
    t_dev = traj.cpu().numpy().astype(np.float64)
    K, N, H = w.K, w.N, w.H
    rows = t_dev.reshape(-1, 4)
    acts = np.repeat(w.cands[:, None, :], N, axis=1).reshape(-1)
    nzr = np.stack([oracle.normals(w.plan_seed, i, k, t, 4, 2) for k in range(K) for i in range(N) for t in range(H)])
    o_em = oracle.observe(w.model, rows, acts, noise=nzr, bf16=True).reshape(K, N, H, 2)
    e_roll = float(np.max(np.abs(obs.cpu().numpy() - o_em)) / np.max(np.abs(o_em)))
    o1_em = oracle.observe(w.model, w.states, np.full(N, w.update_action, np.int32), noise=nz, bf16=True)
    e_one = float(np.max(np.abs(o1.cpu().numpy() - o1_em)) / np.max(np.abs(o1_em)))
    print(f"  rollout observations vs emulation {e_roll:.2e}; belief observations {e_one:.2e}", flush=True)
    assert e_roll <= BOUND_OBS_EMUL and e_one <= BOUND_OBS_EMUL


def test_deep_observations_large_counts_sampled(V):
    w = workloads.deep(seed=8, N=4096, K=256, H=20, with_obs=True)
    vm = V.Model(w.model, compute="bf16")
    print("deep bf16 per-step observations K=256 N=4096 H=20", flush=True)
    Cd = dev(w.cands, torch.int32)
    _, traj = V.plan(vm, dev(w.states), Cd, w.gamma, w.goal, seed=w.plan_seed, return_traj=True)
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    obs = V.plan_observe(vm, traj, Cd, seed=w.plan_seed, status=st)
    torch.cuda.synchronize()
    assert int(st.item()) == 0
    rng = np.random.default_rng(3)
    picks = [(int(rng.integers(0, w.K)), int(rng.integers(0, w.N)), int(rng.integers(0, w.H))) for _ in range(48)]
    picks.append((w.K - 1, w.N - 1, w.H - 1))
    s_rows = np.stack([traj[k, i, t].cpu().numpy() for k, i, t in picks]).astype(np.float64)
    acts = np.array([w.cands[k, t] for k, _, t in picks], np.int32)
    nzr = np.stack([oracle.normals(w.plan_seed, i, k, t, 4, 2) for k, i, t in picks])
    o_em = oracle.observe(w.model, s_rows, acts, noise=nzr, bf16=True)
    got = np.stack([obs[k, i, t].cpu().numpy() for k, i, t in picks])
    e = float(np.max(np.abs(got - o_em)) / np.max(np.abs(o_em)))
    print(f"  sampled observations vs emulation {e:.2e}", flush=True)
    assert e <= BOUND_OBS_EMUL
    assert np.all(np.isfinite(obs[:, ::512].cpu().numpy()))


def test_deep_bad_action_sets_status(V):
    w = workloads.deep(N=64, K=4, H=3)
    vm = V.Model(w.model, compute="bf16")
    C = w.cands.copy()
    C[2, 1] = 7
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    V.plan(vm, dev(w.states), dev(C, torch.int32), w.gamma, w.goal, seed=1, status=st)
    torch.cuda.synchronize()
    assert int(st.item()) != 0
    st.zero_()
    V.plan(vm, dev(w.states), dev(w.cands, torch.int32), w.gamma, w.goal, seed=1, status=st)
    torch.cuda.synchronize()
    assert int(st.item()) == 0


def test_deep_plan_within_bounds(V):
    w = workloads.deep(seed=6)
    print("deep bf16 plan seed 6 (K=32 N=128 H=10)", flush=True)
    vm = V.Model(w.model, compute="bf16")
    S = dev(w.states)
    C = dev(w.cands, torch.int32)
    q = V.plan(vm, S, C, w.gamma, w.goal, seed=w.plan_seed).cpu().numpy().astype(np.float64)
    q64 = oracle.plan(w.model, w.states, w.cands, w.gamma, w.goal, seed=w.plan_seed)
    qem = oracle.plan(w.model, w.states, w.cands, w.gamma, w.goal, seed=w.plan_seed, bf16=True)
    e64 = float(np.max(np.abs(q - q64) / np.abs(q64)))
    eem = float(np.max(np.abs(q - qem) / np.abs(qem)))
    # belief weights: Q = sum_i w_i G_ik from the same returns
    bw = np.random.default_rng(7).random(w.N)
    bw /= bw.sum()
    qw, G = V.plan(vm, S, C, w.gamma, w.goal, seed=w.plan_seed, belief_w=dev(bw, torch.float64), return_G=True)
    G64 = G.cpu().numpy().astype(np.float64)
    qw_ref = G64 @ bw
    ew = float(np.max(np.abs(qw.cpu().numpy() - qw_ref) / np.abs(qw_ref)))
    print(f"  Q err vs fp64 {e64:.2e} vs bf16-emulation {eem:.2e}; weighted Q vs its returns {ew:.2e}", flush=True)
    assert e64 <= BOUND_Q_FP64 and eem <= BOUND_Q_EMUL
    assert ew <= 1e-5
    # the unweighted Q is the mean of the same returns
    assert np.max(np.abs(q - G64.mean(axis=1)) / np.abs(q)) <= 1e-5


def test_deep_large_counts_sampled(V):
    w = workloads.deep(seed=8, N=4096, K=256, H=20)
    vm = V.Model(w.model, compute="bf16")
    print("deep bf16 large counts K=256 N=4096 H=20", flush=True)
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    q, G = V.plan(vm, dev(w.states), dev(w.cands, torch.int32), w.gamma, w.goal, seed=w.plan_seed, return_G=True,
                  status=st)
    torch.cuda.synchronize()
    assert int(st.item()) == 0
    G = G.cpu().numpy().astype(np.float64)
    rng = np.random.default_rng(2)
    pairs = [(int(rng.integers(0, w.K)), int(rng.integers(0, w.N))) for _ in range(16)] + [(w.K - 1, w.N - 1)]
    g_em = oracle.rollouts(w.model, w.states, w.cands, w.gamma, w.goal, pairs, seed=w.plan_seed, bf16=True)
    got = np.array([G[k, i] for k, i in pairs])
    e_em = np.abs(got - g_em) / np.abs(g_em)
    print(f"  sampled rollouts vs emulation: max {e_em.max():.2e} median {np.median(e_em):.2e}", flush=True)
    assert e_em.max() <= BOUND_ROLLOUT_EMUL
    qs = G.mean(axis=1)
    assert np.max(np.abs(q.cpu().numpy() - qs) / np.abs(qs)) <= 1e-5
