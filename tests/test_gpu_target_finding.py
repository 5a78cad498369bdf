"""Rollouts and observations at the paper's target-finding shapes (Sec. 5):
a 45-dimensional state, six discrete actions and 36 lidar bins, through
transition and observation networks of four hidden layers of 1024 in
bfloat16 (the split kernels, whose output layers here produce two 32-row
tiles: state and observation features 32 and up come from the second).

* Integer-exact networks (small-integer weights, biases, states and explicit
  noise, discount 1/2): returns, Q, rollout states and per-step observations
  equal the oracle's bit for bit, for a whole group of tiles (N = 64) and a
  ragged one (N = 100).
* Counter noise at small counts: Q against the oracle in binary64 and in
  bfloat16 emulation, unweighted and with belief weights.
* The large counts (K = 256, N = 4,096, H = 20): sampled rollouts against the
  bfloat16 emulation, Q as the mean of the returns, sampled per-step
  observations against the oracle's observation of the device's own states.
* The belief update with the paper's likelihood network of three hidden
  layers of 256 (a shape of its own: proposals in the split kernel, then
  the likelihood of the proposals): integer-exact networks give proposals
  and log-likelihoods bit for bit and the oracle's weights and indices; with
  random networks the proposals and log-likelihoods stay within the bounds
  against the emulation and the device's own weights resample bit-exactly.
  The other users of the likelihood refuse such a model.
"""
import numpy as np
import pytest
import torch

import oracle
import workloads
from test_gpu_wide import integer_mlp

pytestmark = pytest.mark.gpu

D_S, N_ACT, D_O = 45, 6, 36
# Bounds: twice the largest error seen in calibration runs, rounded up to a
# power of two.  Small counts (K 8, N 64, H 5), seeds 16..23: Q vs binary64
# 5.4e-4, Q vs bfloat16 emulation 3.9e-5.  Large counts, seeds 16..19 with 17
# sampled rollouts and 49 sampled observations each: rollouts vs emulation
# 1.8e-3, observations 5.4e-4 of their scale.
BOUND_Q_FP64 = 2.0 ** -9
BOUND_Q_EMUL = 2.0 ** -13
BOUND_ROLLOUT_EMUL = 2.0 ** -8
BOUND_OBS_EMUL = 2.0 ** -9
# The update at N = 4,096 against the emulation, relative to the largest
# magnitude, seeds 16..23: proposals 7.6e-4, log-likelihoods 7.0e-3.
BOUND_PROP_EMUL = 2.0 ** -9
BOUND_LL_EMUL = 2.0 ** -6


@pytest.fixture(scope="module")
def V():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2606_19729_amd as lib
    return lib


def dev(a, dtype=torch.float32):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def integer_workload(seed, N):
    rng = np.random.default_rng(seed)
    model = workloads.Model(d_s=D_S, n_actions=N_ACT, d_a=0, d_w=D_S, d_o=D_O, d_wz=D_O,
                            trans=integer_mlp(rng, [D_S + N_ACT + D_S] + [1024] * 4 + [D_S]), obs=[], lik=[])
    model.obs = integer_mlp(np.random.default_rng(seed + 1), [D_S + N_ACT + D_O] + [1024] * 4 + [D_O])
    lrng = np.random.default_rng(seed + 2)
    model.lik = integer_mlp(lrng, [D_S + N_ACT + D_O] + [256] * 3 + [1])
    # a likelihood that reads 16 units of the last hidden layer (the sparse
    # output row of integer_mlp may read none)
    W, b = model.lik[-1]
    W[0, lrng.choice(256, 16, replace=False)] = lrng.choice([-1.0, 1.0], 16)
    K, H = 4, 3
    S = rng.integers(-3, 4, (N, D_S)).astype(np.float32)
    C = rng.integers(0, N_ACT, (K, H)).astype(np.int32)
    noise = rng.integers(-2, 3, (K, N, H, D_S)).astype(np.float32)
    obs_noise = rng.integers(-2, 3, (K, N, H, D_O)).astype(np.float32)
    goal = rng.integers(-2, 3, D_S).astype(np.float32)
    return model, S, C, noise, obs_noise, goal


@pytest.mark.parametrize("N", [64, 100])
def test_integer_exact_target_finding_matches_bitwise(V, N):
    model, S, C, noise, obs_noise, goal = integer_workload(80 + N, N)
    print(f"integer-exact target-finding plan + observations N={N}", flush=True)
    vm = V.Model(model, compute="bf16")
    Cd = dev(C, torch.int32)
    q, G, traj = V.plan(vm, dev(S), Cd, 0.5, goal, noise=dev(noise), return_G=True, return_traj=True)
    obs = V.plan_observe(vm, traj, Cd, noise=dev(obs_noise))
    o1 = V.observe(vm, dev(S), 4, noise=dev(obs_noise[0, :, 0]))
    torch.cuda.synchronize()
    q_ref, G_ref = oracle.plan(model, S, C, 0.5, goal, noise=noise, return_G=True)
    t_ref, o_ref = oracle.plan_steps(model, S, C, noise=noise, obs_noise=obs_noise)
    # the pins are not vacuous: both output tiles of each network move
    assert np.max(np.abs(G_ref)) > 1.0
    assert np.any(t_ref[..., 32:] != S[None, :, None, 32:]) and np.any(t_ref[..., :32] != S[None, :, None, :32])
    assert np.max(np.abs(o_ref[..., 32:])) >= 1.0 and np.max(np.abs(o_ref[..., :32])) >= 1.0
    assert np.array_equal(G.cpu().numpy().astype(np.float64), G_ref)
    assert np.array_equal(traj.cpu().numpy().astype(np.float64), t_ref)
    assert np.array_equal(obs.cpu().numpy().astype(np.float64), o_ref)
    o1_ref = oracle.observe(model, S, np.full(N, 4, np.int32), noise=obs_noise[0, :, 0])
    assert np.array_equal(o1.cpu().numpy().astype(np.float64), o1_ref)
    q = q.cpu().numpy().astype(np.float64)
    if N & (N - 1) == 0:
        assert np.array_equal(q, q_ref)
    else:
        assert np.max(np.abs(q - q_ref) / np.abs(q_ref)) <= 2.0 ** -22


def test_target_finding_refusals(V):
    w = workloads.target_finding(N=64, K=1, H=1)
    with pytest.raises(V.VoilaError) as e:
        V.Model(w.model, compute="f32")
    assert e.value.status == V.VOILA_ERR_UNSUPPORTED
    # a likelihood of the samplers' shape is not compiled
    rng = np.random.default_rng(0)
    lik = workloads.random_mlp(rng, [D_S + N_ACT + D_O] + [1024] * 4 + [1])
    with pytest.raises(V.VoilaError) as e:
        V.Model(workloads.Model(**{**w.model.__dict__, "lik": lik}), compute="bf16")
    assert e.value.status == V.VOILA_ERR_UNSUPPORTED
    # the likelihood of its own shape serves the update only
    vm = V.Model(w.model, compute="bf16")
    S = dev(w.states)
    O = dev(np.zeros((8, D_O), np.float32))
    with pytest.raises(V.VoilaError) as e:
        V.info_nce(vm, S[:8], dev(np.zeros(8, np.int32), torch.int32), O)
    assert e.value.status == V.VOILA_ERR_UNSUPPORTED


def q_errors(V, seed, K=8, N=64, H=5):
    w = workloads.target_finding(seed=seed, N=N, K=K, H=H)
    vm = V.Model(w.model, compute="bf16")
    S, C = dev(w.states), dev(w.cands, torch.int32)
    q = V.plan(vm, S, C, w.gamma, w.goal, seed=w.plan_seed).cpu().numpy().astype(np.float64)
    bw = np.random.default_rng(seed).random(w.N)
    bw /= bw.sum()
    qw, G = V.plan(vm, S, C, w.gamma, w.goal, seed=w.plan_seed, belief_w=dev(bw, torch.float64), return_G=True)
    torch.cuda.synchronize()
    q64 = oracle.plan(w.model, w.states, w.cands, w.gamma, w.goal, seed=w.plan_seed)
    qem = oracle.plan(w.model, w.states, w.cands, w.gamma, w.goal, seed=w.plan_seed, bf16=True)
    G64 = G.cpu().numpy().astype(np.float64)
    return (float(np.max(np.abs(q - q64) / np.abs(q64))), float(np.max(np.abs(q - qem) / np.abs(qem))),
            float(np.max(np.abs(qw.cpu().numpy() - G64 @ bw) / np.abs(G64 @ bw))),
            float(np.max(np.abs(q - G64.mean(axis=1)) / np.abs(q))))


def test_target_finding_plan_within_bounds(V):
    print("target-finding bf16 plan seed 16 (K=8 N=64 H=5)", flush=True)
    e64, eem, ew, em = q_errors(V, 16)
    print(f"  Q err vs fp64 {e64:.2e} vs bf16-emulation {eem:.2e}; weighted {ew:.2e}", flush=True)
    assert e64 <= BOUND_Q_FP64 and eem <= BOUND_Q_EMUL
    assert ew <= 1e-5 and em <= 1e-5


def large_errors(V, seed, n_roll=16, n_obs=48):
    w = workloads.target_finding(seed=seed, N=4096, K=256, H=20)
    vm = V.Model(w.model, compute="bf16")
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    Cd = dev(w.cands, torch.int32)
    q, G, traj = V.plan(vm, dev(w.states), Cd, w.gamma, w.goal, seed=w.plan_seed, return_G=True, return_traj=True,
                        status=st)
    obs = V.plan_observe(vm, traj, Cd, seed=w.plan_seed, status=st)
    torch.cuda.synchronize()
    assert int(st.item()) == 0
    G = G.cpu().numpy().astype(np.float64)
    rng = np.random.default_rng(seed)
    pairs = [(int(rng.integers(0, w.K)), int(rng.integers(0, w.N))) for _ in range(n_roll)] + [(w.K - 1, w.N - 1)]
    g_em = oracle.rollouts(w.model, w.states, w.cands, w.gamma, w.goal, pairs, seed=w.plan_seed, bf16=True)
    got = np.array([G[k, i] for k, i in pairs])
    e_roll = float(np.max(np.abs(got - g_em) / np.abs(g_em)))
    qs = G.mean(axis=1)
    e_q = float(np.max(np.abs(q.cpu().numpy() - qs) / np.abs(qs)))
    picks = [(int(rng.integers(0, w.K)), int(rng.integers(0, w.N)), int(rng.integers(0, w.H))) for _ in range(n_obs)]
    picks.append((w.K - 1, w.N - 1, w.H - 1))
    s_rows = np.stack([traj[k, i, t].cpu().numpy() for k, i, t in picks]).astype(np.float64)
    acts = np.array([w.cands[k, t] for k, _, t in picks], np.int32)
    nzr = np.stack([oracle.normals(w.plan_seed, i, k, t, 4, D_O) for k, i, t in picks])
    o_em = oracle.observe(w.model, s_rows, acts, noise=nzr, bf16=True)
    o_got = np.stack([obs[k, i, t].cpu().numpy() for k, i, t in picks])
    e_obs = float(np.max(np.abs(o_got - o_em)) / np.max(np.abs(o_em)))
    finite = bool(np.all(np.isfinite(obs[:, ::512].cpu().numpy())))
    return e_roll, e_q, e_obs, finite


def test_target_finding_large_counts_sampled(V):
    print("target-finding bf16 large counts K=256 N=4096 H=20", flush=True)
    e_roll, e_q, e_obs, finite = large_errors(V, 16)
    print(f"  sampled rollouts {e_roll:.2e}; Q vs mean {e_q:.2e}; sampled observations {e_obs:.2e}", flush=True)
    assert e_roll <= BOUND_ROLLOUT_EMUL and e_obs <= BOUND_OBS_EMUL and e_q <= 1e-5 and finite


def test_integer_exact_target_finding_update(V):
    N = 100
    model, S, C, noise, obs_noise, goal = integer_workload(90, N)
    rng = np.random.default_rng(91)
    o = rng.integers(-2, 3, D_O).astype(np.float32)
    unoise = rng.integers(-2, 3, (N, D_S)).astype(np.float32)
    prior = rng.random(N)
    prior /= prior.sum()
    print("integer-exact target-finding update N=100", flush=True)
    vm = V.Model(model, compute="bf16")
    out = V.update(vm, dev(S), 3, o, lam=4.0, prior_w=dev(prior, torch.float64), seed=5, U=12345,
                   noise=dev(unoise))
    torch.cuda.synchronize()
    ref = oracle.update(model, S, 3, o, lam=4.0, prior_w=prior, noise=unoise, seed=5, U=12345)
    ll = out["loglik"].cpu().numpy().astype(np.float64)
    assert np.max(np.abs(ref["loglik"])) >= 1.0 and np.ptp(ref["loglik"]) > 0  # the pin is not vacuous
    assert np.array_equal(out["prop"].cpu().numpy().astype(np.float64), ref["S_prop"])
    assert np.array_equal(ll, ref["loglik"])
    assert np.max(np.abs(out["w"].cpu().numpy() - ref["w"]) / np.max(ref["w"])) <= 1e-13
    assert np.array_equal(out["idx"].cpu().numpy(), ref["idx"])
    assert np.array_equal(out["states"].cpu().numpy().astype(np.float64), ref["S_new"])


def update_errors(V, seed, N=4096):
    w = workloads.target_finding(seed=seed, N=N, K=1, H=1)
    vm = V.Model(w.model, compute="bf16")
    o = (0.5 * np.random.default_rng(seed).standard_normal(D_O)).astype(np.float32)
    out = V.update(vm, dev(w.states), w.update_action, o, lam=w.lam, seed=w.update_seed, U=w.resample_u)
    torch.cuda.synchronize()
    ref = oracle.update(w.model, w.states, w.update_action, o, lam=w.lam, seed=w.update_seed, U=w.resample_u,
                        bf16=True)
    prop = out["prop"].cpu().numpy().astype(np.float64)
    ll = out["loglik"].cpu().numpy().astype(np.float64)
    e_prop = float(np.max(np.abs(prop - ref["S_prop"])) / np.max(np.abs(ref["S_prop"])))
    e_ll = float(np.max(np.abs(ll - ref["loglik"])) / np.max(np.abs(ref["loglik"])))
    wd = out["w"].cpu().numpy()
    w_same, _ = oracle.normalize(ll, w.lam, None)
    e_w = float(np.max(np.abs(wd - w_same) / np.max(w_same)))
    exact = bool(np.array_equal(out["idx"].cpu().numpy(), oracle.resample(wd, w.resample_u)))
    return e_prop, e_ll, e_w, exact


def test_target_finding_update_within_bounds(V):
    print("target-finding bf16 update seed 16 N=4096", flush=True)
    e_prop, e_ll, e_w, exact = update_errors(V, 16)
    print(f"  proposals {e_prop:.2e}; log-likelihoods {e_ll:.2e}; weights(same l) {e_w:.2e}", flush=True)
    assert e_prop <= BOUND_PROP_EMUL and e_ll <= BOUND_LL_EMUL
    assert e_w <= 1e-12 and exact
