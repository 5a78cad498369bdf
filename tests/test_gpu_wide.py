"""Hidden width 1024 (bfloat16 networks, grouped evaluation of the second
hidden layer) and an integer-exact pin of every packed network shape.

* Integer-exact networks: small-integer weights, biases, states, actions and
  explicit noise, with discount 1/2 and N = 64, so every binary32 and
  bfloat16 operation on the device and every binary64 operation in the oracle
  is exact: Q, the returns, the rollout states and the per-step observations
  must equal the oracle's bit for bit, for every compiled shape and both
  precisions.  Any misplaced weight fragment changes the result.
* Width 1024 in bfloat16 at the small workload's counts (K = 32, N = 128,
  H = 10): Q, observations and the update against the oracle in binary64 and
  in bfloat16 emulation, within the stated bounds; at the large counts
  (K = 1024, N = 4096, H = 20) on sampled rollouts.
"""
import numpy as np
import pytest
import torch

import oracle
import workloads

pytestmark = pytest.mark.gpu

# Bounds for width 1024, calibrated like the width-64/256 ones: twice the
# largest error seen over 13 seeds (3..14 and 31) at these counts, rounded up
# to a power of two.  Largest seen: Q vs binary64 9.9e-3, Q vs bfloat16
# emulation 2.9e-4, observations vs emulation 7.5e-4 (of their scale),
# posterior mean 1.7e-3 posterior standard deviations.
BOUND_Q_FP64 = 2.0 ** -5
BOUND_Q_EMUL = 2.0 ** -10
BOUND_OBS = 2.0 ** -9
BOUND_POST = 2.0 ** -8
# Single rollouts at the large counts (horizon 20), calibrated the same way
# over 10 seeds x 32 sampled rollouts: largest seen 9.5e-3 against the
# bfloat16 emulation (median 1.3e-7; the large ones come from an activation
# whose bfloat16 rounding falls the other way under binary32 and binary64
# sums, one bfloat16 unit carried through the later steps).
BOUND_ROLLOUT_EMUL = 2.0 ** -5


@pytest.fixture(scope="module")
def V():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2606_19729_amd as lib
    return lib


def dev(a, dtype=torch.float32):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def integer_mlp(rng, dims, fan=2):
    """Layers with a few +-1 weights per row and biases in {-1, 0, 1, 2}:
    activations stay small integers, exact in bfloat16 and binary32."""
    layers = []
    for l in range(len(dims) - 1):
        n_in, n_out = dims[l], dims[l + 1]
        W = np.zeros((n_out, n_in), np.float32)
        for r in range(n_out):
            cols = rng.choice(n_in, size=min(fan if l == 0 else 1, n_in), replace=False)
            W[r, cols] = rng.choice([-1.0, 1.0], size=cols.size)
        if l == len(dims) - 2:
            W *= (rng.random((n_out, 1)) < 0.5)  # sparse output rows keep the states small
        b = rng.integers(-1, 3, n_out).astype(np.float32)
        layers.append((W, b))
    return layers


def integer_workload(shape, seed, N=64):
    d_s, n_act, d_a, d_w, d_o, d_wz, width, n_hid = shape
    rng = np.random.default_rng(seed)
    aw = n_act if n_act > 0 else d_a
    hid = [width] * n_hid
    model = workloads.Model(d_s=d_s, n_actions=n_act, d_a=d_a, d_w=d_w, d_o=d_o, d_wz=d_wz,
                            trans=integer_mlp(rng, [d_s + aw + d_w] + hid + [d_s]),
                            obs=integer_mlp(rng, [d_s + aw + d_wz] + hid + [d_o]),
                            lik=integer_mlp(rng, [d_s + aw + d_o] + hid + [1]))
    K, H = 6, 4
    S = rng.integers(-3, 4, (N, d_s)).astype(np.float32)
    if n_act > 0:
        C = rng.integers(0, n_act, (K, H)).astype(np.int32)
    else:
        C = rng.integers(-1, 2, (K, H, d_a)).astype(np.float32)
    noise = rng.integers(-2, 3, (K, N, H, d_w)).astype(np.float32)
    goal = rng.integers(-2, 3, d_s).astype(np.float32)
    obs_noise = rng.integers(-2, 3, (K, N, H, d_wz)).astype(np.float32)
    return model, S, C, noise, goal, obs_noise


SHAPES = {
    "small": (4, 5, 0, 4, 2, 2, 64, 2),
    "realistic": (16, 0, 4, 16, 32, 32, 256, 3),
    "continuous": (4, 0, 4, 4, 2, 2, 64, 2),
    "wide": (4, 5, 0, 4, 2, 2, 1024, 2),
}


# N = 70 and 100 give the paired bfloat16 evaluations (two 32-row tiles per
# wave) an odd tile count (the last pair's second tile masked) and a ragged
# last tile
@pytest.mark.parametrize("name,compute,N", [("small", "f32", 64), ("small", "bf16", 64), ("realistic", "f32", 64),
                                            ("realistic", "bf16", 64), ("realistic", "bf16", 70),
                                            ("realistic", "bf16", 100), ("continuous", "f32", 64),
                                            ("continuous", "bf16", 64), ("wide", "bf16", 64)])
def test_integer_exact_networks_match_bitwise(V, name, compute, N):
    model, S, C, noise, goal, obs_noise = integer_workload(SHAPES[name], seed=len(name) * 7 + len(compute) + N - 64,
                                                           N=N)
    print(f"integer-exact plan: {name} {compute} N={N}", flush=True)
    vm = V.Model(model, compute=compute)
    Cd = dev(C, torch.int32 if model.n_actions > 0 else torch.float32)
    q, G, traj = V.plan(vm, dev(S), Cd, 0.5, goal, noise=dev(noise), return_G=True, return_traj=True)
    obs = V.plan_observe(vm, traj, Cd, noise=dev(obs_noise))
    torch.cuda.synchronize()
    q_ref, G_ref = oracle.plan(model, S, C, 0.5, goal, noise=noise, return_G=True)
    assert np.max(np.abs(G_ref)) > 1.0  # the pin is not vacuous
    assert np.array_equal(G.cpu().numpy().astype(np.float64), G_ref)
    q = q.cpu().numpy().astype(np.float64)
    if N & (N - 1) == 0:
        assert np.array_equal(q, q_ref)
    else:  # Q = (integer sum) x binary32(1/N): one rounding
        assert np.max(np.abs(q - q_ref) / np.abs(q_ref)) <= 2.0 ** -22
    # the rollout states and the per-step observations, bit for bit
    t_ref, o_ref = oracle.plan_steps(model, S, C, noise=noise, obs_noise=obs_noise)
    assert np.max(np.abs(o_ref)) >= 1.0
    assert np.array_equal(traj.cpu().numpy().astype(np.float64), t_ref)
    assert np.array_equal(obs.cpu().numpy().astype(np.float64), o_ref)


def test_binary32_wide_model_is_refused(V):
    w = workloads.wide(N=8, K=1, H=1)
    with pytest.raises(V.VoilaError) as e:
        V.Model(w.model, compute="f32")
    assert e.value.status == V.VOILA_ERR_UNSUPPORTED


@pytest.mark.parametrize("seed", [3, 31])
def test_wide_plan_update_observe_within_bounds(V, seed):
    w = workloads.wide(seed=seed)
    print(f"wide bf16 case seed {seed}", flush=True)
    mb = V.Model(w.model, compute="bf16")
    S = dev(w.states)
    q = V.plan(mb, S, dev(w.cands, torch.int32), w.gamma, w.goal, seed=w.plan_seed).cpu().numpy().astype(np.float64)
    q64 = oracle.plan(w.model, w.states, w.cands, w.gamma, w.goal, seed=w.plan_seed)
    qem = oracle.plan(w.model, w.states, w.cands, w.gamma, w.goal, seed=w.plan_seed, bf16=True)
    e64 = float(np.max(np.abs(q - q64) / np.abs(q64)))
    eem = float(np.max(np.abs(q - qem) / np.abs(qem)))
    # observations of the belief under action 2 (the bfloat16 emulation rounds the same inputs)
    acts = np.full(w.N, w.update_action, np.int32)
    nz = np.random.default_rng(seed).standard_normal((w.N, w.model.d_wz)).astype(np.float32)
    o_dev = V.observe(mb, S, w.update_action, noise=dev(nz)).cpu().numpy().astype(np.float64)
    o_em = oracle.observe(w.model, w.states, acts, noise=nz, bf16=True)
    e_obs = float(np.max(np.abs(o_dev - o_em)) / np.max(np.abs(o_em)))
    o = oracle.draw_observation(w).astype(np.float32)
    out = V.update(mb, S, w.update_action, o, lam=w.lam, seed=w.update_seed, U=w.resample_u)
    ref = oracle.update(w.model, w.states, w.update_action, o, lam=w.lam, seed=w.update_seed, U=w.resample_u)
    wd = out["w"].cpu().numpy()
    mean_d = wd @ out["prop"].cpu().numpy().astype(np.float64)
    mean_r = ref["w"] @ ref["S_prop"]
    sd_r = np.sqrt(ref["w"] @ (ref["S_prop"] - mean_r) ** 2)
    post = float(np.max(np.abs(mean_d - mean_r) / sd_r))
    print(f"  Q err vs fp64 {e64:.2e} vs bf16-emulation {eem:.2e}; obs vs emulation {e_obs:.2e}; "
          f"posterior mean {post:.2e} sd", flush=True)
    assert e64 <= BOUND_Q_FP64 and eem <= BOUND_Q_EMUL
    assert e_obs <= BOUND_OBS
    assert post <= BOUND_POST
    assert np.array_equal(out["idx"].cpu().numpy(), oracle.resample(wd, w.resample_u))


def test_wide_large_counts_sampled(V):
    # the large counts: 1024 candidates x 4096 particles x 20 steps
    w = workloads.wide(seed=5, N=4096, K=1024, H=20)
    mb = V.Model(w.model, compute="bf16")
    print("wide bf16 large counts K=1024 N=4096 H=20", flush=True)
    q, G = V.plan(mb, dev(w.states), dev(w.cands, torch.int32), w.gamma, w.goal, seed=w.plan_seed, return_G=True)
    torch.cuda.synchronize()
    G = G.cpu().numpy().astype(np.float64)
    rng = np.random.default_rng(2)
    pairs = [(int(rng.integers(0, w.K)), int(rng.integers(0, w.N))) for _ in range(24)] + [(w.K - 1, w.N - 1)]
    g_em = oracle.rollouts(w.model, w.states, w.cands, w.gamma, w.goal, pairs, seed=w.plan_seed, bf16=True)
    got = np.array([G[k, i] for k, i in pairs])
    e_em = np.abs(got - g_em) / np.abs(g_em)
    print(f"  sampled rollouts vs emulation: max {e_em.max():.2e} median {np.median(e_em):.2e}", flush=True)
    assert e_em.max() <= BOUND_ROLLOUT_EMUL
    # Q is the mean of the returns
    qs = G.mean(axis=1)
    assert np.max(np.abs(q.cpu().numpy() - qs) / np.abs(qs)) <= 1e-5
