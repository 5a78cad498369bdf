"""Rollout states and per-step observations of the plan rollouts, through the
C ABI, against the oracle.

* binary32: states s_1..s_H and observations within 1e-5 of the array's
  scale (the proposal / observation tolerance of the parity tests), with
  counter-RNG and explicit noise, common random numbers, ragged sizes and
  K = 0 / H = 0, for the small, continuous-action and (reduced) realistic
  workloads; at the realistic workload's full size on sampled rollouts and
  sampled observation rows, and the returns recomputed from all the states.
* bfloat16: against the oracle's bfloat16 emulation within stated bounds,
  calibrated as twice the largest error seen over 10 seeds (40..49) of each
  workload, rounded up to a power of two.  Largest seen, as a fraction of the
  array's scale: states 2.5e-3 / 4.5e-3 / 2.0e-3 and observations 3.6e-3 /
  7.1e-3 / 5.7e-3 (small / realistic / width 1024): single activations whose
  bfloat16 rounding falls the other way carry a 2^-8 relative change.
* asking for the states leaves Q and the returns bit for bit unchanged.
The integer-exact networks (test_gpu_wide) pin both outputs bit for bit for
every compiled shape.
"""
import numpy as np
import pytest
import torch

import oracle
import workloads

pytestmark = pytest.mark.gpu

TOL = 1e-5
BOUND_TRAJ_EMUL = 2.0 ** -6
BOUND_OBS_EMUL = 2.0 ** -6


@pytest.fixture(scope="module")
def V():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2606_19729_amd as lib
    return lib


def dev(a, dtype=torch.float32):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def host(t):
    return t.detach().cpu().numpy().astype(np.float64)


def scaled_err(got, ref):
    got, ref = np.asarray(got, np.float64), np.asarray(ref, np.float64)
    if ref.size == 0:
        return 0.0
    return float(np.max(np.abs(got - ref)) / max(np.max(np.abs(ref)), 1e-30))


def cands_dev(w):
    return dev(w.cands, torch.int32 if w.model.n_actions > 0 else torch.float32)


def run(V, w, m, crn=False, noise=None, obs_noise=None):
    q, G, traj = V.plan(m, dev(w.states), cands_dev(w), w.gamma, w.goal, seed=w.plan_seed, crn=crn,
                        noise=None if noise is None else dev(noise), return_G=True, return_traj=True)
    o = V.plan_observe(m, traj, cands_dev(w), seed=w.plan_seed, crn=crn,
                       noise=None if obs_noise is None else dev(obs_noise))
    torch.cuda.synchronize()
    return host(q), host(G), host(traj), host(o)


def check_f32(V, w, crn=False, explicit=False):
    m = V.Model(w.model)
    noise = workloads.explicit_plan_noise(w) if explicit else None
    obs_noise = workloads.explicit_obs_noise(w) if explicit else None
    print(f"plan states/observations {w.name} N={w.N} K={w.K} H={w.H} crn={crn} explicit={explicit}", flush=True)
    q, G, traj, o = run(V, w, m, crn, noise, obs_noise)
    rt, ro = oracle.plan_steps(w.model, w.states, w.cands, noise=noise, obs_noise=obs_noise, seed=w.plan_seed,
                               crn=crn)
    e_t, e_o = scaled_err(traj, rt), scaled_err(o, ro)
    print(f"  states err {e_t:.2e} observations err {e_o:.2e}", flush=True)
    assert traj.shape == rt.shape and o.shape == ro.shape
    assert e_t <= TOL and e_o <= TOL
    return m, q, G


@pytest.mark.parametrize("N,K,H", [(1, 1, 1), (33, 3, 7), (100, 2, 5), (257, 4, 3)])
def test_small_states_and_observations(V, N, K, H):
    w = workloads.small(seed=N + 2 * K + H, N=N, K=K, H=H)
    check_f32(V, w)
    check_f32(V, w, explicit=True)


def test_common_random_numbers_and_continuous_actions(V):
    check_f32(V, workloads.small(seed=7, N=70, K=5, H=6), crn=True)
    w = workloads.continuous(N=45, K=4, H=6)
    check_f32(V, w)
    check_f32(V, w, explicit=True)


def test_realistic_reduced(V):
    w = workloads.realistic(N=70, K=6, H=5)
    check_f32(V, w)
    check_f32(V, w, explicit=True, crn=True)


def test_requesting_states_leaves_the_plan_unchanged(V):
    for w in [workloads.small(seed=21, N=90, K=6, H=8), workloads.realistic(seed=22, N=64, K=3, H=4)]:
        m = V.Model(w.model)
        q0, G0 = V.plan(m, dev(w.states), cands_dev(w), w.gamma, w.goal, seed=w.plan_seed, return_G=True)
        q1, G1, _ = V.plan(m, dev(w.states), cands_dev(w), w.gamma, w.goal, seed=w.plan_seed, return_G=True,
                           return_traj=True)
        torch.cuda.synchronize()
        assert torch.equal(q0, q1) and torch.equal(G0, G1)


def test_zero_sizes_write_nothing(V):
    w = workloads.small(seed=5, N=40, K=3, H=4)
    m = V.Model(w.model)
    traj = torch.full((3, 40, 0, 4), 7.0, device="cuda")
    o = V.plan_observe(m, traj, dev(w.cands[:, :0], torch.int32), seed=1)
    assert o.shape == (3, 40, 0, 2)
    traj = torch.zeros((0, 40, 4, 4), device="cuda")
    o = V.plan_observe(m, traj, dev(w.cands[:0], torch.int32), seed=1)
    assert o.shape == (0, 40, 4, 2)


def test_bad_action_sets_status(V):
    w = workloads.small(seed=6, N=40, K=3, H=4)
    m = V.Model(w.model)
    _, traj = V.plan(m, dev(w.states), cands_dev(w), w.gamma, w.goal, seed=1, return_traj=True)
    bad = w.cands.copy()
    bad[1, 2] = 9
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    V.plan_observe(m, traj, dev(bad, torch.int32), seed=1, status=st)
    torch.cuda.synchronize()
    assert int(st.item()) == V.VOILA_ERR_INVALID_ARG


@pytest.mark.parametrize("name,seed", [("small", 101), ("realistic", 203), ("wide", 3)])
def test_bf16_within_stated_bounds(V, name, seed):
    if name == "small":
        w = workloads.small(seed=seed, N=96, K=8, H=10)
    elif name == "realistic":
        w = workloads.realistic(seed=seed, N=64, K=4, H=20)
    else:
        w = workloads.wide(seed=seed, N=64, K=4, H=10)
    print(f"bf16 plan states/observations {name} seed {seed}", flush=True)
    m = V.Model(w.model, compute="bf16")
    _, _, traj, o = run(V, w, m)
    rt, ro = oracle.plan_steps(w.model, w.states, w.cands, seed=w.plan_seed, bf16=True)
    e_t, e_o = scaled_err(traj, rt), scaled_err(o, ro)
    print(f"  vs bf16 emulation: states {e_t:.2e} observations {e_o:.2e}", flush=True)
    assert e_t <= BOUND_TRAJ_EMUL and e_o <= BOUND_OBS_EMUL


def test_realistic_full_size_sampled(V):
    # the benchmark's launch configuration (1024 x 4096 x 20): 5.4 GB of states
    # and 10.7 GB of observations on the device
    w = workloads.realistic()
    m = V.Model(w.model)
    print("realistic full size 1024 x 4096 x 20: states and observations", flush=True)
    S = dev(w.states)
    C = cands_dev(w)
    q, G, traj = V.plan(m, S, C, w.gamma, w.goal, seed=w.plan_seed, return_G=True, return_traj=True)
    o = V.plan_observe(m, traj, C, seed=w.plan_seed)
    torch.cuda.synchronize()
    # the returns are the discounted rewards of the written states (float64 on the device)
    goal = torch.as_tensor(w.goal, dtype=torch.float64, device="cuda")
    disc = torch.as_tensor(w.gamma ** np.arange(w.H), dtype=torch.float64, device="cuda")
    G_ref = torch.zeros((w.K, w.N), dtype=torch.float64, device="cuda")
    for k0 in range(0, w.K, 128):
        r = -((traj[k0:k0 + 128].double() - goal) ** 2).sum(-1)
        G_ref[k0:k0 + 128] = (r * disc).sum(-1)
    e_g = float(((G.double() - G_ref).abs() / G_ref.abs()).max())
    print(f"  returns from the states: max rel err {e_g:.2e}", flush=True)
    assert e_g <= 1e-5
    rng = np.random.default_rng(4)
    pairs = [(int(rng.integers(0, w.K)), int(rng.integers(0, w.N))) for _ in range(16)] + [(w.K - 1, w.N - 1)]
    for k, i in pairs:
        # the oracle's transition sampler, stepped with the rollout's counter noise
        s = np.asarray(w.states[i], np.float64)[None, :]
        ref_t = np.zeros((w.H, w.model.d_s))
        for t in range(w.H):
            nz = oracle.normals(w.plan_seed, i, k, t, 3, w.model.d_w)
            s = oracle.transition(w.model, s, w.cands[k, t][None, :], nz[None, :])
            ref_t[t] = s[0]
        got_t = host(traj[k, i])
        e_t = scaled_err(got_t, ref_t)
        # the oracle's observation sampler on the device's states, with the rollout's counter noise
        nzo = np.stack([oracle.normals(w.plan_seed, i, k, t, 4, w.model.d_wz) for t in range(w.H)])
        ref_o = oracle.observe(w.model, got_t, w.cands[k], noise=nzo)
        e_o = scaled_err(host(o[k, i]), ref_o)
        assert e_t <= TOL and e_o <= TOL, (k, i, e_t, e_o)
    print(f"  {len(pairs)} sampled rollouts within {TOL}", flush=True)
