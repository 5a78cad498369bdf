"""bfloat16 form of the networks (bf16 operands, binary32 accumulation) against
the oracle in two modes: binary64 with the binary32 master weights, and the
oracle's bfloat16 emulation (weights and layer inputs rounded to bfloat16,
binary64 accumulation).

Stated bounds, calibrated over 20 seeds of the small and the (reduced)
realistic workload as twice the largest error seen, rounded up to a power of
two (largest seen: 1.01e-2, 2.6e-4 and 1.9e-3 posterior standard deviations):
* Q relative error vs the binary64 oracle:            <= 2^-5
* Q relative error vs the bfloat16-emulation oracle:  <= 2^-10
* pre-resampling posterior mean vs the binary64 oracle, per state
  coordinate, in units of the posterior standard deviation: <= 2^-8

Single rollouts (no averaging over particles) are bounded per result,
calibrated the same way over 20 seeds x 64 sampled rollouts of the realistic
networks at horizon 20 (largest seen: 7.7e-3 vs the emulation, 2.9e-2 vs
binary64):
* return of every sampled rollout vs the bfloat16-emulation oracle: <= 2^-6
* return of every sampled rollout vs the binary64 oracle:           <= 2^-4
Most rollouts agree with the emulation to binary32 rounding (median 5e-8);
the largest errors come from the rounding of an activation to bfloat16
falling the other way when the binary32 sum and the emulation's binary64 sum
sit on either side of a rounding midpoint, which changes that activation by
one bfloat16 unit and propagates through the later steps.
"""
import numpy as np
import pytest
import torch

import oracle
import workloads

pytestmark = pytest.mark.gpu

BOUND_Q_FP64 = 2.0 ** -5
BOUND_Q_EMUL = 2.0 ** -10
BOUND_POST = 2.0 ** -8
BOUND_ROLLOUT_EMUL = 2.0 ** -6
BOUND_ROLLOUT_FP64 = 2.0 ** -4


@pytest.fixture(scope="module")
def V():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2606_19729_amd as lib
    return lib


CASES = [("small", 101), ("small", 117), ("realistic", 203), ("realistic", 219)]


def make(name, seed):
    if name == "small":
        return workloads.small(seed=seed)
    return workloads.realistic(seed=seed, N=256, K=16, H=20)


@pytest.mark.parametrize("name,seed", CASES)
def test_bf16_plan_and_update_within_stated_bounds(V, name, seed):
    w = make(name, seed)
    print(f"bf16 case {name} seed {seed}", flush=True)
    mb = V.Model(w.model, compute="bf16")
    S = torch.as_tensor(w.states, device="cuda")
    C = torch.as_tensor(w.cands, device="cuda")
    q = V.plan(mb, S, C, w.gamma, w.goal, seed=w.plan_seed).cpu().numpy().astype(np.float64)
    q64 = oracle.plan(w.model, w.states, w.cands, w.gamma, w.goal, seed=w.plan_seed)
    qem = oracle.plan(w.model, w.states, w.cands, w.gamma, w.goal, seed=w.plan_seed, bf16=True)
    e64 = float(np.max(np.abs(q - q64) / np.abs(q64)))
    eem = float(np.max(np.abs(q - qem) / np.abs(qem)))
    o = oracle.draw_observation(w).astype(np.float32)
    out = V.update(mb, S, w.update_action, o, lam=w.lam, seed=w.update_seed, U=w.resample_u)
    ref = oracle.update(w.model, w.states, w.update_action, o, lam=w.lam, seed=w.update_seed, U=w.resample_u)
    wd = out["w"].cpu().numpy()
    mean_d = wd @ out["prop"].cpu().numpy().astype(np.float64)
    mean_r = ref["w"] @ ref["S_prop"]
    sd_r = np.sqrt(ref["w"] @ (ref["S_prop"] - mean_r) ** 2)
    post = float(np.max(np.abs(mean_d - mean_r) / sd_r))
    print(f"  Q err vs fp64 {e64:.2e} vs bf16-emulation {eem:.2e}; posterior mean {post:.2e} sd; "
          f"argmax agrees {np.argmax(q) == np.argmax(q64)}", flush=True)
    assert e64 <= BOUND_Q_FP64
    assert eem <= BOUND_Q_EMUL
    assert post <= BOUND_POST
    # resampling of the device's own weights stays bit-exact
    assert np.array_equal(out["idx"].cpu().numpy(), oracle.resample(wd, w.resample_u))


def test_bf16_realistic_full_size_sampled(V):
    w = workloads.realistic()
    mb = V.Model(w.model, compute="bf16")
    q, G = V.plan(mb, torch.as_tensor(w.states, device="cuda"), torch.as_tensor(w.cands, device="cuda"),
                  w.gamma, w.goal, seed=w.plan_seed, return_G=True)
    G = G.cpu().numpy().astype(np.float64)
    rng = np.random.default_rng(1)
    pairs = [(int(rng.integers(0, w.K)), int(rng.integers(0, w.N))) for _ in range(32)]
    g_em = oracle.rollouts(w.model, w.states, w.cands, w.gamma, w.goal, pairs, seed=w.plan_seed, bf16=True)
    g64 = oracle.rollouts(w.model, w.states, w.cands, w.gamma, w.goal, pairs, seed=w.plan_seed)
    got = np.array([G[k, i] for k, i in pairs])
    # every sampled rollout against the per-rollout bounds
    e_em = np.abs(got - g_em) / np.abs(g_em)
    e64 = np.abs(got - g64) / np.abs(g64)
    print(f"  sampled rollouts: err vs emulation max {e_em.max():.2e} (median {np.median(e_em):.2e}), "
          f"vs fp64 max {e64.max():.2e} (median {np.median(e64):.2e})", flush=True)
    assert e_em.max() <= BOUND_ROLLOUT_EMUL
    assert e64.max() <= BOUND_ROLLOUT_FP64
