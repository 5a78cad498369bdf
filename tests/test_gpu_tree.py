"""One-level closed-loop tree with the preference backup (voila_plan_closed_loop,
through the C ABI), checked stage by stage against the oracle on the device's
own intermediate results:
* R(b, a): the horizon-1 plan value, within 1e-5 relative;
* child beliefs: every row is one of its first action's successors (within
  1e-5 of the oracle's), each child holds N rows;
* child values: the oracle's continuation returns from the device's child
  beliefs (key seed + 1), mean per child and L_eta, within 1e-5 relative;
* Psi, V(b), pi and the greedy action from the device's R and child values:
  the backup within 1e-12, the soft value as voila_soft_value's bound;
* the whole composition against the oracle's: first every child row equals
  the oracle's own child row within 1e-5 of the scale (every resampling
  decision fell the same way for these seeded cases; a decision could fall
  the other way only if binary32 and binary64 weights straddled a quantisation
  boundary), then Psi within 1e-5 relative -- R, the prior term and the child
  values are all non-positive, so no cancellation amplifies their 1e-5
  relative errors in the sum.
"""
import numpy as np
import pytest
import torch

import oracle
import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def V():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2606_19729_amd as lib
    return lib


def dev(a, dtype=torch.float32):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def rel(a, b):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    return float(np.max(np.abs(a - b) / np.maximum(np.abs(b), 1e-30)))


def run_case(V, w, first, n_obs, cont, gamma=0.95, eta=2.0, lam=1.0, seed=1234, log_pi0=None):
    m = V.Model(w.model)
    A, N = len(first), w.N
    rng = np.random.default_rng(seed)
    U = rng.integers(0, 2**32, A * n_obs, dtype=np.uint64).astype(np.uint32)
    is_disc = w.model.n_actions > 0
    print(f"closed-loop tree {w.name}: N={N} A={A} n_obs={n_obs} K={cont.shape[0]} H={cont.shape[1]}", flush=True)
    r = V.plan_closed_loop(m, dev(w.states), dev(first, torch.int32 if is_disc else torch.float32), n_obs,
                           dev(cont, torch.int32 if is_disc else torch.float32), gamma, eta, lam, w.goal, seed,
                           dev(U.view(np.int32), torch.int32),
                           log_pi0=None if log_pi0 is None else dev(log_pi0, torch.float64), want_child=True)
    torch.cuda.synchronize()
    d = {k: (v.cpu().numpy() if v is not None else None) for k, v in r.items()}
    # 1. R(b, a)
    cands1 = first.reshape(A, 1) if is_disc else first.reshape(A, 1, -1)
    R_ref = oracle.plan(w.model, w.states, cands1, 1.0, w.goal, seed=seed)
    e_R = rel(d["R"], R_ref)
    # 2. child beliefs: rows of the right successor sets
    traj, _ = oracle.plan_steps(w.model, w.states, cands1, seed=seed, want_obs=False)
    child = d["child"].reshape(A * n_obs, N, -1)
    for g in range(A * n_obs):
        succ = traj[g // n_obs, :, 0]
        dist = np.abs(child[g][:, None, :] - succ[None, :, :]).max(-1).min(-1)
        assert np.all(dist <= 1e-5 * np.abs(succ).max()), g
    # 3. child values from the device's child beliefs
    _, G2 = oracle.plan(w.model, d["child"], cont, gamma, w.goal, seed=seed + 1, return_G=True)
    Qc = G2.reshape(cont.shape[0], A * n_obs, N).mean(axis=2).T
    Vc_ref, _, _ = oracle.soft_value(Qc, eta)
    e_Vc = rel(d["V_child"], Vc_ref)
    # 4. backup and root soft value from the device's R and child values
    lp = np.full(A, -np.log(A)) if log_pi0 is None else log_pi0
    psi_ref = lp / eta + d["R"] + gamma * d["V_child"].reshape(A, n_obs).mean(axis=1)
    e_psi = rel(d["psi"], psi_ref)
    V_ref, pi_ref, best_ref = oracle.soft_value(d["psi"][None, :], eta, log_pi0=np.zeros((1, A)))
    # 5. the whole composition
    full = oracle.plan_closed_loop(w.model, w.states, first, n_obs, cont, gamma, eta, lam, w.goal, seed, U,
                                   log_pi0=log_pi0)
    e_child = float(np.max(np.abs(d["child"] - full["child"]))) / float(np.max(np.abs(full["child"])))
    assert e_child <= 1e-5, e_child
    e_full = rel(d["psi"], full["psi"])
    print(f"  R {e_R:.2e}; V_child {e_Vc:.2e}; psi {e_psi:.2e}; child rows vs full oracle {e_child:.2e}; "
          f"psi vs full oracle {e_full:.2e}; "
          f"best {int(d['best'][0])} (oracle {full['best']})", flush=True)
    assert e_R <= 1e-5 and e_Vc <= 1e-5 and e_psi <= 1e-12
    assert rel(d["V"], V_ref) <= 1e-12 and rel(d["pi"], pi_ref[0]) <= 1e-12 and int(d["best"][0]) == best_ref[0]
    assert e_full <= 1e-5


def test_small_tree(V):
    w = workloads.small(seed=91, N=128, K=16, H=5)
    run_case(V, w, np.arange(5, dtype=np.int32), 4, w.cands)


def test_small_tree_prior_and_single_branch(V):
    w = workloads.small(seed=92, N=40, K=6, H=3)
    lp = np.log(np.array([0.4, 0.1, 0.2, 0.2, 0.1]))
    run_case(V, w, np.array([3, 1, 4, 0, 2], np.int32), 1, w.cands, log_pi0=lp, gamma=0.5, eta=0.7)


def test_realistic_tree_continuous_actions(V):
    w = workloads.realistic(seed=93, N=96, K=8, H=4)
    first = np.random.default_rng(5).uniform(-1, 1, (3, 4)).astype(np.float32)
    run_case(V, w, first, 3, w.cands)
