"""Soft value, soft policy and greedy action of candidate preferences
(voila_soft_value, through the C ABI) against the oracle: V and the policy
within 1e-12 relative (binary64 on both sides, different summation order),
the greedy action exact (both sides compare the same binary64 x_k), ties to
the lowest index, the uniform prior, K = 1, non-finite preferences, and the
plan's own Q as input."""
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


def check(Vlib, Q, eta, lp):
    Qd = torch.as_tensor(np.ascontiguousarray(Q, np.float32), device="cuda")
    lpd = None if lp is None else torch.as_tensor(np.ascontiguousarray(lp), device="cuda")
    v, pi, best = Vlib.soft_value(Qd, eta, lpd)
    torch.cuda.synchronize()
    v_ref, pi_ref, best_ref = oracle.soft_value(np.asarray(Q, np.float32).astype(np.float64), eta, lp)
    v, pi, best = v.cpu().numpy(), pi.cpu().numpy(), best.cpu().numpy()
    e_v = float(np.max(np.abs(v - v_ref) / np.maximum(np.abs(v_ref), 1.0)))
    e_pi = float(np.max(np.abs(pi - pi_ref) / np.maximum(pi_ref, 1e-300)))
    print(f"  M={Q.shape[0]} K={Q.shape[1]} eta={eta}: V err {e_v:.2e} pi err {e_pi:.2e}", flush=True)
    assert e_v <= 1e-12 and e_pi <= 1e-12
    assert np.array_equal(best, best_ref)


@pytest.mark.parametrize("M,K", [(1, 1), (37, 1024), (5, 3000)])
@pytest.mark.parametrize("eta", [0.3, 5.0])
def test_soft_value_matches_oracle(V, M, K, eta):
    rng = np.random.default_rng(M * K)
    Q = (rng.standard_normal((M, K)) * 4).astype(np.float32)
    check(V, Q, eta, None)
    check(V, Q, eta, np.log(rng.dirichlet(np.ones(K), size=M)))


def test_ties_go_to_the_lowest_index(V):
    Q = np.zeros((3, 700), np.float32)
    Q[0, [5, 300, 650]] = 2.0
    Q[1, [699, 256, 257]] = 1.0
    check(V, Q, 1.0, None)
    _, _, best = V.soft_value(torch.as_tensor(Q, device="cuda"), 1.0)
    assert best.cpu().tolist() == [5, 256, 0]


def test_plan_q_as_preferences(V):
    w = workloads.small()
    m = V.Model(w.model)
    q = V.plan(m, torch.as_tensor(w.states, device="cuda"), torch.as_tensor(w.cands, device="cuda"), w.gamma,
               w.goal, seed=w.plan_seed)
    torch.cuda.synchronize()
    check(V, q.cpu().numpy()[None, :], 2.0, None)


def test_non_finite_preference_sets_status(V):
    Q = np.zeros((2, 10), np.float32)
    Q[1, 3] = np.nan
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    v, _, _ = V.soft_value(torch.as_tensor(Q, device="cuda"), 1.0, status=st)
    torch.cuda.synchronize()
    assert int(st.item()) == V.VOILA_ERR_NUMERIC
    assert v[0].item() == pytest.approx(0.0, abs=1e-15)
