"""Grouped progressive widening (voila_pw_step, through the C ABI) against
the oracle.

* widening flags, chosen branches and branch counts: exact (both sides take
  the widening test in binary64 and draw the reused branch from the same
  Philox word);
* new branch observations and log-likelihoods: binary32 within 1e-5 of the
  array's scale; bfloat16 against the oracle's emulation within 2^-6 of the
  scale (the per-step observation bound);
* weights from the device's own log-likelihoods within 1e-13 relative of the
  oracle's normalisation, resampling indices bit-exact given the device's
  weights, gathered rows exact;
* ragged and empty groups, the 8192-successor group limit, and the realistic
  networks at 2,048 groups / ~2 M successors on sampled groups.
"""
import numpy as np
import pytest
import torch

import oracle
import workloads

pytestmark = pytest.mark.gpu

TOL = 1e-5
BOUND_EMUL = 2.0 ** -6


@pytest.fixture(scope="module")
def V():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2606_19729_amd as lib
    return lib


def dev(a, dtype=torch.float32):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def host(t):
    return t.detach().cpu().numpy()


def scaled_err(got, ref):
    got, ref = np.asarray(got, np.float64), np.asarray(ref, np.float64)
    if ref.size == 0:
        return 0.0
    return float(np.max(np.abs(got - ref)) / max(np.max(np.abs(ref)), 1e-30))


def make_case(model, seed, M, d_max, B=6):
    rng = np.random.default_rng(seed)
    sizes = rng.integers(0, d_max + 1, M)
    sizes[:3] = [0, 1, d_max]
    seg = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int32)
    T = int(seg[-1])
    succ = (rng.standard_normal((T, model.d_s)) * 0.8).astype(np.float32)
    actions = rng.integers(0, model.n_actions, M).astype(np.int32) if model.n_actions > 0 else \
        rng.uniform(-1, 1, (M, model.d_a)).astype(np.float32)
    children = rng.integers(0, B + 1, M).astype(np.int32)
    visits = (children.astype(np.int64) ** 2 + rng.integers(-2, 3, M)).clip(0).astype(np.int32)
    table = rng.standard_normal((M, B, model.d_o)).astype(np.float32)
    U = rng.integers(0, 2**32, M, dtype=np.uint64).astype(np.uint32)
    return dict(succ=succ, seg=seg, actions=actions, visits=visits, children=children, table=table, U=U)


def run_dev(V, m, c, k_o=1.0, alpha_o=0.5, lam=0.8, seed=1234, status=None):
    ch = dev(c["children"], torch.int32)
    tab = dev(c["table"])
    res = V.pw_step(m, dev(c["succ"]), dev(c["seg"], torch.int32),
                    dev(c["actions"], torch.int32 if c["actions"].dtype == np.int32 else torch.float32),
                    dev(c["visits"], torch.int32), ch, tab, dev(c["U"].view(np.int32), torch.int32), k_o, alpha_o,
                    lam=lam, seed=seed, status=status)
    torch.cuda.synchronize()
    out = {k: host(v) for k, v in res.items()}
    out["children"] = host(ch)
    out["table"] = host(tab)
    return out


def check_groups(c, d, lam, groups=None):
    """Weights / statistics from the device's own log-likelihoods, indices
    given the device's weights, gathered rows."""
    seg = c["seg"]
    for g in (range(len(seg) - 1) if groups is None else groups):
        lo, hi = seg[g], seg[g + 1]
        if hi == lo:
            assert d["branch"][g] == -1 and d["widen"][g] == 0
            continue
        w_ref, st_ref = oracle.normalize(d["loglik"][lo:hi].astype(np.float64), lam)
        wd = d["w"][lo:hi]
        assert np.max(np.abs(wd - w_ref) / np.maximum(w_ref, 1e-300)) <= 1e-13, g
        assert np.allclose(d["stats"][g], st_ref, rtol=1e-12, atol=1e-12), g
        idx_ref = oracle.resample(wd, int(c["U"][g]))
        assert np.array_equal(d["idx"][lo:hi], idx_ref), g
        assert np.array_equal(d["succ"][lo:hi], c["succ"][lo:hi][idx_ref]), g


def compare(V, model, c, compute, lam=0.8, seed=1234):
    m = V.Model(model, compute=compute)
    d = run_dev(V, m, c, lam=lam, seed=seed)
    r = oracle.pw_step(model, c["succ"], c["seg"], c["actions"], c["visits"], c["children"], c["table"], 1.0, 0.5,
                       lam, seed, c["U"], bf16=(compute == "bf16"))
    assert np.array_equal(d["widen"], r["widen"])
    assert np.array_equal(d["branch"], r["branch"])
    assert np.array_equal(d["children"], r["children"])
    e_tab = scaled_err(d["table"], r["obs_table"])
    e_ll = scaled_err(d["loglik"], r["loglik"])
    print(f"  {compute}: widened {int(d['widen'].sum())} of {len(d['widen'])}; table err {e_tab:.2e}, "
          f"loglik err {e_ll:.2e}", flush=True)
    bound = TOL if compute == "f32" else BOUND_EMUL
    assert e_tab <= bound and e_ll <= bound
    check_groups(c, d, lam)
    return d


@pytest.mark.parametrize("compute", ["f32", "bf16"])
def test_small_groups(V, compute):
    w = workloads.small(seed=61)
    print(f"pw step small {compute}", flush=True)
    compare(V, w.model, make_case(w.model, 61, M=45, d_max=300), compute)


def test_continuous_actions(V):
    w = workloads.continuous(seed=62)
    print("pw step continuous f32", flush=True)
    compare(V, w.model, make_case(w.model, 62, M=30, d_max=200), "f32")


@pytest.mark.parametrize("compute", ["f32", "bf16"])
def test_realistic_groups(V, compute):
    w = workloads.realistic(seed=63, N=8, K=1, H=1)
    print(f"pw step realistic {compute}", flush=True)
    compare(V, w.model, make_case(w.model, 63, M=24, d_max=700), compute)


def test_wide_groups(V):
    w = workloads.wide(seed=64, N=8, K=1, H=1)
    print("pw step width 1024 bf16", flush=True)
    compare(V, w.model, make_case(w.model, 64, M=12, d_max=150), "bf16")


def test_group_limit_sets_status(V):
    w = workloads.small(seed=65)
    c = make_case(w.model, 65, M=4, d_max=10)
    sizes = np.array([8192, 8193, 5, 0])
    c["seg"] = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int32)
    c["succ"] = np.random.default_rng(1).standard_normal((int(sizes.sum()), 4)).astype(np.float32)
    m = V.Model(w.model)
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    d = run_dev(V, m, c, status=st)
    assert int(st.item()) == V.VOILA_ERR_INVALID_ARG
    assert d["branch"][1] == -1 and d["widen"][1] == 0
    check_groups(c, d, 0.8, groups=[0, 2, 3])


def test_realistic_many_groups_sampled(V):
    # 2,048 action nodes with 1..2,000 successors each (~2 M successors), the
    # realistic networks; sampled groups checked against the oracle's steps
    w = workloads.realistic(seed=66, N=8, K=1, H=1)
    model = w.model
    c = make_case(model, 66, M=2048, d_max=2000, B=8)
    m = V.Model(model)
    seed, lam = 77, 0.8
    print(f"pw step realistic, {len(c['seg']) - 1} groups, {int(c['seg'][-1])} successors", flush=True)
    d = run_dev(V, m, c, lam=lam, seed=seed)
    rng = np.random.default_rng(5)
    groups = sorted(set([1, 2, 2047] + [int(x) for x in rng.integers(0, 2048, 10)]))
    key = [seed & 0xFFFFFFFF, seed >> 32]
    B = c["table"].shape[1]
    for g in groups:
        lo, hi = c["seg"][g], c["seg"][g + 1]
        if hi == lo:
            continue
        wid = oracle.pw_widen(c["visits"][g], c["children"][g], 1.0, 0.5, B)
        assert d["widen"][g] == wid
        if wid:
            assert d["branch"][g] == c["children"][g] and d["children"][g] == c["children"][g] + 1
            nz = oracle.normals(seed, 0, g, 0, 4, model.d_wz)
            o_ref = oracle.observe(model, c["succ"][lo][None, :], c["actions"][g][None, :], noise=nz[None, :])[0]
            assert scaled_err(d["table"][g, d["branch"][g]], o_ref) <= TOL
        else:
            word = oracle.philox([g, 1, 0, 6 << 16], key)[0]
            assert d["branch"][g] == int(np.floor(oracle.uniform(word) * c["children"][g]))
        o = d["table"][g, d["branch"][g]].astype(np.float64)
        X = np.concatenate([c["succ"][lo:hi].astype(np.float64), np.tile(c["actions"][g], (hi - lo, 1)),
                            np.tile(o, (hi - lo, 1))], axis=1)
        ll = oracle.mlp(model.lik, X)[:, 0]
        assert scaled_err(d["loglik"][lo:hi], ll) <= TOL, g
    check_groups(c, d, lam, groups=groups)
    print(f"  {len(groups)} sampled groups match; widened {int(d['widen'].sum())}", flush=True)
