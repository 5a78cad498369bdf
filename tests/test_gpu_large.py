"""Beliefs above one workgroup (N > 8192): the multi-workgroup normalisation,
exact blocked prefix sum and two-level binary-search resampler against the
oracle -- indices bit-exact given the oracle's weights, weights within 1e-13
given the same log-likelihoods.

Above 2^20 particles the quantised weights keep b(N) = 52 - ceil(log2 N) < 32
fraction bits (31 at 2^20 + 1, 30 at 2^22, 28 at 2^24, 26 at 2^26), so the
offset is u = U >> (32 - b) and the output step 2^b is smaller; those sizes
are checked bit for bit too, with offsets whose dropped low bits are all set,
all clear, or random."""
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


@pytest.mark.parametrize("N", [8193, 50000, 1 << 20])
def test_large_resample_bit_exact(V, N):
    rng = np.random.default_rng(N)
    cases = [np.full(N, 1.0 / N), rng.dirichlet(np.full(N, 0.2))]
    oh = np.zeros(N)
    oh[N // 3] = 1.0
    cases.append(oh)
    z = rng.dirichlet(np.ones(N))
    z[rng.integers(0, N, N // 3)] = 0.0
    cases.append(z / z.sum())
    for ci, wv in enumerate(cases):
        for U in [0, 0xFFFFFFFF, int(rng.integers(0, 2**32))]:
            print(f"large resample N={N} case {ci} U={U}", flush=True)
            idx = V.resample(dev(wv, torch.float64), U)
            torch.cuda.synchronize()
            assert np.array_equal(idx.cpu().numpy(), oracle.resample(wv, U)), (N, ci, U)


def weight_cases(rng, N, full=True):
    """Uniform, one-hot, sparse Dirichlet and zero-mass-subset weights."""
    cases = [np.full(N, 1.0 / N)]
    oh = np.zeros(N)
    oh[N // 3] = 1.0
    cases.append(oh)
    if full:
        cases.append(rng.dirichlet(np.full(N, 0.2)))
        z = rng.gamma(1.0, size=N)
        z[rng.integers(0, N, N // 3)] = 0.0
        cases.append(z / z.sum())
    else:
        g = rng.gamma(0.3, size=N)
        cases.append(g / g.sum())
    return cases


@pytest.mark.parametrize("N", [(1 << 20) + 1, 1 << 22, 1 << 24, 1 << 26])
def test_large_resample_reduced_fraction_bits(V, N):
    b = V.resample_bits(N)
    assert b == oracle.resample_bits(N) and b == 52 - (N - 1).bit_length() and b < 32
    rng = np.random.default_rng(N + 1)
    drop = 32 - b
    Us = [0, 0xFFFFFFFF, (1 << drop) - 1, 1 << drop, int(rng.integers(0, 2**32))]
    for ci, wv in enumerate(weight_cases(rng, N, full=N <= (1 << 24))):
        wd = dev(wv, torch.float64)
        for U in (Us if N <= (1 << 24) else Us[1:3]):
            print(f"large resample N={N} b={b} case {ci} U={U:#x}", flush=True)
            idx = V.resample(wd, U)
            torch.cuda.synchronize()
            got = idx.cpu().numpy()
            ref = oracle.resample(wv, U)
            assert np.array_equal(got, ref), (N, ci, U, int(np.sum(got != ref)))
            if ci == 0:
                assert np.array_equal(got, np.arange(N))  # uniform weights: the identity
        del wd


@pytest.mark.parametrize("N", [(1 << 20) + 1, 1 << 22, 1 << 24])
def test_reweight_resample_reduced_fraction_bits(V, N):
    """The fused weights + resampling path above 2^20 particles: weights
    within 1e-13 of the oracle's, indices bit-exact given them, rows gathered."""
    rng = np.random.default_rng(N + 5)
    ll = (rng.standard_normal(N) * 3).astype(np.float32)
    src = rng.standard_normal((N, 16)).astype(np.float32)
    U = int(rng.integers(0, 2**32)) | ((1 << (32 - V.resample_bits(N))) - 1)
    print(f"reweight_resample N={N} b={V.resample_bits(N)} U={U:#x}", flush=True)
    out = V.reweight_resample(dev(ll), U, 1.0, src=dev(src), want_w=True)
    torch.cuda.synchronize()
    w = out["w"].cpu().numpy()
    wr, sr = oracle.normalize(ll.astype(np.float64), 1.0)
    assert np.max(np.abs(w - wr) / wr) < 1e-13
    st = out["stats"].cpu().numpy()
    assert abs(st[0] - sr[0]) / abs(sr[0]) < 1e-12
    # ESS = 1 / sum w^2: the oracle sums the N squares in sequence, whose
    # rounding error alone can reach (N - 1) 2^-53 of the sum
    assert abs(st[1] - sr[1]) / sr[1] <= max(1e-12, 2 * N * 2.0 ** -53)
    idx = out["idx"].cpu().numpy()
    assert np.array_equal(idx, oracle.resample(w, U))
    assert np.array_equal(out["dst"].cpu().numpy(), src[idx])


def test_large_resample_gathers_rows(V):
    rng = np.random.default_rng(3)
    N = 30000
    wv = rng.dirichlet(np.ones(N))
    src = rng.standard_normal((N, 16)).astype(np.float32)
    idx, dst = V.resample(dev(wv, torch.float64), 99, src=dev(src))
    torch.cuda.synchronize()
    ref = oracle.resample(wv, 99)
    assert np.array_equal(idx.cpu().numpy(), ref)
    assert np.array_equal(dst.cpu().numpy(), src[ref])


@pytest.mark.parametrize("N", [8193, 100000])
def test_large_normalize(V, N):
    rng = np.random.default_rng(N)
    ll = (rng.standard_normal(N) * 4).astype(np.float32)
    for lam, prior in [(1.0, None), (1.25, rng.dirichlet(np.ones(N)))]:
        w, st = V.normalize(dev(ll), lam, None if prior is None else dev(prior, torch.float64))
        torch.cuda.synchronize()
        wr, sr = oracle.normalize(ll.astype(np.float64), lam, prior)
        assert np.max(np.abs(w.cpu().numpy() - wr) / wr) < 1e-13
        assert np.max(np.abs(st.cpu().numpy() - sr) / np.abs(sr)) < 1e-12
    w, st = V.normalize(dev(np.full(N, 0.5, np.float32)), 1.0)
    torch.cuda.synchronize()
    assert np.all(w.cpu().numpy() == 1.0 / N)


def test_large_update_matches_oracle(V):
    w = workloads.small(seed=41, N=20000)
    m = V.Model(w.model)
    o = oracle.draw_observation(w).astype(np.float32)
    out = V.update(m, dev(w.states), w.update_action, o, lam=w.lam, seed=w.update_seed, U=w.resample_u)
    torch.cuda.synchronize()
    ref = oracle.update(w.model, w.states, w.update_action, o, lam=w.lam, seed=w.update_seed, U=w.resample_u)
    prop = out["prop"].cpu().numpy()
    assert np.max(np.abs(prop - ref["S_prop"])) <= 1e-5 * np.max(np.abs(ref["S_prop"]))
    wd, st = oracle.normalize(out["loglik"].cpu().numpy().astype(np.float64), w.lam)
    assert np.max(np.abs(out["w"].cpu().numpy() - wd) / wd) < 1e-12
    idx = out["idx"].cpu().numpy()
    assert np.array_equal(idx, oracle.resample(out["w"].cpu().numpy(), w.resample_u))
    assert np.array_equal(out["states"].cpu().numpy(), prop[idx])


def test_large_zero_mass_sets_status(V):
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    V.resample(dev(np.zeros(20000), torch.float64), 5, status=st)
    torch.cuda.synchronize()
    assert int(st.item()) == V.VOILA_ERR_NUMERIC


@pytest.mark.parametrize("N", [1000, 8192, 8193, 300000])
def test_reweight_resample_fused(V, N):
    """The one-call weights + resampling path: weights within 1e-13 of the
    oracle's, indices bit-exact with the oracle's resampler on those weights,
    and identical to the two-call normalise-then-resample path."""
    rng = np.random.default_rng(N + 7)
    ll = (rng.standard_normal(N) * 3).astype(np.float32)
    src = rng.standard_normal((N, 8)).astype(np.float32)
    U = int(rng.integers(0, 2**32))
    for lam, prior in [(1.0, None), (0.7, rng.dirichlet(np.ones(N)))]:
        pw = None if prior is None else dev(prior, torch.float64)
        print(f"reweight_resample N={N} lam={lam}", flush=True)
        out = V.reweight_resample(dev(ll), U, lam, prior_w=pw, src=dev(src), want_w=True)
        w2, st2 = V.normalize(dev(ll), lam, pw)
        idx2 = V.resample(w2, U)
        torch.cuda.synchronize()
        w = out["w"].cpu().numpy()
        wr, sr = oracle.normalize(ll.astype(np.float64), lam, prior)
        assert np.max(np.abs(w - wr) / wr) < 1e-13
        assert np.max(np.abs(out["stats"].cpu().numpy() - sr) / np.abs(sr)) < 1e-12
        idx = out["idx"].cpu().numpy()
        assert np.array_equal(idx, oracle.resample(w, U))
        assert np.array_equal(out["dst"].cpu().numpy(), src[idx])
        assert np.array_equal(w, w2.cpu().numpy()) and np.array_equal(idx, idx2.cpu().numpy())


def test_large_update_without_index_output(V):
    # the gather reads the indices back from the workspace when the caller keeps none
    w = workloads.small(seed=43, N=30000)
    m = V.Model(w.model)
    o = oracle.draw_observation(w).astype(np.float32)
    a = V.update(m, dev(w.states), w.update_action, o, lam=w.lam, seed=w.update_seed, U=w.resample_u)
    b = V.update(m, dev(w.states), w.update_action, o, lam=w.lam, seed=w.update_seed, U=w.resample_u,
                 want_idx=False)
    torch.cuda.synchronize()
    assert b["idx"] is None
    assert torch.equal(a["states"], b["states"])
