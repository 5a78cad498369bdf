"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Tolerances (binary32 network arithmetic):
* Q and per-rollout returns G: relative error <= 1e-5.  The oracle's own
  sensitivity to a one-ulp binary32 perturbation of every input and weight is
  below ~10 ulps per rollout for these networks, so binary32 evaluation in a
  different summation order stays well inside 1e-5.
* proposal states, observations and log-likelihoods: every element within
  1e-5 of the array's scale, i.e. max_i |got_i - ref_i| <= 1e-5 max_i |ref_i|
  (an element-wise relative bound is ill-posed for entries near zero, such
  as a state coordinate or a log-likelihood that crosses zero).
* normalised weights from the same binary32 log-likelihoods: relative 1e-13
  (binary64 exp / log of two libraries differ by an ulp or so).
* resampling indices given the oracle's weights: bit-exact.
"""
import numpy as np
import pytest
import torch

import oracle
import workloads

pytestmark = pytest.mark.gpu

V = None
TOL = 1e-5


@pytest.fixture(scope="module", autouse=True)
def _lib():
    global V
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2606_19729_amd as lib
    V = lib
    yield


def dev(a, dtype=torch.float32):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def host(t):
    return t.detach().cpu().numpy().astype(np.float64)


def max_rel(got, ref):
    got, ref = np.asarray(got, np.float64), np.asarray(ref, np.float64)
    return float(np.max(np.abs(got - ref) / np.maximum(np.abs(ref), 1e-300)))


def scaled_err(got, ref):
    got, ref = np.asarray(got, np.float64), np.asarray(ref, np.float64)
    return float(np.max(np.abs(got - ref)) / max(np.max(np.abs(ref)), 1e-30))


def cands_dev(w):
    return dev(w.cands, torch.int32 if w.model.n_actions > 0 else torch.float32)


def say(*a):
    print(*a, flush=True)


# ----------------------------------------------------------------------------- RNG
def test_philox_words_and_normals_match_oracle():
    seed = 0x0123456789ABCDEF
    for (c1, c2, stream, d) in [(0, 0, 3, 4), (7, 11, 5, 16), (3, 0, 4, 2), (0xFFFFFFFF, 5, 3, 13)]:
        say("philox case", c1, c2, stream, d)
        z, words = V.philox_normals(seed, 1000, c1, c2, stream, 300, d)
        torch.cuda.synchronize()
        words = words.cpu().numpy().view(np.uint32)
        z = z.cpu().numpy().astype(np.float64)
        for r in [0, 1, 77, 299]:
            nb = (d + 3) // 4
            for b in range(nb):
                ref = oracle.philox([1000 + r, c1, c2, (stream << 16) | b], [seed & 0xFFFFFFFF, seed >> 32])
                assert np.array_equal(words[r, 4 * b:4 * b + 4], ref)
            refz = oracle.normals(seed, 1000 + r, c1, c2, stream, d)
            assert np.max(np.abs(z[r] - refz)) < 4e-6 * max(1.0, np.max(np.abs(refz)))


# ----------------------------------------------------------------------------- plan
def run_plan(w, compute="f32", noise=None, seed=None, **kw):
    m = V.Model(w.model, compute=compute)
    q, G = V.plan(m, dev(w.states), cands_dev(w), w.gamma, w.goal,
                  seed=w.plan_seed if seed is None else seed,
                  noise=None if noise is None else dev(noise), return_G=True, **kw)
    torch.cuda.synchronize()
    return host(q), host(G)


def check_plan(w, noise=None, reward_at=0, crn=False, belief_w=None, tol=TOL):
    kw = dict(reward_at=reward_at, crn=crn)
    if belief_w is not None:
        kw["belief_w"] = dev(belief_w, torch.float64)
    q, G = run_plan(w, noise=noise, **kw)
    Qr, Gr = oracle.plan(w.model, w.states, w.cands, w.gamma, w.goal, belief_w=belief_w, noise=noise,
                         seed=w.plan_seed, crn=crn, reward_at=reward_at, return_G=True)
    eq, eg = max_rel(q, Qr), max_rel(G, Gr)
    say(f"  {w.name} K={w.K} N={w.N} H={w.H} noise={'explicit' if noise is not None else 'philox'} "
        f"max rel err Q={eq:.2e} G={eg:.2e}")
    assert eq <= tol and eg <= tol
    return q, G


def test_plan_small_explicit_noise():
    w = workloads.small()
    check_plan(w, noise=workloads.explicit_plan_noise(w))


def test_plan_small_philox():
    check_plan(workloads.small())


@pytest.mark.parametrize("N,K,H", [(1, 1, 1), (33, 3, 7), (100, 2, 0), (31, 5, 4), (257, 4, 3)])
def test_plan_small_ragged_sizes(N, K, H):
    w = workloads.small(seed=N + K + H, N=N, K=K, H=H)
    check_plan(w)
    check_plan(w, noise=workloads.explicit_plan_noise(w))


def test_plan_options():
    w = workloads.small(seed=9, N=70, K=6, H=5)
    check_plan(w, reward_at=1)
    bw = np.random.default_rng(2).dirichlet(np.ones(70))
    check_plan(w, belief_w=bw)
    check_plan(w, crn=True)


def test_plan_crn_identical_candidates_are_bitwise_equal():
    w = workloads.small(seed=3, N=64, K=4, H=6)
    w.cands[:] = w.cands[0]
    q, G = run_plan(w, crn=True)
    assert np.all(q == q[0]) and np.all(G == G[0])
    q2, _ = run_plan(w, crn=False)
    assert not np.all(q2 == q2[0])


def test_plan_is_deterministic():
    w = workloads.small(seed=5, N=300, K=17, H=9)
    a = run_plan(w)
    b = run_plan(w)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_plan_bad_action_sets_status():
    w = workloads.small(seed=4, N=40, K=3, H=4)
    w.cands[1, 2] = 7
    m = V.Model(w.model)
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    V.plan(m, dev(w.states), cands_dev(w), w.gamma, w.goal, seed=1, status=st)
    torch.cuda.synchronize()
    assert int(st.item()) == V.VOILA_ERR_INVALID_ARG


def test_plan_realistic_reduced():
    w = workloads.realistic(N=70, K=6, H=5)
    check_plan(w)
    check_plan(w, noise=workloads.explicit_plan_noise(w))


def test_plan_realistic_full_size_sampled():
    # the benchmark's launch configuration (1024 x 4096 x 20); the oracle
    # recomputes 64 sampled rollouts and the full Q of two candidates
    w = workloads.realistic()
    q, G = run_plan(w)
    rng = np.random.default_rng(0)
    pairs = [(int(rng.integers(0, w.K)), int(rng.integers(0, w.N))) for _ in range(64)]
    g_ref = oracle.rollouts(w.model, w.states, w.cands, w.gamma, w.goal, pairs, seed=w.plan_seed)
    e = max_rel([G[k, i] for k, i in pairs], g_ref)
    say(f"  sampled rollouts max rel err {e:.2e}")
    assert e <= TOL
    for k in [0, w.K - 1]:
        gk = oracle.rollouts(w.model, w.states, w.cands, w.gamma, w.goal, [(k, i) for i in range(w.N)],
                             seed=w.plan_seed)
        qk = oracle.weighted_mean(gk)
        say(f"  Q[{k}] rel err {max_rel(q[k], qk):.2e}")
        assert max_rel(q[k], qk) <= TOL
    # Q is the mean of the returns for every candidate
    assert max_rel(q, G.mean(axis=1)) <= 1e-6


# ----------------------------------------------------------------------------- update stages
@pytest.mark.parametrize("N", [1, 2, 31, 128, 1000, 4096, 8192])
def test_normalize_matches_oracle(N):
    rng = np.random.default_rng(N)
    ll = (rng.standard_normal(N) * 3).astype(np.float32)
    for lam, prior in [(1.0, None), (1.25, None), (1.0, rng.dirichlet(np.ones(N)))]:
        w, st = V.normalize(dev(ll), lam, None if prior is None else dev(prior, torch.float64))
        torch.cuda.synchronize()
        wr, sr = oracle.normalize(ll.astype(np.float64), lam, prior)
        assert max_rel(host(w), wr) < 1e-13
        assert max_rel(host(st), sr) < 1e-13
    w, st = V.normalize(dev(np.full(N, -2.0, np.float32)), 1.25)
    torch.cuda.synchronize()
    assert np.all(host(w) == 1.0 / N)
    assert host(st)[0] == pytest.approx(-1.6, abs=1e-15)


def _weight_cases(N, rng):
    yield np.full(N, 1.0 / N)
    oh = np.zeros(N)
    oh[(3 * N) // 7] = 1.0
    yield oh
    for conc in [0.05, 1.0, 20.0]:
        w = rng.dirichlet(np.full(N, conc))
        if N > 4:
            w[rng.integers(0, N, N // 5)] = 0.0
            w /= w.sum()
        yield w


@pytest.mark.parametrize("N", [1, 2, 31, 128, 1000, 4096, 8191, 8192])
def test_resample_bit_exact_given_oracle_weights(N):
    rng = np.random.default_rng(100 + N)
    for wv in _weight_cases(N, rng):
        for U in [0, 0xFFFFFFFF, int(rng.integers(0, 2**32))]:
            idx = V.resample(dev(wv, torch.float64), U)
            torch.cuda.synchronize()
            ref = oracle.resample(wv, U)
            assert np.array_equal(idx.cpu().numpy(), ref), (N, U)


def test_resample_gathers_rows_and_flags_zero_mass():
    rng = np.random.default_rng(1)
    wv = rng.dirichlet(np.ones(500))
    src = rng.standard_normal((500, 16)).astype(np.float32)
    idx, dst = V.resample(dev(wv, torch.float64), 12345, src=dev(src))
    torch.cuda.synchronize()
    ref = oracle.resample(wv, 12345)
    assert np.array_equal(idx.cpu().numpy(), ref)
    assert np.array_equal(dst.cpu().numpy(), src[ref])
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    V.resample(dev(np.zeros(64), torch.float64), 1, status=st)
    torch.cuda.synchronize()
    assert int(st.item()) == V.VOILA_ERR_NUMERIC


# ----------------------------------------------------------------------------- observe / update
def test_observe_matches_oracle():
    for w in [workloads.small(N=77), workloads.realistic(N=90, K=1, H=1)]:
        m = V.Model(w.model)
        a = w.update_action
        noise = np.random.default_rng(3).standard_normal((w.N, w.model.d_wz)).astype(np.float32)
        for nz in [noise, None]:
            o = V.observe(m, dev(w.states), a, seed=99, noise=None if nz is None else dev(nz))
            torch.cuda.synchronize()
            acts = [int(a)] * w.N if w.model.n_actions > 0 else np.repeat(np.asarray(a)[None], w.N, 0)
            ref = oracle.observe(w.model, w.states, acts, noise=nz, seed=99)
            e = scaled_err(host(o), ref)
            say(f"  observe {w.name} noise={'explicit' if nz is not None else 'philox'} err {e:.2e}")
            assert e <= TOL


def check_update(w, noise=None, prior=None):
    m = V.Model(w.model)
    o = oracle.draw_observation(w).astype(np.float32)
    out = V.update(m, dev(w.states), w.update_action, o, lam=w.lam,
                   prior_w=None if prior is None else dev(prior, torch.float64), seed=w.update_seed,
                   U=w.resample_u, noise=None if noise is None else dev(noise))
    torch.cuda.synchronize()
    ref = oracle.update(w.model, w.states, w.update_action, o, lam=w.lam, prior_w=prior, noise=noise,
                        seed=w.update_seed, U=w.resample_u)
    e_prop = scaled_err(host(out["prop"]), ref["S_prop"])
    e_ll = scaled_err(host(out["loglik"]), ref["loglik"])
    # weights from the device's binary32 log-likelihoods, normalised by the oracle
    w_from_dev, st_from_dev = oracle.normalize(host(out["loglik"]), w.lam, prior)
    e_w = max_rel(host(out["w"]), w_from_dev)
    e_w_ref = scaled_err(host(out["w"]), ref["w"])
    say(f"  update {w.name} N={w.N}: prop {e_prop:.2e} loglik {e_ll:.2e} w(same l) {e_w:.2e} "
        f"w(vs fp64) {e_w_ref:.2e} stats {host(out['stats'])} vs {ref['stats']}")
    assert e_prop <= TOL and e_ll <= TOL
    assert e_w <= 1e-12
    assert max_rel(host(out["stats"]), st_from_dev) <= 1e-12
    # resampling of the device weights is bit-exact with the definition
    idx = out["idx"].cpu().numpy()
    assert np.array_equal(idx, oracle.resample(host(out["w"]), w.resample_u))
    assert np.array_equal(host(out["states"]), host(out["prop"])[idx])
    return out, ref


def test_update_small():
    w = workloads.small()
    check_update(w, noise=workloads.explicit_update_noise(w))
    check_update(w)
    check_update(w, prior=np.random.default_rng(5).dirichlet(np.ones(w.N)))


@pytest.mark.parametrize("N", [1, 37, 8192])
def test_update_small_sizes(N):
    check_update(workloads.small(seed=N, N=N))


def test_update_realistic():
    w = workloads.realistic(K=1, H=1)
    check_update(w)


def test_update_nonfinite_likelihood_sets_status():
    w = workloads.small(N=50)
    m_desc = w.model
    W, b = m_desc.lik[-1]
    bad = workloads.Model(**{**m_desc.__dict__, "lik": m_desc.lik[:-1] + [(W, np.full_like(b, np.inf))]})
    m = V.Model(bad)
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    V.update(m, dev(w.states), 2, np.zeros(2, np.float32), seed=1, U=1, status=st)
    torch.cuda.synchronize()
    assert int(st.item()) == V.VOILA_ERR_NUMERIC


def test_update_is_deterministic():
    w = workloads.realistic(N=1000, K=1, H=1)
    m = V.Model(w.model)
    o = np.zeros(w.model.d_o, np.float32)
    a = V.update(m, dev(w.states), w.update_action, o, seed=3, U=7)
    b = V.update(m, dev(w.states), w.update_action, o, seed=3, U=7)
    torch.cuda.synchronize()
    for k in ["states", "idx", "w", "loglik", "stats"]:
        assert torch.equal(a[k], b[k]), k
