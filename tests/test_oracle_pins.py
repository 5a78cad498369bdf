"""Pins of the FP64 oracle against facts that do not come from the oracle.

The paper prints no worked numeric example of its generators, weights or
resampling, so every pin here is a closed form, an invariant, an independent
library routine or an independent implementation:

* Philox4x32-10 against rocRAND's engine run on the host;
* networks against numpy matrix products, bfloat16 rounding against torch;
* plan against the closed-form Gaussian propagation of a generator whose
  ReLUs are all active (the network is then affine), and special cases
  (H = 0, gamma = 0, constant state, common random numbers, the shift between
  the two reward timings);
* normalisation against scipy's logsumexp and exact special cases;
* resampling against numpy's searchsorted, the copy-count bounds of
  systematic resampling, exact unbiasedness over the offset, and a
  count-based formulation;
* the whole update against the exponential-tilting closed form of a
  Gaussian proposal weighted by an affine log-likelihood.
"""
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest
import scipy.special
import torch

import oracle
import workloads
from workloads import Model

HERE = os.path.dirname(os.path.abspath(__file__))


# ----------------------------------------------------------------------------- RNG
@pytest.fixture(scope="module")
def rocrand_host():
    if shutil.which("hipcc") is None:
        pytest.skip("hipcc not available")
    d = tempfile.mkdtemp()
    exe = os.path.join(d, "rr")
    subprocess.run(["hipcc", "-O1", "-x", "hip", "--offload-arch=gfx950", "-w",
                    os.path.join(HERE, "rocrand_philox_host.cpp"), "-o", exe], check=True)
    return exe


@pytest.mark.parametrize("seed", [0x123456789ABCDEF, 1, 0xFFFFFFFFFFFFFFFF])
def test_philox_matches_rocrand_engine(rocrand_host, seed):
    key = [seed & 0xFFFFFFFF, seed >> 32]
    # rocRAND's (subsequence, offset) move counter words 2-3 and 0-1; every word
    # of the counter and of the key is exercised.
    cases = [((0, 0), [0, 0, 0, 0]), ((0, 4), [1, 0, 0, 0]), ((1, 0), [0, 0, 1, 0]),
             ((1 << 32, 0), [0, 0, 0, 1]), ((0, 4 << 32), [0, 1, 0, 0]),
             ((0x00050003, 4 * 0x0000000700000009), [9, 7, 0x00050003, 0])]
    for (sub, off), ctr in cases:
        out = subprocess.run([rocrand_host, hex(seed), hex(sub), hex(off), "4"], check=True,
                             capture_output=True, text=True).stdout.split()
        ref = [int(x, 16) for x in out]
        got = [int(x) for x in oracle.philox(ctr, key)]
        assert got == ref, (hex(seed), ctr)


def test_uniform_is_open_and_exact_in_binary32():
    for x in [0, 1, 511, 512, 0x7FFFFFFF, 0xFFFFFFFF, 0x12345678]:
        u = oracle.uniform(x)
        assert 0.0 < u < 1.0
        assert float(np.float32(u)) == u
    assert oracle.uniform(0) == 2.0 ** -24
    assert oracle.uniform(0xFFFFFFFF) == 1.0 - 2.0 ** -24


def test_box_muller_moments():
    z = np.concatenate([oracle.normals(77, i, 3, 5, 3, 16) for i in range(8000)])
    n = z.size
    assert abs(z.mean()) < 5 / np.sqrt(n)
    assert abs(z.var() - 1.0) < 5 * np.sqrt(2.0 / n)
    assert abs(scipy.stats.skew(z)) < 5 * np.sqrt(6.0 / n)
    assert abs(scipy.stats.kurtosis(z)) < 5 * np.sqrt(24.0 / n)
    # the two draws of a pair share the radius: z0^2 + z1^2 = -2 ln u0
    w = oracle.philox([4, 0, 0, (3 << 16) | 0], [9, 0])
    zz = oracle.normals(9, 4, 0, 0, 3, 4)
    assert np.isclose(zz[0] ** 2 + zz[1] ** 2, -2 * np.log(oracle.uniform(w[0])), rtol=1e-13)
    assert np.isclose(zz[2] ** 2 + zz[3] ** 2, -2 * np.log(oracle.uniform(w[2])), rtol=1e-13)


def test_normals_are_prefix_consistent_and_counter_separated():
    a = oracle.normals(5, 1, 2, 3, 3, 7)
    b = oracle.normals(5, 1, 2, 3, 3, 16)
    assert np.array_equal(a, b[:7])
    assert not np.allclose(oracle.normals(5, 1, 2, 4, 3, 4), oracle.normals(5, 1, 2, 3, 3, 4))
    assert not np.allclose(oracle.normals(5, 1, 2, 3, 4, 4), oracle.normals(5, 1, 2, 3, 3, 4))


# ----------------------------------------------------------------------------- networks
def _numpy_mlp(layers, X):
    h = np.asarray(X, np.float64)
    for j, (W, b) in enumerate(layers):
        h = h @ np.asarray(W, np.float64).T + np.asarray(b, np.float64)
        if j < len(layers) - 1:
            h = np.maximum(h, 0.0)
    return h


@pytest.mark.parametrize("dims", [[1, 1], [3, 5, 2], [5, 4, 3, 1], [2, 5, 5, 5, 4], [13, 64, 64, 4]])
def test_mlp_matches_numpy(dims):
    rng = np.random.default_rng(sum(dims))
    layers = workloads.random_mlp(rng, dims)
    X = rng.standard_normal((37, dims[0]))
    np.testing.assert_allclose(oracle.mlp(layers, X), _numpy_mlp(layers, X), rtol=1e-12, atol=1e-12)


def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(3)
    x = np.concatenate([rng.standard_normal(4000).astype(np.float32),
                        np.float32([1.0, -1.0, 1.00390625, 1.01171875, 3.0e-30, 65504.0, 0.0])])
    # exact ties in bfloat16: 1 + 2^-8 (-> 1), 1 + 3 * 2^-8 (-> 1 + 2^-6)
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(oracle.round_bf16(x), ref)


def test_mlp_bf16_mode_matches_numpy_with_rounded_operands():
    rng = np.random.default_rng(4)
    layers = workloads.random_mlp(rng, [6, 16, 16, 3])
    X = rng.standard_normal((20, 6)).astype(np.float32)
    rb = oracle.round_bf16
    h = rb(X)
    for j, (W, b) in enumerate(layers):
        h = h @ rb(W).T + np.asarray(b, np.float64)
        if j < len(layers) - 1:
            h = rb(np.maximum(h, 0.0))
    np.testing.assert_allclose(oracle.mlp(layers, X, bf16=True), h, rtol=1e-12, atol=1e-12)


# ----------------------------------------------------------------------------- affine generator
def affine_model(rng, d_s=4, n_actions=5, d_a=0, d_w=4, d_o=2, width=32, in_scale=0.08,
                 out_scale=0.05, bias=20.0, lik_scale=0.05):
    """Networks whose hidden ReLUs stay active on the inputs used here (large
    positive hidden biases, small first-layer weights), so that each network is
    an affine map of its input.  The output bias is re-centred so that the
    constant term of the affine map is small."""
    aw = n_actions if n_actions > 0 else d_a

    def net(d_in, d_out, first, last):
        W1 = (rng.standard_normal((width, d_in)) * first).astype(np.float32)
        b1 = np.full(width, bias, np.float32)
        W2 = (rng.standard_normal((width, width)) * 0.02).astype(np.float32)
        b2 = np.full(width, bias, np.float32)
        W3 = (rng.standard_normal((d_out, width)) * last).astype(np.float32)
        layers = [(W1, b1), (W2, b2), (W3, np.zeros(d_out, np.float32))]
        _, c = composite(layers)
        b3 = (-c + rng.standard_normal(d_out) * 0.1).astype(np.float32)
        return [(W1, b1), (W2, b2), (W3, b3)]

    m = Model(d_s=d_s, n_actions=n_actions, d_a=d_a, d_w=d_w, d_o=d_o, d_wz=d_o,
              trans=net(d_s + aw + d_w, d_s, in_scale, out_scale),
              obs=net(d_s + aw + d_o, d_o, in_scale, out_scale),
              lik=net(d_s + aw + d_o, 1, in_scale, lik_scale))
    return m


def composite(layers):
    """(A, c) with net(x) = A x + c when every ReLU is active."""
    A = np.eye(layers[0][0].shape[1])
    c = np.zeros(layers[0][0].shape[1])
    for W, b in layers:
        A = np.asarray(W, np.float64) @ A
        c = np.asarray(W, np.float64) @ c + np.asarray(b, np.float64)
    return A, c


def split_transition(m):
    A, c = composite(m.trans)
    aw = m.action_width
    As, Aa, Aw = A[:, :m.d_s], A[:, m.d_s:m.d_s + aw], A[:, m.d_s + aw:]
    return np.eye(m.d_s) + As, Aa, Aw, c


def test_affine_generator_one_step_is_affine():
    rng = np.random.default_rng(10)
    m = affine_model(rng)
    F, B, C, c = split_transition(m)
    S = rng.standard_normal((50, 4))
    a = rng.integers(0, 5, 50)
    w = rng.standard_normal((50, 4))
    ref = S @ F.T + B[:, a].T + w @ C.T + c
    np.testing.assert_allclose(oracle.transition(m, S, a, w), ref, rtol=1e-10, atol=1e-10)


def closed_form_q(m, states, cands, gamma, goal):
    """E[Q_k] under s_{t+1} = F s_t + B a_t + C w + c, w ~ N(0, I)."""
    F, B, C, c = split_transition(m)
    K, H = cands.shape[0], cands.shape[1]
    out = np.zeros(K)
    for k in range(K):
        mu = np.asarray(states, np.float64).copy()      # [N, d_s], one mean per particle
        Sig = np.zeros((m.d_s, m.d_s))
        disc, acc = 1.0, np.zeros(mu.shape[0])
        for t in range(H):
            act = B[:, cands[k, t]] if m.n_actions > 0 else B @ cands[k, t]
            mu = mu @ F.T + act + c
            Sig = F @ Sig @ F.T + C @ C.T
            acc += disc * -(((mu - goal) ** 2).sum(1) + np.trace(Sig))
            disc *= gamma
        out[k] = acc.mean()
    return out


@pytest.mark.parametrize("noise_source", ["philox", "explicit"])
def test_plan_matches_gaussian_propagation(noise_source):
    rng = np.random.default_rng(11)
    m = affine_model(rng)
    N, K, H = 3000, 4, 8
    states = (rng.standard_normal((N, 4)) * 0.5).astype(np.float32)
    cands = rng.integers(0, 5, (K, H)).astype(np.int32)
    goal = np.array([1, 1, 0, 0], np.float32)
    noise = None if noise_source == "philox" else rng.standard_normal((K, N, H, 4)).astype(np.float32)
    Q, G = oracle.plan(m, states, cands, 0.9, goal, noise=noise, seed=1234, return_G=True)
    ref = closed_form_q(m, states, cands, 0.9, goal)
    sigma = G.std(axis=1) / np.sqrt(N)
    assert np.all(np.abs(Q - ref) < 5 * sigma), (Q, ref, sigma)
    # the MC error is small compared with the value itself
    assert np.all(np.abs(Q - ref) < 0.05 * np.abs(ref))


def test_plan_continuous_actions_gaussian_propagation():
    rng = np.random.default_rng(12)
    m = affine_model(rng, d_s=6, n_actions=0, d_a=3, d_w=6, d_o=3)
    N, K, H = 3000, 3, 6
    states = (rng.standard_normal((N, 6)) * 0.5).astype(np.float32)
    cands = rng.uniform(-1, 1, (K, H, 3)).astype(np.float32)
    goal = np.zeros(6, np.float32)
    goal[:2] = 1
    Q, G = oracle.plan(m, states, cands, 0.97, goal, seed=99, return_G=True)
    ref = closed_form_q(m, states, cands, 0.97, goal)
    assert np.all(np.abs(Q - ref) < 5 * G.std(axis=1) / np.sqrt(N))


def test_plan_special_cases():
    w = workloads.small(N=16, K=6, H=5)
    m = w.model
    # H = 0: nothing accumulates
    Q0 = oracle.plan(m, w.states, w.cands[:, :0], w.gamma, w.goal, seed=1)
    assert np.array_equal(Q0, np.zeros(6))
    # gamma = 0: the first reward only, r_0 = R(s_1)
    Qg, G = oracle.plan(m, w.states, w.cands, 0.0, w.goal, seed=1, return_G=True)
    Q1 = oracle.plan(m, w.states, w.cands[:, :1], 0.7, w.goal, seed=1)
    np.testing.assert_allclose(Qg, Q1, rtol=1e-15)
    # constant state (zero output layer): Q = -mean ||s - g||^2 (1 - gamma^H) / (1 - gamma)
    zero = Model(**{**m.__dict__, "trans": m.trans[:-1] + [(np.zeros_like(m.trans[-1][0]),
                                                             np.zeros_like(m.trans[-1][1]))]})
    Qz = oracle.plan(zero, w.states, w.cands, w.gamma, w.goal, seed=1)
    d2 = ((w.states.astype(np.float64) - w.goal) ** 2).sum(1).mean()
    np.testing.assert_allclose(Qz, -d2 * (1 - w.gamma ** 5) / (1 - w.gamma), rtol=1e-13)
    # identical candidates under common random numbers give identical Q
    same = np.repeat(w.cands[:1], 3, axis=0)
    Qc = oracle.plan(m, w.states, same, w.gamma, w.goal, seed=5, crn=True)
    assert Qc[0] == Qc[1] == Qc[2]
    Qi = oracle.plan(m, w.states, same, w.gamma, w.goal, seed=5, crn=False)
    assert Qi[0] != Qi[1]
    # weighted belief: Q is the weighted mean of the per-particle returns
    bw = np.random.default_rng(1).dirichlet(np.ones(16))
    Qw, Gw = oracle.plan(m, w.states, w.cands, w.gamma, w.goal, belief_w=bw, seed=1, return_G=True)
    np.testing.assert_allclose(Qw, Gw @ bw, rtol=1e-13)


def test_reward_timing_shift_identity():
    # reward of the acted-from state over H steps equals R(s_0) plus gamma times
    # the arrival-reward return over the first H-1 steps (same noise).
    w = workloads.small(N=20, K=5, H=6)
    noise = workloads.explicit_plan_noise(w)
    Qcur = oracle.plan(w.model, w.states, w.cands, w.gamma, w.goal, noise=noise, reward_at=1)
    Qnext = oracle.plan(w.model, w.states, w.cands[:, :5], w.gamma, w.goal, noise=noise[:, :, :5], reward_at=0)
    r0 = -((w.states.astype(np.float64) - w.goal) ** 2).sum(1).mean()
    np.testing.assert_allclose(Qcur, r0 + w.gamma * Qnext, rtol=1e-12)


def test_rollouts_subset_matches_full_plan():
    w = workloads.small(N=12, K=7, H=4)
    Q, G = oracle.plan(w.model, w.states, w.cands, w.gamma, w.goal, seed=w.plan_seed, return_G=True)
    pairs = [(0, 0), (6, 11), (3, 5)]
    g = oracle.rollouts(w.model, w.states, w.cands, w.gamma, w.goal, pairs, seed=w.plan_seed)
    assert np.array_equal(g, np.array([G[k, i] for k, i in pairs]))


# ----------------------------------------------------------------------------- normalisation
def test_normalize_uniform_is_exact():
    for N in [1, 3, 128, 4096, 5000]:
        w, st = oracle.normalize(np.full(N, -3.25), lam=1.25)
        assert np.all(w == 1.0 / N)
        assert st[0] == pytest.approx(-3.25 / 1.25, abs=1e-15)
        assert st[1] == pytest.approx(N, rel=1e-12)


def test_normalize_against_logsumexp_and_invariances():
    rng = np.random.default_rng(21)
    ll = rng.standard_normal(1000) * 4
    for lam in [1.0, 1.25]:
        w, st = oracle.normalize(ll, lam=lam)
        ref_logz = scipy.special.logsumexp(ll / lam) - np.log(1000)
        assert st[0] == pytest.approx(ref_logz, rel=1e-13)
        ref_w = scipy.special.softmax(ll / lam)
        np.testing.assert_allclose(w, ref_w, rtol=1e-12)
        assert abs(w.sum() - 1) <= 1001 * 2.0 ** -53
        assert st[1] == pytest.approx(1.0 / (ref_w ** 2).sum(), rel=1e-12)
        w2, st2 = oracle.normalize(ll + 37.5, lam=lam)
        np.testing.assert_allclose(w2, w, rtol=1e-12)
        assert st2[0] == pytest.approx(st[0] + 37.5 / lam, rel=1e-13)
        w3, _ = oracle.normalize(ll / lam, lam=1.0)
        np.testing.assert_allclose(w3, w, rtol=1e-12)
    prior = rng.dirichlet(np.ones(1000))
    w, st = oracle.normalize(ll, lam=1.0, prior_w=prior)
    assert st[0] == pytest.approx(scipy.special.logsumexp(ll, b=prior), rel=1e-13)
    np.testing.assert_allclose(w, scipy.special.softmax(ll + np.log(prior)), rtol=1e-12)


def test_normalize_rejects_non_finite():
    with pytest.raises(oracle.OracleError):
        oracle.normalize(np.array([0.0, np.nan, 1.0]))
    with pytest.raises(oracle.OracleError):
        oracle.normalize(np.array([0.0, np.inf]))


# ----------------------------------------------------------------------------- resampling
def quantised_cumsum(w):
    N = len(w)
    b = oracle.resample_bits(N)
    q = np.rint(np.asarray(w, np.float64) * (N * 2.0 ** b))
    return np.cumsum(q), b


def test_resample_bits():
    assert oracle.resample_bits(1) == 32
    assert oracle.resample_bits(8192) == 32
    assert oracle.resample_bits(1 << 20) == 32
    assert oracle.resample_bits((1 << 20) + 1) == 31
    assert oracle.resample_bits(1 << 24) == 28


def test_resample_uniform_is_identity_and_one_hot_is_constant():
    for N in [1, 2, 5, 128, 4096, 8191]:
        w = np.full(N, 1.0 / N)
        for U in [0, 1, 0x80000000, 0xFFFFFFFF]:
            assert np.array_equal(oracle.resample(w, U), np.arange(N))
        oh = np.zeros(N)
        oh[N // 3] = 1.0
        assert np.all(oracle.resample(oh, 0x1234) == N // 3)


@pytest.mark.parametrize("N", [3, 17, 128, 1000, 4096])
def test_resample_matches_searchsorted_and_count_bounds(N):
    rng = np.random.default_rng(N)
    for trial in range(5):
        w = rng.dirichlet(np.full(N, 0.3))
        w[rng.integers(0, N, N // 4)] = 0.0
        w /= w.sum()
        U = int(rng.integers(0, 2**32))
        idx = oracle.resample(w, U)
        C, b = quantised_cumsum(w)
        P = np.arange(N, dtype=np.float64) * 2.0 ** b + (U >> (32 - b))
        ref = np.searchsorted(C, P, side="right")
        last = np.nonzero(np.diff(np.concatenate([[0.0], C])) > 0)[0][-1]
        ref = np.where(ref >= N, last, ref)
        assert np.array_equal(idx, ref)
        assert np.all(np.diff(idx) >= 0)
        counts = np.bincount(idx, minlength=N)
        assert counts.sum() == N
        assert np.all(counts[w == 0] == 0)
        top_edge = C[-1] != N * 2.0 ** b
        inner = np.ones(N, bool)
        if top_edge:
            inner[last] = False
        assert np.all(counts[inner] >= np.floor(N * w[inner] - 1e-9))
        assert np.all(counts[inner] <= np.ceil(N * w[inner] + 1e-9))


def test_resample_count_formulation():
    # copies of particle i = ceil((C_i - u) / 2^b) - ceil((C_{i-1} - u) / 2^b)
    rng = np.random.default_rng(5)
    N = 300
    w = rng.dirichlet(np.ones(N))
    U = 0xDEADBEEF
    C, b = quantised_cumsum(w)
    u = U >> (32 - b)
    Cm = np.concatenate([[0.0], C])
    start = np.ceil((Cm - u) / 2.0 ** b).clip(0, N)
    counts = np.diff(start).astype(int)
    assert np.array_equal(np.bincount(oracle.resample(w, U), minlength=N), counts)


def test_resample_is_exactly_unbiased_over_the_offset():
    # averaging the copy count of particle i over every offset u in [0, 2^b)
    # gives q_i / 2^b exactly; integrate the piecewise-constant count.
    rng = np.random.default_rng(6)
    N = 7
    w = rng.dirichlet(np.ones(N))
    C, b = quantised_cumsum(w)
    q = np.diff(np.concatenate([[0.0], C]))
    step = 2.0 ** b
    # breakpoints of the count as a function of u: C_i mod 2^b
    brk = np.unique(np.concatenate([[0.0, step], np.mod(C, step)]))
    mean = np.zeros(N)
    for lo, hi in zip(brk[:-1], brk[1:]):
        if hi <= lo:
            continue
        U = int(lo) << (32 - b)
        idx = oracle.resample(w, U)
        mean += np.bincount(idx, minlength=N) * (hi - lo) / step
    if C[-1] == N * step:
        np.testing.assert_allclose(mean, q / step, rtol=0, atol=1e-9)


def test_resample_quantisation_rounds_to_nearest():
    # N = 2, b = 32: q_0 = rint(w_0 * 2^33) = 2^31 + 1 for w_0 * 2^33 = 2^31 + 0.6;
    # with u = 2^31 the first output is the first particle only if q_0 was
    # rounded up (C_0 = 2^31 + 1 > u), the second if it was truncated
    w0 = (2.0 ** 31 + 0.6) / 2.0 ** 33
    w = np.array([w0, 1.0 - w0])
    assert oracle.resample_bits(2) == 32
    idx = oracle.resample(w, 1 << 31)
    assert idx[0] == 0
    w0 = (2.0 ** 31 + 0.4) / 2.0 ** 33  # rounds down: C_0 = 2^31 = u, not above it
    assert oracle.resample(np.array([w0, 1.0 - w0]), 1 << 31)[0] == 1


def test_resample_rejects_zero_mass():
    with pytest.raises(oracle.OracleError):
        oracle.resample(np.zeros(5), 0)


# ----------------------------------------------------------------------------- update
def test_update_matches_exponential_tilting():
    # all particles at one state: proposal s' ~ N(mu, C C^T); an affine
    # likelihood l = c.s' + d tilts it to mean mu + C C^T c / lambda, and
    # log E[exp(l / lambda)] = (c.mu + d) / lambda + c^T C C^T c / (2 lambda^2).
    rng = np.random.default_rng(31)
    m = affine_model(rng, width=32, in_scale=0.5, out_scale=1.0, lik_scale=0.5)
    F, B, C, c = split_transition(m)
    Al, cl = composite(m.lik)
    N = 1 << 15
    s0 = np.array([0.3, -0.2, 0.1, 0.5], np.float32)
    states = np.repeat(s0[None, :], N, axis=0)
    a = 2
    o = np.array([0.25, -0.5], np.float32)
    lam = 1.25
    out = oracle.update(m, states, a, o, lam=lam, seed=77, U=0x9E3779B9)
    mu = F @ s0 + B[:, a] + c
    Sig = C @ C.T
    grad = Al[0, :4]
    dconst = Al[0, 4:4 + 5] @ np.eye(5)[a] + Al[0, 9:] @ o + cl[0]
    tilted = mu + Sig @ grad / lam
    wmean = out["w"] @ out["S_prop"]
    sd = np.sqrt((out["w"][:, None] ** 2 * (out["S_prop"] - wmean) ** 2).sum(0))
    assert np.all(np.abs(wmean - tilted) < 5 * sd + 1e-12), (wmean, tilted, sd)
    assert np.linalg.norm(tilted - mu) > 10 * sd.max()  # the tilt is resolved
    logz = (grad @ mu + dconst) / lam + grad @ Sig @ grad / (2 * lam ** 2)
    ll = out["loglik"]
    sd_logz = np.exp(ll / lam - (ll / lam).max()).std() / np.exp(ll / lam - (ll / lam).max()).mean() / np.sqrt(N)
    assert abs(out["stats"][0] - logz) < 5 * sd_logz + 1e-12
    # resampled particles are proposal particles, and their mean follows the weights
    assert np.allclose(out["S_new"], out["S_prop"][out["idx"]])
    assert np.all(np.abs(out["S_new"].mean(0) - wmean) < 5 * sd + 1e-3)


def test_update_philox_noise_is_stream_5():
    w = workloads.small(N=40)
    o = oracle.draw_observation(w)
    a = oracle.update(w.model, w.states, w.update_action, o, seed=w.update_seed, U=w.resample_u)
    noise = np.stack([oracle.normals(w.update_seed, i, 0, 0, 5, w.model.d_w) for i in range(40)])
    b = oracle.update(w.model, w.states, w.update_action, o, noise=noise, U=w.resample_u)
    for key in ["S_prop", "loglik", "w", "stats", "idx", "S_new"]:
        assert np.array_equal(a[key], b[key]), key


def test_update_constant_likelihood_keeps_the_proposal_set():
    w = workloads.small(N=64)
    m = w.model
    flat = Model(**{**m.__dict__, "lik": m.lik[:-1] + [(np.zeros_like(m.lik[-1][0]),
                                                        np.full_like(m.lik[-1][1], 2.5))]})
    out = oracle.update(flat, w.states, 2, np.zeros(2), seed=3, U=12345)
    assert np.all(out["w"] == 1.0 / 64)
    assert np.array_equal(out["idx"], np.arange(64))
    assert np.array_equal(out["S_new"], out["S_prop"])
    assert out["stats"][0] == pytest.approx(2.5)


def test_observe_is_affine_for_the_affine_sampler():
    rng = np.random.default_rng(41)
    m = affine_model(rng)
    A, c = composite(m.obs)
    S = rng.standard_normal((30, 4))
    a = rng.integers(0, 5, 30)
    wz = rng.standard_normal((30, 2))
    X = np.concatenate([S, np.eye(5)[a], wz], axis=1)
    np.testing.assert_allclose(oracle.observe(m, S, a, noise=wz), X @ A.T + c, rtol=1e-10, atol=1e-10)


# ----------------------------------------------------------------------------- per-step observations
def affine_steps(m, states, cands, noise, obs_noise):
    """States and observations of every rollout step, written out with the
    affine maps of the two samplers (every ReLU active)."""
    F, B, C, c = split_transition(m)
    Az, cz = composite(m.obs)
    K, N, H = noise.shape[0], states.shape[0], noise.shape[2]
    aw = m.action_width
    traj = np.zeros((K, N, H, m.d_s))
    obs = np.zeros((K, N, H, m.d_o))
    for k in range(K):
        s = np.asarray(states, np.float64).copy()
        for t in range(H):
            a = np.eye(aw)[cands[k, t]] if m.n_actions > 0 else np.asarray(cands[k, t], np.float64)
            s = s @ F.T + a @ B.T + noise[k, :, t] @ C.T + c
            traj[k, :, t] = s
            x = np.concatenate([s, np.broadcast_to(a, (N, aw)), obs_noise[k, :, t]], axis=1)
            obs[k, :, t] = x @ Az.T + cz
    return traj, obs


@pytest.mark.parametrize("discrete", [True, False])
def test_plan_steps_follow_the_affine_samplers(discrete):
    rng = np.random.default_rng(43)
    m = affine_model(rng) if discrete else affine_model(rng, d_s=6, n_actions=0, d_a=3, d_w=6, d_o=3)
    N, K, H = 7, 3, 5
    states = (rng.standard_normal((N, m.d_s)) * 0.5).astype(np.float32)
    cands = rng.integers(0, 5, (K, H)).astype(np.int32) if discrete else \
        rng.uniform(-1, 1, (K, H, 3)).astype(np.float32)
    noise = rng.standard_normal((K, N, H, m.d_w)).astype(np.float32)
    obs_noise = rng.standard_normal((K, N, H, m.d_wz)).astype(np.float32)
    traj, obs = oracle.plan_steps(m, states, cands, noise=noise, obs_noise=obs_noise)
    rt, ro = affine_steps(m, states, cands, noise, obs_noise)
    np.testing.assert_allclose(traj, rt, rtol=1e-9, atol=1e-9)
    np.testing.assert_allclose(obs, ro, rtol=1e-9, atol=1e-9)


@pytest.mark.parametrize("crn", [False, True])
def test_plan_steps_counter_noise(crn):
    """Observation noise is stream 4 at counter (particle, candidate or 0 under
    common random numbers, step); the transition noise is the plan's."""
    rng = np.random.default_rng(44)
    m = affine_model(rng)
    N, K, H, seed = 5, 3, 4, 0xABCDEF012345
    states = (rng.standard_normal((N, 4)) * 0.5).astype(np.float32)
    cands = rng.integers(0, 5, (K, H)).astype(np.int32)
    noise = np.zeros((K, N, H, m.d_w))
    obs_noise = np.zeros((K, N, H, m.d_wz))
    for k in range(K):
        for i in range(N):
            for t in range(H):
                kk = 0 if crn else k
                noise[k, i, t] = oracle.normals(seed, i, kk, t, 3, m.d_w)
                obs_noise[k, i, t] = oracle.normals(seed, i, kk, t, 4, m.d_wz)
    traj, obs = oracle.plan_steps(m, states, cands, seed=seed, crn=crn)
    rt, ro = affine_steps(m, states, cands, noise, obs_noise)
    np.testing.assert_allclose(traj, rt, rtol=1e-9, atol=1e-9)
    np.testing.assert_allclose(obs, ro, rtol=1e-9, atol=1e-9)


def test_plan_steps_are_the_states_the_returns_are_taken_on():
    """The returns of plan are the discounted rewards of the written states."""
    w = workloads.small(N=16, K=4, H=6)
    goal = np.asarray(w.goal, np.float64)
    traj, obs = oracle.plan_steps(w.model, w.states, w.cands, seed=w.plan_seed)
    _, G = oracle.plan(w.model, w.states, w.cands, w.gamma, w.goal, seed=w.plan_seed, return_G=True)
    r = -((traj - goal) ** 2).sum(-1)                       # [K, N, H]
    G_ref = (r * w.gamma ** np.arange(w.H)).sum(-1)
    np.testing.assert_allclose(G, G_ref, rtol=1e-12, atol=1e-12)
    # each observation equals the observation sampler applied to its row
    acts = np.repeat(w.cands[:, None, :], w.N, axis=1)      # [K, N, H]
    nz = np.zeros((w.K, w.N, w.H, w.model.d_wz))
    for k in range(w.K):
        for i in range(w.N):
            for t in range(w.H):
                nz[k, i, t] = oracle.normals(w.plan_seed, i, k, t, 4, w.model.d_wz)
    o_ref = oracle.observe(w.model, traj.reshape(-1, w.model.d_s), acts.reshape(-1),
                           noise=nz.reshape(-1, w.model.d_wz))
    np.testing.assert_allclose(obs.reshape(-1, w.model.d_o), o_ref, rtol=0, atol=0)
    # H = 0 and K = 0 write nothing
    t0, o0 = oracle.plan_steps(w.model, w.states, w.cands[:, :0], seed=1)
    assert t0.shape == (w.K, w.N, 0, w.model.d_s) and o0.shape == (w.K, w.N, 0, w.model.d_o)


# ----------------------------------------------------------------------------- progressive widening
def test_pw_widen_matches_integer_forms():
    """|C| < k N^alpha in integer form where the threshold is exact:
    k = 1, alpha = 1/2 -> C^2 < N; k = 1/2, alpha = 1 -> 2C < N; plus the
    no-branch and capacity rules."""
    B = 16
    for N in range(0, 300):
        for C in range(0, B + 2):
            got1 = oracle.pw_widen(N, C, 1.0, 0.5, B)
            got2 = oracle.pw_widen(N, C, 0.5, 1.0, B)
            if C >= B:
                assert got1 == 0 and got2 == 0
            elif C == 0:
                assert got1 == 1 and got2 == 1
            else:
                assert got1 == int(C * C < N), (N, C)
                assert got2 == int(2 * C < N), (N, C)


def pw_case(seed, M=40, B=6, d_max=60, model=None):
    rng = np.random.default_rng(seed)
    w = workloads.small(seed=seed, N=8, K=1, H=1) if model is None else None
    m = model or w.model
    sizes = rng.integers(0, d_max, M)
    sizes[:3] = [0, 1, d_max]
    seg = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int32)
    T = int(seg[-1])
    succ = rng.standard_normal((T, m.d_s)).astype(np.float32)
    actions = rng.integers(0, m.n_actions, M).astype(np.int32) if m.n_actions > 0 else \
        rng.uniform(-1, 1, (M, m.d_a)).astype(np.float32)
    children = rng.integers(0, B + 1, M).astype(np.int32)
    visits = (children.astype(np.int64) ** 2 + rng.integers(-2, 3, M)).clip(0).astype(np.int32)
    table = rng.standard_normal((M, B, m.d_o)).astype(np.float32)
    U = rng.integers(0, 2**32, M, dtype=np.uint64).astype(np.uint32)
    return m, succ, seg, actions, visits, children, table, U


def test_pw_step_branch_choice_and_new_observations():
    m, succ, seg, actions, visits, children, table, U = pw_case(51)
    seed = 0x5EED
    out = oracle.pw_step(m, succ, seg, actions, visits, children, table, 1.0, 0.5, 1.0, seed, U)
    M, B = len(visits), table.shape[1]
    key = [seed & 0xFFFFFFFF, seed >> 32]
    n_new = n_reuse = 0
    for g in range(M):
        if seg[g + 1] == seg[g]:
            assert out["branch"][g] == -1 and out["widen"][g] == 0
            assert out["children"][g] == children[g]
            continue
        wid = oracle.pw_widen(visits[g], children[g], 1.0, 0.5, B)
        assert out["widen"][g] == wid
        if wid:
            n_new += 1
            assert out["branch"][g] == children[g] and out["children"][g] == children[g] + 1
            nz = oracle.normals(seed, 0, g, 0, 4, m.d_wz)
            o_ref = oracle.observe(m, succ[seg[g]][None, :], [int(actions[g])], noise=nz[None, :])[0]
            np.testing.assert_array_equal(out["obs_table"][g, children[g]], o_ref)
        else:
            n_reuse += 1
            word = oracle.philox([g, 1, 0, 6 << 16], key)[0]
            assert out["branch"][g] == int(np.floor(oracle.uniform(word) * children[g]))
            assert 0 <= out["branch"][g] < children[g]
            assert out["children"][g] == children[g]
        untouched = [b for b in range(B) if not (wid and b == children[g])]
        np.testing.assert_array_equal(out["obs_table"][g, untouched], np.asarray(table[g, untouched], np.float64))
    assert n_new > 5 and n_reuse > 5


def test_pw_step_groups_are_independent_updates():
    """Each group: l from the likelihood network against the chosen branch's
    observation, weights and resampling of the single-belief definitions."""
    m, succ, seg, actions, visits, children, table, U = pw_case(52)
    out = oracle.pw_step(m, succ, seg, actions, visits, children, table, 1.0, 0.5, 0.7, 99, U)
    aw = m.n_actions
    for g in range(len(visits)):
        lo, hi = seg[g], seg[g + 1]
        if hi == lo:
            continue
        o = out["obs_table"][g, out["branch"][g]]
        X = np.concatenate([succ[lo:hi].astype(np.float64), np.tile(np.eye(aw)[actions[g]], (hi - lo, 1)),
                            np.tile(o, (hi - lo, 1))], axis=1)
        ll = oracle.mlp(m.lik, X)[:, 0]
        np.testing.assert_array_equal(out["loglik"][lo:hi], ll)
        w, st = oracle.normalize(ll, 0.7)
        np.testing.assert_array_equal(out["w"][lo:hi], w)
        np.testing.assert_array_equal(out["stats"][g], st)
        idx = oracle.resample(w, U[g])
        np.testing.assert_array_equal(out["idx"][lo:hi], idx)
        np.testing.assert_array_equal(out["S_out"][lo:hi], succ[lo:hi][idx])


def test_pw_reused_branches_are_uniform():
    M, C = 5000, 5
    rng = np.random.default_rng(53)
    w = workloads.small(seed=53, N=8, K=1, H=1)
    m = w.model
    seg = np.arange(M + 1, dtype=np.int32)
    succ = rng.standard_normal((M, 4)).astype(np.float32)
    out = oracle.pw_step(m, succ, seg, np.zeros(M, np.int32), np.full(M, 4, np.int32), np.full(M, C, np.int32),
                         np.zeros((M, C, 2)), 1.0, 0.5, 1.0, 7, np.zeros(M, np.uint32))
    assert not out["widen"].any()
    counts = np.bincount(out["branch"], minlength=C)
    chi2 = ((counts - M / C) ** 2 / (M / C)).sum()
    assert chi2 < 20.5   # 4 degrees of freedom, p ~ 4e-4


# ----------------------------------------------------------------------------- soft value
def test_soft_value_against_scipy_and_limits():
    rng = np.random.default_rng(71)
    Q = rng.standard_normal((6, 50)) * 3
    lp = np.log(rng.dirichlet(np.ones(50), size=6))
    for eta in [0.1, 1.0, 7.0]:
        V, pi, best = oracle.soft_value(Q, eta, lp)
        x = eta * Q + lp
        np.testing.assert_allclose(V, scipy.special.logsumexp(x, axis=1) / eta, rtol=1e-14, atol=1e-14)
        np.testing.assert_allclose(pi, scipy.special.softmax(x, axis=1), rtol=1e-12, atol=1e-15)
        assert np.array_equal(best, np.argmax(x, axis=1))
    # uniform prior: V = (1/eta) log mean exp(eta Q); constant Q gives V = Q exactly
    V, pi, _ = oracle.soft_value(np.full((1, 8), 2.5), 0.5)
    assert V[0] == 2.5 and np.all(pi == 0.125)
    # a single candidate: V = Q + log pi0 / eta
    V, _, _ = oracle.soft_value(np.array([[1.25]]), 2.0, np.array([[np.log(0.5)]]))
    assert V[0] == pytest.approx(1.25 + np.log(0.5) / 2.0, abs=1e-15)
    # eta -> infinity: the maximum; eta -> 0 under the uniform prior: the mean
    V, _, _ = oracle.soft_value(Q, 1e6)
    np.testing.assert_allclose(V, Q.max(axis=1), atol=1e-5)
    V, _, _ = oracle.soft_value(Q, 1e-7)
    np.testing.assert_allclose(V, Q.mean(axis=1), rtol=1e-5)
    # shift invariance and ties to the lowest index
    V2, _, _ = oracle.soft_value(Q + 10.0, 1.0, lp)
    V1, _, _ = oracle.soft_value(Q, 1.0, lp)
    np.testing.assert_allclose(V2, V1 + 10.0, rtol=1e-14)
    _, _, b = oracle.soft_value(np.array([[1.0, 3.0, 3.0, 2.0]]), 1.0)
    assert b[0] == 1


# ----------------------------------------------------------------------------- one-level closed-loop tree
def test_closed_loop_tree_special_cases():
    w = workloads.small(seed=81, N=24, K=6, H=4)
    m = w.model
    first = np.arange(5, dtype=np.int32)
    U = np.arange(5 * 3, dtype=np.uint32) * 2654435761
    cont = w.cands[:, :3]
    # gamma = 0: Psi = log pi0 / eta + R(b, a), R the horizon-1 plan value
    out = oracle.plan_closed_loop(m, w.states, first, 3, cont, 0.0, 2.0, 1.0, w.goal, 11, U)
    R1 = oracle.plan(m, w.states, first[:, None], 1.0, w.goal, seed=11)
    np.testing.assert_allclose(out["R"], R1, rtol=0, atol=0)
    np.testing.assert_allclose(out["psi"], -np.log(5) / 2.0 + R1, rtol=1e-15, atol=1e-15)
    x = 2.0 * out["psi"]
    assert out["V"] == pytest.approx(scipy.special.logsumexp(x) / 2.0, rel=1e-14)
    np.testing.assert_allclose(out["pi"], scipy.special.softmax(x), rtol=1e-12)
    assert out["best"] == int(np.argmax(out["psi"]))
    # gamma > 0: the backup adds gamma times the mean child value, each child
    # value being the soft value of the continuation returns from that child
    out2 = oracle.plan_closed_loop(m, w.states, first, 3, cont, 0.9, 2.0, 1.0, w.goal, 11, U)
    np.testing.assert_allclose(out2["psi"] - out["psi"], 0.9 * out2["V_child"].reshape(5, 3).mean(axis=1),
                               rtol=1e-12, atol=1e-12)
    child = out2["child"].reshape(15, 24, 4)
    for g in [0, 7, 14]:
        # every child is a resampled copy of its action's successors
        traj, _ = oracle.plan_steps(m, w.states, first[:, None], seed=11, want_obs=False)
        succ = traj[g // 3, :, 0]
        assert all(any(np.array_equal(r, s) for s in succ) for r in child[g])
    # eta -> infinity: V(b) tends to the best preference
    out3 = oracle.plan_closed_loop(m, w.states, first, 2, cont, 0.9, 1e6, 1.0, w.goal, 11, U[:10])
    assert out3["V"] == pytest.approx(out3["psi"].max(), abs=1e-4)


# ----------------------------------------------------------------------------- InfoNCE (Eq. 6)
def test_info_nce_scores_exact_two_by_two():
    # row 0: scores (0, log 3) -> softmax (1/4, 3/4), loss log 4 - 0
    # row 1: scores (0, 0)     -> softmax (1/2, 1/2), loss log 2 - 0
    L = np.array([[0.0, np.log(3.0)], [0.0, 0.0]])
    rl, G = oracle.info_nce_from_scores(L)
    np.testing.assert_allclose(rl, [2 * np.log(2.0), np.log(2.0)], rtol=1e-15)
    assert rl.mean() == pytest.approx(1.5 * np.log(2.0), rel=1e-15)
    np.testing.assert_allclose(G, [[-3 / 8, 3 / 8], [1 / 4, -1 / 4]], rtol=1e-15, atol=1e-16)
    # the diagonal entry is the row's own column: listing row 1 alone
    rl1, G1 = oracle.info_nce_from_scores(L[1:], rows=[1])
    np.testing.assert_allclose(rl1, rl[1:], rtol=0)
    np.testing.assert_allclose(G1, G[1:], rtol=0)


def test_info_nce_gradient_matches_finite_differences():
    rng = np.random.default_rng(3)
    B = 7
    L = rng.standard_normal((B, B)) * 2.0
    _, G = oracle.info_nce_from_scores(L)
    h = 1e-6
    for i, j in [(0, 0), (0, 5), (3, 3), (6, 1), (4, 2)]:
        Lp, Lm = L.copy(), L.copy()
        Lp[i, j] += h
        Lm[i, j] -= h
        fd = (oracle.info_nce_from_scores(Lp)[0].mean() - oracle.info_nce_from_scores(Lm)[0].mean()) / (2 * h)
        assert G[i, j] == pytest.approx(fd, abs=1e-9)
    np.testing.assert_allclose(G.sum(axis=1), 0.0, atol=1e-15)


def linear_score_model(rng, d_s, n_actions, d_a, d_o, width=16):
    """A likelihood network that computes the affine score u = v . x + c
    exactly: hidden unit 0 is relu(u), unit 1 is relu(-u), the second hidden
    layer copies them (they are non-negative) and the output is their
    difference."""
    aw = n_actions if n_actions > 0 else d_a
    d_in = d_s + aw + d_o
    v = rng.standard_normal(d_in).astype(np.float32)
    c = np.float32(0.375)
    W1 = np.zeros((width, d_in), np.float32)
    W1[0], W1[1] = v, -v
    b1 = np.zeros(width, np.float32)
    b1[0], b1[1] = c, -c
    W2 = np.eye(width, dtype=np.float32)
    W3 = np.zeros((1, width), np.float32)
    W3[0, 0], W3[0, 1] = 1.0, -1.0
    lik = [(W1, b1), (W2, np.zeros(width, np.float32)), (W3, np.zeros(1, np.float32))]
    trans = workloads.random_mlp(rng, [d_s + aw + 1, width, width, d_s])
    return Model(d_s=d_s, n_actions=n_actions, d_a=d_a, d_w=1, d_o=d_o, d_wz=1, trans=trans, lik=lik), v, c


@pytest.mark.parametrize("n_actions,d_a", [(5, 0), (0, 3)])
def test_info_nce_affine_score_closed_form(n_actions, d_a):
    # With l = v_s . s' + v_a . a + v_o . o + c the state-action part is
    # constant along a row, so row i's loss is log sum_j exp(v_o . o_j) - v_o . o_i
    # whatever the states and actions: only the observation varies along a row.
    rng = np.random.default_rng(17)
    d_s, d_o, B = 4, 3, 11
    m, v, c = linear_score_model(rng, d_s, n_actions, d_a, d_o)
    aw = m.action_width
    S = rng.standard_normal((B, d_s)).astype(np.float32)
    A = rng.integers(0, n_actions, B).astype(np.int32) if n_actions else rng.standard_normal((B, d_a)).astype(np.float32)
    O = rng.standard_normal((B, d_o)).astype(np.float32)
    out = oracle.info_nce(m, S, A, O)
    vo = O.astype(np.float64) @ v[d_s + aw:].astype(np.float64)
    lse = np.log(np.sum(np.exp(vo - vo.max()))) + vo.max()
    np.testing.assert_allclose(out["row_loss"], lse - vo, rtol=1e-12, atol=1e-12)
    assert out["loss"] == pytest.approx(np.mean(lse - vo), rel=1e-12)
    # the scores themselves: the row's state-action and the column's observation
    Aoh = np.eye(n_actions)[A] if n_actions else A.astype(np.float64)
    sa = S.astype(np.float64) @ v[:d_s].astype(np.float64) + Aoh @ v[d_s:d_s + aw].astype(np.float64)
    np.testing.assert_allclose(out["scores"], sa[:, None] + vo[None, :] + float(c), rtol=1e-12, atol=1e-12)
    # the derivative: softmax of the observation scores, minus the identity, over B
    p = np.exp(vo - vo.max())
    p /= p.sum()
    np.testing.assert_allclose(out["G"], (p[None, :] - np.eye(B)) / B, rtol=1e-12, atol=1e-14)


def test_info_nce_special_cases_and_invariances():
    w = workloads.small(seed=91, N=16)
    m = w.model
    rng = np.random.default_rng(5)
    B = 13
    S = w.states[:B]
    A = rng.integers(0, m.n_actions, B).astype(np.int32)
    O = rng.standard_normal((B, m.d_o)).astype(np.float32)
    out = oracle.info_nce(m, S, A, O)
    # B = 1: a single positive pair, zero loss and zero derivative
    one = oracle.info_nce(m, S[:1], A[:1], O[:1])
    assert one["loss"] == 0.0 and one["G"][0, 0] == 0.0
    # identical observations: every row's scores are equal, loss log B
    same = oracle.info_nce(m, S, A, np.repeat(O[:1], B, axis=0))
    np.testing.assert_allclose(same["row_loss"], np.log(B), rtol=1e-13)
    np.testing.assert_allclose(same["G"], (1.0 / B - np.eye(B)) / B, rtol=1e-12, atol=1e-15)
    # a constant added to every score (the output bias) changes nothing
    lik2 = [(W.copy(), b.copy()) for W, b in m.lik]
    lik2[-1] = (lik2[-1][0], lik2[-1][1] + np.float32(8.0))
    m2 = Model(**{**m.__dict__, "lik": lik2})
    out2 = oracle.info_nce(m2, S, A, O)
    shift = float(lik2[-1][1][0]) - float(m.lik[-1][1][0])
    np.testing.assert_allclose(out2["scores"], out["scores"] + shift, rtol=1e-12)
    np.testing.assert_allclose(out2["row_loss"], out["row_loss"], rtol=1e-10, atol=1e-12)
    # permuting the batch permutes rows and columns
    perm = rng.permutation(B)
    outp = oracle.info_nce(m, S[perm], A[perm], O[perm])
    np.testing.assert_allclose(outp["scores"], out["scores"][perm][:, perm], rtol=0)
    np.testing.assert_allclose(outp["row_loss"], out["row_loss"][perm], rtol=1e-14)
    assert outp["loss"] == pytest.approx(out["loss"], rel=1e-14)
    # a subset of rows is the same rows of the full evaluation
    sub = oracle.info_nce(m, S, A, O, rows=[12, 0, 5])
    np.testing.assert_allclose(sub["scores"], out["scores"][[12, 0, 5]], rtol=0)
    np.testing.assert_allclose(sub["row_loss"], out["row_loss"][[12, 0, 5]], rtol=0)
    np.testing.assert_allclose(sub["G"], out["G"][[12, 0, 5]], rtol=0)
    # scores are the likelihood network on [s'_i, a_i, o_j]
    X = np.concatenate([S[3], np.eye(m.n_actions)[A[3]], O[8]]).astype(np.float64)
    assert out["scores"][3, 8] == pytest.approx(_numpy_mlp(m.lik, X[None, :])[0, 0], rel=1e-12)


# ----------------------------------------------------------------------------- DDIM teacher sampler
def test_cosine_schedule_end_points_and_monotone():
    assert oracle.cosine_abar(0.0) == 1.0
    assert 0.0 <= oracle.cosine_abar(1.0) < 1e-30
    a = [oracle.cosine_abar(t) for t in np.linspace(0.0, 1.0, 201)]
    assert all(x > y for x, y in zip(a[:-1], a[1:]))


@pytest.mark.parametrize("n_steps", [1, 2, 7, 50])
def test_ddim_recovers_a_point_mass_exactly(n_steps):
    # with the exact v of a point-mass data distribution the clean-sample
    # estimate is the point itself at every step, so the deterministic
    # sampler lands on it from any noise and with any number of steps
    rng = np.random.default_rng(n_steps)
    x0, x1 = rng.standard_normal(6), rng.standard_normal(6) * 3.0
    np.testing.assert_allclose(oracle.ddim_point_mass(x0, x1, n_steps), x0, rtol=0, atol=1e-12)


@pytest.mark.parametrize("sigma", [0.5, 2.0])
@pytest.mark.parametrize("n_steps", [1, 3, 10, 50])
def test_ddim_gaussian_data_closed_form(sigma, n_steps):
    # Data N(mu, sigma^2) with its exact denoiser.  In the standardised
    # coordinate z = (x - sqrt(a) mu) / sqrt(a sigma^2 + 1 - a) a deterministic
    # step multiplies z by cos(phi - phi'), phi = atan2(sqrt(1 - a), sqrt(a) sigma)
    # (the estimates' directions at the two times), so from z = x1 at tau = 1
    # the sample is mu + sigma x1 prod_k cos(phi_k - phi_{k+1}); every step's
    # clean and noise estimates enter the product.
    rng = np.random.default_rng(n_steps)
    mu, x1 = rng.standard_normal(5), rng.standard_normal(5)
    a = np.array([oracle.cosine_abar(1.0 - k / n_steps) for k in range(n_steps + 1)])
    phi = np.arctan2(np.sqrt(1.0 - a), np.sqrt(a) * sigma)
    shrink = np.prod(np.cos(phi[:-1] - phi[1:]))
    np.testing.assert_allclose(oracle.ddim_gaussian(mu, sigma, x1, n_steps), mu + sigma * x1 * shrink,
                               rtol=1e-12, atol=1e-12)
    if n_steps == 50:
        assert 0.96 < shrink < 1.0  # the discretisation shrinks less with more steps (0.57 at 3, 0.97 at 50)


@pytest.mark.parametrize("n_actions,d_a", [(5, 0), (0, 3)])
def test_ddim_one_step_is_minus_v_at_tau_one(n_actions, d_a):
    # one step from tau = 1 (abar = 0) to tau = 0 (abar = 1): the sample is the
    # clean estimate sqrt(abar) x - sqrt(1 - abar) v = -v([s, a, x1, 1])
    layers = workloads.denoiser(seed=5, d_c=5, d_x=3, n_actions=n_actions, d_a=d_a, width=16, n_hidden=3)
    S, X1 = workloads.ddim_batch(9, d_c=5, d_x=3, seed=6)
    a = 2 if n_actions else np.array([0.5, -0.25, 1.0], np.float32)
    out = oracle.ddim_sample(layers, 5, 3, n_actions, d_a, S, a, X1, 1)
    A = np.tile(np.eye(n_actions)[a] if n_actions else a, (9, 1))
    X = np.concatenate([S, A, X1, np.ones((9, 1))], axis=1).astype(np.float64)
    np.testing.assert_allclose(out, -_numpy_mlp(layers, X), rtol=1e-12, atol=1e-12)


def test_ddim_zero_denoiser_single_step_and_rows_independent():
    layers = workloads.denoiser(seed=7, width=8, n_hidden=2)
    zero = [(np.zeros_like(W), np.zeros_like(b)) for W, b in layers]
    S, X1 = workloads.ddim_batch(5, seed=8)
    # v = 0 and abar(1) = 0: one step erases the noise
    np.testing.assert_allclose(oracle.ddim_sample(zero, 4, 4, 5, 0, S, 1, X1, 1), 0.0, atol=1e-15)
    # rows are independent samples
    full = oracle.ddim_sample(layers, 4, 4, 5, 0, S, 1, X1, 12)
    part = oracle.ddim_sample(layers, 4, 4, 5, 0, S[2:4], 1, X1[2:4], 12)
    np.testing.assert_array_equal(full[2:4], part)


def _flat_lik(m):
    return np.concatenate([np.concatenate([W.ravel(), b.ravel()]) for W, b in m.lik]).astype(np.float64)


def _with_flat_lik(m, theta):
    layers, off = [], 0
    for W, b in m.lik:
        nW, nb = W.size, b.size
        layers.append((theta[off:off + nW].reshape(W.shape), theta[off + nW:off + nW + nb]))
        off += nW + nb
    return Model(**{**m.__dict__, "lik": layers})


@pytest.mark.parametrize("which", ["small", "continuous"])
def test_info_nce_param_grad_matches_finite_differences(which):
    w = workloads.small(seed=93, N=16) if which == "small" else workloads.continuous(seed=94, N=16)
    m = w.model
    S, A, O = workloads.nce_batch(w, 9, seed=3)
    loss, g = oracle.info_nce_param_grad(m, S, A, O)
    assert loss == pytest.approx(oracle.info_nce(m, S, A, O)["loss"], rel=1e-14)
    theta = _flat_lik(m)
    # the output bias shifts every score equally: its derivative is zero
    assert abs(g[-1]) < 1e-14
    rng = np.random.default_rng(4)
    h = 1e-6
    checked = 0
    # random coordinates plus the first weights and biases of every layer
    fixed, off = [], 0
    for W, b in m.lik:
        fixed += [off, off + 1, off + W.size, off + W.size + 1]
        off += W.size + b.size
    coords = sorted(set(int(q) for q in rng.choice(theta.size - 1, 40, replace=False)) |
                    set(q for q in fixed if q < theta.size - 1))
    for q in coords:
        tp, tm = theta.copy(), theta.copy()
        tp[q] += h
        tm[q] -= h
        fp = oracle.info_nce(_with_flat_lik(m, tp), S, A, O)["loss"]
        fm = oracle.info_nce(_with_flat_lik(m, tm), S, A, O)["loss"]
        f2 = oracle.info_nce(_with_flat_lik(m, theta), S, A, O)["loss"]
        # skip coordinates whose step crosses a ReLU kink (one-sided slopes differ)
        if abs((fp - f2) / h - (f2 - fm) / h) > 1e-4 * max(1.0, abs(g[q])):
            continue
        assert g[q] == pytest.approx((fp - fm) / (2 * h), abs=1e-7, rel=1e-5), q
        checked += 1
    assert checked >= 30


def _deep_lik_model(seed, width=10, n_hidden=3):
    """The small workload's model with a likelihood network of n_hidden ReLU
    layers (the depth of the realistic likelihood network, narrower)."""
    w = workloads.small(seed=seed, N=16)
    rng = np.random.default_rng(seed)
    m = w.model
    lik = workloads.random_mlp(rng, [m.d_s + m.n_actions + m.d_o] + [width] * n_hidden + [1])
    return w, Model(**{**m.__dict__, "lik": lik})


def test_info_nce_param_grad_three_hidden_layers_matches_finite_differences():
    # the reverse sweep through every hidden->hidden layer, as in the
    # realistic (three hidden layer) likelihood network
    w, m = _deep_lik_model(95)
    S, A, O = workloads.nce_batch(w, 7, seed=5)
    _, g = oracle.info_nce_param_grad(m, S, A, O)
    theta = _flat_lik(m)
    h, checked = 1e-6, 0
    for q in range(theta.size - 1):
        tp, tm = theta.copy(), theta.copy()
        tp[q] += h
        tm[q] -= h
        fp = oracle.info_nce(_with_flat_lik(m, tp), S, A, O)["loss"]
        fm = oracle.info_nce(_with_flat_lik(m, tm), S, A, O)["loss"]
        f2 = oracle.info_nce(_with_flat_lik(m, theta), S, A, O)["loss"]
        if abs((fp - f2) / h - (f2 - fm) / h) > 1e-4 * max(1.0, abs(g[q])):
            continue
        assert g[q] == pytest.approx((fp - fm) / (2 * h), abs=1e-7, rel=1e-5), q
        checked += 1
    assert checked >= 0.9 * (theta.size - 1)


def _bf16_values(x):
    """x rounded to bfloat16 (nearest, ties to even) by bit manipulation of its
    binary32 value, returned as float32."""
    u = np.asarray(x, np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32)


def test_info_nce_param_grad_bf16_emulation_within_rounding_of_exact():
    # the emulation rounds weights, layer inputs and hidden adjoints to
    # bfloat16 (8 significant bits).  Against the exact gradient of the
    # network whose weights are already bfloat16 values (so only the rounding
    # of activations and adjoints differs) it stays within a few units of
    # 2^-8 of the gradient's scale, and differs from it (the rounding takes
    # effect); the rounded weights alone change the function, so that is the
    # reference
    w, m = _deep_lik_model(96, width=24)
    m_r = Model(**{**m.__dict__, "lik": [(_bf16_values(W), b) for W, b in m.lik]})
    S, A, O = workloads.nce_batch(w, 12, seed=6)
    _, g = oracle.info_nce_param_grad(m_r, S, A, O)
    loss_b, gb = oracle.info_nce_param_grad(m, S, A, O, bf16=True)
    assert loss_b == pytest.approx(oracle.info_nce(m, S, A, O, bf16=True)["loss"], rel=1e-14)
    scale = np.max(np.abs(g))
    err = np.max(np.abs(gb - g)) / scale
    assert 1e-5 < err < 16 * 2.0 ** -8
    # per layer, the emulated gradient points the same way as the exact one
    off = 0
    for W, b in m.lik:
        n = W.size + b.size
        a, e = gb[off:off + n], g[off:off + n]
        assert np.dot(a, e) / (np.linalg.norm(a) * np.linalg.norm(e)) > 0.99
        off += n
    # with weights and inputs already bfloat16 values, rounding the inputs
    # changes nothing: only activations and adjoints are rounded
    S_r, O_r = _bf16_values(S), _bf16_values(O)
    _, g1 = oracle.info_nce_param_grad(m_r, S_r, A, O_r, bf16=True)
    _, g2 = oracle.info_nce_param_grad(m, S_r, A, O_r, bf16=True)
    assert np.array_equal(g1, g2)
