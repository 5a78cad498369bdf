"""Contrastive objective of the likelihood network (voila_info_nce, through
the C ABI) against the oracle (Eq. 6).

* scores l_ij: binary32 within 1e-5 of the matrix's scale, bfloat16 against
  the oracle's emulation within 2^-6 of the scale (the likelihood bounds of
  the other parity tests);
* row losses, the mean loss and the derivative from the device's own scores:
  the oracle's row reduction on those scores within 1e-12 (binary64 on both
  sides, different summation order), the derivative within binary32 rounding;
* end to end against the oracle's scores: each row loss moves by at most
  twice the largest score error of its row (log-sum-exp and the diagonal
  term are each 1-Lipschitz in the max norm), each derivative entry by at
  most p_ij (e^{2 delta} - 1) / B;
* ragged batches (B not a multiple of the 32-column tile), B = 1 and B = 32,
  continuous actions, the realistic and width-1024 networks, sampled rows at
  B = 4,096, bit-identical repeated runs, and the status word for a bad
  action or a non-finite score.
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


def run_dev(V, m, S, A, O, status=None):
    res = V.info_nce(m, dev(S), dev(A, torch.int32 if A.dtype == np.int32 else torch.float32), dev(O),
                     status=status)
    torch.cuda.synchronize()
    return {k: (host(v) if v is not None else None) for k, v in res.items()}


def check_against_own_scores(d, rows=None):
    sc = d["scores"].astype(np.float64)
    B = sc.shape[1]
    sel = np.arange(B) if rows is None else np.asarray(rows)
    rl, G = oracle.info_nce_from_scores(sc[sel], rows=sel)
    np.testing.assert_allclose(d["row_loss"][sel], rl, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(d["grad"][sel], G, rtol=2.0 ** -23, atol=1e-15)
    if rows is None:
        assert d["loss"][0] == pytest.approx(d["row_loss"].mean(), rel=1e-13, abs=1e-13)


def check_against_oracle(d, r, bound, rows=None):
    B = d["scores"].shape[1]
    sel = np.arange(B) if rows is None else np.asarray(rows)
    ref = r["scores"]
    got = d["scores"][sel].astype(np.float64)
    scale = max(float(np.max(np.abs(ref))), 1e-30)
    err = np.abs(got - ref)
    e = float(err.max()) / scale
    delta = err.max(axis=1)
    dl = np.abs(d["row_loss"][sel] - r["row_loss"])
    dg = np.abs(d["grad"][sel].astype(np.float64) - r["G"])
    p = r["G"] * B + (sel[:, None] == np.arange(B)[None, :])
    gb = p * np.expm1(2.0 * delta)[:, None] / B * 1.01 + 2.0 ** -23 * np.abs(r["G"]) + 1e-15
    print(f"  scores err {e:.2e} of scale; row-loss err {dl.max():.2e}; grad err {dg.max():.2e}", flush=True)
    assert e <= bound
    assert np.all(dl <= 2.0 * delta * 1.01 + 1e-12)
    assert np.all(dg <= gb)
    if rows is None:
        assert abs(d["loss"][0] - r["loss"]) <= 2.0 * delta.max() * 1.01 + 1e-12


def compare(V, w, B, compute, seed=14):
    model = w.model
    S, A, O = workloads.nce_batch(w, B, seed=seed)
    m = V.Model(model, compute=compute)
    print(f"info_nce {w.name} {compute} B={B}", flush=True)
    d = run_dev(V, m, S, A, O)
    check_against_own_scores(d)
    r = oracle.info_nce(model, S, A, O, bf16=(compute == "bf16"))
    check_against_oracle(d, r, TOL if compute == "f32" else BOUND_EMUL)
    return d


@pytest.mark.parametrize("compute,B", [("f32", 100), ("bf16", 77), ("f32", 32), ("f32", 33)])
def test_small(V, compute, B):
    compare(V, workloads.small(seed=71), B, compute)


def test_single_pair_is_zero(V):
    w = workloads.small(seed=72)
    S, A, O = workloads.nce_batch(w, 1)
    d = run_dev(V, V.Model(w.model), S, A, O)
    assert d["row_loss"][0] == 0.0 and d["loss"][0] == 0.0 and d["grad"][0, 0] == 0.0


def test_continuous_actions(V):
    compare(V, workloads.continuous(seed=73), 65, "f32")


@pytest.mark.parametrize("compute,B", [("f32", 96), ("bf16", 130)])
def test_realistic(V, compute, B):
    compare(V, workloads.realistic(seed=74, N=256, K=1, H=1), B, compute)


def test_wide(V):
    compare(V, workloads.wide(seed=75, N=64, K=1, H=1), 40, "bf16")


@pytest.mark.parametrize("compute", ["f32", "bf16"])
def test_realistic_full_batch_sampled_rows(V, compute):
    # B = 4,096 (16.8 M pairs) with the realistic networks; sampled rows
    # against the oracle, every row against the device's own scores
    w = workloads.realistic(seed=76, N=4096, K=1, H=1)
    B = 4096
    S, A, O = workloads.nce_batch(w, B, seed=15)
    m = V.Model(w.model, compute=compute)
    print(f"info_nce realistic {compute} B={B}", flush=True)
    d = run_dev(V, m, S, A, O)
    check_against_own_scores(d)
    rows = [0, 1, 31, 32, 2047, 4095]
    r = oracle.info_nce(w.model, S, A, O, rows=rows, bf16=(compute == "bf16"))
    check_against_oracle(d, r, TOL if compute == "f32" else BOUND_EMUL, rows=rows)
    np.testing.assert_allclose(d["grad"].astype(np.float64).sum(axis=1), 0.0, atol=1e-6)


def test_repeatable(V):
    w = workloads.realistic(seed=77, N=256, K=1, H=1)
    S, A, O = workloads.nce_batch(w, 300)
    m = V.Model(w.model, compute="bf16")
    a = run_dev(V, m, S, A, O)
    b = run_dev(V, m, S, A, O)
    for k in a:
        assert np.array_equal(a[k], b[k]), k


def test_status_word(V):
    w = workloads.small(seed=78)
    S, A, O = workloads.nce_batch(w, 40)
    m = V.Model(w.model)
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    A_bad = A.copy()
    A_bad[7] = w.model.n_actions
    run_dev(V, m, S, A_bad, O, status=st)
    assert int(st.item()) == V.VOILA_ERR_INVALID_ARG
    W, b = w.model.lik[-1]
    bad = workloads.Model(**{**w.model.__dict__, "lik": w.model.lik[:-1] + [(W, np.full_like(b, np.inf))]})
    st.zero_()
    run_dev(V, V.Model(bad), S, A, O, status=st)
    assert int(st.item()) == V.VOILA_ERR_NUMERIC


def test_rejects_bad_sizes(V):
    w = workloads.small(seed=79)
    m = V.Model(w.model)
    S, A, O = workloads.nce_batch(w, 4)
    with pytest.raises(V.VoilaError):
        V.info_nce(m, dev(S[:0]), dev(A[:0], torch.int32), dev(O[:0]))


# ----------------------------------------------------------------------------- parameter derivative
def run_grad(V, m, S, A, O):
    res = V.info_nce_grad(m, dev(S), dev(A, torch.int32 if A.dtype == np.int32 else torch.float32), dev(O))
    torch.cuda.synchronize()
    return float(res["loss"].item()), host(res["grad"]).astype(np.float64)


@pytest.mark.parametrize("which,B", [("small", 100), ("small", 256), ("continuous", 65), ("small", 32),
                                     ("small", 1024)])
def test_param_grad_against_oracle(V, which, B):
    # max |g_dev - g_ref| <= 1e-5 max |g_ref|: the binary32 tolerance relative
    # to the gradient's scale (binary32 forward and reverse passes over B^2
    # pairs against binary64)
    w = workloads.small(seed=81) if which == "small" else workloads.continuous(seed=82)
    S, A, O = workloads.nce_batch(w, B, seed=17)
    m = V.Model(w.model)
    print(f"info_nce grad {which} B={B}", flush=True)
    loss, g = run_grad(V, m, S, A, O)
    loss_ref, g_ref = oracle.info_nce_param_grad(w.model, S, A, O)
    err = float(np.max(np.abs(g - g_ref))) / float(np.max(np.abs(g_ref)))
    print(f"  grad err {err:.2e} of scale {np.max(np.abs(g_ref)):.3e}; loss {loss:.6f} vs {loss_ref:.6f}", flush=True)
    assert g.shape == g_ref.shape
    assert err <= TOL
    assert abs(loss - loss_ref) <= 1e-5 * max(1.0, abs(loss_ref))
    assert abs(g[-1]) <= 1e-5 * float(np.max(np.abs(g_ref)))  # output bias: the scores' derivatives sum to zero


def test_param_grad_single_pair_repeatable_and_unsupported(V):
    w = workloads.small(seed=83)
    m = V.Model(w.model)
    S, A, O = workloads.nce_batch(w, 1)
    loss, g = run_grad(V, m, S, A, O)
    assert loss == 0.0 and np.all(g == 0.0)
    S, A, O = workloads.nce_batch(w, 300)
    assert np.array_equal(run_grad(V, m, S, A, O)[1], run_grad(V, m, S, A, O)[1])
    r = workloads.realistic(seed=84, N=64, K=1, H=1)
    S, A, O = workloads.nce_batch(r, 8)
    with pytest.raises(V.VoilaError):
        V.info_nce_grad(V.Model(r.model), dev(S), dev(A), dev(O))


def test_param_grad_bench_size_properties(V):
    # B = 4,096 (16.8 M pairs, the measured size): the output-bias derivative
    # vanishes, the result is finite and repeatable, and the loss equals the
    # forward call's
    w = workloads.small(seed=9)
    S, A, O = workloads.nce_batch(w, 4096, seed=18)
    m = V.Model(w.model)
    print("info_nce grad small B=4096", flush=True)
    loss, g = run_grad(V, m, S, A, O)
    assert np.all(np.isfinite(g))
    assert abs(g[-1]) <= 1e-5 * float(np.max(np.abs(g)))
    d = run_dev(V, m, S, A, O)
    assert loss == pytest.approx(float(d["loss"][0]), rel=1e-12)
    assert np.array_equal(run_grad(V, m, S, A, O)[1], g)


def test_maximum_batch(V):
    # B = 32,768 (the largest accepted; 1.07e9 pairs) with the small networks:
    # sampled rows against the oracle; one more tuple is refused
    w = workloads.small(seed=85, N=4096)
    B = 32768
    S, A, O = workloads.nce_batch(w, B, seed=19)
    m = V.Model(w.model)
    print(f"info_nce small f32 B={B}", flush=True)
    d = run_dev(V, m, S, A, O)
    rows = [0, 12345, B - 1]
    check_against_own_scores(d, rows=rows)
    r = oracle.info_nce(w.model, S, A, O, rows=rows)
    check_against_oracle(d, r, TOL, rows=rows)
    assert np.isfinite(d["loss"][0])
    S1, A1, O1 = workloads.nce_batch(w, B + 1, seed=20)
    with pytest.raises(V.VoilaError):
        V.info_nce(m, dev(S1), dev(A1, torch.int32), dev(O1), want_scores=False, want_grad=False)
