"""voila_update_noalloc (the belief update with its workspace in the
library's fixed device scratch) against voila_update with a caller workspace:
identical results, bit for bit, on consecutive calls that reuse the scratch
with different sizes (the second call smaller), across the single-workgroup
and the multi-workgroup resampling paths; sizes beyond the scratch are
refused before anything is enqueued; given its output buffers and device
inputs, the call allocates nothing."""
import numpy as np
import pytest
import torch

import workloads

pytestmark = pytest.mark.gpu

V = None
KEYS = ["states", "idx", "w", "loglik", "prop", "stats"]


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


def buffers(N, d_s):
    d = torch.device("cuda")
    return {"states": torch.empty((N, d_s), dtype=torch.float32, device=d),
            "idx": torch.empty(N, dtype=torch.int32, device=d),
            "w": torch.empty(N, dtype=torch.float64, device=d),
            "loglik": torch.empty(N, dtype=torch.float32, device=d),
            "prop": torch.empty((N, d_s), dtype=torch.float32, device=d),
            "stats": torch.empty(2, dtype=torch.float64, device=d)}


def run_pair(w, N, seed, prior=False):
    m = V.Model(w.model)
    S = dev(w.states[:N])
    act = dev([w.update_action], torch.int32) if w.model.n_actions > 0 else dev(np.asarray(w.update_action))
    obs = dev(np.random.default_rng(seed).standard_normal(w.model.d_o))
    pw = None
    if prior:
        pw = dev(np.random.default_rng(seed + 1).dirichlet(np.ones(N)), torch.float64)
    ref = V.update(m, S, act, obs, lam=w.lam, prior_w=pw, seed=seed, U=w.resample_u + seed)
    out = buffers(N, w.model.d_s)
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    torch.cuda.synchronize()
    before = torch.cuda.memory_allocated()
    got = V.update_noalloc(m, S, act, obs, lam=w.lam, prior_w=pw, seed=seed, U=w.resample_u + seed, out=out,
                           status=st)
    assert torch.cuda.memory_allocated() == before  # nothing allocated for the call
    torch.cuda.synchronize()
    assert int(st.item()) == 0
    for k in KEYS:
        assert torch.equal(got[k], ref[k]), (N, k)
    print(f"  no-alloc update {w.name} N={N}: identical to voila_update", flush=True)


def test_noalloc_matches_update_on_consecutive_calls():
    # 20,000 particles take the multi-workgroup resampling path, 3,000 and 1
    # the single-workgroup one; each call reuses what the previous left
    w = workloads.realistic(N=20000, K=1, H=1)
    run_pair(w, 20000, seed=5)
    run_pair(w, 3000, seed=6)
    run_pair(w, 1, seed=7)
    run_pair(w, 9000, seed=8, prior=True)
    ws = workloads.small(N=4096)
    run_pair(ws, 4096, seed=9)
    run_pair(ws, 100, seed=10, prior=True)


def test_noalloc_refuses_sizes_beyond_the_scratch():
    w = workloads.realistic(N=200000, K=1, H=1)
    m = V.Model(w.model)
    N = 200000
    assert V.lib.voila_update_workspace_size(m.handle, N) > 8 << 20
    S = dev(w.states)
    out = buffers(N, w.model.d_s)
    with pytest.raises(V.VoilaError) as e:
        V.update_noalloc(m, S, np.asarray(w.update_action, np.float32), np.zeros(w.model.d_o, np.float32), out=out)
    assert e.value.status == V.VOILA_ERR_UNSUPPORTED
    # the largest size the documentation promises still runs
    n_max = 65536
    assert V.lib.voila_update_workspace_size(m.handle, n_max) <= 8 << 20
    run_pair(w, n_max, seed=11)
