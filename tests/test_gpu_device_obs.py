"""The belief update reads the executed action and the received observation
from device memory (the update of Sec. 3 takes (b, a, o); an observation drawn
by the observation sampler of Eq. 5 on the GPU never visits the host).

* observe -> update chained on one stream with no host copy: results equal,
  bit for bit, the update given the same observation copied from the host.
* the chain captured in a hipGraph (torch.cuda.CUDAGraph over the C ABI) and
  replayed after the state the observation is drawn from and the observation
  noise were changed in device memory: every replay equals, bit for bit, the
  eager chain on the same inputs, with eager work and synchronisations between
  replays; a captured update alone follows an observation overwritten in place.
* a bad action or observation in device memory sets the status word.
"""
import numpy as np
import pytest
import torch

import oracle
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


def say(msg):
    print(msg, flush=True)


def _action(w):
    if w.model.n_actions > 0:
        return dev([w.update_action], torch.int32)
    return dev(np.asarray(w.update_action, np.float32))


def _buffers(w, N):
    d = torch.device("cuda")
    return {"states": torch.empty((N, w.model.d_s), dtype=torch.float32, device=d),
            "idx": torch.empty(N, dtype=torch.int32, device=d),
            "w": torch.empty(N, dtype=torch.float64, device=d),
            "loglik": torch.empty(N, dtype=torch.float32, device=d),
            "prop": torch.empty((N, w.model.d_s), dtype=torch.float32, device=d),
            "stats": torch.empty(2, dtype=torch.float64, device=d)}


@pytest.mark.parametrize("name", ["small", "realistic", "small_continuous"])
def test_observe_then_update_device_chain(name):
    w = {"small": lambda: workloads.small(N=300),
         "realistic": lambda: workloads.realistic(N=1000, K=1, H=1),
         "small_continuous": lambda: workloads.continuous(N=300)}[name]()
    m = V.Model(w.model)
    S = dev(w.states)
    act = _action(w)
    s_true = dev(w.states[5:6])
    nz = dev(np.random.default_rng(11).standard_normal((1, w.model.d_wz)))
    obs = V.observe(m, s_true, act, noise=nz)
    got = V.update(m, S, act, obs[0], lam=w.lam, seed=w.update_seed, U=w.resample_u)
    torch.cuda.synchronize()
    o_host = obs[0].cpu().numpy()
    via_host = V.update(m, S, w.update_action, o_host, lam=w.lam, seed=w.update_seed, U=w.resample_u)
    torch.cuda.synchronize()
    for k in KEYS:
        assert torch.equal(got[k], via_host[k]), k
    # the chain against the oracle: the observation, then the update given it
    acts = [int(w.update_action)] if w.model.n_actions > 0 else np.asarray(w.update_action)[None]
    o_ref = oracle.observe(w.model, w.states[5:6], acts, noise=nz.cpu().numpy())[0]
    e_o = float(np.max(np.abs(o_host - o_ref)) / np.max(np.abs(o_ref)))
    ref = oracle.update(w.model, w.states, w.update_action, o_host, lam=w.lam, seed=w.update_seed, U=w.resample_u)
    e_l = float(np.max(np.abs(got["loglik"].cpu().numpy() - ref["loglik"])) / np.max(np.abs(ref["loglik"])))
    say(f"  {name}: observation err {e_o:.2e}, loglik err {e_l:.2e}")
    assert e_o <= 1e-5 and e_l <= 1e-5
    assert np.array_equal(got["idx"].cpu().numpy(), oracle.resample(got["w"].cpu().numpy().astype(np.float64),
                                                                      w.resample_u))


@pytest.mark.parametrize("N", [1000, 20000])
def test_captured_chain_follows_device_inputs(N):
    """N = 20,000 takes the multi-workgroup resampling path."""
    w = workloads.realistic(N=N, K=1, H=1)
    m = V.Model(w.model)
    S = dev(w.states)
    act = _action(w)
    rng = np.random.default_rng(N)
    s_true = dev(w.states[:1])
    nz = dev(rng.standard_normal((1, w.model.d_wz)))
    obs_buf = torch.empty((1, w.model.d_o), dtype=torch.float32, device="cuda")
    ws_o = m.observe_workspace()
    ws_u = m.update_workspace(N)
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    out_g = _buffers(w, N)

    def chain(out):
        V.observe(m, s_true, act, noise=nz, out=obs_buf, workspace=ws_o, status=status)
        V.update(m, S, act, obs_buf[0], lam=w.lam, seed=w.update_seed, U=w.resample_u, out=out, workspace=ws_u,
                 status=status)

    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        chain(out_g)  # warm-up outside the capture
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        chain(out_g)
    torch.cuda.synchronize()
    seen = set()
    for rep in range(4):
        # new inputs in device memory: the state the observation is drawn from
        # and its noise; eager work on the stream between replays
        s_true.copy_(dev(w.states[rep * 7 + 3:rep * 7 + 4]))
        nz.copy_(dev(rng.standard_normal((1, w.model.d_wz))))
        g.replay()
        torch.cuda.synchronize()
        got = {k: v.clone() for k, v in out_g.items()}
        o_graph = obs_buf.clone()
        out_e = _buffers(w, N)
        chain(out_e)
        torch.cuda.synchronize()
        assert torch.equal(o_graph, obs_buf)
        for k in KEYS:
            assert torch.equal(got[k], out_e[k]), (rep, k)
        seen.add(tuple(got["idx"][:64].cpu().tolist()))
        _ = torch.randn(1000, device="cuda").sum()  # unrelated eager work between replays
    assert int(status.item()) == 0
    assert len(seen) > 1  # the replays followed the new observations
    say(f"  captured observe->update N={N}: 4 replays bit-identical to eager, {len(seen)} distinct resamplings")

    # a captured update on its own follows an observation overwritten in place
    o2 = torch.zeros(w.model.d_o, dtype=torch.float32, device="cuda")
    out_u = _buffers(w, N)
    with torch.cuda.stream(side):
        V.update(m, S, act, o2, lam=w.lam, seed=w.update_seed, U=w.resample_u, out=out_u, workspace=ws_u)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g2 = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g2):
        V.update(m, S, act, o2, lam=w.lam, seed=w.update_seed, U=w.resample_u, out=out_u, workspace=ws_u)
    for rep in range(3):
        o_new = rng.standard_normal(w.model.d_o).astype(np.float32)
        o2.copy_(dev(o_new))
        g2.replay()
        torch.cuda.synchronize()
        ref = V.update(m, S, w.update_action, o_new, lam=w.lam, seed=w.update_seed, U=w.resample_u)
        torch.cuda.synchronize()
        for k in KEYS:
            assert torch.equal(out_u[k], ref[k]), (rep, k)


def test_bad_device_action_or_observation_sets_status():
    w = workloads.small(N=64)
    m = V.Model(w.model)
    S = dev(w.states)
    o = torch.zeros(w.model.d_o, dtype=torch.float32, device="cuda")
    for bad_a in [5, -1]:
        st = torch.zeros(1, dtype=torch.int32, device="cuda")
        V.update(m, S, dev([bad_a], torch.int32), o, seed=1, U=1, status=st)
        torch.cuda.synchronize()
        assert int(st.item()) == V.VOILA_ERR_INVALID_ARG
        st.zero_()
        V.observe(m, S, dev([bad_a], torch.int32), status=st)
        torch.cuda.synchronize()
        assert int(st.item()) == V.VOILA_ERR_INVALID_ARG
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    V.update(m, S, dev([2], torch.int32), dev([0.0, float("nan")]), seed=1, U=1, status=st)
    torch.cuda.synchronize()
    assert int(st.item()) != 0
    # a valid call leaves the status word alone
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    V.update(m, S, dev([2], torch.int32), o, seed=1, U=1, status=st)
    V.observe(m, S, dev([4], torch.int32), status=st)
    torch.cuda.synchronize()
    assert int(st.item()) == 0
    # host values are still checked before anything is enqueued
    with pytest.raises(V.VoilaError):
        V.update(m, S, 7, o, seed=1, U=1)
    with pytest.raises(V.VoilaError):
        V.update(m, S, 2, [0.0, float("inf")], seed=1, U=1)
