"""Python face of the FP64 oracle (test infrastructure only).

The oracle is a plain binary64 CPU implementation of the VOiLA planning hot
path (``voila_oracle.c``).  Only the tests, the smoke check and the
benchmark's CPU-baseline leg may import this package; the product library
never does.  Inputs are converted to binary64 here (binary32 inputs convert
exactly), the C code does all of the arithmetic.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_double, c_int, c_int32, c_uint32, c_uint64, c_size_t

import numpy as np

from . import build as _build

_LIB = None

OR_OK, OR_ERR_ARG, OR_ERR_NUMERIC = 0, 1, 2


class OracleError(RuntimeError):
    pass


class _CModel(ctypes.Structure):
    _fields_ = [
        ("d_s", c_int), ("n_actions", c_int), ("d_a", c_int), ("d_w", c_int),
        ("d_o", c_int), ("d_wz", c_int), ("residual", c_int),
        ("t_layers", c_int), ("t_dims", POINTER(c_int)), ("t_params", POINTER(c_double)),
        ("z_layers", c_int), ("z_dims", POINTER(c_int)), ("z_params", POINTER(c_double)),
        ("l_layers", c_int), ("l_dims", POINTER(c_int)), ("l_params", POINTER(c_double)),
    ]


def lib():
    global _LIB
    if _LIB is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        L = ctypes.CDLL(_build.LIB)
        dp, ip, i32p, u32p = POINTER(c_double), POINTER(c_int), POINTER(c_int32), POINTER(c_uint32)
        mp = POINTER(_CModel)
        L.or_philox4x32_10.argtypes = [u32p, u32p, u32p]
        L.or_uniform.argtypes = [c_uint32]
        L.or_uniform.restype = c_double
        L.or_normals.argtypes = [c_uint64, c_uint32, c_uint32, c_uint32, c_uint32, c_int, dp]
        L.or_round_bf16.argtypes = [c_double]
        L.or_round_bf16.restype = c_double
        L.or_mlp.argtypes = [c_int, ip, dp, c_int, dp, dp, c_int]
        L.or_plan.argtypes = [mp, c_int, dp, dp, c_int, c_int, i32p, dp, c_double, dp, c_int,
                              dp, c_uint64, c_int, c_int, dp, dp]
        L.or_rollouts.argtypes = [mp, c_int, dp, c_int, c_int, i32p, dp, c_double, dp, c_int,
                                  c_uint64, c_int, c_int, c_int, i32p, i32p, dp]
        L.or_weighted_mean.argtypes = [c_int, dp, dp]
        L.or_weighted_mean.restype = c_double
        L.or_normalize.argtypes = [c_int, dp, dp, c_double, dp, dp]
        L.or_resample_bits.argtypes = [c_int]
        L.or_resample.argtypes = [c_int, dp, c_uint32, i32p]
        L.or_update.argtypes = [mp, c_int, dp, dp, c_int, dp, dp, c_double, dp, c_uint64, c_uint32,
                                c_int, dp, dp, dp, dp, i32p, dp]
        L.or_observe.argtypes = [mp, c_int, dp, i32p, dp, dp, c_uint64, c_int, dp]
        L.or_transition.argtypes = [mp, c_int, dp, i32p, dp, dp, c_int, dp]
        L.or_pw_widen.argtypes = [c_int, c_int, c_double, c_double, c_int]
        L.or_pw_step.argtypes = [mp, c_int, dp, c_int, i32p, i32p, dp, i32p, i32p, c_int, dp, c_double, c_double,
                                 c_double, c_uint64, u32p, c_int, i32p, i32p, dp, dp, dp, i32p, dp]
        L.or_soft_value.argtypes = [c_int, c_int, dp, dp, c_double, dp, dp, i32p]
        L.or_plan_steps.argtypes = [mp, c_int, dp, c_int, c_int, i32p, dp, dp, dp, c_uint64, c_int, c_int,
                                    dp, dp]
        L.or_info_nce_rows.argtypes = [c_int, c_int, i32p, dp, dp, dp]
        L.or_info_nce.argtypes = [mp, c_int, dp, i32p, dp, dp, c_int, i32p, c_int, dp, dp, dp, dp]
        L.or_info_nce_param_grad.argtypes = [mp, c_int, dp, i32p, dp, dp, c_int, dp, dp]
        L.or_cosine_abar.argtypes = [c_double]
        L.or_cosine_abar.restype = c_double
        L.or_ddim_sample.argtypes = [c_int, ip, dp, c_int, c_int, c_int, c_int, c_int, dp, c_int, dp, dp, c_int, c_int,
                                     dp]
        L.or_ddim_point_mass.argtypes = [c_int, dp, dp, c_int, dp]
        L.or_ddim_gaussian.argtypes = [c_int, dp, c_double, dp, c_int, dp]
        L.or_mlp_param_count.argtypes = [c_int, ip]
        L.or_mlp_param_count.restype = c_size_t
        L.or_set_threads.argtypes = [c_int]
        L.or_set_threads.restype = c_int
        _LIB = L
    return _LIB


# --------------------------------------------------------------------------- helpers
def _d(a):
    """Contiguous binary64 copy (exact for binary32 input) or None."""
    if a is None:
        return None
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _p(a, ctype=c_double):
    return None if a is None else a.ctypes.data_as(POINTER(ctype))


def _check(rc, what):
    if rc != OR_OK:
        raise OracleError(f"oracle {what} failed with code {rc}")


def flatten_layers(layers):
    """(dims int32 array, params float64 array) from [(W, b), ...]."""
    dims = [int(layers[0][0].shape[1])] + [int(W.shape[0]) for W, _ in layers]
    parts = []
    for W, b in layers:
        parts.append(np.asarray(W, np.float64).ravel())
        parts.append(np.asarray(b, np.float64).ravel())
    return np.array(dims, dtype=np.int32), np.ascontiguousarray(np.concatenate(parts))


class _Bound:
    """A C model struct together with the arrays it points into."""

    def __init__(self, model):
        self.keep = []
        cm = _CModel()
        cm.d_s, cm.n_actions, cm.d_a = model.d_s, model.n_actions, model.d_a
        cm.d_w, cm.d_o, cm.d_wz = model.d_w, model.d_o, model.d_wz
        cm.residual = 1 if model.residual else 0
        for tag, layers in (("t", model.trans), ("z", model.obs), ("l", model.lik)):
            if layers:
                dims, params = flatten_layers(layers)
                self.keep += [dims, params]
                setattr(cm, f"{tag}_layers", len(layers))
                setattr(cm, f"{tag}_dims", dims.ctypes.data_as(POINTER(c_int)))
                setattr(cm, f"{tag}_params", params.ctypes.data_as(POINTER(c_double)))
            else:
                setattr(cm, f"{tag}_layers", 0)
        self.c = cm

    def ref(self):
        return ctypes.byref(self.c)


def _cands(model, cands):
    if model.n_actions > 0:
        return np.ascontiguousarray(np.asarray(cands, np.int32)), None
    return None, _d(cands)


# --------------------------------------------------------------------------- RNG
def philox(counter, key):
    """Philox4x32-10 of one 4-word counter under a 2-word key -> 4 uint32."""
    c = np.ascontiguousarray(np.asarray(counter, np.uint32))
    k = np.ascontiguousarray(np.asarray(key, np.uint32))
    out = np.zeros(4, np.uint32)
    lib().or_philox4x32_10(_p(c, c_uint32), _p(k, c_uint32), _p(out, c_uint32))
    return out


def uniform(x: int) -> float:
    return lib().or_uniform(int(x))


def normals(seed, c0, c1, c2, stream, d):
    out = np.zeros(d, np.float64)
    lib().or_normals(int(seed), int(c0), int(c1), int(c2), int(stream), int(d), _p(out))
    return out


def normals_rows(seed, n, c1, c2, stream, d):
    """Normals of counters (r, c1, c2) for r = 0..n-1 as an [n, d] array."""
    L = lib()
    if not hasattr(L, "_rows_ready"):
        L.or_normals_rows.argtypes = [c_uint64, c_int, c_uint32, c_uint32, c_uint32, c_int, POINTER(c_double)]
        L._rows_ready = True
    out = np.zeros((n, d), np.float64)
    L.or_normals_rows(int(seed), int(n), int(c1), int(c2), int(stream), int(d), _p(out))
    return out


def round_bf16(x):
    x = np.asarray(x, np.float64)
    f = np.vectorize(lambda v: lib().or_round_bf16(float(v)), otypes=[np.float64])
    return f(x)


# --------------------------------------------------------------------------- networks
def mlp(layers, X, bf16=False):
    """Rows of X through the network: ReLU hidden layers, linear output."""
    dims, params = flatten_layers(layers)
    X = _d(np.atleast_2d(X))
    Y = np.zeros((X.shape[0], int(dims[-1])), np.float64)
    _check(lib().or_mlp(len(layers), dims.ctypes.data_as(POINTER(c_int)), _p(params), X.shape[0],
                        _p(X), _p(Y), int(bf16)), "mlp")
    return Y


def transition(model, S, actions, noise, bf16=False):
    """s' = s + f_T([s, a, w]) for given rows (actions one per row)."""
    S = _d(np.atleast_2d(S))
    n = S.shape[0]
    a_disc, a_cont = (np.ascontiguousarray(np.asarray(actions, np.int32).reshape(n)), None) \
        if model.n_actions > 0 else (None, _d(np.asarray(actions).reshape(n, model.d_a)))
    W = _d(np.asarray(noise).reshape(n, model.d_w))
    out = np.zeros((n, model.d_s), np.float64)
    b = _Bound(model)
    _check(lib().or_transition(b.ref(), n, _p(S), _p(a_disc, c_int32), _p(a_cont), _p(W),
                               int(bf16), _p(out)), "transition")
    return out


def observe(model, S, actions, noise=None, seed=0, bf16=False):
    """o = f_Z([s', a, w_Z]) per row; noise given or drawn from stream 4."""
    S = _d(np.atleast_2d(S))
    n = S.shape[0]
    a_disc, a_cont = (np.ascontiguousarray(np.asarray(actions, np.int32).reshape(n)), None) \
        if model.n_actions > 0 else (None, _d(np.asarray(actions).reshape(n, model.d_a)))
    W = None if noise is None else _d(np.asarray(noise).reshape(n, model.d_wz))
    out = np.zeros((n, model.d_o), np.float64)
    b = _Bound(model)
    _check(lib().or_observe(b.ref(), n, _p(S), _p(a_disc, c_int32), _p(a_cont), _p(W), int(seed),
                            int(bf16), _p(out)), "observe")
    return out


# --------------------------------------------------------------------------- plan
def plan(model, states, cands, gamma, goal, belief_w=None, noise=None, seed=0, crn=False,
         reward_at=0, bf16=False, return_G=False):
    """Q[K] (and G[K, N]) of open-loop candidate sequences from a particle belief."""
    S = _d(states)
    N = S.shape[0]
    cd, cc = _cands(model, cands)
    K, H = int(np.asarray(cands).shape[0]), int(np.asarray(cands).shape[1])
    Q = np.zeros(K, np.float64)
    G = np.zeros((K, N), np.float64)
    nz = None if noise is None else _d(noise)
    if nz is not None:
        assert nz.shape == (K, N, H, model.d_w), nz.shape
    b = _Bound(model)
    _check(lib().or_plan(b.ref(), N, _p(S), _p(_d(belief_w)), K, H, _p(cd, c_int32), _p(cc),
                         float(gamma), _p(_d(goal)), int(reward_at), _p(nz), int(seed), int(crn),
                         int(bf16), _p(Q), _p(G)), "plan")
    return (Q, G) if return_G else Q


def rollouts(model, states, cands, gamma, goal, pairs, seed=0, crn=False, reward_at=0, bf16=False):
    """Returns G of selected rollouts [(k, i), ...] under counter-RNG noise."""
    S = _d(states)
    N = S.shape[0]
    cd, cc = _cands(model, cands)
    K, H = int(np.asarray(cands).shape[0]), int(np.asarray(cands).shape[1])
    pairs = np.asarray(pairs, np.int32).reshape(-1, 2)
    ks = np.ascontiguousarray(pairs[:, 0])
    is_ = np.ascontiguousarray(pairs[:, 1])
    out = np.zeros(len(pairs), np.float64)
    b = _Bound(model)
    _check(lib().or_rollouts(b.ref(), N, _p(S), K, H, _p(cd, c_int32), _p(cc), float(gamma),
                             _p(_d(goal)), int(reward_at), int(seed), int(crn), int(bf16), len(pairs),
                             _p(ks, c_int32), _p(is_, c_int32), _p(out)), "rollouts")
    return out


def plan_steps(model, states, cands, noise=None, obs_noise=None, seed=0, crn=False, bf16=False, want_obs=True):
    """(traj [K, N, H, d_s], obs [K, N, H, d_o] or None): the rollout states
    s_1..s_H of plan and an observation f_Z([s_{t+1}, a_t, w_Z]) per step."""
    S = _d(states)
    N = S.shape[0]
    cd, cc = _cands(model, cands)
    K, H = int(np.asarray(cands).shape[0]), int(np.asarray(cands).shape[1])
    nz = None if noise is None else _d(noise)
    if nz is not None:
        assert nz.shape == (K, N, H, model.d_w), nz.shape
    oz = None if obs_noise is None else _d(obs_noise)
    if oz is not None:
        assert oz.shape == (K, N, H, model.d_wz), oz.shape
    traj = np.zeros((K, N, H, model.d_s), np.float64)
    obs = np.zeros((K, N, H, model.d_o), np.float64) if want_obs else None
    b = _Bound(model)
    _check(lib().or_plan_steps(b.ref(), N, _p(S), K, H, _p(cd, c_int32), _p(cc), _p(nz), _p(oz), int(seed),
                               int(crn), int(bf16), _p(traj), _p(obs)), "plan_steps")
    return traj, obs


def pw_widen(visits, children, k_o, alpha_o, capacity):
    """Progressive-widening test of one action node (1: add a branch)."""
    return lib().or_pw_widen(int(visits), int(children), float(k_o), float(alpha_o), int(capacity))


def pw_step(model, succ, seg, actions, visits, children, obs_table, k_o, alpha_o, lam, seed, U, bf16=False):
    """Grouped progressive-widening step over M action nodes.  Returns a dict
    (widen, branch, loglik, w, stats, idx, S_out, children, obs_table); the
    last two are updated copies of the inputs."""
    S = _d(succ)
    T = S.shape[0]
    seg = np.ascontiguousarray(np.asarray(seg, np.int32))
    M = seg.shape[0] - 1
    a_disc, a_cont = (np.ascontiguousarray(np.asarray(actions, np.int32).reshape(M)), None) \
        if model.n_actions > 0 else (None, _d(np.asarray(actions).reshape(M, model.d_a)))
    vis = np.ascontiguousarray(np.asarray(visits, np.int32))
    ch = np.array(children, np.int32)
    tab = np.array(obs_table, np.float64)
    B = tab.shape[1]
    assert tab.shape == (M, B, model.d_o)
    Uv = np.ascontiguousarray(np.asarray(U, np.uint32))
    out = dict(widen=np.zeros(M, np.int32), branch=np.zeros(M, np.int32), loglik=np.zeros(T), w=np.zeros(T),
               stats=np.zeros((M, 2)), idx=np.zeros(T, np.int32), S_out=np.zeros((T, model.d_s)))
    b = _Bound(model)
    _check(lib().or_pw_step(b.ref(), T, _p(S), M, _p(seg, c_int32), _p(a_disc, c_int32), _p(a_cont),
                            _p(vis, c_int32), _p(ch, c_int32), B, _p(tab), float(k_o), float(alpha_o), float(lam),
                            int(seed), _p(Uv, c_uint32), int(bf16), _p(out["widen"], c_int32),
                            _p(out["branch"], c_int32), _p(out["loglik"]), _p(out["w"]), _p(out["stats"]),
                            _p(out["idx"], c_int32), _p(out["S_out"])), "pw_step")
    out["children"] = ch
    out["obs_table"] = tab
    return out


def soft_value(Q, eta, log_pi0=None):
    """(V [M], pi [M, K], best [M]) of preferences Q [M, K] (1-D: one node)
    with reference-policy log-probabilities log_pi0 (None: uniform)."""
    Qa = np.atleast_2d(_d(Q))
    M, K = Qa.shape
    lp = None if log_pi0 is None else np.ascontiguousarray(np.atleast_2d(_d(log_pi0)))
    V = np.zeros(M)
    pi = np.zeros((M, K))
    best = np.zeros(M, np.int32)
    _check(lib().or_soft_value(M, K, _p(np.ascontiguousarray(Qa)), _p(lp), float(eta), _p(V), _p(pi),
                               _p(best, c_int32)), "soft_value")
    return V, pi, best


def plan_closed_loop(model, states, first, n_obs, cont, gamma, eta, lam, goal, seed, U, log_pi0=None, bf16=False):
    """One-level closed-loop tree of the preference backup (Eq. 1), built
    from the functions above:
      1. every particle is moved one step under each first action a (plan of
         horizon 1, key `seed`): successors s'_{a,i} and R(b, a) = mean_i R(s'_{a,i});
      2. n_obs observation branches per first action: branch j of action a is
         the successor set of a starting at successor j, widened once by the
         grouped progressive-widening step (key `seed`, offsets U[a n_obs + j]),
         which draws its observation at that successor and resamples the set
         against it -- the child belief tau(b, a, o_j);
      3. every child belief is valued by the continuation candidates (plan of
         their horizon, key seed + 1): Q_child[k] = mean over the child's
         particles of the returns, V_child = L_eta Q_child (uniform prior);
      4. Psi(b, a) = (1/eta) log pi0(a) + R(b, a) + gamma mean_j V_child(a, j),
         V(b) = L_eta Psi, with the soft policy and the greedy first action.
    Returns a dict (psi, V, pi, best, R, V_child, child)."""
    S = np.asarray(states, np.float64)
    N = S.shape[0]
    first = np.asarray(first)
    A = first.shape[0]
    cands1 = first.reshape(A, 1) if model.n_actions > 0 else first.reshape(A, 1, model.d_a)
    R, _ = plan(model, S, cands1, 1.0, goal, seed=seed, bf16=bf16, return_G=True)
    traj, _ = plan_steps(model, S, cands1, seed=seed, bf16=bf16, want_obs=False)
    M = A * n_obs
    succ = np.concatenate([np.roll(traj[a, :, 0], -j, axis=0) for a in range(A) for j in range(n_obs)])
    seg = np.arange(M + 1, dtype=np.int32) * N
    acts = np.repeat(first, n_obs, axis=0)
    out = pw_step(model, succ, seg, acts, np.zeros(M, np.int32), np.zeros(M, np.int32),
                  np.zeros((M, 1, model.d_o)), 1.0, 1.0, lam, seed, U, bf16=bf16)
    child = out["S_out"]
    cont = np.asarray(cont)
    K = cont.shape[0]
    _, G2 = plan(model, child, cont, gamma, goal, seed=seed + 1, bf16=bf16, return_G=True)
    Qc = G2.reshape(K, M, N).mean(axis=2).T
    Vc, _, _ = soft_value(Qc, eta)
    lp = np.full(A, -np.log(A)) if log_pi0 is None else np.asarray(log_pi0, np.float64)
    psi = lp / eta + R + gamma * Vc.reshape(A, n_obs).mean(axis=1)
    V, pi, best = soft_value(psi[None, :], eta, log_pi0=np.zeros((1, A)))
    return dict(psi=psi, V=V[0], pi=pi[0], best=int(best[0]), R=R, V_child=Vc, child=child)


def info_nce_from_scores(scores, rows=None):
    """(row_loss [R], G [R, B]) of score rows [R, B] (Eq. 6): row r is the
    state-action of tuple rows[r] (None: r) against all B observations,
    row_loss_r = log sum_j exp(l_rj) - l_r,rows[r], and G the derivative of
    the batch's mean row loss with respect to each score."""
    L = np.atleast_2d(_d(scores))
    R, B = L.shape
    rw = None if rows is None else np.ascontiguousarray(np.asarray(rows, np.int32))
    if rw is None:
        assert R == B
    rl = np.zeros(R)
    G = np.zeros((R, B))
    _check(lib().or_info_nce_rows(B, R, _p(rw, c_int32), _p(np.ascontiguousarray(L)), _p(rl), _p(G)),
           "info_nce_rows")
    return rl, G


def info_nce(model, states, actions, obs, rows=None, bf16=False):
    """InfoNCE objective of the likelihood network on a mini-batch of B
    tuples (s'_i, a_i, o_i) (Sec. 4.2, Eq. 6).  Returns a dict with scores
    [R, B] (l([s'_i, a_i, o_j]) for the listed rows i, None: all), row_loss
    [R], G [R, B] (derivative of the loss with respect to each score) and,
    with all rows, loss (the mean row loss)."""
    S = _d(states)
    B = S.shape[0]
    O = _d(np.asarray(obs).reshape(B, model.d_o))
    if model.n_actions > 0:
        a_disc, a_cont = np.ascontiguousarray(np.asarray(actions, np.int32).reshape(B)), None
    else:
        a_disc, a_cont = None, _d(np.asarray(actions).reshape(B, model.d_a))
    rw = None if rows is None else np.ascontiguousarray(np.asarray(rows, np.int32))
    R = B if rw is None else rw.shape[0]
    out = dict(scores=np.zeros((R, B)), row_loss=np.zeros(R), G=np.zeros((R, B)))
    loss = np.zeros(1)
    b = _Bound(model)
    _check(lib().or_info_nce(b.ref(), B, _p(S), _p(a_disc, c_int32), _p(a_cont), _p(O), R, _p(rw, c_int32),
                             int(bf16), _p(out["scores"]), _p(out["row_loss"]), _p(out["G"]),
                             _p(loss if rw is None else None)), "info_nce")
    if rw is None:
        out["loss"] = float(loss[0])
    return out


def info_nce_param_grad(model, states, actions, obs, bf16=False):
    """(loss, gradient) of the InfoNCE loss with respect to the likelihood
    network's parameters, packed per layer as W (row-major [out, in]) then b.
    bf16=True: the bfloat16 emulation (weights, layer inputs and hidden
    adjoints rounded to bfloat16, binary64 accumulation)."""
    S = _d(states)
    B = S.shape[0]
    O = _d(np.asarray(obs).reshape(B, model.d_o))
    if model.n_actions > 0:
        a_disc, a_cont = np.ascontiguousarray(np.asarray(actions, np.int32).reshape(B)), None
    else:
        a_disc, a_cont = None, _d(np.asarray(actions).reshape(B, model.d_a))
    dims, _ = flatten_layers(model.lik)
    g = np.zeros(int(lib().or_mlp_param_count(len(model.lik), dims.ctypes.data_as(POINTER(c_int)))))
    loss = np.zeros(1)
    b = _Bound(model)
    _check(lib().or_info_nce_param_grad(b.ref(), B, _p(S), _p(a_disc, c_int32), _p(a_cont), _p(O), int(bf16),
                                        _p(g), _p(loss)), "info_nce_param_grad")
    return float(loss[0]), g


def cosine_abar(tau):
    """Cosine cumulative noise schedule abar(tau), abar(0) = 1."""
    return lib().or_cosine_abar(float(tau))


def ddim_sample(layers, d_c, d_x, n_actions, d_a, cond, action, x1, n_steps, bf16=False):
    """Teacher samples [n, d_x]: the DDIM (ODE) sampler of the v-prediction
    denoiser `layers` (input [c, a, x_tau, tau], output v [d_x]) in n_steps
    uniform steps from x1 [n, d_x] (the latent noise at tau = 1),
    conditioned on cond [n, d_c] and one action (index or [d_a] values)."""
    C = _d(cond)
    n = C.shape[0]
    X1 = _d(np.asarray(x1).reshape(n, d_x))
    dims, params = flatten_layers(layers)
    a_disc, a_cont = (int(action), None) if n_actions > 0 else (0, _d(np.asarray(action).reshape(d_a)))
    out = np.zeros((n, d_x))
    _check(lib().or_ddim_sample(len(layers), dims.ctypes.data_as(POINTER(c_int)), _p(params), d_c, d_x, n_actions,
                                d_a, n, _p(C), a_disc, _p(a_cont), _p(X1), int(n_steps), int(bf16), _p(out)),
           "ddim_sample")
    return out


def ddim_gaussian(mu, sigma, x1, n_steps):
    """The sampler's steps driven by the exact v of Gaussian data N(mu, sigma^2 I)."""
    mu, x1 = _d(np.ravel(mu)), _d(np.ravel(x1))
    out = np.zeros_like(x1)
    _check(lib().or_ddim_gaussian(x1.shape[0], _p(mu), float(sigma), _p(x1), int(n_steps), _p(out)), "ddim_gaussian")
    return out


def ddim_point_mass(x0, x1, n_steps):
    """The sampler's steps driven by the exact v of a point mass at x0."""
    x0, x1 = _d(np.ravel(x0)), _d(np.ravel(x1))
    out = np.zeros_like(x1)
    _check(lib().or_ddim_point_mass(x1.shape[0], _p(x0), _p(x1), int(n_steps), _p(out)), "ddim_point_mass")
    return out


def weighted_mean(G, w=None):
    G = _d(G)
    return lib().or_weighted_mean(G.shape[0], _p(G), _p(_d(w)))


# --------------------------------------------------------------------------- update
def normalize(loglik, lam=1.0, prior_w=None):
    """(w', [log evidence, ESS]) for weights proportional to prior * exp(l / lam)."""
    ll = _d(loglik)
    N = ll.shape[0]
    w = np.zeros(N, np.float64)
    st = np.zeros(2, np.float64)
    _check(lib().or_normalize(N, _p(ll), _p(_d(prior_w)), float(lam), _p(w), _p(st)), "normalize")
    return w, st


def resample_bits(N: int) -> int:
    return lib().or_resample_bits(int(N))


def resample(w, U):
    """Systematic resampling indices [N] int32 on quantised weights."""
    w = _d(w)
    N = w.shape[0]
    idx = np.zeros(N, np.int32)
    _check(lib().or_resample(N, _p(w), int(U) & 0xFFFFFFFF, _p(idx, c_int32)), "resample")
    return idx


def update(model, states, action, obs, lam=1.0, prior_w=None, noise=None, seed=0, U=0, bf16=False):
    """SIR belief update.  Returns a dict with S_prop, loglik, w, stats, idx, S_new."""
    S = _d(states)
    N = S.shape[0]
    if model.n_actions > 0:
        a_disc, a_cont = int(action), None
    else:
        a_disc, a_cont = 0, _d(np.asarray(action).reshape(model.d_a))
    o = _d(np.asarray(obs).reshape(model.d_o))
    nz = None if noise is None else _d(np.asarray(noise).reshape(N, model.d_w))
    out = dict(S_prop=np.zeros((N, model.d_s)), loglik=np.zeros(N), w=np.zeros(N),
               stats=np.zeros(2), idx=np.zeros(N, np.int32), S_new=np.zeros((N, model.d_s)))
    b = _Bound(model)
    _check(lib().or_update(b.ref(), N, _p(S), _p(_d(prior_w)), a_disc, _p(a_cont), _p(o), float(lam),
                           _p(nz), int(seed), int(U) & 0xFFFFFFFF, int(bf16), _p(out["S_prop"]),
                           _p(out["loglik"]), _p(out["w"]), _p(out["stats"]),
                           _p(out["idx"], c_int32), _p(out["S_new"])), "update")
    return out


def draw_observation(w, bf16=False):
    """The observation of a workload: a true state drawn from the belief is moved
    by the transition sampler with the executed action and observed through the
    observation sampler, both with the workload's explicit noise."""
    m = w.model
    s_true = np.asarray(w.states[w.true_index], np.float64)[None, :]
    a = np.asarray(w.update_action)
    s_next = transition(m, s_true, a.reshape(1, -1) if m.n_actions == 0 else [int(a)],
                        w.true_noise[None, :], bf16=bf16)
    return observe(m, s_next, a.reshape(1, -1) if m.n_actions == 0 else [int(a)],
                   noise=w.obs_noise[None, :], bf16=bf16)[0]


# --------------------------------------------------------------------------- gradients
DISTILL, RETURN = 0, 1


def _grad_args(model, S0, actions, H, particles, noise, targets, goal):
    S0 = _d(S0)
    B = S0.shape[0]
    if model.n_actions > 0:
        ad = np.ascontiguousarray(np.asarray(actions, np.int32).reshape(B, H))
        ac = None
    else:
        ad = None
        ac = _d(np.asarray(actions).reshape(-1, H, model.d_a))
    nz = None if noise is None else _d(np.asarray(noise).reshape(B, H, model.d_w))
    tg = None if targets is None else _d(np.asarray(targets).reshape(B, H, model.d_s))
    g = _d(goal) if goal is not None else np.zeros(model.d_s)
    return S0, B, ad, ac, nz, tg, g


def _lib_grad():
    L = lib()
    if not hasattr(L, "_grad_ready"):
        dp, i32p, mp = POINTER(c_double), POINTER(c_int32), POINTER(_CModel)
        L.or_rollout_objective.argtypes = [mp, c_int, c_int, c_int, dp, i32p, dp, dp, c_uint64, c_int, dp,
                                           c_double, dp, POINTER(c_uint64)]
        L.or_rollout_objective.restype = c_double
        L.or_rollout_grad.argtypes = [mp, c_int, c_int, c_int, dp, i32p, dp, dp, c_uint64, c_int, dp, c_double,
                                      dp, dp, dp, dp]
        L._grad_ready = True
    return L


def rollout_objective(model, S0, actions, H, objective, targets=None, gamma=1.0, goal=None, particles=1,
                      noise=None, seed=0, patterns=False):
    """Distillation loss (objective 0) or mean discounted return (objective 1)
    of free-running rollouts; with patterns=True also each rollout's ReLU
    sign-pattern hash (to detect finite differences that straddle a kink)."""
    S0, B, ad, ac, nz, tg, g = _grad_args(model, S0, actions, H, particles, noise, targets, goal)
    pat = np.zeros(B, np.uint64) if patterns else None
    b = _Bound(model)
    v = _lib_grad().or_rollout_objective(b.ref(), B, H, particles, _p(S0), _p(ad, c_int32), _p(ac), _p(nz),
                                         int(seed), int(objective), _p(tg), float(gamma), _p(g),
                                         None if pat is None else pat.ctypes.data_as(POINTER(c_uint64)))
    return (v, pat) if patterns else v


def rollout_grad(model, S0, actions, H, objective, targets=None, gamma=1.0, goal=None, particles=1, noise=None,
                 seed=0, want_params=True, want_actions=False):
    """(objective value, d/dparams as [(dW, db), ...] or None, d/dA or None)."""
    S0, B, ad, ac, nz, tg, g = _grad_args(model, S0, actions, H, particles, noise, targets, goal)
    dims, params = flatten_layers(model.trans)
    gp = np.zeros_like(params) if want_params else None
    ga = np.zeros_like(ac) if (want_actions and ac is not None) else None
    loss = np.zeros(1)
    b = _Bound(model)
    _check(_lib_grad().or_rollout_grad(b.ref(), B, H, particles, _p(S0), _p(ad, c_int32), _p(ac), _p(nz), int(seed),
                                       int(objective), _p(tg), float(gamma), _p(g), _p(loss), _p(gp), _p(ga)),
           "rollout_grad")
    layers = None
    if gp is not None:
        layers, off = [], 0
        for n_in, n_out in zip(dims[:-1], dims[1:]):
            W = gp[off:off + n_out * n_in].reshape(n_out, n_in)
            off += n_out * n_in
            bb = gp[off:off + n_out]
            off += n_out
            layers.append((W, bb))
    return float(loss[0]), layers, ga


def teacher_targets(teacher_model, S0, actions, H, particles=1, noise=None, seed=0):
    """States s_1..s_H [B, H, d_s] of the teacher network's rollouts from the
    same initial states, actions and noise (the distillation targets)."""
    S0 = _d(S0)
    B, d_s = S0.shape
    out = np.zeros((B, H, d_s))
    s = S0.copy()
    for t in range(H):
        if teacher_model.n_actions > 0:
            a = np.asarray(actions, np.int32).reshape(B, H)[:, t]
        else:
            A = np.asarray(actions, np.float64).reshape(-1, H, teacher_model.d_a)
            a = A[np.arange(B) // particles, t]
        if noise is not None:
            w = np.asarray(noise, np.float64).reshape(B, H, teacher_model.d_w)[:, t]
        else:
            w = normals_rows(seed, B, 0, t, 3, teacher_model.d_w)
        s = transition(teacher_model, s, a, w)
        out[:, t] = s
    return out


def set_threads(n):
    """Threads of the oracle's parallel loops (results do not depend on it); returns the previous count."""
    return int(lib().or_set_threads(int(n)))
