"""Python binding of libvoila: the VOiLA planning hot path on MI355X (gfx950).

Argument marshalling only.  Every step of plan / update / observe runs in the
HIP kernels of ``libvoila.so`` (built by ``build.py``); torch provides device
memory and the stream.  There is no CPU fallback: importing this package
raises if the library has not been built, and every call raises
``VoilaError`` when the library reports a failure.

Functions mirror include/voila.h:

* ``Model(desc, compute="f32"|"bf16", device=0)``  voila_model_create
* ``plan(model, states, cands, gamma, goal, ...)`` -> Q [K] (and G [K, N])
* ``update(model, states, action, obs, ...)``      -> dict of the new belief
* ``normalize(loglik, lam, prior_w)``              -> (w, stats)
* ``resample(w, U, src=None)``                     -> idx (and gathered rows)
* ``observe(model, states, action, ...)``          -> o [n, d_o]
* ``philox_normals(seed, c0, c1, c2, stream, n, d)`` -> (normals, words)
"""
from __future__ import annotations

import ctypes
import math
import os
from ctypes import POINTER, c_double, c_float, c_int32, c_size_t, c_uint32, c_uint64, c_void_p

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libvoila.so")

VOILA_OK = 0
VOILA_ERR_INVALID_ARG = 1
VOILA_ERR_UNSUPPORTED = 2
VOILA_ERR_WORKSPACE = 3
VOILA_ERR_DEVICE = 4
VOILA_ERR_NUMERIC = 5
VOILA_F32 = 0
VOILA_BF16 = 1


class VoilaError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"voila status {status}: {msg}")
        self.status = status


class _Mlp(ctypes.Structure):
    _fields_ = [("n_layers", c_int32), ("h_dims", POINTER(c_int32)),
                ("h_W", POINTER(POINTER(c_float))), ("h_b", POINTER(POINTER(c_float)))]


class _ModelDesc(ctypes.Structure):
    _fields_ = [("d_s", c_int32), ("n_actions", c_int32), ("d_a", c_int32), ("d_w", c_int32),
                ("d_o", c_int32), ("d_wz", c_int32), ("trans", _Mlp), ("obs", _Mlp), ("lik", _Mlp),
                ("compute", c_int32)]


class _PlanOpts(ctypes.Structure):
    _fields_ = [("gamma", c_double), ("h_goal", POINTER(c_float)), ("seed", c_uint64), ("crn", c_int32),
                ("reward_at", c_int32), ("d_noise", c_void_p), ("d_traj_out", c_void_p)]


class _UpdateOpts(ctypes.Structure):
    _fields_ = [("lambda_", c_double), ("seed", c_uint64), ("resample_u", c_uint32), ("d_noise", c_void_p)]


class _BatchItem(ctypes.Structure):
    _fields_ = [("model", c_void_p), ("d_states", c_void_p), ("d_belief_w", c_void_p), ("N", c_int32),
                ("d_cands", c_void_p), ("K", c_int32), ("H", c_int32), ("gamma", c_double),
                ("h_goal", POINTER(c_float)), ("seed", c_uint64), ("crn", c_int32), ("reward_at", c_int32),
                ("d_q_out", c_void_p), ("d_returns_out", c_void_p), ("lambda_", c_double),
                ("update_seed", c_uint64), ("d_states_out", c_void_p), ("d_idx_out", c_void_p),
                ("d_w_out", c_void_p), ("d_stats_out", c_void_p)]


class _PwOpts(ctypes.Structure):
    _fields_ = [("k_o", c_double), ("alpha_o", c_double), ("lambda_", c_double), ("seed", c_uint64),
                ("capacity", c_int32)]


class _ClosedLoopOpts(ctypes.Structure):
    _fields_ = [("gamma", c_double), ("eta", c_double), ("lambda_", c_double), ("h_goal", POINTER(c_float)),
                ("seed", c_uint64), ("n_obs", c_int32), ("d_log_pi0", c_void_p), ("d_U", c_void_p)]


class _GradOpts(ctypes.Structure):
    _fields_ = [("B", c_int32), ("H", c_int32), ("checkpoint", c_int32), ("d_s0", c_void_p),
                ("d_actions", c_void_p), ("particles", c_int32), ("d_noise", c_void_p), ("seed", c_uint64),
                ("objective", c_int32), ("d_targets", c_void_p), ("gamma", c_double), ("h_goal", POINTER(c_float)),
                ("d_loss_out", c_void_p), ("d_grad_params", c_void_p), ("d_grad_actions", c_void_p)]


VOILA_OBJ_DISTILL = 0
VOILA_OBJ_RETURN = 1


class _BatchTuning(ctypes.Structure):
    _fields_ = [("waves_per_block", c_int32), ("blocks_per_cu", c_int32), ("dynamic", c_int32)]


VOILA_BATCH_PLAN = 1
VOILA_BATCH_UPDATE = 2


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_2606_19729_amd/build.py "
                          "(the HIP library is the only implementation; there is no fallback)")
    L = ctypes.CDLL(LIB_PATH)
    vp = c_void_p
    L.voila_version.restype = c_int32
    L.voila_status_string.argtypes = [c_int32]
    L.voila_status_string.restype = ctypes.c_char_p
    L.voila_last_error.restype = ctypes.c_char_p
    L.voila_model_create.argtypes = [POINTER(_ModelDesc), c_int32, POINTER(vp)]
    L.voila_model_create.restype = c_int32
    L.voila_model_destroy.argtypes = [vp]
    L.voila_model_destroy.restype = c_int32
    L.voila_plan_workspace_size.argtypes = [vp, c_int32, c_int32, c_int32]
    L.voila_plan_workspace_size.restype = c_size_t
    L.voila_plan.argtypes = [vp, vp, vp, c_int32, vp, c_int32, c_int32, POINTER(_PlanOpts), vp, c_size_t,
                             vp, vp, vp, vp]
    L.voila_plan.restype = c_int32
    L.voila_update_workspace_size.argtypes = [vp, c_int32]
    L.voila_update_workspace_size.restype = c_size_t
    L.voila_update.argtypes = [vp, vp, vp, c_int32, vp, vp, POINTER(_UpdateOpts), vp, c_size_t,
                               vp, vp, vp, vp, vp, vp, vp, vp]
    L.voila_update.restype = c_int32
    L.voila_update_noalloc.argtypes = [vp, vp, vp, c_int32, vp, vp, POINTER(_UpdateOpts), vp, vp, vp, vp, vp, vp,
                                       vp, vp]
    L.voila_update_noalloc.restype = c_int32
    L.voila_update_max_particles.restype = c_int32
    L.voila_normalize.argtypes = [vp, vp, c_int32, c_double, vp, vp, vp, vp, c_size_t, vp]
    L.voila_normalize.restype = c_int32
    L.voila_resample_bits.argtypes = [c_int32]
    L.voila_resample_bits.restype = c_int32
    L.voila_resample.argtypes = [vp, c_int32, c_uint32, vp, vp, vp, c_int32, vp, vp, c_size_t, vp]
    L.voila_reweight_resample.argtypes = [vp, vp, c_int32, c_double, c_uint32, vp, vp, vp, vp, vp, c_int32, vp,
                                          vp, c_size_t, vp]
    L.voila_reweight_resample.restype = c_int32
    L.voila_weights_workspace_size.argtypes = [c_int32]
    L.voila_weights_workspace_size.restype = c_size_t
    L.voila_resample.restype = c_int32
    L.voila_observe_workspace_size.argtypes = [vp]
    L.voila_observe_workspace_size.restype = c_size_t
    L.voila_observe.argtypes = [vp, vp, c_int32, vp, c_uint64, vp, vp, c_size_t, vp, vp, vp]
    L.voila_observe.restype = c_int32
    L.voila_plan_observe_workspace_size.argtypes = [vp, c_int32, c_int32]
    L.voila_plan_observe_workspace_size.restype = c_size_t
    L.voila_plan_observe.argtypes = [vp, vp, c_int32, vp, c_int32, c_int32, c_uint64, c_int32, vp, vp, c_size_t, vp,
                                     vp, vp]
    L.voila_plan_observe.restype = c_int32
    L.voila_soft_value.argtypes = [vp, vp, c_int32, c_int32, c_double, vp, vp, vp, vp, vp]
    L.voila_soft_value.restype = c_int32
    L.voila_plan_closed_loop_workspace_size.argtypes = [vp, c_int32, c_int32, c_int32, c_int32, c_int32]
    L.voila_plan_closed_loop_workspace_size.restype = c_size_t
    L.voila_plan_closed_loop.argtypes = [vp, vp, c_int32, vp, c_int32, vp, c_int32, c_int32,
                                         POINTER(_ClosedLoopOpts), vp, c_size_t, vp, vp, vp, vp, vp, vp, vp, vp, vp]
    L.voila_plan_closed_loop.restype = c_int32
    L.voila_pw_step_workspace_size.argtypes = [vp, c_int32, c_int32]
    L.voila_pw_step_workspace_size.restype = c_size_t
    L.voila_pw_step.argtypes = [vp, vp, c_int32, vp, c_int32, vp, vp, vp, vp, vp, POINTER(_PwOpts), vp, c_size_t,
                                vp, vp, vp, vp, vp, vp, vp, vp, vp]
    L.voila_pw_step.restype = c_int32
    L.voila_info_nce_workspace_size.argtypes = [vp, c_int32]
    L.voila_info_nce_workspace_size.restype = c_size_t
    L.voila_info_nce.argtypes = [vp, vp, vp, vp, c_int32, vp, c_size_t, vp, vp, vp, vp, vp, vp]
    L.voila_info_nce.restype = c_int32
    L.voila_info_nce_param_count.argtypes = [vp]
    L.voila_info_nce_param_count.restype = c_int32
    L.voila_info_nce_grad_workspace_size.argtypes = [vp, c_int32]
    L.voila_info_nce_grad_workspace_size.restype = c_size_t
    L.voila_info_nce_grad.argtypes = [vp, vp, vp, vp, c_int32, vp, c_size_t, vp, vp, vp, vp]
    L.voila_info_nce_grad.restype = c_int32
    L.voila_denoiser_create.argtypes = [POINTER(_Mlp), c_int32, c_int32, c_int32, c_int32, c_int32, c_int32,
                                        POINTER(vp)]
    L.voila_denoiser_create.restype = c_int32
    L.voila_denoiser_destroy.argtypes = [vp]
    L.voila_denoiser_destroy.restype = c_int32
    L.voila_ddim_workspace_size.argtypes = [vp, c_int32]
    L.voila_ddim_workspace_size.restype = c_size_t
    L.voila_ddim_sample.argtypes = [vp, vp, vp, vp, c_int32, c_int32, vp, c_size_t, vp, vp]
    L.voila_ddim_sample.restype = c_int32
    L.voila_philox_normals.argtypes = [c_uint64, c_uint32, c_uint32, c_uint32, c_uint32, c_int32, c_int32, vp,
                                       vp, vp]
    L.voila_philox_normals.restype = c_int32
    L.voila_batch_create.argtypes = [POINTER(_BatchItem), c_int32, POINTER(_BatchTuning), POINTER(vp)]
    L.voila_batch_create.restype = c_int32
    L.voila_batch_destroy.argtypes = [vp]
    L.voila_batch_destroy.restype = c_int32
    L.voila_batch_run.argtypes = [vp, c_int32, vp, vp, vp, vp, vp]
    L.voila_batch_run.restype = c_int32
    L.voila_batch_capture.argtypes = [vp, c_int32, vp, vp, vp, vp]
    L.voila_batch_capture.restype = c_int32
    L.voila_batch_replay.argtypes = [vp, vp]
    L.voila_batch_replay.restype = c_int32
    L.voila_grad_param_count.argtypes = [vp]
    L.voila_grad_param_count.restype = c_int32
    L.voila_rollout_grad_workspace_size.argtypes = [vp, POINTER(_GradOpts)]
    L.voila_rollout_grad_workspace_size.restype = c_size_t
    L.voila_rollout_grad.argtypes = [vp, POINTER(_GradOpts), vp, c_size_t, vp]
    L.voila_rollout_grad.restype = c_int32
    return L


lib = _load()

# the exported C symbols (checked by the test-suite against include/voila.h)
EXPORTED = ["voila_version", "voila_status_string", "voila_last_error", "voila_model_create",
            "voila_model_destroy", "voila_plan_workspace_size", "voila_plan", "voila_update_workspace_size",
            "voila_update", "voila_update_noalloc", "voila_update_max_particles", "voila_weights_workspace_size", "voila_normalize",
            "voila_reweight_resample",
            "voila_resample_bits",
            "voila_resample", "voila_observe_workspace_size", "voila_observe", "voila_plan_observe_workspace_size",
            "voila_plan_observe", "voila_pw_step_workspace_size", "voila_pw_step", "voila_soft_value",
            "voila_plan_closed_loop_workspace_size", "voila_plan_closed_loop",
            "voila_info_nce_workspace_size", "voila_info_nce", "voila_info_nce_param_count",
            "voila_info_nce_grad_workspace_size", "voila_info_nce_grad", "voila_denoiser_create", "voila_denoiser_destroy",
            "voila_ddim_workspace_size", "voila_ddim_sample",
            "voila_philox_normals",
            "voila_batch_create", "voila_batch_destroy", "voila_batch_run", "voila_batch_capture",
            "voila_batch_replay", "voila_grad_param_count", "voila_rollout_grad_workspace_size",
            "voila_rollout_grad"]


def _check(st):
    if st != VOILA_OK:
        raise VoilaError(st, lib.voila_last_error().decode() or lib.voila_status_string(st).decode())


def _ptr(t):
    return None if t is None else c_void_p(t.data_ptr())


def _stream(stream):
    s = stream if stream is not None else torch.cuda.current_stream()
    return c_void_p(s.cuda_stream)


def _dev(t, dtype, shape=None, name="tensor"):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise VoilaError(VOILA_ERR_INVALID_ARG, f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise VoilaError(VOILA_ERR_INVALID_ARG, f"{name} must have dtype {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise VoilaError(VOILA_ERR_INVALID_ARG, f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise VoilaError(VOILA_ERR_INVALID_ARG, f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    return t


def version() -> int:
    return lib.voila_version()


def resample_bits(N: int) -> int:
    return lib.voila_resample_bits(int(N))


def max_update_particles() -> int:
    return lib.voila_update_max_particles()


def _mlp_desc(layers, keep):
    """_Mlp view of [(W [out, in], b [out]), ...] (arrays kept alive in `keep`)."""
    import numpy as np
    m = _Mlp()
    if not layers:
        m.n_layers = 0
        return m
    dims = [int(layers[0][0].shape[1])] + [int(W.shape[0]) for W, _ in layers]
    dims_arr = (c_int32 * len(dims))(*dims)
    Ws = [np.ascontiguousarray(np.asarray(W, np.float32)) for W, _ in layers]
    bs = [np.ascontiguousarray(np.asarray(b, np.float32)) for _, b in layers]
    W_arr = (POINTER(c_float) * len(Ws))(*[w.ctypes.data_as(POINTER(c_float)) for w in Ws])
    b_arr = (POINTER(c_float) * len(bs))(*[b.ctypes.data_as(POINTER(c_float)) for b in bs])
    keep.extend([dims_arr, Ws, bs, W_arr, b_arr])
    m.n_layers = len(layers)
    m.h_dims = dims_arr
    m.h_W = W_arr
    m.h_b = b_arr
    return m


class Denoiser:
    """Packed device copy of a v-prediction denoiser (layers [(W, b), ...]
    with input [c, a, x_tau, tau] -- conditioning input c of width d_c --
    and output v [d_x])."""

    def __init__(self, layers, d_c: int, d_x: int, n_actions: int, d_a: int = 0, compute: str = "bf16",
                 device: int = 0):
        self.d_c, self.d_x, self.n_actions, self.d_a = int(d_c), int(d_x), int(n_actions), int(d_a)
        self.compute = compute
        self.device = device
        self.handle = c_void_p()
        keep = []
        desc = _mlp_desc(layers, keep)
        _check(lib.voila_denoiser_create(ctypes.byref(desc), self.d_c, self.d_x, self.n_actions, self.d_a,
                                         {"f32": VOILA_F32, "bf16": VOILA_BF16}[compute], int(device),
                                         ctypes.byref(self.handle)))

    def close(self):
        if self.handle:
            lib.voila_denoiser_destroy(self.handle)
            self.handle = c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def ddim_sample(den: Denoiser, cond, action, x1, n_steps, out=None, workspace=None, stream=None):
    """Teacher samples [N, d_x] float32: n_steps deterministic DDIM steps of
    the denoiser from x1 [N, d_x] (the latent noise at tau = 1) conditioned
    on cond [N, d_c] and one action (index, or d_a values)."""
    N = int(cond.shape[0])
    _dev(cond, torch.float32, (N, den.d_c), "cond")
    _dev(x1, torch.float32, (N, den.d_x), "x1")
    if den.n_actions > 0:
        h_action = (c_int32 * 1)(int(action))
    else:
        vals = [float(x) for x in (action.tolist() if hasattr(action, "tolist") else action)]
        if len(vals) != den.d_a:
            raise VoilaError(VOILA_ERR_INVALID_ARG, f"continuous action must have {den.d_a} values")
        h_action = (c_float * den.d_a)(*vals)
    res = out if out is not None else torch.empty((N, den.d_x), dtype=torch.float32, device=cond.device)
    if workspace is None:
        n = lib.voila_ddim_workspace_size(den.handle, int(n_steps))
        workspace = torch.empty(max(int(n), 1), dtype=torch.uint8, device=cond.device)
    _check(lib.voila_ddim_sample(den.handle, _ptr(cond), h_action, _ptr(x1), N, int(n_steps), _ptr(workspace),
                                 workspace.numel(), _ptr(res), _stream(stream)))
    return res


class Model:
    """Packed device copy of the transition / observation / likelihood networks.

    ``desc`` has attributes d_s, n_actions, d_a, d_w, d_o, d_wz and lists
    ``trans``, ``obs``, ``lik`` of (W [out, in], b [out]) float32 arrays.
    """

    def __init__(self, desc, compute: str = "f32", device: int = 0):
        import numpy as np
        self.desc = desc
        self.compute = compute
        self.device = device
        self.handle = c_void_p()
        keep = []

        def mlp(layers):
            return _mlp_desc(layers, keep)

        d = _ModelDesc()
        d.d_s, d.n_actions, d.d_a = desc.d_s, desc.n_actions, desc.d_a
        d.d_w, d.d_o, d.d_wz = desc.d_w, desc.d_o, desc.d_wz
        d.trans, d.obs, d.lik = mlp(desc.trans), mlp(desc.obs), mlp(desc.lik)
        d.compute = {"f32": VOILA_F32, "bf16": VOILA_BF16}[compute]
        _check(lib.voila_model_create(ctypes.byref(d), int(device), ctypes.byref(self.handle)))

    def close(self):
        if self.handle:
            lib.voila_model_destroy(self.handle)
            self.handle = c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def torch_device(self):
        return torch.device("cuda", self.device)

    def plan_workspace(self, N, K, H):
        n = lib.voila_plan_workspace_size(self.handle, int(N), int(K), int(H))
        return torch.empty(max(n, 1), dtype=torch.uint8, device=self.torch_device)

    def update_workspace(self, N):
        n = lib.voila_update_workspace_size(self.handle, int(N))
        return torch.empty(max(n, 1), dtype=torch.uint8, device=self.torch_device)

    def observe_workspace(self):
        n = lib.voila_observe_workspace_size(self.handle)
        return torch.empty(max(n, 1), dtype=torch.uint8, device=self.torch_device)


def plan(model: Model, states, cands, gamma, goal, belief_w=None, seed=0, crn=False, reward_at=0, noise=None,
         return_G=False, q_out=None, G_out=None, workspace=None, status=None, stream=None, return_traj=False,
         traj_out=None):
    """Q [K] float32 (then G [K, N] if return_G, then the rollout states
    [K, N, H, d_s] if return_traj) of candidate action sequences."""
    d = model.desc
    N = int(states.shape[0])
    _dev(states, torch.float32, (N, d.d_s), "states")
    if d.n_actions > 0:
        _dev(cands, torch.int32, None, "cands")
        K, H = int(cands.shape[0]), int(cands.shape[1])
    else:
        _dev(cands, torch.float32, None, "cands")
        K, H = int(cands.shape[0]), int(cands.shape[1])
        if cands.dim() != 3 or cands.shape[2] != d.d_a:
            raise VoilaError(VOILA_ERR_INVALID_ARG, "continuous cands must be [K, H, d_a]")
    if belief_w is not None:
        _dev(belief_w, torch.float64, (N,), "belief_w")
    if noise is not None:
        _dev(noise, torch.float32, (K, N, H, d.d_w), "noise")
    goal_arr = (c_float * d.d_s)(*[float(x) for x in goal])
    traj = None
    if return_traj:
        traj = traj_out if traj_out is not None else \
            torch.empty((K, N, H, d.d_s), dtype=torch.float32, device=states.device)
        _dev(traj, torch.float32, (K, N, H, d.d_s), "traj_out")
    opts = _PlanOpts(float(gamma), goal_arr, int(seed) & (2**64 - 1), int(bool(crn)), int(reward_at),
                     _ptr(noise), _ptr(traj))
    q = q_out if q_out is not None else torch.empty(K, dtype=torch.float32, device=states.device)
    G = None
    if return_G:
        G = G_out if G_out is not None else torch.empty((K, N), dtype=torch.float32, device=states.device)
    ws = workspace if workspace is not None else model.plan_workspace(N, K, H)
    _check(lib.voila_plan(model.handle, _ptr(states), _ptr(belief_w), N, _ptr(cands), K, H, ctypes.byref(opts),
                          _ptr(ws), ws.numel(), _ptr(q), _ptr(G), _ptr(status), _stream(stream)))
    out = (q,) + ((G,) if return_G else ()) + ((traj,) if return_traj else ())
    return out if len(out) > 1 else q


def plan_observe(model: Model, traj, cands, seed=0, crn=False, noise=None, out=None, workspace=None, status=None,
                 stream=None):
    """Observations [K, N, H, d_o] drawn at every step of the rollouts whose
    states `traj` [K, N, H, d_s] plan returned (same candidates, seed, crn)."""
    d = model.desc
    if traj.dim() != 4:
        raise VoilaError(VOILA_ERR_INVALID_ARG, "traj must be [K, N, H, d_s]")
    K, N, H = int(traj.shape[0]), int(traj.shape[1]), int(traj.shape[2])
    _dev(traj, torch.float32, (K, N, H, d.d_s), "traj")
    if d.n_actions > 0:
        _dev(cands, torch.int32, (K, H), "cands")
    else:
        _dev(cands, torch.float32, (K, H, d.d_a), "cands")
    if noise is not None:
        _dev(noise, torch.float32, (K, N, H, d.d_wz), "noise")
    o = out if out is not None else torch.empty((K, N, H, d.d_o), dtype=torch.float32, device=traj.device)
    _dev(o, torch.float32, (K, N, H, d.d_o), "out")
    if workspace is None:
        n = lib.voila_plan_observe_workspace_size(model.handle, K, H)
        workspace = torch.empty(max(int(n), 1), dtype=torch.uint8, device=traj.device)
    _check(lib.voila_plan_observe(model.handle, _ptr(traj), N, _ptr(cands), K, H, int(seed) & (2**64 - 1),
                                  int(bool(crn)), _ptr(noise), _ptr(workspace), workspace.numel(), _ptr(o),
                                  _ptr(status), _stream(stream)))
    return o


def soft_value(Q, eta, log_pi0=None, want_pi=True, status=None, stream=None):
    """(V [M] float64, pi [M, K] float64 or None, best [M] int32) of
    preferences Q [M, K] float32 under a reference policy (log-probabilities
    [M, K] float64, None: uniform)."""
    if Q.dim() != 2:
        raise VoilaError(VOILA_ERR_INVALID_ARG, "Q must be [M, K]")
    M, K = int(Q.shape[0]), int(Q.shape[1])
    _dev(Q, torch.float32, (M, K), "Q")
    if log_pi0 is not None:
        _dev(log_pi0, torch.float64, (M, K), "log_pi0")
    V = torch.empty(M, dtype=torch.float64, device=Q.device)
    pi = torch.empty((M, K), dtype=torch.float64, device=Q.device) if want_pi else None
    best = torch.empty(M, dtype=torch.int32, device=Q.device)
    _check(lib.voila_soft_value(_ptr(Q), _ptr(log_pi0), M, K, float(eta), _ptr(V), _ptr(pi), _ptr(best),
                                _ptr(status), _stream(stream)))
    return V, pi, best


def info_nce(model: Model, states, actions, obs, want_scores=True, want_grad=True, out=None, workspace=None,
             status=None, stream=None):
    """Contrastive objective of the likelihood network over a mini-batch of
    B tuples: states [B, d_s] float32, actions int32 [B] or float32 [B, d_a],
    obs [B, d_o] float32.  Returns dict(loss [1] float64, row_loss [B]
    float64, scores [B, B] float32 or None, grad [B, B] float32 or None)."""
    d = model.desc
    B = int(states.shape[0])
    _dev(states, torch.float32, (B, d.d_s), "states")
    if d.n_actions > 0:
        _dev(actions, torch.int32, (B,), "actions")
    else:
        _dev(actions, torch.float32, (B, d.d_a), "actions")
    _dev(obs, torch.float32, (B, d.d_o), "obs")
    dev = states.device
    o = out if out is not None else {}
    res = {"loss": o.get("loss", torch.empty(1, dtype=torch.float64, device=dev)),
           "row_loss": o.get("row_loss", torch.empty(B, dtype=torch.float64, device=dev)),
           "scores": o.get("scores", torch.empty((B, B), dtype=torch.float32, device=dev)) if want_scores else None,
           "grad": o.get("grad", torch.empty((B, B), dtype=torch.float32, device=dev)) if want_grad else None}
    if workspace is None:
        n = lib.voila_info_nce_workspace_size(model.handle, B)
        workspace = torch.empty(max(int(n), 1), dtype=torch.uint8, device=dev)
    _check(lib.voila_info_nce(model.handle, _ptr(states), _ptr(actions), _ptr(obs), B, _ptr(workspace),
                              workspace.numel(), _ptr(res["scores"]), _ptr(res["row_loss"]), _ptr(res["grad"]),
                              _ptr(res["loss"]), _ptr(status), _stream(stream)))
    return res


def info_nce_grad(model: Model, states, actions, obs, out=None, workspace=None, status=None, stream=None):
    """Derivative of the contrastive objective with respect to the likelihood
    network's parameters (binary32 width-64 networks of the small shapes, and
    the width-256 network in binary32 or bfloat16).  Returns dict(loss [1]
    float64, grad [n_params] float32, per layer W [out, in] row-major then b)."""
    d = model.desc
    B = int(states.shape[0])
    _dev(states, torch.float32, (B, d.d_s), "states")
    if d.n_actions > 0:
        _dev(actions, torch.int32, (B,), "actions")
    else:
        _dev(actions, torch.float32, (B, d.d_a), "actions")
    _dev(obs, torch.float32, (B, d.d_o), "obs")
    n_params = int(lib.voila_info_nce_param_count(model.handle))
    if n_params == 0:
        raise VoilaError(VOILA_ERR_UNSUPPORTED, "no compiled parameter derivative for this likelihood network")
    dev = states.device
    o = out if out is not None else {}
    res = {"loss": o.get("loss", torch.empty(1, dtype=torch.float64, device=dev)),
           "grad": o.get("grad", torch.empty(n_params, dtype=torch.float32, device=dev))}
    if workspace is None:
        n = lib.voila_info_nce_grad_workspace_size(model.handle, B)
        workspace = torch.empty(max(int(n), 1), dtype=torch.uint8, device=dev)
    _check(lib.voila_info_nce_grad(model.handle, _ptr(states), _ptr(actions), _ptr(obs), B, _ptr(workspace),
                                   workspace.numel(), _ptr(res["loss"]), _ptr(res["grad"]), _ptr(status),
                                   _stream(stream)))
    return res


def plan_closed_loop(model: Model, states, first, n_obs, cont, gamma, eta, lam, goal, seed, U, log_pi0=None,
                     want_child=False, workspace=None, status=None, stream=None):
    """One-level closed-loop tree with the preference backup.  `first`:
    int32 [A] action indices or float32 [A, d_a]; `cont`: continuation
    candidates as for plan; `U` [A n_obs] int32 holds the child resampling
    offsets' 32-bit patterns.  Returns dict(psi [A], V [1], pi [A], best [1],
    R [A], V_child [A n_obs], child [A n_obs N, d_s] or None)."""
    d = model.desc
    N = int(states.shape[0])
    _dev(states, torch.float32, (N, d.d_s), "states")
    A = int(first.shape[0])
    if d.n_actions > 0:
        _dev(first, torch.int32, (A,), "first")
        _dev(cont, torch.int32, None, "cont")
    else:
        _dev(first, torch.float32, (A, d.d_a), "first")
        _dev(cont, torch.float32, None, "cont")
    K, H = int(cont.shape[0]), int(cont.shape[1])
    _dev(U, torch.int32, (A * n_obs,), "U")
    if log_pi0 is not None:
        _dev(log_pi0, torch.float64, (A,), "log_pi0")
    dev = states.device
    f64 = dict(dtype=torch.float64, device=dev)
    res = {"psi": torch.empty(A, **f64), "V": torch.empty(1, **f64), "pi": torch.empty(A, **f64),
           "best": torch.empty(1, dtype=torch.int32, device=dev), "R": torch.empty(A, **f64),
           "V_child": torch.empty(A * n_obs, **f64),
           "child": torch.empty((A * n_obs * N, d.d_s), dtype=torch.float32, device=dev) if want_child else None}
    goal_arr = (c_float * d.d_s)(*[float(x) for x in goal])
    opts = _ClosedLoopOpts(float(gamma), float(eta), float(lam), goal_arr, int(seed) & (2**64 - 1), int(n_obs),
                           _ptr(log_pi0), _ptr(U))
    if workspace is None:
        n = lib.voila_plan_closed_loop_workspace_size(model.handle, N, A, int(n_obs), K, H)
        if n == 0:
            raise VoilaError(VOILA_ERR_INVALID_ARG, "sizes out of range")
        workspace = torch.empty(int(n), dtype=torch.uint8, device=dev)
    _check(lib.voila_plan_closed_loop(model.handle, _ptr(states), N, _ptr(first), A, _ptr(cont), K, H,
                                      ctypes.byref(opts), _ptr(workspace), workspace.numel(), _ptr(res["psi"]),
                                      _ptr(res["V"]), _ptr(res["pi"]), _ptr(res["best"]), _ptr(res["R"]),
                                      _ptr(res["V_child"]), _ptr(res["child"]), _ptr(status), _stream(stream)))
    return res


def pw_step(model: Model, succ, seg, actions, visits, children, obs_table, U, k_o, alpha_o, lam=1.0, seed=0,
            out=None, workspace=None, status=None, stream=None):
    """Grouped progressive widening over M action nodes (successors
    succ[seg[m]:seg[m+1]], seg [M + 1] int32).  `children` [M] int32 and
    `obs_table` [M, capacity, d_o] float32 are updated in place; `U` [M]
    int32 holds the resampling offsets' 32-bit patterns.  Returns dict(widen,
    branch, loglik, w, stats, idx, succ)."""
    d = model.desc
    T = int(succ.shape[0])
    M = int(seg.shape[0]) - 1
    _dev(succ, torch.float32, (T, d.d_s), "succ")
    _dev(seg, torch.int32, (M + 1,), "seg")
    if d.n_actions > 0:
        _dev(actions, torch.int32, (M,), "actions")
    else:
        _dev(actions, torch.float32, (M, d.d_a), "actions")
    _dev(visits, torch.int32, (M,), "visits")
    _dev(children, torch.int32, (M,), "children")
    if obs_table.dim() != 3:
        raise VoilaError(VOILA_ERR_INVALID_ARG, "obs_table must be [M, capacity, d_o]")
    B = int(obs_table.shape[1])
    _dev(obs_table, torch.float32, (M, B, d.d_o), "obs_table")
    _dev(U, torch.int32, (M,), "U")
    dev = succ.device
    o = out if out is not None else {}
    res = {"widen": o.get("widen", torch.empty(M, dtype=torch.int32, device=dev)),
           "branch": o.get("branch", torch.empty(M, dtype=torch.int32, device=dev)),
           "loglik": o.get("loglik", torch.empty(T, dtype=torch.float32, device=dev)),
           "w": o.get("w", torch.empty(T, dtype=torch.float64, device=dev)),
           "stats": o.get("stats", torch.empty((M, 2), dtype=torch.float64, device=dev)),
           "idx": o.get("idx", torch.empty(T, dtype=torch.int32, device=dev)),
           "succ": o.get("succ", torch.empty((T, d.d_s), dtype=torch.float32, device=dev))}
    opts = _PwOpts(float(k_o), float(alpha_o), float(lam), int(seed) & (2**64 - 1), B)
    if workspace is None:
        n = lib.voila_pw_step_workspace_size(model.handle, T, M)
        workspace = torch.empty(max(int(n), 1), dtype=torch.uint8, device=dev)
    _check(lib.voila_pw_step(model.handle, _ptr(succ), T, _ptr(seg), M, _ptr(actions), _ptr(visits), _ptr(children),
                             _ptr(obs_table), _ptr(U), ctypes.byref(opts), _ptr(workspace), workspace.numel(),
                             _ptr(res["widen"]), _ptr(res["branch"]), _ptr(res["loglik"]), _ptr(res["w"]),
                             _ptr(res["stats"]), _ptr(res["idx"]), _ptr(res["succ"]), _ptr(status),
                             _stream(stream)))
    return res


def _action_dev(model, action, device):
    """The executed action as the device buffer the library reads: a CUDA
    tensor is passed through (int32 [1] index, or float32 [d_a]); a host value
    is checked and copied to a small device tensor."""
    d = model.desc
    if isinstance(action, torch.Tensor) and action.is_cuda:
        if d.n_actions > 0:
            return _dev(action.reshape(1), torch.int32, (1,), "action")
        return _dev(action.reshape(-1), torch.float32, (d.d_a,), "action")
    if d.n_actions > 0:
        a = int(action.item() if hasattr(action, "item") else action)
        if not 0 <= a < d.n_actions:
            raise VoilaError(VOILA_ERR_INVALID_ARG, "action index out of range")
        return torch.tensor([a], dtype=torch.int32, device=device)
    vals = [float(x) for x in (action.tolist() if hasattr(action, "tolist") else action)]
    if len(vals) != d.d_a:
        raise VoilaError(VOILA_ERR_INVALID_ARG, f"continuous action must have {d.d_a} values")
    if not all(math.isfinite(v) for v in vals):
        raise VoilaError(VOILA_ERR_INVALID_ARG, "non-finite action")
    return torch.tensor(vals, dtype=torch.float32, device=device)


def _obs_dev(model, obs, device):
    """The observation as a device float32 [d_o] buffer (a CUDA tensor is
    passed through; a host value is checked and copied)."""
    d = model.desc
    if isinstance(obs, torch.Tensor) and obs.is_cuda:
        return _dev(obs.reshape(-1), torch.float32, (d.d_o,), "observation")
    vals = [float(x) for x in (obs.tolist() if hasattr(obs, "tolist") else obs)]
    if len(vals) != d.d_o:
        raise VoilaError(VOILA_ERR_INVALID_ARG, f"observation must have {d.d_o} values")
    if not all(math.isfinite(v) for v in vals):
        raise VoilaError(VOILA_ERR_INVALID_ARG, "non-finite observation")
    return torch.tensor(vals, dtype=torch.float32, device=device)


def update(model: Model, states, action, obs, lam=1.0, prior_w=None, seed=0, U=0, noise=None, want_idx=True,
           want_w=True, want_loglik=True, want_prop=True, out=None, workspace=None, status=None, stream=None):
    """SIR belief update; returns dict(states, idx, w, loglik, prop, stats).
    `action` and `obs` are read on the device: CUDA tensors are passed as they
    are (no host round trip, capturable), host values are copied first."""
    d = model.desc
    N = int(states.shape[0])
    _dev(states, torch.float32, (N, d.d_s), "states")
    if prior_w is not None:
        _dev(prior_w, torch.float64, (N,), "prior_w")
    if noise is not None:
        _dev(noise, torch.float32, (N, d.d_w), "noise")
    dev = states.device
    a_dev = _action_dev(model, action, dev)
    o_dev = _obs_dev(model, obs, dev)
    if stream is not None:  # the copies of host values must outlive the call on that stream
        a_dev.record_stream(stream)
        o_dev.record_stream(stream)
    o = out if out is not None else {}
    res = {
        "states": o.get("states", torch.empty((N, d.d_s), dtype=torch.float32, device=dev)),
        "idx": o.get("idx", torch.empty(N, dtype=torch.int32, device=dev)) if want_idx else None,
        "w": o.get("w", torch.empty(N, dtype=torch.float64, device=dev)) if want_w else None,
        "loglik": o.get("loglik", torch.empty(N, dtype=torch.float32, device=dev)) if want_loglik else None,
        "prop": o.get("prop", torch.empty((N, d.d_s), dtype=torch.float32, device=dev)) if want_prop else None,
        "stats": o.get("stats", torch.empty(2, dtype=torch.float64, device=dev)),
    }
    opts = _UpdateOpts(float(lam), int(seed) & (2**64 - 1), int(U) & 0xFFFFFFFF, _ptr(noise))
    ws = workspace if workspace is not None else model.update_workspace(N)
    _check(lib.voila_update(model.handle, _ptr(states), _ptr(prior_w), N, _ptr(a_dev), _ptr(o_dev),
                            ctypes.byref(opts), _ptr(ws), ws.numel(), _ptr(res["states"]),
                            _ptr(res["idx"]), _ptr(res["w"]), _ptr(res["loglik"]), _ptr(res["prop"]),
                            _ptr(res["stats"]), _ptr(status), _stream(stream)))
    return res


def update_noalloc(model: Model, states, action, obs, lam=1.0, prior_w=None, seed=0, U=0, noise=None, out=None,
                   status=None, stream=None):
    """update() through voila_update_noalloc: the library takes the workspace
    from its fixed device scratch (no workspace argument, nothing allocated by
    the call).  `out` holds the output buffers (states, idx, w, loglik, prop,
    stats); entries left out are allocated here, by the caller's side."""
    d = model.desc
    N = int(states.shape[0])
    _dev(states, torch.float32, (N, d.d_s), "states")
    if prior_w is not None:
        _dev(prior_w, torch.float64, (N,), "prior_w")
    if noise is not None:
        _dev(noise, torch.float32, (N, d.d_w), "noise")
    dev = states.device
    a_dev = _action_dev(model, action, dev)
    o_dev = _obs_dev(model, obs, dev)
    if stream is not None:
        a_dev.record_stream(stream)
        o_dev.record_stream(stream)
    o = out if out is not None else {}
    res = {k: o[k] if k in o else None for k in ["states", "idx", "w", "loglik", "prop", "stats"]}
    if res["states"] is None:
        res["states"] = torch.empty((N, d.d_s), dtype=torch.float32, device=dev)
    opts = _UpdateOpts(float(lam), int(seed) & (2**64 - 1), int(U) & 0xFFFFFFFF, _ptr(noise))
    _check(lib.voila_update_noalloc(model.handle, _ptr(states), _ptr(prior_w), N, _ptr(a_dev), _ptr(o_dev),
                                    ctypes.byref(opts), _ptr(res["states"]), _ptr(res["idx"]), _ptr(res["w"]),
                                    _ptr(res["loglik"]), _ptr(res["prop"]), _ptr(res["stats"]), _ptr(status),
                                    _stream(stream)))
    return res


def weights_workspace(N, device):
    n = lib.voila_weights_workspace_size(int(N))
    return None if n == 0 else torch.empty(n, dtype=torch.uint8, device=device)


def normalize(loglik, lam=1.0, prior_w=None, status=None, workspace=None, stream=None):
    """(w [N] float64, stats [2] float64) of weights proportional to prior * exp(l / lam)."""
    N = int(loglik.shape[0])
    _dev(loglik, torch.float32, (N,), "loglik")
    if prior_w is not None:
        _dev(prior_w, torch.float64, (N,), "prior_w")
    w = torch.empty(N, dtype=torch.float64, device=loglik.device)
    st = torch.empty(2, dtype=torch.float64, device=loglik.device)
    ws = workspace if workspace is not None else weights_workspace(N, loglik.device)
    _check(lib.voila_normalize(_ptr(loglik), _ptr(prior_w), N, float(lam), _ptr(w), _ptr(st), _ptr(status), _ptr(ws),
                               0 if ws is None else ws.numel(), _stream(stream)))
    return w, st


def resample(w, U, src=None, status=None, workspace=None, dst=None, idx=None, stream=None):
    """Systematic resampling indices [N] int32 (and src rows gathered by them)."""
    N = int(w.shape[0])
    _dev(w, torch.float64, (N,), "w")
    idx = idx if idx is not None else torch.empty(N, dtype=torch.int32, device=w.device)
    rf = 0
    if src is not None:
        _dev(src, torch.float32, None, "src")
        if src.shape[0] != N:
            raise VoilaError(VOILA_ERR_INVALID_ARG, "src must have N rows")
        rf = int(src.numel() // N)
        dst = dst if dst is not None else torch.empty_like(src)
    ws = workspace if workspace is not None else weights_workspace(N, w.device)
    _check(lib.voila_resample(_ptr(w), N, int(U) & 0xFFFFFFFF, _ptr(idx), _ptr(src), _ptr(dst), rf, _ptr(status),
                              _ptr(ws), 0 if ws is None else ws.numel(), _stream(stream)))
    return (idx, dst) if src is not None else idx


def reweight_resample(loglik, U, lam=1.0, prior_w=None, src=None, want_w=False, status=None, workspace=None,
                      idx=None, dst=None, stats=None, stream=None):
    """Weights exp(l / lam) (x prior) normalised in binary64, then systematic
    resampling (and the gathered rows of src): dict(idx, w, stats, dst)."""
    N = int(loglik.shape[0])
    _dev(loglik, torch.float32, (N,), "loglik")
    if prior_w is not None:
        _dev(prior_w, torch.float64, (N,), "prior_w")
    d = loglik.device
    idx = idx if idx is not None else torch.empty(N, dtype=torch.int32, device=d)
    w = torch.empty(N, dtype=torch.float64, device=d) if want_w else None
    stats = stats if stats is not None else torch.empty(2, dtype=torch.float64, device=d)
    rf = 0
    if src is not None:
        _dev(src, torch.float32, None, "src")
        if src.shape[0] != N:
            raise VoilaError(VOILA_ERR_INVALID_ARG, "src must have N rows")
        rf = int(src.numel() // N)
        dst = dst if dst is not None else torch.empty_like(src)
    ws = workspace if workspace is not None else weights_workspace(N, d)
    _check(lib.voila_reweight_resample(_ptr(loglik), _ptr(prior_w), N, float(lam), int(U) & 0xFFFFFFFF, _ptr(idx),
                                       _ptr(w), _ptr(stats), _ptr(src), _ptr(dst), rf, _ptr(status), _ptr(ws),
                                       0 if ws is None else ws.numel(), _stream(stream)))
    return {"idx": idx, "w": w, "stats": stats, "dst": dst}


def observe(model: Model, states, action, seed=0, noise=None, workspace=None, out=None, status=None, stream=None):
    """o [n, d_o] float32 from the observation network (`action` as in update)."""
    d = model.desc
    n = int(states.shape[0])
    _dev(states, torch.float32, (n, d.d_s), "states")
    if noise is not None:
        _dev(noise, torch.float32, (n, d.d_wz), "noise")
    o = out if out is not None else torch.empty((n, d.d_o), dtype=torch.float32, device=states.device)
    ws = workspace if workspace is not None else model.observe_workspace()
    a_dev = _action_dev(model, action, states.device)
    if stream is not None:
        a_dev.record_stream(stream)
    _check(lib.voila_observe(model.handle, _ptr(states), n, _ptr(a_dev), int(seed) & (2**64 - 1), _ptr(noise),
                             _ptr(ws), ws.numel(), _ptr(o), _ptr(status), _stream(stream)))
    return o


def philox_normals(seed, c0, c1, c2, stream_id, n, d, device=0, stream=None):
    """(normals [n, d] float32, words [n, 4 * ceil(d / 4)] int32 view of the uint32 words)."""
    dev = torch.device("cuda", device)
    out = torch.empty((n, d), dtype=torch.float32, device=dev)
    words = torch.empty((n, 4 * ((d + 3) // 4)), dtype=torch.int32, device=dev)
    _check(lib.voila_philox_normals(int(seed) & (2**64 - 1), int(c0), int(c1), int(c2), int(stream_id), int(n),
                                    int(d), _ptr(out), _ptr(words), _stream(stream)))
    return out, words


class Batch:
    """Many planning instances (+ their belief updates) in one persistent launch.

    ``instances`` is a list of dicts with keys: model (Model), states [N, d_s],
    cands, gamma, goal, seed, and optionally belief_w, crn, reward_at,
    want_returns, and for the update: lam, update_seed.  Output tensors are
    allocated here and exposed as ``q[j]``, ``returns[j]``, ``new_states[j]``,
    ``idx[j]``, ``w[j]``, ``stats[j]``.
    """

    def __init__(self, instances, with_update=True, waves_per_block=4, blocks_per_cu=0, dynamic=True):
        self.n = len(instances)
        self.keep = []
        items = (_BatchItem * self.n)()
        self.q, self.returns, self.new_states, self.idx, self.w, self.stats = [], [], [], [], [], []
        self.models = [inst["model"] for inst in instances]
        for j, inst in enumerate(instances):
            m = inst["model"]
            d = m.desc
            S = inst["states"]
            N = int(S.shape[0])
            _dev(S, torch.float32, (N, d.d_s), f"instances[{j}].states")
            C = inst["cands"]
            _dev(C, torch.int32 if d.n_actions > 0 else torch.float32, None, f"instances[{j}].cands")
            K, H = int(C.shape[0]), int(C.shape[1])
            bw = inst.get("belief_w")
            if bw is not None:
                _dev(bw, torch.float64, (N,), f"instances[{j}].belief_w")
            dev = S.device
            q = torch.empty(K, dtype=torch.float32, device=dev)
            G = torch.empty((K, N), dtype=torch.float32, device=dev) if inst.get("want_returns") else None
            goal = (c_float * d.d_s)(*[float(x) for x in inst["goal"]])
            self.keep += [S, C, bw, goal]
            it = items[j]
            it.model, it.d_states, it.d_belief_w, it.N = m.handle, _ptr(S), _ptr(bw), N
            it.d_cands, it.K, it.H = _ptr(C), K, H
            it.gamma, it.h_goal, it.seed = float(inst["gamma"]), goal, int(inst.get("seed", 0)) & (2**64 - 1)
            it.crn, it.reward_at = int(bool(inst.get("crn", False))), int(inst.get("reward_at", 0))
            it.d_q_out, it.d_returns_out = _ptr(q), _ptr(G)
            self.q.append(q)
            self.returns.append(G)
            if with_update:
                ns = torch.empty((N, d.d_s), dtype=torch.float32, device=dev)
                ix = torch.empty(N, dtype=torch.int32, device=dev)
                ww = torch.empty(N, dtype=torch.float64, device=dev)
                st = torch.empty(2, dtype=torch.float64, device=dev)
                it.lambda_ = float(inst.get("lam", 1.0))
                it.update_seed = int(inst.get("update_seed", 0)) & (2**64 - 1)
                it.d_states_out, it.d_idx_out, it.d_w_out, it.d_stats_out = _ptr(ns), _ptr(ix), _ptr(ww), _ptr(st)
                self.new_states.append(ns)
                self.idx.append(ix)
                self.w.append(ww)
                self.stats.append(st)
        tun = _BatchTuning(int(waves_per_block), int(blocks_per_cu), int(bool(dynamic)))
        self.handle = c_void_p()
        _check(lib.voila_batch_create(items, self.n, ctypes.byref(tun), ctypes.byref(self.handle)))
        self.items = items

    def run(self, what=VOILA_BATCH_PLAN | VOILA_BATCH_UPDATE, actions=None, obs=None, resample_u=None, status=None,
            stream=None):
        _check(lib.voila_batch_run(self.handle, int(what), _ptr(actions), _ptr(obs), _ptr(resample_u), _ptr(status),
                                   _stream(stream)))

    def capture(self, what=VOILA_BATCH_PLAN | VOILA_BATCH_UPDATE, actions=None, obs=None, resample_u=None,
                status=None):
        self._graph_args = (actions, obs, resample_u, status)
        _check(lib.voila_batch_capture(self.handle, int(what), _ptr(actions), _ptr(obs), _ptr(resample_u),
                                       _ptr(status)))

    def replay(self, stream=None):
        _check(lib.voila_batch_replay(self.handle, _stream(stream)))

    def close(self):
        if self.handle:
            lib.voila_batch_destroy(self.handle)
            self.handle = c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def grad_param_count(model: Model) -> int:
    return lib.voila_grad_param_count(model.handle)


def unflatten_params(model: Model, flat):
    """[(dW [out, in], db [out]), ...] views of a flat parameter vector."""
    dims = [int(model.desc.trans[0][0].shape[1])] + [int(W.shape[0]) for W, _ in model.desc.trans]
    out, off = [], 0
    for n_in, n_out in zip(dims[:-1], dims[1:]):
        W = flat[off:off + n_out * n_in].reshape(n_out, n_in)
        off += n_out * n_in
        out.append((W, flat[off:off + n_out]))
        off += n_out
    return out


def rollout_grad(model: Model, s0, actions, H, objective, targets=None, gamma=1.0, goal=None, particles=1,
                 noise=None, seed=0, checkpoint=5, want_params=True, want_actions=False, workspace=None,
                 stream=None):
    """(objective [1], d/dparams [P] or None, d/dA (like actions) or None) through H-step rollouts."""
    d = model.desc
    B = int(s0.shape[0])
    _dev(s0, torch.float32, (B, d.d_s), "s0")
    if d.n_actions > 0:
        _dev(actions, torch.int32, (B, H), "actions")
    else:
        _dev(actions, torch.float32, (B // max(particles, 1), H, d.d_a), "actions")
    if targets is not None:
        _dev(targets, torch.float32, (B, H, d.d_s), "targets")
    if noise is not None:
        _dev(noise, torch.float32, (B, H, d.d_w), "noise")
    dev = s0.device
    loss = torch.empty(1, dtype=torch.float32, device=dev)
    gp = torch.empty(grad_param_count(model), dtype=torch.float32, device=dev) if want_params else None
    ga = torch.empty_like(actions) if want_actions else None
    goal_arr = (c_float * d.d_s)(*[float(x) for x in (goal if goal is not None else [0.0] * d.d_s)])
    o = _GradOpts(B, int(H), int(checkpoint), _ptr(s0), _ptr(actions), int(particles), _ptr(noise),
                  int(seed) & (2**64 - 1), int(objective), _ptr(targets), float(gamma), goal_arr, _ptr(loss),
                  _ptr(gp), _ptr(ga))
    n = lib.voila_rollout_grad_workspace_size(model.handle, ctypes.byref(o))
    if n == 0:
        _check(lib.voila_rollout_grad(model.handle, ctypes.byref(o), None, 0, _stream(stream)))
    ws = workspace if workspace is not None else torch.empty(n, dtype=torch.uint8, device=dev)
    _check(lib.voila_rollout_grad(model.handle, ctypes.byref(o), _ptr(ws), ws.numel(), _stream(stream)))
    return loss, gp, ga
