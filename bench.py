"""Throughput of the VOiLA planning hot path on one MI355X.

One step = plan (every candidate sequence x every belief particle x the
horizon, through the transition network) + one SIR belief update of the whole
belief, on the "realistic" synthetic workload: state dim 16, continuous
actions in [-1,1]^4, noise dim 16, observation dim 32, three hidden layers of
width 256 in every network, N = 4096 particles, K = 1024 candidates, H = 20,
gamma = 0.99, binary32 network arithmetic.  Inputs are resident on the GPU
before timing starts.

Prints one JSON line: `value` is rollout steps per second of the whole step
(K * N * H / step time); the update's particles per second, the plan-only rate,
the bfloat16 form of the same workload, the roofline of the rollout kernel
and the FP64 oracle's rate on the host cores are reported beside it.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "generator rollout steps/s + belief-update particles/s, BF16 vs FP32 at tol"
PEAK_F32_TFLOPS = 157.3
PEAK_BF16_TFLOPS = 2500.0

# rocprofv3 counters of the hot kernels, valid only for the kernel sources
# they were taken on (the commands and raw figures are under profiles/):
#   mfma_busy      SQ_VALU_MFMA_BUSY_CYCLES / (GRBM_GUI_ACTIVE per XCD x 1024 SIMDs)
#   valu_per_mfma  (SQ_INSTS_VALU - SQ_INSTS_MFMA) / SQ_INSTS_MFMA
#   valu_issue     (SQ_INSTS_VALU - SQ_INSTS_MFMA) x 4 cycles / (launch cycles at 2.4 GHz x 1024 SIMDs):
#                  the share of the SIMDs' issue time the vector instructions alone take
#   hbm_bytes      FETCH_SIZE x 2 + WRITE_SIZE per launch (the factors are what the two
#                  counters read for an elementwise kernel of 256 MiB in + 256 MiB out)
MEASURED = {
    "sources_sha256_16": "c7dd443124fe6725",
    "kernels": {
        "plan_kernel f32 realistic": {"mfma_busy": 0.890, "valu_per_mfma": 0.53, "valu_issue": 0.03,
                                      "hbm_bytes": (5627 * 2 + 1024) * 1024},
        "plan_kernel bf16 realistic": {"mfma_busy": 0.613, "valu_per_mfma": 2.69, "valu_issue": 0.17,
                                       "hbm_bytes": (4223 * 2 + 512) * 1024},
        "plan_batch_kernel bf16": {"mfma_busy": 0.511, "valu_per_mfma": 10.75, "valu_issue": 0.58,
                                   "valu_per_tile_step": 150, "mfma_per_tile_step": 14.0,
                                   "hbm_bytes": (88821 * 2 + 76897) * 1024},
        "plan_kernel bf16 width 1024": {"mfma_busy": 0.598, "valu_per_mfma": 1.47, "valu_issue": 0.10,
                                        "hbm_bytes": (9510 * 2 + 1024) * 1024},
        "plan_split_kernel bf16 4 x 1024": {"mfma_busy": 0.473, "valu_per_mfma": 1.86, "valu_issue": 0.10,
                                            "l2_hit": 0.749, "hbm_bytes": (260881759 * 2 + 164361) * 1024},
        "plan_split_kernel bf16 target finding": {"mfma_busy": 0.457, "valu_per_mfma": 1.97, "valu_issue": 0.10,
                                                  "l2_hit": 0.788, "hbm_bytes": (925838188 * 2 + 4277267) * 1024},
        "observe_kernel f32 realistic rollouts": {"mfma_busy": 0.854, "valu_per_mfma": 0.52},
        "observe_kernel bf16 realistic rollouts": {"mfma_busy": 0.431, "valu_per_mfma": 3.08},
        "observe_split_kernel bf16 4 x 1024": {"mfma_busy": 0.468, "valu_per_mfma": 1.86, "l2_hit": 0.742},
        "observe_split_kernel bf16 target finding": {"mfma_busy": 0.452, "valu_per_mfma": 1.97, "l2_hit": 0.843},
        "nce_wide_bwd_kernel f32": {"mfma_busy": 0.705, "valu_per_mfma": 0.77},
        "nce_wide_wgrad_kernel f32": {"mfma_busy": 0.548, "valu_per_mfma": 0.91},
        "nce_wide_bwd_kernel bf16": {"mfma_busy": 0.144, "valu_per_mfma": 7.23},
        "nce_wide_wgrad_kernel bf16": {"mfma_busy": 0.109, "valu_per_mfma": 12.35},
        "ddim_split_kernel 5 x 1024": {"mfma_busy": 0.476, "valu_per_mfma": 1.82},
        "ddim_split_kernel 5 x 512": {"mfma_busy": 0.437, "valu_per_mfma": 2.76},
        "ddim_split_kernel 5 x 512, 64-d latent": {"mfma_busy": 0.404, "valu_per_mfma": 3.37},
        "lg_resample_kernel 2^24": {"hbm_bytes": (541267 * 2 + 1114115) * 1024},
    },
}


# rocprofv3 figures attached to each bench section
SECTION_COUNTERS = {
    "batched": ["plan_batch_kernel bf16"],
    "wide_bf16": ["plan_kernel bf16 width 1024"],
    "deep_bf16": ["plan_split_kernel bf16 4 x 1024", "observe_split_kernel bf16 4 x 1024"],
    "target_finding_bf16": ["plan_split_kernel bf16 target finding", "observe_split_kernel bf16 target finding"],
    "plan_observe": ["observe_kernel f32 realistic rollouts", "observe_kernel bf16 realistic rollouts"],
    "info_nce": ["nce_wide_bwd_kernel f32", "nce_wide_wgrad_kernel f32", "nce_wide_bwd_kernel bf16",
                 "nce_wide_wgrad_kernel bf16"],
    "ddim": ["ddim_split_kernel 5 x 1024", "ddim_split_kernel 5 x 512", "ddim_split_kernel 5 x 512, 64-d latent"],
}


def measured(kernel):
    """The rocprofv3 figures of `kernel`, or None once the kernel sources changed."""
    if kernel_sources_hash() != MEASURED["sources_sha256_16"]:
        return None
    return MEASURED["kernels"][kernel]


def kernel_sources_hash():
    import glob
    import hashlib
    h = hashlib.sha256()
    files = sorted(glob.glob(os.path.join(ROOT, "paper_2606_19729_amd", "csrc", "*")))
    for f in files + [os.path.join(ROOT, "paper_2606_19729_amd", "build.py")]:  # sources and compiler flags
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def trans_flops_per_step(model):
    """2 * MACs of one transition-network evaluation, one-hot inputs excluded."""
    dims = [model.d_s + model.d_a + model.d_w] + [int(W.shape[0]) for W, _ in model.trans]
    return 2 * sum(a * b for a, b in zip(dims[:-1], dims[1:]))


def small_flops_per_step():
    """2 * MACs of the small transition network, one-hot inputs excluded: (4 + 4) x 64 + 64 x 64 + 64 x 4."""
    return 2 * ((4 + 4) * 64 + 64 * 64 + 64 * 4)


def bench_batched(V, torch, reps):
    """64 uneven small-network instances + their updates: bf16 persistent batch replayed
    from a hipGraph vs the plain f32 form (one voila_plan / voila_update call each)."""
    import workloads
    works = workloads.batched()
    dev = torch.device("cuda", 0)
    ev = lambda: torch.cuda.Event(enable_timing=True)  # noqa: E731
    steps = sum(w.N * w.K * w.H for w in works)
    parts = sum(w.N for w in works)
    out = {"instances": len(works), "rollout_steps": steps, "particles": parts}
    obs = torch.zeros((len(works), 2), dtype=torch.float32, device=dev)
    acts = torch.tensor([w.update_action for w in works], dtype=torch.int32, device=dev)
    us = torch.as_tensor(np.array([w.resample_u for w in works], np.uint32).view(np.int32), device=dev)
    S = [torch.as_tensor(w.states, device=dev) for w in works]
    C = [torch.as_tensor(w.cands, device=dev) for w in works]
    for form in ["bf16", "f32"]:
        models = [V.Model(w.model, compute=form) for w in works]
        insts = [dict(model=m, states=s, cands=c, gamma=w.gamma, goal=w.goal, seed=w.plan_seed, lam=w.lam,
                      update_seed=w.update_seed) for m, s, c, w in zip(models, S, C, works)]
        if form == "bf16":
            from paper_2606_19729_amd import autotune
            tuned = autotune.tune(insts, run_args=dict(actions=acts, obs=obs, resample_u=us), reps=2)
            b = V.Batch(insts, with_update=True, **tuned["schedule"])
            b.capture(actions=acts, obs=obs, resample_u=us)
            for what, key in [(V.VOILA_BATCH_PLAN | V.VOILA_BATCH_UPDATE, "plan+update")]:
                b.replay()
                torch.cuda.synchronize()
                e0, e1 = ev(), ev()
                e0.record()
                for _ in range(reps):
                    b.replay()
                e1.record()
                torch.cuda.synchronize()
                ms = e0.elapsed_time(e1) / reps
            e0, e1 = ev(), ev()
            b2 = V.Batch(insts, with_update=False, **tuned["schedule"])
            b2.run(V.VOILA_BATCH_PLAN)
            torch.cuda.synchronize()
            e0.record()
            for _ in range(reps):
                b2.run(V.VOILA_BATCH_PLAN)
            e1.record()
            torch.cuda.synchronize()
            plan_ms = e0.elapsed_time(e1) / reps
            out["bf16_persistent_graph"] = {"ms": ms, "plan_ms": plan_ms, "rollout_steps_per_s": steps / (plan_ms / 1e3),
                                            "step_rate_incl_updates": steps / (ms / 1e3),
                                            "schedule": tuned["schedule"],
                                            "mfma_frac_bf16_peak": small_flops_per_step() * steps / (plan_ms / 1e3) / 1e12
                                            / PEAK_BF16_TFLOPS}
            b.close()
            b2.close()
        else:
            ws = [m.plan_workspace(w.N, w.K, w.H) for m, w in zip(models, works)]
            q = [torch.empty(w.K, dtype=torch.float32, device=dev) for w in works]

            def plain():
                for m, s, c, w, wsp, qq in zip(models, S, C, works, ws, q):
                    V.plan(m, s, c, w.gamma, w.goal, seed=w.plan_seed, q_out=qq, workspace=wsp)
            plain()
            torch.cuda.synchronize()
            e0, e1 = ev(), ev()
            e0.record()
            for _ in range(reps):
                plain()
            e1.record()
            torch.cuda.synchronize()
            plan_ms = e0.elapsed_time(e1) / reps
            out["f32_plain"] = {"plan_ms": plan_ms, "rollout_steps_per_s": steps / (plan_ms / 1e3),
                                "mfma_frac_f32_peak": small_flops_per_step() * steps / (plan_ms / 1e3) / 1e12
                                / PEAK_F32_TFLOPS}
        for m in models:
            m.close()
    out["bf16_over_f32_rollout_rate"] = (out["bf16_persistent_graph"]["rollout_steps_per_s"]
                                         / out["f32_plain"]["rollout_steps_per_s"])
    return out


def bench_deep(V, torch, reps, paper_dims=False):
    """Four hidden layers of 1024 in bfloat16 (the depth and width of the
    paper's distilled samplers), run by the split rollout kernel: 4096
    particles x 20 steps, plan and per-step observations; with the small
    workload's dimensions (256 candidates), or with `paper_dims` the paper's
    target-finding task (45-dimensional state, six actions, 36 lidar bins,
    1024 candidates) and its belief update through the 3 x 256 likelihood."""
    import workloads
    dev = torch.device("cuda", 0)
    if paper_dims:
        w = workloads.target_finding(seed=16, N=4096, K=1024, H=20)
    else:
        w = workloads.deep(seed=8, N=4096, K=256, H=20, with_obs=True)
    mb = V.Model(w.model, compute="bf16")
    S = torch.as_tensor(w.states, device=dev)
    C = torch.as_tensor(w.cands, device=dev)
    q = torch.empty(w.K, dtype=torch.float32, device=dev)
    ws = mb.plan_workspace(w.N, w.K, w.H)
    V.plan(mb, S, C, w.gamma, w.goal, seed=w.plan_seed, q_out=q, workspace=ws)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for r in range(reps):
        V.plan(mb, S, C, w.gamma, w.goal, seed=w.plan_seed + r, q_out=q, workspace=ws)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    steps = w.K * w.N * w.H
    fps = trans_flops_per_step(w.model)
    tflops = fps * steps / (ms / 1e3) / 1e12
    # per-step observations through the observation network of the same depth
    _, traj = V.plan(mb, S, C, w.gamma, w.goal, seed=w.plan_seed, q_out=q, workspace=ws, return_traj=True)
    obs = V.plan_observe(mb, traj, C, seed=w.plan_seed)
    torch.cuda.synchronize()
    e0.record(stream)
    for r in range(reps):
        V.plan_observe(mb, traj, C, seed=w.plan_seed, out=obs)
    e1.record(stream)
    torch.cuda.synchronize()
    oms = e0.elapsed_time(e1) / reps
    # [s', w_Z] -> 1024 x 4 -> o, the one-hot action folded into the bias row
    ofl = 2 * ((w.model.d_s + w.model.d_wz) * 1024 + 3 * 1024 * 1024 + 1024 * w.model.d_o)
    dims = {"d_s": w.model.d_s, "n_actions": w.model.n_actions, "d_w": w.model.d_w, "d_o": w.model.d_o,
            "d_wz": w.model.d_wz}
    otf = ofl * steps / (oms / 1e3) / 1e12
    upd = None
    if w.model.lik:
        # the belief update with the paper's 3 x 256 likelihood: proposals
        # through the split transition kernel, likelihood of the proposals,
        # normalisation and resampling (inputs resident, one observation)
        o = torch.as_tensor((0.5 * np.random.default_rng(1).standard_normal(w.model.d_o)).astype(np.float32),
                            device=dev)
        a = torch.tensor([w.update_action], dtype=torch.int32, device=dev)
        uws = torch.empty(int(V.lib.voila_update_workspace_size(mb.handle, w.N)), dtype=torch.uint8, device=dev)
        V.update(mb, S, a, o, lam=w.lam, seed=w.update_seed, U=w.resample_u, workspace=uws)
        torch.cuda.synchronize()
        e0.record(stream)
        for r in range(reps):
            V.update(mb, S, a, o, lam=w.lam, seed=w.update_seed + r, U=w.resample_u, workspace=uws)
        e1.record(stream)
        torch.cuda.synchronize()
        ums = e0.elapsed_time(e1) / reps
        upd = {"N": w.N, "likelihood_hidden": [256] * 3, "ms": ums, "particles_per_s": w.N / (ums / 1e3)}
    mb.close()
    return {"K": w.K, "N": w.N, "H": w.H, "hidden": [1024] * 4, "dims": dims, "update": upd, "plan_ms": ms,
            "rollout_steps_per_s": steps / (ms / 1e3), "achieved_tflops": tflops,
            "mfma_frac_bf16_peak": tflops / PEAK_BF16_TFLOPS, "flop_per_rollout_step": fps,
            "observe": {"ms": oms, "observations_per_s": steps / (oms / 1e3), "flop_per_observation": ofl,
                        "achieved_tflops": otf, "mfma_frac_bf16_peak": otf / PEAK_BF16_TFLOPS}}


def bench_wide(V, torch, reps):
    """Hidden width 1024 in bfloat16: throughput at 1024 candidates x 4096
    particles x 20 steps, and plan + update latency at the small counts."""
    import workloads
    dev = torch.device("cuda", 0)
    out = {}
    w = workloads.wide(seed=3, N=4096, K=1024, H=20)
    mb = V.Model(w.model, compute="bf16")
    S = torch.as_tensor(w.states, device=dev)
    C = torch.as_tensor(w.cands, device=dev)
    q = torch.empty(w.K, dtype=torch.float32, device=dev)
    ws = mb.plan_workspace(w.N, w.K, w.H)
    V.plan(mb, S, C, w.gamma, w.goal, seed=w.plan_seed, q_out=q, workspace=ws)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for r in range(reps):
        V.plan(mb, S, C, w.gamma, w.goal, seed=w.plan_seed + r, q_out=q, workspace=ws)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    steps = w.K * w.N * w.H
    tflops = trans_flops_per_step(w.model) * steps / (ms / 1e3) / 1e12
    out["large_counts"] = {"K": w.K, "N": w.N, "H": w.H, "plan_ms": ms, "rollout_steps_per_s": steps / (ms / 1e3),
                           "achieved_tflops": tflops, "mfma_frac_bf16_peak": tflops / PEAK_BF16_TFLOPS,
                           "flop_per_rollout_step": trans_flops_per_step(w.model)}
    w = workloads.wide(seed=3)
    mb = V.Model(w.model, compute="bf16")
    S = torch.as_tensor(w.states, device=dev)
    C = torch.as_tensor(w.cands, device=dev)
    q = torch.empty(w.K, dtype=torch.float32, device=dev)
    ws = mb.plan_workspace(w.N, w.K, w.H)
    wsu = mb.update_workspace(w.N)
    obs = torch.zeros(w.model.d_o, dtype=torch.float32, device=dev)
    act = torch.tensor([w.update_action], dtype=torch.int32, device=dev)
    upd_out = {"states": torch.empty((w.N, 4), dtype=torch.float32, device=dev),
               "idx": torch.empty(w.N, dtype=torch.int32, device=dev),
               "w": torch.empty(w.N, dtype=torch.float64, device=dev),
               "loglik": torch.empty(w.N, dtype=torch.float32, device=dev),
               "prop": torch.empty((w.N, 4), dtype=torch.float32, device=dev),
               "stats": torch.empty(2, dtype=torch.float64, device=dev)}

    def once(r):
        V.plan(mb, S, C, w.gamma, w.goal, seed=r, q_out=q, workspace=ws)
        e_mid.record(stream)
        V.update(mb, S, act, obs, lam=w.lam, seed=r + 1, U=w.resample_u, out=upd_out, workspace=wsu)

    e_mid = torch.cuda.Event(enable_timing=True)
    once(0)
    torch.cuda.synchronize()
    pm, um = [], []
    for r in range(max(3, reps)):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e_mid = torch.cuda.Event(enable_timing=True)
        a.record(stream)
        once(10 + r)
        b.record(stream)
        torch.cuda.synchronize()
        pm.append(a.elapsed_time(e_mid))
        um.append(e_mid.elapsed_time(b))
    out["small_counts"] = {"K": w.K, "N": w.N, "H": w.H, "plan_ms": float(np.median(pm)),
                           "update_ms": float(np.median(um))}
    return out


def bench_small(V, torch, reps):
    """The small workload (32 candidates x 128 particles x 10 steps, one
    128-particle update), binary32: latency of plan and update."""
    import workloads
    dev = torch.device("cuda", 0)
    w = workloads.small()
    m = V.Model(w.model, compute="f32")
    S = torch.as_tensor(w.states, device=dev)
    C = torch.as_tensor(w.cands, device=dev)
    q = torch.empty(w.K, dtype=torch.float32, device=dev)
    ws = m.plan_workspace(w.N, w.K, w.H)
    wsu = m.update_workspace(w.N)
    obs = torch.zeros(w.model.d_o, dtype=torch.float32, device=dev)
    act = torch.tensor([w.update_action], dtype=torch.int32, device=dev)
    upd_out = {"states": torch.empty((w.N, w.model.d_s), dtype=torch.float32, device=dev),
               "idx": torch.empty(w.N, dtype=torch.int32, device=dev),
               "w": torch.empty(w.N, dtype=torch.float64, device=dev),
               "loglik": torch.empty(w.N, dtype=torch.float32, device=dev),
               "prop": torch.empty((w.N, w.model.d_s), dtype=torch.float32, device=dev),
               "stats": torch.empty(2, dtype=torch.float64, device=dev)}
    stream = torch.cuda.current_stream()
    pm, um = [], []
    for r in range(max(5, reps) + 1):
        a, mid, b = (torch.cuda.Event(enable_timing=True) for _ in range(3))
        a.record(stream)
        V.plan(m, S, C, w.gamma, w.goal, seed=r, q_out=q, workspace=ws)
        mid.record(stream)
        V.update(m, S, act, obs, lam=w.lam, seed=r + 1, U=w.resample_u, out=upd_out, workspace=wsu)
        b.record(stream)
        torch.cuda.synchronize()
        if r > 0:
            pm.append(a.elapsed_time(mid))
            um.append(mid.elapsed_time(b))
    return {"K": w.K, "N": w.N, "H": w.H, "plan_ms": float(np.median(pm)), "update_ms": float(np.median(um)),
            "rollout_steps_per_s": w.K * w.N * w.H / (float(np.median(pm)) / 1e3),
            "update_particles_per_s": w.N / (float(np.median(um)) / 1e3)}


def obs_flops_per_row(model):
    """2 * MACs of one observation-network evaluation at its full input width."""
    dims = [model.d_s + model.d_a + model.d_wz] + [int(W.shape[0]) for W, _ in model.obs]
    return 2 * sum(a * b for a, b in zip(dims[:-1], dims[1:]))


def bench_plan_observe(V, torch, reps, w, S, C):
    """The realistic plan with its rollout states written out (K x N x H x d_s
    floats) and an observation drawn at every rollout step (K x N x H x d_o):
    binary32 and bfloat16."""
    dev = S.device
    out = {}
    traj = torch.empty((w.K, w.N, w.H, w.model.d_s), dtype=torch.float32, device=dev)
    obs = torch.empty((w.K, w.N, w.H, w.model.d_o), dtype=torch.float32, device=dev)
    rows = w.K * w.N * w.H
    stream = torch.cuda.current_stream()
    for compute in ["f32", "bf16"]:
        m = V.Model(w.model, compute=compute)
        ws = m.plan_workspace(w.N, w.K, w.H)
        q = torch.empty(w.K, dtype=torch.float32, device=dev)
        n_ws = V.lib.voila_plan_observe_workspace_size(m.handle, w.K, w.H)
        wso = torch.empty(int(n_ws), dtype=torch.uint8, device=dev)
        pm, om = [], []
        for r in range(reps + 1):
            a, mid, b = (torch.cuda.Event(enable_timing=True) for _ in range(3))
            a.record(stream)
            V.plan(m, S, C, w.gamma, w.goal, seed=w.plan_seed + r, q_out=q, workspace=ws, return_traj=True,
                   traj_out=traj)
            mid.record(stream)
            V.plan_observe(m, traj, C, seed=w.plan_seed + r, out=obs, workspace=wso)
            b.record(stream)
            torch.cuda.synchronize()
            if r > 0:
                pm.append(a.elapsed_time(mid))
                om.append(mid.elapsed_time(b))
        p_ms, o_ms = float(np.median(pm)), float(np.median(om))
        peak = PEAK_F32_TFLOPS if compute == "f32" else PEAK_BF16_TFLOPS
        out[compute] = {"plan_with_states_ms": p_ms, "observe_ms": o_ms,
                        "observations_per_s": rows / (o_ms / 1e3),
                        "observe_mfma_frac": obs_flops_per_row(w.model) * rows / (o_ms / 1e3) / 1e12 / peak,
                        "states_GB_per_s": rows * w.model.d_s * 4 / (p_ms / 1e3) / 1e9}
        print(f"[bench]   {compute}: plan + states {p_ms:.2f} ms, observations {o_ms:.2f} ms",
              file=sys.stderr, flush=True)
    out["rows"] = rows
    out["flop_per_observation"] = obs_flops_per_row(w.model)
    return out


def bench_pw(V, torch, reps):
    """Grouped progressive widening with the realistic networks: 4,096 action
    nodes with U{1..1024} successors each (about 2.1 M successors), binary32
    and bfloat16."""
    import workloads
    dev = torch.device("cuda", 0)
    w = workloads.realistic(seed=7, N=8, K=1, H=1)
    rng = np.random.default_rng(7)
    M, B = 4096, 8
    sizes = rng.integers(1, 1025, M)
    seg = torch.as_tensor(np.concatenate([[0], np.cumsum(sizes)]).astype(np.int32), device=dev)
    T = int(sizes.sum())
    succ = torch.as_tensor(rng.standard_normal((T, w.model.d_s)).astype(np.float32), device=dev)
    actions = torch.as_tensor(rng.uniform(-1, 1, (M, w.model.d_a)).astype(np.float32), device=dev)
    children0 = rng.integers(0, B + 1, M).astype(np.int32)
    visits = torch.as_tensor((children0.astype(np.int64) ** 2 + rng.integers(-2, 3, M)).clip(0).astype(np.int32),
                             device=dev)
    table0 = torch.as_tensor(rng.standard_normal((M, B, w.model.d_o)).astype(np.float32), device=dev)
    U = torch.as_tensor(rng.integers(0, 2**31, M).astype(np.int32), device=dev)
    out = {"groups": M, "successors": T}
    stream = torch.cuda.current_stream()
    for compute in ["f32", "bf16"]:
        m = V.Model(w.model, compute=compute)
        ws = torch.empty(int(V.lib.voila_pw_step_workspace_size(m.handle, T, M)), dtype=torch.uint8, device=dev)
        res = None
        ms = []
        for r in range(reps + 1):
            ch = torch.as_tensor(children0, device=dev)
            tab = table0.clone()
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            res = V.pw_step(m, succ, seg, actions, visits, ch, tab, U, 1.0, 0.5, lam=1.0, seed=r, out=res,
                            workspace=ws)
            b.record(stream)
            torch.cuda.synchronize()
            if r > 0:
                ms.append(a.elapsed_time(b))
        t = float(np.median(ms))
        out[compute] = {"ms": t, "successors_per_s": T / (t / 1e3),
                        "widened": int(res["widen"].sum().item())}
        print(f"[bench]   {compute}: {t:.3f} ms", file=sys.stderr, flush=True)
    return out


def lik_flops(model, first_inputs):
    """2 * MACs of one likelihood-network evaluation whose first layer takes
    `first_inputs` inputs."""
    dims = [first_inputs] + [int(W.shape[0]) for W, _ in model.lik]
    return 2 * sum(a * b for a, b in zip(dims[:-1], dims[1:]))


def bench_info_nce(V, torch, reps):
    """The contrastive objective of the likelihood network with the realistic
    networks on a mini-batch of B = 4,096 tuples (16.8 M scored pairs):
    scores, row losses, mean loss and the derivative by every score, binary32
    and bfloat16."""
    import workloads
    dev = torch.device("cuda", 0)
    w = workloads.realistic(seed=8, N=4096, K=1, H=1)
    B = 4096
    S, A, O = (torch.as_tensor(x, device=dev) for x in workloads.nce_batch(w, B, seed=16))
    m0 = w.model
    pairs = B * B
    # the state and action columns are folded once per row; every pair runs
    # the rest of the network with the observation as its input
    f_pair = lik_flops(m0, m0.d_o)
    out = {"B": B, "pairs": pairs, "flop_per_pair_executed": f_pair,
           "flop_per_pair_full_input": lik_flops(m0, m0.d_s + m0.action_width + m0.d_o)}
    stream = torch.cuda.current_stream()
    for compute in ["f32", "bf16"]:
        m = V.Model(m0, compute=compute)
        ws = torch.empty(int(V.lib.voila_info_nce_workspace_size(m.handle, B)), dtype=torch.uint8, device=dev)
        res = None
        ms = []
        for r in range(reps + 1):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            res = V.info_nce(m, S, A, O, out=res, workspace=ws)
            b.record(stream)
            torch.cuda.synchronize()
            if r > 0:
                ms.append(a.elapsed_time(b))
        t = float(np.median(ms))
        peak = PEAK_F32_TFLOPS if compute == "f32" else PEAK_BF16_TFLOPS
        out[compute] = {"ms": t, "pairs_per_s": pairs / (t / 1e3),
                        "mfma_frac": f_pair * pairs / (t / 1e3) / 1e12 / peak,
                        "loss": float(res["loss"].item())}
        print(f"[bench]   {compute}: {t:.3f} ms", file=sys.stderr, flush=True)
    # the derivative with respect to the network's parameters, small binary32
    # networks (11 -> 64 -> 64 -> 1), the same B
    ws_small = workloads.small(seed=9)
    S2, A2, O2 = (torch.as_tensor(x, device=dev) for x in workloads.nce_batch(ws_small, B, seed=18))
    m2 = V.Model(ws_small.model, compute="f32")
    ws2 = torch.empty(int(V.lib.voila_info_nce_grad_workspace_size(m2.handle, B)), dtype=torch.uint8, device=dev)
    res2 = None
    ms = []
    for r in range(reps + 1):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        res2 = V.info_nce_grad(m2, S2, A2, O2, out=res2, workspace=ws2)
        b.record(stream)
        torch.cuda.synchronize()
        if r > 0:
            ms.append(a.elapsed_time(b))
    t = float(np.median(ms))
    out["small_param_grad_f32"] = {"ms": t, "pairs_per_s": pairs / (t / 1e3),
                                   "n_params": int(res2["grad"].numel())}
    print(f"[bench]   small-network parameter derivative f32: {t:.3f} ms", file=sys.stderr, flush=True)
    # the derivative for the realistic likelihood network: per pair the
    # forward pass over the observation inputs, the two transposed hidden
    # products of the reverse sweep and the weight-derivative products
    Wd = int(m0.lik[0][0].shape[0])
    d_in = m0.d_s + m0.action_width + m0.d_o
    f_grad = f_pair + 2 * 2 * Wd * Wd + 2 * (2 * Wd * Wd + Wd * d_in)
    out["realistic_param_grad"] = {"flop_per_pair": f_grad}
    for compute in ["f32", "bf16"]:
        m = V.Model(m0, compute=compute)
        wsg = torch.empty(int(V.lib.voila_info_nce_grad_workspace_size(m.handle, B)), dtype=torch.uint8, device=dev)
        res3 = None
        ms = []
        for r in range(reps + 1):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            res3 = V.info_nce_grad(m, S, A, O, out=res3, workspace=wsg)
            b.record(stream)
            torch.cuda.synchronize()
            if r > 0:
                ms.append(a.elapsed_time(b))
        t = float(np.median(ms))
        peak = PEAK_F32_TFLOPS if compute == "f32" else PEAK_BF16_TFLOPS
        out["realistic_param_grad"][compute] = {
            "ms": t, "pairs_per_s": pairs / (t / 1e3), "achieved_tflops": f_grad * pairs / (t / 1e3) / 1e12,
            "mfma_frac": f_grad * pairs / (t / 1e3) / 1e12 / peak, "n_params": int(res3["grad"].numel())}
        print(f"[bench]   realistic parameter derivative {compute}: {t:.3f} ms", file=sys.stderr, flush=True)
        del wsg
    return out


def bench_ddim(V, torch, reps):
    """The teacher samplers the generators are distilled from (bfloat16,
    65,536 samples, 50 deterministic DDIM steps): the paper's 5 x 1024
    transition denoiser, beside one evaluation of a 4 x 1024 network (the
    paper's distilled sampler shape) through the same kernel -- the
    distilled-versus-diffusion sampling-rate comparison -- and two 5 x 512
    observation denoisers: a 32-dimensional observation given a
    16-dimensional state and 4 continuous action inputs, and the paper's
    64-dimensional latent observation given the 39-dimensional state with a
    one-hot environment index (44 inputs) and one of six actions."""
    import workloads
    dev = torch.device("cuda", 0)
    N, steps = 65536, 50
    out = {"samples": N}
    stream = torch.cuda.current_stream()
    cases = [("teacher_5x1024", 4, 4, 5, 0, 1024, 5, steps, 2),
             ("distilled_4x1024", 4, 4, 5, 0, 1024, 4, 1, 2),
             ("observation_teacher_5x512", 16, 32, 0, 4, 512, 5, steps, [0.5, -1.0, 0.25, 0.0]),
             ("observation_teacher_5x512_o64", 44, 64, 6, 0, 512, 5, steps, 4)]
    for name, d_c, d_x, n_act, d_a, width, nh, n_steps, action in cases:
        C, X1 = (torch.as_tensor(x, device=dev) for x in workloads.ddim_batch(N, d_c=d_c, d_x=d_x, seed=23))
        layers = workloads.denoiser(seed=24, d_c=d_c, d_x=d_x, n_actions=n_act, d_a=d_a, width=width, n_hidden=nh)
        den = V.Denoiser(layers, d_c, d_x, n_act, d_a, compute="bf16")
        ws = torch.empty(int(V.lib.voila_ddim_workspace_size(den.handle, n_steps)), dtype=torch.uint8, device=dev)
        res = torch.empty((N, d_x), dtype=torch.float32, device=dev)
        ms = []
        for r in range(reps + 1):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            V.ddim_sample(den, C, action, X1, n_steps, out=res, workspace=ws)
            b.record(stream)
            torch.cuda.synchronize()
            if r > 0:
                ms.append(a.elapsed_time(b))
        t = float(np.median(ms))
        # executed flop per network evaluation: the first layer over the slot
        # inputs (x_tau and c; action and tau folded per step)
        dims = [d_x + d_c] + [int(W.shape[0]) for W, _ in layers]
        f_eval = 2 * sum(x * y for x, y in zip(dims[:-1], dims[1:]))
        out[name] = {"steps": n_steps, "ms": t, "samples_per_s": N / (t / 1e3), "flop_per_evaluation": f_eval,
                     "mfma_frac": f_eval * N * n_steps / (t / 1e3) / 1e12 / PEAK_BF16_TFLOPS}
        print(f"[bench]   {name}: {t:.3f} ms", file=sys.stderr, flush=True)
    out["distilled_over_teacher"] = out["distilled_4x1024"]["samples_per_s"] / out["teacher_5x1024"]["samples_per_s"]
    out["precision_note"] = ("teacher and distilled shape both in bfloat16 (binary32 accumulation); the paper "
                             "states no precision for its 283x")
    return out


def bench_tree(V, torch, reps):
    """One-level closed-loop tree with the realistic networks: 1,024 particles,
    8 continuous first actions x 4 observation branches, 128 continuation
    candidates of horizon 10 (42 M continuation rollout steps), binary32 and
    bfloat16."""
    import workloads
    dev = torch.device("cuda", 0)
    w = workloads.realistic(seed=9, N=1024, K=128, H=10)
    rng = np.random.default_rng(9)
    A, n_obs = 8, 4
    first = torch.as_tensor(rng.uniform(-1, 1, (A, 4)).astype(np.float32), device=dev)
    U = torch.as_tensor(rng.integers(0, 2**31, A * n_obs).astype(np.int32), device=dev)
    S = torch.as_tensor(w.states, device=dev)
    C = torch.as_tensor(w.cands, device=dev)
    steps = A * n_obs * w.N * w.K * w.H + A * w.N
    out = {"N": w.N, "first_actions": A, "branches": n_obs, "K": w.K, "H": w.H, "rollout_steps": steps}
    stream = torch.cuda.current_stream()
    for compute in ["f32", "bf16"]:
        m = V.Model(w.model, compute=compute)
        ws = torch.empty(int(V.lib.voila_plan_closed_loop_workspace_size(m.handle, w.N, A, n_obs, w.K, w.H)),
                         dtype=torch.uint8, device=dev)
        ms = []
        for r in range(reps + 1):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            V.plan_closed_loop(m, S, first, n_obs, C, w.gamma, 2.0, w.lam, w.goal, r, U, workspace=ws)
            b.record(stream)
            torch.cuda.synchronize()
            if r > 0:
                ms.append(a.elapsed_time(b))
        t = float(np.median(ms))
        out[compute] = {"ms": t, "rollout_steps_per_s": steps / (t / 1e3)}
        print(f"[bench]   {compute}: {t:.2f} ms", file=sys.stderr, flush=True)
    return out


def bench_gemm_reference(torch, reps):
    """Matrix-core throughput a vendor library GEMM (torch.matmul -> hipBLASLt)
    reaches on this GPU, 8192^3 in bfloat16 and binary32: the re-measured
    counterpart of the datasheet MFMA peaks the roofline fractions use."""
    dev = torch.device("cuda", 0)
    n = 8192
    out = {"n": n}
    stream = torch.cuda.current_stream()
    for name, dt in [("bf16", torch.bfloat16), ("f32", torch.float32)]:
        a = torch.randn((n, n), device=dev, dtype=dt)
        b = torch.randn((n, n), device=dev, dtype=dt)
        c = torch.matmul(a, b)
        torch.cuda.synchronize()
        ms = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            torch.matmul(a, b, out=c)
            e1.record(stream)
            torch.cuda.synchronize()
            ms.append(e0.elapsed_time(e1))
        t = float(np.median(ms))
        out[name + "_tflops"] = 2.0 * n ** 3 / (t / 1e3) / 1e12
        del a, b, c
    out["f32_allow_tf32"] = bool(torch.backends.cuda.matmul.allow_tf32)
    return out


def bench_grad(V, torch, reps):
    """Adjoint through 65,536 rollouts x 20 steps (checkpoint every 5): distillation
    gradient w.r.t. the 5,316 parameters; return gradient w.r.t. [1024, 20, 4] actions."""
    import workloads
    dev = torch.device("cuda", 0)
    rng = np.random.default_rng(5)
    B, H = 65536, 20
    out = {"rollouts": B, "H": H, "checkpoint": 5}
    w = workloads.small(seed=11)
    m = V.Model(w.model)
    S0 = torch.as_tensor(rng.standard_normal((B, 4)).astype(np.float32), device=dev)
    A = torch.as_tensor(rng.integers(0, 5, (B, H)).astype(np.int32), device=dev)
    T = torch.as_tensor(rng.standard_normal((B, H, 4)).astype(np.float32), device=dev)
    mc = V.Model(workloads.make_model(rng, d_s=4, n_actions=0, d_a=4, d_w=4, d_o=2, d_wz=2, width=64, n_hidden=2))
    Ac = torch.as_tensor(rng.uniform(-1, 1, (1024, H, 4)).astype(np.float32), device=dev)
    for key, fn in [("distill_params", lambda: V.rollout_grad(m, S0, A, H, V.VOILA_OBJ_DISTILL, targets=T, seed=3)),
                    ("return_actions", lambda: V.rollout_grad(mc, S0, Ac, H, V.VOILA_OBJ_RETURN, gamma=0.99,
                                                              goal=[1, 1, 0, 0], particles=64, seed=3,
                                                              want_params=False, want_actions=True))]:
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        out[key] = {"ms": ms, "rollout_steps_per_s": B * H / (ms / 1e3)}
    return out


def bench_update_sweep(V, torch, reps):
    """Belief-update HBM sweep: normalise given binary32 log-likelihoods, resample and
    gather 16-float particles; 136 algorithmic bytes per particle (4 B likelihood + 64 B
    particle read + 64 B particle written + 4 B index)."""
    dev = torch.device("cuda", 0)
    out = []
    for lg in (16, 20, 24):
        N = 1 << lg
        rng = np.random.default_rng(lg)
        ll = torch.as_tensor(rng.standard_normal(N).astype(np.float32), device=dev)
        src = torch.as_tensor(rng.standard_normal((N, 16)).astype(np.float32), device=dev)
        ws = V.weights_workspace(N, dev)
        dst = torch.empty_like(src)
        idx = torch.empty(N, dtype=torch.int32, device=dev)

        stats = torch.empty(2, dtype=torch.float64, device=dev)

        def once():
            V.reweight_resample(ll, 12345, src=src, workspace=ws, idx=idx, dst=dst, stats=stats)
        once()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            once()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        gbs = 136.0 * N / (ms / 1e3) / 1e9
        # a plain device copy of the particle rows, for the achievable bandwidth
        dst.copy_(src)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(reps):
            dst.copy_(src)
        e1.record()
        torch.cuda.synchronize()
        copy_gbs = 2.0 * src.numel() * 4 / (e0.elapsed_time(e1) / reps / 1e3) / 1e9
        out.append({"N": N, "ms": ms, "particles_per_s": N / (ms / 1e3), "algorithmic_GB_per_s": gbs,
                    "hbm_frac": gbs / 8000.0, "copy_GB_per_s": copy_gbs, "frac_of_copy": gbs / copy_gbs,
                    "counters": measured("lg_resample_kernel 2^24") if lg == 24 else None})
    return out


def cpu_baseline(w, n_cands):
    """The FP64 oracle on a bounded sample: n_cands candidates x all particles x H,
    plus one full belief update; rate in rollout steps per second."""
    import oracle
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    pairs = [(k, i) for k in range(n_cands) for i in range(w.N)]
    t0 = time.perf_counter()
    oracle.rollouts(w.model, w.states, w.cands, w.gamma, w.goal, pairs, seed=w.plan_seed)
    t_plan = time.perf_counter() - t0
    o = np.zeros(w.model.d_o)
    t0 = time.perf_counter()
    oracle.update(w.model, w.states, w.update_action, o, lam=w.lam, seed=w.update_seed, U=w.resample_u)
    t_upd = time.perf_counter() - t0
    steps = len(pairs) * w.H
    # the same computation on one thread, on a smaller sample (rates scale linearly)
    prev = oracle.set_threads(1)
    pairs1 = [(0, i) for i in range(min(w.N, 256))]
    t0 = time.perf_counter()
    oracle.rollouts(w.model, w.states, w.cands, w.gamma, w.goal, pairs1, seed=w.plan_seed)
    t_plan1 = time.perf_counter() - t0
    oracle.set_threads(prev)
    return {"value": steps / t_plan, "unit": "rollout steps/s", "cores": threads, "kind": "oracle",
            "sample": f"{n_cands} candidates x {w.N} particles x {w.H} steps ({steps} rollout steps) "
                      f"in {t_plan:.2f} s; one {w.N}-particle update in {t_upd:.3f} s "
                      f"({w.N / t_upd:.3g} particles/s); one thread: 1 candidate x {len(pairs1)} particles "
                      f"x {w.H} steps in {t_plan1:.2f} s",
            "update_particles_per_s": w.N / t_upd,
            "value_1thread": len(pairs1) * w.H / t_plan1}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--cpu-cands", type=int, default=12, help="candidates in the oracle's timed sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-bf16", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the batched, gradient and update-sweep measurements")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a 256 MiB read + 256 MiB write elementwise kernel (counter calibration)")
    ap.add_argument("--only", default="",
                    help="comma-separated extra sections to run (for profiling): bf16, batched, gradients, small, "
                         "wide, deep, target_finding, plan_observe, pw_step, info_nce, ddim, tree, update_sweep, gemm")
    args = ap.parse_args()
    only = set(x for x in args.only.split(",") if x)

    def want(section):
        return section in only if only else True
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported (single-GPU library and benchmark)",
              file=sys.stderr, flush=True)
        sys.exit(2)

    import torch
    import paper_2606_19729_amd as V
    import workloads

    dev = torch.device("cuda", 0)
    w = workloads.realistic()
    N, K, H = w.N, w.K, w.H
    print(f"[bench] workload realistic N={N} K={K} H={H}", file=sys.stderr, flush=True)
    m = V.Model(w.model, compute="f32")
    S = torch.as_tensor(w.states, device=dev)
    C = torch.as_tensor(w.cands, device=dev)
    q = torch.empty(K, dtype=torch.float32, device=dev)
    ws_plan = m.plan_workspace(N, K, H)
    ws_upd = m.update_workspace(N)
    obs = np.zeros(w.model.d_o, np.float32)
    upd_out = {"states": torch.empty((N, w.model.d_s), dtype=torch.float32, device=dev),
               "idx": torch.empty(N, dtype=torch.int32, device=dev),
               "w": torch.empty(N, dtype=torch.float64, device=dev),
               "loglik": torch.empty(N, dtype=torch.float32, device=dev),
               "prop": torch.empty((N, w.model.d_s), dtype=torch.float32, device=dev),
               "stats": torch.empty(2, dtype=torch.float64, device=dev)}
    # the observation of the step: the observation network applied to the
    # proposal of the workload's true particle
    V.update(m, S, w.update_action, obs, lam=w.lam, seed=w.update_seed, U=w.resample_u, out=upd_out,
             workspace=ws_upd)
    s_true = upd_out["prop"][w.true_index:w.true_index + 1].clone()
    obs = V.observe(m, s_true, w.update_action, noise=torch.as_tensor(w.obs_noise[None], device=dev))
    obs = obs[0]  # stays in device memory: the update reads it there
    act = torch.as_tensor(np.asarray(w.update_action, dtype=np.float32), device=dev)
    torch.cuda.synchronize()

    stream = torch.cuda.current_stream()
    ev = lambda: torch.cuda.Event(enable_timing=True)  # noqa: E731

    def step(seed, rec=None):
        e0, e1, e2 = (ev(), ev(), ev()) if rec is not None else (None, None, None)
        if e0: e0.record(stream)
        V.plan(m, S, C, w.gamma, w.goal, seed=seed, q_out=q, workspace=ws_plan)
        if e1: e1.record(stream)
        V.update(m, S, act, obs, lam=w.lam, seed=seed + 1, U=w.resample_u, out=upd_out, workspace=ws_upd)
        if e2: e2.record(stream)
        if rec is not None:
            rec.append((e0, e1, e2))

    for i in range(args.warmup):
        step(1000 + i)
    torch.cuda.synchronize()
    rec = []
    t0 = time.perf_counter()
    for i in range(args.steps):
        step(2000 + 2 * i, rec)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    plan_ms = float(np.mean([a.elapsed_time(b) for a, b, _ in rec]))
    upd_ms = float(np.mean([b.elapsed_time(c) for _, b, c in rec]))
    ms_per_step = wall * 1000.0 / args.steps
    steps_per_step = K * N * H
    flops = trans_flops_per_step(w.model) * steps_per_step
    achieved = flops / (plan_ms / 1000.0) / 1e12
    print(f"[bench] f32: {ms_per_step:.2f} ms/step, plan {plan_ms:.2f} ms, update {upd_ms:.3f} ms",
          file=sys.stderr, flush=True)

    result = {
        "metric": METRIC,
        "value": steps_per_step / (ms_per_step / 1000.0),
        "unit": "rollout steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "realistic: d_s=16, continuous d_a=4, d_w=16, d_o=32, three hidden layers "
                               "of 256 (ReLU) per network, N=4096, K=1024, H=20, gamma=0.99; plan + one "
                               "belief update per step", "N": N, "K": K, "H": H},
        "plan_steps_per_s": steps_per_step / (plan_ms / 1000.0),
        "plan_ms": plan_ms,
        "update_ms": upd_ms,
        "update_particles_per_s": N / (upd_ms / 1000.0),
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": PEAK_F32_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_F32_TFLOPS,
                     "traffic": (measured("plan_kernel f32 realistic") or {}).get("hbm_bytes"),
                     "counters": measured("plan_kernel f32 realistic"),
                     "kernel": "plan_kernel (f32, realistic)",
                     "flop_per_rollout_step": trans_flops_per_step(w.model),
                     "rollout_steps_per_launch": steps_per_step},
    }

    if not args.no_bf16 and want("bf16"):
        mb = V.Model(w.model, compute="bf16")
        wsb = mb.plan_workspace(N, K, H)
        qb = torch.empty(K, dtype=torch.float32, device=dev)
        for i in range(args.warmup):
            V.plan(mb, S, C, w.gamma, w.goal, seed=w.plan_seed, q_out=qb, workspace=wsb)
        torch.cuda.synchronize()
        e0, e1 = ev(), ev()
        e0.record(stream)
        for i in range(args.steps):
            V.plan(mb, S, C, w.gamma, w.goal, seed=w.plan_seed, q_out=qb, workspace=wsb)
        e1.record(stream)
        torch.cuda.synchronize()
        bms = e0.elapsed_time(e1) / args.steps
        # accuracy of the bf16 form against the binary32 form on the same noise
        V.plan(m, S, C, w.gamma, w.goal, seed=w.plan_seed, q_out=q, workspace=ws_plan)
        torch.cuda.synchronize()
        qf, qbh = q.cpu().numpy().astype(np.float64), qb.cpu().numpy().astype(np.float64)
        result["bf16"] = {"plan_steps_per_s": steps_per_step / (bms / 1000.0), "plan_ms": bms,
                          "speedup_vs_f32_plan": plan_ms / bms,
                          "max_rel_q_diff_vs_f32": float(np.max(np.abs(qbh - qf) / np.abs(qf))),
                          "roofline_frac_bf16_peak": flops / (bms / 1000.0) / 1e12 / PEAK_BF16_TFLOPS,
                          "counters": measured("plan_kernel bf16 realistic")}
        print(f"[bench] bf16 plan {bms:.2f} ms", file=sys.stderr, flush=True)

    sections = [
        ("batched", "batched instances (bf16 persistent graph vs f32 plain)", "batched",
         lambda: bench_batched(V, torch, max(2, args.steps // 2))),
        ("gradients", "adjoint rollouts", "gradients", lambda: bench_grad(V, torch, max(2, args.steps))),
        ("small", "small workload latency", "small_f32", lambda: bench_small(V, torch, args.steps)),
        ("wide", "hidden width 1024 (bf16)", "wide_bf16", lambda: bench_wide(V, torch, max(2, args.steps // 2))),
        ("deep", "four hidden layers of 1024 (bf16, split rollout kernel)", "deep_bf16",
         lambda: bench_deep(V, torch, max(2, args.steps // 2))),
        ("target_finding", "the paper's target-finding shapes (45-d state, 36 lidar bins; 4 x 1024 bf16)",
         "target_finding_bf16", lambda: bench_deep(V, torch, max(2, args.steps // 2), paper_dims=True)),
        ("plan_observe", "rollout states and per-step observations", "plan_observe",
         lambda: bench_plan_observe(V, torch, max(2, args.steps // 2), w, S, C)),
        ("pw_step", "grouped progressive widening", "pw_step", lambda: bench_pw(V, torch, max(3, args.steps))),
        ("info_nce", "contrastive likelihood objective", "info_nce",
         lambda: bench_info_nce(V, torch, max(3, args.steps))),
        ("ddim", "DDIM teacher sampler vs one distilled-sampler evaluation", "ddim",
         lambda: bench_ddim(V, torch, max(2, args.steps // 2))),
        ("tree", "one-level closed-loop tree", "closed_loop_tree", lambda: bench_tree(V, torch, max(2, args.steps // 2))),
        ("update_sweep", "belief-update sweep", "update_sweep",
         lambda: bench_update_sweep(V, torch, max(3, args.steps))),
    ]
    if not args.no_extras:
        for name, title, key, fn in sections:
            if want(name):
                print(f"[bench] {title}", file=sys.stderr, flush=True)
                result[key] = fn()
                for sect, kernels in SECTION_COUNTERS.items():
                    if sect == key and isinstance(result[key], dict):
                        result[key]["counters"] = {k: measured(k) for k in kernels}

    if not args.no_extras and want("gemm"):
        print("[bench] library GEMM reference (matrix-core peak re-measured)", file=sys.stderr, flush=True)
        result["gemm_reference"] = bench_gemm_reference(torch, 5)
        g = result["gemm_reference"]
        result["roofline"]["frac_of_library_f32_gemm"] = result["roofline"]["achieved"] / g["f32_tflops"]

    if args.calibrate_copy:
        x = torch.ones(64 << 20, dtype=torch.float32, device=dev)
        y = torch.empty_like(x)
        torch.mul(x, 1.0, out=y)
        torch.cuda.synchronize()
        result["calibration"] = {"kernel": "elementwise mul (torch)", "read_bytes": x.numel() * 4,
                                 "write_bytes": y.numel() * 4}

    if not args.no_cpu_baseline:
        print("[bench] timing the FP64 oracle on the host", file=sys.stderr, flush=True)
        result["cpu_baseline"] = cpu_baseline(w, args.cpu_cands)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
