// plan_unit.hpp -- the rollout kernel's per-unit evaluation (one or two
// 32-particle tiles of one candidate over the horizon) and plan_kernel
// itself; included by k_plan.hip and by k_plan_bf16.hip, which compiles the
// bfloat16 instances with the matrix instructions' accumulators in VGPRs.
#pragma once
#include "kcommon.hpp"

namespace voila {

// One (candidate, 32-particle) tile of one planning instance: H steps of the
// transition network with the states in registers, then the tile's returns
// and their (weighted) sum.  `unit_ok` false runs a masked dummy tile (the
// caller's loop is block-uniform) that writes nothing.
template <int DT, int D_S, int N_ACT, int D_A, int D_W, int WIDTH, int NHID, class Src>
__device__ __forceinline__ void plan_unit(Src& src, const NetPtrs& P, const PlanParams& p, const float* goal_src,
                                          long u, bool unit_ok, int lane, int g, int col) {
    constexpr int SS = state_slots(D_S), SA = action_slots(D_A), SW = noise_slots(D_W);
    typedef Net<DT, WIDTH, NHID, in_slots(DT, D_S, D_A, D_W)> NT;
    // the unit (candidate, tile) is uniform over the wave: its candidate's
    // actions are read with scalar loads, which leaves the vector-memory
    // counter to the weight stream
    const int uw = __builtin_amdgcn_readfirstlane(unit_ok ? (int)u : 0);
    const int k = uw / p.n_tiles;
    const int tile = uw - k * p.n_tiles;
    const int i = tile * 32 + col;
    const bool valid = unit_ok && i < p.N;
    float st[SS], goal[SS];
#pragma unroll
    for (int s = 0; s < SS; ++s) {
        int f = 2 * s + g;
        st[s] = (valid && f < D_S) ? p.states[(size_t)i * D_S + f] : 0.0f;
        goal[s] = f < D_S ? goal_src[f] : 0.0f;
    }
    // complete these loads here, once per unit, so that no wait for them (and
    // with them for the weight stream's loads in flight) lands in the step loop
    __builtin_amdgcn_s_waitcnt(waitcnt_vm_lgkm0(0));
    float G = 0.0f;
    double disc = 1.0;
    uint32_t wnow[SW], wnext[SW];  // Philox words of this step's and the next step's noise slots
    for (int t = 0; t < p.H; ++t) {
        float slots[NT::IN_SLOTS];
#pragma unroll
        for (int s = 0; s < NT::IN_SLOTS; ++s) slots[s] = 0.0f;
#pragma unroll
        for (int s = 0; s < SS; ++s) slots[s] = st[s];
        if (D_A > 0) {
            const kconst float* a = (const kconst float*)p.cands + ((size_t)k * p.H + t) * D_A;
#pragma unroll
            for (int s = 0; s < SA; ++s) {
                const float a0 = 2 * s < D_A ? a[2 * s] : 0.0f;
                const float a1 = 2 * s + 1 < D_A ? a[2 * s + 1] : 0.0f;
                slots[SS + s] = g ? a1 : a0;
            }
        }
        if (p.noise) {
            const float* nsrc = p.noise + (((size_t)k * p.N + (valid ? i : 0)) * p.H + t) * D_W;
#pragma unroll
            for (int s = 0; s < SW; ++s) {
                int f = noise_feature(s, g);
                slots[SS + SA + s] = f < D_W ? nsrc[f] : 0.0f;
            }
            // wait on this path only (the merged path would wait on every step)
            __builtin_amdgcn_s_waitcnt(waitcnt_vm_lgkm0(0));
        } else {
            // steps come in pairs: the words of both are drawn at the even step
            if ((t & 1) == 0) {
                philox_two_steps<SW>(wnow, wnext, p.key0, p.key1, (uint32_t)i, p.crn ? 0u : (uint32_t)k,
                                     (uint32_t)t, 3u, g);
            } else {
#pragma unroll
                for (int s = 0; s < SW; ++s) wnow[s] = wnext[s];
            }
            float nz[SW];
            noise_from_words<SW>(nz, wnow);
#pragma unroll
            for (int s = 0; s < SW; ++s) slots[SS + SA + s] = nz[s];
        }
        const float* b0 = P.b0;
        if (N_ACT > 0) {
            int a = ((const kconst int32_t*)p.cands)[(size_t)k * p.H + t];
            if (a < 0 || a >= N_ACT) {
                if (p.status && lane == 0 && unit_ok) p.status[0] = 1;
                a = 0;
            }
            b0 += (size_t)a * p.net.b0_stride;
        }
        float r_cur = 0.0f;
        if (p.reward_at) r_cur = reward_to(st, goal, SS, D_S, g);
        f32x16 out = run_net<NT>(src, P, b0, slots, lane, g);
#pragma unroll
        for (int s = 0; s < SS; ++s) st[s] += out[s];
        if (p.traj && valid) {
            float* dst = p.traj + (((size_t)k * p.N + i) * p.H + t) * D_S;
#pragma unroll
            for (int s = 0; s < SS; ++s)
                if (2 * s + g < D_S) dst[2 * s + g] = st[s];
        }
        float r = p.reward_at ? r_cur : reward_to(st, goal, SS, D_S, g);
        G = __builtin_fmaf((float)disc, r, G);
        disc *= p.gamma;
    }
    if (p.returns && g == 0 && valid) p.returns[(size_t)k * p.N + i] = G;
    float contrib = valid ? (p.belief_w ? (float)p.belief_w[i] * G : G) : 0.0f;
    float tot = sum32(contrib);
    if (lane == 0 && unit_ok) p.partials[(size_t)k * p.n_tiles + tile] = tot;
}

constexpr size_t kPlanStreamLds = (size_t)VOILA_STREAM_NBUF * VOILA_PLAN_STREAM_CHB;  // output tiles per pass of the paired evaluation

// The unit of plan_unit for two tiles (2 tp, 2 tp + 1) of one candidate:
// every weight fragment feeds both tiles' products.
template <int DT, int D_S, int N_ACT, int D_A, int D_W, int WIDTH, int NHID, class Src>
__device__ __forceinline__ void plan_unit_pair(Src& src, const NetPtrs& P, const PlanParams& p, long u, bool unit_ok,
                                               int lane, int g, int col) {
    constexpr int SS = state_slots(D_S), SA = action_slots(D_A), SW = noise_slots(D_W);
    constexpr int ST = 2;
    typedef Net<DT, WIDTH, NHID, in_slots(DT, D_S, D_A, D_W)> NT;
    const int n_pairs = (p.n_tiles + 1) / 2;
    const int uw = __builtin_amdgcn_readfirstlane(unit_ok ? (int)u : 0);
    const int k = uw / n_pairs;
    const int tp = uw - k * n_pairs;
    int i[ST];
    bool valid[ST];
    float st[ST][SS], goal[SS];
#pragma unroll
    for (int q = 0; q < ST; ++q) {
        i[q] = (2 * tp + q) * 32 + col;
        valid[q] = unit_ok && i[q] < p.N;
    }
#pragma unroll
    for (int s = 0; s < SS; ++s) {
        const int f = 2 * s + g;
        goal[s] = f < D_S ? p.goal[f] : 0.0f;
#pragma unroll
        for (int q = 0; q < ST; ++q) st[q][s] = (valid[q] && f < D_S) ? p.states[(size_t)i[q] * D_S + f] : 0.0f;
    }
    __builtin_amdgcn_s_waitcnt(waitcnt_vm_lgkm0(0));
    float G[ST] = {0.0f, 0.0f};
    double disc = 1.0;
    uint32_t wnow[ST][SW], wnext[ST][SW];
    for (int t = 0; t < p.H; ++t) {
        float slots[ST][NT::IN_SLOTS];
#pragma unroll
        for (int q = 0; q < ST; ++q) {
#pragma unroll
            for (int s = 0; s < NT::IN_SLOTS; ++s) slots[q][s] = 0.0f;
#pragma unroll
            for (int s = 0; s < SS; ++s) slots[q][s] = st[q][s];
        }
        if (D_A > 0) {
            const kconst float* a = (const kconst float*)p.cands + ((size_t)k * p.H + t) * D_A;
#pragma unroll
            for (int s = 0; s < SA; ++s) {
                const float a0 = 2 * s < D_A ? a[2 * s] : 0.0f;
                const float a1 = 2 * s + 1 < D_A ? a[2 * s + 1] : 0.0f;
#pragma unroll
                for (int q = 0; q < ST; ++q) slots[q][SS + s] = g ? a1 : a0;
            }
        }
        if (p.noise) {
#pragma unroll
            for (int q = 0; q < ST; ++q) {
                const float* nsrc = p.noise + (((size_t)k * p.N + (valid[q] ? i[q] : 0)) * p.H + t) * D_W;
#pragma unroll
                for (int s = 0; s < SW; ++s) {
                    const int f = noise_feature(s, g);
                    slots[q][SS + SA + s] = f < D_W ? nsrc[f] : 0.0f;
                }
            }
            __builtin_amdgcn_s_waitcnt(waitcnt_vm_lgkm0(0));
        } else {
#pragma unroll
            for (int q = 0; q < ST; ++q) {
                if ((t & 1) == 0) {
                    philox_two_steps<SW>(wnow[q], wnext[q], p.key0, p.key1, (uint32_t)i[q], p.crn ? 0u : (uint32_t)k,
                                         (uint32_t)t, 3u, g);
                } else {
#pragma unroll
                    for (int s = 0; s < SW; ++s) wnow[q][s] = wnext[q][s];
                }
                float nz[SW];
                noise_from_words<SW>(nz, wnow[q]);
#pragma unroll
                for (int s = 0; s < SW; ++s) slots[q][SS + SA + s] = nz[s];
            }
        }
        const float* b0 = P.b0;
        if (N_ACT > 0) {
            int a = ((const kconst int32_t*)p.cands)[(size_t)k * p.H + t];
            if (a < 0 || a >= N_ACT) {
                if (p.status && lane == 0 && unit_ok) p.status[0] = 1;
                a = 0;
            }
            b0 += (size_t)a * p.net.b0_stride;
        }
        float r_cur[ST] = {0.0f, 0.0f};
        if (p.reward_at)
#pragma unroll
            for (int q = 0; q < ST; ++q) r_cur[q] = reward_to(st[q], goal, SS, D_S, g);
        f32x16 out[ST];
#if VOILA_PLAN_FLAT
        run_net_flat<NT, ST, kPlanPassTiles>(src, P, b0, slots, out, lane, g);
#else
        run_net_passes<NT, ST, kPlanPassTiles>(src, P, b0, slots, out, lane, g);
#endif
#pragma unroll
        for (int q = 0; q < ST; ++q) {
#pragma unroll
            for (int s = 0; s < SS; ++s) st[q][s] += out[q][s];
            if (p.traj && valid[q]) {
                float* dst = p.traj + (((size_t)k * p.N + i[q]) * p.H + t) * D_S;
#pragma unroll
                for (int s = 0; s < SS; ++s)
                    if (2 * s + g < D_S) dst[2 * s + g] = st[q][s];
            }
            const float r = p.reward_at ? r_cur[q] : reward_to(st[q], goal, SS, D_S, g);
            G[q] = __builtin_fmaf((float)disc, r, G[q]);
        }
        disc *= p.gamma;
    }
#pragma unroll
    for (int q = 0; q < ST; ++q) {
        if (p.returns && g == 0 && valid[q]) p.returns[(size_t)k * p.N + i[q]] = G[q];
        const float contrib = valid[q] ? (p.belief_w ? (float)p.belief_w[i[q]] * G[q] : G[q]) : 0.0f;
        const float tot = sum32(contrib);
        const int tile = 2 * tp + q;
        if (lane == 0 && unit_ok && tile < p.n_tiles) p.partials[(size_t)k * p.n_tiles + tile] = tot;
    }
}

template <int DT, int D_S, int N_ACT, int D_A, int D_W, int WIDTH, int NHID, int MODE>
__global__ __launch_bounds__(256) void plan_kernel(PlanParams p) {
    if constexpr (!generic_compiled(DT, WIDTH, NHID)) {
        return;  // refused at model creation (binary32 wider than 256) or run by the split rollout kernel
    } else {
    typedef Net<DT, WIDTH, NHID, in_slots(DT, D_S, D_A, D_W)> NT;
    extern __shared__ __attribute__((aligned(16))) char smem[];
    const int lane = threadIdx.x & 63, g = lane >> 5, col = lane & 31;
    const int wpb = blockDim.x >> 6, wave = threadIdx.x >> 6;
    constexpr bool PAIRS = plan_pairs<DT, WIDTH, NHID>();
    const long n_units = (long)p.K * (PAIRS ? (p.n_tiles + 1) / 2 : p.n_tiles);
    with_weights<NT, MODE, (N_ACT > 0 ? N_ACT : 1), VOILA_PLAN_STREAM_CHB>(smem, p.net, [&](auto& src, const NetPtrs& P) {
        // block-uniform loop: every wave of a block walks the same sequence of
        // (unit, step) iterations, idle waves on a masked dummy unit
        for (long ub = blockIdx.x; ub * wpb < n_units; ub += gridDim.x) {
            const long u = ub * wpb + wave;
            if constexpr (PAIRS)
                plan_unit_pair<DT, D_S, N_ACT, D_A, D_W, WIDTH, NHID>(src, P, p, u, u < n_units, lane, g, col);
            else
                plan_unit<DT, D_S, N_ACT, D_A, D_W, WIDTH, NHID>(src, P, p, p.goal, u, u < n_units, lane, g, col);
        }
    });
    }
}

}  // namespace voila
