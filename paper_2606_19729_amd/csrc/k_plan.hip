// k_plan.hip -- the persistent rollout kernel (plan), its batched form and
// the fixed-order Q reduction.
//
// plan_kernel     each wave owns a (candidate, 32-particle) tile, keeps the 32
//                 states in registers for the whole horizon and runs every
//                 transition-network layer on the matrix cores (transposed
//                 evaluation, see device.hpp), with the noise drawn in registers
//                 from Philox.  Small networks are staged in LDS once per block;
//                 wide ones stream their fragments from L2.
// q_reduce_kernel fixed-order sum of the per-tile partial returns into Q.
#include "plan_unit.hpp"

namespace voila {

// Deep wide transition networks (more than two hidden layers wider than 256,
// the depth of the paper's distilled samplers): a block of kPlanSplitWaves
// waves advances kPlanSplitTiles 32-particle tiles of one candidate together,
// each layer split over the waves (run_net_split_owned), so that every
// weight fragment read from L2 serves all of the block's tiles.  Wave q
// carries tile q's states, noise and return, stages the tile's first-layer
// operands in LDS each step and receives the tile's output; the other waves
// hold no per-particle state.  The per-tile partial returns are those of
// plan_kernel.
#ifndef VOILA_PLAN_SPLIT_WAVES
#define VOILA_PLAN_SPLIT_WAVES 8
#endif
#ifndef VOILA_PLAN_SPLIT_TILES
#define VOILA_PLAN_SPLIT_TILES 2
#endif
#ifndef VOILA_PLAN_SPLIT_DEPTH
#define VOILA_PLAN_SPLIT_DEPTH 2
#endif
constexpr int kPlanSplitWaves = VOILA_PLAN_SPLIT_WAVES, kPlanSplitTiles = VOILA_PLAN_SPLIT_TILES,
              kPlanSplitDepth = VOILA_PLAN_SPLIT_DEPTH;

template <int DT, int WIDTH, int NHID>
constexpr bool plan_split() {
    return net_compiled(DT, WIDTH) && !generic_compiled(DT, WIDTH, NHID);
}

// LDS of the split rollout kernel beyond the activations: each owner wave's
// first-layer operands and states ([slot][lane]), then the goal.
template <class NT, int D_S>
struct PlanSplitLds {
    static constexpr int IN = kPlanSplitTiles * SplitIn<NT>::BYTES;
    static constexpr int STATE = kPlanSplitTiles * state_slots(D_S) * 64 * 4;
    static constexpr int BYTES = kPlanSplitTiles * SplitLds<NT>::ACT + IN + STATE + 64 * 4;
};

template <int DT, int D_S, int N_ACT, int D_A, int D_W, int WIDTH, int NHID>
__global__ __launch_bounds__(64 * kPlanSplitWaves) void plan_split_kernel(PlanParams p) {
    if constexpr (!plan_split<DT, WIDTH, NHID>()) {
        return;  // the other networks run in plan_kernel
    } else {
    constexpr int ST = kPlanSplitTiles;
    constexpr int SS = state_slots(D_S), SA = action_slots(D_A), SW = noise_slots(D_W);
    // states wider than 32 come out of the network in two 32-row tiles: state
    // slot s is register s % 16 of output tile s / 16
    constexpr int NO = cdiv(D_S, 32);
    typedef Net<DT, WIDTH, NHID, in_slots(DT, D_S, D_A, D_W), WIDTH / 32, NO> NT;
    typedef PlanSplitLds<NT, D_S> L;
    extern __shared__ __attribute__((aligned(16))) char smem[];
    char* const in_lds = smem + ST * SplitLds<NT>::ACT;
    const int lane = threadIdx.x & 63, g = lane >> 5, col = lane & 31;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    // wave q < ST owns sample tile q of every group: its states (kept in LDS
    // across the network, which needs every register), noise and return; the
    // other waves only evaluate the network
    const bool owner = wave < ST;
    float* const st_lds = reinterpret_cast<float*>(in_lds + L::IN) + (owner ? wave : 0) * SS * 64 + lane;
    float* const goal_lds = reinterpret_cast<float*>(in_lds + L::IN + L::STATE);
    if (threadIdx.x < 64) goal_lds[threadIdx.x] = p.goal[threadIdx.x];
    __syncthreads();
    auto goal_at = [&](int s) { return goal_lds[2 * s + g]; };
    // -|s - goal|^2 over this lane's state slots (both lane groups summed)
    auto reward = [&](const float (&x)[SS]) {
        float part = 0.0f;
#pragma unroll
        for (int s = 0; s < SS; ++s)
            if (2 * s + g < D_S) {
                const float e = x[s] - goal_at(s);
                part = __builtin_fmaf(e, e, part);
            }
        return -(part + __shfl_xor(part, 32));
    };
    const int n_groups = (p.n_tiles + ST - 1) / ST;
    const long n_units = (long)p.K * n_groups;
    const NetPtrs P = net_ptrs(p.net.base, p.net);
    for (long u = blockIdx.x; u < n_units; u += gridDim.x) {
        const int k = (int)(u / n_groups);
        const int grp = (int)(u - (long)k * n_groups);
        const int tile = grp * ST + (owner ? wave : 0);
        const int i = tile * 32 + col;
        const bool valid = owner && i < p.N;
        if (owner) {
            float st[SS];
#pragma unroll
            for (int s = 0; s < SS; ++s) {
                const int f = 2 * s + g;
                st[s] = (valid && f < D_S) ? p.states[(size_t)i * D_S + f] : 0.0f;
            }
#pragma unroll
            for (int s = 0; s < SS; ++s) st_lds[s * 64] = st[s];
        }
        float G = 0.0f;
        double disc = 1.0;
        for (int t = 0; t < p.H; ++t) {
            float r_cur = 0.0f;
            if (owner) {
                float slots[NT::IN_SLOTS], st[SS];
#pragma unroll
                for (int s = 0; s < SS; ++s) st[s] = st_lds[s * 64];
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
                        const int f = noise_feature(s, g);
                        slots[SS + SA + s] = f < D_W ? nsrc[f] : 0.0f;
                    }
                } else {
                    // this step's words only: nothing of the noise lives across the network
                    float nz[SW];
                    noise_slots_philox<SW>(nz, p.key0, p.key1, (uint32_t)i, p.crn ? 0u : (uint32_t)k, (uint32_t)t,
                                           3u, g);
#pragma unroll
                    for (int s = 0; s < SW; ++s) slots[SS + SA + s] = nz[s];
                }
                if (p.reward_at) r_cur = reward(st);
                split_stage_inputs<NT>(in_lds + wave * SplitIn<NT>::BYTES, slots, lane);
            }
            const float* b0 = P.b0;
            if (N_ACT > 0) {
                int a = ((const kconst int32_t*)p.cands)[(size_t)k * p.H + t];
                if (a < 0 || a >= N_ACT) {
                    if (p.status && wave == 0 && lane == 0) p.status[0] = 1;
                    a = 0;
                }
                b0 += (size_t)a * p.net.b0_stride;
            }
            __syncthreads();  // the owners' inputs are in LDS
            float out[NO][16];
            run_net_split_owned<NT, ST, kPlanSplitWaves, kPlanSplitDepth>(P, b0, in_lds, out, lane, g, wave, smem);
            if (owner) {
                float st[SS];
#pragma unroll
                for (int s = 0; s < SS; ++s) st[s] = st_lds[s * 64] + out[s / 16][s % 16];
#pragma unroll
                for (int s = 0; s < SS; ++s) st_lds[s * 64] = st[s];
                if (p.traj && valid) {
                    float* dst = p.traj + (((size_t)k * p.N + i) * p.H + t) * D_S;
#pragma unroll
                    for (int s = 0; s < SS; ++s)
                        if (2 * s + g < D_S) dst[2 * s + g] = st[s];
                }
                const float r = p.reward_at ? r_cur : reward(st);
                G = __builtin_fmaf((float)disc, r, G);
            }
            disc *= p.gamma;
        }
        if (owner) {
            if (p.returns && g == 0 && valid) p.returns[(size_t)k * p.N + i] = G;
            const float contrib = valid ? (p.belief_w ? (float)p.belief_w[i] * G : G) : 0.0f;
            const float tot = sum32(contrib);
            if (lane == 0 && tile < p.n_tiles) p.partials[(size_t)k * p.n_tiles + tile] = tot;
        }
    }
    }
}

// Many planning instances of one network shape in one persistent launch.
// The work list holds block items (instance, first tile unit, number of
// units): a block takes items from a queue (atomic counter, list sorted by
// decreasing cost) or in a static stride, restages the instance's network in
// LDS when the instance changes, and runs one unit per wave.  At most 128
// registers per lane (four waves per SIMD): a small network's step
// alternates between matrix products and the vector work that feeds them
// (noise, ReLU, conversions), and the other waves fill each wave's gaps.
template <int DT, int D_S, int N_ACT, int D_A, int D_W, int WIDTH, int NHID>
__global__ __launch_bounds__(512, 4) void plan_batch_kernel(BatchPlanParams bp) {
    if constexpr (WIDTH > 64) {
        return;  // batches need networks that fit in LDS (the launcher refuses wider ones)
    } else {
    typedef Net<DT, WIDTH, NHID, in_slots(DT, D_S, D_A, D_W)> NT;
    extern __shared__ __attribute__((aligned(16))) char smem[];
    __shared__ int s_item;
    const int lane = threadIdx.x & 63, g = lane >> 5, col = lane & 31;
    const int wave = threadIdx.x >> 6;
    int loaded = -1;
    int item = blockIdx.x;
    for (int iter = 0;; ++iter) {
        if (bp.dynamic) {
            if (threadIdx.x == 0) s_item = atomicAdd(bp.counter, 1);
            __syncthreads();
            item = s_item;
            __syncthreads();
        } else if (iter > 0) {
            item += gridDim.x;
        }
        if (item >= bp.n_items) break;
        const int4 it = bp.items[item];  // (instance, first unit, units, cost)
        PlanParams p = bp.insts[it.x];
        p.status = bp.status;
        if (it.x != loaded) {
            __syncthreads();
            stage_blob(smem, p.net.base, p.net.bytes);
            __syncthreads();
            loaded = it.x;
        }
        const NetPtrs P = net_ptrs(smem, p.net);
        DirectSrc<DT, 8 * NT::HT> src(P.f0);
        const long u = (long)it.y + wave;
        // the goal is read from the instance table (a lane-indexed read of the
        // copy above would place the whole copy in scratch memory)
        plan_unit<DT, D_S, N_ACT, D_A, D_W, WIDTH, NHID>(src, P, p, bp.insts[it.x].goal, u, wave < it.z, lane, g,
                                                         col);
    }
    }
}

__global__ __launch_bounds__(64) void reset_counter_kernel(int* counter) { if (threadIdx.x == 0) *counter = 0; }

__global__ __launch_bounds__(256) void q_reduce_kernel(QReduceParams p) {
    const int lane = threadIdx.x & 63;
    const int k = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (k >= p.K) return;
    float s = 0.0f;
    for (int j = lane; j < p.n_tiles; j += 64) s += p.partials[(size_t)k * p.n_tiles + j];
    s += __shfl_xor(s, 32);
    s = sum32(s);
    if (lane == 0) p.q[k] = s * p.scale;
}

__global__ __launch_bounds__(256) void q_reduce_batch_kernel(const QReduceParams* qs) {
    const QReduceParams p = qs[blockIdx.y];
    const int lane = threadIdx.x & 63;
    const int k = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (k >= p.K) return;
    float s = 0.0f;
    for (int j = lane; j < p.n_tiles; j += 64) s += p.partials[(size_t)k * p.n_tiles + j];
    s += __shfl_xor(s, 32);
    s = sum32(s);
    if (lane == 0) p.q[k] = s * p.scale;
}

// launchers
#define PLAN_K(id, ds, na, da, dw, dox, dwz, w, nh, DT) plan_kernel<DT, ds, na, da, dw, w, nh, plan_mode<w>()>
// The bfloat16 instances of plan_kernel (built in k_plan_bf16.hip).
const void* plan_kernel_bf16(int shape);

size_t plan_stream_lds(int shape, int dt) {
    switch (shape * 2 + dt) {
#define X(id, ds, na, da, dw, dox, dwz, w, nh)                                      \
    case id * 2 + 0:                                                               \
        return stream_lds_of<DT_F32, ds, na, (na > 0 ? 0 : da), dw, w, nh, VOILA_PLAN_STREAM_CHB>(); \
    case id * 2 + 1:                                                               \
        return stream_lds_of<DT_BF16, ds, na, (na > 0 ? 0 : da), dw, w, nh, VOILA_PLAN_STREAM_CHB>();
        VOILA_SHAPES(X)
#undef X
    }
    return kStreamLds;
}
#define PROP_K(id, ds, na, da, dw, dox, dwz, w, nh, DT) propose_kernel<DT, ds, dw, w, nh, pass_mode<w>()>
#define OBS_K(id, ds, na, da, dw, dox, dwz, w, nh, DT) observe_kernel<DT, ds, dwz, dox, w, nh, pass_mode<w>()>

#define PLAN_SK(id, ds, na, da, dw, dox, dwz, w, nh, DT) plan_split_kernel<DT, ds, na, da, dw, w, nh>

template <int DT, int D_S, int D_A, int D_W, int W, int NH>
constexpr size_t plan_split_lds() {
    if constexpr (!plan_split<DT, W, NH>()) {
        return 0;
    } else {
        typedef Net<DT, W, NH, in_slots(DT, D_S, D_A, D_W), W / 32, cdiv(D_S, 32)> NT;
        return (size_t)PlanSplitLds<NT, D_S>::BYTES;
    }
}

bool plan_split_shape(int shape, int dt) {
    switch (shape * 2 + dt) {
#define X(id, ds, na, da, dw, dox, dwz, w, nh) \
    case id * 2 + 0:                           \
        return plan_split<DT_F32, w, nh>();    \
    case id * 2 + 1:                           \
        return plan_split<DT_BF16, w, nh>();
        VOILA_SHAPES(X)
#undef X
    }
    return false;
}

template <class K>
void launch_plan_split_one(K k, size_t lds, int blocks, const PlanParams& p, hipStream_t s) {
    if (lds > 65536) (void)hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL(k, blocks, 64 * kPlanSplitWaves, lds, s, p);
}

hipError_t launch_plan(int shape, int dt, const PlanParams& p, int blocks, hipStream_t s) {
    if (plan_split_shape(shape, dt)) {
        switch (shape * 2 + dt) {
#define X(id, ds, na, da, dw, dox, dwz, w, nh)                                                                      \
    case id * 2 + 0:                                                                                               \
        launch_plan_split_one(PLAN_SK(id, ds, na, da, dw, dox, dwz, w, nh, DT_F32),                                 \
                              plan_split_lds<DT_F32, ds, (na > 0 ? 0 : da), dw, w, nh>(), blocks, p, s);           \
        break;                                                                                                     \
    case id * 2 + 1:                                                                                               \
        launch_plan_split_one(PLAN_SK(id, ds, na, da, dw, dox, dwz, w, nh, DT_BF16),                                \
                              plan_split_lds<DT_BF16, ds, (na > 0 ? 0 : da), dw, w, nh>(), blocks, p, s);          \
        break;
            VOILA_SHAPES(X)
#undef X
            default:
                return hipErrorInvalidValue;
        }
        return hipGetLastError();
    }
    size_t lds = weights_in_lds(shape) ? p.net.bytes : plan_stream_lds(shape, dt) + (p.net.bytes - p.net.off_b0);
    switch (shape * 2 + dt) {
#define X(id, ds, na, da, dw, dox, dwz, w, nh)                                                              \
    case id * 2 + 0:                                                                                       \
        if (lds > 65536)                                                                                   \
            (void)hipFuncSetAttribute((const void*)PLAN_K(id, ds, na, da, dw, dox, dwz, w, nh, DT_F32),     \
                                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);               \
        hipLaunchKernelGGL((PLAN_K(id, ds, na, da, dw, dox, dwz, w, nh, DT_F32)), blocks, 256, lds, s, p);  \
        break;                                                                                             \
    case id * 2 + 1: {                                                                                     \
        const void* k = plan_kernel_bf16(id);                                                              \
        if (lds > 65536) (void)hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds); \
        void* args[] = {(void*)&p};                                                                        \
        (void)hipLaunchKernel(k, dim3(blocks), dim3(256), args, lds, s);                                   \
        break;                                                                                             \
    }
        VOILA_SHAPES(X)
#undef X
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

int plan_pass_tiles(int shape, int dt) {
    switch (shape * 2 + dt) {
#define X(id, ds, na, da, dw, dox, dwz, w, nh)              \
    case id * 2 + 0:                                       \
        return plan_pairs<DT_F32, w, nh>() ? kPlanPassTiles : 0; \
    case id * 2 + 1:                                       \
        return plan_pairs<DT_BF16, w, nh>() ? kPlanPassTiles : 0;
        VOILA_SHAPES(X)
#undef X
    }
    return 0;
}

int plan_tiles_per_unit(int shape, int dt) {
    return plan_split_shape(shape, dt) ? kPlanSplitTiles : plan_pass_tiles(shape, dt) ? 2 : 1;
}
int plan_units_per_block(int shape, int dt) { return plan_split_shape(shape, dt) ? 1 : kWavesPerBlock; }

int plan_blocks_per_cu(int shape, int dt) {
    if (plan_split_shape(shape, dt)) {
        switch (shape * 2 + dt) {
#define X(id, ds, na, da, dw, dox, dwz, w, nh)                                                                 \
    case id * 2 + 0:                                                                                          \
        return occupancy_t(PLAN_SK(id, ds, na, da, dw, dox, dwz, w, nh, DT_F32), 64 * kPlanSplitWaves,          \
                           plan_split_lds<DT_F32, ds, (na > 0 ? 0 : da), dw, w, nh>());                        \
    case id * 2 + 1:                                                                                          \
        return occupancy_t(PLAN_SK(id, ds, na, da, dw, dox, dwz, w, nh, DT_BF16), 64 * kPlanSplitWaves,         \
                           plan_split_lds<DT_BF16, ds, (na > 0 ? 0 : da), dw, w, nh>());
            VOILA_SHAPES(X)
#undef X
        }
        return 1;
    }
    switch (shape * 2 + dt) {
#define X(id, ds, na, da, dw, dox, dwz, w, nh)                                                               \
    case id * 2 + 0:                                                                                        \
        return occupancy(PLAN_K(id, ds, na, da, dw, dox, dwz, w, nh, DT_F32), lds_for_width<w>() ? kLdsGuess : kPlanStreamLds); \
    case id * 2 + 1:                                                                                        \
        return occupancy(plan_kernel_bf16(id), lds_for_width<w>() ? kLdsGuess : kPlanStreamLds);
        VOILA_SHAPES(X)
#undef X
    }
    return 1;
}

#define PLANB_K(id, ds, na, da, dw, dox, dwz, w, nh, DT) plan_batch_kernel<DT, ds, na, da, dw, w, nh>

hipError_t launch_plan_batch(int shape, int dt, const BatchPlanParams& p, int blocks, int wpb, size_t lds,
                             hipStream_t s) {
    if (!weights_in_lds(shape)) return hipErrorInvalidValue;
    switch (shape * 2 + dt) {
#define X(id, ds, na, da, dw, dox, dwz, w, nh)                                                                     \
    case id * 2 + 0:                                                                                              \
        hipLaunchKernelGGL((PLANB_K(id, ds, na, da, dw, dox, dwz, w, nh, DT_F32)), blocks, 64 * wpb, lds, s, p);   \
        break;                                                                                                    \
    case id * 2 + 1:                                                                                              \
        hipLaunchKernelGGL((PLANB_K(id, ds, na, da, dw, dox, dwz, w, nh, DT_BF16)), blocks, 64 * wpb, lds, s, p);  \
        break;
        VOILA_SHAPES(X)
#undef X
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

int plan_batch_blocks_per_cu(int shape, int dt, int wpb, size_t lds) {
    switch (shape * 2 + dt) {
#define X(id, ds, na, da, dw, dox, dwz, w, nh)                                                        \
    case id * 2 + 0:                                                                                 \
        return occupancy_t(PLANB_K(id, ds, na, da, dw, dox, dwz, w, nh, DT_F32), 64 * wpb, lds);      \
    case id * 2 + 1:                                                                                 \
        return occupancy_t(PLANB_K(id, ds, na, da, dw, dox, dwz, w, nh, DT_BF16), 64 * wpb, lds);
        VOILA_SHAPES(X)
#undef X
    }
    return 1;
}


hipError_t launch_q_reduce_batch(const QReduceParams* d_qs, int n_inst, int max_k, hipStream_t s) {
    if (n_inst == 0 || max_k == 0) return hipSuccess;
    hipLaunchKernelGGL(q_reduce_batch_kernel, dim3((max_k + 3) / 4, n_inst), 256, 0, s, d_qs);
    return hipGetLastError();
}

hipError_t launch_reset_counter(int* d_counter, hipStream_t s) {
    hipLaunchKernelGGL(reset_counter_kernel, 1, 64, 0, s, d_counter);
    return hipGetLastError();
}

hipError_t launch_q_reduce(const QReduceParams& p, hipStream_t s) {
    const int blocks = (p.K + 3) / 4;
    if (blocks == 0) return hipSuccess;
    hipLaunchKernelGGL(q_reduce_kernel, blocks, 256, 0, s, p);
    return hipGetLastError();
}

}  // namespace voila
