// kernels.hip -- HIP kernels of the plan / update / observe hot path (gfx950).
//
// plan_kernel     persistent rollout kernel: each wave owns a (candidate, 32-particle)
//                 tile, keeps the 32 states in registers for the whole horizon and
//                 runs every transition-network layer on the matrix cores
//                 (transposed evaluation, see device.hpp), with the noise drawn in
//                 registers from Philox.  Small networks are staged in LDS once per
//                 block; wide ones stream their fragments from L2.
// q_reduce_kernel fixed-order sum of the per-tile partial returns into Q.
// fold_kernel     folds a fixed action (and observation) into a first-layer bias.
// propose_kernel  update stage 1: proposal s' = s + f_T and likelihood l(s', a, o)
//                 for 32 particles per wave; writes s', l and x = l / lambda.
// norm_res_kernel update stage 2 in one workgroup (N <= 8192): binary64 max /
//                 exp / sum normalisation with fixed-order reductions, exact
//                 quantised prefix sum, systematic resampling by binary search,
//                 and the gather of the resampled particles.
#include "kernels.hpp"

#include <math.h>

namespace voila {

namespace {

const ShapeInfo kShapeInfo[kNumShapes] = {
#define X(id, ds, na, da, dw, dox, dwz, w, nh) {ds, na, da, dw, dox, dwz, w, nh},
    VOILA_SHAPES(X)
#undef X
};

// Global memory that no kernel of the launch writes, read through the
// constant address space so wave-uniform reads become scalar loads.
#define kconst __attribute__((address_space(4)))

// r = -||s - g||^2 with the goal already in this lane's slot order.
__device__ __forceinline__ float reward_to(const float* st, const float* goal_slots, int n_slots, int d_s, int g) {
    float part = 0.0f;
    for (int s = 0; s < n_slots; ++s) {
        if (2 * s + g < d_s) {
            float e = st[s] - goal_slots[s];
            part = __builtin_fmaf(e, e, part);
        }
    }
    return -(part + __shfl_xor(part, 32));
}



}  // namespace

const ShapeInfo& shape_info(int shape) { return kShapeInfo[shape]; }

// ---------------------------------------------------------------------------
// plan
// ---------------------------------------------------------------------------
// Binary32 activations of a network wider than 256 do not fit in registers:
// such networks run in bfloat16 only.
constexpr bool net_compiled(int dt, int width) { return dt == DT_BF16 || width <= 256; }

// How a kernel reads the weight fragments of a network.
constexpr int kDirect = 0;    // straight from global memory (L2)
constexpr int kResident = 1;  // whole network staged in LDS once per block
constexpr int kStream = 2;    // streamed through double-buffered LDS chunks
constexpr int kSplit = 3;     // the four waves of a block split each layer of one tile (global memory)

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
            float nz[SW];
            noise_slots_philox<SW>(nz, p.key0, p.key1, (uint32_t)i, p.crn ? 0u : (uint32_t)k, (uint32_t)t, 3u, g);
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

// The weight source of a rollout-sized launch of network NT, handed to
// body(src, P) with the network's pointers: the whole network staged in LDS
// once per block (kResident), streamed through the LDS chunk buffers with the
// biases -- and for a grouped wide network the first layer -- staged after
// them (kStream), or read from L2 (kDirect).  B0_ROWS is the number of
// first-layer bias rows the blob carries (one per discrete action).
template <class NT, int MODE, int B0_ROWS, class Body>
__device__ __forceinline__ void with_weights(char* smem, const NetBlob& net, Body&& body) {
    if (MODE == kResident) {
        stage_blob(smem, net.base, net.bytes);
        __syncthreads();
    }
    NetPtrs P = net_ptrs(MODE == kResident ? (const char*)smem : net.base, net);
    constexpr bool F0_LDS = NT::CT < NT::HT && first_layer_in_lds<NT>(B0_ROWS);
    char* extra = smem;
    if constexpr (MODE == kStream) {
        extra = smem + StreamChunk<NT>::BYTES;
        const uint32_t f0_bytes = F0_LDS ? (uint32_t)(NT::NF0 * NT::FRAG_BYTES) : 0u;
        if (f0_bytes) stage_blob(extra, P.f0, f0_bytes);
        char* bias = extra + f0_bytes;
        stage_blob(bias, net.base + net.off_b0, net.bytes - net.off_b0);
        __syncthreads();
        P.b0 = reinterpret_cast<const float*>(bias);
        P.bh = reinterpret_cast<const float*>(bias + (net.off_bh - net.off_b0));
        P.bo = reinterpret_cast<const float*>(bias + (net.off_bo - net.off_b0));
    }
    if constexpr (MODE == kStream && NT::CT < NT::HT) {
        // grouped wide network: the groups' fragments stream through the LDS
        // chunk buffers, the first layer is read from its LDS copy
        WideSrc<NT, GroupStream<NT>> src(F0_LDS ? (const char*)extra : P.f0, GroupStream<NT>(smem, P.fh));
        src.hid.start();
        body(src, P);
        src.hid.finish();
    } else if constexpr (MODE == kStream) {
        StreamFor<NT> src(smem, P.f0);
        src.start();
        body(src, P);
        src.finish();
    } else {
        DirectSrc<NT::DT, 8 * NT::HT> src(P.f0);
        body(src, P);
    }
}

template <int DT, int D_S, int N_ACT, int D_A, int D_W, int WIDTH, int NHID, int MODE>
__global__ __launch_bounds__(256) void plan_kernel(PlanParams p) {
    if constexpr (!net_compiled(DT, WIDTH)) {
        return;  // binary32 networks wider than 256 are refused at model creation
    } else {
    typedef Net<DT, WIDTH, NHID, in_slots(DT, D_S, D_A, D_W)> NT;
    extern __shared__ __attribute__((aligned(16))) char smem[];
    const int lane = threadIdx.x & 63, g = lane >> 5, col = lane & 31;
    const int wpb = blockDim.x >> 6, wave = threadIdx.x >> 6;
    const long n_units = (long)p.K * p.n_tiles;
    with_weights<NT, MODE, (N_ACT > 0 ? N_ACT : 1)>(smem, p.net, [&](auto& src, const NetPtrs& P) {
        // block-uniform loop: every wave of a block walks the same sequence of
        // (unit, step) iterations, idle waves on a masked dummy unit
        for (long ub = blockIdx.x; ub * wpb < n_units; ub += gridDim.x) {
            const long u = ub * wpb + wave;
            plan_unit<DT, D_S, N_ACT, D_A, D_W, WIDTH, NHID>(src, P, p, p.goal, u, u < n_units, lane, g, col);
        }
    });
    }
}

// Many planning instances of one network shape in one persistent launch.
// The work list holds block items (instance, first tile unit, number of
// units): a block takes items from a queue (atomic counter, list sorted by
// decreasing cost) or in a static stride, restages the instance's network in
// LDS when the instance changes, and runs one unit per wave.
template <int DT, int D_S, int N_ACT, int D_A, int D_W, int WIDTH, int NHID>
__global__ __launch_bounds__(512) void plan_batch_kernel(BatchPlanParams bp) {
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

__global__ __launch_bounds__(256) void fold_kernel(FoldParams p) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= p.width) return;
    float acc = p.b[r];
    for (int c = 0; c < p.nf; ++c) acc += p.w[(size_t)r * p.nf + c] * p.v[c];
    p.out[r] = acc;
}

// First-layer biases with the action of every (candidate, step) group folded
// in, in the column order of fold_kernel.
__global__ __launch_bounds__(256) void fold_steps_kernel(FoldStepsParams p) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= p.width) return;
    for (int j = blockIdx.y; j < p.rows; j += gridDim.y) {
        float acc = p.b[r];
        if (p.n_actions > 0) {
            int a = reinterpret_cast<const int32_t*>(p.cands)[j];
            if (a < 0 || a >= p.n_actions) {
                if (p.status && r == 0) p.status[0] = 1;
                a = 0;
            }
            for (int c = 0; c < p.n_actions; ++c) acc += p.w[(size_t)r * p.nf + c] * (c == a ? 1.0f : 0.0f);
        } else {
            const float* ac = reinterpret_cast<const float*>(p.cands) + (size_t)j * p.d_a;
            for (int c = 0; c < p.d_a; ++c) {
                float v = ac[c];
                if (p.bf16) v = (float)(__bf16)v;
                acc += p.w[(size_t)r * p.nf + c] * v;
            }
        }
        if (p.obs) {
            const int c0 = p.n_actions > 0 ? p.n_actions : p.d_a;
            const float* ob = p.obs + (size_t)j * p.d_o;
            for (int c = 0; c < p.d_o; ++c) {
                float v = ob[c];
                if (p.bf16) v = (float)(__bf16)v;
                acc += p.w[(size_t)r * p.nf + c0 + c] * v;
            }
        }
        p.out[(size_t)j * p.width + r] = acc;
    }
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

// Per-instance first-layer bias with the instance's action (and observation)
// folded in; the fold inputs are read from device memory so the launch can be
// replayed from a graph with new actions / observations.
__global__ __launch_bounds__(256) void fold_batch_kernel(const FoldBatchItem* items, const void* actions,
                                                         const float* obs, int32_t* status) {
    const FoldBatchItem p = items[blockIdx.y];
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= p.width) return;
    float acc = p.b[r];
    int c = 0;
    if (p.n_actions > 0) {
        int a = reinterpret_cast<const int32_t*>(actions)[p.inst];
        if (a < 0 || a >= p.n_actions) {
            if (status && r == 0) status[0] = 1;
            a = 0;
        }
        acc += p.w[(size_t)r * p.nf + a];
        c = p.n_actions;
    } else {
        const float* ac = reinterpret_cast<const float*>(actions) + (size_t)p.inst * p.d_a;
        for (int j = 0; j < p.d_a; ++j, ++c) {
            float v = ac[j];
            if (p.bf16) v = (float)(__bf16)v;
            acc += p.w[(size_t)r * p.nf + c] * v;
        }
    }
    if (p.with_obs) {
        const float* ob = obs + (size_t)p.inst * p.d_o;
        for (int j = 0; j < p.d_o; ++j, ++c) {
            float v = ob[j];
            if (p.bf16) v = (float)(__bf16)v;
            acc += p.w[(size_t)r * p.nf + c] * v;
        }
    }
    p.out[r] = acc;
}

// ---------------------------------------------------------------------------
// update stage 1: proposal and likelihood
// ---------------------------------------------------------------------------
// One 32-particle tile of the update's first stage: proposal through the
// transition network, likelihood of the proposal, x = l / lambda (+ log prior).
template <int DT, int D_S, int D_W, int WIDTH, int NHID, bool SPLIT = false>
__device__ __forceinline__ void propose_tile(const NetPtrs& PT, const NetPtrs& PL, const ProposeParams& p, int tile,
                                             bool tile_ok, int lane, int g, int col, int wave = 0,
                                             char* lds = nullptr) {
    constexpr int SS = state_slots(D_S), SW = noise_slots(D_W);
    typedef Net<DT, WIDTH, NHID, in_slots(DT, D_S, 0, D_W)> NTT;
    typedef Net<DT, WIDTH, NHID, in_slots(DT, D_S, 0, 0)> NTL;
    const int i = tile * 32 + col;
    const bool valid = tile_ok && i < p.N;
    float slots[NTT::IN_SLOTS];
#pragma unroll
    for (int s = 0; s < NTT::IN_SLOTS; ++s) slots[s] = 0.0f;
    float st[SS];
#pragma unroll
    for (int s = 0; s < SS; ++s) {
        int f = 2 * s + g;
        st[s] = (valid && f < D_S) ? p.states[(size_t)i * D_S + f] : 0.0f;
        slots[s] = st[s];
    }
    if (p.noise) {
#pragma unroll
        for (int s = 0; s < SW; ++s) {
            int f = noise_feature(s, g);
            slots[SS + s] = (valid && f < D_W) ? p.noise[(size_t)i * D_W + f] : 0.0f;
        }
    } else {
        float nz[SW];
        noise_slots_philox<SW>(nz, p.key0, p.key1, (uint32_t)i, 0u, 0u, 5u, g);
#pragma unroll
        for (int s = 0; s < SW; ++s) slots[SS + s] = nz[s];
    }
    f32x16 d;
    if constexpr (SPLIT) {
        d = run_net_split<NTT>(PT, p.b0_trans, slots, lane, g, wave, lds);
    } else {
        auto srct = DirectFor<NTT>::make(PT);
        d = run_net<NTT>(srct, PT, p.b0_trans, slots, lane, g);
    }
    const bool writer = !SPLIT || wave == 0;  // a split tile is written by its first wave
    float ls[NTL::IN_SLOTS];
#pragma unroll
    for (int s = 0; s < NTL::IN_SLOTS; ++s) ls[s] = 0.0f;
#pragma unroll
    for (int s = 0; s < SS; ++s) {
        int f = 2 * s + g;
        st[s] += d[s];
        ls[s] = st[s];
        if (writer && valid && f < D_S) p.prop[(size_t)i * D_S + f] = st[s];
    }
    f32x16 lo;
    if constexpr (SPLIT) {
        lo = run_net_split<NTL>(PL, p.b0_lik, ls, lane, g, wave, lds);
    } else {
        auto srcl = DirectFor<NTL>::make(PL);
        lo = run_net<NTL>(srcl, PL, p.b0_lik, ls, lane, g);
    }
    if (writer && g == 0 && valid) {
        float l = lo[0];
        if (p.loglik) p.loglik[i] = l;
        if (!isfinite(l) && p.status) p.status[0] = 5;
        double x = (double)l / p.lambda;
        if (p.prior_w) x += log(p.prior_w[i]);
        p.x[i] = x;
    }
}

template <int DT, int D_S, int D_W, int WIDTH, int NHID, int MODE>
__global__ __launch_bounds__(256) void propose_kernel(ProposeParams p) {
    if constexpr (!net_compiled(DT, WIDTH)) {
        return;  // binary32 networks wider than 256 are refused at model creation
    } else {
    constexpr bool WLDS = MODE == kResident;
    extern __shared__ __attribute__((aligned(16))) char smem[];
    if (WLDS) {
        stage_blob(smem, p.trans.base, p.trans.bytes);
        stage_blob(smem + p.trans.bytes, p.lik.base, p.lik.bytes);
        __syncthreads();
    }
    const NetPtrs PT = net_ptrs(WLDS ? (const char*)smem : p.trans.base, p.trans);
    const NetPtrs PL = net_ptrs(WLDS ? (const char*)smem + p.trans.bytes : p.lik.base, p.lik);
    const int lane = threadIdx.x & 63, g = lane >> 5, col = lane & 31;
    const int wpb = blockDim.x >> 6;
    const int n_tiles = (p.N + 31) / 32;
    if constexpr (MODE == kSplit) {
        const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
        for (int tile = blockIdx.x; tile < n_tiles; tile += gridDim.x)
            propose_tile<DT, D_S, D_W, WIDTH, NHID, true>(PT, PL, p, tile, true, lane, g, col, wave, smem);
    } else {
        for (int tile = blockIdx.x * wpb + (threadIdx.x >> 6); tile < n_tiles; tile += gridDim.x * wpb)
            propose_tile<DT, D_S, D_W, WIDTH, NHID>(PT, PL, p, tile, true, lane, g, col);
    }
    }
}

// Update stage 1 of many instances: block items (instance, first tile, tiles),
// networks restaged in LDS on an instance change.
template <int DT, int D_S, int D_W, int WIDTH, int NHID>
__global__ __launch_bounds__(512) void propose_batch_kernel(BatchProposeParams bp) {
    if constexpr (WIDTH > 64) {
        return;  // batches need networks that fit in LDS (the launcher refuses wider ones)
    } else {
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
        const int4 it = bp.items[item];
        ProposeParams p = bp.insts[it.x];
        p.status = bp.status;
        if (it.x != loaded) {
            __syncthreads();
            stage_blob(smem, p.trans.base, p.trans.bytes);
            stage_blob(smem + p.trans.bytes, p.lik.base, p.lik.bytes);
            __syncthreads();
            loaded = it.x;
        }
        const NetPtrs PT = net_ptrs(smem, p.trans);
        const NetPtrs PL = net_ptrs(smem + p.trans.bytes, p.lik);
        propose_tile<DT, D_S, D_W, WIDTH, NHID>(PT, PL, p, it.y + wave, wave < it.z, lane, g, col);
    }
    }
}

// ---------------------------------------------------------------------------
// observe
// ---------------------------------------------------------------------------
// Rows are (group, particle) pairs: group j = k * H + t has its own folded
// first-layer bias (its action) and 32-particle tiles; row (k, i, t) reads
// state row (k * N + i) * H + t, draws its noise at counter (i, k or 0 under
// common random numbers, t) and writes the same output row.  A plain
// observation of n states is the case K = H = 1.
struct ObsRow {
    size_t r;     // state / noise / output row
    int grp;      // bias row
    bool valid;   // this lane's particle exists
};

// Inputs [s', w_Z] of this lane's row of tile unit u in first-layer slot order.
template <int D_S, int D_WZ, int IN_SLOTS>
__device__ __forceinline__ ObsRow observe_inputs(const ObserveParams& p, long u, int n_tiles, int g, int col,
                                                 float (&slots)[IN_SLOTS]) {
    constexpr int SS = state_slots(D_S), SW = noise_slots(D_WZ);
    ObsRow w;
    w.grp = (int)(u / n_tiles);
    const int tile = (int)(u - (long)w.grp * n_tiles);
    const int k = w.grp / p.H, t = w.grp - k * p.H;
    const int i = tile * 32 + col;
    w.valid = i < p.N;
    w.r = ((size_t)k * p.N + (w.valid ? i : 0)) * p.H + t;
#pragma unroll
    for (int s = 0; s < IN_SLOTS; ++s) slots[s] = 0.0f;
#pragma unroll
    for (int s = 0; s < SS; ++s) {
        int f = 2 * s + g;
        slots[s] = (w.valid && f < D_S) ? p.states[w.r * D_S + f] : 0.0f;
    }
    if (p.noise) {
#pragma unroll
        for (int s = 0; s < SW; ++s) {
            int f = noise_feature(s, g);
            slots[SS + s] = (w.valid && f < D_WZ) ? p.noise[w.r * D_WZ + f] : 0.0f;
        }
    } else {
        float nz[SW];
        noise_slots_philox<SW>(nz, p.key0, p.key1, (uint32_t)i, p.crn ? 0u : (uint32_t)k, (uint32_t)t, 4u, g);
#pragma unroll
        for (int s = 0; s < SW; ++s) slots[SS + s] = nz[s];
    }
    return w;
}

template <int D_O>
__device__ __forceinline__ void observe_store(const ObserveParams& p, const ObsRow& w, const f32x16& o, bool writer,
                                              int g) {
#pragma unroll
    for (int s = 0; s < 16; ++s) {
        int f = 2 * s + g;
        if (writer && w.valid && f < D_O) p.out[w.r * D_O + f] = o[s];
    }
}

// MODE kResident / kSplit / kDirect: sized for one belief (n rows); kStream:
// sized for the rows of whole rollouts, one tile per wave with the weights
// streamed through LDS like the rollout kernel's.
template <int DT, int D_S, int D_WZ, int D_O, int WIDTH, int NHID, int MODE>
__global__ __launch_bounds__(256) void observe_kernel(ObserveParams p) {
    if constexpr (!net_compiled(DT, WIDTH)) {
        return;  // binary32 networks wider than 256 are refused at model creation
    } else {
    typedef Net<DT, WIDTH, NHID, in_slots(DT, D_S, 0, D_WZ)> NTO;
    extern __shared__ __attribute__((aligned(16))) char smem[];
    const int lane = threadIdx.x & 63, g = lane >> 5, col = lane & 31;
    const int n_tiles = (p.N + 31) / 32;
    const long n_units = (long)p.K * p.H * n_tiles;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if constexpr (MODE == kStream) {
        const int wpb = blockDim.x >> 6;
        // each wave keeps the (candidate, step) group's bias row in its own
        // LDS row, refreshed when the group changes (every N/32 units)
        float* rowb = reinterpret_cast<float*>(smem + p.row_bias_lds) + wave * NTO::WIDTH;
        constexpr int RB = NTO::WIDTH / 64;  // bias floats per lane
        static_assert(NTO::WIDTH % 64 == 0 && RB <= 16, "bias row copy: whole lanes");
        int have = -1;
        with_weights<NTO, MODE, 1>(smem, p.obs, [&](auto& src, const NetPtrs& P) {
            // block-uniform loop (the stream's chunk barriers need every wave)
            for (long ub = blockIdx.x; ub * wpb < n_units; ub += gridDim.x) {
                const long u = ub * wpb + wave;
                const bool ok = u < n_units;
                float slots[NTO::IN_SLOTS];
                const ObsRow w = observe_inputs<D_S, D_WZ>(p, ok ? u : 0, n_tiles, g, col, slots);
                const int brow = p.b0_stride ? w.grp : 0;
                const bool fresh = brow != have;  // wave-uniform
                float bv[RB];
                if (fresh) {
                    const float* src_row = p.b0 + (size_t)brow * p.b0_stride;
#pragma unroll
                    for (int q = 0; q < RB; ++q) bv[q] = src_row[q * 64 + lane];
                }
                // complete the row loads here so that the compiler's wait for
                // them does not also drain the weight stream inside the layers
                __builtin_amdgcn_s_waitcnt(waitcnt_vm_lgkm0(0));
                if (fresh) {
#pragma unroll
                    for (int q = 0; q < RB; ++q) rowb[q * 64 + lane] = bv[q];
                    __builtin_amdgcn_s_waitcnt(waitcnt_vm_lgkm0(0));
                    __builtin_amdgcn_wave_barrier();
                    have = brow;
                }
                const f32x16 o = run_net<NTO>(src, P, rowb, slots, lane, g);
                observe_store<D_O>(p, w, o, ok, g);
            }
        });
    } else {
        if (MODE == kResident) {
            stage_blob(smem, p.obs.base, p.obs.bytes);
            __syncthreads();
        }
        const NetPtrs PO = net_ptrs(MODE == kResident ? (const char*)smem : p.obs.base, p.obs);
        // split mode: the block's four waves evaluate one tile together
        const int tpb = MODE == kSplit ? 1 : (int)(blockDim.x >> 6);
        const long first = MODE == kSplit ? (long)blockIdx.x : (long)blockIdx.x * tpb + wave;
        for (long u = first; u < n_units; u += (long)gridDim.x * tpb) {
            float slots[NTO::IN_SLOTS];
            const ObsRow w = observe_inputs<D_S, D_WZ>(p, u, n_tiles, g, col, slots);
            const float* b0 = p.b0 + (size_t)w.grp * p.b0_stride;
            f32x16 o;
            if constexpr (MODE == kSplit) {
                o = run_net_split<NTO>(PO, b0, slots, lane, g, wave, smem);
            } else {
                auto srco = DirectFor<NTO>::make(PO);
                o = run_net<NTO>(srco, PO, b0, slots, lane, g);
            }
            observe_store<D_O>(p, w, o, MODE != kSplit || wave == 0, g);
        }
    }
    }
}

// ---------------------------------------------------------------------------
// update stage 2: normalisation and systematic resampling in one workgroup
// ---------------------------------------------------------------------------
namespace {

constexpr int kNRWaves = kNormResThreads / 64;

__device__ __forceinline__ double wave_sum_d(double v) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m);
    return v;
}
__device__ __forceinline__ double wave_max_d(double v) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v = fmax(v, __shfl_xor(v, m));
    return v;
}
__device__ __forceinline__ int wave_max_i(int v) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v = max(v, __shfl_xor(v, m));
    return v;
}

// Block reductions in a fixed order: lanes (butterfly), then waves 0..15 in order.
__device__ double block_sum_d(double v, double* red) {
    v = wave_sum_d(v);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double s = 0.0;
    for (int w = 0; w < kNRWaves; ++w) s += red[w];
    return s;
}
__device__ double block_max_d(double v, double* red) {
    v = wave_max_d(v);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double m = -INFINITY;
    for (int w = 0; w < kNRWaves; ++w) m = fmax(m, red[w]);
    return m;
}
__device__ int block_max_i(int v, int* red) {
    v = wave_max_i(v);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    int m = -1;
    for (int w = 0; w < kNRWaves; ++w) m = max(m, red[w]);
    return m;
}

}  // namespace

// dst row r = src row ids[r] for r < n (rows of w elements) by the whole
// workgroup: each thread keeps one column and walks rows, so consecutive
// threads move consecutive elements.
template <class T>
__device__ __forceinline__ void block_gather(T* dst, const T* src, const int* ids, int n, int w) {
    const int nt = blockDim.x;
    if (w <= nt) {
        const int rpp = nt / w, r0 = threadIdx.x / w, c = threadIdx.x - r0 * w;
        if (r0 < rpp)
            for (int r = r0; r < n; r += rpp) dst[(size_t)r * w + c] = src[(size_t)ids[r] * w + c];
    } else {
        for (int r = 0; r < n; ++r)
            for (int c = threadIdx.x; c < w; c += nt) dst[(size_t)r * w + c] = src[(size_t)ids[r] * w + c];
    }
}

__device__ void norm_res_body(const NormResParams& p, double* buf, double* redd, int* redi, int* ids) {
    const int tid = threadIdx.x, N = p.N;

    if (!p.w_in) {
        int bad = 0;
        double mx = -INFINITY;
        for (int i = tid; i < N; i += kNormResThreads) {
            double x;
            if (p.x) {
                x = p.x[i];
            } else {
                float l = p.loglik[i];
                if (!isfinite(l)) bad = 1;
                x = (double)l / p.lambda;
                if (p.prior_w) x += log(p.prior_w[i]);
            }
            if (isnan(x) || x == INFINITY) bad = 1;
            buf[i] = x;
            mx = fmax(mx, x);
        }
        mx = block_max_d(mx, redd);
        int anybad = block_max_i(bad, redi);
        if (anybad || !isfinite(mx)) {
            if (tid == 0 && p.status) p.status[0] = 5;
            return;
        }
        double s = 0.0;
        for (int i = tid; i < N; i += kNormResThreads) {
            double e = exp(buf[i] - mx);
            buf[i] = e;
            s += e;
        }
        const double S = block_sum_d(s, redd);
        double sq = 0.0;
        for (int i = tid; i < N; i += kNormResThreads) {
            double w = buf[i] / S;
            buf[i] = w;
            if (p.w_out) p.w_out[i] = w;
            sq += w * w;
        }
        const double SQ = block_sum_d(sq, redd);
        if (tid == 0 && p.stats) {
            p.stats[0] = mx + log(S) - (p.uniform_prior ? log((double)N) : 0.0);
            p.stats[1] = 1.0 / SQ;
        }
    } else {
        int bad = 0;
        for (int i = tid; i < N; i += kNormResThreads) {
            double w = p.w_in[i];
            if (!(w >= 0.0) || w == INFINITY) bad = 1;
            buf[i] = w;
        }
        if (block_max_i(bad, redi)) {
            if (tid == 0 && p.status) p.status[0] = 5;
            return;
        }
    }
    if (!p.do_resample) return;
    __syncthreads();

    // quantise: q_i = rint(w_i * N * 2^b), exact integers below 2^53
    const double scale = ldexp((double)N, p.bits);
    int last = -1;
    for (int i = tid; i < N; i += kNormResThreads) {
        double q = rint(buf[i] * scale);
        buf[i] = q;
        if (q > 0.0) last = i;
    }
    last = block_max_i(last, redi);
    if (last < 0) {
        if (tid == 0 && p.status) p.status[0] = 5;
        return;
    }
    // inclusive prefix sum; every partial sum is an exact integer, so the
    // blocked order gives the same bits as a sequential sum.
    const int per = (N + kNormResThreads - 1) / kNormResThreads;
    const int lo = tid * per, hi = min(N, lo + per);
    double run = 0.0;
    for (int i = lo; i < hi; ++i) {
        run += buf[i];
        buf[i] = run;
    }
    // exclusive scan of the thread totals (wave scan + wave totals)
    double incl = run;
    const int lane = tid & 63;
#pragma unroll
    for (int m = 1; m < 64; m <<= 1) {
        double o = __shfl_up(incl, m);
        if (lane >= m) incl += o;
    }
    __syncthreads();
    if (lane == 63) redd[tid >> 6] = incl;
    __syncthreads();
    double off = incl - run;
    for (int w = 0; w < (tid >> 6); ++w) off += redd[w];
    for (int i = lo; i < hi; ++i) buf[i] += off;
    __syncthreads();

    // systematic positions P_j = j 2^b + u; idx_j = first i with C_i > P_j
    const double step = ldexp(1.0, p.bits);
    const double u = (double)(p.U >> (32 - p.bits));
    for (int j = tid; j < N; j += kNormResThreads) {
        const double P = (double)j * step + u;
        int a = 0, b = N;
        while (a < b) {
            int mid = (a + b) >> 1;
            if (buf[mid] > P) b = mid;
            else a = mid + 1;
        }
        const int idx = a < N ? a : last;
        if (p.idx_out) p.idx_out[j] = idx;
        ids[j] = idx;
    }
    if (p.src && p.dst) {
        __syncthreads();
        const int rf = p.row_floats;
        if (rf % 4 == 0 && ((reinterpret_cast<uintptr_t>(p.src) | reinterpret_cast<uintptr_t>(p.dst)) & 15) == 0)
            block_gather(reinterpret_cast<float4*>(p.dst), reinterpret_cast<const float4*>(p.src), ids, N, rf / 4);
        else
            block_gather(p.dst, p.src, ids, N, rf);
    }
}

__global__ __launch_bounds__(kNormResThreads) void norm_res_kernel(NormResParams p) {
    __shared__ double buf[kNormResMaxN];
    __shared__ int ids[kNormResMaxN];
    __shared__ double redd[kNRWaves];
    __shared__ int redi[kNRWaves];
    norm_res_body(p, buf, redd, redi, ids);
}

// One workgroup per instance.
__global__ __launch_bounds__(kNormResThreads) void norm_res_batch_kernel(const NormResParams* ps, const uint32_t* us,
                                                                          int32_t* status) {
    __shared__ double buf[kNormResMaxN];
    __shared__ int ids[kNormResMaxN];
    __shared__ double redd[kNRWaves];
    __shared__ int redi[kNRWaves];
    NormResParams p = ps[blockIdx.x];
    if (us) p.U = us[blockIdx.x];
    p.status = status;
    norm_res_body(p, buf, redd, redi, ids);
}

// ---------------------------------------------------------------------------
// soft value: V = (1/eta) log sum_k exp(eta Q_k + log pi0_k), per node
// ---------------------------------------------------------------------------
constexpr int kSoftThreads = 256;

__global__ __launch_bounds__(kSoftThreads) void soft_value_kernel(SoftValueParams p) {
    __shared__ double redd[kSoftThreads / 64];
    __shared__ int redi[kSoftThreads / 64];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const double lp_uniform = p.no_prior ? 0.0 : -log((double)p.K);
    for (int m = blockIdx.x; m < p.M; m += gridDim.x) {
        const float* qf = p.Q ? p.Q + (size_t)m * p.K : nullptr;
        const double* qd = p.Qd ? p.Qd + (size_t)m * p.K : nullptr;
        auto q = [&](int k) { return qd ? qd[k] : (double)qf[k]; };
        const double* lp = p.log_pi0 ? p.log_pi0 + (size_t)m * p.K : nullptr;
        // x_k = eta Q_k + log pi0_k; maximum and its first index
        double mx = -INFINITY;
        int arg = p.K;
        int bad = 0;
        for (int k = tid; k < p.K; k += kSoftThreads) {
            const double x = p.eta * q(k) + (lp ? lp[k] : lp_uniform);
            if (isnan(x) || x == INFINITY) bad = 1;
            if (x > mx) {
                mx = x;
                arg = k;
            }
        }
        // (max, lowest index) over the block, in a fixed order
#pragma unroll
        for (int d = 32; d >= 1; d >>= 1) {
            const double om = __shfl_xor(mx, d);
            const int oa = __shfl_xor(arg, d);
            if (om > mx || (om == mx && oa < arg)) {
                mx = om;
                arg = oa;
            }
            bad |= __shfl_xor(bad, d);
        }
        __syncthreads();
        if (lane == 0) {
            redd[wave] = mx;
            redi[wave] = bad ? -1 : arg;
        }
        __syncthreads();
        mx = redd[0];
        arg = redi[0];
        bad = redi[0] < 0;
        for (int w = 1; w < kSoftThreads / 64; ++w) {
            bad |= redi[w] < 0;
            if (redd[w] > mx || (redd[w] == mx && redi[w] < arg)) {
                mx = redd[w];
                arg = redi[w];
            }
        }
        if (bad || !isfinite(mx)) {
            if (tid == 0 && p.status) p.status[0] = 5;
            __syncthreads();
            continue;
        }
        double s = 0.0;
        for (int k = tid; k < p.K; k += kSoftThreads)
            s += exp(p.eta * q(k) + (lp ? lp[k] : lp_uniform) - mx);
#pragma unroll
        for (int d = 32; d >= 1; d >>= 1) s += __shfl_xor(s, d);
        __syncthreads();
        if (lane == 0) redd[wave] = s;
        __syncthreads();
        double S = 0.0;
        for (int w = 0; w < kSoftThreads / 64; ++w) S += redd[w];
        if (tid == 0) {
            p.V[m] = (mx + log(S)) / p.eta;
            if (p.best) p.best[m] = arg;
        }
        if (p.pi)
            for (int k = tid; k < p.K; k += kSoftThreads)
                p.pi[(size_t)m * p.K + k] = exp(p.eta * q(k) + (lp ? lp[k] : lp_uniform) - mx) / S;
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// one-level closed-loop tree (preference backup over observation branches)
// ---------------------------------------------------------------------------
// Successor set of branch group (a, j): the successors of first action a
// starting at successor j; the group's offsets, action and empty branch table.
__global__ __launch_bounds__(256) void tree_groups_kernel(TreeParams p) {
    const int M = p.A * p.n_obs;
    const long n_el = (long)M * p.N * p.d_s;
    for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < n_el; e += (long)gridDim.x * blockDim.x) {
        const long row = e / p.d_s;
        const int c = (int)(e - row * p.d_s);
        const int m = (int)(row / p.N), i = (int)(row - (long)m * p.N);
        const int a = m / p.n_obs, j = m - a * p.n_obs;
        int src = i + j % p.N;
        if (src >= p.N) src -= p.N;
        p.succ[e] = p.succ0[((size_t)a * p.N + src) * p.d_s + c];
    }
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m <= M) p.seg[m] = m * p.N;
    if (m < M) {
        const int a = m / p.n_obs;
        p.zeros[m] = 0;
        p.zeros[M + m] = 0;
        if (p.n_actions > 0) {
            reinterpret_cast<int32_t*>(p.acts)[m] = reinterpret_cast<const int32_t*>(p.first)[a];
        } else {
            for (int c = 0; c < p.d_a; ++c)
                reinterpret_cast<float*>(p.acts)[(size_t)m * p.d_a + c] =
                    reinterpret_cast<const float*>(p.first)[(size_t)a * p.d_a + c];
        }
    }
}

// Child preferences: the mean continuation return of candidate k over the
// particles of child m, one wave per (m, k), fixed summation order.
__global__ __launch_bounds__(256) void tree_child_q_kernel(TreeParams p) {
    const int M = p.A * p.n_obs;
    const int lane = threadIdx.x & 63;
    const long item = (long)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (item >= (long)M * p.K) return;
    const int m = (int)(item / p.K), k = (int)(item - (long)m * p.K);
    const float* g = p.G2 + (size_t)k * ((size_t)M * p.N) + (size_t)m * p.N;
    double s = 0.0;
    for (int i = lane; i < p.N; i += 64) s += (double)g[i];
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) s += __shfl_xor(s, d);
    if (lane == 0) p.Qc[(size_t)m * p.K + k] = s / p.N;
}

// Psi(b, a) = (1/eta) log pi0(a) + R(b, a) + gamma mean_j V_child(a, j).
__global__ __launch_bounds__(64) void tree_backup_kernel(TreeParams p) {
    const int a = blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= p.A) return;
    double v = 0.0;
    for (int j = 0; j < p.n_obs; ++j) v += p.Vc[(size_t)a * p.n_obs + j];
    const double lp = p.log_pi0 ? p.log_pi0[a] : -log((double)p.A);
    p.psi[a] = lp / p.eta + (double)p.R[a] + p.gamma * (v / p.n_obs);
    if (p.R_out) p.R_out[a] = (double)p.R[a];
}

// ---------------------------------------------------------------------------
// grouped progressive widening (simulations grouped by parent action node)
// ---------------------------------------------------------------------------
namespace {
// Group m's successors [lo, lo + n) if the offsets are consistent and the
// group fits one workgroup; otherwise the group is skipped and *status set.
__device__ __forceinline__ bool pw_group(const PwParams& p, int m, int& lo, int& n) {
    lo = p.seg[m];
    const int hi = p.seg[m + 1];
    n = hi - lo;
    if (lo < 0 || hi < lo || hi > p.T || n > kPwMaxGroup) {
        if (p.status) p.status[0] = 1;
        n = 0;
        return false;
    }
    return true;
}
}  // namespace

// First successor of each group (the state a new branch's observation is drawn at).
__global__ __launch_bounds__(256) void pw_first_kernel(PwParams p) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= p.M * p.d_s) return;
    const int m = e / p.d_s, c = e - m * p.d_s;
    int lo, n;
    pw_group(p, m, lo, n);
    p.first[e] = n > 0 ? p.succ[(size_t)lo * p.d_s + c] : 0.0f;
}

// Widening test, branch choice and table update, one thread per action node.
__global__ __launch_bounds__(256) void pw_branch_kernel(PwParams p) {
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= p.M) return;
    int lo, n;
    pw_group(p, m, lo, n);
    int wid = 0, br = -1;
    const int C = p.children[m];
    if (C < 0 || C > p.B) {
        if (p.status) p.status[0] = 1;
        n = 0;
    }
    if (n > 0) {
        wid = C < p.B && (C == 0 || (double)C < p.k_o * pow((double)p.visits[m], p.alpha_o));
        float* row = p.table + (size_t)m * p.B * p.d_o;
        if (wid) {
            br = C;
            for (int c = 0; c < p.d_o; ++c) row[(size_t)br * p.d_o + c] = p.o_new[(size_t)m * p.d_o + c];
            p.children[m] = C + 1;
        } else {
            const uint4 w = philox4x32_10(make_uint4((uint32_t)m, 1u, 0u, 6u << 16), p.key0, p.key1);
            br = (int)floor((double)word_to_uniform(w.x) * (double)C);
        }
        for (int c = 0; c < p.d_o; ++c) p.o_sel[(size_t)m * p.d_o + c] = row[(size_t)br * p.d_o + c];
    } else {
        for (int c = 0; c < p.d_o; ++c) p.o_sel[(size_t)m * p.d_o + c] = 0.0f;
    }
    if (p.widen) p.widen[m] = wid;
    if (p.branch) p.branch[m] = br;
}

// Exclusive prefix of the groups' 32-row tile counts (one workgroup).
__global__ __launch_bounds__(1024) void pw_tiles_kernel(PwParams p) {
    __shared__ int wtot[16];
    const int tid = threadIdx.x, lane = tid & 63;
    const int per = (p.M + 1023) / 1024;
    const int a = tid * per, b = min(p.M, a + per);
    int run = 0;
    for (int m = a; m < b; ++m) {
        int lo, n;
        pw_group(p, m, lo, n);
        run += (n + 31) / 32;
    }
    int incl = run;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        int o = __shfl_up(incl, d);
        if (lane >= d) incl += o;
    }
    if (lane == 63) wtot[tid >> 6] = incl;
    __syncthreads();
    int off = incl - run;
    for (int w = 0; w < (tid >> 6); ++w) off += wtot[w];
    for (int m = a; m < b; ++m) {
        int lo, n;
        pw_group(p, m, lo, n);
        p.tiles[m] = off;
        off += (n + 31) / 32;
    }
    if (tid == 1023) p.tiles[p.M] = off;
}

// Likelihood of every successor against its group's chosen observation:
// x_j = l([s'_j, a_m, o_m]) / lambda, one 32-row tile of one group per wave.
template <int DT, int D_S, int WIDTH, int NHID, int MODE>
__global__ __launch_bounds__(256) void pw_lik_kernel(PwParams p) {
    if constexpr (!net_compiled(DT, WIDTH)) {
        return;  // binary32 networks wider than 256 are refused at model creation
    } else {
    typedef Net<DT, WIDTH, NHID, in_slots(DT, D_S, 0, 0)> NTL;
    constexpr int SS = state_slots(D_S);
    extern __shared__ __attribute__((aligned(16))) char smem[];
    const int lane = threadIdx.x & 63, g = lane >> 5, col = lane & 31;
    const int wpb = blockDim.x >> 6;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const kconst int32_t* tiles = (const kconst int32_t*)p.tiles;
    const kconst int32_t* seg = (const kconst int32_t*)p.seg;
    const long n_units = tiles[p.M];
    with_weights<NTL, MODE, 1>(smem, p.lik, [&](auto& src, const NetPtrs& P) {
        // block-uniform loop (a streamed network's chunk barriers need every wave)
        for (long ub = blockIdx.x; ub * wpb < n_units; ub += gridDim.x) {
            const int u = (int)(ub * wpb + wave);
            const bool ok = u < n_units;
            // the group of this tile: the last m with tiles[m] <= u
            int a = 0, b = p.M;
            while (a < b) {
                const int mid = (a + b + 1) >> 1;
                if (tiles[mid] <= u) a = mid;
                else b = mid - 1;
            }
            const int m = ok ? a : 0;
            const int lo = seg[m], hi = seg[m + 1];
            const int j = ok ? lo + (u - tiles[m]) * 32 + col : 0;
            const bool valid = ok && j < hi;
            float slots[NTL::IN_SLOTS];
#pragma unroll
            for (int s = 0; s < NTL::IN_SLOTS; ++s) slots[s] = 0.0f;
#pragma unroll
            for (int s = 0; s < SS; ++s) {
                const int f = 2 * s + g;
                slots[s] = (valid && f < D_S) ? p.succ[(size_t)j * D_S + f] : 0.0f;
            }
            __builtin_amdgcn_s_waitcnt(waitcnt_vm_lgkm0(0));
            const f32x16 o = run_net<NTL>(src, P, p.b0_lik + (size_t)m * NTL::WIDTH, slots, lane, g);
            if (g == 0 && valid) {
                const float l = o[0];
                if (p.loglik) p.loglik[j] = l;
                if (!isfinite(l) && p.status) p.status[0] = 5;
                p.x[j] = (double)l / p.lambda;
            }
        }
    });
    }
}

// Weights, statistics and systematic resampling of every group, one
// workgroup per group (the single-belief procedure on the group's rows).
__global__ __launch_bounds__(kNormResThreads) void pw_norm_res_kernel(PwParams pw) {
    __shared__ double buf[kNormResMaxN];
    __shared__ int ids[kNormResMaxN];
    __shared__ double redd[kNRWaves];
    __shared__ int redi[kNRWaves];
    for (int m = blockIdx.x; m < pw.M; m += gridDim.x) {
        int lo, n;
        pw_group(pw, m, lo, n);
        if (n == 0) continue;
        int c = 0;
        while ((1 << c) < n) ++c;
        NormResParams p{};
        p.x = pw.x + lo;
        p.lambda = pw.lambda;
        p.N = n;
        p.bits = 52 - c < 32 ? 52 - c : 32;
        p.uniform_prior = 1;
        p.do_resample = 1;
        p.U = pw.U[m];
        p.w_out = pw.w ? pw.w + lo : nullptr;
        p.stats = pw.stats ? pw.stats + 2 * (size_t)m : nullptr;
        p.idx_out = pw.idx ? pw.idx + lo : nullptr;
        p.src = pw.succ_out ? pw.succ + (size_t)lo * pw.d_s : nullptr;
        p.dst = pw.succ_out ? pw.succ_out + (size_t)lo * pw.d_s : nullptr;
        p.row_floats = pw.d_s;
        p.status = pw.status;
        norm_res_body(p, buf, redd, redi, ids);
        __syncthreads();
    }
}

// Scores of all B x B pairs of a contrastive mini-batch: tile (i, jt) is
// state-action i against the 32 observations of column tile jt.  Row i's
// state and action sit in its folded first-layer bias row, which each wave
// copies into its own LDS row when the row changes; the observations are the
// network's input slots.
template <int DT, int D_O, int WIDTH, int NHID, int MODE>
__global__ __launch_bounds__(256) void nce_scores_kernel(NceParams p) {
    if constexpr (!net_compiled(DT, WIDTH)) {
        return;  // binary32 networks wider than 256 are refused at model creation
    } else {
    typedef Net<DT, WIDTH, NHID, in_slots(DT, D_O, 0, 0)> NTL;
    constexpr int SO = state_slots(D_O);
    extern __shared__ __attribute__((aligned(16))) char smem[];
    const int lane = threadIdx.x & 63, g = lane >> 5, col = lane & 31;
    const int wpb = blockDim.x >> 6;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int jtiles = (p.B + 31) / 32;
    const long n_units = (long)p.B * jtiles;
    float* rowb = reinterpret_cast<float*>(smem + p.row_bias_lds) + wave * NTL::WIDTH;
    constexpr int RB = NTL::WIDTH / 64;  // bias floats per lane
    static_assert(NTL::WIDTH % 64 == 0 && RB <= 16, "bias row copy: whole lanes");
    int have = -1;  // row held in this wave's LDS bias row
    with_weights<NTL, MODE, 1>(smem, p.lik, [&](auto& src, const NetPtrs& P) {
        // block-uniform loop (a streamed network's chunk barriers need every wave)
        for (long ub = blockIdx.x; ub * wpb < n_units; ub += gridDim.x) {
            const long u = ub * wpb + wave;
            const bool ok = u < n_units;
            const int i = ok ? (int)(u / jtiles) : 0;
            const int j = ok ? (int)(u - (long)i * jtiles) * 32 + col : 0;
            const bool valid = ok && j < p.B;
            float slots[NTL::IN_SLOTS];
#pragma unroll
            for (int s = 0; s < NTL::IN_SLOTS; ++s) slots[s] = 0.0f;
#pragma unroll
            for (int s = 0; s < SO; ++s) {
                const int f = 2 * s + g;
                slots[s] = (valid && f < D_O) ? p.obs[(size_t)j * D_O + f] : 0.0f;
            }
            const bool fresh = i != have;  // wave-uniform
            float bv[RB];
            if (fresh) {
                const float* brow = p.b0 + (size_t)i * NTL::WIDTH;
#pragma unroll
                for (int q = 0; q < RB; ++q) bv[q] = brow[q * 64 + lane];
            }
            __builtin_amdgcn_s_waitcnt(waitcnt_vm_lgkm0(0));
            if (fresh) {
#pragma unroll
                for (int q = 0; q < RB; ++q) rowb[q * 64 + lane] = bv[q];
                __builtin_amdgcn_s_waitcnt(waitcnt_vm_lgkm0(0));
                __builtin_amdgcn_wave_barrier();
                have = i;
            }
            const f32x16 o = run_net<NTL>(src, P, rowb, slots, lane, g);
            if (g == 0 && valid) {
                const float l = o[0];
                p.scores[(size_t)i * p.B + j] = l;
                if (!isfinite(l) && p.status) p.status[0] = 5;
            }
        }
    });
    }
}

// Row i of the objective, one workgroup per row in binary64:
// row_loss_i = m + log sum_j exp(l_ij - m) - l_ii with m = max_j l_ij, and
// grad_ij = (exp(l_ij - m) / sum - [i == j]) / B.
__global__ __launch_bounds__(kNormResThreads) void nce_rows_kernel(NceParams p) {
    __shared__ double red[kNRWaves];
    const int tid = threadIdx.x, B = p.B;
    for (int i = blockIdx.x; i < B; i += gridDim.x) {
        const float* l = p.scores + (size_t)i * B;
        double mx = -INFINITY;
        for (int j = tid; j < B; j += kNormResThreads) mx = fmax(mx, (double)l[j]);
        mx = block_max_d(mx, red);
        double sum = 0.0;
        for (int j = tid; j < B; j += kNormResThreads) sum += exp((double)l[j] - mx);
        sum = block_sum_d(sum, red);
        if (tid == 0) {
            if (!isfinite(mx) && p.status) p.status[0] = 5;
            p.row_loss[i] = mx + log(sum) - (double)l[i];
        }
        if (p.grad) {
            const double inv_b = 1.0 / (double)B;
            for (int j = tid; j < B; j += kNormResThreads)
                p.grad[(size_t)i * B + j] = (float)((exp((double)l[j] - mx) / sum - (j == i ? 1.0 : 0.0)) * inv_b);
        }
    }
}

// The mean of the B row losses (fixed-order sums).
__global__ __launch_bounds__(kNormResThreads) void nce_mean_kernel(NceParams p) {
    __shared__ double red[kNRWaves];
    double s = 0.0;
    for (int i = threadIdx.x; i < p.B; i += kNormResThreads) s += p.row_loss[i];
    s = block_sum_d(s, red);
    if (threadIdx.x == 0) p.loss[0] = s / (double)p.B;
}

// Cosine cumulative schedule, abar(0) = 1 (offset 0.008), clamped to [0, 1].
__device__ __forceinline__ double cosine_abar(double tau) {
    const double s = 0.008, h = 1.5707963267948966;
    const double c = cos(h * (tau + s) / (1.0 + s)), c0 = cos(h * s / (1.0 + s));
    const double a = (c * c) / (c0 * c0);
    return a < 0.0 ? 0.0 : (a > 1.0 ? 1.0 : a);
}

// Per-step first-layer biases (the action and tau_k = 1 - k/n folded in) and
// the step coefficients of the deterministic sampler: with a = abar(tau_k),
// a' = abar(tau_{k+1}), the v-prediction estimates x0 = sqrt(a) x - sqrt(1-a) v
// and eps = sqrt(1-a) x + sqrt(a) v re-noised to tau_{k+1} give
// x' = A x + B v, A = sqrt(a' a) + sqrt((1-a')(1-a)), B = sqrt((1-a') a) - sqrt(a' (1-a)).
// A - 1 is stored rather than A: with many steps A is within binary32
// resolution of 1, and x' = x + ((A - 1) x + B v) keeps its effect.
__global__ __launch_bounds__(256) void ddim_prep_kernel(DdimPrepParams p) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    for (int t = blockIdx.y; t < p.n_steps; t += gridDim.y) {
        const double tau = 1.0 - (double)t / p.n_steps, tau_n = 1.0 - (double)(t + 1) / p.n_steps;
        if (r < p.width) {
            float tf = (float)tau;
            if (p.bf16) tf = (float)(__bf16)tf;
            const int nf = p.aw + 1;
            float acc = p.b[r];
            for (int c = 0; c < p.aw; ++c) acc += p.w[(size_t)r * nf + c] * p.v[c];
            acc += p.w[(size_t)r * nf + p.aw] * tf;
            p.b0[(size_t)t * p.width + r] = acc;
        }
        if (r == 0) {
            const double a = cosine_abar(tau), an = cosine_abar(tau_n);
            p.coef[2 * t] = (float)((sqrt(an * a) + sqrt((1.0 - an) * (1.0 - a))) - 1.0);
            p.coef[2 * t + 1] = (float)(sqrt((1.0 - an) * a) - sqrt(an * (1.0 - a)));
        }
    }
}

// One 32-sample tile of the teacher sampler: x_tau in the state slots (the
// output tile's layout, so v updates it in place), the conditioning state in
// the noise slots, n_steps network evaluations.  Small networks run one tile
// per wave from LDS; deep wide networks are split over the block's four waves
// with the activations in LDS and the weights read from L2.
template <int DT, int D_X, int D_C, int WIDTH, int NHID, int MODE>
__global__ __launch_bounds__(256) void ddim_kernel(DdimParams p) {
    if constexpr (!net_compiled(DT, WIDTH)) {
        return;  // binary32 networks wider than 256 are refused at creation
    } else {
    constexpr bool SPLIT = MODE == kSplit;
    typedef Net<DT, WIDTH, NHID, in_slots(DT, D_X, 0, D_C), (SPLIT ? WIDTH / 32 : chunk_tiles(WIDTH))> NT;
    constexpr int SS = state_slots(D_X), SW = noise_slots(D_C);
    extern __shared__ __attribute__((aligned(16))) char smem[];
    const int lane = threadIdx.x & 63, g = lane >> 5, col = lane & 31;
    const int wpb = blockDim.x >> 6;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int n_tiles = (p.N + 31) / 32;
    const kconst float* coef = (const kconst float*)p.coef;
    // one tile: returns after writing (by `writer`) the final samples
    auto run_tile = [&](int tile, bool ok, bool writer, auto&& eval) {
        const int i = (ok ? tile : 0) * 32 + col;
        const bool valid = ok && i < p.N;
        float x[SS], cond[SW];
#pragma unroll
        for (int s = 0; s < SS; ++s) {
            const int f = 2 * s + g;
            x[s] = (valid && f < D_X) ? p.x1[(size_t)i * D_X + f] : 0.0f;
        }
#pragma unroll
        for (int s = 0; s < SW; ++s) {
            const int f = noise_feature(s, g);
            cond[s] = (valid && f < D_C) ? p.states[(size_t)i * D_C + f] : 0.0f;
        }
        __builtin_amdgcn_s_waitcnt(waitcnt_vm_lgkm0(0));
        for (int t = 0; t < p.n_steps; ++t) {
            float slots[NT::IN_SLOTS];
#pragma unroll
            for (int s = 0; s < NT::IN_SLOTS; ++s) slots[s] = 0.0f;
#pragma unroll
            for (int s = 0; s < SS; ++s) slots[s] = x[s];
#pragma unroll
            for (int s = 0; s < SW; ++s) slots[SS + s] = cond[s];
            const f32x16 v = eval(p.b0 + (size_t)t * WIDTH, slots);
            const float Am1 = coef[2 * t], B = coef[2 * t + 1];
#pragma unroll
            for (int s = 0; s < SS; ++s) x[s] += __builtin_fmaf(B, v[s], Am1 * x[s]);
        }
        if (writer && valid)
#pragma unroll
            for (int s = 0; s < SS; ++s)
                if (2 * s + g < D_X) p.out[(size_t)i * D_X + 2 * s + g] = x[s];
    };
    if constexpr (SPLIT) {
        return;  // deep wide networks run in ddim_split_kernel
    } else {
        with_weights<NT, MODE, 1>(smem, p.net, [&](auto& src, const NetPtrs& P) {
            // block-uniform loop (a streamed network's chunk barriers need every wave)
            for (long ub = blockIdx.x; ub * wpb < n_tiles; ub += gridDim.x) {
                const int tile = (int)(ub * wpb + wave);
                run_tile(tile, tile < n_tiles, true, [&](const float* b0, const float (&slots)[NT::IN_SLOTS]) {
                    return run_net<NT>(src, P, b0, slots, lane, g);
                });
            }
        });
    }
    }
}

// The teacher sampler for deep wide networks: a block of kDdimSplitWaves
// waves advances kDdimSplitTiles 32-sample tiles together, each layer split
// over the waves (run_net_split_multi), so that every weight fragment read
// from L2 serves all of the block's tiles.  Every wave keeps the tiles'
// samples; the first wave writes them.
#ifndef VOILA_DDIM_SPLIT_WAVES
#define VOILA_DDIM_SPLIT_WAVES 8
#endif
#ifndef VOILA_DDIM_SPLIT_TILES
#define VOILA_DDIM_SPLIT_TILES 2
#endif
#ifndef VOILA_DDIM_SPLIT_DEPTH
#define VOILA_DDIM_SPLIT_DEPTH 2
#endif
constexpr int kDdimSplitWaves = VOILA_DDIM_SPLIT_WAVES, kDdimSplitTiles = VOILA_DDIM_SPLIT_TILES,
              kDdimSplitDepth = VOILA_DDIM_SPLIT_DEPTH;
template <int DT, int D_X, int D_C, int WIDTH, int NHID>
__global__ __launch_bounds__(64 * kDdimSplitWaves) void ddim_split_kernel(DdimParams p) {
    if constexpr (!net_compiled(DT, WIDTH) || WIDTH <= 64) {
        return;  // small networks run one tile per wave in ddim_kernel
    } else {
    constexpr int ST = kDdimSplitTiles;
    typedef Net<DT, WIDTH, NHID, in_slots(DT, D_X, 0, D_C), WIDTH / 32> NT;
    constexpr int SS = state_slots(D_X), SW = noise_slots(D_C);
    extern __shared__ __attribute__((aligned(16))) char smem[];
    const int lane = threadIdx.x & 63, g = lane >> 5, col = lane & 31;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int n_groups = (p.N + 32 * ST - 1) / (32 * ST);
    const kconst float* coef = (const kconst float*)p.coef;
    const NetPtrs P = net_ptrs(p.net.base, p.net);
    for (int grp = blockIdx.x; grp < n_groups; grp += gridDim.x) {
        float x[ST][SS], cond[ST][SW];
        bool valid[ST];
        int row[ST];
#pragma unroll
        for (int st = 0; st < ST; ++st) {
            row[st] = (grp * ST + st) * 32 + col;
            valid[st] = row[st] < p.N;
#pragma unroll
            for (int s = 0; s < SS; ++s) {
                const int f = 2 * s + g;
                x[st][s] = (valid[st] && f < D_X) ? p.x1[(size_t)row[st] * D_X + f] : 0.0f;
            }
#pragma unroll
            for (int s = 0; s < SW; ++s) {
                const int f = noise_feature(s, g);
                cond[st][s] = (valid[st] && f < D_C) ? p.states[(size_t)row[st] * D_C + f] : 0.0f;
            }
        }
        __builtin_amdgcn_s_waitcnt(waitcnt_vm_lgkm0(0));
        for (int t = 0; t < p.n_steps; ++t) {
            float slots[ST][NT::IN_SLOTS];
#pragma unroll
            for (int st = 0; st < ST; ++st) {
#pragma unroll
                for (int s = 0; s < NT::IN_SLOTS; ++s) slots[st][s] = 0.0f;
#pragma unroll
                for (int s = 0; s < SS; ++s) slots[st][s] = x[st][s];
#pragma unroll
                for (int s = 0; s < SW; ++s) slots[st][SS + s] = cond[st][s];
            }
            f32x16 v[ST];
            run_net_split_multi<NT, ST, kDdimSplitWaves, kDdimSplitDepth>(P, p.b0 + (size_t)t * WIDTH, slots, v, lane, g, wave, smem);
            const float Am1 = coef[2 * t], B = coef[2 * t + 1];
#pragma unroll
            for (int st = 0; st < ST; ++st)
#pragma unroll
                for (int s = 0; s < SS; ++s) x[st][s] += __builtin_fmaf(B, v[st][s], Am1 * x[st][s]);
        }
        if (wave == 0)
#pragma unroll
            for (int st = 0; st < ST; ++st)
                if (valid[st])
#pragma unroll
                    for (int s = 0; s < SS; ++s)
                        if (2 * s + g < D_X) p.out[(size_t)row[st] * D_X + 2 * s + g] = x[st][s];
    }
    }
}

__global__ __launch_bounds__(256) void philox_kernel(PhiloxParams p) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= p.n) return;
    const int nb = (p.d + 3) / 4;
    for (int b = 0; b < nb; ++b) {
        uint4 w = philox4x32_10(make_uint4(p.c0 + (uint32_t)r, p.c1, p.c2, (p.stream << 16) | (uint32_t)b), p.key0,
                                p.key1);
        if (p.words) {
            uint32_t* o = p.words + ((size_t)r * nb + b) * 4;
            o[0] = w.x; o[1] = w.y; o[2] = w.z; o[3] = w.w;
        }
        float z[4];
        box_muller(w.x, w.y, z[0], z[1]);
        box_muller(w.z, w.w, z[2], z[3]);
        for (int j = 0; j < 4; ++j)
            if (4 * b + j < p.d) p.out[(size_t)r * p.d + 4 * b + j] = z[j];
    }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
namespace {

template <int W> constexpr bool lds_for_width() { return W <= 64; }
// weight access of the rollout kernel and of the single-pass kernels
template <int W> constexpr int plan_mode() { return W <= 64 ? kResident : kStream; }
template <int W> constexpr int pass_mode() { return W <= 64 ? kResident : W <= 256 ? kSplit : kDirect; }
constexpr size_t kStreamLds = (size_t)VOILA_STREAM_NBUF * VOILA_STREAM_CHB;

}  // namespace

bool weights_in_lds(int shape) { return kShapeInfo[shape].width <= 64; }

#define VOILA_IN_SLOTS(fn, expr)                                                                   \
    int fn(int shape, int dt) {                                                                     \
        const ShapeInfo& s = kShapeInfo[shape];                                                     \
        (void)s;                                                                                    \
        return expr;                                                                                \
    }
VOILA_IN_SLOTS(plan_in_slots, in_slots(dt, s.d_s, s.n_actions > 0 ? 0 : s.d_a, s.d_w))
VOILA_IN_SLOTS(update_in_slots, in_slots(dt, s.d_s, 0, s.d_w))
VOILA_IN_SLOTS(obs_in_slots, in_slots(dt, s.d_s, 0, s.d_wz))
VOILA_IN_SLOTS(lik_in_slots, in_slots(dt, s.d_s, 0, 0))
VOILA_IN_SLOTS(nce_in_slots, in_slots(dt, s.d_o, 0, 0))
#undef VOILA_IN_SLOTS

#define PLAN_K(id, ds, na, da, dw, dox, dwz, w, nh, DT) plan_kernel<DT, ds, na, da, dw, w, nh, plan_mode<w>()>

// LDS of a streaming rollout kernel before its staged biases: the two chunk
// buffers (and the first layer of a grouped wide network).
template <int DT, int D_S, int N_ACT, int D_AIN, int D_W, int WIDTH, int NHID>
constexpr size_t stream_lds_of() {
    if constexpr (!net_compiled(DT, WIDTH) || WIDTH <= 64) {
        return kStreamLds;
    } else {
        typedef Net<DT, WIDTH, NHID, in_slots(DT, D_S, D_AIN, D_W)> NT;
        return (size_t)StreamChunk<NT>::BYTES +
               (NT::CT < NT::HT && first_layer_in_lds<NT>(N_ACT > 0 ? N_ACT : 1) ? (size_t)NT::NF0 * NT::FRAG_BYTES
                                                                                : 0);
    }
}
size_t plan_stream_lds(int shape, int dt) {
    switch (shape * 2 + dt) {
#define X(id, ds, na, da, dw, dox, dwz, w, nh)                                      \
    case id * 2 + 0:                                                               \
        return stream_lds_of<DT_F32, ds, na, (na > 0 ? 0 : da), dw, w, nh>();            \
    case id * 2 + 1:                                                               \
        return stream_lds_of<DT_BF16, ds, na, (na > 0 ? 0 : da), dw, w, nh>();
        VOILA_SHAPES(X)
#undef X
    }
    return kStreamLds;
}
#define PROP_K(id, ds, na, da, dw, dox, dwz, w, nh, DT) propose_kernel<DT, ds, dw, w, nh, pass_mode<w>()>
#define OBS_K(id, ds, na, da, dw, dox, dwz, w, nh, DT) observe_kernel<DT, ds, dwz, dox, w, nh, pass_mode<w>()>

hipError_t launch_plan(int shape, int dt, const PlanParams& p, int blocks, hipStream_t s) {
    size_t lds = weights_in_lds(shape) ? p.net.bytes : plan_stream_lds(shape, dt) + (p.net.bytes - p.net.off_b0);
    switch (shape * 2 + dt) {
#define X(id, ds, na, da, dw, dox, dwz, w, nh)                                                              \
    case id * 2 + 0:                                                                                       \
        if (lds > 65536)                                                                                   \
            (void)hipFuncSetAttribute((const void*)PLAN_K(id, ds, na, da, dw, dox, dwz, w, nh, DT_F32),     \
                                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);               \
        hipLaunchKernelGGL((PLAN_K(id, ds, na, da, dw, dox, dwz, w, nh, DT_F32)), blocks, 256, lds, s, p);  \
        break;                                                                                             \
    case id * 2 + 1:                                                                                       \
        if (lds > 65536)                                                                                   \
            (void)hipFuncSetAttribute((const void*)PLAN_K(id, ds, na, da, dw, dox, dwz, w, nh, DT_BF16),    \
                                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);               \
        hipLaunchKernelGGL((PLAN_K(id, ds, na, da, dw, dox, dwz, w, nh, DT_BF16)), blocks, 256, lds, s, p); \
        break;
        VOILA_SHAPES(X)
#undef X
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// Split-mode passes (one tile per block, LDS for activations and partials).
bool pass_split(int shape) { return kShapeInfo[shape].width > 64 && kShapeInfo[shape].width <= 256; }
int pass_tiles_per_block(int shape) { return pass_split(shape) ? 1 : 4; }
constexpr size_t kSplitLds = 48 * 1024;  // binary32 width 256: 32 KB activations + 16 KB partials

hipError_t launch_propose(int shape, int dt, const ProposeParams& p, int blocks, hipStream_t s) {
    const size_t lds = weights_in_lds(shape) ? (size_t)p.trans.bytes + p.lik.bytes : pass_split(shape) ? kSplitLds : 0;
    switch (shape * 2 + dt) {
#define X(id, ds, na, da, dw, dox, dwz, w, nh)                                                              \
    case id * 2 + 0:                                                                                       \
        hipLaunchKernelGGL((PROP_K(id, ds, na, da, dw, dox, dwz, w, nh, DT_F32)), blocks, 256, lds, s, p);  \
        break;                                                                                             \
    case id * 2 + 1:                                                                                       \
        hipLaunchKernelGGL((PROP_K(id, ds, na, da, dw, dox, dwz, w, nh, DT_BF16)), blocks, 256, lds, s, p); \
        break;
        VOILA_SHAPES(X)
#undef X
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_observe(int shape, int dt, const ObserveParams& p, int blocks, hipStream_t s) {
    const size_t lds = weights_in_lds(shape) ? p.obs.bytes : pass_split(shape) ? kSplitLds : 0;
    switch (shape * 2 + dt) {
#define X(id, ds, na, da, dw, dox, dwz, w, nh)                                                             \
    case id * 2 + 0:                                                                                      \
        hipLaunchKernelGGL((OBS_K(id, ds, na, da, dw, dox, dwz, w, nh, DT_F32)), blocks, 256, lds, s, p);  \
        break;                                                                                            \
    case id * 2 + 1:                                                                                      \
        hipLaunchKernelGGL((OBS_K(id, ds, na, da, dw, dox, dwz, w, nh, DT_BF16)), blocks, 256, lds, s, p); \
        break;
        VOILA_SHAPES(X)
#undef X
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

#define OBSR_K(id, ds, na, da, dw, dox, dwz, w, nh, DT) observe_kernel<DT, ds, dwz, dox, w, nh, plan_mode<w>()>

size_t observe_rollout_lds(int shape, int dt, const NetBlob& obs) {
    if (weights_in_lds(shape)) return obs.bytes;
    size_t chunks = kStreamLds;
    switch (shape * 2 + dt) {
#define X(id, ds, na, da, dw, dox, dwz, w, nh)                       \
    case id * 2 + 0:                                                \
        chunks = stream_lds_of<DT_F32, ds, 0, 0, dwz, w, nh>();     \
        break;                                                      \
    case id * 2 + 1:                                                \
        chunks = stream_lds_of<DT_BF16, ds, 0, 0, dwz, w, nh>();    \
        break;
        VOILA_SHAPES(X)
#undef X
    }
    return chunks + (obs.bytes - obs.off_b0);
}

hipError_t launch_observe_rollouts(int shape, int dt, const ObserveParams& p0, int blocks, hipStream_t s) {
    ObserveParams p = p0;
    size_t lds = observe_rollout_lds(shape, dt, p.obs);
    if (!weights_in_lds(shape)) {
        // one first-layer bias row per wave after the stream buffers and staged biases
        lds = (lds + 15) / 16 * 16;
        p.row_bias_lds = (uint32_t)lds;
        lds += (size_t)kWavesPerBlock * kShapeInfo[shape].width * 4;
    }
    switch (shape * 2 + dt) {
#define X(id, ds, na, da, dw, dox, dwz, w, nh)                                                                \
    case id * 2 + 0:                                                                                         \
        if (lds > 65536)                                                                                     \
            (void)hipFuncSetAttribute((const void*)OBSR_K(id, ds, na, da, dw, dox, dwz, w, nh, DT_F32),       \
                                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);                 \
        hipLaunchKernelGGL((OBSR_K(id, ds, na, da, dw, dox, dwz, w, nh, DT_F32)), blocks, 256, lds, s, p);    \
        break;                                                                                               \
    case id * 2 + 1:                                                                                         \
        if (lds > 65536)                                                                                     \
            (void)hipFuncSetAttribute((const void*)OBSR_K(id, ds, na, da, dw, dox, dwz, w, nh, DT_BF16),      \
                                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);                 \
        hipLaunchKernelGGL((OBSR_K(id, ds, na, da, dw, dox, dwz, w, nh, DT_BF16)), blocks, 256, lds, s, p);   \
        break;
        VOILA_SHAPES(X)
#undef X
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

namespace {
template <class KernelT>
int occupancy(KernelT k, size_t lds) {
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k, 256, lds) != hipSuccess || n < 1) n = 1;
    return n;
}
template <class KernelT>
int occupancy_t(KernelT k, int threads, size_t lds) {
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k, threads, lds) != hipSuccess || n < 1) n = 1;
    return n;
}
// LDS bytes assumed for occupancy: the blob sizes of the small shape are a few tens of KB.
constexpr size_t kLdsGuess = 32 * 1024;
}  // namespace

int plan_blocks_per_cu(int shape, int dt) {
    switch (shape * 2 + dt) {
#define X(id, ds, na, da, dw, dox, dwz, w, nh)                                                               \
    case id * 2 + 0:                                                                                        \
        return occupancy(PLAN_K(id, ds, na, da, dw, dox, dwz, w, nh, DT_F32), lds_for_width<w>() ? kLdsGuess : kStreamLds); \
    case id * 2 + 1:                                                                                        \
        return occupancy(PLAN_K(id, ds, na, da, dw, dox, dwz, w, nh, DT_BF16), lds_for_width<w>() ? kLdsGuess : kStreamLds);
        VOILA_SHAPES(X)
#undef X
    }
    return 1;
}
int propose_blocks_per_cu(int shape, int dt) {
    switch (shape * 2 + dt) {
#define X(id, ds, na, da, dw, dox, dwz, w, nh)                                                                   \
    case id * 2 + 0:                                                                                            \
        return occupancy(PROP_K(id, ds, na, da, dw, dox, dwz, w, nh, DT_F32), lds_for_width<w>() ? 2 * kLdsGuess : kSplitLds); \
    case id * 2 + 1:                                                                                            \
        return occupancy(PROP_K(id, ds, na, da, dw, dox, dwz, w, nh, DT_BF16), lds_for_width<w>() ? 2 * kLdsGuess : kSplitLds);
        VOILA_SHAPES(X)
#undef X
    }
    return 1;
}
int observe_blocks_per_cu(int shape, int dt) {
    switch (shape * 2 + dt) {
#define X(id, ds, na, da, dw, dox, dwz, w, nh)                                                              \
    case id * 2 + 0:                                                                                       \
        return occupancy(OBS_K(id, ds, na, da, dw, dox, dwz, w, nh, DT_F32), lds_for_width<w>() ? kLdsGuess : kSplitLds); \
    case id * 2 + 1:                                                                                       \
        return occupancy(OBS_K(id, ds, na, da, dw, dox, dwz, w, nh, DT_BF16), lds_for_width<w>() ? kLdsGuess : kSplitLds);
        VOILA_SHAPES(X)
#undef X
    }
    return 1;
}

#define PWL_K(id, ds, na, da, dw, dox, dwz, w, nh, DT) pw_lik_kernel<DT, ds, w, nh, plan_mode<w>()>

hipError_t launch_pw_lik(int shape, int dt, const PwParams& p, int blocks, hipStream_t s) {
    size_t lds = p.lik.bytes;
    if (!weights_in_lds(shape)) {
        switch (shape * 2 + dt) {
#define X(id, ds, na, da, dw, dox, dwz, w, nh)                           \
    case id * 2 + 0:                                                    \
        lds = stream_lds_of<DT_F32, ds, 0, 0, 0, w, nh>();              \
        break;                                                          \
    case id * 2 + 1:                                                    \
        lds = stream_lds_of<DT_BF16, ds, 0, 0, 0, w, nh>();             \
        break;
            VOILA_SHAPES(X)
#undef X
        }
        lds += p.lik.bytes - p.lik.off_b0;
    }
    switch (shape * 2 + dt) {
#define X(id, ds, na, da, dw, dox, dwz, w, nh)                                                                \
    case id * 2 + 0:                                                                                         \
        if (lds > 65536)                                                                                     \
            (void)hipFuncSetAttribute((const void*)PWL_K(id, ds, na, da, dw, dox, dwz, w, nh, DT_F32),        \
                                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);                 \
        hipLaunchKernelGGL((PWL_K(id, ds, na, da, dw, dox, dwz, w, nh, DT_F32)), blocks, 256, lds, s, p);     \
        break;                                                                                               \
    case id * 2 + 1:                                                                                         \
        if (lds > 65536)                                                                                     \
            (void)hipFuncSetAttribute((const void*)PWL_K(id, ds, na, da, dw, dox, dwz, w, nh, DT_BF16),       \
                                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);                 \
        hipLaunchKernelGGL((PWL_K(id, ds, na, da, dw, dox, dwz, w, nh, DT_BF16)), blocks, 256, lds, s, p);    \
        break;
        VOILA_SHAPES(X)
#undef X
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

int pw_lik_blocks_per_cu(int shape, int dt) {
    switch (shape * 2 + dt) {
#define X(id, ds, na, da, dw, dox, dwz, w, nh)                                                               \
    case id * 2 + 0:                                                                                        \
        return occupancy(PWL_K(id, ds, na, da, dw, dox, dwz, w, nh, DT_F32), lds_for_width<w>() ? kLdsGuess : kStreamLds); \
    case id * 2 + 1:                                                                                        \
        return occupancy(PWL_K(id, ds, na, da, dw, dox, dwz, w, nh, DT_BF16), lds_for_width<w>() ? kLdsGuess : kStreamLds);
        VOILA_SHAPES(X)
#undef X
    }
    return 1;
}

#define NCE_K(id, ds, na, da, dw, dox, dwz, w, nh, DT) nce_scores_kernel<DT, dox, w, nh, plan_mode<w>()>

hipError_t launch_nce_scores(int shape, int dt, const NceParams& p0, int blocks, hipStream_t s) {
    NceParams p = p0;
    size_t lds = p.lik.bytes;
    if (!weights_in_lds(shape)) {
        switch (shape * 2 + dt) {
#define X(id, ds, na, da, dw, dox, dwz, w, nh)                           \
    case id * 2 + 0:                                                    \
        lds = stream_lds_of<DT_F32, dox, 0, 0, 0, w, nh>();             \
        break;                                                          \
    case id * 2 + 1:                                                    \
        lds = stream_lds_of<DT_BF16, dox, 0, 0, 0, w, nh>();            \
        break;
            VOILA_SHAPES(X)
#undef X
        }
        lds += p.lik.bytes - p.lik.off_b0;
    }
    // one first-layer bias row per wave after the staged weights and biases
    lds = (lds + 15) / 16 * 16;
    p.row_bias_lds = (uint32_t)lds;
    lds += (size_t)kWavesPerBlock * shape_info(shape).width * 4;
    switch (shape * 2 + dt) {
#define X(id, ds, na, da, dw, dox, dwz, w, nh)                                                                \
    case id * 2 + 0:                                                                                         \
        if (lds > 65536)                                                                                     \
            (void)hipFuncSetAttribute((const void*)NCE_K(id, ds, na, da, dw, dox, dwz, w, nh, DT_F32),        \
                                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);                 \
        hipLaunchKernelGGL((NCE_K(id, ds, na, da, dw, dox, dwz, w, nh, DT_F32)), blocks, 256, lds, s, p);     \
        break;                                                                                               \
    case id * 2 + 1:                                                                                         \
        if (lds > 65536)                                                                                     \
            (void)hipFuncSetAttribute((const void*)NCE_K(id, ds, na, da, dw, dox, dwz, w, nh, DT_BF16),       \
                                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);                 \
        hipLaunchKernelGGL((NCE_K(id, ds, na, da, dw, dox, dwz, w, nh, DT_BF16)), blocks, 256, lds, s, p);    \
        break;
        VOILA_SHAPES(X)
#undef X
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

int nce_scores_blocks_per_cu(int shape, int dt) {
    switch (shape * 2 + dt) {
#define X(id, ds, na, da, dw, dox, dwz, w, nh)                                                               \
    case id * 2 + 0:                                                                                        \
        return occupancy(NCE_K(id, ds, na, da, dw, dox, dwz, w, nh, DT_F32), lds_for_width<w>() ? kLdsGuess : kStreamLds); \
    case id * 2 + 1:                                                                                        \
        return occupancy(NCE_K(id, ds, na, da, dw, dox, dwz, w, nh, DT_BF16), lds_for_width<w>() ? kLdsGuess : kStreamLds);
        VOILA_SHAPES(X)
#undef X
    }
    return 1;
}

hipError_t launch_nce_rows(const NceParams& p, int blocks, hipStream_t s) {
    if (p.B == 0) return hipSuccess;
    hipLaunchKernelGGL(nce_rows_kernel, blocks, kNormResThreads, 0, s, p);
    return hipGetLastError();
}

hipError_t launch_nce_mean(const NceParams& p, hipStream_t s) {
    if (p.B == 0 || !p.loss) return hipSuccess;
    hipLaunchKernelGGL(nce_mean_kernel, 1, kNormResThreads, 0, s, p);
    return hipGetLastError();
}

template <int W> constexpr int ddim_mode() { return W <= 64 ? kResident : kSplit; }
#define DDIM_K(id, dx, dc, w, nh, DT) ddim_kernel<DT, dx, dc, w, nh, ddim_mode<w>()>
#define DDIM_SK(id, dx, dc, w, nh, DT) ddim_split_kernel<DT, dx, dc, w, nh>

int ddim_shape(int d_x, int d_c, int width, int n_hidden) {
#define X(id, dx, dc, w, nh) \
    if (d_x == dx && d_c == dc && width == w && n_hidden == nh) return id;
    VOILA_DDIM_SHAPES(X)
#undef X
    return -1;
}
int ddim_in_slots(int shape, int dt) {
    switch (shape) {
#define X(id, dx, dc, w, nh) \
    case id:                 \
        return in_slots(dt, dx, 0, dc);
        VOILA_DDIM_SHAPES(X)
#undef X
    }
    return 0;
}
bool ddim_split(int shape) {
    switch (shape) {
#define X(id, dx, dc, w, nh) \
    case id:                 \
        return ddim_mode<w>() == kSplit;
        VOILA_DDIM_SHAPES(X)
#undef X
    }
    return false;
}

template <int DT, int D_X, int D_C, int W, int NH>
constexpr size_t ddim_split_lds() {
    if constexpr (!net_compiled(DT, W)) {
        return 0;
    } else {
        return (size_t)kDdimSplitTiles * SplitLds<Net<DT, W, NH, in_slots(DT, D_X, 0, D_C), W / 32>>::ACT;
    }
}
int ddim_tiles_per_block(int shape) { return ddim_split(shape) ? kDdimSplitTiles : kWavesPerBlock; }

hipError_t launch_ddim_prep(const DdimPrepParams& p, hipStream_t s) {
    if (p.n_steps == 0) return hipSuccess;
    hipLaunchKernelGGL(ddim_prep_kernel, dim3((p.width + 255) / 256, p.n_steps < 65535 ? p.n_steps : 65535), 256,
                       0, s, p);
    return hipGetLastError();
}

template <class K>
void launch_ddim_one(K k, bool split, size_t lds, int blocks, const DdimParams& p, hipStream_t s) {
    if (lds > 65536) (void)hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL(k, blocks, split ? 64 * kDdimSplitWaves : 256, lds, s, p);
}

hipError_t launch_ddim(int shape, int dt, const DdimParams& p, int blocks, hipStream_t s) {
    switch (shape * 2 + dt) {
#define X(id, dx, dc, w, nh)                                                                                       \
    case id * 2 + 0:                                                                                          \
        if (ddim_mode<w>() == kSplit)                                                                         \
            launch_ddim_one(DDIM_SK(id, dx, dc, w, nh, DT_F32), true, ddim_split_lds<DT_F32, dx, dc, w, nh>(), blocks, p, s); \
        else                                                                                                  \
            launch_ddim_one(DDIM_K(id, dx, dc, w, nh, DT_F32), false, p.net.bytes, blocks, p, s);                  \
        break;                                                                                                \
    case id * 2 + 1:                                                                                          \
        if (ddim_mode<w>() == kSplit)                                                                         \
            launch_ddim_one(DDIM_SK(id, dx, dc, w, nh, DT_BF16), true, ddim_split_lds<DT_BF16, dx, dc, w, nh>(), blocks, p, s); \
        else                                                                                                  \
            launch_ddim_one(DDIM_K(id, dx, dc, w, nh, DT_BF16), false, p.net.bytes, blocks, p, s);                 \
        break;
        VOILA_DDIM_SHAPES(X)
#undef X
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

int ddim_blocks_per_cu(int shape, int dt) {
    switch (shape * 2 + dt) {
#define X(id, dx, dc, w, nh)                                                                                    \
    case id * 2 + 0:                                                                                       \
        return ddim_mode<w>() == kSplit                                                                    \
                   ? occupancy_t(DDIM_SK(id, dx, dc, w, nh, DT_F32), 64 * kDdimSplitWaves,                     \
                                 ddim_split_lds<DT_F32, dx, dc, w, nh>())                                      \
                   : occupancy(DDIM_K(id, dx, dc, w, nh, DT_F32), kLdsGuess);                                  \
    case id * 2 + 1:                                                                                       \
        return ddim_mode<w>() == kSplit                                                                    \
                   ? occupancy_t(DDIM_SK(id, dx, dc, w, nh, DT_BF16), 64 * kDdimSplitWaves,                    \
                                 ddim_split_lds<DT_BF16, dx, dc, w, nh>())                                     \
                   : occupancy(DDIM_K(id, dx, dc, w, nh, DT_BF16), kLdsGuess);
        VOILA_DDIM_SHAPES(X)
#undef X
    }
    return 1;
}

int observe_rollout_blocks_per_cu(int shape, int dt) {
    switch (shape * 2 + dt) {
#define X(id, ds, na, da, dw, dox, dwz, w, nh)                                                               \
    case id * 2 + 0:                                                                                        \
        return occupancy(OBSR_K(id, ds, na, da, dw, dox, dwz, w, nh, DT_F32), lds_for_width<w>() ? kLdsGuess : kStreamLds); \
    case id * 2 + 1:                                                                                        \
        return occupancy(OBSR_K(id, ds, na, da, dw, dox, dwz, w, nh, DT_BF16), lds_for_width<w>() ? kLdsGuess : kStreamLds);
        VOILA_SHAPES(X)
#undef X
    }
    return 1;
}

#define PLANB_K(id, ds, na, da, dw, dox, dwz, w, nh, DT) plan_batch_kernel<DT, ds, na, da, dw, w, nh>
#define PROPB_K(id, ds, na, da, dw, dox, dwz, w, nh, DT) propose_batch_kernel<DT, ds, dw, w, nh>

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

hipError_t launch_propose_batch(int shape, int dt, const BatchProposeParams& p, int blocks, int wpb, size_t lds,
                                hipStream_t s) {
    if (!weights_in_lds(shape)) return hipErrorInvalidValue;
    switch (shape * 2 + dt) {
#define X(id, ds, na, da, dw, dox, dwz, w, nh)                                                                     \
    case id * 2 + 0:                                                                                              \
        hipLaunchKernelGGL((PROPB_K(id, ds, na, da, dw, dox, dwz, w, nh, DT_F32)), blocks, 64 * wpb, lds, s, p);   \
        break;                                                                                                    \
    case id * 2 + 1:                                                                                              \
        hipLaunchKernelGGL((PROPB_K(id, ds, na, da, dw, dox, dwz, w, nh, DT_BF16)), blocks, 64 * wpb, lds, s, p);  \
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

int propose_batch_blocks_per_cu(int shape, int dt, int wpb, size_t lds) {
    switch (shape * 2 + dt) {
#define X(id, ds, na, da, dw, dox, dwz, w, nh)                                                        \
    case id * 2 + 0:                                                                                 \
        return occupancy_t(PROPB_K(id, ds, na, da, dw, dox, dwz, w, nh, DT_F32), 64 * wpb, lds);      \
    case id * 2 + 1:                                                                                 \
        return occupancy_t(PROPB_K(id, ds, na, da, dw, dox, dwz, w, nh, DT_BF16), 64 * wpb, lds);
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

hipError_t launch_fold_batch(const FoldBatchItem* d_items, int n_items, int max_width, const void* d_actions,
                             const float* d_obs, int32_t* d_status, hipStream_t s) {
    if (n_items == 0) return hipSuccess;
    hipLaunchKernelGGL(fold_batch_kernel, dim3((max_width + 255) / 256, n_items), 256, 0, s, d_items, d_actions, d_obs,
                       d_status);
    return hipGetLastError();
}

hipError_t launch_norm_res_batch(const NormResParams* d_ps, int n_inst, const uint32_t* d_u, int32_t* d_status,
                                 hipStream_t s) {
    if (n_inst == 0) return hipSuccess;
    hipLaunchKernelGGL(norm_res_batch_kernel, n_inst, kNormResThreads, 0, s, d_ps, d_u, d_status);
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

hipError_t launch_fold(const FoldParams& p, hipStream_t s) {
    hipLaunchKernelGGL(fold_kernel, (p.width + 255) / 256, 256, 0, s, p);
    return hipGetLastError();
}

hipError_t launch_fold_steps(const FoldStepsParams& p, hipStream_t s) {
    if (p.rows == 0) return hipSuccess;
    hipLaunchKernelGGL(fold_steps_kernel, dim3((p.width + 255) / 256, p.rows < 65535 ? p.rows : 65535), 256, 0, s, p);
    return hipGetLastError();
}

hipError_t launch_tree_groups(const TreeParams& p, hipStream_t s) {
    const int M = p.A * p.n_obs;
    const long n_el = (long)M * p.N * p.d_s;
    long blocks = (n_el + 255) / 256;
    if (blocks < (M + 1 + 255) / 256) blocks = (M + 1 + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(tree_groups_kernel, (int)blocks, 256, 0, s, p);
    return hipGetLastError();
}

hipError_t launch_tree_child_q(const TreeParams& p, hipStream_t s) {
    const long items = (long)p.A * p.n_obs * p.K;
    hipLaunchKernelGGL(tree_child_q_kernel, (int)((items + 3) / 4), 256, 0, s, p);
    return hipGetLastError();
}

hipError_t launch_tree_backup(const TreeParams& p, hipStream_t s) {
    hipLaunchKernelGGL(tree_backup_kernel, (p.A + 63) / 64, 64, 0, s, p);
    return hipGetLastError();
}

hipError_t launch_soft_value(const SoftValueParams& p, int blocks, hipStream_t s) {
    if (p.M == 0 || blocks == 0) return hipSuccess;
    hipLaunchKernelGGL(soft_value_kernel, blocks, kSoftThreads, 0, s, p);
    return hipGetLastError();
}

hipError_t launch_pw_first(const PwParams& p, hipStream_t s) {
    const int n = p.M * p.d_s;
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(pw_first_kernel, (n + 255) / 256, 256, 0, s, p);
    return hipGetLastError();
}

hipError_t launch_pw_branch(const PwParams& p, hipStream_t s) {
    if (p.M == 0) return hipSuccess;
    hipLaunchKernelGGL(pw_branch_kernel, (p.M + 255) / 256, 256, 0, s, p);
    return hipGetLastError();
}

hipError_t launch_pw_tiles(const PwParams& p, hipStream_t s) {
    hipLaunchKernelGGL(pw_tiles_kernel, 1, 1024, 0, s, p);
    return hipGetLastError();
}

hipError_t launch_pw_norm_res(const PwParams& p, int blocks, hipStream_t s) {
    if (p.M == 0 || blocks == 0) return hipSuccess;
    hipLaunchKernelGGL(pw_norm_res_kernel, blocks, kNormResThreads, 0, s, p);
    return hipGetLastError();
}

hipError_t launch_norm_res(const NormResParams& p, hipStream_t s) {
    hipLaunchKernelGGL(norm_res_kernel, 1, kNormResThreads, 0, s, p);
    return hipGetLastError();
}

hipError_t launch_philox(const PhiloxParams& p, hipStream_t s) {
    if (p.n == 0) return hipSuccess;
    hipLaunchKernelGGL(philox_kernel, (p.n + 255) / 256, 256, 0, s, p);
    return hipGetLastError();
}

}  // namespace voila
