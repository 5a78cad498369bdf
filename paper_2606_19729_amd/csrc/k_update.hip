// k_update.hip -- the belief update: action/observation folds, proposal and
// likelihood (update stage 1), single-workgroup normalisation and systematic
// resampling (stage 2), their batched forms, and the counter-based noise hook.
#include "kcommon.hpp"

namespace voila {

const ShapeInfo& shape_info(int shape) { return kShapeInfo[shape]; }

// First-layer biases with the action (then the observation) of every row
// folded in: the first layer's weight columns of those inputs times their
// values (a one-hot action selects its column), added to the bias.  Inputs are
// read from device memory; a discrete action outside [0, n_actions) or a
// non-finite action or observation value sets the status word to
// VOILA_ERR_INVALID_ARG (an out-of-range action is then taken as action 0).
__global__ __launch_bounds__(256) void fold_steps_kernel(FoldStepsParams p) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= p.width) return;
    for (int j = blockIdx.y; j < p.rows; j += gridDim.y) {
        float acc = p.b[r];
        bool bad = false;
        if (p.n_actions > 0) {
            int a = reinterpret_cast<const int32_t*>(p.cands)[j];
            if (a < 0 || a >= p.n_actions) {
                bad = true;
                a = 0;
            }
            for (int c = 0; c < p.n_actions; ++c) acc += p.w[(size_t)r * p.nf + c] * (c == a ? 1.0f : 0.0f);
        } else {
            const float* ac = reinterpret_cast<const float*>(p.cands) + (size_t)j * p.d_a;
            for (int c = 0; c < p.d_a; ++c) {
                float v = ac[c];
                bad |= !isfinite(v);
                if (p.bf16) v = (float)(__bf16)v;
                acc += p.w[(size_t)r * p.nf + c] * v;
            }
        }
        if (p.obs) {
            const int c0 = p.n_actions > 0 ? p.n_actions : p.d_a;
            const float* ob = p.obs + (size_t)j * p.d_o;
            for (int c = 0; c < p.d_o; ++c) {
                float v = ob[c];
                bad |= !isfinite(v);
                if (p.bf16) v = (float)(__bf16)v;
                acc += p.w[(size_t)r * p.nf + c0 + c] * v;
            }
        }
        if (bad && p.status && r == 0) p.status[0] = 1;
        p.out[(size_t)j * p.width + r] = acc;
    }
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
    if constexpr (!generic_compiled(DT, WIDTH, NHID)) {
        return;  // refused at model creation (binary32 wider than 256) or run by the split rollout kernel
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

// Proposals of models whose transition network runs in the split evaluation
// (more than two hidden layers wider than 256): a block of kPropSplitWaves
// waves advances two 32-particle tiles, every layer split over the waves
// (run_net_split_owned); wave q forms tile q's inputs [s, w] (noise as in
// propose_tile) and writes its proposals s + f_T(s, a, w).
constexpr int kPropSplitWaves = 8, kPropSplitDepth = 2;

template <int DT, int D_S, int D_W, int WIDTH, int NHID>
__global__ __launch_bounds__(64 * kPropSplitWaves) void propose_split_kernel(ProposeParams p) {
    if constexpr (!net_compiled(DT, WIDTH) || generic_compiled(DT, WIDTH, NHID)) {
        return;  // the other networks run in propose_kernel
    } else {
    constexpr int ST = kPropSplitTiles, SS = state_slots(D_S), SW = noise_slots(D_W), NO = cdiv(D_S, 32);
    typedef Net<DT, WIDTH, NHID, in_slots(DT, D_S, 0, D_W), WIDTH / 32, NO> NT;
    extern __shared__ __attribute__((aligned(16))) char smem[];
    char* const in_lds = smem + ST * SplitLds<NT>::ACT;
    const int lane = threadIdx.x & 63, g = lane >> 5, col = lane & 31;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const bool owner = wave < ST;
    const int n_groups = ((p.N + 31) / 32 + ST - 1) / ST;
    const NetPtrs P = net_ptrs(p.trans.base, p.trans);
    for (int u = blockIdx.x; u < n_groups; u += gridDim.x) {
        const int i = (u * ST + (owner ? wave : 0)) * 32 + col;
        const bool valid = owner && i < p.N;
        if (owner) {
            float slots[NT::IN_SLOTS];
#pragma unroll
            for (int s = 0; s < NT::IN_SLOTS; ++s) slots[s] = 0.0f;
#pragma unroll
            for (int s = 0; s < SS; ++s) {
                const int f = 2 * s + g;
                slots[s] = (valid && f < D_S) ? p.states[(size_t)i * D_S + f] : 0.0f;
            }
            if (p.noise) {
#pragma unroll
                for (int s = 0; s < SW; ++s) {
                    const int f = noise_feature(s, g);
                    slots[SS + s] = (valid && f < D_W) ? p.noise[(size_t)i * D_W + f] : 0.0f;
                }
            } else {
                float nz[SW];
                noise_slots_philox<SW>(nz, p.key0, p.key1, (uint32_t)i, 0u, 0u, 5u, g);
#pragma unroll
                for (int s = 0; s < SW; ++s) slots[SS + s] = nz[s];
            }
            split_stage_inputs<NT>(in_lds + wave * SplitIn<NT>::BYTES, slots, lane);
        }
        __syncthreads();  // the owners' inputs are in LDS
        float d[NO][16];
        run_net_split_owned<NT, ST, kPropSplitWaves, kPropSplitDepth>(P, p.b0_trans, in_lds, d, lane, g, wave, smem);
        if (valid)
#pragma unroll
            for (int s = 0; s < SS; ++s) {
                const int f = 2 * s + g;
                if (f < D_S) p.prop[(size_t)i * D_S + f] = p.states[(size_t)i * D_S + f] + d[s / 16][s % 16];
            }
    }
    }
}

// The likelihood of the proposals for those models, x = l / lambda (+ log
// prior): the block's four waves split one 32-particle tile's layers
// (run_net_split), as the update of width-256 networks does.
template <int DT, int D_S, int LW, int LNH>
__global__ __launch_bounds__(256) void lik_rows_kernel(ProposeParams p) {
    static_assert(pass_mode<LW>() == kSplit, "likelihood widths above 64 and up to 256");
    typedef Net<DT, LW, LNH, in_slots(DT, D_S, 0, 0)> NTL;
    constexpr int SS = state_slots(D_S);
    extern __shared__ __attribute__((aligned(16))) char smem[];
    const int lane = threadIdx.x & 63, g = lane >> 5, col = lane & 31;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const NetPtrs PL = net_ptrs(p.lik.base, p.lik);
    const int n_tiles = (p.N + 31) / 32;
    for (int tile = blockIdx.x; tile < n_tiles; tile += gridDim.x) {
        const int i = tile * 32 + col;
        const bool valid = i < p.N;
        float ls[NTL::IN_SLOTS];
#pragma unroll
        for (int s = 0; s < NTL::IN_SLOTS; ++s) ls[s] = 0.0f;
#pragma unroll
        for (int s = 0; s < SS; ++s) {
            const int f = 2 * s + g;
            ls[s] = (valid && f < D_S) ? p.prop[(size_t)i * D_S + f] : 0.0f;
        }
        const f32x16 lo = run_net_split<NTL>(PL, p.b0_lik, ls, lane, g, wave, smem);
        if (wave == 0 && g == 0 && valid) {
            const float l = lo[0];
            if (p.loglik) p.loglik[i] = l;
            if (!isfinite(l) && p.status) p.status[0] = 5;
            double x = (double)l / p.lambda;
            if (p.prior_w) x += log(p.prior_w[i]);
            p.x[i] = x;
        }
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

// launchers
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

#define PROP_K(id, ds, na, da, dw, dox, dwz, w, nh, DT) propose_kernel<DT, ds, dw, w, nh, pass_mode<w>()>

int pass_tiles_per_block(int shape) { return pass_split(shape) ? 1 : 4; }

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

int lik_shape_width(int shape) {
#define X(id, ds, lw, lnh) \
    if (shape == id) return lw;
    VOILA_LIK_SHAPES(X)
#undef X
    return 0;
}
int lik_shape_hidden(int shape) {
#define X(id, ds, lw, lnh) \
    if (shape == id) return lnh;
    VOILA_LIK_SHAPES(X)
#undef X
    return 0;
}

#define PROPS_K(id, ds, na, da, dw, dox, dwz, w, nh, DT) propose_split_kernel<DT, ds, dw, w, nh>

template <int DT, int D_S, int D_W, int W, int NH>
constexpr size_t propose_split_lds() {
    if constexpr (!net_compiled(DT, W) || generic_compiled(DT, W, NH)) {
        return 0;
    } else {
        typedef Net<DT, W, NH, in_slots(DT, D_S, 0, D_W), W / 32, cdiv(D_S, 32)> NT;
        return (size_t)kPropSplitTiles * (SplitLds<NT>::ACT + SplitIn<NT>::BYTES);
    }
}

hipError_t launch_propose_split(int shape, int dt, const ProposeParams& p, int blocks, hipStream_t s) {
    switch (shape * 2 + dt) {
#define X(id, ds, na, da, dw, dox, dwz, w, nh)                                                                  \
    case id * 2 + 0: {                                                                                         \
        const size_t lds = propose_split_lds<DT_F32, ds, dw, w, nh>();                                          \
        if (lds == 0) return hipErrorInvalidValue;                                                             \
        if (lds > 65536)                                                                                       \
            (void)hipFuncSetAttribute((const void*)PROPS_K(id, ds, na, da, dw, dox, dwz, w, nh, DT_F32),          \
                                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);                   \
        hipLaunchKernelGGL((PROPS_K(id, ds, na, da, dw, dox, dwz, w, nh, DT_F32)), blocks, 64 * kPropSplitWaves, \
                           lds, s, p);                                                                         \
        break;                                                                                                 \
    }                                                                                                          \
    case id * 2 + 1: {                                                                                         \
        const size_t lds = propose_split_lds<DT_BF16, ds, dw, w, nh>();                                         \
        if (lds == 0) return hipErrorInvalidValue;                                                             \
        if (lds > 65536)                                                                                       \
            (void)hipFuncSetAttribute((const void*)PROPS_K(id, ds, na, da, dw, dox, dwz, w, nh, DT_BF16),         \
                                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);                   \
        hipLaunchKernelGGL((PROPS_K(id, ds, na, da, dw, dox, dwz, w, nh, DT_BF16)), blocks, 64 * kPropSplitWaves, \
                           lds, s, p);                                                                         \
        break;                                                                                                 \
    }
        VOILA_SHAPES(X)
#undef X
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

int propose_split_blocks_per_cu(int shape, int dt) {
    switch (shape * 2 + dt) {
#define X(id, ds, na, da, dw, dox, dwz, w, nh)                                                              \
    case id * 2 + 0:                                                                                       \
        return occupancy_t(PROPS_K(id, ds, na, da, dw, dox, dwz, w, nh, DT_F32), 64 * kPropSplitWaves,       \
                           propose_split_lds<DT_F32, ds, dw, w, nh>());                                     \
    case id * 2 + 1:                                                                                       \
        return occupancy_t(PROPS_K(id, ds, na, da, dw, dox, dwz, w, nh, DT_BF16), 64 * kPropSplitWaves,      \
                           propose_split_lds<DT_BF16, ds, dw, w, nh>());
        VOILA_SHAPES(X)
#undef X
    }
    return 1;
}

hipError_t launch_lik_rows(int shape, int dt, const ProposeParams& p, int blocks, hipStream_t s) {
    switch (shape * 2 + dt) {
#define X(id, ds, lw, lnh)                                                                                 \
    case id * 2 + 0:                                                                                      \
        hipLaunchKernelGGL((lik_rows_kernel<DT_F32, ds, lw, lnh>), blocks, 256, kSplitLds, s, p);         \
        break;                                                                                            \
    case id * 2 + 1:                                                                                      \
        hipLaunchKernelGGL((lik_rows_kernel<DT_BF16, ds, lw, lnh>), blocks, 256, kSplitLds, s, p);        \
        break;
        VOILA_LIK_SHAPES(X)
#undef X
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

int lik_rows_blocks_per_cu(int shape, int dt) {
    switch (shape * 2 + dt) {
#define X(id, ds, lw, lnh)                                                          \
    case id * 2 + 0:                                                               \
        return occupancy(lik_rows_kernel<DT_F32, ds, lw, lnh>, kSplitLds);         \
    case id * 2 + 1:                                                               \
        return occupancy(lik_rows_kernel<DT_BF16, ds, lw, lnh>, kSplitLds);
        VOILA_LIK_SHAPES(X)
#undef X
    }
    return 1;
}

#define PROPB_K(id, ds, na, da, dw, dox, dwz, w, nh, DT) propose_batch_kernel<DT, ds, dw, w, nh>

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

hipError_t launch_fold_steps(const FoldStepsParams& p, hipStream_t s) {
    if (p.rows == 0) return hipSuccess;
    hipLaunchKernelGGL(fold_steps_kernel, dim3((p.width + 255) / 256, p.rows < 65535 ? p.rows : 65535), 256, 0, s, p);
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
