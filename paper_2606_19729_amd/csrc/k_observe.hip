// k_observe.hip -- the observation sampler f_Z over belief rows and over the
// rows of whole rollouts (per-step observations).
#include "kcommon.hpp"

namespace voila {

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
    int i;        // particle
    bool valid;   // this lane's particle exists
};

// This lane's row of tile unit u (index arithmetic only).
__device__ __forceinline__ ObsRow observe_row(const ObserveParams& p, long u, int n_tiles, int col) {
    ObsRow w;
    w.grp = (int)(u / n_tiles);
    const int tile = (int)(u - (long)w.grp * n_tiles);
    const int k = w.grp / p.H, t = w.grp - k * p.H;
    w.i = tile * 32 + col;
    w.valid = w.i < p.N;
    w.r = ((size_t)k * p.N + (w.valid ? w.i : 0)) * p.H + t;
    return w;
}

// This lane's state slots s' of row w (zero past the belief).
template <int D_S>
__device__ __forceinline__ void observe_states(const ObserveParams& p, const ObsRow& w, int g,
                                               float (&st)[state_slots(D_S)]) {
#pragma unroll
    for (int s = 0; s < state_slots(D_S); ++s) {
        const int f = 2 * s + g;
        st[s] = (w.valid && f < D_S) ? p.states[w.r * D_S + f] : 0.0f;
    }
}

// Inputs [s', w_Z] of row w in first-layer slot order, from its state slots.
template <int D_S, int D_WZ, int IN_SLOTS>
__device__ __forceinline__ void observe_slots(const ObserveParams& p, const ObsRow& w, int g,
                                              const float (&st)[state_slots(D_S)], float (&slots)[IN_SLOTS]) {
    constexpr int SS = state_slots(D_S), SW = noise_slots(D_WZ);
#pragma unroll
    for (int s = 0; s < IN_SLOTS; ++s) slots[s] = 0.0f;
#pragma unroll
    for (int s = 0; s < SS; ++s) slots[s] = st[s];
    if (p.noise) {
#pragma unroll
        for (int s = 0; s < SW; ++s) {
            int f = noise_feature(s, g);
            slots[SS + s] = (w.valid && f < D_WZ) ? p.noise[w.r * D_WZ + f] : 0.0f;
        }
    } else {
        const int k = w.grp / p.H, t = w.grp - k * p.H;
        float nz[SW];
        noise_slots_philox<SW>(nz, p.key0, p.key1, (uint32_t)w.i, p.crn ? 0u : (uint32_t)k, (uint32_t)t, 4u, g);
#pragma unroll
        for (int s = 0; s < SW; ++s) slots[SS + s] = nz[s];
    }
}

// Inputs [s', w_Z] of this lane's row of tile unit u in first-layer slot order.
template <int D_S, int D_WZ, int IN_SLOTS>
__device__ __forceinline__ ObsRow observe_inputs(const ObserveParams& p, long u, int n_tiles, int g, int col,
                                                 float (&slots)[IN_SLOTS]) {
    const ObsRow w = observe_row(p, u, n_tiles, col);
    float st[state_slots(D_S)];
    observe_states<D_S>(p, w, g, st);
    observe_slots<D_S, D_WZ>(p, w, g, st, slots);
    return w;
}

// Writes this lane's outputs: feature 2 s + g is register s % 16 of output
// tile s / 16 (observations wider than 32 come in NO 32-row tiles).
template <int D_O, int NO, class T>
__device__ __forceinline__ void observe_store(const ObserveParams& p, const ObsRow& w, const T (&o)[NO], bool writer,
                                              int g) {
#pragma unroll
    for (int s = 0; s < 16 * NO; ++s) {
        int f = 2 * s + g;
        if (writer && w.valid && f < D_O) p.out[w.r * D_O + f] = o[s / 16][s % 16];
    }
}
template <int D_O>
__device__ __forceinline__ void observe_store(const ObserveParams& p, const ObsRow& w, const f32x16& o, bool writer,
                                              int g) {
    const f32x16 one[1] = {o};
    observe_store<D_O, 1, f32x16>(p, w, one, writer, g);
}

// MODE kResident / kSplit / kDirect: sized for one belief (n rows); kStream:
// sized for the rows of whole rollouts, one tile per wave with the weights
// streamed through LDS like the rollout kernel's.
template <int DT, int D_S, int D_WZ, int D_O, int WIDTH, int NHID, int MODE>
__global__ __launch_bounds__(256) void observe_kernel(ObserveParams p) {
    if constexpr (!generic_compiled(DT, WIDTH, NHID)) {
        return;  // refused at model creation (binary32 wider than 256) or run by the split rollout kernel
    } else {
    typedef Net<DT, WIDTH, NHID, in_slots(DT, D_S, 0, D_WZ)> NTO;
    extern __shared__ __attribute__((aligned(16))) char smem[];
    const int lane = threadIdx.x & 63, g = lane >> 5, col = lane & 31;
    const int n_tiles = (p.N + 31) / 32;
    const long n_units = (long)p.K * p.H * n_tiles;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if constexpr (MODE == kStream) {
        const int wpb = blockDim.x >> 6;
        // each wave keeps its unit's (candidate, step) group bias row in an
        // LDS row of its own, rewritten when the group changes
        float* rowb = reinterpret_cast<float*>(smem + p.row_bias_lds) + wave * NTO::WIDTH;
        constexpr int RB = NTO::WIDTH / 64;  // bias floats per lane
        static_assert(NTO::WIDTH % 64 == 0 && RB <= 16, "bias row copy: whole lanes");
        // paired evaluation: a unit is two tiles of one group, every weight
        // fragment (streamed in pass-major order) feeding both
        constexpr bool PAIRS = plan_pairs<DT, WIDTH, NHID>();
        constexpr int TPU = PAIRS ? 2 : 1;
        const int n_tu = (n_tiles + TPU - 1) / TPU;  // units per group
        const long n_pu = (long)p.K * p.H * n_tu;
        int have = -1;
        // the rows, states and bias row of the wave's next unit, read one
        // unit ahead: their memory latency passes while the current unit
        // multiplies (a wave's consecutive units lie in different groups)
        constexpr int SS = state_slots(D_S);
        ObsRow nw[TPU];
        float nst[TPU][SS];
        float nbv[RB];
        auto next_rows = [&](long u) {
            const bool ok = u < n_pu;
            const long uu = ok ? u : 0;
            const long grp = uu / n_tu;
            const int t0 = (int)(uu - grp * n_tu) * TPU;
#pragma unroll
            for (int q = 0; q < TPU; ++q) {
                // a tile past the group's last reads that tile and writes nothing
                const int tile = t0 + q < n_tiles ? t0 + q : t0;
                nw[q] = observe_row(p, grp * n_tiles + tile, n_tiles, col);
                nw[q].valid = nw[q].valid && ok && t0 + q < n_tiles;
                observe_states<D_S>(p, nw[q], g, nst[q]);
            }
            const float* src_row = p.b0 + (size_t)(p.b0_stride ? nw[0].grp : 0) * p.b0_stride;
#pragma unroll
            for (int q = 0; q < RB; ++q) nbv[q] = ok ? src_row[q * 64 + lane] : 0.0f;
        };
        with_weights<NTO, MODE, 1, PAIRS ? VOILA_PLAN_STREAM_CHB : VOILA_STREAM_CHB>(
            smem, p.obs, [&](auto& src, const NetPtrs& P) {
            next_rows((long)blockIdx.x * wpb + wave);
            // block-uniform loop (the stream's chunk barriers need every wave)
            for (long ub = blockIdx.x; ub * wpb < n_pu; ub += gridDim.x) {
                const bool ok = ub * wpb + wave < n_pu;
                float slots[TPU][NTO::IN_SLOTS];
                ObsRow w[TPU];
#pragma unroll
                for (int q = 0; q < TPU; ++q) {
                    w[q] = nw[q];
                    observe_slots<D_S, D_WZ>(p, w[q], g, nst[q], slots[q]);
                }
                const int brow = p.b0_stride ? w[0].grp : 0;
                if (brow != have) {  // wave-uniform; the row's reads of the last unit precede these writes
#pragma unroll
                    for (int q = 0; q < RB; ++q) rowb[q * 64 + lane] = nbv[q];
                    have = brow;
                }
                next_rows((ub + gridDim.x) * wpb + wave);
                if constexpr (PAIRS) {
                    f32x16 o[2];
                    run_net_flat<NTO, 2, kPlanPassTiles>(src, P, rowb, slots, o, lane, g);
#pragma unroll
                    for (int q = 0; q < 2; ++q) observe_store<D_O>(p, w[q], o[q], w[q].valid, g);
                } else {
                    const f32x16 o = run_net<NTO>(src, P, rowb, slots[0], lane, g);
                    observe_store<D_O>(p, w[0], o, ok, g);
                }
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

// Observation networks of more than two hidden layers wider than 256 (the
// depth of the paper's distilled samplers): a block of kObsSplitWaves waves
// evaluates two 32-row tiles of one (candidate, step) group together, each
// layer split over the waves (run_net_split_owned), every weight fragment
// read from L2 serving both tiles.  Wave q forms tile q's inputs, stages
// them in LDS and writes the tile's observations (observations wider than
// 32 come in two output tiles).
constexpr int kObsSplitWaves = 8, kObsSplitTiles = 2, kObsSplitDepth = 2;

template <int DT, int WIDTH, int NHID>
constexpr bool obs_split() {
    return net_compiled(DT, WIDTH) && !generic_compiled(DT, WIDTH, NHID);
}

template <int DT, int D_S, int D_WZ, int D_O, int WIDTH, int NHID>
__global__ __launch_bounds__(64 * kObsSplitWaves) void observe_split_kernel(ObserveParams p) {
    if constexpr (!obs_split<DT, WIDTH, NHID>()) {
        return;  // the other networks run in observe_kernel
    } else {
    constexpr int ST = kObsSplitTiles, NO = cdiv(D_O, 32);
    typedef Net<DT, WIDTH, NHID, in_slots(DT, D_S, 0, D_WZ), WIDTH / 32, NO> NT;
    extern __shared__ __attribute__((aligned(16))) char smem[];
    char* const in_lds = smem + ST * SplitLds<NT>::ACT;
    const int lane = threadIdx.x & 63, g = lane >> 5, col = lane & 31;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const bool owner = wave < ST;  // wave q forms and writes tile q of the group
    const int n_tiles = (p.N + 31) / 32;
    const int n_pairs = (n_tiles + ST - 1) / ST;
    const long n_units = (long)p.K * p.H * n_pairs;
    const NetPtrs P = net_ptrs(p.obs.base, p.obs);
    for (long u = blockIdx.x; u < n_units; u += gridDim.x) {
        const long grp = u / n_pairs;
        const int tp = (int)(u - grp * n_pairs);
        ObsRow w{};
        if (owner) {
            // a tile past the last of the group reads row 0 and writes nothing
            const int tile = tp * ST + wave;
            float slots[NT::IN_SLOTS];
            w = observe_inputs<D_S, D_WZ>(p, grp * n_tiles + (tile < n_tiles ? tile : 0), n_tiles, g, col, slots);
            w.valid = w.valid && tile < n_tiles;
            split_stage_inputs<NT>(in_lds + wave * SplitIn<NT>::BYTES, slots, lane);
        }
        const float* b0 = p.b0 + (size_t)(p.b0_stride ? grp : 0) * p.b0_stride;
        __syncthreads();  // the owners' inputs are in LDS
        float o[NO][16];
        run_net_split_owned<NT, ST, kObsSplitWaves, kObsSplitDepth>(P, b0, in_lds, o, lane, g, wave, smem);
        if (owner) observe_store<D_O, NO, float[16]>(p, w, o, true, g);
    }
    }
}

#define OBS_SK(id, ds, na, da, dw, dox, dwz, w, nh, DT) observe_split_kernel<DT, ds, dwz, dox, w, nh>

template <int DT, int D_S, int D_WZ, int D_O, int W, int NH>
constexpr size_t obs_split_lds() {
    if constexpr (!obs_split<DT, W, NH>()) {
        return 0;
    } else {
        typedef Net<DT, W, NH, in_slots(DT, D_S, 0, D_WZ), W / 32, cdiv(D_O, 32)> NT;
        return (size_t)kObsSplitTiles * (SplitLds<NT>::ACT + SplitIn<NT>::BYTES);
    }
}

bool observe_split_shape(int shape, int dt) {
    switch (shape * 2 + dt) {
#define X(id, ds, na, da, dw, dox, dwz, w, nh) \
    case id * 2 + 0:                           \
        return obs_split<DT_F32, w, nh>();     \
    case id * 2 + 1:                           \
        return obs_split<DT_BF16, w, nh>();
        VOILA_SHAPES(X)
#undef X
    }
    return false;
}

// Rows (k, i, t) of an observation launch in the split kernel: one unit of
// two tiles per block, the grid capped (the kernel strides over units).
hipError_t launch_observe_split(int shape, int dt, const ObserveParams& p, hipStream_t s) {
    const long n_pairs = ((long)(p.N + 31) / 32 + kObsSplitTiles - 1) / kObsSplitTiles;
    const long units = (long)p.K * p.H * n_pairs;
    if (units == 0) return hipSuccess;
    const int blocks = (int)(units < 4096 ? units : 4096);
    switch (shape * 2 + dt) {
#define X(id, ds, na, da, dw, dox, dwz, w, nh)                                                               \
    case id * 2 + 0: {                                                                                      \
        const size_t lds = obs_split_lds<DT_F32, ds, dwz, dox, w, nh>();                                         \
        if (lds > 65536)                                                                                    \
            (void)hipFuncSetAttribute((const void*)OBS_SK(id, ds, na, da, dw, dox, dwz, w, nh, DT_F32),      \
                                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);                \
        hipLaunchKernelGGL((OBS_SK(id, ds, na, da, dw, dox, dwz, w, nh, DT_F32)), blocks,                    \
                           64 * kObsSplitWaves, lds, s, p);                                                 \
        break;                                                                                              \
    }                                                                                                       \
    case id * 2 + 1: {                                                                                      \
        const size_t lds = obs_split_lds<DT_BF16, ds, dwz, dox, w, nh>();                                        \
        if (lds > 65536)                                                                                    \
            (void)hipFuncSetAttribute((const void*)OBS_SK(id, ds, na, da, dw, dox, dwz, w, nh, DT_BF16),     \
                                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);                \
        hipLaunchKernelGGL((OBS_SK(id, ds, na, da, dw, dox, dwz, w, nh, DT_BF16)), blocks,                   \
                           64 * kObsSplitWaves, lds, s, p);                                                 \
        break;                                                                                              \
    }
        VOILA_SHAPES(X)
#undef X
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// launchers
#define OBS_K(id, ds, na, da, dw, dox, dwz, w, nh, DT) observe_kernel<DT, ds, dwz, dox, w, nh, pass_mode<w>()>

hipError_t launch_observe(int shape, int dt, const ObserveParams& p, int blocks, hipStream_t s) {
    if (observe_split_shape(shape, dt)) return launch_observe_split(shape, dt, p, s);
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

template <int DT, int D_S, int D_WZ, int W, int NH>
constexpr size_t obs_stream_lds() {
    return plan_pairs<DT, W, NH>() ? stream_lds_of<DT, D_S, 0, 0, D_WZ, W, NH, VOILA_PLAN_STREAM_CHB>()
                                   : stream_lds_of<DT, D_S, 0, 0, D_WZ, W, NH>();
}

size_t observe_rollout_lds(int shape, int dt, const NetBlob& obs) {
    if (weights_in_lds(shape)) return obs.bytes;
    size_t chunks = kStreamLds;
    switch (shape * 2 + dt) {
#define X(id, ds, na, da, dw, dox, dwz, w, nh)                  \
    case id * 2 + 0:                                           \
        chunks = obs_stream_lds<DT_F32, ds, dwz, w, nh>();     \
        break;                                                 \
    case id * 2 + 1:                                           \
        chunks = obs_stream_lds<DT_BF16, ds, dwz, w, nh>();    \
        break;
        VOILA_SHAPES(X)
#undef X
    }
    return chunks + (obs.bytes - obs.off_b0);
}

hipError_t launch_observe_rollouts(int shape, int dt, const ObserveParams& p0, int blocks, hipStream_t s) {
    if (observe_split_shape(shape, dt)) return launch_observe_split(shape, dt, p0, s);
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

int observe_rollout_blocks_per_cu(int shape, int dt) {
    switch (shape * 2 + dt) {
#define X(id, ds, na, da, dw, dox, dwz, w, nh)                                                               \
    case id * 2 + 0:                                                                                        \
        return occupancy(OBSR_K(id, ds, na, da, dw, dox, dwz, w, nh, DT_F32),                               \
                         lds_for_width<w>() ? kLdsGuess : obs_stream_lds<DT_F32, ds, dwz, w, nh>());          \
    case id * 2 + 1:                                                                                        \
        return occupancy(OBSR_K(id, ds, na, da, dw, dox, dwz, w, nh, DT_BF16),                              \
                         lds_for_width<w>() ? kLdsGuess : obs_stream_lds<DT_BF16, ds, dwz, w, nh>());
        VOILA_SHAPES(X)
#undef X
    }
    return 1;
}

}  // namespace voila
