// k_ddim.hip -- the DDIM teacher samplers of v-prediction denoisers.
#include "kcommon.hpp"

namespace voila {

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
    if constexpr (!net_compiled(DT, WIDTH) || D_X > 32) {
        return;  // binary32 wider than 256 is refused at creation; wider samples run split
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
    constexpr int ST = kDdimSplitTiles, NO = cdiv(D_X, 32);
    typedef Net<DT, WIDTH, NHID, in_slots(DT, D_X, 0, D_C), WIDTH / 32, NO> NT;
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
            f32x16 v[ST * NO];
            run_net_split_multi<NT, ST, kDdimSplitWaves, kDdimSplitDepth>(P, p.b0 + (size_t)t * WIDTH, slots, v, lane, g, wave, smem);
            const float Am1 = coef[2 * t], B = coef[2 * t + 1];
            // state slot s holds feature 2 s + g: output tile s / 16, register s % 16
#pragma unroll
            for (int st = 0; st < ST; ++st)
#pragma unroll
                for (int s = 0; s < SS; ++s)
                    x[st][s] += __builtin_fmaf(B, v[st * NO + s / 16][s % 16], Am1 * x[st][s]);
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

// launchers
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
        return (size_t)kDdimSplitTiles * SplitLds<Net<DT, W, NH, in_slots(DT, D_X, 0, D_C), W / 32, cdiv(D_X, 32)>>::ACT;
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

}  // namespace voila
