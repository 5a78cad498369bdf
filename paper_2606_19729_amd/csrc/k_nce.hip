// k_nce.hip -- the contrastive (InfoNCE) objective of the likelihood network:
// all-pairs scores, binary64 row losses and score derivatives, the mean loss.
#include "kcommon.hpp"

namespace voila {


// Scores of all B x B pairs of a contrastive mini-batch: tile (i, jt) is
// state-action i against the 32 observations of column tile jt.  Row i's
// state and action sit in its folded first-layer bias row, which each wave
// copies into its own LDS row when the row changes; the observations are the
// network's input slots.
template <int DT, int D_O, int WIDTH, int NHID, int MODE>
__global__ __launch_bounds__(256) void nce_scores_kernel(NceParams p) {
    if constexpr (!generic_compiled(DT, WIDTH, NHID)) {
        return;  // refused at model creation (binary32 wider than 256) or run by the split rollout kernel
    } else {
    typedef Net<DT, WIDTH, NHID, in_slots(DT, D_O, 0, 0)> NTL;
    constexpr int SO = state_slots(D_O);
    // paired evaluation: a unit is two column tiles of one row, every weight
    // fragment (streamed in pass-major order) feeding both
    constexpr bool PAIRS = MODE == kStream && plan_pairs<DT, WIDTH, NHID>();
    constexpr int TPU = PAIRS ? 2 : 1;
    extern __shared__ __attribute__((aligned(16))) char smem[];
    const int lane = threadIdx.x & 63, g = lane >> 5, col = lane & 31;
    const int wpb = blockDim.x >> 6;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int jtiles = (p.B + 31) / 32;
    const int jun = (jtiles + TPU - 1) / TPU;  // units per row
    const long n_units = (long)p.B * jun;
    float* rowb = reinterpret_cast<float*>(smem + p.row_bias_lds) + wave * NTL::WIDTH;
    constexpr int RB = NTL::WIDTH / 64;  // bias floats per lane
    static_assert(NTL::WIDTH % 64 == 0 && RB <= 16, "bias row copy: whole lanes");
    int have = -1;  // row held in this wave's LDS bias row
    // the observations and bias row of the wave's next unit, read one unit
    // ahead: their memory latency passes while the current unit multiplies
    // (a wave's consecutive units lie in different rows)
    float nob[TPU][SO];
    float nbv[RB];
    auto next_inputs = [&](long u) {
        const bool ok = u < n_units;  // wave-uniform
        const int i = ok ? (int)(u / jun) : 0;
        const int jt0 = ok ? (int)(u - (long)i * jun) * TPU : 0;
#pragma unroll
        for (int q = 0; q < TPU; ++q) {
            const int j = (jt0 + q) * 32 + col;
            const bool v = ok && jt0 + q < jtiles && j < p.B;
#pragma unroll
            for (int s = 0; s < SO; ++s) {
                const int f = 2 * s + g;
                nob[q][s] = (v && f < D_O) ? p.obs[(size_t)j * D_O + f] : 0.0f;
            }
        }
        const float* brow = p.b0 + (size_t)i * NTL::WIDTH;
#pragma unroll
        for (int q = 0; q < RB; ++q) nbv[q] = ok ? brow[q * 64 + lane] : 0.0f;
    };
    with_weights<NTL, MODE, 1, PAIRS ? VOILA_PLAN_STREAM_CHB : VOILA_STREAM_CHB>(smem, p.lik, [&](auto& src,
                                                                                            const NetPtrs& P) {
        next_inputs((long)blockIdx.x * wpb + wave);
        // block-uniform loop (a streamed network's chunk barriers need every wave)
        for (long ub = blockIdx.x; ub * wpb < n_units; ub += gridDim.x) {
            const long u = ub * wpb + wave;
            const bool ok = u < n_units;
            const int i = ok ? (int)(u / jun) : 0;
            const int jt0 = ok ? (int)(u - (long)i * jun) * TPU : 0;
            int j[TPU];
            bool valid[TPU];
            float slots[TPU][NTL::IN_SLOTS];
#pragma unroll
            for (int q = 0; q < TPU; ++q) {
                j[q] = (jt0 + q) * 32 + col;
                valid[q] = ok && jt0 + q < jtiles && j[q] < p.B;
#pragma unroll
                for (int s = 0; s < NTL::IN_SLOTS; ++s) slots[q][s] = 0.0f;
#pragma unroll
                for (int s = 0; s < SO; ++s) slots[q][s] = nob[q][s];
            }
            if (i != have) {  // wave-uniform; the row's reads of the last unit precede these writes
#pragma unroll
                for (int q = 0; q < RB; ++q) rowb[q * 64 + lane] = nbv[q];
                have = i;
            }
            next_inputs(u + (long)gridDim.x * wpb);
            f32x16 o[TPU];
            if constexpr (PAIRS) {
                run_net_flat<NTL, 2, kPlanPassTiles>(src, P, rowb, slots, o, lane, g);
            } else {
                o[0] = run_net<NTL>(src, P, rowb, slots[0], lane, g);
            }
#pragma unroll
            for (int q = 0; q < TPU; ++q)
                if (g == 0 && valid[q]) {
                    const float l = o[q][0];
                    p.scores[(size_t)i * p.B + j[q]] = l;
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

// launchers
#define NCE_K(id, ds, na, da, dw, dox, dwz, w, nh, DT) nce_scores_kernel<DT, dox, w, nh, plan_mode<w>()>

template <int DT, int D_O, int W, int NH>
constexpr size_t nce_stream_lds() {
    return plan_pairs<DT, W, NH>() ? stream_lds_of<DT, D_O, 0, 0, 0, W, NH, VOILA_PLAN_STREAM_CHB>()
                                   : stream_lds_of<DT, D_O, 0, 0, 0, W, NH>();
}

hipError_t launch_nce_scores(int shape, int dt, const NceParams& p0, int blocks, hipStream_t s) {
    NceParams p = p0;
    size_t lds = p.lik.bytes;
    if (!weights_in_lds(shape)) {
        switch (shape * 2 + dt) {
#define X(id, ds, na, da, dw, dox, dwz, w, nh)                  \
    case id * 2 + 0:                                           \
        lds = nce_stream_lds<DT_F32, dox, w, nh>();            \
        break;                                                 \
    case id * 2 + 1:                                           \
        lds = nce_stream_lds<DT_BF16, dox, w, nh>();           \
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
        return occupancy(NCE_K(id, ds, na, da, dw, dox, dwz, w, nh, DT_F32),                                \
                         lds_for_width<w>() ? kLdsGuess : nce_stream_lds<DT_F32, dox, w, nh>());             \
    case id * 2 + 1:                                                                                        \
        return occupancy(NCE_K(id, ds, na, da, dw, dox, dwz, w, nh, DT_BF16),                               \
                         lds_for_width<w>() ? kLdsGuess : nce_stream_lds<DT_BF16, dox, w, nh>());
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

}  // namespace voila
