// kcommon.hpp -- device helpers and launch constants shared by the kernel
// translation units (weight sources of rollout-sized launches, binary64
// block reductions, the single-workgroup normalisation and resampling body).
#pragma once

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

// Binary32 activations of a network wider than 256 do not fit in registers:
// such networks run in bfloat16 only.
constexpr bool net_compiled(int dt, int width) { return dt == DT_BF16 || width <= 256; }
// The kernels that evaluate one network per wave or per block (rollouts,
// proposals, observations, likelihoods) hold a wide network's first hidden
// layer in registers and group the second: networks wider than 256 with
// more than two hidden layers run in the split rollout kernel only.
constexpr bool generic_compiled(int dt, int width, int nhid) {
    return net_compiled(dt, width) && (width <= 256 || nhid == 2);
}

// How a kernel reads the weight fragments of a network.
constexpr int kDirect = 0;    // straight from global memory (L2)
constexpr int kResident = 1;  // whole network staged in LDS once per block
constexpr int kStream = 2;    // streamed through double-buffered LDS chunks
constexpr int kSplit = 3;     // the four waves of a block split each layer of one tile (global memory)

// The weight source of a rollout-sized launch of network NT, handed to
// body(src, P) with the network's pointers: the whole network staged in LDS
// once per block (kResident), streamed through the LDS chunk buffers with the
// biases -- and for a grouped wide network the first layer -- staged after
// them (kStream), or read from L2 (kDirect).  B0_ROWS is the number of
// first-layer bias rows the blob carries (one per discrete action).
template <class NT, int MODE, int B0_ROWS, int CHB = VOILA_STREAM_CHB, class Body>
__device__ __forceinline__ void with_weights(char* smem, const NetBlob& net, Body&& body) {
    if (MODE == kResident) {
        stage_blob(smem, net.base, net.bytes);
        __syncthreads();
    }
    NetPtrs P = net_ptrs(MODE == kResident ? (const char*)smem : net.base, net);
    constexpr bool F0_LDS = NT::CT < NT::HT && first_layer_in_lds<NT>(B0_ROWS);
    char* extra = smem;
    if constexpr (MODE == kStream) {
        extra = smem + StreamChunk<NT, CHB>::BYTES;
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
        StreamFor<NT, CHB> src(smem, P.f0);
        src.start();
        body(src, P);
        src.finish();
    } else {
        DirectSrc<NT::DT, 8 * NT::HT> src(P.f0);
        body(src, P);
    }
}

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

namespace {
template <int W> constexpr bool lds_for_width() { return W <= 64; }
// weight access of the rollout kernel and of the single-pass kernels
template <int W> constexpr int plan_mode() { return W <= 64 ? kResident : kStream; }
template <int W> constexpr int pass_mode() { return W <= 64 ? kResident : W <= 256 ? kSplit : kDirect; }
constexpr size_t kStreamLds = (size_t)VOILA_STREAM_NBUF * VOILA_STREAM_CHB;

// Split-mode passes (one tile per block, LDS for activations and partials).
inline bool pass_split(int shape) { return kShapeInfo[shape].width > 64 && kShapeInfo[shape].width <= 256; }
constexpr size_t kSplitLds = 48 * 1024;  // binary32 width 256: 32 KB activations + 16 KB partials
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

// Whether the rollout kernels (plan, per-step observations) run two
// 32-particle tiles per wave through a pass-major fragment stream
// (run_net_flat): the streamed bfloat16 layered networks, where reading each
// weight fragment once for 64 rollouts halves the LDS traffic per matrix
// instruction.
template <int DT, int WIDTH, int NHID>
constexpr bool plan_pairs() {
    return DT == DT_BF16 && WIDTH > 64 && chunk_tiles(WIDTH) == WIDTH / 32 && NHID >= 2;
}
#ifndef VOILA_PLAN_PASS_TILES
#define VOILA_PLAN_PASS_TILES 2
#endif
constexpr int kPlanPassTiles = VOILA_PLAN_PASS_TILES;
#ifndef VOILA_PLAN_FLAT
#define VOILA_PLAN_FLAT 1
#endif
// LDS of a streaming rollout kernel before its staged biases: the two chunk
// buffers (and the first layer of a grouped wide network).
template <int DT, int D_S, int N_ACT, int D_AIN, int D_W, int WIDTH, int NHID, int CHB = VOILA_STREAM_CHB>
constexpr size_t stream_lds_of() {
    if constexpr (!generic_compiled(DT, WIDTH, NHID) || WIDTH <= 64) {
        return (size_t)VOILA_STREAM_NBUF * CHB;
    } else {
        typedef Net<DT, WIDTH, NHID, in_slots(DT, D_S, D_AIN, D_W)> NT;
        return (size_t)StreamChunk<NT, CHB>::BYTES +
               (NT::CT < NT::HT && first_layer_in_lds<NT>(N_ACT > 0 ? N_ACT : 1) ? (size_t)NT::NF0 * NT::FRAG_BYTES
                                                                                : 0);
    }
}

}  // namespace voila
