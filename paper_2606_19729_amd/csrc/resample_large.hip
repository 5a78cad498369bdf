// resample_large.hip -- weight normalisation and systematic resampling for
// beliefs larger than one workgroup can hold (N > 8192), streamed through HBM.
//
// Chunks of 4096 particles (256 threads x 16 consecutive particles):
//   pass 1  per-chunk max of x_i = l_i / lambda (+ log w_i)            -> bmax
//   red 1   m = max over chunks (one workgroup, fixed order)
//   pass 2  per-chunk sum of exp(x_i - m) (thread order, then tree)     -> bsum
//   red 2   S = sum over chunks in chunk order
//   pass 3  w_i = exp(x_i - m) / S (or given weights), q_i = rint(w_i N 2^b),
//           chunk-relative inclusive prefix C_i (exact integers), chunk
//           total, sum of w_i^2, last positive-mass particle
//   red 3   exclusive scan of the chunk totals (exact), statistics
//   pass 4  per output j: P_j = j 2^b + u, first chunk whose inclusive
//           prefix exceeds P_j (binary search over chunks), then first
//           particle of that chunk with C_i > P_j - offset (binary search),
//           gather of the particle's row.
// Every prefix is an integer below 2^53, so the blocked scan gives the same
// bits as a sequential one and the indices equal those of the one-workgroup
// kernel and of the definition.
#include "kernels.hpp"

#include <math.h>

namespace voila {

namespace {

constexpr int kLgThreads = 256;
constexpr int kLgItems = 16;
constexpr int kLgChunk = kLgThreads * kLgItems;

__device__ __forceinline__ double lg_x(const LargeResParams& p, int i, int& bad) {
    if (p.x) {
        double x = p.x[i];
        if (isnan(x) || x == INFINITY) bad = 1;
        return x;
    }
    float l = p.loglik[i];
    if (!isfinite(l)) bad = 1;
    double x = (double)l / p.lambda;
    if (p.prior_w) x += log(p.prior_w[i]);
    return x;
}

__device__ double blk_reduce(double v, double* red, bool is_max) {
    for (int m = 32; m >= 1; m >>= 1) {
        double o = __shfl_xor(v, m);
        v = is_max ? fmax(v, o) : v + o;
    }
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double r = is_max ? -INFINITY : 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) r = is_max ? fmax(r, red[w]) : r + red[w];
    return r;
}

__device__ int blk_max_i(int v, int* red) {
    for (int m = 32; m >= 1; m >>= 1) v = max(v, __shfl_xor(v, m));
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    int r = -1;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) r = max(r, red[w]);
    return r;
}

}  // namespace

__global__ __launch_bounds__(kLgThreads) void lg_max_kernel(LargeResParams p) {
    __shared__ double red[kLgThreads / 64];
    __shared__ int redi[kLgThreads / 64];
    const int base = blockIdx.x * kLgChunk + threadIdx.x * kLgItems;
    double mx = -INFINITY;
    int bad = 0;
    for (int k = 0; k < kLgItems; ++k)
        if (base + k < p.N) mx = fmax(mx, lg_x(p, base + k, bad));
    mx = blk_reduce(mx, red, true);
    bad = blk_max_i(bad, redi);
    if (threadIdx.x == 0) {
        p.ws.bmax[blockIdx.x] = mx;
        if (bad && p.status) p.status[0] = 5;
    }
}

__global__ __launch_bounds__(kLgThreads) void lg_reduce_max_kernel(LargeResParams p) {
    __shared__ double red[kLgThreads / 64];
    double mx = -INFINITY;
    for (int c = threadIdx.x; c < p.n_chunks; c += blockDim.x) mx = fmax(mx, p.ws.bmax[c]);
    mx = blk_reduce(mx, red, true);
    if (threadIdx.x == 0) {
        p.ws.scal[0] = mx;
        if (!isfinite(mx) && p.status) p.status[0] = 5;
    }
}

__global__ __launch_bounds__(kLgThreads) void lg_sum_kernel(LargeResParams p) {
    __shared__ double red[kLgThreads / 64];
    const double m = p.ws.scal[0];
    const int base = blockIdx.x * kLgChunk + threadIdx.x * kLgItems;
    double s = 0.0;
    int bad = 0;
    for (int k = 0; k < kLgItems; ++k)
        if (base + k < p.N) s += exp(lg_x(p, base + k, bad) - m);
    s = blk_reduce(s, red, false);
    if (threadIdx.x == 0) p.ws.bsum[blockIdx.x] = s;
}

__global__ __launch_bounds__(64) void lg_reduce_sum_kernel(LargeResParams p) {
    if (threadIdx.x != 0) return;
    double s = 0.0;
    for (int c = 0; c < p.n_chunks; ++c) s += p.ws.bsum[c];
    p.ws.scal[1] = s;
}

__global__ __launch_bounds__(kLgThreads) void lg_quant_kernel(LargeResParams p) {
    __shared__ double red[kLgThreads / 64];
    __shared__ int redi[kLgThreads / 64];
    __shared__ double tot[kLgThreads / 64];
    const int base = blockIdx.x * kLgChunk + threadIdx.x * kLgItems;
    const double m = p.ws.scal[0], S = p.ws.scal[1];
    const double scale = ldexp((double)p.N, p.bits);
    double q[kLgItems];
    double sq = 0.0, run = 0.0;
    int last = -1, bad = 0;
    for (int k = 0; k < kLgItems; ++k) {
        const int i = base + k;
        double w = 0.0;
        if (i < p.N) {
            if (p.w_in) {
                w = p.w_in[i];
                if (!(w >= 0.0) || w == INFINITY) bad = 1;
            } else {
                w = exp(lg_x(p, i, bad) - m) / S;
                if (p.w_out) p.w_out[i] = w;
            }
        }
        sq += w * w;
        q[k] = rint(w * scale);
        if (q[k] > 0.0) last = i;
        run += q[k];
        q[k] = run;
    }
    // chunk-level exclusive scan of the thread totals (exact integers)
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    double incl = run;
    for (int d = 1; d < 64; d <<= 1) {
        double o = __shfl_up(incl, d);
        if (lane >= d) incl += o;
    }
    if (lane == 63) tot[wave] = incl;
    __syncthreads();
    double off = incl - run;
    for (int w2 = 0; w2 < wave; ++w2) off += tot[w2];
    if (p.do_resample)
        for (int k = 0; k < kLgItems; ++k)
            if (base + k < p.N) p.ws.cloc[base + k] = q[k] + off;
    double total = 0.0;
    for (int w2 = 0; w2 < (int)(blockDim.x >> 6); ++w2) total += tot[w2];
    sq = blk_reduce(sq, red, false);
    last = blk_max_i(last, redi);
    bad = blk_max_i(bad, redi);
    if (threadIdx.x == 0) {
        p.ws.btot[blockIdx.x] = total;
        p.ws.bsq[blockIdx.x] = sq;
        p.ws.blast[blockIdx.x] = last;
        if (bad && p.status) p.status[0] = 5;
    }
}

// One workgroup: exclusive scan of the chunk totals, global statistics.
__global__ __launch_bounds__(1024) void lg_scan_kernel(LargeResParams p) {
    __shared__ double tot[1024 / 64];
    __shared__ double red[1024 / 64];
    __shared__ int redi[1024 / 64];
    const int nc = p.n_chunks;
    const int per = (nc + blockDim.x - 1) / blockDim.x;
    const int lo = threadIdx.x * per, hi = min(nc, lo + per);
    double run = 0.0, sq = 0.0;
    int last = -1;
    for (int c = lo; c < hi; ++c) {
        run += p.ws.btot[c];
        sq += p.ws.bsq[c];
        last = max(last, p.ws.blast[c]);
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    double incl = run;
    for (int d = 1; d < 64; d <<= 1) {
        double o = __shfl_up(incl, d);
        if (lane >= d) incl += o;
    }
    if (lane == 63) tot[wave] = incl;
    __syncthreads();
    double off = incl - run;
    for (int w2 = 0; w2 < wave; ++w2) off += tot[w2];
    for (int c = lo; c < hi; ++c) {
        p.ws.boff[c] = off;
        off += p.ws.btot[c];
        p.ws.bincl[c] = off;
    }
    sq = blk_reduce(sq, red, false);
    last = blk_max_i(last, redi);
    if (threadIdx.x == 0) {
        p.ws.last[0] = last;
        if (last < 0 && p.status) p.status[0] = 5;
        if (p.stats && !p.w_in) {
            const double m = p.ws.scal[0], S = p.ws.scal[1];
            p.stats[0] = m + log(S) - (p.uniform_prior ? log((double)p.N) : 0.0);
            p.stats[1] = 1.0 / sq;
        }
    }
}

__global__ __launch_bounds__(256) void lg_search_kernel(LargeResParams p) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= p.N) return;
    const int last = p.ws.last[0];
    if (last < 0) return;  // no particle has mass: outputs left untouched, status set
    const double P = (double)j * ldexp(1.0, p.bits) + (double)(p.U >> (32 - p.bits));
    int a = 0, b = p.n_chunks;
    while (a < b) {
        int mid = (a + b) >> 1;
        if (p.ws.bincl[mid] > P) b = mid;
        else a = mid + 1;
    }
    int idx = last;
    if (a < p.n_chunks) {
        const double rel = P - p.ws.boff[a];
        int lo = a * kLgChunk, hi = min(p.N, lo + kLgChunk);
        while (lo < hi) {
            int mid = (lo + hi) >> 1;
            if (p.ws.cloc[mid] > rel) hi = mid;
            else lo = mid + 1;
        }
        idx = lo;
    }
    if (p.idx_out) p.idx_out[j] = idx;
    if (p.src && p.dst)
        for (int c = 0; c < p.row_floats; ++c) p.dst[(size_t)j * p.row_floats + c] = p.src[(size_t)idx * p.row_floats + c];
}

size_t large_res_workspace_bytes(int N) {
    const size_t nc = ((size_t)N + kLgChunk - 1) / kLgChunk;
    auto al = [](size_t x) { return (x + 255) / 256 * 256; };
    return al(nc * 8) * 6 + al(nc * 4) + al((size_t)N * 8) + al(64);
}

LargeResWs carve_large_res(void* base, int N) {
    const size_t nc = ((size_t)N + kLgChunk - 1) / kLgChunk;
    auto al = [](size_t x) { return (x + 255) / 256 * 256; };
    char* b = reinterpret_cast<char*>(base);
    LargeResWs w;
    w.bmax = reinterpret_cast<double*>(b); b += al(nc * 8);
    w.bsum = reinterpret_cast<double*>(b); b += al(nc * 8);
    w.btot = reinterpret_cast<double*>(b); b += al(nc * 8);
    w.bsq = reinterpret_cast<double*>(b); b += al(nc * 8);
    w.boff = reinterpret_cast<double*>(b); b += al(nc * 8);
    w.bincl = reinterpret_cast<double*>(b); b += al(nc * 8);
    w.blast = reinterpret_cast<int*>(b); b += al(nc * 4);
    w.cloc = reinterpret_cast<double*>(b); b += al((size_t)N * 8);
    w.scal = reinterpret_cast<double*>(b);
    w.last = reinterpret_cast<int*>(b + 32);
    return w;
}

hipError_t launch_large_res(LargeResParams p, hipStream_t s) {
    p.n_chunks = (p.N + kLgChunk - 1) / kLgChunk;
    const int nc = p.n_chunks;
    if (!p.w_in) {
        hipLaunchKernelGGL(lg_max_kernel, nc, kLgThreads, 0, s, p);
        hipLaunchKernelGGL(lg_reduce_max_kernel, 1, kLgThreads, 0, s, p);
        hipLaunchKernelGGL(lg_sum_kernel, nc, kLgThreads, 0, s, p);
        hipLaunchKernelGGL(lg_reduce_sum_kernel, 1, 64, 0, s, p);
    }
    hipLaunchKernelGGL(lg_quant_kernel, nc, kLgThreads, 0, s, p);
    hipLaunchKernelGGL(lg_scan_kernel, 1, 1024, 0, s, p);
    if (p.do_resample) hipLaunchKernelGGL(lg_search_kernel, (p.N + 255) / 256, 256, 0, s, p);
    return hipGetLastError();
}

}  // namespace voila
