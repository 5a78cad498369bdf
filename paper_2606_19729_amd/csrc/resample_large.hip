// resample_large.hip -- weight normalisation and systematic resampling for
// beliefs larger than one workgroup can hold (N > 8192), streamed through HBM.
//
// Chunks of 4096 particles, 256 threads; thread t touches particles
// chunk_base + 256 k + t (k < 16), so every global access is coalesced.
//   pass 1  per-chunk (max, sum exp(x - max)) of x_i = l_i / lambda (+ log w_i),
//           accumulated online (the running sum is rescaled when the running
//           max grows), in a fixed order                        -> bmax, bsum
//   red 1   m = max over chunks, S = sum_c bsum_c exp(bmax_c - m) in chunk order
//   pass 2  w_i = exp(x_i - m) / S (or given weights), q_i = rint(w_i N 2^b);
//           the chunk-relative inclusive prefix C_i is formed in LDS (each
//           thread scans 16 consecutive entries, then the thread totals are
//           scanned); chunk total, sum of w_i^2, last positive particle
//   red 2   exclusive scan of the chunk totals, statistics
//   starts  per block of 4096 outputs, the particle of its first output
//           (global two-level search, one thread per block)
//   pass 3  one workgroup per 4096 consecutive outputs j: the particles
//           [start of this block, start of the next] own all of them; each
//           particle writes its index to the outputs it owns (the count form
//           of the search: its copies are the outputs between its two prefix
//           boundaries), the rest take the last positive-mass particle
//   gather  dst row j = src row idx_j, 16-byte vectors where the rows allow,
//           consecutive threads on consecutive elements
// Every prefix is an integer below 2^53, so the blocked sums give the same
// bits as a sequential sum and the indices equal those of the definition.
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

__device__ __forceinline__ int lg_pad(int r) { return r + (r >> 4); }

// (m, s) <- (m, s) combined with (m2, s2), where s = sum exp(x - m).
__device__ __forceinline__ void lse_merge(double& m, double& s, double m2, double s2) {
    if (m2 == -INFINITY) return;
    if (m == -INFINITY) {
        m = m2;
        s = s2;
        return;
    }
    if (m2 > m) {
        s = s * exp(m - m2) + s2;
        m = m2;
    } else {
        s += s2 * exp(m2 - m);
    }
}

__device__ double blk_sum(double v, double* red) {
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double r = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) r += red[w];
    return r;
}

__device__ int blk_max_i(int v, int* red) {
    for (int d = 32; d >= 1; d >>= 1) v = max(v, __shfl_xor(v, d));
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    int r = -1;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) r = max(r, red[w]);
    return r;
}

// Global prefix of particle i (exact integer).
__device__ __forceinline__ double gprefix(const LargeResParams& p, int i) {
    return p.ws.boff[i / kLgChunk] + p.ws.cloc[i];
}

// First particle with prefix > P (global memory), or `last` if none.
__device__ int global_search(const LargeResParams& p, double P, int last) {
    int a = 0, b = p.n_chunks;
    while (a < b) {
        int mid = (a + b) >> 1;
        if (p.ws.bincl[mid] > P) b = mid;
        else a = mid + 1;
    }
    if (a >= p.n_chunks) return last;
    const double rel = P - p.ws.boff[a];
    int lo = a * kLgChunk, hi = min(p.N, lo + kLgChunk);
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (p.ws.cloc[mid] > rel) hi = mid;
        else lo = mid + 1;
    }
    return lo;
}

// dst row j0 + r = src row ids[r] for r < n_out (rows of w elements): each
// thread keeps one column c and walks the rows, so consecutive threads move
// consecutive elements of a row and of consecutive rows.
template <class T>
__device__ __forceinline__ void gather_rows(T* dst, const T* src, const int* ids, int j0, int n_out, int w) {
    if (w <= kLgThreads) {
        const int rpp = kLgThreads / w, r0 = threadIdx.x / w, c = threadIdx.x - r0 * w;
        if (r0 < rpp)
            for (int r = r0; r < n_out; r += rpp) dst[(size_t)(j0 + r) * w + c] = src[(size_t)ids[r] * w + c];
    } else {
        for (int r = 0; r < n_out; ++r)
            for (int c = threadIdx.x; c < w; c += kLgThreads) dst[(size_t)(j0 + r) * w + c] = src[(size_t)ids[r] * w + c];
    }
}

}  // namespace

__global__ __launch_bounds__(kLgThreads) void lg_lse_kernel(LargeResParams p) {
    __shared__ double rm[kLgThreads], rs[kLgThreads];
    __shared__ int redi[kLgThreads / 64];
    const int base = blockIdx.x * kLgChunk + threadIdx.x;
    int bad = 0;
    // this thread's 16 values: their maximum, then the sum of exp(x - max)
    // (independent exponentials, no serial merge chain)
    double xs[kLgItems];
    double m = -INFINITY;
#pragma unroll
    for (int k = 0; k < kLgItems; ++k) {
        const int i = base + k * kLgThreads;
        xs[k] = i < p.N ? lg_x(p, i, bad) : -INFINITY;
        m = fmax(m, xs[k]);
    }
    double s = 0.0;
    if (m != -INFINITY) {
#pragma unroll
        for (int k = 0; k < kLgItems; ++k) s += exp(xs[k] - m);
    }
    rm[threadIdx.x] = m;
    rs[threadIdx.x] = s;
    bad = blk_max_i(bad, redi);
    // fixed-shape tree: thread t merges t + h into t for h = 128, 64, ..., 1
    for (int h = kLgThreads / 2; h >= 1; h >>= 1) {
        __syncthreads();
        if (threadIdx.x < h) {
            double mm = rm[threadIdx.x], ss = rs[threadIdx.x];
            lse_merge(mm, ss, rm[threadIdx.x + h], rs[threadIdx.x + h]);
            rm[threadIdx.x] = mm;
            rs[threadIdx.x] = ss;
        }
    }
    if (threadIdx.x == 0) {
        p.ws.bmax[blockIdx.x] = rm[0];
        p.ws.bsum[blockIdx.x] = rs[0];
        if (bad && p.status) p.status[0] = 5;
    }
}

constexpr int kRedThreads = 1024;
__global__ __launch_bounds__(kRedThreads) void lg_lse_reduce_kernel(LargeResParams p) {
    __shared__ double rm[kRedThreads], rs[kRedThreads];
    double m = -INFINITY, s = 0.0;
    for (int c = threadIdx.x; c < p.n_chunks; c += kRedThreads) lse_merge(m, s, p.ws.bmax[c], p.ws.bsum[c]);
    rm[threadIdx.x] = m;
    rs[threadIdx.x] = s;
    for (int h = kRedThreads / 2; h >= 1; h >>= 1) {
        __syncthreads();
        if (threadIdx.x < h) {
            double mm = rm[threadIdx.x], ss = rs[threadIdx.x];
            lse_merge(mm, ss, rm[threadIdx.x + h], rs[threadIdx.x + h]);
            rm[threadIdx.x] = mm;
            rs[threadIdx.x] = ss;
        }
    }
    if (threadIdx.x == 0) {
        p.ws.scal[0] = rm[0];
        p.ws.scal[1] = rs[0];
        if (!isfinite(rm[0]) && p.status) p.status[0] = 5;
    }
}

__global__ __launch_bounds__(kLgThreads) void lg_quant_kernel(LargeResParams p) {
    // one pad slot per 16 entries keeps the per-thread scans of 16
    // consecutive entries off a single LDS bank
    __shared__ double q[kLgChunk + kLgChunk / 16];
    __shared__ double red[kLgThreads / 64];
    __shared__ int redi[kLgThreads / 64];
    __shared__ double tot[kLgThreads / 64];
    const int cbase = blockIdx.x * kLgChunk;
    const double m = p.ws.scal[0], S = p.ws.scal[1];
    const double scale = ldexp((double)p.N, p.bits);
    double sq = 0.0;
    int last = -1, bad = 0;
    for (int k = 0; k < kLgItems; ++k) {
        const int r = k * kLgThreads + threadIdx.x, i = cbase + r;
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
        const double qi = rint(w * scale);
        if (qi > 0.0) last = i;
        q[lg_pad(r)] = qi;
    }
    __syncthreads();
    // chunk-relative inclusive prefix: 16 consecutive entries per thread, then the thread totals
    double run = 0.0;
    for (int k = 0; k < kLgItems; ++k) {
        run += q[lg_pad(threadIdx.x * kLgItems + k)];
        q[lg_pad(threadIdx.x * kLgItems + k)] = run;
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
    for (int k = 0; k < kLgItems; ++k) q[lg_pad(threadIdx.x * kLgItems + k)] += off;
    double total = 0.0;
    for (int w2 = 0; w2 < kLgThreads / 64; ++w2) total += tot[w2];
    __syncthreads();
    if (p.do_resample)
        for (int k = 0; k < kLgItems; ++k) {
            const int r = k * kLgThreads + threadIdx.x;
            if (cbase + r < p.N) p.ws.cloc[cbase + r] = q[lg_pad(r)];
        }
    sq = blk_sum(sq, red);
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
    sq = blk_sum(sq, red);
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

// Particle index of the first output of every block of 4096 outputs (and
// `last` after the final block): the search range of each output block.
__global__ __launch_bounds__(256) void lg_starts_kernel(LargeResParams p) {
    const int blk = blockIdx.x * blockDim.x + threadIdx.x;
    if (blk > p.n_chunks) return;
    const int last = p.ws.last[0];
    if (last < 0) return;
    if (blk == p.n_chunks) {
        p.ws.starts[blk] = last;
        return;
    }
    const double step = ldexp(1.0, p.bits), u = (double)(p.U >> (32 - p.bits));
    p.ws.starts[blk] = global_search(p, (double)blk * kLgChunk * step + u, last);
}

constexpr int kHeavyCopies = 16;  // copies above which a particle's outputs are filled cooperatively
constexpr int kHeavySlots = 64;
__global__ __launch_bounds__(kLgThreads) void lg_search_kernel(LargeResParams p) {
    __shared__ int ids[kLgChunk];
    __shared__ int3 heavy[kHeavySlots];
    __shared__ int n_heavy;
    const int last = p.ws.last[0];
    if (last < 0) return;  // no particle has mass: outputs left untouched, status set
    const int j0 = blockIdx.x * kLgChunk;
    const int n_out = min(kLgChunk, p.N - j0);
    const double inv_step = ldexp(1.0, -p.bits), u = (double)(p.U >> (32 - p.bits));
    // every output of this block is owned by a particle in [starts[blk], starts[blk + 1]]
    const int a = p.ws.starts[blockIdx.x], b = max(a, p.ws.starts[blockIdx.x + 1]);
    // outputs past the total mass (the top edge) take the last positive-mass particle
    for (int r = threadIdx.x; r < n_out; r += kLgThreads) ids[r] = last;
    __syncthreads();
    // particle i owns the outputs j with C_{i-1} <= j 2^b + u < C_i, i.e.
    // ceil((C_{i-1} - u) / 2^b) <= j < ceil((C_i - u) / 2^b): the same index as
    // the first i with C_i > j 2^b + u (all quantities exact integers / powers of two)
    // particles with many copies in this block are filled by the whole workgroup
    for (int base = a; base <= b; base += kLgThreads) {
        if (threadIdx.x == 0) n_heavy = 0;
        __syncthreads();
        const int i = base + threadIdx.x;
        if (i <= b) {
            const double ci = gprefix(p, i);
            const double cp = i > 0 ? gprefix(p, i - 1) : 0.0;
            if (ci > cp) {
                const int js = max(j0, (int)ceil((cp - u) * inv_step));
                const int je = min(j0 + n_out, (int)min(ceil((ci - u) * inv_step), (double)p.N));
                int slot = -1;
                if (je - js > kHeavyCopies) slot = atomicAdd(&n_heavy, 1);
                if (slot >= 0 && slot < kHeavySlots) {
                    heavy[slot] = make_int3(i, js, je);
                } else {
                    for (int j = js; j < je; ++j) ids[j - j0] = i;
                }
            }
        }
        __syncthreads();
        const int nh = min(n_heavy, kHeavySlots);
        for (int h = 0; h < nh; ++h) {
            const int3 e = heavy[h];
            for (int j = e.y + threadIdx.x; j < e.z; j += kLgThreads) ids[j - j0] = e.x;
        }
        __syncthreads();
    }
    for (int r = threadIdx.x; r < n_out; r += kLgThreads) p.idx_out[j0 + r] = ids[r];
}

// The resampled rows: dst row j = src row idx_j, 1024 rows per workgroup.
constexpr int kGatherRows = 1024;
__global__ __launch_bounds__(kLgThreads) void lg_gather_kernel(LargeResParams p) {
    if (p.ws.last[0] < 0) return;
    const int j0 = blockIdx.x * kGatherRows;
    const int n_out = min(kGatherRows, p.N - j0);
    const int rf = p.row_floats;
    const int* ids = p.idx_out + j0;
    if (rf % 4 == 0 && ((reinterpret_cast<uintptr_t>(p.src) | reinterpret_cast<uintptr_t>(p.dst)) & 15) == 0)
        gather_rows(reinterpret_cast<float4*>(p.dst), reinterpret_cast<const float4*>(p.src), ids, j0, n_out, rf / 4);
    else
        gather_rows(p.dst, p.src, ids, j0, n_out, rf);
}

size_t large_res_workspace_bytes(int N) {
    const size_t nc = ((size_t)N + kLgChunk - 1) / kLgChunk;
    auto al = [](size_t x) { return (x + 255) / 256 * 256; };
    return al(nc * 8) * 6 + al(nc * 4) + al((size_t)N * 8) + al(64) + al((nc + 1) * 4) + al((size_t)N * 4);
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
    b += al(64);
    w.starts = reinterpret_cast<int*>(b);
    b += al((nc + 1) * 4);
    w.idx = reinterpret_cast<int*>(b);
    return w;
}

hipError_t launch_large_res(LargeResParams p, hipStream_t s) {
    p.n_chunks = (p.N + kLgChunk - 1) / kLgChunk;
    if (!p.idx_out) p.idx_out = p.ws.idx;  // the gather reads the indices back
    const int nc = p.n_chunks;
    if (!p.w_in) {
        hipLaunchKernelGGL(lg_lse_kernel, nc, kLgThreads, 0, s, p);
        hipLaunchKernelGGL(lg_lse_reduce_kernel, 1, kRedThreads, 0, s, p);
    }
    hipLaunchKernelGGL(lg_quant_kernel, nc, kLgThreads, 0, s, p);
    hipLaunchKernelGGL(lg_scan_kernel, 1, 1024, 0, s, p);
    if (p.do_resample) {
        hipLaunchKernelGGL(lg_starts_kernel, (nc + 1 + 255) / 256, 256, 0, s, p);
        hipLaunchKernelGGL(lg_search_kernel, nc, kLgThreads, 0, s, p);
        if (p.src && p.dst)
            hipLaunchKernelGGL(lg_gather_kernel, (p.N + kGatherRows - 1) / kGatherRows, kLgThreads, 0, s, p);
    }
    return hipGetLastError();
}

}  // namespace voila
