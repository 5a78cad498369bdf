// resample_large.hip -- weight normalisation and systematic resampling for
// beliefs larger than one workgroup can hold (N > 8192), streamed through HBM.
//
// Blocks of 4096 particles (256 threads, thread t touching particles
// block_base + 256 k + t, k < 16, so global reads are coalesced) for the
// first two passes; the quantised prefix is kept at the granularity of
// 1024-particle chunks.
//   pass 1  per-block (max, sum exp(x - max)) of x_i = l_i / lambda (+ log w_i)
//           in a fixed order                                    -> bmax, bsum
//   red 1   m = max over blocks, S = sum_b bsum_b exp(bmax_b - m) in block order
//   pass 2  w_i = exp(x_i - m) (1 / S) (or given weights), q_i = rint(w_i N 2^b):
//           the total of q of every 1024-particle chunk and of every block
//           (exact), and per block the sum of w_i^2 and the last positive
//           particle (the per-particle prefix is not stored)
//   red 2   exclusive scan of the block totals (one workgroup), statistics
//   pass 3  one workgroup per 1024 consecutive outputs j: the first block
//           whose prefix range reaches the block's first position j0 2^b + u
//           is found by search over the block prefix, and the chunks from
//           there on get their prefix from it and the chunk totals (a running
//           sum of exact integers); for each chunk that meets the positions the
//           q_i are recomputed (the same arithmetic as pass 2; thread t holds
//           particles 4 t .. 4 t + 3) and their chunk-relative inclusive
//           prefix is formed in registers (thread scan, then a scan of the
//           thread totals); each particle writes its index to the outputs it
//           owns (the count form of the search: a particle's copies are the
//           outputs between its two prefix boundaries); outputs past the total
//           mass take the last positive-mass particle; the block then writes
//           its indices and gathers its rows dst_j = src_{idx_j}
// Every prefix is an integer below 2^53, so the blocked sums give the same
// bits as a sequential sum and the indices equal those of the definition.
#include "kernels.hpp"

#include <math.h>

namespace voila {

namespace {

constexpr int kLgThreads = 256;
constexpr int kLgItems = 16;                      // particles per thread in passes 1 and 2
constexpr int kLgBlock = kLgThreads * kLgItems;   // particles per workgroup of passes 1 and 2
constexpr int kLgChunk = 1024;                    // particles per chunk of the quantised prefix
constexpr int kSubPerBlock = kLgBlock / kLgChunk;
constexpr int kChunkItems = kLgChunk / kLgThreads;  // particles per thread in pass 3

__device__ __forceinline__ double lg_x(const LargeResParams& p, int i, int& bad) {
    if (p.x) {
        double x = p.x[i];
        if (isnan(x) || x == INFINITY) bad = 1;
        return x;
    }
    float l = p.loglik[i];
    if (!isfinite(l)) bad = 1;
    // a binary64 division costs a dozen instructions: skipped when lambda = 1
    double x = p.lambda == 1.0 ? (double)l : (double)l / p.lambda;
    if (p.prior_w) x += log(p.prior_w[i]);
    return x;
}

// exp(x) for x <= 0 in binary64, table-driven (P. T. P. Tang, Table-driven
// implementation of the exponential function in IEEE floating-point
// arithmetic, ACM TOMS 15(2), 1989): x = (256 e + j) ln2/256 + r with
// |r| <= ln2/512, exp(x) = 2^e 2^(j/256) exp(r), exp(r) from its degree-5
// Taylor polynomial (truncation below 2^-66 of the result).  ln2/256 is
// split into a 32-bit head (k ln2/256 exact for |k| < 2^21) and a tail.
// `tab` holds 2^(j/256), j < 256 (fill_exp_tab).  Within a few units in the
// last place of exp; x below -745.2 (under the smallest subnormal, and -inf)
// gives 0.
constexpr int kExpTab = 256;
__device__ __forceinline__ void fill_exp_tab(double* tab) {
    for (int j = threadIdx.x; j < kExpTab; j += blockDim.x) tab[j] = exp2((double)j / kExpTab);
    __syncthreads();
}
__device__ __forceinline__ double exp_tab(double x, const double* tab) {
    if (!(x > -745.2)) return 0.0;
    const double kd = rint(x * 369.3299304675746);  // 256 / ln 2
    const int k = (int)kd;
    const double r = fma(-kd, -0x1.718432a1b0e26p-43, fma(-kd, 0x1.62e42ff000000p-9, x));
    const double poly = fma(fma(fma(fma(fma(1.0 / 120, r, 1.0 / 24), r, 1.0 / 6), r, 0.5), r, 1.0), r, 1.0);
    return ldexp(tab[k & (kExpTab - 1)] * poly, k >> 8);
}

// (m, s) <- (m, s) combined with (m2, s2), where s = sum exp(x - m)
// (exponentials of non-positive arguments from the table).
__device__ __forceinline__ void lse_merge(double& m, double& s, double m2, double s2, const double* tab) {
    if (m2 == -INFINITY) return;
    if (m == -INFINITY) {
        m = m2;
        s = s2;
        return;
    }
    if (m2 > m) {
        s = s * exp_tab(m - m2, tab) + s2;
        m = m2;
    } else {
        s += s2 * exp_tab(m2 - m, tab);
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

}  // namespace

__global__ __launch_bounds__(kLgThreads) void lg_lse_kernel(LargeResParams p) {
    __shared__ double rm[kLgThreads / 64], rs[kLgThreads / 64];
    __shared__ int redi[kLgThreads / 64];
    __shared__ double etab[kExpTab];
    fill_exp_tab(etab);
    const int base = blockIdx.x * kLgBlock + threadIdx.x;
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
        for (int k = 0; k < kLgItems; ++k) s += exp_tab(xs[k] - m, etab);
    }
    // fixed-shape tree: lanes merge across the wave (butterfly), then the
    // four wave results in order
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) lse_merge(m, s, __shfl_xor(m, d), __shfl_xor(s, d), etab);
    if ((threadIdx.x & 63) == 0) {
        rm[threadIdx.x >> 6] = m;
        rs[threadIdx.x >> 6] = s;
    }
    bad = blk_max_i(bad, redi);
    if (threadIdx.x == 0) {
        double mm = rm[0], ss = rs[0];
        for (int w = 1; w < kLgThreads / 64; ++w) lse_merge(mm, ss, rm[w], rs[w], etab);
        p.ws.bmax[blockIdx.x] = mm;
        p.ws.bsum[blockIdx.x] = ss;
        if (bad && p.status) p.status[0] = 5;
    }
}

constexpr int kRedThreads = 1024;
__global__ __launch_bounds__(kRedThreads) void lg_lse_reduce_kernel(LargeResParams p) {
    __shared__ double rm[kRedThreads], rs[kRedThreads];
    __shared__ double etab[kExpTab];
    fill_exp_tab(etab);
    double m = -INFINITY, s = 0.0;
    for (int c = threadIdx.x; c < p.n_blocks; c += kRedThreads) lse_merge(m, s, p.ws.bmax[c], p.ws.bsum[c], etab);
    rm[threadIdx.x] = m;
    rs[threadIdx.x] = s;
    for (int h = kRedThreads / 2; h >= 1; h >>= 1) {
        __syncthreads();
        if (threadIdx.x < h) {
            double mm = rm[threadIdx.x], ss = rs[threadIdx.x];
            lse_merge(mm, ss, rm[threadIdx.x + h], rs[threadIdx.x + h], etab);
            rm[threadIdx.x] = mm;
            rs[threadIdx.x] = ss;
        }
    }
    if (threadIdx.x == 0) {
        p.ws.scal[0] = rm[0];
        p.ws.scal[1] = rs[0];
        p.ws.scal[2] = 1.0 / rs[0];  // the weights multiply by 1 / S (one rounding more than a division)
        if (!isfinite(rm[0]) && p.status) p.status[0] = 5;
    }
}

// q_i = rint(w_i N 2^b) of particle i with w_i = exp(x_i - m) (1 / S), or
// the given weight (checked); pass 2 and pass 3 call this same function.
__device__ __forceinline__ double quant_w(const LargeResParams& p, int i, double m, double invS, int& bad, double& w,
                                         const double* etab) {
    if (p.w_in) {
        w = p.w_in[i];
        if (!(w >= 0.0) || w == INFINITY) bad = 1;
    } else {
        w = exp_tab(lg_x(p, i, bad) - m, etab) * invS;
    }
    return rint(w * ldexp((double)p.N, p.bits));
}

__global__ __launch_bounds__(kLgThreads) void lg_quant_kernel(LargeResParams p) {
    __shared__ double red[kLgThreads / 64];
    __shared__ int redi[kLgThreads / 64];
    __shared__ double etab[kExpTab];
    fill_exp_tab(etab);
    const int bbase = blockIdx.x * kLgBlock;
    const double m = p.ws.scal[0], invS = p.ws.scal[2];
    double sq = 0.0, tq[kSubPerBlock];
    int last = -1, bad = 0;
#pragma unroll
    for (int c = 0; c < kSubPerBlock; ++c) tq[c] = 0.0;
#pragma unroll
    for (int k = 0; k < kLgItems; ++k) {
        const int i = bbase + k * kLgThreads + threadIdx.x;  // chunk k / kChunkItems of the block
        if (i < p.N) {
            double w;
            const double q = quant_w(p, i, m, invS, bad, w, etab);
            if (!p.w_in && p.w_out) p.w_out[i] = w;
            sq += w * w;
            tq[k / kChunkItems] += q;  // exact: integers below 2^53
            if (q > 0.0) last = i;
        }
    }
    double bt = 0.0;  // exact: integers below 2^53
#pragma unroll
    for (int c = 0; c < kSubPerBlock; ++c) {
        const double t = blk_sum(tq[c], red);
        const int ci = blockIdx.x * kSubPerBlock + c;
        if (threadIdx.x == 0 && ci < p.n_chunks) p.ws.btot[ci] = t;
        bt += t;
    }
    if (threadIdx.x == 0) p.ws.bbt[blockIdx.x] = bt;
    sq = blk_sum(sq, red);
    last = blk_max_i(last, redi);
    bad = blk_max_i(bad, redi);
    if (threadIdx.x == 0) {
        p.ws.bsq[blockIdx.x] = sq;
        p.ws.blast[blockIdx.x] = last;
        if (bad && p.status) p.status[0] = 5;
    }
}

// One workgroup: exclusive scan of the block totals, global statistics.
// Rounds of 4096 blocks: coalesced loads (the next round's issued before this
// round is scanned), a transpose through LDS so that each thread scans four
// consecutive totals, a scan of the thread totals, coalesced stores.  The
// totals are integers below 2^53: every order of addition gives the same bits.
__global__ __launch_bounds__(1024) void lg_scan_kernel(LargeResParams p) {
    constexpr int T = 1024, R = 4, SPAN = T * R;
    __shared__ double vals[SPAN];
    __shared__ double tot[T / 64];
    __shared__ double red[T / 64];
    __shared__ int redi[T / 64];
    const int nc = p.n_blocks, lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    // the statistics' loads issued together (added in the same order as one
    // at a time: b = t, t + T, ...)
    double sq = 0.0;
    int last = -1;
    for (int b0 = 0; b0 < p.n_blocks; b0 += R * T) {
        double q[R];
        int l[R];
#pragma unroll
        for (int k = 0; k < R; ++k) {
            const int b = b0 + threadIdx.x + T * k;
            q[k] = b < p.n_blocks ? p.ws.bsq[b] : 0.0;
            l[k] = b < p.n_blocks ? p.ws.blast[b] : -1;
        }
#pragma unroll
        for (int k = 0; k < R; ++k) {
            sq += q[k];
            last = max(last, l[k]);
        }
    }
    double v[R], vn[R];
#pragma unroll
    for (int k = 0; k < R; ++k) {
        const int c = threadIdx.x + T * k;
        v[k] = c < nc ? p.ws.bbt[c] : 0.0;
    }
    double carry = 0.0;
    for (int c0 = 0; c0 < nc; c0 += SPAN) {
#pragma unroll
        for (int k = 0; k < R; ++k) vals[threadIdx.x + T * k] = v[k];
#pragma unroll
        for (int k = 0; k < R; ++k) {
            const int c = c0 + SPAN + threadIdx.x + T * k;
            vn[k] = c < nc ? p.ws.bbt[c] : 0.0;
        }
        __syncthreads();
        double e[R], run = 0.0;
#pragma unroll
        for (int k = 0; k < R; ++k) {
            e[k] = run;
            run += vals[R * threadIdx.x + k];
        }
        double incl = run;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const double o = __shfl_up(incl, d);
            if (lane >= d) incl += o;
        }
        if (lane == 63) tot[wave] = incl;
        __syncthreads();
        double off = carry + incl - run, round_total = 0.0;
        for (int w2 = 0; w2 < T / 64; ++w2) {
            if (w2 < wave) off += tot[w2];
            round_total += tot[w2];
        }
#pragma unroll
        for (int k = 0; k < R; ++k) vals[R * threadIdx.x + k] = off + e[k];  // this thread's own slots
        __syncthreads();
#pragma unroll
        for (int k = 0; k < R; ++k) {
            const int c = c0 + threadIdx.x + T * k;
            if (c < nc) {
                const double o = vals[threadIdx.x + T * k];
                p.ws.boff[c] = o;
                p.ws.bincl[c] = o + v[k];
            }
        }
        carry += round_total;
#pragma unroll
        for (int k = 0; k < R; ++k) v[k] = vn[k];
        __syncthreads();  // vals and tot are rewritten by the next round
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

constexpr int kHeavyCopies = 16;  // copies above which a particle's outputs are filled cooperatively
constexpr int kHeavySlots = 64;
constexpr int kOutBlock = kLgChunk;  // outputs per workgroup of pass 3

// dst row j0 + r = src row ids[r] for r < n_out (rows of w elements): each
// thread keeps one column and walks rows, so consecutive threads move
// consecutive elements of a row and of consecutive rows.  The rows are
// streamed with non-temporal loads and stores (read once / written once).
typedef float f32x4_nt __attribute__((ext_vector_type(4)));
template <class T> struct NtType { typedef T type; };
template <> struct NtType<float4> { typedef f32x4_nt type; };
constexpr int kGatherBatch = 16;
template <class T>
__device__ __forceinline__ void gather_rows(T* dst0, const T* src0, const int* ids, int j0, int n_out, int w) {
    typedef typename NtType<T>::type V;
    V* dst = reinterpret_cast<V*>(dst0);
    const V* src = reinterpret_cast<const V*>(src0);
    if (w <= kLgThreads) {
        // up to kGatherBatch rows per thread loaded before any is stored, so
        // that many loads are in flight (the rows never overlap: the sources
        // and the destination are distinct buffers)
        const int rpp = kLgThreads / w, r0 = threadIdx.x / w, c = threadIdx.x - r0 * w;
        if (r0 < rpp) {
            for (int rb = r0; rb < n_out; rb += kGatherBatch * rpp) {
                V v[kGatherBatch];
#pragma unroll
                for (int q = 0; q < kGatherBatch; ++q) {
                    const int r = rb + q * rpp;
                    if (r < n_out) v[q] = __builtin_nontemporal_load(src + (size_t)ids[r] * w + c);
                }
#pragma unroll
                for (int q = 0; q < kGatherBatch; ++q) {
                    const int r = rb + q * rpp;
                    if (r < n_out) __builtin_nontemporal_store(v[q], dst + (size_t)(j0 + r) * w + c);
                }
            }
        }
    } else {
        for (int r = 0; r < n_out; ++r)
            for (int c = threadIdx.x; c < w; c += kLgThreads)
                __builtin_nontemporal_store(__builtin_nontemporal_load(src + (size_t)ids[r] * w + c),
                                            dst + (size_t)(j0 + r) * w + c);
    }
}

__global__ __launch_bounds__(kLgThreads) void lg_resample_kernel(LargeResParams p) {
    __shared__ int ids[kOutBlock];
    __shared__ double etab[kExpTab];
    fill_exp_tab(etab);
    __shared__ int3 heavy[kHeavySlots];
    __shared__ double wtot[kLgThreads / 64];
    __shared__ int n_heavy, s_first;
    const int last = p.ws.last[0];
    if (last < 0) return;  // no particle has mass: outputs left untouched, status set
    const int j0 = blockIdx.x * kOutBlock;
    const int n_out = min(kOutBlock, p.N - j0);
    const double step = ldexp(1.0, p.bits), inv_step = ldexp(1.0, -p.bits);
    const double u = (double)(p.U >> (32 - p.bits));
    const double P0 = (double)j0 * step + u, P1 = (double)(j0 + n_out - 1) * step + u;
    const double m = p.ws.scal[0], invS = p.ws.scal[2];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    // outputs past the total mass (the top edge) take the last positive-mass particle
    for (int r = threadIdx.x; r < n_out; r += kLgThreads) ids[r] = last;
    // first particle block whose inclusive total exceeds the first position:
    // the inclusive totals are non-decreasing, so it is the count of blocks
    // with bincl <= P0, found in two rounds of one test per thread
    if (threadIdx.x == 0) {
        s_first = 0;
        n_heavy = 0;
    }
    __syncthreads();
    {
        const int nb = p.n_blocks;
        const int stride = (nb + kLgThreads - 1) / kLgThreads;  // blocks per segment
        const int c1 = threadIdx.x * stride;
        // segments whose first block is at or below P0 (the answer lies in the last of them)
        const int below = (c1 < nb && p.ws.bincl[c1] <= P0) ? 1 : 0;
        const int nseg = __syncthreads_count(below);
        if (nseg > 0) {
            const int seg0 = (nseg - 1) * stride;
            const int c2 = seg0 + threadIdx.x;
            const int in = (threadIdx.x < stride && c2 < nb && p.ws.bincl[c2] <= P0) ? 1 : 0;
            const int cnt = __syncthreads_count(in);
            if (threadIdx.x == 0) s_first = seg0 + cnt;
        }
    }
    __syncthreads();
    // chunk prefixes from the block's exclusive prefix plus the chunk totals
    // (exact integer sums: the values a chunk-level scan gives)
    const int bf = min(s_first, p.n_blocks - 1);
    double cnext = p.ws.boff[bf];
    for (int c = bf * kSubPerBlock; c < p.n_chunks; ++c) {
        const double coff = cnext;
        cnext = coff + p.ws.btot[c];
        if (cnext <= P0) continue;  // the chunk ends before the block's first position
        if (coff > P1) break;       // this and later chunks own no output of the block
        if (cnext == coff) continue;  // no mass in the chunk
        // this thread's particles i0 .. i0 + 3: q and their inclusive prefix
        const int i0 = c * kLgChunk + kChunkItems * threadIdx.x;
        double qk[kChunkItems], run = 0.0;
        int bad = 0;
#pragma unroll
        for (int k = 0; k < kChunkItems; ++k) {
            double w;
            qk[k] = i0 + k < p.N ? quant_w(p, i0 + k, m, invS, bad, w, etab) : 0.0;
            run += qk[k];
            qk[k] = run;
        }
        // exclusive scan of the thread totals (exact integers: any order gives the same bits)
        double incl = run;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const double o = __shfl_up(incl, d);
            if (lane >= d) incl += o;
        }
        if (lane == 63) wtot[wave] = incl;
        __syncthreads();
        double off = coff + incl - run;
        for (int w2 = 0; w2 < wave; ++w2) off += wtot[w2];
        // particle i owns the outputs j with C_{i-1} <= j 2^b + u < C_i, i.e.
        // ceil((C_{i-1} - u) / 2^b) <= j < ceil((C_i - u) / 2^b): the same index
        // as the first i with C_i > j 2^b + u (exact integers / powers of two);
        // particles with many copies in this block are filled by the whole workgroup
        double cp = off;
#pragma unroll
        for (int k = 0; k < kChunkItems; ++k) {
            const double ci = off + qk[k];
            if (ci > cp) {
                const int js = max(j0, (int)ceil((cp - u) * inv_step));
                const int je = min(j0 + n_out, (int)min(ceil((ci - u) * inv_step), (double)p.N));
                if (je - js > kHeavyCopies) {
                    const int slot = atomicAdd(&n_heavy, 1);
                    if (slot < kHeavySlots) heavy[slot] = make_int3(i0 + k, js, je);
                    else
                        for (int j = js; j < je; ++j) ids[j - j0] = i0 + k;
                } else {
                    for (int j = js; j < je; ++j) ids[j - j0] = i0 + k;
                }
            }
            cp = ci;
        }
        __syncthreads();
        const int nh = min(n_heavy, kHeavySlots);
        for (int h = 0; h < nh; ++h) {
            const int3 e = heavy[h];
            for (int j = e.y + threadIdx.x; j < e.z; j += kLgThreads) ids[j - j0] = e.x;
        }
        __syncthreads();
        if (threadIdx.x == 0) n_heavy = 0;
        __syncthreads();
    }
    if (p.idx_out)
        for (int r = threadIdx.x; r < n_out; r += kLgThreads) p.idx_out[j0 + r] = ids[r];
    if (p.src && p.dst) {
        const int rf = p.row_floats;
        if (rf % 4 == 0 && ((reinterpret_cast<uintptr_t>(p.src) | reinterpret_cast<uintptr_t>(p.dst)) & 15) == 0)
            gather_rows(reinterpret_cast<float4*>(p.dst), reinterpret_cast<const float4*>(p.src), ids, j0, n_out,
                        rf / 4);
        else
            gather_rows(p.dst, p.src, ids, j0, n_out, rf);
    }
}

size_t large_res_workspace_bytes(int N) {
    const size_t nb = ((size_t)N + kLgBlock - 1) / kLgBlock, nc = ((size_t)N + kLgChunk - 1) / kLgChunk;
    auto al = [](size_t x) { return (x + 255) / 256 * 256; };
    return al(nb * 8) * 6 + al(nb * 4) + al(nc * 8) + al(64);
}

LargeResWs carve_large_res(void* base, int N) {
    const size_t nb = ((size_t)N + kLgBlock - 1) / kLgBlock, nc = ((size_t)N + kLgChunk - 1) / kLgChunk;
    auto al = [](size_t x) { return (x + 255) / 256 * 256; };
    char* b = reinterpret_cast<char*>(base);
    LargeResWs w;
    w.bmax = reinterpret_cast<double*>(b); b += al(nb * 8);
    w.bsum = reinterpret_cast<double*>(b); b += al(nb * 8);
    w.bsq = reinterpret_cast<double*>(b); b += al(nb * 8);
    w.blast = reinterpret_cast<int*>(b); b += al(nb * 4);
    w.btot = reinterpret_cast<double*>(b); b += al(nc * 8);
    w.bbt = reinterpret_cast<double*>(b); b += al(nb * 8);
    w.boff = reinterpret_cast<double*>(b); b += al(nb * 8);
    w.bincl = reinterpret_cast<double*>(b); b += al(nb * 8);
    w.scal = reinterpret_cast<double*>(b);
    w.last = reinterpret_cast<int*>(b + 32);
    return w;
}

hipError_t launch_large_res(LargeResParams p, hipStream_t s) {
    p.n_blocks = (p.N + kLgBlock - 1) / kLgBlock;
    p.n_chunks = (p.N + kLgChunk - 1) / kLgChunk;
    if (!p.w_in) {
        hipLaunchKernelGGL(lg_lse_kernel, p.n_blocks, kLgThreads, 0, s, p);
        hipLaunchKernelGGL(lg_lse_reduce_kernel, 1, kRedThreads, 0, s, p);
    }
    hipLaunchKernelGGL(lg_quant_kernel, p.n_blocks, kLgThreads, 0, s, p);
    hipLaunchKernelGGL(lg_scan_kernel, 1, 1024, 0, s, p);
    if (p.do_resample) {
        if (p.idx_out || (p.src && p.dst))
            hipLaunchKernelGGL(lg_resample_kernel, (p.N + kOutBlock - 1) / kOutBlock, kLgThreads, 0, s, p);
    }
    return hipGetLastError();
}

}  // namespace voila
