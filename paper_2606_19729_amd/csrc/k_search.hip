// k_search.hip -- planner steps above the rollout core: soft value and action
// selection, the one-level closed-loop tree, grouped progressive widening.
#include "kcommon.hpp"

namespace voila {

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
    if constexpr (!generic_compiled(DT, WIDTH, NHID)) {
        return;  // refused at model creation (binary32 wider than 256) or run by the split rollout kernel
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

// launchers
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

}  // namespace voila
