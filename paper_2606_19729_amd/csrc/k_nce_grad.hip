// k_nce_grad.hip -- derivative of the contrastive (InfoNCE) objective with
// respect to the parameters of a likelihood network evaluated layer by layer
// (hidden width 256), in two stages per chunk of pairs:
//   1. nce_wide_bwd_kernel: every pair (i, j) runs the network forward on
//      [s'_i, a_i, o_j] and the reverse sweep with weight G_ij (Eq. 6), and
//      stores the hidden activations h_1..h_L and the hidden adjoints
//      delta_1..delta_{L-1} in HBM, per unit of 32 pairs (row i, 32
//      consecutive columns j) feature by feature: [array][unit][feature][32];
//   2. nce_wide_wgrad_kernel: the weight derivatives as products over the
//      chunk's pairs, dW_l = sum_p delta_l,p h_{l-1},p^T, on the matrix cores,
//      each workgroup over its own range of pairs (split K) into its own
//      partial sums; the partials are summed in a fixed order at the end.
#include "kcommon.hpp"

namespace voila {

// The shape the streaming source walks: a layered network followed by the
// transposed hidden->hidden layers of the reverse sweep (no output layer).
template <class N> struct BwdStreamShape {
    static constexpr int DT = N::DT, HT = N::HT, FRAG_BYTES = N::FRAG_BYTES, NF0 = N::NF0, NFH = N::NFH;
    static constexpr int NHID = 2 * N::NHID - 1;  // NHID - 1 forward and NHID - 1 transposed blocks
    static constexpr int NFO = 0;
};

template <int DT> struct Elem;
template <> struct Elem<DT_F32> { typedef float type; };
template <> struct Elem<DT_BF16> { typedef __bf16 type; };

// Binary32 values as B operands without the ReLU (adjoints may be negative).
template <int HT>
__device__ __forceinline__ void set_plain(Act<DT_F32, HT>& a, const f32x16 (&acc)[HT]) {
#pragma unroll
    for (int t = 0; t < HT; ++t) a.v[t] = acc[t];
}
template <int HT>
__device__ __forceinline__ void set_plain(Act<DT_BF16, HT>& a, const f32x16 (&acc)[HT]) {
#pragma unroll
    for (int t = 0; t < HT; ++t)
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            bf16x8 r;
#pragma unroll
            for (int q = 0; q < 8; ++q) r[q] = (__bf16)acc[t][8 * h + q];
            a.v[2 * t + h] = r;
        }
}
// Element (t, i) of an operand set (the value the matrix cores consume).
template <int HT>
__device__ __forceinline__ float act_at(const Act<DT_F32, HT>& a, int t, int i) { return a.v[t][i]; }
template <int HT>
__device__ __forceinline__ __bf16 act_at(const Act<DT_BF16, HT>& a, int t, int i) { return a.v[2 * t + (i >> 3)][i & 7]; }

template <int DT, int D_O, int WIDTH, int NHID>
__global__ __launch_bounds__(256) void nce_wide_bwd_kernel(NceWideParams p) {
    typedef Net<DT, WIDTH, NHID, in_slots(DT, D_O, 0, 0), WIDTH / 32> NT;
    typedef BwdStreamShape<NT> SH;
    typedef typename Frag<DT>::type FT;
    typedef FragIdx<NT> FI;
    typedef typename Elem<DT>::type ET;
    constexpr int HT = NT::HT, SO = state_slots(D_O);
#ifndef VOILA_NCE_BWD_DEPTH
#define VOILA_NCE_BWD_DEPTH 4
#endif
    constexpr int DEPTH = DT == DT_F32 ? VOILA_NCE_BWD_DEPTH : kPfDepth;
    static_assert(HT % 2 == 0, "two tiles of ReLU bits per mask word");
    extern __shared__ __attribute__((aligned(16))) char smem[];
    const int lane = threadIdx.x & 63, g = lane >> 5, col = lane & 31;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    float* bh = reinterpret_cast<float*>(smem + p.lds_bias);
    float* wo = bh + (NHID - 1) * WIDTH;
    float* rowb = wo + WIDTH + wave * WIDTH;
    for (int k = threadIdx.x; k < (NHID - 1) * WIDTH; k += blockDim.x) bh[k] = p.bh[k];
    for (int k = threadIdx.x; k < WIDTH; k += blockDim.x) wo[k] = p.w_out[k];
    __syncthreads();
    StreamSrc<SH> src(smem, p.stream);
    src.start();
    constexpr int RB = WIDTH / 64;  // bias floats per lane
    const int jtiles = (p.B + 31) / 32;
    int have = -1;
    // block-uniform loop: the stream's chunk barriers need every wave
    for (long ub = blockIdx.x; p.u0 + ub * 4 < p.u1; ub += gridDim.x) {
        const long u = p.u0 + ub * 4 + wave;
        const bool ok = u < p.u1;
        const int i = ok ? (int)(u / jtiles) : 0;
        const int j = ok ? (int)(u - (long)i * jtiles) * 32 + col : 0;
        const bool valid = ok && j < p.B;
        float slots[NT::IN_SLOTS];
#pragma unroll
        for (int s = 0; s < NT::IN_SLOTS; ++s) slots[s] = 0.0f;
#pragma unroll
        for (int s = 0; s < SO; ++s) {
            const int f = 2 * s + g;
            slots[s] = (valid && f < D_O) ? p.obs[(size_t)j * D_O + f] : 0.0f;
        }
        const bool fresh = i != have;  // wave-uniform
        float bv[RB];
        if (fresh) {
            const float* brow = p.b0 + (size_t)i * WIDTH;
#pragma unroll
            for (int q = 0; q < RB; ++q) bv[q] = brow[q * 64 + lane];
        }
        const float gc = valid ? p.grad[(size_t)i * p.B + j] : 0.0f;
        __builtin_amdgcn_s_waitcnt(waitcnt_vm_lgkm0(0));
        if (fresh) {
#pragma unroll
            for (int q = 0; q < RB; ++q) rowb[q * 64 + lane] = bv[q];
            __builtin_amdgcn_s_waitcnt(waitcnt_vm_lgkm0(0));
            __builtin_amdgcn_wave_barrier();
            have = i;
        }
        // feature 32 t + out_row(r, g) of array a for this lane's pair: a
        // column of the unit's [feature][32] block (every lane of a unit
        // inside the chunk stores; columns past B hold finite values whose
        // adjoints and G are zero)
        const long ul = u - p.u0;
        auto put_all = [&](int a, const Act<DT, HT>& v) {
            ET* base = reinterpret_cast<ET*>(p.act) + (((size_t)a * p.uc + ul) * WIDTH + 4 * g) * 32 + col +
                       opaque_zero();
            if (ok)
#pragma unroll
                for (int t = 0; t < HT; ++t)
#pragma unroll
                    for (int r = 0; r < 16; ++r) base[(32 * t + 8 * (r >> 2) + (r & 3)) * 32] = (ET)act_at(v, t, r);
        };
        f32x16 acc[HT];
        Act<DT, HT> act;
        uint32_t mask[NHID - 1][HT / 2];
        auto keep_mask = [&](int l) {  // ReLU pattern of hidden layer l + 1 (pre-activations in acc)
#pragma unroll
            for (int w = 0; w < HT / 2; ++w) {
                uint32_t m = 0;
#pragma unroll
                for (int h = 0; h < 2; ++h)
#pragma unroll
                    for (int r = 0; r < 16; ++r) m |= (acc[2 * w + h][r] > 0.0f ? 1u : 0u) << (16 * h + r);
                mask[l][w] = m;
            }
        };
        // forward: h_1 = ReLU(b0_i + W_1,obs o_j), h_{l+1} = ReLU(b_{l+1} + W_{l+1} h_l)
        init_bias<HT>(acc, rowb + opaque_zero(), g);
        mfma_layer<NT::IN_KS, HT, 2, FT>(
            acc, [&](int c, int t) { return src.load(FI::first(c, t), lane); },
            [&](int c) { return Slots<DT, NT::IN_SLOTS>::b(slots, c); });
        act.set_relu(acc);
        keep_mask(0);
        put_all(0, act);
        static_for<NHID - 1>([&](auto li) {
            constexpr int l = decltype(li)::value + 1;
            init_bias<HT>(acc, bh + (l - 1) * WIDTH + opaque_zero(), g);
            mfma_layer<NT::HID_KS, HT, DEPTH, FT>(
                acc, [&](int c, int t) { return src.load(FI::hidden(l, c, t), lane); },
                [&](int c) { return act.b(c); });
            act.set_relu(acc);
            if constexpr (l < NHID - 1) keep_mask(l);
            put_all(l, act);
        });
        // adjoint of the last hidden layer's pre-activation: G_ij w_out on its active units
#pragma unroll
        for (int t = 0; t < HT; ++t)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[t][r] = acc[t][r] > 0.0f ? wo[32 * t + out_row(r, g)] * gc : 0.0f;
        set_plain(act, acc);
        // reverse sweep: delta_l = (W_{l+1}^T delta_{l+1}) on the active units of h_l
        static_for<NHID - 1>([&](auto ki) {
            constexpr int k = decltype(ki)::value;
            constexpr int l = NHID - 1 - k;  // layer whose adjoint this step produces
            constexpr int base = NT::NF0 + (NHID - 1 + k) * NT::NFH;
#pragma unroll
            for (int t = 0; t < HT; ++t) acc[t] = f32x16{};
            mfma_layer<NT::HID_KS, HT, DEPTH, FT>(
                acc, [&](int c, int t) { return src.load(base + c * HT + t, lane); },
                [&](int c) { return act.b(c); });
#pragma unroll
            for (int t = 0; t < HT; ++t)
#pragma unroll
                for (int r = 0; r < 16; ++r)
                    if (!((mask[l - 1][t >> 1] >> (16 * (t & 1) + r)) & 1u)) acc[t][r] = 0.0f;
            set_plain(act, acc);
            put_all(NHID - 1 + l, act);
        });
    }
    src.finish();
}

// ---------------------------------------------------------------------------
// stage 2: weight derivatives as split-K products over the chunk's pairs
// ---------------------------------------------------------------------------
template <int DT> struct WgCfg;
template <> struct WgCfg<DT_F32> {
    static constexpr int KC = 32, PAD = 1, VEC = 4;  // pairs per staged chunk, row padding, elements per load
};
template <> struct WgCfg<DT_BF16> {
    static constexpr int KC = 64, PAD = 8, VEC = 8;
};

template <int DT> struct WgVec;
template <> struct WgVec<DT_F32> { typedef f32x4 type; };
template <> struct WgVec<DT_BF16> { typedef bf16x8 type; };

// VEC consecutive elements of a feature-major row (zero past the chunk's
// last pair).
template <int DT>
__device__ __forceinline__ typename WgVec<DT>::type load_vec(const typename Elem<DT>::type* src, int n_ok) {
    typedef typename WgVec<DT>::type VT;
    constexpr int VEC = WgCfg<DT>::VEC;
    if (n_ok >= VEC) return *reinterpret_cast<const VT*>(src);
    VT v;
#pragma unroll
    for (int q = 0; q < VEC; ++q) v[q] = q < n_ok ? src[q] : (typename Elem<DT>::type)0.0f;
    return v;
}

// Writes VEC operand elements into an LDS row.
template <int DT>
__device__ __forceinline__ void store_vec(typename Elem<DT>::type* dst, const typename WgVec<DT>::type& v) {
    if constexpr (DT == DT_F32) {
#pragma unroll
        for (int q = 0; q < 4; ++q) dst[q] = v[q];  // rows are padded to an odd stride: no vector store
    } else {
        *reinterpret_cast<bf16x8*>(dst) = v;
    }
}

template <int DT> struct WgFrag;
template <> struct WgFrag<DT_F32> {
    // A / B operand of k-step s: row r of the staged tile, pair 2 s + (lane / 32)
    __device__ static __forceinline__ float load(const float* t, int row, int s, int lane) {
        return t[row * (WgCfg<DT_F32>::KC + WgCfg<DT_F32>::PAD) + 2 * s + (lane >> 5)];
    }
    static constexpr int KSTEPS = WgCfg<DT_F32>::KC / 2;
};
template <> struct WgFrag<DT_BF16> {
    // pairs 16 s + 8 (lane / 32) .. + 7 of row r
    __device__ static __forceinline__ bf16x8 load(const __bf16* t, int row, int s, int lane) {
        return *reinterpret_cast<const bf16x8*>(t + row * (WgCfg<DT_BF16>::KC + WgCfg<DT_BF16>::PAD) + 16 * s +
                                                8 * (lane >> 5));
    }
    static constexpr int KSTEPS = WgCfg<DT_BF16>::KC / 16;
};

// One weight derivative over this workgroup's units [v0, v1) of the chunk:
// C[m][n] = sum_p A[m][p] B[n][p] with A the layer's output adjoints (formed
// from the last hidden layer, G and w_out when FORMED) and B its inputs (the
// previous hidden layer, or the network input [s'_i, a_i, o_j] when XIN), and
// the adjoint's sum over pairs (the bias derivative).  Results go to the
// workgroup's partial sums: dW at w_off (row-major [WIDTH][n_in]), the bias
// derivative at b_off; with FORMED also the output layer's derivatives
// (sum_p G_p h_L,p at o_off, sum_p G_p at o_off + WIDTH).
template <int DT, int WIDTH, int NB, bool FORMED, bool XIN>
__device__ __forceinline__ void wgrad_pass(const NceWgradParams& p, int a_idx, int b_idx, int n_in, int w_off,
                                           int b_off, int o_off, long v0, long v1, char* smem) {
    typedef typename Elem<DT>::type ET;
    typedef WgCfg<DT> CF;
    typedef typename WgVec<DT>::type VT;
    constexpr int KC = CF::KC, VEC = CF::VEC, STR = KC + CF::PAD;
    constexpr int UPC = KC / 32;                             // units per staged chunk
    constexpr int WR = NB == WIDTH ? 2 : 4, WC = 4 / WR;  // waves along rows / columns of C
    constexpr int RT = WIDTH / 32 / WR, CT = NB / 32 / WC;  // 32x32 tiles per wave
    constexpr int PR = KC / VEC;                             // loads per staged row
    constexpr int A_IT = WIDTH * PR / 256, B_IT = NB * PR / 256;
    static_assert(PR == 8 && WIDTH * PR % 256 == 0 && NB * PR % 256 == 0, "staging map");
    ET* As = reinterpret_cast<ET*>(smem);
    ET* Bs = As + WIDTH * STR;
    const int tid = threadIdx.x, lane = tid & 63, g = lane >> 5, col = lane & 31;
    const int wave = tid >> 6, wr = wave / WC, wc = wave % WC;
    const int cg = tid & 7;            // this thread's column group of a staged row
    const int r0 = tid >> 3;           // its first staged row (then every 32nd)
    const int ku = cg * VEC / 32, c0 = cg * VEC % 32;  // unit within the staged chunk, first column
    const int d_in = n_in;
    const int aw = p.n_actions > 0 ? p.n_actions : p.d_a;
    const int jtiles = (p.B + 31) / 32;

    f32x16 acc[RT][CT];
#pragma unroll
    for (int a = 0; a < RT; ++a)
#pragma unroll
        for (int b = 0; b < CT; ++b) acc[a][b] = f32x16{};
    float sd[A_IT], so[A_IT], sg = 0.0f;  // running sums: adjoint, G h (FORMED), G
#pragma unroll
    for (int it = 0; it < A_IT; ++it) sd[it] = so[it] = 0.0f;
    float wv[A_IT];
    if constexpr (FORMED) {
#pragma unroll
        for (int it = 0; it < A_IT; ++it) wv[it] = p.w_out[r0 + 32 * it];
    }

    VT ra[A_IT], rb[B_IT];
    auto fetch = [&](long v) {
        const long uu = v + ku;  // this thread's unit (local to the chunk)
        const bool in = uu < v1;
        // pairs of this thread's columns: row i, columns j0 .. j0 + VEC - 1
        const long ug = p.u0 + uu;
        const int i = (int)(ug / jtiles), j0 = (int)(ug - (long)i * jtiles) * 32 + c0;
        float gv[VEC];
        if constexpr (FORMED) {
#pragma unroll
            for (int e = 0; e < VEC; ++e) gv[e] = (in && j0 + e < p.B) ? p.grad[(size_t)i * p.B + j0 + e] : 0.0f;
        }
        const ET* Ab = reinterpret_cast<const ET*>(p.act) +
                       (((size_t)a_idx * p.uc + (in ? uu : 0)) * WIDTH + r0) * 32 + c0 + opaque_zero();
#pragma unroll
        for (int it = 0; it < A_IT; ++it) {
            if (in) {
                ra[it] = *reinterpret_cast<const VT*>(Ab + it * 32 * 32);
            } else {
#pragma unroll
                for (int e = 0; e < VEC; ++e) ra[it][e] = (ET)0.0f;
            }
            if constexpr (FORMED) {
                // delta = G w_out on the active units of the last hidden layer
#pragma unroll
                for (int e = 0; e < VEC; ++e) {
                    const float h = (float)ra[it][e];
                    so[it] = __builtin_fmaf(gv[e], h, so[it]);
                    ra[it][e] = (ET)(h > 0.0f ? wv[it] * gv[e] : 0.0f);
                }
                if (r0 == 0 && it == 0)
#pragma unroll
                    for (int e = 0; e < VEC; ++e) sg += gv[e];
            }
#pragma unroll
            for (int e = 0; e < VEC; ++e) sd[it] += (float)ra[it][e];
        }
        if constexpr (XIN) {
            // network input [s'_i, a_i, o_j] of the pairs, zero past d_in and past B
            int a = 0;
            if (p.n_actions > 0 && in) {
                a = reinterpret_cast<const int32_t*>(p.actions)[i];
                if (a < 0 || a >= p.n_actions) a = 0;  // as the forward pass
            }
#pragma unroll
            for (int it = 0; it < B_IT; ++it) {
                const int r = r0 + 32 * it;
#pragma unroll
                for (int e = 0; e < VEC; ++e) {
                    const int j = j0 + e;
                    float v = 0.0f;
                    if (in && j < p.B && r < d_in) {
                        if (r < p.d_s) {
                            v = p.states[(size_t)i * p.d_s + r];
                        } else if (r < p.d_s + aw) {
                            if (p.n_actions > 0) v = (r - p.d_s == a) ? 1.0f : 0.0f;
                            else v = reinterpret_cast<const float*>(p.actions)[(size_t)i * p.d_a + (r - p.d_s)];
                        } else {
                            v = p.obs[(size_t)j * p.d_o + (r - p.d_s - aw)];
                        }
                    }
                    rb[it][e] = (ET)v;
                }
            }
        } else {
            const ET* Bb = reinterpret_cast<const ET*>(p.act) +
                           (((size_t)b_idx * p.uc + (in ? uu : 0)) * WIDTH + r0) * 32 + c0 + opaque_zero();
#pragma unroll
            for (int it = 0; it < B_IT; ++it) {
                if (in) {
                    rb[it] = *reinterpret_cast<const VT*>(Bb + it * 32 * 32);
                } else {
#pragma unroll
                    for (int e = 0; e < VEC; ++e) rb[it][e] = (ET)0.0f;
                }
            }
        }
    };
    auto stage = [&]() {
#pragma unroll
        for (int it = 0; it < A_IT; ++it) store_vec<DT>(As + (r0 + 32 * it) * STR + cg * VEC, ra[it]);
#pragma unroll
        for (int it = 0; it < B_IT; ++it) store_vec<DT>(Bs + (r0 + 32 * it) * STR + cg * VEC, rb[it]);
    };
    if (v0 < v1) {
        fetch(v0);
        stage();
    }
    __syncthreads();
    for (long v = v0; v < v1; v += UPC) {
        if (v + UPC < v1) fetch(v + UPC);  // next chunk into registers while this one multiplies
#pragma unroll
        for (int s = 0; s < WgFrag<DT>::KSTEPS; ++s) {
            typename Frag<DT>::type af[RT], bf[CT];
#pragma unroll
            for (int a = 0; a < RT; ++a) af[a] = WgFrag<DT>::load(As, 32 * (wr * RT + a) + col, s, lane);
#pragma unroll
            for (int b = 0; b < CT; ++b) bf[b] = WgFrag<DT>::load(Bs, 32 * (wc * CT + b) + col, s, lane);
#pragma unroll
            for (int a = 0; a < RT; ++a)
#pragma unroll
                for (int b = 0; b < CT; ++b) acc[a][b] = mfma(af[a], bf[b], acc[a][b]);
        }
        __syncthreads();
        if (v + UPC < v1) stage();
        __syncthreads();
    }
    // partial sums of this workgroup (written by the first chunk, added to afterwards)
    float* part = p.part + (size_t)blockIdx.x * p.n_params;
#pragma unroll
    for (int a = 0; a < RT; ++a)
#pragma unroll
        for (int b = 0; b < CT; ++b) {
            const int n = 32 * (wc * CT + b) + col;
            if (n < n_in)
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    const int m = 32 * (wr * RT + a) + out_row(r, g);
                    float* d = part + w_off + (size_t)m * n_in + n;
                    *d = (p.accumulate ? *d : 0.0f) + acc[a][b][r];
                }
        }
    // row sums: the eight threads of a staged row combine theirs (fixed order)
#pragma unroll
    for (int it = 0; it < A_IT; ++it) {
        float v = sd[it], o = so[it];
#pragma unroll
        for (int m = 1; m < 8; m <<= 1) {
            v += __shfl_xor(v, m);
            if constexpr (FORMED) o += __shfl_xor(o, m);
        }
        if (cg == 0) {
            const int r = r0 + 32 * it;
            float* d = part + b_off + r;
            *d = (p.accumulate ? *d : 0.0f) + v;
            if constexpr (FORMED) {
                float* e = part + o_off + r;
                *e = (p.accumulate ? *e : 0.0f) + o;
            }
        }
    }
    if constexpr (FORMED) {
#pragma unroll
        for (int m = 1; m < 8; m <<= 1) sg += __shfl_xor(sg, m);
        if (tid == 0) {
            float* e = part + o_off + WIDTH;
            *e = (p.accumulate ? *e : 0.0f) + sg;
        }
    }
    __syncthreads();
}

template <int DT, int WIDTH, int NHID, int XW>
__global__ __launch_bounds__(256) void nce_wide_wgrad_kernel(NceWgradParams p) {
    extern __shared__ __attribute__((aligned(16))) char smem[];
    const long per = p.per_split;
    const long q0 = min((long)blockIdx.x * per, p.n_units), q1 = min(q0 + per, p.n_units);
    const int d_in = p.d_in;
    // parameter offsets: layer l has W_l [out][in] then b_l
    int off[NHID + 2];
    off[0] = 0;
    off[1] = WIDTH * d_in + WIDTH;
#pragma unroll
    for (int l = 2; l <= NHID; ++l) off[l] = off[l - 1] + WIDTH * WIDTH + WIDTH;
    // last hidden layer: adjoint formed from h_NHID and G; input h_{NHID-1}; output layer's sums
    wgrad_pass<DT, WIDTH, WIDTH, true, false>(p, NHID - 1, NHID - 2, WIDTH, off[NHID - 1],
                                              off[NHID - 1] + WIDTH * WIDTH, off[NHID], q0, q1, smem);
    // hidden->hidden layers L = NHID - 2 .. 1: stored adjoint delta_{L+1}, input h_L
#pragma unroll
    for (int L = NHID - 2; L >= 1; --L)
        wgrad_pass<DT, WIDTH, WIDTH, false, false>(p, NHID + L, L - 1, WIDTH, off[L], off[L] + WIDTH * WIDTH, 0,
                                                   q0, q1, smem);
    // first layer: adjoint delta_1, input [s'_i, a_i, o_j]
    wgrad_pass<DT, WIDTH, XW, false, true>(p, NHID, 0, d_in, off[0], off[0] + WIDTH * d_in, 0, q0, q1, smem);
}

// ---------------------------------------------------------------------------
// launchers (the realistic shape: width 256, three hidden layers, d_o = 32)
// ---------------------------------------------------------------------------
namespace {
template <int DT> constexpr size_t bwd_lds() {
    typedef Net<DT, 256, 3, in_slots(DT, 32, 0, 0), 8> NT;
    return (size_t)StreamSrc<BwdStreamShape<NT>>::LDS_BYTES;
}
template <int DT> constexpr size_t wgrad_lds() {
    return (size_t)2 * 256 * (WgCfg<DT>::KC + WgCfg<DT>::PAD) * (DT == DT_F32 ? 4 : 2);
}
}  // namespace

bool nce_wide_supported(int shape) { return shape == 1; }

size_t nce_wide_bwd_lds(int dt) {
    // stream buffers, then hidden biases, output weights and one bias row per wave
    const size_t s = dt == DT_F32 ? bwd_lds<DT_F32>() : bwd_lds<DT_BF16>();
    return s + (size_t)(2 + 1 + kWavesPerBlock) * 256 * 4;
}

hipError_t launch_nce_wide_bwd(int shape, int dt, const NceWideParams& p0, int blocks, hipStream_t s) {
    if (shape != 1) return hipErrorInvalidValue;
    NceWideParams p = p0;
    const size_t lds = nce_wide_bwd_lds(dt);
    p.lds_bias = (uint32_t)(dt == DT_F32 ? bwd_lds<DT_F32>() : bwd_lds<DT_BF16>());
    if (dt == DT_F32) {
        (void)hipFuncSetAttribute((const void*)nce_wide_bwd_kernel<DT_F32, 32, 256, 3>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        hipLaunchKernelGGL((nce_wide_bwd_kernel<DT_F32, 32, 256, 3>), blocks, 256, lds, s, p);
    } else {
        (void)hipFuncSetAttribute((const void*)nce_wide_bwd_kernel<DT_BF16, 32, 256, 3>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        hipLaunchKernelGGL((nce_wide_bwd_kernel<DT_BF16, 32, 256, 3>), blocks, 256, lds, s, p);
    }
    return hipGetLastError();
}

hipError_t launch_nce_wide_wgrad(int shape, int dt, const NceWgradParams& p, int blocks, hipStream_t s) {
    if (shape != 1) return hipErrorInvalidValue;
    if (dt == DT_F32) {
        const size_t lds = wgrad_lds<DT_F32>();
        (void)hipFuncSetAttribute((const void*)nce_wide_wgrad_kernel<DT_F32, 256, 3, 64>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        hipLaunchKernelGGL((nce_wide_wgrad_kernel<DT_F32, 256, 3, 64>), blocks, 256, lds, s, p);
    } else {
        const size_t lds = wgrad_lds<DT_BF16>();
        (void)hipFuncSetAttribute((const void*)nce_wide_wgrad_kernel<DT_BF16, 256, 3, 64>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        hipLaunchKernelGGL((nce_wide_wgrad_kernel<DT_BF16, 256, 3, 64>), blocks, 256, lds, s, p);
    }
    return hipGetLastError();
}

int nce_wide_bwd_blocks_per_cu(int dt) {
    return dt == DT_F32 ? occupancy(nce_wide_bwd_kernel<DT_F32, 32, 256, 3>, nce_wide_bwd_lds(DT_F32))
                        : occupancy(nce_wide_bwd_kernel<DT_BF16, 32, 256, 3>, nce_wide_bwd_lds(DT_BF16));
}

int nce_wide_wgrad_blocks_per_cu(int dt) {
    return dt == DT_F32 ? occupancy(nce_wide_wgrad_kernel<DT_F32, 256, 3, 64>, wgrad_lds<DT_F32>())
                        : occupancy(nce_wide_wgrad_kernel<DT_BF16, 256, 3, 64>, wgrad_lds<DT_BF16>());
}

}  // namespace voila
