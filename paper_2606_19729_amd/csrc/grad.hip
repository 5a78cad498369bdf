// grad.hip -- adjoint (reverse-mode) rollout kernel with step checkpointing.
//
// Differentiates free-running rollouts s_{t+1} = s_t + f_T([s_t, a_t, w_t]) of
// a transition network with two hidden layers of width 64 (binary32):
//   distillation objective  L = 1/(B H) sum_b sum_{t=1..H} ||s_{b,t} - T_{b,t}||^2
//   (the distillation loss of Eq. 3 along rollouts, T = teacher states), and
//   return objective        J = 1/B sum_b sum_{t<H} gamma^t (-||s_{b,t+1} - g||^2),
// giving d/d(network parameters) and, for continuous actions, d/dA.
//
// One wave owns a tile of 32 rollouts.  The forward pass keeps the states in
// registers and stores a checkpoint every C steps in the workspace.  The
// reverse sweep walks the segments backwards: it recomputes the segment's
// states from its checkpoint, then for each step (last first) recomputes the
// step's activations, and back-propagates the state adjoint through the
// layers with MFMAs whose A operands are the *transposed* weights packed so
// that every adjoint comes out in exactly the register layout of the matching
// forward activation (ReLU masks are register-wise).  Weight gradients
// dW += dh h^T are products over the 32 rollouts of the tile: the wave writes
// (dh, h) as [rollout][feature] rows into its own LDS scratch (row stride 129
// floats, conflict-free) and accumulates them on MFMA with rollouts as the
// reduction dimension.  Each wave writes its parameter-gradient partial once;
// a second kernel sums the partials in a fixed order (deterministic).
#include "kernels.hpp"

#include <math.h>

namespace voila {

namespace {

constexpr int kRow = 129;  // floats per rollout row of the transpose scratch

// Fragment indices of the transposed pack: [T3: KS3 x HT][T2: 16HT x HT][T1: 16HT x 1]
template <int D_S, int HT> struct BwdIdx {
    static constexpr int KS3 = cdiv(D_S, 2);
    __device__ static constexpr int t3(int c, int mt) { return c * HT + mt; }
    __device__ static constexpr int t2(int c, int mt) { return KS3 * HT + c * HT + mt; }
    __device__ static constexpr int t1(int c) { return KS3 * HT + 16 * HT * HT + c; }
};

__device__ __forceinline__ float lds_frag(const char* base, int f, int lane) {
    return reinterpret_cast<const float*>(base)[f * 64 + lane];
}

}  // namespace

template <int D_S, int N_ACT, int D_A, int D_W>
__global__ __launch_bounds__(256) void grad_kernel(GradParams p) {
    constexpr int WIDTH = 64, NHID = 2, HT = 2;
    constexpr int D_AIN = N_ACT > 0 ? N_ACT : D_A;
    constexpr int SS = state_slots(D_S), SA = action_slots(D_AIN), SW = noise_slots(D_W);
    constexpr int D_IN = D_S + D_AIN + D_W;
    static_assert(D_IN <= 31 && D_S <= 32, "inputs must fit one 32-row tile (column 31 carries the bias)");
    typedef Net<DT_F32, WIDTH, NHID, in_slots(DT_F32, D_S, D_AIN, D_W)> NT;
    typedef BwdIdx<D_S, HT> BI;
    extern __shared__ __attribute__((aligned(16))) char smem[];
    stage_blob(smem, p.fwd.base, p.fwd.bytes);
    stage_blob(smem + p.fwd.bytes, p.bwd.base, p.bwd.bytes);
    __syncthreads();
    const NetPtrs P = net_ptrs(smem, p.fwd);
    const char* bw = smem + p.fwd.bytes;
    const int lane = threadIdx.x & 63, g = lane >> 5, col = lane & 31;
    const int wpb = blockDim.x >> 6, wave = threadIdx.x >> 6;
    float* scr = reinterpret_cast<float*>(smem + p.fwd.bytes + p.bwd.bytes) + wave * 32 * kRow;

    // weight-gradient accumulators (MFMA layouts) and per-lane bias sums
    f32x16 gW1[HT], gW2[HT][HT], gW3[HT];
#pragma unroll
    for (int a = 0; a < HT; ++a) {
        gW1[a] = f32x16{};
        gW3[a] = f32x16{};
#pragma unroll
        for (int b = 0; b < HT; ++b) gW2[a][b] = f32x16{};
    }
    f32x16 gb2[HT];
#pragma unroll
    for (int a = 0; a < HT; ++a) gb2[a] = f32x16{};
    float gb3[SS];
#pragma unroll
    for (int s = 0; s < SS; ++s) gb3[s] = 0.0f;
    float loss_acc = 0.0f;

    // input slots of step t for rollout b from state slots st
    auto make_slots = [&](float (&slots)[NT::IN_SLOTS], const float* st, int b, bool valid, int t) {
#pragma unroll
        for (int s = 0; s < NT::IN_SLOTS; ++s) slots[s] = 0.0f;
#pragma unroll
        for (int s = 0; s < SS; ++s) slots[s] = st[s];
        if (N_ACT > 0) {
            const int a = valid ? reinterpret_cast<const int32_t*>(p.actions)[(size_t)b * p.H + t] : -1;
#pragma unroll
            for (int s = 0; s < SA; ++s) slots[SS + s] = (2 * s + g == a) ? 1.0f : 0.0f;
        } else {
            const float* av =
                reinterpret_cast<const float*>(p.actions) + ((size_t)(valid ? b / p.particles : 0) * p.H + t) * D_A;
#pragma unroll
            for (int s = 0; s < SA; ++s) {
                int f = 2 * s + g;
                slots[SS + s] = f < D_A ? av[f] : 0.0f;
            }
        }
        if (p.noise) {
            const float* nz = p.noise + ((size_t)(valid ? b : 0) * p.H + t) * D_W;
#pragma unroll
            for (int s = 0; s < SW; ++s) {
                int f = noise_feature(s, g);
                slots[SS + SA + s] = f < D_W ? nz[f] : 0.0f;
            }
        } else {
            float nz[SW];
            noise_slots_philox<SW>(nz, p.key0, p.key1, (uint32_t)b, 0u, (uint32_t)t, 3u, g);
#pragma unroll
            for (int s = 0; s < SW; ++s) slots[SS + SA + s] = nz[s];
        }
    };
    // input column of slot s of this lane group (-1: padding)
    auto slot_col = [&](int s) -> int {
        if (s < SS) return 2 * s + g < D_S ? 2 * s + g : -1;
        if (s < SS + SA) return 2 * (s - SS) + g < D_AIN ? D_S + 2 * (s - SS) + g : -1;
        if (s < SS + SA + SW) {
            int f = noise_feature(s - SS - SA, g);
            return f < D_W ? D_S + D_AIN + f : -1;
        }
        return -1;
    };

    const int n_tiles = (p.B + 31) / 32;
    for (long ub = blockIdx.x; ub * wpb < n_tiles; ub += gridDim.x) {
        const int tile = (int)(ub * wpb + wave);
        const bool tile_ok = tile < n_tiles;
        const int b = (tile_ok ? tile : 0) * 32 + col;
        const bool valid = tile_ok && b < p.B;
        float st[SS];
#pragma unroll
        for (int s = 0; s < SS; ++s) {
            int f = 2 * s + g;
            st[s] = (valid && f < D_S) ? p.s0[(size_t)b * D_S + f] : 0.0f;
        }
        // ---- forward with checkpoints
        for (int t = 0; t < p.H; ++t) {
            if (t % p.C == 0 && valid)
#pragma unroll
                for (int s = 0; s < SS; ++s)
                    if (2 * s + g < D_S) p.ckpt[((size_t)b * p.NC + t / p.C) * D_S + 2 * s + g] = st[s];
            float slots[NT::IN_SLOTS];
            make_slots(slots, st, b, valid, t);
            DirectSrc<DT_F32, 8 * HT> src(P.f0);
            f32x16 d = run_net<NT>(src, P, P.b0, slots, lane, g);
            float part = 0.0f;
#pragma unroll
            for (int s = 0; s < SS; ++s) {
                st[s] += d[s];
                int f = 2 * s + g;
                if (f < D_S && valid) {
                    float e = p.objective == 0 ? st[s] - p.targets[((size_t)b * p.H + t) * D_S + f] : st[s] - p.goal[f];
                    part += e * e;
                }
            }
            loss_acc += p.objective == 0 ? part : -p.disc[t] * part;
        }
        // ---- reverse sweep over the segments
        float lam[SS];
#pragma unroll
        for (int s = 0; s < SS; ++s) lam[s] = 0.0f;
        for (int seg = (p.H - 1) / p.C; seg >= 0 && p.H > 0; --seg) {
            const int t0 = seg * p.C, t1 = min(p.H, t0 + p.C);
            // recompute the segment's states s_t0 .. s_t1 into the workspace
#pragma unroll
            for (int s = 0; s < SS; ++s) {
                int f = 2 * s + g;
                st[s] = (valid && f < D_S) ? p.ckpt[((size_t)b * p.NC + seg) * D_S + f] : 0.0f;
            }
            for (int t = t0; t <= t1; ++t) {
                if (valid)
#pragma unroll
                    for (int s = 0; s < SS; ++s)
                        if (2 * s + g < D_S) p.segst[((size_t)b * (p.C + 1) + (t - t0)) * D_S + 2 * s + g] = st[s];
                if (t == t1) break;
                float slots[NT::IN_SLOTS];
                make_slots(slots, st, b, valid, t);
                DirectSrc<DT_F32, 8 * HT> src(P.f0);
                f32x16 d = run_net<NT>(src, P, P.b0, slots, lane, g);
#pragma unroll
                for (int s = 0; s < SS; ++s) st[s] += d[s];
            }
            for (int t = t1 - 1; t >= t0; --t) {
                float s_t[SS], s_n[SS];
#pragma unroll
                for (int s = 0; s < SS; ++s) {
                    int f = 2 * s + g;
                    s_t[s] = (valid && f < D_S) ? p.segst[((size_t)b * (p.C + 1) + (t - t0)) * D_S + f] : 0.0f;
                    s_n[s] = (valid && f < D_S) ? p.segst[((size_t)b * (p.C + 1) + (t - t0 + 1)) * D_S + f] : 0.0f;
                }
                // objective gradient at s_{t+1}
#pragma unroll
                for (int s = 0; s < SS; ++s) {
                    int f = 2 * s + g;
                    if (f < D_S && valid) {
                        float e = p.objective == 0 ? s_n[s] - p.targets[((size_t)b * p.H + t) * D_S + f] : s_n[s] - p.goal[f];
                        lam[s] += (p.objective == 0 ? 2.0f * (float)p.scale : -2.0f * p.disc[t] * (float)p.scale) * e;
                    }
                }
                // recompute the activations of step t
                float slots[NT::IN_SLOTS];
                make_slots(slots, s_t, b, valid, t);
                f32x16 acc[HT];
                Act<DT_F32, HT> h1, h2;
                {
                    DirectSrc<DT_F32, 8 * HT> src(P.f0);
                    init_bias<HT>(acc, P.b0 + opaque_zero(), g);
#pragma unroll
                    for (int c = 0; c < NT::IN_KS; ++c)
#pragma unroll
                        for (int mt = 0; mt < HT; ++mt)
                            acc[mt] = mfma(src.load(FragIdx<NT>::first(c, mt), lane), slots[c], acc[mt]);
                    h1.set_relu(acc);
                    init_bias<HT>(acc, P.bh + opaque_zero(), g);
#pragma unroll
                    for (int c = 0; c < NT::HID_KS; ++c)
#pragma unroll
                        for (int mt = 0; mt < HT; ++mt)
                            acc[mt] = mfma(src.load(FragIdx<NT>::hidden(1, c, mt), lane), h1.b(c), acc[mt]);
                    h2.set_relu(acc);
                }
                const bool wp = p.want_params != 0;
                float lamv[16];
#pragma unroll
                for (int i = 0; i < 16; ++i) lamv[i] = (i < SS && valid) ? lam[i] : 0.0f;
                // (1) dW3 += lam h2^T: rows lam (output features 0..31), h2 at 32..95
                if (wp) {
                    __builtin_amdgcn_wave_barrier();
#pragma unroll
                    for (int i = 0; i < 16; ++i) scr[col * kRow + 2 * i + g] = lamv[i];
#pragma unroll
                    for (int mt = 0; mt < HT; ++mt)
#pragma unroll
                        for (int i = 0; i < 16; ++i)
                            scr[col * kRow + 32 + 32 * mt + out_row(i, g)] = valid ? h2.v[mt][i] : 0.0f;
                    __builtin_amdgcn_wave_barrier();
#pragma unroll
                    for (int c = 0; c < 16; ++c) {
                        const float* r = scr + (2 * c + g) * kRow;
                        float ax = r[col];
#pragma unroll
                        for (int nt = 0; nt < HT; ++nt) gW3[nt] = mfma(ax, r[32 + 32 * nt + col], gW3[nt]);
                    }
#pragma unroll
                    for (int s = 0; s < SS; ++s) gb3[s] += lamv[s];
                }
                // (2) dh2 = (W3^T lam) * [h2 > 0]
                f32x16 dh2[HT];
#pragma unroll
                for (int mt = 0; mt < HT; ++mt) {
                    const char* bwz = bw + opaque_zero();
                    dh2[mt] = f32x16{};
#pragma unroll
                    for (int c = 0; c < BI::KS3; ++c) dh2[mt] = mfma(lds_frag(bwz, BI::t3(c, mt), lane), lam[c], dh2[mt]);
#pragma unroll
                    for (int i = 0; i < 16; ++i) dh2[mt][i] = (valid && h2.v[mt][i] > 0.0f) ? dh2[mt][i] : 0.0f;
                }
                // (3) dW2 += dh2 h1^T: rows dh2 (0..63), h1 at 64..127; b2 += dh2
                if (wp) {
                    __builtin_amdgcn_wave_barrier();
#pragma unroll
                    for (int mt = 0; mt < HT; ++mt)
#pragma unroll
                        for (int i = 0; i < 16; ++i) {
                            scr[col * kRow + 32 * mt + out_row(i, g)] = dh2[mt][i];
                            scr[col * kRow + 64 + 32 * mt + out_row(i, g)] = valid ? h1.v[mt][i] : 0.0f;
                        }
                    __builtin_amdgcn_wave_barrier();
#pragma unroll
                    for (int c = 0; c < 16; ++c) {
                        const float* r = scr + (2 * c + g) * kRow;
#pragma unroll
                        for (int nt = 0; nt < HT; ++nt) {
                            float bx = r[64 + 32 * nt + col];
#pragma unroll
                            for (int mt = 0; mt < HT; ++mt) gW2[mt][nt] = mfma(r[32 * mt + col], bx, gW2[mt][nt]);
                        }
                    }
#pragma unroll
                    for (int mt = 0; mt < HT; ++mt) gb2[mt] += dh2[mt];
                }
                // (4) dh1 = (W2^T dh2) * [h1 > 0]
                f32x16 dh1[HT];
#pragma unroll
                for (int mt = 0; mt < HT; ++mt) dh1[mt] = f32x16{};
#pragma unroll
                for (int c0 = 0; c0 < 16 * HT; c0 += 8) {
                    const char* bwz = bw + opaque_zero();
#pragma unroll
                    for (int c = c0; c < c0 + 8; ++c)
#pragma unroll
                        for (int mt = 0; mt < HT; ++mt)
                            dh1[mt] = mfma(lds_frag(bwz, BI::t2(c, mt), lane), dh2[c >> 4][c & 15], dh1[mt]);
                }
#pragma unroll
                for (int mt = 0; mt < HT; ++mt)
#pragma unroll
                    for (int i = 0; i < 16; ++i) dh1[mt][i] = h1.v[mt][i] > 0.0f ? dh1[mt][i] : 0.0f;
                // (5) dW1 (+ b1 through the ones column 31) += dh1 x^T: rows dh1 (0..63), x at 64..95
                if (wp) {
                    __builtin_amdgcn_wave_barrier();
#pragma unroll
                    for (int mt = 0; mt < HT; ++mt)
#pragma unroll
                        for (int i = 0; i < 16; ++i) scr[col * kRow + 32 * mt + out_row(i, g)] = dh1[mt][i];
#pragma unroll
                    for (int j = 0; j < 16; ++j) scr[col * kRow + 64 + 16 * g + j] = (16 * g + j == 31) ? 1.0f : 0.0f;
#pragma unroll
                    for (int s = 0; s < NT::IN_SLOTS; ++s) {
                        int cc = slot_col(s);
                        if (cc >= 0) scr[col * kRow + 64 + cc] = slots[s];
                    }
                    __builtin_amdgcn_wave_barrier();
#pragma unroll
                    for (int c = 0; c < 16; ++c) {
                        const float* r = scr + (2 * c + g) * kRow;
                        float bx = r[64 + col];
#pragma unroll
                        for (int mt = 0; mt < HT; ++mt) gW1[mt] = mfma(r[32 * mt + col], bx, gW1[mt]);
                    }
                    __builtin_amdgcn_wave_barrier();
                }
                // (6) dx = W1^T dh1: input feature 2 i + g in register i
                f32x16 dx = f32x16{};
#pragma unroll
                for (int c0 = 0; c0 < 16 * HT; c0 += 8) {
                    const char* bwz = bw + opaque_zero();
#pragma unroll
                    for (int c = c0; c < c0 + 8; ++c) dx = mfma(lds_frag(bwz, BI::t1(c), lane), dh1[c >> 4][c & 15], dx);
                }
                // action gradient of this step (continuous actions), summed over the tile
                if (N_ACT == 0 && p.apart) {
#pragma unroll
                    for (int j = 0; j < D_AIN; ++j) {
                        const int fin = D_S + j;
                        float v = (valid && (fin & 1) == g) ? dx[fin >> 1] : 0.0f;
                        v = sum32(v);
                        v += __shfl_xor(v, 32);
                        if (lane == 0 && tile_ok) p.apart[((size_t)tile * p.H + t) * D_AIN + j] = v;
                    }
                }
                // state adjoint: lam_t = lam_{t+1} + d(f_T)/ds_t^T lam_{t+1}
#pragma unroll
                for (int s = 0; s < SS; ++s)
                    if (2 * s + g < D_S) lam[s] += dx[s];
            }
        }
    }
    // ---- per-wave partials
    const int wid = blockIdx.x * wpb + wave;
    float lsum = sum32(loss_acc) + __shfl_xor(sum32(loss_acc), 32);
    if (lane == 0) p.lpart[wid] = lsum;
    if (!p.want_params) return;
    float* out = p.wpart + (size_t)wid * p.n_params;
    // layout: W1 [64][D_IN], b1 [64], W2 [64][64], b2 [64], W3 [D_S][64], b3 [D_S]
    const int oW1 = 0, ob1 = 64 * D_IN, oW2 = ob1 + 64, ob2 = oW2 + 64 * 64, oW3 = ob2 + 64, ob3 = oW3 + D_S * 64;
#pragma unroll
    for (int mt = 0; mt < HT; ++mt)
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const int m = 32 * mt + out_row(i, g);
            if (col < D_IN) out[oW1 + m * D_IN + col] = gW1[mt][i];
            if (col == 31) out[ob1 + m] = gW1[mt][i];
#pragma unroll
            for (int nt = 0; nt < HT; ++nt) out[oW2 + m * 64 + 32 * nt + col] = gW2[mt][nt][i];
        }
#pragma unroll
    for (int nt = 0; nt < HT; ++nt)
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const int m = out_row(i, g);
            if (m < D_S) out[oW3 + m * 64 + 32 * nt + col] = gW3[nt][i];
        }
#pragma unroll
    for (int mt = 0; mt < HT; ++mt)
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            float v = sum32(gb2[mt][i]);
            if (col == 0) out[ob2 + 32 * mt + out_row(i, g)] = v;
        }
#pragma unroll
    for (int s = 0; s < SS; ++s) {
        float v = sum32(gb3[s]);
        if (col == 0 && 2 * s + g < D_S) out[ob3 + 2 * s + g] = v;
    }
}

// Fixed-order sums of the per-wave partials: parameters, objective, actions.
__global__ __launch_bounds__(256) void grad_reduce_kernel(GradReduceParams p) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (p.grad_params && q < p.n_params) {
        float s = 0.0f;
        for (int w = 0; w < p.n_waves; ++w) s += p.wpart[(size_t)w * p.n_params + q];
        p.grad_params[q] = s;
    }
    if (p.grad_actions && q < p.n_action_values) {
        // q = (sequence k, step t, component j); tiles of sequence k are consecutive
        const int per_step = p.H * p.d_a;
        const int k = q / per_step, rem = q % per_step;
        float s = 0.0f;
        for (int tl = 0; tl < p.tiles_per_seq; ++tl)
            s += p.apart[(size_t)(k * p.tiles_per_seq + tl) * per_step + rem];
        p.grad_actions[q] = s;
    }
    if (p.loss && q == 0) {
        double s = 0.0;
        for (int w = 0; w < p.n_waves; ++w) s += (double)p.lpart[w];
        p.loss[0] = (float)(s * p.scale);
    }
}

// Parameter derivative of the contrastive objective (Eq. 6): for every pair
// (i, j) the likelihood network is re-run on [s'_i, a_i, o_j] (row i's state
// and action folded into its first-layer bias row, the observation in the
// input slots) and its parameters' derivative is accumulated with weight
// G_ij = d loss / d l_ij.  One wave owns a (row i, 32 observations) tile; the
// output layer is a dot product, so its adjoint is w3 * G_ij on the active
// units; the hidden adjoints use the transposed pack; the weight gradients
// are products over the tile's 32 pairs through the wave's LDS scratch, the
// first layer's over the full input [s'_i, a_i, o_j, 1] (column 31 carries
// the bias).  Each wave writes its partial once; grad_reduce_kernel sums them
// in a fixed order.
template <int D_S, int N_ACT, int D_A, int D_O>
__global__ __launch_bounds__(256) void nce_grad_kernel(NceGradParams p) {
    constexpr int WIDTH = 64, NHID = 2, HT = 2;
    constexpr int D_AIN = N_ACT > 0 ? N_ACT : D_A;
    constexpr int D_IN = D_S + D_AIN + D_O;
    static_assert(D_IN <= 31, "inputs must fit one 32-row tile (column 31 carries the bias)");
    typedef Net<DT_F32, WIDTH, NHID, in_slots(DT_F32, D_O, 0, 0)> NT;
    typedef BwdIdx<1, HT> BI;
    constexpr int SO = state_slots(D_O);
    extern __shared__ __attribute__((aligned(16))) char smem[];
    stage_blob(smem, p.fwd.base, p.fwd.bytes);
    stage_blob(smem + p.fwd.bytes, p.bwd.base, p.bwd.bytes);
    __syncthreads();
    const NetPtrs P = net_ptrs(smem, p.fwd);
    const char* bw = smem + p.fwd.bytes;
    const int lane = threadIdx.x & 63, g = lane >> 5, col = lane & 31;
    const int wpb = blockDim.x >> 6, wave = threadIdx.x >> 6;
    float* scr = reinterpret_cast<float*>(smem + p.fwd.bytes + p.bwd.bytes) + wave * 32 * kRow;

    f32x16 gW1[HT], gW2[HT][HT], gb2[HT], gw3[HT];
#pragma unroll
    for (int a = 0; a < HT; ++a) {
        gW1[a] = f32x16{};
        gb2[a] = f32x16{};
        gw3[a] = f32x16{};
#pragma unroll
        for (int b = 0; b < HT; ++b) gW2[a][b] = f32x16{};
    }
    float gb3 = 0.0f;

    const int B = p.B, jtiles = (B + 31) / 32;
    const long n_units = (long)B * jtiles;
    for (long u = (long)blockIdx.x * wpb + wave; u < n_units; u += (long)gridDim.x * wpb) {
        const int i = (int)(u / jtiles);
        const int j = (int)(u - (long)i * jtiles) * 32 + col;
        const bool valid = j < B;
        float slots[NT::IN_SLOTS];
#pragma unroll
        for (int s = 0; s < NT::IN_SLOTS; ++s) slots[s] = 0.0f;
#pragma unroll
        for (int s = 0; s < SO; ++s) {
            const int f = 2 * s + g;
            slots[s] = (valid && f < D_O) ? p.obs[(size_t)j * D_O + f] : 0.0f;
        }
        // forward: the two hidden layers' activations of the tile
        f32x16 acc[HT];
        Act<DT_F32, HT> h1, h2;
        {
            DirectSrc<DT_F32, 8 * HT> src(P.f0);
            init_bias<HT>(acc, p.b0 + (size_t)i * WIDTH, g);
#pragma unroll
            for (int c = 0; c < NT::IN_KS; ++c)
#pragma unroll
                for (int mt = 0; mt < HT; ++mt)
                    acc[mt] = mfma(src.load(FragIdx<NT>::first(c, mt), lane), slots[c], acc[mt]);
            h1.set_relu(acc);
            init_bias<HT>(acc, P.bh + opaque_zero(), g);
#pragma unroll
            for (int c = 0; c < NT::HID_KS; ++c)
#pragma unroll
                for (int mt = 0; mt < HT; ++mt)
                    acc[mt] = mfma(src.load(FragIdx<NT>::hidden(1, c, mt), lane), h1.b(c), acc[mt]);
            h2.set_relu(acc);
        }
        const float gc = valid ? p.grad[(size_t)i * B + j] : 0.0f;
        // output layer: dw3 += G h2, db3 += G; adjoint of h2 = w3 G on active units
        f32x16 d2[HT];
#pragma unroll
        for (int mt = 0; mt < HT; ++mt)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const float hv = h2.v[mt][r];
                gw3[mt][r] = __builtin_fmaf(gc, hv, gw3[mt][r]);
                d2[mt][r] = hv > 0.0f ? p.w3[32 * mt + out_row(r, g)] * gc : 0.0f;
            }
        if (g == 0) gb3 += gc;
        // dW2 += d2 h1^T over the tile's pairs (rows d2 at 0..63, h1 at 64..127); b2 += d2
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int mt = 0; mt < HT; ++mt)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                scr[col * kRow + 32 * mt + out_row(r, g)] = d2[mt][r];
                scr[col * kRow + 64 + 32 * mt + out_row(r, g)] = valid ? h1.v[mt][r] : 0.0f;
            }
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int c = 0; c < 16; ++c) {
            const float* rw = scr + (2 * c + g) * kRow;
#pragma unroll
            for (int nt = 0; nt < HT; ++nt) {
                const float bx = rw[64 + 32 * nt + col];
#pragma unroll
                for (int mt = 0; mt < HT; ++mt) gW2[mt][nt] = mfma(rw[32 * mt + col], bx, gW2[mt][nt]);
            }
        }
#pragma unroll
        for (int mt = 0; mt < HT; ++mt) gb2[mt] += d2[mt];
        // adjoint of h1 = (W2^T d2) on active units
        f32x16 d1[HT];
#pragma unroll
        for (int mt = 0; mt < HT; ++mt) d1[mt] = f32x16{};
#pragma unroll
        for (int c0 = 0; c0 < 16 * HT; c0 += 8) {
            const char* bwz = bw + opaque_zero();
#pragma unroll
            for (int c = c0; c < c0 + 8; ++c)
#pragma unroll
                for (int mt = 0; mt < HT; ++mt)
                    d1[mt] = mfma(lds_frag(bwz, BI::t2(c, mt), lane), d2[c >> 4][c & 15], d1[mt]);
        }
#pragma unroll
        for (int mt = 0; mt < HT; ++mt)
#pragma unroll
            for (int r = 0; r < 16; ++r) d1[mt][r] = h1.v[mt][r] > 0.0f ? d1[mt][r] : 0.0f;
        // dW1 (+ b1 through column 31) += d1 x^T, x = [s'_i, a_i, o_j, 0, ..., 1]
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int mt = 0; mt < HT; ++mt)
#pragma unroll
            for (int r = 0; r < 16; ++r) scr[col * kRow + 32 * mt + out_row(r, g)] = d1[mt][r];
        int a_i = 0;
        if (N_ACT > 0) {
            a_i = reinterpret_cast<const int32_t*>(p.actions)[i];
            if (a_i < 0 || a_i >= N_ACT) a_i = 0;  // flagged by the fold, which uses action 0 as well
        }
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const int c = 16 * g + q;
            float v = 0.0f;
            if (c < D_S) {
                v = p.states[(size_t)i * D_S + c];
            } else if (c < D_S + D_AIN) {
                if (N_ACT > 0) v = (c - D_S == a_i) ? 1.0f : 0.0f;
                else v = reinterpret_cast<const float*>(p.actions)[(size_t)i * D_AIN + (c - D_S)];
            } else if (c < D_IN) {
                v = p.obs[(size_t)(valid ? j : 0) * D_O + (c - D_S - D_AIN)];
            } else if (c == 31) {
                v = 1.0f;
            }
            scr[col * kRow + 64 + c] = valid ? v : 0.0f;
        }
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int c = 0; c < 16; ++c) {
            const float* rw = scr + (2 * c + g) * kRow;
            const float bx = rw[64 + col];
#pragma unroll
            for (int mt = 0; mt < HT; ++mt) gW1[mt] = mfma(rw[32 * mt + col], bx, gW1[mt]);
        }
        __builtin_amdgcn_wave_barrier();
    }
    // per-wave partials: W1 [64][D_IN], b1 [64], W2 [64][64], b2 [64], W3 [1][64], b3 [1]
    const int wid = blockIdx.x * wpb + wave;
    float* out = p.wpart + (size_t)wid * p.n_params;
    constexpr int oW1 = 0, ob1 = 64 * D_IN, oW2 = ob1 + 64, ob2 = oW2 + 64 * 64, oW3 = ob2 + 64, ob3 = oW3 + 64;
#pragma unroll
    for (int mt = 0; mt < HT; ++mt)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int m = 32 * mt + out_row(r, g);
            if (col < D_IN) out[oW1 + m * D_IN + col] = gW1[mt][r];
            if (col == 31) out[ob1 + m] = gW1[mt][r];
#pragma unroll
            for (int nt = 0; nt < HT; ++nt) out[oW2 + m * 64 + 32 * nt + col] = gW2[mt][nt][r];
            const float vb = sum32(gb2[mt][r]);
            const float vw = sum32(gw3[mt][r]);
            if (col == 0) {
                out[ob2 + m] = vb;
                out[oW3 + m] = vw;
            }
        }
    const float v3 = sum32(gb3);
    if (lane == 0) out[ob3] = v3;
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
#define GRAD_SHAPES(X) X(0, 4, 5, 0, 4) X(2, 4, 0, 4, 4)

bool grad_supported(int shape) {
#define X(id, ds, na, da, dw) if (shape == id) return true;
    GRAD_SHAPES(X)
#undef X
    return false;
}

hipError_t launch_grad(int shape, const GradParams& p, int blocks, size_t lds, hipStream_t s) {
    switch (shape) {
#define X(id, ds, na, da, dw)                                                                                \
    case id:                                                                                                \
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(grad_kernel<ds, na, da, dw>),                 \
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);                     \
        hipLaunchKernelGGL((grad_kernel<ds, na, da, dw>), blocks, 256, lds, s, p);                           \
        break;
        GRAD_SHAPES(X)
#undef X
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

int grad_blocks_per_cu(int shape, size_t lds) {
    int n = 0;
    switch (shape) {
#define X(id, ds, na, da, dw)                                                                                  \
    case id:                                                                                                  \
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, grad_kernel<ds, na, da, dw>, 256, lds) != hipSuccess) \
            n = 1;                                                                                            \
        break;
        GRAD_SHAPES(X)
#undef X
    }
    return n < 1 ? 1 : n;
}

// (shape id, d_s, discrete actions, continuous action width, d_o)
#define NCE_GRAD_SHAPES(X) X(0, 4, 5, 0, 2) X(2, 4, 0, 4, 2)

bool nce_grad_supported(int shape) {
#define X(id, ds, na, da, dox) if (shape == id) return true;
    NCE_GRAD_SHAPES(X)
#undef X
    return false;
}

hipError_t launch_nce_grad(int shape, const NceGradParams& p, int blocks, size_t lds, hipStream_t s) {
    switch (shape) {
#define X(id, ds, na, da, dox)                                                                                \
    case id:                                                                                                 \
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(nce_grad_kernel<ds, na, da, dox>),            \
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);                      \
        hipLaunchKernelGGL((nce_grad_kernel<ds, na, da, dox>), blocks, 256, lds, s, p);                       \
        break;
        NCE_GRAD_SHAPES(X)
#undef X
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

int nce_grad_blocks_per_cu(int shape, size_t lds) {
    int n = 0;
    switch (shape) {
#define X(id, ds, na, da, dox)                                                                                 \
    case id:                                                                                                  \
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, nce_grad_kernel<ds, na, da, dox>, 256, lds) != hipSuccess) \
            n = 1;                                                                                            \
        break;
        NCE_GRAD_SHAPES(X)
#undef X
    }
    return n < 1 ? 1 : n;
}

hipError_t launch_grad_reduce(const GradReduceParams& p, hipStream_t s) {
    int n = p.n_params > p.n_action_values ? p.n_params : p.n_action_values;
    if (n < 1) n = 1;
    hipLaunchKernelGGL(grad_reduce_kernel, (n + 255) / 256, 256, 0, s, p);
    return hipGetLastError();
}

}  // namespace voila
