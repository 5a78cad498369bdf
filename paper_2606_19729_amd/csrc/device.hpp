// device.hpp -- wave-level MLP engine on gfx950 matrix cores, counter-based
// noise, and the register layouts shared by the kernels and the host packer.
//
// Register layout (one wave = 64 lanes, lane l, group g = l / 32, column
// n = l % 32):
//   * A 32x32 MFMA output tile D (v_mfma_f32_32x32x2_f32 and
//     v_mfma_f32_32x32x16_bf16 share it) leaves D[row][n] in register i of
//     lane (g, n) with row = out_row(i, g) = 8 (i / 4) + 4 g + i % 4.
//   * The networks are evaluated transposed, h^T = W x^T: the 32 columns of
//     a tile are 32 rollouts (particles), rows are features.  The B operand
//     of the next layer needs, per lane, features of the lane's own column,
//     which is exactly what the D layout holds -- so a layer's output feeds
//     the next layer straight from registers.  k-step c of a hidden layer
//     consumes "register index" ri = c * KPER + j (j < KPER; KPER = 1 for
//     f32, 8 for bf16), i.e. tile ri / 16, register ri % 16, whose feature in
//     group g is 32 (ri / 16) + out_row(ri % 16, g).  The host packs the
//     weight fragments of every layer in that order, so the feature
//     permutation costs nothing at run time.
//   * The first layer's input is assembled per lane in "slots": group g
//     holds state features f = 2 s + g, then continuous-action features
//     2 s + g, then noise features 4 (s / 2) + 2 g + s % 2 (pair g of Philox
//     block s / 2), then zero padding to a multiple of KPER.
//   * The output layer has one 32-row tile; output feature f = 2 i + g sits in
//     register i of group g (row out_row(i, g)), which makes the state update
//     s += f_T(...) a register-to-register add.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>
#include <utility>
#include <stdint.h>

namespace voila {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int DT_F32 = 0;
constexpr int DT_BF16 = 1;

// Pipeline depth (k-steps of weight fragments in registers, including the
// one being multiplied) of the bfloat16 evaluation, chunks per group of the
// grouped wide networks' stream, and the chunk bytes of other streamed
// networks.
#ifndef VOILA_PF_DEPTH
#define VOILA_PF_DEPTH 3
#endif
#ifndef VOILA_WIDE_CPG
#define VOILA_WIDE_CPG 11
#endif
#ifndef VOILA_WIDE_NBUF
#define VOILA_WIDE_NBUF 3
#endif
#ifndef VOILA_STREAM_CHB
#define VOILA_STREAM_CHB 32768
#endif
#ifndef VOILA_STREAM_NBUF
#define VOILA_STREAM_NBUF 2
#endif
// Chunk bytes of the rollout kernel's stream (its single workgroup per CU
// has the LDS for two 64 KB buffers: half the barriers of 32 KB chunks);
// packed networks are padded to whole chunks of the larger size.
#ifndef VOILA_PLAN_STREAM_CHB
#define VOILA_PLAN_STREAM_CHB 65536
#endif
constexpr int kStreamPadBytes = VOILA_PLAN_STREAM_CHB > VOILA_STREAM_CHB ? VOILA_PLAN_STREAM_CHB : VOILA_STREAM_CHB;
constexpr int kPfDepth = VOILA_PF_DEPTH;
#ifndef VOILA_PF_DEPTH_F32
#define VOILA_PF_DEPTH_F32 6
#endif
constexpr int kPfDepthF32 = VOILA_PF_DEPTH_F32;  // binary32 fragments are one register each

__host__ __device__ constexpr int cdiv(int a, int b) { return (a + b - 1) / b; }
__host__ __device__ constexpr int rup(int a, int b) { return cdiv(a, b) * b; }
// Calls f(std::integral_constant<int, i>) for i = 0 .. N-1 (compile-time indices).
template <class F, int... I>
__device__ __forceinline__ void static_for_impl(F&& f, std::integer_sequence<int, I...>) {
    (f(std::integral_constant<int, I>{}), ...);
}
template <int N, class F>
__device__ __forceinline__ void static_for(F&& f) {
    static_for_impl(f, std::make_integer_sequence<int, N>{});
}

__host__ __device__ constexpr int out_row(int i, int g) { return (i >> 2) * 8 + g * 4 + (i & 3); }
__host__ __device__ constexpr int kper(int dt) { return dt == DT_F32 ? 1 : 8; }

// Slots of the first-layer input held by each lane group.
__host__ __device__ constexpr int state_slots(int d_s) { return cdiv(d_s, 2); }
__host__ __device__ constexpr int action_slots(int d_ain) { return cdiv(d_ain, 2); }
__host__ __device__ constexpr int noise_slots(int d_w) { return 2 * cdiv(d_w, 4); }
__host__ __device__ constexpr int in_slots(int dt, int d_s, int d_ain, int d_w) {
    return rup(state_slots(d_s) + action_slots(d_ain) + noise_slots(d_w), kper(dt));
}

// Position of every weight fragment in the packed stream of a network
// (fragment (k-step c, 32-row tile t)), in the order the kernels consume them:
// first layer [c][t], each hidden->hidden layer [c][t], output layer [c].
// Wider networks (two hidden layers) hold only the first hidden layer's
// activations in registers and produce the second in groups of `ct` tiles:
// their hidden->hidden and output fragments are stored group by group, each
// group holding its hidden fragments [c][t % ct] followed by the output-layer
// k-steps that consume the group's tiles.
struct FragLayout {
    int ht, in_ks, hid_ks, ct, nhid;
    __host__ __device__ constexpr bool grouped() const { return ct < ht; }
    __host__ __device__ constexpr int nf0() const { return in_ks * ht; }
    __host__ __device__ constexpr int oks() const { return hid_ks / ht; }  // output k-steps per hidden tile
    __host__ __device__ constexpr int group() const { return hid_ks * ct + oks() * ct; }
    __host__ __device__ constexpr int first(int c, int t) const { return c * ht + t; }
    __host__ __device__ constexpr int hidden(int l, int c, int t) const {
        return grouped() ? nf0() + (t / ct) * group() + c * ct + t % ct
                         : nf0() + (l - 1) * hid_ks * ht + c * ht + t;
    }
    __host__ __device__ constexpr int out(int c) const {
        return grouped() ? nf0() + (c / (oks() * ct)) * group() + hid_ks * ct + c % (oks() * ct)
                         : nf0() + (nhid - 1) * hid_ks * ht + c;
    }
};

// Output tiles produced per group by the grouped evaluation of wide networks.
__host__ __device__ constexpr int chunk_tiles(int width) { return width > 256 ? 4 : width / 32; }
// Tiles per group of a network's default packing: the grouped evaluation
// needs exactly two hidden layers, so deeper networks are packed layer by
// layer (one group of every tile).
__host__ __device__ constexpr int default_ct(int width, int nhid) { return nhid == 2 ? chunk_tiles(width) : width / 32; }

// Compile-time shape of one network as the engine runs it.  CT_ = WIDTH_/32
// packs a wide network layer by layer (for the split evaluation) instead of
// in the groups of the grouped evaluation.  NO_ 32-row output tiles (outputs
// wider than 32 need a layered network; only the split evaluation produces
// more than one): the output fragments of tile t are k-steps
// t HID_KS .. t HID_KS + HID_KS - 1 of the output layer.
template <int DT_, int WIDTH_, int NHID_, int IN_SLOTS_, int CT_ = default_ct(WIDTH_, NHID_), int NO_ = 1>
struct Net {
    static constexpr int DT = DT_;
    static constexpr int WIDTH = WIDTH_;           // hidden width (multiple of 32)
    static constexpr int HT = WIDTH / 32;          // hidden 32-row tiles
    static constexpr int NHID = NHID_;             // hidden layers (>= 1)
    static constexpr int KPER = kper(DT);          // k values per lane per MFMA
    static constexpr int IN_SLOTS = IN_SLOTS_;     // first-layer slots per lane group
    static constexpr int IN_KS = IN_SLOTS / KPER;  // first-layer k-steps
    static constexpr int HID_KS = 16 * HT / KPER;  // k-steps of a layer fed by a hidden layer
    static constexpr int FRAG_BYTES = 64 * KPER * (DT == DT_F32 ? 4 : 2);
    static constexpr int NF0 = IN_KS * HT;         // first-layer fragments
    static constexpr int NFH = HID_KS * HT;        // fragments per hidden->hidden layer
    static constexpr int NO = NO_;                 // output tiles
    static constexpr int NFO = NO_ * HID_KS;       // output-layer fragments
    static constexpr int CT = CT_;                 // tiles per group of the grouped evaluation
    static constexpr int OKS = HID_KS / HT;        // output k-steps per hidden tile
    static_assert(WIDTH % 32 == 0 && NHID >= 1 && IN_SLOTS % KPER == 0, "bad net shape");
    static_assert(CT == HT || (NHID == 2 && HT % CT == 0), "grouped evaluation needs two hidden layers");
    static_assert(NO >= 1 && (NO == 1 || CT == HT), "several output tiles need a layered network");
};

// Device view of one packed network (all pointers into global memory or LDS).
struct NetPtrs {
    const char* f0;     // first-layer fragments  [IN_KS][HT]
    const char* fh;     // hidden fragments       [NHID-1][HID_KS][HT]
    const char* fo;     // output fragments       [HID_KS]
    const float* b0;    // first-layer bias       [WIDTH] (row order)
    const float* bh;    // hidden biases          [NHID-1][WIDTH]
    const float* bo;    // output bias            [32] (row order)
};

// Offsets of the parts of a packed network blob (bytes from the blob start).
struct NetBlob {
    const char* base;
    uint32_t bytes;
    uint32_t off_f0, off_fh, off_fo, off_b0, off_bh, off_bo;
    uint32_t b0_stride;  // floats between first-layer bias variants (discrete actions)
};

__device__ inline NetPtrs net_ptrs(const char* base, const NetBlob& nb) {
    NetPtrs p;
    p.f0 = base + nb.off_f0;
    p.fh = base + nb.off_fh;
    p.fo = base + nb.off_fo;
    p.b0 = reinterpret_cast<const float*>(base + nb.off_b0);
    p.bh = reinterpret_cast<const float*>(base + nb.off_bh);
    p.bo = reinterpret_cast<const float*>(base + nb.off_bo);
    return p;
}

// ----------------------------------------------------------------------------
// Matrix-core primitives.
// ----------------------------------------------------------------------------
__device__ __forceinline__ f32x16 mfma(float a, float b, f32x16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f32x16 mfma(bf16x8 a, bf16x8 b, f32x16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}

template <int DT> struct Frag;
template <> struct Frag<DT_F32> {
    typedef float type;
    __device__ static __forceinline__ float load(const char* p, int idx, int lane) {
        return reinterpret_cast<const float*>(p)[idx * 64 + lane];
    }
};
template <> struct Frag<DT_BF16> {
    typedef bf16x8 type;
    __device__ static __forceinline__ bf16x8 load(const char* p, int idx, int lane) {
        return reinterpret_cast<const bf16x8*>(p)[idx * 64 + lane];
    }
};

// acc[t][i] = bias[32 t + out_row(i, g)]
template <int NT>
__device__ __forceinline__ void init_bias(f32x16 (&acc)[NT], const float* bias, int g) {
#pragma unroll
    for (int t = 0; t < NT; ++t) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            f32x4 v = *reinterpret_cast<const f32x4*>(bias + 32 * t + 8 * q + 4 * g);
            acc[t][4 * q + 0] = v[0];
            acc[t][4 * q + 1] = v[1];
            acc[t][4 * q + 2] = v[2];
            acc[t][4 * q + 3] = v[3];
        }
    }
}

// Hidden activations as the B operands of the next layer.
template <int DT, int HT> struct Act;
// ReLU of a binary32 value as the integer maximum of its bits with 0: values
// with the sign bit set (negatives, -0) become +0, all others are unchanged.
// One instruction, where fmaxf costs two (it first quiets signalling NaNs).
__device__ __forceinline__ float relu_f32(float x) { return __int_as_float(max(__float_as_int(x), 0)); }

typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef short i16x2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
// Two values rounded to bfloat16 (nearest even) in one packed conversion,
// then ReLU on the 16-bit patterns by a packed integer maximum with 0:
// rounding never changes the sign, so this equals rounding the ReLU.
__device__ __forceinline__ uint32_t relu_bf16x2(float a, float b) {
    const bf16x2 p = __builtin_convertvector((f32x2){a, b}, bf16x2);
    const i16x2 q = __builtin_elementwise_max(__builtin_bit_cast(i16x2, p), (i16x2)(short)0);
    return __builtin_bit_cast(uint32_t, q);
}
// Values 8 h .. 8 h + 7 of an accumulator tile as a ReLU'd bfloat16 operand.
__device__ __forceinline__ bf16x8 relu_bf16x8(const f32x16& a, int h) {
    const u32x4 w = {relu_bf16x2(a[8 * h], a[8 * h + 1]), relu_bf16x2(a[8 * h + 2], a[8 * h + 3]),
                     relu_bf16x2(a[8 * h + 4], a[8 * h + 5]), relu_bf16x2(a[8 * h + 6], a[8 * h + 7])};
    return __builtin_bit_cast(bf16x8, w);
}

template <int HT> struct Act<DT_F32, HT> {
    f32x16 v[HT];
    __device__ __forceinline__ void set_relu(const f32x16 (&acc)[HT]) {
#pragma unroll
        for (int t = 0; t < HT; ++t)
#pragma unroll
            for (int i = 0; i < 16; ++i) v[t][i] = relu_f32(acc[t][i]);
    }
    template <int CT>
    __device__ __forceinline__ void set_relu_at(const f32x16 (&acc)[CT], int t0) {
#pragma unroll
        for (int t = 0; t < CT; ++t)
#pragma unroll
            for (int i = 0; i < 16; ++i) v[t0 + t][i] = relu_f32(acc[t][i]);
    }
    __device__ __forceinline__ void set_relu_tile(const f32x16 (&acc)[HT], int t) {
#pragma unroll
        for (int i = 0; i < 16; ++i) v[t][i] = relu_f32(acc[t][i]);
    }
    __device__ __forceinline__ float b(int c) const { return v[c >> 4][c & 15]; }
};
template <int HT> struct Act<DT_BF16, HT> {
    bf16x8 v[2 * HT];
    __device__ __forceinline__ void set_relu(const f32x16 (&acc)[HT]) {
#pragma unroll
        for (int t = 0; t < HT; ++t) {
            v[2 * t] = relu_bf16x8(acc[t], 0);
            v[2 * t + 1] = relu_bf16x8(acc[t], 1);
        }
    }
    template <int CT>
    __device__ __forceinline__ void set_relu_at(const f32x16 (&acc)[CT], int t0) {
#pragma unroll
        for (int t = 0; t < CT; ++t) {
            v[2 * (t0 + t)] = relu_bf16x8(acc[t], 0);
            v[2 * (t0 + t) + 1] = relu_bf16x8(acc[t], 1);
        }
    }
    __device__ __forceinline__ void set_relu_tile(const f32x16 (&acc)[HT], int t) {
        v[2 * t] = relu_bf16x8(acc[t], 0);
        v[2 * t + 1] = relu_bf16x8(acc[t], 1);
    }
    // values 2 j and 2 j + 1 of accumulator tile `a` as the ReLU'd pair j of tile t
    __device__ __forceinline__ void set_relu_pair(const f32x16& a, int t, int j) {
        u32x4 w = __builtin_bit_cast(u32x4, v[2 * t + j / 4]);
        w[j % 4] = relu_bf16x2(a[2 * j], a[2 * j + 1]);
        v[2 * t + j / 4] = __builtin_bit_cast(bf16x8, w);
    }
    __device__ __forceinline__ bf16x8 b(int c) const { return v[c]; }
};

// First-layer B operand from per-lane slot values.
template <int DT, int S> struct Slots;
template <int S> struct Slots<DT_F32, S> {
    __device__ static __forceinline__ float b(const float (&s)[S], int c) { return s[c]; }
};
template <int S> struct Slots<DT_BF16, S> {
    __device__ static __forceinline__ bf16x8 b(const float (&s)[S], int c) {
        bf16x8 r;
#pragma unroll
        for (int j = 0; j < 8; ++j) r[j] = (__bf16)s[8 * c + j];
        return r;
    }
};

// A zero the compiler cannot see through.  Adding it to a fragment address
// keeps the (loop-invariant) weight loads inside the window of fragments that
// uses them instead of letting them be hoisted out of the rollout loop, which
// would need one register per weight.
__device__ __forceinline__ int opaque_zero() {
    int z = 0;
    asm volatile("" : "+s"(z));
    return z;
}

// A wave-uniform 32-bit value the compiler cannot see through.
__device__ __forceinline__ uint32_t opaque_u32(uint32_t v) {
    asm volatile("" : "+s"(v));
    return v;
}

// Fragment source reading a resident copy of the packed network (global
// memory or LDS) directly; the address is refreshed every WIN fragments.
template <int DT, int WIN>
struct DirectSrc {
    const char* base;
    const char* cur;
    __device__ __forceinline__ explicit DirectSrc(const char* b) : base(b), cur(b) {}
    __device__ __forceinline__ typename Frag<DT>::type load(int f, int lane) {
        if (f % WIN == 0) cur = base + opaque_zero();
        return Frag<DT>::load(cur, f, lane);
    }
    __device__ __forceinline__ void finish() {}
};

// s_waitcnt immediate: wait until at most `vm` vector-memory operations of
// this wave are outstanding and all of its LDS operations are done.
__host__ __device__ constexpr int waitcnt_vm_lgkm0(int vm) { return (vm & 15) | ((vm >> 4) << 14) | (7 << 4); }

// Fragment source streaming the packed network from global memory through
// NBUF LDS chunk buffers shared by the workgroup's four waves; the network's
// evaluation is unrolled at compile time and the packed stream is padded to
// whole chunks.  Every wave walks the same fragment sequence (the rollout
// loop is block-uniform).
template <class N, int CHB = VOILA_STREAM_CHB, int NBUF = VOILA_STREAM_NBUF, int WIN = 4 * N::HT>
struct StreamSrc {
    static constexpr int FB = N::FRAG_BYTES;
    static constexpr int FPC = CHB / FB;  // fragments per chunk
    static constexpr int NFR = N::NF0 + (N::NHID - 1) * N::NFH + N::NFO;
    static constexpr int NCH = cdiv(NFR, FPC);  // the packed stream is padded to whole chunks
    static constexpr int kWaves = 4;            // waves of the workgroup
    static constexpr int ROUNDS = CHB / 1024 / kWaves;
    static constexpr int LDS_BYTES = NBUF * CHB;
    static_assert(CHB % (1024 * kWaves) == 0 && CHB % FB == 0, "chunk must be whole DMA rounds and fragments");
    static_assert(NBUF >= 2 && (NBUF - 2) * ROUNDS <= 63 && NCH >= NBUF, "bad chunk pipeline");
    char* lds;          // NBUF * CHB bytes of LDS
    const char* src;    // packed fragment stream in global memory
    const char* lsrc;   // this lane's 16-byte slot of this wave's first 1 KB round
    int cur, nxt_buf;   // buffer of the current chunk, buffer of the next load
    const char* win;    // current chunk's buffer, refreshed every WIN fragments

    __device__ __forceinline__ StreamSrc(char* l, const char* s)
        : lds(l), src(s),
          lsrc(s + (size_t)__builtin_amdgcn_readfirstlane(threadIdx.x >> 6) * 1024 + (threadIdx.x & 63) * 16),
          cur(NBUF - 1), nxt_buf(NBUF - 1), win(l) {}

    // Copies chunk ch into buffer b: each wave moves a quarter, 1 KB per
    // round (64 lanes x 16 B), with direct-to-LDS loads.
    __device__ __forceinline__ void fetch(int ch, int b) const {
        const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
        const int lane = threadIdx.x & 63;
        const char* base = src + opaque_zero() + (size_t)ch * CHB;
        auto round = [&](int r) {
            const int off = (r * kWaves + wave) * 1024;
            __builtin_amdgcn_global_load_lds((const void*)(base + off + lane * 16),
                                             (__attribute__((address_space(3))) void*)(lds + b * CHB + off), 16, 0,
                                             0);
        };
#pragma unroll
        for (int r = 0; r < ROUNDS; ++r) round(r);
    }
    __device__ __forceinline__ void start() {
#pragma unroll
        for (int j = 0; j < NBUF - 1; ++j) fetch(j, j);
    }
    // At the first fragment of a chunk: wait until only this wave's loads of
    // the NBUF - 2 newer chunks are outstanding and its LDS reads are done,
    // meet the workgroup (the chunk is then complete and the buffer read
    // before it free), and start loading the chunk NBUF - 1 ahead there.
    // The loads of the chunk NBUF - 1 ahead are spread over the fragments the
    // current chunk actually serves (the last chunk is padding past its end):
    // round r is issued at fragment floor(r * V / ROUNDS) of a chunk of V
    // served fragments (positions are compile-time constants).
    static constexpr int LASTF = NFR - (NCH - 1) * FPC;
    int nxt_ch = 0;
    __device__ __forceinline__ typename Frag<N::DT>::type load(int f, int lane) {
        const int ch = f / FPC, within = f % FPC;
        if (within == 0) {
            __builtin_amdgcn_s_waitcnt(waitcnt_vm_lgkm0((NBUF - 2) * ROUNDS));
            __builtin_amdgcn_s_barrier();
            cur = cur + 1 == NBUF ? 0 : cur + 1;
            int nxt = ch + NBUF - 1;
            nxt_ch = nxt < NCH ? nxt : nxt - NCH;
        }
        const int served = ch == NCH - 1 ? LASTF : FPC;
#pragma unroll
        for (int r = 0; r < ROUNDS; ++r) {
            if ((r * served) / ROUNDS != within) continue;
            const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
            const int off = (r * kWaves + wave) * 1024;
            __builtin_amdgcn_global_load_lds(
                (const void*)(lsrc + opaque_u32((uint32_t)(nxt_ch * CHB + r * kWaves * 1024))),
                (__attribute__((address_space(3))) void*)(lds + nxt_buf * CHB + off), 16, 0, 0);
            if (r == ROUNDS - 1) nxt_buf = nxt_buf + 1 == NBUF ? 0 : nxt_buf + 1;
        }
        if (within % WIN == 0) win = lds + cur * CHB + opaque_zero();
        return Frag<N::DT>::load(win, within, lane);
    }
    __device__ __forceinline__ void finish() { __builtin_amdgcn_s_waitcnt(0); }
};

// Instruction classes of the scheduling-group barriers: LDS or vector-memory
// reads, matrix-core instructions.
constexpr int kSchedReads = 0x100 | 0x020;
constexpr int kSchedMfma = 0x008;

// acc[t] += A(c, t) B(c) over k-steps c < KS and tiles t < NT, with the A
// fragments of the next D - 1 k-steps already loading while k-step c is
// multiplied (register ring indexed at compile time).  `ld(c, t)` issues the
// load of fragment (c, t) (in increasing c, so a streaming source meets its
// chunk boundaries in order); `bop(c)` gives the B operand of k-step c.
template <int KS, int NT, int D, class FT, class LD, class BOP>
__device__ __forceinline__ void mfma_layer(f32x16 (&acc)[NT], LD&& ld, BOP&& bop) {
    constexpr int DD = D < KS ? D : KS;
    FT ring[DD][NT];
    static_for<DD - 1>([&](auto pi) {
        constexpr int c = decltype(pi)::value;
        static_for<NT>([&](auto ti) { ring[c][decltype(ti)::value] = ld(c, decltype(ti)::value); });
    });
    static_for<KS>([&](auto ci) {
        constexpr int c = decltype(ci)::value;
        if constexpr (c + DD - 1 < KS) {
            static_for<NT>([&](auto ti) {
                ring[(c + DD - 1) % DD][decltype(ti)::value] = ld(c + DD - 1, decltype(ti)::value);
            });
        }
        auto b = bop(ci);
        static_for<NT>([&](auto ti) {
            constexpr int t = decltype(ti)::value;
            acc[t] = mfma(ring[c % DD][t], b, acc[t]);
        });
        // issue this k-step's prefetch loads before its products, and keep the
        // scheduler from hoisting later loads (one register set per k-step)
        if constexpr (c + DD - 1 < KS) __builtin_amdgcn_sched_group_barrier(kSchedReads, NT, 0);
        __builtin_amdgcn_sched_group_barrier(kSchedMfma, NT, 0);
        __builtin_amdgcn_sched_barrier(0);
    });
}

// Fragment index of (k-step c, tile t) in each layer of the packed stream.
// (The layout is rebuilt from the shape constants in each call: a static
// constexpr layout object would be read from memory at run time.)
template <class N> struct FragIdx {
    __device__ static constexpr FragLayout lay() { return FragLayout{N::HT, N::IN_KS, N::HID_KS, N::CT, N::NHID}; }
    __device__ static constexpr int first(int c, int t) { return lay().first(c, t); }
    __device__ static constexpr int hidden(int l, int c, int t) { return lay().hidden(l, c, t); }
    __device__ static constexpr int out(int c) { return lay().out(c); }
};

template <class N, class Src>
__device__ __forceinline__ f32x16 run_net_grouped(Src& src, const NetPtrs& P, const float* b0,
                                                  const float (&slots)[N::IN_SLOTS], int lane, int g);

// Runs one network on the 32 columns of a wave.  `slots` is the first-layer
// input of this lane, `b0` the first-layer bias (row order, possibly with an
// action folded in).  Returns the output tile: feature 2 i + g in out[i].
template <class N, class Src>
__device__ __forceinline__ f32x16 run_net(Src& src, const NetPtrs& P, const float* b0,
                                          const float (&slots)[N::IN_SLOTS], int lane, int g) {
    if constexpr (N::CT < N::HT) {
        return run_net_grouped<N>(src, P, b0, slots, lane, g);
    } else if constexpr (N::DT == DT_BF16 && N::WIDTH > 64) {
        // streamed bfloat16: every loop unrolled at compile time, weight fragments of
        // the next k-steps loaded while this one multiplies, and two
        // accumulator sets so that each layer's ReLU and conversion run tile by
        // tile inside the next layer, one tile ahead of the k-steps that read
        // it, overlapped with the matrix cores instead of between layers
        typedef FragIdx<N> FI;
        typedef typename Frag<N::DT>::type FT;
        constexpr int KPT = N::HID_KS / N::HT;  // k-steps that read one tile of the previous layer
        f32x16 acc[2][N::HT];
        Act<N::DT, N::HT> act;
        init_bias<N::HT>(acc[0], b0 + opaque_zero(), g);
        mfma_layer<N::IN_KS, N::HT, 2, FT>(
            acc[0], [&](int c, int t) { return src.load(FI::first(c, t), lane); },
            [&](int c) { return Slots<N::DT, N::IN_SLOTS>::b(slots, c); });
        act.set_relu_tile(acc[0], 0);
        auto lazy_b = [&](const f32x16 (&prev)[N::HT], auto ci) {
            constexpr int c = decltype(ci)::value;
            if constexpr (c % KPT == 0 && c / KPT + 1 < N::HT) act.set_relu_tile(prev, c / KPT + 1);
            return act.b(c);
        };
        static_for<N::NHID - 1>([&](auto li) {
            constexpr int l = decltype(li)::value + 1;
            init_bias<N::HT>(acc[l % 2], P.bh + (l - 1) * N::WIDTH + opaque_zero(), g);
            mfma_layer<N::HID_KS, N::HT, kPfDepth, FT>(
                acc[l % 2], [&](int c, int t) { return src.load(FI::hidden(l, c, t), lane); },
                [&](auto ci) { return lazy_b(acc[(l - 1) % 2], ci); });
            act.set_relu_tile(acc[l % 2], 0);
        });
        f32x16 out[1];
        init_bias<1>(out, P.bo + opaque_zero(), g);
        mfma_layer<N::HID_KS, 1, 4, FT>(
            out, [&](int c, int) { return src.load(FI::out(c), lane); },
            [&](auto ci) { return lazy_b(acc[(N::NHID - 1) % 2], ci); });
        return out[0];
    } else if constexpr (N::DT == DT_BF16 || N::WIDTH > 64) {
        // small bfloat16 and streamed binary32 networks: every loop unrolled at
        // compile time (fragment positions, and a streaming source's chunk
        // boundaries, are constants) and the weight fragments of the next
        // k-steps load while this one multiplies
        typedef FragIdx<N> FI;
        typedef typename Frag<N::DT>::type FT;
        f32x16 acc[N::HT];
        Act<N::DT, N::HT> act;
        init_bias<N::HT>(acc, b0 + opaque_zero(), g);
        mfma_layer<N::IN_KS, N::HT, 2, FT>(
            acc, [&](int c, int t) { return src.load(FI::first(c, t), lane); },
            [&](int c) { return Slots<N::DT, N::IN_SLOTS>::b(slots, c); });
        act.set_relu(acc);
        static_for<N::NHID - 1>([&](auto li) {
            constexpr int l = decltype(li)::value + 1;
            init_bias<N::HT>(acc, P.bh + (l - 1) * N::WIDTH + opaque_zero(), g);
            mfma_layer<N::HID_KS, N::HT, (N::DT == DT_F32 ? kPfDepthF32 : kPfDepth), FT>(
                acc, [&](int c, int t) { return src.load(FI::hidden(l, c, t), lane); },
                [&](int c) { return act.b(c); });
            act.set_relu(acc);
        });
        f32x16 out[1];
        init_bias<1>(out, P.bo + opaque_zero(), g);
        mfma_layer<N::HID_KS, 1, 4, FT>(
            out, [&](int c, int) { return src.load(FI::out(c), lane); }, [&](int c) { return act.b(c); });
        return out[0];
    } else {
    typedef FragIdx<N> FI;
    f32x16 acc[N::HT];
    Act<N::DT, N::HT> act;
    init_bias<N::HT>(acc, b0 + opaque_zero(), g);
#pragma unroll
    for (int c = 0; c < N::IN_KS; ++c) {
        auto b = Slots<N::DT, N::IN_SLOTS>::b(slots, c);
#pragma unroll
        for (int t = 0; t < N::HT; ++t) acc[t] = mfma(src.load(FI::first(c, t), lane), b, acc[t]);
    }
    act.set_relu(acc);
#pragma unroll
    for (int l = 1; l < N::NHID; ++l) {
        init_bias<N::HT>(acc, P.bh + (l - 1) * N::WIDTH + opaque_zero(), g);
#pragma unroll
        for (int c = 0; c < N::HID_KS; ++c) {
            auto b = act.b(c);
#pragma unroll
            for (int t = 0; t < N::HT; ++t) acc[t] = mfma(src.load(FI::hidden(l, c, t), lane), b, acc[t]);
        }
        act.set_relu(acc);
    }
    f32x16 out[1];
    init_bias<1>(out, P.bo + opaque_zero(), g);
#pragma unroll
    for (int c = 0; c < N::HID_KS; ++c) out[0] = mfma(src.load(FI::out(c), lane), act.b(c), out[0]);
    return out[0];
    }
}

// Wide two-hidden-layer networks.  The first hidden layer's activations (the
// B operands of the second layer) stay in registers; the second hidden layer
// is produced CT tiles at a time, and each finished group is multiplied into
// the output layer at once, so only CT accumulator tiles of it are live.
//
// Fragment sources of the grouped evaluation: `first` reads the first layer,
// `hid` the hidden->hidden fragments of one group at compile-time positions
// after begin_group(gi), `out` points at the output-layer fragments.
// A window of WINF fragments shares one opaque base address, which bounds how
// many weight loads the compiler can issue ahead (and keeps them in the loop).
template <class N, int WINF = 8>
struct GroupDirect {  // group fragments straight from global memory (L2)
    static constexpr int GF = N::HID_KS * N::CT + N::OKS * N::CT;  // fragments per group
    const char* base;
    const char* grp;
    const char* win;
    __device__ __forceinline__ explicit GroupDirect(const char* b) : base(b), grp(b), win(b) {}
    __device__ __forceinline__ void begin_group(int gi) { grp = base + (size_t)gi * GF * N::FRAG_BYTES; }
    template <int POS>
    __device__ __forceinline__ typename Frag<N::DT>::type load(int lane) {
        if constexpr (POS % WINF == 0) win = grp + POS * N::FRAG_BYTES + opaque_zero();
        return Frag<N::DT>::load(win, POS % WINF, lane);
    }
    __device__ __forceinline__ void start() {}
    __device__ __forceinline__ void finish() {}
};

// Group fragments streamed through NBUF LDS chunk buffers shared by the
// workgroup of four waves; a group is CPG whole chunks, so every chunk
// boundary sits at a compile-time position of the group.  Each wave moves a
// quarter of every chunk with direct-to-LDS loads, issued NBUF - 1 chunks
// ahead.  At the first fragment of a chunk a wave waits until only its loads
// of the NBUF - 2 newer chunks are outstanding (vector-memory loads complete
// in order) and its LDS reads are done, then the workgroup meets at a
// barrier, after which the chunk is complete and the buffer read before it
// is free: the loads of the chunk NBUF - 1 ahead go there.
template <class N, int CPG = VOILA_WIDE_CPG, int NBUF = VOILA_WIDE_NBUF, int WINF = 8>
struct GroupStream {
    static constexpr int FB = N::FRAG_BYTES;
    static constexpr int GF = N::HID_KS * N::CT + N::OKS * N::CT;
    static constexpr int FPC = GF / CPG;                // fragments per chunk
    static constexpr int CHB = FPC * FB;                // chunk bytes
    static constexpr int NCH = (N::HT / N::CT) * CPG;   // chunks per network evaluation
    static constexpr int kWaves = 4;                    // waves of the workgroup
    static constexpr int ROUNDS = CHB / 1024 / kWaves;  // 1 KB loads per wave per chunk
    static constexpr int LDS_BYTES = NBUF * CHB;
    static_assert(GF % CPG == 0 && CHB % (1024 * kWaves) == 0, "a chunk must be whole 1 KB rounds of every wave");
    static_assert(NBUF >= 2 && (NBUF - 2) * ROUNDS <= 63 && NCH >= NBUF, "bad chunk pipeline");
    char* lds;
    const char* src;
    const char* lsrc;  // this lane's 16-byte slot of this wave's first 1 KB round
    int cur, nxt_buf, gch;
    const char* win;
    __device__ __forceinline__ GroupStream(char* l, const char* s)
        : lds(l), src(s),
          lsrc(s + (size_t)__builtin_amdgcn_readfirstlane(threadIdx.x >> 6) * 1024 + (threadIdx.x & 63) * 16),
          cur(NBUF - 1), nxt_buf(NBUF - 1), gch(0), win(l), nxt_ch(0) {}
    __device__ __forceinline__ void fetch(int ch, int b) const {
        const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
        const int lane = threadIdx.x & 63;
        const char* base = src + opaque_zero() + (size_t)ch * CHB;
#pragma unroll
        for (int r = 0; r < ROUNDS; ++r) {
            const int off = (r * kWaves + wave) * 1024;
            __builtin_amdgcn_global_load_lds((const void*)(base + off + lane * 16),
                                             (__attribute__((address_space(3))) void*)(lds + b * CHB + off), 16, 0,
                                             0);
        }
    }
    __device__ __forceinline__ void start() {
#pragma unroll
        for (int j = 0; j < NBUF - 1; ++j) fetch(j, j);
    }
    __device__ __forceinline__ void begin_group(int gi) { gch = gi * CPG; }
    // One 1 KB load of chunk ch into buffer b (round r of this wave).
    __device__ __forceinline__ void fetch_round(int ch, int b, int r) const {
        const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
        const int off = (r * kWaves + wave) * 1024;
        // one scalar offset added to the lane's precomputed address (kept
        // opaque so that its constant part is not split off into a second add)
        __builtin_amdgcn_global_load_lds((const void*)(lsrc + opaque_u32((uint32_t)(ch * CHB + r * kWaves * 1024))),
                                         (__attribute__((address_space(3))) void*)(lds + b * CHB + off), 16, 0, 0);
    }
    // The loads of the chunk NBUF - 1 ahead are spread over the current chunk
    // (one round every SPREAD fragments) rather than issued in a burst at its
    // boundary, where four waves queueing behind the address unit would stall.
    static constexpr int SPREAD = FPC / ROUNDS;
    static_assert(FPC % ROUNDS == 0, "every fragment of a group is served: rounds must divide a chunk");
    int nxt_ch;
    template <int POS>
    __device__ __forceinline__ typename Frag<N::DT>::type load(int lane) {
        constexpr int within = POS % FPC;
        if constexpr (within == 0) {
            __builtin_amdgcn_s_waitcnt(waitcnt_vm_lgkm0((NBUF - 2) * ROUNDS));
            __builtin_amdgcn_s_barrier();
            cur = cur + 1 == NBUF ? 0 : cur + 1;
            int nxt = gch + POS / FPC + NBUF - 1;
            nxt_ch = nxt < NCH ? nxt : nxt - NCH;
        }
        if constexpr (within % SPREAD == 0 && within / SPREAD < ROUNDS) {
            fetch_round(nxt_ch, nxt_buf, within / SPREAD);
            if constexpr (within / SPREAD == ROUNDS - 1) nxt_buf = nxt_buf + 1 == NBUF ? 0 : nxt_buf + 1;
        }
        if constexpr (within % WINF == 0) win = lds + cur * CHB + within * FB + opaque_zero();
        return Frag<N::DT>::load(win, within % WINF, lane);
    }
    __device__ __forceinline__ void finish() { __builtin_amdgcn_s_waitcnt(0); }
};

// Bytes of one LDS chunk buffer of a streaming network source.
// The streaming source of a network evaluated layer by layer.
template <class N, int CHB = VOILA_STREAM_CHB>
using StreamFor = StreamSrc<N, CHB>;

template <class N, int CHB = VOILA_STREAM_CHB, bool G = (N::CT < N::HT)> struct StreamChunk {
    static constexpr int BYTES = StreamFor<N, CHB>::LDS_BYTES;  // LDS of the chunk buffers
};
template <class N, int CHB> struct StreamChunk<N, CHB, true> {
    static constexpr int BYTES = GroupStream<N>::LDS_BYTES;
};

// LDS per workgroup, and whether a grouped wide network's first layer is
// staged in LDS beside its chunk buffers and staged biases (n_var first-layer
// bias variants), or read from L2.
constexpr int kLdsMax = 160 * 1024;
template <class N>
__host__ __device__ constexpr bool first_layer_in_lds(int n_var) {
    if constexpr (N::CT < N::HT)
        return StreamChunk<N>::BYTES + N::NF0 * N::FRAG_BYTES + (n_var + N::NHID - 1) * N::WIDTH * 4 + 1024 <= kLdsMax;
    else
        return false;
}

template <class N, class HS>
struct WideSrc {
    DirectSrc<N::DT, 8> first;
    HS hid;
    __device__ __forceinline__ WideSrc(const char* f0, HS h) : first(f0), hid(h) {}
};

template <class N, class Src>
__device__ __forceinline__ f32x16 run_net_grouped(Src& src, const NetPtrs& P, const float* b0,
                                                  const float (&slots)[N::IN_SLOTS], int lane, int g) {
    typedef FragIdx<N> FI;
    typedef typename Frag<N::DT>::type FT;
    constexpr int CT = N::CT, OKS = N::OKS;
    Act<N::DT, N::HT> act;
    static_for<N::HT / CT>([&](auto gi) {
        constexpr int tc = decltype(gi)::value * CT;
        f32x16 acc[CT];
        init_bias<CT>(acc, b0 + 32 * tc + opaque_zero(), g);
        mfma_layer<N::IN_KS, CT, 2, FT>(
            acc, [&](int c, int t) { return src.first.load(FI::first(c, tc + t), lane); },
            [&](int c) { return Slots<N::DT, N::IN_SLOTS>::b(slots, c); });
        act.template set_relu_at<CT>(acc, tc);
    });
    f32x16 out[1];
    init_bias<1>(out, P.bo + opaque_zero(), g);
#pragma unroll 1
    for (int gi = 0; gi < N::HT / CT; ++gi) {
        src.hid.begin_group(gi);
        f32x16 acc[CT];
        init_bias<CT>(acc, P.bh + 32 * CT * gi + opaque_zero(), g);
        // hidden fragments: ring of two k-steps, positions known at compile time
        constexpr int D = kPfDepth;
        FT ring[D][CT];
        static_for<D - 1>([&](auto pi) {
            constexpr int c = decltype(pi)::value;
            static_for<CT>([&](auto ti) {
                constexpr int t = decltype(ti)::value;
                ring[c][t] = src.hid.template load<c * CT + t>(lane);
            });
        });
        // the group's output-layer k-steps follow its hidden fragments; they
        // load during the last hidden k-step
        constexpr int OB = N::HID_KS * CT;
        FT of[OKS * CT];
        static_for<N::HID_KS>([&](auto ci) {
            constexpr int c = decltype(ci)::value;
            if constexpr (c + D - 1 < N::HID_KS) {
                static_for<CT>([&](auto ti) {
                    constexpr int t = decltype(ti)::value;
                    ring[(c + D - 1) % D][t] = src.hid.template load<(c + D - 1) * CT + t>(lane);
                });
            } else if constexpr (c + 1 == N::HID_KS) {
                static_for<OKS * CT>([&](auto oi) {
                    constexpr int o = decltype(oi)::value;
                    of[o] = src.hid.template load<OB + o>(lane);
                });
            }
            auto b = act.b(c);
            static_for<CT>([&](auto ti) {
                constexpr int t = decltype(ti)::value;
                acc[t] = mfma(ring[c % D][t], b, acc[t]);
            });
            constexpr int NR = c + D - 1 < N::HID_KS ? CT : (c + 1 == N::HID_KS ? OKS * CT : 0);
            if constexpr (NR > 0) __builtin_amdgcn_sched_group_barrier(kSchedReads, NR, 0);
            __builtin_amdgcn_sched_group_barrier(kSchedMfma, CT, 0);
            __builtin_amdgcn_sched_barrier(0);
        });
        Act<N::DT, CT> a2;
        a2.set_relu(acc);
        static_for<OKS * CT>([&](auto ci) {
            constexpr int c = decltype(ci)::value;
            out[0] = mfma(of[c], a2.b(c), out[0]);
        });
        __builtin_amdgcn_sched_barrier(0);
    }
    return out[0];
}

// Layered networks evaluated by the four waves of a workgroup together, on
// the same 32 rollouts (a pass over few particles then keeps four SIMDs busy
// per tile instead of one): wave w produces the 32-row tiles
// [w HT/4, (w + 1) HT/4) of every hidden layer, the activations pass through
// LDS with each tile's registers stored as they are (so k-step c of the next
// layer reads its B operand at [c][lane]), the output layer's k-steps are
// split over the waves and the four partial tiles are added in wave order.
// Weights are read from global memory at per-wave offsets, D - 1 k-steps
// ahead.
template <class N> struct SplitLds {
    static constexpr int ACT = N::DT == DT_F32 ? N::HT * 16 * 64 * 4 : 2 * N::HT * 64 * 16;
    static constexpr int PART = 4 * 16 * 64 * 4;
    static constexpr int BYTES = ACT + PART;
};

template <class N>
__device__ __forceinline__ typename Frag<N::DT>::type split_act(const char* lds, int c, int lane) {
    return reinterpret_cast<const typename Frag<N::DT>::type*>(lds)[c * 64 + lane];
}

template <class N, int TPW>
__device__ __forceinline__ void split_store(char* lds, const f32x16 (&acc)[TPW], int t0, int lane) {
    if constexpr (N::DT == DT_F32) {
        float* a = reinterpret_cast<float*>(lds);
#pragma unroll
        for (int t = 0; t < TPW; ++t)
#pragma unroll
            for (int i = 0; i < 16; ++i) a[((t0 + t) * 16 + i) * 64 + lane] = relu_f32(acc[t][i]);
    } else {
        bf16x8* a = reinterpret_cast<bf16x8*>(lds);
#pragma unroll
        for (int t = 0; t < TPW; ++t)
#pragma unroll
            for (int h = 0; h < 2; ++h) a[(2 * (t0 + t) + h) * 64 + lane] = relu_bf16x8(acc[t], h);
    }
}

template <class N>
__device__ __forceinline__ f32x16 run_net_split(const NetPtrs& P, const float* b0, const float (&slots)[N::IN_SLOTS],
                                                int lane, int g, int wave, char* lds) {
    static_assert(N::HT % 4 == 0 && N::CT == N::HT, "split evaluation needs a layered network of 4k tiles");
    constexpr int TPW = N::HT / 4, KQ = N::HID_KS / 4;
    // k-steps of weight fragments in flight: 32 (binary32) or 16 (bfloat16)
    // fragment loads over the wave's tiles
    constexpr int D = (N::DT == DT_F32 ? 32 : 16) / TPW > 0 ? (N::DT == DT_F32 ? 32 : 16) / TPW : 1;
    typedef typename Frag<N::DT>::type FT;
    typedef FragIdx<N> FI;
    const int t0 = wave * TPW;
    // the fragments of k-step c start HT fragments after those of k-step c - 1;
    // a fresh scalar base per k-step keeps every load's offset small
    auto kstep = [&](const char* base, int c) { return base + (size_t)c * N::HT * N::FRAG_BYTES + opaque_zero(); };
    f32x16 acc[TPW];
    init_bias<TPW>(acc, b0 + 32 * t0 + opaque_zero(), g);
    {
        const char* base = P.f0 + (size_t)FI::first(0, t0) * N::FRAG_BYTES + opaque_zero();
        mfma_layer<N::IN_KS, TPW, D, FT>(
            acc, [&](int c, int t) { return Frag<N::DT>::load(kstep(base, c), t, lane); },
            [&](int c) { return Slots<N::DT, N::IN_SLOTS>::b(slots, c); });
    }
    split_store<N, TPW>(lds, acc, t0, lane);
    __syncthreads();
    static_for<N::NHID - 1>([&](auto li) {
        constexpr int l = decltype(li)::value + 1;
        init_bias<TPW>(acc, P.bh + (l - 1) * N::WIDTH + 32 * t0 + opaque_zero(), g);
        const char* base = P.f0 + (size_t)FI::hidden(l, 0, t0) * N::FRAG_BYTES + opaque_zero();
        mfma_layer<N::HID_KS, TPW, D, FT>(
            acc, [&](int c, int t) { return Frag<N::DT>::load(kstep(base, c), t, lane); },
            [&](int c) { return split_act<N>(lds, c, lane); });
        __syncthreads();
        split_store<N, TPW>(lds, acc, t0, lane);
        __syncthreads();
    });
    f32x16 part[1];
    init_bias<1>(part, P.bo + opaque_zero(), g);
    if (wave != 0) part[0] = f32x16{};
    {
        const int k0 = wave * KQ;
        const char* base = P.f0 + (size_t)(FI::out(0) + k0) * N::FRAG_BYTES + opaque_zero();
        mfma_layer<KQ, 1, D, FT>(
            part, [&](int c, int) { return Frag<N::DT>::load(base + (size_t)c * N::FRAG_BYTES + opaque_zero(), 0, lane); },
            [&](int c) { return split_act<N>(lds, k0 + c, lane); });
    }
    float* pl = reinterpret_cast<float*>(lds + SplitLds<N>::ACT);
#pragma unroll
    for (int i = 0; i < 16; ++i) pl[(wave * 16 + i) * 64 + lane] = part[0][i];
    __syncthreads();
    f32x16 out;
#pragma unroll
    for (int i = 0; i < 16; ++i)
        out[i] = ((pl[i * 64 + lane] + pl[(16 + i) * 64 + lane]) + pl[(32 + i) * 64 + lane]) + pl[(48 + i) * 64 + lane];
    __syncthreads();
    return out;
}

// mfma_layer for ST sample tiles at once: every weight fragment loaded (and
// prefetched D k-steps ahead) feeds the products of all ST tiles; bop(c, st)
// is tile st's B operand of k-step c.
template <int KS, int NT, int ST, int D, class FT, class LD, class BOP>
__device__ __forceinline__ void mfma_layer_multi(f32x16 (&acc)[ST][NT], LD&& ld, BOP&& bop) {
    constexpr int DD = D < KS ? D : KS;
    FT ring[DD][NT];
    static_for<DD - 1>([&](auto pi) {
        constexpr int c = decltype(pi)::value;
        static_for<NT>([&](auto ti) { ring[c][decltype(ti)::value] = ld(c, decltype(ti)::value); });
    });
    static_for<KS>([&](auto ci) {
        constexpr int c = decltype(ci)::value;
        if constexpr (c + DD - 1 < KS) {
            static_for<NT>([&](auto ti) {
                ring[(c + DD - 1) % DD][decltype(ti)::value] = ld(c + DD - 1, decltype(ti)::value);
            });
        }
        static_for<ST>([&](auto si) {
            constexpr int st = decltype(si)::value;
            auto b = bop(c, st);
            static_for<NT>([&](auto ti) {
                constexpr int t = decltype(ti)::value;
                acc[st][t] = mfma(ring[c % DD][t], b, acc[st][t]);
            });
        });
        if constexpr (c + DD - 1 < KS) __builtin_amdgcn_sched_group_barrier(kSchedReads, NT, 0);
        __builtin_amdgcn_sched_group_barrier(kSchedMfma, NT * ST, 0);
        __builtin_amdgcn_sched_barrier(0);
    });
}

// Pass-major fragment order of a layered network whose layers are produced
// RP output tiles at a time (run_net_passes): within each layer the
// fragments of pass p (tiles RP p .. RP p + RP - 1) come first, k-step by
// k-step; the output layer follows as usual.
__host__ __device__ constexpr int pass_first(int in_ks, int rp, int c, int t) { return ((t / rp) * in_ks + c) * rp + t % rp; }
__host__ __device__ constexpr int pass_hidden(int nf0, int nfh, int hid_ks, int rp, int l, int c, int t) {
    return nf0 + (l - 1) * nfh + ((t / rp) * hid_ks + c) * rp + t % rp;
}

// A layered network (streamed in the pass-major order) on ST sample tiles of
// one wave: every layer is produced RP output tiles at a time, each weight
// fragment read from the stream serves all ST sample tiles, and the next
// layer's operands are converted pass by pass while the current layer's
// remain in registers.  out[st] is sample tile st's output tile.
template <class N, int ST, int RP, class Src>
__device__ __forceinline__ void run_net_passes(Src& src, const NetPtrs& P, const float* b0,
                                               const float (&slots)[ST][N::IN_SLOTS], f32x16 (&out)[ST], int lane,
                                               int g) {
    static_assert(N::CT == N::HT && N::HT % RP == 0, "pass evaluation needs a layered network");
    typedef typename Frag<N::DT>::type FT;
    constexpr int NP = N::HT / RP;
#ifdef VOILA_PASS_DEPTH
    constexpr int D = VOILA_PASS_DEPTH;
#else
    constexpr int D = N::DT == DT_F32 ? kPfDepthF32 : kPfDepth;
#endif
    Act<N::DT, N::HT> act[ST];
    static_for<NP>([&](auto pi) {
        constexpr int p = decltype(pi)::value;
        f32x16 acc[ST][RP];
#pragma unroll
        for (int st = 0; st < ST; ++st) init_bias<RP>(acc[st], b0 + 32 * RP * p + opaque_zero(), g);
        mfma_layer_multi<N::IN_KS, RP, ST, 2, FT>(
            acc, [&](int c, int t) { return src.load(pass_first(N::IN_KS, RP, c, RP * p + t), lane); },
            [&](int c, int st) { return Slots<N::DT, N::IN_SLOTS>::b(slots[st], c); });
#pragma unroll
        for (int st = 0; st < ST; ++st) act[st].template set_relu_at<RP>(acc[st], RP * p);
    });
    static_for<N::NHID - 1>([&](auto li) {
        constexpr int l = decltype(li)::value + 1;
        Act<N::DT, N::HT> nxt[ST];
        static_for<NP>([&](auto pi) {
            constexpr int p = decltype(pi)::value;
            f32x16 acc[ST][RP];
#pragma unroll
            for (int st = 0; st < ST; ++st)
                init_bias<RP>(acc[st], P.bh + (l - 1) * N::WIDTH + 32 * RP * p + opaque_zero(), g);
            mfma_layer_multi<N::HID_KS, RP, ST, D, FT>(
                acc,
                [&](int c, int t) {
                    return src.load(pass_hidden(N::NF0, N::NFH, N::HID_KS, RP, l, c, RP * p + t), lane);
                },
                [&](int c, int st) { return act[st].b(c); });
#pragma unroll
            for (int st = 0; st < ST; ++st) nxt[st].template set_relu_at<RP>(acc[st], RP * p);
        });
#pragma unroll
        for (int st = 0; st < ST; ++st) act[st] = nxt[st];
    });
    f32x16 o[ST][1];
#pragma unroll
    for (int st = 0; st < ST; ++st) init_bias<1>(o[st], P.bo + opaque_zero(), g);
    mfma_layer_multi<N::HID_KS, 1, ST, 4, FT>(
        o, [&](int c, int) { return src.load(N::NF0 + (N::NHID - 1) * N::NFH + c, lane); },
        [&](int c, int st) { return act[st].b(c); });
#pragma unroll
    for (int st = 0; st < ST; ++st) out[st] = o[st][0];
}

// run_net_passes as one pipelined sequence (bfloat16): the fragments are
// consumed in stream order with a single register ring that prefetches
// across pass and layer boundaries; the ReLU / bfloat16 conversion of each
// finished pass is spread over the matrix instructions of the pass that
// follows it (accumulators double-buffered by pass), so that the vector
// instructions issue in the shadow of the matrix core; and the biases of
// the next pass are read LEAD fragment-steps before it starts.  The
// conversion of a layer's last pass completes before the next layer's first
// k-step that reads it.  Same products, in the same order, as run_net_passes.
#ifndef VOILA_FLAT_DEPTH
#define VOILA_FLAT_DEPTH 3
#endif
#ifndef VOILA_FLAT_VALU
#define VOILA_FLAT_VALU 4
#endif
#ifndef VOILA_FLAT_LEAD
#define VOILA_FLAT_LEAD 4
#endif
template <class N, int RP, int LEAD>
struct FlatSeq {
    static constexpr int NP = N::HT / RP;
    static constexpr int NQ = N::NHID * NP;  // hidden-producing passes; pass NQ is the output layer
    static constexpr int NFR = N::NF0 + (N::NHID - 1) * N::NFH + N::NFO;
    static constexpr int OUT0 = N::NF0 + (N::NHID - 1) * N::NFH;  // first output-layer fragment
    static constexpr int KPT = 32 / (2 * N::KPER);                // k-steps per 32-row tile
    // layer, pass, k-step and output tile of fragment f (output layer: layer NHID, pass 0, tile 0)
    __host__ __device__ static constexpr int layer(int f) {
        return f < N::NF0 ? 0 : f >= OUT0 ? N::NHID : 1 + (f - N::NF0) / N::NFH;
    }
    __host__ __device__ static constexpr int rel(int f) {
        return f < N::NF0 ? f : f >= OUT0 ? f - OUT0 : (f - N::NF0) % N::NFH;
    }
    __host__ __device__ static constexpr int ks(int f) { return layer(f) == 0 ? N::IN_KS : N::HID_KS; }
    __host__ __device__ static constexpr int pass(int f) { return f >= OUT0 ? 0 : rel(f) / (ks(f) * RP); }
    __host__ __device__ static constexpr int kstep(int f) { return f >= OUT0 ? rel(f) : (rel(f) / RP) % ks(f); }
    __host__ __device__ static constexpr int tile(int f) { return f >= OUT0 ? 0 : rel(f) % RP; }
    __host__ __device__ static constexpr int gpass(int f) { return layer(f) * NP + pass(f); }
    // first fragment and length (fragment-steps) of global pass q
    __host__ __device__ static constexpr int pass_start(int q) {
        return q / NP == 0 ? (q % NP) * N::IN_KS * RP
               : q >= NQ   ? OUT0
                           : N::NF0 + (q / NP - 1) * N::NFH + (q % NP) * N::HID_KS * RP;
    }
    __host__ __device__ static constexpr int pass_len(int q) {
        return q >= NQ ? N::NFO : (q / NP == 0 ? N::IN_KS : N::HID_KS) * RP;
    }
    // fragment-step of pass q at which the biases of pass q + 1 are read
    __host__ __device__ static constexpr int bias_at(int q) { return pass_len(q) > LEAD ? pass_len(q) - LEAD : 0; }
    // fragment-steps of pass q + 1 over which pass q (q < NQ) is converted:
    // before pass q + 1 reads the biases of pass q + 2 into pass q's
    // accumulators, and before the next layer first reads pass q's tiles
    __host__ __device__ static constexpr int window(int q) {
        const int w = (q + 1) % NP != 0 ? pass_len(q + 1)
                      : KPT * RP * (NP - 1) * ((q + 1) >= NQ ? 1 : RP);
        return q + 2 < NQ && bias_at(q + 1) < w ? (bias_at(q + 1) > 0 ? bias_at(q + 1) : 1) : w;
    }
};

template <class N, int ST, int RP, class Src>
__device__ __forceinline__ void run_net_flat(Src& src, const NetPtrs& P, const float* b0,
                                             const float (&slots)[ST][N::IN_SLOTS], f32x16 (&out)[ST], int lane,
                                             int g) {
    static_assert(N::DT == DT_BF16 && N::CT == N::HT && N::HT % RP == 0 && N::NHID >= 2,
                  "flat evaluation needs a layered bfloat16 network");
    typedef typename Frag<N::DT>::type FT;
    typedef FlatSeq<N, RP, VOILA_FLAT_LEAD> Q;
    constexpr int NP = Q::NP, NQ = Q::NQ, NFR = Q::NFR;
    constexpr int PF = (VOILA_FLAT_DEPTH - 1) * RP;
    constexpr int R = PF + 1;
    constexpr int NPAIR = ST * RP * 8;  // converted value pairs per pass
    static_assert(NP >= 2, "a layer's last pass is converted while the next layer reads its first tiles");
    Act<N::DT, N::HT> A[2][ST];
    f32x16 acc[2][ST][RP];
    f32x16 o[ST];
    FT ring[R];
    // the biases of pass q into the first sample tile's accumulators: the
    // other tiles' first products of the pass take them as their addend
    // (D = A B + C with C the first tile's bias registers), so each bias is
    // read from LDS once per pass, not once per sample tile
    auto bias_of = [&](auto qi) {
        constexpr int q = decltype(qi)::value;
        if constexpr (q < NQ) {
            const float* bias = (q / NP == 0 ? b0 : P.bh + (q / NP - 1) * N::WIDTH) + 32 * RP * (q % NP);
            init_bias<RP>(acc[q % 2][0], bias + opaque_zero(), g);
        } else {
            f32x16 ob[1];
            init_bias<1>(ob, P.bo + opaque_zero(), g);
            o[0] = ob[0];
        }
    };
    bias_of(std::integral_constant<int, 0>{});
    static_for<PF>([&](auto fi) {
        constexpr int f = decltype(fi)::value;
        ring[f % R] = src.load(f, lane);
    });
    static_for<NFR>([&](auto fi) {
        constexpr int f = decltype(fi)::value;
        constexpr int L = Q::layer(f), c = Q::kstep(f), t = Q::tile(f);
        constexpr bool OUT = L == N::NHID;
        constexpr int q = Q::gpass(f);
        constexpr int s0 = f - Q::pass_start(q);  // fragment-step within the pass
        // conversion of the previous pass q - 1 into the activations of its
        // layer (before this step's bias reads, which may reuse its registers)
        if constexpr (q >= 1) {
            constexpr int qc = q - 1;
            constexpr int W = Q::window(qc);
            constexpr int PPS = (NPAIR + W - 1) / W;
            if constexpr (s0 < W) {
                constexpr int Lc = qc / NP, pc = qc % NP;
                static_for<PPS>([&](auto ji) {
                    constexpr int j = s0 * PPS + decltype(ji)::value;
                    if constexpr (j < NPAIR) {
                        constexpr int st = j / (RP * 8), tt = (j / 8) % RP, pr = j % 8;
                        A[Lc % 2][st].set_relu_pair(acc[qc % 2][st][tt], RP * pc + tt, pr);
                    }
                });
            }
        }
        if constexpr (q < NQ && s0 == Q::bias_at(q)) bias_of(std::integral_constant<int, q + 1>{});
        if constexpr (f + PF < NFR) ring[(f + PF) % R] = src.load(f + PF, lane);
        // the last sample tile first: at the pass's first k-step the tiles
        // after the first add to its bias registers before it is updated
        static_for<ST>([&](auto si) {
            constexpr int st = ST - 1 - decltype(si)::value;
            constexpr bool FROM0 = st > 0 && c == 0;
            if constexpr (L == 0) {
                acc[q % 2][st][t] = mfma(ring[f % R], Slots<N::DT, N::IN_SLOTS>::b(slots[st], c),
                                         acc[q % 2][FROM0 ? 0 : st][t]);
            } else if constexpr (!OUT) {
                acc[q % 2][st][t] = mfma(ring[f % R], A[(L - 1) % 2][st].b(c), acc[q % 2][FROM0 ? 0 : st][t]);
            } else {
                o[st] = mfma(ring[f % R], A[(L - 1) % 2][st].b(c), o[FROM0 ? 0 : st]);
            }
        });
        __builtin_amdgcn_sched_group_barrier(kSchedReads, 1, 0);
        static_for<ST>([&](auto) {
            __builtin_amdgcn_sched_group_barrier(kSchedMfma, 1, 0);
            __builtin_amdgcn_sched_group_barrier(0x002, VOILA_FLAT_VALU, 0);
        });
        __builtin_amdgcn_sched_barrier(0);
    });
#pragma unroll
    for (int st = 0; st < ST; ++st) out[st] = o[st];
}

// Split evaluation of ST sample tiles by the NW waves of a block: wave w
// computes output tiles [w HT/NW, (w+1) HT/NW) of every layer for all ST
// sample tiles, so each weight fragment read from L2 serves ST tiles.  The
// activations of sample tile st live at lds + st * ACT; the output layer's
// per-wave partials reuse that space.  bin(c, st) is the first-layer B
// operand of sample tile st at k-step c.  The outputs go to sink(st, t, i,
// v): value i of output tile t of sample tile st; with OWN false every wave
// receives every sample tile's, with OWN true wave w < ST only its own
// sample tile's (st = w) and the other waves none.  D k-steps of weight
// fragments are in flight.
template <class N, int ST, int NW, int D, bool OWN, class BIN, class SINK>
__device__ __forceinline__ void run_net_split_core(const NetPtrs& P, const float* b0, BIN&& bin, SINK&& sink,
                                                   int lane, int g, int wave, char* lds) {
    static_assert(N::HT % NW == 0 && N::HID_KS % NW == 0 && N::CT == N::HT, "split needs a layered network");
    static_assert(!OWN || ST <= NW, "every sample tile needs an owner wave");
    constexpr int TPW = N::HT / NW, KQ = N::HID_KS / NW;
    constexpr int ACT = SplitLds<N>::ACT;
    static_assert(ST * NW * 16 * 64 * 4 <= ST * ACT, "partials must fit the activation space");
    typedef typename Frag<N::DT>::type FT;
    typedef FragIdx<N> FI;
    const int t0 = wave * TPW;
    auto kstep = [&](const char* base, int c) { return base + (size_t)c * N::HT * N::FRAG_BYTES + opaque_zero(); };
    // one base register per sample tile's activations, the k-steps as
    // immediate offsets (a folded constant base past 64 KB would need one
    // address register per k-step, which the compiler hoists and spills)
    char* act[ST];
#pragma unroll
    for (int st = 0; st < ST; ++st) act[st] = lds + st * ACT + opaque_zero();
    f32x16 acc[ST][TPW];
#pragma unroll
    for (int st = 0; st < ST; ++st) init_bias<TPW>(acc[st], b0 + 32 * t0 + opaque_zero(), g);
    {
        const char* base = P.f0 + (size_t)FI::first(0, t0) * N::FRAG_BYTES + opaque_zero();
        mfma_layer_multi<N::IN_KS, TPW, ST, D, FT>(
            acc, [&](int c, int t) { return Frag<N::DT>::load(kstep(base, c), t, lane); }, bin);
    }
#pragma unroll
    for (int st = 0; st < ST; ++st) split_store<N, TPW>(act[st], acc[st], t0, lane);
    __syncthreads();
    static_for<N::NHID - 1>([&](auto li) {
        constexpr int l = decltype(li)::value + 1;
#pragma unroll
        for (int st = 0; st < ST; ++st) init_bias<TPW>(acc[st], P.bh + (l - 1) * N::WIDTH + 32 * t0 + opaque_zero(), g);
        const char* base = P.f0 + (size_t)FI::hidden(l, 0, t0) * N::FRAG_BYTES + opaque_zero();
        mfma_layer_multi<N::HID_KS, TPW, ST, D, FT>(
            acc, [&](int c, int t) { return Frag<N::DT>::load(kstep(base, c), t, lane); },
            [&](int c, int st) { return split_act<N>(act[st], c, lane); });
        __syncthreads();
#pragma unroll
        for (int st = 0; st < ST; ++st) split_store<N, TPW>(act[st], acc[st], t0, lane);
        __syncthreads();
    });
    // the output layer: each wave multiplies its k-steps for every output
    // tile, then the partial tiles are added in wave order, tile by tile (the
    // partials reuse the activation space once every wave has read it)
    f32x16 part[ST][N::NO];
#pragma unroll
    for (int st = 0; st < ST; ++st) {
        init_bias<N::NO>(part[st], P.bo + opaque_zero(), g);
        if (wave != 0)
#pragma unroll
            for (int t = 0; t < N::NO; ++t) part[st][t] = f32x16{};
    }
    {
        const int k0 = wave * KQ;
        const char* base = P.f0 + (size_t)(FI::out(0) + k0) * N::FRAG_BYTES + opaque_zero();
        mfma_layer_multi<KQ, N::NO, ST, D, FT>(
            part,
            [&](int c, int t) {
                return Frag<N::DT>::load(base + (size_t)(t * N::HID_KS + c) * N::FRAG_BYTES + opaque_zero(), 0, lane);
            },
            [&](int c, int st) { return split_act<N>(act[st], k0 + c, lane); });
    }
    __syncthreads();  // every wave has read the activations the partials overwrite
    float* pl = reinterpret_cast<float*>(lds);
    auto total = [&](int st, int i) {
        float v = pl[((st * NW) * 16 + i) * 64 + lane];
        for (int w = 1; w < NW; ++w) v += pl[((st * NW + w) * 16 + i) * 64 + lane];
        return v;
    };
#pragma unroll
    for (int t = 0; t < N::NO; ++t) {
#pragma unroll
        for (int st = 0; st < ST; ++st)
#pragma unroll
            for (int i = 0; i < 16; ++i) pl[((st * NW + wave) * 16 + i) * 64 + lane] = part[st][t][i];
        __syncthreads();
        if constexpr (OWN) {
            if (wave < ST)
#pragma unroll
                for (int i = 0; i < 16; ++i) sink(wave, t, i, total(wave, i));
        } else {
#pragma unroll
            for (int st = 0; st < ST; ++st)
#pragma unroll
                for (int i = 0; i < 16; ++i) sink(st, t, i, total(st, i));
        }
        __syncthreads();
    }
}

// The split evaluation with the first-layer inputs of every sample tile in
// each wave's slots; every wave receives every output tile.
template <class N, int ST, int NW, int D>
__device__ __forceinline__ void run_net_split_multi(const NetPtrs& P, const float* b0,
                                                    const float (&slots)[ST][N::IN_SLOTS],
                                                    f32x16 (&out)[ST * N::NO], int lane, int g, int wave,
                                                    char* lds) {
    run_net_split_core<N, ST, NW, D, false>(
        P, b0, [&](int c, int st) { return Slots<N::DT, N::IN_SLOTS>::b(slots[st], c); },
        [&](int st, int t, int i, float v) { out[st * N::NO + t][i] = v; }, lane, g, wave, lds);
}

// First-layer operands of one sample tile staged in LDS by the wave that owns
// the tile (the others then carry no per-sample state).
template <class N> struct SplitIn {
    static constexpr int BYTES = N::IN_KS * 64 * (int)sizeof(typename Frag<N::DT>::type);
};
template <class N>
__device__ __forceinline__ void split_stage_inputs(char* lds_in, const float (&slots)[N::IN_SLOTS], int lane) {
    typedef typename Frag<N::DT>::type FT;
    FT* d = reinterpret_cast<FT*>(lds_in);
#pragma unroll
    for (int c = 0; c < N::IN_KS; ++c) d[c * 64 + lane] = Slots<N::DT, N::IN_SLOTS>::b(slots, c);
}

// The split evaluation with the first-layer operands of sample tile st at
// lds_in + st * SplitIn<N>::BYTES (written, before a barrier, by its owner
// wave st); wave w < ST receives its own sample tile's output tiles as
// out[t][i] (plain scalars: no vector register tuple is rebuilt per value).
template <class N, int ST, int NW, int D>
__device__ __forceinline__ void run_net_split_owned(const NetPtrs& P, const float* b0, const char* lds_in,
                                                    float (&out)[N::NO][16], int lane, int g, int wave, char* lds) {
    typedef typename Frag<N::DT>::type FT;
    const FT* in[ST];
#pragma unroll
    for (int st = 0; st < ST; ++st)
        in[st] = reinterpret_cast<const FT*>(lds_in + st * SplitIn<N>::BYTES + opaque_zero());
    run_net_split_core<N, ST, NW, D, true>(
        P, b0, [&](int c, int st) { return in[st][c * 64 + lane]; },
        [&](int, int t, int i, float v) { out[t][i] = v; }, lane, g, wave, lds);
}

// Fragment source of a network read straight from global memory: the plain
// source for networks evaluated layer by layer, the grouped bundle otherwise.
template <class N, bool GROUPED = (N::CT < N::HT)> struct DirectFor;
template <class N> struct DirectFor<N, false> {
    typedef DirectSrc<N::DT, 4 * N::HT> type;
    __device__ static __forceinline__ type make(const NetPtrs& P) { return type(P.f0); }
};
template <class N> struct DirectFor<N, true> {
    typedef WideSrc<N, GroupDirect<N>> type;
    __device__ static __forceinline__ type make(const NetPtrs& P) { return type(P.f0, GroupDirect<N>(P.fh)); }
};

// ----------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) and Box-Muller draws.
// ----------------------------------------------------------------------------
__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        // one 32 x 32 -> 64-bit product per multiplier (v_mad_u64_u32) gives
        // both halves, where separate high and low products take two
        const uint64_t p0 = (uint64_t)0xD2511F53u * c.x, p1 = (uint64_t)0xCD9E8D57u * c.z;
        const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        // each three-way exclusive or in one instruction (v_bitop3_b32 with
        // the truth table 0x96 of a ^ b ^ c), where separate ones take two
        c = make_uint4(__builtin_amdgcn_bitop3_b32(hi1, c.y, k0, 0x96), lo1,
                       __builtin_amdgcn_bitop3_b32(hi0, c.w, k1, 0x96), lo0);
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c;
}

// u = (2 (x >> 9) + 1) 2^-24, exact in binary32, inside (0, 1).
__device__ __forceinline__ float word_to_uniform(uint32_t x) {
    return (float)((x >> 8) | 1u) * 0x1p-24f;
}

// Box-Muller pair from two words: (r cos 2 pi u_b, r sin 2 pi u_b), r = sqrt(-2 ln u_a),
// on the hardware transcendental units: -2 ln u_a = -2 ln 2 log2 u_a (v_log_f32),
// v_sqrt_f32, and v_sin_f32 / v_cos_f32, which take their argument in turns
// (sin 2 pi x), so u_b in (0, 1) needs no range reduction.
__device__ __forceinline__ void box_muller(uint32_t wa, uint32_t wb, float& z_cos, float& z_sin) {
    const float ua = word_to_uniform(wa), ub = word_to_uniform(wb);
    const float r = __builtin_amdgcn_sqrtf(-1.3862943611198906f * __builtin_amdgcn_logf(ua));
    z_cos = r * __builtin_amdgcn_cosf(ub);
    z_sin = r * __builtin_amdgcn_sinf(ub);
}

// The value of the lane 32 positions away: lanes l < 32 get lane l + 32's
// value and lanes l >= 32 lane l - 32's (one v_permlane32_swap; every lane of
// the wave must be active).
__device__ __forceinline__ uint32_t swap_halves(uint32_t v) {
    const auto r = __builtin_amdgcn_permlane32_swap(v, v, false, false);
    return (threadIdx.x & 32) ? r[0] : r[1];
}

// The noise slots of lane group g: slot s holds feature 4 (s / 2) + 2 g + s % 2,
// i.e. pair g of Philox block s / 2 of counter (c0, c1, c2, (stream << 16) | block).
// The two lane groups of a column need the two halves of the same blocks:
// with an even number of blocks each group computes every other block and
// hands the other group the pair it needs, so each block is computed once.
template <int NS>
__device__ __forceinline__ void noise_slots_philox(float (&out)[NS], uint32_t key0, uint32_t key1, uint32_t c0,
                                                   uint32_t c1, uint32_t c2, uint32_t stream, int g) {
    constexpr int NB = NS / 2;
    if constexpr (NB % 2 == 0) {
#pragma unroll
        for (int q = 0; q < NB / 2; ++q) {
            // group g computes block 2 q + g
            const uint4 w = philox4x32_10(make_uint4(c0, c1, c2, (stream << 16) | (uint32_t)(2 * q + g)), key0, key1);
            const uint32_t own_a = g ? w.z : w.x, own_b = g ? w.w : w.y;
            const uint32_t got_a = swap_halves(g ? w.x : w.z), got_b = swap_halves(g ? w.y : w.w);
            // block 2 q: group 0's own pair, group 1 receives it; block 2 q + 1 the other way round
            box_muller(g ? got_a : own_a, g ? got_b : own_b, out[4 * q], out[4 * q + 1]);
            box_muller(g ? own_a : got_a, g ? own_b : got_b, out[4 * q + 2], out[4 * q + 3]);
        }
    } else {
#pragma unroll
        for (int blk = 0; blk < NB; ++blk) {
            uint4 w = philox4x32_10(make_uint4(c0, c1, c2, (stream << 16) | (uint32_t)blk), key0, key1);
            uint32_t wa = g ? w.z : w.x;
            uint32_t wb = g ? w.w : w.y;
            box_muller(wa, wb, out[2 * blk], out[2 * blk + 1]);
        }
    }
}

// Philox words of the noise slots of lane group g for steps c2 and c2 + 1
// (counter (c0, c1, step, (stream << 16) | block)), each block computed once:
// group g computes the blocks of step c2 + g, keeps its own pair and hands the
// other group its pair of the same step.  now[2 b], now[2 b + 1] are the
// words of block b at step c2, next[] those at step c2 + 1.
template <int NS>
__device__ __forceinline__ void philox_two_steps(uint32_t (&now)[NS], uint32_t (&next)[NS], uint32_t key0,
                                                 uint32_t key1, uint32_t c0, uint32_t c1, uint32_t c2,
                                                 uint32_t stream, int g) {
#pragma unroll
    for (int blk = 0; blk < NS / 2; ++blk) {
        const uint4 w = philox4x32_10(make_uint4(c0, c1, c2 + (uint32_t)g, (stream << 16) | (uint32_t)blk), key0, key1);
        const uint32_t own_a = g ? w.z : w.x, own_b = g ? w.w : w.y;
        const uint32_t got_a = swap_halves(g ? w.x : w.z), got_b = swap_halves(g ? w.y : w.w);
        now[2 * blk] = g ? got_a : own_a;
        now[2 * blk + 1] = g ? got_b : own_b;
        next[2 * blk] = g ? own_a : got_a;
        next[2 * blk + 1] = g ? own_b : got_b;
    }
}

// Box-Muller draws of the noise slots from their Philox words.
template <int NS>
__device__ __forceinline__ void noise_from_words(float (&out)[NS], const uint32_t (&wd)[NS]) {
#pragma unroll
    for (int blk = 0; blk < NS / 2; ++blk) box_muller(wd[2 * blk], wd[2 * blk + 1], out[2 * blk], out[2 * blk + 1]);
}

// Noise feature held by slot s of group g.
__host__ __device__ constexpr int noise_feature(int s, int g) { return 4 * (s / 2) + 2 * g + (s % 2); }

// Copies a packed network blob into LDS (bytes is a multiple of 16).
__device__ __forceinline__ void stage_blob(char* dst, const char* src, uint32_t bytes) {
    const uint4* s = reinterpret_cast<const uint4*>(src);
    uint4* d = reinterpret_cast<uint4*>(dst);
    for (uint32_t i = threadIdx.x; i < bytes / 16; i += blockDim.x) d[i] = s[i];
}

// Wave-wide reductions across the 32 columns of one lane group (fixed order).
__device__ __forceinline__ float sum32(float v) {
    v += __shfl_xor(v, 16);
    v += __shfl_xor(v, 8);
    v += __shfl_xor(v, 4);
    v += __shfl_xor(v, 2);
    v += __shfl_xor(v, 1);
    return v;
}

}  // namespace voila
