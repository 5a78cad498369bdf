// abi.hip -- the extern "C" entry points of include/voila.h: argument checks,
// packing of the networks into MFMA fragment order, workspace carving and
// kernel launches.  Nothing here computes a result on the host.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <algorithm>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/voila.h"
#include "kernels.hpp"

using namespace voila;

namespace {

thread_local std::string g_last_error;

voila_status_t fail(voila_status_t st, const std::string& msg) {
    g_last_error = msg;
    return st;
}

#define VOILA_CHECK_HIP(expr)                                                            \
    do {                                                                                 \
        hipError_t e_ = (expr);                                                          \
        if (e_ != hipSuccess) return fail(VOILA_ERR_DEVICE, std::string(#expr) + ": " + \
                                                                hipGetErrorString(e_)); \
    } while (0)

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Round a binary32 value to bfloat16 (nearest, ties to even) and back.
float bf16_round(float v) {
    uint32_t u;
    std::memcpy(&u, &v, 4);
    if ((u & 0x7f800000u) == 0x7f800000u) return v;
    u += 0x7fffu + ((u >> 16) & 1u);
    u &= 0xffff0000u;
    float r;
    std::memcpy(&r, &u, 4);
    return r;
}
uint16_t bf16_bits(float v) {
    float r = bf16_round(v);
    uint32_t u;
    std::memcpy(&u, &r, 4);
    return (uint16_t)(u >> 16);
}

struct HostNet {
    int n_layers = 0;
    std::vector<int> dims;
    std::vector<const float*> W, b;
    bool present() const { return n_layers > 0; }
    int width() const { return dims[1]; }
    int out() const { return dims[n_layers]; }
    float w(int l, int o, int c) const { return W[l][(size_t)o * dims[l] + c]; }
};

// Input column of first-layer slot si of lane group g (-1: padding).
struct SlotMap {
    int d_s, d_ain, d_w, col_a, col_w;
    int col_s = 0;  // input column of the first "state" slot feature
    int operator()(int si, int g) const {
        const int SS = state_slots(d_s), SA = action_slots(d_ain), SW = noise_slots(d_w);
        if (si < SS) {
            int f = 2 * si + g;
            return f < d_s ? col_s + f : -1;
        }
        si -= SS;
        if (si < SA) {
            int f = 2 * si + g;
            return f < d_ain ? col_a + f : -1;
        }
        si -= SA;
        if (si < SW) {
            int f = noise_feature(si, g);
            return f < d_w ? col_w + f : -1;
        }
        return -1;
    }
};

// Output feature held by row r of the output tile (feature 2 i + g sits at out_row(i, g)).
int row_feature(int r) {
    int i = (r / 8) * 4 + (r % 4), g = (r / 4) % 2;
    return 2 * i + g;
}

// Packs one network into a blob: fragments of every layer in the order the
// kernels consume them, then the biases.  b0_variants holds n_var rows of
// `width` first-layer biases.
std::vector<char> pack_net(const HostNet& n, int dt, int in_slots_per_group, const SlotMap& map,
                           const std::vector<float>& b0_variants, int n_var, NetBlob& nb, bool layered = false,
                           int pass_tiles = 0) {
    const int W = n.width(), HT = W / 32, NHID = n.n_layers - 1, KP = kper(dt);
    const int CT = layered ? HT : default_ct(W, NHID);
    const int esz = dt == DT_F32 ? 4 : 2;
    const size_t fb = (size_t)64 * KP * esz;
    const int IN_KS = in_slots_per_group / KP, HID_KS = 16 * HT / KP;
    // 32-row output tiles: more than one only for networks packed layer by
    // layer (the split evaluation), tile t's k-steps following tile t - 1's
    const int NO = (layered || (CT == HT && !pass_tiles)) ? (n.out() + 31) / 32 : 1;
    const size_t nf0 = (size_t)IN_KS * HT, nfh = (size_t)HID_KS * HT, nfo = (size_t)NO * HID_KS;
    const size_t off_f0 = 0;
    const size_t off_fh = off_f0 + nf0 * fb;
    const size_t off_fo = off_fh + (size_t)(NHID - 1) * nfh * fb;
    // networks streamed whole through LDS chunk buffers are padded to whole chunks
    const size_t nfr = nf0 + (size_t)(NHID - 1) * nfh + nfo;
    const size_t fpc = kStreamPadBytes / fb;
    const size_t pad = (W > 64 && CT == HT) ? (nfr + fpc - 1) / fpc * fpc - nfr : 0;
    const size_t off_b0 = align_up(off_fo + (nfo + pad) * fb, 16);
    const size_t off_bh = align_up(off_b0 + (size_t)n_var * W * 4, 16);
    const size_t off_bo = align_up(off_bh + (size_t)(NHID - 1) * W * 4, 16);
    const size_t total = align_up(off_bo + (size_t)NO * 32 * 4, 16);
    std::vector<char> blob(total, 0);
    auto put = [&](size_t frag_off, size_t frag, int lane, int j, float v) {
        size_t e = (frag * 64 + lane) * KP + j;
        char* p = blob.data() + frag_off + e * esz;
        if (dt == DT_F32) {
            std::memcpy(p, &v, 4);
        } else {
            uint16_t h = bf16_bits(v);
            std::memcpy(p, &h, 2);
        }
    };
    auto hidden_in = [](int ri, int g) { return 32 * (ri / 16) + out_row(ri % 16, g); };
    // every fragment goes to its position in the consumption order (FragLayout,
    // or the pass-major order of the paired plan evaluation)
    const FragLayout lay{HT, IN_KS, HID_KS, CT, NHID};
    const int rp = pass_tiles;
    auto first_pos = [&](int c, int t) { return rp ? pass_first(IN_KS, rp, c, t) : lay.first(c, t); };
    auto hidden_pos = [&](int l, int c, int t) {
        return rp ? pass_hidden((int)nf0, (int)nfh, HID_KS, rp, l, c, t) : lay.hidden(l, c, t);
    };
    for (int c = 0; c < IN_KS; ++c)
        for (int t = 0; t < HT; ++t)
            for (int lane = 0; lane < 64; ++lane)
                for (int j = 0; j < KP; ++j) {
                    int col = map(c * KP + j, lane / 32);
                    put(off_f0, first_pos(c, t), lane, j, col >= 0 ? n.w(0, 32 * t + lane % 32, col) : 0.0f);
                }
    for (int l = 1; l <= NHID - 1; ++l)
        for (int c = 0; c < HID_KS; ++c)
            for (int t = 0; t < HT; ++t)
                for (int lane = 0; lane < 64; ++lane)
                    for (int j = 0; j < KP; ++j)
                        put(off_f0, hidden_pos(l, c, t), lane, j,
                            n.w(l, 32 * t + lane % 32, hidden_in(c * KP + j, lane / 32)));
    const int L = NHID;
    for (int t = 0; t < NO; ++t)
        for (int c = 0; c < HID_KS; ++c)
            for (int lane = 0; lane < 64; ++lane)
                for (int j = 0; j < KP; ++j) {
                    int f = 32 * t + row_feature(lane % 32);
                    put(off_f0, lay.out(t * HID_KS + c), lane, j,
                        f < n.out() ? n.w(L, f, hidden_in(c * KP + j, lane / 32)) : 0.0f);
                }
    std::memcpy(blob.data() + off_b0, b0_variants.data(), (size_t)n_var * W * 4);
    for (int l = 1; l <= NHID - 1; ++l) std::memcpy(blob.data() + off_bh + (size_t)(l - 1) * W * 4, n.b[l], (size_t)W * 4);
    std::vector<float> bo((size_t)NO * 32);
    for (int r = 0; r < NO * 32; ++r) {
        int f = 32 * (r / 32) + row_feature(r % 32);
        bo[r] = f < n.out() ? n.b[L][f] : 0.0f;
    }
    std::memcpy(blob.data() + off_bo, bo.data(), bo.size() * 4);
    nb.base = nullptr;
    nb.bytes = (uint32_t)total;
    nb.off_f0 = (uint32_t)off_f0;
    nb.off_fh = (uint32_t)off_fh;
    nb.off_fo = (uint32_t)off_fo;
    nb.off_b0 = (uint32_t)off_b0;
    nb.off_bh = (uint32_t)off_bh;
    nb.off_bo = (uint32_t)off_bo;
    nb.b0_stride = (uint32_t)W;
    return blob;
}

// The likelihood network for the contrastive objective's parameter
// derivative, as one fragment stream in the order the backward kernel
// consumes it: the first layer over the observation inputs (the state and
// action are folded into per-row biases), the hidden->hidden layers, then the
// transposed hidden->hidden layers from the last to the first (the products
// W_l^T delta_l of the reverse sweep), padded to whole stream chunks.
std::vector<char> pack_nce_wide(const HostNet& n, int dt, int in_slots_per_group, const SlotMap& map) {
    const int W = n.width(), HT = W / 32, NHID = n.n_layers - 1, KP = kper(dt);
    const int esz = dt == DT_F32 ? 4 : 2;
    const size_t fb = (size_t)64 * KP * esz;
    const int IN_KS = in_slots_per_group / KP, HID_KS = 16 * HT / KP;
    const size_t nf0 = (size_t)IN_KS * HT, nfh = (size_t)HID_KS * HT;
    const size_t nfr = nf0 + 2 * (size_t)(NHID - 1) * nfh;
    const size_t fpc = VOILA_STREAM_CHB / fb;
    std::vector<char> blob((nfr + fpc - 1) / fpc * fpc * fb, 0);
    auto put = [&](size_t frag, int lane, int j, float v) {
        char* p = blob.data() + ((frag * 64 + lane) * KP + j) * esz;
        if (dt == DT_F32) {
            std::memcpy(p, &v, 4);
        } else {
            uint16_t h = bf16_bits(v);
            std::memcpy(p, &h, 2);
        }
    };
    auto hidden_in = [](int ri, int g) { return 32 * (ri / 16) + out_row(ri % 16, g); };
    for (int c = 0; c < IN_KS; ++c)
        for (int t = 0; t < HT; ++t)
            for (int lane = 0; lane < 64; ++lane)
                for (int j = 0; j < KP; ++j) {
                    int col = map(c * KP + j, lane / 32);
                    put((size_t)c * HT + t, lane, j, col >= 0 ? n.w(0, 32 * t + lane % 32, col) : 0.0f);
                }
    for (int l = 1; l <= NHID - 1; ++l)
        for (int c = 0; c < HID_KS; ++c)
            for (int t = 0; t < HT; ++t)
                for (int lane = 0; lane < 64; ++lane)
                    for (int j = 0; j < KP; ++j)
                        put(nf0 + (size_t)(l - 1) * nfh + (size_t)c * HT + t, lane, j,
                            n.w(l, 32 * t + lane % 32, hidden_in(c * KP + j, lane / 32)));
    for (int k = 0; k < NHID - 1; ++k) {
        const int l = NHID - 1 - k;  // W_{l+1}^T maps the adjoint of h_{l+1} to h_l
        for (int c = 0; c < HID_KS; ++c)
            for (int t = 0; t < HT; ++t)
                for (int lane = 0; lane < 64; ++lane)
                    for (int j = 0; j < KP; ++j)
                        put(nf0 + (size_t)(NHID - 1 + k) * nfh + (size_t)c * HT + t, lane, j,
                            n.w(l, hidden_in(c * KP + j, lane / 32), 32 * t + lane % 32));
    }
    return blob;
}

// First-layer columns [c0, c0 + nf) of a network (rounded to bfloat16 for
// bfloat16 models), row-major [width][nf], for folding fixed inputs into the bias.
std::vector<float> fold_columns(const HostNet& n, int c0, int nf, int dt) {
    const int W = n.width();
    std::vector<float> out((size_t)W * nf);
    for (int o = 0; o < W; ++o)
        for (int c = 0; c < nf; ++c) {
            float v = n.w(0, o, c0 + c);
            out[(size_t)o * nf + c] = dt == DT_BF16 ? bf16_round(v) : v;
        }
    return out;
}

// Transposed weights of a two-hidden-layer network for the adjoint kernel, as
// f32 MFMA fragments [T3: ceil(d_out/2) x HT][T2: 16 HT x HT][T1: 16 HT]:
// T3 maps the output-layer adjoint (output feature 2 c + g in k-step c) to
// the second hidden layer, T2 the second hidden layer to the first (k-step c
// = feature 32 (c / 16) + out_row(c % 16, g)), T1 the first hidden layer to
// the input (row r of the tile = input feature row_feature(r)).
std::vector<char> pack_bwd(const HostNet& n, NetBlob& nb) {
    const int W = n.width(), HT = W / 32, d_out = n.out(), d_in = n.dims[0];
    const int KS3 = (d_out + 1) / 2;
    const size_t nfr = (size_t)KS3 * HT + (size_t)16 * HT * HT + 16 * HT;
    std::vector<char> blob(align_up(nfr * 256, 1024), 0);
    float* f = reinterpret_cast<float*>(blob.data());
    auto hidden_in = [](int ri, int g) { return 32 * (ri / 16) + out_row(ri % 16, g); };
    size_t fr = 0;
    for (int c = 0; c < KS3; ++c)
        for (int mt = 0; mt < HT; ++mt, ++fr)
            for (int lane = 0; lane < 64; ++lane) {
                int o = 2 * c + lane / 32;
                f[fr * 64 + lane] = o < d_out ? n.w(2, o, 32 * mt + lane % 32) : 0.0f;
            }
    for (int c = 0; c < 16 * HT; ++c)
        for (int mt = 0; mt < HT; ++mt, ++fr)
            for (int lane = 0; lane < 64; ++lane)
                f[fr * 64 + lane] = n.w(1, hidden_in(c, lane / 32), 32 * mt + lane % 32);
    for (int c = 0; c < 16 * HT; ++c, ++fr)
        for (int lane = 0; lane < 64; ++lane) {
            int fin = row_feature(lane % 32);
            f[fr * 64 + lane] = fin < d_in ? n.w(0, hidden_in(c, lane / 32), fin) : 0.0f;
        }
    nb = NetBlob{};
    nb.bytes = (uint32_t)blob.size();
    return blob;
}

struct DeviceGuard {
    int prev = -1;
    bool ok = true;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) ok = hipSetDevice(dev) == hipSuccess;
    }
    ~DeviceGuard() {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

}  // namespace

struct voila_model_s {
    int device = 0, shape = -1, dt = DT_F32, cus = 1;
    int d_s = 0, n_actions = 0, d_a = 0, d_w = 0, d_o = 0, d_wz = 0, width = 0, n_hidden = 0;
    bool has_obs = false, has_lik = false;
    // a likelihood network of its own shape (VOILA_LIK_SHAPES): hidden width
    // lik_width; such models update beliefs through the split proposal and
    // likelihood-rows kernels, and the other likelihood users refuse them
    bool lik_split = false;
    int lik_width = 0;
    int lik_bpc = 1;
    char* mem = nullptr;
    NetBlob trans_plan{}, trans_upd{}, obs{}, lik{}, lik_nce{};
    // the observation network for the rows of whole rollouts: in the paired
    // plan evaluation's pass-major order where that evaluation applies, else obs
    NetBlob obs_roll{};
    const float* fold_w_trans = nullptr;
    const float* fold_b_trans = nullptr;
    const float* fold_w_obs = nullptr;
    const float* fold_b_obs = nullptr;
    const float* fold_w_lik = nullptr;
    const float* fold_b_lik = nullptr;
    const float* fold_w_nce = nullptr;  // [width][a_width + d_s]: action columns, then state columns
    int nf_trans = 0, nf_obs = 0, nf_lik = 0;
    int plan_bpc = 1, prop_bpc = 1, obs_bpc = 1, obs_roll_bpc = 1, pw_bpc = 1, nce_bpc = 1;
    bool has_grad = false;
    NetBlob grad_fwd{}, grad_bwd{};
    int grad_bpc = 1, n_params = 0;
    bool has_nce_grad = false;       // parameter derivative of the contrastive objective compiled
    NetBlob lik_bwd{};               // transposed likelihood pack
    const float* lik_w3 = nullptr;   // [width] output-layer weights of the likelihood network
    int nce_grad_bpc = 1, n_lik_params = 0;
    // the same derivative for likelihood networks evaluated layer by layer
    bool has_nce_wide = false;
    const char* nce_wide_stream = nullptr;  // first layer, hidden layers, transposed hidden layers
    const float* nce_wide_bh = nullptr;     // [n_hidden - 1][width]
    const float* nce_wide_wout = nullptr;   // [width] (bfloat16 values for bfloat16 models)
    int nce_wide_bpc = 1, nce_wgrad_bpc = 1;
    int action_width() const { return n_actions > 0 ? n_actions : d_a; }
};

namespace {
constexpr const char* kLikSplitOnlyUpdate =
    "a likelihood network of another shape than the samplers' is used by the belief update only";
constexpr int kGradWaves = 4;
size_t grad_lds_bytes(const voila_model_s* m) {
    return (size_t)m->grad_fwd.bytes + m->grad_bwd.bytes + (size_t)kGradWaves * 32 * 129 * sizeof(float);
}
size_t nce_grad_lds_bytes(const voila_model_s* m) {
    return (size_t)m->lik_nce.bytes + m->lik_bwd.bytes + (size_t)kGradWaves * 32 * 129 * sizeof(float);
}
}  // namespace

extern "C" {

int32_t voila_version(void) { return 100; }

const char* voila_status_string(voila_status_t s) {
    switch (s) {
        case VOILA_OK: return "ok";
        case VOILA_ERR_INVALID_ARG: return "invalid argument";
        case VOILA_ERR_UNSUPPORTED: return "unsupported shape or size";
        case VOILA_ERR_WORKSPACE: return "workspace missing or too small";
        case VOILA_ERR_DEVICE: return "HIP runtime error";
        case VOILA_ERR_NUMERIC: return "non-finite likelihood or zero total weight";
        default: return "unknown status";
    }
}

const char* voila_last_error(void) { return g_last_error.c_str(); }

static voila_status_t read_net(const voila_mlp_desc_t& d, HostNet& n, const char* name) {
    n = HostNet();
    if (d.n_layers == 0) return VOILA_OK;
    if (d.n_layers < 2 || !d.h_dims || !d.h_W || !d.h_b)
        return fail(VOILA_ERR_INVALID_ARG, std::string(name) + ": needs >= 2 layers and non-NULL arrays");
    n.n_layers = d.n_layers;
    for (int l = 0; l <= d.n_layers; ++l) {
        if (d.h_dims[l] < 1) return fail(VOILA_ERR_INVALID_ARG, std::string(name) + ": non-positive width");
        n.dims.push_back(d.h_dims[l]);
    }
    for (int l = 0; l < d.n_layers; ++l) {
        if (!d.h_W[l] || !d.h_b[l]) return fail(VOILA_ERR_INVALID_ARG, std::string(name) + ": NULL layer array");
        n.W.push_back(d.h_W[l]);
        n.b.push_back(d.h_b[l]);
    }
    for (int l = 1; l < d.n_layers; ++l)
        if (n.dims[l] != n.dims[1]) return fail(VOILA_ERR_UNSUPPORTED, std::string(name) + ": hidden widths differ");
    return VOILA_OK;
}

voila_status_t voila_model_create(const voila_model_desc_t* desc, int32_t device, voila_model_t* out) {
    if (!desc || !out) return fail(VOILA_ERR_INVALID_ARG, "NULL descriptor or output handle");
    *out = nullptr;
    if (desc->compute != VOILA_F32 && desc->compute != VOILA_BF16)
        return fail(VOILA_ERR_INVALID_ARG, "compute must be VOILA_F32 or VOILA_BF16");
    HostNet T, Z, L;
    voila_status_t st;
    if ((st = read_net(desc->trans, T, "trans")) != VOILA_OK) return st;
    if ((st = read_net(desc->obs, Z, "obs")) != VOILA_OK) return st;
    if ((st = read_net(desc->lik, L, "lik")) != VOILA_OK) return st;
    if (!T.present()) return fail(VOILA_ERR_INVALID_ARG, "the transition network is required");
    const int aw = desc->n_actions > 0 ? desc->n_actions : desc->d_a;
    if (desc->d_s < 1 || desc->n_actions < 0 || desc->d_a < 0 || desc->d_w < 0 || desc->d_o < 0 || desc->d_wz < 0)
        return fail(VOILA_ERR_INVALID_ARG, "negative or zero dimension");
    if (T.dims[0] != desc->d_s + aw + desc->d_w || T.out() != desc->d_s)
        return fail(VOILA_ERR_INVALID_ARG, "trans dims must be [d_s + a_width + d_w, ..., d_s]");
    if (Z.present() && (Z.dims[0] != desc->d_s + aw + desc->d_wz || Z.out() != desc->d_o))
        return fail(VOILA_ERR_INVALID_ARG, "obs dims must be [d_s + a_width + d_wz, ..., d_o]");
    if (L.present() && (L.dims[0] != desc->d_s + aw + desc->d_o || L.out() != 1))
        return fail(VOILA_ERR_INVALID_ARG, "lik dims must be [d_s + a_width + d_o, ..., 1]");
    int shape = -1;
    for (int s = 0; s < kNumShapes; ++s) {
        const ShapeInfo& si = shape_info(s);
        bool ok = si.d_s == desc->d_s && si.n_actions == desc->n_actions &&
                  (desc->n_actions > 0 || si.d_a == desc->d_a) && si.d_w == desc->d_w &&
                  si.width == T.width() && si.n_hidden == T.n_layers - 1;
        if (Z.present()) ok = ok && si.d_wz == desc->d_wz && si.d_o == desc->d_o && Z.width() == si.width &&
                              Z.n_layers - 1 == si.n_hidden;
        const int lw = lik_shape_width(s) ? lik_shape_width(s) : si.width;
        const int lnh = lik_shape_hidden(s) ? lik_shape_hidden(s) : si.n_hidden;
        if (L.present()) ok = ok && si.d_o == desc->d_o && L.width() == lw && L.n_layers - 1 == lnh;
        if (ok) {
            shape = s;
            break;
        }
    }
    if (shape < 0) return fail(VOILA_ERR_UNSUPPORTED, "no compiled kernel for this network shape");
    if (plan_split_shape(shape, DT_BF16) && L.present() && !lik_shape_width(shape))
        return fail(VOILA_ERR_UNSUPPORTED,
                    "networks wider than 256 with more than two hidden layers: transition and observation "
                    "networks only (no likelihood network of the same shape)");
    if (T.width() > 256 && desc->compute != VOILA_BF16)
        return fail(VOILA_ERR_UNSUPPORTED, "hidden widths above 256 run in bfloat16 only");

    int ndev = 0;
    VOILA_CHECK_HIP(hipGetDeviceCount(&ndev));
    if (device < 0 || device >= ndev) return fail(VOILA_ERR_INVALID_ARG, "device index out of range");
    DeviceGuard guard(device);
    if (!guard.ok) return fail(VOILA_ERR_DEVICE, "hipSetDevice failed");

    voila_model_s* m = new voila_model_s();
    m->device = device;
    m->shape = shape;
    m->dt = desc->compute;
    m->d_s = desc->d_s;
    m->n_actions = desc->n_actions;
    m->d_a = desc->n_actions > 0 ? 0 : desc->d_a;
    m->d_w = desc->d_w;
    m->d_o = desc->d_o;
    m->d_wz = desc->d_wz;
    m->width = T.width();
    m->n_hidden = T.n_layers - 1;
    m->has_obs = Z.present();
    m->has_lik = L.present();
    m->lik_split = L.present() && lik_shape_width(shape) > 0;
    m->lik_width = L.present() ? L.width() : 0;
    const int dt = m->dt, W = m->width, LW = m->lik_width;

    // first-layer bias variants of the plan: one per discrete action (the
    // one-hot column folded in), or the plain bias for continuous actions
    std::vector<float> b0_plan;
    int n_var = 1;
    if (m->n_actions > 0) {
        n_var = m->n_actions;
        for (int a = 0; a < m->n_actions; ++a)
            for (int o = 0; o < W; ++o) {
                float wv = T.w(0, o, m->d_s + a);
                b0_plan.push_back(T.b[0][o] + (dt == DT_BF16 ? bf16_round(wv) : wv));
            }
    } else {
        b0_plan.assign(T.b[0], T.b[0] + W);
    }
    std::vector<float> b0_plain_T(T.b[0], T.b[0] + W);
    SlotMap map_plan{m->d_s, m->d_a, m->d_w, m->d_s, m->d_s + aw};
    SlotMap map_upd{m->d_s, 0, m->d_w, m->d_s, m->d_s + aw};
    std::vector<std::vector<char>> blobs;
    blobs.push_back(pack_net(T, dt, plan_in_slots(shape, dt), map_plan, b0_plan, n_var, m->trans_plan, false,
                             plan_pass_tiles(shape, dt)));
    blobs.push_back(pack_net(T, dt, update_in_slots(shape, dt), map_upd, b0_plain_T, 1, m->trans_upd));
    if (Z.present()) {
        std::vector<float> b0(Z.b[0], Z.b[0] + W);
        SlotMap mz{m->d_s, 0, m->d_wz, m->d_s, m->d_s + aw};
        blobs.push_back(pack_net(Z, dt, obs_in_slots(shape, dt), mz, b0, 1, m->obs));
    } else {
        blobs.emplace_back();
    }
    if (L.present()) {
        std::vector<float> b0(L.b[0], L.b[0] + LW);
        SlotMap ml{m->d_s, 0, 0, m->d_s, m->d_s};
        blobs.push_back(pack_net(L, dt, lik_in_slots(shape, dt), ml, b0, 1, m->lik));
    } else {
        blobs.emplace_back();
    }
    // adjoint packs (binary32 models of the shapes the adjoint kernel supports)
    m->has_grad = grad_supported(shape) && dt == DT_F32;
    if (m->has_grad) {
        SlotMap mg{m->d_s, aw, m->d_w, m->d_s, m->d_s + aw};
        blobs.push_back(pack_net(T, dt, in_slots(DT_F32, m->d_s, aw, m->d_w), mg, b0_plain_T, 1, m->grad_fwd));
        blobs.push_back(pack_bwd(T, m->grad_bwd));
        for (int l = 0; l < T.n_layers; ++l) m->n_params += T.dims[l + 1] * T.dims[l] + T.dims[l + 1];
    } else {
        blobs.emplace_back();
        blobs.emplace_back();
    }
    // the likelihood network with its first layer over the observation
    // columns (state and action folded per row) for the contrastive objective
    if (L.present() && !m->lik_split) {
        // pass-major where the scores kernel runs the paired evaluation (this
        // pack serves only that kernel there)
        std::vector<float> b0(L.b[0], L.b[0] + LW);
        SlotMap mo{m->d_o, 0, 0, 0, 0, m->d_s + aw};
        blobs.push_back(pack_net(L, dt, nce_in_slots(shape, dt), mo, b0, 1, m->lik_nce, false,
                                 plan_pass_tiles(shape, dt)));
    } else {
        blobs.emplace_back();
    }
    // transposed likelihood pack for the objective's parameter derivative
    m->has_nce_grad = L.present() && !m->lik_split && nce_grad_supported(shape) && dt == DT_F32;
    if (m->has_nce_grad) {
        blobs.push_back(pack_bwd(L, m->lik_bwd));
        for (int l = 0; l < L.n_layers; ++l) m->n_lik_params += L.dims[l + 1] * L.dims[l] + L.dims[l + 1];
    } else {
        blobs.emplace_back();
    }
    // the layered form of the same derivative (hidden width 256)
    m->has_nce_wide = L.present() && !m->lik_split && nce_wide_supported(shape);
    if (m->has_nce_wide) {
        SlotMap mo{m->d_o, 0, 0, 0, 0, m->d_s + aw};
        blobs.push_back(pack_nce_wide(L, dt, nce_in_slots(shape, dt), mo));
        if (m->n_lik_params == 0)
            for (int l = 0; l < L.n_layers; ++l) m->n_lik_params += L.dims[l + 1] * L.dims[l] + L.dims[l + 1];
    } else {
        blobs.emplace_back();
    }
    // the observation network in pass-major order for per-step observations
    const int obs_pt = Z.present() ? plan_pass_tiles(shape, dt) : 0;
    if (obs_pt) {
        std::vector<float> b0(Z.b[0], Z.b[0] + W);
        SlotMap mz{m->d_s, 0, m->d_wz, m->d_s, m->d_s + aw};
        blobs.push_back(pack_net(Z, dt, obs_in_slots(shape, dt), mz, b0, 1, m->obs_roll, false, obs_pt));
    } else {
        blobs.emplace_back();
    }
    const size_t nb = blobs.size();
    std::vector<std::vector<float>> folds;
    m->nf_trans = aw;
    folds.push_back(fold_columns(T, m->d_s, aw, dt));
    folds.push_back(b0_plain_T);
    if (Z.present()) {
        m->nf_obs = aw;
        folds.push_back(fold_columns(Z, m->d_s, aw, dt));
        folds.push_back(std::vector<float>(Z.b[0], Z.b[0] + W));
    } else {
        folds.emplace_back();
        folds.emplace_back();
    }
    if (L.present()) {
        m->nf_lik = aw + m->d_o;
        folds.push_back(fold_columns(L, m->d_s, aw + m->d_o, dt));
        folds.push_back(std::vector<float>(L.b[0], L.b[0] + LW));
        std::vector<float> fa = fold_columns(L, m->d_s, aw, dt), fs = fold_columns(L, 0, m->d_s, dt);
        std::vector<float> fn((size_t)LW * (aw + m->d_s));
        for (int o = 0; o < LW; ++o) {
            for (int c = 0; c < aw; ++c) fn[(size_t)o * (aw + m->d_s) + c] = fa[(size_t)o * aw + c];
            for (int c = 0; c < m->d_s; ++c) fn[(size_t)o * (aw + m->d_s) + aw + c] = fs[(size_t)o * m->d_s + c];
        }
        folds.push_back(fn);
        folds.push_back(std::vector<float>(L.W[L.n_layers - 1], L.W[L.n_layers - 1] + LW));
    } else {
        folds.emplace_back();
        folds.emplace_back();
        folds.emplace_back();
        folds.emplace_back();
    }
    if (m->has_nce_wide) {
        std::vector<float> bh;
        for (int l = 1; l < L.n_layers - 1; ++l) bh.insert(bh.end(), L.b[l], L.b[l] + W);
        folds.push_back(bh);
        std::vector<float> wo(L.W[L.n_layers - 1], L.W[L.n_layers - 1] + W);
        if (dt == DT_BF16)
            for (float& v : wo) v = bf16_round(v);
        folds.push_back(wo);
    } else {
        folds.emplace_back();
        folds.emplace_back();
    }
    size_t total = 0;
    std::vector<size_t> offs;
    for (auto& b : blobs) {
        offs.push_back(total);
        total = align_up(total + b.size(), 256);
    }
    for (auto& f : folds) {
        offs.push_back(total);
        total = align_up(total + f.size() * 4, 256);
    }
    if (hipMalloc(&m->mem, total) != hipSuccess) {
        delete m;
        return fail(VOILA_ERR_DEVICE, "hipMalloc of the packed model failed");
    }
    std::vector<char> host(total, 0);
    for (size_t i = 0; i < blobs.size(); ++i)
        if (!blobs[i].empty()) std::memcpy(host.data() + offs[i], blobs[i].data(), blobs[i].size());
    for (size_t i = 0; i < folds.size(); ++i)
        if (!folds[i].empty()) std::memcpy(host.data() + offs[blobs.size() + i], folds[i].data(), folds[i].size() * 4);
    if (hipMemcpy(m->mem, host.data(), total, hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipFree(m->mem);
        delete m;
        return fail(VOILA_ERR_DEVICE, "upload of the packed model failed");
    }
    m->trans_plan.base = m->mem + offs[0];
    m->trans_upd.base = m->mem + offs[1];
    m->obs.base = m->mem + offs[2];
    m->lik.base = m->mem + offs[3];
    m->grad_fwd.base = m->mem + offs[4];
    m->grad_bwd.base = m->mem + offs[5];
    m->lik_nce.base = m->mem + offs[6];
    m->lik_bwd.base = m->mem + offs[7];
    if (obs_pt) {
        m->obs_roll.base = m->mem + offs[9];
    } else {
        m->obs_roll = m->obs;
    }
    m->fold_w_trans = reinterpret_cast<const float*>(m->mem + offs[nb + 0]);
    m->fold_b_trans = reinterpret_cast<const float*>(m->mem + offs[nb + 1]);
    m->fold_w_obs = reinterpret_cast<const float*>(m->mem + offs[nb + 2]);
    m->fold_b_obs = reinterpret_cast<const float*>(m->mem + offs[nb + 3]);
    m->fold_w_lik = reinterpret_cast<const float*>(m->mem + offs[nb + 4]);
    m->fold_b_lik = reinterpret_cast<const float*>(m->mem + offs[nb + 5]);
    m->fold_w_nce = reinterpret_cast<const float*>(m->mem + offs[nb + 6]);
    m->lik_w3 = reinterpret_cast<const float*>(m->mem + offs[nb + 7]);
    if (m->has_nce_wide) {
        m->nce_wide_stream = m->mem + offs[8];
        m->nce_wide_bh = reinterpret_cast<const float*>(m->mem + offs[nb + 8]);
        m->nce_wide_wout = reinterpret_cast<const float*>(m->mem + offs[nb + 9]);
    }

    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) == hipSuccess) m->cus = prop.multiProcessorCount;
    m->plan_bpc = plan_blocks_per_cu(shape, dt);
    m->prop_bpc = m->lik_split ? propose_split_blocks_per_cu(shape, dt) : propose_blocks_per_cu(shape, dt);
    if (m->lik_split) m->lik_bpc = lik_rows_blocks_per_cu(shape, dt);
    m->obs_bpc = observe_blocks_per_cu(shape, dt);
    m->obs_roll_bpc = observe_rollout_blocks_per_cu(shape, dt);
    m->pw_bpc = pw_lik_blocks_per_cu(shape, dt);
    m->nce_bpc = nce_scores_blocks_per_cu(shape, dt);
    if (m->has_nce_grad) m->nce_grad_bpc = nce_grad_blocks_per_cu(shape, nce_grad_lds_bytes(m));
    if (m->has_nce_wide) {
        m->nce_wide_bpc = nce_wide_bwd_blocks_per_cu(dt);
        m->nce_wgrad_bpc = nce_wide_wgrad_blocks_per_cu(dt);
    }
    if (m->has_grad) m->grad_bpc = grad_blocks_per_cu(shape, grad_lds_bytes(m));
    *out = m;
    return VOILA_OK;
}

voila_status_t voila_model_destroy(voila_model_t m) {
    if (!m) return VOILA_OK;
    {
        DeviceGuard guard(m->device);
        if (m->mem) (void)hipFree(m->mem);
    }
    delete m;
    return VOILA_OK;
}

// ---------------------------------------------------------------------------
// plan
// ---------------------------------------------------------------------------
static size_t plan_ws(int N, int K) {
    const size_t n_tiles = ((size_t)N + 31) / 32;
    return align_up((size_t)K * n_tiles * sizeof(float), 256);
}

size_t voila_plan_workspace_size(voila_model_t model, int32_t N, int32_t K, int32_t H) {
    (void)model;
    (void)H;
    if (N < 1 || K < 0) return 0;
    return plan_ws(N, K);
}

voila_status_t voila_plan(voila_model_t m, const float* d_states, const double* d_belief_w, int32_t N,
                          const void* d_cands, int32_t K, int32_t H, const voila_plan_opts_t* o, void* ws,
                          size_t ws_bytes, float* d_q_out, float* d_returns_out, int32_t* d_status, void* stream) {
    if (!m) return fail(VOILA_ERR_INVALID_ARG, "NULL model");
    if (!o) return fail(VOILA_ERR_INVALID_ARG, "NULL options");
    if (N < 1) return fail(VOILA_ERR_INVALID_ARG, "N must be >= 1");
    if (K < 0 || H < 0) return fail(VOILA_ERR_INVALID_ARG, "K and H must be >= 0");
    if ((long long)K * N > (1LL << 31) - 1 || (long long)K * H > (1LL << 31) - 1)
        return fail(VOILA_ERR_UNSUPPORTED, "K * N and K * H must fit in 31 bits");
    if (!(o->gamma >= 0.0 && o->gamma <= 1.0)) return fail(VOILA_ERR_INVALID_ARG, "gamma must lie in [0, 1]");
    if (!o->h_goal) return fail(VOILA_ERR_INVALID_ARG, "NULL goal");
    if (o->reward_at != 0 && o->reward_at != 1) return fail(VOILA_ERR_INVALID_ARG, "reward_at must be 0 or 1");
    if (K == 0) return VOILA_OK;
    if (!d_states || !d_q_out || (!d_cands && H > 0)) return fail(VOILA_ERR_INVALID_ARG, "NULL device buffer");
    if (!ws || ws_bytes < plan_ws(N, K)) return fail(VOILA_ERR_WORKSPACE, "plan workspace too small");
    DeviceGuard guard(m->device);
    if (!guard.ok) return fail(VOILA_ERR_DEVICE, "hipSetDevice failed");
    const int n_tiles = (N + 31) / 32;
    PlanParams p{};
    p.net = m->trans_plan;
    p.states = d_states;
    p.belief_w = d_belief_w;
    p.cands = d_cands;
    p.noise = o->d_noise;
    p.returns = d_returns_out;
    p.traj = o->d_traj_out;
    p.partials = reinterpret_cast<float*>(ws);
    p.status = d_status;
    p.N = N;
    p.K = K;
    p.H = H;
    p.n_tiles = n_tiles;
    p.gamma = o->gamma;
    p.key0 = (uint32_t)(o->seed & 0xffffffffu);
    p.key1 = (uint32_t)(o->seed >> 32);
    p.crn = o->crn ? 1 : 0;
    p.reward_at = o->reward_at;
    for (int j = 0; j < 64; ++j) p.goal[j] = j < m->d_s ? o->h_goal[j] : 0.0f;
    // units: (candidate, tile), or (candidate, group of tiles) for the paired
    // and the split evaluations
    const int tpu = plan_tiles_per_unit(m->shape, m->dt), upb = plan_units_per_block(m->shape, m->dt);
    const long units = (long)K * ((n_tiles + tpu - 1) / tpu);
    const long want = (units + upb - 1) / upb;
    const long cap = (long)m->cus * m->plan_bpc;
    const int blocks = (int)(want < cap ? want : cap);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    VOILA_CHECK_HIP(launch_plan(m->shape, m->dt, p, blocks, s));
    QReduceParams q{};
    q.partials = p.partials;
    q.q = d_q_out;
    q.K = K;
    q.n_tiles = n_tiles;
    q.scale = d_belief_w ? 1.0f : (float)(1.0 / (double)N);
    VOILA_CHECK_HIP(launch_q_reduce(q, s));
    return VOILA_OK;
}

// ---------------------------------------------------------------------------
// update
// ---------------------------------------------------------------------------
int32_t voila_update_max_particles(void) { return kLargeMaxN; }

size_t voila_weights_workspace_size(int32_t N) {
    if (N <= kNormResMaxN) return 0;
    if (N > kLargeMaxN) return 0;
    return large_res_workspace_bytes(N);
}

int32_t voila_resample_bits(int32_t N) {
    if (N < 1) return 0;
    int c = 0;
    while ((1LL << c) < (long long)N) ++c;
    return 52 - c < 32 ? 52 - c : 32;
}

namespace {
struct UpdateWs {
    float* b0_trans;
    float* b0_lik;
    double* x;
    float* prop;
    char* large;   // multi-workgroup resampling workspace (N > 8192)
    size_t bytes;
};
UpdateWs carve_update(char* base, int width, int N, int d_s) {
    UpdateWs w{};
    size_t off = 0;
    w.b0_trans = reinterpret_cast<float*>(base + off);
    off = align_up(off + (size_t)width * 4, 256);
    w.b0_lik = reinterpret_cast<float*>(base + off);
    off = align_up(off + (size_t)width * 4, 256);
    w.x = reinterpret_cast<double*>(base + off);
    off = align_up(off + (size_t)N * 8, 256);
    w.prop = reinterpret_cast<float*>(base + off);
    off = align_up(off + (size_t)N * d_s * 4, 256);
    w.large = base + off;
    if (N > kNormResMaxN) off = align_up(off + large_res_workspace_bytes(N), 256);
    w.bytes = off;
    return w;
}

// First-layer bias of one network with the executed action (and, for the
// likelihood, the observation) read from device memory and folded in, so the
// fold follows whatever those buffers hold when the stream reaches it.
FoldStepsParams fold_one(voila_model_t m, const float* w, const float* b, int nf, const void* d_action,
                         const float* d_obs, float* out, int32_t* d_status, int width = 0) {
    FoldStepsParams f{};
    f.w = w;
    f.b = b;
    f.out = out;
    f.cands = d_action;
    f.obs = d_obs;
    f.width = width ? width : m->width;
    f.nf = nf;
    f.rows = 1;
    f.n_actions = m->n_actions;
    f.d_a = m->d_a;
    f.d_o = d_obs ? m->d_o : 0;
    f.bf16 = m->dt == DT_BF16 ? 1 : 0;
    f.status = d_status;
    return f;
}
}  // namespace

size_t voila_update_workspace_size(voila_model_t m, int32_t N) {
    if (!m || N < 1) return 0;
    return carve_update(nullptr, m->width, N, m->d_s).bytes;
}

voila_status_t voila_update(voila_model_t m, const float* d_states, const double* d_prior_w, int32_t N,
                            const void* d_action, const float* d_obs, const voila_update_opts_t* o, void* ws,
                            size_t ws_bytes, float* d_states_out, int32_t* d_idx_out, double* d_w_out,
                            float* d_loglik_out, float* d_prop_out, double* d_stats_out, int32_t* d_status,
                            void* stream) {
    if (!m) return fail(VOILA_ERR_INVALID_ARG, "NULL model");
    if (!m->has_lik) return fail(VOILA_ERR_INVALID_ARG, "the model has no likelihood network");
    if (!o || !d_action || !d_obs) return fail(VOILA_ERR_INVALID_ARG, "NULL options, action or observation");
    if (N < 1) return fail(VOILA_ERR_INVALID_ARG, "N must be >= 1");
    if (N > kLargeMaxN) return fail(VOILA_ERR_UNSUPPORTED, "N above voila_update_max_particles()");
    if (!(o->lambda > 0.0) || !std::isfinite(o->lambda)) return fail(VOILA_ERR_INVALID_ARG, "lambda must be > 0");
    if (!d_states || !d_states_out) return fail(VOILA_ERR_INVALID_ARG, "NULL device buffer");
    UpdateWs w = carve_update(reinterpret_cast<char*>(ws), m->width, N, m->d_s);
    if (!ws || ws_bytes < w.bytes) return fail(VOILA_ERR_WORKSPACE, "update workspace too small");
    DeviceGuard guard(m->device);
    if (!guard.ok) return fail(VOILA_ERR_DEVICE, "hipSetDevice failed");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    VOILA_CHECK_HIP(launch_fold_steps(
        fold_one(m, m->fold_w_trans, m->fold_b_trans, m->nf_trans, d_action, nullptr, w.b0_trans, d_status), s));
    VOILA_CHECK_HIP(launch_fold_steps(
        fold_one(m, m->fold_w_lik, m->fold_b_lik, m->nf_lik, d_action, d_obs, w.b0_lik, d_status, m->lik_width),
        s));
    ProposeParams p{};
    p.trans = m->trans_upd;
    p.lik = m->lik;
    p.b0_trans = w.b0_trans;
    p.b0_lik = w.b0_lik;
    p.states = d_states;
    p.prior_w = d_prior_w;
    p.noise = o->d_noise;
    p.prop = d_prop_out ? d_prop_out : w.prop;
    p.loglik = d_loglik_out;
    p.x = w.x;
    p.status = d_status;
    p.N = N;
    p.lambda = o->lambda;
    p.key0 = (uint32_t)(o->seed & 0xffffffffu);
    p.key1 = (uint32_t)(o->seed >> 32);
    const int n_tiles = (N + 31) / 32;
    if (m->lik_split) {
        const int want = (n_tiles + kPropSplitTiles - 1) / kPropSplitTiles, cap = m->cus * m->prop_bpc;
        VOILA_CHECK_HIP(launch_propose_split(m->shape, m->dt, p, want < cap ? want : cap, s));
        const int lcap = m->cus * m->lik_bpc;
        VOILA_CHECK_HIP(launch_lik_rows(m->shape, m->dt, p, n_tiles < lcap ? n_tiles : lcap, s));
    } else {
        const int tpb = pass_tiles_per_block(m->shape);
        const int want = (n_tiles + tpb - 1) / tpb;
        const int cap = m->cus * m->prop_bpc;
        VOILA_CHECK_HIP(launch_propose(m->shape, m->dt, p, want < cap ? want : cap, s));
    }
    if (N > kNormResMaxN) {
        LargeResParams r{};
        r.x = w.x;
        r.lambda = o->lambda;
        r.N = N;
        r.bits = voila_resample_bits(N);
        r.uniform_prior = d_prior_w ? 0 : 1;
        r.do_resample = 1;
        r.U = o->resample_u;
        r.w_out = d_w_out;
        r.stats = d_stats_out;
        r.idx_out = d_idx_out;
        r.src = p.prop;
        r.dst = d_states_out;
        r.row_floats = m->d_s;
        r.status = d_status;
        r.ws = carve_large_res(w.large, N);
        VOILA_CHECK_HIP(launch_large_res(r, s));
        return VOILA_OK;
    }
    NormResParams r{};
    r.x = w.x;
    r.N = N;
    r.bits = voila_resample_bits(N);
    r.uniform_prior = d_prior_w ? 0 : 1;
    r.do_resample = 1;
    r.U = o->resample_u;
    r.lambda = o->lambda;
    r.w_out = d_w_out;
    r.stats = d_stats_out;
    r.idx_out = d_idx_out;
    r.src = p.prop;
    r.dst = d_states_out;
    r.row_floats = m->d_s;
    r.status = d_status;
    VOILA_CHECK_HIP(launch_norm_res(r, s));
    return VOILA_OK;
}

// ---------------------------------------------------------------------------
// update without allocation: the workspace is a fixed device array
// ---------------------------------------------------------------------------
namespace {
constexpr size_t kUpdateScratchBytes = VOILA_UPDATE_NOALLOC_SCRATCH_BYTES;
// The workspace of voila_update_noalloc, one copy per device (loaded with the
// library's code object).  In host code this name only identifies the array
// for hipGetSymbolAddress; it is never a device address.
__device__ __align__(256) char scratch[kUpdateScratchBytes];
constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxScratchDevices] = {};

// Device address of the current device's copy of `scratch`, looked up once
// per device (the caller has made `device` current).
voila_status_t scratch_address(int device, void** out) {
    if (device < 0 || device >= kMaxScratchDevices) return fail(VOILA_ERR_UNSUPPORTED, "device index above 63");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail(VOILA_ERR_DEVICE, std::string("hipGetSymbolAddress of the update scratch: ") +
                                              hipGetErrorString(e));
        g_scratch_ptr[device] = ptr;
    }
    *out = g_scratch_ptr[device];
    return VOILA_OK;
}
}  // namespace

voila_status_t voila_update_noalloc(voila_model_t m, const float* d_states, const double* d_prior_w, int32_t N,
                                    const void* d_action, const float* d_obs, const voila_update_opts_t* o,
                                    float* d_states_out, int32_t* d_idx_out, double* d_w_out, float* d_loglik_out,
                                    float* d_prop_out, double* d_stats_out, int32_t* d_status, void* stream) {
    if (!m) return fail(VOILA_ERR_INVALID_ARG, "NULL model");
    if (N < 1) return fail(VOILA_ERR_INVALID_ARG, "N must be >= 1");
    const size_t need = voila_update_workspace_size(m, N);
    if (need > kUpdateScratchBytes)
        return fail(VOILA_ERR_UNSUPPORTED, "N = " + std::to_string(N) + " needs " + std::to_string(need) +
                                               " bytes of workspace; the fixed scratch of voila_update_noalloc "
                                               "holds " + std::to_string(kUpdateScratchBytes));
    DeviceGuard guard(m->device);
    if (!guard.ok) return fail(VOILA_ERR_DEVICE, "hipSetDevice failed");
    void* ws = nullptr;
    const voila_status_t st = scratch_address(m->device, &ws);
    if (st != VOILA_OK) return st;
    // every part of the workspace is written before it is read within the
    // call, so nothing needs clearing between calls
    return voila_update(m, d_states, d_prior_w, N, d_action, d_obs, o, ws, kUpdateScratchBytes, d_states_out,
                        d_idx_out, d_w_out, d_loglik_out, d_prop_out, d_stats_out, d_status, stream);
}

voila_status_t voila_normalize(const float* d_loglik, const double* d_prior_w, int32_t N, double lambda,
                               double* d_w_out, double* d_stats_out, int32_t* d_status, void* ws, size_t ws_bytes,
                               void* stream) {
    if (N < 1) return fail(VOILA_ERR_INVALID_ARG, "N must be >= 1");
    if (N > kLargeMaxN) return fail(VOILA_ERR_UNSUPPORTED, "N above voila_update_max_particles()");
    if (!(lambda > 0.0) || !std::isfinite(lambda)) return fail(VOILA_ERR_INVALID_ARG, "lambda must be > 0");
    if (!d_loglik || !d_w_out) return fail(VOILA_ERR_INVALID_ARG, "NULL device buffer");
    if (N > kNormResMaxN) {
        if (!ws || ws_bytes < voila_weights_workspace_size(N)) return fail(VOILA_ERR_WORKSPACE, "workspace too small");
        LargeResParams r{};
        r.loglik = d_loglik;
        r.prior_w = d_prior_w;
        r.lambda = lambda;
        r.N = N;
        r.bits = voila_resample_bits(N);
        r.uniform_prior = d_prior_w ? 0 : 1;
        r.w_out = d_w_out;
        r.stats = d_stats_out;
        r.status = d_status;
        r.ws = carve_large_res(ws, N);
        VOILA_CHECK_HIP(launch_large_res(r, reinterpret_cast<hipStream_t>(stream)));
        return VOILA_OK;
    }
    NormResParams r{};
    r.loglik = d_loglik;
    r.prior_w = d_prior_w;
    r.lambda = lambda;
    r.N = N;
    r.bits = voila_resample_bits(N);
    r.uniform_prior = d_prior_w ? 0 : 1;
    r.do_resample = 0;
    r.w_out = d_w_out;
    r.stats = d_stats_out;
    r.status = d_status;
    VOILA_CHECK_HIP(launch_norm_res(r, reinterpret_cast<hipStream_t>(stream)));
    return VOILA_OK;
}

voila_status_t voila_resample(const double* d_w, int32_t N, uint32_t U, int32_t* d_idx_out, const float* d_src,
                              float* d_dst, int32_t row_floats, int32_t* d_status, void* ws, size_t ws_bytes,
                              void* stream) {
    if (N < 1) return fail(VOILA_ERR_INVALID_ARG, "N must be >= 1");
    if (N > kLargeMaxN) return fail(VOILA_ERR_UNSUPPORTED, "N above voila_update_max_particles()");
    if (!d_w || !d_idx_out) return fail(VOILA_ERR_INVALID_ARG, "NULL device buffer");
    if ((d_src != nullptr) != (d_dst != nullptr)) return fail(VOILA_ERR_INVALID_ARG, "give both or neither of src and dst");
    if (d_src && row_floats < 1) return fail(VOILA_ERR_INVALID_ARG, "row_floats must be >= 1");
    if (N > kNormResMaxN) {
        if (!ws || ws_bytes < voila_weights_workspace_size(N)) return fail(VOILA_ERR_WORKSPACE, "workspace too small");
        LargeResParams r{};
        r.w_in = d_w;
        r.N = N;
        r.bits = voila_resample_bits(N);
        r.do_resample = 1;
        r.U = U;
        r.idx_out = d_idx_out;
        r.src = d_src;
        r.dst = d_dst;
        r.row_floats = row_floats;
        r.status = d_status;
        r.ws = carve_large_res(ws, N);
        VOILA_CHECK_HIP(launch_large_res(r, reinterpret_cast<hipStream_t>(stream)));
        return VOILA_OK;
    }
    NormResParams r{};
    r.w_in = d_w;
    r.N = N;
    r.bits = voila_resample_bits(N);
    r.do_resample = 1;
    r.U = U;
    r.idx_out = d_idx_out;
    r.src = d_src;
    r.dst = d_dst;
    r.row_floats = row_floats;
    r.status = d_status;
    VOILA_CHECK_HIP(launch_norm_res(r, reinterpret_cast<hipStream_t>(stream)));
    return VOILA_OK;
}

voila_status_t voila_reweight_resample(const float* d_loglik, const double* d_prior_w, int32_t N, double lambda,
                                       uint32_t U, int32_t* d_idx_out, double* d_w_out, double* d_stats_out,
                                       const float* d_src, float* d_dst, int32_t row_floats, int32_t* d_status,
                                       void* ws, size_t ws_bytes, void* stream) {
    if (N < 1) return fail(VOILA_ERR_INVALID_ARG, "N must be >= 1");
    if (N > kLargeMaxN) return fail(VOILA_ERR_UNSUPPORTED, "N above voila_update_max_particles()");
    if (!(lambda > 0.0) || !std::isfinite(lambda)) return fail(VOILA_ERR_INVALID_ARG, "lambda must be > 0");
    if (!d_loglik || !d_idx_out) return fail(VOILA_ERR_INVALID_ARG, "NULL device buffer");
    if ((d_src != nullptr) != (d_dst != nullptr)) return fail(VOILA_ERR_INVALID_ARG, "give both or neither of src and dst");
    if (d_src && row_floats < 1) return fail(VOILA_ERR_INVALID_ARG, "row_floats must be >= 1");
    if (N > kNormResMaxN) {
        if (!ws || ws_bytes < voila_weights_workspace_size(N)) return fail(VOILA_ERR_WORKSPACE, "workspace too small");
        LargeResParams r{};
        r.loglik = d_loglik;
        r.prior_w = d_prior_w;
        r.lambda = lambda;
        r.N = N;
        r.bits = voila_resample_bits(N);
        r.uniform_prior = d_prior_w ? 0 : 1;
        r.do_resample = 1;
        r.U = U;
        r.w_out = d_w_out;
        r.stats = d_stats_out;
        r.idx_out = d_idx_out;
        r.src = d_src;
        r.dst = d_dst;
        r.row_floats = row_floats;
        r.status = d_status;
        r.ws = carve_large_res(ws, N);
        VOILA_CHECK_HIP(launch_large_res(r, reinterpret_cast<hipStream_t>(stream)));
        return VOILA_OK;
    }
    NormResParams r{};
    r.loglik = d_loglik;
    r.prior_w = d_prior_w;
    r.lambda = lambda;
    r.N = N;
    r.bits = voila_resample_bits(N);
    r.uniform_prior = d_prior_w ? 0 : 1;
    r.do_resample = 1;
    r.U = U;
    r.w_out = d_w_out;
    r.stats = d_stats_out;
    r.idx_out = d_idx_out;
    r.src = d_src;
    r.dst = d_dst;
    r.row_floats = row_floats;
    r.status = d_status;
    VOILA_CHECK_HIP(launch_norm_res(r, reinterpret_cast<hipStream_t>(stream)));
    return VOILA_OK;
}

namespace {
// Blocks of an observe launch over `tiles` 32-row tiles: enough to cover
// them, at most the resident blocks of the whole chip.
int observe_blocks(voila_model_t m, long tiles) {
    const long tpb = pass_tiles_per_block(m->shape);
    const long want = (tiles + tpb - 1) / tpb;
    const long cap = (long)m->cus * m->obs_bpc;
    return (int)(want < cap ? want : cap);
}
}  // namespace

size_t voila_observe_workspace_size(voila_model_t m) {
    if (!m) return 0;
    return align_up((size_t)m->width * 4, 256);
}

voila_status_t voila_observe(voila_model_t m, const float* d_states, int32_t n, const void* d_action, uint64_t seed,
                             const float* d_noise, void* ws, size_t ws_bytes, float* d_obs_out, int32_t* d_status,
                             void* stream) {
    if (!m) return fail(VOILA_ERR_INVALID_ARG, "NULL model");
    if (!m->has_obs) return fail(VOILA_ERR_INVALID_ARG, "the model has no observation network");
    if (n < 0) return fail(VOILA_ERR_INVALID_ARG, "n must be >= 0");
    if (!d_action) return fail(VOILA_ERR_INVALID_ARG, "NULL action");
    if (n == 0) return VOILA_OK;
    if (!d_states || !d_obs_out) return fail(VOILA_ERR_INVALID_ARG, "NULL device buffer");
    if (!ws || ws_bytes < voila_observe_workspace_size(m)) return fail(VOILA_ERR_WORKSPACE, "observe workspace too small");
    DeviceGuard guard(m->device);
    if (!guard.ok) return fail(VOILA_ERR_DEVICE, "hipSetDevice failed");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const FoldStepsParams f = fold_one(m, m->fold_w_obs, m->fold_b_obs, m->nf_obs, d_action, nullptr,
                                       reinterpret_cast<float*>(ws), d_status);
    VOILA_CHECK_HIP(launch_fold_steps(f, s));
    ObserveParams p{};
    p.obs = m->obs;
    p.b0 = f.out;
    p.b0_stride = 0;
    p.states = d_states;
    p.noise = d_noise;
    p.out = d_obs_out;
    p.N = n;
    p.K = 1;
    p.H = 1;
    p.key0 = (uint32_t)(seed & 0xffffffffu);
    p.key1 = (uint32_t)(seed >> 32);
    VOILA_CHECK_HIP(launch_observe(m->shape, m->dt, p, observe_blocks(m, (n + 31) / 32), s));
    return VOILA_OK;
}

namespace {
struct PwWs {
    float* first;
    float* b0_obs;
    float* o_new;
    float* o_sel;
    float* b0_lik;
    int32_t* tiles;
    double* x;
    size_t bytes;
};
PwWs carve_pw(char* base, voila_model_t m, int T, int M) {
    PwWs w{};
    size_t off = 0;
    auto take = [&](size_t bytes) {
        char* p = base + off;
        off = align_up(off + bytes, 256);
        return p;
    };
    w.first = reinterpret_cast<float*>(take((size_t)M * m->d_s * 4));
    w.b0_obs = reinterpret_cast<float*>(take((size_t)M * m->width * 4));
    w.o_new = reinterpret_cast<float*>(take((size_t)M * m->d_o * 4));
    w.o_sel = reinterpret_cast<float*>(take((size_t)M * m->d_o * 4));
    w.b0_lik = reinterpret_cast<float*>(take((size_t)M * m->width * 4));
    w.tiles = reinterpret_cast<int32_t*>(take(((size_t)M + 1) * 4));
    w.x = reinterpret_cast<double*>(take((size_t)T * 8));
    w.bytes = off;
    return w;
}
}  // namespace

size_t voila_pw_step_workspace_size(voila_model_t m, int32_t T, int32_t M) {
    if (!m || T < 0 || M < 0) return 0;
    return carve_pw(nullptr, m, T, M).bytes;
}

voila_status_t voila_pw_step(voila_model_t m, const float* d_succ, int32_t T, const int32_t* d_seg, int32_t M,
                             const void* d_actions, const int32_t* d_visits, int32_t* d_children,
                             float* d_obs_table, const uint32_t* d_U, const voila_pw_opts_t* o, void* ws,
                             size_t ws_bytes, int32_t* d_widen_out, int32_t* d_branch_out, float* d_loglik_out,
                             double* d_w_out, double* d_stats_out, int32_t* d_idx_out, float* d_succ_out,
                             int32_t* d_status, void* stream) {
    if (!m) return fail(VOILA_ERR_INVALID_ARG, "NULL model");
    if (!m->has_obs || !m->has_lik) return fail(VOILA_ERR_INVALID_ARG, "the model needs observation and likelihood networks");
    if (m->lik_split) return fail(VOILA_ERR_UNSUPPORTED, kLikSplitOnlyUpdate);
    if (!o) return fail(VOILA_ERR_INVALID_ARG, "NULL options");
    if (T < 0 || M < 0) return fail(VOILA_ERR_INVALID_ARG, "T and M must be >= 0");
    if (o->capacity < 1) return fail(VOILA_ERR_INVALID_ARG, "capacity must be >= 1");
    if (!(o->k_o > 0.0) || !(o->alpha_o > 0.0) || !std::isfinite(o->k_o) || !std::isfinite(o->alpha_o))
        return fail(VOILA_ERR_INVALID_ARG, "k_o and alpha_o must be finite and > 0");
    if (!(o->lambda > 0.0) || !std::isfinite(o->lambda)) return fail(VOILA_ERR_INVALID_ARG, "lambda must be > 0");
    if ((long long)M * o->capacity * m->d_o > (1LL << 31) - 1)
        return fail(VOILA_ERR_UNSUPPORTED, "M * capacity * d_o must fit in 31 bits");
    if (M == 0) return VOILA_OK;
    if (!d_seg || !d_actions || !d_visits || !d_children || !d_obs_table || !d_U || (T > 0 && !d_succ))
        return fail(VOILA_ERR_INVALID_ARG, "NULL device buffer");
    PwWs w = carve_pw(reinterpret_cast<char*>(ws), m, T, M);
    if (!ws || ws_bytes < w.bytes) return fail(VOILA_ERR_WORKSPACE, "progressive-widening workspace too small");
    DeviceGuard guard(m->device);
    if (!guard.ok) return fail(VOILA_ERR_DEVICE, "hipSetDevice failed");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    PwParams p{};
    p.lik = m->lik;
    p.succ = d_succ;
    p.seg = d_seg;
    p.actions = d_actions;
    p.visits = d_visits;
    p.children = d_children;
    p.table = d_obs_table;
    p.U = d_U;
    p.first = w.first;
    p.o_new = w.o_new;
    p.o_sel = w.o_sel;
    p.b0_lik = w.b0_lik;
    p.tiles = w.tiles;
    p.x = w.x;
    p.widen = d_widen_out;
    p.branch = d_branch_out;
    p.loglik = d_loglik_out;
    p.w = d_w_out;
    p.stats = d_stats_out;
    p.idx = d_idx_out;
    p.succ_out = d_succ_out;
    p.status = d_status;
    p.T = T;
    p.M = M;
    p.B = o->capacity;
    p.d_s = m->d_s;
    p.d_o = m->d_o;
    p.k_o = o->k_o;
    p.alpha_o = o->alpha_o;
    p.lambda = o->lambda;
    p.key0 = (uint32_t)(o->seed & 0xffffffffu);
    p.key1 = (uint32_t)(o->seed >> 32);
    // 1. an observation drawn at each group's first successor (used by the groups that widen)
    VOILA_CHECK_HIP(launch_pw_first(p, s));
    FoldStepsParams fo{};
    fo.w = m->fold_w_obs;
    fo.b = m->fold_b_obs;
    fo.out = w.b0_obs;
    fo.cands = d_actions;
    fo.width = m->width;
    fo.nf = m->nf_obs;
    fo.rows = M;
    fo.n_actions = m->n_actions;
    fo.d_a = m->d_a;
    fo.bf16 = m->dt == DT_BF16 ? 1 : 0;
    fo.status = d_status;
    VOILA_CHECK_HIP(launch_fold_steps(fo, s));
    ObserveParams op{};
    op.obs = m->obs;
    op.b0 = w.b0_obs;
    op.b0_stride = m->width;
    op.states = w.first;
    op.out = w.o_new;
    op.N = 1;
    op.K = M;
    op.H = 1;
    op.key0 = p.key0;
    op.key1 = p.key1;
    VOILA_CHECK_HIP(launch_observe(m->shape, m->dt, op, observe_blocks(m, M), s));
    // 2. widening test, branch choice, table update
    VOILA_CHECK_HIP(launch_pw_branch(p, s));
    // 3. likelihood of every successor against its group's branch observation
    FoldStepsParams fl = fo;
    fl.w = m->fold_w_lik;
    fl.b = m->fold_b_lik;
    fl.out = w.b0_lik;
    fl.nf = m->nf_lik;
    fl.obs = w.o_sel;
    fl.d_o = m->d_o;
    VOILA_CHECK_HIP(launch_fold_steps(fl, s));
    VOILA_CHECK_HIP(launch_pw_tiles(p, s));
    const long units = (long)T / 32 + M;
    const long want = (units + kWavesPerBlock - 1) / kWavesPerBlock;
    const long cap = (long)m->cus * m->pw_bpc;
    VOILA_CHECK_HIP(launch_pw_lik(m->shape, m->dt, p, (int)(want < cap ? want : cap), s));
    // 4. per-group weights and systematic resampling
    VOILA_CHECK_HIP(launch_pw_norm_res(p, M < m->cus ? M : m->cus, s));
    return VOILA_OK;
}

namespace {
struct NceWs {
    float* b0;
    float* scores;
    double* row_loss;
    size_t bytes;
};
NceWs carve_nce(char* base, voila_model_t m, int B) {
    NceWs w{};
    size_t off = 0;
    auto take = [&](size_t bytes) {
        char* p = base + off;
        off = align_up(off + bytes, 256);
        return p;
    };
    w.b0 = reinterpret_cast<float*>(take((size_t)B * m->width * 4));
    w.scores = reinterpret_cast<float*>(take((size_t)B * B * 4));
    w.row_loss = reinterpret_cast<double*>(take((size_t)B * 8));
    w.bytes = off;
    return w;
}
}  // namespace

size_t voila_info_nce_workspace_size(voila_model_t m, int32_t B) {
    if (!m || B < 1 || B > kNceMaxBatch) return 0;
    return carve_nce(nullptr, m, B).bytes;
}

voila_status_t voila_info_nce(voila_model_t m, const float* d_states, const void* d_actions, const float* d_obs,
                              int32_t B, void* ws, size_t ws_bytes, float* d_scores_out, double* d_row_loss_out,
                              float* d_grad_out, double* d_loss_out, int32_t* d_status, void* stream) {
    if (!m) return fail(VOILA_ERR_INVALID_ARG, "NULL model");
    if (!m->has_lik) return fail(VOILA_ERR_INVALID_ARG, "the model has no likelihood network");
    if (m->lik_split) return fail(VOILA_ERR_UNSUPPORTED, kLikSplitOnlyUpdate);
    if (B < 1) return fail(VOILA_ERR_INVALID_ARG, "B must be >= 1");
    if (B > kNceMaxBatch) return fail(VOILA_ERR_UNSUPPORTED, "B must be <= 32768");
    if (!d_states || !d_actions || !d_obs) return fail(VOILA_ERR_INVALID_ARG, "NULL device buffer");
    NceWs w = carve_nce(reinterpret_cast<char*>(ws), m, B);
    if (!ws || ws_bytes < w.bytes) return fail(VOILA_ERR_WORKSPACE, "contrastive-objective workspace too small");
    DeviceGuard guard(m->device);
    if (!guard.ok) return fail(VOILA_ERR_DEVICE, "hipSetDevice failed");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    // 1. row i's state and action folded into its first-layer bias row
    FoldStepsParams f{};
    f.w = m->fold_w_nce;
    f.b = m->fold_b_lik;
    f.out = w.b0;
    f.cands = d_actions;
    f.obs = d_states;
    f.width = m->width;
    f.nf = m->action_width() + m->d_s;
    f.rows = B;
    f.n_actions = m->n_actions;
    f.d_a = m->d_a;
    f.d_o = m->d_s;
    f.bf16 = m->dt == DT_BF16 ? 1 : 0;
    f.status = d_status;
    VOILA_CHECK_HIP(launch_fold_steps(f, s));
    // 2. scores of all pairs, 3. per-row losses and derivatives, 4. the mean
    NceParams p{};
    p.lik = m->lik_nce;
    p.obs = d_obs;
    p.b0 = w.b0;
    p.scores = d_scores_out ? d_scores_out : w.scores;
    p.row_loss = d_row_loss_out ? d_row_loss_out : w.row_loss;
    p.grad = d_grad_out;
    p.loss = d_loss_out;
    p.status = d_status;
    p.B = B;
    p.d_o = m->d_o;
    const int tpu = plan_pass_tiles(m->shape, m->dt) ? 2 : 1;  // column tiles per wave unit (paired evaluation)
    const long units = (long)B * (((B + 31) / 32 + tpu - 1) / tpu);
    const long want = (units + kWavesPerBlock - 1) / kWavesPerBlock;
    const long cap = (long)m->cus * m->nce_bpc;
    VOILA_CHECK_HIP(launch_nce_scores(m->shape, m->dt, p, (int)(want < cap ? want : cap), s));
    VOILA_CHECK_HIP(launch_nce_rows(p, B < 8 * m->cus ? B : 8 * m->cus, s));
    VOILA_CHECK_HIP(launch_nce_mean(p, s));
    return VOILA_OK;
}

struct voila_denoiser_s {
    int device = 0, shape = -1, dt = DT_F32, cus = 1, bpc = 1;
    int d_c = 0, d_x = 0, n_actions = 0, d_a = 0, width = 0;
    char* mem = nullptr;
    NetBlob net{};
    const float* fold_w = nullptr;  // [width][a_width + 1]
    const float* fold_b = nullptr;  // [width]
    int action_width() const { return n_actions > 0 ? n_actions : d_a; }
};

voila_status_t voila_denoiser_create(const voila_mlp_desc_t* net, int32_t d_c, int32_t d_x, int32_t n_actions,
                                     int32_t d_a, int32_t compute, int32_t device, voila_denoiser_t* out) {
    if (!net || !out) return fail(VOILA_ERR_INVALID_ARG, "NULL descriptor or output handle");
    *out = nullptr;
    if (compute != VOILA_F32 && compute != VOILA_BF16)
        return fail(VOILA_ERR_INVALID_ARG, "compute must be VOILA_F32 or VOILA_BF16");
    if (d_c < 1 || d_x < 1 || n_actions < 0 || d_a < 0 || (n_actions == 0 && d_a < 1))
        return fail(VOILA_ERR_INVALID_ARG, "bad conditioning, sample or action dimension");
    const int aw = n_actions > 0 ? n_actions : d_a;
    if (aw > 63) return fail(VOILA_ERR_UNSUPPORTED, "at most 63 action inputs");
    HostNet D;
    voila_status_t st;
    if ((st = read_net(*net, D, "denoiser")) != VOILA_OK) return st;
    if (!D.present()) return fail(VOILA_ERR_INVALID_ARG, "the denoiser network is required");
    if (D.dims[0] != d_c + aw + d_x + 1 || D.out() != d_x)
        return fail(VOILA_ERR_INVALID_ARG, "denoiser dims must be [d_c + a_width + d_x + 1, ..., d_x]");
    const int shape = ddim_shape(d_x, d_c, D.width(), D.n_layers - 1);
    if (shape < 0) return fail(VOILA_ERR_UNSUPPORTED, "no compiled sampler kernel for this denoiser shape");
    if (D.width() > 256 && compute != VOILA_BF16)
        return fail(VOILA_ERR_UNSUPPORTED, "hidden widths above 256 run in bfloat16 only");
    int ndev = 0;
    VOILA_CHECK_HIP(hipGetDeviceCount(&ndev));
    if (device < 0 || device >= ndev) return fail(VOILA_ERR_INVALID_ARG, "device index out of range");
    DeviceGuard guard(device);
    if (!guard.ok) return fail(VOILA_ERR_DEVICE, "hipSetDevice failed");
    voila_denoiser_s* m = new voila_denoiser_s();
    m->device = device;
    m->shape = shape;
    m->dt = compute;
    m->d_c = d_c;
    m->d_x = d_x;
    m->n_actions = n_actions;
    m->d_a = n_actions > 0 ? 0 : d_a;
    m->width = D.width();
    const int W = m->width, dt = m->dt;
    // input [c, a, x_tau, tau]: x_tau in the state slots, c in the noise slots
    SlotMap map{d_x, 0, d_c, d_c, 0, d_c + aw};
    std::vector<float> b0(D.b[0], D.b[0] + W);
    std::vector<char> blob = pack_net(D, dt, ddim_in_slots(shape, dt), map, b0, 1, m->net, ddim_split(shape));
    std::vector<float> fa = fold_columns(D, d_c, aw, dt), ft = fold_columns(D, d_c + aw + d_x, 1, dt);
    std::vector<float> fw((size_t)W * (aw + 1));
    for (int o = 0; o < W; ++o) {
        for (int c = 0; c < aw; ++c) fw[(size_t)o * (aw + 1) + c] = fa[(size_t)o * aw + c];
        fw[(size_t)o * (aw + 1) + aw] = ft[o];
    }
    const size_t off_w = align_up(blob.size(), 256), off_b = align_up(off_w + fw.size() * 4, 256);
    const size_t total = align_up(off_b + (size_t)W * 4, 256);
    std::vector<char> host(total, 0);
    std::memcpy(host.data(), blob.data(), blob.size());
    std::memcpy(host.data() + off_w, fw.data(), fw.size() * 4);
    std::memcpy(host.data() + off_b, D.b[0], (size_t)W * 4);
    if (hipMalloc(&m->mem, total) != hipSuccess) {
        delete m;
        return fail(VOILA_ERR_DEVICE, "hipMalloc of the packed denoiser failed");
    }
    if (hipMemcpy(m->mem, host.data(), total, hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipFree(m->mem);
        delete m;
        return fail(VOILA_ERR_DEVICE, "upload of the packed denoiser failed");
    }
    m->net.base = m->mem;
    m->fold_w = reinterpret_cast<const float*>(m->mem + off_w);
    m->fold_b = reinterpret_cast<const float*>(m->mem + off_b);
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) == hipSuccess) m->cus = prop.multiProcessorCount;
    m->bpc = ddim_blocks_per_cu(shape, dt);
    *out = m;
    return VOILA_OK;
}

voila_status_t voila_denoiser_destroy(voila_denoiser_t m) {
    if (!m) return VOILA_OK;
    DeviceGuard guard(m->device);
    if (m->mem) (void)hipFree(m->mem);
    delete m;
    return VOILA_OK;
}

size_t voila_ddim_workspace_size(voila_denoiser_t m, int32_t n_steps) {
    if (!m || n_steps < 1 || n_steps > kDdimMaxSteps) return 0;
    return align_up((size_t)n_steps * m->width * 4, 256) + align_up((size_t)n_steps * 2 * 4, 256);
}

voila_status_t voila_ddim_sample(voila_denoiser_t m, const float* d_states, const void* h_action, const float* d_x1,
                                 int32_t N, int32_t n_steps, void* ws, size_t ws_bytes, float* d_out, void* stream) {
    if (!m) return fail(VOILA_ERR_INVALID_ARG, "NULL denoiser");
    if (N < 0) return fail(VOILA_ERR_INVALID_ARG, "N must be >= 0");
    if (n_steps < 1 || n_steps > kDdimMaxSteps) return fail(VOILA_ERR_INVALID_ARG, "n_steps must be in [1, 4096]");
    if (!h_action) return fail(VOILA_ERR_INVALID_ARG, "NULL action");
    DdimPrepParams pp{};
    if (m->n_actions > 0) {
        const int a = *reinterpret_cast<const int32_t*>(h_action);
        if (a < 0 || a >= m->n_actions) return fail(VOILA_ERR_INVALID_ARG, "action index out of range");
        for (int j = 0; j < m->n_actions; ++j) pp.v[j] = j == a ? 1.0f : 0.0f;
    } else {
        const float* a = reinterpret_cast<const float*>(h_action);
        for (int j = 0; j < m->d_a; ++j) {
            if (!std::isfinite(a[j])) return fail(VOILA_ERR_INVALID_ARG, "non-finite action");
            pp.v[j] = m->dt == DT_BF16 ? bf16_round(a[j]) : a[j];
        }
    }
    if (N == 0) return VOILA_OK;
    if (!d_states || !d_x1 || !d_out) return fail(VOILA_ERR_INVALID_ARG, "NULL device buffer");
    const size_t need = voila_ddim_workspace_size(m, n_steps);
    if (!ws || ws_bytes < need) return fail(VOILA_ERR_WORKSPACE, "sampler workspace too small");
    DeviceGuard guard(m->device);
    if (!guard.ok) return fail(VOILA_ERR_DEVICE, "hipSetDevice failed");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    char* base = reinterpret_cast<char*>(ws);
    pp.w = m->fold_w;
    pp.b = m->fold_b;
    pp.b0 = reinterpret_cast<float*>(base);
    pp.coef = reinterpret_cast<float*>(base + align_up((size_t)n_steps * m->width * 4, 256));
    pp.width = m->width;
    pp.aw = m->action_width();
    pp.n_steps = n_steps;
    pp.bf16 = m->dt == DT_BF16 ? 1 : 0;
    VOILA_CHECK_HIP(launch_ddim_prep(pp, s));
    DdimParams p{};
    p.net = m->net;
    p.states = d_states;
    p.x1 = d_x1;
    p.b0 = pp.b0;
    p.coef = pp.coef;
    p.out = d_out;
    p.N = N;
    p.n_steps = n_steps;
    const long tiles = ((long)N + 31) / 32;
    const long tpb = ddim_tiles_per_block(m->shape);
    const long want = (tiles + tpb - 1) / tpb;
    const long cap = (long)m->cus * m->bpc;
    VOILA_CHECK_HIP(launch_ddim(m->shape, m->dt, p, (int)(want < cap ? want : cap), s));
    return VOILA_OK;
}

int32_t voila_info_nce_param_count(voila_model_t m) {
    return m && (m->has_nce_grad || m->has_nce_wide) ? m->n_lik_params : 0;
}

namespace {
struct NceGradWs {
    char* nce;
    size_t nce_bytes;
    float* G;
    float* wpart;
    int blocks;
    // layered networks: activation arrays of one chunk of units, per-workgroup partials
    void* act;
    long uc;
    size_t bytes;
};
// Units (32 pairs each) held by one chunk of the layered derivative's arrays
// at most, and the array bytes per unit.
long nce_wide_unit_cap(const voila_model_s* m) { return m->dt == DT_F32 ? (1L << 14) : (1L << 15); }
size_t nce_wide_unit_bytes(const voila_model_s* m) {
    return (2 * (size_t)m->n_hidden - 1) * m->width * 32 * (m->dt == DT_F32 ? 4 : 2);
}
// uc = 0: as many units per chunk as the workspace of ws_bytes holds (the
// default workspace holds min(all units, the cap)).
NceGradWs carve_nce_grad(char* base, voila_model_t m, int B, size_t ws_bytes = 0) {
    NceGradWs w{};
    w.nce = base;
    w.nce_bytes = voila_info_nce_workspace_size(m, B);
    size_t off = align_up(w.nce_bytes, 256);
    w.G = reinterpret_cast<float*>(base + off);
    off = align_up(off + (size_t)B * B * 4, 256);
    const long units = (long)B * ((B + 31) / 32);
    if (m->has_nce_wide) {
        w.blocks = m->cus * m->nce_wgrad_bpc;
    } else {
        const long want = (units + kGradWaves - 1) / kGradWaves;
        const long cap = (long)m->cus * m->nce_grad_bpc;
        w.blocks = (int)(want < cap ? want : cap) * kGradWaves;
    }
    w.wpart = reinterpret_cast<float*>(base + off);
    off = align_up(off + (size_t)w.blocks * m->n_lik_params * 4, 256);
    if (m->has_nce_wide) {
        long uc = units < nce_wide_unit_cap(m) ? units : nce_wide_unit_cap(m);
        if (ws_bytes > off) {
            const long fit = (long)((ws_bytes - off) / nce_wide_unit_bytes(m));
            uc = fit < uc ? fit : uc;
        }
        w.uc = uc < 1 ? 1 : uc;
        w.act = base + off;
        off = align_up(off + (size_t)w.uc * nce_wide_unit_bytes(m), 256);
    }
    w.bytes = off;
    return w;
}
}  // namespace

size_t voila_info_nce_grad_workspace_size(voila_model_t m, int32_t B) {
    if (!m || !(m->has_nce_grad || m->has_nce_wide) || B < 1 || B > kNceMaxBatch) return 0;
    return carve_nce_grad(nullptr, m, B).bytes;
}

voila_status_t voila_info_nce_grad(voila_model_t m, const float* d_states, const void* d_actions, const float* d_obs,
                                   int32_t B, void* ws, size_t ws_bytes, double* d_loss_out, float* d_param_grad_out,
                                   int32_t* d_status, void* stream) {
    if (!m) return fail(VOILA_ERR_INVALID_ARG, "NULL model");
    if (!m->has_nce_grad && !m->has_nce_wide)
        return fail(VOILA_ERR_UNSUPPORTED,
                    "the parameter derivative is compiled for binary32 width-64 likelihood networks of the small "
                    "shapes and for the width-256 likelihood network");
    if (B < 1) return fail(VOILA_ERR_INVALID_ARG, "B must be >= 1");
    if (B > kNceMaxBatch) return fail(VOILA_ERR_UNSUPPORTED, "B must be <= 32768");
    if (!d_states || !d_actions || !d_obs || !d_param_grad_out) return fail(VOILA_ERR_INVALID_ARG, "NULL device buffer");
    NceGradWs w = carve_nce_grad(reinterpret_cast<char*>(ws), m, B, ws_bytes);
    if (!ws || ws_bytes < w.bytes) return fail(VOILA_ERR_WORKSPACE, "contrastive-gradient workspace too small");
    voila_status_t st = voila_info_nce(m, d_states, d_actions, d_obs, B, w.nce, w.nce_bytes, nullptr, nullptr, w.G,
                                       d_loss_out, d_status, stream);
    if (st != VOILA_OK) return st;
    DeviceGuard guard(m->device);
    if (!guard.ok) return fail(VOILA_ERR_DEVICE, "hipSetDevice failed");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    NceWs nw = carve_nce(reinterpret_cast<char*>(w.nce), m, B);
    if (m->has_nce_wide) {
        // chunks of units: forward and reverse sweep of every pair, then the
        // split-K products into per-workgroup partial sums
        const long units = (long)B * ((B + 31) / 32);
        const int upc = m->dt == DT_F32 ? 1 : 2;  // units per staged chunk of the product kernel
        for (long u0 = 0; u0 < units; u0 += w.uc) {
            const long u1 = u0 + w.uc < units ? u0 + w.uc : units;
            NceWideParams a{};
            a.stream = m->nce_wide_stream;
            a.bh = m->nce_wide_bh;
            a.w_out = m->nce_wide_wout;
            a.b0 = nw.b0;
            a.obs = d_obs;
            a.grad = w.G;
            a.act = w.act;
            a.uc = w.uc;
            a.u0 = u0;
            a.u1 = u1;
            a.B = B;
            const long want = (u1 - u0 + 3) / 4;
            const long cap = (long)m->cus * m->nce_wide_bpc;
            VOILA_CHECK_HIP(launch_nce_wide_bwd(m->shape, m->dt, a, (int)(want < cap ? want : cap), s));
            NceWgradParams b{};
            b.act = w.act;
            b.uc = w.uc;
            b.u0 = u0;
            b.n_units = u1 - u0;
            const long per = (b.n_units + w.blocks - 1) / w.blocks;
            b.per_split = (per + upc - 1) / upc * upc;
            b.grad = w.G;
            b.w_out = m->nce_wide_wout;
            b.states = d_states;
            b.actions = d_actions;
            b.obs = d_obs;
            b.B = B;
            b.n_actions = m->n_actions;
            b.d_a = m->d_a;
            b.d_s = m->d_s;
            b.d_o = m->d_o;
            b.d_in = m->d_s + m->action_width() + m->d_o;
            b.part = w.wpart;
            b.n_params = m->n_lik_params;
            b.accumulate = u0 > 0 ? 1 : 0;
            VOILA_CHECK_HIP(launch_nce_wide_wgrad(m->shape, m->dt, b, w.blocks, s));
        }
        GradReduceParams r{};
        r.wpart = w.wpart;
        r.grad_params = d_param_grad_out;
        r.n_params = m->n_lik_params;
        r.n_waves = w.blocks;
        VOILA_CHECK_HIP(launch_grad_reduce(r, s));
        return VOILA_OK;
    }
    NceGradParams p{};
    p.fwd = m->lik_nce;
    p.bwd = m->lik_bwd;
    p.w3 = m->lik_w3;
    p.b0 = nw.b0;
    p.obs = d_obs;
    p.states = d_states;
    p.actions = d_actions;
    p.grad = w.G;
    p.wpart = w.wpart;
    p.status = d_status;
    p.B = B;
    p.n_params = m->n_lik_params;
    VOILA_CHECK_HIP(launch_nce_grad(m->shape, p, w.blocks / kGradWaves, nce_grad_lds_bytes(m), s));
    GradReduceParams r{};
    r.wpart = w.wpart;
    r.grad_params = d_param_grad_out;
    r.n_params = m->n_lik_params;
    r.n_waves = w.blocks;
    VOILA_CHECK_HIP(launch_grad_reduce(r, s));
    return VOILA_OK;
}

voila_status_t voila_soft_value(const float* d_Q, const double* d_log_pi0, int32_t M, int32_t K, double eta,
                                double* d_V_out, double* d_pi_out, int32_t* d_best_out, int32_t* d_status,
                                void* stream) {
    if (M < 0 || K < 1) return fail(VOILA_ERR_INVALID_ARG, "M must be >= 0 and K >= 1");
    if (!(eta > 0.0) || !std::isfinite(eta)) return fail(VOILA_ERR_INVALID_ARG, "eta must be finite and > 0");
    if ((long long)M * K > (1LL << 31) - 1) return fail(VOILA_ERR_UNSUPPORTED, "M * K must fit in 31 bits");
    if (M == 0) return VOILA_OK;
    if (!d_Q || !d_V_out) return fail(VOILA_ERR_INVALID_ARG, "NULL device buffer");
    SoftValueParams p{};
    p.Q = d_Q;
    p.log_pi0 = d_log_pi0;
    p.V = d_V_out;
    p.pi = d_pi_out;
    p.best = d_best_out;
    p.status = d_status;
    p.M = M;
    p.K = K;
    p.eta = eta;
    VOILA_CHECK_HIP(launch_soft_value(p, M < 4096 ? M : 4096, reinterpret_cast<hipStream_t>(stream)));
    return VOILA_OK;
}

namespace {
struct TreeWs {
    char* plan1;
    float* succ0;
    float* q1;
    float* succ;
    int32_t* seg;
    char* acts;
    int32_t* zeros;
    float* table;
    char* pw;
    float* child;
    char* plan2;
    float* q2;
    float* G2;
    double* Qc;
    double* Vc;
    size_t bytes;
};
TreeWs carve_tree(char* base, voila_model_t m, int N, int A, int n_obs, int K) {
    TreeWs w{};
    size_t off = 0;
    auto take = [&](size_t bytes) {
        char* p = base + off;
        off = align_up(off + bytes, 256);
        return p;
    };
    const size_t M = (size_t)A * n_obs, T = M * N;
    w.plan1 = take(plan_ws(N, A));
    w.succ0 = reinterpret_cast<float*>(take((size_t)A * N * m->d_s * 4));
    w.q1 = reinterpret_cast<float*>(take((size_t)A * 4));
    w.succ = reinterpret_cast<float*>(take(T * m->d_s * 4));
    w.seg = reinterpret_cast<int32_t*>(take((M + 1) * 4));
    w.acts = take(M * (m->n_actions > 0 ? 4 : (size_t)m->d_a * 4));
    w.zeros = reinterpret_cast<int32_t*>(take(2 * M * 4));
    w.table = reinterpret_cast<float*>(take(M * m->d_o * 4));
    w.pw = take(voila_pw_step_workspace_size(m, (int)T, (int)M));
    w.child = reinterpret_cast<float*>(take(T * m->d_s * 4));
    w.plan2 = take(plan_ws((int)T, K));
    w.q2 = reinterpret_cast<float*>(take((size_t)K * 4));
    w.G2 = reinterpret_cast<float*>(take((size_t)K * T * 4));
    w.Qc = reinterpret_cast<double*>(take(M * K * 8));
    w.Vc = reinterpret_cast<double*>(take(M * 8));
    w.bytes = off;
    return w;
}
bool tree_sizes_ok(int N, int A, int n_obs, int K, int H) {
    if (N < 1 || A < 1 || n_obs < 1 || K < 1 || H < 0) return false;
    const long long T = (long long)A * n_obs * N;
    return T <= (1LL << 31) - 1 && (long long)K * T <= (1LL << 31) - 1 && (long long)A * N <= (1LL << 31) - 1;
}
}  // namespace

size_t voila_plan_closed_loop_workspace_size(voila_model_t m, int32_t N, int32_t A, int32_t n_obs, int32_t K,
                                             int32_t H) {
    if (!m || !tree_sizes_ok(N, A, n_obs, K, H)) return 0;
    return carve_tree(nullptr, m, N, A, n_obs, K).bytes;
}

voila_status_t voila_plan_closed_loop(voila_model_t m, const float* d_states, int32_t N, const void* d_first,
                                      int32_t A, const void* d_cont, int32_t K, int32_t H,
                                      const voila_closed_loop_opts_t* o, void* ws, size_t ws_bytes,
                                      double* d_psi_out, double* d_V_out, double* d_pi_out, int32_t* d_best_out,
                                      double* d_R_out, double* d_Vchild_out, float* d_child_out, int32_t* d_status,
                                      void* stream) {
    if (!m) return fail(VOILA_ERR_INVALID_ARG, "NULL model");
    if (!m->has_obs || !m->has_lik) return fail(VOILA_ERR_INVALID_ARG, "the model needs observation and likelihood networks");
    if (m->lik_split) return fail(VOILA_ERR_UNSUPPORTED, kLikSplitOnlyUpdate);
    if (!o || !o->h_goal) return fail(VOILA_ERR_INVALID_ARG, "NULL options or goal");
    if (!tree_sizes_ok(N, A, o->n_obs, K, H))
        return fail(VOILA_ERR_INVALID_ARG, "N, A, n_obs, K >= 1, H >= 0, and the branch and rollout counts must fit in 31 bits");
    if (N > kPwMaxGroup) return fail(VOILA_ERR_UNSUPPORTED, "N above 8192 (one workgroup resamples a branch)");
    if (!(o->gamma >= 0.0 && o->gamma <= 1.0)) return fail(VOILA_ERR_INVALID_ARG, "gamma must lie in [0, 1]");
    if (!(o->eta > 0.0) || !std::isfinite(o->eta)) return fail(VOILA_ERR_INVALID_ARG, "eta must be finite and > 0");
    if (!(o->lambda > 0.0) || !std::isfinite(o->lambda)) return fail(VOILA_ERR_INVALID_ARG, "lambda must be > 0");
    if (!d_states || !d_first || (!d_cont && H > 0) || !o->d_U || !d_psi_out || !d_V_out)
        return fail(VOILA_ERR_INVALID_ARG, "NULL device buffer");
    TreeWs w = carve_tree(reinterpret_cast<char*>(ws), m, N, A, o->n_obs, K);
    if (!ws || ws_bytes < w.bytes) return fail(VOILA_ERR_WORKSPACE, "closed-loop workspace too small");
    DeviceGuard guard(m->device);
    if (!guard.ok) return fail(VOILA_ERR_DEVICE, "hipSetDevice failed");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const int M = A * o->n_obs, T = M * N;
    voila_status_t st;
    // 1. one step from every particle under each first action: successors and R(b, a)
    voila_plan_opts_t p1{};
    p1.gamma = 1.0;
    p1.h_goal = o->h_goal;
    p1.seed = o->seed;
    p1.d_traj_out = w.succ0;
    if ((st = voila_plan(m, d_states, nullptr, N, d_first, A, 1, &p1, w.plan1, plan_ws(N, A), w.q1, nullptr,
                         d_status, stream)) != VOILA_OK)
        return st;
    // 2. the observation branches and their child beliefs
    TreeParams tp{};
    tp.succ0 = w.succ0;
    tp.succ = w.succ;
    tp.seg = w.seg;
    tp.first = d_first;
    tp.acts = w.acts;
    tp.zeros = w.zeros;
    tp.A = A;
    tp.n_obs = o->n_obs;
    tp.N = N;
    tp.K = K;
    tp.d_s = m->d_s;
    tp.n_actions = m->n_actions;
    tp.d_a = m->d_a;
    tp.gamma = o->gamma;
    tp.eta = o->eta;
    VOILA_CHECK_HIP(launch_tree_groups(tp, s));
    float* child = d_child_out ? d_child_out : w.child;
    voila_pw_opts_t po{};
    po.k_o = 1.0;
    po.alpha_o = 1.0;
    po.lambda = o->lambda;
    po.seed = o->seed;
    po.capacity = 1;
    if ((st = voila_pw_step(m, w.succ, T, w.seg, M, w.acts, w.zeros, w.zeros + M, w.table, o->d_U, &po, w.pw,
                            voila_pw_step_workspace_size(m, T, M), nullptr, nullptr, nullptr, nullptr, nullptr,
                            nullptr, child, d_status, stream)) != VOILA_OK)
        return st;
    // 3. child values from the continuation candidates (rollout key seed + 1)
    voila_plan_opts_t p2{};
    p2.gamma = o->gamma;
    p2.h_goal = o->h_goal;
    p2.seed = o->seed + 1;
    if ((st = voila_plan(m, child, nullptr, T, d_cont, K, H, &p2, w.plan2, plan_ws(T, K), w.q2, w.G2, d_status,
                         stream)) != VOILA_OK)
        return st;
    tp.G2 = w.G2;
    tp.Qc = w.Qc;
    VOILA_CHECK_HIP(launch_tree_child_q(tp, s));
    double* Vc = d_Vchild_out ? d_Vchild_out : w.Vc;
    SoftValueParams sv{};
    sv.Qd = w.Qc;
    sv.V = Vc;
    sv.status = d_status;
    sv.M = M;
    sv.K = K;
    sv.eta = o->eta;
    VOILA_CHECK_HIP(launch_soft_value(sv, M < 4096 ? M : 4096, s));
    // 4. backup and the root's soft value
    tp.Vc = Vc;
    tp.R = w.q1;
    tp.log_pi0 = o->d_log_pi0;
    tp.psi = d_psi_out;
    tp.R_out = d_R_out;
    VOILA_CHECK_HIP(launch_tree_backup(tp, s));
    SoftValueParams sr{};
    sr.Qd = d_psi_out;
    sr.no_prior = 1;
    sr.V = d_V_out;
    sr.pi = d_pi_out;
    sr.best = d_best_out;
    sr.status = d_status;
    sr.M = 1;
    sr.K = A;
    sr.eta = o->eta;
    VOILA_CHECK_HIP(launch_soft_value(sr, 1, s));
    return VOILA_OK;
}

size_t voila_plan_observe_workspace_size(voila_model_t m, int32_t K, int32_t H) {
    if (!m || K < 0 || H < 0) return 0;
    return align_up((size_t)K * H * m->width * 4, 256);
}

voila_status_t voila_plan_observe(voila_model_t m, const float* d_traj, int32_t N, const void* d_cands, int32_t K,
                                  int32_t H, uint64_t seed, int32_t crn, const float* d_noise, void* ws,
                                  size_t ws_bytes, float* d_obs_out, int32_t* d_status, void* stream) {
    if (!m) return fail(VOILA_ERR_INVALID_ARG, "NULL model");
    if (!m->has_obs) return fail(VOILA_ERR_INVALID_ARG, "the model has no observation network");
    if (N < 1) return fail(VOILA_ERR_INVALID_ARG, "N must be >= 1");
    if (K < 0 || H < 0) return fail(VOILA_ERR_INVALID_ARG, "K and H must be >= 0");
    if ((long long)K * N > (1LL << 31) - 1 || (long long)K * H > (1LL << 31) - 1)
        return fail(VOILA_ERR_UNSUPPORTED, "K * N and K * H must fit in 31 bits");
    if ((long long)K * H * ((N + 31) / 32) > (1LL << 31) - 1)
        return fail(VOILA_ERR_UNSUPPORTED, "K * H * ceil(N / 32) must fit in 31 bits");
    if (K == 0 || H == 0) return VOILA_OK;
    if (!d_traj || !d_cands || !d_obs_out) return fail(VOILA_ERR_INVALID_ARG, "NULL device buffer");
    if (!ws || ws_bytes < voila_plan_observe_workspace_size(m, K, H))
        return fail(VOILA_ERR_WORKSPACE, "plan-observe workspace too small");
    DeviceGuard guard(m->device);
    if (!guard.ok) return fail(VOILA_ERR_DEVICE, "hipSetDevice failed");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    FoldStepsParams f{};
    f.w = m->fold_w_obs;
    f.b = m->fold_b_obs;
    f.out = reinterpret_cast<float*>(ws);
    f.cands = d_cands;
    f.width = m->width;
    f.nf = m->nf_obs;
    f.rows = K * H;
    f.n_actions = m->n_actions;
    f.d_a = m->d_a;
    f.bf16 = m->dt == DT_BF16 ? 1 : 0;
    f.status = d_status;
    VOILA_CHECK_HIP(launch_fold_steps(f, s));
    ObserveParams p{};
    p.obs = m->obs_roll;
    p.b0 = f.out;
    p.b0_stride = m->width;
    p.states = d_traj;
    p.noise = d_noise;
    p.out = d_obs_out;
    p.N = N;
    p.K = K;
    p.H = H;
    p.crn = crn ? 1 : 0;
    p.key0 = (uint32_t)(seed & 0xffffffffu);
    p.key1 = (uint32_t)(seed >> 32);
    const int tpu = plan_pass_tiles(m->shape, m->dt) ? 2 : 1;  // tiles per wave unit (paired evaluation)
    const long units = (long)K * H * (((N + 31) / 32 + tpu - 1) / tpu);
    const long want = (units + kWavesPerBlock - 1) / kWavesPerBlock;
    const long cap = (long)m->cus * m->obs_roll_bpc;
    VOILA_CHECK_HIP(launch_observe_rollouts(m->shape, m->dt, p, (int)(want < cap ? want : cap), s));
    return VOILA_OK;
}

voila_status_t voila_philox_normals(uint64_t seed, uint32_t c0_base, uint32_t c1, uint32_t c2, uint32_t stream_id,
                                    int32_t n, int32_t d, float* d_out, uint32_t* d_words, void* stream) {
    if (n < 0 || d < 1) return fail(VOILA_ERR_INVALID_ARG, "n must be >= 0 and d >= 1");
    if (stream_id > 0xffffu) return fail(VOILA_ERR_INVALID_ARG, "stream id must fit in 16 bits");
    if (n > 0 && !d_out) return fail(VOILA_ERR_INVALID_ARG, "NULL output");
    PhiloxParams p{};
    p.out = d_out;
    p.words = d_words;
    p.n = n;
    p.d = d;
    p.key0 = (uint32_t)(seed & 0xffffffffu);
    p.key1 = (uint32_t)(seed >> 32);
    p.c0 = c0_base;
    p.c1 = c1;
    p.c2 = c2;
    p.stream = stream_id;
    VOILA_CHECK_HIP(launch_philox(p, reinterpret_cast<hipStream_t>(stream)));
    return VOILA_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// batches
// ---------------------------------------------------------------------------
struct voila_batch_s {
    int device = 0, shape = 0, dt = 0, n = 0, cus = 1, wpb = 4, dynamic = 1;
    bool has_update = false;
    char* mem = nullptr;
    PlanParams* d_plan = nullptr;
    QReduceParams* d_qr = nullptr;
    ProposeParams* d_prop = nullptr;
    FoldBatchItem* d_fold = nullptr;
    NormResParams* d_nr = nullptr;
    int4* d_plan_items = nullptr;
    int4* d_prop_items = nullptr;
    int* d_counters = nullptr;
    int n_plan_items = 0, n_prop_items = 0, max_k = 0, width = 0;
    size_t plan_lds = 0, prop_lds = 0;
    int plan_blocks = 1, prop_blocks = 1;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace {

// Work items of `count` units split into pieces of at most `wpb`: (instance, first, units, cost).
void add_items(std::vector<int4>& out, int inst, long units, int wpb, int cost_per_unit) {
    for (long u0 = 0; u0 < units; u0 += wpb) {
        int c = (int)std::min<long>(wpb, units - u0);
        out.push_back(make_int4(inst, (int)u0, c, cost_per_unit * c));
    }
}

}  // namespace

extern "C" {

voila_status_t voila_batch_create(const voila_batch_item_t* items, int32_t n, const voila_batch_tuning_t* tuning,
                                  voila_batch_t* out) {
    if (!items || !out || n < 1) return fail(VOILA_ERR_INVALID_ARG, "NULL items / output or n < 1");
    *out = nullptr;
    voila_batch_tuning_t tu{4, 0, 1};
    if (tuning) tu = *tuning;
    if (tu.waves_per_block < 1 || tu.waves_per_block > 8 || tu.blocks_per_cu < 0)
        return fail(VOILA_ERR_INVALID_ARG, "waves_per_block must be 1..8 and blocks_per_cu >= 0");
    const voila_model_s* m0 = items[0].model;
    if (!m0) return fail(VOILA_ERR_INVALID_ARG, "NULL model in item 0");
    const bool upd = items[0].d_states_out != nullptr;
    for (int j = 0; j < n; ++j) {
        const voila_batch_item_t& it = items[j];
        const std::string tag = "item " + std::to_string(j) + ": ";
        if (!it.model) return fail(VOILA_ERR_INVALID_ARG, tag + "NULL model");
        if (it.model->shape != m0->shape || it.model->dt != m0->dt || it.model->device != m0->device)
            return fail(VOILA_ERR_INVALID_ARG, tag + "models must share shape, precision and device");
        if (it.N < 1 || it.K < 0 || it.H < 0) return fail(VOILA_ERR_INVALID_ARG, tag + "N >= 1, K >= 0, H >= 0");
        if ((long long)it.K * it.N > (1LL << 31) - 1) return fail(VOILA_ERR_UNSUPPORTED, tag + "K * N too large");
        if (!(it.gamma >= 0.0 && it.gamma <= 1.0)) return fail(VOILA_ERR_INVALID_ARG, tag + "gamma outside [0, 1]");
        if (!it.h_goal || !it.d_states) return fail(VOILA_ERR_INVALID_ARG, tag + "NULL goal or states");
        if (it.K > 0 && (!it.d_q_out || (it.H > 0 && !it.d_cands)))
            return fail(VOILA_ERR_INVALID_ARG, tag + "NULL q_out or candidates");
        if (it.reward_at != 0 && it.reward_at != 1) return fail(VOILA_ERR_INVALID_ARG, tag + "reward_at must be 0 or 1");
        if ((it.d_states_out != nullptr) != upd)
            return fail(VOILA_ERR_INVALID_ARG, tag + "either every item or no item has update outputs");
        if (upd) {
            if (!it.model->has_lik) return fail(VOILA_ERR_INVALID_ARG, tag + "model has no likelihood network");
            if (!(it.lambda > 0.0) || !std::isfinite(it.lambda)) return fail(VOILA_ERR_INVALID_ARG, tag + "lambda must be > 0");
            if (it.N > kNormResMaxN) return fail(VOILA_ERR_UNSUPPORTED, tag + "N above voila_update_max_particles()");
        }
    }
    if (!weights_in_lds(m0->shape))
        return fail(VOILA_ERR_UNSUPPORTED, "batches need networks that fit in LDS (hidden width <= 64)");
    DeviceGuard guard(m0->device);
    if (!guard.ok) return fail(VOILA_ERR_DEVICE, "hipSetDevice failed");

    voila_batch_s* b = new voila_batch_s();
    b->device = m0->device;
    b->shape = m0->shape;
    b->dt = m0->dt;
    b->n = n;
    b->cus = m0->cus;
    b->wpb = tu.waves_per_block;
    b->dynamic = tu.dynamic ? 1 : 0;
    b->has_update = upd;
    b->width = m0->width;
    const int d_s = m0->d_s, W = m0->width;

    // device memory plan: tables, work lists, partial sums, update workspace, counters
    std::vector<PlanParams> hp(n);
    std::vector<QReduceParams> hq(n);
    std::vector<ProposeParams> hpr(upd ? n : 0);
    std::vector<FoldBatchItem> hf(upd ? 2 * n : 0);
    std::vector<NormResParams> hn(upd ? n : 0);
    std::vector<int4> plan_items, prop_items;
    std::vector<size_t> part_off(n), ws_off(n);
    size_t part_bytes = 0, ws_bytes = 0;
    for (int j = 0; j < n; ++j) {
        const voila_batch_item_t& it = items[j];
        const int n_tiles = (it.N + 31) / 32;
        part_off[j] = part_bytes;
        part_bytes = align_up(part_bytes + (size_t)it.K * n_tiles * 4, 256);
        if (upd) {
            ws_off[j] = ws_bytes;
            ws_bytes += carve_update(nullptr, W, it.N, d_s).bytes;
        }
        add_items(plan_items, j, (long)it.K * n_tiles, b->wpb, it.H);
        if (upd) add_items(prop_items, j, n_tiles, b->wpb, 1);
        b->max_k = std::max(b->max_k, it.K);
    }
    if (b->dynamic) {
        // longest first; items of one instance stay contiguous (equal cost per unit)
        std::stable_sort(plan_items.begin(), plan_items.end(), [&](const int4& a, const int4& c) {
            int ha = items[a.x].H, hc = items[c.x].H;
            return ha != hc ? ha > hc : a.x < c.x;
        });
    }
    b->n_plan_items = (int)plan_items.size();
    b->n_prop_items = (int)prop_items.size();
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off = align_up(off + bytes, 256);
        return o;
    };
    const size_t o_plan = take(sizeof(PlanParams) * n), o_qr = take(sizeof(QReduceParams) * n);
    const size_t o_prop = take(sizeof(ProposeParams) * hpr.size()), o_fold = take(sizeof(FoldBatchItem) * hf.size());
    const size_t o_nr = take(sizeof(NormResParams) * hn.size());
    const size_t o_pi = take(sizeof(int4) * plan_items.size()), o_ri = take(sizeof(int4) * prop_items.size());
    const size_t o_cnt = take(2 * sizeof(int));
    const size_t o_part = take(part_bytes), o_ws = take(ws_bytes);
    if (hipMalloc(&b->mem, off) != hipSuccess) {
        delete b;
        return fail(VOILA_ERR_DEVICE, "hipMalloc of the batch workspace failed");
    }
    char* base = b->mem;
    for (int j = 0; j < n; ++j) {
        const voila_batch_item_t& it = items[j];
        const voila_model_s* m = it.model;
        const int n_tiles = (it.N + 31) / 32;
        PlanParams& p = hp[j];
        p = PlanParams{};
        p.net = m->trans_plan;
        p.states = it.d_states;
        p.belief_w = it.d_belief_w;
        p.cands = it.d_cands;
        p.returns = it.d_returns_out;
        p.partials = reinterpret_cast<float*>(base + o_part + part_off[j]);
        p.N = it.N;
        p.K = it.K;
        p.H = it.H;
        p.n_tiles = n_tiles;
        p.gamma = it.gamma;
        p.key0 = (uint32_t)(it.seed & 0xffffffffu);
        p.key1 = (uint32_t)(it.seed >> 32);
        p.crn = it.crn ? 1 : 0;
        p.reward_at = it.reward_at;
        for (int c = 0; c < 64; ++c) p.goal[c] = c < d_s ? it.h_goal[c] : 0.0f;
        hq[j] = QReduceParams{p.partials, it.d_q_out, it.K, n_tiles,
                              it.d_belief_w ? 1.0f : (float)(1.0 / (double)it.N)};
        b->plan_lds = std::max<size_t>(b->plan_lds, m->trans_plan.bytes);
        if (upd) {
            UpdateWs w = carve_update(base + o_ws + ws_off[j], W, it.N, d_s);
            const int aw = m->action_width();
            hf[2 * j] = FoldBatchItem{m->fold_w_trans, m->fold_b_trans, w.b0_trans, W, m->nf_trans, m->n_actions,
                                      m->d_a, m->d_o, m->dt == DT_BF16, 0, j};
            hf[2 * j + 1] = FoldBatchItem{m->fold_w_lik, m->fold_b_lik, w.b0_lik, W, m->nf_lik, m->n_actions,
                                          m->d_a, m->d_o, m->dt == DT_BF16, 1, j};
            (void)aw;
            ProposeParams& q = hpr[j];
            q = ProposeParams{};
            q.trans = m->trans_upd;
            q.lik = m->lik;
            q.b0_trans = w.b0_trans;
            q.b0_lik = w.b0_lik;
            q.states = it.d_states;
            q.prior_w = it.d_belief_w;
            q.prop = w.prop;
            q.x = w.x;
            q.N = it.N;
            q.lambda = it.lambda;
            q.key0 = (uint32_t)(it.update_seed & 0xffffffffu);
            q.key1 = (uint32_t)(it.update_seed >> 32);
            NormResParams& r = hn[j];
            r = NormResParams{};
            r.x = w.x;
            r.N = it.N;
            r.bits = voila_resample_bits(it.N);
            r.uniform_prior = it.d_belief_w ? 0 : 1;
            r.do_resample = 1;
            r.lambda = it.lambda;
            r.w_out = it.d_w_out;
            r.stats = it.d_stats_out;
            r.idx_out = it.d_idx_out;
            r.src = w.prop;
            r.dst = it.d_states_out;
            r.row_floats = d_s;
            b->prop_lds = std::max<size_t>(b->prop_lds, (size_t)m->trans_upd.bytes + m->lik.bytes);
        }
    }
    b->d_plan = reinterpret_cast<PlanParams*>(base + o_plan);
    b->d_qr = reinterpret_cast<QReduceParams*>(base + o_qr);
    b->d_prop = reinterpret_cast<ProposeParams*>(base + o_prop);
    b->d_fold = reinterpret_cast<FoldBatchItem*>(base + o_fold);
    b->d_nr = reinterpret_cast<NormResParams*>(base + o_nr);
    b->d_plan_items = reinterpret_cast<int4*>(base + o_pi);
    b->d_prop_items = reinterpret_cast<int4*>(base + o_ri);
    b->d_counters = reinterpret_cast<int*>(base + o_cnt);
    std::vector<char> host(o_part, 0);
    auto put = [&](size_t o, const void* src, size_t bytes) {
        if (bytes) std::memcpy(host.data() + o, src, bytes);
    };
    put(o_plan, hp.data(), sizeof(PlanParams) * n);
    put(o_qr, hq.data(), sizeof(QReduceParams) * n);
    put(o_prop, hpr.data(), sizeof(ProposeParams) * hpr.size());
    put(o_fold, hf.data(), sizeof(FoldBatchItem) * hf.size());
    put(o_nr, hn.data(), sizeof(NormResParams) * hn.size());
    put(o_pi, plan_items.data(), sizeof(int4) * plan_items.size());
    put(o_ri, prop_items.data(), sizeof(int4) * prop_items.size());
    if (hipMemcpy(b->mem, host.data(), o_part, hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipFree(b->mem);
        delete b;
        return fail(VOILA_ERR_DEVICE, "upload of the batch tables failed");
    }
    const int bpc_plan = tu.blocks_per_cu ? tu.blocks_per_cu
                                          : plan_batch_blocks_per_cu(b->shape, b->dt, b->wpb, b->plan_lds);
    b->plan_blocks = std::max(1, std::min(b->n_plan_items, b->cus * bpc_plan));
    if (upd) {
        const int bpc_prop = tu.blocks_per_cu ? tu.blocks_per_cu
                                              : propose_batch_blocks_per_cu(b->shape, b->dt, b->wpb, b->prop_lds);
        b->prop_blocks = std::max(1, std::min(b->n_prop_items, b->cus * bpc_prop));
    }
    *out = b;
    return VOILA_OK;
}

voila_status_t voila_batch_destroy(voila_batch_t b) {
    if (!b) return VOILA_OK;
    {
        DeviceGuard guard(b->device);
        if (b->exec) (void)hipGraphExecDestroy(b->exec);
        if (b->graph) (void)hipGraphDestroy(b->graph);
        if (b->mem) (void)hipFree(b->mem);
    }
    delete b;
    return VOILA_OK;
}

static voila_status_t batch_enqueue(voila_batch_t b, int32_t what, const void* d_actions, const float* d_obs,
                                    const uint32_t* d_u, int32_t* d_status, hipStream_t s) {
    if (what & VOILA_BATCH_PLAN) {
        if (b->dynamic) VOILA_CHECK_HIP(launch_reset_counter(b->d_counters, s));
        BatchPlanParams p{b->d_plan, b->d_plan_items, b->n_plan_items, b->dynamic, b->d_counters, d_status};
        VOILA_CHECK_HIP(launch_plan_batch(b->shape, b->dt, p, b->plan_blocks, b->wpb, b->plan_lds, s));
        VOILA_CHECK_HIP(launch_q_reduce_batch(b->d_qr, b->n, b->max_k, s));
    }
    if (what & VOILA_BATCH_UPDATE) {
        VOILA_CHECK_HIP(launch_fold_batch(b->d_fold, 2 * b->n, b->width, d_actions, d_obs, d_status, s));
        if (b->dynamic) VOILA_CHECK_HIP(launch_reset_counter(b->d_counters + 1, s));
        BatchProposeParams p{b->d_prop, b->d_prop_items, b->n_prop_items, b->dynamic, b->d_counters + 1, d_status};
        VOILA_CHECK_HIP(launch_propose_batch(b->shape, b->dt, p, b->prop_blocks, b->wpb, b->prop_lds, s));
        VOILA_CHECK_HIP(launch_norm_res_batch(b->d_nr, b->n, d_u, d_status, s));
    }
    return VOILA_OK;
}

static voila_status_t batch_check(voila_batch_t b, int32_t what, const void* d_actions, const float* d_obs,
                                  const uint32_t* d_u) {
    if (!b) return fail(VOILA_ERR_INVALID_ARG, "NULL batch");
    if (what < 1 || what > 3) return fail(VOILA_ERR_INVALID_ARG, "what must combine VOILA_BATCH_PLAN / _UPDATE");
    if (what & VOILA_BATCH_UPDATE) {
        if (!b->has_update) return fail(VOILA_ERR_INVALID_ARG, "the batch was created without update outputs");
        if (!d_actions || !d_obs || !d_u) return fail(VOILA_ERR_INVALID_ARG, "NULL actions, observations or offsets");
    }
    return VOILA_OK;
}

voila_status_t voila_batch_run(voila_batch_t b, int32_t what, const void* d_actions, const float* d_obs,
                               const uint32_t* d_u, int32_t* d_status, void* stream) {
    voila_status_t st = batch_check(b, what, d_actions, d_obs, d_u);
    if (st != VOILA_OK) return st;
    DeviceGuard guard(b->device);
    if (!guard.ok) return fail(VOILA_ERR_DEVICE, "hipSetDevice failed");
    return batch_enqueue(b, what, d_actions, d_obs, d_u, d_status, reinterpret_cast<hipStream_t>(stream));
}

voila_status_t voila_batch_capture(voila_batch_t b, int32_t what, const void* d_actions, const float* d_obs,
                                   const uint32_t* d_u, int32_t* d_status) {
    voila_status_t st = batch_check(b, what, d_actions, d_obs, d_u);
    if (st != VOILA_OK) return st;
    DeviceGuard guard(b->device);
    if (!guard.ok) return fail(VOILA_ERR_DEVICE, "hipSetDevice failed");
    hipStream_t s = nullptr;
    VOILA_CHECK_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        st = batch_enqueue(b, what, d_actions, d_obs, d_u, d_status, s);
        hipError_t e2 = hipStreamEndCapture(s, &g);
        if (st == VOILA_OK && e2 != hipSuccess) st = fail(VOILA_ERR_DEVICE, "hipStreamEndCapture failed");
    } else {
        st = fail(VOILA_ERR_DEVICE, std::string("hipStreamBeginCapture: ") + hipGetErrorString(e));
    }
    (void)hipStreamDestroy(s);
    if (st != VOILA_OK) {
        if (g) (void)hipGraphDestroy(g);
        return st;
    }
    hipGraphExec_t ex = nullptr;
    e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(g);
        return fail(VOILA_ERR_DEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
    }
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->graph = g;
    b->exec = ex;
    return VOILA_OK;
}

voila_status_t voila_batch_replay(voila_batch_t b, void* stream) {
    if (!b) return fail(VOILA_ERR_INVALID_ARG, "NULL batch");
    if (!b->exec) return fail(VOILA_ERR_INVALID_ARG, "no captured graph: call voila_batch_capture first");
    DeviceGuard guard(b->device);
    if (!guard.ok) return fail(VOILA_ERR_DEVICE, "hipSetDevice failed");
    VOILA_CHECK_HIP(hipGraphLaunch(b->exec, reinterpret_cast<hipStream_t>(stream)));
    return VOILA_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// gradients through rollouts
// ---------------------------------------------------------------------------
namespace {
struct GradWs {
    float* ckpt;
    float* segst;
    float* wpart;
    float* lpart;
    float* apart;
    size_t bytes;
    int blocks;
};
GradWs carve_grad(const voila_model_s* m, const voila_grad_opts_t* o, char* base) {
    GradWs w{};
    const int n_tiles = (o->B + 31) / 32;
    const int C = o->checkpoint, NC = (o->H + C - 1) / C;
    const int want = (n_tiles + kGradWaves - 1) / kGradWaves;
    const int cap = m->cus * m->grad_bpc;
    w.blocks = std::max(1, std::min(want, cap));
    const int n_waves = w.blocks * kGradWaves;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        char* p = base ? base + off : nullptr;
        off = align_up(off + bytes, 256);
        return reinterpret_cast<float*>(p);
    };
    w.ckpt = take((size_t)o->B * std::max(NC, 1) * m->d_s * 4);
    w.segst = take((size_t)o->B * (C + 1) * m->d_s * 4);
    w.wpart = take((size_t)n_waves * m->n_params * 4);
    w.lpart = take((size_t)n_waves * 4);
    w.apart = take((size_t)n_tiles * std::max(o->H, 1) * std::max(m->d_a, 1) * 4);
    w.bytes = off;
    return w;
}
voila_status_t grad_check(const voila_model_s* m, const voila_grad_opts_t* o) {
    if (!m) return fail(VOILA_ERR_INVALID_ARG, "NULL model");
    if (!o) return fail(VOILA_ERR_INVALID_ARG, "NULL options");
    if (!m->has_grad) return fail(VOILA_ERR_UNSUPPORTED, "gradients need a binary32 model with two hidden layers of 64");
    if (o->B < 1 || o->H < 0 || o->H > 64 || o->checkpoint < 1)
        return fail(VOILA_ERR_INVALID_ARG, "B >= 1, 0 <= H <= 64, checkpoint >= 1");
    if (o->objective != VOILA_OBJ_DISTILL && o->objective != VOILA_OBJ_RETURN)
        return fail(VOILA_ERR_INVALID_ARG, "unknown objective");
    if (!o->d_s0 || (o->H > 0 && !o->d_actions)) return fail(VOILA_ERR_INVALID_ARG, "NULL states or actions");
    if (o->objective == VOILA_OBJ_DISTILL && o->H > 0 && !o->d_targets)
        return fail(VOILA_ERR_INVALID_ARG, "the distillation objective needs teacher states");
    if (o->objective == VOILA_OBJ_RETURN && (!o->h_goal || !(o->gamma >= 0.0 && o->gamma <= 1.0)))
        return fail(VOILA_ERR_INVALID_ARG, "the return objective needs a goal and gamma in [0, 1]");
    if (m->n_actions == 0 && (o->particles < 1 || o->B % o->particles != 0))
        return fail(VOILA_ERR_INVALID_ARG, "particles must divide B");
    if (o->d_grad_actions && (m->n_actions > 0 || o->particles % 32 != 0))
        return fail(VOILA_ERR_INVALID_ARG, "action gradients need continuous actions and particles % 32 == 0");
    return VOILA_OK;
}
}  // namespace

extern "C" {

int32_t voila_grad_param_count(voila_model_t m) { return m && m->has_grad ? m->n_params : 0; }

size_t voila_rollout_grad_workspace_size(voila_model_t m, const voila_grad_opts_t* o) {
    if (grad_check(m, o) != VOILA_OK) return 0;
    return carve_grad(m, o, nullptr).bytes;
}

voila_status_t voila_rollout_grad(voila_model_t m, const voila_grad_opts_t* o, void* ws, size_t ws_bytes,
                                  void* stream) {
    voila_status_t st = grad_check(m, o);
    if (st != VOILA_OK) return st;
    GradWs w = carve_grad(m, o, reinterpret_cast<char*>(ws));
    if (!ws || ws_bytes < w.bytes) return fail(VOILA_ERR_WORKSPACE, "gradient workspace too small");
    DeviceGuard guard(m->device);
    if (!guard.ok) return fail(VOILA_ERR_DEVICE, "hipSetDevice failed");
    GradParams p{};
    p.fwd = m->grad_fwd;
    p.bwd = m->grad_bwd;
    p.s0 = o->d_s0;
    p.actions = o->d_actions;
    p.noise = o->d_noise;
    p.targets = o->d_targets;
    p.ckpt = w.ckpt;
    p.segst = w.segst;
    p.wpart = w.wpart;
    p.lpart = w.lpart;
    p.apart = o->d_grad_actions ? w.apart : nullptr;
    p.B = o->B;
    p.H = o->H;
    p.C = o->checkpoint;
    p.NC = (o->H + o->checkpoint - 1) / o->checkpoint;
    p.particles = m->n_actions > 0 ? 1 : o->particles;
    p.objective = o->objective;
    p.want_params = o->d_grad_params ? 1 : 0;
    p.n_params = m->n_params;
    p.scale = o->objective == VOILA_OBJ_DISTILL ? 1.0 / ((double)o->B * std::max(o->H, 1)) : 1.0 / (double)o->B;
    p.key0 = (uint32_t)(o->seed & 0xffffffffu);
    p.key1 = (uint32_t)(o->seed >> 32);
    for (int j = 0; j < 32; ++j) p.goal[j] = (o->h_goal && j < m->d_s) ? o->h_goal[j] : 0.0f;
    double d = 1.0;
    for (int t = 0; t < 64; ++t) {
        p.disc[t] = (float)d;
        d *= o->gamma;
    }
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    VOILA_CHECK_HIP(launch_grad(m->shape, p, w.blocks, grad_lds_bytes(m), s));
    GradReduceParams r{};
    r.wpart = w.wpart;
    r.lpart = w.lpart;
    r.apart = p.apart;
    r.grad_params = o->d_grad_params;
    r.grad_actions = o->d_grad_actions;
    r.loss = o->d_loss_out;
    r.n_params = o->d_grad_params ? m->n_params : 0;
    r.n_waves = w.blocks * kGradWaves;
    r.H = o->H;
    r.d_a = m->d_a;
    r.tiles_per_seq = m->n_actions > 0 ? 1 : o->particles / 32;
    r.n_action_values = o->d_grad_actions ? (o->B / o->particles) * o->H * m->d_a : 0;
    r.scale = p.scale;
    VOILA_CHECK_HIP(launch_grad_reduce(r, s));
    return VOILA_OK;
}

}  // extern "C"
