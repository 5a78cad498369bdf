// kernels.hpp -- host-visible parameter blocks and launchers of the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device.hpp"

namespace voila {

// Network shapes with compiled kernels: X(id, d_s, n_actions, d_a, d_w, d_o, d_wz, width, n_hidden)
// (n_actions > 0: discrete one-hot actions; d_a > 0: continuous actions).
#define VOILA_SHAPES(X)                                 \
    X(0, 4, 5, 0, 4, 2, 2, 64, 2)     /* small */        \
    X(1, 16, 0, 4, 16, 32, 32, 256, 3) /* realistic */    \
    X(2, 4, 0, 4, 4, 2, 2, 64, 2)      /* small, continuous actions */ \
    X(3, 4, 5, 0, 4, 2, 2, 1024, 2)    /* small, hidden width 1024 */ \
    X(4, 4, 5, 0, 4, 2, 2, 1024, 4)    /* small, four hidden layers of 1024 (no likelihood network) */ \
    X(5, 45, 6, 0, 45, 36, 36, 1024, 4) /* target finding: 45-d state, six actions, 36 lidar bins */

constexpr int kNumShapes = 6;

// Model shapes whose likelihood network has a shape of its own (the paper
// pairs four-layer samplers of width 1024 with a likelihood of three hidden
// layers of 256): X(id, d_s, likelihood width, likelihood hidden layers).
// Such models update beliefs (proposal and likelihood in separate kernels);
// the other likelihood users refuse them.
#define VOILA_LIK_SHAPES(X) X(5, 45, 256, 3)
int lik_shape_width(int shape);   // 0: the likelihood has the model's width and depth
int lik_shape_hidden(int shape);

struct ShapeInfo {
    int d_s, n_actions, d_a, d_w, d_o, d_wz, width, n_hidden;
};
const ShapeInfo& shape_info(int shape);

// First-layer slots per lane group for each use of a network.
int plan_in_slots(int shape, int dt);     // transition net in plan: state + continuous action + noise
int update_in_slots(int shape, int dt);   // transition net in update: state + noise (action folded)
int obs_in_slots(int shape, int dt);      // observation net: state + obs noise (action folded)
int lik_in_slots(int shape, int dt);      // likelihood net: state (action, observation folded)
int nce_in_slots(int shape, int dt);      // likelihood net: observation (state, action folded)

struct PlanParams {
    NetBlob net;
    const float* states;     // [N][d_s]
    const double* belief_w;  // [N] or NULL
    const void* cands;       // int32 [K][H] or float [K][H][d_a]
    const float* noise;      // [K][N][H][d_w] or NULL
    float* returns;          // [K][N] or NULL
    float* traj;             // [K][N][H][d_s] rollout states s_1..s_H, or NULL
    float* partials;         // [K][n_tiles]
    int32_t* status;         // or NULL
    int N, K, H, n_tiles;
    double gamma;
    uint32_t key0, key1;
    int crn, reward_at;
    float goal[64];
};

struct QReduceParams {
    const float* partials;
    float* q;
    int K, n_tiles;
    float scale;
};

struct ProposeParams {
    NetBlob trans, lik;
    const float* b0_trans;   // folded first-layer bias of the transition net [width]
    const float* b0_lik;     // folded first-layer bias of the likelihood net [width]
    const float* states;     // [N][d_s]
    const double* prior_w;   // [N] or NULL
    const float* noise;      // [N][d_w] or NULL
    float* prop;             // [N][d_s]
    float* loglik;           // [N] or NULL
    double* x;               // [N]  l / lambda (+ log prior)
    int32_t* status;         // or NULL
    int N;
    double lambda;
    uint32_t key0, key1;
};

// Observations of rows (k, i, t), k < K, i < N, t < H (K = H = 1: n plain rows).
struct ObserveParams {
    NetBlob obs;
    const float* b0;         // folded first-layer biases, row k * H + t at b0 + (k * H + t) * b0_stride
    int b0_stride;           // 0: one bias for every row
    const float* states;     // [K][N][H][d_s]
    const float* noise;      // [K][N][H][d_wz] or NULL
    float* out;              // [K][N][H][d_o]
    int N, K, H, crn;
    uint32_t key0, key1;
    uint32_t row_bias_lds;   // LDS offset of the per-wave bias rows (whole-rollout launches; set by the launcher)
};

// First-layer biases with the action (and observation) of each row folded in.
struct FoldStepsParams {
    const float* w;      // [width][nf] action (then observation) columns of the first layer
    const float* b;      // [width]
    float* out;          // [rows][width]
    const void* cands;   // int32 [rows] action indices or float [rows][d_a]
    const float* obs;    // [rows][d_o] observations to fold, or NULL
    int width, nf, rows, n_actions, d_a, d_o, bf16;
    int32_t* status;     // or NULL
};

// Soft value of M nodes' candidate preferences (one workgroup per node).
struct SoftValueParams {
    const float* Q;          // [M][K] preferences (plan's Q), or NULL when Qd is given
    const double* Qd;        // [M][K] binary64 preferences, or NULL
    const double* log_pi0;   // [M][K] reference-policy log-probabilities, or NULL (uniform)
    int no_prior;            // 1: no prior term at all (the preferences already hold it)
    double* V;               // [M]
    double* pi;              // [M][K] or NULL
    int32_t* best;           // [M] or NULL
    int32_t* status;         // or NULL
    int M, K;
    double eta;
};
hipError_t launch_soft_value(const SoftValueParams& p, int blocks, hipStream_t s);

// One-level closed-loop tree: A first actions, n_obs observation branches
// each (M = A n_obs groups of N successors), K continuation candidates.
struct TreeParams {
    const float* succ0;      // [A][N][d_s] successors of each first action
    float* succ;             // [M][N][d_s] group (a, j): successors of a from successor j on
    int32_t* seg;            // [M + 1]
    const void* first;       // int32 [A] or float [A][d_a]
    void* acts;              // int32 [M] or float [M][d_a]
    int32_t* zeros;          // [2 M] visits and branch counts (all 0)
    const float* G2;         // [K][M N] continuation returns from the children
    double* Qc;              // [M][K] child preferences
    const double* Vc;        // [M] child values
    const float* R;          // [A] first-step reward estimates
    const double* log_pi0;   // [A] or NULL (uniform)
    double* psi;             // [A]
    double* R_out;           // [A] or NULL
    int A, n_obs, N, K, d_s, n_actions, d_a;
    double gamma, eta;
};
hipError_t launch_tree_groups(const TreeParams& p, hipStream_t s);
hipError_t launch_tree_child_q(const TreeParams& p, hipStream_t s);
hipError_t launch_tree_backup(const TreeParams& p, hipStream_t s);

// Grouped progressive-widening step over M action nodes (groups of successors
// seg[m] .. seg[m+1]).
struct PwParams {
    NetBlob lik;
    const float* succ;        // [T][d_s]
    const int32_t* seg;       // [M + 1]
    const void* actions;      // int32 [M] or float [M][d_a]
    const int32_t* visits;    // [M]
    int32_t* children;        // [M], updated
    float* table;             // [M][B][d_o], updated
    const uint32_t* U;        // [M] resampling offsets
    float* first;             // [M][d_s] first successor of each group (workspace)
    const float* o_new;       // [M][d_o] observation drawn at the first successor
    float* o_sel;             // [M][d_o] observation of the chosen branch (workspace)
    const float* b0_lik;      // [M][width] folded likelihood biases
    int32_t* tiles;           // [M + 1] exclusive prefix of the groups' 32-row tile counts
    double* x;                // [T] l / lambda
    int32_t* widen;           // [M] or NULL
    int32_t* branch;          // [M] or NULL
    float* loglik;            // [T] or NULL
    double* w;                // [T] or NULL
    double* stats;            // [M][2] or NULL
    int32_t* idx;             // [T] indices within the group, or NULL
    float* succ_out;          // [T][d_s] or NULL
    int32_t* status;          // or NULL
    int T, M, B, d_s, d_o;
    double k_o, alpha_o, lambda;
    uint32_t key0, key1;
};

// Contrastive objective of the likelihood network over a mini-batch of B
// tuples (s'_i, a_i, o_i): scores l_ij = l([s'_i, a_i, o_j]) of all pairs.
struct NceParams {
    NetBlob lik;          // likelihood network packed with its first layer over the observation columns
    const float* obs;     // [B][d_o]
    const float* b0;      // [B][width] first-layer biases with row i's state and action folded in
    float* scores;        // [B][B] l_ij, row i = state-action i
    double* row_loss;     // [B] log sum_j exp(l_ij) - l_ii
    float* grad;          // [B][B] derivative of the mean row loss by l_ij, or NULL
    double* loss;         // [1] mean row loss, or NULL
    int32_t* status;      // or NULL
    int B, d_o;
    uint32_t row_bias_lds;  // LDS offset of the per-wave bias rows (set by the launcher)
};

// Teacher sampler of a v-prediction denoiser (input [c, a, x_tau, tau],
// output v): n_steps deterministic DDIM steps per sample.
struct DdimParams {
    NetBlob net;          // state slots: x_tau; noise slots: the conditioning input
    const float* states;  // [N][d_c] conditioning inputs
    const float* x1;      // [N][d_x] latent noise at tau = 1
    const float* b0;      // [n_steps][width] first-layer biases with the action and tau_k folded in
    const float* coef;    // [n_steps][2]: x <- x + (coef[0] x + coef[1] v), coef[0] = A - 1
    float* out;           // [N][d_x]
    int N, n_steps;
};
struct DdimPrepParams {
    const float* w;       // [width][a_width + 1]: action columns, then the tau column
    const float* b;       // [width]
    float* b0;            // [n_steps][width]
    float* coef;          // [n_steps][2]
    int width, aw, n_steps, bf16;
    float v[64];          // action values (one-hot or continuous)
};

struct NormResParams {
    const double* x;         // [N] precomputed l / lambda (+ log prior), or NULL
    const float* loglik;     // [N] used when x is NULL and w_in is NULL
    const double* prior_w;   // [N] or NULL (with loglik)
    const double* w_in;      // [N] given normalised weights (resample only), or NULL
    double lambda;
    int N, bits, uniform_prior, do_resample;
    uint32_t U;
    double* w_out;           // [N] or NULL
    double* stats;           // [2] or NULL
    int32_t* idx_out;        // [N] or NULL
    const float* src;        // gather source rows or NULL
    float* dst;              // gather destination rows or NULL
    int row_floats;
    int32_t* status;         // or NULL
};

// Many instances in one launch.  items[j] = (instance, first unit, units in
// this item (<= waves per block), cost used for ordering).
struct BatchPlanParams {
    const PlanParams* insts;
    const int4* items;
    int n_items;
    int dynamic;   // 1: items taken from the atomic counter in list order
    int* counter;
    int32_t* status;
};

struct BatchProposeParams {
    const ProposeParams* insts;
    const int4* items;
    int n_items;
    int dynamic;
    int* counter;
    int32_t* status;
};

// Fold of instance `inst`'s action (and observation) into a first-layer bias;
// actions and observations are read at run time from arrays indexed by inst.
struct FoldBatchItem {
    const float* w;   // [width][nf]
    const float* b;   // [width]
    float* out;       // [width]
    int width, nf, n_actions, d_a, d_o, bf16, with_obs, inst;
};

// Adjoint rollouts (two hidden layers of width 64, binary32).
struct GradParams {
    NetBlob fwd, bwd;          // forward pack (actions as inputs) and transposed pack
    const float* s0;           // [B][d_s]
    const void* actions;       // int32 [B][H] or float [B / particles][H][d_a]
    const float* noise;        // [B][H][d_w] or NULL
    const float* targets;      // [B][H][d_s] (distillation)
    float* ckpt;               // [B][NC][d_s] checkpoints
    float* segst;              // [B][C + 1][d_s] states of the segment being reversed
    float* wpart;              // [waves][n_params] parameter-gradient partials
    float* lpart;              // [waves] objective partials
    float* apart;              // [tiles][H][d_a] action-gradient partials or NULL
    int B, H, C, NC, particles, objective, want_params, n_params;
    double scale;
    uint32_t key0, key1;
    float goal[32];
    float disc[64];            // gamma^t
};

// Parameter derivative of the contrastive objective for binary32 width-64
// likelihood networks with two hidden layers.
struct NceGradParams {
    NetBlob fwd, bwd;     // first layer over the observation columns; transposed pack
    const float* w3;      // [64] output-layer weights
    const float* b0;      // [B][64] first-layer biases with row i's state and action folded in
    const float* obs;     // [B][d_o]
    const float* states;  // [B][d_s]
    const void* actions;  // int32 [B] or float [B][d_a]
    const float* grad;    // [B][B] derivative of the loss by each score
    float* wpart;         // [waves][n_params] per-wave partials
    int32_t* status;      // or NULL
    int B, n_params;
};
bool nce_grad_supported(int shape);
hipError_t launch_nce_grad(int shape, const NceGradParams& p, int blocks, size_t lds, hipStream_t s);
int nce_grad_blocks_per_cu(int shape, size_t lds);

struct GradReduceParams {
    const float* wpart;
    const float* lpart;
    const float* apart;
    float* grad_params;
    float* grad_actions;
    float* loss;
    int n_params, n_waves, n_action_values, H, d_a, tiles_per_seq;
    double scale;
};

// Multi-workgroup normalisation / resampling for large beliefs.
struct LargeResWs {
    double* bmax;    // per-block max
    double* bsum;    // per-block sum of exp
    double* bsq;     // per-block sum of squared weights
    int* blast;      // per-block last positive-mass particle
    double* btot;    // per-chunk total of quantised weights
    double* bbt;     // per-block total of quantised weights (the sum of its chunks')
    double* boff;    // exclusive prefix of the block totals
    double* bincl;   // inclusive prefix of the block totals
    double* scal;    // [0] max, [1] sum
    int* last;       // last positive-mass particle overall
};

struct LargeResParams {
    const double* x;        // [N] l / lambda (+ log prior), or NULL
    const float* loglik;    // [N] used when x and w_in are NULL
    const double* prior_w;  // with loglik, or NULL
    const double* w_in;     // given normalised weights (resample only), or NULL
    double lambda;
    int N, bits, uniform_prior, do_resample, n_chunks, n_blocks;
    uint32_t U;
    double* w_out;
    double* stats;
    int32_t* idx_out;
    const float* src;
    float* dst;
    int row_floats;
    int32_t* status;
    LargeResWs ws;
};

size_t large_res_workspace_bytes(int N);
LargeResWs carve_large_res(void* base, int N);
hipError_t launch_large_res(LargeResParams p, hipStream_t s);
constexpr int kLargeMaxN = 1 << 26;

struct PhiloxParams {
    float* out;
    uint32_t* words;
    int n, d;
    uint32_t key0, key1, c0, c1, c2, stream;
};

constexpr int kNormResMaxN = 8192;
constexpr int kNormResThreads = 1024;

// Kernel launchers (return the launch status).
hipError_t launch_plan(int shape, int dt, const PlanParams& p, int blocks, hipStream_t s);
hipError_t launch_q_reduce(const QReduceParams& p, hipStream_t s);
hipError_t launch_fold_steps(const FoldStepsParams& p, hipStream_t s);
// Grouped progressive-widening stages.
hipError_t launch_pw_first(const PwParams& p, hipStream_t s);
hipError_t launch_pw_branch(const PwParams& p, hipStream_t s);
hipError_t launch_pw_tiles(const PwParams& p, hipStream_t s);
hipError_t launch_pw_lik(int shape, int dt, const PwParams& p, int blocks, hipStream_t s);
int pw_lik_blocks_per_cu(int shape, int dt);
hipError_t launch_pw_norm_res(const PwParams& p, int blocks, hipStream_t s);
// Contrastive-objective stages: all-pairs scores, per-row losses and
// derivatives (one workgroup per row), the mean loss (one workgroup).
hipError_t launch_nce_scores(int shape, int dt, const NceParams& p, int blocks, hipStream_t s);
int nce_scores_blocks_per_cu(int shape, int dt);
hipError_t launch_nce_rows(const NceParams& p, int blocks, hipStream_t s);
hipError_t launch_nce_mean(const NceParams& p, hipStream_t s);
// Denoiser shapes of the teacher sampler: (id, denoised width d_x,
// conditioning width d_c, hidden width, hidden layers).
#define VOILA_DDIM_SHAPES(X) \
    X(0, 4, 4, 64, 2)        \
    X(1, 4, 4, 1024, 5)      \
    X(2, 4, 4, 1024, 4)      \
    X(3, 32, 16, 512, 5)     \
    X(4, 64, 44, 512, 5)
constexpr int kNumDdimShapes = 5;
int ddim_shape(int d_x, int d_c, int width, int n_hidden);  // -1 when not compiled
int ddim_in_slots(int shape, int dt);
bool ddim_split(int shape);                        // evaluated by all waves of a block per group of tiles
int ddim_tiles_per_block(int shape);
hipError_t launch_ddim_prep(const DdimPrepParams& p, hipStream_t s);
hipError_t launch_ddim(int shape, int dt, const DdimParams& p, int blocks, hipStream_t s);
int ddim_blocks_per_cu(int shape, int dt);
constexpr int kDdimMaxSteps = 4096;
constexpr int kNceMaxBatch = 32768;  // B <= this (the score matrix holds B^2 binary32 values)
constexpr int kPwMaxGroup = 8192;  // successors per group (one workgroup normalises and resamples a group)
hipError_t launch_propose(int shape, int dt, const ProposeParams& p, int blocks, hipStream_t s);
// Update stage 1 of the models of VOILA_LIK_SHAPES: proposals through the split
// transition kernel (two 32-particle tiles per block), then the likelihood of
// the proposals (one tile per block of four waves).
hipError_t launch_propose_split(int shape, int dt, const ProposeParams& p, int blocks, hipStream_t s);
int propose_split_blocks_per_cu(int shape, int dt);
constexpr int kPropSplitTiles = 2;
hipError_t launch_lik_rows(int shape, int dt, const ProposeParams& p, int blocks, hipStream_t s);
int lik_rows_blocks_per_cu(int shape, int dt);
hipError_t launch_observe(int shape, int dt, const ObserveParams& p, int blocks, hipStream_t s);
// The observe kernel sized for the rows of whole rollouts (weights streamed like the rollout kernel's).
hipError_t launch_observe_rollouts(int shape, int dt, const ObserveParams& p, int blocks, hipStream_t s);
int observe_rollout_blocks_per_cu(int shape, int dt);
hipError_t launch_norm_res(const NormResParams& p, hipStream_t s);
hipError_t launch_philox(const PhiloxParams& p, hipStream_t s);
hipError_t launch_plan_batch(int shape, int dt, const BatchPlanParams& p, int blocks, int waves_per_block,
                             size_t lds, hipStream_t s);
hipError_t launch_q_reduce_batch(const QReduceParams* d_qs, int n_inst, int max_k, hipStream_t s);
hipError_t launch_fold_batch(const FoldBatchItem* d_items, int n_items, int max_width, const void* d_actions,
                             const float* d_obs, int32_t* d_status, hipStream_t s);
hipError_t launch_propose_batch(int shape, int dt, const BatchProposeParams& p, int blocks, int waves_per_block,
                                size_t lds, hipStream_t s);
hipError_t launch_norm_res_batch(const NormResParams* d_ps, int n_inst, const uint32_t* d_u, int32_t* d_status,
                                 hipStream_t s);
hipError_t launch_reset_counter(int* d_counter, hipStream_t s);
int plan_batch_blocks_per_cu(int shape, int dt, int waves_per_block, size_t lds);
bool grad_supported(int shape);
hipError_t launch_grad(int shape, const GradParams& p, int blocks, size_t lds, hipStream_t s);
hipError_t launch_grad_reduce(const GradReduceParams& p, hipStream_t s);
int grad_blocks_per_cu(int shape, size_t lds);
int propose_batch_blocks_per_cu(int shape, int dt, int waves_per_block, size_t lds);

// Output tiles per pass of the plan kernel's paired evaluation (two
// 32-particle tiles per wave, weights in pass-major order), 0 when the shape
// runs one tile per wave in the layer-major order.
int plan_pass_tiles(int shape, int dt);
// Rollout work units: 32-particle tiles per unit (1, 2 for the paired
// evaluation, or the split kernel's tiles per block) and units per block.
int plan_tiles_per_unit(int shape, int dt);
int plan_units_per_block(int shape, int dt);
bool plan_split_shape(int shape, int dt);

// Resident blocks per CU of the plan / propose / observe kernels.
int plan_blocks_per_cu(int shape, int dt);
int propose_blocks_per_cu(int shape, int dt);
int pass_tiles_per_block(int shape);  // 32-particle tiles one propose / observe block covers
int observe_blocks_per_cu(int shape, int dt);
// Whether a shape's kernels stage the packed network in LDS.
bool weights_in_lds(int shape);

// Derivative of the contrastive objective for likelihood networks evaluated
// layer by layer: stage 1 (forward and reverse sweep of every pair of a
// chunk, activations and adjoints stored) and stage 2 (split-K products).
struct NceWideParams {
    const char* stream;    // fragments: first layer (observation inputs), hidden layers, transposed hidden layers
    const float* bh;       // [NHID - 1][width] hidden biases
    const float* w_out;    // [width] output-layer weights (bfloat16 values for bfloat16 models)
    const float* b0;       // [B][width] first-layer bias rows with s'_i and a_i folded in
    const float* obs;      // [B][d_o]
    const float* grad;     // [B][B] d loss / d l_ij
    void* act;             // [2 NHID - 1][uc][width][32]: h_1..h_NHID, then delta_1..delta_{NHID-1}
    long uc;               // unit capacity of the arrays
    long u0, u1;           // units of the chunk (unit u: row u / jtiles, 32 columns from 32 (u % jtiles))
    int B;
    uint32_t lds_bias;     // LDS offset of the staged biases (set by the launcher)
};
struct NceWgradParams {
    const void* act;       // the chunk's arrays (as NceWideParams::act)
    long uc, u0;           // as NceWideParams
    long n_units;          // units in the chunk
    long per_split;        // units per workgroup (a multiple of the staged chunk)
    const float* grad;     // [B][B]
    const float* w_out;    // [width]
    const float* states;   // [B][d_s]
    const void* actions;   // int32 [B] or float [B][d_a]
    const float* obs;      // [B][d_o]
    int B, n_actions, d_a, d_s, d_o, d_in;
    float* part;           // [workgroups][n_params] partial sums
    int n_params;
    int accumulate;        // 0: the first chunk writes the partials, 1: later chunks add
};
bool nce_wide_supported(int shape);
size_t nce_wide_bwd_lds(int dt);
hipError_t launch_nce_wide_bwd(int shape, int dt, const NceWideParams& p, int blocks, hipStream_t s);
hipError_t launch_nce_wide_wgrad(int shape, int dt, const NceWgradParams& p, int blocks, hipStream_t s);
int nce_wide_bwd_blocks_per_cu(int dt);
int nce_wide_wgrad_blocks_per_cu(int dt);

constexpr int kWavesPerBlock = 4;

}  // namespace voila
