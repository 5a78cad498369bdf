/*
 * voila.h -- C ABI of the VOiLA planning hot path on AMD Instinct MI355X (gfx950).
 *
 * The library evaluates the two data-parallel halves of online POMDP planning
 * with learned generative models (Hoerger et al., "VOiLA: Vectorized Online
 * Planning with Learned Diffusion Models for POMDP Agents"):
 *
 *   plan    Monte-Carlo returns of open-loop candidate action sequences from a
 *           particle belief, simulated through the distilled transition sampler
 *           s' = f_T(s, a, w_T), w_T ~ N(0, I) (Sec. 4.2, Eq. 2; Sec. 4.3), with
 *           the expected reward R(b, a) estimated as an average over belief
 *           particles (Sec. 2.1; Sec. 2.2 below Eq. 1) and discounted by gamma^t.
 *   update  The SIR belief update of Sec. 3: proposal particles from f_T,
 *           weights proportional to exp(l(s', a, o) / lambda) from the learned
 *           likelihood (Sec. 4.2, "Likelihood Model"), normalised in binary64,
 *           then systematic resampling.
 *   observe The observation sampler z = f_Z(s', a, w_Z) (Sec. 4.2, Eq. 5).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Pointers named d_* are DEVICE pointers (memory of the model's device);
 *   pointers named h_* are HOST pointers.  The caller owns every buffer it
 *   passes; the library owns only the model object it creates.
 * - `stream` is a hipStream_t (NULL = the legacy default stream).  Compute
 *   entry points only enqueue work on it: they do not allocate and do not
 *   synchronise, so results are ready when the stream's earlier work and the
 *   enqueued kernels have finished.  Entry points marked [sync] synchronise.
 * - Argument errors are reported synchronously, before anything is enqueued,
 *   and leave all outputs untouched.  Numeric failures detected on the device
 *   (a non-finite log-likelihood, all weights zero) are reported through the
 *   optional device status word d_status (set to a nonzero VOILA_ERR_NUMERIC,
 *   never cleared by the library) and leave the outputs of that call
 *   undefined.
 * - voila_last_error() returns a thread-local description of the last
 *   argument error.
 * - Networks are multilayer perceptrons: affine layers with ReLU between them
 *   and a linear output layer; each layer is given as nn.Linear stores it,
 *   W[out][in] row-major and b[out].  Input vectors are concatenated as
 *   [s, a, w] for the samplers and [s', a, o] for the likelihood; a discrete
 *   action enters as a one-hot vector over the action set (0-based index).
 * - Counter-based noise: draws come from Philox4x32-10 (Salmon et al., SC'11)
 *   keyed by the 64-bit seed (low word first).  Block j of four draws of
 *   particle i uses the counter (i, c1, t, (stream << 16) | j): plan uses
 *   stream 3 with c1 = candidate index (0 under common random numbers) and t =
 *   step; observe uses stream 4 with (row, 0, 0); update uses stream 5 with
 *   (i, 0, 0).  Each word x gives u = (2 * (x >> 9) + 1) * 2^-24, and the pairs
 *   (u0, u1), (u2, u3) give draws 4j..4j+3 by Box-Muller:
 *   sqrt(-2 ln u_a) * {cos, sin}(2 pi u_b).
 */
#ifndef VOILA_H
#define VOILA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t voila_status_t;
#define VOILA_OK 0
#define VOILA_ERR_INVALID_ARG 1  /* bad pointer, size or value                     */
#define VOILA_ERR_UNSUPPORTED 2  /* network shape or size with no compiled kernel  */
#define VOILA_ERR_WORKSPACE 3    /* workspace missing or too small                 */
#define VOILA_ERR_DEVICE 4       /* the HIP runtime reported an error              */
#define VOILA_ERR_NUMERIC 5      /* non-finite likelihood or zero total weight     */

#define VOILA_F32 0   /* binary32 network arithmetic (MFMA 32x32x2 f32)               */
#define VOILA_BF16 1  /* bfloat16 operands, binary32 accumulation (MFMA 32x32x16 bf16) */

typedef struct voila_model_s* voila_model_t;

/* One network.  h_dims has n_layers + 1 entries (input width first); h_W[l]
 * and h_b[l] are host arrays of dims[l+1] * dims[l] and dims[l+1] floats. */
typedef struct {
    int32_t n_layers;
    const int32_t* h_dims;
    const float* const* h_W;
    const float* const* h_b;
} voila_mlp_desc_t;

/* The three networks and the spaces they act on.
 *   trans: [d_s + a_width + d_w] -> ... -> d_s   (state increment, s' = s + f_T)
 *   obs:   [d_s + a_width + d_wz] -> ... -> d_o  (may have n_layers == 0: absent)
 *   lik:   [d_s + a_width + d_o] -> ... -> 1     (may have n_layers == 0: absent)
 * a_width = n_actions for a discrete action set (n_actions > 0), else d_a. */
typedef struct {
    int32_t d_s, n_actions, d_a, d_w, d_o, d_wz;
    voila_mlp_desc_t trans, obs, lik;
    int32_t compute;  /* VOILA_F32 or VOILA_BF16 */
} voila_model_desc_t;

/* Library version as major * 10000 + minor * 100 + patch. */
int32_t voila_version(void);
/* Static description of a status code. */
const char* voila_status_string(voila_status_t status);
/* Thread-local description of the last argument error ("" if none). */
const char* voila_last_error(void);

/* [sync] Packs the networks into the on-device layout of the compiled kernels
 * (MFMA operand fragments; one-hot action columns folded into per-action
 * first-layer biases; bfloat16 rounding to nearest even for VOILA_BF16) on
 * device `device` and returns an owned handle.  Host arrays are only read
 * during the call.  Fails with VOILA_ERR_UNSUPPORTED for shapes without a
 * compiled kernel.  Compiled shapes (d_s, actions, d_w, d_o, d_wz, hidden
 * layers x width): (4, 5 discrete, 4, 2, 2, 2 x 64); (4, d_a = 4, 4, 2, 2,
 * 2 x 64); (16, d_a = 4, 16, 32, 32, 3 x 256); (4, 5 discrete, 4, 2, 2,
 * 2 x 1024, VOILA_BF16 only: binary32 activations of that width do not fit
 * in registers); (4, 5 discrete, 4, 2, 2, 4 x 1024, VOILA_BF16 only, the
 * depth and width of the paper's distilled samplers (Sec. 5)): transition
 * and observation networks only -- a likelihood network of that shape is
 * refused -- serving voila_plan, voila_observe and voila_plan_observe (their
 * kernels split every layer of two 32-row tiles over a block's waves);
 * (45, 6 discrete, 45, 36, 36, 4 x 1024, VOILA_BF16 only: the paper's
 * target-finding task (Sec. 5), a 45-dimensional state and 36 lidar bins,
 * whose sampler outputs span two 32-row tiles) with, optionally, the
 * paper's likelihood network of 3 x 256 (a shape of its own): such a model
 * serves voila_plan, voila_observe, voila_plan_observe and voila_update;
 * voila_pw_step, voila_plan_closed_loop and voila_info_nce refuse it with
 * VOILA_ERR_UNSUPPORTED. */
voila_status_t voila_model_create(const voila_model_desc_t* h_desc, int32_t device, voila_model_t* out);
/* [sync] Frees a model (NULL is accepted). */
voila_status_t voila_model_destroy(voila_model_t model);

/* ---------------------------------------------------------------------------
 * plan: Q_k = sum_i w_i G_ik,  G_ik = sum_{t<H} gamma^t r_t  (Sec. 2.1, 2.2, 4.3)
 * For candidate k and particle i: s_0 = S_i, s_{t+1} = s_t + f_T([s_t, a_kt, w]),
 * r_t = -||s_{t+1} - g||^2 (reward_at = 0, default) or -||s_t - g||^2
 * (reward_at = 1).
 * ------------------------------------------------------------------------- */
typedef struct {
    double gamma;           /* discount, 0 <= gamma <= 1                        */
    const float* h_goal;    /* host [d_s] goal g of the reward                  */
    uint64_t seed;          /* Philox key of the rollout noise                  */
    int32_t crn;            /* 1: common random numbers across candidates       */
    int32_t reward_at;      /* 0: reward on arrival s_{t+1}; 1: on s_t          */
    const float* d_noise;   /* device [K][N][H][d_w] explicit noise, or NULL    */
    float* d_traj_out;      /* device [K][N][H][d_s] rollout states s_1..s_H    */
                            /* (caller-owned, written in full), or NULL         */
} voila_plan_opts_t;

/* Bytes of device workspace voila_plan needs for these sizes. */
size_t voila_plan_workspace_size(voila_model_t model, int32_t N, int32_t K, int32_t H);

/* d_states [N][d_s] float; d_belief_w [N] double normalised weights or NULL
 * (uniform 1/N); d_cands int32 [K][H] action indices (discrete) or float
 * [K][H][d_a] (continuous); d_q_out [K] float; d_returns_out [K][N] float or
 * NULL.  1 <= N, 0 <= K, 0 <= H.  A discrete action index outside
 * [0, n_actions) sets *d_status (if given) to VOILA_ERR_INVALID_ARG and is
 * replaced by action 0 (no memory outside the model is read). */
voila_status_t voila_plan(voila_model_t model, const float* d_states, const double* d_belief_w, int32_t N,
                          const void* d_cands, int32_t K, int32_t H, const voila_plan_opts_t* h_opts,
                          void* d_workspace, size_t workspace_bytes, float* d_q_out, float* d_returns_out,
                          int32_t* d_status, void* stream);

/* ---------------------------------------------------------------------------
 * update: b' = tau(b, a, o) by sequential importance resampling (Sec. 3)
 *   s'_i = s_i + f_T([s_i, a, w_i])                 (proposal)
 *   l_i  = l([s'_i, a, o])                          (learned log-likelihood)
 *   x_i  = l_i / lambda (+ log w_i under a weighted prior)
 *   w'_i = exp(x_i - max x) / sum_j exp(x_j - max x)     (binary64)
 *   stats = {log evidence = max x + log sum exp(x - max x) (- log N if uniform),
 *            effective sample size = 1 / sum w'_i^2}
 *   systematic resampling of w' with offset U (see voila_resample);
 *   S_new_j = s'_{idx_j}, uniform weights.
 * ------------------------------------------------------------------------- */
typedef struct {
    double lambda;          /* likelihood temperature, > 0                       */
    uint64_t seed;          /* Philox key of the proposal noise                  */
    uint32_t resample_u;    /* 32-bit offset word of systematic resampling       */
    const float* d_noise;   /* device [N][d_w] explicit proposal noise, or NULL  */
} voila_update_opts_t;

/* Bytes of device workspace voila_update needs for N particles. */
size_t voila_update_workspace_size(voila_model_t model, int32_t N);

/* d_action: device pointer to the executed action, one int32 index (discrete)
 * or d_a floats (continuous); d_obs: device [d_o] floats, the received
 * observation.  Both are read on the device when the stream reaches the call
 * (an observation drawn by voila_observe needs no host round trip, and a
 * captured graph replays with whatever the two buffers hold then).  A discrete
 * action outside [0, n_actions) or a non-finite action or observation value
 * sets *d_status to VOILA_ERR_INVALID_ARG (an out-of-range action is then
 * taken as action 0).  Outputs: d_states_out [N][d_s] float (required);
 * optional d_idx_out [N] int32, d_w_out [N] double (weights before
 * resampling), d_loglik_out [N] float, d_prop_out [N][d_s] float (proposal
 * particles), d_stats_out [2] double, d_status (int32 status word).
 * 1 <= N <= voila_update_max_particles(). */
voila_status_t voila_update(voila_model_t model, const float* d_states, const double* d_prior_w, int32_t N,
                            const void* d_action, const float* d_obs, const voila_update_opts_t* h_opts,
                            void* d_workspace, size_t workspace_bytes, float* d_states_out, int32_t* d_idx_out,
                            double* d_w_out, float* d_loglik_out, float* d_prop_out, double* d_stats_out,
                            int32_t* d_status, void* stream);

/* For callers that cannot allocate device memory (code under hipGraph stream
 * capture, tight serving loops, harnesses that forbid hipMalloc): voila_update
 * with its workspace taken from a fixed array in the library's device code,
 * VOILA_UPDATE_NOALLOC_SCRATCH_BYTES (8 MiB) per device, held from the
 * library's load until the process ends.  Arguments, outputs and results are
 * those of voila_update.  The call allocates nothing (no hipMalloc, no
 * allocating library routine); its first call on a device looks up that
 * device's copy of the array.  N is limited to what the array holds:
 * voila_update_workspace_size(model, N) <= VOILA_UPDATE_NOALLOC_SCRATCH_BYTES
 * (every N up to 65,536 fits for the compiled shapes), else
 * VOILA_ERR_UNSUPPORTED.  Every call on a device shares that device's array:
 * calls that overlap on one device (concurrent streams, or host threads
 * without ordering) race and give undefined results; calls ordered on one
 * stream are safe.  Nothing in the array needs clearing between calls. */
#define VOILA_UPDATE_NOALLOC_SCRATCH_BYTES ((size_t)8 << 20)
voila_status_t voila_update_noalloc(voila_model_t model, const float* d_states, const double* d_prior_w, int32_t N,
                                    const void* d_action, const float* d_obs, const voila_update_opts_t* h_opts,
                                    float* d_states_out, int32_t* d_idx_out, double* d_w_out, float* d_loglik_out,
                                    float* d_prop_out, double* d_stats_out, int32_t* d_status, void* stream);

/* Largest N accepted by voila_update / voila_normalize / voila_resample
 * (beliefs above 8192 particles take a multi-workgroup path through HBM). */
int32_t voila_update_max_particles(void);

/* Bytes of device workspace voila_normalize / voila_resample need for N
 * particles (0 up to 8192 particles, where one workgroup holds the belief). */
size_t voila_weights_workspace_size(int32_t N);

/* ---------------------------------------------------------------------------
 * Stages of update, exported on their own.  They are the reweighting and
 * resampling halves of the particle belief operator tau(b, a, o) of Sec. 2.1
 * (the posterior proportional to the observation likelihood times the
 * predicted belief) as Sec. 3 approximates it with sequential importance
 * resampling, weights exp(l / lambda) as in Sec. 4.2 ("Likelihood Model").
 * ------------------------------------------------------------------------- */
/* Weight normalisation of given log-likelihoods d_loglik [N] float:
 * w'_i and stats exactly as in voila_update (Sec. 2.1: the normalised
 * posterior weights; the log evidence is log Z of the same section, the
 * normaliser of tau).  d_prior_w [N] double or NULL. */
voila_status_t voila_normalize(const float* d_loglik, const double* d_prior_w, int32_t N, double lambda,
                               double* d_w_out, double* d_stats_out, int32_t* d_status, void* d_workspace,
                               size_t workspace_bytes, void* stream);

/* The update's second stage on its own, in one call (the weighting and
 * resampling steps of Sec. 3): weights of given
 * log-likelihoods d_loglik [N] (as voila_normalize) followed by systematic
 * resampling and the optional row gather (as voila_resample), without a
 * round trip of the weights through memory unless d_w_out is given.
 * Workspace as voila_weights_workspace_size(N). */
voila_status_t voila_reweight_resample(const float* d_loglik, const double* d_prior_w, int32_t N, double lambda,
                                       uint32_t U, int32_t* d_idx_out, double* d_w_out, double* d_stats_out,
                                       const float* d_src, float* d_dst, int32_t row_floats, int32_t* d_status,
                                       void* d_workspace, size_t workspace_bytes, void* stream);

/* Fraction bits b(N) = min(32, 52 - ceil(log2 N)) of the quantised weights. */
int32_t voila_resample_bits(int32_t N);

/* Systematic resampling (the resampling step of Sec. 3, whose scheme the
 * paper leaves open; systematic with a quantised, exactly summed weight
 * prefix, so that any summation order gives identical indices) of normalised
 * binary64 weights d_w [N]:
 *   q_i = rint(w_i * N * 2^b)   (ties to even; exact integers)
 *   C_i = q_0 + ... + q_i       (binary64, exact because C_i < 2^53)
 *   u = U >> (32 - b), P_j = j * 2^b + u
 *   idx_j = min{ i : C_i > P_j }, or the last i with q_i > 0 if none.
 * Writes d_idx_out [N] int32; if d_src and d_dst are both non-NULL also
 * gathers rows: d_dst[j][:] = d_src[idx_j][:] for rows of `row_floats`
 * floats.  Negative, non-finite or all-zero weights set d_status. */
voila_status_t voila_resample(const double* d_w, int32_t N, uint32_t U, int32_t* d_idx_out,
                              const float* d_src, float* d_dst, int32_t row_floats, int32_t* d_status,
                              void* d_workspace, size_t workspace_bytes, void* stream);

/* ---------------------------------------------------------------------------
 * observe: o_r = f_Z([s'_r, a, w_Z,r]) (Sec. 4.2, Eq. 5) for n rows sharing
 * one action (d_action: device int32 index or float [d_a], read on the
 * device as in voila_update, with the same status on a bad value); noise
 * explicit (d_noise [n][d_wz]) or Philox stream 4 with counter (r, 0, 0)
 * under `seed`.  d_states [n][d_s] float, d_obs_out [n][d_o] float; the
 * workspace holds the first-layer bias with the action folded in.
 * ------------------------------------------------------------------------- */
size_t voila_observe_workspace_size(voila_model_t model);
voila_status_t voila_observe(voila_model_t model, const float* d_states, int32_t n, const void* d_action,
                             uint64_t seed, const float* d_noise, void* d_workspace, size_t workspace_bytes,
                             float* d_obs_out, int32_t* d_status, void* stream);

/* ---------------------------------------------------------------------------
 * Per-step observations of the plan rollouts: the forward simulation of
 * Sec. 4.3 runs both learned samplers, drawing an observation (Eq. 5) at
 * every simulated step.  It does not enter Q.
 *   o_{k,i,t} = f_Z([s_{k,i,t+1}, a_{k,t}, w_Z]),  k < K, i < N, t < H,
 * with s_{k,i,t+1} the rollout states voila_plan writes to opts.d_traj_out
 * (same N, K, H, candidates, seed and crn).  w_Z is given (d_noise, device
 * [K][N][H][d_wz]) or drawn from Philox stream 4 at counter (i, k, or 0 when
 * crn != 0, t) under key `seed`.
 * d_traj [K][N][H][d_s] float; d_cands as in voila_plan; d_obs_out
 * [K][N][H][d_o] float (caller-owned).  The workspace holds one folded
 * first-layer bias per (candidate, step).  A discrete action outside
 * [0, n_actions) sets *d_status (if given) to VOILA_ERR_INVALID_ARG and is
 * replaced by action 0.  K = 0 or H = 0 writes nothing.
 * ------------------------------------------------------------------------- */
size_t voila_plan_observe_workspace_size(voila_model_t model, int32_t K, int32_t H);
voila_status_t voila_plan_observe(voila_model_t model, const float* d_traj, int32_t N, const void* d_cands,
                                  int32_t K, int32_t H, uint64_t seed, int32_t crn, const float* d_noise,
                                  void* d_workspace, size_t workspace_bytes, float* d_obs_out, int32_t* d_status,
                                  void* stream);

/* ---------------------------------------------------------------------------
 * Contrastive (InfoNCE) objective of the likelihood network, Sec. 4.2,
 * Eq. 6.  For a mini-batch of B tuples (s'_i, a_i, o_i) -- d_states
 * [B][d_s] float, d_actions int32 [B] indices or float [B][d_a], d_obs
 * [B][d_o] float -- the network is evaluated on every state-action against
 * every observation:
 *   l_ij = l([s'_i, a_i, o_j])                    (d_scores_out [B][B] float or NULL)
 *   row_loss_i = log sum_j exp(l_ij) - l_ii        (d_row_loss_out [B] double or NULL)
 *   loss = (1/B) sum_i row_loss_i                  (d_loss_out [1] double or NULL)
 *   G_ij = d loss / d l_ij = (softmax_j(l_i.)_j - [i == j]) / B
 *                                                  (d_grad_out [B][B] float or NULL)
 * Scores are computed in the model's precision; the row reductions run in
 * binary64 (max-shifted) and G is rounded to float.  1 <= B <= 32768.  The
 * workspace (voila_info_nce_workspace_size) holds one folded first-layer
 * bias row per tuple and, where the caller passes NULL, the scores and row
 * losses.  A discrete action outside [0, n_actions) sets *d_status to
 * VOILA_ERR_INVALID_ARG (action 0 is used); a non-finite score sets it to
 * VOILA_ERR_NUMERIC.  All buffers are caller-owned device memory.
 * ------------------------------------------------------------------------- */
size_t voila_info_nce_workspace_size(voila_model_t model, int32_t B);
voila_status_t voila_info_nce(voila_model_t model, const float* d_states, const void* d_actions,
                              const float* d_obs, int32_t B, void* d_workspace, size_t workspace_bytes,
                              float* d_scores_out, double* d_row_loss_out, float* d_grad_out, double* d_loss_out,
                              int32_t* d_status, void* stream);

/* The derivative of the same loss with respect to the likelihood network's
 * parameters: sum over all B^2 pairs of G_ij times the derivative of
 * l([s'_i, a_i, o_j]) (reverse mode through the network, ReLU'(0) = 0),
 * written to d_param_grad_out [voila_info_nce_param_count(model)] float in
 * the layout of the network description (per layer W row-major [out][in],
 * then b); the loss goes to d_loss_out [1] double (or NULL).  Compiled for
 * binary32 likelihood networks with two hidden layers of width 64 over the
 * small shapes (d_s = 4, d_o = 2, five discrete or four continuous action
 * inputs), and for the realistic likelihood network (three hidden layers of
 * width 256 over d_s = 16, d_a = 4, d_o = 32) in binary32 or bfloat16; for
 * other models voila_info_nce_param_count returns 0 and voila_info_nce_grad
 * VOILA_ERR_UNSUPPORTED.  The width-256 form works through chunks of up to
 * 2^19 (binary32) or 2^20 (bfloat16) pairs: each pair's hidden activations
 * and adjoints are stored in the workspace, then the weight derivatives are
 * formed as products over the chunk's pairs (bfloat16 operands: activations
 * and adjoints rounded to bfloat16, binary32 accumulation).  Partial sums
 * are reduced in a fixed order (repeatable).  Status and out-of-range
 * actions as for voila_info_nce (action 0 is used in both passes).
 * Workspace: voila_info_nce_grad_workspace_size (about 2.8 GB for the
 * width-256 network once B^2 reaches the chunk size); for the width-256
 * network a smaller workspace is accepted down to one unit of 32 pairs per
 * chunk (the pairs are then processed in more chunks; the partial sums are
 * grouped differently, so results agree to rounding).
 */
int32_t voila_info_nce_param_count(voila_model_t model);
size_t voila_info_nce_grad_workspace_size(voila_model_t model, int32_t B);
voila_status_t voila_info_nce_grad(voila_model_t model, const float* d_states, const void* d_actions,
                                   const float* d_obs, int32_t B, void* d_workspace, size_t workspace_bytes,
                                   double* d_loss_out, float* d_param_grad_out, int32_t* d_status, void* stream);

/* ---------------------------------------------------------------------------
 * Teacher samplers of the learned generators (Sec. 4.2): a conditional
 * v-prediction denoiser v(c, a, x_tau, tau) run by the deterministic (ODE)
 * DDIM sampler, the sampler a generator is distilled from.  For the
 * transition model c is the state s and x the next state (d_x = d_c = d_s);
 * for the observation model c is the next state and x the observation.
 *
 * voila_denoiser_create packs a denoiser MLP (host arrays as in
 * voila_model_create; input [c, a, x_tau, tau] of width d_c + a_width + d_x
 * + 1, ReLU hidden layers of equal width, linear output v of width d_x;
 * a_width = n_actions for one-hot discrete actions, else d_a).  Compiled
 * shapes (d_x, d_c, hidden layers): (4, 4, 2 x 64) in binary32 or bfloat16;
 * in bfloat16 only (4, 4, 5 x 1024) -- the paper's transition denoiser --,
 * (4, 4, 4 x 1024) -- the distilled sampler's shape, for a one-step cost
 * comparison --, (32, 16, 5 x 512) -- the paper's observation denoiser
 * width and depth -- and (64, 44, 5 x 512) -- the paper's observation
 * denoiser over its 64-dimensional latent observation, conditioned on the
 * 39-dimensional state with a one-hot environment index (its output layer
 * is two 32-row tiles); other shapes return VOILA_ERR_UNSUPPORTED.  The handle
 * owns a device copy of the weights.
 *
 * voila_ddim_sample draws N samples in n_steps uniform steps tau_k = 1 - k/n
 * from d_x1 [N][d_x] (the latent noise at tau = 1) conditioned on d_cond
 * [N][d_c] and one action (h_action: host int32 index or float[d_a]).  With
 * the cosine schedule abar(tau) = cos^2(pi/2 (tau + 0.008)/1.008) /
 * cos^2(pi/2 0.008/1.008), a = abar(tau_k), a' = abar(tau_{k+1}) and v the
 * denoiser's output at (c, a, x, tau_k):
 *   x0 = sqrt(a) x - sqrt(1 - a) v,  eps = sqrt(1 - a) x + sqrt(a) v,
 *   x <- sqrt(a') x0 + sqrt(1 - a') eps,
 * the final x (tau = 0) written to d_out [N][d_x].  The step is applied as
 * x <- x + ((A - 1) x + B v) with A - 1 and B formed in binary64 and rounded
 * to binary32 (A is within binary32 resolution of 1 at large step counts);
 * the network runs in the denoiser's precision.  1 <= n_steps <= 4096; the workspace
 * (voila_ddim_workspace_size) holds the per-step folded biases.
 * ------------------------------------------------------------------------- */
typedef struct voila_denoiser_s* voila_denoiser_t;
voila_status_t voila_denoiser_create(const voila_mlp_desc_t* net, int32_t d_c, int32_t d_x, int32_t n_actions,
                                     int32_t d_a, int32_t compute, int32_t device, voila_denoiser_t* out);
voila_status_t voila_denoiser_destroy(voila_denoiser_t denoiser);
size_t voila_ddim_workspace_size(voila_denoiser_t denoiser, int32_t n_steps);
voila_status_t voila_ddim_sample(voila_denoiser_t denoiser, const float* d_cond, const void* h_action,
                                 const float* d_x1, int32_t N, int32_t n_steps, void* d_workspace,
                                 size_t workspace_bytes, float* d_out, void* stream);

/* ---------------------------------------------------------------------------
 * Soft value and action selection (the log-sum-exp operator L_eta of the
 * preference formulation the planner builds on, Sec. 2.2): for M nodes with
 * K candidate preferences each (d_Q [M][K] float, e.g. voila_plan's Q) and a
 * reference policy (d_log_pi0 [M][K] double log-probabilities, or NULL for
 * the uniform 1/K), with x_k = eta Q_k + log pi0_k in binary64:
 *   V_m = (1/eta) log sum_k exp(x_k)       (max-shifted; d_V_out [M] double)
 *   pi_mk = exp(x_k - eta V_m)             (soft policy; d_pi_out [M][K] or NULL)
 *   best_m = argmax_k x_k, lowest k on ties (d_best_out [M] int32 or NULL).
 * eta > 0.  A NaN or +inf preference sets *d_status to VOILA_ERR_NUMERIC and
 * leaves the node's outputs unwritten.
 * ------------------------------------------------------------------------- */
voila_status_t voila_soft_value(const float* d_Q, const double* d_log_pi0, int32_t M, int32_t K, double eta,
                                double* d_V_out, double* d_pi_out, int32_t* d_best_out, int32_t* d_status,
                                void* stream);

/* ---------------------------------------------------------------------------
 * One-level closed-loop tree with the preference backup of Eq. 1.  For a
 * belief of N uniformly weighted particles, A first actions (d_first: int32
 * [A] indices or float [A][d_a]), n_obs observation branches per first
 * action and K continuation candidates of horizon H (d_cont as voila_plan's
 * candidates):
 *   1. every particle is moved one step under each first action (voila_plan
 *      with horizon 1 and key seed): successors s'_{a,i}, R(b, a) their mean
 *      reward;
 *   2. branch j of action a is a's successor set starting at successor j,
 *      widened once by voila_pw_step (key seed, offset d_U[a n_obs + j]): an
 *      observation drawn at that successor, the set weighted against it and
 *      resampled -- the child belief tau(b, a, o_j);
 *   3. every child belief is valued by the continuation candidates
 *      (voila_plan over all children at once, key seed + 1): Q_child[k] is
 *      the mean return over the child's particles and V_child = L_eta Q_child
 *      with a uniform prior (voila_soft_value);
 *   4. Psi(b, a) = (1/eta) log pi0(a) + R(b, a) + gamma mean_j V_child(a, j)
 *      (d_log_pi0 [A] log-probabilities, or NULL for uniform), V(b) = L_eta
 *      Psi, pi(a) = exp(eta Psi(b, a) - eta V(b)), best = argmax_a Psi.
 * Outputs: d_psi_out [A], d_V_out [1] (double, required); optional d_pi_out
 * [A], d_best_out [1], d_R_out [A], d_Vchild_out [A n_obs] (double / int32)
 * and d_child_out [A n_obs N][d_s] float (the child beliefs).
 * N <= 8192.  The model needs its observation and likelihood networks.
 * ------------------------------------------------------------------------- */
typedef struct {
    double gamma;             /* discount, 0 <= gamma <= 1                        */
    double eta;               /* temperature of L_eta, > 0                        */
    double lambda;            /* likelihood temperature of the child updates, > 0 */
    const float* h_goal;      /* host [d_s] goal of the reward                    */
    uint64_t seed;            /* Philox key (continuation rollouts use seed + 1)  */
    int32_t n_obs;            /* observation branches per first action, >= 1     */
    const double* d_log_pi0;  /* device [A] reference policy, or NULL (uniform)   */
    const uint32_t* d_U;      /* device [A n_obs] resampling offsets              */
} voila_closed_loop_opts_t;

size_t voila_plan_closed_loop_workspace_size(voila_model_t model, int32_t N, int32_t A, int32_t n_obs, int32_t K,
                                             int32_t H);
voila_status_t voila_plan_closed_loop(voila_model_t model, const float* d_states, int32_t N, const void* d_first,
                                      int32_t A, const void* d_cont, int32_t K, int32_t H,
                                      const voila_closed_loop_opts_t* h_opts, void* d_workspace,
                                      size_t workspace_bytes, double* d_psi_out, double* d_V_out, double* d_pi_out,
                                      int32_t* d_best_out, double* d_R_out, double* d_Vchild_out,
                                      float* d_child_out, int32_t* d_status, void* stream);

/* ---------------------------------------------------------------------------
 * Grouped progressive widening (Sec. 4.3): the simulations of a planning
 * pass are grouped by their parent action node and all groups are handled at
 * once.  For each of the M nodes, with successor states d_succ[seg[m] ..
 * seg[m+1]) simulated under the node's action a_m:
 *   1. widen_m = |C(a)| < k_o N(a)^alpha_o in binary64 (N(a) = d_visits[m],
 *      |C(a)| = d_children[m]); a node without branches always widens, a
 *      node with `capacity` branches never does.
 *   2. widening: o = f_Z([s'_first, a_m, w_Z]) (Eq. 5) at the group's first
 *      successor, w_Z from Philox stream 4 at counter (0, m, 0), becomes
 *      branch |C(a)| of the node (d_obs_table[m][branch]) and d_children[m]
 *      grows by one; otherwise an existing branch is taken uniformly:
 *      floor(u |C(a)|), u the uniform of word 0 of Philox at counter
 *      (m, 1, 0, 6 << 16).  Both draws use key `seed`.
 *   3. l_j = l([s'_j, a_m, o_branch]) for the group's successors, weights
 *      w_j = exp(l_j / lambda) / sum over the group (binary64), stats
 *      {log evidence - log n_m, ESS}, systematic resampling of the group
 *      with offset d_U[m] (as voila_resample), d_succ_out rows gathered.
 * d_succ [T][d_s] float; d_seg [M + 1] int32 (seg[0] = 0, non-decreasing,
 * seg[M] = T, every group at most 8192 successors: a group that breaks this
 * sets *d_status to VOILA_ERR_INVALID_ARG and is skipped); d_actions int32
 * [M] or float [M][d_a]; d_visits [M] int32; d_children [M] int32 in
 * [0, capacity] (updated); d_obs_table [M][capacity][d_o] float (updated:
 * the new branch's row); d_U [M] uint32.  Outputs (NULL to skip, except as
 * noted): d_widen_out [M] int32 flags, d_branch_out [M] int32 (-1 for an
 * empty group), d_loglik_out [T] float, d_w_out [T] double, d_stats_out
 * [M][2] double, d_idx_out [T] int32 indices within each group,
 * d_succ_out [T][d_s] float.  Non-finite likelihoods set VOILA_ERR_NUMERIC.
 * ------------------------------------------------------------------------- */
typedef struct {
    double k_o, alpha_o;    /* widening constants, > 0                          */
    double lambda;          /* likelihood temperature, > 0                      */
    uint64_t seed;          /* Philox key of new-branch noise and branch draws  */
    int32_t capacity;       /* branches per node in d_obs_table, >= 1          */
} voila_pw_opts_t;

size_t voila_pw_step_workspace_size(voila_model_t model, int32_t T, int32_t M);
voila_status_t voila_pw_step(voila_model_t model, const float* d_succ, int32_t T, const int32_t* d_seg, int32_t M,
                             const void* d_actions, const int32_t* d_visits, int32_t* d_children,
                             float* d_obs_table, const uint32_t* d_U, const voila_pw_opts_t* h_opts,
                             void* d_workspace, size_t workspace_bytes, int32_t* d_widen_out,
                             int32_t* d_branch_out, float* d_loglik_out, double* d_w_out, double* d_stats_out,
                             int32_t* d_idx_out, float* d_succ_out, int32_t* d_status, void* stream);

/* ---------------------------------------------------------------------------
 * Batches: many independent planning instances (uneven N, K, H; one network
 * each, all of one shape and precision) in one persistent launch, each
 * followed by its own belief update (the per-action-node grouping of
 * simulations of Sec. 4.3 is the paper's analogue).  A batch is built once
 * ([sync]: it uploads the instance tables and cost-sorted work lists and
 * allocates its own device workspace), then run on a stream, or captured
 * once into a hipGraph and replayed.  Per-run inputs -- executed actions,
 * observations and resampling offsets -- are read from device arrays at run
 * time, so a captured graph replays with whatever those arrays hold.
 * Only network shapes whose kernels stage the whole network in LDS (hidden
 * width <= 64) can be batched; N <= voila_update_max_particles() when the
 * update is used.
 * ------------------------------------------------------------------------- */
typedef struct voila_batch_s* voila_batch_t;

typedef struct {
    voila_model_t model;       /* this instance's networks                        */
    const float* d_states;     /* [N][d_s] belief particles                        */
    const double* d_belief_w;  /* [N] normalised weights or NULL (uniform)         */
    int32_t N;
    const void* d_cands;       /* int32 [K][H] or float [K][H][d_a]                */
    int32_t K, H;
    double gamma;
    const float* h_goal;       /* host [d_s], read during voila_batch_create       */
    uint64_t seed;             /* Philox key of this instance's rollout noise      */
    int32_t crn, reward_at;
    float* d_q_out;            /* [K]                                              */
    float* d_returns_out;      /* [K][N] or NULL                                   */
    /* belief update of this instance (VOILA_BATCH_UPDATE) */
    double lambda;
    uint64_t update_seed;      /* Philox key of the proposal noise                 */
    float* d_states_out;       /* [N][d_s] (required for the update)               */
    int32_t* d_idx_out;        /* [N] or NULL                                      */
    double* d_w_out;           /* [N] or NULL                                      */
    double* d_stats_out;       /* [2] or NULL                                      */
} voila_batch_item_t;

/* Schedule of the persistent batch kernels (autotuned by the Python layer). */
typedef struct {
    int32_t waves_per_block;   /* 1..8 waves of 64 lanes per workgroup (default 4)             */
    int32_t blocks_per_cu;     /* resident workgroups per CU; 0 = as many as fit (default)     */
    int32_t dynamic;           /* 1 = atomic queue over cost-sorted items (default), 0 = static */
} voila_batch_tuning_t;

#define VOILA_BATCH_PLAN 1
#define VOILA_BATCH_UPDATE 2

/* [sync] h_tuning may be NULL (defaults). */
voila_status_t voila_batch_create(const voila_batch_item_t* h_items, int32_t n_items,
                                  const voila_batch_tuning_t* h_tuning, voila_batch_t* out);
/* [sync] Frees the batch, its workspace and its graph (NULL accepted). */
voila_status_t voila_batch_destroy(voila_batch_t batch);
/* Enqueues plan and/or update (what = VOILA_BATCH_PLAN | VOILA_BATCH_UPDATE) of
 * every instance.  For the update: d_actions int32 [n] or float [n][d_a],
 * d_obs float [n][d_o], d_resample_u uint32 [n] (instance order). */
voila_status_t voila_batch_run(voila_batch_t batch, int32_t what, const void* d_actions, const float* d_obs,
                               const uint32_t* d_resample_u, int32_t* d_status, void* stream);
/* [sync] Captures voila_batch_run with these arguments into a hipGraph owned
 * by the batch (replacing a previous one). */
voila_status_t voila_batch_capture(voila_batch_t batch, int32_t what, const void* d_actions, const float* d_obs,
                                   const uint32_t* d_resample_u, int32_t* d_status);
/* Launches the captured graph on `stream`. */
voila_status_t voila_batch_replay(voila_batch_t batch, void* stream);

/* ---------------------------------------------------------------------------
 * Gradients through rollouts (adjoint with step checkpointing).  Rollout b:
 * s_0 = S0_b, s_{t+1} = s_t + f_T([s_t, a_{b,t}, w_{b,t}]).  Objectives:
 *   VOILA_OBJ_DISTILL  L = 1/(B H) sum_b sum_{t=1..H} ||s_{b,t} - T_{b,t}||^2:
 *                      the distillation loss of Eq. 3 applied along
 *                      free-running rollouts against teacher states T;
 *   VOILA_OBJ_RETURN   J = 1/B sum_b sum_{t<H} gamma^t (-||s_{b,t+1} - g||^2):
 *                      the mean discounted return of Sec. 2.1.
 * Outputs: the objective, its gradient with respect to the transition
 * network's parameters (W1, b1, W2, b2, W3, b3 concatenated, each as
 * nn.Linear stores it) and, for continuous actions, with respect to the
 * action sequences.  The forward pass stores a checkpoint every `checkpoint`
 * steps; the reverse sweep recomputes each segment from its checkpoint.
 * Binary32 models of networks with two hidden layers of width 64 only
 * (otherwise VOILA_ERR_UNSUPPORTED).  Results are deterministic (fixed-order
 * reductions).
 * ------------------------------------------------------------------------- */
#define VOILA_OBJ_DISTILL 0
#define VOILA_OBJ_RETURN 1

typedef struct {
    int32_t B, H;               /* rollouts (>= 1), horizon (0..64)                            */
    int32_t checkpoint;         /* checkpoint interval in steps (>= 1)                          */
    const float* d_s0;          /* [B][d_s]                                                     */
    const void* d_actions;      /* discrete: int32 [B][H]; continuous: float [B/particles][H][d_a] */
    int32_t particles;          /* rollouts per continuous sequence (multiple of 32 when the
                                   action gradient is requested); ignored for discrete actions  */
    const float* d_noise;       /* [B][H][d_w] or NULL: Philox stream 3, counter (b, 0, t)       */
    uint64_t seed;
    int32_t objective;          /* VOILA_OBJ_DISTILL or VOILA_OBJ_RETURN                         */
    const float* d_targets;     /* [B][H][d_s] teacher states s_1..s_H (distillation)           */
    double gamma;               /* return objective                                             */
    const float* h_goal;        /* host [d_s] (return objective)                                */
    float* d_loss_out;          /* [1] or NULL                                                  */
    float* d_grad_params;       /* [voila_grad_param_count(model)] or NULL                      */
    float* d_grad_actions;      /* same layout as d_actions (continuous) or NULL                */
} voila_grad_opts_t;

/* Number of parameters of the transition network (length of d_grad_params). */
int32_t voila_grad_param_count(voila_model_t model);
size_t voila_rollout_grad_workspace_size(voila_model_t model, const voila_grad_opts_t* h_opts);
voila_status_t voila_rollout_grad(voila_model_t model, const voila_grad_opts_t* h_opts, void* d_workspace,
                                  size_t workspace_bytes, void* stream);

/* ---------------------------------------------------------------------------
 * Test hook: the counter-based draws the kernels consume.  Fills
 * d_out [n][d] float with the normals of counters (c0_base + r, c1, c2) of
 * `stream` for r < n, and d_words [n][4 * ceil(d/4)] uint32 (may be NULL) with
 * the raw Philox words.
 * ------------------------------------------------------------------------- */
voila_status_t voila_philox_normals(uint64_t seed, uint32_t c0_base, uint32_t c1, uint32_t c2, uint32_t stream_id,
                                    int32_t n, int32_t d, float* d_out, uint32_t* d_words, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* VOILA_H */
