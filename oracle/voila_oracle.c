/*
 * voila_oracle.c -- plain FP64 CPU reference of the VOiLA planning hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test-suite, the smoke check and the benchmark's
 * CPU-baseline leg do.  It shares no header, helper, table or constant with
 * the HIP implementation: every step below is written out from the paper
 * (Hoerger et al., "VOiLA: Vectorized Online Planning with Learned Diffusion
 * Models for POMDP Agents") and from the published definitions it relies on.
 *
 * What it computes (all arithmetic in IEEE binary64, sums in ascending index
 * order, built with -ffp-contract=off so no fused multiply-adds appear):
 *
 *   mlp       Feed-forward generator / likelihood network: affine layers with
 *             ReLU between them, linear output layer (Sec. 4.2, Eq. 2 and
 *             Eq. 5 for the samplers, Sec. 4.2 "Likelihood Model" for l).
 *   plan      Monte-Carlo estimate of the discounted return of open-loop
 *             action sequences from a particle belief: the expected reward
 *             R(b,a) is a Monte-Carlo average over belief particles (Sec. 2.1,
 *             Sec. 2.2 below Eq. 1), forward simulation draws successor
 *             states from the learned transition sampler s'=f_T(s,a,w_T),
 *             w_T ~ N(0,I) (Eq. 2, Sec. 4.3), and the return is discounted
 *             by gamma^t (Sec. 2.1, value definition).
 *   update    Sequential-importance-resampling belief update (Sec. 3, last
 *             paragraph): proposal particles from f_T, weights
 *             exp(l(s',a,o)/lambda) from the likelihood network (Sec. 4.2,
 *             "Likelihood Model", last paragraph), normalisation of the
 *             weights (the proportionality in the belief operator tau of
 *             Sec. 2.1), then resampling.
 *   resample  Systematic resampling on weights quantised to integer
 *             multiples of 2^-b of a particle (the paper leaves the scheme
 *             open; this reading makes every prefix sum exact in binary64).
 *   observe   Observation sampler z=f_Z(s',a,w_Z) (Eq. 5).
 *   pw_step   Progressive widening of many action nodes at once (Sec. 4.3):
 *             the widening test, a new or reused observation branch per node,
 *             and each node's successors weighted and resampled as a group.
 *   soft_value  The log-sum-exp operator of the preference formulation
 *             (Sec. 2.2): soft value, soft policy and greedy action of the
 *             candidates' preferences, with a reference-policy prior.
 *   info_nce  The contrastive objective of the likelihood network (Sec. 4.2,
 *             Eq. 6): scores of all B x B state-action / observation pairs of
 *             a mini-batch, per-row log-sum-exp losses, their mean, its
 *             derivative with respect to every score and, by reverse mode
 *             through the network, with respect to its parameters.
 *   ddim      The teacher sampler of the transition model (Sec. 4.2): the
 *             deterministic DDIM sampler (Song, Meng, Ermon, "Denoising
 *             diffusion implicit models", ICLR 2021) of a v-prediction
 *             denoiser (Salimans and Ho, "Progressive distillation for fast
 *             sampling of diffusion models", ICLR 2022) under the cosine
 *             schedule, from the latent noise at tau = 1 to a next state.
 *   plan_steps  The states of the plan rollouts and an observation drawn
 *             from f_Z at every step (Sec. 4.3 forward-simulates with both
 *             learned samplers).
 *   philox    Philox4x32-10 counter-based generator (Salmon, Moraes, Dror,
 *             Shaw, "Parallel random numbers: as easy as 1, 2, 3", SC'11),
 *             Box-Muller transform for N(0,1) draws.
 *
 * Input vector convention: x = [s, a, w] where a discrete action is one-hot
 * over the action set (0-based index) and a continuous action is used as
 * given; the likelihood network takes [s', a, o]; the observation sampler
 * takes [s', a, w_Z].  Layer parameters are packed per layer as W (rows =
 * outputs, row-major, i.e. W[n*in + k]) followed by the bias b[n].
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_OK 0
#define OR_ERR_ARG 1
#define OR_ERR_NUMERIC 2

#define OR_MAX_WIDTH 4096
#define OR_MAX_LAYERS 8

/* ------------------------------------------------------------------------- */
/* Philox4x32-10 (SC'11 paper: Philox-4x32 with R = 10 rounds).              */
/* One round multiplies the even words by the two published multipliers,    */
/* xors the high halves into the odd words together with the round key, and */
/* permutes; the key is bumped by the two published Weyl constants between  */
/* rounds.                                                                   */
/* ------------------------------------------------------------------------- */
static const uint32_t PHILOX_MUL0 = 0xD2511F53u;
static const uint32_t PHILOX_MUL1 = 0xCD9E8D57u;
static const uint32_t PHILOX_WEYL0 = 0x9E3779B9u;
static const uint32_t PHILOX_WEYL1 = 0xBB67AE85u;

void or_philox4x32_10(const uint32_t counter[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = counter[0], c1 = counter[1], c2 = counter[2], c3 = counter[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        uint64_t prod0 = (uint64_t)PHILOX_MUL0 * (uint64_t)c0;
        uint64_t prod1 = (uint64_t)PHILOX_MUL1 * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(prod0 >> 32), lo0 = (uint32_t)prod0;
        uint32_t hi1 = (uint32_t)(prod1 >> 32), lo1 = (uint32_t)prod1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
        k0 += PHILOX_WEYL0;
        k1 += PHILOX_WEYL1;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Uniform on the open interval (0,1) from the top 23 bits of a word:
 * u = (2*(x >> 9) + 1) * 2^-24.  The value has at most 24 significant bits,
 * so it is exact in binary32 as well as binary64, and it is never 0 or 1. */
double or_uniform(uint32_t x)
{
    return (2.0 * (double)(x >> 9) + 1.0) * 0x1p-24;
}

/* d standard normal draws for one counter triple (c0,c1,c2) of a stream.
 * Block j of four draws uses counter (c0, c1, c2, (stream << 16) | j); its
 * four words give two uniform pairs (u0,u1), (u2,u3), each turned into two
 * normals by the Box-Muller transform:
 *   z_a = sqrt(-2 ln u_a) cos(2 pi u_b),  z_b = sqrt(-2 ln u_a) sin(2 pi u_b). */
void or_normals(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t stream,
                int d, double* z)
{
    const double two_pi = 6.283185307179586476925286766559;
    uint32_t key[2] = {(uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32)};
    for (int block = 0; 4 * block < d; ++block) {
        uint32_t ctr[4] = {c0, c1, c2, (stream << 16) | (uint32_t)block};
        uint32_t w[4];
        or_philox4x32_10(ctr, key, w);
        double u0 = or_uniform(w[0]), u1 = or_uniform(w[1]);
        double u2 = or_uniform(w[2]), u3 = or_uniform(w[3]);
        double r0 = sqrt(-2.0 * log(u0));
        double r1 = sqrt(-2.0 * log(u2));
        double four[4] = {r0 * cos(two_pi * u1), r0 * sin(two_pi * u1),
                          r1 * cos(two_pi * u3), r1 * sin(two_pi * u3)};
        for (int j = 0; j < 4; ++j)
            if (4 * block + j < d) z[4 * block + j] = four[j];
    }
}

/* ------------------------------------------------------------------------- */
/* bfloat16 emulation: round to 8 significant bits, ties to even.           */
/* ------------------------------------------------------------------------- */
double or_round_bf16(double x)
{
    if (x == 0.0 || !isfinite(x)) return x;
    int e;
    double m = frexp(x, &e);           /* x = m * 2^e, 0.5 <= |m| < 1 */
    double scaled = ldexp(m, 8);       /* 128 <= |scaled| < 256       */
    double r = nearbyint(scaled);      /* default mode: ties to even  */
    return ldexp(r, e - 8);
}

/* ------------------------------------------------------------------------- */
/* Multilayer perceptron (Sec. 4.2; layer widths Sec. 5.2).                  */
/* ------------------------------------------------------------------------- */
static size_t mlp_param_count(int n_layers, const int* dims)
{
    size_t n = 0;
    for (int l = 0; l < n_layers; ++l) n += (size_t)dims[l + 1] * dims[l] + dims[l + 1];
    return n;
}

static int mlp_check(int n_layers, const int* dims)
{
    if (n_layers < 1) return OR_ERR_ARG;
    for (int l = 0; l <= n_layers; ++l)
        if (dims[l] < 1 || dims[l] > OR_MAX_WIDTH) return OR_ERR_ARG;
    return OR_OK;
}

/* y = MLP(x).  Hidden layers: h = max(W h_prev + b, 0); output layer linear.
 * With bf16 != 0 each layer input is first rounded to bfloat16, and the
 * weights must already be bfloat16 values (round_weights; biases,
 * accumulation and outputs stay binary64). */
static void mlp_forward(int n_layers, const int* dims, const double* params,
                        const double* x, double* y, int bf16)
{
    double buf0[OR_MAX_WIDTH], buf1[OR_MAX_WIDTH];
    double* in = buf0;
    double* out = buf1;
    for (int k = 0; k < dims[0]; ++k) in[k] = bf16 ? or_round_bf16(x[k]) : x[k];
    const double* p = params;
    for (int l = 0; l < n_layers; ++l) {
        int n_in = dims[l], n_out = dims[l + 1];
        const double* W = p;
        const double* b = p + (size_t)n_out * n_in;
        for (int n = 0; n < n_out; ++n) {
            double acc = 0.0;
            for (int k = 0; k < n_in; ++k) {
                acc += W[(size_t)n * n_in + k] * in[k];
            }
            acc += b[n];
            if (l < n_layers - 1) {
                if (acc < 0.0) acc = 0.0;
                if (bf16) acc = or_round_bf16(acc);
            }
            out[n] = acc;
        }
        p += (size_t)n_out * n_in + n_out;
        double* t = in; in = out; out = t;
    }
    for (int n = 0; n < dims[n_layers]; ++n) y[n] = in[n];
}

/* Copy of a parameter vector with every weight rounded to bfloat16 and the
 * biases unchanged (the bfloat16 emulation rounds each weight once). */
static double* round_weights(int n_layers, const int* dims, const double* params)
{
    double* out = (double*)malloc(sizeof(double) * (mlp_param_count(n_layers, dims) + 1));
    if (!out) return NULL;
    const double* p = params;
    double* q = out;
    for (int l = 0; l < n_layers; ++l) {
        size_t nw = (size_t)dims[l + 1] * dims[l];
        for (size_t j = 0; j < nw; ++j) q[j] = or_round_bf16(p[j]);
        for (int j = 0; j < dims[l + 1]; ++j) q[nw + j] = p[nw + j];
        p += nw + dims[l + 1];
        q += nw + dims[l + 1];
    }
    return out;
}

int or_mlp(int n_layers, const int* dims, const double* params, int rows,
           const double* X, double* Y, int bf16)
{
    if (mlp_check(n_layers, dims) != OR_OK || rows < 0) return OR_ERR_ARG;
    double* rw = bf16 ? round_weights(n_layers, dims, params) : NULL;
    if (bf16 && !rw) return OR_ERR_ARG;
    const double* P = bf16 ? rw : params;
    #pragma omp parallel for schedule(static)
    for (int r = 0; r < rows; ++r)
        mlp_forward(n_layers, dims, P, X + (size_t)r * dims[0], Y + (size_t)r * dims[n_layers], bf16);
    free(rw);
    return OR_OK;
}

/* ------------------------------------------------------------------------- */
/* Generator model: transition sampler f_T (Eq. 2, used with a residual     */
/* state update s' = s + f_T(x), the increment form of Eq. 2), observation  */
/* sampler f_Z (Eq. 5) and likelihood l (Sec. 4.2).                         */
/* ------------------------------------------------------------------------- */
typedef struct {
    int d_s;        /* state dimension                                   */
    int n_actions;  /* > 0: discrete action set fed one-hot; 0: continuous */
    int d_a;        /* continuous action dimension (ignored if discrete)  */
    int d_w;        /* transition-noise dimension                         */
    int d_o;        /* observation dimension                              */
    int d_wz;       /* observation-noise dimension                        */
    int residual;   /* 1: s' = s + f_T(x); 0: s' = f_T(x)                 */
    int t_layers; const int* t_dims; const double* t_params;
    int z_layers; const int* z_dims; const double* z_params;
    int l_layers; const int* l_dims; const double* l_params;
} or_model;

/* The model with bfloat16-rounded weights for the bfloat16 emulation
 * (m itself when bf16 == 0).  release_rounded frees the copies. */
typedef struct {
    or_model m;
    double* buf[3];
} rounded_model;

static const or_model* rounded(const or_model* m, int bf16, rounded_model* r)
{
    r->buf[0] = r->buf[1] = r->buf[2] = NULL;
    if (!bf16) return m;
    r->m = *m;
    if (m->t_params && m->t_layers > 0 && mlp_check(m->t_layers, m->t_dims) == OR_OK)
        r->m.t_params = r->buf[0] = round_weights(m->t_layers, m->t_dims, m->t_params);
    if (m->z_params && m->z_layers > 0 && mlp_check(m->z_layers, m->z_dims) == OR_OK)
        r->m.z_params = r->buf[1] = round_weights(m->z_layers, m->z_dims, m->z_params);
    if (m->l_params && m->l_layers > 0 && mlp_check(m->l_layers, m->l_dims) == OR_OK)
        r->m.l_params = r->buf[2] = round_weights(m->l_layers, m->l_dims, m->l_params);
    return &r->m;
}

static void release_rounded(rounded_model* r)
{
    for (int j = 0; j < 3; ++j) free(r->buf[j]);
}

static int action_width(const or_model* m)
{
    return m->n_actions > 0 ? m->n_actions : m->d_a;
}

/* Writes the action part of an input vector. */
static void put_action(const or_model* m, double* dst, int a_disc, const double* a_cont)
{
    if (m->n_actions > 0) {
        for (int j = 0; j < m->n_actions; ++j) dst[j] = (j == a_disc) ? 1.0 : 0.0;
    } else {
        for (int j = 0; j < m->d_a; ++j) dst[j] = a_cont[j];
    }
}

/* One transition draw s_next = s + f_T([s, a, w]) (or f_T(...) if not residual). */
static void transition(const or_model* m, const double* s, int a_disc, const double* a_cont,
                       const double* w, double* s_next, int bf16)
{
    double x[OR_MAX_WIDTH], d[OR_MAX_WIDTH];
    int aw = action_width(m);
    for (int j = 0; j < m->d_s; ++j) x[j] = s[j];
    put_action(m, x + m->d_s, a_disc, a_cont);
    for (int j = 0; j < m->d_w; ++j) x[m->d_s + aw + j] = w[j];
    mlp_forward(m->t_layers, m->t_dims, m->t_params, x, d, bf16);
    for (int j = 0; j < m->d_s; ++j) s_next[j] = m->residual ? s[j] + d[j] : d[j];
}

static int model_check(const or_model* m)
{
    if (m->d_s < 1 || m->d_w < 0 || m->n_actions < 0) return OR_ERR_ARG;
    if (m->n_actions == 0 && m->d_a < 0) return OR_ERR_ARG;
    if (mlp_check(m->t_layers, m->t_dims) != OR_OK) return OR_ERR_ARG;
    if (m->t_dims[0] != m->d_s + action_width(m) + m->d_w) return OR_ERR_ARG;
    if (m->t_dims[m->t_layers] != m->d_s) return OR_ERR_ARG;
    return OR_OK;
}

/* Reward R(s) = -||s - g||^2 (action independent). */
static double reward(int d_s, const double* s, const double* goal)
{
    double acc = 0.0;
    for (int j = 0; j < d_s; ++j) {
        double e = s[j] - goal[j];
        acc += e * e;
    }
    return -acc;
}

/* Noise of the plan rollouts: stream 3, counter (particle, candidate or 0
 * under common random numbers, step). */
#define OR_STREAM_PLAN 3u
#define OR_STREAM_OBS 4u
#define OR_STREAM_UPDATE 5u

/* Discounted return of rollout (k, i):
 *   s_0 = S_i;  s_{t+1} = s_t + f_T([s_t, a_{k,t}, w_{k,i,t}]);
 *   reward_at == 0: r_t = R(s_{t+1})   (reward on arrival, default)
 *   reward_at == 1: r_t = R(s_t)       (reward of the state acted from)
 *   G = sum_{t<H} gamma^t r_t.
 * traj (NULL or [H][d_s]) receives s_1 .. s_H. */
static double rollout_return(const or_model* m, const double* S_i, int k, int i, int N, int H,
                             const int32_t* cand_disc, const double* cand_cont,
                             double gamma, const double* goal, int reward_at,
                             const double* noise, uint64_t seed, int crn, int bf16, double* traj)
{
    double s[OR_MAX_WIDTH], s_next[OR_MAX_WIDTH], w[OR_MAX_WIDTH];
    for (int j = 0; j < m->d_s; ++j) s[j] = S_i[j];
    double G = 0.0, disc = 1.0;
    for (int t = 0; t < H; ++t) {
        if (noise) {
            const double* src = noise + (((size_t)k * N + i) * H + t) * m->d_w;
            for (int j = 0; j < m->d_w; ++j) w[j] = src[j];
        } else {
            or_normals(seed, (uint32_t)i, crn ? 0u : (uint32_t)k, (uint32_t)t, OR_STREAM_PLAN, m->d_w, w);
        }
        int a_disc = cand_disc ? cand_disc[(size_t)k * H + t] : 0;
        const double* a_cont = cand_cont ? cand_cont + ((size_t)k * H + t) * m->d_a : NULL;
        transition(m, s, a_disc, a_cont, w, s_next, bf16);
        double r = reward_at ? reward(m->d_s, s, goal) : reward(m->d_s, s_next, goal);
        G += disc * r;
        disc *= gamma;
        for (int j = 0; j < m->d_s; ++j) s[j] = s_next[j];
        if (traj)
            for (int j = 0; j < m->d_s; ++j) traj[(size_t)t * m->d_s + j] = s_next[j];
    }
    return G;
}

/* Neumaier-compensated sum of a[i] * b[i] (b may be NULL: uniform 1/n). */
static double weighted_sum(int n, const double* a, const double* b, size_t stride)
{
    double sum = 0.0, comp = 0.0;
    for (int i = 0; i < n; ++i) {
        double term = a[(size_t)i * stride] * (b ? b[i] : 1.0 / (double)n);
        double t = sum + term;
        if (fabs(sum) >= fabs(term)) comp += (sum - t) + term;
        else comp += (term - t) + sum;
        sum = t;
    }
    return sum + comp;
}

int or_plan(const or_model* m0, int N, const double* S, const double* belief_w,
            int K, int H, const int32_t* cand_disc, const double* cand_cont,
            double gamma, const double* goal, int reward_at,
            const double* noise, uint64_t seed, int crn, int bf16,
            double* Q, double* G)
{
    if (model_check(m0) != OR_OK || N < 1 || K < 0 || H < 0) return OR_ERR_ARG;
    if (m0->n_actions > 0 ? !cand_disc : !cand_cont) return OR_ERR_ARG;
    double* Gbuf = G ? G : (double*)malloc(sizeof(double) * (size_t)K * N + 1);
    if (!Gbuf) return OR_ERR_ARG;
    rounded_model rm;
    const or_model* m = rounded(m0, bf16, &rm);
    #pragma omp parallel for schedule(dynamic, 16)
    for (long r = 0; r < (long)K * N; ++r) {
        int k = (int)(r / N), i = (int)(r % N);
        Gbuf[r] = rollout_return(m, S + (size_t)i * m->d_s, k, i, N, H, cand_disc, cand_cont,
                                 gamma, goal, reward_at, noise, seed, crn, bf16, NULL);
    }
    for (int k = 0; k < K; ++k) Q[k] = weighted_sum(N, Gbuf + (size_t)k * N, belief_w, 1);
    if (!G) free(Gbuf);
    release_rounded(&rm);
    return OR_OK;
}

/* Returns of selected rollouts (k_list[p], i_list[p]) only -- used to check
 * sampled outputs of full-size workloads. */
int or_rollouts(const or_model* m0, int N, const double* S, int K, int H,
                const int32_t* cand_disc, const double* cand_cont,
                double gamma, const double* goal, int reward_at,
                uint64_t seed, int crn, int bf16,
                int n_pairs, const int32_t* k_list, const int32_t* i_list, double* G_out)
{
    if (model_check(m0) != OR_OK || N < 1 || K < 0 || H < 0 || n_pairs < 0) return OR_ERR_ARG;
    for (int p = 0; p < n_pairs; ++p)
        if (k_list[p] < 0 || k_list[p] >= K || i_list[p] < 0 || i_list[p] >= N) return OR_ERR_ARG;
    rounded_model rm;
    const or_model* m = rounded(m0, bf16, &rm);
    #pragma omp parallel for schedule(dynamic, 1)
    for (int p = 0; p < n_pairs; ++p) {
        int k = k_list[p], i = i_list[p];
        G_out[p] = rollout_return(m, S + (size_t)i * m->d_s, k, i, N, H, cand_disc, cand_cont,
                                  gamma, goal, reward_at, NULL, seed, crn, bf16, NULL);
    }
    release_rounded(&rm);
    return OR_OK;
}

/* Weighted sum of given returns: Q = sum_i w_i G_i (w NULL: 1/N). */
double or_weighted_mean(int n, const double* G, const double* w)
{
    return weighted_sum(n, G, w, 1);
}

/* ------------------------------------------------------------------------- */
/* Belief update (Sec. 3; Sec. 4.2 likelihood model; Sec. 2.1 operator tau). */
/* ------------------------------------------------------------------------- */

/* Weight normalisation.  x_i = l_i / lambda (+ log w_i for a weighted prior),
 * m = max x_i, e_i = exp(x_i - m), S = sum e_i, w'_i = e_i / S;
 * stats[0] = log evidence = m + log S (- log N under a uniform prior),
 * stats[1] = effective sample size 1 / sum w'_i^2. */
int or_normalize(int N, const double* loglik, const double* prior_w, double lambda,
                 double* w_out, double* stats)
{
    if (N < 1 || !(lambda > 0.0)) return OR_ERR_ARG;
    double* x = (double*)malloc(sizeof(double) * (size_t)N);
    if (!x) return OR_ERR_ARG;
    double mx = -INFINITY;
    for (int i = 0; i < N; ++i) {
        if (!isfinite(loglik[i])) { free(x); return OR_ERR_NUMERIC; }
        x[i] = loglik[i] / lambda;
        if (prior_w) x[i] += log(prior_w[i]);
        if (x[i] > mx) mx = x[i];
    }
    if (!isfinite(mx)) { free(x); return OR_ERR_NUMERIC; }
    double sum = 0.0, comp = 0.0;
    for (int i = 0; i < N; ++i) {
        x[i] = exp(x[i] - mx);
        double t = sum + x[i];
        if (fabs(sum) >= fabs(x[i])) comp += (sum - t) + x[i];
        else comp += (x[i] - t) + sum;
        sum = t;
    }
    double S = sum + comp;
    double sq = 0.0;
    for (int i = 0; i < N; ++i) {
        w_out[i] = x[i] / S;
        sq += w_out[i] * w_out[i];
    }
    if (stats) {
        stats[0] = mx + log(S) - (prior_w ? 0.0 : log((double)N));
        stats[1] = 1.0 / sq;
    }
    free(x);
    return OR_OK;
}

/* Fraction bits of the quantised weights: b(N) = min(32, 52 - ceil(log2 N)),
 * so every partial sum of the integers q_i stays below 2^53. */
int or_resample_bits(int N)
{
    int c = 0;
    while (((int64_t)1 << c) < (int64_t)N) ++c;
    return 52 - c < 32 ? 52 - c : 32;
}

/* Systematic resampling on quantised weights.
 *   q_i = rint(w_i * N * 2^b)       (one binary64 product, ties to even)
 *   C_i = q_0 + ... + q_i           (integers below 2^53: exact)
 *   u   = U >> (32 - b),  P_j = j * 2^b + u
 *   idx_j = smallest i with C_i > P_j; if none, the last i with q_i > 0.
 * This is systematic resampling with offset u / 2^b in [0,1) on the weights
 * rounded to multiples of 2^-b particles. */
int or_resample(int N, const double* w, uint32_t U, int32_t* idx)
{
    if (N < 1) return OR_ERR_ARG;
    int b = or_resample_bits(N);
    double scale = ldexp((double)N, b);
    double* C = (double*)malloc(sizeof(double) * (size_t)N);
    if (!C) return OR_ERR_ARG;
    double run = 0.0;
    int last_positive = -1;
    for (int i = 0; i < N; ++i) {
        if (!(w[i] >= 0.0) || !isfinite(w[i])) { free(C); return OR_ERR_NUMERIC; }
        double q = nearbyint(w[i] * scale);
        if (q > 0.0) last_positive = i;
        run += q;
        C[i] = run;
    }
    if (last_positive < 0) { free(C); return OR_ERR_NUMERIC; }
    double u = (double)(U >> (32 - b));
    double step = ldexp(1.0, b);
    int i = 0;
    for (int j = 0; j < N; ++j) {
        double P = (double)j * step + u;
        while (i < N && !(C[i] > P)) ++i;
        idx[j] = (i < N) ? i : last_positive;
    }
    free(C);
    return OR_OK;
}

/* Full SIR update for one executed action a and received observation o.
 *   s'_i = s_i + f_T([s_i, a, w_i])          w_i: given noise or stream 5,
 *                                              counter (i, 0, 0)
 *   l_i  = l([s'_i, a, o])
 *   w'   = normalise(l / lambda, prior)
 *   idx  = resample(w', U);  S_new_j = s'_{idx_j}
 * Outputs may be NULL except S_new. */
int or_update(const or_model* m0, int N, const double* S, const double* prior_w,
              int a_disc, const double* a_cont, const double* o, double lambda,
              const double* noise, uint64_t seed, uint32_t U, int bf16,
              double* S_prop, double* loglik, double* w_out, double* stats,
              int32_t* idx, double* S_new)
{
    if (model_check(m0) != OR_OK || N < 1) return OR_ERR_ARG;
    if (mlp_check(m0->l_layers, m0->l_dims) != OR_OK) return OR_ERR_ARG;
    if (m0->l_dims[0] != m0->d_s + action_width(m0) + m0->d_o || m0->l_dims[m0->l_layers] != 1) return OR_ERR_ARG;
    if (m0->n_actions > 0 ? (a_disc < 0 || a_disc >= m0->n_actions) : !a_cont) return OR_ERR_ARG;
    int d_s = m0->d_s, aw = action_width(m0);
    double* sp = (double*)malloc(sizeof(double) * (size_t)N * d_s);
    double* ll = (double*)malloc(sizeof(double) * (size_t)N);
    double* wn = (double*)malloc(sizeof(double) * (size_t)N);
    int32_t* ix = (int32_t*)malloc(sizeof(int32_t) * (size_t)N);
    if (!sp || !ll || !wn || !ix) { free(sp); free(ll); free(wn); free(ix); return OR_ERR_ARG; }
    rounded_model rm;
    const or_model* m = rounded(m0, bf16, &rm);
    #pragma omp parallel for schedule(static)
    for (int i = 0; i < N; ++i) {
        double w[OR_MAX_WIDTH], x[OR_MAX_WIDTH], y[1];
        if (noise) {
            for (int j = 0; j < m->d_w; ++j) w[j] = noise[(size_t)i * m->d_w + j];
        } else {
            or_normals(seed, (uint32_t)i, 0u, 0u, OR_STREAM_UPDATE, m->d_w, w);
        }
        transition(m, S + (size_t)i * d_s, a_disc, a_cont, w, sp + (size_t)i * d_s, bf16);
        for (int j = 0; j < d_s; ++j) x[j] = sp[(size_t)i * d_s + j];
        put_action(m, x + d_s, a_disc, a_cont);
        for (int j = 0; j < m->d_o; ++j) x[d_s + aw + j] = o[j];
        mlp_forward(m->l_layers, m->l_dims, m->l_params, x, y, bf16);
        ll[i] = y[0];
    }
    int rc = or_normalize(N, ll, prior_w, lambda, wn, stats);
    if (rc == OR_OK) rc = or_resample(N, wn, U, ix);
    if (rc == OR_OK) {
        for (int j = 0; j < N; ++j)
            for (int c = 0; c < d_s; ++c) S_new[(size_t)j * d_s + c] = sp[(size_t)ix[j] * d_s + c];
        if (S_prop) memcpy(S_prop, sp, sizeof(double) * (size_t)N * d_s);
        if (loglik) memcpy(loglik, ll, sizeof(double) * (size_t)N);
        if (w_out) memcpy(w_out, wn, sizeof(double) * (size_t)N);
        if (idx) memcpy(idx, ix, sizeof(int32_t) * (size_t)N);
    }
    free(sp); free(ll); free(wn); free(ix);
    release_rounded(&rm);
    return rc;
}

/* One observation draw o = f_Z([s', a, w_Z]) (Eq. 5). */
static void observation(const or_model* m, const double* s_next, int a_disc, const double* a_cont,
                        const double* wz, double* o, int bf16)
{
    double x[OR_MAX_WIDTH];
    int aw = action_width(m);
    for (int j = 0; j < m->d_s; ++j) x[j] = s_next[j];
    put_action(m, x + m->d_s, a_disc, a_cont);
    for (int j = 0; j < m->d_wz; ++j) x[m->d_s + aw + j] = wz[j];
    mlp_forward(m->z_layers, m->z_dims, m->z_params, x, o, bf16);
}

static int obs_net_check(const or_model* m)
{
    if (mlp_check(m->z_layers, m->z_dims) != OR_OK) return OR_ERR_ARG;
    if (m->z_dims[0] != m->d_s + action_width(m) + m->d_wz || m->z_dims[m->z_layers] != m->d_o) return OR_ERR_ARG;
    return OR_OK;
}

/* Observation sampler (Eq. 5): o_r = f_Z([s'_r, a_r, w_Z,r]) for n rows;
 * noise given or stream 4 with counter (row, 0, 0).  Actions: one per row. */
int or_observe(const or_model* m0, int n, const double* S, const int32_t* a_disc,
               const double* a_cont, const double* noise, uint64_t seed, int bf16, double* O)
{
    if (n < 0 || obs_net_check(m0) != OR_OK) return OR_ERR_ARG;
    if (m0->n_actions > 0 ? !a_disc : !a_cont) return OR_ERR_ARG;
    rounded_model rm;
    const or_model* m = rounded(m0, bf16, &rm);
    #pragma omp parallel for schedule(static)
    for (int r = 0; r < n; ++r) {
        double w[OR_MAX_WIDTH];
        if (noise) {
            for (int j = 0; j < m->d_wz; ++j) w[j] = noise[(size_t)r * m->d_wz + j];
        } else {
            or_normals(seed, (uint32_t)r, 0u, 0u, OR_STREAM_OBS, m->d_wz, w);
        }
        observation(m, S + (size_t)r * m->d_s, a_disc ? a_disc[r] : 0,
                    a_cont ? a_cont + (size_t)r * m->d_a : NULL, w, O + (size_t)r * m->d_o, bf16);
    }
    release_rounded(&rm);
    return OR_OK;
}

/* States and observations along the plan rollouts (Sec. 4.3 simulates with
 * both samplers; Eq. 2 and Eq. 5).  For candidate k, particle i and step
 * t < H: s_{t+1} is the rollout state of rollout_return (same transition
 * noise: given [K][N][H][d_w] or stream 3), written to traj[k][i][t] ([K][N]
 * [H][d_s], may be NULL); o_{k,i,t} = f_Z([s_{t+1}, a_{k,t}, w_Z]) with w_Z
 * given (obs_noise [K][N][H][d_wz]) or drawn from stream 4 at counter
 * (i, k or 0 under common random numbers, t), written to obs[k][i][t]
 * ([K][N][H][d_o], may be NULL). */
int or_plan_steps(const or_model* m0, int N, const double* S, int K, int H,
                  const int32_t* cand_disc, const double* cand_cont, const double* noise,
                  const double* obs_noise, uint64_t seed, int crn, int bf16, double* traj, double* obs)
{
    if (model_check(m0) != OR_OK || N < 1 || K < 0 || H < 0) return OR_ERR_ARG;
    if (m0->n_actions > 0 ? !cand_disc : !cand_cont) return OR_ERR_ARG;
    if (obs && obs_net_check(m0) != OR_OK) return OR_ERR_ARG;
    rounded_model rm;
    const or_model* m = rounded(m0, bf16, &rm);
    int rc = OR_OK;
    #pragma omp parallel for schedule(dynamic, 16)
    for (long r = 0; r < (long)K * N; ++r) {
        int k = (int)(r / N), i = (int)(r % N);
        double* tr = (double*)malloc(sizeof(double) * ((size_t)H * m->d_s + 1));
        if (!tr) {
            #pragma omp atomic write
            rc = OR_ERR_ARG;
            continue;
        }
        double goal0[OR_MAX_WIDTH] = {0};
        rollout_return(m, S + (size_t)i * m->d_s, k, i, N, H, cand_disc, cand_cont, 1.0, goal0, 0,
                       noise, seed, crn, bf16, tr);
        for (int t = 0; t < H; ++t) {
            size_t row = (size_t)r * H + t;
            if (traj)
                for (int j = 0; j < m->d_s; ++j) traj[row * m->d_s + j] = tr[(size_t)t * m->d_s + j];
            if (!obs) continue;
            double wz[OR_MAX_WIDTH];
            if (obs_noise) {
                for (int j = 0; j < m->d_wz; ++j) wz[j] = obs_noise[row * m->d_wz + j];
            } else {
                or_normals(seed, (uint32_t)i, crn ? 0u : (uint32_t)k, (uint32_t)t, OR_STREAM_OBS, m->d_wz, wz);
            }
            observation(m, tr + (size_t)t * m->d_s, cand_disc ? cand_disc[(size_t)k * H + t] : 0,
                        cand_cont ? cand_cont + ((size_t)k * H + t) * m->d_a : NULL, wz,
                        obs + row * m->d_o, bf16);
        }
        free(tr);
    }
    release_rounded(&rm);
    return rc;
}

/* Transition draws for n given (state, action, noise) rows: s'_r. */
int or_transition(const or_model* m0, int n, const double* S, const int32_t* a_disc,
                  const double* a_cont, const double* noise, int bf16, double* S_next)
{
    if (model_check(m0) != OR_OK || n < 0) return OR_ERR_ARG;
    if (m0->n_actions > 0 ? !a_disc : !a_cont) return OR_ERR_ARG;
    rounded_model rm;
    const or_model* m = rounded(m0, bf16, &rm);
    #pragma omp parallel for schedule(static)
    for (int r = 0; r < n; ++r)
        transition(m, S + (size_t)r * m->d_s, a_disc ? a_disc[r] : 0,
                   a_cont ? a_cont + (size_t)r * m->d_a : NULL,
                   noise + (size_t)r * m->d_w, S_next + (size_t)r * m->d_s, bf16);
    release_rounded(&rm);
    return OR_OK;
}

size_t or_mlp_param_count(int n_layers, const int* dims)
{
    return mlp_param_count(n_layers, dims);
}

/* ------------------------------------------------------------------------- */
/* Gradients through rollouts of the transition sampler (reverse mode).      */
/*                                                                           */
/* Rollout b: s_0 = S0_b; for t < H: s_{t+1} = s_t + f_T([s_t, a_{b,t}, w_{b,t}]). */
/* Objectives:                                                               */
/*   distill (objective 0): L = 1/(B H) sum_b sum_{t=1..H} ||s_{b,t} - T_{b,t}||^2 */
/*            with teacher states T (the distillation loss of Eq. 3 applied  */
/*            along free-running rollouts);                                  */
/*   return  (objective 1): J = 1/B sum_b sum_{t<H} gamma^t (-||s_{b,t+1} - g||^2). */
/* Actions: discrete a_{b,t} = actions[b*H + t] (one-hot), or continuous     */
/* sequences A[k][t][:] shared by `particles` consecutive rollouts           */
/* (rollout b uses k = b / particles).  Noise: given [B][H][d_w] or Philox   */
/* stream 3 with counter (b, 0, t).  The reverse sweep stores the whole     */
/* trajectory (no checkpointing) and uses ReLU'(0) = 0.                      */
/* ------------------------------------------------------------------------- */
#define OR_GRAD_CHUNK 64

static void grad_action(const or_model* m, int H, int particles, const int32_t* a_disc, const double* a_cont,
                        int b, int t, int* ad, const double** ac)
{
    *ad = 0;
    *ac = NULL;
    if (m->n_actions > 0) *ad = a_disc[(size_t)b * H + t];
    else *ac = a_cont + ((size_t)(b / particles) * H + t) * m->d_a;
}

static void grad_noise(const or_model* m, int H, const double* noise, uint64_t seed, int b, int t, double* w)
{
    if (noise) {
        for (int j = 0; j < m->d_w; ++j) w[j] = noise[((size_t)b * H + t) * m->d_w + j];
    } else {
        or_normals(seed, (uint32_t)b, 0u, (uint32_t)t, OR_STREAM_PLAN, m->d_w, w);
    }
}

/* Objective of one rollout and the hash of its ReLU sign pattern. */
static double rollout_objective(const or_model* m, int B, int H, int particles, const double* S0,
                                const int32_t* a_disc, const double* a_cont, const double* noise, uint64_t seed,
                                int objective, const double* targets, double gamma, const double* goal, int b,
                                uint64_t* pattern)
{
    double s[OR_MAX_WIDTH], x[OR_MAX_WIDTH], h[2][OR_MAX_WIDTH], w[OR_MAX_WIDTH];
    int d_s = m->d_s, aw = action_width(m);
    for (int j = 0; j < d_s; ++j) s[j] = S0[(size_t)b * d_s + j];
    double acc = 0.0, disc = 1.0;
    uint64_t hsh = 1469598103934665603ull;
    for (int t = 0; t < H; ++t) {
        int ad;
        const double* ac;
        grad_action(m, H, particles, a_disc, a_cont, b, t, &ad, &ac);
        grad_noise(m, H, noise, seed, b, t, w);
        for (int j = 0; j < d_s; ++j) x[j] = s[j];
        put_action(m, x + d_s, ad, ac);
        for (int j = 0; j < m->d_w; ++j) x[d_s + aw + j] = w[j];
        /* forward through the layers, recording the ReLU signs */
        const double* p = m->t_params;
        const double* in = x;
        int cur = 0;
        for (int l = 0; l < m->t_layers; ++l) {
            int n_in = m->t_dims[l], n_out = m->t_dims[l + 1];
            const double* W = p;
            const double* bb = p + (size_t)n_out * n_in;
            double* out = h[cur];
            for (int n = 0; n < n_out; ++n) {
                double z = 0.0;
                for (int k = 0; k < n_in; ++k) z += W[(size_t)n * n_in + k] * in[k];
                z += bb[n];
                if (l < m->t_layers - 1) {
                    int on = z > 0.0;
                    hsh = (hsh ^ (uint64_t)on) * 1099511628211ull;
                    z = on ? z : 0.0;
                }
                out[n] = z;
            }
            p += (size_t)n_out * n_in + n_out;
            in = out;
            cur ^= 1;
        }
        for (int j = 0; j < d_s; ++j) s[j] += in[j];
        if (objective == 0) {
            const double* T = targets + ((size_t)b * H + t) * d_s;
            for (int j = 0; j < d_s; ++j) acc += (s[j] - T[j]) * (s[j] - T[j]);
        } else {
            acc += disc * reward(d_s, s, goal);
            disc *= gamma;
        }
    }
    if (pattern) *pattern = hsh;
    return acc;
}

/* Objective value over all rollouts (Neumaier over b) and, if `patterns` is
 * non-NULL, each rollout's ReLU sign-pattern hash. */
double or_rollout_objective(const or_model* m, int B, int H, int particles, const double* S0,
                            const int32_t* a_disc, const double* a_cont, const double* noise, uint64_t seed,
                            int objective, const double* targets, double gamma, const double* goal,
                            uint64_t* patterns)
{
    double* per = (double*)malloc(sizeof(double) * (size_t)(B > 0 ? B : 1));
    #pragma omp parallel for schedule(static)
    for (int b = 0; b < B; ++b)
        per[b] = rollout_objective(m, B, H, particles, S0, a_disc, a_cont, noise, seed, objective, targets, gamma,
                                   goal, b, patterns ? patterns + b : NULL);
    /* Neumaier-compensated mean of the per-rollout values in rollout order
     * (terms per[b] / B), times B: the compensated sum over b */
    double total = weighted_sum(B, per, NULL, 1) * (double)B;
    free(per);
    double scale = objective == 0 ? 1.0 / ((double)B * H) : 1.0 / (double)B;
    return total * scale;
}

/* Reverse-mode gradient.  grad_params (may be NULL) receives d/d(parameters)
 * in the packed per-layer order (W then b); grad_actions (may be NULL,
 * continuous actions only) receives d/dA in the layout of a_cont. */
int or_rollout_grad(const or_model* m, int B, int H, int particles, const double* S0, const int32_t* a_disc,
                    const double* a_cont, const double* noise, uint64_t seed, int objective, const double* targets,
                    double gamma, const double* goal, double* loss, double* grad_params, double* grad_actions)
{
    if (model_check(m) != OR_OK || B < 1 || H < 0 || particles < 1) return OR_ERR_ARG;
    if (objective != 0 && objective != 1) return OR_ERR_ARG;
    if (objective == 0 && !targets) return OR_ERR_ARG;
    if (m->n_actions > 0 ? !a_disc : !a_cont) return OR_ERR_ARG;
    if (grad_actions && m->n_actions > 0) return OR_ERR_ARG;
    const int L = m->t_layers, d_s = m->d_s, aw = action_width(m);
    const size_t P = mlp_param_count(L, m->t_dims);
    int maxw = 0;
    for (int l = 0; l <= L; ++l) if (m->t_dims[l] > maxw) maxw = m->t_dims[l];
    const double scale = objective == 0 ? 1.0 / ((double)B * H) : 1.0 / (double)B;
    const int n_seq = m->n_actions > 0 ? 0 : (B + particles - 1) / particles;
    /* parameter gradients accumulate per chunk of OR_GRAD_CHUNK consecutive
     * rollouts (sequentially inside a chunk); chunks are summed in order
     * afterwards, so the result does not depend on the thread count */
    const int n_chunks = (B + OR_GRAD_CHUNK - 1) / OR_GRAD_CHUNK;
    double* gp = grad_params ? (double*)calloc((size_t)n_chunks * P, sizeof(double)) : NULL;
    double* ga = grad_actions ? (double*)calloc((size_t)B * H * (aw > 0 ? aw : 1), sizeof(double)) : NULL;
    double* lo = (double*)malloc(sizeof(double) * (size_t)B);
    int rc = OR_OK;
    #pragma omp parallel for schedule(dynamic, 1)
    for (int chunk = 0; chunk < n_chunks; ++chunk)
    for (int b = chunk * OR_GRAD_CHUNK; b < B && b < (chunk + 1) * OR_GRAD_CHUNK; ++b) {
        /* forward: store the layer inputs and pre-activations of every step */
        double* acts = (double*)malloc(sizeof(double) * (size_t)(H > 0 ? H : 1) * (L + 1) * maxw);
        double* pre = (double*)malloc(sizeof(double) * (size_t)(H > 0 ? H : 1) * L * maxw);
        double* st = (double*)malloc(sizeof(double) * (size_t)(H + 1) * d_s);
        double* dsc = (double*)malloc(sizeof(double) * (size_t)(H > 0 ? H : 1));
        double w[OR_MAX_WIDTH];
        for (int j = 0; j < d_s; ++j) st[j] = S0[(size_t)b * d_s + j];
        double acc = 0.0, disc = 1.0;
        for (int t = 0; t < H; ++t) {
            int ad;
            const double* ac;
            grad_action(m, H, particles, a_disc, a_cont, b, t, &ad, &ac);
            grad_noise(m, H, noise, seed, b, t, w);
            double* x = acts + ((size_t)t * (L + 1)) * maxw;
            for (int j = 0; j < d_s; ++j) x[j] = st[(size_t)t * d_s + j];
            put_action(m, x + d_s, ad, ac);
            for (int j = 0; j < m->d_w; ++j) x[d_s + aw + j] = w[j];
            const double* p = m->t_params;
            for (int l = 0; l < L; ++l) {
                int n_in = m->t_dims[l], n_out = m->t_dims[l + 1];
                const double* Wl = p;
                const double* bl = p + (size_t)n_out * n_in;
                const double* in = acts + ((size_t)t * (L + 1) + l) * maxw;
                double* zz = pre + ((size_t)t * L + l) * maxw;
                double* out = acts + ((size_t)t * (L + 1) + l + 1) * maxw;
                for (int n = 0; n < n_out; ++n) {
                    double z = 0.0;
                    for (int k = 0; k < n_in; ++k) z += Wl[(size_t)n * n_in + k] * in[k];
                    z += bl[n];
                    zz[n] = z;
                    out[n] = (l < L - 1) ? (z > 0.0 ? z : 0.0) : z;
                }
                p += (size_t)n_out * n_in + n_out;
            }
            const double* d = acts + ((size_t)t * (L + 1) + L) * maxw;
            for (int j = 0; j < d_s; ++j) st[(size_t)(t + 1) * d_s + j] = st[(size_t)t * d_s + j] + d[j];
            const double* s1 = st + (size_t)(t + 1) * d_s;
            if (objective == 0) {
                const double* T = targets + ((size_t)b * H + t) * d_s;
                for (int j = 0; j < d_s; ++j) acc += (s1[j] - T[j]) * (s1[j] - T[j]);
            } else {
                dsc[t] = disc;
                acc += disc * reward(d_s, s1, goal);
                disc *= gamma;
            }
        }
        lo[b] = acc;
        /* reverse sweep: lam = dObjective/ds_{t+1} */
        double lam[OR_MAX_WIDTH], g_out[OR_MAX_WIDTH], g_in[OR_MAX_WIDTH];
        for (int j = 0; j < d_s; ++j) lam[j] = 0.0;
        for (int t = H - 1; t >= 0; --t) {
            const double* s1 = st + (size_t)(t + 1) * d_s;
            if (objective == 0) {
                const double* T = targets + ((size_t)b * H + t) * d_s;
                for (int j = 0; j < d_s; ++j) lam[j] += 2.0 * (s1[j] - T[j]) * scale;
            } else {
                for (int j = 0; j < d_s; ++j) lam[j] += dsc[t] * (-2.0 * (s1[j] - goal[j])) * scale;
            }
            /* back through the layers of step t; d(out of last layer) = lam */
            for (int j = 0; j < d_s; ++j) g_out[j] = lam[j];
            size_t off_end = P;
            for (int l = L - 1; l >= 0; --l) {
                int n_in = m->t_dims[l], n_out = m->t_dims[l + 1];
                size_t off = off_end - ((size_t)n_out * n_in + n_out);
                const double* Wl = m->t_params + off;
                const double* in = acts + ((size_t)t * (L + 1) + l) * maxw;
                const double* zz = pre + ((size_t)t * L + l) * maxw;
                if (l < L - 1)
                    for (int n = 0; n < n_out; ++n) if (!(zz[n] > 0.0)) g_out[n] = 0.0;
                if (gp) {
                    double* G = gp + (size_t)chunk * P + off;
                    for (int n = 0; n < n_out; ++n) {
                        for (int k = 0; k < n_in; ++k) G[(size_t)n * n_in + k] += g_out[n] * in[k];
                        G[(size_t)n_out * n_in + n] += g_out[n];
                    }
                }
                for (int k = 0; k < n_in; ++k) {
                    double a = 0.0;
                    for (int n = 0; n < n_out; ++n) a += Wl[(size_t)n * n_in + k] * g_out[n];
                    g_in[k] = a;
                }
                for (int k = 0; k < n_in; ++k) g_out[k] = g_in[k];
                off_end = off;
            }
            /* g_out now holds d/dx_t: state part adds to lam, action part to dA */
            if (ga)
                for (int j = 0; j < aw; ++j) ga[((size_t)b * H + t) * aw + j] = g_out[d_s + j];
            for (int j = 0; j < d_s; ++j) lam[j] += g_out[j];
        }
        free(acts);
        free(pre);
        free(st);
        free(dsc);
    }
    if (loss) {
        double tot = weighted_sum(B, lo, NULL, 1) * (double)B;
        *loss = tot * scale;
    }
    if (gp) {
        for (size_t q = 0; q < P; ++q) {
            double sum = 0.0, comp = 0.0;
            for (int c = 0; c < n_chunks; ++c) {
                double term = gp[(size_t)c * P + q];
                double tt = sum + term;
                if (fabs(sum) >= fabs(term)) comp += (sum - tt) + term; else comp += (term - tt) + sum;
                sum = tt;
            }
            grad_params[q] = sum + comp;
        }
    }
    if (ga) {
        for (int k = 0; k < n_seq; ++k)
            for (int t = 0; t < H; ++t)
                for (int j = 0; j < aw; ++j) {
                    double sum = 0.0;
                    for (int b = k * particles; b < (k + 1) * particles && b < B; ++b)
                        sum += ga[((size_t)b * H + t) * aw + j];
                    grad_actions[((size_t)k * H + t) * aw + j] = sum;
                }
    }
    free(gp);
    free(ga);
    free(lo);
    return rc;
}

/* Normals of n consecutive first counter words c0 = 0..n-1 (rows of out[n][d]). */
void or_normals_rows(uint64_t seed, int n, uint32_t c1, uint32_t c2, uint32_t stream, int d, double* out)
{
    #pragma omp parallel for schedule(static)
    for (int r = 0; r < n; ++r) or_normals(seed, (uint32_t)r, c1, c2, stream, d, out + (size_t)r * d);
}

/* Threads of the OpenMP loops (the results do not depend on it); returns
 * the previous setting.  Used to time the oracle on one core. */
int or_set_threads(int n)
{
#ifdef _OPENMP
    int prev = omp_get_max_threads();
    if (n > 0) omp_set_num_threads(n);
    return prev;
#else
    (void)n;
    return 1;
#endif
}

/* ------------------------------------------------------------------------- */
/* Grouped progressive-widening step (Sec. 4.3): simulations are grouped by  */
/* their parent action node and every group is handled at once.             */
/* ------------------------------------------------------------------------- */
#define OR_STREAM_BRANCH 6u

/* Widening test of one action node with n_visits visits and n_children
 * observation branches: widen when |C(a)| < k_o N(a)^alpha_o (binary64), or
 * when the node has no branch yet; never beyond `capacity` branches. */
int or_pw_widen(int n_visits, int n_children, double k_o, double alpha_o, int capacity)
{
    if (n_children >= capacity) return 0;
    if (n_children == 0) return 1;
    return (double)n_children < k_o * pow((double)n_visits, alpha_o);
}

/* For M action nodes whose successor states S[seg[m] .. seg[m+1]) (rows of
 * d_s) were simulated under the node's action:
 *   1. widen_m = or_pw_widen(visits[m], children[m], k_o, alpha_o, B).
 *   2. widening: a new observation o = f_Z([S[seg[m]], a_m, w_Z]) (Eq. 5),
 *      w_Z drawn from stream 4 at counter (0, m, 0), is stored as branch
 *      children[m] of the node's table obs_table[m][B][d_o] and children[m]
 *      grows by one; otherwise an existing branch is taken uniformly:
 *      floor(u * children[m]) with u the uniform of word 0 of Philox at
 *      counter (m, 1, 0, stream 6 << 16).
 *   3. every successor of the node is weighted against the chosen branch's
 *      observation, l_j = l([s'_j, a_m, o_branch]) (Sec. 4.2), and the group is
 *      normalised (or_normalize, uniform prior) and resampled (or_resample
 *      with the node's offset U[m]); idx holds indices within the group and
 *      S_out[j] = S[seg[m] + idx_j].
 * Empty groups are skipped (branch -1, nothing written).  Outputs: widen [M],
 * branch [M], loglik [T], w [T], stats [M][2], idx [T], S_out [T][d_s];
 * children and obs_table are updated in place. */
int or_pw_step(const or_model* m0, int T, const double* S, int M, const int32_t* seg,
               const int32_t* a_disc, const double* a_cont, const int32_t* visits, int32_t* children,
               int B, double* obs_table, double k_o, double alpha_o, double lambda, uint64_t seed,
               const uint32_t* U, int bf16, int32_t* widen, int32_t* branch, double* loglik, double* w,
               double* stats, int32_t* idx, double* S_out)
{
    if (M < 0 || T < 0 || B < 1 || !(lambda > 0.0) || obs_net_check(m0) != OR_OK) return OR_ERR_ARG;
    if (mlp_check(m0->l_layers, m0->l_dims) != OR_OK) return OR_ERR_ARG;
    if (m0->l_dims[0] != m0->d_s + action_width(m0) + m0->d_o || m0->l_dims[m0->l_layers] != 1) return OR_ERR_ARG;
    if (m0->n_actions > 0 ? !a_disc : !a_cont) return OR_ERR_ARG;
    if (seg[0] != 0 || seg[M] != T) return OR_ERR_ARG;
    for (int g = 0; g < M; ++g)
        if (seg[g + 1] < seg[g] || children[g] < 0 || children[g] > B) return OR_ERR_ARG;
    const int d_s = m0->d_s, d_o = m0->d_o, aw = action_width(m0);
    rounded_model rm;
    const or_model* m = rounded(m0, bf16, &rm);
    int rc = OR_OK;
    for (int g = 0; g < M && rc == OR_OK; ++g) {
        const int lo = seg[g], n = seg[g + 1] - lo;
        const int ad = a_disc ? a_disc[g] : 0;
        const double* ac = a_cont ? a_cont + (size_t)g * m->d_a : NULL;
        if (n == 0) {
            widen[g] = 0;
            branch[g] = -1;
            continue;
        }
        double* row = obs_table + (size_t)g * B * d_o;
        widen[g] = or_pw_widen(visits[g], children[g], k_o, alpha_o, B);
        if (widen[g]) {
            double wz[OR_MAX_WIDTH];
            or_normals(seed, 0u, (uint32_t)g, 0u, OR_STREAM_OBS, m->d_wz, wz);
            observation(m, S + (size_t)lo * d_s, ad, ac, wz, row + (size_t)children[g] * d_o, bf16);
            branch[g] = children[g];
            children[g] += 1;
        } else {
            uint32_t ctr[4] = {(uint32_t)g, 1u, 0u, OR_STREAM_BRANCH << 16};
            uint32_t key[2] = {(uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32)};
            uint32_t word[4];
            or_philox4x32_10(ctr, key, word);
            branch[g] = (int32_t)floor(or_uniform(word[0]) * (double)children[g]);
        }
        const double* o = row + (size_t)branch[g] * d_o;
        #pragma omp parallel for schedule(static)
        for (int j = 0; j < n; ++j) {
            double x[OR_MAX_WIDTH], y[1];
            for (int c = 0; c < d_s; ++c) x[c] = S[(size_t)(lo + j) * d_s + c];
            put_action(m, x + d_s, ad, ac);
            for (int c = 0; c < d_o; ++c) x[d_s + aw + c] = o[c];
            mlp_forward(m->l_layers, m->l_dims, m->l_params, x, y, bf16);
            loglik[lo + j] = y[0];
        }
        rc = or_normalize(n, loglik + lo, NULL, lambda, w + lo, stats + 2 * (size_t)g);
        if (rc == OR_OK) rc = or_resample(n, w + lo, U[g], idx + lo);
        if (rc == OR_OK)
            for (int j = 0; j < n; ++j)
                for (int c = 0; c < d_s; ++c)
                    S_out[(size_t)(lo + j) * d_s + c] = S[(size_t)(lo + idx[lo + j]) * d_s + c];
    }
    release_rounded(&rm);
    return rc;
}

/* ------------------------------------------------------------------------- */
/* Soft value and action selection (Sec. 2.2): the log-sum-exp operator      */
/* L_eta over the preferences of M nodes with K candidates each.             */
/* ------------------------------------------------------------------------- */
/* x_k = eta Q_k + log pi0_k (pi0 given as log-probabilities, NULL: uniform
 * 1/K), i.e. eta times the preference Q_k + (1/eta) log pi0_k;
 *   V = (1/eta) log sum_k exp(x_k)      (max-shifted, compensated sum)
 *   pi_k = exp(x_k - eta V)             (the soft policy)
 *   best = argmax_k x_k                 (lowest k on ties). */
int or_soft_value(int M, int K, const double* Q, const double* log_pi0, double eta,
                  double* V, double* pi, int32_t* best)
{
    if (M < 0 || K < 1 || !(eta > 0.0) || !isfinite(eta)) return OR_ERR_ARG;
    double* x = (double*)malloc(sizeof(double) * (size_t)K);
    if (!x) return OR_ERR_ARG;
    int rc = OR_OK;
    for (int m = 0; m < M && rc == OR_OK; ++m) {
        double mx = -INFINITY;
        int arg = 0;
        for (int k = 0; k < K; ++k) {
            size_t e = (size_t)m * K + k;
            x[k] = eta * Q[e] + (log_pi0 ? log_pi0[e] : -log((double)K));
            if (isnan(x[k]) || x[k] == INFINITY) { rc = OR_ERR_NUMERIC; break; }
            if (x[k] > mx) { mx = x[k]; arg = k; }
        }
        if (rc != OR_OK) break;
        if (!isfinite(mx)) { rc = OR_ERR_NUMERIC; break; }
        double sum = 0.0, comp = 0.0;
        for (int k = 0; k < K; ++k) {
            double v = exp(x[k] - mx);
            double t = sum + v;
            if (fabs(sum) >= fabs(v)) comp += (sum - t) + v;
            else comp += (v - t) + sum;
            sum = t;
        }
        double S = sum + comp;
        V[m] = (mx + log(S)) / eta;
        if (pi)
            for (int k = 0; k < K; ++k) pi[(size_t)m * K + k] = exp(x[k] - mx) / S;
        if (best) best[m] = arg;
    }
    free(x);
    return rc;
}

/* ------------------------------------------------------------------------- */
/* Contrastive likelihood objective (Sec. 4.2, Eq. 6): every state-action of */
/* a mini-batch of B tuples (s'_i, a_i, o_i) against every observation.      */
/* ------------------------------------------------------------------------- */
/* Given the all-pairs scores l_ij = l(s'_i, a_i, o_j) (row i, column j) of
 * the rows listed in rows[r] (n_rows of them; the diagonal entry of row r is
 * column rows[r]):
 *   row_loss_r = log sum_j exp(l_ij) - l_ii     (max-shifted, compensated sum)
 *   G_rj       = (exp(l_ij) / sum_j' exp(l_ij') - [j == i]) / B,
 * the derivative of the mean of the B row losses with respect to l_ij. */
int or_info_nce_rows(int B, int n_rows, const int32_t* rows, const double* Lg, double* row_loss, double* G)
{
    if (B < 1 || n_rows < 0) return OR_ERR_ARG;
    for (int r = 0; r < n_rows; ++r) {
        const int i = rows ? rows[r] : r;
        if (i < 0 || i >= B) return OR_ERR_ARG;
        const double* l = Lg + (size_t)r * B;
        double mx = -INFINITY;
        for (int j = 0; j < B; ++j) {
            if (!isfinite(l[j])) return OR_ERR_NUMERIC;
            if (l[j] > mx) mx = l[j];
        }
        double sum = 0.0, comp = 0.0;
        for (int j = 0; j < B; ++j) {
            double v = exp(l[j] - mx);
            double t = sum + v;
            if (fabs(sum) >= fabs(v)) comp += (sum - t) + v;
            else comp += (v - t) + sum;
            sum = t;
        }
        const double S = sum + comp;
        if (row_loss) row_loss[r] = mx + log(S) - l[i];
        if (G)
            for (int j = 0; j < B; ++j)
                G[(size_t)r * B + j] = (exp(l[j] - mx) / S - (j == i ? 1.0 : 0.0)) / (double)B;
    }
    return OR_OK;
}

/* The scores l_ij = l([s'_i, a_i, o_j]) of rows rows[r] (NULL: all B rows in
 * order) against all B observations, then their row losses and derivatives
 * (or_info_nce_rows).  With all rows, *loss = (1/B) sum_i row_loss_i (the
 * InfoNCE loss of Eq. 6); loss may be NULL. */
int or_info_nce(const or_model* m0, int B, const double* S, const int32_t* a_disc, const double* a_cont,
                const double* O, int n_rows, const int32_t* rows, int bf16, double* Lg, double* row_loss,
                double* G, double* loss)
{
    if (B < 1 || n_rows < 0 || (!rows && n_rows != B)) return OR_ERR_ARG;
    if (mlp_check(m0->l_layers, m0->l_dims) != OR_OK) return OR_ERR_ARG;
    if (m0->l_dims[0] != m0->d_s + action_width(m0) + m0->d_o || m0->l_dims[m0->l_layers] != 1) return OR_ERR_ARG;
    if (m0->n_actions > 0 ? !a_disc : !a_cont) return OR_ERR_ARG;
    for (int r = 0; r < n_rows; ++r) {
        const int i = rows ? rows[r] : r;
        if (i < 0 || i >= B) return OR_ERR_ARG;
        if (m0->n_actions > 0 && (a_disc[i] < 0 || a_disc[i] >= m0->n_actions)) return OR_ERR_ARG;
    }
    const int d_s = m0->d_s, d_o = m0->d_o, aw = action_width(m0);
    rounded_model rm;
    const or_model* m = rounded(m0, bf16, &rm);
    #pragma omp parallel for schedule(static)
    for (long e = 0; e < (long)n_rows * B; ++e) {
        const int r = (int)(e / B), j = (int)(e % B);
        const int i = rows ? rows[r] : r;
        double x[OR_MAX_WIDTH], y[1];
        for (int c = 0; c < d_s; ++c) x[c] = S[(size_t)i * d_s + c];
        put_action(m, x + d_s, a_disc ? a_disc[i] : 0, a_cont ? a_cont + (size_t)i * m->d_a : NULL);
        for (int c = 0; c < d_o; ++c) x[d_s + aw + c] = O[(size_t)j * d_o + c];
        mlp_forward(m->l_layers, m->l_dims, m->l_params, x, y, bf16);
        Lg[e] = y[0];
    }
    release_rounded(&rm);
    int rc = or_info_nce_rows(B, n_rows, rows, Lg, row_loss, G);
    if (rc == OR_OK && loss && !rows && row_loss) {
        double sum = 0.0, comp = 0.0;
        for (int i = 0; i < B; ++i) {
            double v = row_loss[i];
            double t = sum + v;
            if (fabs(sum) >= fabs(v)) comp += (sum - t) + v;
            else comp += (v - t) + sum;
            sum = t;
        }
        *loss = (sum + comp) / (double)B;
    }
    return rc;
}

/* ------------------------------------------------------------------------- */
/* Teacher sampler of the transition model (Sec. 4.2): the deterministic     */
/* (ODE) DDIM sampler of a v-prediction denoiser under the cosine schedule.  */
/* ------------------------------------------------------------------------- */
/* Cosine cumulative schedule (Nichol and Dhariwal, "Improved denoising
 * diffusion probabilistic models", 2021) with offset 0.008, normalised so
 * that abar(0) = 1:  abar(tau) = cos^2(pi/2 (tau + s)/(1 + s)) / cos^2(pi/2 s/(1 + s)).
 * At tau = 1 the numerator's angle is pi/2 and abar is 0 up to rounding; it
 * is clamped to [0, 1]. */
double or_cosine_abar(double tau)
{
    const double s = 0.008, h = 1.5707963267948966;
    double c = cos(h * (tau + s) / (1.0 + s)), c0 = cos(h * s / (1.0 + s));
    double a = (c * c) / (c0 * c0);
    return a < 0.0 ? 0.0 : (a > 1.0 ? 1.0 : a);
}

typedef void (*or_vfun)(const void* ctx, const double* s, const double* x, double tau, double* v);

/* The ODE sampler from x at tau = 1 (the latent noise) to tau = 0 in n
 * uniform steps tau_k = 1 - k/n.  With a = abar(tau_k), a' = abar(tau_{k+1})
 * and the predicted v at (x, tau_k), the clean-sample and noise estimates of
 * v-prediction are x0 = sqrt(a) x - sqrt(1-a) v and eps = sqrt(1-a) x +
 * sqrt(a) v, and the step re-noises x0 with eps to the next time:
 * x <- sqrt(a') x0 + sqrt(1-a') eps. */
static void ddim_run(int d, const double* s, double* x, int n_steps, or_vfun vf, const void* ctx)
{
    double v[OR_MAX_WIDTH];
    for (int k = 0; k < n_steps; ++k) {
        const double tau = 1.0 - (double)k / n_steps, tau_next = 1.0 - (double)(k + 1) / n_steps;
        const double a = or_cosine_abar(tau), an = or_cosine_abar(tau_next);
        vf(ctx, s, x, tau, v);
        for (int c = 0; c < d; ++c) {
            double x0 = sqrt(a) * x[c] - sqrt(1.0 - a) * v[c];
            double eps = sqrt(1.0 - a) * x[c] + sqrt(a) * v[c];
            x[c] = sqrt(an) * x0 + sqrt(1.0 - an) * eps;
        }
    }
}

typedef struct {
    int n_layers; const int* dims; const double* params;
    int d_c, d_x, n_actions, d_a, a_disc; const double* a_cont; int bf16;
} ddim_net_ctx;

/* v = denoiser([c, a, x, tau]) (a one-hot over n_actions, or continuous). */
static void ddim_net_v(const void* cp, const double* cond, const double* x, double tau, double* v)
{
    const ddim_net_ctx* c = (const ddim_net_ctx*)cp;
    double in[OR_MAX_WIDTH];
    const int aw = c->n_actions > 0 ? c->n_actions : c->d_a;
    for (int j = 0; j < c->d_c; ++j) in[j] = cond[j];
    for (int j = 0; j < aw; ++j) in[c->d_c + j] = c->n_actions > 0 ? (j == c->a_disc ? 1.0 : 0.0) : c->a_cont[j];
    for (int j = 0; j < c->d_x; ++j) in[c->d_c + aw + j] = x[j];
    in[c->d_c + aw + c->d_x] = tau;
    mlp_forward(c->n_layers, c->dims, c->params, in, v, c->bf16);
}

/* Teacher samples of n rows: X1 [n][d_x] the latent noise at tau = 1,
 * C [n][d_c] the conditioning inputs (the state for the transition
 * denoiser, the next state for the observation denoiser), one action for
 * all rows, a denoiser with input [c, a, x_tau, tau] and output v [d_x].
 * Out [n][d_x]. */
int or_ddim_sample(int n_layers, const int* dims, const double* params, int d_c, int d_x, int n_actions, int d_a,
                   int n, const double* C, int a_disc, const double* a_cont, const double* X1, int n_steps,
                   int bf16, double* out)
{
    const int aw = n_actions > 0 ? n_actions : d_a;
    if (mlp_check(n_layers, dims) != OR_OK || n < 0 || n_steps < 1 || d_c < 1 || d_x < 1) return OR_ERR_ARG;
    if (dims[0] != d_c + aw + d_x + 1 || dims[n_layers] != d_x) return OR_ERR_ARG;
    if (n_actions > 0 ? (a_disc < 0 || a_disc >= n_actions) : !a_cont) return OR_ERR_ARG;
    double* rw = bf16 ? round_weights(n_layers, dims, params) : NULL;
    if (bf16 && !rw) return OR_ERR_ARG;
    ddim_net_ctx c = {n_layers, dims, bf16 ? rw : params, d_c, d_x, n_actions, d_a, a_disc, a_cont, bf16};
    #pragma omp parallel for schedule(static)
    for (int r = 0; r < n; ++r) {
        double x[OR_MAX_WIDTH];
        for (int j = 0; j < d_x; ++j) x[j] = X1[(size_t)r * d_x + j];
        ddim_run(d_x, C + (size_t)r * d_c, x, n_steps, ddim_net_v, &c);
        for (int j = 0; j < d_x; ++j) out[(size_t)r * d_x + j] = x[j];
    }
    free(rw);
    return OR_OK;
}

/* The same sampler driven by the exact v of a point-mass data distribution
 * at x0 (the conditioning input s is taken as x0): with a = abar(tau),
 * eps = (x - sqrt(a) x0) / sqrt(1 - a) and v = sqrt(a) eps - sqrt(1 - a) x0.
 * For tau = 1 (a = 0) eps = x.  Test hook of the step arithmetic. */
static void ddim_point_v(const void* cp, const double* s, const double* x, double tau, double* v)
{
    const int d = *(const int*)cp;
    const double a = or_cosine_abar(tau);
    for (int j = 0; j < d; ++j) {
        double eps = a > 0.0 ? (x[j] - sqrt(a) * s[j]) / sqrt(1.0 - a) : x[j];
        v[j] = sqrt(a) * eps - sqrt(1.0 - a) * s[j];
    }
}

/* The exact v of Gaussian data N(mu, sigma^2 I): with a = abar(tau), the
 * posterior mean is x0 = mu + sqrt(a) sigma^2 (x - sqrt(a) mu) / (a sigma^2
 * + 1 - a), eps = (x - sqrt(a) x0) / sqrt(1 - a) and v = sqrt(a) eps -
 * sqrt(1 - a) x0 (the conditioning input is taken as mu).  Test hook. */
typedef struct { int d; double sigma; } ddim_gauss_ctx;
static void ddim_gauss_v(const void* cp, const double* mu, const double* x, double tau, double* v)
{
    const ddim_gauss_ctx* c = (const ddim_gauss_ctx*)cp;
    const double a = or_cosine_abar(tau), s2 = c->sigma * c->sigma;
    for (int j = 0; j < c->d; ++j) {
        double x0 = mu[j] + sqrt(a) * s2 * (x[j] - sqrt(a) * mu[j]) / (a * s2 + 1.0 - a);
        double eps = (x[j] - sqrt(a) * x0) / sqrt(1.0 - a);
        v[j] = sqrt(a) * eps - sqrt(1.0 - a) * x0;
    }
}

int or_ddim_gaussian(int d, const double* mu, double sigma, const double* x1, int n_steps, double* out)
{
    if (d < 1 || d > OR_MAX_WIDTH || n_steps < 1 || !(sigma > 0.0)) return OR_ERR_ARG;
    ddim_gauss_ctx c = {d, sigma};
    for (int j = 0; j < d; ++j) out[j] = x1[j];
    ddim_run(d, mu, out, n_steps, ddim_gauss_v, &c);
    return OR_OK;
}

int or_ddim_point_mass(int d, const double* x0, const double* x1, int n_steps, double* out)
{
    if (d < 1 || d > OR_MAX_WIDTH || n_steps < 1) return OR_ERR_ARG;
    for (int j = 0; j < d; ++j) out[j] = x1[j];
    ddim_run(d, x0, out, n_steps, ddim_point_v, &d);
    return OR_OK;
}

/* Derivative of the InfoNCE loss (Eq. 6) with respect to the likelihood
 * network's parameters (packed per layer as W then b, the layout of the
 * parameter vector): sum over all pairs of G_ij times the derivative of
 * l([s'_i, a_i, o_j]), by reverse mode through the network (ReLU'(0) = 0),
 * accumulated over each row's pairs in order, then over rows in order.
 * Also returns the loss.  bf16 != 0 is the bfloat16 emulation of C.9
 * extended to the reverse sweep: weights and every layer's input rounded to
 * bfloat16 (the scores and G from the emulated forward pass), and the
 * derivative with respect to each hidden layer's pre-activation rounded to
 * bfloat16 before it enters a product or a sum (the output adjoint G stays
 * unrounded); biases unrounded, accumulation in binary64. */
int or_info_nce_param_grad(const or_model* m0, int B, const double* S, const int32_t* a_disc, const double* a_cont,
                           const double* O, int bf16, double* grad, double* loss)
{
    if (B < 1 || mlp_check(m0->l_layers, m0->l_dims) != OR_OK || m0->l_layers > OR_MAX_LAYERS) return OR_ERR_ARG;
    const int L = m0->l_layers, d_s = m0->d_s, d_o = m0->d_o, aw = action_width(m0);
    const int* dims = m0->l_dims;
    if (dims[0] != d_s + aw + d_o || dims[L] != 1) return OR_ERR_ARG;
    const size_t np = mlp_param_count(L, dims);
    double* Lg = (double*)malloc(sizeof(double) * (size_t)B * B);
    double* G = (double*)malloc(sizeof(double) * (size_t)B * B);
    double* rl = (double*)malloc(sizeof(double) * (size_t)B);
    if (!Lg || !G || !rl) { free(Lg); free(G); free(rl); return OR_ERR_ARG; }
    int rc = or_info_nce(m0, B, S, a_disc, a_cont, O, B, NULL, bf16, Lg, rl, G, loss);
    rounded_model rm;
    const or_model* m = rounded(m0, bf16, &rm);
    /* one partial gradient per row, summed in row order afterwards (the
     * result does not depend on the number of threads) */
    double* part = rc == OR_OK ? (double*)calloc((size_t)B * np, sizeof(double)) : NULL;
    if (rc == OR_OK && !part) rc = OR_ERR_ARG;
    #pragma omp parallel for schedule(dynamic, 1)
    for (int i = 0; i < (rc == OR_OK ? B : 0); ++i) {
        /* activations of every layer for one pair: act[l] is layer l's input */
        double act[OR_MAX_LAYERS + 1][OR_MAX_WIDTH], delta[OR_MAX_WIDTH], prev[OR_MAX_WIDTH];
        double* gi = part + (size_t)i * np;
        for (int j = 0; j < B; ++j) {
            double* x = act[0];
            for (int c = 0; c < d_s; ++c) x[c] = S[(size_t)i * d_s + c];
            put_action(m, x + d_s, a_disc ? a_disc[i] : 0, a_cont ? a_cont + (size_t)i * m->d_a : NULL);
            for (int c = 0; c < d_o; ++c) x[d_s + aw + c] = O[(size_t)j * d_o + c];
            if (bf16)
                for (int c = 0; c < dims[0]; ++c) x[c] = or_round_bf16(x[c]);
            const double* p = m->l_params;
            for (int l = 0; l < L; ++l) {
                const int n_in = dims[l], n_out = dims[l + 1];
                for (int n = 0; n < n_out; ++n) {
                    double acc = 0.0;
                    for (int k = 0; k < n_in; ++k) acc += p[(size_t)n * n_in + k] * act[l][k];
                    acc += p[(size_t)n_out * n_in + n];
                    act[l + 1][n] = (l < L - 1 && acc < 0.0) ? 0.0 : acc;
                    if (bf16 && l < L - 1) act[l + 1][n] = or_round_bf16(act[l + 1][n]);
                }
                p += (size_t)n_out * n_in + n_out;
            }
            /* reverse sweep: delta = d loss / d (pre-activation of layer l) */
            delta[0] = G[(size_t)i * B + j];
            size_t off = np;
            for (int l = L - 1; l >= 0; --l) {
                const int n_in = dims[l], n_out = dims[l + 1];
                off -= (size_t)n_out * n_in + n_out;
                const double* W = m->l_params + off;
                double* gW = gi + off;
                for (int n = 0; n < n_out; ++n) {
                    for (int k = 0; k < n_in; ++k) gW[(size_t)n * n_in + k] += delta[n] * act[l][k];
                    gW[(size_t)n_out * n_in + n] += delta[n];
                }
                if (l > 0) {
                    for (int k = 0; k < n_in; ++k) {
                        double acc = 0.0;
                        for (int n = 0; n < n_out; ++n) acc += W[(size_t)n * n_in + k] * delta[n];
                        prev[k] = act[l][k] > 0.0 ? acc : 0.0;
                    }
                    for (int k = 0; k < n_in; ++k) delta[k] = bf16 ? or_round_bf16(prev[k]) : prev[k];
                }
            }
        }
    }
    release_rounded(&rm);
    for (size_t q = 0; q < np; ++q) grad[q] = 0.0;
    if (part)
        for (int i = 0; i < B; ++i)
            for (size_t q = 0; q < np; ++q) grad[q] += part[(size_t)i * np + q];
    free(part);
    free(Lg); free(G); free(rl);
    return rc;
}
