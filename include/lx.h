/* lx.h -- C ABI of liblx: ensemble adaptive explicit/implicit tau-leaping on
 * AMD Instinct MI355X (gfx950).
 *
 * The library advances P independent trajectories of a mass-action reaction
 * network to a final time, one trajectory per GPU lane, with the adaptive
 * explicit/implicit tau-leaping method packaged by matLeap (Feigelman,
 * Ganscha & Claassen, arXiv 1608.07058), and returns for every trajectory the
 * final state X(t_end), the firing counts r_j and the integrals G_j of g_j(X)
 * that feed the conjugate Gamma(alpha_j + r_j, beta_j + G_j) posterior
 * (Background section of the paper).
 *
 * Conventions
 *  - Every function returns an lx_status; LX_OK (0) on success, a negative
 *    code on error.  lx_last_error() returns a thread-local message for the
 *    last non-OK status.  No C++ exception crosses this interface.
 *  - Buffers marked "device" are GPU memory owned by the caller (e.g. torch
 *    tensors); the library never frees them.  Host arrays are read during the
 *    call only.
 *  - Work is enqueued on the caller's HIP stream (passed as void*, NULL for
 *    the default stream) and is asynchronous: the call returns once the
 *    kernels are launched.  Argument and launch errors are reported
 *    synchronously.  Per-trajectory conditions are reported in lx_stats.
 *  - Network handles are immutable after creation; simulations with distinct
 *    handles may run from different host threads.  A handle may be shared by
 *    threads; its kernel cache is internally locked.
 *  - The first simulation of a network with given precision/schedule compiles
 *    a network-specialised kernel (hipRTC, gfx950) and caches the code object
 *    in memory and in the directory named by LX_KERNEL_CACHE (default: a
 *    "kcache" directory beside liblx.so).
 */
#ifndef LX_H_
#define LX_H_

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t lx_status;
#define LX_OK 0
#define LX_E_INVALID (-1)     /* invalid argument or network table */
#define LX_E_COMPILE (-2)     /* run-time kernel compilation failed */
#define LX_E_HIP (-3)         /* HIP runtime error (launch, module load) */
#define LX_E_UNSUPPORTED (-4) /* device is not gfx950, or network too large */
#define LX_E_NOMEM (-5)       /* host or device allocation failed */
/* Warning (positive): the simulation ran, and some trajectories ended with a
 * status other than LX_LANE_OK (only with lx_options.check_lanes set). */
#define LX_W_LANE_FAIL 1

/* Simulation modes (paper, Results section: adaptive by default, or fully
 * explicit tau-leaping, or SSA only). */
#define LX_MODE_ADAPTIVE 0 /* explicit/implicit/SSA switching */
#define LX_MODE_EXPLICIT 1 /* explicit leaps and SSA bursts, never implicit */
#define LX_MODE_SSA 2      /* exact SSA (Gillespie direct method) only */

/* Precision policies. */
#define LX_PREC_FP64 0  /* every floating-point quantity in binary64 */
#define LX_PREC_MIXED 1 /* propensities, tau bounds, Poisson means and samplers in
                           binary32; time t, G and the implicit Newton solve in
                           binary64; counts int32 */

/* Schedules. */
#define LX_SCHED_PLAIN 0   /* one lane per particle for its whole life */
#define LX_SCHED_BATCHED 1 /* persistent blocks; each block owns a contiguous range of
                              particles and refills finished lanes from it (work
                              stealing through an LDS cursor); lanes in SSA bursts
                              take several SSA steps per leap iteration of the
                              other lanes (divergence balancing); waves may run
                              with 16 or 32 active lanes when the ensemble is too
                              small to give every SIMD a full wave */

/* Jacobian of the implicit solve (lx_options.jacobian). */
#define LX_JAC_ANALYTIC 0
#define LX_JAC_FD 1
#define LX_JAC_USER 2 /* the derivative terms given to lx_network_create_jac */

/* Per-trajectory status codes (lx_stats.status). */
#define LX_LANE_OK 0
#define LX_LANE_STEP_BUDGET 1     /* max_steps attempts used before t_end */
#define LX_LANE_LAMBDA_OVERFLOW 2 /* a Poisson mean beyond the sampler's range
                                     (2^30; in mixed precision means
                                     from 2^22 are drawn in binary64) */
#define LX_LANE_BAD_INPUT 3       /* negative/non-finite theta or negative x0 */
#define LX_LANE_COUNT_OVERFLOW 4  /* a copy number or firing count beyond int32 */

/* Options.  Obtain defaults from lx_options_default() and override fields.
 * The control constants are the tuning parameters the paper leaves to its
 * supplement (Implementation section); the defaults are stated readings. */
typedef struct lx_options {
  int32_t precision;    /* LX_PREC_*                          default FP64 */
  int32_t schedule;     /* LX_SCHED_*                         default PLAIN */
  uint64_t seed;        /* Philox key                         default 160807058 */
  uint32_t rng_stream;  /* added to the high key word (e.g. an interval index) */
  uint32_t pid_base;    /* particle p uses RNG particle id pid_base + p */
  double t_start;       /* start time                         default 0 */
  int32_t accumulate;   /* nonzero: r_out and G_out hold starting values and
                           are accumulated into (split runs) */
  int32_t n_c;          /* critical threshold on L_j          default 10 */
  double delta;         /* partial-equilibrium tolerance      default 0.05 */
  double n_stiff;       /* implicit if tau_im > n_stiff*tau_ex, default 100 */
  double k_ssa;         /* SSA burst if tau' < k_ssa / a0     default 10 */
  double k_crit;        /* SSA burst if a0c >= a0 / k_crit    default 10 */
  int32_t n_ssa_ex;     /* SSA burst length after an explicit choice, default 100 */
  int32_t n_ssa_im;     /* SSA burst length after an implicit choice, default 10 */
  double lambda_thr;    /* Poisson inversion below, PTRS (valid from 10) at or
                           above, default 15, in [10,30] */
  double newton_tol;    /* Newton stop: |dy|inf <= tol*max(1,|y|inf), default 1e-10 */
  int32_t newton_maxit; /* default 20 */
  int32_t block_size;   /* threads per block (64..256, multiple of 64); 0 = default (64
                           plain, 256 batched); networks beyond 16 species or 32
                           reactions run 64 with one trajectory per lane */
  int64_t max_steps;    /* attempt budget per trajectory      default 10^7 (< 2^32) */
  int32_t lanes_per_wave; /* batched: active lanes per wave, 4/8/16/32/64; 0 = chosen from P */
  int32_t ssa_k;        /* batched: SSA steps per leap iteration, 1..64; 0 = default 4 */
  int32_t blocks_per_cu;/* batched: resident blocks per CU, 1..8; 0 = default 2 (for
                           networks beyond 16 species or 32 reactions: as many as their
                           LDS fits, at most 8, with one trajectory per wave; 4 with one
                           per lane) */
  uint32_t pid_stride;  /* row p uses RNG particle id pid_base + p * pid_stride;
                           0 means 1 (interleaved ids for sharding or mixed sets) */
  int32_t regroup;      /* batched: every `regroup` iterations the lanes of a block are
                           regrouped by next action (SSA step or leap) so that waves are
                           homogeneous; 0 = off, 1..64 (one lane per trajectory only) */
  int32_t lanes_per_traj; /* batched: lanes per trajectory, 1, 2, 4, 8 or 16 (0 = 1); the lanes of a
                           trajectory split its Poisson draws and upcoming SSA draws;
                           lanes_per_wave counts lanes, so a wave holds
                           lanes_per_wave / lanes_per_traj trajectories.  Networks
                           beyond 16 species or 32 reactions: 0 = one trajectory per
                           wave, 1 = one per lane */
  int32_t jacobian;     /* Jacobian of the implicit solve: LX_JAC_ANALYTIC (0, default,
                           the exact mass-action derivative, which is what a symbolic
                           Jacobian gives) or LX_JAC_FD (1, forward differences with the
                           step 2^-26 max(|y_k|, 1): the numerically estimated Jacobian
                           (Background section), or LX_JAC_USER (2, the caller's symbolic
                           derivative terms, lx_network_create_jac) */
  int32_t check_lanes;  /* 1: after launching, wait for the stream and read the status
                           of every trajectory from `stats` (which must then be
                           given); return LX_W_LANE_FAIL if any is not LX_LANE_OK,
                           with the count and the first one in lx_last_error().
                           The call is then synchronous.  0 (default): return at
                           once; statuses are in `stats` when the stream is done */
  uint64_t cycles;      /* 0 (default), or the device address of a uint64 [P][4] buffer:
                           the simulation then runs a variant that reads the GPU clock
                           and writes, per trajectory, the cycles spent in (0) assembling
                           the implicit solve's Jacobian, (1) its LU solves, (2) the whole
                           implicit solves (Newton iterations and count rounding) and (3)
                           the whole trajectory.  Measurement only; results unchanged.
                           lx_simulate and lx_simulate_grid, regroup 0 */
  int32_t tail_lanes;   /* batched, one lane per trajectory: once a block has no particles
                           left to hand out and at most 64 / tail_lanes trajectories are
                           still running in a wave, the wave gives each of them a group
                           of tail_lanes lanes (as lanes_per_traj) to finish it; 0 = off
                           (default), 2, 4, 8 or 16.  Results unchanged */
  int32_t waves_per_simd; /* register budget: 0 = the compiler's choice (default; for
                           the one-trajectory-per-wave kernel of large networks, the
                           waves per SIMD of the blocks its LDS lets be resident,
                           rounded up, at most 4), else
                           1..8 -- the kernel is compiled to keep at least this many
                           waves resident per SIMD (fewer registers per lane, spills if
                           needed).  Results unchanged */
} lx_options;

/* Per-trajectory statistics (80 bytes). */
typedef struct lx_stats {
  int32_t status;      /* LX_LANE_* */
  uint32_t crit_fired; /* accepted leaps in which a critical reaction fired
                          (at most the attempts, so below 2^32) */
  double t_final; /* time reached (t_end unless status != OK) */
  int64_t steps_ssa, steps_explicit, steps_implicit; /* accepted actions by kind */
  int64_t rejections;   /* leap attempts rejected (negative state, failed solve) */
  int64_t newton_iters; /* Newton iterations */
  int64_t newton_fail;  /* implicit solves that did not converge */
  int64_t kclip;        /* implicit counts clipped at zero */
  int64_t attempts;     /* SSA steps + leap attempts (RNG attempt index) */
} lx_stats;

typedef struct lx_network_s* lx_network;

/* Fill *opt with the defaults above.  opt must be non-null. */
void lx_options_default(lx_options* opt);

/* Thread-local message describing the last non-OK status of this thread. */
const char* lx_last_error(void);

/* Compile a network from a flat table (paper, Background section: mass-action
 * propensities a_j = theta_j g_j(X), g_j a function of the reactant copy
 * numbers).
 *   N, M              species and reactions, N, M >= 1.
 *   reactant_order    host int32 [M][N], m_ij >= 0 molecules of species i
 *                     consumed by reaction j; order_j = sum_i m_ij <= 3.
 *   product_coeff     host int32 [M][N], p_ij >= 0 molecules produced.
 * g_j(X) = prod_i C(X_i, m_ij) (distinct-combination convention).
 * Sizes: N <= 64, M <= 256.  Networks with N <= 16 and M <= 32 run kernels
 * whose per-lane state lives in registers; larger ones run kernels that read
 * the stoichiometry as compressed tables and solve implicit leaps with the
 * whole wave on one Newton system in LDS: the batched schedule runs one
 * trajectory per wave (reactions and species spread over the lanes, the
 * waves of a block sharing the Newton area), the plain schedule, or the
 * batched one with lanes_per_traj = 1, one trajectory per lane with its
 * arrays in the lane-interleaved private segment (no network sets, no
 * particle filter, lanes_per_traj at most 1, regroup and tail_lanes 0).
 * Errors: LX_E_INVALID for a bad table or a network above those sizes.
 * *out receives a handle owned by the caller and released with
 * lx_network_destroy. */
lx_status lx_network_create(int32_t N, int32_t M, const int32_t* reactant_order,
                            const int32_t* product_coeff, lx_network* out);

/* lx_network_create with a caller-supplied Jacobian for the implicit solve
 * (paper, Background section: the Jacobian of the implicit leap is
 * estimated numerically unless a symbolic one is provided).  The caller gives
 * d g_j / d y_k, for reactions j and their reactant species k, as polynomial
 * terms: term t contributes coef[t] * prod_i y_i^powers[t][i] to
 * d g_j / d y_k with (j, k) = (rxn[t], wrt[t]); the solve multiplies by
 * theta_j.  Evaluation: per term, coef times repeated products in ascending
 * species order; per (j, k), the terms summed from zero in table order; a
 * reactant pair with no terms has derivative 0.  Simulations with
 * opt->jacobian = LX_JAC_USER use these terms (the other choices stay
 * available).
 *   n_terms   1 .. 65536.
 *   rxn, wrt  host int32 [n_terms]: reaction index in [0, M) and one of its
 *             reactant species (m_kj > 0).
 *   coef      host double [n_terms], finite.
 *   powers    host int32 [n_terms][N], each in [0, 16].
 * Arrays are read during the call only.  Errors: those of
 * lx_network_create, and LX_E_INVALID for a term outside these rules. */
lx_status lx_network_create_jac(int32_t N, int32_t M, const int32_t* reactant_order,
                                const int32_t* product_coeff, int32_t n_terms,
                                const int32_t* rxn, const int32_t* wrt, const double* coef,
                                const int32_t* powers, lx_network* out);

/* Compile (hipRTC, gfx950) and cache on disk the simulation kernel of a
 * network for a precision, schedule and block size (0 = default) without
 * running it; needs no GPU.  Optional: lx_simulate compiles on first use. */
lx_status lx_network_prepare(lx_network net, int32_t precision, int32_t schedule,
                             int32_t block_size);

/* Release a handle and its compiled kernels.  NULL is accepted. */
lx_status lx_network_destroy(lx_network net);

/* Query sizes and the number of reversible pairs found (reactions with
 * exactly opposite net-change vectors, paired in ascending index). */
lx_status lx_network_info(lx_network net, int32_t* N, int32_t* M, int32_t* n_pairs);

/* Simulate P trajectories from t_start to t_end (paper: Implementation
 * section -- adaptive explicit-implicit tau-leaping with critical reactions,
 * the implicit switch when excluding reaction pairs in partial equilibrium
 * gives a much larger leap, and the switch to SSA when the wait for the next
 * critical reaction is comparable to the wait for the next reaction; tau
 * bounded by the relative change of the propensities with accuracy eps,
 * Background section).
 *   theta   device double [P][M]: rate constants per trajectory (>= 0, finite).
 *   x0      device int32  [P][N]: initial copy numbers (>= 0).
 *   t_end   final time (>= opt->t_start); eps > 0 (the paper uses 0.03).
 *   mode    LX_MODE_*.
 *   opt     options or NULL for the defaults.
 *   x_out   device int32  [P][N]: X(t_end).
 *   r_out   device int32  [P][M]: firing counts (input too if accumulate).
 *   G_out   device double [P][M]: integral of g_j over [t_start, t_end] --
 *           trapezoid rule over leaps, exact over SSA steps (input too if
 *           accumulate).
 *   stats   device lx_stats [P] or NULL.
 *   stream  hipStream_t or NULL.
 * Rows are trajectories, row-major.  Results depend only on (seed,
 * rng_stream, pid_base + p) and the inputs, never on the schedule or block
 * size.  P = 0 is a no-op.  Errors: LX_E_INVALID (null pointers with P > 0,
 * bad options), LX_E_UNSUPPORTED (not gfx950), LX_E_COMPILE, LX_E_HIP. */
lx_status lx_simulate(lx_network net, int64_t P, const double* theta, const int32_t* x0,
                      double t_end, double eps, int32_t mode, const lx_options* opt,
                      int32_t* x_out, int32_t* r_out, double* G_out, lx_stats* stats,
                      void* stream);

/* lx_simulate with observation times: the trajectories also stop at each of
 * times[0..n_times) and their states there are written out (the paper
 * measures accuracy on species distributions at fixed time points, Results
 * section).  A trajectory stops at an observation time as it stops at t_end
 * (a leap is shortened to end there and no critical reaction fires; an SSA
 * step whose waiting time passes it integrates g up to it and does not fire;
 * an absorbing state integrates g up to it), records its state, and goes on
 * from there with fresh step decisions and the same random stream.  The
 * simulation ends at times[n_times - 1].
 *   times   device double [n_times]: non-decreasing, from opt->t_start, finite.
 *           A trajectory meeting a time below its current time, or not
 *           finite, ends with status LX_LANE_BAD_INPUT.
 *   x_grid  device int32 [P][n_times][N]: X(times[k]); -1 in every row whose
 *           time the trajectory did not reach with status OK.
 *   other arguments as lx_simulate; x_out, r_out, G_out and stats describe
 *   the end of the simulation (or where the trajectory stopped).
 * n_times = 1 with times[0] = t_end gives exactly lx_simulate's results.
 * Errors as lx_simulate, and LX_E_INVALID for n_times < 1 or a null times /
 * x_grid pointer with P > 0. */
lx_status lx_simulate_grid(lx_network net, int64_t P, const double* theta, const int32_t* x0,
                           int32_t n_times, const double* times, double eps, int32_t mode,
                           const lx_options* opt, int32_t* x_grid, int32_t* x_out,
                           int32_t* r_out, double* G_out, lx_stats* stats, void* stream);

/* One network of a multi-network simulation. */
typedef struct lx_set_item {
  lx_network net;
  int64_t P;
  const double* theta; /* device [P][M of net] */
  const int32_t* x0;   /* device [P][N of net] */
  int32_t* x_out;      /* device [P][N] */
  int32_t* r_out;      /* device [P][M] */
  double* G_out;       /* device [P][M] */
  lx_stats* stats;     /* device [P] or NULL */
  uint32_t pid_base;   /* RNG particle id of row p: pid_base + p * pid_stride */
  uint32_t pid_stride; /* 0 means 1 */
} lx_set_item;

/* Simulate several networks in one launch (batched schedule): K in [1, 8]
 * items, each with its own network, ensemble and buffers.  Every block owns
 * an equal slice of every item and runs the items one after another (a wave
 * moves to the next item as soon as its lanes have drained the block's slice
 * of the current one), so networks of very different cost still load every
 * block alike and no wave mixes networks at a time.  Results are identical to K separate lx_simulate calls
 * with the same ids.  t_end, eps, mode and options (precision, control
 * constants, seed, rng_stream, accumulate, tuning) are shared; opt->schedule,
 * pid_base and pid_stride are ignored in favour of the items.  Errors as for
 * lx_simulate. */
lx_status lx_simulate_set(int32_t K, const lx_set_item* items, double t_end, double eps,
                          int32_t mode, const lx_options* opt, void* stream);

/* ---- Particle filter over observation intervals ---------------------------
 * The paper's motivating use (Background and Discussion sections): particle-
 * filter Bayesian inference with the conjugate update theta_j | path ~
 * Gamma(alpha_j + r_j, beta_j + G_j).  Interval k = 1..K covers
 * [(k-1) dt, k dt]:
 *   1. every particle is simulated over the interval (lx_simulate semantics,
 *      r and G accumulated, RNG stream opt->rng_stream + k, particle id = row);
 *   2. weight = Gaussian density of observation y[k-1] of species obs_species
 *      with sd obs_sd; particles whose simulation failed weigh zero;
 *   3. weights become integer codes floor(exp(lw - max lw) 2^40) (all equal if
 *      every code is zero) and P ancestors are drawn by multinomial
 *      resampling with exact integer prefix sums;
 *   4. each new particle takes its ancestor's state and cumulative r, G and
 *      draws theta_j ~ Gamma(alpha_j + r_j, rate beta_j + G_j);
 *   5. loglik[k-1] = max lw + log(mean code 2^-40) (-inf if every weight is 0).
 * All buffers are device memory owned by the caller; the workspace replaces
 * any allocation by the library. */
typedef struct lx_pf_problem {
  lx_network net;
  int64_t P;            /* particles, 1 .. 2^23 */
  int32_t K;            /* observation intervals >= 1 */
  int32_t obs_species;  /* observed species index */
  double dt;            /* interval length > 0 */
  double obs_sd;        /* observation noise sd > 0 */
  const double* y;      /* [K] observations */
  const double* alpha;  /* [M] prior shapes (> 0) */
  const double* beta;   /* [M] prior rates (> 0; a shape or rate out of range makes the
                           refreshed theta invalid and its particle ends the next
                           interval with LX_LANE_BAD_INPUT, weight zero) */
  double* theta;        /* [P][M] in: initial parameters; out: last refresh */
  int32_t* x;           /* [P][N] in: initial states; out: states at K dt */
  int32_t* r;           /* [P][M] cumulative firing counts (normally zero at entry) */
  double* G;            /* [P][M] cumulative integrals of g (normally zero at entry) */
  double* loglik;       /* [K] log-likelihood increments */
  void* workspace;      /* >= lx_pf_workspace_size bytes, 256-byte aligned */
  size_t workspace_bytes;
} lx_pf_problem;

/* Bytes of workspace the filter needs for P particles of an N x M network. */
lx_status lx_pf_workspace_size(int64_t P, int32_t N, int32_t M, size_t* bytes);

/* Enqueue the K intervals on `stream` (direct launches).  eps, mode and opt as
 * for lx_simulate (opt->t_start, accumulate, pid_base/stride are set by the
 * filter). */
lx_status lx_pf_run(const lx_pf_problem* pb, double eps, int32_t mode, const lx_options* opt,
                    void* stream);

/* lx_pf_run for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation): the
 * same filter, with pb->workspace and pb->workspace_bytes ignored in favour
 * of a scratch array inside the library (64 MiB, a file-scope device array
 * that each GPU the library runs on holds until the process ends; 2^18
 * particles of a 4 x 6 network fit).  The call allocates nothing: it calls no
 * hipMalloc/hipFree and loads no kernel.  Its first call on a device looks up
 * the array's device address (which may load the library's own device code
 * there).  Every call on a GPU shares that GPU's array, so calls that overlap
 * on one GPU race; stream-ordered calls do not.  Errors: as lx_pf_run, and
 * LX_E_INVALID when the filter needs more scratch than the array holds
 * (lx_pf_workspace_size above 64 MiB) or when the simulation kernel for these
 * options has not been loaded on this device yet (run the same filter once
 * through lx_pf_run, which loads it). */
lx_status lx_pf_run_static(const lx_pf_problem* pb, double eps, int32_t mode,
                           const lx_options* opt, void* stream);

/* A captured filter: all K intervals recorded once into a HIP graph on a
 * non-default `stream` (capture happens during the call; nothing executes),
 * then replayed by lx_pf_graph_launch on any stream.  The graph refers to the
 * problem's buffers, which must outlive it.  Every replay runs the whole
 * filter again from the buffers' current contents. */
typedef struct lx_pf_graph_s* lx_pf_graph;
lx_status lx_pf_graph_create(const lx_pf_problem* pb, double eps, int32_t mode,
                             const lx_options* opt, void* stream, lx_pf_graph* out);
lx_status lx_pf_graph_launch(lx_pf_graph g, void* stream);
lx_status lx_pf_graph_destroy(lx_pf_graph g);

/* ---- Test hooks: run the production device functions on fixed inputs. ----
 * All pointers are device memory; n elements; enqueued on stream. */

/* Philox4x32-10 (Salmon et al. 2011): ctr [n][4], key [n][2] -> out [n][4]. */
lx_status lx_test_philox(int64_t n, const uint32_t* ctr, const uint32_t* key, uint32_t* out,
                         void* stream);
/* Uniform maps: f64 from word pairs w [n][2]; f32 from words w [n]. */
lx_status lx_test_uniform_f64(int64_t n, const uint32_t* w, double* out, void* stream);
lx_status lx_test_uniform_f32(int64_t n, const uint32_t* w, float* out, void* stream);
/* Elementary functions used by the samplers: fn = 0 exp_f64, 1 log_f64,
 * 2 lfact (log k!), 3 sqrt_f64 (in/out double); 10 exp_f32, 11 log_f32,
 * 12 sqrt_f32 (in/out float). */
lx_status lx_test_math(int32_t fn, int64_t n, const void* in, void* out, void* stream);
/* Poisson(lam[q]) drawn at site (pid[q], e[q], site[q]) with key (seed,
 * stream_id); lambda_thr in [10,30] as in lx_options; precision LX_PREC_*;
 * out int64 (-1 = beyond range). */
lx_status lx_test_poisson(int64_t n, const double* lam, const uint32_t* pid, const uint32_t* e,
                          const uint32_t* site, uint64_t seed, uint32_t stream_id,
                          double lambda_thr, int32_t precision, int64_t* out, void* stream);
/* Gamma(shape[q], 1) at site (pid[q], e[q], Gamma site + j[q]) (the
 * particle filter's refresh sampler); out double. */
lx_status lx_test_gamma(int64_t n, const double* shape, const uint32_t* pid, const uint32_t* e,
                        const uint32_t* j, uint64_t seed, uint32_t stream_id, double* out,
                        void* stream);
/* Exponential(1) = -log(U) at site (pid[q], e[q], SSA site). */
lx_status lx_test_exponential(int64_t n, const uint32_t* pid, const uint32_t* e, uint64_t seed,
                              uint32_t stream_id, int32_t precision, double* out, void* stream);
/* Step decision for Q states of a network: propensities a [Q][M] (as double),
 * critical and equilibrium masks crit/eq [Q][W], W = ceil(M/32) words per
 * state (reaction j is bit j % 32 of word j / 32; W = 1 up to 32 reactions), tau [Q][2]
 * = (tau_ex, tau_im or +inf), action [Q] (0 explicit leap, 1 implicit leap,
 * 2 SSA burst, 3 absorbing).  theta [Q][M], x [Q][N].  Uses opt->precision
 * and the control constants; eps and mode as in lx_simulate. */
lx_status lx_test_tau_select(lx_network net, int64_t Q, const double* theta, const int32_t* x,
                             double eps, int32_t mode, const lx_options* opt, double* a,
                             uint32_t* crit, uint32_t* eq, double* tau, int32_t* action,
                             void* stream);
/* Implicit-leap solve for Q cases: given tau [Q], Poisson draws Pj [Q][M]
 * (int64) and critical firing jc [Q] (-1 none), the non-critical set
 * {j : a_j > 0, j != jc}; outputs k [Q][M] (int64), ok [Q], iters [Q].
 * opt->jacobian selects the analytic or forward-difference Jacobian;
 * newton_tol and newton_maxit apply. */
lx_status lx_test_implicit(lx_network net, int64_t Q, const double* theta, const int32_t* x,
                           const double* tau, const int64_t* Pj, const int32_t* jc,
                           const lx_options* opt, int64_t* k, int32_t* ok, int32_t* iters,
                           void* stream);

#ifdef __cplusplus
}
#endif

#endif /* LX_H_ */
