// lx_params.h -- plain-data structures shared by the host library and the
// kernels it compiles at run time (no includes, no HIP types).
#pragma once

namespace lx {

enum Mode { MODE_ADAPTIVE = 0, MODE_EXPLICIT = 1, MODE_SSA = 2 };

// Per-trajectory status (lx_stats.status).
enum LaneStatus {
  LANE_OK = 0,
  LANE_STEP_BUDGET = 1,      // max_steps attempts used before t_end
  LANE_LAMBDA_OVERFLOW = 2,  // a Poisson mean beyond the sampler's range
  LANE_BAD_INPUT = 3,        // negative or non-finite theta, negative x0
  LANE_COUNT_OVERFLOW = 4    // a copy number or firing count beyond int32
};

// Kernel parameters, passed by value.
struct SimParams {
  double t_start, t_end;
  double eps, delta, n_stiff, k_ssa, k_crit, lam_thr, newton_tol;
  long long max_steps;
  long long P;
  unsigned int k0, k1, pid_base, pid_stride;
  int n_c, n_ssa_ex, n_ssa_im, newton_maxit, kcap, mode, accumulate;
  int jacobian;           // implicit solve: 0 analytic Jacobian, 1 forward differences
  // batched scheduler
  long long per_block;    // particles owned by each block (contiguous range)
  int lanes;              // active lanes per wave (4 to 64)
  int ssa_k;              // SSA steps a lane in an SSA burst takes per leap iteration
  int regroup;            // regroup lanes by next action every `regroup` iterations (0: never)
  int tail;               // lanes per trajectory for the end of a block's range (0: off)
  int waves;              // register budget: waves per SIMD the kernel is compiled for (0: default)
  // observation times (kernels compiled with LX_GRID): the state at
  // times[k], k < n_times, goes to x_grid [P][n_times][N]
  const double* times;
  int* x_grid;
  int n_times;
  // clock cycles per trajectory [P][4] (kernels compiled with LX_TIMERS)
  unsigned long long* cycles;
};

// Register budget of the simulation kernels (waves_per_simd option).
#ifdef LX_WAVES
#define LX_WAVES_ATTR __attribute__((amdgpu_waves_per_eu(LX_WAVES)))
#else
#define LX_WAVES_ATTR
#endif

// Cycle timers of the LX_TIMERS variant: LX_CLOCK reads the GPU's clock.
#ifdef LX_TIMERS
#define LX_CLOCK() __builtin_amdgcn_s_memtime()
#else
#define LX_CLOCK() 0ull
#endif

// Per-trajectory statistics (layout of the public lx_stats).
// Method constants of a launch (the fields of SimParams named below).  A
// generated kernel source may define LX_CONST together with a struct LxConst
// holding them as compile-time values -- the host then compiles one kernel
// per set of values, so they fold into immediates and occupy no scalar
// registers; otherwise they are read from the launch parameters.
#ifdef LX_CONST
#define LXP(prm, f) (::LxConst::f)
#else
#define LXP(prm, f) ((prm).f)
#endif

struct Stats {
  int status;
  unsigned int crit_fired;  // accepted leaps in which a critical reaction fired
  double t_final;
  long long steps_ssa, steps_explicit, steps_implicit, rejections, newton_iters, newton_fail,
      kclip, attempts;
};

// One network of a multi-network launch (lx_simulate_set): every block of
// the launch owns the slice [blk * per_block, (blk + 1) * per_block) of it.
struct SetItem {
  const double* theta;
  const int* x0;
  int* x_out;
  int* r_out;
  double* G_out;
  Stats* stats;
  long long P, per_block;
  int lanes, pad;
  unsigned int pid_base, pid_stride;
};

constexpr int SET_MAX = 8;
struct SetArgs {
  int K, pad;
  SetItem it[SET_MAX];
};
// Particle-filter workspace pieces (lx_pf.hip), carved from the caller's buffer.
struct PfWork {
  int* x2;
  int* r2;
  double* G2;
  double* lw;
  unsigned long long* codes;
  unsigned long long* scan;
  Stats* stats;
  double* bmax;
  unsigned long long* bsum;
  double* mx;
  unsigned long long* total;
};
}  // namespace lx
