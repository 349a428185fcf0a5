// lx_sim.h -- network-specialised simulation of one trajectory per lane.
//
// Compiled at run time by hipRTC after lx_device.h, lx_params.h and a
// generated block that defines one traits struct per network (LxNet0, LxNet1,
// ...; LxNet is the first) with static constexpr members:
//   N, M         species and reactions (M <= 32, N <= 16 here; larger
//                networks run the kernels of lx_sim_large.h)
//   RO[M][N]     reactant orders m_ij
//   NU[M][N]     net changes nu_ij = p_ij - m_ij
//   PHI[N]       case of the tau-bound factor of each species (0: not a reactant)
//   PARTNER[M]   reversible partner reaction or -1;  NPAIRS
// Every loop over species or reactions has a compile-time trip count and is
// unrolled, so per-lane state lives in registers and the tables fold into
// immediate operands.
//
// The method (matLeap, arXiv 1608.07058): a_j = theta_j g_j(X) and the
// statistics r_j (firings), G_j = integral of g_j (trapezoid while leaping,
// exact during SSA) -- Background section; adaptive explicit/implicit leaping
// with critical reactions, the partial-equilibrium implicit switch and the
// switch to SSA when critical reactions are fast -- Implementation section;
// tau bounded by the relative-change rule of Cao et al. 2006 -- Background.
#pragma once

namespace lx {

__device__ __forceinline__ double binom_real(double y, int mult) {
  if (mult == 1) return y;
  if (mult == 2) return (y * (y - 1.0)) * 0.5;
  return ((y * (y - 1.0)) * (y - 2.0)) / 6.0;
}

__device__ __forceinline__ double binom_real_deriv(double y, int mult) {
  if (mult == 1) return 1.0;
  if (mult == 2) return y - 0.5;
  return ((3.0 * y - 6.0) * y + 2.0) / 6.0;
}

// g_j(y) = prod over reactant species (ascending) of C(y_i, m_ij).
template <class NET>
__device__ __forceinline__ void g_all(const double (&y)[NET::N], double (&g)[NET::M]) {
#pragma unroll
  for (int j = 0; j < NET::M; ++j) {
    double gj = 1.0;
#pragma unroll
    for (int i = 0; i < NET::N; ++i)
      if (NET::RO[j][i] > 0) gj = gj * binom_real(y[i], NET::RO[j][i]);
    g[j] = gj;
  }
}

// g_j(y) with y_k replaced by yk (a forward-difference evaluation).
template <class NET>
__device__ __forceinline__ double g_moved(int j, int k, const double (&y)[NET::N], double yk) {
  double gj = 1.0;
#pragma unroll
  for (int i = 0; i < NET::N; ++i)
    if (NET::RO[j][i] > 0) gj = gj * binom_real(i == k ? yk : y[i], NET::RO[j][i]);
  return gj;
}

// Forward-difference step of species k at y: the step 2^-26 max(|y_k|, 1)
// (square root of the binary64 epsilon, scaled), taken as the representable
// difference (y_k + step) - y_k; returns the moved coordinate in *yh.
__device__ __forceinline__ double fd_step(double yk, double* yh) {
  const double ak = __builtin_fabs(yk);
  const double step = 0x1p-26 * (ak < 1.0 ? 1.0 : ak);
  *yh = yk + step;
  return *yh - yk;
}

// d g_j / d y_k.
template <class NET>
__device__ __forceinline__ double dg_of(int j, int k, const double (&y)[NET::N]) {
  double gj = 1.0;
#pragma unroll
  for (int i = 0; i < NET::N; ++i) {
    if (NET::RO[j][i] == 0) continue;
    gj = gj * (i == k ? binom_real_deriv(y[i], NET::RO[j][i]) : binom_real(y[i], NET::RO[j][i]));
  }
  return gj;
}

// d g_j / d y_k from the caller's derivative terms of (j, k) (NET::JT_*):
// each term its coefficient times repeated products of y in ascending species
// order, summed from zero in table order.  j and k are compile-time after
// unrolling, so only that pair's terms remain.
template <class NET>
__device__ __forceinline__ double dg_user(int j, int k, const double (&y)[NET::N]) {
  double s = 0.0;
#pragma unroll
  for (int t = 0; t < NET::NJT; ++t) {
    if (NET::JT_J[t] != j || NET::JT_K[t] != k) continue;
    double v = NET::JT_C[t];
#pragma unroll
    for (int f = NET::JT_PTR[t]; f < NET::JT_PTR[t + 1]; ++f)
#pragma unroll
      for (int e = 0; e < NET::JT_PW[f]; ++e) v = v * y[NET::JT_SP[f]];
    s = s + v;
  }
  return s;
}

// Cross-lane read within groups of TPL lanes (lane s of the caller's group).
// Groups of 2 and 4 lanes lie within a quad of the wave, so the read is a
// DPP quad permutation (a VALU move, no LDS round trip); a group of 16 is a
// DPP row, read with a row broadcast, and a group of 8 is half a row, read
// with two row broadcasts whose bank masks select the half.  `s` is a
// compile-time constant after unrolling, so the branches fold away.
template <int W, int S = 0>
__device__ __forceinline__ int row_group_read(int v, int s) {
  if constexpr (S + 1 < W) {
    if (s != S) return row_group_read<W, S + 1>(v, s);
  }
  if constexpr (W == 16) {
    return __builtin_amdgcn_update_dpp(0, v, 0x150 + S, 0xF, 0xF, false);  // row_newbcast:S
  } else {
    // lanes 0-7 of the row (banks 0, 1) read lane S, lanes 8-15 lane 8 + S
    const int lo = __builtin_amdgcn_update_dpp(0, v, 0x150 + S, 0xF, 0x3, false);
    return __builtin_amdgcn_update_dpp(lo, v, 0x158 + S, 0xF, 0xC, false);
  }
}

template <int TPL>
__device__ __forceinline__ int group_read_b32(int v, int s) {
  if constexpr (TPL == 16 || TPL == 8) {
    return row_group_read<TPL>(v, s);
  } else if constexpr (TPL == 4) {
    switch (s) {
      case 0: return __builtin_amdgcn_update_dpp(0, v, 0x00, 0xF, 0xF, false);
      case 1: return __builtin_amdgcn_update_dpp(0, v, 0x55, 0xF, 0xF, false);
      case 2: return __builtin_amdgcn_update_dpp(0, v, 0xAA, 0xF, 0xF, false);
      default: return __builtin_amdgcn_update_dpp(0, v, 0xFF, 0xF, 0xF, false);
    }
  } else if constexpr (TPL == 2) {
    if (s == 0) return __builtin_amdgcn_update_dpp(0, v, 0xA0, 0xF, 0xF, false);
    return __builtin_amdgcn_update_dpp(0, v, 0xF5, 0xF, 0xF, false);
  } else {
    return __shfl(v, s, TPL);
  }
}

template <int TPL, class T>
__device__ __forceinline__ T group_read(T v, int s) {
  if constexpr (TPL == 2 || TPL == 4 || TPL == 8 || TPL == 16) {
    if constexpr (sizeof(T) == 4) {
      return __builtin_bit_cast(T, group_read_b32<TPL>(__builtin_bit_cast(int, v), s));
    } else {
      static_assert(sizeof(T) == 8, "32- or 64-bit values");
      const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
      const unsigned lo = (unsigned)group_read_b32<TPL>((int)(unsigned)b, s);
      const unsigned hi = (unsigned)group_read_b32<TPL>((int)(unsigned)(b >> 32), s);
      return __builtin_bit_cast(T, ((unsigned long long)hi << 32) | lo);
    }
  } else {
    return __shfl(v, s, TPL);
  }
}

// Lane state of one trajectory.  With TPL > 1 a trajectory occupies TPL lanes
// that hold identical state and run identical control flow; they split the
// Poisson draws of a leap (one reaction each) and the draws of upcoming SSA
// steps (one attempt each) and exchange the results, so every value is the
// one the single-lane form computes.  With GRID the trajectory also stops at
// observation times (prm.times) and records its state there (grid_next).
template <class P, class NET, int TPL = 1, bool GRID = false>
struct Lane {
  typedef typename P::R R;
  static constexpr int N = NET::N;
  static constexpr int M = NET::M;
  static_assert(M <= 32, "reaction masks are 32-bit");

  // particle state
  u32 pid;
  double th[M];
  R thr[M];
  int x[N];
  int r[M];
  double G[M];
  double t;
  u32 e;
  int status;
  double tend;  // end of the current stretch: the next observation time (GRID)
  int kt;       // index of that time (GRID)
  // step state
  double g[M];
  R a[M];
  R a0, a0c;
  u32 crit, ncr;  // reaction bitmasks
  bool plan, gvalid, implicit;
  R tau_p;
  int ssa_left;
  // counters
  u32 n_ssa, n_ex, n_im, n_rej, n_nfail, n_clip, n_cf;  // < 2^32: attempts are bounded by max_steps
  long long n_nit;
  // clock cycles (LX_TIMERS): Jacobian assembly, LU solves, implicit solves, start
  unsigned long long cy_jac, cy_lu, cy_imp, cy_t0;

  // The time the trajectory runs to now: t_end, or the next observation time.
  __device__ __forceinline__ double t_end_(const SimParams& prm) const {
    if constexpr (GRID) return tend;
    else return prm.t_end;
  }

  __device__ __forceinline__ bool active(const SimParams& prm) const {
    return (status == LANE_OK) & (t < t_end_(prm));  // no short circuit: one condition
  }

  __device__ __forceinline__ void load(long long p, const double* __restrict__ theta,
                                       const int* __restrict__ x0, const int* r_in,
                                       const double* G_in, const SimParams& prm) {
    pid = prm.pid_base + (u32)p * prm.pid_stride;
    bool bad = false;
#pragma unroll
    for (int j = 0; j < M; ++j) {
      th[j] = theta[p * M + j];
      thr[j] = (R)th[j];
      bad = bad || !(th[j] >= 0.0) || th[j] == LX_INF_F64;
      r[j] = LXP(prm, accumulate) ? r_in[p * M + j] : 0;
      G[j] = LXP(prm, accumulate) ? G_in[p * M + j] : 0.0;
    }
#pragma unroll
    for (int i = 0; i < N; ++i) {
      x[i] = x0[p * N + i];
      bad = bad || x[i] < 0;
    }
    status = bad ? LANE_BAD_INPUT : LANE_OK;
    t = prm.t_start;
    if constexpr (GRID) {
      kt = 0;
      tend = prm.times[0];
      if (!(tend >= t) || tend == LX_INF_F64) status = LANE_BAD_INPUT;
    }
    e = 0;
    plan = false;
    gvalid = false;
    implicit = false;
    ssa_left = 0;
    n_ssa = n_ex = n_im = n_rej = n_nit = n_nfail = n_clip = n_cf = 0;
    cy_jac = cy_lu = cy_imp = 0;
    cy_t0 = LX_CLOCK();
  }

  // Cycle timers of the trajectory (LX_TIMERS variant) as row p of prm.cycles.
  __device__ __forceinline__ void store_cycles(long long p, const SimParams& prm) const {
#ifdef LX_TIMERS
    unsigned long long* c = prm.cycles + p * 4;
    c[0] = cy_jac;
    c[1] = cy_lu;
    c[2] = cy_imp;
    c[3] = LX_CLOCK() - cy_t0;
#endif
  }

  __device__ __forceinline__ void store(long long p, int* x_out, int* r_out, double* G_out,
                                        Stats* stats) const {
#pragma unroll
    for (int i = 0; i < N; ++i) x_out[p * N + i] = x[i];
#pragma unroll
    for (int j = 0; j < M; ++j) {
      r_out[p * M + j] = r[j];
      G_out[p * M + j] = G[j];
    }
    if (stats) {
      Stats s;
      s.status = status;
      s.crit_fired = n_cf;
      s.t_final = t;
      s.steps_ssa = n_ssa;
      s.steps_explicit = n_ex;
      s.steps_implicit = n_im;
      s.rejections = n_rej;
      s.newton_iters = n_nit;
      s.newton_fail = n_nfail;
      s.kclip = n_clip;
      s.attempts = e;
      stats[p] = s;
    }
  }

  // Observation times: called when the lane has stopped, at its current
  // time tend (status OK) or for good.  Records the state as row kt of
  // x_grid [P][n_times][N] (-1 where the time was not reached in status OK;
  // only `writer` stores) and opens the stretch to the next time, with fresh
  // step decisions and the same random stream.  A next time below the
  // current one, or not finite, ends the trajectory with BAD_INPUT.  Returns
  // true if the trajectory goes on.
  __device__ __forceinline__ bool grid_next(long long p, const SimParams& prm, bool writer) {
    const bool ok = status == LANE_OK;
    int* row = prm.x_grid + ((long long)p * prm.n_times + kt) * N;
    if (writer) {
#pragma unroll
      for (int i = 0; i < N; ++i) row[i] = ok ? x[i] : -1;
    }
    kt += 1;
    if (ok && kt < prm.n_times) {
      const double tn = prm.times[kt];
      if ((tn >= t) & (tn != LX_INF_F64)) {
        tend = tn;
        ssa_left = 0;
        plan = false;
        return true;
      }
      status = LANE_BAD_INPUT;
    }
    if (writer) {
      for (int k = kt; k < prm.n_times; ++k) {
        row += N;
#pragma unroll
        for (int i = 0; i < N; ++i) row[i] = -1;
      }
    }
    return false;
  }

  // Number of 32-bit words of the state moved when lanes are regrouped.
  static constexpr int STATE_WORDS = 21 + N + 3 * M + (GRID ? 3 : 0);

  // Write the trajectory's state to an LDS slot (regrouping).  theta, g, a
  // and the plan's masks are not moved: they are reloaded or recomputed.
  __device__ __forceinline__ void save(long long p, u32* w) const {
    int q = 0;
    w[q++] = (u32)p;
    w[q++] = (u32)((unsigned long long)p >> 32);
    w[q++] = pid;
#pragma unroll
    for (int i = 0; i < N; ++i) w[q++] = (u32)x[i];
#pragma unroll
    for (int j = 0; j < M; ++j) w[q++] = (u32)r[j];
#pragma unroll
    for (int j = 0; j < M; ++j) {
      const unsigned long long b = __builtin_bit_cast(unsigned long long, G[j]);
      w[q++] = (u32)b;
      w[q++] = (u32)(b >> 32);
    }
    const unsigned long long tb = __builtin_bit_cast(unsigned long long, t);
    w[q++] = (u32)tb;
    w[q++] = (u32)(tb >> 32);
    w[q++] = e;
    w[q++] = (u32)status;
    w[q++] = (plan ? 1u : 0u) | (implicit ? 2u : 0u);
    const double tp = (double)tau_p;
    const unsigned long long pb = __builtin_bit_cast(unsigned long long, tp);
    w[q++] = (u32)pb;
    w[q++] = (u32)(pb >> 32);
    w[q++] = (u32)ssa_left;
    w[q++] = n_ssa;
    w[q++] = n_ex;
    w[q++] = n_im;
    w[q++] = n_rej;
    w[q++] = n_nfail;
    w[q++] = n_clip;
    w[q++] = n_cf;
    w[q++] = (u32)n_nit;
    w[q++] = (u32)((unsigned long long)n_nit >> 32);
    if constexpr (GRID) {
      const unsigned long long eb = __builtin_bit_cast(unsigned long long, tend);
      w[q++] = (u32)eb;
      w[q++] = (u32)(eb >> 32);
      w[q++] = (u32)kt;
    }
  }

  // Read a state written by save(); theta is reloaded from the input, the
  // propensities (and, for a lane retrying a leap, its plan's critical set)
  // are recomputed from the state, which reproduces them exactly.
  __device__ __forceinline__ long long restore(const u32* w, const double* __restrict__ theta,
                                               const SimParams& prm) {
    int q = 0;
    const long long p = (long long)((unsigned long long)w[0] | ((unsigned long long)w[1] << 32));
    q = 2;
    pid = w[q++];
#pragma unroll
    for (int i = 0; i < N; ++i) x[i] = (int)w[q++];
#pragma unroll
    for (int j = 0; j < M; ++j) r[j] = (int)w[q++];
#pragma unroll
    for (int j = 0; j < M; ++j) {
      const unsigned long long b = (unsigned long long)w[q] | ((unsigned long long)w[q + 1] << 32);
      q += 2;
      G[j] = __builtin_bit_cast(double, b);
    }
    const unsigned long long tb = (unsigned long long)w[q] | ((unsigned long long)w[q + 1] << 32);
    q += 2;
    t = __builtin_bit_cast(double, tb);
    e = w[q++];
    status = (int)w[q++];
    const u32 flags = w[q++];
    const unsigned long long pb = (unsigned long long)w[q] | ((unsigned long long)w[q + 1] << 32);
    q += 2;
    const double tp = __builtin_bit_cast(double, pb);
    ssa_left = (int)w[q++];
    n_ssa = w[q++];
    n_ex = w[q++];
    n_im = w[q++];
    n_rej = w[q++];
    n_nfail = w[q++];
    n_clip = w[q++];
    n_cf = w[q++];
    n_nit = (long long)((unsigned long long)w[q] | ((unsigned long long)w[q + 1] << 32));
    if constexpr (GRID) {
      q += 2;
      const unsigned long long eb = (unsigned long long)w[q] | ((unsigned long long)w[q + 1] << 32);
      q += 2;
      tend = __builtin_bit_cast(double, eb);
      kt = (int)w[q++];
    }
#pragma unroll
    for (int j = 0; j < M; ++j) {
      th[j] = theta[p * M + j];
      thr[j] = (R)th[j];
    }
    gvalid = false;
    plan = false;
    implicit = false;
    if (flags & 1u) {  // retrying a leap: rebuild the plan, keep the halved tau'
      propensities();
      make_plan(prm);
      implicit = (flags & 2u) != 0;
      tau_p = (R)tp;
    }
    return p;
  }

  // a_j = theta_j g_j (Background section); a0 summed in ascending j.
  __device__ __forceinline__ void propensities() {
    if (!gvalid) {
      double xd[N];
#pragma unroll
      for (int i = 0; i < N; ++i) xd[i] = (double)x[i];
      g_all<NET>(xd, g);
      gvalid = true;
    }
    a0 = (R)0;
#pragma unroll
    for (int j = 0; j < M; ++j) {
      a[j] = thr[j] * (R)g[j];
      a0 = a0 + a[j];
    }
  }

  // Factor phi_i of the highest-order reaction of species i (Cao 2006).
  __device__ __forceinline__ R phi(int i) const {
    const int c = NET::PHI[i];
    if (c == 1) return (R)1;
    if (c == 2) return (R)2;
    if (c == 4) return (R)3;
    const R xm1 = (R)(x[i] - 1 > 1 ? x[i] - 1 : 1);
    if (c == 3) return (R)2 + (R)1 / xm1;
    if (c == 5) return (R)1.5 * ((R)2 + (R)1 / xm1);
    const R xm2 = (R)(x[i] - 2 > 1 ? x[i] - 2 : 1);
    return ((R)3 + (R)1 / xm1) + (R)2 / xm2;
  }

  // Tau selection over the reaction mask `use` (Cao 2006): bound the expected
  // change and variance of every reactant species by max(eps x_i/phi_i, 1).
  __device__ __forceinline__ R tau_select(u32 use, R eps) const {
    R tau = P::inf();
#pragma unroll
    for (int i = 0; i < N; ++i) {
      if (NET::PHI[i] == 0) continue;
      R mu = (R)0, s2 = (R)0;
#pragma unroll
      for (int j = 0; j < M; ++j) {
        const int v = NET::NU[j][i];
        if (v == 0) continue;
        if ((use >> j) & 1u) {
          mu = mu + (R)v * a[j];
          s2 = s2 + (R)(v * v) * a[j];
        }
      }
      R num = eps * (R)x[i];
      if (NET::PHI[i] != 1) num = num / phi(i);
      const R bound = num < (R)1 ? (R)1 : num;
      // bound >= 1, so a zero sum gives +inf by IEEE division (s2 >= +0)
      const R t1 = bound / P::fabs_(mu);
      const R t2 = (bound * bound) / s2;
      const R ti = t2 < t1 ? t2 : t1;
      tau = ti < tau ? ti : tau;
    }
    return tau;
  }

  // Critical set, tau_ex, partial equilibrium, tau_im and the leap type.
  __device__ __forceinline__ void make_plan(const SimParams& prm) {
    R tau_ex, tau_im;
    u32 eq;
    decide(prm, &tau_ex, &tau_im, &eq);
  }

  __device__ __forceinline__ void decide(const SimParams& prm, R* tau_ex_out, R* tau_im_out,
                                         u32* eq_out) {
    crit = 0;
    ncr = 0;
    a0c = (R)0;
#pragma unroll
    for (int j = 0; j < M; ++j) {
      int L = 0x7fffffff;
#pragma unroll
      for (int i = 0; i < N; ++i) {
        const int v = NET::NU[j][i];
        if (v < 0) {
          const int q = x[i] / (-v);
          L = q < L ? q : L;
        }
      }
      const bool pos = a[j] > (R)0;
      const bool c = pos && L < LXP(prm, n_c);
      crit |= (c ? 1u : 0u) << j;
      ncr |= ((pos && !c) ? 1u : 0u) << j;
      if (c) a0c = a0c + a[j];
    }
    const R eps = (R)LXP(prm, eps);
    const R tau_ex = tau_select(ncr, eps);
    implicit = false;
    tau_p = tau_ex;
    *tau_ex_out = tau_ex;
    *tau_im_out = P::inf();
    *eq_out = 0;
    if (NET::NPAIRS > 0 && LXP(prm, mode) == MODE_ADAPTIVE) {
      u32 eq = 0;
      const R delta = (R)LXP(prm, delta);
#pragma unroll
      for (int j = 0; j < M; ++j) {
        const int k = NET::PARTNER[j];
        if (k <= j) continue;
        if (((ncr >> j) & 1u) && ((ncr >> k) & 1u)) {
          const R lo = a[k] < a[j] ? a[k] : a[j];
          if (P::fabs_(a[j] - a[k]) <= delta * lo) eq |= (1u << j) | (1u << k);
        }
      }
      *eq_out = eq;
      if (eq) {
        const R tau_im = tau_select(ncr & ~eq, eps);
        *tau_im_out = tau_im;
        if (tau_im > (R)LXP(prm, n_stiff) * tau_ex) {
          implicit = true;
          tau_p = tau_im;
        }
      }
    }
    plan = true;
  }

  __device__ __forceinline__ void absorb(const SimParams& prm) {
    const double rem = t_end_(prm) - t;
#pragma unroll
    for (int j = 0; j < M; ++j) G[j] = G[j] + g[j] * rem;
    t = t_end_(prm);
  }

  // One SSA step (Gillespie 1977 direct method) with exact G.
  __device__ __forceinline__ void ssa_step(const SimParams& prm, const Key& key) {
    const Words4 w = draw_block(key, pid, e, SITE_SSA, 0);
    R u1, u2;
    P::uniforms(w, &u1, &u2);
    ssa_apply(prm, -P::ulog(u1), u2);
  }

  // The SSA step given its draws: E = -log(u1) of the step's first uniform and
  // the second uniform u2.  With `zero` (a0 = 0) it is the absorption instead
  // (G_j += g_j (t_end - t), no step counted), with `budget` nothing happens
  // but the lane's status; a step whose waiting time reaches t_end counts and
  // absorbs.  Every outcome is selected, without divergent branches; each
  // quantity is computed by the operations of its own branch.
  __device__ __forceinline__ void ssa_apply(const SimParams& prm, R E, R u2, bool zero = false,
                                            bool budget = false) {
    const bool stepping = !zero && !budget;
    e = e + (stepping ? 1u : 0u);
    n_ssa += stepping ? 1u : 0u;
    status = budget ? (int)LANE_STEP_BUDGET : status;
    const double tau_s = (double)(E / a0);  // +inf when a0 = 0 (E > 0)
    const double rem = t_end_(prm) - t;
    const bool past = tau_s >= rem;
    const bool absorbing = zero || (stepping && past);
    const bool fire = stepping && !past;
    const double dt = absorbing ? rem : tau_s;
    // Selection without branches: the partial sums before the first one
    // above u2 a0 are those of the ascending search (sums after it are never
    // compared), and the last reaction with a_j > 0 is used only when no sum
    // exceeds it, i.e. after every term.
    const R thr_ = u2 * a0;
    R cum = (R)0;
    int jf = -1, jlast = -1;
    bool found = false;
#pragma unroll
    for (int j = 0; j < M; ++j) {
      jlast = a[j] > (R)0 ? j : jlast;
      cum = cum + a[j];
      const bool hit = !found && cum > thr_;
      jf = hit ? j : jf;
      found = found || hit;
    }
    jf = found ? jf : jlast;
    const bool moves = absorbing || fire;
#pragma unroll
    for (int j = 0; j < M; ++j) {
      const double Gn = G[j] + g[j] * dt;
      G[j] = moves ? Gn : G[j];
    }
    // x += nu_jf, r_jf += 1 as selected increments (a firing only)
    jf = fire ? jf : -1;
#pragma unroll
    for (int i = 0; i < N; ++i) {
      int d = 0;
#pragma unroll
      for (int j = 0; j < M; ++j)
        if (NET::NU[j][i] != 0) d = (j == jf) ? NET::NU[j][i] : d;
      x[i] = x[i] + d;
    }
#pragma unroll
    for (int j = 0; j < M; ++j) r[j] = r[j] + (j == jf ? 1 : 0);
    t = absorbing ? t_end_(prm) : (fire ? t + tau_s : t);
    gvalid = fire ? false : gvalid;
  }

  // Dense LU with partial pivoting (first maximal pivot), in registers.
  __device__ __forceinline__ static bool lu_solve(double (&A)[N][N], double (&b)[N]) {
#pragma unroll
    for (int c = 0; c < N; ++c) {
      int piv = c;
      double best = __builtin_fabs(A[c][c]);
#pragma unroll
      for (int rr = c + 1; rr < N; ++rr) {
        const double v = __builtin_fabs(A[rr][c]);
        if (v > best) {
          best = v;
          piv = rr;
        }
      }
      if (!(best > 0.0)) return false;
#pragma unroll
      for (int rr = c + 1; rr < N; ++rr) {
        if (rr == piv) {
#pragma unroll
          for (int q = 0; q < N; ++q) {
            const double tmp = A[c][q];
            A[c][q] = A[rr][q];
            A[rr][q] = tmp;
          }
          const double tb = b[c];
          b[c] = b[rr];
          b[rr] = tb;
        }
      }
#pragma unroll
      for (int rr = c + 1; rr < N; ++rr) {
        const double l = A[rr][c] / A[c][c];
#pragma unroll
        for (int q = c; q < N; ++q) A[rr][q] = A[rr][q] - l * A[c][q];
        b[rr] = b[rr] - l * b[c];
      }
    }
#pragma unroll
    for (int rr = N - 1; rr >= 0; --rr) {
      double s = b[rr];
#pragma unroll
      for (int q = rr + 1; q < N; ++q) s = s - A[rr][q] * b[q];
      b[rr] = s / A[rr][rr];
    }
    return true;
  }

  // Implicit leap (Rathinam et al. 2003): Newton on
  //   F(y) = y - c - tau sum_{j noncritical} nu_j a_j(y),
  //   c = x + sum_j nu_j (P_j - tau a_j(x)) + nu_jc [fired],
  // with the analytic Jacobian I - tau sum_j nu_j grad a_j(y)^T.  On entry k
  // holds the Poisson draws P_j, on success the rounded counts.
  __device__ __forceinline__ bool implicit_counts(double tau, long long (&k)[M], int jc,
                                                  const SimParams& prm) {
    const unsigned long long ti0 = LX_CLOCK();
    double ax[M], c[N], y[N];
#pragma unroll
    for (int j = 0; j < M; ++j) ax[j] = th[j] * g[j];
#pragma unroll
    for (int i = 0; i < N; ++i) {
      double ci = (double)x[i];
#pragma unroll
      for (int j = 0; j < M; ++j) {
        if (NET::NU[j][i] == 0) continue;
        if ((ncr >> j) & 1u) {
          const double d = (double)k[j] - tau * ax[j];
          ci = ci + (double)NET::NU[j][i] * d;
        }
      }
#pragma unroll
      for (int j = 0; j < M; ++j)
        if (NET::NU[j][i] != 0 && j == jc) ci = ci + (double)NET::NU[j][i];
      c[i] = ci;
      y[i] = (double)x[i];
    }
    bool converged = false;
    for (int it = 0; it < LXP(prm, newton_maxit); ++it) {
      n_nit += 1;
      double ay[M], gy[M];
      g_all<NET>(y, gy);
#pragma unroll
      for (int j = 0; j < M; ++j) ay[j] = ((ncr >> j) & 1u) ? th[j] * gy[j] : 0.0;
      double A[N][N], b[N];
#pragma unroll
      for (int i = 0; i < N; ++i) {
        double s = 0.0;
#pragma unroll
        for (int j = 0; j < M; ++j)
          if (NET::NU[j][i] != 0 && ((ncr >> j) & 1u)) s = s + (double)NET::NU[j][i] * ay[j];
        b[i] = -((y[i] - c[i]) - tau * s);
      }
      // d a_j / d y_k: analytic, forward differences (a_j re-evaluated with
      // y_k moved by the representable step h_k), or the caller's terms
      const unsigned long long tj0 = LX_CLOCK();
      double yh[N], h[N];
      if (LXP(prm, jacobian) == 1) {
#pragma unroll
        for (int kk = 0; kk < N; ++kk) h[kk] = fd_step(y[kk], &yh[kk]);
      }
#pragma unroll
      for (int i = 0; i < N; ++i) {
#pragma unroll
        for (int kk = 0; kk < N; ++kk) {
          double s = 0.0;
#pragma unroll
          for (int j = 0; j < M; ++j) {
            if (NET::NU[j][i] == 0 || NET::RO[j][kk] == 0) continue;
            if ((ncr >> j) & 1u) {
              const double d =
                  LXP(prm, jacobian) == 1
                      ? (th[j] * g_moved<NET>(j, kk, y, yh[kk]) - ay[j]) / h[kk]
                      : (LXP(prm, jacobian) == 2 ? th[j] * dg_user<NET>(j, kk, y)
                                                 : th[j] * dg_of<NET>(j, kk, y));
              s = s + (double)NET::NU[j][i] * d;
            }
          }
          A[i][kk] = (i == kk ? 1.0 : 0.0) - tau * s;
        }
      }
      const unsigned long long tl0 = LX_CLOCK();
      cy_jac += tl0 - tj0;
      const bool lu_ok = lu_solve(A, b);
      cy_lu += LX_CLOCK() - tl0;
      if (!lu_ok) break;
      double dmax = 0.0, ymax = 0.0;
#pragma unroll
      for (int i = 0; i < N; ++i) {
        y[i] = y[i] + b[i];
        const double ad = __builtin_fabs(b[i]);
        const double ay_ = __builtin_fabs(y[i]);
        dmax = dmax < ad ? ad : dmax;
        ymax = ymax < ay_ ? ay_ : ymax;
      }
      if (!(dmax == dmax)) break;
      if (dmax <= LXP(prm, newton_tol) * (ymax < 1.0 ? 1.0 : ymax)) {
        converged = true;
        break;
      }
    }
    if (!converged) {
      n_nfail += 1;
      cy_imp += LX_CLOCK() - ti0;
      return false;
    }
    double gy[M];
    g_all<NET>(y, gy);
#pragma unroll
    for (int j = 0; j < M; ++j) {
      if (!((ncr >> j) & 1u)) {
        k[j] = 0;
        continue;
      }
      const double v = (tau * (th[j] * gy[j]) - tau * ax[j]) + (double)k[j];
      double kr = __builtin_round(v);
      if (kr < 0.0) {
        kr = 0.0;
        n_clip += 1;
      }
      if (kr > 1073741824.0) kr = 1073741824.0;
      k[j] = (long long)kr;
    }
    cy_imp += LX_CLOCK() - ti0;
    return true;
  }

  // One leap attempt with the current plan.  Returns false on rejection.
  __device__ __forceinline__ void leap_attempt(const SimParams& prm, const Key& key) {
    const u32 ea = e;
    e = e + 1;
    R tau_pp = P::inf();
    int jc = -1;
    R uc1 = (R)0, uc2 = (R)0;
    if (a0c > (R)0) {
      const Words4 w = draw_block(key, pid, ea, SITE_CRIT, 0);
      P::uniforms(w, &uc1, &uc2);
      tau_pp = -P::ulog(uc1) / a0c;
    }
    R tau_r;
    if (tau_p < tau_pp) {
      tau_r = tau_p;
    } else {
      tau_r = tau_pp;
      // branch-free search over the critical set, as in the SSA selection
      const R thr_ = uc2 * a0c;
      R cum = (R)0;
      int jlast = -1;
      bool found = false;
#pragma unroll
      for (int j = 0; j < M; ++j) {
        const bool cj = ((crit >> j) & 1u) != 0u;
        jlast = cj ? j : jlast;
        cum = cj ? cum + a[j] : cum;
        const bool hit = cj && !found && cum > thr_;
        jc = hit ? j : jc;
        found = found || hit;
      }
      jc = found ? jc : jlast;
    }
    double tau = (double)tau_r;
    const double rem = t_end_(prm) - t;
    bool last = false;
    if (tau >= rem) {
      tau = rem;
      jc = -1;
      last = true;
    }
    const R tau_rr = (R)tau;
    const R lam_thr = (R)LXP(prm, lam_thr);
    long long k[M];
    bool overflow = false;
    if constexpr (TPL == 1) {
#pragma unroll
      for (int j = 0; j < M; ++j) {
        k[j] = 0;
        if ((ncr >> j) & 1u) {
          long long kj;
          if constexpr (M > 4)
            kj = poisson_sample_call<P>(a[j] * tau_rr, lam_thr, LXP(prm, kcap), key, pid, ea, (u32)j);
          else
            kj = poisson_sample<P>(a[j] * tau_rr, lam_thr, LXP(prm, kcap), key, pid, ea, (u32)j);
          overflow = overflow | (kj < 0);
          k[j] = kj;
        }
      }
    } else {
      // lane `sub` of the group draws reaction g*TPL + sub of each group g
      const int sub = (int)(threadIdx.x & (TPL - 1));
#pragma unroll
      for (int g = 0; g < (M + TPL - 1) / TPL; ++g) {
        R aj = (R)0;
        bool nc = false;
#pragma unroll
        for (int q = 0; q < TPL; ++q) {
          if (g * TPL + q < M && sub == q) {
            aj = a[g * TPL + q];
            nc = ((ncr >> (g * TPL + q)) & 1u) != 0;
          }
        }
        long long kj = 0;
        if (nc) {
          if constexpr ((M + TPL - 1) / TPL > 4)
            kj = poisson_sample_call<P>(aj * tau_rr, lam_thr, LXP(prm, kcap), key, pid, ea,
                                        (u32)(g * TPL + sub));
          else
            kj = poisson_sample<P>(aj * tau_rr, lam_thr, LXP(prm, kcap), key, pid, ea,
                                   (u32)(g * TPL + sub));
        }
#pragma unroll
        for (int q = 0; q < TPL; ++q) {
          if (g * TPL + q < M) {
            const long long v = group_read<TPL>(kj, q);
            k[g * TPL + q] = v;
            overflow = overflow | (v < 0);
          }
        }
      }
    }
    if (overflow) {
      status = LANE_LAMBDA_OVERFLOW;
      return;
    }
    bool ok = true;
    if (implicit) ok = implicit_counts(tau, k, jc, prm);
    long long xn[N];
    if (ok) {
#pragma unroll
      for (int j = 0; j < M; ++j)
        if (j == jc) k[j] = 1;
#pragma unroll
      for (int i = 0; i < N; ++i) {
        long long v = x[i];
#pragma unroll
        for (int j = 0; j < M; ++j)
          if (NET::NU[j][i] != 0) v = v + (long long)NET::NU[j][i] * k[j];
        xn[i] = v;
        ok = ok & (v >= 0);
      }
    }
    if (!ok) {
      n_rej += 1;
      tau_p = tau_p / (R)2;
      return;
    }
    bool big = false;
#pragma unroll
    for (int i = 0; i < N; ++i) big = big | (xn[i] > 2147483647LL);
#pragma unroll
    for (int j = 0; j < M; ++j) big = big | ((long long)r[j] + k[j] > 2147483647LL);
    if (big) {
      status = LANE_COUNT_OVERFLOW;
      return;
    }
    double xd[N], gn[M];
#pragma unroll
    for (int i = 0; i < N; ++i) xd[i] = (double)xn[i];
    g_all<NET>(xd, gn);
#pragma unroll
    for (int j = 0; j < M; ++j) {
      G[j] = G[j] + (tau * (g[j] + gn[j])) * 0.5;
      r[j] = r[j] + (int)k[j];
      g[j] = gn[j];
    }
#pragma unroll
    for (int i = 0; i < N; ++i) x[i] = (int)xn[i];
    t = last ? t_end_(prm) : t + tau;
    if (implicit) n_im += 1;
    else n_ex += 1;
    n_cf += jc >= 0 ? 1u : 0u;
    plan = false;
    gvalid = true;
  }

  // One action: an SSA step, a leap attempt, or absorption.  Equivalent to
  // the nested loops of the method (leap retries with halved tau', SSA bursts
  // of n_ssa steps) flattened so that every lane makes progress on every
  // iteration; a burst decided here starts with its first SSA step at once.
  __device__ __forceinline__ void step(const SimParams& prm, const Key& key) {
    if (!plan) propensities();
    if (a0 == (R)0) {
      absorb(prm);
      return;
    }
    if (LXP(prm, mode) != MODE_SSA && ssa_left == 0) {
      if (!plan) make_plan(prm);
      if (tau_p < (R)LXP(prm, k_ssa) / a0 || a0c >= a0 / (R)LXP(prm, k_crit))
        ssa_left = implicit ? LXP(prm, n_ssa_im) : LXP(prm, n_ssa_ex);
    }
    if ((long long)e >= LXP(prm, max_steps)) {
      status = LANE_STEP_BUDGET;
      return;
    }
    if (LXP(prm, mode) == MODE_SSA || ssa_left > 0) {
      ssa_step(prm, key);
      if (ssa_left > 0) ssa_left -= 1;
      plan = false;
      return;
    }
    leap_attempt(prm, key);
  }

  // True when the next action is an SSA step (a burst in progress, or SSA
  // mode); such a lane needs no plan.
  __device__ __forceinline__ bool in_ssa(const SimParams& prm) const {
    return LXP(prm, mode) == MODE_SSA || ssa_left > 0;
  }

  // An SSA step of a lane in a burst (the SSA branch of step()).
  __device__ __forceinline__ void ssa_only(const SimParams& prm, const Key& key) {
    propensities();
    if (a0 == (R)0) {
      absorb(prm);
      return;
    }
    if ((long long)e >= LXP(prm, max_steps)) {
      status = LANE_STEP_BUDGET;
      return;
    }
    ssa_step(prm, key);
    if (ssa_left > 0) ssa_left -= 1;
    plan = false;
  }

  // Up to kmax SSA steps while the lane stays in an SSA burst.  With TPL > 1
  // the draws of the next TPL attempts are made in parallel (lane s of the
  // group draws attempt e + s) and applied in order.
  __device__ __forceinline__ void ssa_burst(const SimParams& prm, const Key& key, int kmax) {
    if constexpr (TPL == 1) {
      for (int k = 0; k < kmax; ++k) {
        if (!(active(prm) && in_ssa(prm))) break;
        ssa_only(prm, key);
      }
    } else {
      const u32 sub = threadIdx.x & (TPL - 1);
      int done = 0;
      while ((done < kmax) & active(prm) & in_ssa(prm)) {
        const Words4 w = draw_block(key, pid, e + sub, SITE_SSA, 0);
        R u1, u2;
        P::uniforms(w, &u1, &u2);
        const R E = -P::ulog(u1);
#pragma unroll
        for (int s = 0; s < TPL; ++s) {
          const R Es = group_read<TPL>(E, s);
          const R u2s = group_read<TPL>(u2, s);
          if ((done < kmax) & active(prm) & in_ssa(prm)) {
            propensities();
            const bool zero = a0 == (R)0;
            const bool budget = !zero && (long long)e >= LXP(prm, max_steps);
            ssa_apply(prm, Es, u2s, zero, budget);
            const bool stepped = !zero && !budget;
            ssa_left = (stepped && ssa_left > 0) ? ssa_left - 1 : ssa_left;
            plan = stepped ? false : plan;
            ++done;
          }
        }
      }
    }
  }
};

// ---------------------------------------------------------------------------
// Kernels.
// ---------------------------------------------------------------------------
#ifndef LX_POLICY
#define LX_POLICY lx::F64
#endif
#ifndef LX_BLOCK
#define LX_BLOCK 64
#endif
#ifndef LX_TPL
#define LX_TPL 1
#endif
#ifdef LX_GRID
#define LX_GRID_ON true
#else
#define LX_GRID_ON false
#endif

}  // namespace lx

#if !defined(LX_BATCHED) && !defined(LX_SET) && !defined(LX_LARGE)
// Plain form: lane = particle for life, 64 lanes per wave.
extern "C" __global__ void __launch_bounds__(LX_BLOCK) LX_WAVES_ATTR
    lx_sim_plain(const double* __restrict__ theta, const int* __restrict__ x0, int* x_out,
                 int* r_out, double* G_out, lx::Stats* stats, lx::SimParams prm) {
  const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= prm.P) return;
  const lx::Key key{prm.k0, prm.k1};
  lx::Lane<LX_POLICY, LxNet, 1, LX_GRID_ON> lane;
  lane.load(p, theta, x0, r_out, G_out, prm);
  for (;;) {
    while (lane.active(prm)) lane.step(prm, key);
    if constexpr (LX_GRID_ON) {
      if (lane.grid_next(p, prm, true)) continue;
    }
    break;
  }
  lane.store(p, x_out, r_out, G_out, stats);
  lane.store_cycles(p, prm);
}
#endif

#if defined(LX_BATCHED) || defined(LX_SET)
namespace lx {
// Batched form.  Block `blk` owns particles [blk*per_block, (blk+1)*per_block);
// its waves run `lanes` active lanes each and refill a finished lane with the
// block's next particle through an LDS cursor (work stealing within the
// block), until the range is exhausted.  Every iteration, lanes in an SSA
// burst take up to ssa_k SSA steps while the other lanes plan and take one
// leap attempt, which balances the divergent paths (an SSA step costs a
// fraction of a leap).  Per trajectory the sequence of actions, and hence
// every result, is the one of the plain form.
// The end of a block's range (tail_lanes): the n <= 64 / G trajectories still
// running in the wave are saved to LDS and each is finished by a group of G
// lanes (lane s of group g restores trajectory g), with the lane-group code
// of lanes_per_traj; per trajectory the actions, and so the results, are
// those of one lane.
template <class NET, int G>
__device__ __forceinline__ void finish_in_groups(Lane<LX_POLICY, NET, 1, LX_GRID_ON>& lane, bool has,
                                                 long long p, const double* __restrict__ theta,
                                                 int* x_out, int* r_out, double* G_out,
                                                 Stats* stats, const SimParams& prm, u32* slots) {
  typedef Lane<LX_POLICY, NET, 1, LX_GRID_ON> One;
  constexpr int STRIDE = One::STATE_WORDS;
  const int lane_id = threadIdx.x & 63;
  const unsigned long long live = __ballot(has);
  const int n = __popcll(live);
  if (has) lane.save(p, slots + __popcll(live & ((1ull << lane_id) - 1ull)) * STRIDE);
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
  const int g = lane_id / G;
  const int sub = lane_id & (G - 1);
  if (g >= n) return;
  const Key key{prm.k0, prm.k1};
  Lane<LX_POLICY, NET, G, LX_GRID_ON> lg;
  const long long pg = lg.restore(slots + g * STRIDE, theta, prm);
  for (;;) {
    if (lg.active(prm)) {
      lg.ssa_burst(prm, key, LXP(prm, ssa_k));
      if (lg.active(prm) && !lg.in_ssa(prm)) lg.step(prm, key);
    }
    if (!lg.active(prm)) {
      if constexpr (LX_GRID_ON) {
        if (lg.grid_next(pg, prm, sub == 0)) continue;
      }
      if (sub == 0) lg.store(pg, x_out, r_out, G_out, stats);
      return;
    }
  }
}

template <class NET>
__device__ __forceinline__ void run_batched(long long blk, const double* __restrict__ theta,
                                            const int* __restrict__ x0, int* x_out, int* r_out,
                                            double* G_out, Stats* stats, const SimParams& prm,
                                            unsigned long long* next, bool cursor_ready) {
  constexpr int TPL = LX_TPL;
#ifdef LX_CONST
  constexpr int TAIL = ::LxConst::tail;
#else
  constexpr int TAIL = 0;
#endif
  const int lane_id = threadIdx.x & 63;
  const int slot = lane_id / TPL;  // trajectory slot of this lane in its wave
  const int sub = lane_id & (TPL - 1);
  const int wave = threadIdx.x >> 6;
  const int waves = blockDim.x >> 6;
  const long long lo = blk * prm.per_block;
  long long hi = lo + prm.per_block;
  if (hi > prm.P) hi = prm.P;
  if (!cursor_ready) {
    if (threadIdx.x == 0) *next = (unsigned long long)(lo + (long long)waves * prm.lanes);
    __syncthreads();
  }
  const Key key{prm.k0, prm.k1};
  long long p = lo + (long long)wave * prm.lanes + slot;
  bool has = slot < prm.lanes && p < hi;
  Lane<LX_POLICY, NET, TPL, LX_GRID_ON> lane;
  if (has) lane.load(p, theta, x0, r_out, G_out, prm);
  if constexpr (TPL == 1 && TAIL > 1) {
    // wave-uniform loop: the wave switches to lane groups once the block's
    // range is exhausted and few of its trajectories are left
    __shared__ u32 tail_slots[(LX_BLOCK / 64) * (64 / (TAIL > 1 ? TAIL : 1)) *
                              Lane<LX_POLICY, NET, 1, LX_GRID_ON>::STATE_WORDS];
    u32* slots = tail_slots + wave * (64 / TAIL) * Lane<LX_POLICY, NET, 1, LX_GRID_ON>::STATE_WORDS;
    for (;;) {
      const unsigned long long live = __ballot(has);
      if (!live) return;
      if (__popcll(live) <= 64 / TAIL && *((volatile unsigned long long*)next) >= (unsigned long long)hi) {
        finish_in_groups<NET, TAIL>(lane, has, p, theta, x_out, r_out, G_out, stats, prm, slots);
        return;
      }
      if (has) {
        if (lane.active(prm)) {
          lane.ssa_burst(prm, key, LXP(prm, ssa_k));
          if (lane.active(prm) && !lane.in_ssa(prm)) lane.step(prm, key);
        }
        if (!lane.active(prm)) {
          bool again = false;
          if constexpr (LX_GRID_ON) again = lane.grid_next(p, prm, true);
          if (!again) {
            lane.store(p, x_out, r_out, G_out, stats);
            lane.store_cycles(p, prm);
            p = (long long)atomicAdd(next, 1ull);
            has = p < hi;
            if (has) lane.load(p, theta, x0, r_out, G_out, prm);
          }
        }
      }
    }
  }
  while (has) {
    if (lane.active(prm)) {
      lane.ssa_burst(prm, key, LXP(prm, ssa_k));
      if (lane.active(prm) && !lane.in_ssa(prm)) lane.step(prm, key);
    }
    if (!lane.active(prm)) {
      if constexpr (LX_GRID_ON) {
        if (lane.grid_next(p, prm, sub == 0)) continue;
      }
      if (sub == 0) {
        lane.store(p, x_out, r_out, G_out, stats);
        lane.store_cycles(p, prm);
      }
      long long pn = 0;
      if (sub == 0) pn = (long long)atomicAdd(next, 1ull);
      p = group_read<TPL>(pn, 0);
      has = p < hi;
      if (has) lane.load(p, theta, x0, r_out, G_out, prm);
    }
  }
}

// Batched form with regrouping by next action.  Every `regroup` iterations
// the lanes of the block write their state to LDS in the order (lanes whose
// next action is an SSA step, lanes that plan or leap, empty lanes) and read
// back the state of their new position, so that waves hold one kind of lane.
// A wave that still holds both kinds (the boundary wave) lets one kind act per
// iteration, alternating, so every lane acts at least every second iteration
// and no wave pays for both paths.  Refill from the block's range as in
// run_batched.  Each trajectory's actions, and hence every result, are
// unchanged.
template <class NET>
__device__ __forceinline__ void run_regroup(long long blk, const double* __restrict__ theta,
                                            const int* __restrict__ x0, int* x_out, int* r_out,
                                            double* G_out, Stats* stats, const SimParams& prm,
                                            unsigned long long* next, bool cursor_ready) {
  typedef Lane<LX_POLICY, NET, 1, LX_GRID_ON> LaneT;
  constexpr int STRIDE = LaneT::STATE_WORDS;
  __shared__ u32 slots[LX_BLOCK * STRIDE];
  __shared__ int counts[2 * (LX_BLOCK / 64)];
  const int lane_id = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int waves = blockDim.x >> 6;
  const bool slot_thread = lane_id < prm.lanes;
  const int vslot = wave * prm.lanes + lane_id;
  const long long lo = blk * prm.per_block;
  long long hi = lo + prm.per_block;
  if (hi > prm.P) hi = prm.P;
  if (!cursor_ready) {
    if (threadIdx.x == 0) *next = (unsigned long long)(lo + (long long)waves * prm.lanes);
    __syncthreads();
  }
  const Key key{prm.k0, prm.k1};
  long long p = lo + vslot;
  bool has = slot_thread && p < hi;
  LaneT lane;
  if (has) lane.load(p, theta, x0, r_out, G_out, prm);
  for (int iter = 0;; ++iter) {
    while (has && !lane.active(prm)) {  // store finished trajectories, refill
      if constexpr (LX_GRID_ON) {
        if (lane.grid_next(p, prm, true)) continue;
      }
      lane.store(p, x_out, r_out, G_out, stats);
      p = (long long)atomicAdd(next, 1ull);
      has = p < hi;
      if (has) lane.load(p, theta, x0, r_out, G_out, prm);
    }
    if (!__syncthreads_or(has ? 1 : 0)) break;
    int cls = has ? (lane.in_ssa(prm) ? 0 : 1) : 2;
    if (LXP(prm, regroup) > 0 && iter % LXP(prm, regroup) == 0) {
      const unsigned long long b0 = __ballot(cls == 0);
      const unsigned long long b1 = __ballot(cls == 1);
      if (lane_id == 0) {
        counts[2 * wave] = __popcll(b0);
        counts[2 * wave + 1] = __popcll(b1);
      }
      __syncthreads();
      int n0 = 0, n1 = 0, before0 = 0, before1 = 0;
      for (int w = 0; w < waves; ++w) {
        if (w < wave) {
          before0 += counts[2 * w];
          before1 += counts[2 * w + 1];
        }
        n0 += counts[2 * w];
        n1 += counts[2 * w + 1];
      }
      const unsigned long long below = (1ull << lane_id) - 1ull;
      if (cls == 0) lane.save(p, slots + (before0 + __popcll(b0 & below)) * STRIDE);
      if (cls == 1) lane.save(p, slots + (n0 + before1 + __popcll(b1 & below)) * STRIDE);
      __syncthreads();
      has = slot_thread && vslot < n0 + n1;
      if (has) p = lane.restore(slots + vslot * STRIDE, theta, prm);
      cls = has ? (lane.in_ssa(prm) ? 0 : 1) : 2;
    }
    const bool any0 = __ballot(cls == 0) != 0ull;
    const bool any1 = __ballot(cls == 1) != 0ull;
    const bool run_ssa = any0 && (!any1 || (iter & 1) == 0);
    if (cls == 0 && run_ssa) {
      for (int k = 0; k < LXP(prm, ssa_k); ++k) {
        if (!(lane.active(prm) && lane.in_ssa(prm))) break;
        lane.ssa_only(prm, key);
      }
    } else if (cls == 1 && !run_ssa) {
      lane.step(prm, key);
    }
  }
}

// `cursor_ready`: the caller has set *next to the first particle after the
// block's initial lanes and synchronised the block (network sets set every
// network's cursor at once and run the networks back to back).
template <class NET>
__device__ __forceinline__ void run_sched(long long blk, const double* __restrict__ theta,
                                          const int* __restrict__ x0, int* x_out, int* r_out,
                                          double* G_out, Stats* stats, const SimParams& prm,
                                          unsigned long long* next, bool cursor_ready = false) {
  if (LX_TPL == 1 && LXP(prm, regroup) > 0)
    run_regroup<NET>(blk, theta, x0, x_out, r_out, G_out, stats, prm, next, cursor_ready);
  else run_batched<NET>(blk, theta, x0, x_out, r_out, G_out, stats, prm, next, cursor_ready);
}
}  // namespace lx
#endif

#if defined(LX_BATCHED) && !defined(LX_LARGE)
extern "C" __global__ void __launch_bounds__(LX_BLOCK) LX_WAVES_ATTR
    lx_sim_batched(const double* __restrict__ theta, const int* __restrict__ x0, int* x_out,
                   int* r_out, double* G_out, lx::Stats* stats, lx::SimParams prm) {
  __shared__ unsigned long long next;
  lx::run_sched<LxNet>(blockIdx.x, theta, x0, x_out, r_out, G_out, stats, prm, &next);
}
#endif

#if defined(LX_HOOKS) && !defined(LX_LARGE)
// Step decision on fixed states (test hook).
extern "C" __global__ void __launch_bounds__(64)
    lx_hook_tau(const double* __restrict__ theta, const int* __restrict__ xs, double* a_out,
                unsigned int* crit_out, unsigned int* eq_out, double* tau_out, int* action,
                lx::SimParams prm) {
  typedef LX_POLICY::R R;
  const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= prm.P) return;
  lx::Lane<LX_POLICY, LxNet> lane;
  lx::SimParams p2 = prm;
  p2.accumulate = 0;
  p2.pid_base = 0;
  lane.load(q, theta, xs, nullptr, nullptr, p2);
  lane.propensities();
  R tau_ex, tau_im;
  unsigned int eq;
  lane.decide(prm, &tau_ex, &tau_im, &eq);
  for (int j = 0; j < LxNet::M; ++j) a_out[q * LxNet::M + j] = (double)lane.a[j];
  crit_out[q] = lane.crit;
  eq_out[q] = eq;
  tau_out[2 * q] = (double)tau_ex;
  tau_out[2 * q + 1] = (double)tau_im;
  int act;
  if (lane.a0 == (R)0) act = 3;
  else if (lane.tau_p < (R)LXP(prm, k_ssa) / lane.a0 || lane.a0c >= lane.a0 / (R)LXP(prm, k_crit)) act = 2;
  else act = lane.implicit ? 1 : 0;
  action[q] = act;
}

// Implicit-leap solve on fixed inputs (test hook); binary64 policy.
extern "C" __global__ void __launch_bounds__(64)
    lx_hook_implicit(const double* __restrict__ theta, const int* __restrict__ xs,
                     const double* __restrict__ tau, const long long* __restrict__ Pj,
                     const int* __restrict__ jc, long long* k_out, int* ok_out, int* it_out,
                     lx::SimParams prm) {
  const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= prm.P) return;
  lx::Lane<lx::F64, LxNet> lane;
  lx::SimParams p2 = prm;
  p2.accumulate = 0;
  p2.pid_base = 0;
  lane.load(q, theta, xs, nullptr, nullptr, p2);
  lane.propensities();
  lane.ncr = 0;
  for (int j = 0; j < LxNet::M; ++j)
    if (lane.a[j] > 0.0 && j != jc[q]) lane.ncr |= 1u << j;
  long long k[LxNet::M];
  for (int j = 0; j < LxNet::M; ++j) k[j] = Pj[q * LxNet::M + j];
  const bool ok = lane.implicit_counts(tau[q], k, jc[q], prm);
  for (int j = 0; j < LxNet::M; ++j) k_out[q * LxNet::M + j] = ok ? k[j] : 0;
  ok_out[q] = ok ? 1 : 0;
  it_out[q] = (int)lane.n_nit;
}
#endif
