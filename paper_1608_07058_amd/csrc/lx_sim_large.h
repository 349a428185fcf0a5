// lx_sim_large.h -- one trajectory per lane for networks beyond the
// register-resident kernels of lx_sim.h (up to 64 species, 256 reactions).
//
// The method and every arithmetic operation, in the same order, are those of
// lx::Lane; only the storage differs.  The generated traits struct of a large
// network (LxNet, LARGE = 1) holds compressed stoichiometry instead of dense
// tables:
//   RX_PTR[M+1], RX_SP[], RX_RO[]  reactants of reaction j (ascending species)
//   NJ_PTR[M+1], NJ_SP[], NJ_V[]   nonzero net changes of reaction j (ascending species)
//   NI_PTR[N+1], NI_RX[], NI_V[]   nonzero net changes of species i (ascending reactions)
//   PHI[N], PARTNER[M], NPAIRS
// Loops over species and reactions run at run time with wave-uniform trip
// counts and table indices (scalar loads).  The per-lane arrays (theta in the
// policy's precision, r, G, a, Poisson counts, the Newton system) are private
// arrays indexed at run time, which live in the private segment; it is
// interleaved by lane, so a uniform index across a wave is one contiguous
// access.  The species counts live in LDS; g_j is recomputed from them where
// needed and the reaction sets are bit masks.
#pragma once

namespace lx {

// A pointer into LDS typed as such: accesses through it are LDS instructions
// also where the compiler cannot see where it came from (the Newton solve is
// an out-of-line function).
#define LX_LDS __attribute__((address_space(3)))

// Species counts of one lane in LDS: element i at p[i * LX_BLOCK] (the
// table-driven loops index them at run time; LDS answers in tens of cycles
// where the private segment, not resident in any cache at these sizes, takes
// a trip to memory).
struct XSlot {
  LX_LDS int* p;
  __device__ __forceinline__ LX_LDS int& operator[](int i) const { return p[i * LX_BLOCK]; }
};

template <class NET, class XV>
__device__ __forceinline__ double g_large(int j, const XV& x) {
  double gj = 1.0;
  for (int q = NET::RX_PTR[j]; q < NET::RX_PTR[j + 1]; ++q)
    gj = gj * binom_real((double)x[NET::RX_SP[q]], NET::RX_RO[q]);
  return gj;
}

template <class NET, class YP>
__device__ __forceinline__ double g_large_y(int j, YP y) {
  double gj = 1.0;
  for (int q = NET::RX_PTR[j]; q < NET::RX_PTR[j + 1]; ++q)
    gj = gj * binom_real(y[NET::RX_SP[q]], NET::RX_RO[q]);
  return gj;
}

// d g_j / d y_k.
template <class NET, class YP>
__device__ __forceinline__ double dg_large(int j, int k, YP y) {
  double gj = 1.0;
  for (int q = NET::RX_PTR[j]; q < NET::RX_PTR[j + 1]; ++q) {
    const int i = NET::RX_SP[q];
    gj = gj * (i == k ? binom_real_deriv(y[i], NET::RX_RO[q]) : binom_real(y[i], NET::RX_RO[q]));
  }
  return gj;
}

// d g_j / d y_k from the caller's terms of reactant slot q (reaction j, its
// species k): JT_SLOT_T lists them in table order (as dg_user).
template <class NET, class YP>
__device__ __forceinline__ double dg_user_large(int q, YP y) {
  double s = 0.0;
  for (int u = NET::JT_SLOT_PTR[q]; u < NET::JT_SLOT_PTR[q + 1]; ++u) {
    const int t = NET::JT_SLOT_T[u];
    double v = NET::JT_C[t];
    for (int f = NET::JT_PTR[t]; f < NET::JT_PTR[t + 1]; ++f)
      for (int e = 0; e < NET::JT_PW[f]; ++e) v = v * y[NET::JT_SP[f]];
    s = s + v;
  }
  return s;
}

template <class P, class NET, bool GRID = false>
struct LaneL {
  typedef typename P::R R;
  static constexpr int N = NET::N;
  static constexpr int M = NET::M;

  static constexpr int W = (M + 31) / 32;  // mask words

  // Hot per-lane state (~3.4 KB at M = 128, N = 48 in binary32): g_j is
  // recomputed from x where needed and theta is re-read from the input row
  // by the implicit solve, so neither is stored.
  u32 pid;
  const double* th;  // this trajectory's theta row [M]
  R thr[M];
  XSlot x;  // species counts, in LDS
  int r[M];
  double G[M];
  double t;
  u32 e;
  int status;
  double tend;  // end of the current stretch: the next observation time (GRID)
  int kt;       // index of that time (GRID)
  R a[M];
  R a0, a0c;
  u32 critw[W], ncrw[W], eqw[W];  // reaction sets, bit j % 32 of word j / 32
  bool plan, implicit, any_eq;
  R tau_p;
  int ssa_left;
  u32 n_ssa, n_ex, n_im, n_rej, n_nfail, n_clip, n_cf;
  long long n_nit;
  // clock cycles (LX_TIMERS): Jacobian assembly, LU solves, implicit solves, start
  unsigned long long cy_jac, cy_lu, cy_imp, cy_t0;
  // the current leap's counts (Poisson draws, then the accepted counts)
  int kd[M];
  // an implicit leap parked for the wave's cooperative solve (coop_newton)
  bool pend, pend_ok, pend_last;
  double pend_tau;
  int pend_jc;

  // The time the trajectory runs to now: t_end, or the next observation time.
  __device__ __forceinline__ double t_end_(const SimParams& prm) const {
    if constexpr (GRID) return tend;
    else return prm.t_end;
  }

  __device__ __forceinline__ bool active(const SimParams& prm) const {
    return status == LANE_OK && t < t_end_(prm);
  }

  __device__ static __forceinline__ bool bit(const u32* w, int j) {
    return ((w[j >> 5] >> (j & 31)) & 1u) != 0u;
  }
  __device__ static __forceinline__ void set_bit(u32* w, int j) { w[j >> 5] |= 1u << (j & 31); }
  __device__ __forceinline__ bool crit_(int j) const { return bit(critw, j); }
  __device__ __forceinline__ bool ncr_(int j) const { return bit(ncrw, j); }
  __device__ __forceinline__ bool eq_(int j) const { return bit(eqw, j); }

  __device__ __forceinline__ void load(long long p, const double* __restrict__ theta,
                                       const int* __restrict__ x0, const int* r_in,
                                       const double* G_in, const SimParams& prm) {
    pid = prm.pid_base + (u32)p * prm.pid_stride;
    th = theta + p * M;
    bool bad = false;
    for (int j = 0; j < M; ++j) {
      const double tj = th[j];
      thr[j] = (R)tj;
      bad = bad || !(tj >= 0.0) || tj == LX_INF_F64;
      r[j] = LXP(prm, accumulate) ? r_in[p * M + j] : 0;
      G[j] = LXP(prm, accumulate) ? G_in[p * M + j] : 0.0;
    }
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
    implicit = false;
    ssa_left = 0;
    n_ssa = n_ex = n_im = n_rej = n_nit = n_nfail = n_clip = n_cf = 0;
    cy_jac = cy_lu = cy_imp = 0;
    cy_t0 = LX_CLOCK();
    pend = false;
  }

  // Observation times, as Lane::grid_next: record the state as row kt of
  // x_grid (-1 if the time was not reached in status OK) and open the
  // stretch to the next time; returns true if the trajectory goes on.
  __device__ __forceinline__ bool grid_next(long long p, const SimParams& prm) {
    const bool ok = status == LANE_OK;
    int* row = prm.x_grid + ((long long)p * prm.n_times + kt) * N;
    for (int i = 0; i < N; ++i) row[i] = ok ? x[i] : -1;
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
    for (int k = kt; k < prm.n_times; ++k) {
      row += N;
      for (int i = 0; i < N; ++i) row[i] = -1;
    }
    return false;
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
    for (int i = 0; i < N; ++i) x_out[p * N + i] = x[i];
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

  // a_j = theta_j g_j (Background section); a0 summed in ascending j.
  __device__ __forceinline__ void propensities() {
    a0 = (R)0;
    for (int j = 0; j < M; ++j) {
      a[j] = thr[j] * (R)g_large<NET>(j, x);
      a0 = a0 + a[j];
    }
  }

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

  // Tau selection (Cao 2006) over the non-critical reactions, without those
  // in partial equilibrium when `skip_eq`.
  __device__ __forceinline__ R tau_select(bool skip_eq, R eps) const {
    R tau = P::inf();
    for (int i = 0; i < N; ++i) {
      if (NET::PHI[i] == 0) continue;
      R mu = (R)0, s2 = (R)0;
      for (int q = NET::NI_PTR[i]; q < NET::NI_PTR[i + 1]; ++q) {
        const int j = NET::NI_RX[q];
        const int v = NET::NI_V[q];
        if (ncr_(j) && !(skip_eq && eq_(j))) {
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

  __device__ __forceinline__ void decide(const SimParams& prm, R* tau_ex_out, R* tau_im_out) {
    a0c = (R)0;
    for (int w = 0; w < W; ++w) critw[w] = ncrw[w] = eqw[w] = 0u;
    for (int j = 0; j < M; ++j) {
      int L = 0x7fffffff;
      for (int q = NET::NJ_PTR[j]; q < NET::NJ_PTR[j + 1]; ++q) {
        const int v = NET::NJ_V[q];
        if (v < 0) {
          const int qq = x[NET::NJ_SP[q]] / (-v);
          L = qq < L ? qq : L;
        }
      }
      const bool pos = a[j] > (R)0;
      const bool c = pos && L < LXP(prm, n_c);
      if (c) set_bit(critw, j);
      if (pos && !c) set_bit(ncrw, j);
      if (c) a0c = a0c + a[j];
    }
    const R eps = (R)LXP(prm, eps);
    const R tau_ex = tau_select(false, eps);
    implicit = false;
    tau_p = tau_ex;
    *tau_ex_out = tau_ex;
    *tau_im_out = P::inf();
    any_eq = false;
    if (NET::NPAIRS > 0 && LXP(prm, mode) == MODE_ADAPTIVE) {
      const R delta = (R)LXP(prm, delta);
      for (int j = 0; j < M; ++j) {
        const int k = NET::PARTNER[j];
        if (k <= j) continue;
        if (ncr_(j) && ncr_(k)) {
          const R lo = a[k] < a[j] ? a[k] : a[j];
          if (P::fabs_(a[j] - a[k]) <= delta * lo) {
            set_bit(eqw, j);
            set_bit(eqw, k);
            any_eq = true;
          }
        }
      }
      if (any_eq) {
        const R tau_im = tau_select(true, eps);
        *tau_im_out = tau_im;
        if (tau_im > (R)LXP(prm, n_stiff) * tau_ex) {
          implicit = true;
          tau_p = tau_im;
        }
      }
    }
    plan = true;
  }

  __device__ __forceinline__ void make_plan(const SimParams& prm) {
    R tau_ex, tau_im;
    decide(prm, &tau_ex, &tau_im);
  }

  __device__ __forceinline__ void absorb(const SimParams& prm) {
    const double rem = t_end_(prm) - t;
    for (int j = 0; j < M; ++j) G[j] = G[j] + g_large<NET>(j, x) * rem;
    t = t_end_(prm);
  }

  // One SSA step (Gillespie 1977 direct method) with exact G.
  __device__ __forceinline__ void ssa_step(const SimParams& prm, const Key& key) {
    const Words4 w = draw_block(key, pid, e, SITE_SSA, 0);
    R u1, u2;
    P::uniforms(w, &u1, &u2);
    e = e + 1;
    n_ssa += 1;
    const R E = -P::ulog(u1);
    const double tau_s = (double)(E / a0);
    const double rem = t_end_(prm) - t;
    if (tau_s >= rem) {
      absorb(prm);
      return;
    }
    const R thr_ = u2 * a0;
    R cum = (R)0;
    int jf = -1, jlast = -1;
    for (int j = 0; j < M; ++j) {
      if (a[j] > (R)0) jlast = j;
      cum = cum + a[j];
      if (cum > thr_) {
        jf = j;
        break;
      }
    }
    if (jf < 0) jf = jlast;
    for (int j = 0; j < M; ++j) G[j] = G[j] + g_large<NET>(j, x) * tau_s;
    for (int q = NET::NJ_PTR[jf]; q < NET::NJ_PTR[jf + 1]; ++q) x[NET::NJ_SP[q]] += NET::NJ_V[q];
    r[jf] = r[jf] + 1;
    t = t + tau_s;
  }

  // One leap attempt with the current plan.  An implicit leap draws its
  // Poisson counts and then waits (pend) for the wave's cooperative Newton
  // solve (coop_newton); finish_pending completes it.
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
      const R thr_ = uc2 * a0c;
      R cum = (R)0;
      int jlast = -1;
      for (int j = 0; j < M; ++j) {
        if (crit_(j)) {
          jlast = j;
          cum = cum + a[j];
          if (cum > thr_) {
            jc = j;
            break;
          }
        }
      }
      if (jc < 0) jc = jlast;
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
    // Counts fit int32: the samplers' means are at most 2^30 and the
    // implicit counts are clamped there.
    bool overflow = false;
    for (int j = 0; j < M; ++j) {
      kd[j] = 0;
      if (ncr_(j)) {
        const long long kj =
            poisson_sample_call<P>(a[j] * tau_rr, lam_thr, LXP(prm, kcap), key, pid, ea, (u32)j);
        overflow = overflow || kj < 0;
        kd[j] = (int)kj;
      }
    }
    if (overflow) {
      status = LANE_LAMBDA_OVERFLOW;
      return;
    }
    if (implicit) {
      pend = true;
      pend_tau = tau;
      pend_jc = jc;
      pend_last = last;
      return;
    }
    leap_accept(tau, jc, last, true, prm);
  }

  // The implicit leap after its solve: counts in kd if pend_ok.
  __device__ __forceinline__ void finish_pending(const SimParams& prm) {
    pend = false;
    leap_accept(pend_tau, pend_jc, pend_last, pend_ok, prm);
  }

  // The rest of a leap attempt once its counts kd are known (`ok`: an
  // implicit solve converged, or an explicit leap).
  __device__ __forceinline__ void leap_accept(double tau, int jc, bool last, bool ok,
                                              const SimParams& prm) {
    int xn[N];
    bool big = false;
    if (ok) {
      if (jc >= 0) kd[jc] = 1;
      for (int i = 0; i < N; ++i) {
        long long v = x[i];
        for (int q = NET::NI_PTR[i]; q < NET::NI_PTR[i + 1]; ++q)
          v = v + (long long)NET::NI_V[q] * kd[NET::NI_RX[q]];
        ok = ok && v >= 0;
        big = big || v > 2147483647LL;
        xn[i] = (int)v;
      }
    }
    if (!ok) {
      n_rej += 1;
      tau_p = tau_p / (R)2;
      return;
    }
    for (int j = 0; j < M; ++j) big = big || (long long)r[j] + kd[j] > 2147483647LL;
    if (big) {
      status = LANE_COUNT_OVERFLOW;
      return;
    }
    // trapezoid with the old and the accepted state
    for (int j = 0; j < M; ++j) {
      const double go = g_large<NET>(j, x);
      const double gn = g_large<NET>(j, xn);
      G[j] = G[j] + (tau * (go + gn)) * 0.5;
      r[j] = r[j] + kd[j];
    }
    for (int i = 0; i < N; ++i) x[i] = xn[i];
    t = last ? t_end_(prm) : t + tau;
    if (implicit) n_im += 1;
    else n_ex += 1;
    n_cf += jc >= 0 ? 1u : 0u;
    plan = false;
  }

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

  __device__ __forceinline__ bool in_ssa(const SimParams& prm) const {
    return LXP(prm, mode) == MODE_SSA || ssa_left > 0;
  }

  __device__ __forceinline__ void ssa_burst(const SimParams& prm, const Key& key, int kmax) {
    for (int kk = 0; kk < kmax; ++kk) {
      if (!(active(prm) && in_ssa(prm))) break;
      propensities();
      if (a0 == (R)0) {
        absorb(prm);
        break;
      }
      if ((long long)e >= LXP(prm, max_steps)) {
        status = LANE_STEP_BUDGET;
        break;
      }
      ssa_step(prm, key);
      if (ssa_left > 0) ssa_left -= 1;
      plan = false;
    }
  }
};

// ---------------------------------------------------------------------------
// Wave-cooperative implicit solve.  A lane whose leap is implicit parks it
// (LaneL::pend); the wave then solves the parked leaps one after another,
// all 64 lanes on one Newton system held in LDS: reactions spread over lanes
// for the propensities and derivatives, species (rows) over lanes for the
// residual, the Jacobian rows, the LU elimination and the update.  Partial
// pivoting relabels rows instead of moving them (a row swap only renames
// which stored row is which), so every entry receives exactly the operations
// of the dense row-swapping LU, in the same order.
// ---------------------------------------------------------------------------
template <class NET>
struct SolveArea {
  static constexpr int N = NET::N, M = NET::M, W = (NET::M + 31) / 32, LD = NET::N + 1;
  double A[NET::N * LD];  // row-major, row stride N + 1 (bank spread)
  double b[NET::N], y[NET::N], c[NET::N], sol[NET::N];
  double ax[NET::M], ay[NET::M];
  double d[NET::NSLOT];  // d a_j / d y_k of every reactant slot
  int k[NET::M];         // Poisson draws in, rounded counts out
  const double* th;
  double tau;
  int jc, clips;
  u32 ncr[W];
};

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// Wave reductions with DPP moves (VALU, no LDS round trip): row shifts by 1,
// 2, 4 and 8 leave each row's result in its lane 15, two row broadcasts
// combine the rows into lane 63, which every lane then reads.  `ident` is
// what a lane without a source reads.  Only for operations whose result
// does not depend on the order (max, min, integer sums).
template <int CTRL, int ROWS>
__device__ __forceinline__ int dpp_b32(int v, int ident) {
  return __builtin_amdgcn_update_dpp(ident, v, CTRL, ROWS, 0xF, false);
}

template <int CTRL, int ROWS, class T>
__device__ __forceinline__ T dpp_move(T v, T ident) {
  if constexpr (sizeof(T) == 4) {
    return __builtin_bit_cast(T, dpp_b32<CTRL, ROWS>(__builtin_bit_cast(int, v),
                                                     __builtin_bit_cast(int, ident)));
  } else {
    static_assert(sizeof(T) == 8, "32- or 64-bit values");
    const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
    const unsigned long long c = __builtin_bit_cast(unsigned long long, ident);
    const unsigned lo = (unsigned)dpp_b32<CTRL, ROWS>((int)(unsigned)b, (int)(unsigned)c);
    const unsigned hi = (unsigned)dpp_b32<CTRL, ROWS>((int)(unsigned)(b >> 32), (int)(unsigned)(c >> 32));
    return __builtin_bit_cast(T, ((unsigned long long)hi << 32) | lo);
  }
}

template <class T>
__device__ __forceinline__ T read_lane(T v, int lane) {
  if constexpr (sizeof(T) == 4) {
    return __builtin_bit_cast(T, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), lane));
  } else {
    const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, lane);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), lane);
    return __builtin_bit_cast(T, ((unsigned long long)hi << 32) | lo);
  }
}

template <class T, class Op>
__device__ __forceinline__ T wave_reduce(T v, T ident, Op op) {
  v = op(v, dpp_move<0x111, 0xF>(v, ident));  // row_shr:1
  v = op(v, dpp_move<0x112, 0xF>(v, ident));  // row_shr:2
  v = op(v, dpp_move<0x114, 0xF>(v, ident));  // row_shr:4
  v = op(v, dpp_move<0x118, 0xF>(v, ident));  // row_shr:8
  v = op(v, dpp_move<0x142, 0xA>(v, ident));  // row_bcast:15 into rows 1, 3
  v = op(v, dpp_move<0x143, 0xC>(v, ident));  // row_bcast:31 into rows 2, 3
  return read_lane(v, 63);
}

// Wave maximum of values >= 0 (a NaN counts as 0, as the sequential
// max(m, v) = (m < v ? v : m) from 0 skips it).
__device__ __forceinline__ double wave_max_nonneg(double v) {
  v = v == v ? v : 0.0;
  return wave_reduce(v, 0.0, [](double a, double b) { return a < b ? b : a; });
}

__device__ __forceinline__ int wave_min_int(int v) {
  return wave_reduce(v, 0x7fffffff, [](int a, int b) { return b < a ? b : a; });
}

__device__ __forceinline__ int wave_sum_int(int v) {
  return wave_reduce(v, 0, [](int a, int b) { return a + b; });
}

// g_j(y) with y_k replaced by yk (a forward-difference evaluation).
template <class NET, class YP>
__device__ __forceinline__ double g_large_moved(int j, int k, YP y, double yk) {
  double gj = 1.0;
  for (int q = NET::RX_PTR[j]; q < NET::RX_PTR[j + 1]; ++q) {
    const int i = NET::RX_SP[q];
    gj = gj * binom_real(i == k ? yk : y[i], NET::RX_RO[q]);
  }
  return gj;
}

// The implicit leap of Rathinam et al. (2003), solved by the whole wave:
// Newton on
//   F(y) = y - c - tau sum_{j noncritical} nu_j a_j(y),
//   c = x + sum_j nu_j (P_j - tau a_j(x)) + nu_jc [fired],
// from y = x, with the analytic, forward-difference or caller-supplied
// Jacobian and an LU with partial pivoting per iteration, then the counts
// rounded.  In: S.tau, S.jc, S.th, S.ncr and the Poisson draws S.k, species
// counts xs; out: the rounded counts in S.k when the solve converged.
// Called by every lane of the wave.
// Entries of an LU row loaded per step: 8, except in kernels compiled for
// three or more waves per SIMD, whose register budget (168 or less) the
// larger chunk would exceed (the out-of-line solve adds its registers to the
// kernel's).
#if defined(LX_WAVES) && LX_WAVES >= 3
constexpr int LU_CHUNK = 1;
#else
constexpr int LU_CHUNK = 8;
#endif

struct NewtonOut {
  int iters;
  bool converged;
  int clips;
  unsigned long long cj, cl;  // cycles of Jacobian assembly and LU solves
};

template <class NET, class XV>
__device__ __noinline__ NewtonOut newton_core(SolveArea<NET>& S_area, const XV& xs,
                                              const SimParams& prm) {
  constexpr int N = NET::N, M = NET::M, LD = SolveArea<NET>::LD;
  LX_LDS SolveArea<NET>& S = *(LX_LDS SolveArea<NET>*)&S_area;
  const int lid = threadIdx.x & 63;
  const double tau = S.tau;
  const int jc = S.jc;
  const double* th = S.th;
  auto ncr = [&](int j) { return ((S.ncr[j >> 5] >> (j & 31)) & 1u) != 0u; };
  // tau a_j(x) and c, y = x
  for (int j = lid; j < M; j += 64) S.ax[j] = th[j] * g_large<NET>(j, xs);
  wave_sync();
  if (lid < N) {
    const int i = lid;
    double ci = (double)xs[i];
    for (int q = NET::NI_PTR[i]; q < NET::NI_PTR[i + 1]; ++q) {
      const int j = NET::NI_RX[q];
      if (!ncr(j)) continue;
      const double dj = (double)S.k[j] - tau * S.ax[j];
      ci = ci + (double)NET::NI_V[q] * dj;
    }
    if (jc >= 0)
      for (int q = NET::NJ_PTR[jc]; q < NET::NJ_PTR[jc + 1]; ++q)
        if (NET::NJ_SP[q] == i) ci = ci + (double)NET::NJ_V[q];
    S.c[i] = ci;
    S.y[i] = (double)xs[i];
  }
  wave_sync();
  NewtonOut out{0, false, 0, 0ull, 0ull};
  for (int it = 0; it < LXP(prm, newton_maxit); ++it) {
    out.iters += 1;
    const unsigned long long tj0 = LX_CLOCK();
    // a_j(y) of the non-critical reactions
    for (int j = lid; j < M; j += 64) S.ay[j] = ncr(j) ? th[j] * g_large_y<NET>(j, S.y) : 0.0;
    // d a_j / d y_k of every reactant slot
    for (int sl = lid; sl < NET::NSLOT; sl += 64) {
      const int j = NET::RX_J[sl];
      const int kk = NET::RX_SP[sl];
      double dd = 0.0;
      if (ncr(j)) {
        if (LXP(prm, jacobian) == 2) {
          dd = th[j] * dg_user_large<NET>(sl, S.y);
        } else if (LXP(prm, jacobian) == 1) {
          double yh;
          const double hk = fd_step(S.y[kk], &yh);
          const double ayh = th[j] * g_large_moved<NET>(j, kk, S.y, yh);
          dd = (ayh - th[j] * g_large_y<NET>(j, S.y)) / hk;
        } else {
          dd = th[j] * dg_large<NET>(j, kk, S.y);
        }
      }
      S.d[sl] = dd;
    }
    wave_sync();
    // residual and Jacobian row of species i (terms in ascending reaction order)
    if (lid < N) {
      const int i = lid;
      double si = 0.0;
      LX_LDS double* Ai = S.A + i * LD;
      for (int kk = 0; kk < N; ++kk) Ai[kk] = 0.0;
      for (int q = NET::NI_PTR[i]; q < NET::NI_PTR[i + 1]; ++q) {
        const int j = NET::NI_RX[q];
        if (!ncr(j)) continue;
        const double v = (double)NET::NI_V[q];
        si = si + v * S.ay[j];
        for (int sl = NET::RX_PTR[j]; sl < NET::RX_PTR[j + 1]; ++sl) {
          const int kk = NET::RX_SP[sl];
          Ai[kk] = Ai[kk] + v * S.d[sl];
        }
      }
      S.b[i] = -((S.y[i] - S.c[i]) - tau * si);
      for (int kk = 0; kk < N; ++kk) Ai[kk] = (i == kk ? 1.0 : 0.0) - tau * Ai[kk];
    }
    wave_sync();
    const unsigned long long tl0 = LX_CLOCK();
    out.cj += tl0 - tj0;
    // LU with partial pivoting: lane i holds stored row i, at logical position lp
    int lp = lid;
    bool lu_ok = true;
    for (int cc = 0; cc < N; ++cc) {
      const bool cand = lid < N && lp >= cc;
      const double v = cand ? __builtin_fabs(S.A[lid * LD + cc]) : -1.0;
      // the first maximal |pivot| in logical order from cc; a NaN is never
      // chosen, and a NaN at position cc fails the step
      const double vm = (cand && v == v) ? v : -1.0;
      const double best = wave_max_nonneg(vm < 0.0 ? 0.0 : vm);
      const unsigned long long at_cc = __ballot(cand && lp == cc);
      const int lane_cc = __ffsll((long long)at_cc) - 1;
      const double vcc = read_lane(v, lane_cc);
      const int piv = wave_min_int((cand && vm == best && vm >= 0.0) ? lp : 0x7fffffff);
      if (!(vcc == vcc) || !(best > 0.0) || piv == 0x7fffffff) {
        lu_ok = false;
        break;
      }
      if (lid < N) lp = lp == cc ? piv : (lp == piv ? cc : lp);
      const int pr = __ffsll((long long)__ballot(lid < N && lp == cc)) - 1;
      const LX_LDS double* Ap = S.A + pr * LD;
      if (lid < N && lp > cc) {
        LX_LDS double* Ai = S.A + lid * LD;
        const double l = Ai[cc] / Ap[cc];
        // in chunks of LU_CHUNK: the chunk's loads all issue before its
        // stores (the compiler cannot tell that row Ai is not row Ap); per
        // entry the same operations
        int q = cc;
        for (; q + LU_CHUNK <= N; q += LU_CHUNK) {
          double ai[LU_CHUNK], ap[LU_CHUNK];
#pragma unroll
          for (int u = 0; u < LU_CHUNK; ++u) {
            ai[u] = Ai[q + u];
            ap[u] = Ap[q + u];
          }
#pragma unroll
          for (int u = 0; u < LU_CHUNK; ++u) Ai[q + u] = ai[u] - l * ap[u];
        }
        for (; q < N; ++q) Ai[q] = Ai[q] - l * Ap[q];
        S.b[lid] = S.b[lid] - l * S.b[pr];
      }
      wave_sync();
    }
    if (lu_ok) {
      // back substitution, logical rows from the last (sequential)
      for (int rr = N - 1; rr >= 0; --rr) {
        if (lid < N && lp == rr) {
          const LX_LDS double* Ai = S.A + lid * LD;
          double sum = S.b[lid];
          // ascending q as in the sequential form, operands loaded LU_CHUNK
          // at a time
          int q = rr + 1;
          for (; q + LU_CHUNK <= N; q += LU_CHUNK) {
            double ai[LU_CHUNK], sv[LU_CHUNK];
#pragma unroll
            for (int u = 0; u < LU_CHUNK; ++u) {
              ai[u] = Ai[q + u];
              sv[u] = S.sol[q + u];
            }
#pragma unroll
            for (int u = 0; u < LU_CHUNK; ++u) sum = sum - ai[u] * sv[u];
          }
          for (; q < N; ++q) sum = sum - Ai[q] * S.sol[q];
          S.sol[rr] = sum / Ai[rr];
        }
        wave_sync();
      }
    }
    out.cl += LX_CLOCK() - tl0;
    if (!lu_ok) break;
    double ad = 0.0, ayv = 0.0;
    if (lid < N) {
      const double yi = S.y[lid] + S.sol[lid];
      S.y[lid] = yi;
      ad = __builtin_fabs(S.sol[lid]);
      ayv = __builtin_fabs(yi);
    }
    const double dmax = wave_max_nonneg(ad);
    const double ymax = wave_max_nonneg(ayv);
    wave_sync();
    if (!(dmax == dmax)) break;
    if (dmax <= LXP(prm, newton_tol) * (ymax < 1.0 ? 1.0 : ymax)) {
      out.converged = true;
      break;
    }
  }
  // rounded counts of the non-critical reactions
  int clips = 0;
  if (out.converged) {
    for (int j = lid; j < M; j += 64) {
      if (!ncr(j)) {
        S.k[j] = 0;
        continue;
      }
      const double gy = g_large_y<NET>(j, S.y);
      const double v = (tau * (th[j] * gy) - tau * S.ax[j]) + (double)S.k[j];
      double kr = __builtin_round(v);
      if (kr < 0.0) {
        kr = 0.0;
        clips += 1;
      }
      if (kr > 1073741824.0) kr = 1073741824.0;
      S.k[j] = (int)kr;
    }
  }
  out.clips = wave_sum_int(clips);
  wave_sync();
  return out;
}

// Solve the implicit leap parked by lane s (newton_core): lane s's parked
// data goes in and its counts, statistics and timers come back.  Called by
// every lane of the wave.
template <class P, class NET, bool GRID>
__device__ void coop_newton(LaneL<P, NET, GRID>& me, int s, SolveArea<NET>& S, const int* xcol_s,
                            const SimParams& prm) {
  constexpr int M = NET::M;
  const int lid = threadIdx.x & 63;
  const bool mine = lid == s;
  const unsigned long long ti0 = LX_CLOCK();
  if (mine) {
    S.tau = me.pend_tau;
    S.jc = me.pend_jc;
    S.th = me.th;
    for (int w = 0; w < SolveArea<NET>::W; ++w) S.ncr[w] = me.ncrw[w];
    for (int j = 0; j < M; ++j) S.k[j] = me.kd[j];
  }
  wave_sync();
  const NewtonOut o = newton_core<NET>(S, XSlot{(LX_LDS int*)xcol_s}, prm);
  if (mine) {
    me.n_nit += o.iters;
    me.pend_ok = o.converged;
    if (o.converged) {
      me.n_clip += (u32)o.clips;
      for (int j = 0; j < M; ++j) me.kd[j] = S.k[j];
    } else {
      me.n_nfail += 1;
    }
    me.cy_jac += o.cj;
    me.cy_lu += o.cl;
    me.cy_imp += LX_CLOCK() - ti0;
  }
  wave_sync();
}

// Batched schedule for large networks: block-owned particle ranges refilled
// from an LDS cursor, SSA bursts of up to ssa_k steps per leap iteration.
// The loop runs while any lane of the wave has a trajectory, so that every
// lane takes part in the cooperative solves of the implicit leaps parked in
// an iteration.
template <class NET>
__device__ __forceinline__ void run_large(long long blk, const double* __restrict__ theta,
                                          const int* __restrict__ x0, int* x_out, int* r_out,
                                          double* G_out, Stats* stats, const SimParams& prm,
                                          unsigned long long* next) {
  const int lane_id = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int waves = blockDim.x >> 6;
  const long long lo = blk * prm.per_block;
  long long hi = lo + prm.per_block;
  if (hi > prm.P) hi = prm.P;
  if (threadIdx.x == 0) *next = (unsigned long long)(lo + (long long)waves * prm.lanes);
  __syncthreads();
  const Key key{prm.k0, prm.k1};
  long long p = lo + (long long)wave * prm.lanes + lane_id;
  bool has = lane_id < prm.lanes && p < hi;
  __shared__ int xlds[NET::N * LX_BLOCK];
  __shared__ SolveArea<NET> areas[LX_BLOCK / 64];
  SolveArea<NET>& S = areas[wave];
  const int* xwave = xlds + (threadIdx.x & ~63);
  LaneL<LX_POLICY, NET, LX_GRID_ON> lane;
  lane.x.p = (LX_LDS int*)(xlds + threadIdx.x);
  lane.pend = false;
  if (has) lane.load(p, theta, x0, r_out, G_out, prm);
  while (__ballot(has) != 0ull) {
    if (has && lane.active(prm)) {
      lane.ssa_burst(prm, key, LXP(prm, ssa_k));
      if (lane.active(prm) && !lane.in_ssa(prm)) lane.step(prm, key);
    }
    // the implicit leaps parked in this iteration, one after another
    unsigned long long pend = __ballot(has && lane.pend);
    while (pend) {
      const int s = __ffsll((long long)pend) - 1;
      coop_newton(lane, s, S, xwave + s, prm);
      pend &= pend - 1ull;
    }
    if (has) {
      if (lane.pend) lane.finish_pending(prm);
      if (!lane.active(prm)) {
        bool again = false;
        if constexpr (LX_GRID_ON) again = lane.grid_next(p, prm);
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
}  // namespace lx

#if defined(LX_LARGE) && !defined(LX_WAVE)
extern "C" __global__ void __launch_bounds__(LX_BLOCK) LX_WAVES_ATTR
    lx_sim_large(const double* __restrict__ theta, const int* __restrict__ x0, int* x_out,
                 int* r_out, double* G_out, lx::Stats* stats, lx::SimParams prm) {
  __shared__ unsigned long long next;
  lx::run_large<LxNet>(blockIdx.x, theta, x0, x_out, r_out, G_out, stats, prm, &next);
}
#endif

#if defined(LX_HOOKS) && defined(LX_LARGE)
// Step decision on fixed states (test hook); crit/eq as ceil(M/32) mask words per case.
extern "C" __global__ void __launch_bounds__(64)
    lx_hook_tau(const double* __restrict__ theta, const int* __restrict__ xs, double* a_out,
                unsigned int* crit_out, unsigned int* eq_out, double* tau_out, int* action,
                lx::SimParams prm) {
  typedef LX_POLICY::R R;
  constexpr int M = LxNet::M;
  constexpr int W = (M + 31) / 32;
  const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= prm.P) return;
  __shared__ int xlds[LxNet::N * LX_BLOCK];
  lx::LaneL<LX_POLICY, LxNet> lane;
  lane.x.p = (LX_LDS int*)(xlds + threadIdx.x);
  lx::SimParams p2 = prm;
  p2.accumulate = 0;
  p2.pid_base = 0;
  lane.load(q, theta, xs, nullptr, nullptr, p2);
  lane.propensities();
  R tau_ex, tau_im;
  lane.decide(prm, &tau_ex, &tau_im);
  for (int j = 0; j < M; ++j) a_out[q * M + j] = (double)lane.a[j];
  for (int w = 0; w < W; ++w) {
    crit_out[q * W + w] = lane.critw[w];
    eq_out[q * W + w] = lane.eqw[w];
  }
  tau_out[2 * q] = (double)tau_ex;
  tau_out[2 * q + 1] = (double)tau_im;
  int act;
  if (lane.a0 == (R)0) act = 3;
  else if (lane.tau_p < (R)LXP(prm, k_ssa) / lane.a0 || lane.a0c >= lane.a0 / (R)LXP(prm, k_crit)) act = 2;
  else act = lane.implicit ? 1 : 0;
  action[q] = act;
}

// Implicit-leap solve on fixed states (test hook): the production
// cooperative solve, the wave taking its cases one after another.
extern "C" __global__ void __launch_bounds__(64)
    lx_hook_implicit(const double* __restrict__ theta, const int* __restrict__ xs,
                     const double* __restrict__ tau, const long long* __restrict__ Pj,
                     const int* __restrict__ jc, long long* k_out, int* ok_out, int* it_out,
                     lx::SimParams prm) {
  constexpr int M = LxNet::M;
  const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const bool valid = q < prm.P;
  __shared__ int xlds[LxNet::N * 64];
  __shared__ lx::SolveArea<LxNet> S;
  lx::LaneL<lx::F64, LxNet> lane;
  lane.x.p = (LX_LDS int*)(xlds + threadIdx.x);
  lx::SimParams p2 = prm;
  p2.accumulate = 0;
  p2.pid_base = 0;
  lane.pend = false;
  if (valid) {
    lane.load(q, theta, xs, nullptr, nullptr, p2);
    lane.propensities();
    for (int w = 0; w < lane.W; ++w) lane.ncrw[w] = 0u;
    for (int j = 0; j < M; ++j)
      if (lane.a[j] > 0.0 && j != jc[q]) lane.set_bit(lane.ncrw, j);
    for (int j = 0; j < M; ++j) lane.kd[j] = (int)Pj[q * M + j];
    lane.pend_tau = tau[q];
    lane.pend_jc = jc[q];
  }
  unsigned long long pend = __ballot(valid);
  while (pend) {
    const int s = __ffsll((long long)pend) - 1;
    lx::coop_newton(lane, s, S, xlds + s, prm);
    pend &= pend - 1ull;
  }
  if (!valid) return;
  const bool ok = lane.pend_ok;
  for (int j = 0; j < M; ++j) k_out[q * M + j] = ok ? lane.kd[j] : 0;
  ok_out[q] = ok ? 1 : 0;
  it_out[q] = (int)lane.n_nit;
}
#endif
