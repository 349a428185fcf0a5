// lx_sim_wave.h -- one trajectory per wave for large networks (the batched
// schedule of networks beyond the register-resident kernels of lx_sim.h).
//
// Reaction j belongs to lane j % 64 (slot j / 64 of that lane, at most four
// slots) and species i to lane i: theta, a, g, r, G and the leap's counts of
// a reaction live in registers of its lane, the count of a species in its
// lane and, for the reaction lanes to read, in the wave's LDS area.  The
// control flow is the trajectory's, so it is uniform across the wave; the
// lanes work in parallel on the per-reaction parts of a step (propensities,
// critical set, partial equilibrium, Poisson draws, G) and the per-species
// parts (tau bounds, state update).
//
// Every floating-point operation is that of lx::LaneL and of the oracle, in
// the same order.  The sums the method forms in ascending reaction order run
// as one chain: a0 in lane 0 over the propensities in LDS, whose partial sums
// are also the running sum the SSA step compares against (the chosen
// reaction is the first whose partial sum exceeds u a0), and a0c and the
// critical choice over the critical reactions in ascending order.  The sums
// over a species' reactions run in that species' lane, ascending; the minimum
// of the species' tau bounds does not depend on order.  Implicit leaps are
// solved by the wave (newton_core) with the Newton system in the block's LDS
// area, which the waves of a block take in turn.
#pragma once

namespace lx {

// Species counts in a plain LDS array.
struct XPlain {
  const int* p;
  __device__ __forceinline__ int operator[](int i) const { return p[i]; }
};

// The species' reaction lists (NI) go to LDS as 16-bit entries (reaction |
// net change << 8) when they fit: net changes in [-128, 127], at most 8192
// entries.
template <class NET>
struct NiTable {
  static constexpr int NNI = NET::NI_PTR[NET::N];
  static constexpr bool fits() {
    for (int q = 0; q < NNI; ++q)
      if (NET::NI_V[q] < -128 || NET::NI_V[q] > 127) return false;
    return NNI <= 8192;
  }
  static constexpr bool LDS = fits();
};

// g_j from the packed reactant slots of reaction j (2-bit count, then per
// slot species | order << 6, 8 bits each, ascending species as RX_*).
template <class XV>
__device__ __forceinline__ double g_packed(u32 rp, const XV& x) {
  double gj = 1.0;
  const int n = (int)(rp & 3u);
  for (int q = 0; q < n; ++q) {
    const u32 e = (rp >> (2 + 8 * q)) & 0xffu;
    gj = gj * binom_real((double)x[(int)(e & 63u)], (int)(e >> 6));
  }
  return gj;
}

template <class NET, class R>
struct WaveArea {
  static constexpr int MS = (NET::M + 63) / 64;  // reaction slots per lane
  static constexpr int MP = MS * 64;
  static constexpr int W = MP / 32;
  R a[MP];     // propensities
  R pref[MP];  // running sums a_0 + ... + a_j, ascending j (the a0 chain)
  R ae[MP];    // a_j of the reactions a tau bound sums over, 0 for the others
  int k[MP];   // counts of the current leap
  int x[NET::N];
  int xn[NET::N];
  u32 ncrw[W];  // non-critical reactions, bit j % 32 of word j / 32
  R rb;                           // broadcast of the chain's result
};

// Wave minimum with the sequential rule m = (v < m ? v : m) from +inf: a NaN
// is never chosen.
template <class R>
__device__ __forceinline__ R wave_min_r(R v) {
  v = v == v ? v : (R)__builtin_inf();
  return wave_reduce(v, (R)__builtin_inf(), [](R a, R b) { return b < a ? b : a; });
}

template <class P, class NET, bool GRID = false>
struct WaveTraj {
  typedef typename P::R R;
  static constexpr int N = NET::N;
  static constexpr int M = NET::M;
  static constexpr int MS = WaveArea<NET, R>::MS;

  WaveArea<NET, R>* L;
  int lid;
  // reactions of this lane (j = lid + 64 s)
  R thr[MS], a[MS];
  double g[MS], G[MS];  // g_j(x) of the current propensities, G_j
  int r[MS], kd[MS];
  bool ncr[MS];
  // network constants of those reactions: packed reactant slots (g_packed),
  // packed consumed species (2-bit count, then species | -change << 6 per
  // entry), partner reaction (-1 if none)
  u32 rxp[MS], njp[MS];
  int part[MS];
  // species of this lane (lid < N): its count, the range of its reaction
  // list and its tau-bound case
  int xi;
  int ni_lo, ni_hi, phi_c;
  const unsigned short* ni;  // the reaction lists in LDS (NiTable<NET>::LDS)
  // the trajectory (the same in every lane)
  unsigned long long cmask[MS];  // critical reactions of slot s
  u32 pid;
  const double* th;
  double t;
  u32 e;
  int status;
  double tend;  // end of the current stretch: the next observation time (GRID)
  int kt;       // index of that time (GRID)
  R a0, a0c;
  bool plan, implicit;
  R tau_p;
  int ssa_left;
  u32 n_ssa, n_ex, n_im, n_rej, n_nfail, n_clip, n_cf;
  long long n_nit;
  unsigned long long cy_jac, cy_lu, cy_imp, cy_t0;

  __device__ __forceinline__ int rx(int s) const { return lid + 64 * s; }

  __device__ static __forceinline__ bool bitw(const u32* w, int j) {
    return ((w[j >> 5] >> (j & 31)) & 1u) != 0u;
  }

  __device__ __forceinline__ double t_end_(const SimParams& prm) const {
    if constexpr (GRID) return tend;
    else return prm.t_end;
  }

  __device__ __forceinline__ bool active(const SimParams& prm) const {
    return status == LANE_OK && t < t_end_(prm);
  }

  // This lane's network constants, once per kernel.
  __device__ __forceinline__ void init(WaveArea<NET, R>* area, const unsigned short* ni_lds) {
    L = area;
    lid = threadIdx.x & 63;
    ni = ni_lds;
#pragma unroll
    for (int s = 0; s < MS; ++s) {
      const int j = rx(s);
      u32 rp = 0u, np = 0u;
      int pt = -1;
      if (j < M) {
        const int q0 = NET::RX_PTR[j], q1 = NET::RX_PTR[j + 1];
        rp = (u32)(q1 - q0);
        for (int q = q0; q < q1; ++q)
          rp |= ((u32)NET::RX_SP[q] | ((u32)NET::RX_RO[q] << 6)) << (2 + 8 * (q - q0));
        u32 c = 0u;
        for (int q = NET::NJ_PTR[j]; q < NET::NJ_PTR[j + 1]; ++q) {
          const int v = NET::NJ_V[q];
          if (v < 0) {
            np |= ((u32)NET::NJ_SP[q] | ((u32)(-v) << 6)) << (2u + 8u * c);
            c += 1u;
          }
        }
        np |= c;
        pt = NET::PARTNER[j];
      }
      rxp[s] = rp;
      njp[s] = np;
      part[s] = pt;
    }
    ni_lo = ni_hi = 0;
    phi_c = 0;
    if (lid < N) {
      ni_lo = NET::NI_PTR[lid];
      ni_hi = NET::NI_PTR[lid + 1];
      phi_c = NET::PHI[lid];
    }
  }

  // Entry q of the species' reaction lists: reaction | net change << 8.
  __device__ __forceinline__ void ni_entry(int q, int* j, int* v) const {
    if constexpr (NiTable<NET>::LDS) {
      const u32 w = ni[q];
      *j = (int)(w & 0xffu);
      *v = (int)(signed char)(w >> 8);
    } else {
      *j = NET::NI_RX[q];
      *v = NET::NI_V[q];
    }
  }

  __device__ __forceinline__ void load(long long p, const double* __restrict__ theta,
                                       const int* __restrict__ x0, const int* r_in,
                                       const double* G_in, const SimParams& prm) {
    pid = prm.pid_base + (u32)p * prm.pid_stride;
    th = theta + p * M;
    bool bad = false;
#pragma unroll
    for (int s = 0; s < MS; ++s) {
      const int j = rx(s);
      thr[s] = (R)0;
      a[s] = (R)0;
      g[s] = 0.0;
      G[s] = 0.0;
      r[s] = 0;
      kd[s] = 0;
      ncr[s] = false;
      cmask[s] = 0ull;
      if (j < M) {
        const double tj = th[j];
        thr[s] = (R)tj;
        bad = bad || !(tj >= 0.0) || tj == LX_INF_F64;
        if (LXP(prm, accumulate)) {
          r[s] = r_in[p * M + j];
          G[s] = G_in[p * M + j];
        }
      }
    }
    xi = 0;
    if (lid < N) {
      xi = x0[p * N + lid];
      bad = bad || xi < 0;
      L->x[lid] = xi;
    }
    status = __ballot(bad) != 0ull ? LANE_BAD_INPUT : LANE_OK;
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
    n_ssa = n_ex = n_im = n_rej = n_nfail = n_clip = n_cf = 0;
    n_nit = 0;
    cy_jac = cy_lu = cy_imp = 0;
    cy_t0 = LX_CLOCK();
    wave_sync();
  }

  // Observation times, as Lane::grid_next.
  __device__ __forceinline__ bool grid_next(long long p, const SimParams& prm) {
    const bool ok = status == LANE_OK;
    int* row = prm.x_grid + ((long long)p * prm.n_times + kt) * N;
    if (lid < N) row[lid] = ok ? xi : -1;
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
      if (lid < N) row[lid] = -1;
    }
    return false;
  }

  __device__ __forceinline__ void store_cycles(long long p, const SimParams& prm) const {
#ifdef LX_TIMERS
    if (lid == 0) {
      unsigned long long* c = prm.cycles + p * 4;
      c[0] = cy_jac;
      c[1] = cy_lu;
      c[2] = cy_imp;
      c[3] = LX_CLOCK() - cy_t0;
    }
#endif
  }

  __device__ __forceinline__ void store(long long p, int* x_out, int* r_out, double* G_out,
                                        Stats* stats) const {
    if (lid < N) x_out[p * N + lid] = xi;
#pragma unroll
    for (int s = 0; s < MS; ++s) {
      const int j = rx(s);
      if (j < M) {
        r_out[p * M + j] = r[s];
        G_out[p * M + j] = G[s];
      }
    }
    if (stats && lid == 0) {
      Stats st;
      st.status = status;
      st.crit_fired = n_cf;
      st.t_final = t;
      st.steps_ssa = n_ssa;
      st.steps_explicit = n_ex;
      st.steps_implicit = n_im;
      st.rejections = n_rej;
      st.newton_iters = n_nit;
      st.newton_fail = n_nfail;
      st.kclip = n_clip;
      st.attempts = e;
      stats[p] = st;
    }
  }

  // a_j = theta_j g_j (Background section); a0 summed in ascending j.
  __device__ __forceinline__ void propensities() {
    const XPlain xs{L->x};
#pragma unroll
    for (int s = 0; s < MS; ++s) {
      const int j = rx(s);
      double gj = 0.0;
      R aj = (R)0;
      if (j < M) {
        gj = g_packed(rxp[s], xs);
        aj = thr[s] * (R)gj;
      }
      g[s] = gj;
      a[s] = aj;
      L->a[j] = aj;
    }
    wave_sync();
    if (lid == 0) {
      R c = (R)0;
      for (int j = 0; j < M; ++j) {
        c = c + L->a[j];
        L->pref[j] = c;
      }
      L->rb = c;
    }
    wave_sync();
    a0 = L->rb;
  }

  __device__ __forceinline__ R phi() const {
    const int c = phi_c;
    if (c == 1) return (R)1;
    if (c == 2) return (R)2;
    if (c == 4) return (R)3;
    const R xm1 = (R)(xi - 1 > 1 ? xi - 1 : 1);
    if (c == 3) return (R)2 + (R)1 / xm1;
    if (c == 5) return (R)1.5 * ((R)2 + (R)1 / xm1);
    const R xm2 = (R)(xi - 2 > 1 ? xi - 2 : 1);
    return ((R)3 + (R)1 / xm1) + (R)2 / xm2;
  }

  // Tau selection (Cao 2006) over the reactions whose propensity the caller
  // left in L->ae (the non-critical ones, without those in partial
  // equilibrium for tau_im): species i's bound in lane i.  Where the
  // sequential form skips a reaction, this one adds v * 0 = +-0, which leaves
  // the sums unchanged (they start at +0, so they are never -0).
  __device__ __forceinline__ R tau_select(R eps) const {
    R ti = P::inf();
    if (lid < N && phi_c != 0) {
      R mu = (R)0, s2 = (R)0;
      for (int q = ni_lo; q < ni_hi; ++q) {
        int j, v;
        ni_entry(q, &j, &v);
        const R aj = L->ae[j];
        mu = mu + (R)v * aj;
        s2 = s2 + (R)(v * v) * aj;
      }
      R num = eps * (R)xi;
      if (phi_c != 1) num = num / phi();
      const R bound = num < (R)1 ? (R)1 : num;
      const R t1 = bound / P::fabs_(mu);
      const R t2 = (bound * bound) / s2;
      ti = t2 < t1 ? t2 : t1;
    }
    return wave_min_r<R>(ti);
  }

  __device__ __forceinline__ void decide(const SimParams& prm, R* tau_ex_out, R* tau_im_out) {
    const XPlain xs{L->x};
#pragma unroll
    for (int s = 0; s < MS; ++s) {
      const int j = rx(s);
      bool c = false, nc = false;
      if (j < M) {
        int Lj = 0x7fffffff;
        const int nc_ = (int)(njp[s] & 3u);
        for (int q = 0; q < nc_; ++q) {
          const u32 en = (njp[s] >> (2 + 8 * q)) & 0xffu;
          const int qq = xs[(int)(en & 63u)] / (int)(en >> 6);
          Lj = qq < Lj ? qq : Lj;
        }
        const bool pos = a[s] > (R)0;
        c = pos && Lj < LXP(prm, n_c);
        nc = pos && !c;
      }
      ncr[s] = nc;
      L->ae[j] = nc ? a[s] : (R)0;
      const unsigned long long cm = __ballot(c);
      const unsigned long long nm = __ballot(nc);
      cmask[s] = cm;
      if (lid == 0) {
        L->ncrw[2 * s] = (u32)nm;
        L->ncrw[2 * s + 1] = (u32)(nm >> 32);
      }
    }
    // a0c: the critical propensities in ascending j
    a0c = (R)0;
#pragma unroll
    for (int s = 0; s < MS; ++s) {
      unsigned long long m = cmask[s];
      while (m) {
        const int j = 64 * s + __ffsll((long long)m) - 1;
        m &= m - 1ull;
        a0c = a0c + L->a[j];
      }
    }
    wave_sync();
    const R eps = (R)LXP(prm, eps);
    const R tau_ex = tau_select(eps);
    implicit = false;
    tau_p = tau_ex;
    *tau_ex_out = tau_ex;
    *tau_im_out = P::inf();
    if (NET::NPAIRS > 0 && LXP(prm, mode) == MODE_ADAPTIVE) {
      const R delta = (R)LXP(prm, delta);
      bool any_eq = false;
      bool eqs[MS];
      wave_sync();  // tau_ex has read L->ae
#pragma unroll
      for (int s = 0; s < MS; ++s) {
        const int j = rx(s);
        bool q = false;
        if (j < M) {
          const int k = part[s];
          if (k >= 0 && ncr[s] && bitw(L->ncrw, k)) {
            // the pair's test as the smaller index states it
            const R aj = L->a[j < k ? j : k];
            const R ak = L->a[j < k ? k : j];
            const R lo = ak < aj ? ak : aj;
            q = P::fabs_(aj - ak) <= delta * lo;
          }
        }
        eqs[s] = q;
        const unsigned long long em = __ballot(q);
        any_eq = any_eq || em != 0ull;
      }
      if (any_eq) {
#pragma unroll
        for (int s = 0; s < MS; ++s) L->ae[rx(s)] = (ncr[s] && !eqs[s]) ? a[s] : (R)0;
        wave_sync();
        const R tau_im = tau_select(eps);
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
    for (int s = 0; s < MS; ++s) G[s] = G[s] + g[s] * rem;
    t = t_end_(prm);
  }

  // Species counts after reaction jf fires once (SSA) or the leap's counts
  // (the caller's xn): lanes < N publish theirs to LDS.
  __device__ __forceinline__ void publish_x() {
    if (lid < N) L->x[lid] = xi;
    wave_sync();
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
    // the first reaction whose running sum exceeds thr_, else the last one
    // with a positive propensity
    int jf = -1;
#pragma unroll
    for (int s = 0; s < MS; ++s) {
      const int j = rx(s);
      const unsigned long long m = __ballot(j < M && L->pref[j] > thr_);
      if (jf < 0 && m) jf = 64 * s + __ffsll((long long)m) - 1;
    }
    if (jf < 0) {
#pragma unroll
      for (int s = MS - 1; s >= 0; --s) {
        const int j = rx(s);
        const unsigned long long m = __ballot(j < M && a[s] > (R)0);
        if (jf < 0 && m) jf = 64 * s + 63 - __clzll((long long)m);
      }
    }
#pragma unroll
    for (int s = 0; s < MS; ++s) {
      G[s] = G[s] + g[s] * tau_s;
      if (rx(s) == jf) r[s] = r[s] + 1;
    }
    for (int q = NET::NJ_PTR[jf]; q < NET::NJ_PTR[jf + 1]; ++q)
      if (lid == NET::NJ_SP[q]) xi += NET::NJ_V[q];
    publish_x();
    t = t + tau_s;
  }

  // The implicit leap's counts by the wave's Newton solve in the block's
  // shared area S (taken under `lock` when the block has several waves).
  __device__ __forceinline__ bool solve_implicit(double tau, int jc, SolveArea<NET>& S, int* lock,
                                                 const SimParams& prm) {
    const unsigned long long ti0 = LX_CLOCK();
#pragma unroll
    for (int s = 0; s < MS; ++s) L->k[rx(s)] = kd[s];
    if (lock) {
      if (lid == 0)
        while (atomicCAS(lock, 0, 1) != 0) __builtin_amdgcn_s_sleep(2);
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    }
    wave_sync();
    if (lid == 0) {
      S.tau = tau;
      S.jc = jc;
      S.th = th;
    }
    for (int w = lid; w < SolveArea<NET>::W; w += 64) S.ncr[w] = L->ncrw[w];
    for (int j = lid; j < M; j += 64) S.k[j] = L->k[j];
    wave_sync();
    const NewtonOut o = newton_core<NET>(S, XPlain{L->x}, prm);
    if (o.converged) {
#pragma unroll
      for (int s = 0; s < MS; ++s)
        if (rx(s) < M) kd[s] = S.k[rx(s)];
    }
    wave_sync();
    if (lock) {
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
      if (lid == 0) atomicExch(lock, 0);
    }
    n_nit += o.iters;
    if (o.converged) n_clip += (u32)o.clips;
    else n_nfail += 1;
    cy_jac += o.cj;
    cy_lu += o.cl;
    cy_imp += LX_CLOCK() - ti0;
    return o.converged;
  }

  // One leap attempt with the current plan.
  __device__ __forceinline__ void leap_attempt(const SimParams& prm, const Key& key,
                                               SolveArea<NET>& S, int* lock) {
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
      bool done = false;
#pragma unroll
      for (int s = 0; s < MS; ++s) {
        unsigned long long m = done ? 0ull : cmask[s];
        while (m) {
          const int j = 64 * s + __ffsll((long long)m) - 1;
          m &= m - 1ull;
          jlast = j;
          cum = cum + L->a[j];
          if (cum > thr_) {
            jc = j;
            done = true;
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
    // counts fit int32: the samplers' means are at most 2^30 and the
    // implicit counts are clamped there
    // one inlined sampler in a rolled loop over the slots (the slot's values
    // picked by selects, so that they stay in registers)
    bool overflow = false;
#pragma unroll 1
    for (int s = 0; s < MS; ++s) {
      R as = a[0];
      bool ns = ncr[0];
#pragma unroll
      for (int u = 1; u < MS; ++u)
        if (s == u) {
          as = a[u];
          ns = ncr[u];
        }
      long long kj = 0;
      if (ns) kj = poisson_sample<P>(as * tau_rr, lam_thr, LXP(prm, kcap), key, pid, ea, (u32)rx(s));
      overflow = overflow || kj < 0;
#pragma unroll
      for (int u = 0; u < MS; ++u)
        if (s == u) kd[u] = (int)kj;
    }
    if (__ballot(overflow) != 0ull) {
      status = LANE_LAMBDA_OVERFLOW;
      return;
    }
    bool ok = true;
    if (implicit) ok = solve_implicit(tau, jc, S, lock, prm);
    leap_accept(tau, jc, last, ok, prm);
  }

  // The rest of a leap attempt once its counts kd are known (`ok`: an
  // implicit solve converged, or an explicit leap).
  __device__ __forceinline__ void leap_accept(double tau, int jc, bool last, bool ok,
                                              const SimParams& prm) {
    int xn = 0;
    bool big = false;
    if (ok) {
#pragma unroll
      for (int s = 0; s < MS; ++s) {
        if (rx(s) == jc) kd[s] = 1;
        L->k[rx(s)] = kd[s];
      }
      wave_sync();
      bool okl = true, bigl = false;
      if (lid < N) {
        long long v = xi;
        for (int q = ni_lo; q < ni_hi; ++q) {
          int j, c;
          ni_entry(q, &j, &c);
          v = v + (long long)c * L->k[j];
        }
        okl = v >= 0;
        bigl = v > 2147483647LL;
        xn = (int)v;
      }
      ok = __ballot(!okl) == 0ull;
      big = __ballot(bigl) != 0ull;
    }
    if (!ok) {
      n_rej += 1;
      tau_p = tau_p / (R)2;
      return;
    }
    bool bigr = false;
#pragma unroll
    for (int s = 0; s < MS; ++s) bigr = bigr || (long long)r[s] + kd[s] > 2147483647LL;
    if (big || __ballot(bigr) != 0ull) {
      status = LANE_COUNT_OVERFLOW;
      return;
    }
    if (lid < N) L->xn[lid] = xn;
    wave_sync();
    // trapezoid with the old and the accepted state
    const XPlain xs_new{L->xn};
#pragma unroll
    for (int s = 0; s < MS; ++s) {
      const int j = rx(s);
      if (j < M) {
        const double gn = g_packed(rxp[s], xs_new);
        G[s] = G[s] + (tau * (g[s] + gn)) * 0.5;
        r[s] = r[s] + kd[s];
      }
    }
    xi = xn;
    publish_x();
    t = last ? t_end_(prm) : t + tau;
    if (implicit) n_im += 1;
    else n_ex += 1;
    n_cf += jc >= 0 ? 1u : 0u;
    plan = false;
  }

  __device__ __forceinline__ void step(const SimParams& prm, const Key& key, SolveArea<NET>& S,
                                       int* lock) {
    if (!plan) propensities();
    if (a0 == (R)0) {
      absorb(prm);
      return;
    }
    if (LXP(prm, mode) != MODE_SSA && ssa_left == 0) {
      if (!plan) {
        R tau_ex, tau_im;
        decide(prm, &tau_ex, &tau_im);
      }
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
    leap_attempt(prm, key, S, lock);
  }
};

// Batched schedule, one trajectory per wave: block `blk` owns particles
// [blk*per_block, (blk+1)*per_block); each wave takes the block's next
// particle from an LDS cursor when its trajectory ends.
template <class NET>
__device__ __forceinline__ void run_wave(long long blk, const double* __restrict__ theta,
                                         const int* __restrict__ x0, int* x_out, int* r_out,
                                         double* G_out, Stats* stats, const SimParams& prm) {
  typedef typename LX_POLICY::R R;
  __shared__ WaveArea<NET, R> areas[LX_BLOCK / 64];
  __shared__ SolveArea<NET> S;
  __shared__ unsigned short ni_tab[NiTable<NET>::LDS ? NiTable<NET>::NNI + 1 : 1];
  __shared__ unsigned long long next;
  __shared__ int lock;
  if constexpr (NiTable<NET>::LDS)
    for (int q = threadIdx.x; q < NiTable<NET>::NNI; q += blockDim.x)
      ni_tab[q] = (unsigned short)((u32)NET::NI_RX[q] | (((u32)NET::NI_V[q] & 0xffu) << 8));
  const int wave = threadIdx.x >> 6;
  const int waves = blockDim.x >> 6;
  const long long lo = blk * prm.per_block;
  long long hi = lo + prm.per_block;
  if (hi > prm.P) hi = prm.P;
  if (threadIdx.x == 0) {
    next = (unsigned long long)(lo + waves);
    lock = 0;
  }
  __syncthreads();
  const Key key{prm.k0, prm.k1};
  WaveTraj<LX_POLICY, NET, LX_GRID_ON> tr;
  tr.init(&areas[wave], ni_tab);
  int* lk = waves > 1 ? &lock : nullptr;
  long long p = lo + wave;
  while (p < hi) {
    tr.load(p, theta, x0, r_out, G_out, prm);
    for (;;) {
      while (tr.active(prm)) tr.step(prm, key, S, lk);
      if constexpr (LX_GRID_ON) {
        if (tr.grid_next(p, prm)) continue;
      }
      break;
    }
    tr.store(p, x_out, r_out, G_out, stats);
    tr.store_cycles(p, prm);
    unsigned long long pn = 0;
    if (tr.lid == 0) pn = atomicAdd(&next, 1ull);
    p = (long long)__shfl((long long)pn, 0, 64);
  }
}
}  // namespace lx

#if defined(LX_LARGE) && defined(LX_WAVE)
extern "C" __global__ void __launch_bounds__(LX_BLOCK) LX_WAVES_ATTR
    lx_sim_wave(const double* __restrict__ theta, const int* __restrict__ x0, int* x_out,
                int* r_out, double* G_out, lx::Stats* stats, lx::SimParams prm) {
  lx::run_wave<LxNet>(blockIdx.x, theta, x0, x_out, r_out, G_out, stats, prm);
}
#endif
