// lx_device.h -- device building blocks of the ensemble tau-leaping kernels:
// counter-based RNG, uniform maps, elementary functions and the samplers.
//
// This header is compiled twice: statically by hipcc (test-hook kernels in
// lx_hooks.hip) and at run time by hipRTC, where it is prepended to the
// network-specialised simulation source.  It therefore includes nothing and
// uses only compiler builtins.
//
// Floating point: compiled with -ffp-contract=off; every fused multiply-add is
// an explicit __builtin_fma.  Division and square root are the correctly
// rounded IEEE operations in both precisions.  The operation sequences below
// are fixed so that results are reproducible bit for bit.
#pragma once

namespace lx {

typedef unsigned int u32;
typedef unsigned long long u64;

#define LX_INF_F64 __builtin_inf()
#define LX_INF_F32 __builtin_inff()

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon et al., SC'11): ten rounds of two 32x32->64 products
// and xors with a Weyl-sequence key schedule.  Output is a pure function of
// (counter, key).
// ---------------------------------------------------------------------------
struct Words4 {
  u32 w0, w1, w2, w3;
};

__device__ __forceinline__ Words4 philox(u32 c0, u32 c1, u32 c2, u32 c3, u32 k0, u32 k1) {
#pragma unroll
  for (int round = 0; round < 10; ++round) {
    const u64 p0 = (u64)0xD2511F53u * (u64)c0;
    const u64 p1 = (u64)0xCD9E8D57u * (u64)c2;
    const u32 n0 = (u32)(p1 >> 32) ^ c1 ^ k0;
    const u32 n2 = (u32)(p0 >> 32) ^ c3 ^ k1;
    c1 = (u32)p1;
    c3 = (u32)p0;
    c0 = n0;
    c2 = n2;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  Words4 o;
  o.w0 = c0;
  o.w1 = c1;
  o.w2 = c2;
  o.w3 = c3;
  return o;
}

// Draw-site addressing: counter = (particle id, attempt e, site, trial).
constexpr u32 SITE_CRIT = 0x40000000u;
constexpr u32 SITE_SSA = 0x40000001u;

struct Key {
  u32 k0, k1;
};

__device__ __forceinline__ Words4 draw_block(const Key& key, u32 pid, u32 e, u32 site, u32 trial) {
  return philox(pid, e, site, trial, key.k0, key.k1);
}

// Open-interval uniforms, exact by construction.
__device__ __forceinline__ float uniform_f32(u32 w) {
  return ((float)(w >> 9) + 0.5f) * 0x1p-23f;
}
__device__ __forceinline__ double uniform_f64(u32 hi, u32 lo) {
  return ((double)(hi >> 6) * 67108864.0 + (double)(lo >> 6) + 0.5) * 0x1p-52;
}

// ---------------------------------------------------------------------------
// Elementary functions.
//   exp: x = k ln2 + r (Cody-Waite, ln2 split so k*LN2_HI is exact),
//        e^r by its Taylor polynomial in Horner form, times 2^k.
//   log: x = 2^e m, m in [sqrt(1/2), sqrt(2)), f = m - 1, s = f / (2 + f);
//        log(1 + f) = f - f^2/2 + s (f^2/2 + R(s^2)) with R the tail of the
//        atanh series, plus e ln2 in two parts (reduction and assembly as in
//        the published fdlibm log, e_log.c; the polynomial is the Taylor tail
//        of the atanh series, not fdlibm's minimax coefficients).
// ---------------------------------------------------------------------------
// Each function is a core for ordinary arguments (exp: within the overflow
// and underflow limits; log: positive and finite) and a wrapper that answers
// the special arguments with a final select, without divergent branches.
// The samplers call the cores: their arguments are ordinary by construction.
__device__ __forceinline__ double exp_core_f64(double x) {
  const double kd = __builtin_floor(x * 0x1.71547652b82fep0 + 0.5);
  const double hi = x - kd * 0x1.62e42feep-1;
  const double r = hi - kd * 0x1.a39ef35793c76p-33;
  double p = 1.0 / 6227020800.0;
  p = __builtin_fma(p, r, 1.0 / 479001600.0);
  p = __builtin_fma(p, r, 1.0 / 39916800.0);
  p = __builtin_fma(p, r, 1.0 / 3628800.0);
  p = __builtin_fma(p, r, 1.0 / 362880.0);
  p = __builtin_fma(p, r, 1.0 / 40320.0);
  p = __builtin_fma(p, r, 1.0 / 5040.0);
  p = __builtin_fma(p, r, 1.0 / 720.0);
  p = __builtin_fma(p, r, 1.0 / 120.0);
  p = __builtin_fma(p, r, 1.0 / 24.0);
  p = __builtin_fma(p, r, 1.0 / 6.0);
  p = __builtin_fma(p, r, 0.5);
  p = __builtin_fma(p, r, 1.0);
  p = __builtin_fma(p, r, 1.0);
  return __builtin_amdgcn_ldexp(p, (int)kd);
}

__device__ __forceinline__ double exp_f64(double x0) {
  const bool nan = x0 != x0, big = x0 > 709.782712893384, tiny = x0 < -745.2;
  const double y = exp_core_f64((nan || big || tiny) ? 0.0 : x0);
  return nan ? x0 : (big ? LX_INF_F64 : (tiny ? 0.0 : y));
}

__device__ __forceinline__ double log_core_f64(double x) {
  double m = __builtin_amdgcn_frexp_mant(x);  // [1/2, 1)
  int e = __builtin_amdgcn_frexp_exp(x);
  const bool lo = m < 0x1.6a09e667f3bcdp-1;
  m = lo ? m + m : m;
  e = lo ? e - 1 : e;
  const double f = m - 1.0;
  const double hfsq = (0.5 * f) * f;
  const double s = f / (2.0 + f);
  const double z = s * s;
  double q = 2.0 / 21.0;
  q = __builtin_fma(q, z, 2.0 / 19.0);
  q = __builtin_fma(q, z, 2.0 / 17.0);
  q = __builtin_fma(q, z, 2.0 / 15.0);
  q = __builtin_fma(q, z, 2.0 / 13.0);
  q = __builtin_fma(q, z, 2.0 / 11.0);
  q = __builtin_fma(q, z, 2.0 / 9.0);
  q = __builtin_fma(q, z, 2.0 / 7.0);
  q = __builtin_fma(q, z, 2.0 / 5.0);
  q = __builtin_fma(q, z, 2.0 / 3.0);
  const double R = z * q;
  const double ed = (double)e;
  return ed * 0x1.62e42feep-1 - ((hfsq - (s * (hfsq + R) + ed * 0x1.a39ef35793c76p-33)) - f);
}

__device__ __forceinline__ double log_f64(double x0) {
  const bool normal = x0 > 0.0 && x0 != LX_INF_F64;
  const double y = log_core_f64(normal ? x0 : 1.0);
  return normal ? y : (x0 == 0.0 ? -LX_INF_F64 : (x0 == LX_INF_F64 ? x0 : __builtin_nan("")));
}

__device__ __forceinline__ float exp_core_f32(float x) {
  const float kf = __builtin_floorf(x * 0x1.715476p0f + 0.5f);
  const float hi = x - kf * 0x1.62e4p-1f;
  const float r = hi - kf * 0x1.7f7d1cp-20f;
  float p = 1.0f / 5040.0f;
  p = __builtin_fmaf(p, r, 1.0f / 720.0f);
  p = __builtin_fmaf(p, r, 1.0f / 120.0f);
  p = __builtin_fmaf(p, r, 1.0f / 24.0f);
  p = __builtin_fmaf(p, r, 1.0f / 6.0f);
  p = __builtin_fmaf(p, r, 0.5f);
  p = __builtin_fmaf(p, r, 1.0f);
  p = __builtin_fmaf(p, r, 1.0f);
  return __builtin_amdgcn_ldexpf(p, (int)kf);
}

__device__ __forceinline__ float exp_f32(float x0) {
  const bool nan = x0 != x0, big = x0 > 88.72283f, tiny = x0 < -103.9721f;
  const float y = exp_core_f32((nan || big || tiny) ? 0.0f : x0);
  return nan ? x0 : (big ? LX_INF_F32 : (tiny ? 0.0f : y));
}

__device__ __forceinline__ float log_core_f32(float x) {
  float m = __builtin_amdgcn_frexp_mantf(x);
  int e = __builtin_amdgcn_frexp_expf(x);
  const bool lo = m < 0x1.6a09e6p-1f;
  m = lo ? m + m : m;
  e = lo ? e - 1 : e;
  const float f = m - 1.0f;
  const float hfsq = (0.5f * f) * f;
  const float s = f / (2.0f + f);
  const float z = s * s;
  float q = 2.0f / 11.0f;
  q = __builtin_fmaf(q, z, 2.0f / 9.0f);
  q = __builtin_fmaf(q, z, 2.0f / 7.0f);
  q = __builtin_fmaf(q, z, 2.0f / 5.0f);
  q = __builtin_fmaf(q, z, 2.0f / 3.0f);
  const float R = z * q;
  const float ef = (float)e;
  return ef * 0x1.62e4p-1f - ((hfsq - (s * (hfsq + R) + ef * 0x1.7f7d1cp-20f)) - f);
}

__device__ __forceinline__ float log_f32(float x0) {
  const bool normal = x0 > 0.0f && x0 != LX_INF_F32;
  const float y = log_core_f32(normal ? x0 : 1.0f);
  return normal ? y : (x0 == 0.0f ? -LX_INF_F32 : (x0 == LX_INF_F32 ? x0 : __builtin_nanf("")));
}

// log(k!) for integer-valued k >= 0: exact product for k <= 17, Stirling's
// series for log Gamma(k + 1) with four correction terms above.
__device__ __noinline__ double lfact_f64(double k) {
  if (k <= 17.0) {
    double prod = 1.0;
    for (double i = 2.0; i <= k; i = i + 1.0) prod = prod * i;
    return log_f64(prod);
  }
  const double n = k + 1.0;
  const double rn = 1.0 / n;
  const double rn2 = rn * rn;
  const double corr =
      rn * (1.0 / 12.0 - rn2 * (1.0 / 360.0 - rn2 * (1.0 / 1260.0 - rn2 * (1.0 / 1680.0))));
  return ((k + 0.5) * log_f64(n) - n) + 0x1.d67f1c864beb5p-1 + corr;
}

// ---------------------------------------------------------------------------
// Precision policies.  R is the type of propensities, tau bounds, Poisson
// means and sampler arithmetic; time, G and the implicit solve are double.
// ---------------------------------------------------------------------------
struct F64 {
  typedef double R;
  static constexpr bool mixed = false;
  // samplers' logs and exps: arguments positive and finite, resp. in [-30, 0)
  __device__ static __forceinline__ R ulog(R v) { return log_core_f64(v); }
  __device__ static __forceinline__ R uexp(R v) { return exp_core_f64(v); }
  __device__ static __forceinline__ R sqrt_(R v) { return __builtin_sqrt(v); }
  __device__ static __forceinline__ R floor_(R v) { return __builtin_floor(v); }
  __device__ static __forceinline__ R fabs_(R v) { return __builtin_fabs(v); }
  __device__ static __forceinline__ R fma_(R a, R b, R c) { return __builtin_fma(a, b, c); }
  __device__ static __forceinline__ void uniforms(const Words4& w, R* u1, R* u2) {
    *u1 = uniform_f64(w.w0, w.w1);
    *u2 = uniform_f64(w.w2, w.w3);
  }
  // PTRS candidates per Philox block, and candidate s of a block
  static constexpr u32 TRIALS_PER_BLOCK = 1;
  __device__ static __forceinline__ void candidate(const Words4& w, u32, R* u, R* v) {
    uniforms(w, u, v);
  }
  __device__ static __forceinline__ double wide_from() { return LX_INF_F64; }
  __device__ static __forceinline__ double lambda_max() { return 1073741824.0; }
  __device__ static __forceinline__ R inf() { return LX_INF_F64; }
};

struct Mixed {
  typedef float R;
  static constexpr bool mixed = true;
  __device__ static __forceinline__ R ulog(R v) { return log_core_f32(v); }
  __device__ static __forceinline__ R uexp(R v) { return exp_core_f32(v); }
  __device__ static __forceinline__ R sqrt_(R v) { return __builtin_sqrtf(v); }
  __device__ static __forceinline__ R floor_(R v) { return __builtin_floorf(v); }
  __device__ static __forceinline__ R fabs_(R v) { return __builtin_fabsf(v); }
  __device__ static __forceinline__ R fma_(R a, R b, R c) { return __builtin_fmaf(a, b, c); }
  __device__ static __forceinline__ void uniforms(const Words4& w, R* u1, R* u2) {
    *u1 = uniform_f32(w.w0);
    *u2 = uniform_f32(w.w1);
  }
  // one 32-bit word per uniform: a block holds two PTRS candidates
  static constexpr u32 TRIALS_PER_BLOCK = 2;
  __device__ static __forceinline__ void candidate(const Words4& w, u32 s, R* u, R* v) {
    *u = uniform_f32(s ? w.w2 : w.w0);
    *v = uniform_f32(s ? w.w3 : w.w1);
  }
  // binary32 holds every integer count exactly below 2^24: means at or above
  // 2^22 are drawn by the binary64 sampler (poisson_sample), so the range is
  // binary64's
  __device__ static __forceinline__ double wide_from() { return 4194304.0; }
  __device__ static __forceinline__ double lambda_max() { return 1073741824.0; }
  __device__ static __forceinline__ R inf() { return LX_INF_F32; }
};

// ---------------------------------------------------------------------------
// Poisson sampler: inversion below lam_thr (one uniform), PTRS of Hoermann
// (1993) above, all in the policy's precision.  PTRS candidate t is candidate
// t mod TRIALS_PER_BLOCK of Philox block t / TRIALS_PER_BLOCK.  Returns -1
// when lam is beyond the policy's range.
// ---------------------------------------------------------------------------

// log(1 + d), d > -1: log of the rounded u = 1 + d scaled by d / (u - 1)
// (Goldberg 1991, Theorem 4).
template <class P>
__device__ __forceinline__ typename P::R log1p_r(typename P::R d) {
  typedef typename P::R R;
  const R u = (R)1 + d;
  if (u == (R)1) return d;
  return P::ulog(u) * (d / (u - (R)1));
}

// phi(d) = log(1 + d) - d.  For |d| <= 1/4 by the atanh series in
// s = d / (2 + d): phi = 2 s^3 (1/3 + s^2/5 + ... + s^18/21) - d s; else
// log1p_r(d) - d.
template <class P>
__device__ __forceinline__ typename P::R log1p_minus_id(typename P::R d) {
  typedef typename P::R R;
  if (P::fabs_(d) <= (R)0.25) {
    const R s = d / ((R)2 + d);
    const R z = s * s;
    R q = (R)(2.0 / 21.0);
    q = P::fma_(q, z, (R)(2.0 / 19.0));
    q = P::fma_(q, z, (R)(2.0 / 17.0));
    q = P::fma_(q, z, (R)(2.0 / 15.0));
    q = P::fma_(q, z, (R)(2.0 / 13.0));
    q = P::fma_(q, z, (R)(2.0 / 11.0));
    q = P::fma_(q, z, (R)(2.0 / 9.0));
    q = P::fma_(q, z, (R)(2.0 / 7.0));
    q = P::fma_(q, z, (R)(2.0 / 5.0));
    q = P::fma_(q, z, (R)(2.0 / 3.0));
    return ((s * z) * q) - d * s;
  }
  return log1p_r<P>(d) - d;
}

// The PTRS acceptance test at candidate k (mean lam >= 10) is
// log(ratio * factor) <= rhs with log p(k; lam) = rhs - log(factor): for
// k <= 17 factor = k! (exact product) and rhs = k log lam - lam; beyond,
// Stirling's series for log Gamma(k + 1) with four correction terms c(n),
// n = k + 1, d = (lam - n) / n, rhs = k phi(d) - d - log(2 pi)/2 - c(n) and
// factor = sqrt(n).  Every term is O(1) near the mode.
template <class P>
__device__ __forceinline__ void ptrs_log_density(typename P::R kf, typename P::R lam,
                                                 typename P::R* factor, typename P::R* rhs) {
  typedef typename P::R R;
  if (kf > (R)17) {
    const R n = kf + (R)1;
    const R rn = (R)1 / n;
    const R rn2 = rn * rn;
    const R corr =
        rn * ((R)(1.0 / 12.0) -
              rn2 * ((R)(1.0 / 360.0) - rn2 * ((R)(1.0 / 1260.0) - rn2 * (R)(1.0 / 1680.0))));
    const R d = (lam - n) / n;
    *rhs = (kf * log1p_minus_id<P>(d) - d) - ((R)0x1.d67f1c864beb5p-1 + corr);
    *factor = P::sqrt_(n);
  } else {
    R f = (R)1;
    for (R i = (R)2; i <= kf; i = i + (R)1) f = f * i;
    *rhs = kf * P::ulog(lam) - lam;
    *factor = f;
  }
}

// PTRS constants of a mean (Hoermann 1993).
template <class P>
struct PtrsParams {
  typename P::R lam, a, b, inv_alpha, vr;
};

template <class P>
__device__ __forceinline__ PtrsParams<P> ptrs_params(typename P::R lam) {
  typedef typename P::R R;
  PtrsParams<P> c;
  c.lam = lam;
  const R slam = P::sqrt_(lam);
  c.b = (R)0.931 + (R)2.53 * slam;
  c.a = (R)-0.059 + (R)0.02483 * c.b;
  c.inv_alpha = (R)1.1239 + (R)1.1328 / (c.b - (R)3.4);
  c.vr = (R)0.9277 - (R)3.6224 / (c.b - (R)2);
  return c;
}

// Candidate `slot` of the Philox block `w` (the candidate of trial t is
// slot t mod TRIALS_PER_BLOCK of block t / TRIALS_PER_BLOCK): true with *k
// when accepted.
template <class P>
__device__ __forceinline__ bool ptrs_candidate(const PtrsParams<P>& c, const Words4& w, u32 slot,
                                               long long* k) {
  typedef typename P::R R;
  R u0, v;
  P::candidate(w, slot, &u0, &v);
  const R u = u0 - (R)0.5;
  const R us = (R)0.5 - P::fabs_(u);
  const R kf = P::floor_((((R)2 * c.a) / us + c.b) * u + c.lam + (R)0.43);
  if constexpr (P::mixed) {
    // binary32: the outcomes of the transformed-rejection test evaluated
    // without per-lane branches: out of range, quick acceptance, quick
    // rejection, and the density test, which the wave computes for all its
    // lanes when any of them needs it (a full wave nearly always holds one;
    // a wave down to a few trajectories often does not).  A candidate out of
    // range takes the test at k = 0, harmlessly; the accepted set is the one
    // of the sequential test.  In binary64 the density test costs more than
    // the branches it saves.
    const bool range = (kf >= (R)0) & ((double)kf <= 1073741824.0);
    const bool quick = (us >= (R)0.07) & (v <= c.vr);
    const bool qrej = (us < (R)0.013) & (v > us);
    const R ks = range ? kf : (R)0;
    *k = (long long)ks;
    bool accept = range & quick;
    const bool test = range & !quick & !qrej;
    if (__ballot(test) != 0ull) {
      const R hat = c.a / (us * us) + c.b;
      R fac, rhs;
      ptrs_log_density<P>(ks, c.lam, &fac, &rhs);
      const R lhs = P::ulog(((v * c.inv_alpha) * fac) / hat);
      accept = accept | (test & (lhs <= rhs));
    }
    return accept;
  } else {
    if (kf < (R)0 || (double)kf > 1073741824.0) return false;
    if (us >= (R)0.07 && v <= c.vr) {
      *k = (long long)kf;
      return true;
    }
    if (us < (R)0.013 && v > us) return false;
    const R hat = c.a / (us * us) + c.b;
    R fac, rhs;
    ptrs_log_density<P>(kf, c.lam, &fac, &rhs);
    const R lhs = P::ulog(((v * c.inv_alpha) * fac) / hat);
    *k = (long long)kf;
    return lhs <= rhs;
  }
}

// Trials a PTRS draw makes before giving up (then floor(lam); probability
// below 1e-60).
constexpr u32 PTRS_TRIALS = 64;

template <class P>
__device__ __forceinline__ long long poisson_ptrs(typename P::R lam, const Key& key, u32 pid, u32 e,
                                                  u32 site) {
  const PtrsParams<P> c = ptrs_params<P>(lam);
  Words4 w = Words4{0u, 0u, 0u, 0u};
  for (u32 trial = 0; trial < PTRS_TRIALS; ++trial) {
    if (trial % P::TRIALS_PER_BLOCK == 0u)
      w = draw_block(key, pid, e, site, trial / P::TRIALS_PER_BLOCK);
    long long k;
    if (ptrs_candidate<P>(c, w, trial % P::TRIALS_PER_BLOCK, &k)) return k;
  }
  return (long long)__builtin_floor((double)lam);
}

// The binary64 PTRS draw of a binary32 mean at or beyond 2^22 (inline: an
// out-of-line call costs the simulation kernels more registers than the
// inlined sampler does).
__device__ __forceinline__ long long poisson_wide(double lam, Key key, u32 pid, u32 e, u32 site) {
  return poisson_ptrs<F64>(lam, key, pid, e, site);
}

// Inversion below the PTRS threshold (sequential search of the CDF).
template <class P>
__device__ __forceinline__ long long poisson_inversion(typename P::R lam, int kcap, const Key& key,
                                                       u32 pid, u32 e, u32 site) {
  typedef typename P::R R;
  const Words4 w = draw_block(key, pid, e, site, 0);
  R u, unused;
  P::uniforms(w, &u, &unused);
  R p = P::uexp(-lam);
  R F = p;
  int k = 0;
  while (u > F && k < kcap) {
    k = k + 1;
    p = (p * lam) / (R)k;
    const R Fn = F + p;
    if (Fn == F) break;  // the rest of the tail is below the CDF's resolution
    F = Fn;
  }
  return k;
}

template <class P>
__device__ __forceinline__ long long poisson_sample(typename P::R lam, typename P::R lam_thr,
                                                    int kcap, const Key& key, u32 pid, u32 e,
                                                    u32 site) {
  typedef typename P::R R;
  if (!(lam > (R)0)) return 0;
  if ((double)lam > P::lambda_max()) return -1;
  if constexpr (P::mixed) {
    if ((double)lam >= P::wide_from()) return poisson_wide((double)lam, key, pid, e, site);
  }
  if (lam < lam_thr) return poisson_inversion<P>(lam, kcap, key, pid, e, site);
  return poisson_ptrs<P>(lam, key, pid, e, site);
}

// Out-of-line form for kernels that sample many reactions per lane (keeps one
// copy of the rejection loop instead of one per unrolled call).
template <class P>
__device__ __noinline__ long long poisson_sample_call(typename P::R lam, typename P::R lam_thr,
                                                      int kcap, const Key& key, u32 pid, u32 e,
                                                      u32 site) {
  return poisson_sample<P>(lam, lam_thr, kcap, key, pid, e, site);
}

// ---------------------------------------------------------------------------
// Gamma(a > 0, scale 1): Marsaglia & Tsang (2000) with normal variates from
// the polar method for a >= 1.  Trial t draws block 2t for the polar pair and
// block 2t+1 for the acceptance uniform.  Below 1 their boost:
// Gamma(a) = Gamma(a + 1) U^(1/a), U the first uniform of block 128.  A shape
// that is not positive and finite gives NaN.
// ---------------------------------------------------------------------------
constexpr u32 SITE_RESAMPLE = 0x40000002u;
constexpr u32 SITE_GAMMA = 0x40000010u;  // + reaction index

__device__ __forceinline__ double gamma_ge1(double a, const Key& key, u32 pid, u32 e, u32 site) {
  const double d = a - 1.0 / 3.0;
  const double c = 1.0 / __builtin_sqrt(9.0 * d);
  for (u32 t = 0; t < 64; ++t) {
    const Words4 w = draw_block(key, pid, e, site, 2 * t);
    const double u1 = 2.0 * uniform_f64(w.w0, w.w1) - 1.0;
    const double u2 = 2.0 * uniform_f64(w.w2, w.w3) - 1.0;
    const double s = u1 * u1 + u2 * u2;
    if (s >= 1.0) continue;
    const double z = u1 * __builtin_sqrt((-2.0 * log_f64(s)) / s);
    const double t1 = 1.0 + c * z;
    if (t1 <= 0.0) continue;
    const double v = (t1 * t1) * t1;
    const Words4 w2 = draw_block(key, pid, e, site, 2 * t + 1);
    const double u = uniform_f64(w2.w0, w2.w1);
    const double zz = z * z;
    if (u < 1.0 - 0.0331 * (zz * zz)) return d * v;
    if (log_f64(u) < (((0.5 * zz) + d) - d * v) + d * log_f64(v)) return d * v;
  }
  return d;
}

__device__ __noinline__ double gamma_sample(double a, const Key& key, u32 pid, u32 e, u32 site) {
  if (!(a > 0.0) || a == LX_INF_F64) return __builtin_nan("");
  const bool boost = a < 1.0;
  const double y = gamma_ge1(boost ? a + 1.0 : a, key, pid, e, site);
  if (!boost) return y;
  const Words4 w = draw_block(key, pid, e, site, 128);
  const double u = uniform_f64(w.w0, w.w1);
  return y * exp_f64(log_f64(u) / a);
}

}  // namespace lx
