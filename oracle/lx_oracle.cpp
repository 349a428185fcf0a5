// lx_oracle.cpp -- CPU oracle for ensemble adaptive explicit/implicit tau-leaping.
//
// TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, double-precision
// statement of what the GPU path must compute.  Only the test suite, the smoke
// check and the CPU-baseline leg of the benchmark may load it; the product
// library never links, calls or falls back to it, and it shares no source with
// the HIP path (its RNG, math functions, samplers, LU and step logic are all
// written here, independently).
//
// Method (paper: matLeap, arXiv 1608.07058):
//   * propensity a_j = theta_j * g_j(X), g_j a function of the reactant
//     ("educt") copy numbers -- Background section.
//   * summary statistics r_j (firings) and G_j = integral of g_j(X_s) ds,
//     trapezoid rule while leaping, exact while doing SSA -- Background section.
//   * adaptive explicit/implicit tau-leaping of Cao, Gillespie & Petzold 2007,
//     implicit when the leap computed without the reaction pairs in partial
//     equilibrium is much larger; critical reactions for non-negativity; the
//     matLeap switch to SSA when the expected wait to the next critical
//     reaction is comparable to the wait to the next reaction --
//     Implementation section.
//   * tau bounded by the relative change / variance rule (Cao 2006) --
//     Background section.
//   * exact SSA, Gillespie 1977 direct method -- Background section.
//   * implicit step: Rathinam et al. 2003, solved by Newton with an analytic
//     mass-action Jacobian -- Background section (inverse Jacobian).
//
// Precision.  Everything is double precision ("fp64").  A second instance of
// the same step logic ("mixed") evaluates propensities, tau bounds, Poisson
// means and the samplers in binary32 while time, G and the Newton solve stay
// double; it exists so that the GPU mixed-precision path can be checked
// element by element.  Floating-point contraction is disabled (-ffp-contract=off)
// and every fused multiply-add is an explicit std::fma call.
//
// Readings where the paper is silent are listed at each step ("reading:").
//
// Pins (tests/test_oracle_samplers.py, tests/test_oracle_method.py): Philox
// against its published constants, a second implementation and uniformity;
// exp/log within one ulp of multiple precision; inversion equal to the exact
// Poisson quantile; PTRS and exponential laws; tau selection on hand-worked
// cases; the implicit solve against a direct solve and its residual; exact SSA
// against closed forms and master-equation solutions; the leap modes against
// exact invariants and the laws at the tau-leap error level.  The adaptive
// method as a whole is parity unpinned against matLeap's own program: neither
// its code nor its models nor numbers at these workloads are available.

#include <algorithm>
#include <cstdio>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <limits>
#include <thread>
#include <vector>

namespace {

// Algorithmic operation count of the current trajectory (lane-level
// arithmetic, comparison and integer operations the method performs; a
// division or square root counts as one operation).  Used only to state the
// work behind a measured time; it does not affect any result.
thread_local uint64_t g_ops = 0;
inline void count_ops(uint64_t n) { g_ops += n; }
const uint64_t OPS_PHILOX = 100;  // 10 rounds x (2 mul-hi, 2 mul-lo, 4 xor, 2 key adds)
const uint64_t OPS_EXP = 20;      // 4 reduction, 13 fma, scale, 2 range tests
const uint64_t OPS_LOG = 30;      // split, 3 for f/s, 11 series, 8 assembly, tests
const uint64_t OPS_UNIFORM = 4;

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror & Shaw, SC'11).  Counter-based: the
// output is a pure function of a 128-bit counter and a 64-bit key.
// ---------------------------------------------------------------------------
const uint32_t PHILOX_M0 = 0xD2511F53u;
const uint32_t PHILOX_M1 = 0xCD9E8D57u;
const uint32_t PHILOX_W0 = 0x9E3779B9u;  // golden ratio, 32-bit fraction
const uint32_t PHILOX_W1 = 0xBB67AE85u;  // sqrt(3) - 1, 32-bit fraction

void philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4]) {
  uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
  uint32_t k0 = key_in[0], k1 = key_in[1];
  for (int round = 0; round < 10; ++round) {
    if (round > 0) {  // key schedule: Weyl sequence between rounds
      k0 += PHILOX_W0;
      k1 += PHILOX_W1;
    }
    uint64_t prod0 = (uint64_t)PHILOX_M0 * (uint64_t)c0;
    uint64_t prod1 = (uint64_t)PHILOX_M1 * (uint64_t)c2;
    uint32_t hi0 = (uint32_t)(prod0 >> 32), lo0 = (uint32_t)prod0;
    uint32_t hi1 = (uint32_t)(prod1 >> 32), lo1 = (uint32_t)prod1;
    uint32_t n0 = hi1 ^ c1 ^ k0;
    uint32_t n1 = lo1;
    uint32_t n2 = hi0 ^ c3 ^ k1;
    uint32_t n3 = lo0;
    c0 = n0; c1 = n1; c2 = n2; c3 = n3;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

// Uniform maps, exact by construction so never 0 or 1.
//   binary32: 23 random bits plus one half, scaled by 2^-23.
//   binary64: 26 + 26 random bits plus one half, scaled by 2^-52.
float uniform_f32(uint32_t w) { return ((float)(w >> 9) + 0.5f) * 0x1p-23f; }
double uniform_f64(uint32_t w0, uint32_t w1) {
  return ((double)(w0 >> 6) * 67108864.0 + (double)(w1 >> 6) + 0.5) * 0x1p-52;
}

// Draw sites.  A block of four Philox words is addressed by
//   key     = (seed_lo, seed_hi + rng_stream)
//   counter = (particle id, attempt index e, site, trial)
// where e counts the trajectory's leap attempts and SSA steps, site is the
// reaction index for a Poisson count or one of the two constants below, and
// trial numbers the rejection-sampler rounds.  Results therefore depend only
// on (seed, stream, particle id), never on how particles are scheduled.
const uint32_t SITE_CRIT = 0x40000000u;
const uint32_t SITE_SSA = 0x40000001u;

struct Rng {
  uint32_t key[2];
  uint32_t pid;
  void block(uint32_t e, uint32_t site, uint32_t trial, uint32_t out[4]) const {
    uint32_t ctr[4] = {pid, e, site, trial};
    philox4x32_10(ctr, key, out);
    count_ops(OPS_PHILOX);
  }
};

// ---------------------------------------------------------------------------
// Elementary functions, written from the standard methods so that the same
// operation sequence can be reproduced on another machine:
//   exp: Cody-Waite reduction x = k ln2 + r, |r| <= ln2/2, Taylor polynomial
//        of e^r evaluated by Horner with fma, scaled by 2^k.
//   log: x = 2^e m with m in [sqrt(1/2), sqrt(2)), f = m - 1, s = f/(2+f),
//        log(1+f) = f - f^2/2 + s (f^2/2 + R(s^2)), where R is the tail of the
//        series 2 atanh(s) = 2s + 2s^3/3 + 2s^5/5 + ...; plus e ln2 in two parts.
//        The reduction, the two-part ln 2 and the order in which the result
//        is assembled follow the published fdlibm formulation of log
//        (Sun Microsystems, e_log.c); the polynomial here is the Taylor tail
//        of the atanh series, not fdlibm's minimax coefficients.
// ---------------------------------------------------------------------------
const double LN2_HI = 0x1.62e42feep-1;          // ln 2 truncated to 32 bits
const double LN2_LO = 0x1.a39ef35793c76p-33;    // ln 2 - LN2_HI, rounded
const double LOG2E = 0x1.71547652b82fep0;       // 1 / ln 2, rounded
const double SQRT_HALF = 0x1.6a09e667f3bcdp-1;  // sqrt(1/2), rounded
const float LN2_HI_F = 0x1.62e4p-1f;            // ln 2 truncated to 16 bits
const float LN2_LO_F = 0x1.7f7d1cp-20f;         // ln 2 - LN2_HI_F, rounded
const float LOG2E_F = 0x1.715476p0f;
const float SQRT_HALF_F = 0x1.6a09e6p-1f;

double exp_f64(double x) {
  if (x != x) return x;
  if (x > 709.782712893384) return std::numeric_limits<double>::infinity();
  if (x < -745.2) return 0.0;
  double kd = std::floor(x * LOG2E + 0.5);
  double hi = x - kd * LN2_HI;  // exact (Sterbenz)
  double r = hi - kd * LN2_LO;
  double p = 1.0 / 6227020800.0;          // 1/13!
  p = std::fma(p, r, 1.0 / 479001600.0);  // 1/12!
  p = std::fma(p, r, 1.0 / 39916800.0);   // 1/11!
  p = std::fma(p, r, 1.0 / 3628800.0);    // 1/10!
  p = std::fma(p, r, 1.0 / 362880.0);     // 1/9!
  p = std::fma(p, r, 1.0 / 40320.0);      // 1/8!
  p = std::fma(p, r, 1.0 / 5040.0);       // 1/7!
  p = std::fma(p, r, 1.0 / 720.0);        // 1/6!
  p = std::fma(p, r, 1.0 / 120.0);        // 1/5!
  p = std::fma(p, r, 1.0 / 24.0);         // 1/4!
  p = std::fma(p, r, 1.0 / 6.0);          // 1/3!
  p = std::fma(p, r, 0.5);                // 1/2!
  p = std::fma(p, r, 1.0);                // 1/1!
  p = std::fma(p, r, 1.0);                // 1/0!
  return std::ldexp(p, (int)kd);
}

double log_f64(double x) {
  if (!(x > 0.0)) return x == 0.0 ? -std::numeric_limits<double>::infinity()
                                  : std::numeric_limits<double>::quiet_NaN();
  if (x == std::numeric_limits<double>::infinity()) return x;
  int e;
  double m = std::frexp(x, &e);  // x = m 2^e, m in [1/2, 1)
  if (m < SQRT_HALF) {
    m = m + m;
    e = e - 1;
  }
  double f = m - 1.0;  // exact
  double hfsq = (0.5 * f) * f;
  double s = f / (2.0 + f);
  double z = s * s;
  double q = 2.0 / 21.0;
  q = std::fma(q, z, 2.0 / 19.0);
  q = std::fma(q, z, 2.0 / 17.0);
  q = std::fma(q, z, 2.0 / 15.0);
  q = std::fma(q, z, 2.0 / 13.0);
  q = std::fma(q, z, 2.0 / 11.0);
  q = std::fma(q, z, 2.0 / 9.0);
  q = std::fma(q, z, 2.0 / 7.0);
  q = std::fma(q, z, 2.0 / 5.0);
  q = std::fma(q, z, 2.0 / 3.0);
  double R = z * q;
  double ed = (double)e;
  return ed * LN2_HI - ((hfsq - (s * (hfsq + R) + ed * LN2_LO)) - f);
}

float exp_f32(float x) {
  if (x != x) return x;
  if (x > 88.72283f) return std::numeric_limits<float>::infinity();
  if (x < -103.9721f) return 0.0f;
  float kf = std::floor(x * LOG2E_F + 0.5f);
  float hi = x - kf * LN2_HI_F;  // exact
  float r = hi - kf * LN2_LO_F;
  float p = 1.0f / 5040.0f;           // 1/7!
  p = std::fma(p, r, 1.0f / 720.0f);  // 1/6!
  p = std::fma(p, r, 1.0f / 120.0f);  // 1/5!
  p = std::fma(p, r, 1.0f / 24.0f);   // 1/4!
  p = std::fma(p, r, 1.0f / 6.0f);    // 1/3!
  p = std::fma(p, r, 0.5f);
  p = std::fma(p, r, 1.0f);
  p = std::fma(p, r, 1.0f);
  return std::ldexp(p, (int)kf);
}

float log_f32(float x) {
  if (!(x > 0.0f)) return x == 0.0f ? -std::numeric_limits<float>::infinity()
                                    : std::numeric_limits<float>::quiet_NaN();
  if (x == std::numeric_limits<float>::infinity()) return x;
  int e;
  float m = std::frexp(x, &e);
  if (m < SQRT_HALF_F) {
    m = m + m;
    e = e - 1;
  }
  float f = m - 1.0f;
  float hfsq = (0.5f * f) * f;
  float s = f / (2.0f + f);
  float z = s * s;
  float q = 2.0f / 11.0f;
  q = std::fma(q, z, 2.0f / 9.0f);
  q = std::fma(q, z, 2.0f / 7.0f);
  q = std::fma(q, z, 2.0f / 5.0f);
  q = std::fma(q, z, 2.0f / 3.0f);
  float R = z * q;
  float ef = (float)e;
  return ef * LN2_HI_F - ((hfsq - (s * (hfsq + R) + ef * LN2_LO_F)) - f);
}

// log(k!) for integer k >= 0: the exact product for k <= 17 (17! < 2^53), and
// Stirling's series for log Gamma(n), n = k + 1, with four correction terms
// beyond that.
double lfact_f64(double k) {
  count_ops(k <= 17.0 ? (uint64_t)k + OPS_LOG : 16 + OPS_LOG);
  if (k <= 17.0) {
    double prod = 1.0;
    for (double i = 2.0; i <= k; i = i + 1.0) prod = prod * i;
    return log_f64(prod);
  }
  const double HALF_LOG_2PI = 0x1.d67f1c864beb5p-1;  // log(2 pi) / 2, rounded
  double n = k + 1.0;
  double rn = 1.0 / n;
  double rn2 = rn * rn;
  double corr = rn * (1.0 / 12.0 - rn2 * (1.0 / 360.0 - rn2 * (1.0 / 1260.0 - rn2 * (1.0 / 1680.0))));
  return ((k + 0.5) * log_f64(n) - n) + HALF_LOG_2PI + corr;
}

// Precision policy.  P::R is the type of propensities, tau bounds, Poisson
// means and sampler arithmetic; time, G and the implicit solve are double.
struct PolicyF64 {
  typedef double R;
  static R ulog(R x) { count_ops(OPS_LOG); return log_f64(x); }
  static R uexp(R x) { count_ops(OPS_EXP); return exp_f64(x); }
  // two uniforms from one block of four words
  static void two_uniforms(const uint32_t w[4], R* u1, R* u2) {
    count_ops(2 * OPS_UNIFORM);
    *u1 = uniform_f64(w[0], w[1]);
    *u2 = uniform_f64(w[2], w[3]);
  }
  // PTRS candidates per block of four words, and candidate s of a block
  static constexpr uint32_t TRIALS_PER_BLOCK = 1;
  static void candidate(const uint32_t w[4], uint32_t, R* u, R* v) { two_uniforms(w, u, v); }
  static double wide_from() { return std::numeric_limits<double>::infinity(); }
  static double lambda_max() { return 1073741824.0; }  // 2^30
};
struct PolicyMixed {
  typedef float R;
  static R ulog(R x) { count_ops(OPS_LOG); return log_f32(x); }
  static R uexp(R x) { count_ops(OPS_EXP); return exp_f32(x); }
  static void two_uniforms(const uint32_t w[4], R* u1, R* u2) {
    count_ops(2 * OPS_UNIFORM);
    *u1 = uniform_f32(w[0]);
    *u2 = uniform_f32(w[1]);
  }
  // one 32-bit word per uniform: a block holds two PTRS candidates
  static constexpr uint32_t TRIALS_PER_BLOCK = 2;
  static void candidate(const uint32_t w[4], uint32_t s, R* u, R* v) {
    count_ops(2 * OPS_UNIFORM);
    *u = uniform_f32(w[2 * s]);
    *v = uniform_f32(w[2 * s + 1]);
  }
  // binary32 holds every integer count exactly below 2^24; means at or above
  // 2^22 are handed to the binary64 sampler (poisson_sample), so the range
  // is binary64's
  static double wide_from() { return 4194304.0; }  // 2^22
  static double lambda_max() { return 1073741824.0; }  // 2^30
};

// log(1 + d) for d > -1 from the policy's log: u = 1 + d rounded, then
// log(u) scaled by d / (u - 1), which compensates the rounding of u
// (Goldberg 1991, "What every computer scientist should know about
// floating-point arithmetic", Theorem 4).
template <class P>
typename P::R log1p_r(typename P::R d) {
  typedef typename P::R R;
  R u = (R)1 + d;
  count_ops(1);
  if (u == (R)1) return d;
  count_ops(2);
  return P::ulog(u) * (d / (u - (R)1));
}

// phi(d) = log(1 + d) - d for d > -1.  For |d| <= 1/4 from the series
// log(1 + d) = 2 atanh(s), s = d / (2 + d): phi = -d s + 2 s^3 (1/3 + s^2/5 +
// ... + s^18/21), whose leading terms do not cancel (|s| <= 1/7, ten terms
// reach double precision); beyond that log1p_r(d) - d.
template <class P>
typename P::R log1p_minus_id(typename P::R d) {
  typedef typename P::R R;
  if (std::fabs(d) <= (R)0.25) {
    R s = d / ((R)2 + d);
    R z = s * s;
    R q = (R)(2.0 / 21.0);
    q = std::fma(q, z, (R)(2.0 / 19.0));
    q = std::fma(q, z, (R)(2.0 / 17.0));
    q = std::fma(q, z, (R)(2.0 / 15.0));
    q = std::fma(q, z, (R)(2.0 / 13.0));
    q = std::fma(q, z, (R)(2.0 / 11.0));
    q = std::fma(q, z, (R)(2.0 / 9.0));
    q = std::fma(q, z, (R)(2.0 / 7.0));
    q = std::fma(q, z, (R)(2.0 / 5.0));
    q = std::fma(q, z, (R)(2.0 / 3.0));
    count_ops(16);
    return ((s * z) * q) - d * s;
  }
  count_ops(1);
  return log1p_r<P>(d) - d;
}

// Log-density side of the PTRS acceptance test at candidate k >= 0 for mean
// lam >= 10, in the policy's precision: returns (lhs_factor, rhs) such that
// the candidate is accepted when log(q * lhs_factor) <= rhs, q being the
// ratio v / (alpha * hat(u)).  This equals
//   log q <= log p(k; lam) = k log lam - lam - log k!.
// For k <= 17, log k! is the log of the exact product (lhs_factor = k!,
// rhs = k log lam - lam).  For k > 17 log k! = log Gamma(n), n = k + 1, by
// Stirling's series with four correction terms c(n).  With d = (lam - n)/n,
// log(lam/n) = d + phi(d) and k = n - 1 this gives
//   log p = k phi(d) - d - log(2 pi)/2 - c(n) - log(n)/2,
// every term O(1) near the mode (no large terms cancel); the last term moves
// left as the factor sqrt(n).
template <class P>
void ptrs_log_density(typename P::R kf, typename P::R lam, typename P::R* lhs_factor,
                      typename P::R* rhs) {
  typedef typename P::R R;
  if (kf > (R)17) {
    R n = kf + (R)1;
    R rn = (R)1 / n;
    R rn2 = rn * rn;
    R corr = rn * ((R)(1.0 / 12.0) -
                   rn2 * ((R)(1.0 / 360.0) - rn2 * ((R)(1.0 / 1260.0) - rn2 * (R)(1.0 / 1680.0))));
    R d = (lam - n) / n;
    *rhs = (kf * log1p_minus_id<P>(d) - d) - ((R)0x1.d67f1c864beb5p-1 + corr);
    *lhs_factor = std::sqrt(n);
    count_ops(18);
  } else {
    R f = (R)1;
    for (R i = (R)2; i <= kf; i = i + (R)1) f = f * i;
    *rhs = kf * P::ulog(lam) - lam;
    *lhs_factor = f;
    count_ops(4 + (uint64_t)kf);
  }
}

// ---------------------------------------------------------------------------
// Poisson sampler (Poisson leaping, Background section).
//   lambda < lam_thr: sequential-search inversion of the CDF, one uniform;
//     the search stops where adding the next term no longer changes the
//     summed CDF (the tail is below the precision's resolution; without this
//     a uniform above the rounded CDF's ceiling would run to the cap).
//   lambda >= lam_thr: PTRS, transformed rejection with squeeze
//     (Hoermann 1993, "The transformed rejection method for generating
//     Poisson random variables"), one (U, V) candidate per trial, all in the
//     policy's precision; the final test is ptrs_log_density's.  Candidate t
//     is candidate t mod TRIALS_PER_BLOCK of Philox block t / TRIALS_PER_BLOCK.
// Returns -1 if lambda exceeds the policy's range (lane error).
// ---------------------------------------------------------------------------
template <class P>
int64_t poisson_sample(typename P::R lam, typename P::R lam_thr, int kcap, const Rng& rng,
                       uint32_t e, uint32_t site) {
  typedef typename P::R R;
  if (!(lam > (R)0)) return 0;
  if ((double)lam > P::lambda_max()) return -1;
  // reading: in binary32 a mean of 2^22 or more is drawn by the binary64
  // sampler at the same draw site (its counts near 2^24 would no longer be
  // exact integers in binary32)
  if ((double)lam >= P::wide_from())
    return poisson_sample<PolicyF64>((double)lam, (double)lam_thr, kcap, rng, e, site);
  uint32_t w[4];
  if (lam < lam_thr) {
    rng.block(e, site, 0, w);
    R u, unused;
    P::two_uniforms(w, &u, &unused);
    R p = P::uexp(-lam);
    R F = p;
    int k = 0;
    count_ops(3);
    while (u > F && k < kcap) {
      k = k + 1;
      p = (p * lam) / (R)k;
      const R Fn = F + p;
      count_ops(6);
      if (Fn == F) break;
      F = Fn;
    }
    return k;
  }
  R slam = std::sqrt(lam);
  R b = (R)0.931 + (R)2.53 * slam;
  R a = (R)-0.059 + (R)0.02483 * b;
  R inv_alpha = (R)1.1239 + (R)1.1328 / (b - (R)3.4);
  R vr = (R)0.9277 - (R)3.6224 / (b - (R)2);
  count_ops(12);
  for (uint32_t trial = 0; trial < 64; ++trial) {
    if (trial % P::TRIALS_PER_BLOCK == 0) {
      rng.block(e, site, trial / P::TRIALS_PER_BLOCK, w);
      count_ops(2);
    }
    count_ops(12);
    R u0, v;
    P::candidate(w, trial % P::TRIALS_PER_BLOCK, &u0, &v);
    R u = u0 - (R)0.5;
    R us = (R)0.5 - std::fabs(u);
    R kf = std::floor((((R)2 * a) / us + b) * u + lam + (R)0.43);
    if (kf < (R)0 || (double)kf > 1073741824.0) continue;
    if (us >= (R)0.07 && v <= vr) return (int64_t)kf;
    if (us < (R)0.013 && v > us) continue;
    R hat = a / (us * us) + b;
    R fac, rhs;
    ptrs_log_density<P>(kf, lam, &fac, &rhs);
    R lhs = P::ulog(((v * inv_alpha) * fac) / hat);
    count_ops(4);
    if (lhs <= rhs) return (int64_t)kf;
  }
  return (int64_t)std::floor((double)lam);  // not reached in practice (p < 1e-60)
}

// ---------------------------------------------------------------------------
// Network.
// ---------------------------------------------------------------------------
struct Net {
  int N = 0, M = 0;
  std::vector<int> m;   // [M][N] reactant order m_ij (indexed j*N + i)
  std::vector<int> nu;  // [M][N] net change nu_ij = p_ij - m_ij
  std::vector<int> order;
  std::vector<int> phi_case;   // per species: 0 none, 1 HOR1, 2 HOR2, 3 HOR2 needs 2,
                               //   4 HOR3, 5 HOR3 needs 2, 6 HOR3 needs 3
  std::vector<int> partner;    // reversible partner of each reaction, or -1
  int npairs = 0;
  // operation-count model (see count_ops)
  uint64_t g_cost = 0;         // evaluating all g_j from N copy numbers
  std::vector<int> nu_nnz;     // nonzero net changes per reaction
  uint64_t crit_cost = 0;      // L_j and the critical test for all j
};

// Validation; returns 0 on success.
int build_net(int N, int M, const int32_t* mtab, const int32_t* ptab, Net* net) {
  if (N <= 0 || M <= 0) return -1;
  net->N = N;
  net->M = M;
  net->m.assign((size_t)M * N, 0);
  net->nu.assign((size_t)M * N, 0);
  net->order.assign(M, 0);
  for (int j = 0; j < M; ++j) {
    int ord = 0;
    for (int i = 0; i < N; ++i) {
      int mij = mtab[j * N + i], pij = ptab[j * N + i];
      if (mij < 0 || pij < 0) return -1;
      net->m[j * N + i] = mij;
      net->nu[j * N + i] = pij - mij;
      ord += mij;
    }
    if (ord > 3) return -1;
    net->order[j] = ord;
  }
  // Highest order of reaction (Cao 2006) and how many copies of the species
  // that reaction needs; with several highest-order reactions the largest
  // multiplicity is used (reading: the most conservative bound).
  net->phi_case.assign(N, 0);
  for (int i = 0; i < N; ++i) {
    int hor = 0, mult = 0;
    for (int j = 0; j < M; ++j) {
      int mij = net->m[j * N + i];
      if (mij == 0) continue;
      if (net->order[j] > hor) {
        hor = net->order[j];
        mult = mij;
      } else if (net->order[j] == hor && mij > mult) {
        mult = mij;
      }
    }
    int c = 0;
    if (hor == 1) c = 1;
    else if (hor == 2) c = (mult >= 2) ? 3 : 2;
    else if (hor == 3) c = (mult >= 3) ? 6 : (mult == 2 ? 5 : 4);
    net->phi_case[i] = c;
  }
  // Operation-count model: C(y,1) is free, C(y,2) costs 3 and C(y,3) 5
  // operations, plus one product per factor; L_j costs two per consumed species.
  net->g_cost = (uint64_t)N;
  net->nu_nnz.assign(M, 0);
  net->crit_cost = 0;
  for (int j = 0; j < M; ++j) {
    for (int i = 0; i < N; ++i) {
      int mij = net->m[j * N + i];
      if (mij > 0) net->g_cost += 1 + (mij == 1 ? 0 : (mij == 2 ? 3 : 5));
      if (net->nu[j * N + i] != 0) net->nu_nnz[j] += 1;
      if (net->nu[j * N + i] < 0) net->crit_cost += 2;
    }
    net->crit_cost += 4;
  }
  // Reversible pairs: reactions whose net change vectors are exact negatives,
  // matched greedily in ascending reaction index (reading).
  net->partner.assign(M, -1);
  net->npairs = 0;
  for (int j = 0; j < M; ++j) {
    if (net->partner[j] >= 0) continue;
    bool nonzero = false;
    for (int i = 0; i < N; ++i) nonzero = nonzero || net->nu[j * N + i] != 0;
    if (!nonzero) continue;
    for (int k = j + 1; k < M; ++k) {
      if (net->partner[k] >= 0) continue;
      bool opposite = true;
      for (int i = 0; i < N; ++i) opposite = opposite && net->nu[k * N + i] == -net->nu[j * N + i];
      if (opposite) {
        net->partner[j] = k;
        net->partner[k] = j;
        net->npairs += 1;
        break;
      }
    }
  }
  return 0;
}

// Binomial coefficient C(y, mult) extended to real y, and its derivative.
double binom_real(double y, int mult) {
  if (mult == 1) return y;
  if (mult == 2) return (y * (y - 1.0)) * 0.5;
  return ((y * (y - 1.0)) * (y - 2.0)) / 6.0;
}
double binom_real_deriv(double y, int mult) {
  if (mult == 1) return 1.0;
  if (mult == 2) return y - 0.5;
  return ((3.0 * y - 6.0) * y + 2.0) / 6.0;
}

// g_j(y) = prod_i C(y_i, m_ij) over reactant species in ascending order
// (combinatorial mass-action convention, reading).
double g_of(const Net& net, int j, const double* y) {
  double g = 1.0;
  for (int i = 0; i < net.N; ++i) {
    int mij = net.m[j * net.N + i];
    if (mij > 0) g = g * binom_real(y[i], mij);
  }
  return g;
}
double dg_of(const Net& net, int j, int k, const double* y) {
  if (net.m[j * net.N + k] == 0) return 0.0;
  double g = 1.0;
  for (int i = 0; i < net.N; ++i) {
    int mij = net.m[j * net.N + i];
    if (mij == 0) continue;
    g = g * (i == k ? binom_real_deriv(y[i], mij) : binom_real(y[i], mij));
  }
  return g;
}

// ---------------------------------------------------------------------------
// Options, statistics and status codes.
// ---------------------------------------------------------------------------
enum { MODE_ADAPTIVE = 0, MODE_EXPLICIT = 1, MODE_SSA = 2 };
enum { ST_OK = 0, ST_STEP_BUDGET = 1, ST_LAMBDA_OVERFLOW = 2, ST_BAD_INPUT = 3, ST_COUNT_OVERFLOW = 4 };

}  // namespace

extern "C" {

// Layout shared with the Python wrapper in this directory (not with the HIP
// library, which defines its own).
typedef struct {
  double eps, delta, n_stiff, k_ssa, k_crit, lambda_thr, newton_tol, t_start;
  int64_t max_steps;
  uint64_t seed;
  int32_t n_c, n_ssa_ex, n_ssa_im, newton_maxit;
  uint32_t rng_stream, pid_base;
  int32_t accumulate, mode, precision, nthreads;
  uint32_t pid_stride;  // particle p uses id pid_base + p * pid_stride (0 means 1)
  int32_t jacobian;     // 0: analytic mass-action Jacobian, 1: forward differences,
                        // 2: the caller's derivative terms below
  // caller-supplied derivative terms (jacobian = 2): d g_j / d y_k is the sum,
  // in table order, of coef[t] * prod_i y_i^pow[t][i] over the terms t with
  // (jt_rxn[t], jt_wrt[t]) = (j, k)
  int32_t n_jt;
  const int32_t* jt_rxn;
  const int32_t* jt_wrt;
  const double* jt_coef;
  const int32_t* jt_pow;  // [n_jt][N]
} orc_options;

typedef struct {
  int32_t status;
  uint32_t crit_fired;  // accepted leaps in which a critical reaction fired
  double t_final;
  int64_t steps_ssa, steps_explicit, steps_implicit, rejections, newton_iters, newton_fail,
      kclip, attempts;
  int64_t ops;  // algorithmic operation count (see count_ops)
} orc_stats;

}  // extern "C"

namespace {

struct Ctx {
  const Net* net;
  const orc_options* o;
  double t_end;
};

// Per-step scratch and the method's quantities for one trajectory.
template <class P>
struct Traj {
  typedef typename P::R R;
  const Net& net;
  const orc_options& o;
  double t_end;
  int N, M;
  std::vector<double> theta;  // double parameters
  std::vector<R> theta_r;
  std::vector<int64_t> x, xnew;
  std::vector<int64_t> r;
  std::vector<double> G;
  std::vector<double> g, gnew, xd;
  std::vector<R> a;
  std::vector<int> crit, ncr, eq;
  std::vector<int64_t> k;
  std::vector<double> ysol;  // last converged implicit solution
  R a0 = 0, a0c = 0;
  double t = 0;
  uint32_t e = 0;
  Rng rng;
  orc_stats st;

  Traj(const Net& n, const orc_options& opt, double tend)
      : net(n), o(opt), t_end(tend), N(n.N), M(n.M) {
    theta.resize(M); theta_r.resize(M); x.resize(N); xnew.resize(N); r.resize(M);
    G.resize(M); g.resize(M); gnew.resize(M); xd.resize(N); a.resize(M);
    crit.resize(M); ncr.resize(M); eq.resize(M); k.resize(M);
    std::memset(&st, 0, sizeof(st));
  }

  void g_all(const std::vector<int64_t>& xs, std::vector<double>& out) {
    for (int i = 0; i < N; ++i) xd[i] = (double)xs[i];
    for (int j = 0; j < M; ++j) out[j] = g_of(net, j, xd.data());
  }

  // a_j = theta_j g_j (Background section), a0 = sum in ascending j.
  void propensities() {
    count_ops(net.g_cost + 2 * (uint64_t)M);
    g_all(x, g);
    a0 = 0;
    for (int j = 0; j < M; ++j) {
      a[j] = theta_r[j] * (R)g[j];
      a0 = a0 + a[j];
    }
  }

  // Critical reactions (Cao 2006): L_j = min over consumed species of
  // floor(x_i / |nu_ij|); critical if a_j > 0 and L_j < n_c.
  void critical_set() {
    count_ops(net.crit_cost);
    a0c = 0;
    for (int j = 0; j < M; ++j) {
      int64_t L = std::numeric_limits<int64_t>::max();
      for (int i = 0; i < N; ++i) {
        int v = net.nu[j * N + i];
        if (v < 0) L = std::min(L, x[i] / (int64_t)(-v));
      }
      crit[j] = (a[j] > (R)0 && L < (int64_t)o.n_c) ? 1 : 0;
      ncr[j] = (a[j] > (R)0 && !crit[j]) ? 1 : 0;
      if (crit[j]) a0c = a0c + a[j];
    }
  }

  // Cao 2006 factor g_i (here phi) of the highest-order reaction of species i.
  R phi(int i) {
    R xm1 = (R)std::max<int64_t>(x[i] - 1, 1);
    R xm2 = (R)std::max<int64_t>(x[i] - 2, 1);
    switch (net.phi_case[i]) {
      case 1: return (R)1;
      case 2: return (R)2;
      case 3: return (R)2 + (R)1 / xm1;
      case 4: return (R)3;
      case 5: return (R)1.5 * ((R)2 + (R)1 / xm1);
      case 6: return ((R)3 + (R)1 / xm1) + (R)2 / xm2;
    }
    return (R)1;
  }

  // Tau selection (Cao 2006) over the reaction set `use`: for every reactant
  // species of the network (reading: Cao's set of reactant species, whatever
  // reactions are in `use`), bound the expected change mu_i and the variance
  // sigma2_i accumulated over `use` by max(eps x_i / phi_i, 1).
  R tau_select(const std::vector<int>& use) {
    const R inf = std::numeric_limits<R>::infinity();
    R tau = inf;
    R eps = (R)o.eps;
    for (int i = 0; i < N; ++i) {
      if (net.phi_case[i] == 0) continue;  // not a reactant of any reaction
      count_ops(12);
      R mu = 0, s2 = 0;
      for (int j = 0; j < M; ++j) {
        if (!use[j]) continue;
        int v = net.nu[j * N + i];
        if (v == 0) continue;
        count_ops(4);
        mu = mu + (R)v * a[j];
        s2 = s2 + (R)(v * v) * a[j];
      }
      R bound = std::max((eps * (R)x[i]) / phi(i), (R)1);
      R t1 = (mu != (R)0) ? bound / std::fabs(mu) : inf;
      R t2 = (s2 != (R)0) ? (bound * bound) / s2 : inf;
      tau = std::min(tau, std::min(t1, t2));
    }
    return tau;
  }

  // Reversible pairs in partial equilibrium among the non-critical reactions:
  // |a_j - a_k| <= delta * min(a_j, a_k) (reading of "reaction pairs in
  // equilibrium", Implementation section).
  bool equilibrium_set() {
    bool any = false;
    R delta = (R)o.delta;
    for (int j = 0; j < M; ++j) eq[j] = 0;
    for (int j = 0; j < M; ++j) {
      int kk = net.partner[j];
      if (kk <= j) continue;
      if (!ncr[j] || !ncr[kk]) continue;
      count_ops(5);
      if (std::fabs(a[j] - a[kk]) <= delta * std::min(a[j], a[kk])) {
        eq[j] = 1;
        eq[kk] = 1;
        any = true;
      }
    }
    return any;
  }

  // One SSA step (Gillespie 1977 direct method) with exact G.  Requires
  // propensities() for the current x and a0 > 0.
  void ssa_step() {
    uint32_t w[4];
    rng.block(e, SITE_SSA, 0, w);
    e = e + 1;
    st.steps_ssa += 1;
    R u1, u2;
    P::two_uniforms(w, &u1, &u2);
    double tau_s = (double)(-P::ulog(u1) / a0);
    double rem = t_end - t;
    count_ops(4 + 2 * (uint64_t)M);
    if (tau_s >= rem) {  // the next firing is beyond t_end (reading: no firing)
      for (int j = 0; j < M; ++j) G[j] = G[j] + g[j] * rem;
      t = t_end;
      return;
    }
    R thr = u2 * a0;
    R cum = 0;
    int jf = -1, jlast = -1;
    for (int j = 0; j < M; ++j) {
      if (a[j] > (R)0) jlast = j;
      cum = cum + a[j];
      count_ops(2);
      if (cum > thr) { jf = j; break; }
    }
    if (jf < 0) jf = jlast;
    for (int j = 0; j < M; ++j) G[j] = G[j] + g[j] * tau_s;
    for (int i = 0; i < N; ++i) x[i] = x[i] + net.nu[jf * N + i];
    r[jf] = r[jf] + 1;
    t = t + tau_s;
    count_ops(3 + (uint64_t)net.nu_nnz[jf]);
  }

  // LU with partial pivoting (first maximal |pivot|) on an n x n row-major
  // matrix, solving A z = b in place; returns false on a zero pivot.
  static bool lu_solve(int n, std::vector<double>& A, std::vector<double>& b) {
    uint64_t nn = (uint64_t)n;
    count_ops((2 * nn * nn * nn) / 3 + 2 * nn * nn + nn);
    for (int c = 0; c < n; ++c) {
      int piv = c;
      double best = std::fabs(A[c * n + c]);
      for (int rr = c + 1; rr < n; ++rr) {
        double v = std::fabs(A[rr * n + c]);
        if (v > best) { best = v; piv = rr; }
      }
      if (!(best > 0.0)) return false;
      if (piv != c) {
        for (int q = 0; q < n; ++q) std::swap(A[c * n + q], A[piv * n + q]);
        std::swap(b[c], b[piv]);
      }
      for (int rr = c + 1; rr < n; ++rr) {
        double l = A[rr * n + c] / A[c * n + c];
        for (int q = c; q < n; ++q) A[rr * n + q] = A[rr * n + q] - l * A[c * n + q];
        b[rr] = b[rr] - l * b[c];
      }
    }
    for (int rr = n - 1; rr >= 0; --rr) {
      double s = b[rr];
      for (int q = rr + 1; q < n; ++q) s = s - A[rr * n + q] * b[q];
      b[rr] = s / A[rr * n + rr];
    }
    return true;
  }

  // Forward-difference estimate of d a_j / d y_k at y (the numerically
  // estimated Jacobian the paper names as the alternative to a symbolic one,
  // Background): the step h_k = 2^-26 max(|y_k|, 1) (square root of the
  // binary64 epsilon, scaled), taken as the representable difference
  // (y_k + h_k) - y_k, and a_j re-evaluated with y_k moved by it.
  double fd_dadk(int j, int kk, std::vector<double>& y, double ayj) {
    count_ops(8);
    const double yk = y[kk];
    const double step = 0x1p-26 * std::max(std::fabs(yk), 1.0);
    const double yh = yk + step;
    const double h = yh - yk;
    y[kk] = yh;
    const double ayh = theta[j] * g_of(net, j, y.data());
    y[kk] = yk;
    return (ayh - ayj) / h;
  }

  // Caller-supplied derivative d g_j / d y_k (the symbolic Jacobian the
  // paper allows in place of the numerical one, Background section): the
  // terms of (j, k) in table order, each coef * prod_i y_i^pow_i by repeated
  // products in ascending species order, summed from zero.
  double dg_user(int j, int kk, const std::vector<double>& y) const {
    double s = 0.0;
    for (int t = 0; t < o.n_jt; ++t) {
      if (o.jt_rxn[t] != j || o.jt_wrt[t] != kk) continue;
      double v = o.jt_coef[t];
      for (int i = 0; i < N; ++i)
        for (int e = 0; e < o.jt_pow[(size_t)t * N + i]; ++e) v = v * y[i];
      s = s + v;
    }
    return s;
  }

  // Implicit tau-leap (Rathinam et al. 2003): solve for real y
  //   y = x + sum_{j noncritical} nu_j (tau a_j(y) - tau a_j(x) + P_j) + nu_jc [fired]
  // by Newton with the Jacobian I - tau sum_j nu_j grad a_j(y)^T, its entries
  // analytic (mass-action derivative) or forward differences (fd_dadk).
  // On success writes k_j = max(0, round(tau a_j(y) - tau a_j(x) + P_j)).
  bool implicit_counts(double tau, const std::vector<int64_t>& Pj, int jc) {
    std::vector<double> c(N), y(N), F(N), J((size_t)N * N), ax(M), ay(M);
    for (int i = 0; i < N; ++i) xd[i] = (double)x[i];
    for (int j = 0; j < M; ++j) ax[j] = theta[j] * g_of(net, j, xd.data());
    for (int i = 0; i < N; ++i) {
      double ci = xd[i];
      for (int j = 0; j < M; ++j) {
        if (!ncr[j] || net.nu[j * N + i] == 0) continue;
        double d = (double)Pj[j] - tau * ax[j];
        ci = ci + (double)net.nu[j * N + i] * d;
      }
      if (jc >= 0 && net.nu[jc * N + i] != 0) ci = ci + (double)net.nu[jc * N + i];
      c[i] = ci;
      y[i] = xd[i];
    }
    count_ops((uint64_t)M + 3 * (uint64_t)N * M);
    bool converged = false;
    for (int it = 0; it < o.newton_maxit; ++it) {
      st.newton_iters += 1;
      // residual: g(y), products and sums
      count_ops(net.g_cost + (uint64_t)M + 5 * (uint64_t)N);
      for (int j = 0; j < M; ++j) ay[j] = ncr[j] ? theta[j] * g_of(net, j, y.data()) : 0.0;
      for (int i = 0; i < N; ++i) {
        double s = 0.0;
        for (int j = 0; j < M; ++j)
          if (ncr[j] && net.nu[j * N + i] != 0) s = s + (double)net.nu[j * N + i] * ay[j];
        F[i] = (y[i] - c[i]) - tau * s;
      }
      for (int i = 0; i < N; ++i) {
        for (int kk = 0; kk < N; ++kk) {
          double s = 0.0;
          for (int j = 0; j < M; ++j) {
            if (!ncr[j] || net.nu[j * N + i] == 0 || net.m[j * N + kk] == 0) continue;
            count_ops(5);  // one Jacobian term: derivative, product, sum
            double d;
            if (o.jacobian == 1) d = fd_dadk(j, kk, y, ay[j]);
            else if (o.jacobian == 2) d = theta[j] * dg_user(j, kk, y);
            else d = theta[j] * dg_of(net, j, kk, y.data());
            s = s + (double)net.nu[j * N + i] * d;
          }
          J[i * N + kk] = (i == kk ? 1.0 : 0.0) - tau * s;
        }
      }
      std::vector<double> rhs(N);
      for (int i = 0; i < N; ++i) rhs[i] = -F[i];
      if (!lu_solve(N, J, rhs)) break;
      double dmax = 0.0, ymax = 0.0;
      for (int i = 0; i < N; ++i) {
        y[i] = y[i] + rhs[i];
        dmax = std::max(dmax, std::fabs(rhs[i]));
        ymax = std::max(ymax, std::fabs(y[i]));
      }
      if (!(dmax == dmax)) break;
      if (dmax <= o.newton_tol * std::max(1.0, ymax)) { converged = true; break; }
    }
    if (!converged) { st.newton_fail += 1; return false; }
    ysol = y;
    count_ops(net.g_cost + 5 * (uint64_t)M);
    for (int j = 0; j < M; ++j) {
      if (!ncr[j]) { k[j] = 0; continue; }
      double v = (tau * (theta[j] * g_of(net, j, y.data())) - tau * ax[j]) + (double)Pj[j];
      double kr = std::round(v);
      if (kr < 0.0) { kr = 0.0; st.kclip += 1; }
      if (kr > 1073741824.0) kr = 1073741824.0;
      k[j] = (int64_t)kr;
    }
    return true;
  }

  // Observation times (time-grid output, reading of the paper's accuracy
  // measurement at fixed time points): with K > 0 the trajectory stops at
  // each times[k] exactly as it stops at t_end (leaps clipped without a
  // critical firing, an SSA step that would pass the time integrates g to it
  // and does not fire, an absorbing state integrates g to it), its state is
  // recorded in xg[k][N], and it goes on from there with the same random
  // stream (attempt counter) and fresh step decisions.  A time below the
  // current time, or not finite, ends the trajectory with BAD_INPUT; rows of
  // times the trajectory does not reach in status OK hold -1.  The last time
  // is the end of the simulation (t_end is not used).
  void run(uint32_t pid, const double* th, const int32_t* x0, int32_t* xo, int32_t* ro,
           double* Go, orc_stats* so, int K = 0, const double* times = nullptr,
           int32_t* xg = nullptr) {
    rng.key[0] = (uint32_t)o.seed;
    rng.key[1] = (uint32_t)(o.seed >> 32) + o.rng_stream;
    rng.pid = pid;
    g_ops = 0;
    t = o.t_start;
    e = 0;
    bool bad = false;
    for (int j = 0; j < M; ++j) {
      theta[j] = th[j];
      theta_r[j] = (R)th[j];
      if (!(th[j] >= 0.0) || th[j] == std::numeric_limits<double>::infinity()) bad = true;
      r[j] = o.accumulate ? ro[j] : 0;
      G[j] = o.accumulate ? Go[j] : 0.0;
    }
    for (int i = 0; i < N; ++i) {
      x[i] = x0[i];
      if (x0[i] < 0) bad = true;
    }
    int status = bad ? ST_BAD_INPUT : ST_OK;
    const R inf = std::numeric_limits<R>::infinity();
    const R k_ssa = (R)o.k_ssa, k_crit = (R)o.k_crit, n_stiff = (R)o.n_stiff;
    const R lam_thr = (R)o.lambda_thr;
    const int kcap = 20 + 4 * (int)std::ceil(o.lambda_thr);

    const int nseg = K > 0 ? K : 1;
    for (int kt = 0; kt < nseg; ++kt) {
      if (K > 0 && status == ST_OK) {
        if (!(times[kt] >= t) || times[kt] == std::numeric_limits<double>::infinity())
          status = ST_BAD_INPUT;
        else
          t_end = times[kt];
      }
      while (status == ST_OK && t < t_end) {
        propensities();
        if (a0 == (R)0) {  // absorbing state (reading): integrate g to t_end
          double rem = t_end - t;
          for (int j = 0; j < M; ++j) G[j] = G[j] + g[j] * rem;
          t = t_end;
          break;
        }
        if (o.mode == MODE_SSA) {
          if ((int64_t)e >= o.max_steps) { status = ST_STEP_BUDGET; break; }
          ssa_step();
          continue;
        }
        critical_set();
        R tau_ex = tau_select(ncr);
        bool implicit = false;
        R tau_p = tau_ex;
        if (o.mode == MODE_ADAPTIVE && net.npairs > 0 && equilibrium_set()) {
          std::vector<int> use(M);
          for (int j = 0; j < M; ++j) use[j] = ncr[j] && !eq[j];
          R tau_im = tau_select(use);
          if (tau_im > n_stiff * tau_ex) {  // "much greater" (Implementation section)
            implicit = true;
            tau_p = tau_im;
          }
        }
        // Leap attempts with the same propensities; tau' halves on rejection.
        for (;;) {
          count_ops(4);
          if (tau_p < k_ssa / a0 || a0c >= a0 / k_crit) {
            // SSA burst: Cao 2006 fallback when the leap is a few SSA steps,
            // and the matLeap switch when critical reactions are fast.
            int n = implicit ? o.n_ssa_im : o.n_ssa_ex;
            for (int s = 0; s < n && t < t_end; ++s) {
              if ((int64_t)e >= o.max_steps) { status = ST_STEP_BUDGET; break; }
              if (s > 0) {
                propensities();
                if (a0 == (R)0) {
                  double rem = t_end - t;
                  for (int j = 0; j < M; ++j) G[j] = G[j] + g[j] * rem;
                  t = t_end;
                  break;
                }
              }
              ssa_step();
            }
            break;
          }
          if ((int64_t)e >= o.max_steps) { status = ST_STEP_BUDGET; break; }
          const uint32_t ea = e;
          e = e + 1;
          // Critical firing: tau'' ~ Exp(a0c); one critical reaction fires if
          // it comes before the leap (Cao 2006).
          R tau_pp = inf;
          int jc = -1;
          uint32_t wc[4];
          R uc1 = 0, uc2 = 0;
          if (a0c > (R)0) {
            rng.block(ea, SITE_CRIT, 0, wc);
            P::two_uniforms(wc, &uc1, &uc2);
            tau_pp = -P::ulog(uc1) / a0c;
          }
          R tau_r;
          if (tau_p < tau_pp) {
            tau_r = tau_p;
          } else {
            tau_r = tau_pp;
            R thr = uc2 * a0c, cum = 0;
            int jlast = -1;
            for (int j = 0; j < M; ++j) {
              if (!crit[j]) continue;
              jlast = j;
              count_ops(2);
              cum = cum + a[j];
              if (cum > thr) { jc = j; break; }
            }
            if (jc < 0) jc = jlast;
          }
          double tau = (double)tau_r;
          double rem = t_end - t;
          bool last = false;
          if (tau >= rem) {  // clip at t_end; no critical firing (reading)
            tau = rem;
            jc = -1;
            last = true;
          }
          R tau_rr = (R)tau;
          count_ops(6);
          // Poisson counts of the non-critical reactions, ascending j.
          bool overflow = false;
          for (int j = 0; j < M; ++j) {
            k[j] = 0;
            if (!ncr[j]) continue;
            count_ops(1);
            int64_t kj = poisson_sample<P>(a[j] * tau_rr, lam_thr, kcap, rng, ea, (uint32_t)j);
            if (kj < 0) overflow = true;
            k[j] = kj;
          }
          if (overflow) { status = ST_LAMBDA_OVERFLOW; break; }
          bool ok = true;
          if (implicit) {
            std::vector<int64_t> Pj(k);
            ok = implicit_counts(tau, Pj, jc);
          }
          if (ok) {
            if (jc >= 0) k[jc] = 1;
            uint64_t nnz = 0;
            for (int j = 0; j < M; ++j) nnz += (uint64_t)net.nu_nnz[j];
            count_ops(2 * nnz + (uint64_t)N);
            for (int i = 0; i < N; ++i) {
              int64_t v = x[i];
              for (int j = 0; j < M; ++j) v = v + (int64_t)net.nu[j * N + i] * k[j];
              xnew[i] = v;
              if (v < 0) ok = false;
            }
          }
          if (!ok) {  // negative population or failed solve: halve tau' (Cao 2006)
            st.rejections += 1;
            tau_p = tau_p / (R)2;
            continue;
          }
          bool big = false;
          for (int i = 0; i < N; ++i) big = big || xnew[i] > 2147483647LL;
          for (int j = 0; j < M; ++j) big = big || r[j] + k[j] > 2147483647LL;
          if (big) { status = ST_COUNT_OVERFLOW; break; }
          // Accept: trapezoid rule for G over the leap, for every reaction.
          count_ops(net.g_cost + 5 * (uint64_t)M + (uint64_t)N + 2);
          g_all(xnew, gnew);
          for (int j = 0; j < M; ++j) {
            G[j] = G[j] + (tau * (g[j] + gnew[j])) * 0.5;
            r[j] = r[j] + k[j];
          }
          for (int i = 0; i < N; ++i) x[i] = xnew[i];
          t = last ? t_end : t + tau;
          if (implicit) st.steps_implicit += 1;
          else st.steps_explicit += 1;
          if (jc >= 0) st.crit_fired += 1;
          break;
        }
      }
      if (K > 0)
        for (int i = 0; i < N; ++i) xg[(size_t)kt * N + i] = status == ST_OK ? (int32_t)x[i] : -1;
    }
    for (int i = 0; i < N; ++i) xo[i] = (int32_t)x[i];
    for (int j = 0; j < M; ++j) {
      ro[j] = (int32_t)r[j];
      Go[j] = G[j];
    }
    st.status = status;
    st.t_final = t;
    st.attempts = e;
    st.ops = (int64_t)g_ops;
    if (so) *so = st;
  }
};

// ---------------------------------------------------------------------------
// Particle-filter interval step (the paper's motivating use: particle-filter
// Bayesian inference with the conjugate update Gamma(alpha + r, beta + G),
// Background section).
// ---------------------------------------------------------------------------
const uint32_t SITE_RESAMPLE = 0x40000002u;
const uint32_t SITE_GAMMA = 0x40000010u;  // + reaction index
const double HALF_LOG_2PI_ = 0x1.d67f1c864beb5p-1;

// Gamma(shape a >= 1, scale 1) by Marsaglia & Tsang (2000), with normal
// variates from the polar method.  Trial t uses block 2t for the polar pair
// and block 2t+1 for the acceptance uniform.
double gamma_ge1(double a, const Rng& rng, uint32_t e, uint32_t site) {
  const double d = a - 1.0 / 3.0;
  const double c = 1.0 / std::sqrt(9.0 * d);
  uint32_t w[4];
  for (uint32_t t = 0; t < 64; ++t) {
    rng.block(e, site, 2 * t, w);
    double U1 = uniform_f64(w[0], w[1]), U2 = uniform_f64(w[2], w[3]);
    double u1 = 2.0 * U1 - 1.0, u2 = 2.0 * U2 - 1.0;
    double s = u1 * u1 + u2 * u2;
    if (s >= 1.0) continue;
    double z = u1 * std::sqrt((-2.0 * log_f64(s)) / s);
    double t1 = 1.0 + c * z;
    if (t1 <= 0.0) continue;
    double v = (t1 * t1) * t1;
    rng.block(e, site, 2 * t + 1, w);
    double u = uniform_f64(w[0], w[1]);
    double zz = z * z;
    if (u < 1.0 - 0.0331 * (zz * zz)) return d * v;
    if (log_f64(u) < (((0.5 * zz) + d) - d * v) + d * log_f64(v)) return d * v;
  }
  return d;
}

// Gamma(shape a > 0, scale 1).  Below 1 by the boost of the same paper:
// Gamma(a) = Gamma(a + 1) U^(1/a), with U the first uniform of block 128 of
// the site (past the 128 blocks of the rounds above).  A shape that is not
// positive and finite gives NaN.
double gamma_sample(double a, const Rng& rng, uint32_t e, uint32_t site) {
  if (!(a > 0.0) || a == std::numeric_limits<double>::infinity())
    return std::numeric_limits<double>::quiet_NaN();
  if (a >= 1.0) return gamma_ge1(a, rng, e, site);
  const double y = gamma_ge1(a + 1.0, rng, e, site);
  uint32_t w[4];
  rng.block(e, site, 128, w);
  const double u = uniform_f64(w[0], w[1]);
  return y * exp_f64(log_f64(u) / a);
}

// floor(U64 * S / 2^64) for the resampling draw: an exact integer in [0, S).
uint64_t scale_u64(uint64_t r, uint64_t S) {
  return (uint64_t)(((unsigned __int128)r * (unsigned __int128)S) >> 64);
}

template <class P>
void run_range(const Net& net, const orc_options& o, double t_end, int64_t lo, int64_t hi,
               const double* theta, const int32_t* x0, int32_t* xo, int32_t* ro, double* Go,
               orc_stats* so, int K, const double* times, int32_t* xg) {
  const int N = net.N, M = net.M;
  for (int64_t p = lo; p < hi; ++p) {
    Traj<P> tr(net, o, t_end);
    const uint32_t stride = o.pid_stride ? o.pid_stride : 1;
    tr.run(o.pid_base + (uint32_t)p * stride, theta + p * M, x0 + p * N, xo + p * N, ro + p * M,
           Go + p * M, so ? so + p : nullptr, K, times, xg ? xg + (size_t)p * K * N : nullptr);
  }
}

// The Jacobian option and, for caller-supplied terms, the table: every term
// names a reaction and one of its reactant species; powers are >= 0 and
// coefficients finite.
bool jacobian_ok(const Net& net, const orc_options& o) {
  if (o.jacobian < 0 || o.jacobian > 2) return false;
  if (o.jacobian != 2) return true;
  if (o.n_jt < 1 || !o.jt_rxn || !o.jt_wrt || !o.jt_coef || !o.jt_pow) return false;
  for (int t = 0; t < o.n_jt; ++t) {
    const int j = o.jt_rxn[t], k = o.jt_wrt[t];
    if (j < 0 || j >= net.M || k < 0 || k >= net.N || net.m[(size_t)j * net.N + k] == 0)
      return false;
    if (!std::isfinite(o.jt_coef[t])) return false;
    for (int i = 0; i < net.N; ++i)
      if (o.jt_pow[(size_t)t * net.N + i] < 0 || o.jt_pow[(size_t)t * net.N + i] > 16) return false;
  }
  return true;
}

int simulate_impl(int32_t N, int32_t M, const int32_t* mtab, const int32_t* ptab, int64_t P,
                  const double* theta, const int32_t* x0, double t_end, const orc_options* opt,
                  int32_t* x_out, int32_t* r_out, double* G_out, orc_stats* stats, int K,
                  const double* times, int32_t* xg) {
  Net net;
  if (build_net(N, M, mtab, ptab, &net) != 0) return -1;
  const orc_options& o = *opt;
  if (!(o.lambda_thr >= 10.0 && o.lambda_thr <= 30.0) || o.n_c < 0 || o.mode < 0 || o.mode > 2 ||
      !(t_end >= o.t_start) || !(o.eps > 0.0) || o.precision < 0 || o.precision > 1 ||
      !jacobian_ok(net, o))
    return -2;
  int nth = o.nthreads > 0 ? o.nthreads : (int)std::max(1u, std::thread::hardware_concurrency());
  nth = (int)std::min<int64_t>(nth, std::max<int64_t>(P, 1));
  std::vector<std::thread> pool;
  int64_t chunk = (P + nth - 1) / nth;
  for (int tix = 0; tix < nth; ++tix) {
    int64_t lo = tix * chunk, hi = std::min(P, lo + chunk);
    if (lo >= hi) break;
    if (o.precision == 0)
      pool.emplace_back(run_range<PolicyF64>, std::cref(net), std::cref(o), t_end, lo, hi, theta,
                        x0, x_out, r_out, G_out, stats, K, times, xg);
    else
      pool.emplace_back(run_range<PolicyMixed>, std::cref(net), std::cref(o), t_end, lo, hi,
                        theta, x0, x_out, r_out, G_out, stats, K, times, xg);
  }
  for (auto& th : pool) th.join();
  return 0;
}

}  // namespace

extern "C" {

void orc_default_options(orc_options* o) {
  std::memset(o, 0, sizeof(*o));
  o->eps = 0.03;
  o->delta = 0.05;
  o->n_stiff = 100.0;
  o->k_ssa = 10.0;
  o->k_crit = 10.0;
  o->lambda_thr = 15.0;
  o->newton_tol = 1e-10;
  o->t_start = 0.0;
  o->max_steps = 10000000;
  o->seed = 160807058ull;
  o->n_c = 10;
  o->n_ssa_ex = 100;
  o->n_ssa_im = 10;
  o->newton_maxit = 20;
  o->mode = MODE_ADAPTIVE;
}

int orc_options_size(void) { return (int)sizeof(orc_options); }
int orc_stats_size(void) { return (int)sizeof(orc_stats); }

// Simulate P independent trajectories on the host.  theta [P][M], x0 [P][N],
// outputs x_out [P][N], r_out [P][M], G_out [P][M] (read as starting values
// when accumulate != 0), stats [P] (nullable).  Returns 0, or -1 for an
// invalid network, -2 for invalid options.
int orc_simulate(int32_t N, int32_t M, const int32_t* mtab, const int32_t* ptab, int64_t P,
                 const double* theta, const int32_t* x0, double t_end, const orc_options* opt,
                 int32_t* x_out, int32_t* r_out, double* G_out, orc_stats* stats) {
  return simulate_impl(N, M, mtab, ptab, P, theta, x0, t_end, opt, x_out, r_out, G_out, stats,
                       0, nullptr, nullptr);
}

// As orc_simulate with observation times times[0..K) (K >= 1): the state at
// each time goes to x_grid [P][K][N] (see Traj::run); the simulation ends at
// times[K-1].  Returns -3 for K < 1.
int orc_simulate_grid(int32_t N, int32_t M, const int32_t* mtab, const int32_t* ptab, int64_t P,
                      const double* theta, const int32_t* x0, int32_t K, const double* times,
                      const orc_options* opt, int32_t* x_grid, int32_t* x_out, int32_t* r_out,
                      double* G_out, orc_stats* stats) {
  if (K < 1 || !times) return -3;
  return simulate_impl(N, M, mtab, ptab, P, theta, x0, opt->t_start, opt, x_out, r_out, G_out,
                       stats, K, times, x_grid);
}

// ---- element-wise hooks on fixed inputs (for pins and bit-exact checks) ----

void orc_philox(int64_t n, const uint32_t* ctr, const uint32_t* key, uint32_t* out) {
  for (int64_t q = 0; q < n; ++q) philox4x32_10(ctr + 4 * q, key + 2 * q, out + 4 * q);
}
void orc_uniform_f64(int64_t n, const uint32_t* w, double* out) {
  for (int64_t q = 0; q < n; ++q) out[q] = uniform_f64(w[2 * q], w[2 * q + 1]);
}
void orc_uniform_f32(int64_t n, const uint32_t* w, float* out) {
  for (int64_t q = 0; q < n; ++q) out[q] = uniform_f32(w[q]);
}
void orc_exp_f64(int64_t n, const double* x, double* out) {
  for (int64_t q = 0; q < n; ++q) out[q] = exp_f64(x[q]);
}
void orc_log_f64(int64_t n, const double* x, double* out) {
  for (int64_t q = 0; q < n; ++q) out[q] = log_f64(x[q]);
}
void orc_exp_f32(int64_t n, const float* x, float* out) {
  for (int64_t q = 0; q < n; ++q) out[q] = exp_f32(x[q]);
}
void orc_log_f32(int64_t n, const float* x, float* out) {
  for (int64_t q = 0; q < n; ++q) out[q] = log_f32(x[q]);
}
void orc_lfact(int64_t n, const double* k, double* out) {
  for (int64_t q = 0; q < n; ++q) out[q] = lfact_f64(k[q]);
}

// Poisson(lam[q]) drawn at site (pid[q], e[q], site[q]); precision 0 = fp64,
// 1 = binary32 (lam rounded to float first).
void orc_poisson(int64_t n, const double* lam, const uint32_t* pid, const uint32_t* e,
                 const uint32_t* site, uint64_t seed, uint32_t stream, double lam_thr,
                 int32_t precision, int64_t* out) {
  Rng rng;
  rng.key[0] = (uint32_t)seed;
  rng.key[1] = (uint32_t)(seed >> 32) + stream;
  int kcap = 20 + 4 * (int)std::ceil(lam_thr);
  for (int64_t q = 0; q < n; ++q) {
    rng.pid = pid[q];
    if (precision == 0)
      out[q] = poisson_sample<PolicyF64>(lam[q], lam_thr, kcap, rng, e[q], site[q]);
    else
      out[q] = poisson_sample<PolicyMixed>((float)lam[q], (float)lam_thr, kcap, rng, e[q], site[q]);
  }
}

// The PTRS log-density split at (k, lam): factor f and right side r with
// log p(k; lam) = r - log f (see ptrs_log_density), in the chosen precision.
void orc_ptrs_log_density(int64_t n, const double* k, const double* lam, int32_t precision,
                          double* fac, double* rhs) {
  for (int64_t q = 0; q < n; ++q) {
    if (precision == 0) {
      double f, r;
      ptrs_log_density<PolicyF64>(k[q], lam[q], &f, &r);
      fac[q] = f;
      rhs[q] = r;
    } else {
      float f, r;
      ptrs_log_density<PolicyMixed>((float)k[q], (float)lam[q], &f, &r);
      fac[q] = f;
      rhs[q] = r;
    }
  }
}

// Exponential(1) = -log(U), U the first uniform of block (pid, e, SITE_SSA, 0).
void orc_exponential(int64_t n, const uint32_t* pid, const uint32_t* e, uint64_t seed,
                     uint32_t stream, int32_t precision, double* out) {
  Rng rng;
  rng.key[0] = (uint32_t)seed;
  rng.key[1] = (uint32_t)(seed >> 32) + stream;
  for (int64_t q = 0; q < n; ++q) {
    rng.pid = pid[q];
    uint32_t w[4];
    rng.block(e[q], SITE_SSA, 0, w);
    if (precision == 0) {
      double u1, u2;
      PolicyF64::two_uniforms(w, &u1, &u2);
      out[q] = -log_f64(u1);
    } else {
      float u1, u2;
      PolicyMixed::two_uniforms(w, &u1, &u2);
      out[q] = (double)(-log_f32(u1));
    }
  }
}

// Step-decision quantities for Q states: propensities, critical set,
// tau_ex, tau_im (infinity when no pair is in equilibrium) and the chosen
// action (0 explicit leap, 1 implicit leap, 2 SSA burst, 3 absorbing).
// theta [Q][M], x [Q][N]; outputs a [Q][M] (double), crit/eq [Q][M],
// tau [Q][2], action [Q].
int orc_tau_select(int32_t N, int32_t M, const int32_t* mtab, const int32_t* ptab, int64_t Q,
                   const double* theta, const int32_t* xs, const orc_options* opt, double* a_out,
                   int32_t* crit_out, int32_t* eq_out, double* tau_out, int32_t* action) {
  Net net;
  if (build_net(N, M, mtab, ptab, &net) != 0) return -1;
  for (int64_t q = 0; q < Q; ++q) {
    auto body = [&](auto policy_tag) {
      typedef decltype(policy_tag) P;
      typedef typename P::R R;
      Traj<P> tr(net, *opt, 1.0);
      for (int j = 0; j < M; ++j) { tr.theta[j] = theta[q * M + j]; tr.theta_r[j] = (R)theta[q * M + j]; }
      for (int i = 0; i < N; ++i) tr.x[i] = xs[q * N + i];
      tr.propensities();
      tr.critical_set();
      for (int j = 0; j < M; ++j) {
        a_out[q * M + j] = (double)tr.a[j];
        crit_out[q * M + j] = tr.crit[j];
        eq_out[q * M + j] = 0;
      }
      const R inf = std::numeric_limits<R>::infinity();
      R tau_ex = tr.tau_select(tr.ncr), tau_im = inf;
      bool implicit = false;
      if (opt->mode == MODE_ADAPTIVE && net.npairs > 0 && tr.equilibrium_set()) {
        std::vector<int> use(M);
        for (int j = 0; j < M; ++j) use[j] = tr.ncr[j] && !tr.eq[j];
        tau_im = tr.tau_select(use);
        implicit = tau_im > (R)opt->n_stiff * tau_ex;
        for (int j = 0; j < M; ++j) eq_out[q * M + j] = tr.eq[j];
      }
      tau_out[2 * q] = (double)tau_ex;
      tau_out[2 * q + 1] = (double)tau_im;
      R tau_p = implicit ? tau_im : tau_ex;
      int act;
      if (tr.a0 == (R)0) act = 3;
      else if (tau_p < (R)opt->k_ssa / tr.a0 || tr.a0c >= tr.a0 / (R)opt->k_crit) act = 2;
      else act = implicit ? 1 : 0;
      action[q] = act;
    };
    if (opt->precision == 0) body(PolicyF64());
    else body(PolicyMixed());
  }
  return 0;
}

// Implicit-leap solve for Q cases with given tau, Poisson draws P_j and
// critical firing jc (-1 for none); the non-critical set is taken as
// {j : a_j > 0} minus jc.  Outputs y [Q][N], k [Q][M], ok [Q], iters [Q].
int orc_implicit(int32_t N, int32_t M, const int32_t* mtab, const int32_t* ptab, int64_t Q,
                 const double* theta, const int32_t* xs, const double* tau, const int64_t* Pj,
                 const int32_t* jc, const orc_options* opt, double* y_out, int64_t* k_out,
                 int32_t* ok, int32_t* iters) {
  Net net;
  if (build_net(N, M, mtab, ptab, &net) != 0) return -1;
  if (!jacobian_ok(net, *opt)) return -2;
  for (int64_t q = 0; q < Q; ++q) {
    Traj<PolicyF64> tr(net, *opt, 1.0);
    for (int j = 0; j < M; ++j) { tr.theta[j] = theta[q * M + j]; tr.theta_r[j] = theta[q * M + j]; }
    for (int i = 0; i < N; ++i) tr.x[i] = xs[q * N + i];
    tr.propensities();
    for (int j = 0; j < M; ++j) tr.ncr[j] = (tr.a[j] > 0.0 && j != jc[q]) ? 1 : 0;
    std::vector<int64_t> P(Pj + q * M, Pj + (q + 1) * M);
    bool good = tr.implicit_counts(tau[q], P, jc[q]);
    ok[q] = good ? 1 : 0;
    iters[q] = (int32_t)tr.st.newton_iters;
    for (int j = 0; j < M; ++j) k_out[q * M + j] = good ? tr.k[j] : 0;
    for (int i = 0; i < N; ++i) y_out[q * N + i] = good ? tr.ysol[i] : 0.0;
  }
  return 0;
}


// Gamma(shape[q], 1) at site (pid[q], e[q], SITE_GAMMA + j[q]) -- test hook.
void orc_gamma(int64_t n, const double* shape, const uint32_t* pid, const uint32_t* e,
               const uint32_t* j, uint64_t seed, uint32_t stream, double* out) {
  Rng rng;
  rng.key[0] = (uint32_t)seed;
  rng.key[1] = (uint32_t)(seed >> 32) + stream;
  for (int64_t q = 0; q < n; ++q) {
    rng.pid = pid[q];
    out[q] = gamma_sample(shape[q], rng, e[q], SITE_GAMMA + j[q]);
  }
}

// Multinomial resampling from integer weight codes (test hook): ancestors of
// P new particles at interval k.
void orc_resample(int64_t P, const uint64_t* codes, uint64_t seed, uint32_t stream, uint32_t k,
                  int32_t* anc) {
  std::vector<uint64_t> S(P);
  uint64_t acc = 0;
  for (int64_t p = 0; p < P; ++p) { acc += codes[p]; S[p] = acc; }
  Rng rng;
  rng.key[0] = (uint32_t)seed;
  rng.key[1] = (uint32_t)(seed >> 32) + stream;
  for (int64_t q = 0; q < P; ++q) {
    rng.pid = (uint32_t)q;
    uint32_t w[4];
    rng.block(k, SITE_RESAMPLE, 0, w);
    uint64_t U = scale_u64(((uint64_t)w[0] << 32) | w[1], acc);
    anc[q] = (int32_t)(std::upper_bound(S.begin(), S.end(), U) - S.begin());
  }
}

// Particle filter over K observation intervals of length dt.  Per interval k
// (1-based): every particle is simulated from (k-1) dt to k dt with r and G
// accumulated (RNG stream k); its log-weight is the Gaussian log-density of
// observation y[k-1] of species obs_species with sd obs_sd; weights become
// integer codes floor(exp(lw - max lw) 2^40) (all 1 if every code is 0; lanes
// with a non-OK status weigh 0); P ancestors are drawn by multinomial
// resampling; the new particles take their ancestors' state and cumulative
// r, G, and draw theta_j ~ Gamma(alpha_j + r_j, rate beta_j + G_j).  loglik[k-1]
// = max lw + log(sum of codes 2^-40 / P).  theta, x, r, G are in/out.
// Algorithmic operations (count_ops) of the simulations of the last
// orc_pf_run on this thread, summed over particles and intervals.
static thread_local double g_pf_ops = 0.0;

double orc_pf_last_ops() { return g_pf_ops; }

int orc_pf_run(int32_t N, int32_t M, const int32_t* mtab, const int32_t* ptab, int64_t P,
               int32_t K, double dt, int32_t obs_species, double obs_sd, const double* y,
               const double* alpha, const double* beta, double* theta, int32_t* x, int32_t* r,
               double* G, double* loglik, const orc_options* opt) {
  Net net;
  if (build_net(N, M, mtab, ptab, &net) != 0) return -1;
  orc_options o = *opt;
  o.accumulate = 1;
  o.pid_base = 0;
  o.pid_stride = 1;
  std::vector<orc_stats> st(P);
  std::vector<double> lw(P);
  std::vector<uint64_t> code(P);
  std::vector<int32_t> anc(P);
  std::vector<int32_t> x2((size_t)P * N), r2((size_t)P * M);
  std::vector<double> G2((size_t)P * M);
  const double Lc = log_f64(obs_sd) + HALF_LOG_2PI_;
  g_pf_ops = 0.0;
  for (int k = 1; k <= K; ++k) {
    o.t_start = (double)(k - 1) * dt;
    o.rng_stream = opt->rng_stream + (uint32_t)k;
    int rc = orc_simulate(N, M, mtab, ptab, P, theta, x, (double)k * dt, &o, x, r, G, st.data());
    if (rc != 0) return rc;
    for (int64_t p = 0; p < P; ++p) g_pf_ops += (double)st[p].ops;
    double mx = -std::numeric_limits<double>::infinity();
    for (int64_t p = 0; p < P; ++p) {
      if (st[p].status != ST_OK) {
        lw[p] = -std::numeric_limits<double>::infinity();
        continue;
      }
      double dz = (y[k - 1] - (double)x[p * N + obs_species]) / obs_sd;
      lw[p] = (-0.5 * (dz * dz)) - Lc;
      mx = std::max(mx, lw[p]);
    }
    uint64_t S = 0;
    for (int64_t p = 0; p < P; ++p) {
      code[p] = (lw[p] == -std::numeric_limits<double>::infinity())
                    ? 0
                    : (uint64_t)std::floor(exp_f64(lw[p] - mx) * 0x1p40);
      S += code[p];
    }
    if (S == 0) {  // every particle weighs zero: resample uniformly
      loglik[k - 1] = -std::numeric_limits<double>::infinity();
      for (int64_t p = 0; p < P; ++p) code[p] = 1;
    } else {
      loglik[k - 1] = mx + log_f64(((double)S * 0x1p-40) / (double)P);
    }
    orc_resample(P, code.data(), o.seed, opt->rng_stream, (uint32_t)k, anc.data());
    Rng rng;
    rng.key[0] = (uint32_t)o.seed;
    rng.key[1] = (uint32_t)(o.seed >> 32) + opt->rng_stream;
    for (int64_t q = 0; q < P; ++q) {
      const int64_t a = anc[q];
      for (int i = 0; i < N; ++i) x2[q * N + i] = x[a * N + i];
      rng.pid = (uint32_t)q;
      for (int j = 0; j < M; ++j) {
        r2[q * M + j] = r[a * M + j];
        G2[q * M + j] = G[a * M + j];
        double shape = alpha[j] + (double)r2[q * M + j];
        double rate = beta[j] + G2[q * M + j];
        theta[q * M + j] = gamma_sample(shape, rng, (uint32_t)k, SITE_GAMMA + (uint32_t)j) / rate;
      }
    }
    std::copy(x2.begin(), x2.end(), x);
    std::copy(r2.begin(), r2.end(), r);
    std::copy(G2.begin(), G2.end(), G);
  }
  return 0;
}

}  // extern "C"
