// lx_pf.hip -- particle-filter interval kernels (network independent).
//
// After every trajectory has been simulated over an observation interval
// (lx_simulate with accumulated r and G), one interval of the filter is:
//   1. log-weights: Gaussian log-density of the observed species, -inf for
//      lanes whose simulation failed; per-block maxima;
//   2. integer weight codes floor(exp(lw - max) 2^40) and per-block sums;
//   3. inclusive prefix sums of the codes (exact uint64 arithmetic, so the
//      result does not depend on the order of the parallel scan);
//   4. multinomial resampling: particle q draws U in [0, S) from its Philox
//      site and takes the smallest ancestor whose prefix sum exceeds U; it
//      inherits the ancestor's state and cumulative r, G and draws
//      theta_j ~ Gamma(alpha_j + r_j, rate beta_j + G_j) (the conjugate update
//      of the paper's Background section);
//   5. copy back and the interval's log-likelihood increment.
#include <hip/hip_runtime.h>

#include <mutex>

#include "lx_device.h"
#include "lx_params.h"

namespace lxpf {

constexpr int BLOCK = 256;

__device__ __forceinline__ double block_max(double v, double* sh) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int s = BLOCK / 2; s > 0; s >>= 1) {
    if (t < s) sh[t] = sh[t + s] > sh[t] ? sh[t + s] : sh[t];
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

__device__ __forceinline__ unsigned long long block_sum(unsigned long long v,
                                                        unsigned long long* sh) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int s = BLOCK / 2; s > 0; s >>= 1) {
    if (t < s) sh[t] = sh[t] + sh[t + s];
    __syncthreads();
  }
  const unsigned long long r = sh[0];
  __syncthreads();
  return r;
}

__global__ void __launch_bounds__(BLOCK)
    logw_kernel(long long P, int N, const int* __restrict__ x, int obs, const double* y, double sd,
                const lx::Stats* __restrict__ st, double* lw, double* bmax) {
  __shared__ double sh[BLOCK];
  const double Lc = lx::log_f64(sd) + 0x1.d67f1c864beb5p-1;  // log(sd) + log(2 pi)/2
  const long long p = (long long)blockIdx.x * BLOCK + threadIdx.x;
  const double ninf = -__builtin_inf();
  double v = ninf;
  if (p < P && st[p].status == lx::LANE_OK) {
    const double dz = (y[0] - (double)x[p * N + obs]) / sd;
    v = (-0.5 * (dz * dz)) - Lc;
  }
  if (p < P) lw[p] = v;
  const double m = block_max(v, sh);
  if (threadIdx.x == 0) bmax[blockIdx.x] = m;
}

__global__ void __launch_bounds__(BLOCK)
    codes_kernel(long long P, const double* __restrict__ lw, const double* __restrict__ bmax,
                 int nb, unsigned long long* codes, unsigned long long* bsum, double* mx_out) {
  __shared__ double shd[BLOCK];
  __shared__ unsigned long long shu[BLOCK];
  double m = -__builtin_inf();
  for (int b = threadIdx.x; b < nb; b += BLOCK) m = bmax[b] > m ? bmax[b] : m;
  m = block_max(m, shd);
  const long long p = (long long)blockIdx.x * BLOCK + threadIdx.x;
  unsigned long long c = 0;
  if (p < P) {
    const double v = lw[p];
    if (v != -__builtin_inf())
      c = (unsigned long long)__builtin_floor(lx::exp_f64(v - m) * 0x1p40);
    codes[p] = c;
  }
  const unsigned long long s = block_sum(c, shu);
  if (threadIdx.x == 0) {
    bsum[blockIdx.x] = s;
    if (blockIdx.x == 0) *mx_out = m;
  }
}

__global__ void __launch_bounds__(BLOCK)
    scan_kernel(long long P, const unsigned long long* __restrict__ codes,
                const unsigned long long* __restrict__ bsum, int nb, unsigned long long* scan,
                unsigned long long* total_out) {
  __shared__ unsigned long long sh[BLOCK];
  unsigned long long off = 0, tot = 0;
  for (int b = threadIdx.x; b < nb; b += BLOCK) {
    if (b < (int)blockIdx.x) off += bsum[b];
    tot += bsum[b];
  }
  off = block_sum(off, sh);
  tot = block_sum(tot, sh);
  const long long p = (long long)blockIdx.x * BLOCK + threadIdx.x;
  unsigned long long v = p < P ? codes[p] : 0ull;
  // inclusive scan within the block (Hillis-Steele, exact integers)
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int s = 1; s < BLOCK; s <<= 1) {
    const unsigned long long add = threadIdx.x >= s ? sh[threadIdx.x - s] : 0ull;
    __syncthreads();
    sh[threadIdx.x] += add;
    __syncthreads();
  }
  if (p < P) scan[p] = sh[threadIdx.x] + off;
  if (blockIdx.x == 0 && threadIdx.x == 0) *total_out = tot;
}

// Multinomial resampling: particle q draws its ancestor a(q), the smallest
// a with scan[a] > U, U uniform on the integers below the total; then the
// block's particles take their ancestors' state and cumulative r, G, and
// draw theta_j ~ Gamma(alpha_j + r_j, rate beta_j + G_j).  The rows of the
// block's particles are written together, consecutive threads writing
// consecutive words.
__global__ void __launch_bounds__(BLOCK)
    resample_kernel(long long P, int N, int M, const unsigned long long* __restrict__ scan,
                    const unsigned long long* __restrict__ total_in, lx::Key key, unsigned k,
                    const int* __restrict__ x, const int* __restrict__ r,
                    const double* __restrict__ G, int* x2, int* r2, double* G2, double* theta,
                    const double* __restrict__ alpha, const double* __restrict__ beta) {
  __shared__ long long anc[BLOCK];
  const long long q0 = (long long)blockIdx.x * BLOCK;
  const long long q = q0 + threadIdx.x;
  if (q < P) {
    const unsigned long long S = *total_in;
    const lx::Words4 w = lx::draw_block(key, (unsigned)q, k, lx::SITE_RESAMPLE, 0);
    const unsigned long long r64 = ((unsigned long long)w.w0 << 32) | (unsigned long long)w.w1;
    long long a;
    if (S == 0) {  // every particle weighs zero: uniform resampling
      a = (long long)__umul64hi(r64, (unsigned long long)P);
    } else {
      const unsigned long long U = __umul64hi(r64, S);
      long long lo = 0, hi = P - 1;  // smallest a with scan[a] > U
      while (lo < hi) {
        const long long mid = (lo + hi) >> 1;
        if (scan[mid] > U) hi = mid;
        else lo = mid + 1;
      }
      a = lo;
    }
    anc[threadIdx.x] = a;
  }
  __syncthreads();
  const long long rest = P - q0;
  const int nq = rest < BLOCK ? (int)rest : BLOCK;
  for (int e = threadIdx.x; e < nq * N; e += BLOCK) {
    const int qq = e / N, i = e - qq * N;
    x2[(q0 + qq) * N + i] = x[anc[qq] * N + i];
  }
  for (int e = threadIdx.x; e < nq * M; e += BLOCK) {
    const int qq = e / M, j = e - qq * M;
    const long long a = anc[qq];
    const int rj = r[a * M + j];
    const double Gj = G[a * M + j];
    const long long o = (q0 + qq) * M + j;
    r2[o] = rj;
    G2[o] = Gj;
    const double shape = alpha[j] + (double)rj;
    const double rate = beta[j] + Gj;
    theta[o] = lx::gamma_sample(shape, key, (unsigned)(q0 + qq), k, lx::SITE_GAMMA + (unsigned)j) / rate;
  }
}

// The resampled state back into the caller's arrays (flat copies), and the
// interval's log-likelihood.
__global__ void __launch_bounds__(BLOCK)
    copyback_kernel(long long P, int N, int M, const int* __restrict__ x2,
                    const int* __restrict__ r2, const double* __restrict__ G2, int* x, int* r,
                    double* G, const double* mx, const unsigned long long* total, double* ll) {
  const long long t = (long long)blockIdx.x * BLOCK + threadIdx.x;
  const long long stride = (long long)gridDim.x * BLOCK;
  for (long long e = t; e < P * N; e += stride) x[e] = x2[e];
  for (long long e = t; e < P * M; e += stride) {
    r[e] = r2[e];
    G[e] = G2[e];
  }
  if (t == 0) {
    const unsigned long long S = *total;
    ll[0] = S == 0 ? -__builtin_inf()
                   : *mx + lx::log_f64(((double)S * 0x1p-40) / (double)P);
  }
}

}  // namespace lxpf

// Workspace layout (256-byte aligned pieces).
static size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

size_t lxpf_workspace_layout(long long P, int N, int M, char* base, lx::PfWork* w) {
  const long long nb = (P + lxpf::BLOCK - 1) / lxpf::BLOCK;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    char* p = base ? base + off : nullptr;
    off += align256(bytes);
    return p;
  };
  lx::PfWork t;
  t.x2 = (int*)take((size_t)P * N * 4);
  t.r2 = (int*)take((size_t)P * M * 4);
  t.G2 = (double*)take((size_t)P * M * 8);
  t.lw = (double*)take((size_t)P * 8);
  t.codes = (unsigned long long*)take((size_t)P * 8);
  t.scan = (unsigned long long*)take((size_t)P * 8);
  t.stats = (lx::Stats*)take((size_t)P * sizeof(lx::Stats));
  t.bmax = (double*)take((size_t)nb * 8);
  t.bsum = (unsigned long long*)take((size_t)nb * 8);
  t.mx = (double*)take(8);
  t.total = (unsigned long long*)take(8);
  if (w) *w = t;
  return off;
}

// Enqueue steps 1-5 of interval k (1-based) on stream s.
hipError_t lxpf_launch_interval(long long P, int N, int M, int* x, int* r, double* G,
                                double* theta, const double* y_k, int obs, double sd,
                                const double* alpha, const double* beta, unsigned k0,
                                unsigned k1, unsigned k, double* ll_k, const lx::PfWork& w,
                                hipStream_t s) {
  const unsigned nb = (unsigned)((P + lxpf::BLOCK - 1) / lxpf::BLOCK);
  const dim3 g(nb), b(lxpf::BLOCK);
  hipLaunchKernelGGL(lxpf::logw_kernel, g, b, 0, s, P, N, x, obs, y_k, sd, w.stats, w.lw,
                     w.bmax);
  hipLaunchKernelGGL(lxpf::codes_kernel, g, b, 0, s, P, w.lw, w.bmax, (int)nb, w.codes, w.bsum,
                     w.mx);
  hipLaunchKernelGGL(lxpf::scan_kernel, g, b, 0, s, P, w.codes, w.bsum, (int)nb, w.scan, w.total);
  const lx::Key key{k0, k1};
  hipLaunchKernelGGL(lxpf::resample_kernel, g, b, 0, s, P, N, M, w.scan, w.total, key, k, x, r, G,
                     w.x2, w.r2, w.G2, theta, alpha, beta);
  hipLaunchKernelGGL(lxpf::copyback_kernel, g, b, 0, s, P, N, M, w.x2, w.r2, w.G2, x, r, G, w.mx,
                     w.total, ll_k);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Scratch of lx_pf_run_static, the filter entry point for callers that cannot
// allocate device memory: a file-scope device array that each GPU holds for
// the life of the process.  Host code never passes `scratch` itself (on the
// host the name is only a stand-in): it passes the device address looked up
// here once per device, with that device current.  Every piece of the
// workspace carved from it is written before it is read within each
// interval, so nothing needs clearing; calls that overlap on one GPU share
// the array and race.
// ---------------------------------------------------------------------------
constexpr size_t LXPF_STATIC_BYTES = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[LXPF_STATIC_BYTES];

constexpr int LXPF_MAX_DEVICES = 64;

hipError_t lxpf_static_scratch(void** ptr, size_t* bytes) {
  static std::mutex mu;
  static void* addr[LXPF_MAX_DEVICES] = {};
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= LXPF_MAX_DEVICES) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[dev]) {
    void* a = nullptr;
    e = hipGetSymbolAddress(&a, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    addr[dev] = a;
  }
  *ptr = addr[dev];
  *bytes = LXPF_STATIC_BYTES;
  return hipSuccess;
}
