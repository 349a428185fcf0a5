// lx_hooks.hip -- statically compiled test-hook kernels that run the
// production device functions of lx_device.h on fixed inputs, one thread per
// element.  Network-independent; the network-specialised hooks are compiled
// at run time with the simulation kernels (lx_sim.h).
#include <hip/hip_runtime.h>

#include "lx_device.h"

namespace lxh {

constexpr int BLOCK = 256;

__global__ void __launch_bounds__(BLOCK)
    philox_kernel(long long n, const unsigned* ctr, const unsigned* key, unsigned* out) {
  const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n) return;
  const lx::Words4 w = lx::philox(ctr[4 * q], ctr[4 * q + 1], ctr[4 * q + 2], ctr[4 * q + 3],
                                  key[2 * q], key[2 * q + 1]);
  out[4 * q] = w.w0;
  out[4 * q + 1] = w.w1;
  out[4 * q + 2] = w.w2;
  out[4 * q + 3] = w.w3;
}

__global__ void __launch_bounds__(BLOCK)
    uniform_f64_kernel(long long n, const unsigned* w, double* out) {
  const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (q < n) out[q] = lx::uniform_f64(w[2 * q], w[2 * q + 1]);
}

__global__ void __launch_bounds__(BLOCK)
    uniform_f32_kernel(long long n, const unsigned* w, float* out) {
  const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (q < n) out[q] = lx::uniform_f32(w[q]);
}

__global__ void __launch_bounds__(BLOCK)
    math_f64_kernel(int fn, long long n, const double* in, double* out) {
  const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n) return;
  const double v = in[q];
  double r;
  if (fn == 0) r = lx::exp_f64(v);
  else if (fn == 1) r = lx::log_f64(v);
  else if (fn == 2) r = lx::lfact_f64(v);
  else r = lx::F64::sqrt_(v);
  out[q] = r;
}

__global__ void __launch_bounds__(BLOCK)
    math_f32_kernel(int fn, long long n, const float* in, float* out) {
  const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n) return;
  const float v = in[q];
  float r;
  if (fn == 10) r = lx::exp_f32(v);
  else if (fn == 11) r = lx::log_f32(v);
  else r = lx::Mixed::sqrt_(v);
  out[q] = r;
}

template <class P>
__global__ void __launch_bounds__(BLOCK)
    poisson_kernel(long long n, const double* lam, const unsigned* pid, const unsigned* e,
                   const unsigned* site, lx::Key key, double lam_thr, int kcap, long long* out) {
  const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n) return;
  typedef typename P::R R;
  out[q] = lx::poisson_sample<P>((R)lam[q], (R)lam_thr, kcap, key, pid[q], e[q], site[q]);
}

template <class P>
__global__ void __launch_bounds__(BLOCK)
    exponential_kernel(long long n, const unsigned* pid, const unsigned* e, lx::Key key,
                       double* out) {
  const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n) return;
  typedef typename P::R R;
  const lx::Words4 w = lx::draw_block(key, pid[q], e[q], lx::SITE_SSA, 0);
  R u1, u2;
  P::uniforms(w, &u1, &u2);
  out[q] = (double)(-P::ulog(u1));
}

__global__ void __launch_bounds__(BLOCK)
    gamma_kernel(long long n, const double* shape, const unsigned* pid, const unsigned* e,
                 const unsigned* j, lx::Key key, double* out) {
  const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (q < n) out[q] = lx::gamma_sample(shape[q], key, pid[q], e[q], lx::SITE_GAMMA + j[q]);
}

static unsigned grid_of(long long n) { return (unsigned)((n + BLOCK - 1) / BLOCK); }

}  // namespace lxh

// Launchers used by lx_api.cpp (C++ linkage, same library).
hipError_t lxh_launch_philox(long long n, const unsigned* ctr, const unsigned* key, unsigned* out,
                             hipStream_t s) {
  hipLaunchKernelGGL(lxh::philox_kernel, dim3(lxh::grid_of(n)), dim3(lxh::BLOCK), 0, s, n, ctr,
                     key, out);
  return hipGetLastError();
}
hipError_t lxh_launch_uniform_f64(long long n, const unsigned* w, double* out, hipStream_t s) {
  hipLaunchKernelGGL(lxh::uniform_f64_kernel, dim3(lxh::grid_of(n)), dim3(lxh::BLOCK), 0, s, n, w,
                     out);
  return hipGetLastError();
}
hipError_t lxh_launch_uniform_f32(long long n, const unsigned* w, float* out, hipStream_t s) {
  hipLaunchKernelGGL(lxh::uniform_f32_kernel, dim3(lxh::grid_of(n)), dim3(lxh::BLOCK), 0, s, n, w,
                     out);
  return hipGetLastError();
}
hipError_t lxh_launch_math(int fn, long long n, const void* in, void* out, hipStream_t s) {
  if (fn < 10)
    hipLaunchKernelGGL(lxh::math_f64_kernel, dim3(lxh::grid_of(n)), dim3(lxh::BLOCK), 0, s, fn, n,
                       (const double*)in, (double*)out);
  else
    hipLaunchKernelGGL(lxh::math_f32_kernel, dim3(lxh::grid_of(n)), dim3(lxh::BLOCK), 0, s, fn, n,
                       (const float*)in, (float*)out);
  return hipGetLastError();
}
hipError_t lxh_launch_poisson(long long n, const double* lam, const unsigned* pid,
                              const unsigned* e, const unsigned* site, unsigned k0, unsigned k1,
                              double lam_thr, int kcap, int mixed, long long* out, hipStream_t s) {
  const lx::Key key{k0, k1};
  if (mixed)
    hipLaunchKernelGGL(lxh::poisson_kernel<lx::Mixed>, dim3(lxh::grid_of(n)), dim3(lxh::BLOCK), 0,
                       s, n, lam, pid, e, site, key, lam_thr, kcap, out);
  else
    hipLaunchKernelGGL(lxh::poisson_kernel<lx::F64>, dim3(lxh::grid_of(n)), dim3(lxh::BLOCK), 0,
                       s, n, lam, pid, e, site, key, lam_thr, kcap, out);
  return hipGetLastError();
}
hipError_t lxh_launch_gamma(long long n, const double* shape, const unsigned* pid,
                            const unsigned* e, const unsigned* j, unsigned k0, unsigned k1,
                            double* out, hipStream_t s) {
  const lx::Key key{k0, k1};
  hipLaunchKernelGGL(lxh::gamma_kernel, dim3(lxh::grid_of(n)), dim3(lxh::BLOCK), 0, s, n, shape,
                     pid, e, j, key, out);
  return hipGetLastError();
}
hipError_t lxh_launch_exponential(long long n, const unsigned* pid, const unsigned* e, unsigned k0,
                                  unsigned k1, int mixed, double* out, hipStream_t s) {
  const lx::Key key{k0, k1};
  if (mixed)
    hipLaunchKernelGGL(lxh::exponential_kernel<lx::Mixed>, dim3(lxh::grid_of(n)),
                       dim3(lxh::BLOCK), 0, s, n, pid, e, key, out);
  else
    hipLaunchKernelGGL(lxh::exponential_kernel<lx::F64>, dim3(lxh::grid_of(n)), dim3(lxh::BLOCK),
                       0, s, n, pid, e, key, out);
  return hipGetLastError();
}
