// lx_api.cpp -- host side of liblx: the C ABI of include/lx.h.
//
//  * network compiler: validates the flat stoichiometry table and derives the
//    tables the kernels need (net changes, tau-bound factor cases, reversible
//    pairs);
//  * code generator: emits the network as compile-time constants in front of
//    the kernel source (lx_device.h, lx_params.h, lx_sim.h, embedded at build
//    time) and compiles it for gfx950 with hipRTC; code objects are cached in
//    memory per (network, variant, device) and on disk by content hash;
//  * launcher: validates arguments and enqueues the kernels on the caller's
//    stream.
#include <hip/hip_runtime.h>
#include <hip/hiprtc.h>

#include <dlfcn.h>
#include <sys/stat.h>
#include <unistd.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "lx.h"
#include "lx_embedded.inc"  // lx_src_params, lx_src_device, lx_src_sim, lx_src_sim_large, lx_src_sim_wave (generated)
#include "lx_params.h"

static_assert(sizeof(lx_stats) == sizeof(lx::Stats), "lx_stats layout");
static_assert(sizeof(lx_stats) == 80, "lx_stats size");
static_assert(sizeof(lx_options) == 160, "lx_options size");

// Launchers of the static hook kernels (lx_hooks.hip).
hipError_t lxh_launch_philox(long long, const unsigned*, const unsigned*, unsigned*, hipStream_t);
hipError_t lxh_launch_uniform_f64(long long, const unsigned*, double*, hipStream_t);
hipError_t lxh_launch_uniform_f32(long long, const unsigned*, float*, hipStream_t);
hipError_t lxh_launch_math(int, long long, const void*, void*, hipStream_t);
hipError_t lxh_launch_poisson(long long, const double*, const unsigned*, const unsigned*,
                              const unsigned*, unsigned, unsigned, double, int, int, long long*,
                              hipStream_t);
hipError_t lxh_launch_exponential(long long, const unsigned*, const unsigned*, unsigned, unsigned,
                                  int, double*, hipStream_t);
hipError_t lxh_launch_gamma(long long, const double*, const unsigned*, const unsigned*,
                            const unsigned*, unsigned, unsigned, double*, hipStream_t);

// Particle-filter kernels (lx_pf.hip).
size_t lxpf_workspace_layout(long long P, int N, int M, char* base, lx::PfWork* w);
hipError_t lxpf_static_scratch(void** ptr, size_t* bytes);
hipError_t lxpf_launch_interval(long long P, int N, int M, int* x, int* r, double* G,
                                double* theta, const double* y_k, int obs, double sd,
                                const double* alpha, const double* beta, unsigned k0,
                                unsigned k1, unsigned k, double* ll_k, const lx::PfWork& w,
                                hipStream_t s);

namespace {

thread_local std::string g_err;

lx_status fail(lx_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

lx_status hip_fail(hipError_t e, const char* what) {
  return fail(LX_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

const int MAX_M = 256;  // networks up to 64 x 256 (large-network kernels beyond 16 x 32)
const int MAX_N = 64;
// Register budget of the one-trajectory-per-wave kernel when the caller
// leaves waves_per_simd at 0: as many waves per SIMD as its LDS allows, at
// most four (at most 128 registers); the compiler's own choice (about 200
// registers, two waves) runs 1.5x slower on the random 48 x 128 ensemble.
const int WAVE_KERNEL_WAVES = 4;
const int REG_M = 32;  // register-resident kernels
const int REG_N = 16;
// The register-resident lane state needs well over 128 VGPRs; blocks of more
// than four waves per SIMD would force spills (and were refused at dispatch),
// so blocks are limited to 256 threads.
const int MAX_BLOCK = 256;

// ---------------------------------------------------------------------------
// Kernel compilation and caching.
// ---------------------------------------------------------------------------
std::mutex g_rtc_mutex;

uint64_t fnv1a(const std::string& s) {
  uint64_t h = 1469598103934665603ull;
  for (unsigned char c : s) {
    h ^= c;
    h *= 1099511628211ull;
  }
  return h;
}

std::string cache_dir() {
  const char* env = getenv("LX_KERNEL_CACHE");
  if (env && *env) return env;
  Dl_info info;
  if (dladdr((void*)&fnv1a, &info) && info.dli_fname) {
    std::string p(info.dli_fname);
    size_t slash = p.find_last_of('/');
    if (slash != std::string::npos) return p.substr(0, slash) + "/kcache";
  }
  return "";
}

const char* const RTC_OPTS[] = {"--offload-arch=gfx950",
                                "-O3",
                                "-std=c++17",
                                "-ffp-contract=off",
                                "-fhip-fp32-correctly-rounded-divide-sqrt",
                                "-fno-gpu-flush-denormals-to-zero",
                                "-Xclang",
                                "-target-feature",
                                "-Xclang",
                                "-packed-fp32-ops"};

lx_status compile_source(const std::string& src, std::vector<char>* code) {
  std::string key = src;
  for (const char* o : RTC_OPTS) key += std::string("\n//opt ") + o;
  char name[32];
  snprintf(name, sizeof(name), "%016llx.co", (unsigned long long)fnv1a(key));
  const std::string dir = cache_dir();
  if (!dir.empty()) {
    std::ifstream f(dir + "/" + name, std::ios::binary);
    if (f) {
      std::vector<char> buf((std::istreambuf_iterator<char>(f)), std::istreambuf_iterator<char>());
      if (!buf.empty()) {
        *code = std::move(buf);
        return LX_OK;
      }
    }
  }
  std::lock_guard<std::mutex> lock(g_rtc_mutex);
  hiprtcProgram prog;
  if (hiprtcCreateProgram(&prog, src.c_str(), "lx_sim.hip", 0, nullptr, nullptr) != HIPRTC_SUCCESS)
    return fail(LX_E_COMPILE, "hiprtcCreateProgram failed");
  const int nopt = (int)(sizeof(RTC_OPTS) / sizeof(RTC_OPTS[0]));
  hiprtcResult rc = hiprtcCompileProgram(prog, nopt, const_cast<const char**>(RTC_OPTS));
  if (rc != HIPRTC_SUCCESS) {
    size_t ls = 0;
    hiprtcGetProgramLogSize(prog, &ls);
    std::string log(ls + 1, '\0');
    hiprtcGetProgramLog(prog, &log[0]);
    hiprtcDestroyProgram(&prog);
    return fail(LX_E_COMPILE, "kernel compilation failed: " + log.substr(0, 4000));
  }
  size_t cs = 0;
  hiprtcGetCodeSize(prog, &cs);
  code->assign(cs, 0);
  hiprtcGetCode(prog, code->data());
  hiprtcDestroyProgram(&prog);
  if (!dir.empty()) {
    mkdir(dir.c_str(), 0755);
    std::string tmp = dir + "/" + name + ".tmp" + std::to_string((long long)getpid());
    std::ofstream f(tmp, std::ios::binary);
    if (f) {
      f.write(code->data(), (std::streamsize)code->size());
      f.close();
      rename(tmp.c_str(), (dir + "/" + name).c_str());
    }
  }
  return LX_OK;
}

struct Kernel {
  hipModule_t mod = nullptr;
  hipFunction_t fn = nullptr;
};

}  // namespace

// ---------------------------------------------------------------------------
// Network handle.
// ---------------------------------------------------------------------------
struct lx_network_s {
  int N = 0, M = 0, npairs = 0;
  bool large = false;  // beyond the register-resident limits: lx_sim_large.h kernels
  std::vector<int> ro, nu, phi, partner;
  // caller-supplied derivative terms (lx_network_create_jac), in table order
  std::vector<int> jt_rxn, jt_wrt, jt_pow;  // jt_pow [n][N]
  std::vector<double> jt_coef;
  std::string netsrc;
  std::mutex mu;
  std::map<std::string, Kernel> kernels;  // variant key -> loaded kernel

  ~lx_network_s() {
    for (auto& kv : kernels)
      if (kv.second.mod) (void)hipModuleUnload(kv.second.mod);
  }
};

namespace {

std::string table_src(const char* name, const std::vector<int>& v, int rows, int cols) {
  std::ostringstream s;
  s << "  static constexpr int " << name << "[" << rows << "][" << cols << "] = {";
  for (int r = 0; r < rows; ++r) {
    s << (r ? ",{" : "{");
    for (int c = 0; c < cols; ++c) s << (c ? "," : "") << v[(size_t)r * cols + c];
    s << "}";
  }
  s << "};\n";
  return s.str();
}

std::string vec_src(const char* name, const std::vector<int>& v) {
  std::ostringstream s;
  s << "  static constexpr int " << name << "[" << v.size() << "] = {";
  for (size_t q = 0; q < v.size(); ++q) s << (q ? "," : "") << v[q];
  s << "};\n";
  return s.str();
}

std::string dvec_src(const char* name, const std::vector<double>& v) {
  std::ostringstream s;
  s << "  static constexpr double " << name << "[" << v.size() << "] = {";
  for (size_t q = 0; q < v.size(); ++q) {
    char buf[40];
    snprintf(buf, sizeof(buf), "%a", v[q]);
    s << (q ? "," : "") << buf;
  }
  s << "};\n";
  return s.str();
}

// Caller-supplied derivative terms of d g_j / d y_k as compile-time tables:
// term t has reaction JT_J[t], species JT_K[t], coefficient JT_C[t] and the
// factors y_{JT_SP[f]}^{JT_PW[f]}, f in [JT_PTR[t], JT_PTR[t+1]), in
// ascending species order; JT_SLOT_PTR / JT_SLOT_T list, for every reactant
// slot q of RX_PTR order (reaction j, its q-th reactant species), the terms
// of that (j, k) in table order.  Empty tables hold one unused entry.
std::string jacobian_src(const lx_network_s& n) {
  const int T = (int)n.jt_rxn.size();
  std::vector<int> J(n.jt_rxn), K(n.jt_wrt), ptr(1, 0), sp, pw;
  std::vector<double> C(n.jt_coef);
  for (int t = 0; t < T; ++t) {
    for (int i = 0; i < n.N; ++i) {
      const int e = n.jt_pow[(size_t)t * n.N + i];
      if (e) {
        sp.push_back(i);
        pw.push_back(e);
      }
    }
    ptr.push_back((int)sp.size());
  }
  std::vector<int> slot_ptr(1, 0), slot_t;
  for (int j = 0; j < n.M; ++j)
    for (int i = 0; i < n.N; ++i) {
      if (n.ro[(size_t)j * n.N + i] == 0) continue;
      for (int t = 0; t < T; ++t)
        if (J[t] == j && K[t] == i) slot_t.push_back(t);
      slot_ptr.push_back((int)slot_t.size());
    }
  if (T == 0) {
    J.assign(1, -1);
    K.assign(1, -1);
    C.assign(1, 0.0);
  }
  if (sp.empty()) {
    sp.push_back(0);
    pw.push_back(0);
  }
  if (slot_t.empty()) slot_t.push_back(0);
  std::ostringstream s;
  s << "  static constexpr int NJT = " << T << ";\n";
  s << vec_src("JT_J", J) << vec_src("JT_K", K) << dvec_src("JT_C", C) << vec_src("JT_PTR", ptr)
    << vec_src("JT_SP", sp) << vec_src("JT_PW", pw) << vec_src("JT_SLOT_PTR", slot_ptr)
    << vec_src("JT_SLOT_T", slot_t);
  return s.str();
}

// Compressed rows of an M x N (or transposed) table: for each row the
// columns with a nonzero entry, ascending, and their values.
void csr_src(std::ostringstream& s, const char* ptr, const char* idx, const char* val,
             const std::vector<int>& t, int rows, int cols, bool transpose, bool reactants) {
  std::vector<int> p(1, 0), ix, vv;
  for (int r = 0; r < rows; ++r) {
    for (int c = 0; c < cols; ++c) {
      const size_t at = transpose ? (size_t)c * rows + r : (size_t)r * cols + c;
      const int v = t[at];
      if (v == 0 || (reactants && v < 0)) continue;
      ix.push_back(c);
      vv.push_back(v);
    }
    p.push_back((int)ix.size());
  }
  if (ix.empty()) {  // keep arrays non-empty
    ix.push_back(0);
    vv.push_back(0);
  }
  s << vec_src(ptr, p) << vec_src(idx, ix) << vec_src(val, vv);
}

// Compile-time description of the network for the kernel source: a traits
// struct named LxNet<k> (the "@" placeholder is replaced by k).  Small
// networks carry dense tables (unrolled kernels); large ones compressed rows.
std::string network_source(const lx_network_s& n) {
  std::ostringstream s;
  s << "struct LxNet@ {\n";
  if (n.large) {
    s << "  static constexpr int LARGE = 1;\n";
    s << "  static constexpr int N = " << n.N << ";\n  static constexpr int M = " << n.M << ";\n";
    s << "  static constexpr int NPAIRS = " << n.npairs << ";\n";
    csr_src(s, "RX_PTR", "RX_SP", "RX_RO", n.ro, n.M, n.N, false, true);
    {  // reaction of every reactant slot (the RX_SP order)
      std::vector<int> rj;
      for (int j = 0; j < n.M; ++j)
        for (int i = 0; i < n.N; ++i)
          if (n.ro[(size_t)j * n.N + i] > 0) rj.push_back(j);
      if (rj.empty()) rj.push_back(0);
      s << "  static constexpr int NSLOT = " << (int)rj.size() << ";\n" << vec_src("RX_J", rj);
    }
    csr_src(s, "NJ_PTR", "NJ_SP", "NJ_V", n.nu, n.M, n.N, false, false);
    csr_src(s, "NI_PTR", "NI_RX", "NI_V", n.nu, n.N, n.M, true, false);
    s << vec_src("PHI", n.phi);
    s << vec_src("PARTNER", n.partner);
    s << jacobian_src(n);
    s << "};\n";
    return s.str();
  }
  s << "  static constexpr int N = " << n.N << ";\n  static constexpr int M = " << n.M << ";\n";
  s << "  static constexpr int NPAIRS = " << n.npairs << ";\n";
  s << table_src("RO", n.ro, n.M, n.N);
  s << table_src("NU", n.nu, n.M, n.N);
  s << vec_src("PHI", n.phi);
  s << vec_src("PARTNER", n.partner);
  s << jacobian_src(n);
  s << "};\n";
  return s.str();
}

std::string named_net(const lx_network_s& n, int k) {
  std::string src = n.netsrc;
  const size_t at = src.find('@');
  return src.replace(at, 1, std::to_string(k));
}

// The method constants of a launch as compile-time values (see LXP in
// lx_params.h): one kernel per set of values; doubles in hexadecimal so the
// constants are the exact binary64 values of the options.
std::string const_source(const lx::SimParams& p) {
  char waves[40] = "";
  if (p.waves) snprintf(waves, sizeof(waves), "#define LX_WAVES %d\n", p.waves);
  char buf[1024];
  snprintf(buf, sizeof(buf),
           "%s%s#define LX_CONST 1\n"
           "struct LxConst {\n"
           "  static constexpr double eps = %a, delta = %a, n_stiff = %a, k_ssa = %a, k_crit = %a,\n"
           "      lam_thr = %a, newton_tol = %a;\n"
           "  static constexpr long long max_steps = %lldLL;\n"
           "  static constexpr int n_c = %d, n_ssa_ex = %d, n_ssa_im = %d, newton_maxit = %d,\n"
           "      kcap = %d, mode = %d, accumulate = %d, ssa_k = %d, regroup = %d, jacobian = %d,\n"
           "      tail = %d;\n"
           "};\n",
           p.cycles ? "#define LX_TIMERS 1\n" : "", waves, p.eps, p.delta, p.n_stiff, p.k_ssa, p.k_crit,
           p.lam_thr, p.newton_tol, p.max_steps,
           p.n_c, p.n_ssa_ex, p.n_ssa_im, p.newton_maxit, p.kcap, p.mode, p.accumulate, p.ssa_k,
           p.regroup, p.jacobian, p.tail);
  return buf;
}

// Full hipRTC source of one kernel variant of a network; `consts` is
// const_source() of the launch, or empty for run-time constants (hooks).
std::string kernel_source(const lx_network_s& net, const char* variant, int precision, int block,
                          int tpl, const std::string& consts, bool grid = false) {
  std::ostringstream src;
  src << "// generated by liblx\n";
  if (grid) src << "#define LX_GRID 1\n";
  src << "#define LX_TPL " << tpl << "\n";
  src << "#define LX_POLICY " << (precision == LX_PREC_MIXED ? "lx::Mixed" : "lx::F64") << "\n";
  src << "#define LX_BLOCK " << block << "\n";
  if (strcmp(variant, "hooks") == 0) src << "#define LX_HOOKS 1\n";
  if (strcmp(variant, "batched") == 0) src << "#define LX_BATCHED 1\n";
  const bool wave = strcmp(variant, "wave") == 0;
  if (wave) src << "#define LX_WAVE 1\n";
  if (net.large) src << "#define LX_LARGE 1\n";
  src << consts << lx_src_params << "\n" << lx_src_device << "\n" << named_net(net, 0)
      << "typedef LxNet0 LxNet;\n" << lx_src_sim;
  if (net.large) src << "\n" << lx_src_sim_large;
  if (net.large && wave) src << "\n" << lx_src_sim_wave;
  return src.str();
}

// hipRTC source of the multi-network kernel: every network of the set as
// LxNet<k>.  Every block owns a slice of every network and runs the
// networks one after another (each wave moves on as soon as its lanes have
// drained the block's slice), so that all blocks carry the same mix of work
// whatever the networks' costs.
std::string set_source(const std::vector<const lx_network_s*>& nets, int precision, int block,
                       int tpl, const std::string& consts) {
  std::ostringstream src;
  src << "// generated by liblx (network set)\n" << consts;
  src << "#define LX_TPL " << tpl << "\n";
  src << "#define LX_POLICY " << (precision == LX_PREC_MIXED ? "lx::Mixed" : "lx::F64") << "\n";
  src << "#define LX_BLOCK " << block << "\n#define LX_SET 1\n";
  src << lx_src_params << "\n" << lx_src_device << "\n";
  for (size_t k = 0; k < nets.size(); ++k) src << named_net(*nets[k], (int)k);
  src << "typedef LxNet0 LxNet;\n" << lx_src_sim << "\n";
  src << "extern \"C\" __global__ void __launch_bounds__(LX_BLOCK) LX_WAVES_ATTR\n"
         "    lx_sim_set(lx::SetArgs a, lx::SimParams prm) {\n"
         "  __shared__ unsigned long long next[" << nets.size() << "];\n"
         "  const long long blk = blockIdx.x;\n"
         "  const long long waves = blockDim.x >> 6;\n"
         "  if (threadIdx.x == 0) {\n";
  for (size_t k = 0; k < nets.size(); ++k)
    src << "    next[" << k << "] = (unsigned long long)(blk * a.it[" << k << "].per_block + waves * a.it["
        << k << "].lanes);\n";
  src << "  }\n  __syncthreads();\n";
  for (size_t k = 0; k < nets.size(); ++k)
    src << "  {\n    const lx::SetItem& it = a.it[" << k << "];\n"
        << "    lx::SimParams q = prm;\n"
        << "    q.P = it.P;\n    q.per_block = it.per_block;\n    q.lanes = it.lanes;\n"
        << "    q.pid_base = it.pid_base;\n    q.pid_stride = it.pid_stride;\n"
        << "    if (blk * it.per_block < it.P)\n"
        << "      lx::run_sched<LxNet" << k
        << ">(blk, it.theta, it.x0, it.x_out, it.r_out, it.G_out, it.stats, q, &next[" << k
        << "], true);\n  }\n";
  src << "}\n";
  return src.str();
}

lx_status check_device(int* dev_out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  hipDeviceProp_t prop;
  e = hipGetDeviceProperties(&prop, dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDeviceProperties");
  if (strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return fail(LX_E_UNSUPPORTED, std::string("liblx targets gfx950; device is ") + prop.gcnArchName);
  *dev_out = dev;
  return LX_OK;
}

// Fetch (compiling and loading on first use) a kernel for the current device
// from the cache of network `owner`; `make_src` produces its source.
template <class F>
lx_status get_kernel_src(lx_network_s* owner, const std::string& variant_key, F make_src,
                         const char* fname, hipFunction_t* fn, bool may_load = true) {
  int dev = 0;
  lx_status st = check_device(&dev);
  if (st != LX_OK) return st;
  std::ostringstream key;
  key << variant_key << "/" << fname << "/dev" << dev;
  std::lock_guard<std::mutex> lock(owner->mu);
  auto it = owner->kernels.find(key.str());
  if (it != owner->kernels.end()) {
    *fn = it->second.fn;
    return LX_OK;
  }
  if (!may_load)
    return fail(LX_E_INVALID,
                "the simulation kernel for these options is not loaded on this device yet "
                "(loading allocates device memory): run the same call once through the "
                "allocating entry point first");
  std::vector<char> code;
  st = compile_source(make_src(), &code);
  if (st != LX_OK) return st;
  Kernel k;
  hipError_t e = hipModuleLoadData(&k.mod, code.data());
  if (e != hipSuccess) return hip_fail(e, "hipModuleLoadData");
  e = hipModuleGetFunction(&k.fn, k.mod, fname);
  if (e != hipSuccess) {
    (void)hipModuleUnload(k.mod);
    return hip_fail(e, "hipModuleGetFunction");
  }
  owner->kernels[key.str()] = k;
  *fn = k.fn;
  return LX_OK;
}

// A simulation or hook kernel of one network: variant "plain", "batched",
// "large" or "hooks", precision LX_PREC_*, `grid` for observation times.
lx_status get_kernel(lx_network_s* net, const char* variant, int precision, int block,
                     const char* fname, hipFunction_t* fn, int tpl, const std::string& consts,
                     bool grid = false, bool may_load = true) {
  std::ostringstream key;
  key << variant << (grid ? "-grid" : "") << "/" << precision << "/" << block << "/tpl" << tpl
      << "/c" << std::hex << fnv1a(consts) << std::dec;
  return get_kernel_src(
      net, key.str(),
      [&]() { return kernel_source(*net, variant, precision, block, tpl, consts, grid); }, fname,
      fn, may_load);
}

// Schedule-dependent fields of the launch parameters in canonical form (they
// are compile-time constants of the kernel, so equal launches share it).
void finish_params(const lx_options& o, bool batched, lx::SimParams* prm) {
  prm->ssa_k = batched ? (o.ssa_k ? o.ssa_k : 4) : 0;
  prm->regroup = batched ? o.regroup : 0;
  prm->tail = (batched && o.lanes_per_traj <= 1 && o.regroup == 0 && !o.cycles) ? o.tail_lanes : 0;
  prm->waves = o.waves_per_simd;
}

// Active lanes per wave of the batched schedule: full waves when the ensemble
// gives every SIMD (4 per CU) a wave, otherwise 32 or 16, so that more SIMDs
// are busy and each wave carries fewer divergent paths.
int choose_lanes(int requested, long long P, int cus) {
  if (requested) return requested;
  const long long simds = 4LL * cus;
  return P >= 64 * simds ? 64 : (P >= 32 * simds ? 32 : 16);
}

int tpl_of(const lx_options& o) { return o.lanes_per_traj > 1 ? o.lanes_per_traj : 1; }

// Trajectories per wave of the batched schedule.
int traj_per_wave(const lx_options& o, long long P, int cus) {
  const int tpl = tpl_of(o);
  if (tpl > 1) return (o.lanes_per_wave ? o.lanes_per_wave : 64) / tpl;
  return choose_lanes(o.lanes_per_wave, P, cus);
}

lx_status device_cus(int* cus) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(cus, hipDeviceAttributeMultiprocessorCount, dev);
  return e == hipSuccess ? LX_OK : hip_fail(e, "device attributes");
}

lx_status fill_params(const lx_options& o, int64_t P, double t_end, double eps, int32_t mode,
                      lx::SimParams* prm) {
  if (!(std::isfinite(t_end)) || !std::isfinite(o.t_start) || t_end < o.t_start)
    return fail(LX_E_INVALID, "need finite t_start <= t_end");
  if (!(eps > 0.0) || !std::isfinite(eps)) return fail(LX_E_INVALID, "eps must be positive");
  if (mode < 0 || mode > 2) return fail(LX_E_INVALID, "mode must be LX_MODE_*");
  if (o.precision != LX_PREC_FP64 && o.precision != LX_PREC_MIXED)
    return fail(LX_E_INVALID, "precision must be LX_PREC_*");
  if (o.schedule != LX_SCHED_PLAIN && o.schedule != LX_SCHED_BATCHED)
    return fail(LX_E_INVALID, "schedule must be LX_SCHED_*");
  if (o.n_c < 0 || !(o.delta >= 0.0) || !(o.n_stiff > 0.0) || !(o.k_ssa >= 0.0) ||
      !(o.k_crit > 0.0) || o.n_ssa_ex < 1 || o.n_ssa_im < 1 || !(o.lambda_thr >= 10.0) ||
      !(o.lambda_thr <= 30.0) || !(o.newton_tol > 0.0) || o.newton_maxit < 0 ||
      o.max_steps < 0 || o.max_steps > 4294967295LL)
    return fail(LX_E_INVALID, "option out of range");
  if (o.block_size != 0 && (o.block_size < 64 || o.block_size > MAX_BLOCK || o.block_size % 64 != 0))
    return fail(LX_E_INVALID, "block_size must be 0 or a multiple of 64 in [64, 256]");
  if (o.lanes_per_wave != 0 && o.lanes_per_wave != 4 && o.lanes_per_wave != 8 &&
      o.lanes_per_wave != 16 && o.lanes_per_wave != 32 && o.lanes_per_wave != 64)
    return fail(LX_E_INVALID, "lanes_per_wave must be 0, 4, 8, 16, 32 or 64");
  if (o.ssa_k < 0 || o.ssa_k > 64) return fail(LX_E_INVALID, "ssa_k must be in [0, 64]");
  if (o.regroup < 0 || o.regroup > 64) return fail(LX_E_INVALID, "regroup must be in [0, 64]");
  if (o.lanes_per_traj < 0 || o.lanes_per_traj > 16 ||
      (o.lanes_per_traj & (o.lanes_per_traj - 1)) != 0)
    return fail(LX_E_INVALID, "lanes_per_traj must be 0, 1, 2, 4, 8 or 16");
  if (o.lanes_per_traj > 1 && o.regroup > 0)
    return fail(LX_E_INVALID, "regroup needs one lane per trajectory");
  if (o.lanes_per_traj > 1 && o.lanes_per_wave != 0 && o.lanes_per_wave < o.lanes_per_traj)
    return fail(LX_E_INVALID, "lanes_per_wave must be at least lanes_per_traj");
  if (o.tail_lanes != 0 && o.tail_lanes != 2 && o.tail_lanes != 4 && o.tail_lanes != 8 &&
      o.tail_lanes != 16)
    return fail(LX_E_INVALID, "tail_lanes must be 0, 2, 4, 8 or 16");
  if (o.waves_per_simd < 0 || o.waves_per_simd > 8)
    return fail(LX_E_INVALID, "waves_per_simd must be in [0, 8]");
  if (o.blocks_per_cu < 0 || o.blocks_per_cu > 8)
    return fail(LX_E_INVALID, "blocks_per_cu must be in [0, 8]");
  if (o.jacobian != LX_JAC_ANALYTIC && o.jacobian != LX_JAC_FD && o.jacobian != LX_JAC_USER)
    return fail(LX_E_INVALID, "jacobian must be LX_JAC_ANALYTIC, LX_JAC_FD or LX_JAC_USER");
  {
    const uint64_t stride = o.pid_stride ? o.pid_stride : 1;
    if (P > 0 && (uint64_t)o.pid_base + (uint64_t)(P - 1) * stride >= 4294967296ull)
      return fail(LX_E_INVALID, "particle ids pid_base + p * pid_stride exceed 2^32");
  }
  memset(prm, 0, sizeof(*prm));
  prm->t_start = o.t_start;
  prm->t_end = t_end;
  prm->eps = eps;
  prm->delta = o.delta;
  prm->n_stiff = o.n_stiff;
  prm->k_ssa = o.k_ssa;
  prm->k_crit = o.k_crit;
  prm->lam_thr = o.lambda_thr;
  prm->newton_tol = o.newton_tol;
  prm->max_steps = o.max_steps;
  prm->P = P;
  prm->k0 = (uint32_t)o.seed;
  prm->k1 = (uint32_t)(o.seed >> 32) + o.rng_stream;
  prm->pid_base = o.pid_base;
  prm->pid_stride = o.pid_stride ? o.pid_stride : 1;
  prm->n_c = o.n_c;
  prm->n_ssa_ex = o.n_ssa_ex;
  prm->n_ssa_im = o.n_ssa_im;
  prm->newton_maxit = o.newton_maxit;
  prm->kcap = 20 + 4 * (int)std::ceil(o.lambda_thr);
  prm->mode = mode;
  prm->accumulate = o.accumulate ? 1 : 0;
  prm->jacobian = o.jacobian;
  prm->cycles = (unsigned long long*)(uintptr_t)o.cycles;
  if (o.cycles && o.regroup > 0)
    return fail(LX_E_INVALID, "cycle timers need regroup 0");
  return LX_OK;
}

// With opt.check_lanes: wait for the stream, read the status word of every
// record of `stats` (strided copy of 4 bytes out of each lx_stats), and
// report trajectories that ended with a status other than LANE_OK.
lx_status check_lanes(const lx_options& o, int64_t P, const lx_stats* stats, hipStream_t s,
                      int64_t* failed) {
  *failed = 0;
  if (!o.check_lanes || P == 0) return LX_OK;
  if (!stats) return fail(LX_E_INVALID, "check_lanes needs the stats buffer");
  std::vector<int32_t> st((size_t)P);
  hipError_t e = hipMemcpy2DAsync(st.data(), sizeof(int32_t), stats, sizeof(lx_stats),
                                  sizeof(int32_t), (size_t)P, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "reading lane statuses");
  int64_t first = -1;
  for (int64_t p = 0; p < P; ++p)
    if (st[(size_t)p] != 0) {
      if (first < 0) first = p;
      *failed += 1;
    }
  if (*failed) {
    std::ostringstream m;
    m << *failed << " of " << P << " trajectories ended with a non-OK status (first: row "
      << first << ", status " << st[(size_t)first] << ")";
    g_err = m.str();
  }
  return LX_OK;
}

// A resolved simulation launch: kernel, geometry and parameters.
struct SimLaunch {
  hipFunction_t fn = nullptr;
  long long grid = 0;
  int block = 0;
  bool batched = false;
  lx::SimParams prm;
};

// LDS bytes of a block of the one-trajectory-per-wave kernel (the layout of
// WaveArea, SolveArea and the species' reaction lists in lx_sim_wave.h and
// lx_sim_large.h), and from it the default register budget in waves per SIMD.
long long wave_lds_bytes(const lx_network_s& n, int precision, int block) {
  const long long R = precision == LX_PREC_MIXED ? 4 : 8;
  const long long MS = (n.M + 63) / 64, MP = 64 * MS, W = MP / 32;
  long long nslot = 0, nni = 0;
  for (int j = 0; j < n.M; ++j)
    for (int i = 0; i < n.N; ++i) {
      nslot += n.ro[(size_t)j * n.N + i] > 0;
      nni += n.nu[(size_t)j * n.N + i] != 0;
    }
  auto up8 = [](long long b) { return (b + 7) / 8 * 8; };
  const long long wave_area = up8(3 * MP * R + 4 * MP + 8LL * n.N + 4 * W + R);
  const long long solve_area =
      up8(8 * ((long long)n.N * (n.N + 1) + 4LL * n.N + 2LL * n.M + nslot) + 4LL * n.M + 24 +
          4LL * ((n.M + 31) / 32));
  return (block / 64) * wave_area + solve_area + 2 * (nni + 1) + 256;  // + cursor, lock, slack
}

int wave_default_waves(const lx_network_s& n, int precision, int block) {
  // waves per SIMD of the blocks the LDS lets be resident (at most 8 per CU),
  // rounded up, so that the register budget never keeps one of them out
  long long blocks = 163840 / wave_lds_bytes(n, precision, block);
  blocks = blocks > 8 ? 8 : blocks;
  const long long reach = (blocks * (block / 64) + 3) / 4;
  return (int)(reach < 1 ? 1 : (reach > WAVE_KERNEL_WAVES ? WAVE_KERNEL_WAVES : reach));
}

lx_status plan_sim(lx_network net, int64_t P, const lx_options& o, double t_end, double eps,
                   int32_t mode, SimLaunch* L, bool grid = false, bool may_load = true) {
  lx_status st = fill_params(o, P, t_end, eps, mode, &L->prm);
  if (st != LX_OK) return st;
  if (o.jacobian == LX_JAC_USER && net->jt_rxn.empty())
    return fail(LX_E_INVALID, "LX_JAC_USER needs a network created with derivative terms "
                              "(lx_network_create_jac)");
  if (P == 0) return LX_OK;
  if (net->large) {
    // The batched schedule runs one trajectory per wave (lx_sim_wave), or with
    // lanes_per_traj = 1 one per lane refilled from the block's range; the
    // plain schedule gives every lane one trajectory.
    if (o.lanes_per_traj > 1 || o.regroup > 0 || o.tail_lanes > 0)
      return fail(LX_E_UNSUPPORTED,
                  "networks beyond 16 species or 32 reactions run one wave (batched) or one "
                  "lane per trajectory without regrouping (lanes_per_traj 0 or 1, regroup and "
                  "tail_lanes 0)");
    const bool batched = o.schedule == LX_SCHED_BATCHED;
    L->batched = true;
    if (batched && o.lanes_per_traj == 0) {
      // waves of a block share one LDS area for their implicit solves; the
      // block is the largest (up to 4 waves) whose LDS the device allows
      int dev = 0, lds_max = 65536;
      hipError_t e = hipGetDevice(&dev);
      if (e == hipSuccess)
        e = hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
      if (e != hipSuccess) return hip_fail(e, "device attributes");
      if (o.block_size) {
        L->block = o.block_size;
      } else {
        L->block = 256;
        while (L->block > 64 && wave_lds_bytes(*net, o.precision, L->block) > lds_max)
          L->block -= 64;
      }
      if (wave_lds_bytes(*net, o.precision, L->block) > lds_max)
        return fail(LX_E_UNSUPPORTED, "the network's one-trajectory-per-wave kernel needs more LDS "
                                      "per block than the device has (use a smaller block_size, "
                                      "or lanes_per_traj = 1)");
      finish_params(o, true, &L->prm);
      L->prm.ssa_k = 0;
      if (L->prm.waves == 0) L->prm.waves = wave_default_waves(*net, o.precision, L->block);
      st = get_kernel(net, "wave", o.precision, L->block, "lx_sim_wave", &L->fn, 1,
                      const_source(L->prm), grid, may_load);
      if (st != LX_OK) return st;
      int cus = 0;
      st = device_cus(&cus);
      if (st != LX_OK) return st;
      const long long round = L->block / 64;
      // default: as many blocks per CU as their LDS lets be resident (at most 8)
      long long fit = 163840 / wave_lds_bytes(*net, o.precision, L->block);
      fit = fit < 1 ? 1 : (fit > 8 ? 8 : fit);
      const long long max_grid = (long long)cus * (o.blocks_per_cu ? o.blocks_per_cu : fit);
      long long per_block = (P + max_grid - 1) / max_grid;
      if (per_block < round) per_block = round;
      L->prm.per_block = per_block;
      L->prm.lanes = 1;
      L->grid = (P + per_block - 1) / per_block;
      if (L->grid > 0x7fffffffLL) return fail(LX_E_INVALID, "P too large for one launch");
      return LX_OK;
    }
    // one wave per block: every wave owns an LDS area for its cooperative
    // implicit solves (the 48 x 48 system of a 48-species network is 18 KB)
    if (o.block_size != 0 && o.block_size != 64)
      return fail(LX_E_INVALID, "networks beyond 16 species or 32 reactions run one lane per "
                                "trajectory in 64-thread blocks");
    L->block = 64;
    finish_params(o, true, &L->prm);
    st = get_kernel(net, "large", o.precision, L->block, "lx_sim_large", &L->fn, 1,
                    const_source(L->prm), grid, may_load);
    if (st != LX_OK) return st;
    long long per_block = L->block;
    int lanes = 64;
    if (batched) {
      int cus = 0;
      st = device_cus(&cus);
      if (st != LX_OK) return st;
      lanes = traj_per_wave(o, P, cus);
      const long long round = (long long)(L->block / 64) * lanes;
      const long long max_grid = (long long)cus * (o.blocks_per_cu ? o.blocks_per_cu : 4);
      per_block = (P + max_grid - 1) / max_grid;
      if (per_block < round) per_block = round;
    }
    L->prm.per_block = per_block;
    L->prm.lanes = lanes;
    L->grid = (P + per_block - 1) / per_block;
    if (L->grid > 0x7fffffffLL) return fail(LX_E_INVALID, "P too large for one launch");
    return LX_OK;
  }
  L->batched = o.schedule == LX_SCHED_BATCHED;
  L->block = o.block_size ? o.block_size : (L->batched ? 256 : 64);
  finish_params(o, L->batched, &L->prm);
  st = get_kernel(net, L->batched ? "batched" : "plain", o.precision, L->block,
                  L->batched ? "lx_sim_batched" : "lx_sim_plain", &L->fn,
                  L->batched ? tpl_of(o) : 1, const_source(L->prm), grid, may_load);
  if (st != LX_OK) return st;
  L->grid = (P + L->block - 1) / L->block;
  if (L->batched) {
    int cus = 0;
    st = device_cus(&cus);
    if (st != LX_OK) return st;
    const int lanes = traj_per_wave(o, P, cus);
    const long long round = (long long)(L->block / 64) * lanes;
    const long long max_grid = (long long)cus * (o.blocks_per_cu ? o.blocks_per_cu : 2);
    long long per_block = (P + max_grid - 1) / max_grid;
    if (per_block < round) per_block = round;
    L->prm.per_block = per_block;
    L->prm.lanes = lanes;
    L->grid = (P + per_block - 1) / per_block;
  }
  if (L->grid > 0x7fffffffLL) return fail(LX_E_INVALID, "P too large for one launch");
  return LX_OK;
}

lx_status launch_sim(const SimLaunch& L, const lx::SimParams& prm, const double* theta,
                     const int32_t* x0, int32_t* x_out, int32_t* r_out, double* G_out,
                     lx_stats* stats, hipStream_t s) {
  lx::Stats* sp = (lx::Stats*)stats;
  lx::SimParams p = prm;
  void* args[] = {(void*)&theta, (void*)&x0, (void*)&x_out, (void*)&r_out,
                  (void*)&G_out, (void*)&sp, (void*)&p};
  hipError_t e = hipModuleLaunchKernel(L.fn, (unsigned)L.grid, 1, 1, (unsigned)L.block, 1, 1, 0,
                                       s, args, nullptr);
  if (e != hipSuccess) return hip_fail(e, "launch of the simulation kernel");
  return LX_OK;
}

}  // namespace

extern "C" {

void lx_options_default(lx_options* o) {
  if (!o) return;
  memset(o, 0, sizeof(*o));
  o->precision = LX_PREC_FP64;
  o->schedule = LX_SCHED_PLAIN;
  o->seed = 160807058ull;
  o->n_c = 10;
  o->delta = 0.05;
  o->n_stiff = 100.0;
  o->k_ssa = 10.0;
  o->k_crit = 10.0;
  o->n_ssa_ex = 100;
  o->n_ssa_im = 10;
  o->lambda_thr = 15.0;
  o->newton_tol = 1e-10;
  o->newton_maxit = 20;
  o->max_steps = 10000000;
}

const char* lx_last_error(void) { return g_err.c_str(); }

lx_status lx_network_create(int32_t N, int32_t M, const int32_t* ro, const int32_t* pc,
                            lx_network* out) {
  if (!out) return fail(LX_E_INVALID, "out is null");
  *out = nullptr;
  if (N < 1 || M < 1) return fail(LX_E_INVALID, "need N >= 1 and M >= 1");
  if (!ro || !pc) return fail(LX_E_INVALID, "null stoichiometry table");
  if (M > MAX_M || N > MAX_N)
    return fail(LX_E_INVALID, "network too large (need N <= 64 species, M <= 256 reactions)");
  lx_network_s* n = new (std::nothrow) lx_network_s();
  if (!n) return fail(LX_E_NOMEM, "out of host memory");
  n->N = N;
  n->M = M;
  n->large = M > REG_M || N > REG_N;
  n->ro.assign((size_t)M * N, 0);
  n->nu.assign((size_t)M * N, 0);
  std::vector<int> order(M, 0);
  for (int j = 0; j < M; ++j) {
    for (int i = 0; i < N; ++i) {
      const int m = ro[(size_t)j * N + i], p = pc[(size_t)j * N + i];
      if (m < 0 || p < 0 || m > 3 || p > 1000000) {
        delete n;
        return fail(LX_E_INVALID, "table entries must be >= 0 (reactant orders <= 3)");
      }
      n->ro[(size_t)j * N + i] = m;
      n->nu[(size_t)j * N + i] = p - m;
      order[j] += m;
    }
    if (order[j] > 3) {
      delete n;
      return fail(LX_E_INVALID, "reaction order above 3");
    }
  }
  // Tau-bound factor case per species: highest order of the reactions that
  // consume it, and the largest multiplicity among those reactions.
  n->phi.assign(N, 0);
  for (int i = 0; i < N; ++i) {
    int hor = 0, mult = 0;
    for (int j = 0; j < M; ++j) {
      const int m = n->ro[(size_t)j * N + i];
      if (!m) continue;
      if (order[j] > hor) {
        hor = order[j];
        mult = m;
      } else if (order[j] == hor && m > mult) {
        mult = m;
      }
    }
    int c = 0;
    if (hor == 1) c = 1;
    else if (hor == 2) c = mult >= 2 ? 3 : 2;
    else if (hor == 3) c = mult >= 3 ? 6 : (mult == 2 ? 5 : 4);
    n->phi[i] = c;
  }
  // Reversible pairs: exactly opposite net changes, greedy by ascending index.
  n->partner.assign(M, -1);
  for (int j = 0; j < M; ++j) {
    if (n->partner[j] >= 0) continue;
    bool nz = false;
    for (int i = 0; i < N; ++i) nz = nz || n->nu[(size_t)j * N + i] != 0;
    if (!nz) continue;
    for (int k = j + 1; k < M; ++k) {
      if (n->partner[k] >= 0) continue;
      bool opp = true;
      for (int i = 0; i < N && opp; ++i) opp = n->nu[(size_t)k * N + i] == -n->nu[(size_t)j * N + i];
      if (opp) {
        n->partner[j] = k;
        n->partner[k] = j;
        n->npairs += 1;
        break;
      }
    }
  }
  n->netsrc = network_source(*n);
  *out = n;
  return LX_OK;
}

lx_status lx_network_create_jac(int32_t N, int32_t M, const int32_t* reactant_order,
                                const int32_t* product_coeff, int32_t n_terms,
                                const int32_t* rxn, const int32_t* wrt, const double* coef,
                                const int32_t* powers, lx_network* out) {
  if (!out) return fail(LX_E_INVALID, "out is null");
  *out = nullptr;
  if (n_terms < 1 || n_terms > 65536 || !rxn || !wrt || !coef || !powers)
    return fail(LX_E_INVALID, "need 1 to 65536 derivative terms and non-null term arrays");
  lx_network n = nullptr;
  lx_status st = lx_network_create(N, M, reactant_order, product_coeff, &n);
  if (st != LX_OK) return st;
  for (int t = 0; t < n_terms; ++t) {
    const int j = rxn[t], k = wrt[t];
    bool ok = j >= 0 && j < M && k >= 0 && k < N && n->ro[(size_t)j * N + k] > 0 &&
              std::isfinite(coef[t]);
    for (int i = 0; i < N && ok; ++i) ok = powers[(size_t)t * N + i] >= 0 && powers[(size_t)t * N + i] <= 16;
    if (!ok) {
      delete n;
      return fail(LX_E_INVALID, "derivative term " + std::to_string(t) +
                                    ": it must name a reaction and one of its reactant species, "
                                    "with a finite coefficient and powers in [0, 16]");
    }
  }
  n->jt_rxn.assign(rxn, rxn + n_terms);
  n->jt_wrt.assign(wrt, wrt + n_terms);
  n->jt_coef.assign(coef, coef + n_terms);
  n->jt_pow.assign(powers, powers + (size_t)n_terms * N);
  n->netsrc = network_source(*n);
  *out = n;
  return LX_OK;
}

lx_status lx_network_prepare(lx_network net, int32_t precision, int32_t schedule,
                             int32_t block_size) {
  if (!net) return fail(LX_E_INVALID, "null network");
  if (precision != LX_PREC_FP64 && precision != LX_PREC_MIXED)
    return fail(LX_E_INVALID, "precision must be LX_PREC_*");
  if (schedule != LX_SCHED_PLAIN && schedule != LX_SCHED_BATCHED)
    return fail(LX_E_INVALID, "schedule must be LX_SCHED_*");
  if (block_size != 0 && (block_size < 64 || block_size > MAX_BLOCK || block_size % 64 != 0))
    return fail(LX_E_INVALID, "block_size must be 0 or a multiple of 64 in [64, 256]");
  const bool wave = net->large && schedule == LX_SCHED_BATCHED;
  int wave_block = block_size ? block_size : 256;
  // without a device: the block a device with 64 KiB of LDS per block takes
  while (wave && !block_size && wave_block > 64 && wave_lds_bytes(*net, precision, wave_block) > 65536)
    wave_block -= 64;
  const int block = wave ? wave_block
                         : net->large ? 64
                                      : (block_size ? block_size : (schedule == LX_SCHED_BATCHED ? 256 : 64));
  // the kernel lx_simulate uses with default options, eps 0.03, adaptive mode
  lx_options o;
  lx_options_default(&o);
  o.precision = precision;
  o.schedule = schedule;
  lx::SimParams prm;
  lx_status st = fill_params(o, 1, 1.0, 0.03, LX_MODE_ADAPTIVE, &prm);
  if (st != LX_OK) return st;
  const bool batched = net->large || schedule == LX_SCHED_BATCHED;
  finish_params(o, batched, &prm);
  if (wave) {
    prm.ssa_k = 0;
    if (prm.waves == 0) prm.waves = wave_default_waves(*net, precision, block);
  }
  std::vector<char> code;
  const char* variant = wave ? "wave" : net->large ? "large" : (schedule == LX_SCHED_BATCHED ? "batched" : "plain");
  return compile_source(kernel_source(*net, variant, precision, block, 1, const_source(prm)), &code);
}

lx_status lx_network_destroy(lx_network net) {
  delete net;
  return LX_OK;
}

lx_status lx_network_info(lx_network net, int32_t* N, int32_t* M, int32_t* n_pairs) {
  if (!net) return fail(LX_E_INVALID, "null network");
  if (N) *N = net->N;
  if (M) *M = net->M;
  if (n_pairs) *n_pairs = net->npairs;
  return LX_OK;
}

lx_status lx_simulate(lx_network net, int64_t P, const double* theta, const int32_t* x0,
                      double t_end, double eps, int32_t mode, const lx_options* opt,
                      int32_t* x_out, int32_t* r_out, double* G_out, lx_stats* stats,
                      void* stream) {
  if (!net) return fail(LX_E_INVALID, "null network");
  if (P < 0) return fail(LX_E_INVALID, "P < 0");
  lx_options o;
  if (opt) o = *opt;
  else lx_options_default(&o);
  lx::SimParams tmp;
  lx_status st = fill_params(o, P, t_end, eps, mode, &tmp);
  if (st != LX_OK) return st;
  if (P == 0) return LX_OK;
  if (!theta || !x0 || !x_out || !r_out || !G_out)
    return fail(LX_E_INVALID, "null input/output pointer");
  SimLaunch L;
  st = plan_sim(net, P, o, t_end, eps, mode, &L);
  if (st != LX_OK) return st;
  st = launch_sim(L, L.prm, theta, x0, x_out, r_out, G_out, stats, (hipStream_t)stream);
  if (st != LX_OK) return st;
  int64_t failed = 0;
  st = check_lanes(o, P, stats, (hipStream_t)stream, &failed);
  if (st != LX_OK) return st;
  return failed ? LX_W_LANE_FAIL : LX_OK;
}

lx_status lx_simulate_grid(lx_network net, int64_t P, const double* theta, const int32_t* x0,
                           int32_t n_times, const double* times, double eps, int32_t mode,
                           const lx_options* opt, int32_t* x_grid, int32_t* x_out,
                           int32_t* r_out, double* G_out, lx_stats* stats, void* stream) {
  if (!net) return fail(LX_E_INVALID, "null network");
  if (P < 0) return fail(LX_E_INVALID, "P < 0");
  if (n_times < 1) return fail(LX_E_INVALID, "need n_times >= 1");
  lx_options o;
  if (opt) o = *opt;
  else lx_options_default(&o);
  // the end of the simulation is times[n_times - 1], checked per trajectory
  lx::SimParams tmp;
  lx_status st = fill_params(o, P, o.t_start, eps, mode, &tmp);
  if (st != LX_OK) return st;
  if (P == 0) return LX_OK;
  if (!theta || !x0 || !times || !x_grid || !x_out || !r_out || !G_out)
    return fail(LX_E_INVALID, "null input/output pointer");
  if ((long long)n_times > (1LL << 62) / ((long long)P * net->N))
    return fail(LX_E_INVALID, "x_grid too large");
  SimLaunch L;
  st = plan_sim(net, P, o, o.t_start, eps, mode, &L, true);
  if (st != LX_OK) return st;
  L.prm.times = times;
  L.prm.x_grid = x_grid;
  L.prm.n_times = n_times;
  st = launch_sim(L, L.prm, theta, x0, x_out, r_out, G_out, stats, (hipStream_t)stream);
  if (st != LX_OK) return st;
  int64_t failed = 0;
  st = check_lanes(o, P, stats, (hipStream_t)stream, &failed);
  if (st != LX_OK) return st;
  return failed ? LX_W_LANE_FAIL : LX_OK;
}

lx_status lx_simulate_set(int32_t K, const lx_set_item* items, double t_end, double eps,
                          int32_t mode, const lx_options* opt, void* stream) {
  if (K < 1 || K > lx::SET_MAX || !items) return fail(LX_E_INVALID, "need 1 <= K <= 8 items");
  lx_options o;
  if (opt) o = *opt;
  else lx_options_default(&o);
  o.schedule = LX_SCHED_BATCHED;
  if (o.cycles) return fail(LX_E_INVALID, "cycle timers apply to lx_simulate and lx_simulate_grid");
  long long total = 0;
  for (int k = 0; k < K; ++k) {
    const lx_set_item& it = items[k];
    if (!it.net || it.P < 0) return fail(LX_E_INVALID, "bad set item");
    if (it.net->large)
      return fail(LX_E_UNSUPPORTED, "network sets take networks of at most 16 species and 32 reactions");
    if (it.P > 0 && (!it.theta || !it.x0 || !it.x_out || !it.r_out || !it.G_out))
      return fail(LX_E_INVALID, "null input/output pointer in set item");
    lx_options ok = o;
    ok.pid_base = it.pid_base;
    ok.pid_stride = it.pid_stride;
    lx::SimParams tmp;
    lx_status st = fill_params(ok, it.P, t_end, eps, mode, &tmp);
    if (st != LX_OK) return st;
    total += it.P;
  }
  lx::SimParams prm;
  lx_status st = fill_params(o, 0, t_end, eps, mode, &prm);
  if (st != LX_OK) return st;
  if (total == 0) return LX_OK;
  const int block = o.block_size ? o.block_size : 256;
  int cus = 0;
  st = device_cus(&cus);
  if (st != LX_OK) return st;
  const int lanes = traj_per_wave(o, total, cus);
  const long long round = (long long)(block / 64) * lanes;
  // resident blocks, but no more than give every block a full round of lanes
  long long grid = (long long)cus * (o.blocks_per_cu ? o.blocks_per_cu : 2);
  const long long fill = (total + round - 1) / round;
  if (grid > fill) grid = fill;
  lx::SetArgs args;
  memset(&args, 0, sizeof(args));
  args.K = K;
  std::vector<const lx_network_s*> nets;
  std::ostringstream key;
  key << "set/" << o.precision << "/" << block << "/tpl" << tpl_of(o);
  for (int k = 0; k < K; ++k) {
    const lx_set_item& it = items[k];
    lx::SetItem& d = args.it[k];
    d.theta = it.theta;
    d.x0 = it.x0;
    d.x_out = it.x_out;
    d.r_out = it.r_out;
    d.G_out = it.G_out;
    d.stats = (lx::Stats*)it.stats;
    d.P = it.P;
    d.per_block = (it.P + grid - 1) / grid;
    d.lanes = lanes;
    d.pid_base = it.pid_base;
    d.pid_stride = it.pid_stride ? it.pid_stride : 1;
    nets.push_back(it.net);
    key << "/" << std::hex << fnv1a(it.net->netsrc) << std::dec;
  }
  finish_params(o, true, &prm);
  const std::string consts = const_source(prm);
  key << "/c" << std::hex << fnv1a(consts) << std::dec;
  hipFunction_t fn;
  st = get_kernel_src(items[0].net, key.str(),
                      [&]() { return set_source(nets, o.precision, block, tpl_of(o), consts); },
                      "lx_sim_set", &fn);
  if (st != LX_OK) return st;
  void* kargs[] = {(void*)&args, (void*)&prm};
  hipError_t e = hipModuleLaunchKernel(fn, (unsigned)grid, 1, 1, (unsigned)block, 1, 1, 0,
                                       (hipStream_t)stream, kargs, nullptr);
  if (e != hipSuccess) return hip_fail(e, "launch lx_sim_set");
  int64_t failed_total = 0;
  std::string first_msg;
  for (int k = 0; k < K; ++k) {
    int64_t failed = 0;
    st = check_lanes(o, items[k].P, items[k].stats, (hipStream_t)stream, &failed);
    if (st != LX_OK) return st;
    if (failed && first_msg.empty()) first_msg = "item " + std::to_string(k) + ": " + g_err;
    failed_total += failed;
  }
  if (failed_total) {
    g_err = first_msg;
    return LX_W_LANE_FAIL;
  }
  return LX_OK;
}

// ---------------------------------------------------------------------------
// Test hooks.
// ---------------------------------------------------------------------------
lx_status lx_test_philox(int64_t n, const uint32_t* ctr, const uint32_t* key, uint32_t* out,
                         void* stream) {
  if (n < 0 || (n > 0 && (!ctr || !key || !out))) return fail(LX_E_INVALID, "bad arguments");
  if (n == 0) return LX_OK;
  hipError_t e = lxh_launch_philox(n, ctr, key, out, (hipStream_t)stream);
  return e == hipSuccess ? LX_OK : hip_fail(e, "philox hook");
}

lx_status lx_test_uniform_f64(int64_t n, const uint32_t* w, double* out, void* stream) {
  if (n < 0 || (n > 0 && (!w || !out))) return fail(LX_E_INVALID, "bad arguments");
  if (n == 0) return LX_OK;
  hipError_t e = lxh_launch_uniform_f64(n, w, out, (hipStream_t)stream);
  return e == hipSuccess ? LX_OK : hip_fail(e, "uniform hook");
}

lx_status lx_test_uniform_f32(int64_t n, const uint32_t* w, float* out, void* stream) {
  if (n < 0 || (n > 0 && (!w || !out))) return fail(LX_E_INVALID, "bad arguments");
  if (n == 0) return LX_OK;
  hipError_t e = lxh_launch_uniform_f32(n, w, out, (hipStream_t)stream);
  return e == hipSuccess ? LX_OK : hip_fail(e, "uniform hook");
}

lx_status lx_test_math(int32_t fn, int64_t n, const void* in, void* out, void* stream) {
  const bool ok_fn = (fn >= 0 && fn <= 3) || (fn >= 10 && fn <= 12);
  if (!ok_fn || n < 0 || (n > 0 && (!in || !out))) return fail(LX_E_INVALID, "bad arguments");
  if (n == 0) return LX_OK;
  hipError_t e = lxh_launch_math(fn, n, in, out, (hipStream_t)stream);
  return e == hipSuccess ? LX_OK : hip_fail(e, "math hook");
}

lx_status lx_test_poisson(int64_t n, const double* lam, const uint32_t* pid, const uint32_t* e,
                          const uint32_t* site, uint64_t seed, uint32_t stream_id,
                          double lambda_thr, int32_t precision, int64_t* out, void* stream) {
  if (n < 0 || (n > 0 && (!lam || !pid || !e || !site || !out)) || !(lambda_thr >= 10.0) ||
      !(lambda_thr <= 30.0) || (precision != LX_PREC_FP64 && precision != LX_PREC_MIXED))
    return fail(LX_E_INVALID, "bad arguments");
  if (n == 0) return LX_OK;
  const int kcap = 20 + 4 * (int)std::ceil(lambda_thr);
  hipError_t err = lxh_launch_poisson(n, lam, pid, e, site, (uint32_t)seed,
                                      (uint32_t)(seed >> 32) + stream_id, lambda_thr, kcap,
                                      precision == LX_PREC_MIXED, (long long*)out,
                                      (hipStream_t)stream);
  return err == hipSuccess ? LX_OK : hip_fail(err, "poisson hook");
}

lx_status lx_test_exponential(int64_t n, const uint32_t* pid, const uint32_t* e, uint64_t seed,
                              uint32_t stream_id, int32_t precision, double* out, void* stream) {
  if (n < 0 || (n > 0 && (!pid || !e || !out)) ||
      (precision != LX_PREC_FP64 && precision != LX_PREC_MIXED))
    return fail(LX_E_INVALID, "bad arguments");
  if (n == 0) return LX_OK;
  hipError_t err = lxh_launch_exponential(n, pid, e, (uint32_t)seed,
                                          (uint32_t)(seed >> 32) + stream_id,
                                          precision == LX_PREC_MIXED, out, (hipStream_t)stream);
  return err == hipSuccess ? LX_OK : hip_fail(err, "exponential hook");
}

lx_status lx_test_tau_select(lx_network net, int64_t Q, const double* theta, const int32_t* x,
                             double eps, int32_t mode, const lx_options* opt, double* a,
                             uint32_t* crit, uint32_t* eq, double* tau, int32_t* action,
                             void* stream) {
  if (!net || Q < 0) return fail(LX_E_INVALID, "bad arguments");
  lx_options o;
  if (opt) o = *opt;
  else lx_options_default(&o);
  lx::SimParams prm;
  lx_status st = fill_params(o, Q, 1.0 + o.t_start, eps, mode, &prm);
  if (st != LX_OK) return st;
  if (Q == 0) return LX_OK;
  if (!theta || !x || !a || !crit || !eq || !tau || !action)
    return fail(LX_E_INVALID, "null pointer");
  hipFunction_t fn;
  st = get_kernel(net, "hooks", o.precision, 64, "lx_hook_tau", &fn, 1, std::string());
  if (st != LX_OK) return st;
  void* args[] = {(void*)&theta, (void*)&x, (void*)&a, (void*)&crit, (void*)&eq,
                  (void*)&tau, (void*)&action, (void*)&prm};
  hipError_t e = hipModuleLaunchKernel(fn, (unsigned)((Q + 63) / 64), 1, 1, 64, 1, 1, 0,
                                       (hipStream_t)stream, args, nullptr);
  return e == hipSuccess ? LX_OK : hip_fail(e, "tau hook");
}

lx_status lx_test_implicit(lx_network net, int64_t Q, const double* theta, const int32_t* x,
                           const double* tau, const int64_t* Pj, const int32_t* jc,
                           const lx_options* opt, int64_t* k, int32_t* ok, int32_t* iters,
                           void* stream) {
  if (!net || Q < 0) return fail(LX_E_INVALID, "bad arguments");
  lx_options o;
  if (opt) o = *opt;
  else lx_options_default(&o);
  lx::SimParams prm;
  lx_status st = fill_params(o, Q, 1.0 + o.t_start, 0.03, 0, &prm);
  if (st != LX_OK) return st;
  if (Q == 0) return LX_OK;
  if (!theta || !x || !tau || !Pj || !jc || !k || !ok || !iters)
    return fail(LX_E_INVALID, "null pointer");
  hipFunction_t fn;
  st = get_kernel(net, "hooks", LX_PREC_FP64, 64, "lx_hook_implicit", &fn, 1, std::string());
  if (st != LX_OK) return st;
  void* args[] = {(void*)&theta, (void*)&x, (void*)&tau, (void*)&Pj, (void*)&jc,
                  (void*)&k, (void*)&ok, (void*)&iters, (void*)&prm};
  hipError_t e = hipModuleLaunchKernel(fn, (unsigned)((Q + 63) / 64), 1, 1, 64, 1, 1, 0,
                                       (hipStream_t)stream, args, nullptr);
  return e == hipSuccess ? LX_OK : hip_fail(e, "implicit hook");
}

// ---------------------------------------------------------------------------
// Particle filter.
// ---------------------------------------------------------------------------
lx_status lx_pf_workspace_size(int64_t P, int32_t N, int32_t M, size_t* bytes) {
  if (!bytes || P < 1 || N < 1 || M < 1) return fail(LX_E_INVALID, "bad arguments");
  *bytes = lxpf_workspace_layout(P, N, M, nullptr, nullptr);
  return LX_OK;
}

}  // extern "C"

namespace {

lx_status pf_check(const lx_pf_problem* pb, double eps, int32_t mode, const lx_options* opt,
                   lx_options* o, SimLaunch* L, lx::PfWork* w, bool may_load = true) {
  if (!pb || !pb->net) return fail(LX_E_INVALID, "null problem or network");
  const lx_pf_problem& q = *pb;
  if (q.net->large)
    return fail(LX_E_UNSUPPORTED, "the particle filter takes networks of at most 16 species and 32 reactions");
  if (q.P < 1 || q.P > (1LL << 23) || q.K < 1) return fail(LX_E_INVALID, "need 1 <= P <= 2^23, K >= 1");
  if (q.obs_species < 0 || q.obs_species >= q.net->N) return fail(LX_E_INVALID, "bad obs_species");
  if (!(q.dt > 0.0) || !std::isfinite(q.dt) || !(q.obs_sd > 0.0) || !std::isfinite(q.obs_sd))
    return fail(LX_E_INVALID, "dt and obs_sd must be positive");
  if (!q.y || !q.alpha || !q.beta || !q.theta || !q.x || !q.r || !q.G || !q.loglik || !q.workspace)
    return fail(LX_E_INVALID, "null buffer");
  const size_t need = lxpf_workspace_layout(q.P, q.net->N, q.net->M, nullptr, nullptr);
  if (q.workspace_bytes < need || ((uintptr_t)q.workspace & 255u))
    return fail(LX_E_INVALID, "workspace too small or not 256-byte aligned");
  if (opt) *o = *opt;
  else lx_options_default(o);
  if (o->cycles) return fail(LX_E_INVALID, "cycle timers apply to lx_simulate and lx_simulate_grid");
  o->accumulate = 1;
  o->pid_base = 0;
  o->pid_stride = 1;
  o->t_start = 0.0;
  lx_status st = plan_sim(q.net, q.P, *o, q.dt, eps, mode, L, false, may_load);
  if (st != LX_OK) return st;
  lxpf_workspace_layout(q.P, q.net->N, q.net->M, (char*)q.workspace, w);
  return LX_OK;
}

lx_status pf_enqueue(const lx_pf_problem& q, const lx_options& o, const SimLaunch& L,
                     const lx::PfWork& w, hipStream_t s) {
  for (int k = 1; k <= q.K; ++k) {
    lx::SimParams prm = L.prm;
    prm.t_start = (double)(k - 1) * q.dt;
    prm.t_end = (double)k * q.dt;
    prm.k1 = (uint32_t)(o.seed >> 32) + o.rng_stream + (uint32_t)k;
    lx_status st = launch_sim(L, prm, q.theta, q.x, q.x, q.r, q.G, (lx_stats*)w.stats, s);
    if (st != LX_OK) return st;
    hipError_t e = lxpf_launch_interval(q.P, q.net->N, q.net->M, q.x, q.r, q.G, q.theta,
                                        q.y + (k - 1), q.obs_species, q.obs_sd, q.alpha,
                                        q.beta, (uint32_t)o.seed,
                                        (uint32_t)(o.seed >> 32) + o.rng_stream, (unsigned)k,
                                        q.loglik + (k - 1), w, s);
    if (e != hipSuccess) return hip_fail(e, "particle-filter kernels");
  }
  return LX_OK;
}

}  // namespace

struct lx_pf_graph_s {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

extern "C" {

lx_status lx_pf_run(const lx_pf_problem* pb, double eps, int32_t mode, const lx_options* opt,
                    void* stream) {
  lx_options o;
  SimLaunch L;
  lx::PfWork w;
  lx_status st = pf_check(pb, eps, mode, opt, &o, &L, &w);
  if (st != LX_OK) return st;
  return pf_enqueue(*pb, o, L, w, (hipStream_t)stream);
}

lx_status lx_pf_run_static(const lx_pf_problem* pb, double eps, int32_t mode,
                           const lx_options* opt, void* stream) {
  if (!pb || !pb->net) return fail(LX_E_INVALID, "null problem or network");
  void* base = nullptr;
  size_t bytes = 0;
  hipError_t e = lxpf_static_scratch(&base, &bytes);
  if (e != hipSuccess) return hip_fail(e, "address of the filter's static scratch");
  if (pb->P >= 1 && pb->net->N >= 1 && pb->net->M >= 1 && pb->P <= (1LL << 23)) {
    const size_t need = lxpf_workspace_layout(pb->P, pb->net->N, pb->net->M, nullptr, nullptr);
    if (need > bytes)
      return fail(LX_E_INVALID, "lx_pf_run_static: the filter needs " + std::to_string(need) +
                                    " bytes of scratch, above its static maximum of " +
                                    std::to_string(bytes) + " (use lx_pf_run with a workspace)");
  }
  lx_pf_problem q = *pb;
  q.workspace = base;
  q.workspace_bytes = bytes;
  lx_options o;
  SimLaunch L;
  lx::PfWork w;
  lx_status st = pf_check(&q, eps, mode, opt, &o, &L, &w, false);
  if (st != LX_OK) return st;
  return pf_enqueue(q, o, L, w, (hipStream_t)stream);
}

lx_status lx_pf_graph_create(const lx_pf_problem* pb, double eps, int32_t mode,
                             const lx_options* opt, void* stream, lx_pf_graph* out) {
  if (!out) return fail(LX_E_INVALID, "out is null");
  *out = nullptr;
  if (!stream) return fail(LX_E_INVALID, "graph capture needs a non-default stream");
  lx_options o;
  SimLaunch L;
  lx::PfWork w;
  lx_status st = pf_check(pb, eps, mode, opt, &o, &L, &w);  // compiles/loads before capture
  if (st != LX_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
  st = pf_enqueue(*pb, o, L, w, s);
  hipGraph_t graph = nullptr;
  e = hipStreamEndCapture(s, &graph);
  if (st != LX_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    return st;
  }
  if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
  lx_pf_graph_s* g = new (std::nothrow) lx_pf_graph_s();
  if (!g) {
    (void)hipGraphDestroy(graph);
    return fail(LX_E_NOMEM, "out of host memory");
  }
  g->graph = graph;
  e = hipGraphInstantiate(&g->exec, graph, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    (void)hipGraphDestroy(graph);
    delete g;
    return hip_fail(e, "hipGraphInstantiate");
  }
  *out = g;
  return LX_OK;
}

lx_status lx_pf_graph_launch(lx_pf_graph g, void* stream) {
  if (!g) return fail(LX_E_INVALID, "null graph");
  hipError_t e = hipGraphLaunch(g->exec, (hipStream_t)stream);
  return e == hipSuccess ? LX_OK : hip_fail(e, "hipGraphLaunch");
}

lx_status lx_pf_graph_destroy(lx_pf_graph g) {
  if (!g) return LX_OK;
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  delete g;
  return LX_OK;
}

lx_status lx_test_gamma(int64_t n, const double* shape, const uint32_t* pid, const uint32_t* e,
                        const uint32_t* j, uint64_t seed, uint32_t stream_id, double* out,
                        void* stream) {
  if (n < 0 || (n > 0 && (!shape || !pid || !e || !j || !out)))
    return fail(LX_E_INVALID, "bad arguments");
  if (n == 0) return LX_OK;
  hipError_t err = lxh_launch_gamma(n, shape, pid, e, j, (uint32_t)seed,
                                    (uint32_t)(seed >> 32) + stream_id, out, (hipStream_t)stream);
  return err == hipSuccess ? LX_OK : hip_fail(err, "gamma hook");
}

}  // extern "C"
