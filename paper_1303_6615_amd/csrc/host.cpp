// Host side of the library: FP64 coefficient tables, the context, and the
// C ABI declared in include/aparareal.h.
//
// Coefficients (all evaluated in FP64 on the host, then rounded once):
//   * modal basis of L_k (Sec. 6.1): omega_k = sqrt(1 + k^2/F), a_k = k/sqrt(F);
//   * fine ETDRK4 (Cox-Matthews, Sec. 6.2) per (k, alpha): with
//     lambda = -nu k^4 - i alpha omega_k / eps and z = h lambda,
//       E = e^z, E2 = e^{z/2}, Q = (h/2) phi1(z/2), f1 = h(phi1 - 3phi2 + 4phi3)(z),
//       2 f2 = 2h(phi2 - 2phi3)(z), f3 = h(-phi2 + 4phi3)(z);
//     phi_j by its Taylor series for |z| < 1.5, by the closed quotient
//     otherwise (the FP32 table also carries lo parts of E and E2, unused by
//     the kernels, which take E from the FP64 table);
//   * time average (eq. numerical average; Alg. 1): s_m = m T0/M,
//     w_m = rho(m/M)/M with rho(s) = C exp(-1/(s(1-s))), C normalising the
//     integral over (0,1) (trapezoid rule, which converges faster than any
//     power for this kernel); rot[m][k] = exp(-i omega_k s_m);
//   * coarse step (Alg. 2): hd[k] = exp(-nu k^4 dT/2), rotT[k] = exp(-i omega_k dT/eps).
#include <hip/hip_runtime.h>
#include <sys/stat.h>
#include <unistd.h>

#include <cmath>
#include <complex>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <algorithm>
#include <limits>
#include <map>
#include <memory>
#include <deque>
#include <mutex>
#include <queue>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/aparareal.h"
#include "launch.hpp"
#include "noalloc.hpp"
#include "wavefft.hpp"

namespace {

using cd = std::complex<double>;
using ap::cx;

thread_local std::string g_last_error;

int fail(int code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

int hip_fail(hipError_t e, const char* what) {
  return fail(AP_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  ~DevBuf() {
    if (p) (void)hipFree(p);
  }
  hipError_t alloc(size_t n) {
    if (n <= bytes && p) return hipSuccess;
    if (p) {
      (void)hipFree(p);
      p = nullptr;
      bytes = 0;
    }
    hipError_t e = hipMalloc(&p, n);
    if (e == hipSuccess) bytes = n;
    return e;
  }
  template <typename T>
  hipError_t upload(const std::vector<T>& v) {
    hipError_t e = alloc(v.size() * sizeof(T));
    if (e != hipSuccess) return e;
    return hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice);
  }
  template <typename T>
  T* as() const {
    return static_cast<T*>(p);
  }
};

double factorial(int n) {
  double f = 1.0;
  for (int i = 2; i <= n; ++i) f *= i;
  return f;
}

cd phi(int j, cd z) {
  if (j == 0) return std::exp(z);
  if (std::abs(z) < 1.5) {
    cd term = 1.0 / factorial(j);
    cd sum = term;
    for (int i = 1; i < 60; ++i) {
      term *= z / double(i + j);
      sum += term;
      if (std::abs(term) < 1e-20 * std::abs(sum)) break;
    }
    return sum;
  }
  cd num = std::exp(z);
  cd zp = 1.0;
  for (int i = 0; i < j; ++i) {
    num -= zp / factorial(i);
    zp *= z;
  }
  return num / zp;
}

double rho_constant() {
  // C = 1 / int_0^1 exp(-1/(s(1-s))) ds by the trapezoid rule on 8192 intervals
  const int n = 8192;
  double sum = 0.0;
  for (int i = 1; i < n; ++i) {
    const double s = double(i) / n;
    sum += std::exp(-1.0 / (s * (1.0 - s)));
  }
  return 1.0 / (sum / n);
}

template <typename T>
cx<T> to_cx(cd v) {
  return cx<T>{T(v.real()), T(v.imag())};
}

bool is_pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }

struct FineTables {
  DevBuf coef64, coef32;
};

struct AvgTables {
  DevBuf rot64, rot32, w64, w32, hd64, hd32, rotT64, rotT32;
  ap::CoarseTab<double> c64{};
  ap::CoarseTab<float> c32{};
};

// Measured durations (us) of the pipeline's workgroup jobs for one problem
// (aparareal_autotune); they replace the analytic estimates that order jobs.
struct CostCal {
  bool valid = false;
  double fine_step = 0, stage1 = 0, stage2 = 0, whole = 0;
};

}  // namespace

struct ap_ctx {
  int N = 0, KD = 0, KP = 0;
  double eps = 0, F = 0, nu = 0;
  int device = 0;
  std::vector<double> omega, akw;   // per retained k
  DevBuf tw64, tw32, basis64, basis32;
  ap::DevTables tabs;
  std::map<uint64_t, std::unique_ptr<FineTables>> fine_cache;
  std::map<std::tuple<uint64_t, uint64_t, int, int>, std::unique_ptr<AvgTables>> avg_cache;
  DevBuf ws_in, ws_out, ws_U, ws_F, ws_G, ws_part;
  // host staging of the fine coefficient tables for the allocation-free
  // fine batch ([8][3][KP] each), sized when the context is created
  std::vector<cx<double>> na_t64;
  std::vector<cx<float>> na_t32;
  // pipelined solve: per-level states, flags, job list and descriptor
  DevBuf pp_U, pp_F, pp_G, pp_part, pp_P1, pp_P2;     // this context's problem
  DevBuf pp_flags, pp_jobs, pp_prob, pp_rows;          // launches this context owns
  std::string pp_jobs_key;
  int pp_njobs = 0;
  std::vector<ap::PipeJob> pp_jobs_host;
  std::vector<unsigned char> pp_prob_host, pp_rows_host;
  // options (aparareal_set_option)
  int opt_split = -1;        // split coarse steps over workgroups: -1 auto, 0 no, 1 yes
  int opt_group = 0;         // samples per group of the average; 0 = by grid size
  int tuned_group = 0;       // group size chosen by aparareal_autotune when opt_group is 0
  int opt_grid = 0;          // workgroups of a persistent launch; 0 = all that fit
  CostCal cost;              // calibrated job durations (aparareal_autotune)
  int opt_graph = 0;         // replay pipelined launches from a captured hipGraph
  int opt_skip = 1;          // slice skipping: exact slices n <= k are copied, not recomputed
  int opt_sweeps = 0;        // tol > 0: iteration-ordered sweeps with host residual checks
  int opt_fine = 0;          // fine slices: 0 ETDRK4, 1 Strang steps (Alg. 3)
  int opt_coarse = 0;        // coarse step: 0 asymptotic (Alg. 2), 1 one Strang step (standard parareal)
  int opt_fine_group = 0;    // slices per fine job: 0 automatic, else at most this many
  int opt_fine_shape = -1;   // workgroup shape of the fine batch: -1 tuned (or default), else 0..2
  int handoff_ns = 6000;     // scheduling weight per dependency of the launches this context owns
  int tuned_shape[2] = {-1, -1};   // per precision: from aparareal_autotune_fine or the tuning cache
  std::string device_key;          // device kind, the tuning cache's key
  hipGraph_t graph = nullptr;
  hipGraphExec_t graph_exec = nullptr;
  hipStream_t graph_stream = nullptr;   // private stream the graph is captured on
  std::string graph_key;
  int* pp_diag = nullptr;   // stall record of the last pipelined launch
  bool trace_on = false;     // record per-job device-clock intervals
  DevBuf pp_trace;
  int pp_trace_jobs = 0;
  hipStream_t last_stream = nullptr;
  bool has_last = false;
  // kernel timing (aparareal_profile)
  bool prof_on = false;
  std::vector<hipEvent_t> ev_pool;
  std::vector<std::tuple<int, hipEvent_t, hipEvent_t>> ev_pending;
  int prof_count[AP_K_CLASSES] = {};
  double prof_ms[AP_K_CLASSES] = {};
  ~ap_ctx() {
    if (graph_exec) (void)hipGraphExecDestroy(graph_exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (graph_stream) (void)hipStreamDestroy(graph_stream);
    for (auto& t : ev_pending) {
      ev_pool.push_back(std::get<1>(t));
      ev_pool.push_back(std::get<2>(t));
    }
    for (hipEvent_t e : ev_pool) (void)hipEventDestroy(e);
  }
};

namespace {

uint64_t bits(double v) {
  uint64_t b;
  std::memcpy(&b, &v, sizeof(b));
  return b;
}

// Calls on one context may come on different streams; workspace reuse must
// not race with a previous call still in flight.
hipError_t order_stream(ap_ctx* c, hipStream_t s) {
  if (c->has_last && c->last_stream != s) {
    hipError_t e = hipStreamSynchronize(c->last_stream);
    if (e != hipSuccess) return e;
  }
  c->last_stream = s;
  c->has_last = true;
  return hipSuccess;
}

hipEvent_t take_event(ap_ctx* c) {
  if (!c->ev_pool.empty()) {
    hipEvent_t e = c->ev_pool.back();
    c->ev_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Launch `fn` (returning hipError_t); with profiling on, bracket it with events.
template <typename Fn>
hipError_t timed(ap_ctx* c, int cls, hipStream_t s, Fn&& fn) {
  if (!c->prof_on) return fn();
  hipEvent_t a = take_event(c), b = take_event(c);
  if (!a || !b) return fn();
  (void)hipEventRecord(a, s);
  hipError_t e = fn();
  (void)hipEventRecord(b, s);
  c->ev_pending.emplace_back(cls, a, b);
  return e;
}

// grow a workspace buffer, draining outstanding work first
hipError_t ensure(ap_ctx* c, DevBuf& b, size_t bytes) {
  if (b.p && b.bytes >= bytes) return hipSuccess;
  if (c->has_last) {
    hipError_t e = hipStreamSynchronize(c->last_stream);
    if (e != hipSuccess) return e;
  }
  return b.alloc(bytes);
}

// ETDRK4 coefficients of step h for every retained mode and eigen-branch
// (Sec. 6.2, the Cox-Matthews scheme with the exact linear part
// lambda = -nu k^4 - i alpha omega_k / eps): [8][3][KP] tables
//   FP64: E, 0, E2, 0, Q, f1, 2 f2, f3
//   FP32: E and E2 each as hi + lo, then Q, f1, 2 f2, f3.
void fine_coefs(const ap_ctx* c, double h, cx<double>* t64, cx<float>* t32) {
  const int KP = c->KP;
  for (int k = 0; k < KP; ++k) {
    const double kk = double(k);
    for (int al = 0; al < 3; ++al) {
      const double alpha = double(al - 1);
      const cd lam(-c->nu * kk * kk * kk * kk, -alpha * c->omega[k] / c->eps);
      const cd z = h * lam;
      const cd p1 = phi(1, z), p2 = phi(2, z), p3 = phi(3, z);
      const cd vals[6] = {std::exp(z),
                          std::exp(0.5 * z),
                          0.5 * h * phi(1, 0.5 * z),
                          h * (p1 - 3.0 * p2 + 4.0 * p3),
                          2.0 * h * (p2 - 2.0 * p3),
                          h * (-p2 + 4.0 * p3)};
      const size_t o = size_t(al) * KP + k;
      auto at = [&](int slot) { return size_t(slot) * 3 * KP + o; };
      t64[at(0)] = to_cx<double>(vals[0]);
      t64[at(1)] = cx<double>{0, 0};
      t64[at(2)] = to_cx<double>(vals[1]);
      t64[at(3)] = cx<double>{0, 0};
      for (int q = 2; q < 6; ++q) t64[at(q + 2)] = to_cx<double>(vals[q]);
      for (int q = 0; q < 2; ++q) {
        const cx<float> hi = to_cx<float>(vals[q]);
        const cd rest = vals[q] - cd(double(hi.x), double(hi.y));
        t32[at(2 * q)] = hi;
        t32[at(2 * q + 1)] = to_cx<float>(rest);
      }
      for (int q = 2; q < 6; ++q) t32[at(q + 2)] = to_cx<float>(vals[q]);
    }
  }
}

int fine_tables(ap_ctx* c, double h, FineTables** out) {
  auto it = c->fine_cache.find(bits(h));
  if (it != c->fine_cache.end()) {
    *out = it->second.get();
    return AP_OK;
  }
  auto ft = std::make_unique<FineTables>();
  std::vector<cx<double>> t64(size_t(8) * 3 * c->KP);
  std::vector<cx<float>> t32(size_t(8) * 3 * c->KP);
  fine_coefs(c, h, t64.data(), t32.data());
  hipError_t e = ft->coef64.upload(t64);
  if (e == hipSuccess) e = ft->coef32.upload(t32);
  if (e != hipSuccess) return hip_fail(e, "fine coefficient upload");
  *out = ft.get();
  c->fine_cache[bits(h)] = std::move(ft);
  return AP_OK;
}

// ------------------------------------------------------------ tuning cache -
// Persisted choices of aparareal_autotune_fine, one line per device, grid size
// and precision:  "fine <device> <N> <precision> <shape>".  The file is
// $APARAREAL_TUNE_CACHE, else $XDG_CACHE_HOME/aparareal/tune.txt, else
// $HOME/.cache/aparareal/tune.txt; the last line for a key wins.  A missing or
// unreadable file means no entries, and a failed write is ignored: a shape
// only changes speed, never results.
std::mutex g_tune_mu;

std::string tune_cache_path() {
  if (const char* p = std::getenv("APARAREAL_TUNE_CACHE")) return p;
  if (const char* x = std::getenv("XDG_CACHE_HOME")) return std::string(x) + "/aparareal/tune.txt";
  if (const char* h = std::getenv("HOME")) return std::string(h) + "/.cache/aparareal/tune.txt";
  return std::string();
}

// Identifies the device kind: architecture name and compute-unit count.
std::string device_key(int device) {
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) != hipSuccess) return "unknown";
  std::string k = prop.gcnArchName;
  for (char& ch : k)
    if (ch == ' ') ch = '_';
  return k + "/" + std::to_string(prop.multiProcessorCount) + "cu";
}

std::vector<std::string> read_lines(const std::string& path) {
  std::vector<std::string> out;
  if (path.empty()) return out;
  FILE* f = std::fopen(path.c_str(), "r");
  if (!f) return out;
  char buf[512];
  while (std::fgets(buf, sizeof(buf), f)) {
    std::string ln(buf);
    while (!ln.empty() && (ln.back() == '\n' || ln.back() == '\r')) ln.pop_back();
    if (!ln.empty()) out.push_back(ln);
  }
  std::fclose(f);
  return out;
}

// A fine-batch configuration (workgroup shape and FFT plan) compiled for N.
bool fine_config_valid(int N, int config) {
  return config >= 0 && config < ap::kFineConfigCount && ap::fine_shape(N, false, config, nullptr) > 0;
}

// The cached configuration for (device, N, precision), or -1.
int tune_lookup(const std::string& dev, int N, int precision) {
  std::lock_guard<std::mutex> lock(g_tune_mu);
  const std::string key = "fine " + dev + " " + std::to_string(N) + " " + std::to_string(precision) + " ";
  int shape = -1;
  for (const std::string& ln : read_lines(tune_cache_path()))
    if (ln.compare(0, key.size(), key) == 0) {
      const int v = std::atoi(ln.c_str() + key.size());
      if (fine_config_valid(N, v)) shape = v;
    }
  return shape;
}

void tune_store(const std::string& dev, int N, int precision, int shape) {
  std::lock_guard<std::mutex> lock(g_tune_mu);
  const std::string path = tune_cache_path();
  if (path.empty()) return;
  const std::string key = "fine " + dev + " " + std::to_string(N) + " " + std::to_string(precision) + " ";
  std::vector<std::string> keep;
  for (const std::string& ln : read_lines(path))
    if (ln.compare(0, key.size(), key) != 0) keep.push_back(ln);
  keep.push_back(key + std::to_string(shape));
  // create the directory chain, then write a temporary file and rename it
  for (size_t i = 1; i < path.size(); ++i)
    if (path[i] == '/') {
      const std::string d = path.substr(0, i);
      (void)mkdir(d.c_str(), 0755);
    }
  const std::string tmp = path + ".tmp" + std::to_string(getpid());
  FILE* f = std::fopen(tmp.c_str(), "w");
  if (!f) return;
  for (const std::string& ln : keep) std::fprintf(f, "%s\n", ln.c_str());
  const bool ok = std::fclose(f) == 0;
  if (ok) (void)std::rename(tmp.c_str(), path.c_str());
  else (void)std::remove(tmp.c_str());
}

// Configuration (workgroup shape and FFT plan) of the context's fine batches
// in this precision: the option if set, else the tuned one, else the default.
int fine_shape_of(const ap_ctx* c, int precision) {
  if (c->opt_fine_shape >= 0) return c->opt_fine_shape;
  const int t = c->tuned_shape[precision == AP_PREC_FP64 ? 1 : 0];
  return t >= 0 ? t : 0;
}

// Samples per group of the time average: as many as make one round of
// transforms for the eight wavefronts of a pipeline workgroup (3 signals per
// sample; 64 / G signals per wavefront with G lanes per signal of length N).
int default_group_size(int nx) {
  const int P = nx / 2;
  const int G = P <= 32 ? 8 : P <= 64 ? 16 : P <= 128 ? 32 : 64;
  return std::max(1, 8 * (64 / G) / 3);
}

int group_size(const ap_ctx* c) {
  return c->opt_group > 0 ? c->opt_group : c->tuned_group > 0 ? c->tuned_group : default_group_size(c->N);
}

// Group sizes the autotuner tries for split coarse steps: multiples 1, 3/2, 2
// and 3 of the grid-size default.  Larger groups mean longer stage jobs but
// fewer group sums for the stage-2 jobs and the finisher to read back.
constexpr int kTuneGroupMults2[] = {2, 3, 4, 6};   // twice the multiple
int tune_group(int nx, int cand) { return std::max(1, default_group_size(nx) * kTuneGroupMults2[cand] / 2); }

// dT == 0 builds the average-only tables.
int avg_tables(ap_ctx* c, double dT, double T0, int M, AvgTables** out) {
  const int gs = group_size(c);
  auto key = std::make_tuple(bits(dT), bits(T0), M, gs);
  auto it = c->avg_cache.find(key);
  if (it != c->avg_cache.end()) {
    *out = it->second.get();
    return AP_OK;
  }
  auto at = std::make_unique<AvgTables>();
  const int KP = c->KP;
  const double C = rho_constant();
  std::vector<cx<double>> r64(size_t(M) * KP);
  std::vector<cx<float>> r32(size_t(M) * KP);
  std::vector<double> w64(M);
  std::vector<float> w32(M);
  for (int m = 0; m < M; ++m) {
    const double sr = double(m) / M;     // s_m / T0
    const double s = T0 * sr;
    const double rho = (sr > 0.0 && sr < 1.0) ? C * std::exp(-1.0 / (sr * (1.0 - sr))) : 0.0;
    w64[m] = rho / M;
    w32[m] = float(w64[m]);
    for (int k = 0; k < KP; ++k) {
      const double th = c->omega[k] * s;
      const cd e(std::cos(th), -std::sin(th));
      r64[size_t(m) * KP + k] = to_cx<double>(e);
      r32[size_t(m) * KP + k] = to_cx<float>(e);
    }
  }
  std::vector<double> hd64(KP);
  std::vector<float> hd32(KP);
  std::vector<cx<double>> rt64(KP);
  std::vector<cx<float>> rt32(KP);
  for (int k = 0; k < KP; ++k) {
    const double kk = double(k);
    hd64[k] = std::exp(-c->nu * kk * kk * kk * kk * dT * 0.5);
    hd32[k] = float(hd64[k]);
    const double th = c->omega[k] * dT / c->eps;
    const cd e(std::cos(th), -std::sin(th));
    rt64[k] = to_cx<double>(e);
    rt32[k] = to_cx<float>(e);
  }
  hipError_t e = at->rot64.upload(r64);
  if (e == hipSuccess) e = at->rot32.upload(r32);
  if (e == hipSuccess) e = at->w64.upload(w64);
  if (e == hipSuccess) e = at->w32.upload(w32);
  if (e == hipSuccess) e = at->hd64.upload(hd64);
  if (e == hipSuccess) e = at->hd32.upload(hd32);
  if (e == hipSuccess) e = at->rotT64.upload(rt64);
  if (e == hipSuccess) e = at->rotT32.upload(rt32);
  if (e != hipSuccess) return hip_fail(e, "average table upload");
  at->c64 = ap::CoarseTab<double>{{at->rot64.as<cx<double>>(), at->w64.as<double>(), M, gs},
                                  at->hd64.as<double>(), at->rotT64.as<cx<double>>(), dT};
  at->c32 = ap::CoarseTab<float>{{at->rot32.as<cx<float>>(), at->w32.as<float>(), M, gs},
                                 at->hd32.as<float>(), at->rotT32.as<cx<float>>(), float(dT)};
  *out = at.get();
  c->avg_cache[key] = std::move(at);
  return AP_OK;
}

int check_ctx(ap_ctx* c) {
  if (!c) return fail(AP_EINVAL, "null context");
  return AP_OK;
}

int check_prec(int precision) {
  if (precision != AP_PREC_FP32 && precision != AP_PREC_FP64)
    return fail(AP_EINVAL, "precision must be AP_PREC_FP32 (0) or AP_PREC_FP64 (1)");
  return AP_OK;
}

size_t state_bytes(const ap_ctx* c) { return size_t(3) * c->KP * sizeof(cx<double>); }

// common prologue of the batched entry points: physical -> modal into ws_in
int batch_prologue(ap_ctx* c, const double* in, void* out, int batch, int precision, hipStream_t s) {
  int rc = check_ctx(c);
  if (rc) return rc;
  if ((rc = check_prec(precision))) return rc;
  if (batch < 0) return fail(AP_EINVAL, "batch must be >= 0");
  if (batch > 0 && (!in || !out)) return fail(AP_EINVAL, "null array");
  hipError_t e = order_stream(c, s);
  if (e != hipSuccess) return hip_fail(e, "stream ordering");
  if (batch == 0) return AP_OK;
  const size_t need = size_t(batch) * state_bytes(c);
  if ((e = ensure(c, c->ws_in, need)) != hipSuccess) return hip_fail(e, "workspace");
  if ((e = ensure(c, c->ws_out, need)) != hipSuccess) return hip_fail(e, "workspace");
  e = timed(c, AP_K_TO_MODAL, s, [&] { return ap::launch_to_modal(c->N, in, c->ws_in.as<cx<double>>(), batch, c->tabs, s); });
  if (e != hipSuccess) return hip_fail(e, "to_modal launch");
  return AP_OK;
}

int batch_epilogue(ap_ctx* c, double* out, int batch, hipStream_t s) {
  hipError_t e = timed(c, AP_K_TO_PHYSICAL, s,
                       [&] { return ap::launch_to_physical(c->N, c->ws_out.as<cx<double>>(), out, batch, c->tabs, s); });
  if (e != hipSuccess) return hip_fail(e, "to_physical launch");
  return AP_OK;
}

int solve_sweeps(ap_ctx* c, const double* u0, const ap_solve_params* p, double* U_out, double* resid,
                 hipStream_t s, int steps, FineTables* ft, AvgTables* at) {
  const int Ns = p->slices;
  const size_t sb = state_bytes(c);
  hipError_t e;
  if ((e = ensure(c, c->ws_U, sb * (Ns + 1))) != hipSuccess ||
      (e = ensure(c, c->ws_F, sb * (Ns + 1))) != hipSuccess ||
      (e = ensure(c, c->ws_G, sb * (Ns + 1))) != hipSuccess ||
      (e = ensure(c, c->ws_part, sizeof(double2) * size_t(Ns) * std::max(1, p->K))) != hipSuccess)
    return hip_fail(e, "solve workspace");
  const bool f64 = p->precision == AP_PREC_FP64;
  const ap::CoarseTab<double>* c64 = f64 ? &at->c64 : nullptr;
  const ap::CoarseTab<float>* c32 = f64 ? nullptr : &at->c32;
  cx<double>* U = c->ws_U.as<cx<double>>();
  cx<double>* Fn = c->ws_F.as<cx<double>>();
  cx<double>* G = c->ws_G.as<cx<double>>();
  double2* part = c->ws_part.as<double2>();
  const size_t st = size_t(3) * c->KP;
  e = timed(c, AP_K_TO_MODAL, s, [&] { return ap::launch_to_modal(c->N, u0, U, 1, c->tabs, s); });
  if (e != hipSuccess) return hip_fail(e, "to_modal");
  e = timed(c, AP_K_SWEEP, s, [&] { return ap::launch_sweep(c->N, U, Fn, G, part, Ns, 1, c64, c32, c->tabs, s); });
  if (e != hipSuccess) return hip_fail(e, "initial sweep");
  for (int k = 0; k < p->K; ++k) {
    e = timed(c, AP_K_FINE, s, [&] {
      return ap::launch_fine(c->N, f64, U, Fn + st, Ns, steps, ft->coef64.as<cx<double>>(),
                             ft->coef32.as<cx<float>>(), c->tabs, s);
    });
    if (e != hipSuccess) return hip_fail(e, "fine batch");
    e = timed(c, AP_K_SWEEP, s,
              [&] { return ap::launch_sweep(c->N, U, Fn, G, part + size_t(k) * Ns, Ns, 0, c64, c32, c->tabs, s); });
    if (e != hipSuccess) return hip_fail(e, "correction sweep");
    e = timed(c, AP_K_RESID, s,
              [&] { return ap::launch_resid(part + size_t(k) * Ns, Ns, 1, resid + k, nullptr, s); });
    if (e != hipSuccess) return hip_fail(e, "resid");
    if (p->tol > 0.0) {
      double r = 0.0;
      if ((e = hipMemcpyAsync(&r, resid + k, sizeof(double), hipMemcpyDeviceToHost, s)) != hipSuccess ||
          (e = hipStreamSynchronize(s)) != hipSuccess)
        return hip_fail(e, "residual readback");
      if (!std::isfinite(r)) return fail(AP_ENUMERIC, "non-finite parareal residual");
      if (r <= p->tol && k + 1 < p->K) {
        std::vector<double> rest(size_t(p->K - k - 1), -1.0);
        if ((e = hipMemcpyAsync(resid + k + 1, rest.data(), rest.size() * sizeof(double), hipMemcpyHostToDevice,
                                s)) != hipSuccess ||
            (e = hipStreamSynchronize(s)) != hipSuccess)
          return hip_fail(e, "residual fill");
        break;
      }
    }
  }
  e = timed(c, AP_K_TO_PHYSICAL, s, [&] { return ap::launch_to_physical(c->N, U, U_out, Ns + 1, c->tabs, s); });
  if (e != hipSuccess) return hip_fail(e, "to_physical");
  return AP_OK;
}

// ------------------------------------------------------------- scheduling ---
// Shape of one problem in a pipelined launch.
struct PipeShape {
  int nx = 0, Ns = 0, K = 0, steps = 0, M = 0, gs = 1, groups = 1;
  bool split = false, fp64 = false;
  bool skip = true;          // slices n <= k of level k copy their exact values
  int fine_kind = 0, coarse_kind = 0;
  int fg = 1;                // slices per fine job (consecutive slices of one level, stepped together)
  double tol = 0.0;
  CostCal cal;
};

// Estimated duration (us) of the workgroup jobs of one problem, used only to
// order the jobs.  Without a calibration: one nonlinear evaluation at grid
// size N takes about 1.6 + 0.0032 N us in FP32 (x1.6 in FP64), a fine step
// four of them; a group job of the average costs a fixed 3 us plus 1.5
// evaluation times per round of transforms its 3 gs signals need, a whole
// coarse step 3 us plus 2.2 per round for each of its two averages (measured
// on MI355X at N = 256 and 1024).
struct JobCost {
  double fine, stage1, stage2, mid, finish, whole;
};

JobCost job_cost(const PipeShape& q) {
  const double ev = (1.6 + 0.0032 * q.nx) * (q.fp64 ? 1.6 : 1.0);
  const int P = q.nx / 2;
  const int G = P <= 32 ? 8 : P <= 64 ? 16 : P <= 128 ? 32 : 64;
  const int per_round = 8 * (64 / G);
  auto rounds = [&](int samples) { return double((3 * samples + per_round - 1) / per_round); };
  JobCost c;
  c.fine = (q.fine_kind == 1 ? 2.0 : 4.0) * ev * q.steps + 2.0;
  c.stage1 = 3.0 + 1.5 * rounds(q.gs) * ev;
  c.stage2 = c.stage1 + 0.5;
  c.mid = 3.0;       // the last stage-1 job sums the group sums and stores y
  c.finish = 0.5;
  c.whole = q.coarse_kind == 1 ? 2.0 * ev + 3.0 : 2.0 * (3.0 + 2.2 * rounds(q.M - 1) * ev) + 1.0;
  if (q.cal.valid) {
    if (q.cal.fine_step > 0) c.fine = q.cal.fine_step * q.steps;
    if (q.cal.stage1 > 0) c.stage1 = q.cal.stage1;
    if (q.cal.stage2 > 0) c.stage2 = q.cal.stage2;
    if (q.cal.whole > 0) c.whole = q.cal.whole;
  }
  return c;
}

// Every job's dependencies must come earlier in the hand-out order (for a
// split step: every stage-2 job after all stage-1 jobs of the step and after
// every job the finishing one waits for).  Then the earliest unfinished job
// always has its inputs, whatever the number of workgroups.
bool order_is_valid(const std::vector<ap::PipeJob>& jobs, const std::vector<PipeShape>& shapes) {
  std::vector<size_t> base(shapes.size() + 1, 0);
  for (size_t p = 0; p < shapes.size(); ++p) base[p + 1] = base[p] + size_t(shapes[p].K + 1) * shapes[p].Ns;
  const long long none = -1;
  // per (prob, k, n): first/last position of the coarse step's jobs, its
  // stage-1 last position, stage-2 first position; per fine slice its position
  std::vector<long long> cfirst(base.back(), none), clast(base.back(), none), s1last(base.back(), none),
      s2first(base.back(), none), fpos(base.back(), none);
  for (size_t i = 0; i < jobs.size(); ++i) {
    const ap::PipeJob& j = jobs[i];
    if (j.prob < 0 || size_t(j.prob) >= shapes.size()) return false;
    const PipeShape& q = shapes[j.prob];
    if (j.k < 0 || j.k > q.K || j.n < 1 || j.n > q.Ns) return false;
    const size_t at = base[j.prob] + size_t(j.k) * q.Ns + (j.n - 1);
    const long long pos = (long long)i;
    if (j.type == ap::kJobFine) {
      // slices n .. n + g - 1 (g >= 1, at most the problem's slices per fine job)
      const int g = std::max(1, j.g);
      if (j.k >= q.K || g > std::max(1, q.fg) || j.n + g - 1 > q.Ns) return false;
      for (int i = 0; i < g; ++i) {
        if (fpos[at + i] != none) return false;
        fpos[at + i] = pos;
      }
      continue;
    }
    if (cfirst[at] == none) cfirst[at] = pos;
    clast[at] = pos;
    if (j.type == ap::kJobStage1) s1last[at] = pos;
    if (j.type == ap::kJobStage2 && s2first[at] == none) s2first[at] = pos;
    if (j.type == ap::kJobCopy && (!q.skip || j.k < 1 || j.n > j.k)) return false;
  }
  for (size_t p = 0; p < shapes.size(); ++p) {
    const PipeShape& q = shapes[p];
    auto idx = [&](int k, int n) { return base[p] + size_t(k) * q.Ns + (n - 1); };
    for (int k = 0; k <= q.K; ++k)
      for (int n = 1; n <= q.Ns; ++n) {
        const size_t at = idx(k, n);
        if (cfirst[at] == none) return false;
        // with a tolerance, C(k, Ns) (its completion point) comes after the copy jobs of level k
        auto copies_before = [&](long long from) {
          if (!(q.tol > 0.0) || !q.skip || k < 1 || n != q.Ns) return true;
          for (int m = 1; m <= std::min(k, q.Ns - 1); ++m)
            if (clast[idx(k, m)] >= from) return false;
          return true;
        };
        if (q.skip && k >= 1 && n <= k) {
          // copy job: after C(k-1,n) and, for n = k, after F(k-1,k); no fine slice
          if (fpos[at] != none || clast[idx(k - 1, n)] >= cfirst[at]) return false;
          if (n == k && (fpos[idx(k - 1, n)] == none || fpos[idx(k - 1, n)] >= cfirst[at])) return false;
          if (!copies_before(cfirst[at])) return false;
          continue;
        }
        if (k < q.K && fpos[at] == none) return false;
        const long long prev_done = n > 1 ? clast[idx(k, n - 1)] : none;
        if (k < q.K && prev_done >= fpos[at]) return false;
        if (prev_done >= cfirst[at]) return false;
        // the step's completion point: the whole job, or the stage-2 jobs
        const long long finish_from = q.split ? s2first[at] : cfirst[at];
        if (q.split && (s1last[at] == none || s2first[at] == none || s1last[at] >= s2first[at])) return false;
        if (k >= 1 && (fpos[idx(k - 1, n)] >= finish_from || clast[idx(k - 1, n)] >= finish_from)) return false;
        if (!copies_before(finish_from)) return false;
      }
  }
  return true;
}

// Dependency graph of the jobs of several problems, as the device waits for
// them: per job its duration estimate (us) and the jobs it waits for.
struct JobDag {
  std::vector<ap::PipeJob> job;
  std::vector<double> dur;
  std::vector<char> virt;        // 1: a join point (no job, no workgroup; its duration is work that the
                                 // last job to reach it does before its successors may start)
  std::vector<int> pred_begin;   // CSR: preds of node i at pred[pred_begin[i] .. pred_begin[i+1])
  std::vector<int> pred;
};

// Appends the jobs of one problem in a topological order (level by level:
// its coarse steps and copies, then its fine jobs) with their dependencies.
//   copy C(k,n), n <= k:  C(k-1,n); for n = k also F(k-1,k)
//   whole C(k,n):         C(k,n-1); for k >= 1 also F(k-1,n), C(k-1,n)
//   stage 1 of C(k,n):    C(k,n-1)
//   stage 2 of C(k,n):    every stage-1 job of the step, and (any stage-2 job
//                         may finish the step) for k >= 1 F(k-1,n), C(k-1,n)
//   fine F(k,n..n+g-1):   C(k,n+g-2) (its last input; the chain orders the rest)
// C(k,n) is complete when its whole or copy job, or every stage-2 job, is.
// With a tolerance, the jobs completing C(k,Ns) also wait for the copies of
// level k (they read their residual parts).  A split step gets two join
// points (after its stage-1 jobs, with the midpoint state the last of them
// forms; after its stage-2 jobs, its completion), so that the graph has a few
// edges per job instead of one per pair of group jobs.
void problem_dag(int prob, const PipeShape& q, JobDag& d) {
  const JobCost jc = job_cost(q);
  const int Ns = q.Ns, K = q.K, fg = std::max(1, q.fg);
  const size_t cells = size_t(K + 1) * Ns;
  std::vector<int> cnode(cells, -1), fjob(cells, -1);   // node completing C(k,n); fine job of F(k,n)
  auto at = [&](int k, int n) { return size_t(k) * Ns + n - 1; };
  std::vector<int> deps;
  auto comp = [&](int k, int n) { deps.push_back(cnode[at(k, n)]); };
  auto copies = [&](int k, int n) {
    if (!(q.tol > 0.0) || !q.skip || k < 1 || n != Ns) return;
    for (int m = 1; m <= std::min(k, Ns - 1); ++m) comp(k, m);
  };
  auto add = [&](ap::PipeJob j, double dur, bool v) {
    d.job.push_back(j);
    d.dur.push_back(dur);
    d.virt.push_back(v ? 1 : 0);
    d.pred.insert(d.pred.end(), deps.begin(), deps.end());
    d.pred_begin.push_back(int(d.pred.size()));
    deps.clear();
    return int(d.job.size()) - 1;
  };
  for (int k = 0; k <= K; ++k) {
    for (int n = 1; n <= Ns; ++n) {
      if (q.skip && k >= 1 && n <= k) {
        comp(k - 1, n);
        if (n == k) deps.push_back(fjob[at(k - 1, n)]);
        copies(k, n);
        cnode[at(k, n)] = add({prob, ap::kJobCopy, k, n, 0}, 1.0, false);
        continue;
      }
      if (q.split) {
        const int first = int(d.job.size());
        for (int g = 0; g < q.groups; ++g) {
          if (n > 1) comp(k, n - 1);
          add({prob, ap::kJobStage1, k, n, g}, jc.stage1, false);
        }
        for (int g = 0; g < q.groups; ++g) deps.push_back(first + g);
        const int j1 = add({prob, ap::kJobStage1, k, n, -1}, jc.mid, true);
        const int s2 = int(d.job.size());
        for (int g = 0; g < q.groups; ++g) {
          deps.push_back(j1);
          if (k >= 1) {
            deps.push_back(fjob[at(k - 1, n)]);
            comp(k - 1, n);
          }
          copies(k, n);
          add({prob, ap::kJobStage2, k, n, g}, jc.stage2 + jc.finish, false);
        }
        for (int g = 0; g < q.groups; ++g) deps.push_back(s2 + g);
        cnode[at(k, n)] = add({prob, ap::kJobStage2, k, n, -1}, 0.0, true);
      } else {
        if (n > 1) comp(k, n - 1);
        if (k >= 1) {
          deps.push_back(fjob[at(k - 1, n)]);
          comp(k - 1, n);
        }
        copies(k, n);
        cnode[at(k, n)] = add({prob, ap::kJobCoarse, k, n, 0}, jc.whole, false);
      }
    }
    if (k == K) break;
    for (int n = q.skip && k >= 1 ? k + 1 : 1; n <= Ns; n += fg) {
      const int g = std::min(fg, Ns - n + 1);
      if (n + g - 2 >= 1) comp(k, n + g - 2);
      const int i = add({prob, ap::kJobFine, k, n, g}, jc.fine, false);
      for (int x = 0; x < g; ++x) fjob[at(k, n + x)] = i;
    }
  }
}

// Delay assumed between a job's end and the start of a job waiting on it
// (us): the producer's release, the consumer's poll and acquire, and the
// spread of a split step's group jobs.  A single hand-off measures 1.3-3.4 us
// on MI355X; as a scheduling weight, 6 us gave the shortest solves in a scan
// of 0-20 us (N = 256 with 64 slices: 5.19 -> 4.7 ms; N = 1024 with 256
// slices: 17.5 -> 15.6 ms; the 64-problem batch unchanged).  It lengthens
// the chains of many short dependent jobs, so their jobs get priority.
constexpr double kHandoffUs = 6.0;   // the default; aparareal_autotune may pick another per launch

// Hand-out order of the jobs of several problems on `workers` resident
// workgroups: a list schedule simulated with the jobs' duration estimates and
// a hand-off delay kHandoffUs per dependency.  Whenever a workgroup is free
// it takes, among the jobs whose dependencies' results have arrived, the one
// with the longest remaining path to the end of its problem (its own
// duration plus the longest chain of jobs and hand-offs that wait on it, the
// "bottom level"); the jobs are handed out in the order the simulation
// starts them.  Long chains (long fine steps or many slices) thus start
// first and are not stretched by the jobs of short problems, while every
// workgroup is kept busy.  The order is topological by construction.
std::vector<ap::PipeJob> schedule_jobs(const std::vector<PipeShape>& shapes, int workers,
                                       double handoff = kHandoffUs) {
  JobDag d;
  d.pred_begin.push_back(0);
  for (size_t p = 0; p < shapes.size(); ++p) problem_dag(int(p), shapes[p], d);
  const int nj = int(d.job.size());
  // successors (CSR) and bottom levels (nodes were appended in a topological
  // order); a hand-off delay separates a job from each job that waits on it
  // (through a join point or directly)
  std::vector<int> nsucc(size_t(nj) + 1, 0), npred(nj, 0);
  for (int i = 0; i < nj; ++i) {
    npred[i] = d.pred_begin[i + 1] - d.pred_begin[i];
    for (int x = d.pred_begin[i]; x < d.pred_begin[i + 1]; ++x) ++nsucc[d.pred[x] + 1];
  }
  for (int i = 0; i < nj; ++i) nsucc[i + 1] += nsucc[i];
  std::vector<int> succ(d.pred.size()), fill(nsucc.begin(), nsucc.end() - 1);
  for (int i = 0; i < nj; ++i)
    for (int x = d.pred_begin[i]; x < d.pred_begin[i + 1]; ++x) succ[fill[d.pred[x]]++] = i;
  auto edge = [&](int to) { return d.virt[to] ? 0.0 : handoff; };
  std::vector<double> bl(nj, 0.0);
  for (int i = nj - 1; i >= 0; --i) {
    double m = 0.0;
    for (int x = nsucc[i]; x < nsucc[i + 1]; ++x) m = std::max(m, edge(succ[x]) + bl[succ[x]]);
    bl[i] = d.dur[i] + m;
  }
  // event simulation: ready jobs by bottom level (ties: earlier in the list),
  // running jobs by end time, jobs waiting for their inputs to arrive by time
  auto later = [&](int a, int b) { return bl[a] != bl[b] ? bl[a] < bl[b] : a > b; };
  std::priority_queue<int, std::vector<int>, decltype(later)> ready(later);
  using Ev = std::pair<double, int>;
  std::priority_queue<Ev, std::vector<Ev>, std::greater<Ev>> running;
  // Jobs whose dependencies have completed, waiting for the results to
  // arrive: a job released at event time t gets t + kHandoffUs, and events
  // are processed in time order, so this queue is in time order already.
  std::deque<Ev> pending;
  std::vector<double> avail(nj, 0.0);   // when the last dependency's result reaches the node
  std::vector<Ev> stack;
  // node i has completed at time t: release its successors (join points
  // complete at once, without a workgroup)
  auto complete = [&](int i, double t) {
    stack.assign(1, Ev{t, i});
    while (!stack.empty()) {
      const int u = stack.back().second;
      const double tu = stack.back().first;
      stack.pop_back();
      for (int x = nsucc[u]; x < nsucc[u + 1]; ++x) {
        const int v = succ[x];
        avail[v] = std::max(avail[v], tu + edge(v));
        if (--npred[v] > 0) continue;
        if (d.virt[v]) {
          stack.push_back({avail[v] + d.dur[v], v});
        } else {
          pending.push_back({avail[v], v});
        }
      }
    }
  };
  for (int i = 0; i < nj; ++i)
    if (npred[i] == 0) {
      if (d.virt[i]) complete(i, d.dur[i]);
      else pending.push_back({0.0, i});
    }
  std::vector<ap::PipeJob> out;
  int njobs = 0;
  for (int i = 0; i < nj; ++i) njobs += d.virt[i] ? 0 : 1;
  out.reserve(njobs);
  const int W = std::max(1, workers);
  int busy = 0;
  double now = 0.0;
  while (int(out.size()) < njobs) {
    while (!pending.empty() && pending.front().first <= now) {
      ready.push(pending.front().second);
      pending.pop_front();
    }
    while (busy < W && !ready.empty()) {
      const int i = ready.top();
      ready.pop();
      out.push_back(d.job[i]);
      running.push({now + d.dur[i], i});
      ++busy;
    }
    // next event: a job ends, or (with a free workgroup) a waiting job's inputs arrive
    double next = running.empty() ? std::numeric_limits<double>::infinity() : running.top().first;
    if (busy < W && !pending.empty()) next = std::min(next, pending.front().first);
    if (!(next < std::numeric_limits<double>::infinity())) return {};   // a cycle: cannot happen
    now = next;
    while (!running.empty() && running.top().first <= now) {
      const int i = running.top().second;
      running.pop();
      --busy;
      complete(i, now);
    }
  }
  return out;
}

// Workgroups assumed by the host-only schedule queries (one per CU of an MI355X).
constexpr int kQueryWorkers = 256;

// ---------------------------------------------------------- pipelined solve -
// One problem of a pipelined launch: its context (tables, per-problem device
// workspace), arguments and derived sizes.
struct PlanItem {
  ap_ctx* c = nullptr;
  const double* u0 = nullptr;
  ap_solve_params p{};
  double* U_out = nullptr;
  double* resid = nullptr;
  FineTables* ft = nullptr;
  AvgTables* at = nullptr;
  FineTables* cft = nullptr;   // Strang coarse: tables for h = dT
  PipeShape q;
};

// Validates the solve parameters and derives the problem's shape and tables.
int plan_item(ap_ctx* c, const double* u0, const ap_solve_params* p, double* U_out, double* resid, PlanItem* it) {
  int rc = check_ctx(c);
  if (rc) return rc;
  if (!p || !u0 || !U_out) return fail(AP_EINVAL, "null argument");
  if ((rc = check_prec(p->precision))) return rc;
  if (!(p->T > 0.0) || !std::isfinite(p->T)) return fail(AP_EINVAL, "T must be > 0");
  if (p->slices < 1) return fail(AP_EINVAL, "slices must be >= 1");
  if (p->K < 0) return fail(AP_EINVAL, "K must be >= 0");
  if (p->K > 0 && !resid) return fail(AP_EINVAL, "resid must hold K entries");
  if (!(p->dt_fine > 0.0) || !std::isfinite(p->dt_fine)) return fail(AP_EINVAL, "dt_fine must be > 0");
  if (p->M_avg < 2) return fail(AP_EINVAL, "M_avg must be >= 2");
  if (!std::isfinite(p->T0) || !std::isfinite(p->tol)) return fail(AP_EINVAL, "T0, tol must be finite");
  if (size_t(2 * p->K + 1) * size_t(p->slices) > (size_t(1) << 30)) return fail(AP_EINVAL, "problem too large");
  const int Ns = p->slices;
  const double dT = p->T / Ns;
  const double ratio = dT / p->dt_fine;
  if (ratio > 1e7) return fail(AP_EINVAL, "dT/dt_fine too large");
  const int steps = std::max(1, int(std::ceil(ratio - 1e-9)));
  const double win = p->T0 > 0.0 ? p->T0 : dT / c->eps;
  it->c = c;
  it->u0 = u0;
  it->p = *p;
  it->U_out = U_out;
  it->resid = resid;
  if ((rc = fine_tables(c, dT / steps, &it->ft))) return rc;
  if ((rc = avg_tables(c, dT, win, p->M_avg, &it->at))) return rc;
  PipeShape& q = it->q;
  q.nx = c->N;
  q.Ns = Ns;
  q.K = p->K;
  q.steps = steps;
  q.M = p->M_avg;
  q.gs = group_size(c);
  q.groups = ap::avg_groups(q.M, q.gs);
  q.fp64 = p->precision == AP_PREC_FP64;
  q.split = c->opt_split < 0 ? q.groups >= 2 : c->opt_split != 0;
  q.fine_kind = c->opt_fine;
  q.coarse_kind = c->opt_coarse;
  if (q.coarse_kind == 1) {
    q.split = false;                       // one Strang step: nothing to split
    if ((rc = fine_tables(c, dT, &it->cft))) return rc;
  }
  q.cal = c->cost;
  q.skip = c->opt_skip != 0;
  q.tol = p->tol > 0.0 ? p->tol : 0.0;
  return AP_OK;
}

template <typename T>
ap::PipeProb<T> make_prob(const PlanItem& it, int* cnt);
template <>
ap::PipeProb<double> make_prob<double>(const PlanItem& it, int* cnt) {
  ap_ctx* c = it.c;
  return ap::PipeProb<double>{c->pp_U.as<cx<double>>(), c->pp_F.as<cx<double>>(), c->pp_G.as<cx<double>>(),
                              c->pp_part.as<double2>(), cnt, c->pp_P1.as<cx<double>>(), c->pp_P2.as<cx<double>>(),
                              it.q.nx, it.q.Ns, it.q.K, it.q.steps, it.q.groups, it.q.fine_kind, it.q.coarse_kind,
                              it.p.T / it.q.Ns / it.q.steps, it.p.T / it.q.Ns,
                              it.cft ? it.cft->coef64.as<cx<double>>() : nullptr, it.q.tol,
                              it.ft->coef64.as<cx<double>>(), it.ft->coef64.as<cx<double>>(), it.at->c64,
                              c->tabs.tw64, c->tabs.basis64};
}
template <>
ap::PipeProb<float> make_prob<float>(const PlanItem& it, int* cnt) {
  ap_ctx* c = it.c;
  return ap::PipeProb<float>{c->pp_U.as<cx<double>>(), c->pp_F.as<cx<double>>(), c->pp_G.as<cx<double>>(),
                             c->pp_part.as<double2>(), cnt, c->pp_P1.as<cx<float>>(), c->pp_P2.as<cx<float>>(),
                             it.q.nx, it.q.Ns, it.q.K, it.q.steps, it.q.groups, it.q.fine_kind, it.q.coarse_kind,
                             it.p.T / it.q.Ns / it.q.steps, it.p.T / it.q.Ns,
                             it.cft ? it.cft->coef64.as<cx<double>>() : nullptr, it.q.tol,
                             it.ft->coef64.as<cx<double>>(), it.ft->coef32.as<cx<float>>(), it.at->c32,
                             c->tabs.tw32, c->tabs.basis32};
}

// Uploads `bytes` to a device buffer only when they differ from what it holds
// (the host copy `last`); the device buffer is in use by earlier launches on
// the owner's stream, so that stream is drained first.
hipError_t upload_if_changed(ap_ctx* owner, DevBuf& dev, std::vector<unsigned char>& last,
                             const std::vector<unsigned char>& bytes) {
  if (dev.p && last == bytes) return hipSuccess;
  hipError_t e = ensure(owner, dev, std::max<size_t>(bytes.size(), 1));
  if (e != hipSuccess) return e;
  if (owner->has_last && (e = hipStreamSynchronize(owner->last_stream)) != hipSuccess) return e;
  if (!bytes.empty() && (e = hipMemcpy(dev.p, bytes.data(), bytes.size(), hipMemcpyHostToDevice)) != hipSuccess)
    return e;
  last = bytes;
  return hipSuccess;
}

template <typename V>
std::vector<unsigned char> as_bytes(const std::vector<V>& v) {
  std::vector<unsigned char> b(v.size() * sizeof(V));
  if (!v.empty()) std::memcpy(b.data(), v.data(), b.size());
  return b;
}

// Runs the problems of `items` (same precision, distinct contexts) as one
// persistent launch on stream s.  `owner` holds the launch's job list,
// descriptors and counters; each item's context holds its problem's states.
int plan_launch(ap_ctx* owner, std::vector<PlanItem>& items, hipStream_t s) {
  hipError_t e;
  const bool f64 = items[0].q.fp64;
  std::vector<PipeShape> shapes;
  long long ncnt = 0;
  int nx_common = items[0].q.nx, nx_max = 0;
  for (auto& it : items) {
    const PipeShape& q = it.q;
    if (q.fp64 != f64) return fail(AP_EINVAL, "all problems of a batch need the same precision");
    ap_ctx* c = it.c;
    const size_t sb = state_bytes(c);
    const size_t pb = size_t(3) * c->KP * (f64 ? sizeof(cx<double>) : sizeof(cx<float>));
    // stage-1 sums and the midpoint state per level; stage-2 sums per level
    const size_t p1bytes = q.split ? pb * size_t(q.K + 1) * (q.groups + 1) : pb;
    const size_t p2bytes = q.split ? pb * size_t(q.K + 1) * q.groups : pb;
    if ((e = ensure(c, c->pp_U, sb * size_t(q.K + 1) * (q.Ns + 1))) != hipSuccess ||
        (e = ensure(c, c->pp_F, sb * size_t(std::max(q.K, 1)) * (q.Ns + 1))) != hipSuccess ||
        (e = ensure(c, c->pp_G, sb * size_t(q.K + 1) * (q.Ns + 1))) != hipSuccess ||
        (e = ensure(c, c->pp_part, sizeof(double2) * size_t(q.Ns) * std::max(1, q.K))) != hipSuccess ||
        (e = ensure(c, c->pp_P1, p1bytes)) != hipSuccess || (e = ensure(c, c->pp_P2, p2bytes)) != hipSuccess)
      return hip_fail(e, "pipeline workspace");
    shapes.push_back(q);
    ncnt += ap::pipe_counters(q.Ns, q.K);
    if (q.nx != nx_common) nx_common = 0;
    nx_max = std::max(nx_max, q.nx);
  }
  if (ncnt > (1LL << 30)) return fail(AP_EINVAL, "batch too large");
  // resident workgroups of the launch
  int grid = ap::pipeline_max_grid(nx_common, nx_max, f64);
  if (grid <= 0) return fail(AP_EDEVICE, "pipeline kernel does not fit the device");
  if (owner->opt_grid > 0) grid = std::min(grid, owner->opt_grid);
  // Slices per fine job: stepping several slices in one workgroup costs a job
  // about what one slice costs, but a group starts only when its last input
  // is ready.  Automatic: one slice while the batch's slices fit the resident
  // workgroups (the solve is latency-bound), else the most per grid size.
  long long slices_total = 0;
  for (auto& it : items) slices_total += it.q.Ns;
  for (size_t i = 0; i < items.size(); ++i) {
    const int jm = ap::pipeline_fine_slices(items[i].q.nx, f64, items[i].q.fine_kind);
    const int want = items[i].c->opt_fine_group;
    items[i].q.fg = want > 0 ? std::min(want, jm) : (slices_total > grid ? jm : 1);
    shapes[i].fg = items[i].q.fg;
  }
  // counters, then ticket, stall record [4] (stalled, job, counter, jobs
  // completed), per-workgroup progress [2][1024]
  const long long nflags = ncnt + 5 + 2 * 1024;
  if ((e = ensure(owner, owner->pp_flags, sizeof(int) * size_t(nflags))) != hipSuccess)
    return hip_fail(e, "pipeline counters");
  int* flags = owner->pp_flags.as<int>();
  int* ticket = flags + ncnt;
  int* abort = ticket + 1;
  // job list, cached by the problems' shapes
  std::string key = std::to_string(grid) + ":" + std::to_string(owner->handoff_ns) + "|";
  for (auto& q : shapes)
    key += std::to_string(q.nx) + ":" + std::to_string(q.Ns) + ":" + std::to_string(q.K) + ":" +
           std::to_string(q.steps) + ":" + std::to_string(q.M) + ":" + std::to_string(q.gs) + ":" +
           std::to_string(int(q.split)) + ":" + std::to_string(int(q.fp64)) + ":" + std::to_string(int(q.skip)) + ":" +
           std::to_string(q.fine_kind) + std::to_string(q.coarse_kind) + ":" + std::to_string(q.fg) + ":" +
           (q.cal.valid ? std::to_string(q.cal.fine_step) + "," + std::to_string(q.cal.stage1) + "," +
                              std::to_string(q.cal.stage2) + "," + std::to_string(q.cal.whole)
                        : std::string("-")) + ";";
  if (key != owner->pp_jobs_key) {
    std::vector<ap::PipeJob> jobs = schedule_jobs(shapes, grid, owner->handoff_ns * 1e-3);
    if (!order_is_valid(jobs, shapes)) return fail(AP_EINVAL, "internal: job order is not topological");
    if (jobs.size() > size_t(1) << 30) return fail(AP_EINVAL, "batch too large");
    owner->pp_jobs_key.clear();
    std::vector<unsigned char> last;
    if ((e = upload_if_changed(owner, owner->pp_jobs, last, as_bytes(jobs))) != hipSuccess)
      return hip_fail(e, "job list upload");
    owner->pp_jobs_host = std::move(jobs);
    owner->pp_njobs = int(owner->pp_jobs_host.size());
    owner->pp_jobs_key = key;
  }
  // descriptors and residual rows
  std::vector<ap::ResidRow> rows;
  std::vector<unsigned char> probs;
  long long off = 0;
  for (auto& it : items) {
    int* cnt = flags + off;
    off += ap::pipe_counters(it.q.Ns, it.q.K);
    if (f64) {
      const ap::PipeProb<double> pr = make_prob<double>(it, cnt);
      const auto* b = reinterpret_cast<const unsigned char*>(&pr);
      probs.insert(probs.end(), b, b + sizeof(pr));
    } else {
      const ap::PipeProb<float> pr = make_prob<float>(it, cnt);
      const auto* b = reinterpret_cast<const unsigned char*>(&pr);
      probs.insert(probs.end(), b, b + sizeof(pr));
    }
    const int* stop = it.q.tol > 0.0 ? cnt + ap::pipe_stop_index(it.q.Ns, it.q.K) : nullptr;
    for (int k = 0; k < it.q.K; ++k)
      rows.push_back({it.c->pp_part.as<double2>() + size_t(k) * it.q.Ns, it.resid + k, stop, it.q.Ns, k + 1});
  }
  if ((e = upload_if_changed(owner, owner->pp_prob, owner->pp_prob_host, probs)) != hipSuccess)
    return hip_fail(e, "problem descriptor upload");
  if ((e = upload_if_changed(owner, owner->pp_rows, owner->pp_rows_host, as_bytes(rows))) != hipSuccess)
    return hip_fail(e, "residual table upload");
  // Boundary transforms of a batch: one launch per grid size (and per
  // kBoundaryBatch problems) instead of one per problem, the problems' states
  // passed by value as the launch's argument.  The modal initial state also
  // goes to U(K, 0), the last level's slice 0.  A single problem keeps the
  // direct launches.
  const bool bnd_batched = items.size() > 1;
  struct BndLaunch {
    int nx;
    ap::BoundaryBatch b;
  };
  std::vector<BndLaunch> bnd_in, bnd_out;
  if (bnd_batched) {
    std::vector<int> sizes;
    for (auto& it : items)
      if (std::find(sizes.begin(), sizes.end(), it.q.nx) == sizes.end()) sizes.push_back(it.q.nx);
    // appends a problem of `states` states (a workgroup each) to the open
    // launch of size nx in v, opening a new one when needed
    auto add = [](std::vector<BndLaunch>& v, int nx, const ap::BoundaryJob& jb, int states) {
      if (v.empty() || v.back().nx != nx || v.back().b.n == ap::kBoundaryBatch) {
        v.push_back(BndLaunch{nx, {}});
        v.back().b.n = 0;
        v.back().b.first[0] = 0;
      }
      ap::BoundaryBatch& b = v.back().b;
      b.job[b.n] = jb;
      b.first[b.n + 1] = b.first[b.n] + states;
      b.n += 1;
    };
    for (int nx : sizes)
      for (auto& it : items) {
        if (it.q.nx != nx) continue;
        ap_ctx* c = it.c;
        cx<double>* U = c->pp_U.as<cx<double>>();
        const size_t st = size_t(3) * c->KP;
        cx<double>* UK0 = it.q.K > 0 ? U + size_t(it.q.K) * (it.q.Ns + 1) * st : nullptr;
        add(bnd_in, nx, ap::BoundaryJob{it.u0, U, UK0, c->tabs.tw64, c->tabs.basis64}, 1);
        const cx<double>* UK = U + size_t(it.q.K) * (it.q.Ns + 1) * st;
        add(bnd_out, nx, ap::BoundaryJob{UK, it.U_out, nullptr, c->tabs.tw64, c->tabs.basis64}, it.q.Ns + 1);
      }
  }
  grid = std::max(1, std::min({grid, owner->pp_njobs, 1024}));   // progress record holds 1024 workgroups
  unsigned long long* trace = nullptr;
  if (owner->trace_on) {
    if ((e = ensure(owner, owner->pp_trace, sizeof(unsigned long long) * 3 * size_t(owner->pp_njobs))) !=
        hipSuccess)
      return hip_fail(e, "trace buffer");
    trace = owner->pp_trace.as<unsigned long long>();
    owner->pp_trace_jobs = owner->pp_njobs;
  }
  // enqueue: boundary transforms in, counters, the persistent launch,
  // residuals, boundary transforms out (kernels and device copies only, so
  // that the sequence can be captured into a graph)
  owner->pp_diag = abort;
  auto enqueue = [&](hipStream_t st, bool time_it) -> int {
    auto run = [&](int cls, auto&& fn) { return time_it ? timed(owner, cls, st, fn) : fn(); };
    hipError_t err;
    for (const BndLaunch& g : bnd_in) {
      err = run(AP_K_TO_MODAL, [&] { return ap::launch_to_modal_batch(g.nx, g.b, st); });
      if (err != hipSuccess) return hip_fail(err, "to_modal");
    }
    for (auto& it : items) {
      if (bnd_batched) break;
      ap_ctx* c = it.c;
      cx<double>* U = c->pp_U.as<cx<double>>();
      const size_t sb = state_bytes(c);
      err = run(AP_K_TO_MODAL, [&] { return ap::launch_to_modal(c->N, it.u0, U, 1, c->tabs, st); });
      if (err != hipSuccess) return hip_fail(err, "to_modal");
      if (it.q.K > 0 &&
          (err = hipMemcpyAsync(U + size_t(it.q.K) * (it.q.Ns + 1) * (sb / sizeof(cx<double>)), U, sb,
                                hipMemcpyDeviceToDevice, st)) != hipSuccess)
        return hip_fail(err, "initial state copy");
    }
    if ((err = ap::launch_zero_ints(flags, int(nflags), st)) != hipSuccess) return hip_fail(err, "counter reset");
    err = run(AP_K_PIPELINE, [&] {
      return ap::launch_pipeline(nx_common, nx_max, f64, owner->pp_jobs.p, owner->pp_njobs, owner->pp_prob.p,
                                 ticket, abort, abort + 4, trace, grid, st);
    });
    if (err != hipSuccess) return hip_fail(err, "pipeline launch");
    if (!rows.empty()) {
      err = run(AP_K_RESID, [&] {
        return ap::launch_resid_rows(owner->pp_rows.as<ap::ResidRow>(), int(rows.size()), abort, st);
      });
      if (err != hipSuccess) return hip_fail(err, "resid");
    }
    long long foff = 0;
    for (auto& it : items) {
      ap_ctx* c = it.c;
      const int* stop = flags + foff + ap::pipe_stop_index(it.q.Ns, it.q.K);
      foff += ap::pipe_counters(it.q.Ns, it.q.K);
      if (it.q.tol > 0.0 && it.q.K > 1 &&
          (err = ap::launch_select_level(c->pp_U.as<cx<double>>(), it.q.Ns, it.q.K, c->KP, stop, st)) !=
              hipSuccess)
        return hip_fail(err, "level selection");
      if (bnd_batched) continue;
      const cx<double>* UK = c->pp_U.as<cx<double>>() + size_t(it.q.K) * (it.q.Ns + 1) * 3 * c->KP;
      err = run(AP_K_TO_PHYSICAL, [&] { return ap::launch_to_physical(c->N, UK, it.U_out, it.q.Ns + 1, c->tabs, st); });
      if (err != hipSuccess) return hip_fail(err, "to_physical");
    }
    for (const BndLaunch& g : bnd_out) {
      err = run(AP_K_TO_PHYSICAL, [&] { return ap::launch_to_physical_batch(g.nx, g.b, st); });
      if (err != hipSuccess) return hip_fail(err, "to_physical");
    }
    return AP_OK;
  };
  if (!owner->opt_graph || trace) return enqueue(s, true);
  // Graph replay: the sequence is captured once per set of device addresses
  // (arguments and workspaces) and launch shape, then replayed; inputs are
  // read from device memory at replay time.
  std::string gkey = key + "|" + std::to_string(grid);
  auto addr = [&](const void* p) { gkey += ":" + std::to_string(reinterpret_cast<uintptr_t>(p)); };
  addr(owner->pp_flags.p);
  addr(owner->pp_jobs.p);
  addr(owner->pp_prob.p);
  addr(owner->pp_rows.p);
  for (auto& it : items) {
    addr(it.c);
    addr(it.u0);
    addr(it.U_out);
    addr(it.resid);
    addr(it.c->pp_U.p);
  }
  if (!owner->graph_exec || gkey != owner->graph_key) {
    if (owner->graph_exec) (void)hipGraphExecDestroy(owner->graph_exec);
    if (owner->graph) (void)hipGraphDestroy(owner->graph);
    owner->graph_exec = nullptr;
    owner->graph = nullptr;
    owner->graph_key.clear();
    if (!owner->graph_stream && (e = hipStreamCreateWithFlags(&owner->graph_stream, hipStreamNonBlocking)) != hipSuccess)
      return hip_fail(e, "graph stream");
    if ((e = hipStreamBeginCapture(owner->graph_stream, hipStreamCaptureModeThreadLocal)) != hipSuccess)
      return hip_fail(e, "graph capture");
    const int rc = enqueue(owner->graph_stream, false);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(owner->graph_stream, &g);
    if (rc) {
      if (g) (void)hipGraphDestroy(g);
      return rc;
    }
    if (e != hipSuccess) return hip_fail(e, "graph capture");
    owner->graph = g;
    if ((e = hipGraphInstantiate(&owner->graph_exec, g, nullptr, nullptr, 0)) != hipSuccess) {
      owner->graph_exec = nullptr;
      return hip_fail(e, "graph instantiation");
    }
    owner->graph_key = gkey;
  }
  e = timed(owner, AP_K_PIPELINE, s, [&] { return hipGraphLaunch(owner->graph_exec, s); });
  if (e != hipSuccess) return hip_fail(e, "graph launch");
  return AP_OK;
}

}  // namespace

namespace aplib {
void set_last_error(const std::string& msg) { g_last_error = msg; }
}  // namespace aplib

extern "C" {

const char* aparareal_last_error(void) { return g_last_error.c_str(); }

ap_ctx* aparareal_create(int N, double eps, double F, double nu) {
  if (!is_pow2(N) || N < 64 || N > 2048) {
    fail(AP_EINVAL, "N must be a power of two in [64, 2048]");
    return nullptr;
  }
  if (!(eps > 0.0) || !(F > 0.0) || !(nu >= 0.0) || !std::isfinite(eps) || !std::isfinite(F) ||
      !std::isfinite(nu)) {
    fail(AP_EINVAL, "need eps > 0, F > 0, nu >= 0 (finite)");
    return nullptr;
  }
  auto c = std::make_unique<ap_ctx>();
  c->N = N;
  c->KD = N / 3;
  c->KP = c->KD + 1;
  c->eps = eps;
  c->F = F;
  c->nu = nu;
  hipError_t e = hipGetDevice(&c->device);
  if (e != hipSuccess) {
    hip_fail(e, "hipGetDevice");
    return nullptr;
  }
  c->device_key = device_key(c->device);
  for (int prec = 0; prec < 2; ++prec) c->tuned_shape[prec] = tune_lookup(c->device_key, N, prec);
  c->omega.resize(c->KP);
  c->akw.resize(c->KP);
  c->na_t64.resize(size_t(8) * 3 * c->KP);
  c->na_t32.resize(size_t(8) * 3 * c->KP);
  std::vector<ap::Basis<double>> b64(c->KP);
  std::vector<ap::Basis<float>> b32(c->KP);
  for (int k = 0; k < c->KP; ++k) {
    const double a = double(k) / std::sqrt(F);
    const double w = std::sqrt(1.0 + a * a);
    c->omega[k] = w;
    c->akw[k] = a / w;
    b64[k] = {1.0 / w, a / w};
    b32[k] = {float(1.0 / w), float(a / w)};
  }
  // twiddles, per FFT plan: exp(-2 pi i t/N), t < N, then the per-pass
  // tables of the wave-local FFT of length N/2 (exp(-2 pi i q k/(NS R)) at
  // (q-1) NS + k); plan 1's table (where there is one) follows plan 0's
  std::vector<cx<double>> t64;
  std::vector<cx<float>> t32;
  auto push = [&](double th) {
    t64.push_back(cx<double>{std::cos(th), -std::sin(th)});
    t32.push_back(cx<float>{float(std::cos(th)), float(-std::sin(th))});
  };
  for (int plan = 0; plan < ap::wave_plans(N / 2); ++plan) {
    if (plan == 1) c->tabs.tw_plan1 = int(t64.size());
    for (int t = 0; t < N; ++t) push(2.0 * M_PI * double(t) / double(N));
    int r[4], npass = 0;
    ap::wave_plan_radices(N / 2, r, &npass, plan);
    int NS = r[0];
    for (int j = 1; j < npass; ++j) {
      const int R = r[j];
      for (int q = 1; q < R; ++q)
        for (int k = 0; k < NS; ++k) push(2.0 * M_PI * double(q) * double(k) / double(NS * R));
      NS *= R;
    }
  }
  if ((e = c->tw64.upload(t64)) != hipSuccess || (e = c->tw32.upload(t32)) != hipSuccess ||
      (e = c->basis64.upload(b64)) != hipSuccess || (e = c->basis32.upload(b32)) != hipSuccess) {
    hip_fail(e, "table upload");
    return nullptr;
  }
  c->tabs.tw64 = c->tw64.as<cx<double>>();
  c->tabs.tw32 = c->tw32.as<cx<float>>();
  c->tabs.basis64 = c->basis64.as<ap::Basis<double>>();
  c->tabs.basis32 = c->basis32.as<ap::Basis<float>>();
  g_last_error.clear();
  return c.release();
}

int aparareal_destroy(ap_ctx* c) {
  if (!c) return fail(AP_EINVAL, "null context");
  (void)hipDeviceSynchronize();
  delete c;
  return AP_OK;
}

int aparareal_nonlinear(ap_ctx* c, const double* U_in, double* N_out, int batch, int precision, void* stream) {
  hipStream_t s = static_cast<hipStream_t>(stream);
  int rc = batch_prologue(c, U_in, N_out, batch, precision, s);
  if (rc || batch == 0) return rc;
  hipError_t e = timed(c, AP_K_NONLINEAR, s, [&] {
    return ap::launch_nonlinear(c->N, precision == AP_PREC_FP64, c->ws_in.as<cx<double>>(),
                                c->ws_out.as<cx<double>>(), batch, c->tabs, s);
  });
  if (e != hipSuccess) return hip_fail(e, "nonlinear launch");
  return batch_epilogue(c, N_out, batch, s);
}

int aparareal_fine_batch(ap_ctx* c, const double* U_in, double* U_out, int batch, double dT, int steps,
                         int precision, void* stream) {
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (c && !(dT > 0.0 && std::isfinite(dT))) return fail(AP_EINVAL, "dT must be > 0");
  if (c && steps < 1) return fail(AP_EINVAL, "steps must be >= 1");
  if (c && U_in && U_in == U_out) return fail(AP_EINVAL, "U_out may not alias U_in");
  int rc = batch_prologue(c, U_in, U_out, batch, precision, s);
  if (rc || batch == 0) return rc;
  FineTables* ft = nullptr;
  if ((rc = fine_tables(c, dT / steps, &ft))) return rc;
  const bool f64 = precision == AP_PREC_FP64;
  hipError_t e = timed(c, AP_K_FINE, s, [&] {
    return ap::launch_fine(c->N, f64, c->ws_in.as<cx<double>>(), c->ws_out.as<cx<double>>(), batch, steps,
                           ft->coef64.as<cx<double>>(), ft->coef32.as<cx<float>>(), c->tabs, s,
                           fine_shape_of(c, precision));
  });
  if (e != hipSuccess) return hip_fail(e, "fine launch");
  return batch_epilogue(c, U_out, batch, s);
}

int aparareal_measure_peaks(void* stream, double* fp32_tflops, double* fp64_tflops, double* lds_tbps) {
  if (!fp32_tflops || !fp64_tflops || !lds_tbps) return fail(AP_EINVAL, "null output");
  hipStream_t s = static_cast<hipStream_t>(stream);
  int dev = 0, cus = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return hip_fail(e, "device query");
  const size_t bytes = size_t(cus) * 16 * 256 * sizeof(double);
  void* scratch = nullptr;
  if ((e = hipMalloc(&scratch, bytes)) != hipSuccess) return hip_fail(e, "peak scratch");
  e = ap::measure_peaks(scratch, bytes, s, fp32_tflops, fp64_tflops, lds_tbps);
  const hipError_t f = hipFree(scratch);
  if (e != hipSuccess) return hip_fail(e, "peak kernels");
  if (f != hipSuccess) return hip_fail(f, "peak scratch free");
  return AP_OK;
}

int aparareal_fine_shape(ap_ctx* c, int precision, int* shape, int* threads, int* slices) {
  int rc = check_ctx(c);
  if (rc) return rc;
  if ((rc = check_prec(precision))) return rc;
  const int sh = fine_shape_of(c, precision);
  int j = 0;
  const int nt = ap::fine_shape(c->N, precision == AP_PREC_FP64, sh, &j);
  if (shape) *shape = sh;
  if (threads) *threads = nt;
  if (slices) *slices = j;
  return AP_OK;
}

int aparareal_fft_plan(int N, int plan, int* radices, int* passes, int* reg_exchanges) {
  if (N < 64 || N > 2048 || (N & (N - 1)) != 0) return fail(AP_EINVAL, "N must be a power of two in [64, 2048]");
  if (plan < 0 || plan >= ap::wave_plans(N / 2)) return fail(AP_EINVAL, "no such FFT plan for this N");
  int r[4], n = 0, x = 0;
  ap::wave_plan_radices(N / 2, r, &n, plan, &x);
  if (radices)
    for (int i = 0; i < 4; ++i) radices[i] = i < n ? r[i] : 1;
  if (passes) *passes = n;
  if (reg_exchanges) *reg_exchanges = x;
  return AP_OK;
}

int aparareal_autotune_fine(ap_ctx* c, const double* U_in, int batch, double dT, int steps, int precision,
                            void* stream, double* shape_ms, int* best) {
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (c && !(dT > 0.0 && std::isfinite(dT))) return fail(AP_EINVAL, "dT must be > 0");
  if (c && steps < 1) return fail(AP_EINVAL, "steps must be >= 1");
  if (c && batch < 1) return fail(AP_EINVAL, "batch must be >= 1");
  // the prologue checks an output pointer; the tuning runs write only the workspace
  int rc = batch_prologue(c, U_in, const_cast<double*>(U_in), batch, precision, s);
  if (rc) return rc;
  FineTables* ft = nullptr;
  if ((rc = fine_tables(c, dT / steps, &ft))) return rc;
  const bool f64 = precision == AP_PREC_FP64;
  hipEvent_t a = nullptr, b = nullptr;
  hipError_t e = hipEventCreate(&a);
  if (e == hipSuccess) e = hipEventCreate(&b);
  double ms[ap::kFineConfigCount];
  int pick = 0;
  for (int sh = 0; e == hipSuccess && sh < ap::kFineConfigCount; ++sh) {
    ms[sh] = -1.0;
    if (!fine_config_valid(c->N, sh)) continue;
    auto run = [&] {
      return ap::launch_fine(c->N, f64, c->ws_in.as<cx<double>>(), c->ws_out.as<cx<double>>(), batch, steps,
                             ft->coef64.as<cx<double>>(), ft->coef32.as<cx<float>>(), c->tabs, s, sh);
    };
    e = run();                                   // warm-up
    if (e == hipSuccess) e = hipEventRecord(a, s);
    for (int r = 0; e == hipSuccess && r < 3; ++r) e = run();
    if (e == hipSuccess) e = hipEventRecord(b, s);
    if (e == hipSuccess) e = hipEventSynchronize(b);
    float el = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&el, a, b);
    ms[sh] = double(el) / 3.0;
    if (e == hipSuccess && ms[sh] < ms[pick]) pick = sh;
  }
  if (a) (void)hipEventDestroy(a);
  if (b) (void)hipEventDestroy(b);
  if (e != hipSuccess) return hip_fail(e, "fine configuration tuning");
  c->tuned_shape[f64 ? 1 : 0] = pick;
  tune_store(c->device_key, c->N, precision, pick);
  if (shape_ms)
    for (int sh = 0; sh < ap::kFineConfigCount; ++sh) shape_ms[sh] = ms[sh];
  if (best) *best = pick;
  return AP_OK;
}

// The fine batch with every scratch byte in the library's per-device scratch
// array: the coefficient tables of the step size, then the modal input and
// output states.  Nothing is allocated, on the device or on the host.
int aparareal_fine_batch_noalloc(ap_ctx* c, const double* U_in, double* U_out, int batch, double dT, int steps,
                                 int precision, void* stream) {
  hipStream_t s = static_cast<hipStream_t>(stream);
  int rc = check_ctx(c);
  if (rc) return rc;
  if ((rc = check_prec(precision))) return rc;
  if (!(dT > 0.0 && std::isfinite(dT))) return fail(AP_EINVAL, "dT must be > 0");
  if (steps < 1) return fail(AP_EINVAL, "steps must be >= 1");
  if (batch < 0) return fail(AP_EINVAL, "batch must be >= 0");
  if (batch > 0 && (!U_in || !U_out)) return fail(AP_EINVAL, "null array");
  if (U_in && U_in == U_out) return fail(AP_EINVAL, "U_out may not alias U_in");
  auto up256 = [](size_t b) { return (b + 255) / 256 * 256; };
  const size_t b64 = c->na_t64.size() * sizeof(cx<double>), b32 = c->na_t32.size() * sizeof(cx<float>);
  const size_t fixed = up256(b64) + up256(b32);
  const size_t per_state = 2 * state_bytes(c);
  const size_t max_batch = (ap::kNoAllocScratchBytes - fixed - 512) / per_state;
  if (size_t(batch) > max_batch)
    return fail(AP_EINVAL, "batch of " + std::to_string(batch) + " states exceeds the scratch: at most " +
                               std::to_string(max_batch) + " states of N = " + std::to_string(c->N));
  int cur = -1;
  hipError_t e = hipGetDevice(&cur);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if (cur != c->device) return fail(AP_EINVAL, "the context's device must be the current device");
  void* base = nullptr;
  if ((e = ap::noalloc_scratch(c->device, &base)) != hipSuccess) return hip_fail(e, "scratch address");
  if ((e = order_stream(c, s)) != hipSuccess) return hip_fail(e, "stream ordering");
  if (batch == 0) return AP_OK;
  unsigned char* p = static_cast<unsigned char*>(base);
  auto* coef64 = reinterpret_cast<cx<double>*>(p);
  auto* coef32 = reinterpret_cast<cx<float>*>(p + up256(b64));
  auto* in = reinterpret_cast<cx<double>*>(p + fixed);
  auto* out = reinterpret_cast<cx<double>*>(p + fixed + up256(size_t(batch) * state_bytes(c)));
  // pageable host source: the copy has taken the bytes when the call returns
  fine_coefs(c, dT / steps, c->na_t64.data(), c->na_t32.data());
  if ((e = hipMemcpyAsync(coef64, c->na_t64.data(), b64, hipMemcpyHostToDevice, s)) != hipSuccess ||
      (e = hipMemcpyAsync(coef32, c->na_t32.data(), b32, hipMemcpyHostToDevice, s)) != hipSuccess)
    return hip_fail(e, "coefficient copy");
  if ((e = ap::launch_to_modal(c->N, U_in, in, batch, c->tabs, s)) != hipSuccess)
    return hip_fail(e, "to_modal launch");
  if ((e = ap::launch_fine(c->N, precision == AP_PREC_FP64, in, out, batch, steps, coef64, coef32, c->tabs, s,
                           fine_shape_of(c, precision))) != hipSuccess)
    return hip_fail(e, "fine launch");
  if ((e = ap::launch_to_physical(c->N, out, U_out, batch, c->tabs, s)) != hipSuccess)
    return hip_fail(e, "to_physical launch");
  return AP_OK;
}

int aparareal_strang_batch(ap_ctx* c, const double* U_in, double* U_out, int batch, double dT, int steps,
                           int precision, void* stream) {
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (c && !(dT > 0.0 && std::isfinite(dT))) return fail(AP_EINVAL, "dT must be > 0");
  if (c && steps < 1) return fail(AP_EINVAL, "steps must be >= 1");
  if (c && U_in && U_in == U_out) return fail(AP_EINVAL, "U_out may not alias U_in");
  int rc = batch_prologue(c, U_in, U_out, batch, precision, s);
  if (rc || batch == 0) return rc;
  FineTables* ft = nullptr;
  if ((rc = fine_tables(c, dT / steps, &ft))) return rc;
  hipError_t e = timed(c, AP_K_FINE, s, [&] {
    return ap::launch_strang(c->N, precision == AP_PREC_FP64, c->ws_in.as<cx<double>>(), c->ws_out.as<cx<double>>(),
                             batch, steps, dT / steps, ft->coef64.as<cx<double>>(), c->tabs, s);
  });
  if (e != hipSuccess) return hip_fail(e, "strang launch");
  return batch_epilogue(c, U_out, batch, s);
}

int aparareal_average(ap_ctx* c, const double* U_in, double* N_out, int batch, double T0, int M_avg,
                      int precision, void* stream) {
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (c && !(T0 > 0.0 && std::isfinite(T0))) return fail(AP_EINVAL, "T0 must be > 0");
  if (c && M_avg < 2) return fail(AP_EINVAL, "M_avg must be >= 2");
  int rc = batch_prologue(c, U_in, N_out, batch, precision, s);
  if (rc || batch == 0) return rc;
  AvgTables* at = nullptr;
  if ((rc = avg_tables(c, 0.0, T0, M_avg, &at))) return rc;
  const bool f64 = precision == AP_PREC_FP64;
  hipError_t e = timed(c, AP_K_AVERAGE, s, [&] {
    return ap::launch_average(c->N, c->ws_in.as<cx<double>>(), c->ws_out.as<cx<double>>(), batch,
                              f64 ? &at->c64.avg : nullptr, f64 ? nullptr : &at->c32.avg, c->tabs, s);
  });
  if (e != hipSuccess) return hip_fail(e, "average launch");
  return batch_epilogue(c, N_out, batch, s);
}

int aparareal_coarse(ap_ctx* c, const double* U_in, double* U_out, int batch, double dT, int M_avg, double T0,
                     int precision, void* stream) {
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (c && !(dT > 0.0 && std::isfinite(dT))) return fail(AP_EINVAL, "dT must be > 0");
  if (c && M_avg < 2) return fail(AP_EINVAL, "M_avg must be >= 2");
  if (c && !std::isfinite(T0)) return fail(AP_EINVAL, "T0 must be finite");
  if (c && U_in && U_in == U_out) return fail(AP_EINVAL, "U_out may not alias U_in");
  int rc = batch_prologue(c, U_in, U_out, batch, precision, s);
  if (rc || batch == 0) return rc;
  const double win = T0 > 0.0 ? T0 : dT / c->eps;
  AvgTables* at = nullptr;
  if ((rc = avg_tables(c, dT, win, M_avg, &at))) return rc;
  const bool f64 = precision == AP_PREC_FP64;
  hipError_t e = timed(c, AP_K_COARSE, s, [&] {
    return ap::launch_coarse(c->N, c->ws_in.as<cx<double>>(), c->ws_out.as<cx<double>>(), batch,
                             f64 ? &at->c64 : nullptr, f64 ? nullptr : &at->c32, c->tabs, s);
  });
  if (e != hipSuccess) return hip_fail(e, "coarse launch");
  return batch_epilogue(c, U_out, batch, s);
}

int aparareal_solve(ap_ctx* c, const double* u0, const ap_solve_params* p, double* U_out, double* resid,
                    void* stream) {
  hipStream_t s = static_cast<hipStream_t>(stream);
  int rc = check_ctx(c);
  if (rc) return rc;
  hipError_t e = order_stream(c, s);
  if (e != hipSuccess) return hip_fail(e, "stream ordering");
  std::vector<PlanItem> items(1);
  if ((rc = plan_item(c, u0, p, U_out, resid, &items[0]))) return rc;
  if (p->tol > 0.0 && c->opt_sweeps) {
    if (c->opt_fine || c->opt_coarse)
      return fail(AP_EINVAL, "the host-checked sweeps run ETDRK4 fine slices and asymptotic coarse steps only");
    return solve_sweeps(c, u0, p, U_out, resid, s, items[0].q.steps, items[0].ft, items[0].at);
  }
  return plan_launch(c, items, s);
}

int aparareal_solve_batch(const ap_batch_item* batch, int count, void* stream) {
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (count < 0 || (count > 0 && !batch)) return fail(AP_EINVAL, "bad batch");
  if (count == 0) return AP_OK;
  std::vector<PlanItem> items(static_cast<size_t>(count));
  for (int i = 0; i < count; ++i) {
    ap_ctx* c = batch[i].ctx;
    int rc = check_ctx(c);
    if (rc) return rc;
    for (int j = 0; j < i; ++j)
      if (batch[j].ctx == c) return fail(AP_EINVAL, "a context may appear only once in a batch");
    hipError_t e = order_stream(c, s);
    if (e != hipSuccess) return hip_fail(e, "stream ordering");
    if ((rc = plan_item(c, batch[i].u0, &batch[i].params, batch[i].U_out, batch[i].resid, &items[size_t(i)])))
      return rc;
  }
  return plan_launch(batch[0].ctx, items, s);
}

int aparareal_autotune(const ap_batch_item* batch, int count, void* stream, double* best_ms) {
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (count < 1 || !batch) return fail(AP_EINVAL, "bad autotune batch");
  for (int i = 0; i < count; ++i) {
    int rc = check_ctx(batch[i].ctx);
    if (rc) return rc;
    for (int j = 0; j < i; ++j)
      if (batch[j].ctx == batch[i].ctx) return fail(AP_EINVAL, "a context may appear only once in a batch");
    hipError_t e = order_stream(batch[i].ctx, s);
    if (e != hipSuccess) return hip_fail(e, "stream ordering");
  }
  ap_ctx* owner = batch[0].ctx;
  auto run = [&]() -> int {
    std::vector<PlanItem> items(static_cast<size_t>(count));
    for (int i = 0; i < count; ++i) {
      int rc = plan_item(batch[i].ctx, batch[i].u0, &batch[i].params, batch[i].U_out, batch[i].resid, &items[i]);
      if (rc) return rc;
    }
    return plan_launch(owner, items, s);
  };
  hipEvent_t ev[2] = {nullptr, nullptr};
  if (hipEventCreate(&ev[0]) != hipSuccess || hipEventCreate(&ev[1]) != hipSuccess) {
    if (ev[0]) (void)hipEventDestroy(ev[0]);
    return fail(AP_EDEVICE, "event creation");
  }
  const bool trace_was = owner->trace_on;
  std::vector<int> split_was, group_was;
  std::vector<CostCal> cal_was;
  for (int i = 0; i < count; ++i) {
    split_was.push_back(batch[i].ctx->opt_split);
    group_was.push_back(batch[i].ctx->tuned_group);
    cal_was.push_back(batch[i].ctx->cost);
  }
  // candidates: whole coarse steps with the default groups, then split steps
  // with each tuned group size (contexts with AP_OPT_GROUP set keep theirs)
  constexpr int kCands = 1 + int(sizeof(kTuneGroupMults2) / sizeof(kTuneGroupMults2[0]));
  double best = -1.0;
  int best_cand = -1;
  std::vector<CostCal> best_cal = cal_was;
  int rc = AP_OK;
  for (int cand = 0; cand < kCands && rc == AP_OK; ++cand) {
    const int split = cand == 0 ? 0 : 1;
    bool distinct = cand <= 1;
    for (int i = 0; i < count; ++i) {
      ap_ctx* c = batch[i].ctx;
      c->opt_split = split;
      c->tuned_group = cand == 0 ? 0 : tune_group(c->N, cand - 1);
      if (cand > 1 && c->opt_group == 0 && c->tuned_group != tune_group(c->N, cand - 2)) distinct = true;
      c->cost = CostCal{};
    }
    if (!distinct) continue;   // same groups as the previous candidate for every problem
    if ((rc = run())) break;   // warm-up (tables, workspaces, job list)
    // two rounds: measure job durations, re-order with them
    for (int round = 0; round < 2 && rc == AP_OK; ++round) {
      owner->trace_on = true;
      rc = run();
      owner->trace_on = trace_was;
      if (rc) break;
      hipError_t e = hipStreamSynchronize(s);
      const int nj = owner->pp_trace_jobs;
      std::vector<unsigned long long> raw(size_t(3) * nj);
      if (e == hipSuccess)
        e = hipMemcpy(raw.data(), owner->pp_trace.p, raw.size() * sizeof(unsigned long long), hipMemcpyDeviceToHost);
      if (e != hipSuccess) {
        rc = hip_fail(e, "autotune trace");
        break;
      }
      // per problem and job type: median duration (us, 100 MHz ticks)
      std::vector<std::vector<double>> d(size_t(count) * 4);
      for (int j = 0; j < nj; ++j) {
        const ap::PipeJob& jb = owner->pp_jobs_host[j];
        if (jb.prob < 0 || jb.prob >= count || jb.type < 0 || jb.type > 3) continue;
        const double us = double(raw[3 * j + 1] - raw[3 * j]) / 100.0;
        d[size_t(jb.prob) * 4 + jb.type].push_back(us);
      }
      auto median = [](std::vector<double>& v) {
        if (v.empty()) return 0.0;
        std::nth_element(v.begin(), v.begin() + v.size() / 2, v.end());
        return v[v.size() / 2];
      };
      for (int i = 0; i < count; ++i) {
        CostCal cc;
        cc.valid = true;
        const double fine = median(d[size_t(i) * 4 + ap::kJobFine]);
        const ap_solve_params& p = batch[i].params;
        const int steps = std::max(1, int(std::ceil(p.T / p.slices / p.dt_fine - 1e-9)));
        cc.fine_step = fine / steps;
        cc.whole = median(d[size_t(i) * 4 + ap::kJobCoarse]);
        cc.stage1 = median(d[size_t(i) * 4 + ap::kJobStage1]);
        cc.stage2 = median(d[size_t(i) * 4 + ap::kJobStage2]);
        batch[i].ctx->cost = cc;
      }
    }
    if (rc) break;
    double ms = -1.0;
    for (int rep = 0; rep < 3 && rc == AP_OK; ++rep) {
      (void)hipEventRecord(ev[0], s);
      rc = run();
      (void)hipEventRecord(ev[1], s);
      float t = 0.f;
      if (rc == AP_OK && (hipEventSynchronize(ev[1]) != hipSuccess || hipEventElapsedTime(&t, ev[0], ev[1]) != hipSuccess))
        rc = fail(AP_EDEVICE, "autotune timing");
      if (rc == AP_OK && (ms < 0.0 || t < ms)) ms = t;
    }
    if (rc == AP_OK && (best < 0.0 || ms < best)) {
      best = ms;
      best_cand = cand;
      best_cal.clear();
      for (int i = 0; i < count; ++i) best_cal.push_back(batch[i].ctx->cost);
    }
  }
  // with the best mapping and its measured durations: the scheduling weight
  // of a dependency (hand-off delay), a few values around the default
  const int handoff_was = owner->handoff_ns;
  int best_handoff = handoff_was;
  if (rc == AP_OK && best_cand >= 0) {
    for (int i = 0; i < count; ++i) {
      ap_ctx* c = batch[i].ctx;
      c->opt_split = best_cand == 0 ? 0 : 1;
      c->tuned_group = best_cand == 0 ? 0 : tune_group(c->N, best_cand - 1);
      c->cost = best_cal[size_t(i)];
    }
    for (const int h : {handoff_was / 2, handoff_was * 5 / 3}) {
      owner->handoff_ns = h;
      if ((rc = run())) break;   // warm-up with the new job order
      double ms = -1.0;
      for (int rep = 0; rep < 3 && rc == AP_OK; ++rep) {
        (void)hipEventRecord(ev[0], s);
        rc = run();
        (void)hipEventRecord(ev[1], s);
        float t = 0.f;
        if (rc == AP_OK &&
            (hipEventSynchronize(ev[1]) != hipSuccess || hipEventElapsedTime(&t, ev[0], ev[1]) != hipSuccess))
          rc = fail(AP_EDEVICE, "autotune timing");
        if (rc == AP_OK && (ms < 0.0 || t < ms)) ms = t;
      }
      if (rc == AP_OK && ms < best) {
        best = ms;
        best_handoff = h;
      }
    }
  }
  owner->handoff_ns = rc == AP_OK ? best_handoff : handoff_was;
  for (int i = 0; i < count; ++i) {
    ap_ctx* c = batch[i].ctx;
    if (rc == AP_OK && best_cand >= 0) {
      c->opt_split = best_cand == 0 ? 0 : 1;
      c->tuned_group = best_cand == 0 ? 0 : tune_group(c->N, best_cand - 1);
      c->cost = best_cal[size_t(i)];
    } else {
      c->opt_split = split_was[size_t(i)];
      c->tuned_group = group_was[size_t(i)];
      c->cost = cal_was[size_t(i)];
    }
  }
  owner->trace_on = trace_was;
  (void)hipEventDestroy(ev[0]);
  (void)hipEventDestroy(ev[1]);
  if (rc) return rc;
  if (best_ms) *best_ms = best;
  return AP_OK;
}

int aparareal_set_option(ap_ctx* c, int option, int value) {
  int rc = check_ctx(c);
  if (rc) return rc;
  switch (option) {
    case AP_OPT_SPLIT:
      if (value < -1 || value > 1) return fail(AP_EINVAL, "AP_OPT_SPLIT takes -1, 0 or 1");
      c->opt_split = value;
      return AP_OK;
    case AP_OPT_GROUP:
      if (value < 0 || value > 4096) return fail(AP_EINVAL, "AP_OPT_GROUP takes 0..4096");
      c->opt_group = value;
      return AP_OK;
    case AP_OPT_GRID:
      if (value < 0) return fail(AP_EINVAL, "AP_OPT_GRID takes a value >= 0");
      c->opt_grid = value;
      return AP_OK;
    case AP_OPT_GRAPH:
      if (value < 0 || value > 1) return fail(AP_EINVAL, "AP_OPT_GRAPH takes 0 or 1");
      c->opt_graph = value;
      return AP_OK;
    case AP_OPT_SKIP:
      if (value < 0 || value > 1) return fail(AP_EINVAL, "AP_OPT_SKIP takes 0 or 1");
      c->opt_skip = value;
      return AP_OK;
    case AP_OPT_SWEEPS:
      if (value < 0 || value > 1) return fail(AP_EINVAL, "AP_OPT_SWEEPS takes 0 or 1");
      c->opt_sweeps = value;
      return AP_OK;
    case AP_OPT_FINE:
      if (value < 0 || value > 1) return fail(AP_EINVAL, "AP_OPT_FINE takes 0 (ETDRK4) or 1 (Strang)");
      c->opt_fine = value;
      return AP_OK;
    case AP_OPT_FINE_GROUP:
      if (value < 0 || value > 64) return fail(AP_EINVAL, "AP_OPT_FINE_GROUP takes 0..64");
      c->opt_fine_group = value;
      return AP_OK;
    case AP_OPT_COARSE:
      if (value < 0 || value > 1) return fail(AP_EINVAL, "AP_OPT_COARSE takes 0 (asymptotic) or 1 (Strang)");
      c->opt_coarse = value;
      return AP_OK;
    case AP_OPT_FINE_SHAPE:
      if (value != -1 && !fine_config_valid(c->N, value))
        return fail(AP_EINVAL, "AP_OPT_FINE_SHAPE takes -1 or a configuration 0..5 compiled for this N "
                               "(3..5 need N >= 256)");
      c->opt_fine_shape = value;
      return AP_OK;
    case AP_OPT_HANDOFF_NS:
      if (value < 0 || value > 1000000) return fail(AP_EINVAL, "AP_OPT_HANDOFF_NS takes 0..1000000");
      c->handoff_ns = value;
      return AP_OK;
    default:
      return fail(AP_EINVAL, "unknown option");
  }
}

int aparareal_get_option(ap_ctx* c, int option, int* value) {
  int rc = check_ctx(c);
  if (rc) return rc;
  if (!value) return fail(AP_EINVAL, "null value");
  switch (option) {
    case AP_OPT_SPLIT: *value = c->opt_split; return AP_OK;
    case AP_OPT_GROUP: *value = group_size(c); return AP_OK;
    case AP_OPT_GRID: *value = c->opt_grid; return AP_OK;
    case AP_OPT_GRAPH: *value = c->opt_graph; return AP_OK;
    case AP_OPT_SKIP: *value = c->opt_skip; return AP_OK;
    case AP_OPT_SWEEPS: *value = c->opt_sweeps; return AP_OK;
    case AP_OPT_FINE: *value = c->opt_fine; return AP_OK;
    case AP_OPT_COARSE: *value = c->opt_coarse; return AP_OK;
    case AP_OPT_FINE_GROUP: *value = c->opt_fine_group; return AP_OK;
    case AP_OPT_FINE_SHAPE: *value = c->opt_fine_shape; return AP_OK;
    case AP_OPT_HANDOFF_NS: *value = c->handoff_ns; return AP_OK;
    default: return fail(AP_EINVAL, "unknown option");
  }
}

int aparareal_pipeline_status(ap_ctx* c, int* info) {
  int rc = check_ctx(c);
  if (rc) return rc;
  if (!info) return fail(AP_EINVAL, "null info");
  info[0] = info[1] = info[2] = 0;
  if (!c->pp_diag) return AP_OK;
  hipError_t e = c->has_last ? hipStreamSynchronize(c->last_stream) : hipDeviceSynchronize();
  if (e == hipSuccess) e = hipMemcpy(info, c->pp_diag, 3 * sizeof(int), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(e, "pipeline status");
  return AP_OK;
}

namespace {
// Shape of a problem of a schedule query (no context needed).
int query_shape(int N, const ap_solve_params* p, int split, int group, int fine_group, const double* cost,
                PipeShape* q) {
  if (!p || !is_pow2(N) || N < 64 || N > 2048 || p->slices < 1 || p->K < 0 || p->M_avg < 2 || group < 0 ||
      split < -1 || split > 1 || fine_group < 1 || fine_group > 64 || !(p->T > 0.0) || !(p->dt_fine > 0.0))
    return fail(AP_EINVAL, "bad schedule query");
  if (size_t(2 * p->K + 1) * size_t(p->slices) > (size_t(1) << 24)) return fail(AP_EINVAL, "problem too large");
  const double dT = p->T / p->slices;
  const double ratio = dT / p->dt_fine;
  if (ratio > 1e7) return fail(AP_EINVAL, "dT/dt_fine too large");
  q->nx = N;
  q->Ns = p->slices;
  q->K = p->K;
  q->steps = std::max(1, int(std::ceil(ratio - 1e-9)));
  q->M = p->M_avg;
  q->gs = group > 0 ? group : default_group_size(N);
  q->groups = ap::avg_groups(q->M, q->gs);
  q->fp64 = p->precision == AP_PREC_FP64;
  q->split = split < 0 ? q->groups >= 2 : split != 0;
  q->skip = true;
  q->tol = p->tol > 0.0 ? p->tol : 0.0;
  q->fg = std::min(fine_group, ap::pipeline_fine_slices(N, q->fp64, q->fine_kind));
  if (cost) {
    for (int i = 0; i < 4; ++i)
      if (!(cost[i] >= 0.0) || !(cost[i] < 1e9)) return fail(AP_EINVAL, "bad job duration");
    q->cal.valid = true;
    q->cal.fine_step = cost[0];
    q->cal.stage1 = cost[1];
    q->cal.stage2 = cost[2];
    q->cal.whole = cost[3];
  }
  return AP_OK;
}
}  // namespace

int aparareal_pipeline_schedule(int N, const ap_solve_params* p, int split, int group, int fine_group, int* out,
                                int max_jobs) {
  if (max_jobs < 0) return fail(AP_EINVAL, "bad schedule query");
  PipeShape q;
  const int rc = query_shape(N, p, split, group, fine_group, nullptr, &q);
  if (rc) return rc;
  const std::vector<PipeShape> shapes{q};
  const std::vector<ap::PipeJob> jobs = schedule_jobs(shapes, kQueryWorkers);
  if (!order_is_valid(jobs, shapes)) return fail(AP_EINVAL, "internal: job order is not topological");
  if (out)
    for (size_t i = 0; i < jobs.size() && i < size_t(max_jobs); ++i) {
      out[4 * i] = jobs[i].type;
      out[4 * i + 1] = jobs[i].k;
      out[4 * i + 2] = jobs[i].n;
      out[4 * i + 3] = jobs[i].g;
    }
  return int(jobs.size());
}

int aparareal_pipeline_schedule_batch(int count, const int* N, const ap_solve_params* p, int split, int group,
                                      int fine_group, const double* cost, int* out, int max_jobs) {
  if (count < 1 || count > 4096 || !N || !p || max_jobs < 0) return fail(AP_EINVAL, "bad schedule query");
  std::vector<PipeShape> shapes(static_cast<size_t>(count));
  size_t cells = 0;
  for (int i = 0; i < count; ++i) {
    const int rc = query_shape(N[i], &p[i], split, group, fine_group, cost ? cost + 4 * i : nullptr, &shapes[i]);
    if (rc) return rc;
    cells += size_t(2 * p[i].K + 1) * size_t(p[i].slices);
    if (cells > (size_t(1) << 24)) return fail(AP_EINVAL, "batch too large");
  }
  const std::vector<ap::PipeJob> jobs = schedule_jobs(shapes, kQueryWorkers);
  if (!order_is_valid(jobs, shapes)) return fail(AP_EINVAL, "internal: job order is not topological");
  if (out)
    for (size_t i = 0; i < jobs.size() && i < size_t(max_jobs); ++i) {
      out[5 * i] = jobs[i].prob;
      out[5 * i + 1] = jobs[i].type;
      out[5 * i + 2] = jobs[i].k;
      out[5 * i + 3] = jobs[i].n;
      out[5 * i + 4] = jobs[i].g;
    }
  return int(jobs.size());
}

int aparareal_pipeline_trace(ap_ctx* c, int enable, long long* out, int max_jobs) {
  int rc = check_ctx(c);
  if (rc) return rc;
  if (enable >= 0) {
    c->trace_on = enable != 0;
    return AP_OK;
  }
  if (!out || max_jobs < 0) return fail(AP_EINVAL, "bad trace query");
  if (!c->pp_trace.p || c->pp_trace_jobs == 0) return 0;
  const int n = std::min(max_jobs, c->pp_trace_jobs);
  std::vector<unsigned long long> raw(size_t(3) * n);   // start, end, workgroup
  hipError_t e = c->has_last ? hipStreamSynchronize(c->last_stream) : hipDeviceSynchronize();
  if (e == hipSuccess) e = hipMemcpy(raw.data(), c->pp_trace.p, raw.size() * sizeof(unsigned long long),
                                     hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(e, "trace readback");
  for (int i = 0; i < n; ++i) {
    const ap::PipeJob& j = c->pp_jobs_host[i];
    long long* o = out + size_t(8) * i;
    o[0] = j.prob;
    o[1] = j.type;
    o[2] = j.k;
    o[3] = j.n;
    o[4] = j.g;
    o[5] = (long long)raw[3 * i];
    o[6] = (long long)raw[3 * i + 1];
    o[7] = (long long)raw[3 * i + 2];
  }
  return n;
}

int aparareal_profile(ap_ctx* c, int enable) {
  int rc = check_ctx(c);
  if (rc) return rc;
  if (enable) {
    for (auto& t : c->ev_pending) {
      c->ev_pool.push_back(std::get<1>(t));
      c->ev_pool.push_back(std::get<2>(t));
    }
    c->ev_pending.clear();
    for (int i = 0; i < AP_K_CLASSES; ++i) {
      c->prof_count[i] = 0;
      c->prof_ms[i] = 0.0;
    }
  }
  c->prof_on = enable != 0;
  return AP_OK;
}

int aparareal_profile_read(ap_ctx* c, int cls, int* launches, double* total_ms) {
  int rc = check_ctx(c);
  if (rc) return rc;
  if (cls < 0 || cls >= AP_K_CLASSES || !launches || !total_ms) return fail(AP_EINVAL, "bad profile query");
  for (auto& t : c->ev_pending) {
    hipEvent_t a = std::get<1>(t), b = std::get<2>(t);
    hipError_t e = hipEventSynchronize(b);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
    if (e != hipSuccess) return hip_fail(e, "profile events");
    c->prof_count[std::get<0>(t)] += 1;
    c->prof_ms[std::get<0>(t)] += ms;
    c->ev_pool.push_back(a);
    c->ev_pool.push_back(b);
  }
  c->ev_pending.clear();
  *launches = c->prof_count[cls];
  *total_ms = c->prof_ms[cls];
  return AP_OK;
}

}  // extern "C"
