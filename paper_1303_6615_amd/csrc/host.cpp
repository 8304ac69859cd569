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

#include <cmath>
#include <complex>
#include <cstring>
#include <algorithm>
#include <map>
#include <memory>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/aparareal.h"
#include "launch.hpp"

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

}  // namespace

struct ap_ctx {
  int N = 0, KD = 0, KP = 0;
  double eps = 0, F = 0, nu = 0;
  int device = 0;
  std::vector<double> omega, akw;   // per retained k
  DevBuf tw64, tw32, basis64, basis32;
  ap::DevTables tabs;
  std::map<uint64_t, std::unique_ptr<FineTables>> fine_cache;
  std::map<std::tuple<uint64_t, uint64_t, int>, std::unique_ptr<AvgTables>> avg_cache;
  DevBuf ws_in, ws_out, ws_U, ws_F, ws_G, ws_part;
  // pipelined solve: per-level states, flags, job list and descriptor
  DevBuf pp_U, pp_F, pp_G, pp_part, pp_flags, pp_jobs, pp_prob;
  std::tuple<int, int, int, int> pp_jobs_key{-1, -1, -1, -1};
  int pp_njobs = 0;
  std::vector<ap::PipeJob> pp_jobs_host;
  std::vector<unsigned char> pp_prob_host;
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

int fine_tables(ap_ctx* c, double h, FineTables** out) {
  auto it = c->fine_cache.find(bits(h));
  if (it != c->fine_cache.end()) {
    *out = it->second.get();
    return AP_OK;
  }
  auto ft = std::make_unique<FineTables>();
  const int KP = c->KP;
  std::vector<cx<double>> t64(size_t(8) * 3 * KP);
  std::vector<cx<float>> t32(size_t(8) * 3 * KP);
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
      // FP64: E, 0, E2, 0, Q, f1, 2f2, f3
      t64[at(0)] = to_cx<double>(vals[0]);
      t64[at(1)] = cx<double>{0, 0};
      t64[at(2)] = to_cx<double>(vals[1]);
      t64[at(3)] = cx<double>{0, 0};
      for (int q = 2; q < 6; ++q) t64[at(q + 2)] = to_cx<double>(vals[q]);
      // FP32: E and E2 as hi + lo
      for (int q = 0; q < 2; ++q) {
        const cx<float> hi = to_cx<float>(vals[q]);
        const cd rest = vals[q] - cd(double(hi.x), double(hi.y));
        t32[at(2 * q)] = hi;
        t32[at(2 * q + 1)] = to_cx<float>(rest);
      }
      for (int q = 2; q < 6; ++q) t32[at(q + 2)] = to_cx<float>(vals[q]);
    }
  }
  hipError_t e = ft->coef64.upload(t64);
  if (e == hipSuccess) e = ft->coef32.upload(t32);
  if (e != hipSuccess) return hip_fail(e, "fine coefficient upload");
  *out = ft.get();
  c->fine_cache[bits(h)] = std::move(ft);
  return AP_OK;
}

// dT == 0 builds the average-only tables.
int avg_tables(ap_ctx* c, double dT, double T0, int M, AvgTables** out) {
  auto key = std::make_tuple(bits(dT), bits(T0), M);
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
  at->c64 = ap::CoarseTab<double>{{at->rot64.as<cx<double>>(), at->w64.as<double>(), M},
                                  at->hd64.as<double>(), at->rotT64.as<cx<double>>(), dT};
  at->c32 = ap::CoarseTab<float>{{at->rot32.as<cx<float>>(), at->w32.as<float>(), M},
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

// Jobs of the pipelined solve in a topological order: by estimated ready time
// t(C(k,n)) = n tc + k tf, t(F(k,n)) = (n-1) tc + k tf (tc, tf: nonlinear
// evaluations per coarse step / fine slice), coarse before fine on ties.  Every
// dependency of a job has a smaller t or is a coarse job of equal t, so the
// ticket order lets the earliest unfinished job always run.
std::vector<ap::PipeJob> pipeline_jobs(int prob, int Ns, int K, int steps, int M) {
  struct Item {
    long long t;
    ap::PipeJob j;
  };
  const long long tc = 2LL * (M - 1) > 0 ? 2LL * (M - 1) : 1, tf = 4LL * steps;
  std::vector<Item> it;
  it.reserve(size_t(2 * K + 1) * Ns);
  for (int k = 0; k <= K; ++k)
    for (int n = 1; n <= Ns; ++n) it.push_back({n * tc + k * tf, {prob, 0, k, n}});
  for (int k = 0; k < K; ++k)
    for (int n = 1; n <= Ns; ++n) it.push_back({(n - 1) * tc + k * tf, {prob, 1, k, n}});
  std::stable_sort(it.begin(), it.end(), [](const Item& a, const Item& b) {
    if (a.t != b.t) return a.t < b.t;
    if (a.j.type != b.j.type) return a.j.type < b.j.type;
    if (a.j.k != b.j.k) return a.j.k < b.j.k;
    return a.j.n < b.j.n;
  });
  std::vector<ap::PipeJob> out;
  out.reserve(it.size());
  for (auto& x : it) out.push_back(x.j);
  return out;
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

int solve_pipelined(ap_ctx* c, const double* u0, const ap_solve_params* p, double* U_out, double* resid,
                    hipStream_t s, int steps, FineTables* ft, AvgTables* at) {
  const int Ns = p->slices, K = p->K;
  const size_t sb = state_bytes(c);
  // job flags, ticket, stall record [3], per-workgroup progress [2][256]
  const int nflags = (2 * K + 1) * Ns + 4 + 2 * 256;
  hipError_t e;
  if ((e = ensure(c, c->pp_U, sb * size_t(K + 1) * (Ns + 1))) != hipSuccess ||
      (e = ensure(c, c->pp_F, sb * size_t(std::max(K, 1)) * (Ns + 1))) != hipSuccess ||
      (e = ensure(c, c->pp_G, sb * size_t(K + 1) * (Ns + 1))) != hipSuccess ||
      (e = ensure(c, c->pp_part, sizeof(double2) * size_t(Ns) * std::max(1, K))) != hipSuccess ||
      (e = ensure(c, c->pp_flags, sizeof(int) * size_t(nflags))) != hipSuccess ||
      (e = ensure(c, c->pp_prob, sizeof(ap::PipeProb<double>))) != hipSuccess)
    return hip_fail(e, "pipeline workspace");
  const auto key = std::make_tuple(Ns, K, steps, p->M_avg);
  if (key != c->pp_jobs_key) {
    c->pp_jobs_host = pipeline_jobs(0, Ns, K, steps, p->M_avg);
    c->pp_njobs = int(c->pp_jobs_host.size());
    if ((e = ensure(c, c->pp_jobs, sizeof(ap::PipeJob) * c->pp_jobs_host.size())) != hipSuccess ||
        (e = hipMemcpy(c->pp_jobs.p, c->pp_jobs_host.data(), sizeof(ap::PipeJob) * c->pp_jobs_host.size(),
                       hipMemcpyHostToDevice)) != hipSuccess)
      return hip_fail(e, "job list upload");
    c->pp_jobs_key = key;
  }
  const bool f64 = p->precision == AP_PREC_FP64;
  cx<double>* U = c->pp_U.as<cx<double>>();
  int* flags = c->pp_flags.as<int>();
  int* ticket = flags + (2 * K + 1) * Ns;
  int* abort = ticket + 1;
  c->pp_prob_host.resize(sizeof(ap::PipeProb<double>));
  if (f64) {
    ap::PipeProb<double> pr{U, c->pp_F.as<cx<double>>(), c->pp_G.as<cx<double>>(), c->pp_part.as<double2>(),
                            flags, Ns, K, steps, ft->coef64.as<cx<double>>(), ft->coef64.as<cx<double>>(), at->c64};
    std::memcpy(c->pp_prob_host.data(), &pr, sizeof(pr));
  } else {
    ap::PipeProb<float> pr{U, c->pp_F.as<cx<double>>(), c->pp_G.as<cx<double>>(), c->pp_part.as<double2>(),
                           flags, Ns, K, steps, ft->coef64.as<cx<double>>(), ft->coef32.as<cx<float>>(), at->c32};
    std::memcpy(c->pp_prob_host.data(), &pr, sizeof(pr));
  }
  if ((e = hipMemcpyAsync(c->pp_prob.p, c->pp_prob_host.data(), c->pp_prob_host.size(), hipMemcpyHostToDevice, s)) !=
      hipSuccess)
    return hip_fail(e, "problem descriptor upload");
  const size_t st = size_t(3) * c->KP;
  e = timed(c, AP_K_TO_MODAL, s, [&] { return ap::launch_to_modal(c->N, u0, U, 1, c->tabs, s); });
  if (e != hipSuccess) return hip_fail(e, "to_modal");
  if (K > 0 && (e = hipMemcpyAsync(U + size_t(K) * (Ns + 1) * st, U, sb, hipMemcpyDeviceToDevice, s)) != hipSuccess)
    return hip_fail(e, "initial state copy");
  if ((e = ap::launch_zero_ints(flags, nflags, s)) != hipSuccess) return hip_fail(e, "flag reset");
  c->pp_diag = abort;
  const int grid = std::min(c->pp_njobs, 256);
  unsigned long long* trace = nullptr;
  if (c->trace_on) {
    if ((e = ensure(c, c->pp_trace, sizeof(unsigned long long) * 3 * size_t(c->pp_njobs))) != hipSuccess)
      return hip_fail(e, "trace buffer");
    trace = c->pp_trace.as<unsigned long long>();
    c->pp_trace_jobs = c->pp_njobs;
  }
  e = timed(c, AP_K_PIPELINE, s, [&] {
    return ap::launch_pipeline(c->N, f64, c->pp_jobs.p, c->pp_njobs, c->pp_prob.p, ticket, abort, abort + 3, trace,
                               grid, c->tabs, s);
  });
  if (e != hipSuccess) return hip_fail(e, "pipeline launch");
  if (K > 0) {
    e = timed(c, AP_K_RESID, s,
              [&] { return ap::launch_resid(c->pp_part.as<double2>(), Ns, K, resid, abort, s); });
    if (e != hipSuccess) return hip_fail(e, "resid");
  }
  cx<double>* UK = U + size_t(K) * (Ns + 1) * st;
  e = timed(c, AP_K_TO_PHYSICAL, s, [&] { return ap::launch_to_physical(c->N, UK, U_out, Ns + 1, c->tabs, s); });
  if (e != hipSuccess) return hip_fail(e, "to_physical");
  return AP_OK;
}

}  // namespace

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
  c->omega.resize(c->KP);
  c->akw.resize(c->KP);
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
  std::vector<cx<double>> t64(N);
  std::vector<cx<float>> t32(N);
  for (int t = 0; t < N; ++t) {
    const double th = 2.0 * M_PI * double(t) / double(N);
    t64[t] = cx<double>{std::cos(th), -std::sin(th)};
    t32[t] = cx<float>{float(std::cos(th)), float(-std::sin(th))};
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
                           ft->coef64.as<cx<double>>(), ft->coef32.as<cx<float>>(), c->tabs, s);
  });
  if (e != hipSuccess) return hip_fail(e, "fine launch");
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
  const double h = dT / steps;
  const double win = p->T0 > 0.0 ? p->T0 : dT / c->eps;
  hipError_t e = order_stream(c, s);
  if (e != hipSuccess) return hip_fail(e, "stream ordering");
  FineTables* ft = nullptr;
  AvgTables* at = nullptr;
  if ((rc = fine_tables(c, h, &ft))) return rc;
  if ((rc = avg_tables(c, dT, win, p->M_avg, &at))) return rc;
  if (p->tol > 0.0) return solve_sweeps(c, u0, p, U_out, resid, s, steps, ft, at);
  return solve_pipelined(c, u0, p, U_out, resid, s, steps, ft, at);
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

int aparareal_pipeline_schedule(int slices, int K, int steps, int M_avg, int* out) {
  if (slices < 1 || K < 0 || steps < 1 || M_avg < 2 || !out) return fail(AP_EINVAL, "bad schedule query");
  if (size_t(2 * K + 1) * size_t(slices) > (size_t(1) << 30)) return fail(AP_EINVAL, "problem too large");
  const std::vector<ap::PipeJob> jobs = pipeline_jobs(0, slices, K, steps, M_avg);
  for (size_t i = 0; i < jobs.size(); ++i) {
    out[3 * i] = jobs[i].type;
    out[3 * i + 1] = jobs[i].k;
    out[3 * i + 2] = jobs[i].n;
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
  std::vector<unsigned long long> raw(size_t(3) * n);
  hipError_t e = c->has_last ? hipStreamSynchronize(c->last_stream) : hipDeviceSynchronize();
  if (e == hipSuccess) e = hipMemcpy(raw.data(), c->pp_trace.p, raw.size() * sizeof(unsigned long long),
                                     hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(e, "trace readback");
  for (int i = 0; i < n; ++i) {
    out[6 * i + 0] = c->pp_jobs_host[i].type;
    out[6 * i + 1] = c->pp_jobs_host[i].k;
    out[6 * i + 2] = c->pp_jobs_host[i].n;
    out[6 * i + 3] = (long long)raw[3 * i];
    out[6 * i + 4] = (long long)raw[3 * i + 1];
    out[6 * i + 5] = (long long)raw[3 * i + 2];
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
