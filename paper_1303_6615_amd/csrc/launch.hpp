// Host-visible kernel launch interface of the HIP path (internal to the library).
#pragma once
#include <hip/hip_runtime.h>

#include "rsw_device.hpp"

namespace ap {

// Per-context device tables that depend only on the grid and F.
struct DevTables {
  const cx<double>* tw64 = nullptr;      // exp(-2 pi i t / N), t < N, then FFT plan 0's pass tables
  const cx<float>* tw32 = nullptr;
  const Basis<double>* basis64 = nullptr;  // per retained k: 1/omega_k, a_k/omega_k
  const Basis<float>* basis32 = nullptr;
  int tw_plan1 = 0;                      // entry where FFT plan 1's table starts (same layout)
  template <typename T> const cx<T>* tw() const;
  template <typename T> const Basis<T>* basis() const;
  template <typename T> const cx<T>* tw_plan(int plan) const { return tw<T>() + (plan == 1 ? tw_plan1 : 0); }
};
template <> inline const cx<double>* DevTables::tw<double>() const { return tw64; }
template <> inline const cx<float>* DevTables::tw<float>() const { return tw32; }
template <> inline const Basis<double>* DevTables::basis<double>() const { return basis64; }
template <> inline const Basis<float>* DevTables::basis<float>() const { return basis32; }

// Kernel-weighted time average: rot[m][k] = exp(-i omega_k s_m), w[m] = rho(m/M)/M.
// The samples m = 1..M-1 are summed in groups of gs consecutive samples: each
// group's contributions in increasing m, then the group sums in increasing
// group order.  Every kernel uses this association, whatever the number of
// workgroups that evaluate one average, so results do not depend on it.
template <typename T>
struct AvgTab {
  const cx<T>* rot;
  const T* w;
  int M;
  int gs;
};
inline int avg_groups(int M, int gs) { return (M - 1 + gs - 1) / gs; }

// Asymptotic coarse step of length dT: hd[k] = exp(-nu k^4 dT/2),
// rotT[k] = exp(-i omega_k dT/eps) (the alpha = +1 factor of exp(-(dT/eps) L)).
template <typename T>
struct CoarseTab {
  AvgTab<T> avg;
  const T* hd;
  const cx<T>* rotT;
  T dT;
};

// Pipelined solve: jobs of problem `prob` at iteration level k for slice n
// (1-based).  A coarse step is either one job (kJobCoarse) or, split over
// workgroups, one job per sample group g for each of its two averages
// (kJobStage1, kJobStage2); the last stage-2 job of a step to finish applies
// the step and the correction.  kJobCopy is the step C(k,n) of a slice that
// iteration k has made exact (n <= k): its inputs equal those of C(k-1,n), so
// U(k,n) = U(k-1,n) (n < k) or F(k-1,k) (n = k) and G(k,n) = G(k-1,n), and
// the fine slices F(k,n), n <= k, are not run at all.
enum : int { kJobCoarse = 0, kJobFine = 1, kJobStage1 = 2, kJobStage2 = 3, kJobCopy = 4 };
struct PipeJob {
  int prob, type, k, n, g;
};

// Counter layout of one problem (int32, zeroed before the launch), in units
// of kCounterStride ints: every counter has a 128-byte line of its own, so
// that workgroups polling different counters do not queue on one line.
//   C(k,n) done     at             k Ns + n-1   (k = 0..K)
//   F(k,n) done     at (K+1) Ns +  k Ns + n-1   (k = 0..K-1)
//   stage-1 count   at (2K+1) Ns + k Ns + n-1   (k = 0..K)
//   stage-2 count   at (3K+2) Ns + k Ns + n-1   (k = 0..K)
//   stopped level   at (4K+3) Ns                (0: running; k: residual r^k <= tol)
constexpr int kCounterStride = 32;
inline long long pipe_counters(int Ns, int K) { return ((4LL * K + 3) * Ns + 1) * kCounterStride; }
inline long long pipe_stop_index(int Ns, int K) { return (4LL * K + 3) * Ns * kCounterStride; }

// Per-problem device descriptor of the pipelined solve.
template <typename T>
struct PipeProb {
  cx<double>* U;       // [K+1][Ns+1][3][KP]
  cx<double>* F;       // [K][Ns+1][3][KP]
  cx<double>* G;       // [K+1][Ns+1][3][KP]
  double2* part;       // [K][Ns] residual partial sums
  int* cnt;            // counters, layout above
  cx<T>* P1;           // [K+1][groups + 1][3][KP] stage-1 group sums, then the step's midpoint state (split steps)
  cx<T>* P2;           // [K+1][groups][3][KP] stage-2 group sums
  int nx, Ns, K, steps, groups;
  int fine_kind;       // 0: ETDRK4 fine slices; 1: Strang steps (Alg. 3)
  int coarse_kind;     // 0: asymptotic coarse step (Alg. 2); 1: one Strang step of dT
  double hf, hc;       // fine step size; coarse (Strang) step size dT
  const cx<double>* ccoef64;   // Strang coarse: [8][3][KP] table for h = dT (slot 2: e^{(dT/2) lambda})
  double tol;          // > 0: stop after the first level k with r^k <= tol
  const cx<double>* coef64;
  const cx<T>* coef;
  CoarseTab<T> ct;
  const cx<T>* tw;     // exp(-2 pi i t / nx)
  const Basis<T>* basis;
};

// Boundary transforms of up to kBoundaryBatch problems of one grid size in
// one launch, passed by value as the kernel's argument (no device table, so
// nothing to upload or wait for).  Problem i covers workgroups first[i] ..
// first[i+1] - 1, one state each: state j of problem i is read from src and
// written to dst, each advanced by j states of its form.
constexpr int kBoundaryBatch = 64;
struct BoundaryJob {
  const void* src;              // to modal: double [3][N] per state; to physical: cx<double> [3][KP]
  void* dst;                    // the other form
  cx<double>* dst2;             // to modal: a second copy of the modal state, or null
  const cx<double>* tw;         // the problem's FP64 twiddles
  const Basis<double>* basis;   // the problem's FP64 modal basis
};
struct BoundaryBatch {
  int n;                              // problems
  int first[kBoundaryBatch + 1];      // prefix sums of their workgroups
  BoundaryJob job[kBoundaryBatch];
};
static_assert(sizeof(BoundaryBatch) <= 4096, "a kernel argument of at most 4 KiB");

hipError_t launch_to_modal(int nx, const double* phys, cx<double>* modal, int batch, const DevTables& t,
                           hipStream_t s);
hipError_t launch_to_modal_batch(int nx, const BoundaryBatch& b, hipStream_t s);
hipError_t launch_to_physical_batch(int nx, const BoundaryBatch& b, hipStream_t s);
hipError_t launch_to_physical(int nx, const cx<double>* modal, double* phys, int batch, const DevTables& t,
                              hipStream_t s);
hipError_t launch_nonlinear(int nx, bool fp64, const cx<double>* in, cx<double>* out, int batch,
                            const DevTables& t, hipStream_t s);
// The fine batch in configuration `shape` (0 .. 5: workgroup shape
// shape % 3, FFT plan shape / 3; 0 the default); the workgroup shape changes
// no result, plan 1 rounds differently at N = 1024 only.
hipError_t launch_fine(int nx, bool fp64, const cx<double>* in, cx<double>* out, int batch, int steps,
                       const cx<double>* coef64, const cx<float>* coef32, const DevTables& t, hipStream_t s,
                       int shape = 0);
hipError_t launch_fine_f32(int nx, int shape, const cx<double>* in, cx<double>* out, int batch, int steps,
                           const cx<double>* coef64, const cx<float>* coef32, const DevTables& t, hipStream_t s);
hipError_t launch_fine_f64(int nx, int shape, const cx<double>* in, cx<double>* out, int batch, int steps,
                           const cx<double>* coef64, const DevTables& t, hipStream_t s);
// Threads per workgroup of a fine-batch configuration (0 if it is not
// compiled at this grid size) and its slices per workgroup.
int fine_shape_f32(int nx, int shape, int* slices);
int fine_shape_f64(int nx, int shape, int* slices);
inline int fine_shape(int nx, bool fp64, int shape, int* slices) {
  return fp64 ? fine_shape_f64(nx, shape, slices) : fine_shape_f32(nx, shape, slices);
}
constexpr int kFineConfigCount = 6;   // 3 workgroup shapes x 2 FFT plans
// `steps` Strang steps of size h (coef64 slot 2: e^{(h/2) lambda}) per state.
hipError_t launch_strang(int nx, bool fp64, const cx<double>* in, cx<double>* out, int batch, int steps, double h,
                         const cx<double>* coef64, const DevTables& t, hipStream_t s);
hipError_t launch_average(int nx, const cx<double>* in, cx<double>* out, int batch, const AvgTab<double>* av64,
                          const AvgTab<float>* av32, const DevTables& t, hipStream_t s);
hipError_t launch_coarse(int nx, const cx<double>* in, cx<double>* out, int batch, const CoarseTab<double>* c64,
                         const CoarseTab<float>* c32, const DevTables& t, hipStream_t s);
hipError_t launch_sweep(int nx, cx<double>* U, const cx<double>* Fine, cx<double>* Gold, double2* part, int Ns,
                        int initial, const CoarseTab<double>* c64, const CoarseTab<float>* c32,
                        const DevTables& t, hipStream_t s);
// nx = the grid size of every problem, or 0 for problems of several grid
// sizes (up to nx_max) in one launch.
hipError_t launch_pipeline(int nx, int nx_max, bool fp64, const void* jobs, int njobs, const void* probs,
                           int* ticket, int* abort, int* progress, unsigned long long* trace, int grid,
                           hipStream_t s);
// LDS bytes of one pipeline workgroup for grid size nx (0 if unsupported).
size_t pipeline_lds(int nx, int nx_max, bool fp64);
// Pipeline workgroups resident on the current device at once (0 on error).
int pipeline_max_grid(int nx, int nx_max, bool fp64);
// Most slices one fine job of the pipelined solve steps together at grid size
// nx, for fine propagator `kind` (0 ETDRK4, 1 Strang).
int pipeline_fine_slices(int nx, bool fp64, int kind);
// Per-translation-unit pipeline kernels (pipe_*.hip): launch with `lds`
// bytes of LDS, and workgroups resident at once.
#define AP_PIPE_TU(tag)                                                                                  \
  hipError_t pipe_launch_##tag(int nx, size_t lds, const PipeJob* jobs, int njobs, const void* probs,    \
                               int* ticket, int* abort, int* progress, unsigned long long* trace, int grid, \
                               hipStream_t s);                                                           \
  int pipe_occupancy_##tag(int nx, size_t lds);
AP_PIPE_TU(f32)
AP_PIPE_TU(f64)
AP_PIPE_TU(mix1024_f32)
AP_PIPE_TU(mix2048_f32)
AP_PIPE_TU(mix2048_f64)
#undef AP_PIPE_TU

hipError_t launch_zero_ints(int* p, int n, hipStream_t s);
// FP32 / FP64 vector FMA throughput (TFLOP/s) and LDS read bandwidth (TB/s)
// of the current device, from microbenchmark kernels writing to `scratch`
// (at least 16 x CUs x 256 doubles); synchronises `s`.
hipError_t measure_peaks(void* scratch, size_t scratch_bytes, hipStream_t s, double* fp32_tflops,
                         double* fp64_tflops, double* lds_tbps);
// out[r] = max_n sqrt(part[r][n].x / part[r][n].y) for r < rows; NaN if *abort
hipError_t launch_resid(const double2* part, int Ns, int rows, double* out, const int* abort, hipStream_t s);
// Residual rows of several problems in one launch: row r reads Ns[r] partial
// sums at part[r] and writes out[r].
struct ResidRow {
  const double2* part;
  double* out;
  const int* stop;     // the problem's stopped level (NULL: never stops); rows past it get -1
  int Ns, level;
};
hipError_t launch_resid_rows(const ResidRow* rows, int nrows, const int* abort, hipStream_t s);
// If *stop = k in 1..K-1, copies U(k, 1..Ns) over U(K, 1..Ns) (the output rows).
hipError_t launch_select_level(cx<double>* U, int Ns, int K, int KP, const int* stop, hipStream_t s);

}  // namespace ap
