// Host-visible kernel launch interface of the HIP path (internal to the library).
#pragma once
#include <hip/hip_runtime.h>

#include "rsw_device.hpp"

namespace ap {

// Per-context device tables that depend only on the grid and F.
struct DevTables {
  const cx<double>* tw64 = nullptr;      // exp(-2 pi i t / N), t < N
  const cx<float>* tw32 = nullptr;
  const Basis<double>* basis64 = nullptr;  // per retained k: 1/omega_k, a_k/omega_k
  const Basis<float>* basis32 = nullptr;
  template <typename T> const cx<T>* tw() const;
  template <typename T> const Basis<T>* basis() const;
};
template <> inline const cx<double>* DevTables::tw<double>() const { return tw64; }
template <> inline const cx<float>* DevTables::tw<float>() const { return tw32; }
template <> inline const Basis<double>* DevTables::basis<double>() const { return basis64; }
template <> inline const Basis<float>* DevTables::basis<float>() const { return basis32; }

// Kernel-weighted time average: rot[m][k] = exp(-i omega_k s_m), w[m] = rho(m/M)/M.
template <typename T>
struct AvgTab {
  const cx<T>* rot;
  const T* w;
  int M;
};

// Asymptotic coarse step of length dT: hd[k] = exp(-nu k^4 dT/2),
// rotT[k] = exp(-i omega_k dT/eps) (the alpha = +1 factor of exp(-(dT/eps) L)).
template <typename T>
struct CoarseTab {
  AvgTab<T> avg;
  const T* hd;
  const cx<T>* rotT;
  T dT;
};

// Pipelined solve: one job = one coarse step (type 0) or one fine slice
// (type 1) of problem `prob` at iteration level k for slice n (1-based).
struct PipeJob {
  int prob, type, k, n;
};

// Per-problem device descriptor of the pipelined solve (layout in kernels.hip).
template <typename T>
struct PipeProb {
  cx<double>* U;       // [K+1][Ns+1][3][KP]
  cx<double>* F;       // [K][Ns+1][3][KP]
  cx<double>* G;       // [K+1][Ns+1][3][KP]
  double2* part;       // [K][Ns] residual partial sums
  int* done;           // [(2K+1) Ns] job flags
  int Ns, K, steps;
  const cx<double>* coef64;
  const cx<T>* coef;
  CoarseTab<T> ct;
};

hipError_t launch_to_modal(int nx, const double* phys, cx<double>* modal, int batch, const DevTables& t,
                           hipStream_t s);
hipError_t launch_to_physical(int nx, const cx<double>* modal, double* phys, int batch, const DevTables& t,
                              hipStream_t s);
hipError_t launch_nonlinear(int nx, bool fp64, const cx<double>* in, cx<double>* out, int batch,
                            const DevTables& t, hipStream_t s);
hipError_t launch_fine(int nx, bool fp64, const cx<double>* in, cx<double>* out, int batch, int steps,
                       const cx<double>* coef64, const cx<float>* coef32, const DevTables& t, hipStream_t s);
hipError_t launch_average(int nx, const cx<double>* in, cx<double>* out, int batch, const AvgTab<double>* av64,
                          const AvgTab<float>* av32, const DevTables& t, hipStream_t s);
hipError_t launch_coarse(int nx, const cx<double>* in, cx<double>* out, int batch, const CoarseTab<double>* c64,
                         const CoarseTab<float>* c32, const DevTables& t, hipStream_t s);
hipError_t launch_sweep(int nx, cx<double>* U, const cx<double>* Fine, cx<double>* Gold, double2* part, int Ns,
                        int initial, const CoarseTab<double>* c64, const CoarseTab<float>* c32,
                        const DevTables& t, hipStream_t s);
hipError_t launch_pipeline(int nx, bool fp64, const void* jobs, int njobs, const void* probs, int* ticket,
                           int* abort, int* progress, unsigned long long* trace, int grid, const DevTables& t,
                           hipStream_t s);
hipError_t launch_zero_ints(int* p, int n, hipStream_t s);
// out[r] = max_n sqrt(part[r][n].x / part[r][n].y) for r < rows; NaN if *abort
hipError_t launch_resid(const double2* part, int Ns, int rows, double* out, const int* abort, hipStream_t s);

}  // namespace ap
