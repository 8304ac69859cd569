// HIP kernels of the asymptotic parareal path (gfx950).
//
//   k_to_modal / k_to_physical : FP64 boundary transforms, physical grid values
//                                <-> modal amplitudes of the retained band
//   k_nonlinear                : dealiased N (Sec. 6.1)
//   k_fine                     : (fine_*.hip) ETDRK4 over `steps` steps, the
//                                parallel fine sweep of Alg. 4
//   k_average                  : kernel-weighted time average (eq. numerical
//                                average; Alg. 1), samples in flight together
//   k_coarse                   : one asymptotic coarse step per state (Alg. 2)
//   k_sweep                    : one serial coarse sweep of a parareal iteration
//                                with the FP64 correction (eq. HMM parareal
//                                iteration), used by the tolerance-driven solve
//   k_pipeline                 : the whole iteration as one persistent launch:
//                                coarse steps C(k,n) and fine slices F(k,n) of all
//                                iterations k are jobs taken in a topological
//                                order from one ticket counter, each waiting on
//                                the done flags of the jobs it reads
//   k_resid_rows               : r^k = max_n sqrt(num_n / den_n) per iteration
#include <algorithm>

#include "dispatch.hpp"
#include "fine_kernel.hpp"
#include "pipeline.hpp"

namespace ap {

// ------------------------------------------------- boundary transforms -----
// One state in one workgroup: physical [3][N] float64 -> modal [3][KP]
// complex float64 (projected), written to dst and, when dst2 is not null, to
// dst2 as well.
template <int NX, int NT>
__device__ __forceinline__ void to_modal_block(const double* __restrict__ src, cx<double>* __restrict__ dst,
                                               cx<double>* __restrict__ dst2, const cx<double>* __restrict__ tw_g,
                                               const Basis<double>* __restrict__ basis) {
  using G = Geo<NX>;
  using T = double;
  constexpr int P = G::P;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<T>* tw = reinterpret_cast<cx<T>*>(smem_raw);
  cx<T>* a = tw + NX;
  cx<T>* b = a + 3 * P;
  for (int i = threadIdx.x; i < NX; i += NT) tw[i] = tw_g[i];
  for (int i = threadIdx.x; i < 3 * P; i += NT) {
    const int f = i / P, n = i - f * P;
    a[f * P + n] = cx<T>{src[f * NX + 2 * n], src[f * NX + 2 * n + 1]};
  }
  __syncthreads();
  cx<T>* R = fft_lds<T, P, -1, NT>(a, b, 3, tw);
  const T half_over_n = T(0.5) / T(NX);
  for (int k = threadIdx.x; k < G::KP; k += NT) {
    const cx<T> w = tw[k];
    const int kc = (P - k) & (P - 1);
    cx<T> X[3];
    for (int f = 0; f < 3; ++f) {
      const cx<T> zk = R[f * P + k], zc = conj(R[f * P + kc]);
      X[f] = half_over_n * ((zk + zc) - mul_i(w * (zk - zc)));
    }
    if (k == 0) X[0].y = X[1].y = X[2].y = T(0);   // real signals: the mean is real
    cx<T> c[3];
    fields_to_modal<T>(X[0], X[1], X[2], basis[k], c);
    for (int al = 0; al < 3; ++al) dst[al * G::KP + k] = c[al];
    if (dst2)
      for (int al = 0; al < 3; ++al) dst2[al * G::KP + k] = c[al];
  }
}

// physical [B][3][N] float64 -> modal [B][3][KP] complex float64 (projected)
template <int NX, int NT>
__global__ void __launch_bounds__(NT) k_to_modal(const double* __restrict__ phys, cx<double>* __restrict__ modal,
                                                 const cx<double>* __restrict__ tw_g,
                                                 const Basis<double>* __restrict__ basis) {
  to_modal_block<NX, NT>(phys + size_t(blockIdx.x) * 3 * NX, modal + size_t(blockIdx.x) * 3 * Geo<NX>::KP, nullptr,
                         tw_g, basis);
}

// The problem of a batch that workgroup `block` belongs to, and the state's
// index within it.
__device__ __forceinline__ int batch_problem(const BoundaryBatch& b, int block, int& state) {
  int i = 0;
  while (i + 1 < b.n && block >= b.first[i + 1]) ++i;
  state = block - b.first[i];
  return i;
}

// One state per workgroup over a batch of problems of one grid size.
template <int NX, int NT>
__global__ void __launch_bounds__(NT) k_to_modal_batch(const BoundaryBatch b) {
  int j = 0;
  const BoundaryJob& jb = b.job[batch_problem(b, blockIdx.x, j)];
  constexpr size_t KS = size_t(3) * Geo<NX>::KP;
  cx<double>* dst2 = jb.dst2 ? jb.dst2 + j * KS : nullptr;
  to_modal_block<NX, NT>(static_cast<const double*>(jb.src) + j * size_t(3) * NX,
                         static_cast<cx<double>*>(jb.dst) + j * KS, dst2, jb.tw, jb.basis);
}

// One state in one workgroup: modal [3][KP] -> physical [3][N].
template <int NX, int NT>
__device__ __forceinline__ void to_physical_block(const cx<double>* __restrict__ src, double* __restrict__ dst,
                                                  const cx<double>* __restrict__ tw_g,
                                                  const Basis<double>* __restrict__ basis) {
  using G = Geo<NX>;
  using T = double;
  constexpr int P = G::P;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  // spec [3][P+1] shares the second FFT buffer: it is dead once the
  // pre-processed spectra are in `a`.
  cx<T>* tw = reinterpret_cast<cx<T>*>(smem_raw);
  cx<T>* a = tw + NX;
  cx<T>* spec = a + 3 * P;
  cx<T>* b = spec;
  for (int i = threadIdx.x; i < NX; i += NT) tw[i] = tw_g[i];
  zero_spec_tail<T, NX, NT>(spec, 1);
  const T s = T(0.70710678118654752440);
  for (int k = threadIdx.x; k < G::KP; k += NT) {
    const cx<T> c0 = src[k], c1 = src[G::KP + k], c2 = src[2 * G::KP + k];
    const Basis<T> bs = basis[k];
    spec[k] = s * (c0 + c2);
    spec[(P + 1) + k] = mul_i((bs.iw * s) * (c0 - c2) + bs.aw * c1);
    spec[2 * (P + 1) + k] = (bs.aw * s) * (c2 - c0) + bs.iw * c1;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < 3 * P; i += NT) {
    const int v = i / P, k = i - v * P;
    const cx<T>* X = spec + v * (P + 1);
    const cx<T> xk = X[k], xc = conj(X[P - k]);
    a[v * P + k] = (xk + xc) + mul_i(conj(tw[k]) * (xk - xc));
  }
  __syncthreads();
  cx<T>* R = fft_lds<T, P, +1, NT>(a, b, 3, tw);
  for (int i = threadIdx.x; i < 3 * P; i += NT) {
    const int f = i / P, n = i - f * P;
    const cx<T> z = R[f * P + n];
    dst[f * NX + 2 * n] = z.x;
    dst[f * NX + 2 * n + 1] = z.y;
  }
}

// modal [B][3][KP] -> physical [B][3][N]
template <int NX, int NT>
__global__ void __launch_bounds__(NT) k_to_physical(const cx<double>* __restrict__ modal, double* __restrict__ phys,
                                                    const cx<double>* __restrict__ tw_g,
                                                    const Basis<double>* __restrict__ basis) {
  to_physical_block<NX, NT>(modal + size_t(blockIdx.x) * 3 * Geo<NX>::KP, phys + size_t(blockIdx.x) * 3 * NX, tw_g,
                            basis);
}

template <int NX, int NT>
__global__ void __launch_bounds__(NT) k_to_physical_batch(const BoundaryBatch b) {
  int j = 0;
  const BoundaryJob& jb = b.job[batch_problem(b, blockIdx.x, j)];
  to_physical_block<NX, NT>(static_cast<const cx<double>*>(jb.src) + j * size_t(3) * Geo<NX>::KP,
                            static_cast<double*>(jb.dst) + j * size_t(3) * NX, jb.tw, jb.basis);
}

// ------------------------------------------------------- nonlinear term -----
template <typename T, int NX, int NT>
__global__ void __launch_bounds__(NT) k_nonlinear(const cx<double>* __restrict__ Uin, cx<double>* __restrict__ Nout,
                                                  const cx<T>* __restrict__ tw, const Basis<T>* __restrict__ basis) {
  using E_ = Engine<T, NX, NT, 1>;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  E_ en(smem_raw, tw);
  const cx<double>* src = Uin + size_t(blockIdx.x) * 3 * E_::KP;
  cx<double>* dst = Nout + size_t(blockIdx.x) * 3 * E_::KP;
  cx<T> c[E_::MPT][3], n[E_::MPT][3];
  Basis<T> bs[E_::MPT];
#pragma unroll
  for (int j = 0; j < E_::MPT; ++j) {
    const int k = en.valid(j) ? en.mode(j) : 0;
    bs[j] = basis[k];
    for (int al = 0; al < 3; ++al) c[j][al] = en.valid(j) ? cvt<T>(src[al * E_::KP + k]) : czero<T>();
  }
  en.neval(0, c, n, bs);
#pragma unroll
  for (int j = 0; j < E_::MPT; ++j)
    if (en.valid(j))
      for (int al = 0; al < 3; ++al) dst[al * E_::KP + en.mode(j)] = cvt<double>(n[j][al]);
}

template <typename T, int NX, int NT>
__global__ void __launch_bounds__(NT) k_strang(const cx<double>* __restrict__ Uin, cx<double>* __restrict__ Uout,
                                               int batch, int steps, double h, const cx<double>* __restrict__ coef64,
                                               const cx<T>* __restrict__ tw, const Basis<T>* __restrict__ basis) {
  constexpr int S = fine_slots<T, NX, NT>();
  using E_ = Engine<T, NX, NT, S>;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  E_ en(smem_raw, tw);
  const size_t st = size_t(3) * E_::KP;
  const int first = blockIdx.x * E_::jmax();
  const int J = min(E_::jmax(), batch - first);
  strang_job<T, NX, NT, S>(en, J, Uin + first * st, Uin + (first + 1) * st, Uout + first * st, steps, coef64, h,
                           basis);
}

// ---------------------------------------------------- average and coarse ---
template <typename T, int NX, int NT, int S>
__global__ void __launch_bounds__(NT) k_average(const cx<double>* __restrict__ Uin, cx<double>* __restrict__ Nout,
                                                AvgTab<T> av, const cx<T>* __restrict__ tw,
                                                const Basis<T>* __restrict__ basis) {
  using E_ = Engine<T, NX, NT, S>;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  E_ en(smem_raw, tw);
  const cx<double>* src = Uin + size_t(blockIdx.x) * 3 * E_::KP;
  cx<double>* dst = Nout + size_t(blockIdx.x) * 3 * E_::KP;
  cx<T> y[E_::MPT][3], acc[E_::MPT][3];
  load_owned<T, NX, NT, S>(en, src, y);
  nbar_owned<T, NX, NT, S>(en, y, acc, av, basis);
#pragma unroll
  for (int j = 0; j < E_::MPT; ++j)
    if (en.valid(j))
      for (int al = 0; al < 3; ++al) dst[al * E_::KP + en.mode(j)] = cvt<double>(acc[j][al]);
}

template <typename T, int NX, int NT, int S>
__global__ void __launch_bounds__(NT) k_coarse(const cx<double>* __restrict__ Uin, cx<double>* __restrict__ Uout,
                                               CoarseTab<T> ct, const cx<T>* __restrict__ tw,
                                               const Basis<T>* __restrict__ basis) {
  using E_ = Engine<T, NX, NT, S>;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  E_ en(smem_raw, tw);
  const size_t st = size_t(3) * E_::KP;
  cx<double>* o = Uout + blockIdx.x * st;
  coarse_job<T, NX, NT, S>(en, ct, basis, Uin + blockIdx.x * st, o, o, nullptr, nullptr, nullptr, nullptr);
}

// One workgroup runs the serial sweep over n = 1..Ns of one iteration.
// U, Fine, Gold: modal FP64 [Ns+1][3][KP], updated in place.
template <typename T, int NX, int NT, int S>
__global__ void __launch_bounds__(NT) k_sweep(cx<double>* __restrict__ U, const cx<double>* __restrict__ Fine,
                                              cx<double>* __restrict__ Gold, double2* __restrict__ part, int Ns,
                                              int initial, CoarseTab<T> ct, const cx<T>* __restrict__ tw,
                                              const Basis<T>* __restrict__ basis) {
  using E_ = Engine<T, NX, NT, S>;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  E_ en(smem_raw, tw);
  const size_t st = size_t(3) * E_::KP;
  for (int n = 1; n <= Ns; ++n) {
    cx<double>* Un = U + n * st;
    cx<double>* Gn = Gold + n * st;
    if (initial)
      coarse_job<T, NX, NT, S>(en, ct, basis, U + (n - 1) * st, Un, Gn, nullptr, nullptr, nullptr, nullptr);
    else
      coarse_job<T, NX, NT, S>(en, ct, basis, U + (n - 1) * st, Un, Gn, Gn, Fine + n * st, Un, part + (n - 1));
  }
}

__global__ void k_zero_ints(int* p, int n) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = 0;
}

// rows r = 0..R-1: out[r] = max_n sqrt(part[r][n].x / part[r][n].y); NaN after an abort.
__device__ __forceinline__ void resid_row(const double2* __restrict__ row, int Ns, double* out, bool aborted) {
  __shared__ double red[256];
  double m = 0.0;
  for (int n = threadIdx.x; n < Ns; n += 256) {
    const double2 p = row[n];
    const double r = p.y > 0.0 ? sqrt(p.x / p.y) : (p.x > 0.0 ? INFINITY : 0.0);
    m = (r > m || r != r) ? r : m;
  }
  red[threadIdx.x] = m;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (threadIdx.x < off) {
      const double o = red[threadIdx.x + off];
      if (o > red[threadIdx.x] || o != o) red[threadIdx.x] = o;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = aborted ? NAN : red[0];
}

__global__ void __launch_bounds__(256) k_resid_rows(const double2* __restrict__ part, int Ns,
                                                     double* __restrict__ out, const int* __restrict__ abort) {
  resid_row(part + size_t(blockIdx.x) * Ns, Ns, out + blockIdx.x, abort && *abort);
}

__global__ void __launch_bounds__(256) k_resid_table(const ResidRow* __restrict__ rows,
                                                      const int* __restrict__ abort) {
  const ResidRow r = rows[blockIdx.x];
  if (r.stop && *r.stop > 0 && r.level > *r.stop) {       // iteration not run: the solve stopped before it
    if (threadIdx.x == 0) *r.out = -1.0;
    return;
  }
  resid_row(r.part, r.Ns, r.out, abort && *abort);
}

// U(K, 1..Ns) <- U(k, 1..Ns) when the solve stopped at level k < K (the
// output rows; slice 0, the initial state, is held at level K only).
__global__ void __launch_bounds__(256) k_select_level(cx<double>* __restrict__ U, int Ns, int K, int KP,
                                                       const int* __restrict__ stop) {
  const int k = *stop;
  if (k <= 0 || k >= K) return;
  const size_t row = size_t(Ns + 1) * 3 * KP;
  const size_t n = size_t(Ns) * 3 * KP;
  const cx<double>* src = U + size_t(k) * row + 3 * KP;
  cx<double>* dst = U + size_t(K) * row + 3 * KP;
  for (size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += size_t(gridDim.x) * blockDim.x)
    dst[i] = src[i];
}

// ------------------------------------------------------------- launchers ---
// Threads per workgroup: the fine batch uses three wavefronts (one per field
// transform) or enough threads to own every retained mode; the
// sample-parallel kernels use 512 threads with as many state slots as the
// LDS budget allows.
// 512 threads: eight wavefronts with up to 256 VGPRs each (the jobs keep the
// ETDRK4 state, coefficients and a register DFT live at once).
template <typename T, int NX>
constexpr int avg_threads() {
  return 512;
}

template <int NX>
static hipError_t to_modal_nx(const double* phys, cx<double>* modal, int batch, const DevTables& t, hipStream_t s) {
  constexpr int NT = 256;
  const size_t lds = (NX + 6 * Geo<NX>::P) * sizeof(cx<double>);
  prep_lds(k_to_modal<NX, NT>, lds);
  hipLaunchKernelGGL((k_to_modal<NX, NT>), dim3(batch), dim3(NT), lds, s, phys, modal, t.tw64, t.basis64);
  return hipGetLastError();
}

template <int NX>
static hipError_t to_physical_nx(const cx<double>* modal, double* phys, int batch, const DevTables& t, hipStream_t s) {
  constexpr int NT = 256;
  const size_t lds = (NX + 3 * (Geo<NX>::P + 1) + 3 * Geo<NX>::P) * sizeof(cx<double>);
  prep_lds(k_to_physical<NX, NT>, lds);
  hipLaunchKernelGGL((k_to_physical<NX, NT>), dim3(batch), dim3(NT), lds, s, modal, phys, t.tw64, t.basis64);
  return hipGetLastError();
}

template <int NX>
static hipError_t to_modal_batch_nx(const BoundaryBatch& b, hipStream_t s) {
  constexpr int NT = 256;
  const size_t lds = (NX + 6 * Geo<NX>::P) * sizeof(cx<double>);
  prep_lds(k_to_modal_batch<NX, NT>, lds);
  hipLaunchKernelGGL((k_to_modal_batch<NX, NT>), dim3(b.first[b.n]), dim3(NT), lds, s, b);
  return hipGetLastError();
}

template <int NX>
static hipError_t to_physical_batch_nx(const BoundaryBatch& b, hipStream_t s) {
  constexpr int NT = 256;
  const size_t lds = (NX + 3 * (Geo<NX>::P + 1) + 3 * Geo<NX>::P) * sizeof(cx<double>);
  prep_lds(k_to_physical_batch<NX, NT>, lds);
  hipLaunchKernelGGL((k_to_physical_batch<NX, NT>), dim3(b.first[b.n]), dim3(NT), lds, s, b);
  return hipGetLastError();
}

template <typename T, int NX>
static hipError_t nonlinear_nx(const cx<double>* in, cx<double>* out, int batch, const DevTables& t, hipStream_t s) {
  constexpr int NT = fine_threads<T, NX>();
  const size_t lds = Engine<T, NX, NT, 1>::lds_bytes();
  prep_lds(k_nonlinear<T, NX, NT>, lds);
  hipLaunchKernelGGL((k_nonlinear<T, NX, NT>), dim3(batch), dim3(NT), lds, s, in, out, t.tw<T>(), t.basis<T>());
  return hipGetLastError();
}

template <typename T, int NX>
static hipError_t strang_nx(const cx<double>* in, cx<double>* out, int batch, int steps, double h,
                            const cx<double>* coef64, const DevTables& t, hipStream_t s) {
  constexpr int NT = fine_threads<T, NX>();
  const size_t lds = Engine<T, NX, NT, fine_slots<T, NX, NT>()>::lds_bytes();
  const int J = fine_slices<T, NX>();
  prep_lds(k_strang<T, NX, NT>, lds);
  hipLaunchKernelGGL((k_strang<T, NX, NT>), dim3((batch + J - 1) / J), dim3(NT), lds, s, in, out, batch, steps, h,
                     coef64, t.tw<T>(), t.basis<T>());
  return hipGetLastError();
}

template <typename T, int NX>
static hipError_t average_nx(const cx<double>* in, cx<double>* out, int batch, const AvgTab<T>& av,
                             const DevTables& t, hipStream_t s) {
  constexpr int NT = avg_threads<T, NX>();
  constexpr int S = max_slots<T, NX, NT>();
  const size_t lds = Engine<T, NX, NT, S>::lds_bytes();
  prep_lds(k_average<T, NX, NT, S>, lds);
  hipLaunchKernelGGL((k_average<T, NX, NT, S>), dim3(batch), dim3(NT), lds, s, in, out, av, t.tw<T>(), t.basis<T>());
  return hipGetLastError();
}

template <typename T, int NX>
static hipError_t coarse_nx(const cx<double>* in, cx<double>* out, int batch, const CoarseTab<T>& ct,
                            const DevTables& t, hipStream_t s) {
  constexpr int NT = avg_threads<T, NX>();
  constexpr int S = max_slots<T, NX, NT>();
  const size_t lds = Engine<T, NX, NT, S>::lds_bytes();
  prep_lds(k_coarse<T, NX, NT, S>, lds);
  hipLaunchKernelGGL((k_coarse<T, NX, NT, S>), dim3(batch), dim3(NT), lds, s, in, out, ct, t.tw<T>(), t.basis<T>());
  return hipGetLastError();
}

template <typename T, int NX>
static hipError_t sweep_nx(cx<double>* U, const cx<double>* Fine, cx<double>* Gold, double2* part, int Ns,
                           int initial, const CoarseTab<T>& ct, const DevTables& t, hipStream_t s) {
  constexpr int NT = avg_threads<T, NX>();
  constexpr int S = max_slots<T, NX, NT>();
  const size_t lds = Engine<T, NX, NT, S>::lds_bytes();
  prep_lds(k_sweep<T, NX, NT, S>, lds);
  hipLaunchKernelGGL((k_sweep<T, NX, NT, S>), dim3(1), dim3(NT), lds, s, U, Fine, Gold, part, Ns, initial, ct,
                     t.tw<T>(), t.basis<T>());
  return hipGetLastError();
}

hipError_t launch_to_modal(int nx, const double* phys, cx<double>* modal, int batch, const DevTables& t,
                           hipStream_t s) {
  AP_DISPATCH_NX(nx, to_modal_nx<NX>(phys, modal, batch, t, s));
}
hipError_t launch_to_physical(int nx, const cx<double>* modal, double* phys, int batch, const DevTables& t,
                              hipStream_t s) {
  AP_DISPATCH_NX(nx, to_physical_nx<NX>(modal, phys, batch, t, s));
}
hipError_t launch_to_modal_batch(int nx, const BoundaryBatch& b, hipStream_t s) {
  if (b.n < 1 || b.n > kBoundaryBatch || b.first[b.n] <= 0) return hipErrorInvalidValue;
  AP_DISPATCH_NX(nx, to_modal_batch_nx<NX>(b, s));
}
hipError_t launch_to_physical_batch(int nx, const BoundaryBatch& b, hipStream_t s) {
  if (b.n < 1 || b.n > kBoundaryBatch || b.first[b.n] <= 0) return hipErrorInvalidValue;
  AP_DISPATCH_NX(nx, to_physical_batch_nx<NX>(b, s));
}
hipError_t launch_nonlinear(int nx, bool fp64, const cx<double>* in, cx<double>* out, int batch,
                            const DevTables& t, hipStream_t s) {
  if (fp64) AP_DISPATCH_NX(nx, (nonlinear_nx<double, NX>(in, out, batch, t, s)));
  AP_DISPATCH_NX(nx, (nonlinear_nx<float, NX>(in, out, batch, t, s)));
}
hipError_t launch_fine(int nx, bool fp64, const cx<double>* in, cx<double>* out, int batch, int steps,
                       const cx<double>* coef64, const cx<float>* coef32, const DevTables& t, hipStream_t s,
                       int shape) {
  return fp64 ? launch_fine_f64(nx, shape, in, out, batch, steps, coef64, t, s)
              : launch_fine_f32(nx, shape, in, out, batch, steps, coef64, coef32, t, s);
}
hipError_t launch_strang(int nx, bool fp64, const cx<double>* in, cx<double>* out, int batch, int steps, double h,
                         const cx<double>* coef64, const DevTables& t, hipStream_t s) {
  if (fp64) AP_DISPATCH_NX(nx, (strang_nx<double, NX>(in, out, batch, steps, h, coef64, t, s)));
  AP_DISPATCH_NX(nx, (strang_nx<float, NX>(in, out, batch, steps, h, coef64, t, s)));
}
hipError_t launch_average(int nx, const cx<double>* in, cx<double>* out, int batch, const AvgTab<double>* av64,
                          const AvgTab<float>* av32, const DevTables& t, hipStream_t s) {
  if (av64) AP_DISPATCH_NX(nx, (average_nx<double, NX>(in, out, batch, *av64, t, s)));
  AP_DISPATCH_NX(nx, (average_nx<float, NX>(in, out, batch, *av32, t, s)));
}
hipError_t launch_coarse(int nx, const cx<double>* in, cx<double>* out, int batch, const CoarseTab<double>* c64,
                         const CoarseTab<float>* c32, const DevTables& t, hipStream_t s) {
  if (c64) AP_DISPATCH_NX(nx, (coarse_nx<double, NX>(in, out, batch, *c64, t, s)));
  AP_DISPATCH_NX(nx, (coarse_nx<float, NX>(in, out, batch, *c32, t, s)));
}
hipError_t launch_sweep(int nx, cx<double>* U, const cx<double>* Fine, cx<double>* Gold, double2* part, int Ns,
                        int initial, const CoarseTab<double>* c64, const CoarseTab<float>* c32,
                        const DevTables& t, hipStream_t s) {
  if (c64) AP_DISPATCH_NX(nx, (sweep_nx<double, NX>(U, Fine, Gold, part, Ns, initial, *c64, t, s)));
  AP_DISPATCH_NX(nx, (sweep_nx<float, NX>(U, Fine, Gold, part, Ns, initial, *c32, t, s)));
}
// pipelined solve: the kernels live in the pipe_*.hip translation units
size_t pipeline_lds(int nx, int nx_max, bool fp64) {
  return fp64 ? pipeline_lds_t<double>(nx, nx_max) : pipeline_lds_t<float>(nx, nx_max);
}

using PipeLaunchFn = hipError_t (*)(int, size_t, const PipeJob*, int, const void*, int*, int*, int*,
                                    unsigned long long*, int, hipStream_t);
using PipeOccFn = int (*)(int, size_t);

// kernel for grid size nx (0: several sizes up to nx_max in one launch)
static bool pipe_kernel(int nx, int nx_max, bool fp64, PipeLaunchFn* fn, PipeOccFn* occ) {
  if (nx > 0) {
    *fn = fp64 ? pipe_launch_f64 : pipe_launch_f32;
    *occ = fp64 ? pipe_occupancy_f64 : pipe_occupancy_f32;
  } else if (fp64) {
    *fn = pipe_launch_mix2048_f64;
    *occ = pipe_occupancy_mix2048_f64;
  } else if (nx_max <= 1024) {
    *fn = pipe_launch_mix1024_f32;
    *occ = pipe_occupancy_mix1024_f32;
  } else {
    *fn = pipe_launch_mix2048_f32;
    *occ = pipe_occupancy_mix2048_f32;
  }
  return true;
}

template <typename T>
static int pipeline_fine_slices_t(int nx, int kind) {
  switch (nx) {
    case 64: return pipe_fine_slices<T, 64>(kind);
    case 128: return pipe_fine_slices<T, 128>(kind);
    case 256: return pipe_fine_slices<T, 256>(kind);
    case 512: return pipe_fine_slices<T, 512>(kind);
    case 1024: return pipe_fine_slices<T, 1024>(kind);
    default: return pipe_fine_slices<T, 2048>(kind);
  }
}
int pipeline_fine_slices(int nx, bool fp64, int kind) {
  return fp64 ? pipeline_fine_slices_t<double>(nx, kind) : pipeline_fine_slices_t<float>(nx, kind);
}

int pipeline_max_grid(int nx, int nx_max, bool fp64) {
  const size_t lds = pipeline_lds(nx, nx_max, fp64);
  PipeLaunchFn fn;
  PipeOccFn occ;
  if (lds == 0 || !pipe_kernel(nx, nx_max, fp64, &fn, &occ)) return 0;
  return occ(nx, lds);
}

hipError_t launch_pipeline(int nx, int nx_max, bool fp64, const void* jobs, int njobs, const void* probs,
                           int* ticket, int* abort, int* progress, unsigned long long* trace, int grid,
                           hipStream_t s) {
  const size_t lds = pipeline_lds(nx, nx_max, fp64);
  PipeLaunchFn fn;
  PipeOccFn occ;
  if (lds == 0 || !pipe_kernel(nx, nx_max, fp64, &fn, &occ)) return hipErrorInvalidValue;
  return fn(nx, lds, static_cast<const PipeJob*>(jobs), njobs, probs, ticket, abort, progress, trace, grid, s);
}


hipError_t launch_zero_ints(int* p, int n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int blocks = (n + 255) / 256 < 64 ? (n + 255) / 256 : 64;
  hipLaunchKernelGGL(k_zero_ints, dim3(blocks), dim3(256), 0, s, p, n);
  return hipGetLastError();
}
hipError_t launch_resid(const double2* part, int Ns, int rows, double* out, const int* abort, hipStream_t s) {
  if (rows <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_resid_rows, dim3(rows), dim3(256), 0, s, part, Ns, out, abort);
  return hipGetLastError();
}
hipError_t launch_select_level(cx<double>* U, int Ns, int K, int KP, const int* stop, hipStream_t s) {
  const size_t n = size_t(Ns) * 3 * KP;
  const int blocks = int(std::max<size_t>(1, std::min<size_t>((n + 255) / 256, 1024)));
  hipLaunchKernelGGL(k_select_level, dim3(blocks), dim3(256), 0, s, U, Ns, K, KP, stop);
  return hipGetLastError();
}
hipError_t launch_resid_rows(const ResidRow* rows, int nrows, const int* abort, hipStream_t s) {
  if (nrows <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_resid_table, dim3(nrows), dim3(256), 0, s, rows, abort);
  return hipGetLastError();
}

}  // namespace ap
