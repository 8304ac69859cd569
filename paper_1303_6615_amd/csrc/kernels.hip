// HIP kernels of the asymptotic parareal path (gfx950).
//
//   k_to_modal / k_to_physical : FP64 boundary transforms, physical grid values
//                                <-> modal amplitudes of the retained band
//   k_nonlinear                : dealiased N (Sec. 6.1)
//   k_fine                     : ETDRK4 over `steps` steps, one slice per workgroup
//                                (the parallel fine sweep of Alg. 4)
//   k_average                  : kernel-weighted time average (eq. numerical
//                                average; Alg. 1), samples in flight together
//   k_coarse                   : one asymptotic coarse step per state (Alg. 2)
//   k_sweep                    : the serial coarse sweep of one parareal
//                                iteration with the FP64 correction
//                                U_n = Fine_n + (G_new - G_old) and the residual
//                                partial sums (eq. HMM parareal iteration; Alg. 4)
//   k_resid                    : r^k = max_n sqrt(num_n / den_n)
#include "launch.hpp"
#include "rsw_device.hpp"

namespace ap {

// ------------------------------------------------------------ helpers -----
template <int NX, int NT>
struct Own {
  static constexpr int KP = Geo<NX>::KP;
  static constexpr int MPT = (KP + NT - 1) / NT;
  static __device__ __forceinline__ int mode(int j) { return threadIdx.x + j * NT; }
  static __device__ __forceinline__ bool valid(int j) { return mode(j) < KP; }
};

template <typename T>
__device__ __forceinline__ cx<T> rot_in(cx<T> c, cx<T> e, int alpha_idx) {
  // exp(-i alpha omega s) with e = exp(-i omega s): alpha=+1 -> e, -1 -> conj(e), 0 -> 1
  return alpha_idx == 2 ? c * e : (alpha_idx == 0 ? c * conj(e) : c);
}
template <typename T>
__device__ __forceinline__ cx<T> rot_out(cx<T> c, cx<T> e, int alpha_idx) {
  return alpha_idx == 2 ? c * conj(e) : (alpha_idx == 0 ? c * e : c);
}

// ------------------------------------------------- boundary transforms -----
// physical [B][3][N] float64 -> modal [B][3][KP] complex float64 (projected)
template <int NX, int NT>
__global__ void __launch_bounds__(NT) k_to_modal(const double* __restrict__ phys, cx<double>* __restrict__ modal,
                                                 const cx<double>* __restrict__ tw,
                                                 const Basis<double>* __restrict__ basis) {
  using G = Geo<NX>;
  using T = double;
  constexpr int P = G::P;
  extern __shared__ unsigned char smem_raw[];
  cx<T>* a = reinterpret_cast<cx<T>*>(smem_raw);
  cx<T>* b = a + 3 * P;
  const double* src = phys + size_t(blockIdx.x) * 3 * NX;
  for (int i = threadIdx.x; i < 3 * P; i += NT) {
    const int f = i / P, n = i - f * P;
    a[f * P + n] = cx<T>{src[f * NX + 2 * n], src[f * NX + 2 * n + 1]};
  }
  __syncthreads();
  cx<T>* R = fft_lds<T, P, -1, NT>(a, b, 3, tw);
  const T half_over_n = T(0.5) / T(NX);
  cx<double>* dst = modal + size_t(blockIdx.x) * 3 * G::KP;
  for (int k = threadIdx.x; k < G::KP; k += NT) {
    const cx<T> w = tw[k];
    const int kc = (P - k) & (P - 1);
    cx<T> X[3];
    for (int f = 0; f < 3; ++f) {
      const cx<T> zk = R[f * P + k], zc = conj(R[f * P + kc]);
      X[f] = half_over_n * ((zk + zc) - mul_i(w * (zk - zc)));
    }
    if (k == 0) {  // real signals: the mean is real
      X[0].y = X[1].y = X[2].y = T(0);
    }
    cx<T> c[3];
    fields_to_modal<T>(X[0], X[1], X[2], basis[k], c);
    for (int al = 0; al < 3; ++al) dst[al * G::KP + k] = c[al];
  }
}

// modal [B][3][KP] -> physical [B][3][N]
template <int NX, int NT>
__global__ void __launch_bounds__(NT) k_to_physical(const cx<double>* __restrict__ modal, double* __restrict__ phys,
                                                    const cx<double>* __restrict__ tw,
                                                    const Basis<double>* __restrict__ basis) {
  using G = Geo<NX>;
  using T = double;
  constexpr int P = G::P;
  extern __shared__ unsigned char smem_raw[];
  cx<T>* spec = reinterpret_cast<cx<T>*>(smem_raw);
  cx<T>* a = spec + 3 * (P + 1);
  cx<T>* b = a + 3 * P;
  zero_spec_tail<T, NX, NT>(spec, 1);
  const cx<double>* src = modal + size_t(blockIdx.x) * 3 * G::KP;
  const T s = T(0.70710678118654752440);
  for (int k = threadIdx.x; k < G::KP; k += NT) {
    const cx<T> c0 = src[k], c1 = src[G::KP + k], c2 = src[2 * G::KP + k];
    const Basis<T> bs = basis[k];
    const cx<T> v1 = s * (c0 + c2);
    const cx<T> v2 = mul_i((bs.iw * s) * (c0 - c2) + bs.aw * c1);
    const cx<T> h = (bs.aw * s) * (c2 - c0) + bs.iw * c1;
    spec[k] = v1;
    spec[(P + 1) + k] = v2;
    spec[2 * (P + 1) + k] = h;
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
  double* dst = phys + size_t(blockIdx.x) * 3 * NX;
  for (int i = threadIdx.x; i < 3 * P; i += NT) {
    const int f = i / P, n = i - f * P;
    const cx<T> z = R[f * P + n];
    dst[f * NX + 2 * n] = z.x;
    dst[f * NX + 2 * n + 1] = z.y;
  }
}

// ------------------------------------------------------- nonlinear term -----
template <typename T, int NX, int NT>
__global__ void __launch_bounds__(NT) k_nonlinear(const cx<double>* __restrict__ Uin, cx<double>* __restrict__ Nout,
                                                  const cx<T>* __restrict__ tw, const Basis<T>* __restrict__ basis) {
  using G = Geo<NX>;
  using O = Own<NX, NT>;
  extern __shared__ unsigned char smem_raw[];
  cx<T>* spec = reinterpret_cast<cx<T>*>(smem_raw);
  cx<T>* a = spec + Lds<T, NX>::spec_elems(1);
  cx<T>* b = a + Lds<T, NX>::work_elems(1);
  zero_spec_tail<T, NX, NT>(spec, 1);
  const cx<double>* src = Uin + size_t(blockIdx.x) * 3 * G::KP;
  cx<double>* dst = Nout + size_t(blockIdx.x) * 3 * G::KP;
#pragma unroll
  for (int j = 0; j < O::MPT; ++j) {
    if (!O::valid(j)) continue;
    const int k = O::mode(j);
    cx<T> c[3];
    for (int al = 0; al < 3; ++al) c[al] = cvt<T>(src[al * G::KP + k]);
    put_fields<T, NX>(spec, 0, k, c, basis[k]);
  }
  __syncthreads();
  cx<T>* R = nonlinear_core<T, NX, NT>(spec, a, b, 1, tw);
#pragma unroll
  for (int j = 0; j < O::MPT; ++j) {
    if (!O::valid(j)) continue;
    const int k = O::mode(j);
    cx<T> n[3];
    get_N<T, NX>(R, 0, k, basis[k], tw, n);
    for (int al = 0; al < 3; ++al) dst[al * G::KP + k] = cvt<double>(n[al]);
  }
}

// ------------------------------------------------------------ fine ETDRK4 ---
// Coefficient tables [8][3][KP] per precision: E_hi, E_lo, E2_hi, E2_lo, Q, f1,
// 2*f2, f3 for each (alpha, k).  The state and the step accumulator
// u+ = E u + f1 N(u) + 2f2 (N(a) + N(b)) + f3 N(c) are kept in FP64 in both
// precisions (E from the FP64 table): the slowly varying modes change by less
// than half an FP32 ulp per step, so an FP32 state would drop those increments
// coherently step after step.  With T = float the stage states a, b, c, the
// nonlinear evaluations and the products f*N run in FP32.
template <typename T, int NX, int NT>
__global__ void __launch_bounds__(NT) k_fine(const cx<double>* __restrict__ Uin, cx<double>* __restrict__ Uout,
                                             int steps, const cx<double>* __restrict__ coef64,
                                             const cx<T>* __restrict__ coef, const cx<T>* __restrict__ tw,
                                             const Basis<T>* __restrict__ basis) {
  using G = Geo<NX>;
  using O = Own<NX, NT>;
  constexpr int KP = G::KP;
  constexpr int MPT = O::MPT;
  extern __shared__ unsigned char smem_raw[];
  cx<T>* spec = reinterpret_cast<cx<T>*>(smem_raw);
  cx<T>* a_buf = spec + Lds<T, NX>::spec_elems(1);
  cx<T>* b_buf = a_buf + Lds<T, NX>::work_elems(1);
  zero_spec_tail<T, NX, NT>(spec, 1);

  const cx<double>* src = Uin + size_t(blockIdx.x) * 3 * KP;
  cx<double>* dst = Uout + size_t(blockIdx.x) * 3 * KP;

  cx<double> c[MPT][3], cE[MPT][3];
  cx<T> cE2[MPT][3], cQ[MPT][3], cf1[MPT][3], cf2[MPT][3], cf3[MPT][3];
  Basis<T> bs[MPT];
#pragma unroll
  for (int j = 0; j < MPT; ++j) {
    const int k = O::mode(j) < KP ? O::mode(j) : KP - 1;
    bs[j] = basis[k];
#pragma unroll
    for (int al = 0; al < 3; ++al) {
      const int o = al * KP + k;
      c[j][al] = src[o];
      cE[j][al] = coef64[0 * 3 * KP + o];
      cE2[j][al] = coef[2 * 3 * KP + o];
      cQ[j][al] = coef[4 * 3 * KP + o];
      cf1[j][al] = coef[5 * 3 * KP + o];
      cf2[j][al] = coef[6 * 3 * KP + o];
      cf3[j][al] = coef[7 * 3 * KP + o];
    }
  }

  // N of the modal state x (per owned mode) -> n
  auto neval = [&](cx<T> (&x)[MPT][3], cx<T> (&n)[MPT][3]) {
#pragma unroll
    for (int j = 0; j < MPT; ++j)
      if (O::valid(j)) put_fields<T, NX>(spec, 0, O::mode(j), x[j], bs[j]);
    __syncthreads();
    cx<T>* R = nonlinear_core<T, NX, NT>(spec, a_buf, b_buf, 1, tw);
#pragma unroll
    for (int j = 0; j < MPT; ++j)
      if (O::valid(j)) get_N<T, NX>(R, 0, O::mode(j), bs[j], tw, n[j]);
  };

  cx<T> Nx[MPT][3], st[MPT][3], E2c[MPT][3], Nu[MPT][3];
  cx<double> acc[MPT][3];
  for (int step = 0; step < steps; ++step) {
#pragma unroll
    for (int j = 0; j < MPT; ++j)
#pragma unroll
      for (int al = 0; al < 3; ++al) st[j][al] = cvt<T>(c[j][al]);
    neval(st, Nu);
#pragma unroll
    for (int j = 0; j < MPT; ++j)
#pragma unroll
      for (int al = 0; al < 3; ++al) {
        E2c[j][al] = cE2[j][al] * st[j][al];
        st[j][al] = cfma(cQ[j][al], Nu[j][al], E2c[j][al]);                                   // a
        acc[j][al] = cE[j][al] * c[j][al] + cvt<double>(cf1[j][al] * Nu[j][al]);
      }
    neval(st, Nx);                                                                            // N(a)
#pragma unroll
    for (int j = 0; j < MPT; ++j)
#pragma unroll
      for (int al = 0; al < 3; ++al) {
        acc[j][al] = acc[j][al] + cvt<double>(cf2[j][al] * Nx[j][al]);
        const cx<T> a_ = st[j][al];
        st[j][al] = cfma(cQ[j][al], Nx[j][al], E2c[j][al]);                                   // b
        E2c[j][al] = cE2[j][al] * a_;                                                         // E2 a
      }
    neval(st, Nx);                                                                            // N(b)
#pragma unroll
    for (int j = 0; j < MPT; ++j)
#pragma unroll
      for (int al = 0; al < 3; ++al) {
        acc[j][al] = acc[j][al] + cvt<double>(cf2[j][al] * Nx[j][al]);
        st[j][al] = cfma(cQ[j][al], T(2) * Nx[j][al] - Nu[j][al], E2c[j][al]);                // c
      }
    neval(st, Nx);                                                                            // N(c)
#pragma unroll
    for (int j = 0; j < MPT; ++j)
#pragma unroll
      for (int al = 0; al < 3; ++al) c[j][al] = acc[j][al] + cvt<double>(cf3[j][al] * Nx[j][al]);
  }
#pragma unroll
  for (int j = 0; j < MPT; ++j)
    if (O::valid(j))
      for (int al = 0; al < 3; ++al) dst[al * KP + O::mode(j)] = c[j][al];
}

// ----------------------------------------------------------- time average ---
// Nbar of the owned-mode state y (registers) -> acc, S samples in flight.
template <typename T, int NX, int NT, int S>
__device__ __forceinline__ void nbar_owned(const cx<T> (&y)[Own<NX, NT>::MPT][3], cx<T> (&acc)[Own<NX, NT>::MPT][3],
                                           const Basis<T> (&bs)[Own<NX, NT>::MPT], const AvgTab<T>& av,
                                           cx<T>* spec, cx<T>* a_buf, cx<T>* b_buf,
                                           const cx<T>* __restrict__ tw) {
  using G = Geo<NX>;
  using O = Own<NX, NT>;
  constexpr int KP = G::KP;
#pragma unroll
  for (int j = 0; j < O::MPT; ++j)
    for (int al = 0; al < 3; ++al) acc[j][al] = czero<T>();
  for (int m0 = 1; m0 < av.M; m0 += S) {
    const int ns = min(S, av.M - m0);
    for (int s = 0; s < ns; ++s) {
      const cx<T>* rot = av.rot + size_t(m0 + s) * KP;
#pragma unroll
      for (int j = 0; j < O::MPT; ++j) {
        if (!O::valid(j)) continue;
        const int k = O::mode(j);
        const cx<T> e = rot[k];
        cx<T> x[3];
        for (int al = 0; al < 3; ++al) x[al] = rot_in(y[j][al], e, al);
        put_fields<T, NX>(spec, s, k, x, bs[j]);
      }
    }
    __syncthreads();
    cx<T>* R = nonlinear_core<T, NX, NT>(spec, a_buf, b_buf, ns, tw);
    for (int s = 0; s < ns; ++s) {
      const cx<T>* rot = av.rot + size_t(m0 + s) * KP;
      const T wm = av.w[m0 + s];
#pragma unroll
      for (int j = 0; j < O::MPT; ++j) {
        if (!O::valid(j)) continue;
        const int k = O::mode(j);
        const cx<T> e = rot[k];
        cx<T> n[3];
        get_N<T, NX>(R, s, k, bs[j], tw, n);
        for (int al = 0; al < 3; ++al) acc[j][al] = acc[j][al] + wm * rot_out(n[al], e, al);
      }
    }
  }
}

// One asymptotic coarse step on owned-mode registers u -> g (Alg. 2).
template <typename T, int NX, int NT, int S>
__device__ __forceinline__ void coarse_owned(const cx<T> (&u)[Own<NX, NT>::MPT][3], cx<T> (&g)[Own<NX, NT>::MPT][3],
                                             const Basis<T> (&bs)[Own<NX, NT>::MPT], const CoarseTab<T>& ct,
                                             cx<T>* spec, cx<T>* a_buf, cx<T>* b_buf,
                                             const cx<T>* __restrict__ tw) {
  using O = Own<NX, NT>;
  constexpr int MPT = O::MPT;
  cx<T> w[MPT][3], y[MPT][3], kk[MPT][3];
  T hd[MPT];
  cx<T> rT[MPT];
#pragma unroll
  for (int j = 0; j < MPT; ++j) {
    const int k = O::valid(j) ? O::mode(j) : 0;
    hd[j] = ct.hd[k];
    rT[j] = ct.rotT[k];
    for (int al = 0; al < 3; ++al) w[j][al] = hd[j] * u[j][al];
  }
  nbar_owned<T, NX, NT, S>(w, kk, bs, ct.avg, spec, a_buf, b_buf, tw);
  const T half = T(0.5) * ct.dT;
#pragma unroll
  for (int j = 0; j < MPT; ++j)
    for (int al = 0; al < 3; ++al) y[j][al] = w[j][al] + half * kk[j][al];
  nbar_owned<T, NX, NT, S>(y, kk, bs, ct.avg, spec, a_buf, b_buf, tw);
#pragma unroll
  for (int j = 0; j < MPT; ++j)
    for (int al = 0; al < 3; ++al) {
      const cx<T> v = hd[j] * (w[j][al] + ct.dT * kk[j][al]);
      g[j][al] = al == 2 ? v * rT[j] : (al == 0 ? v * conj(rT[j]) : v);
    }
}

template <typename T, int NX, int NT, int S>
__global__ void __launch_bounds__(NT) k_average(const cx<double>* __restrict__ Uin, cx<double>* __restrict__ Nout,
                                                AvgTab<T> av, const cx<T>* __restrict__ tw,
                                                const Basis<T>* __restrict__ basis) {
  using G = Geo<NX>;
  using O = Own<NX, NT>;
  extern __shared__ unsigned char smem_raw[];
  cx<T>* spec = reinterpret_cast<cx<T>*>(smem_raw);
  cx<T>* a_buf = spec + Lds<T, NX>::spec_elems(S);
  cx<T>* b_buf = a_buf + Lds<T, NX>::work_elems(S);
  zero_spec_tail<T, NX, NT>(spec, S);
  const cx<double>* src = Uin + size_t(blockIdx.x) * 3 * G::KP;
  cx<double>* dst = Nout + size_t(blockIdx.x) * 3 * G::KP;
  cx<T> y[O::MPT][3], acc[O::MPT][3];
  Basis<T> bs[O::MPT];
#pragma unroll
  for (int j = 0; j < O::MPT; ++j) {
    const int k = O::valid(j) ? O::mode(j) : 0;
    bs[j] = basis[k];
    for (int al = 0; al < 3; ++al) y[j][al] = O::valid(j) ? cvt<T>(src[al * G::KP + k]) : czero<T>();
  }
  nbar_owned<T, NX, NT, S>(y, acc, bs, av, spec, a_buf, b_buf, tw);
#pragma unroll
  for (int j = 0; j < O::MPT; ++j)
    if (O::valid(j))
      for (int al = 0; al < 3; ++al) dst[al * G::KP + O::mode(j)] = cvt<double>(acc[j][al]);
}

template <typename T, int NX, int NT, int S>
__global__ void __launch_bounds__(NT) k_coarse(const cx<double>* __restrict__ Uin, cx<double>* __restrict__ Uout,
                                               CoarseTab<T> ct, const cx<T>* __restrict__ tw,
                                               const Basis<T>* __restrict__ basis) {
  using G = Geo<NX>;
  using O = Own<NX, NT>;
  extern __shared__ unsigned char smem_raw[];
  cx<T>* spec = reinterpret_cast<cx<T>*>(smem_raw);
  cx<T>* a_buf = spec + Lds<T, NX>::spec_elems(S);
  cx<T>* b_buf = a_buf + Lds<T, NX>::work_elems(S);
  zero_spec_tail<T, NX, NT>(spec, S);
  const cx<double>* src = Uin + size_t(blockIdx.x) * 3 * G::KP;
  cx<double>* dst = Uout + size_t(blockIdx.x) * 3 * G::KP;
  cx<T> u[O::MPT][3], g[O::MPT][3];
  Basis<T> bs[O::MPT];
#pragma unroll
  for (int j = 0; j < O::MPT; ++j) {
    const int k = O::valid(j) ? O::mode(j) : 0;
    bs[j] = basis[k];
    for (int al = 0; al < 3; ++al) u[j][al] = O::valid(j) ? cvt<T>(src[al * G::KP + k]) : czero<T>();
  }
  coarse_owned<T, NX, NT, S>(u, g, bs, ct, spec, a_buf, b_buf, tw);
#pragma unroll
  for (int j = 0; j < O::MPT; ++j)
    if (O::valid(j))
      for (int al = 0; al < 3; ++al) dst[al * G::KP + O::mode(j)] = cvt<double>(g[j][al]);
}

// ------------------------------------------------------ serial sweep ------
// One workgroup per problem.  U, Fine, Gold: modal FP64 [Ns+1][3][KP].
// initial != 0: U_n = Gold_n = G(U_{n-1}).  Otherwise
// U_n <- Fine_n + (G(U_{n-1}) - Gold_n), Gold_n <- G(U_{n-1}), and
// part[n-1] = (sum |U_n^new - U_n^old|^2, sum |U_n^new|^2) with Parseval
// weights (1 for k = 0, 2 otherwise).
template <typename T, int NX, int NT, int S>
__global__ void __launch_bounds__(NT) k_sweep(cx<double>* __restrict__ U, const cx<double>* __restrict__ Fine,
                                              cx<double>* __restrict__ Gold, double2* __restrict__ part, int Ns,
                                              int initial, CoarseTab<T> ct, const cx<T>* __restrict__ tw,
                                              const Basis<T>* __restrict__ basis) {
  using G = Geo<NX>;
  using O = Own<NX, NT>;
  constexpr int KP = G::KP;
  extern __shared__ unsigned char smem_raw[];
  cx<T>* spec = reinterpret_cast<cx<T>*>(smem_raw);
  cx<T>* a_buf = spec + Lds<T, NX>::spec_elems(S);
  cx<T>* b_buf = a_buf + Lds<T, NX>::work_elems(S);
  double* red = reinterpret_cast<double*>(b_buf + Lds<T, NX>::work_elems(S));   // [2][NT]
  zero_spec_tail<T, NX, NT>(spec, S);
  Basis<T> bs[O::MPT];
#pragma unroll
  for (int j = 0; j < O::MPT; ++j) bs[j] = basis[O::valid(j) ? O::mode(j) : 0];
  const size_t st = size_t(3) * KP;
  for (int n = 1; n <= Ns; ++n) {
    cx<T> u[O::MPT][3], g[O::MPT][3];
#pragma unroll
    for (int j = 0; j < O::MPT; ++j)
      for (int al = 0; al < 3; ++al)
        u[j][al] = O::valid(j) ? cvt<T>(U[(n - 1) * st + al * KP + O::mode(j)]) : czero<T>();
    coarse_owned<T, NX, NT, S>(u, g, bs, ct, spec, a_buf, b_buf, tw);
    double num = 0.0, den = 0.0;
#pragma unroll
    for (int j = 0; j < O::MPT; ++j) {
      if (!O::valid(j)) continue;
      const int k = O::mode(j);
      const double wgt = k == 0 ? 1.0 : 2.0;
      for (int al = 0; al < 3; ++al) {
        const size_t o = n * st + al * KP + k;
        const cx<double> gn = cvt<double>(g[j][al]);
        if (initial) {
          U[o] = gn;
          Gold[o] = gn;
        } else {
          const cx<double> uold = U[o];
          const cx<double> unew = Fine[o] + (gn - Gold[o]);
          const cx<double> d = unew - uold;
          num += wgt * (d.x * d.x + d.y * d.y);
          den += wgt * (unew.x * unew.x + unew.y * unew.y);
          U[o] = unew;
          Gold[o] = gn;
        }
      }
    }
    if (!initial) {
      red[threadIdx.x] = num;
      red[NT + threadIdx.x] = den;
      __syncthreads();
      for (int off = NT / 2; off > 0; off >>= 1) {
        if (threadIdx.x < off) {
          red[threadIdx.x] += red[threadIdx.x + off];
          red[NT + threadIdx.x] += red[NT + threadIdx.x + off];
        }
        __syncthreads();
      }
      if (threadIdx.x == 0) part[n - 1] = make_double2(red[0], red[NT]);
      __syncthreads();
    }
  }
}

// r = max_n sqrt(num_n / den_n) over Ns partials, one workgroup of 256.
__global__ void __launch_bounds__(256) k_resid(const double2* __restrict__ part, int Ns, double* __restrict__ out) {
  __shared__ double red[256];
  double m = 0.0;
  for (int n = threadIdx.x; n < Ns; n += 256) {
    const double2 p = part[n];
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
  if (threadIdx.x == 0) *out = red[0];
}

// ------------------------------------------------------------- launchers ---
template <int NX> struct Cfg;
// block sizes: fine -> enough threads to own every retained mode (<= 512);
// average/coarse -> 256 (N <= 512) or 512, with S samples in flight.
template <> struct Cfg<64>   { static constexpr int FINE = 64,  AVG = 256; static constexpr int S32 = 16, S64 = 16; };
template <> struct Cfg<128>  { static constexpr int FINE = 64,  AVG = 256; static constexpr int S32 = 16, S64 = 8; };
template <> struct Cfg<256>  { static constexpr int FINE = 128, AVG = 256; static constexpr int S32 = 8, S64 = 4; };
template <> struct Cfg<512>  { static constexpr int FINE = 192, AVG = 256; static constexpr int S32 = 4, S64 = 2; };
template <> struct Cfg<1024> { static constexpr int FINE = 384, AVG = 512; static constexpr int S32 = 2, S64 = 1; };
template <> struct Cfg<2048> { static constexpr int FINE = 512, AVG = 512; static constexpr int S32 = 1, S64 = 1; };

template <typename T, int NX> constexpr int samples_in_flight() {
  return sizeof(T) == 4 ? Cfg<NX>::S32 : Cfg<NX>::S64;
}

// Raise the dynamic-LDS limit for launches above 64 KiB (gfx950 has 160 KiB per
// workgroup).  Best effort: a launch that still exceeds the limit fails and is
// reported by the hipGetLastError() that follows it.
template <typename K>
static hipError_t prep_lds(K kernel, size_t bytes) {
  if (bytes > 65536) {
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(kernel), hipFuncAttributeMaxDynamicSharedMemorySize,
                              int(bytes));
    (void)hipGetLastError();
  }
  return hipSuccess;
}

template <int NX>
static hipError_t to_modal_nx(const double* phys, cx<double>* modal, int batch, const DevTables& t, hipStream_t s) {
  constexpr int NT = Cfg<NX>::AVG;
  const size_t lds = 2 * 3 * Geo<NX>::P * sizeof(cx<double>);
  hipError_t e = prep_lds(k_to_modal<NX, NT>, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_to_modal<NX, NT>), dim3(batch), dim3(NT), lds, s, phys, modal, t.tw64, t.basis64);
  return hipGetLastError();
}

template <int NX>
static hipError_t to_physical_nx(const cx<double>* modal, double* phys, int batch, const DevTables& t, hipStream_t s) {
  constexpr int NT = Cfg<NX>::AVG;
  const size_t lds = (3 * (Geo<NX>::P + 1) + 2 * 3 * Geo<NX>::P) * sizeof(cx<double>);
  hipError_t e = prep_lds(k_to_physical<NX, NT>, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_to_physical<NX, NT>), dim3(batch), dim3(NT), lds, s, modal, phys, t.tw64, t.basis64);
  return hipGetLastError();
}

template <typename T, int NX>
static hipError_t nonlinear_nx(const cx<double>* in, cx<double>* out, int batch, const DevTables& t, hipStream_t s) {
  constexpr int NT = Cfg<NX>::FINE;
  const size_t lds = Lds<T, NX>::bytes(1);
  hipError_t e = prep_lds(k_nonlinear<T, NX, NT>, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_nonlinear<T, NX, NT>), dim3(batch), dim3(NT), lds, s, in, out, t.tw<T>(), t.basis<T>());
  return hipGetLastError();
}

template <typename T, int NX>
static hipError_t fine_nx(const cx<double>* in, cx<double>* out, int batch, int steps, const cx<double>* coef64,
                          const cx<T>* coef, const DevTables& t, hipStream_t s) {
  constexpr int NT = Cfg<NX>::FINE;
  const size_t lds = Lds<T, NX>::bytes(1);
  hipError_t e = prep_lds(k_fine<T, NX, NT>, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_fine<T, NX, NT>), dim3(batch), dim3(NT), lds, s, in, out, steps, coef64, coef, t.tw<T>(),
                     t.basis<T>());
  return hipGetLastError();
}

template <typename T, int NX>
static hipError_t average_nx(const cx<double>* in, cx<double>* out, int batch, const AvgTab<T>& av,
                             const DevTables& t, hipStream_t s) {
  constexpr int NT = Cfg<NX>::AVG;
  constexpr int S = samples_in_flight<T, NX>();
  const size_t lds = Lds<T, NX>::bytes(S);
  hipError_t e = prep_lds(k_average<T, NX, NT, S>, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_average<T, NX, NT, S>), dim3(batch), dim3(NT), lds, s, in, out, av, t.tw<T>(), t.basis<T>());
  return hipGetLastError();
}

template <typename T, int NX>
static hipError_t coarse_nx(const cx<double>* in, cx<double>* out, int batch, const CoarseTab<T>& ct,
                            const DevTables& t, hipStream_t s) {
  constexpr int NT = Cfg<NX>::AVG;
  constexpr int S = samples_in_flight<T, NX>();
  const size_t lds = Lds<T, NX>::bytes(S);
  hipError_t e = prep_lds(k_coarse<T, NX, NT, S>, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_coarse<T, NX, NT, S>), dim3(batch), dim3(NT), lds, s, in, out, ct, t.tw<T>(), t.basis<T>());
  return hipGetLastError();
}

template <typename T, int NX>
static hipError_t sweep_nx(cx<double>* U, const cx<double>* Fine, cx<double>* Gold, double2* part, int Ns,
                           int initial, const CoarseTab<T>& ct, const DevTables& t, hipStream_t s) {
  constexpr int NT = Cfg<NX>::AVG;
  constexpr int S = samples_in_flight<T, NX>();
  const size_t lds = Lds<T, NX>::bytes(S) + 2 * NT * sizeof(double);
  hipError_t e = prep_lds(k_sweep<T, NX, NT, S>, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_sweep<T, NX, NT, S>), dim3(1), dim3(NT), lds, s, U, Fine, Gold, part, Ns, initial, ct,
                     t.tw<T>(), t.basis<T>());
  return hipGetLastError();
}

#define AP_DISPATCH_NX(NXV, CALL)                  \
  switch (NXV) {                                   \
    case 64: { constexpr int NX = 64; return CALL; }     \
    case 128: { constexpr int NX = 128; return CALL; }   \
    case 256: { constexpr int NX = 256; return CALL; }   \
    case 512: { constexpr int NX = 512; return CALL; }   \
    case 1024: { constexpr int NX = 1024; return CALL; } \
    case 2048: { constexpr int NX = 2048; return CALL; } \
    default: return hipErrorInvalidValue;          \
  }

hipError_t launch_to_modal(int nx, const double* phys, cx<double>* modal, int batch, const DevTables& t,
                           hipStream_t s) {
  AP_DISPATCH_NX(nx, to_modal_nx<NX>(phys, modal, batch, t, s));
}
hipError_t launch_to_physical(int nx, const cx<double>* modal, double* phys, int batch, const DevTables& t,
                              hipStream_t s) {
  AP_DISPATCH_NX(nx, to_physical_nx<NX>(modal, phys, batch, t, s));
}
hipError_t launch_nonlinear(int nx, bool fp64, const cx<double>* in, cx<double>* out, int batch,
                            const DevTables& t, hipStream_t s) {
  if (fp64) AP_DISPATCH_NX(nx, (nonlinear_nx<double, NX>(in, out, batch, t, s)));
  AP_DISPATCH_NX(nx, (nonlinear_nx<float, NX>(in, out, batch, t, s)));
}
hipError_t launch_fine(int nx, bool fp64, const cx<double>* in, cx<double>* out, int batch, int steps,
                       const cx<double>* coef64, const cx<float>* coef32, const DevTables& t, hipStream_t s) {
  if (fp64) AP_DISPATCH_NX(nx, (fine_nx<double, NX>(in, out, batch, steps, coef64, coef64, t, s)));
  AP_DISPATCH_NX(nx, (fine_nx<float, NX>(in, out, batch, steps, coef64, coef32, t, s)));
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
hipError_t launch_resid(const double2* part, int Ns, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_resid, dim3(1), dim3(256), 0, s, part, Ns, out);
  return hipGetLastError();
}

}  // namespace ap
