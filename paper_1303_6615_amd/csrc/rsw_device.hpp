// Device building blocks for the RSW asymptotic parareal path on gfx950.
//
// State representation.  Every wavenumber 0 <= k <= Kd = floor(N/3) carries
// the three modal amplitudes c^alpha_k (alpha = -1, 0, +1) of u in the
// eigenbasis of the Fourier symbol L_k (Sec. 6.1: L_k r^alpha = i alpha
// omega_k r^alpha, omega_k = sqrt(1 + k^2/F)).  With a = k/sqrt(F) the
// orthonormal eigenvectors are
//     r^0 = (0, i a, 1)/omega,   r^(+-1) = (1, -+ i/omega, +- a/omega)/sqrt(2),
// so every function of -L/eps + D (a scalar per k) is a diagonal multiplier
// per (k, alpha) and only the nonlinear term needs the physical fields.
//
// Physical <-> spectral.  Real fields of length N are transformed through
// complex FFTs of length P = N/2 (x[2n] + i x[2n+1] packed in one complex
// slot) with the standard pre/post twiddle by exp(-+ 2 pi i k / N).  The FFT is
// a Stockham auto-sort radix-4 (one radix-2 stage when log2 P is odd) staged
// in LDS between two ping-pong buffers, all transforms of a workgroup in
// flight together.
#pragma once
#include <hip/hip_runtime.h>

namespace ap {

// This thread's index in its workgroup of NT threads, passed through an empty
// asm statement that also takes `salt`.  A persistent kernel passes the
// number of the job it runs: what a job derives from the index (mode numbers,
// wavenumbers, LDS addresses) then depends on the job, and the compiler cannot
// hoist it out of the job loop, where it would stay live across every other
// kind of job and spill.  The statement has no side effects, so the uses
// within one job still share one value.
template <int NT>
__device__ __forceinline__ unsigned salted_thread(int salt) {
  unsigned t = threadIdx.x;
  asm("" : "+v"(t) : "s"(salt));
  __builtin_assume(t < NT);
  return t;
}

// Complex value aligned to its size, so that LDS and global accesses are
// single 64-bit (float) or 128-bit (double) operations.  Two 32-bit LDS
// accesses to consecutive complex floats would map lanes i and i + 32 to one
// bank; a 64-bit access serves 32 lanes per cycle across all 64 banks.
template <typename T>
struct alignas(2 * sizeof(T)) cx {
  T x, y;
};

template <typename T> __host__ __device__ __forceinline__ cx<T> mk(T a, T b) { return cx<T>{a, b}; }
template <typename T> __host__ __device__ __forceinline__ cx<T> operator+(cx<T> a, cx<T> b) { return {a.x + b.x, a.y + b.y}; }
template <typename T> __host__ __device__ __forceinline__ cx<T> operator-(cx<T> a, cx<T> b) { return {a.x - b.x, a.y - b.y}; }
template <typename T> __host__ __device__ __forceinline__ cx<T> operator*(cx<T> a, cx<T> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename T> __host__ __device__ __forceinline__ cx<T> operator*(T s, cx<T> a) { return {s * a.x, s * a.y}; }
template <typename T> __host__ __device__ __forceinline__ cx<T> conj(cx<T> a) { return {a.x, -a.y}; }
template <typename T> __host__ __device__ __forceinline__ cx<T> mul_i(cx<T> a) { return {-a.y, a.x}; }      // i*a
template <typename T> __host__ __device__ __forceinline__ cx<T> mul_mi(cx<T> a) { return {a.y, -a.x}; }     // -i*a
template <typename T> __host__ __device__ __forceinline__ cx<T> czero() { return {T(0), T(0)}; }
template <typename T, typename U> __host__ __device__ __forceinline__ cx<T> cvt(cx<U> a) { return {T(a.x), T(a.y)}; }
__host__ __device__ __forceinline__ float fmat(float a, float b, float c) { return fmaf(a, b, c); }
__host__ __device__ __forceinline__ double fmat(double a, double b, double c) { return fma(a, b, c); }
// a*b + c with the product written as FMAs
template <typename T> __host__ __device__ __forceinline__ cx<T> cfma(cx<T> a, cx<T> b, cx<T> c) {
  return {fmat(a.x, b.x, fmat(-a.y, b.y, c.x)), fmat(a.x, b.y, fmat(a.y, b.x, c.y))};
}

constexpr int ilog2(int v) { return v <= 1 ? 0 : 1 + ilog2(v / 2); }

// Grid geometry for N grid points.
template <int NX>
struct Geo {
  static constexpr int N = NX;
  static constexpr int P = NX / 2;      // complex FFT length
  static constexpr int KD = NX / 3;     // largest retained wavenumber
  static constexpr int KP = KD + 1;     // retained modes 0..KD
  static_assert((NX & (NX - 1)) == 0 && NX >= 64 && NX <= 2048, "N must be a power of two in [64, 2048]");
};

// Per-wavenumber constants of the modal basis: iw = 1/omega_k, aw = a_k/omega_k.
template <typename T>
struct Basis {
  T iw, aw;
};

// ---------------------------------------------------------------- FFT ------
// y_q = sum_p x_p exp(DIR 2 pi i p q / R)
template <typename T, int R, int DIR>
__device__ __forceinline__ void dft_small(cx<T>* x) {
  if constexpr (R == 2) {
    cx<T> a = x[0] + x[1], b = x[0] - x[1];
    x[0] = a;
    x[1] = b;
  } else {
    static_assert(R == 4, "radix");
    cx<T> a = x[0] + x[2], b = x[0] - x[2];
    cx<T> c = x[1] + x[3], d = x[1] - x[3];
    d = (DIR > 0) ? mul_i(d) : mul_mi(d);
    x[0] = a + c;
    x[2] = a - c;
    x[1] = b + d;
    x[3] = b - d;
  }
}

// One Stockham stage of radix R with NS = product of earlier radices.
// tw[t] = exp(-2 pi i t / (2P)), t < 2P (so exp(-2 pi i u / P) = tw[2u]).
template <typename T, int P, int R, int NS, int DIR, int NT>
__device__ __forceinline__ void stockham_stage(const cx<T>* __restrict__ src, cx<T>* __restrict__ dst,
                                               int nvec, const cx<T>* __restrict__ tw) {
  constexpr int PR = P / R;
  const int total = nvec * PR;
  for (int b = threadIdx.x; b < total; b += NT) {
    const int v = b / PR;
    const int j = b - v * PR;
    const int k = j & (NS - 1);
    const cx<T>* s = src + v * P + j;
    cx<T> x[R];
#pragma unroll
    for (int q = 0; q < R; ++q) x[q] = s[q * PR];
    if constexpr (NS > 1) {
#pragma unroll
      for (int q = 1; q < R; ++q) {
        const int t = q * k * (P / (NS * R));
        cx<T> w = tw[2 * t];
        if (DIR > 0) w = conj(w);
        x[q] = x[q] * w;
      }
    }
    dft_small<T, R, DIR>(x);
    cx<T>* d = dst + v * P + (j - k) * R + k;
#pragma unroll
    for (int q = 0; q < R; ++q) d[q * NS] = x[q];
  }
}

template <typename T, int P, int NS, int DIR, int NT>
struct Radix4Stages {
  // runs the radix-4 stages from NS up to P; returns the buffer holding the result
  static __device__ __forceinline__ cx<T>* run(cx<T>* src, cx<T>* dst, int nvec, const cx<T>* tw) {
    if constexpr (NS >= P) {
      return src;
    } else {
      stockham_stage<T, P, 4, NS, DIR, NT>(src, dst, nvec, tw);
      __syncthreads();
      return Radix4Stages<T, P, NS * 4, DIR, NT>::run(dst, src, nvec, tw);
    }
  }
};

// Unnormalised complex FFT of length P on `nvec` contiguous vectors in `a`
// (scratch `b`), sign DIR; returns a or b, whichever holds the result.
// Entry and exit are workgroup barriers' responsibility of the caller/last stage.
template <typename T, int P, int DIR, int NT>
__device__ __forceinline__ cx<T>* fft_lds(cx<T>* a, cx<T>* b, int nvec, const cx<T>* tw) {
  constexpr int L = ilog2(P);
  if constexpr (L % 2 == 1) {
    stockham_stage<T, P, 2, 1, DIR, NT>(a, b, nvec, tw);
    __syncthreads();
    return Radix4Stages<T, P, 2, DIR, NT>::run(b, a, nvec, tw);
  } else {
    return Radix4Stages<T, P, 1, DIR, NT>::run(a, b, nvec, tw);
  }
}

// Final buffer after a full fft_lds call starting in `a` (compile-time parity).
template <int P>
struct FftParity {
  static constexpr int L = ilog2(P);
  static constexpr int stages = (L % 2 == 1) ? 1 + (L - 1) / 2 : L / 2;
  static constexpr bool in_b = (stages % 2) == 1;
};

// ------------------------------------------------- modal <-> (v1, v2x, h) ---
// (v1^, i k v2^, h^) of the state with modal amplitudes c = (c-, c0, c+).
// With e = c- - c+: v1 = s (c- + c+), v2^ = i (s iw e + aw c0), so
// v2x = i k v2^ = -k s iw e - k aw c0, and h = -s aw e + iw c0 (s = 1/sqrt 2),
// as fused multiply-adds with per-mode real factors.
template <typename T>
__device__ __forceinline__ void modal_to_fields(const cx<T> c[3], T kk, Basis<T> bs, cx<T>& v1,
                                                cx<T>& v2x, cx<T>& h) {
  const T s = T(0.70710678118654752440);
  v1 = s * (c[0] + c[2]);
  const cx<T> e = c[0] - c[2];
  const T al = -(kk * (bs.iw * s)), be = -(kk * bs.aw), ga = -(bs.aw * s);
  v2x = cx<T>{fmat(al, e.x, be * c[1].x), fmat(al, e.y, be * c[1].y)};
  h = cx<T>{fmat(ga, e.x, bs.iw * c[1].x), fmat(ga, e.y, bs.iw * c[1].y)};
}

// modal amplitudes of the spectral vector (n1, n2, n3)
template <typename T>
__device__ __forceinline__ void fields_to_modal(cx<T> n1, cx<T> n2, cx<T> n3, Basis<T> bs, cx<T> out[3]) {
  const T s = T(0.70710678118654752440);
  const cx<T> t2 = bs.iw * mul_i(n2);       // i n2 / omega
  const cx<T> t3 = bs.aw * n3;              // a n3 / omega
  out[0] = s * (n1 - t2 - t3);
  out[1] = bs.iw * n3 - bs.aw * mul_i(n2);
  out[2] = s * (n1 + t2 + t3);
}

// ----------------------------------------------------- LDS working set -----
// For S states: spec[S][3][P+1] (input half spectra, tail k > KD kept zero),
// a, b [S][3][P] ping-pong FFT buffers.
template <typename T, int NX>
struct Lds {
  static constexpr int P = Geo<NX>::P;
  static constexpr size_t spec_elems(int S) { return size_t(S) * 3 * (P + 1); }
  static constexpr size_t work_elems(int S) { return size_t(S) * 3 * P; }
  static constexpr size_t bytes(int S) { return (spec_elems(S) + 2 * work_elems(S)) * sizeof(cx<T>); }
  static constexpr size_t per_state() { return bytes(1); }
};

// Zero the non-retained tail of every spectrum slot (done once per kernel).
template <typename T, int NX, int NT>
__device__ __forceinline__ void zero_spec_tail(cx<T>* spec, int S) {
  using G = Geo<NX>;
  constexpr int tail = G::P - G::KD;   // k = KD+1 .. P
  for (int i = threadIdx.x; i < S * 3 * tail; i += NT) {
    const int v = i / tail;
    const int k = G::KD + 1 + (i - v * tail);
    spec[v * (G::P + 1) + k] = czero<T>();
  }
}

// Write the three physical-field half spectra of a modal state into spec slot s.
template <typename T, int NX>
__device__ __forceinline__ void put_fields(cx<T>* spec, int s, int k, const cx<T> c[3], Basis<T> bs) {
  using G = Geo<NX>;
  cx<T> v1, v2x, h;
  modal_to_fields<T>(c, T(k), bs, v1, v2x, h);
  cx<T>* base = spec + s * 3 * (G::P + 1);
  base[k] = v1;
  base[(G::P + 1) + k] = v2x;
  base[2 * (G::P + 1) + k] = h;
}

// Dealiased N(u) for `nstates` states whose field spectra sit in spec.
// Returns the LDS buffer holding, per state and product (v1^2/2, v1 v2x, h v1),
// the length-P forward FFT of the packed products (post-processing by get_N).
// Must be entered after a barrier that follows the last put_fields.
template <typename T, int NX, int NT>
__device__ __forceinline__ cx<T>* nonlinear_core(cx<T>* spec, cx<T>* a, cx<T>* b, int nstates,
                                                 const cx<T>* tw) {
  using G = Geo<NX>;
  constexpr int P = G::P;
  const int nvec = nstates * 3;
  // inverse real-FFT pre-processing: Z[k] = (X[k] + conj X[P-k]) + i e^{2 pi i k/N} (X[k] - conj X[P-k])
  for (int i = threadIdx.x; i < nvec * P; i += NT) {
    const int v = i / P;
    const int k = i - v * P;
    const cx<T>* X = spec + v * (P + 1);
    const cx<T> xk = X[k];
    const cx<T> xc = conj(X[P - k]);
    const cx<T> w = conj(tw[k]);
    a[v * P + k] = (xk + xc) + mul_i(w * (xk - xc));
  }
  __syncthreads();
  cx<T>* r = fft_lds<T, P, +1, NT>(a, b, nvec, tw);
  cx<T>* o = (r == a) ? b : a;
  (void)o;
  // pointwise quadratic products on the grid, two grid points per slot
  for (int i = threadIdx.x; i < nstates * P; i += NT) {
    const int s = i / P;
    const int n = i - s * P;
    cx<T>* base = r + s * 3 * P + n;
    const cx<T> v1 = base[0], v2x = base[P], h = base[2 * P];
    base[0] = cx<T>{T(0.5) * v1.x * v1.x, T(0.5) * v1.y * v1.y};
    base[P] = cx<T>{v1.x * v2x.x, v1.y * v2x.y};
    base[2 * P] = cx<T>{h.x * v1.x, h.y * v1.y};
  }
  __syncthreads();
  return fft_lds<T, P, -1, NT>(r, (r == a) ? b : a, nvec, tw);
}

// Post-process one retained mode k of state s from the forward-FFT buffer R
// and return modal N amplitudes: N = -(i k P1, P2, i k P3) with
// P_f[k] = (1/N) [ (Z[k] + conj Z[P-k])/2 - i e^{-2 pi i k/N} (Z[k] - conj Z[P-k])/2 ].
template <typename T, int NX>
__device__ __forceinline__ void get_N(const cx<T>* R, int s, int k, Basis<T> bs,
                                      const cx<T>* __restrict__ tw, cx<T> out[3]) {
  using G = Geo<NX>;
  constexpr int P = G::P;
  const T half_over_n = T(0.5) / T(G::N);
  const cx<T> w = tw[k];
  const int kc = (P - k) & (P - 1);
  cx<T> Pf[3];
#pragma unroll
  for (int f = 0; f < 3; ++f) {
    const cx<T>* Z = R + (s * 3 + f) * P;
    const cx<T> zk = Z[k];
    const cx<T> zc = conj(Z[kc]);
    Pf[f] = half_over_n * ((zk + zc) - mul_i(w * (zk - zc)));
  }
  const T kk = T(k);
  const cx<T> n1 = (-kk) * mul_i(Pf[0]);
  const cx<T> n2 = T(-1) * Pf[1];
  const cx<T> n3 = (-kk) * mul_i(Pf[2]);
  fields_to_modal<T>(n1, n2, n3, bs, out);
}

}  // namespace ap
