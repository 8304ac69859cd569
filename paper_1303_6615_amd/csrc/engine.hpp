// Workgroup-level engine: LDS layout, and the per-workgroup jobs of the
// parareal path (one fine slice; one coarse step with the FP64 correction).
//
// LDS layout for S state slots (T = float or double, P = N/2):
//   tw  [N]             exp(-2 pi i t / N), staged once per kernel when it
//                       fits next to one slot (else read from global memory)
//   sp  [S][3][P+1]     field half spectra in, forward transforms out
//   ib  [S][3][P]       inverse transforms (in place); between evaluations it
//                       also holds per-sample contributions and the FP64
//                       reduction scratch [2][NT]
//   y   [3][Kd+1]       the state being averaged (read by every thread)
#pragma once
#include "launch.hpp"
#include "wavefft.hpp"

namespace ap {

constexpr size_t kLdsBudget = 156 * 1024;   // of gfx950's 160 KiB per workgroup

template <typename T, int NX>
constexpr size_t y_bytes() {
  return 3 * size_t(Geo<NX>::KP) * sizeof(cx<T>);
}

template <typename T, int NX, int PLAN = 0>
constexpr bool twiddles_in_lds() {
  return tw_elems<NX / 2, PLAN>() * sizeof(cx<T>) + Slot<T, NX>::bytes + y_bytes<T, NX>() <= kLdsBudget;
}

template <typename T, int NX, int NT, int PLAN = 0>
constexpr int max_slots() {
  const size_t fixed =
      (twiddles_in_lds<T, NX, PLAN>() ? tw_elems<NX / 2, PLAN>() * sizeof(cx<T>) : 0) + y_bytes<T, NX>();
  const size_t s = (kLdsBudget - fixed) / Slot<T, NX>::bytes;
  return s >= 32 ? 32 : (s < 1 ? 1 : int(s));
}

template <typename T, int NX, int NT, int S, int PLAN = 0, int IMAX = 1>
struct Engine {
  using G = Geo<NX>;
  using SL = Slot<T, NX>;
  static constexpr int P = G::P;
  static constexpr int KP = G::KP;
  static constexpr int MPT = (KP + NT - 1) / NT;
  // (slice, mode) items a thread may own in a job over several slices: IMAX
  // (when above MPT) lets a job step more slices than one mode per thread
  // allows, with that many items per thread
  static constexpr int IPT = IMAX > MPT ? IMAX : MPT;
  static constexpr bool TW_LDS = twiddles_in_lds<T, NX, PLAN>();
  static constexpr int TWN = tw_elems<NX / 2, PLAN>();   // twiddle table entries of FFT plan PLAN
  static_assert(NT % 64 == 0, "whole wavefronts");
  static_assert(SL::ib_elems >= size_t(3) * KP, "per-sample contributions fit a slot's ib");
  static constexpr size_t lds_bytes() {
    return (TW_LDS ? TWN * sizeof(cx<T>) : 0) + S * SL::bytes + y_bytes<T, NX>();
  }
  static_assert(lds_bytes() <= 160 * 1024, "LDS budget of gfx950 exceeded");
  const cx<T>* tw;
  cx<T>* sp;
  cx<T>* ib;
  cx<T>* y;
  double* red;

  unsigned tid;   // this thread's index in the workgroup

  // stage == false: the twiddles of this grid size are already in LDS (the
  // previous job of this workgroup staged them and nothing overwrote them).
  __device__ __forceinline__ Engine(unsigned char* smem, const cx<T>* tw_global, bool stage = true)
      : Engine(smem, tw_global, stage, threadIdx.x, ThreadIndex{}) {}
  // For persistent kernels: the thread index salted with the number of the
  // job (salted_thread), so that nothing a job derives from it is hoisted out
  // of the job loop.
  __device__ __forceinline__ Engine(unsigned char* smem, const cx<T>* tw_global, bool stage, int salt)
      : Engine(smem, tw_global, stage, salted_thread<NT>(salt), ThreadIndex{}) {}

 private:
  struct ThreadIndex {};
  __device__ __forceinline__ Engine(unsigned char* smem, const cx<T>* __restrict__ tw_global, bool stage, unsigned t,
                                    ThreadIndex)
      : tid(t) {
    cx<T>* base = reinterpret_cast<cx<T>*>(smem);
    if constexpr (TW_LDS) {
      if (stage) {
        for (int i = tid; i < TWN; i += NT) base[i] = tw_global[i];
        __syncthreads();
      }
      tw = base;
      base += TWN;
    } else {
      tw = tw_global;
    }
    sp = base;
    ib = sp + S * SL::sp_elems;
    y = ib + S * SL::ib_elems;
    red = reinterpret_cast<double*>(ib);
  }

 public:
  __device__ __forceinline__ int mode(int j) const { return tid + j * NT; }
  __device__ __forceinline__ bool valid(int j) const { return mode(j) < KP; }

  // Most slices one job can step together: IPT items per thread (one mode
  // per thread unless IMAX says more), one round of transforms over the
  // wavefronts, and two slots per slice (alternating evaluations need no
  // extra barrier).
  static constexpr int jmax() {
    if (MPT > 1 && IPT <= MPT) return 1;
    const int by_threads = IPT * NT / KP;
    // signals per round of transforms; with several items per thread, two
    // rounds where one would leave more than a fifth of the lane groups idle
    const int per_round = (NT / 64) * (64 / WavePlan<P>::G);
    const int by_waves = IPT > MPT && 5 * 3 * (per_round / 3) < 4 * per_round ? 2 * per_round / 3 : per_round / 3;
    const int by_slots = S / 2 > 0 ? S / 2 : 1;
    int j = by_threads < by_waves ? by_threads : by_waves;
    j = j < by_slots ? j : by_slots;
    j = j < 16 ? j : 16;
    return j > 0 ? j : 1;
  }

  // Items a thread needs for a job over J slices.
  static constexpr int items(int J) { return (J * KP + NT - 1) / NT; }

  // The (slice, mode) items a thread owns in a job over J slices: item j is
  // i = tid + j NT, mode i mod KP of slice i / KP, valid while the slice is
  // below J (for J = 1: the modes tid + j NT below KP; for one item per
  // thread: mode tid mod KP of slice tid / KP), tid the engine's thread index.
  // An invalid item reads as slice 0, mode 0 (addresses in range).
  template <int NI>
  struct OwnT {
    int s[NI], m[NI];
    bool v[NI];
    __device__ __forceinline__ OwnT(unsigned tid, int J) {
#pragma unroll
      for (int j = 0; j < NI; ++j) {
        const int i = int(tid) + j * NT;
        const int q = i / KP;
        v[j] = q < J;
        s[j] = v[j] ? q : 0;
        m[j] = v[j] ? i - q * KP : 0;
      }
    }
    __device__ __forceinline__ int slice(int j) const { return s[j]; }
    __device__ __forceinline__ int mode(int j) const { return m[j]; }
    __device__ __forceinline__ bool valid(int j) const { return v[j]; }
  };
  using Own = OwnT<MPT>;

  // N of the owned items' modal states x -> n for J slices, using slots
  // slot .. slot + J - 1 (callers alternate between slots 0 and S/2, which
  // J <= S/2 keeps apart, so consecutive evaluations need no barrier between
  // them; with S = 1 every evaluation uses slot 0 and ends with a barrier).
  template <int NI>
  __device__ __forceinline__ void neval(int slot, int J, const OwnT<NI>& ow, const cx<T> (&x)[NI][3],
                                        cx<T> (&n)[NI][3], const Basis<T> (&bs)[NI]) {
    cx<T>* sps = sp + slot * SL::sp_elems;
    cx<T>* ibs = ib + slot * SL::ib_elems;
#pragma unroll
    for (int j = 0; j < NI; ++j)
      if (ow.valid(j)) put_fields<T, NX>(sps, ow.slice(j), ow.mode(j), x[j], bs[j]);
    zero_tails<T, NX, NT>(sps, J, tid);
    __syncthreads();
    inverse_fields<T, NX, NT, jmax(), PLAN>(sps, ibs, J, tw, tid);
    __syncthreads();
    forward_products<T, NX, NT, jmax(), PLAN>(sps, ibs, J, tw, tid);
    __syncthreads();
#pragma unroll
    for (int j = 0; j < NI; ++j)
      if (ow.valid(j)) get_N_sp<T, NX>(sps + ow.slice(j) * SL::sp_elems, ow.mode(j), bs[j], tw, n[j]);
    if (S < 2 * J) __syncthreads();
  }
  // one slice (slot, thread-owned modes as mode(j))
  __device__ __forceinline__ void neval(int slot, const cx<T> (&x)[MPT][3], cx<T> (&n)[MPT][3],
                                        const Basis<T> (&bs)[MPT]) {
    neval(slot, 1, Own(tid, 1), x, n, bs);
  }
  // Evaluation H (0 or 1) of an alternating pair: slot 0 or S/2, known when
  // compiling, so that the LDS addresses of the transforms are the same
  // per-lane offsets in every evaluation plus a constant.
  template <int H, int NI>
  __device__ __forceinline__ void neval_half(int J, const OwnT<NI>& ow, const cx<T> (&x)[NI][3], cx<T> (&n)[NI][3],
                                             const Basis<T> (&bs)[NI]) {
    constexpr int slot = H == 0 ? 0 : S / 2;
    neval(slot, J, ow, x, n, bs);
  }

  // Block reductions: a butterfly over the 64 lanes of each wavefront
  // (cross-lane shuffles, no barrier), then the NT / 64 wavefront results
  // combined in wavefront order by every thread, so that every thread returns
  // the same value.  The scratch lives in `ib`: the first barrier waits for
  // its last readers, the last one for this reduction's readers.
  static constexpr int kWaves = NT / 64;

  // FP64 block maximum of x over the workgroup (NaN wins).
  __device__ __forceinline__ double block_max(double x) {
    static_assert(S * SL::ib_elems * sizeof(cx<T>) >= kWaves * sizeof(double), "reduction scratch");
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      const double o = __shfl_xor(x, off);
      if (o > x || o != o) x = o;
    }
    __syncthreads();
    if ((tid & 63) == 0) red[tid >> 6] = x;
    __syncthreads();
    double r = red[0];
    for (int w = 1; w < kWaves; ++w) {
      const double o = red[w];
      if (o > r || o != o) r = o;
    }
    __syncthreads();
    return r;
  }

  // FP64 block sum of (x, y) over the workgroup.
  __device__ __forceinline__ double2 block_sum2(double x, double yv) {
    static_assert(S * SL::ib_elems * sizeof(cx<T>) >= 2 * kWaves * sizeof(double), "reduction scratch");
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      x += __shfl_xor(x, off);
      yv += __shfl_xor(yv, off);
    }
    __syncthreads();
    if ((tid & 63) == 0) {
      red[tid >> 6] = x;
      red[kWaves + (tid >> 6)] = yv;
    }
    __syncthreads();
    double sx = red[0], sy = red[kWaves];
    for (int w = 1; w < kWaves; ++w) {
      sx += red[w];
      sy += red[kWaves + w];
    }
    __syncthreads();
    return make_double2(sx, sy);
  }
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

// ------------------------------------------------------------ fine ETDRK4 ---
// J slices (J <= jmax) stepped together: `steps` ETDRK4 steps of slice s from
// src0 (s = 0) or src1 + (s - 1) 3 KP (modal FP64) to dst + s 3 KP.  The
// slices share the evaluations' transforms (one round over the wavefronts),
// and each rounds exactly as it would alone.  JM = 1 compiles the one-slice
// job (no run-time slice mapping, fewer registers).
// Coefficient tables [8][3][KP]: E_hi, E_lo, E2_hi, E2_lo, Q, f1, 2*f2, f3.
// The state and the step accumulator u+ = E u + f1 N(u) + 2f2 (N(a) + N(b))
// + f3 N(c) stay in FP64 in both precisions (E from the FP64 table): slowly
// varying modes change by less than half an FP32 ulp per step, so an FP32
// state would drop those increments coherently step after step.  With
// T = float the stage states a, b, c, the nonlinear evaluations and the
// products f*N run in FP32.
template <typename T, int NX, int NT, int S, int JM = 0, int PLAN = 0, int IMAX = 1>
__device__ __forceinline__ void fine_job(Engine<T, NX, NT, S, PLAN, IMAX>& en, int Jrun,
                                         const cx<double>* __restrict__ src0, const cx<double>* __restrict__ src1,
                                         cx<double>* __restrict__ dst, int steps,
                                         const cx<double>* __restrict__ coef64, const cx<T>* __restrict__ coef,
                                         const Basis<T>* __restrict__ basis) {
  using E_ = Engine<T, NX, NT, S, PLAN, IMAX>;
  constexpr int KP = E_::KP;
  // items per thread: the modes of one slice (JM = 1), else as many as the
  // largest job of this engine needs
  constexpr int MPT = JM == 1 ? E_::MPT : (E_::items(E_::jmax()) > E_::MPT ? E_::items(E_::jmax()) : E_::MPT);
  const int J = JM == 1 ? 1 : Jrun;   // JM = 1: a single slice, known when compiling
  const typename E_::template OwnT<MPT> ow(en.tid, J);
  // slice s reads src0 (s = 0) or src1 + (s - 1) * 3 KP and writes dst + s * 3 KP
  auto src_of = [&](int sl) { return sl == 0 ? src0 : src1 + size_t(sl - 1) * 3 * KP; };
  cx<double> c[MPT][3], cE[MPT][3];
  cx<T> cE2[MPT][3], cQ[MPT][3], cf1[MPT][3], cf2[MPT][3], cf3[MPT][3];
  Basis<T> bs[MPT];
#pragma unroll
  for (int j = 0; j < MPT; ++j) {
    const int k = ow.valid(j) ? ow.mode(j) : KP - 1;
    const cx<double>* src = src_of(ow.slice(j));
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
  cx<T> Nx[MPT][3], st[MPT][3], E2c[MPT][3], Nu[MPT][3];
  cx<double> acc[MPT][3];
  for (int step = 0; step < steps; ++step) {
#pragma unroll
    for (int j = 0; j < MPT; ++j)
#pragma unroll
      for (int al = 0; al < 3; ++al) st[j][al] = cvt<T>(c[j][al]);
    en.template neval_half<0>(J, ow, st, Nu, bs);
#pragma unroll
    for (int j = 0; j < MPT; ++j)
#pragma unroll
      for (int al = 0; al < 3; ++al) {
        E2c[j][al] = cE2[j][al] * st[j][al];
        st[j][al] = cfma(cQ[j][al], Nu[j][al], E2c[j][al]);                                   // a
        acc[j][al] = cE[j][al] * c[j][al] + cvt<double>(cf1[j][al] * Nu[j][al]);
      }
    en.template neval_half<1>(J, ow, st, Nx, bs);                                             // N(a)
#pragma unroll
    for (int j = 0; j < MPT; ++j)
#pragma unroll
      for (int al = 0; al < 3; ++al) {
        acc[j][al] = acc[j][al] + cvt<double>(cf2[j][al] * Nx[j][al]);
        const cx<T> a_ = st[j][al];
        st[j][al] = cfma(cQ[j][al], Nx[j][al], E2c[j][al]);                                   // b
        E2c[j][al] = cE2[j][al] * a_;                                                         // E2 a
      }
    en.template neval_half<0>(J, ow, st, Nx, bs);                                             // N(b)
#pragma unroll
    for (int j = 0; j < MPT; ++j)
#pragma unroll
      for (int al = 0; al < 3; ++al) {
        acc[j][al] = acc[j][al] + cvt<double>(cf2[j][al] * Nx[j][al]);
        st[j][al] = cfma(cQ[j][al], T(2) * Nx[j][al] - Nu[j][al], E2c[j][al]);                // c
      }
    en.template neval_half<1>(J, ow, st, Nx, bs);                                             // N(c)
#pragma unroll
    for (int j = 0; j < MPT; ++j)
#pragma unroll
      for (int al = 0; al < 3; ++al) c[j][al] = acc[j][al] + cvt<double>(cf3[j][al] * Nx[j][al]);
  }
#pragma unroll
  for (int j = 0; j < MPT; ++j)
    if (ow.valid(j)) {
      cx<double>* out = dst + size_t(ow.slice(j)) * 3 * KP;
      for (int al = 0; al < 3; ++al) out[al * KP + ow.mode(j)] = c[j][al];
    }
}

// --------------------------------------------------------- Strang steps ---
// Strang splitting (Alg. 3) on owned-mode registers c (FP64): per step of
// size h, the half step of the linear flow (E2 = e^{(h/2) lambda} per
// (k, alpha), FP64), the midpoint step of the nonlinear flow
// v <- v + h N(v + (h/2) N(v)), and the second half step.  The evaluations and
// the midpoint state run in T; the state and its update stay in FP64.
template <typename T, int NX, int NT, int S>
__device__ __forceinline__ void strang_regs(Engine<T, NX, NT, S>& en, int J,
                                            const typename Engine<T, NX, NT, S>::Own& ow,
                                            cx<double> (&c)[Engine<T, NX, NT, S>::MPT][3],
                                            int steps, const cx<double> (&cE2)[Engine<T, NX, NT, S>::MPT][3],
                                            double h, const Basis<T> (&bs)[Engine<T, NX, NT, S>::MPT]) {
  using E_ = Engine<T, NX, NT, S>;
  constexpr int MPT = E_::MPT;
  const T hh = T(0.5 * h), hT = T(h);
  cx<T> st[MPT][3], nv[MPT][3];
  cx<double> v[MPT][3];
  for (int step = 0; step < steps; ++step) {
#pragma unroll
    for (int j = 0; j < MPT; ++j)
#pragma unroll
      for (int al = 0; al < 3; ++al) {
        v[j][al] = cE2[j][al] * c[j][al];
        st[j][al] = cvt<T>(v[j][al]);
      }
    en.template neval_half<0>(J, ow, st, nv, bs);
#pragma unroll
    for (int j = 0; j < MPT; ++j)
#pragma unroll
      for (int al = 0; al < 3; ++al) st[j][al] = st[j][al] + hh * nv[j][al];
    en.template neval_half<1>(J, ow, st, nv, bs);
#pragma unroll
    for (int j = 0; j < MPT; ++j)
#pragma unroll
      for (int al = 0; al < 3; ++al) c[j][al] = cE2[j][al] * (v[j][al] + cvt<double>(hT * nv[j][al]));
  }
}
template <typename T, int NX, int NT, int S>
__device__ __forceinline__ void strang_regs(Engine<T, NX, NT, S>& en, cx<double> (&c)[Engine<T, NX, NT, S>::MPT][3],
                                            int steps, const cx<double> (&cE2)[Engine<T, NX, NT, S>::MPT][3],
                                            double h, const Basis<T> (&bs)[Engine<T, NX, NT, S>::MPT]) {
  strang_regs<T, NX, NT, S>(en, 1, typename Engine<T, NX, NT, S>::Own(en.tid, 1), c, steps, cE2, h, bs);
}

// Owned items of the FP64 coefficient slot `slot` of a [8][3][KP] table.
template <typename T, int NX, int NT, int S>
__device__ __forceinline__ void load_coef64(const cx<double>* __restrict__ coef64, int slot,
                                            const typename Engine<T, NX, NT, S>::Own& ow,
                                            cx<double> (&out)[Engine<T, NX, NT, S>::MPT][3]) {
  using E_ = Engine<T, NX, NT, S>;
#pragma unroll
  for (int j = 0; j < E_::MPT; ++j) {
    const int k = ow.valid(j) ? ow.mode(j) : E_::KP - 1;
    for (int al = 0; al < 3; ++al) out[j][al] = coef64[size_t(slot) * 3 * E_::KP + al * E_::KP + k];
  }
}
template <typename T, int NX, int NT, int S>
__device__ __forceinline__ void load_coef64(const Engine<T, NX, NT, S>& en, const cx<double>* __restrict__ coef64,
                                            int slot, cx<double> (&out)[Engine<T, NX, NT, S>::MPT][3]) {
  load_coef64<T, NX, NT, S>(coef64, slot, typename Engine<T, NX, NT, S>::Own(en.tid, 1), out);
}

// `steps` Strang steps of size h for J slices (as fine_job: slice s from src0
// or src1 + (s - 1) 3 KP to dst + s 3 KP; modal FP64; the table's slot 2
// holds E2 = e^{(h/2) lambda}).
template <typename T, int NX, int NT, int S, int JM = 0>
__device__ __forceinline__ void strang_job(Engine<T, NX, NT, S>& en, int Jrun, const cx<double>* __restrict__ src0,
                                           const cx<double>* __restrict__ src1, cx<double>* __restrict__ dst,
                                           int steps, const cx<double>* __restrict__ coef64, double h,
                                           const Basis<T>* __restrict__ basis) {
  using E_ = Engine<T, NX, NT, S>;
  constexpr int MPT = E_::MPT;
  constexpr int KP = E_::KP;
  const int J = JM == 1 ? 1 : Jrun;   // JM = 1: a single slice, known when compiling
  const typename E_::Own ow(en.tid, J);
  cx<double> c[MPT][3], cE2[MPT][3];
  Basis<T> bs[MPT];
#pragma unroll
  for (int j = 0; j < MPT; ++j) {
    const int k = ow.valid(j) ? ow.mode(j) : KP - 1;
    const int sl = ow.slice(j);
    const cx<double>* src = sl == 0 ? src0 : src1 + size_t(sl - 1) * 3 * KP;
    bs[j] = basis[k];
    for (int al = 0; al < 3; ++al) c[j][al] = src[al * KP + k];
  }
  load_coef64<T, NX, NT, S>(coef64, 2, ow, cE2);
  strang_regs<T, NX, NT, S>(en, J, ow, c, steps, cE2, h, bs);
#pragma unroll
  for (int j = 0; j < MPT; ++j)
    if (ow.valid(j)) {
      cx<double>* out = dst + size_t(ow.slice(j)) * 3 * KP;
      for (int al = 0; al < 3; ++al) out[al * KP + ow.mode(j)] = c[j][al];
    }
}

// ----------------------------------------------------------- time average ---
// Nbar contributions of the samples m in [mb, me) of the owned-mode state yv,
// with min(S, me - m0) samples in flight.  [mb, me) covers whole groups of
// av.gs consecutive samples (the last group may be shorter).  Per chunk every
// thread rotates (sample, mode) items into the slots' field spectra; the
// wavefronts run the inverse transforms and the forward transforms of the
// products; every thread turns (sample, mode) items back into weighted,
// rotated modal contributions in the slot's ib; the mode owners then add the
// contributions of each group in increasing sample order.
//   whole:  acc = 0 + S_0 + S_1 + ... over the groups, in increasing order
//   !whole: [mb, me) is one group and acc = its sum S_g
// (S_g = c_first + c_next + ..., the same association in every kernel).
template <typename T, int NX, int NT, int S>
__device__ __forceinline__ void nbar_range(Engine<T, NX, NT, S>& en,
                                           const cx<T> (&yv)[Engine<T, NX, NT, S>::MPT][3],
                                           cx<T> (&acc)[Engine<T, NX, NT, S>::MPT][3], int mb, int me, bool whole,
                                           const AvgTab<T>& av, const Basis<T>* __restrict__ basis) {
  using E_ = Engine<T, NX, NT, S>;
  using SL = Slot<T, NX>;
  constexpr int KP = E_::KP;
  constexpr int MPT = E_::MPT;
  cx<T> pg[MPT][3];
#pragma unroll
  for (int j = 0; j < MPT; ++j) {
    for (int al = 0; al < 3; ++al) {
      acc[j][al] = czero<T>();
      pg[j][al] = czero<T>();
    }
    if (en.valid(j))
      for (int al = 0; al < 3; ++al) en.y[al * KP + en.mode(j)] = yv[j][al];
  }
  __syncthreads();
  for (int m0 = mb; m0 < me; m0 += S) {
    const int ns = min(S, me - m0);
    for (int i = en.tid; i < ns * KP; i += NT) {
      const int s = i / KP, k = i - s * KP;
      const cx<T> e = av.rot[size_t(m0 + s) * KP + k];
      cx<T> x[3];
      for (int al = 0; al < 3; ++al) x[al] = rot_in(en.y[al * KP + k], e, al);
      put_fields<T, NX>(en.sp, s, k, x, basis[k]);
    }
    zero_tails<T, NX, NT>(en.sp, ns, en.tid);
    __syncthreads();
    inverse_fields<T, NX, NT>(en.sp, en.ib, ns, en.tw, en.tid);
    __syncthreads();
    forward_products<T, NX, NT>(en.sp, en.ib, ns, en.tw, en.tid);
    __syncthreads();
    for (int i = en.tid; i < ns * KP; i += NT) {
      const int s = i / KP, k = i - s * KP;
      const cx<T> e = av.rot[size_t(m0 + s) * KP + k];
      const T wm = av.w[m0 + s];
      cx<T> n[3];
      get_N_sp<T, NX>(en.sp + s * SL::sp_elems, k, basis[k], en.tw, n);
      cx<T>* c = en.ib + s * SL::ib_elems;
      for (int al = 0; al < 3; ++al) c[al * KP + k] = wm * rot_out(n[al], e, al);
    }
    __syncthreads();
    for (int s = 0; s < ns; ++s) {
      const int r = (m0 + s - 1) % av.gs;
      const bool first = r == 0;
      const bool last = r == av.gs - 1 || m0 + s == av.M - 1;
      const cx<T>* c = en.ib + s * SL::ib_elems;
#pragma unroll
      for (int j = 0; j < MPT; ++j) {
        if (!en.valid(j)) continue;
        const int k = en.mode(j);
        for (int al = 0; al < 3; ++al) {
          const cx<T> v = c[al * KP + k];
          pg[j][al] = first ? v : pg[j][al] + v;
          if (last) acc[j][al] = whole ? acc[j][al] + pg[j][al] : pg[j][al];
        }
      }
    }
  }
}

// Nbar over all samples (every group, in order).
template <typename T, int NX, int NT, int S>
__device__ __forceinline__ void nbar_owned(Engine<T, NX, NT, S>& en,
                                           const cx<T> (&yv)[Engine<T, NX, NT, S>::MPT][3],
                                           cx<T> (&acc)[Engine<T, NX, NT, S>::MPT][3], const AvgTab<T>& av,
                                           const Basis<T>* __restrict__ basis) {
  nbar_range<T, NX, NT, S>(en, yv, acc, 1, av.M, true, av, basis);
}

// ------------------------------------------------------------ coarse step ---
// The asymptotic coarse step (Alg. 2) on owned-mode registers, in pieces that
// the single-workgroup and the split evaluation share, so that both round
// identically:
//   w = e^{(dT/2) D} u;  y = w + (dT/2) Nbar(w);
//   g = e^{-(dT/eps) L} e^{(dT/2) D} (w + dT Nbar(y)).
template <typename T, int MPT>
struct CoarseRegs {
  T hd[MPT];
  cx<T> rT[MPT];
};

template <typename T, int NX, int NT, int S>
__device__ __forceinline__ void coarse_begin(const Engine<T, NX, NT, S>& en, const CoarseTab<T>& ct,
                                             const cx<T> (&u)[Engine<T, NX, NT, S>::MPT][3],
                                             cx<T> (&w)[Engine<T, NX, NT, S>::MPT][3],
                                             CoarseRegs<T, Engine<T, NX, NT, S>::MPT>& cr) {
  using E_ = Engine<T, NX, NT, S>;
#pragma unroll
  for (int j = 0; j < E_::MPT; ++j) {
    const int k = en.valid(j) ? en.mode(j) : 0;
    cr.hd[j] = ct.hd[k];
    cr.rT[j] = ct.rotT[k];
    for (int al = 0; al < 3; ++al) w[j][al] = cr.hd[j] * u[j][al];
  }
}

template <typename T, int MPT>
__device__ __forceinline__ void coarse_mid(const CoarseTab<T>& ct, const cx<T> (&w)[MPT][3],
                                           const cx<T> (&k1)[MPT][3], cx<T> (&y)[MPT][3]) {
  const T half = T(0.5) * ct.dT;
#pragma unroll
  for (int j = 0; j < MPT; ++j)
    for (int al = 0; al < 3; ++al) y[j][al] = w[j][al] + half * k1[j][al];
}

template <typename T, int MPT>
__device__ __forceinline__ void coarse_end(const CoarseTab<T>& ct, const CoarseRegs<T, MPT>& cr,
                                           const cx<T> (&w)[MPT][3], const cx<T> (&k2)[MPT][3],
                                           cx<T> (&g)[MPT][3]) {
#pragma unroll
  for (int j = 0; j < MPT; ++j)
    for (int al = 0; al < 3; ++al) {
      const cx<T> v = cr.hd[j] * (w[j][al] + ct.dT * k2[j][al]);
      g[j][al] = al == 2 ? v * cr.rT[j] : (al == 0 ? v * conj(cr.rT[j]) : v);
    }
}

// One asymptotic coarse step in one workgroup: u -> g.
template <typename T, int NX, int NT, int S>
__device__ __forceinline__ void coarse_owned(Engine<T, NX, NT, S>& en,
                                             const cx<T> (&u)[Engine<T, NX, NT, S>::MPT][3],
                                             cx<T> (&g)[Engine<T, NX, NT, S>::MPT][3],
                                             const CoarseTab<T>& ct, const Basis<T>* __restrict__ basis) {
  constexpr int MPT = Engine<T, NX, NT, S>::MPT;
  cx<T> w[MPT][3], y[MPT][3], kk[MPT][3];
  CoarseRegs<T, MPT> cr;
  coarse_begin<T, NX, NT, S>(en, ct, u, w, cr);
  nbar_owned<T, NX, NT, S>(en, w, kk, ct.avg, basis);
  coarse_mid<T, MPT>(ct, w, kk, y);
  nbar_owned<T, NX, NT, S>(en, y, kk, ct.avg, basis);
  coarse_end<T, MPT>(ct, cr, w, kk, g);
}

// Owned modes of a modal FP64 state, rounded to T (zero for unowned slots).
template <typename T, int NX, int NT, int S>
__device__ __forceinline__ void load_owned(const Engine<T, NX, NT, S>& en, const cx<double>* __restrict__ src,
                                           cx<T> (&u)[Engine<T, NX, NT, S>::MPT][3]) {
  using E_ = Engine<T, NX, NT, S>;
#pragma unroll
  for (int j = 0; j < E_::MPT; ++j) {
    const int k = en.valid(j) ? en.mode(j) : 0;
    for (int al = 0; al < 3; ++al) u[j][al] = en.valid(j) ? cvt<T>(src[al * E_::KP + k]) : czero<T>();
  }
}

// The parareal correction of a coarse result g (owned modes):
//   gnew <- g;  unew <- g (gold == nullptr, k = 0) or fold + (g - gold) (FP64);
//   uold != nullptr: *part = (sum |unew - uold|^2, sum |unew|^2) with Parseval
//   weights (1 for k = 0, 2 otherwise).
// Every location is read before it is written by the same thread, so unew may
// alias uold and gnew may alias gold (the in-place serial sweep).
template <typename T, int NX, int NT, int S, typename GT = T>
__device__ __forceinline__ void coarse_correct(Engine<T, NX, NT, S>& en,
                                               const cx<GT> (&g)[Engine<T, NX, NT, S>::MPT][3], cx<double>* unew,
                                               cx<double>* gnew, const cx<double>* gold, const cx<double>* fold,
                                               const cx<double>* uold, double2* part) {
  using E_ = Engine<T, NX, NT, S>;
  constexpr int KP = E_::KP;
  double num = 0.0, den = 0.0;
#pragma unroll
  for (int j = 0; j < E_::MPT; ++j) {
    if (!en.valid(j)) continue;
    const int k = en.mode(j);
    const double wgt = k == 0 ? 1.0 : 2.0;
    for (int al = 0; al < 3; ++al) {
      const int o = al * KP + k;
      const cx<double> gn = cvt<double>(g[j][al]);
      cx<double> un = gn;
      if (gold) un = fold[o] + (gn - gold[o]);
      if (uold) {
        const cx<double> d = un - uold[o];
        num += wgt * (d.x * d.x + d.y * d.y);
        den += wgt * (un.x * un.x + un.y * un.y);
      }
      gnew[o] = gn;
      unew[o] = un;
    }
  }
  if (uold) {
    const double2 r = en.block_sum2(num, den);
    if (en.tid == 0) *part = r;
  }
}

// The coarse job of standard parareal: g = one Strang step of size dT
// (table slot 2: e^{(dT/2) lambda}) from uprev, then the correction.
template <typename T, int NX, int NT, int S>
__device__ __forceinline__ void strang_coarse_job(Engine<T, NX, NT, S>& en, const cx<double>* __restrict__ ccoef64,
                                                  double dT, const Basis<T>* __restrict__ basis,
                                                  const cx<double>* uprev, cx<double>* unew, cx<double>* gnew,
                                                  const cx<double>* gold, const cx<double>* fold,
                                                  const cx<double>* uold, double2* part) {
  using E_ = Engine<T, NX, NT, S>;
  constexpr int MPT = E_::MPT;
  cx<double> g[MPT][3], cE2[MPT][3];
  Basis<T> bs[MPT];
#pragma unroll
  for (int j = 0; j < MPT; ++j) {
    const int k = en.valid(j) ? en.mode(j) : 0;
    bs[j] = basis[k];
    for (int al = 0; al < 3; ++al) g[j][al] = en.valid(j) ? uprev[al * E_::KP + k] : czero<double>();
  }
  load_coef64<T, NX, NT, S>(en, ccoef64, 2, cE2);
  strang_regs<T, NX, NT, S>(en, g, 1, cE2, dT, bs);
  coarse_correct<T, NX, NT, S, double>(en, g, unew, gnew, gold, fold, uold, part);
}

// One coarse job of the parareal iteration on modal FP64 states, in one
// workgroup: g = G(uprev), then the correction above.
template <typename T, int NX, int NT, int S>
__device__ __forceinline__ void coarse_job(Engine<T, NX, NT, S>& en, const CoarseTab<T>& ct,
                                           const Basis<T>* __restrict__ basis, const cx<double>* uprev,
                                           cx<double>* unew, cx<double>* gnew, const cx<double>* gold,
                                           const cx<double>* fold, const cx<double>* uold, double2* part) {
  constexpr int MPT = Engine<T, NX, NT, S>::MPT;
  cx<T> u[MPT][3], g[MPT][3];
  load_owned<T, NX, NT, S>(en, uprev, u);
  coarse_owned<T, NX, NT, S>(en, u, g, ct, basis);
  coarse_correct<T, NX, NT, S>(en, g, unew, gnew, gold, fold, uold, part);
}

// The coarse job of a slice that the iteration has made exact (n <= k): the
// state `src` (U(k-1,n) or F(k-1,k)) becomes U(k,n), G(k-1,n) becomes G(k,n),
// and the residual parts are those of the full correction (whose coarse
// difference is exactly zero here).
template <typename T, int NX, int NT, int S>
__device__ __forceinline__ void copy_job(Engine<T, NX, NT, S>& en, const cx<double>* src, cx<double>* unew,
                                         const cx<double>* gold, cx<double>* gnew, const cx<double>* uold,
                                         double2* part) {
  using E_ = Engine<T, NX, NT, S>;
  constexpr int KP = E_::KP;
  double num = 0.0, den = 0.0;
#pragma unroll
  for (int j = 0; j < E_::MPT; ++j) {
    if (!en.valid(j)) continue;
    const int k = en.mode(j);
    const double wgt = k == 0 ? 1.0 : 2.0;
    for (int al = 0; al < 3; ++al) {
      const int o = al * KP + k;
      const cx<double> un = src[o];
      const cx<double> d = un - uold[o];
      num += wgt * (d.x * d.x + d.y * d.y);
      den += wgt * (un.x * un.x + un.y * un.y);
      gnew[o] = gold[o];
      unew[o] = un;
    }
  }
  const double2 r = en.block_sum2(num, den);
  if (en.tid == 0) *part = r;
}

// r^k = max_n sqrt(num_n / den_n) over the residual parts of one level.
template <typename T, int NX, int NT, int S>
__device__ __forceinline__ double level_residual(Engine<T, NX, NT, S>& en, const double2* part, int Ns) {
  __syncthreads();   // the last part was written by thread 0 of this workgroup
  double m = 0.0;
  for (int n = en.tid; n < Ns; n += NT) {
    const double2 q = part[n];
    const double r = q.y > 0.0 ? sqrt(q.x / q.y) : (q.x > 0.0 ? INFINITY : 0.0);
    m = (r > m || r != r) ? r : m;
  }
  return en.block_max(m);
}

// ------------------------------------------------- split coarse step -------
// A coarse step evaluated by several workgroups: the stage-1 job of group g
// stores S_g of Nbar(w); the last stage-1 job to finish sums the stored group
// sums (0 + S_0 + S_1 + ..., the order of the single-workgroup step), forms
// the midpoint state y once and stores it; the stage-2 job of group g loads y
// and stores S_g of Nbar(y).
template <typename T, int NX, int NT, int S>
__device__ __forceinline__ void sum_groups(const Engine<T, NX, NT, S>& en, const cx<T>* __restrict__ P, int groups,
                                           cx<T> (&acc)[Engine<T, NX, NT, S>::MPT][3]) {
  using E_ = Engine<T, NX, NT, S>;
  constexpr int KP = E_::KP;
  constexpr int B = 8;   // group sums in flight per thread (written by other workgroups: long latency)
#pragma unroll
  for (int j = 0; j < E_::MPT; ++j)
    for (int al = 0; al < 3; ++al) acc[j][al] = czero<T>();
  for (int g0 = 0; g0 < groups; g0 += B) {
    const int nb = min(B, groups - g0);
    cx<T> v[B][E_::MPT][3];
    // issue the loads of up to B groups, then add them in increasing group order
#pragma unroll
    for (int b = 0; b < B; ++b) {
      const cx<T>* Pg = P + size_t(g0 + (b < nb ? b : 0)) * 3 * KP;
#pragma unroll
      for (int j = 0; j < E_::MPT; ++j)
        for (int al = 0; al < 3; ++al) v[b][j][al] = en.valid(j) ? Pg[al * KP + en.mode(j)] : czero<T>();
    }
#pragma unroll
    for (int b = 0; b < B; ++b) {
      if (b >= nb) break;
#pragma unroll
      for (int j = 0; j < E_::MPT; ++j)
        for (int al = 0; al < 3; ++al) acc[j][al] = acc[j][al] + v[b][j][al];
    }
  }
}

template <typename T, int NX, int NT, int S>
__device__ __forceinline__ void store_owned(const Engine<T, NX, NT, S>& en, cx<T>* __restrict__ dst,
                                            const cx<T> (&v)[Engine<T, NX, NT, S>::MPT][3]) {
  using E_ = Engine<T, NX, NT, S>;
#pragma unroll
  for (int j = 0; j < E_::MPT; ++j)
    if (en.valid(j))
      for (int al = 0; al < 3; ++al) dst[al * E_::KP + en.mode(j)] = v[j][al];
}

// Stage job of group g: stage 1 stores S_g(Nbar(w)) at Pout; stage 2 loads
// the step's midpoint state y from Y and stores S_g(Nbar(y)) at Pout.  On
// return, w holds the step's w (for the midpoint and the finishing job).
// Stage 2 calls wait_y() (every thread; true when y is published) after
// forming w from uprev, so that loading uprev and the first half step overlap
// the wait for the midpoint; it returns false (and does nothing more) when
// wait_y() does.
template <typename T, int NX, int NT, int S, typename WaitY>
__device__ __forceinline__ bool stage_job(Engine<T, NX, NT, S>& en, const CoarseTab<T>& ct,
                                          const Basis<T>* __restrict__ basis, const cx<double>* uprev, int stage,
                                          int g, const cx<T>* Y, cx<T>* Pout,
                                          cx<T> (&w)[Engine<T, NX, NT, S>::MPT][3],
                                          CoarseRegs<T, Engine<T, NX, NT, S>::MPT>& cr, WaitY&& wait_y) {
  using E_ = Engine<T, NX, NT, S>;
  constexpr int MPT = E_::MPT;
  cx<T> u[MPT][3], y[MPT][3], acc[MPT][3];
  load_owned<T, NX, NT, S>(en, uprev, u);
  coarse_begin<T, NX, NT, S>(en, ct, u, w, cr);
  if (stage == 2) {
    if (!wait_y()) return false;
#pragma unroll
    for (int j = 0; j < MPT; ++j)
      for (int al = 0; al < 3; ++al) y[j][al] = en.valid(j) ? Y[al * E_::KP + en.mode(j)] : czero<T>();
  } else {
#pragma unroll
    for (int j = 0; j < MPT; ++j)
      for (int al = 0; al < 3; ++al) y[j][al] = w[j][al];
  }
  const int mb = 1 + g * ct.avg.gs;
  const int me = min(ct.avg.M, mb + ct.avg.gs);
  nbar_range<T, NX, NT, S>(en, y, acc, mb, me, false, ct.avg, basis);
  store_owned<T, NX, NT, S>(en, Pout, acc);
  return true;
}

// The midpoint state of a split step, formed by its last stage-1 job: the sum
// of the stage-1 group sums at P1 (in group order), then y from w, stored at Y
// in the working precision (the stage-2 jobs load exactly these values).
template <typename T, int NX, int NT, int S>
__device__ __forceinline__ void stage_mid(const Engine<T, NX, NT, S>& en, const CoarseTab<T>& ct, const cx<T>* P1,
                                          int groups, const cx<T> (&w)[Engine<T, NX, NT, S>::MPT][3], cx<T>* Y) {
  constexpr int MPT = Engine<T, NX, NT, S>::MPT;
  cx<T> acc[MPT][3], y[MPT][3];
  sum_groups<T, NX, NT, S>(en, P1, groups, acc);
  coarse_mid<T, MPT>(ct, w, acc, y);
  store_owned<T, NX, NT, S>(en, Y, y);
}

// The finishing part of a split step: Nbar(y) = sum of the stage-2 group sums,
// then the end of the step (the correction follows via coarse_correct).
template <typename T, int NX, int NT, int S>
__device__ __forceinline__ void stage_finish(const Engine<T, NX, NT, S>& en, const CoarseTab<T>& ct, const cx<T>* P2,
                                             int groups, const cx<T> (&w)[Engine<T, NX, NT, S>::MPT][3],
                                             const CoarseRegs<T, Engine<T, NX, NT, S>::MPT>& cr,
                                             cx<T> (&g)[Engine<T, NX, NT, S>::MPT][3]) {
  constexpr int MPT = Engine<T, NX, NT, S>::MPT;
  cx<T> k2[MPT][3];
  sum_groups<T, NX, NT, S>(en, P2, groups, k2);
  coarse_end<T, MPT>(ct, cr, w, k2, g);
}

}  // namespace ap
