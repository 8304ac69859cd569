// Wave-local FFTs and the fused nonlinear evaluation on top of them.
//
// A group of G lanes of one wavefront (G = 8..64 by length) transforms one real
// signal of length N through a complex FFT of length P = N/2, with in-place
// Stockham passes of radix 4, 8 or 16 in LDS: every lane loads its
// butterflies' inputs, computes a register DFT, and after a wavefront-level
// synchronisation stores the outputs at their auto-sorted positions.  No
// workgroup barrier is needed inside a transform; 64/G signals share a
// wavefront and the wavefronts of a workgroup work on further signals.
//
// The real-signal pre/post-processing is fused into the first and last data
// movement: the first inverse pass forms Z[k] = (X[k] + conj X[P-k])
//   + i e^{2 pi i k/N} (X[k] - conj X[P-k]) from the half spectrum on the fly,
// and the first forward pass forms the quadratic products (v1^2/2, v1 v2x,
// h v1) of the inverse outputs on the fly.
#pragma once
#include "rsw_device.hpp"

namespace ap {

// Orders LDS accesses of one wavefront: the hardware executes a wavefront's
// LDS instructions in order; this keeps the compiler from reordering them.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// cos(2 pi j / 16), j = 0..15 (sin(2 pi j/16) = cos(2 pi (j+12)/16))
constexpr double kCos16[16] = {1.0,
                               0.92387953251128675613,
                               0.70710678118654752440,
                               0.38268343236508977173,
                               0.0,
                               -0.38268343236508977173,
                               -0.70710678118654752440,
                               -0.92387953251128675613,
                               -1.0,
                               -0.92387953251128675613,
                               -0.70710678118654752440,
                               -0.38268343236508977173,
                               0.0,
                               0.38268343236508977173,
                               0.70710678118654752440,
                               0.92387953251128675613};

// Register DFT y_q = sum_p x_p exp(DIR 2 pi i p q / R), R a power of two <= 16,
// radix-2 decimation in time with compile-time twiddles.
template <typename T, int R, int DIR, int K>
__device__ __forceinline__ void dft_combine(cx<T> (&x)[R], const cx<T> (&e)[R / 2], const cx<T> (&o)[R / 2]) {
  if constexpr (K < R / 2) {
    cx<T> t;
    if constexpr (K == 0) {
      t = o[0];
    } else if constexpr (4 * K == R) {
      t = DIR > 0 ? mul_i(o[K]) : mul_mi(o[K]);
    } else {
      constexpr int j = K * 16 / R;
      const cx<T> w{T(kCos16[j]), T(DIR > 0 ? kCos16[(j + 12) % 16] : -kCos16[(j + 12) % 16])};
      t = w * o[K];
    }
    x[K] = e[K] + t;
    x[K + R / 2] = e[K] - t;
    dft_combine<T, R, DIR, K + 1>(x, e, o);
  }
}

template <typename T, int R, int DIR>
__device__ __forceinline__ void dft_reg(cx<T> (&x)[R]) {
  if constexpr (R == 2) {
    const cx<T> a = x[0] + x[1], b = x[0] - x[1];
    x[0] = a;
    x[1] = b;
  } else {
    cx<T> e[R / 2], o[R / 2];
#pragma unroll
    for (int i = 0; i < R / 2; ++i) {
      e[i] = x[2 * i];
      o[i] = x[2 * i + 1];
    }
    dft_reg<T, R / 2, DIR>(e);
    dft_reg<T, R / 2, DIR>(o);
    dft_combine<T, R, DIR, 0>(x, e, o);
  }
}

// Plan per transform length: G lanes per signal (64/G signals share a
// wavefront) and n passes of radices r0 .. r3 with product P.  Every pass has
// at least G butterflies where the length allows it (P >= 128): a pass with
// fewer leaves lanes repeating butterflies, so radix-4 passes (and one radix-2
// pass) beat fewer passes of radix 8.  The plans for P = 128, 256, 512 and
// 1024 are also chosen so that some exchanges between passes are row swaps
// in registers rather than LDS round trips (see wave_pass_pair and
// wave_pass_first_pair): at P = 512, radices 8, 4, 4, 4 take the same
// arithmetic as 8, 8, 8 and move the data through LDS four times instead of
// six.
//   PLAN 0 is that plan (the one every kernel uses).  PLAN 1, an alternative
// for the fine batch's autotuner at P >= 128, is the classic Stockham FFT:
// the same radices with every exchange through LDS, and at P = 512 radices
// 8, 8, 8.  PLAN 1 rounds like PLAN 0 except at P = 512.
template <int P, int PLAN = 0> struct WavePlan;
template <> struct WavePlan<32>   { static constexpr int G = 8,  n = 2, r0 = 4,  r1 = 8, r2 = 1, r3 = 1; };
template <> struct WavePlan<64>   { static constexpr int G = 16, n = 3, r0 = 4,  r1 = 4, r2 = 4, r3 = 1; };
template <> struct WavePlan<128>  { static constexpr int G = 32, n = 4, r0 = 4,  r1 = 4, r2 = 4, r3 = 2; };
template <> struct WavePlan<256>  { static constexpr int G = 64, n = 4, r0 = 4,  r1 = 4, r2 = 4, r3 = 4; };
template <> struct WavePlan<512>  { static constexpr int G = 64, n = 4, r0 = 8,  r1 = 4, r2 = 4, r3 = 4; };
template <> struct WavePlan<1024> { static constexpr int G = 64, n = 3, r0 = 16, r1 = 8, r2 = 8, r3 = 1; };
template <int P> struct WavePlan<P, 1> : WavePlan<P, 0> {};
template <> struct WavePlan<512, 1> { static constexpr int G = 64, n = 3, r0 = 8, r1 = 8, r2 = 8, r3 = 1; };

// FFT plans compiled for transform length P (PLAN 1 only where it differs).
constexpr int wave_plans(int P) { return P >= 128 ? 2 : 1; }

// Twiddle table of a grid size N = 2P: entries t < N hold exp(-2 pi i t/N)
// (real-signal pre/post-processing); then, for each pass j after the first,
// exp(-2 pi i q k / (NS R)) at [offset_j + (q-1) NS + k] (q = 1..R-1, k < NS;
// NS points combined before the pass, radix R), contiguous in k so that the
// lanes of a pass read consecutive entries.
// Each plan has a table of its own (the host stores plan 1's after plan 0's).
template <int P, int PLAN = 0>
constexpr int pass1_tw_offset() { return 2 * P; }
template <int P, int PLAN = 0>
constexpr int pass2_tw_offset() { return 2 * P + (WavePlan<P, PLAN>::r1 - 1) * WavePlan<P, PLAN>::r0; }
template <int P, int PLAN = 0>
constexpr int pass3_tw_offset() {
  using PL = WavePlan<P, PLAN>;
  return pass2_tw_offset<P, PLAN>() + (PL::r2 - 1) * PL::r0 * PL::r1;
}
template <int P, int PLAN = 0>
constexpr int tw_elems() {
  using PL = WavePlan<P, PLAN>;
  return PL::n == 4   ? pass3_tw_offset<P, PLAN>() + (PL::r3 - 1) * PL::r0 * PL::r1 * PL::r2
         : PL::n == 3 ? pass3_tw_offset<P, PLAN>()
                      : pass2_tw_offset<P, PLAN>();
}

// The radices of plan `plan` for transform length P (host side, for the
// tables and the plan queries); *regx: exchanges done by row swaps.
inline void wave_plan_radices(int P, int r[4], int* n, int plan = 0, int* regx = nullptr) {
  r[3] = 1;
  int x = 0;
  switch (P) {
    case 32: r[0] = 4; r[1] = 8; r[2] = 1; *n = 2; break;
    case 64: r[0] = 4; r[1] = 4; r[2] = 4; *n = 3; break;
    case 128: r[0] = 4; r[1] = 4; r[2] = 4; r[3] = 2; *n = 4; x = 1; break;
    case 256: r[0] = 4; r[1] = 4; r[2] = 4; r[3] = 4; *n = 4; x = 2; break;
    case 512:
      if (plan == 1) {
        r[0] = 8; r[1] = 8; r[2] = 8; *n = 3;
      } else {
        r[0] = 8; r[1] = 4; r[2] = 4; r[3] = 4; *n = 4; x = 2;
      }
      break;
    default: r[0] = 16; r[1] = 8; r[2] = 8; *n = 3; x = 1; break;
  }
  if (regx) *regx = plan == 1 ? 0 : x;
}

// LDS layouts between passes.  A pass writes position pos to
// (pos with the bits inside its bank row XORed by f(row)), row = pos / E with
// E the elements per row of the 64 four-byte banks (32 complex floats, 16
// complex doubles); the next pass reads through the same map.  Loads of
// E consecutive positions stay one permuted row; f per pass makes the
// stride-R stores of that pass hit distinct banks (chosen by a model of the
// bank mapping).  The last pass writes natural order (its stores are
// consecutive already), which is what the consumers read.
enum : int { kSwzId = 0, kSwzR = 1, kSwzR5 = 2, kSwzR9 = 3, kSwzRx2 = 4, kSwzRx1 = 5, kSwzRh1 = 6 };
template <typename T, int CODE>
__device__ __forceinline__ int swz(int pos) {
  if constexpr (CODE == kSwzId) {
    return pos;
  } else {
    constexpr int rb = sizeof(T) == 4 ? 5 : 4;   // complex float: 32 per row; complex double: 16
    constexpr int m = (1 << rb) - 1;
    const int r = pos >> rb;
    int f;
    if constexpr (CODE == kSwzR) f = r;
    else if constexpr (CODE == kSwzR5) f = r * 5;
    else if constexpr (CODE == kSwzR9) f = r * 9;
    else if constexpr (CODE == kSwzRx2) f = r ^ (r << 2);
    else if constexpr (CODE == kSwzRx1) f = r ^ (r << 1);
    else f = r >> 1;
    return pos ^ (f & m);
  }
}
// layout written by pass 0 / pass 1 (not the last) for transform length P;
// at P = 256 and 512 pass 1 stores in the rotated butterfly order of
// wave_pass_first_pair
template <typename T, int P>
constexpr int swz_pass0() { return kSwzR; }
template <typename T, int P, int PLAN = 0>
constexpr int swz_pass1() {
  if constexpr (PLAN == 1) {
    if constexpr (sizeof(T) == 4) return P <= 256 ? kSwzR5 : kSwzRx2;
    else return P <= 256 ? kSwzR5 : P == 512 ? kSwzRx1 : kSwzId;
  } else if constexpr (sizeof(T) == 4) {
    return P < 256 ? kSwzR5 : P == 256 ? kSwzR9 : P == 512 ? kSwzRx1 : kSwzRx2;
  } else {
    return P < 256 ? kSwzR5 : P == 256 ? kSwzR : P == 512 ? kSwzRh1 : kSwzId;
  }
}
// layout written by pass 2 of a four-pass plan (radix 4 after 16 points)
template <typename T, int P>
constexpr int swz_pass2() { return sizeof(T) == 4 ? kSwzR9 : kSwzR; }

// Sources of a pass's inputs.  fetch(i) issues the LDS loads of input i
// (returning raw values), make(raw) forms the input from them; a pass issues
// every fetch before the first make, so its loads share one LDS round trip.
// Later passes read the previous pass's output through its layout map.
template <typename T, int CODE>
struct ReadLayout {
  const cx<T>* buf;
  using Raw = cx<T>;
  __device__ __forceinline__ Raw fetch(int i) const { return buf[swz<T, CODE>(i)]; }
  __device__ __forceinline__ cx<T> make(const Raw& r) const { return r; }
};

// Twiddles of one Stockham pass, exp(-2 pi i q k/(NS R)), q = 1..R-1, for the
// butterflies of this lane (k = b mod NS), from the pass's contiguous table
// at tw + TWO.  PRE: loaded into registers by the previous pass, with its
// inputs (load), so that they share that pass's LDS round trip; otherwise
// each pass loads its own with its inputs (get).
template <typename T, int P, int R, int NS, int G, int TWO, bool PRE>
struct PassTw {
  static constexpr int NB = P / R;
  static constexpr int BPL = (NB + G - 1) / G;
  cx<T> w[PRE ? BPL : 1][R > 1 ? R - 1 : 1];
  static __device__ __forceinline__ int butterfly(int lig, int i) { return NB < G ? (lig & (NB - 1)) : lig + G * i; }
  __device__ __forceinline__ void load(const cx<T>* tw, int lig) {
    if constexpr (PRE) {
#pragma unroll
      for (int i = 0; i < BPL; ++i) {
        const int k = butterfly(lig, i) & (NS - 1);
#pragma unroll
        for (int q = 1; q < R; ++q) w[i][q - 1] = tw[TWO + (q - 1) * NS + k];
      }
    }
  }
  __device__ __forceinline__ cx<T> get(const cx<T>* tw, int i, int q, int k) const {
    if constexpr (PRE) return w[i][q - 1];
    else return tw[TWO + (q - 1) * NS + k];
  }
};

// No twiddles (the first pass, and the pass after the last).
template <typename T>
struct NoTw {
  __device__ __forceinline__ void load(const cx<T>*, int) {}
  __device__ __forceinline__ cx<T> get(const cx<T>*, int, int, int) const { return cx<T>{T(1), T(0)}; }
};

// Twiddles go to registers one pass ahead where they cost few of them
// (FP32, P <= 128: at most 7 complex values per lane).
template <typename T, int P>
constexpr bool tw_in_registers() {
  return sizeof(T) == 4 && P <= 128;
}

// Pieces of one Stockham pass of radix R after NS points have been combined,
// by the G lanes of one signal group: butterfly b reads positions b + q P/R,
// twiddles by exp(DIR 2 pi i q k/(NS R)) (k = b mod NS), and writes
// (b - k) R + k + q NS.  Lane lig takes butterflies lig, lig + G, ...; when
// the pass has fewer butterflies than lanes (P/R < G), lanes lig and
// lig + P/R repeat the same butterfly and store the same values to the same
// places.
template <int P, int R, int G>
__device__ __forceinline__ int pass_butterfly(int lig, int i) {
  constexpr int NB = P / R;
  return NB < G ? (lig & (NB - 1)) : lig + G * i;
}
// Butterfly of lane lig and slot i in the pass after wave_pass_first_pair
// (NS points combined before it): butterfly b = h NS + k with h = lig mod 16
// and k = 4 i + lig / 16.
template <int NS>
__device__ __forceinline__ int rotated_butterfly(int lig, int i) {
  return (lig & 15) * NS + 4 * i + (lig >> 4);
}
template <int P, int R, int NS, int G, bool ROT>
__device__ __forceinline__ int butterfly_of(int lig, int i) {
  if constexpr (ROT) return rotated_butterfly<NS>(lig, i);
  else return pass_butterfly<P, R, G>(lig, i);
}

// Loads of a pass's inputs from `src`.  BATCH: every load is issued before the
// first input is formed (for small passes; large ones leave the order to the
// compiler, which keeps fewer values live).
template <typename T, int P, int R, int G, bool BATCH, typename Src>
__device__ __forceinline__ void pass_load(cx<T> (&x)[(P / R + G - 1) / G][R], int lig, const Src& src) {
  constexpr int NB = P / R;
  constexpr int BPL = (NB + G - 1) / G;
  static_assert(NB % G == 0 || BPL == 1, "butterflies per lane");
  if constexpr (BATCH) {
    typename Src::Raw raw[BPL][R];
#pragma unroll
    for (int i = 0; i < BPL; ++i)
#pragma unroll
      for (int q = 0; q < R; ++q) raw[i][q] = src.fetch(pass_butterfly<P, R, G>(lig, i) + q * NB);
#pragma unroll
    for (int i = 0; i < BPL; ++i)
#pragma unroll
      for (int q = 0; q < R; ++q) x[i][q] = src.make(raw[i][q]);
  } else {
#pragma unroll
    for (int i = 0; i < BPL; ++i)
#pragma unroll
      for (int q = 0; q < R; ++q) x[i][q] = src.make(src.fetch(pass_butterfly<P, R, G>(lig, i) + q * NB));
  }
}

// Twiddles and register DFTs of a pass whose inputs are in x; `next` loads the
// following pass's register twiddles between the twiddle reads and the
// arithmetic, so that they share this pass's LDS round trip.
template <typename T, int P, int R, int NS, int DIR, int G, bool ROT = false, typename W, typename WN>
__device__ __forceinline__ void pass_compute(cx<T> (&x)[(P / R + G - 1) / G][R], const cx<T>* tw, const W& w, WN& next,
                                             int lig) {
  constexpr int BPL = (P / R + G - 1) / G;
  cx<T> wt[BPL][R > 1 ? R - 1 : 1];
#pragma unroll
  for (int i = 0; i < BPL; ++i) {
    if constexpr (NS > 1) {
      const int b = butterfly_of<P, R, NS, G, ROT>(lig, i);
#pragma unroll
      for (int q = 1; q < R; ++q) wt[i][q - 1] = w.get(tw, i, q, b & (NS - 1));
    }
  }
  next.load(tw, lig);
#pragma unroll
  for (int i = 0; i < BPL; ++i) {
    if constexpr (NS > 1) {
#pragma unroll
      for (int q = 1; q < R; ++q) x[i][q] = x[i][q] * (DIR > 0 ? conj(wt[i][q - 1]) : wt[i][q - 1]);
    }
    dft_reg<T, R, DIR>(x[i]);
  }
}

// Stores of a pass's outputs through the layout map SWO, ordered after every
// lane's loads of the pass (the buffer is updated in place) and before the
// next pass's loads.  The pass has no branch: a branch around the LDS accesses
// would make the compiler wait for the previous pass's stores before the next
// loads, which the in-order LDS queue of a wavefront does not need.
template <typename T, int P, int R, int NS, int G, int SWO, bool ROT = false>
__device__ __forceinline__ void pass_store(cx<T>* buf, const cx<T> (&x)[(P / R + G - 1) / G][R], int lig) {
  constexpr int BPL = (P / R + G - 1) / G;
  wave_sync();
#pragma unroll
  for (int i = 0; i < BPL; ++i) {
    const int b = butterfly_of<P, R, NS, G, ROT>(lig, i);
    const int k = b & (NS - 1);
    const int d = (b - k) * R + k;
#pragma unroll
    for (int q = 0; q < R; ++q) buf[swz<T, SWO>(d + q * NS)] = x[i][q];
  }
  wave_sync();
}

// One in-place Stockham pass through LDS.
template <typename T, int P, int R, int NS, int DIR, int G, int SWO, bool BATCH, typename Src, typename W,
          typename WN>
__device__ __forceinline__ void wave_pass(cx<T>* buf, const cx<T>* tw, const W& w, WN& next, int lig,
                                          const Src& src) {
  cx<T> x[(P / R + G - 1) / G][R];
  pass_load<T, P, R, G, BATCH>(x, lig, src);
  pass_compute<T, P, R, NS, DIR, G>(x, tw, w, next, lig);
  pass_store<T, P, R, NS, G, SWO>(buf, x, lig);
}

// Exchange of 16-lane rows between two registers (v_permlane16_swap, M = 16,
// or v_permlane32_swap, M = 32).  In a lane l with bit M clear, a keeps its
// value and b takes a of lane l + M; in a lane with bit M set, a takes b of
// lane l - M and b keeps its value.  Applied to the pair of registers that
// differ in one bit of the element index, this exchanges that register bit
// with lane bit log2 M.  Pure VALU: no LDS access.
template <int M>
__device__ __forceinline__ void row_swap_u32(unsigned& a, unsigned& b) {
  static_assert(M == 16 || M == 32, "row swaps move lane bit 4 or 5");
  if constexpr (M == 16) {
    const auto r = __builtin_amdgcn_permlane16_swap(a, b, false, false);
    a = r[0];
    b = r[1];
  } else {
    const auto r = __builtin_amdgcn_permlane32_swap(a, b, false, false);
    a = r[0];
    b = r[1];
  }
}
template <int M>
__device__ __forceinline__ void row_swap(float& a, float& b) {
  unsigned ua = __float_as_uint(a), ub = __float_as_uint(b);
  row_swap_u32<M>(ua, ub);
  a = __uint_as_float(ua);
  b = __uint_as_float(ub);
}
template <int M>
__device__ __forceinline__ void row_swap(double& a, double& b) {
  const unsigned long long ua = __double_as_longlong(a), ub = __double_as_longlong(b);
  unsigned alo = unsigned(ua), ahi = unsigned(ua >> 32), blo = unsigned(ub), bhi = unsigned(ub >> 32);
  row_swap_u32<M>(alo, blo);
  row_swap_u32<M>(ahi, bhi);
  a = __longlong_as_double(static_cast<long long>((static_cast<unsigned long long>(ahi) << 32) | alo));
  b = __longlong_as_double(static_cast<long long>((static_cast<unsigned long long>(bhi) << 32) | blo));
}
template <int M, typename T>
__device__ __forceinline__ void row_swap(cx<T>& a, cx<T>& b) {
  row_swap<M>(a.x, b.x);
  row_swap<M>(a.y, b.y);
}

// The last two Stockham passes with the exchange between them in registers.
// Pass A (radix RA after NSA = 16 or 32 points) leaves element
// h NSA RA + q NSA + k of its butterfly b = NSA h + k in register q of the
// lane that ran b: k is lane bits 0-3 (0-4), h lane bits 4-5 (5) and, with
// two butterflies per lane, the slot bit.  The last pass B (radix RB after
// NSA RA points) reads positions b' + q' P/RB; every one of them sits in a
// lane whose bits 4-5 (5) equal bits of q.  Row swaps trade those lane bits
// for register bits, after which lane lig holds exactly the inputs of its
// butterflies lig + G i of pass B, in the order the pass takes them: the same
// values the LDS round trip would have delivered, so the results are
// identical.  Plans with this property:
//   P = 128 (G = 32): A radix 4, B radix 2; lane bit 4 <-> register bit 0;
//   P = 256 (G = 64): A radix 4, B radix 4; lane bits 4, 5 <-> register bits 0, 1;
//   P = 512 (G = 64): A radix 4 after 32 points, 2 butterflies per lane, B
//     radix 4; lane bit 5 <-> register bit 0 of each butterfly;
//   P = 1024 (G = 64): A radix 8 with 2 butterflies per lane, B radix 8;
//     lane bits 4, 5 <-> register bits 0, 1 of each butterfly.
template <int P, int PLAN = 0>
constexpr bool last_pair_in_registers() {
  return PLAN == 0 && (P == 128 || P == 256 || P == 512 || P == 1024);
}

template <typename T, int P, int RA, int NSA, int RB, int NSB, int DIR, int G, bool BATCH, typename Src, typename WA,
          typename WB>
__device__ __forceinline__ void wave_pass_pair(cx<T>* buf, const cx<T>* tw, const WA& wa, WB& wb, int lig,
                                               const Src& src) {
  static_assert((NSA == 16 || (P == 512 && NSA == 32)) && NSB == NSA * RA && NSB * RB == P, "pass pair geometry");
  constexpr int BA = (P / RA + G - 1) / G, BB = (P / RB + G - 1) / G;
  cx<T> x[BA][RA];
  NoTw<T> none;
  pass_load<T, P, RA, G, BATCH>(x, lig, src);
  pass_compute<T, P, RA, NSA, DIR, G>(x, tw, wa, wb, lig);
  cx<T> y[BB][RB];
  if constexpr (P == 128) {
    static_assert(G == 32 && RA == 4 && RB == 2, "plan");
    row_swap<16>(x[0][0], x[0][1]);
    row_swap<16>(x[0][2], x[0][3]);
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int q = 0; q < 2; ++q) y[i][q] = x[0][2 * i + q];
  } else if constexpr (P == 256) {
    static_assert(G == 64 && RA == 4 && RB == 4, "plan");
    row_swap<16>(x[0][0], x[0][1]);
    row_swap<16>(x[0][2], x[0][3]);
    row_swap<32>(x[0][0], x[0][2]);
    row_swap<32>(x[0][1], x[0][3]);
#pragma unroll
    for (int q = 0; q < 4; ++q) y[0][q] = x[0][q];
  } else if constexpr (P == 512) {
    static_assert(G == 64 && RA == 4 && RB == 4, "plan");
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      row_swap<32>(x[i][0], x[i][1]);
      row_swap<32>(x[i][2], x[i][3]);
    }
    // register s of butterfly i now holds q1 = s >> 1 and lane bit 5 = s & 1:
    // input q' = 2 i + (s & 1) of pass-B butterfly s >> 1
#pragma unroll
    for (int ib = 0; ib < 2; ++ib)
#pragma unroll
      for (int q = 0; q < 4; ++q) y[ib][q] = x[q >> 1][2 * ib + (q & 1)];
  } else {
    static_assert(P == 1024 && G == 64 && RA == 8 && RB == 8, "plan");
#pragma unroll
    for (int i = 0; i < 2; ++i) {
#pragma unroll
      for (int q = 0; q < 8; q += 2) row_swap<16>(x[i][q], x[i][q + 1]);
#pragma unroll
      for (int q = 0; q < 8; ++q)
        if ((q & 2) == 0) row_swap<32>(x[i][q], x[i][q + 2]);
    }
    // register s of butterfly i now holds q2 = s >> 2 and lane bits (5, 4) = s & 3:
    // input q' = 4 i + (s & 3) of pass-B butterfly s >> 2
#pragma unroll
    for (int ib = 0; ib < 2; ++ib)
#pragma unroll
      for (int q = 0; q < 8; ++q) y[ib][q] = x[q >> 2][4 * ib + (q & 3)];
  }
  pass_compute<T, P, RB, NSB, DIR, G>(y, tw, wb, none, lig);
  pass_store<T, P, RB, NSB, G, kSwzId>(buf, y, lig);
}

// The first two Stockham passes with the exchange between them in registers
// (P = 256: radices 4, 4; P = 512: radices 8, 4; G = 64).  Pass 0 runs
// butterfly b = lig and leaves element b R0 + q in register q.  Pass 1 (after
// R0 points) reads positions b' + q' P/R1, b' = h NS + k with k = q: its
// inputs q' are the top two bits of b, lane bits 4 and 5.  Row swaps trade
// them for register bits 0 and 1, so that lane lig then holds the inputs of
// pass-1 butterflies h NS + k with h = lig mod 16 and k = 4 i + lig / 16
// (rotated_butterfly), i = register bit 2 at P = 512.  Pass 1 runs those
// butterflies and stores them through layout SW1 for pass 2.  The arithmetic
// is that of the two passes through LDS.
template <int P, int PLAN = 0>
constexpr bool first_pair_in_registers() {
  return PLAN == 0 && (P == 256 || P == 512);
}

template <typename T, int P, int R0, int R1, int DIR, int G, int SW1, bool BATCH, typename Src, typename W1>
__device__ __forceinline__ void wave_pass_first_pair(cx<T>* buf, const cx<T>* tw, const W1& w1, int lig,
                                                     const Src& src) {
  static_assert(G == 64 && P / R0 == G && (R0 == 4 || R0 == 8) && R1 == 4 && R0 * 16 * R1 <= 4 * P,
                "first pair geometry");
  constexpr int B1 = (P / R1 + G - 1) / G;
  cx<T> x[1][R0];
  NoTw<T> none;
  NoTw<T> none2;
  pass_load<T, P, R0, G, BATCH>(x, lig, src);
  pass_compute<T, P, R0, 1, DIR, G>(x, tw, none, none2, lig);
#pragma unroll
  for (int q = 0; q < R0; q += 2) row_swap<16>(x[0][q], x[0][q + 1]);
#pragma unroll
  for (int q = 0; q < R0; ++q)
    if ((q & 2) == 0) row_swap<32>(x[0][q], x[0][q + 2]);
  // register s now holds bit 2 of k (P = 512) and lane bits (5, 4) = s & 3:
  // input q' = s & 3 of slot s >> 2
  cx<T> y[B1][R1];
#pragma unroll
  for (int i = 0; i < B1; ++i)
#pragma unroll
    for (int q = 0; q < R1; ++q) y[i][q] = x[0][4 * i + q];
  pass_compute<T, P, R1, R0, DIR, G, true>(y, tw, w1, none, lig);
  pass_store<T, P, R1, R0, G, SW1, true>(buf, y, lig);
}

// Unnormalised complex FFT of length P by one lane group, result in `buf`
// (natural order); the first pass reads its inputs from `src`.
template <typename T, int P, int DIR, int PLAN = 0, typename Src>
__device__ __forceinline__ void wave_fft(cx<T>* buf, const cx<T>* tw, int lig, const Src& src) {
  using PL = WavePlan<P, PLAN>;
  constexpr bool PRE = tw_in_registers<T, P>();
  constexpr int S0 = swz_pass0<T, P>();
  constexpr int S1 = PL::n >= 3 ? swz_pass1<T, P, PLAN>() : kSwzId;
  NoTw<T> none;
  PassTw<T, P, PL::r1, PL::r0, PL::G, pass1_tw_offset<P, PLAN>(), PRE> w1;
  if constexpr (first_pair_in_registers<P, PLAN>()) {
    static_assert(PL::n == 4 && !PRE && last_pair_in_registers<P, PLAN>(), "plan");
    constexpr int NS2 = PL::r0 * PL::r1, NS3 = NS2 * PL::r2;
    PassTw<T, P, PL::r2, NS2, PL::G, pass2_tw_offset<P, PLAN>(), PRE> w2;
    PassTw<T, P, PL::r3, NS3, PL::G, pass3_tw_offset<P, PLAN>(), PRE> w3;
    wave_pass_first_pair<T, P, PL::r0, PL::r1, DIR, PL::G, S1, PRE>(buf, tw, w1, lig, src);
    wave_pass_pair<T, P, PL::r2, NS2, PL::r3, NS3, DIR, PL::G, PRE>(buf, tw, w2, w3, lig, ReadLayout<T, S1>{buf});
  } else if constexpr (PL::n == 4) {
    constexpr int S2 = swz_pass2<T, P>();
    constexpr int NS2 = PL::r0 * PL::r1, NS3 = NS2 * PL::r2;
    PassTw<T, P, PL::r2, NS2, PL::G, pass2_tw_offset<P, PLAN>(), PRE> w2;
    PassTw<T, P, PL::r3, NS3, PL::G, pass3_tw_offset<P, PLAN>(), PRE> w3;
    wave_pass<T, P, PL::r0, 1, DIR, PL::G, S0, PRE>(buf, tw, none, w1, lig, src);
    wave_pass<T, P, PL::r1, PL::r0, DIR, PL::G, S1, PRE>(buf, tw, w1, w2, lig, ReadLayout<T, S0>{buf});
    if constexpr (last_pair_in_registers<P, PLAN>()) {
      wave_pass_pair<T, P, PL::r2, NS2, PL::r3, NS3, DIR, PL::G, PRE>(buf, tw, w2, w3, lig, ReadLayout<T, S1>{buf});
    } else {
      wave_pass<T, P, PL::r2, NS2, DIR, PL::G, S2, PRE>(buf, tw, w2, w3, lig, ReadLayout<T, S1>{buf});
      wave_pass<T, P, PL::r3, NS3, DIR, PL::G, kSwzId, PRE>(buf, tw, w3, none, lig, ReadLayout<T, S2>{buf});
    }
  } else if constexpr (PL::n == 3) {
    constexpr int NS2 = PL::r0 * PL::r1;
    PassTw<T, P, PL::r2, NS2, PL::G, pass2_tw_offset<P, PLAN>(), PRE> w2;
    wave_pass<T, P, PL::r0, 1, DIR, PL::G, S0, PRE>(buf, tw, none, w1, lig, src);
    if constexpr (last_pair_in_registers<P, PLAN>()) {
      wave_pass_pair<T, P, PL::r1, PL::r0, PL::r2, NS2, DIR, PL::G, PRE>(buf, tw, w1, w2, lig, ReadLayout<T, S0>{buf});
    } else {
      wave_pass<T, P, PL::r1, PL::r0, DIR, PL::G, S1, PRE>(buf, tw, w1, w2, lig, ReadLayout<T, S0>{buf});
      wave_pass<T, P, PL::r2, NS2, DIR, PL::G, kSwzId, PRE>(buf, tw, w2, none, lig, ReadLayout<T, S1>{buf});
    }
  } else {
    wave_pass<T, P, PL::r0, 1, DIR, PL::G, S0, PRE>(buf, tw, none, w1, lig, src);
    wave_pass<T, P, PL::r1, PL::r0, DIR, PL::G, S1, PRE>(buf, tw, w1, none, lig, ReadLayout<T, S0>{buf});
  }
}

// LDS per state slot: SP [3][P+1] (half spectra in; forward transforms out)
// and IB [3][P] (inverse transforms, in place).
template <typename T, int NX>
struct Slot {
  static constexpr int P = Geo<NX>::P;
  static constexpr size_t sp_elems = 3 * (P + 1);
  static constexpr size_t ib_elems = 3 * P;
  static constexpr size_t bytes = (sp_elems + ib_elems) * sizeof(cx<T>);
};

// First-pass source of an inverse transform: Z[k] = (X[k] + conj X[P-k])
// + i conj(t_k) (X[k] - conj X[P-k]) from the half spectrum X (stride P+1),
// t_k = exp(-2 pi i k/N).  With s and d the sum and difference, the product
// i conj(t) d has parts -(t.x d.y - t.y d.x) and t.x d.x + t.y d.y, added to s
// by fused multiply-adds.
template <typename T, int P>
struct ReadHalfSpectrum {
  const cx<T>* X;
  const cx<T>* tw;
  struct Raw {
    cx<T> xk, xm, t;
  };
  __device__ __forceinline__ Raw fetch(int idx) const { return Raw{X[idx], X[P - idx], tw[idx]}; }
  __device__ __forceinline__ cx<T> make(const Raw& r) const {
    const cx<T> s{r.xk.x + r.xm.x, r.xk.y - r.xm.y};
    const cx<T> d{r.xk.x - r.xm.x, r.xk.y + r.xm.y};
    return cx<T>{fmat(r.t.y, d.x, fmat(-r.t.x, d.y, s.x)), fmat(r.t.y, d.y, fmat(r.t.x, d.x, s.y))};
  }
};

// Inverse transforms of the 3*ns field spectra in SP (entries k <= Kd written,
// entries Kd < k <= P zero: see zero_tails) into IB, one signal per lane group
// at a time.  A lane group past the last signal repeats its wavefront's first
// signal (same inputs, same outputs), so no branch surrounds the transforms.
// The loads of the first pass are unconditional: the signal's offset is
// passed through an empty asm statement, so that the compiler cannot tie the
// loads to the zero stores of zero_tails and split them into conditional
// loads (each with its own wait).
// Runs body(v0) for the first signal v0 of each round of transforms of this
// wavefront over nsig signals (tid: the thread's index in the workgroup, as
// in the engine; the field and product transforms take it too).  When MAXNS states (3 MAXNS signals) fit one
// round of the workgroup's wavefronts, the round is straight-line code, and
// the signal's offsets are the same in every evaluation of a job.
template <int NT, int SPW, int MAXNS, typename B>
__device__ __forceinline__ void signal_rounds(int nsig, unsigned tid, B&& body) {
  constexpr int NW = NT / 64;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  if constexpr (MAXNS > 0 && NW * SPW >= 3 * MAXNS) {
    if (wave * SPW < nsig) body(wave * SPW);
  } else {
    for (int v0 = wave * SPW; v0 < nsig; v0 += NW * SPW) body(v0);
  }
}

template <typename T, int NX, int NT, int MAXNS = 0, int PLAN = 0>
__device__ __forceinline__ void inverse_fields(cx<T>* sp, cx<T>* ib, int ns, const cx<T>* tw, unsigned tid) {
  using G_ = Geo<NX>;
  constexpr int P = G_::P;
  constexpr int G = WavePlan<P>::G;
  constexpr int SPW = 64 / G;             // signals per wavefront
  const int lane = tid & 63;
  const int group = lane / G, lig = lane - group * G;
  const int nsig = 3 * ns;
  signal_rounds<NT, SPW, MAXNS>(nsig, tid, [&](int v0) {
    const int v = v0 + group < nsig ? v0 + group : v0;
    int off = v * (P + 1);
    asm volatile("" : "+v"(off));
    wave_fft<T, P, +1, PLAN>(ib + v * P, tw, lig, ReadHalfSpectrum<T, P>{sp + off, tw});
  });
}

// Zeroes the entries Kd < k <= P of the 3*ns field spectra in SP (the forward
// transforms of the previous evaluation overwrote them).  Called by every
// thread between the writes of the retained modes and the barrier before the
// inverse transforms.
template <typename T, int NX, int NT>
__device__ __forceinline__ void zero_tails(cx<T>* sp, int ns, unsigned tid) {
  constexpr int P = Geo<NX>::P;
  constexpr int KD = Geo<NX>::KD;
  constexpr int TL = P - KD;
  for (int i = tid; i < 3 * ns * TL; i += NT) {
    const int v = i / TL;
    sp[v * (P + 1) + KD + 1 + (i - v * TL)] = czero<T>();
  }
}

// First-pass source of a forward transform: the packed product
// (scale v1.x w.x, scale v1.y w.y) of two inverse outputs.
template <typename T>
struct ReadProducts {
  const cx<T>* V1;
  const cx<T>* W;
  T scale;
  struct Raw {
    cx<T> v1, w;
  };
  __device__ __forceinline__ Raw fetch(int idx) const { return Raw{V1[idx], W[idx]}; }
  __device__ __forceinline__ cx<T> make(const Raw& r) const {
    return cx<T>{scale * (r.v1.x * r.w.x), scale * (r.v1.y * r.w.y)};
  }
};

// Forward transforms of the packed products of each state's inverse outputs,
// written into SP (stride P+1): v1^2/2, v1 v2x, h v1.  The first pass reads
// both factors and scales by 1/2 or 1, with no branch on the product; lane
// groups past the last signal repeat their wavefront's first one.
template <typename T, int NX, int NT, int MAXNS = 0, int PLAN = 0>
__device__ __forceinline__ void forward_products(cx<T>* sp, const cx<T>* ib, int ns, const cx<T>* tw,
                                                 unsigned tid) {
  constexpr int P = Geo<NX>::P;
  constexpr int G = WavePlan<P>::G;
  constexpr int SPW = 64 / G;
  const int lane = tid & 63;
  const int group = lane / G, lig = lane - group * G;
  const int nsig = 3 * ns;
  signal_rounds<NT, SPW, MAXNS>(nsig, tid, [&](int v0) {
    const int vv = v0 + group < nsig ? v0 + group : v0;
    const int s = vv / 3, f = vv - 3 * s;
    const cx<T>* V1 = ib + (3 * s) * P;
    const cx<T>* W = ib + (3 * s + (f == 2 ? 2 : f)) * P;   // v1 itself for the square
    const T scale = f == 0 ? T(0.5) : T(1);
    wave_fft<T, P, -1, PLAN>(sp + vv * (P + 1), tw, lig, ReadProducts<T>{V1, W, scale});
  });
}

// Modal N amplitudes of retained mode k from the forward transforms of one
// slot's products (SP base of the slot, stride P+1).
//   Product spectra: Q_f = (Z[k] + conj Z[P-k]) - i w (Z[k] - conj Z[P-k]),
//   w = exp(-2 pi i k/N), so that the product's mode k is h Q_f, h = 1/(2N).
//   N's fields: n1 = -i k h Q_0, n2 = -h Q_1, n3 = -i k h Q_2.
//   Modal amplitudes (fields_to_modal with those fields, s = 1/sqrt 2):
//     out0 = i (R - s h k Q_0),  out2 = -i (R + s h k Q_0),
//     R = s h (iw Q_1 + aw k Q_2),  out1 = i h (aw Q_1 - iw k Q_2),
//   all as fused multiply-adds with per-mode real factors.
template <typename T, int NX>
__device__ __forceinline__ void get_N_sp(const cx<T>* sp_slot, int k, Basis<T> bs, const cx<T>* tw, cx<T> out[3]) {
  using G = Geo<NX>;
  constexpr int P = G::P;
  const cx<T> w = tw[k];
  const int kc = (P - k) & (P - 1);
  cx<T> Q[3];
#pragma unroll
  for (int f = 0; f < 3; ++f) {
    const cx<T>* Z = sp_slot + f * (P + 1);
    const cx<T> zk = Z[k];
    const cx<T> zm = Z[kc];
    const cx<T> s{zk.x + zm.x, zk.y - zm.y};
    const cx<T> d{zk.x - zm.x, zk.y + zm.y};
    Q[f] = cx<T>{fmat(w.y, d.x, fmat(w.x, d.y, s.x)), fmat(w.y, d.y, fmat(-w.x, d.x, s.y))};
  }
  constexpr T h = T(0.5 / double(G::N));
  constexpr T sh = T(0.70710678118654752440 * (0.5 / double(G::N)));
  const T kk = T(k);
  const T a0 = sh * kk, b1 = sh * bs.iw, c2 = a0 * bs.aw, d1 = h * bs.aw, e2 = (h * kk) * bs.iw;
  const cx<T> R{fmat(c2, Q[2].x, b1 * Q[1].x), fmat(c2, Q[2].y, b1 * Q[1].y)};
  // i z = (-z.y, z.x)
  out[0] = cx<T>{fmat(a0, Q[0].y, -R.y), fmat(-a0, Q[0].x, R.x)};
  out[2] = cx<T>{fmat(a0, Q[0].y, R.y), fmat(-a0, Q[0].x, -R.x)};
  out[1] = cx<T>{fmat(e2, Q[2].y, -(d1 * Q[1].y)), fmat(-e2, Q[2].x, d1 * Q[1].x)};
}

}  // namespace ap
