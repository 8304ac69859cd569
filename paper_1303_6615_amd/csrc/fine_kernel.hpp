// The fine batch (the parallel fine sweep of Alg. 4 over independent
// states): one ETDRK4 job (fine_job) per workgroup over the slices its
// threads own modes of.
//
// Workgroup shapes.  Workgroups are small enough that several share a CU
// (VGPRs and LDS permitting); each steps as many slices as its threads own
// modes and its wavefronts transform in one round (Engine::jmax), with two
// slots per slice.  Three shapes per precision and grid size are compiled;
// shape 0 is the default, measured best on MI355X over large batches (FP32:
// 128 / 192 / 192 / 192 / 384 / 704 threads for N = 64 .. 2048; FP64:
// 256 / 256 / 512 / 256 / 384 / 704).  A slice rounds the same way in every
// shape (its transforms and mode arithmetic do not depend on the workgroup),
// so the shape is a performance choice only.  For N >= 256 each shape is
// also compiled with FFT plan 1 (wavefft.hpp: the classic Stockham passes
// through LDS; at N = 1024 other radices, which round differently).  A
// configuration c of the fine batch is shape c mod 3 with plan c / 3;
// aparareal_autotune_fine measures every compiled configuration on the
// caller's batch.
#pragma once
#include "dispatch.hpp"
#include "engine.hpp"

namespace ap {

constexpr int kFineShapes = 3;
constexpr int kFineConfigs = 2 * kFineShapes;   // shapes x FFT plans

template <typename T, int NX, int SHAPE>
constexpr int fine_shape_threads() {
  constexpr int i = NX == 64 ? 0 : NX == 128 ? 1 : NX == 256 ? 2 : NX == 512 ? 3 : NX == 1024 ? 4 : 5;
  constexpr int f32[6][kFineShapes] = {{128, 64, 192},  {192, 256, 128}, {192, 256, 128},
                                       {192, 256, 384}, {384, 512, 448}, {704, 768, 640}};
  constexpr int f64[6][kFineShapes] = {{256, 128, 192}, {256, 192, 384}, {512, 256, 384},
                                       {256, 384, 192}, {384, 512, 448}, {704, 768, 640}};
  return sizeof(T) == 4 ? f32[i][SHAPE] : f64[i][SHAPE];
}

// Threads of the default shape (also the shape of the other batched kernels
// built on the engine: nonlinear term, Strang steps).
template <typename T, int NX>
constexpr int fine_threads() {
  return fine_shape_threads<T, NX, 0>();
}

template <typename T, int NX, int NT, int PLAN = 0>
constexpr int fine_slots() {
  constexpr int KP = Geo<NX>::KP;
  constexpr int MPT = (KP + NT - 1) / NT;
  int j = MPT > 1 ? 1 : NT / KP;
  const int by_waves = (NT / 64) * (64 / WavePlan<NX / 2, PLAN>::G) / 3;
  j = j < by_waves ? j : by_waves;
  j = j < 16 ? (j > 0 ? j : 1) : 16;
  const int s = max_slots<T, NX, NT, PLAN>();
  return 2 * j < s ? 2 * j : s;
}
template <typename T, int NX, int NT, int PLAN = 0>
constexpr int fine_slices_nt() {
  return Engine<T, NX, NT, fine_slots<T, NX, NT, PLAN>(), PLAN>::jmax();
}
template <typename T, int NX>
constexpr int fine_slices() {
  return fine_slices_nt<T, NX, fine_threads<T, NX>()>();
}

// Workgroup b steps slices b J .. min(b J + J, batch) - 1 (J = the shape's
// slices per workgroup).  FP32 kernels keep three wavefronts per SIMD (at
// most 168 VGPRs; the second bound is the minimum of wavefronts per SIMD),
// the occupancy their workgroups are sized for.
template <typename T, int NX, int NT, int PLAN>
__global__ void __launch_bounds__(NT, sizeof(T) == 4 ? 3 : 1) k_fine(const cx<double>* __restrict__ Uin, cx<double>* __restrict__ Uout,
                                             int batch, int steps, const cx<double>* __restrict__ coef64,
                                             const cx<T>* __restrict__ coef, const cx<T>* __restrict__ tw,
                                             const Basis<T>* __restrict__ basis) {
  constexpr int S = fine_slots<T, NX, NT, PLAN>();
  using E_ = Engine<T, NX, NT, S, PLAN>;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  E_ en(smem_raw, tw);
  const size_t st = size_t(3) * E_::KP;
  const int first = blockIdx.x * E_::jmax();
  const int J = min(E_::jmax(), batch - first);
  fine_job<T, NX, NT, S>(en, J, Uin + first * st, Uin + (first + 1) * st, Uout + first * st, steps, coef64, coef,
                         basis);
}

// tw: the twiddle table of FFT plan PLAN
template <typename T, int NX, int NT, int PLAN>
inline hipError_t fine_launch_nt(const cx<double>* in, cx<double>* out, int batch, int steps,
                                 const cx<double>* coef64, const cx<T>* coef, const cx<T>* tw, const Basis<T>* basis,
                                 hipStream_t s) {
  const size_t lds = Engine<T, NX, NT, fine_slots<T, NX, NT, PLAN>(), PLAN>::lds_bytes();
  constexpr int J = fine_slices_nt<T, NX, NT, PLAN>();
  prep_lds(k_fine<T, NX, NT, PLAN>, lds);
  hipLaunchKernelGGL((k_fine<T, NX, NT, PLAN>), dim3((batch + J - 1) / J), dim3(NT), lds, s, in, out, batch, steps,
                     coef64, coef, tw, basis);
  return hipGetLastError();
}

// FFT plans compiled for the fine batch at grid size NX
template <int NX>
constexpr int fine_plans() {
  return wave_plans(NX / 2);
}

template <typename T, int NX, int PLAN>
inline hipError_t fine_launch_plan(int shape, const cx<double>* in, cx<double>* out, int batch, int steps,
                                   const cx<double>* coef64, const cx<T>* coef, const cx<T>* tw,
                                   const Basis<T>* basis, hipStream_t s) {
  switch (shape) {
    case 0: return fine_launch_nt<T, NX, fine_shape_threads<T, NX, 0>(), PLAN>(in, out, batch, steps, coef64, coef, tw, basis, s);
    case 1: return fine_launch_nt<T, NX, fine_shape_threads<T, NX, 1>(), PLAN>(in, out, batch, steps, coef64, coef, tw, basis, s);
    case 2: return fine_launch_nt<T, NX, fine_shape_threads<T, NX, 2>(), PLAN>(in, out, batch, steps, coef64, coef, tw, basis, s);
    default: return hipErrorInvalidValue;
  }
}

// Configuration `config` (shape config % 3, FFT plan config / 3); `t`: the
// context's tables (each plan has its own twiddle table).
template <typename T, int NX>
inline hipError_t fine_launch_config(int config, const cx<double>* in, cx<double>* out, int batch, int steps,
                                     const cx<double>* coef64, const cx<T>* coef, const DevTables& t,
                                     hipStream_t s) {
  if (config < 0 || config >= kFineConfigs) return hipErrorInvalidValue;
  const int shape = config % kFineShapes, plan = config / kFineShapes;
  if (plan == 0)
    return fine_launch_plan<T, NX, 0>(shape, in, out, batch, steps, coef64, coef, t.tw_plan<T>(0), t.basis<T>(), s);
  if constexpr (fine_plans<NX>() > 1)
    return fine_launch_plan<T, NX, 1>(shape, in, out, batch, steps, coef64, coef, t.tw_plan<T>(1), t.basis<T>(), s);
  return hipErrorInvalidValue;
}

// Threads per workgroup of configuration `config` (0 if it is not compiled
// at this grid size); *slices: slices per workgroup.
template <typename T, int NX>
inline int fine_shape_info(int config, int* slices) {
  if (config < 0 || config >= kFineConfigs || config / kFineShapes >= fine_plans<NX>()) return 0;
  int nt = 0, j = 0;
  switch (config % kFineShapes) {
    case 0: nt = fine_shape_threads<T, NX, 0>(); j = fine_slices_nt<T, NX, fine_shape_threads<T, NX, 0>()>(); break;
    case 1: nt = fine_shape_threads<T, NX, 1>(); j = fine_slices_nt<T, NX, fine_shape_threads<T, NX, 1>()>(); break;
    default: nt = fine_shape_threads<T, NX, 2>(); j = fine_slices_nt<T, NX, fine_shape_threads<T, NX, 2>()>(); break;
  }
  if (slices) *slices = j;
  return nt;
}

}  // namespace ap
