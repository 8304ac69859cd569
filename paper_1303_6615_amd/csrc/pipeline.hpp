// The pipelined persistent parareal solve: device scheduler and jobs, and the
// host helpers that launch it.  Instantiated per precision and set of grid
// sizes in the pipe_*.hip translation units.
#pragma once
#include "dispatch.hpp"
#include "engine.hpp"

namespace ap {

// ---------------------------------------------------- pipelined solve -----
// Per problem (the descriptor PipeProb, counter layout in launch.hpp):
//   U [K+1][Ns+1], F [K][Ns+1], G [K+1][Ns+1] modal FP64 states (U(k,0) is
//   read from U(0,0) = u0 for every k), part [K][Ns].
// C(k,n): G(U(k,n-1)) -> G(k,n); U(k,n) = G (k = 0) or F(k-1,n) + (G - G(k-1,n)),
//         needs C(k,n-1), F(k-1,n), C(k-1,n).
// F(k,n): Fine(U(k,n-1)) -> F(k,n), needs C(k,n-1).
// Split C(k,n): stage-1 job of group g needs C(k,n-1); the stage-1 job that
//         finishes last forms the step's midpoint state and publishes the
//         stage-1 counter once more (groups + 1); stage-2 job of group g needs
//         C(k,n-1) to start and that count before it reads the midpoint; the
//         stage-2 job that finishes last also needs F(k-1,n) and C(k-1,n) and
//         publishes C(k,n).
// Stall record `diag` of a launch: [0] stalled, [1] job, [2] counter index,
// [3] jobs completed so far (every workgroup adds 1 per job it publishes).
// A wait ends in a stall only when no job of the launch completes for
// kStallTicks of the constant-rate device clock (100 MHz: 1 s) while it
// waits: the scheduler's order guarantees progress, so this only fires on a
// defect, and it ends the launch instead of hanging the device.  A long wait
// while other jobs keep completing is ordinary (large batches hand out jobs
// long before their inputs exist).
constexpr unsigned long long kStallTicks = 100000000ull;

// Agent-scope acquire by thread 0 on behalf of its workgroup: the cache
// invalidation it issues must complete before the barrier after which the
// other wavefronts read the producers' data (the fence alone orders only this
// wavefront's later loads).
__device__ __forceinline__ void acquire_for_workgroup() {
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
}

// Agent-scope release by thread 0 on behalf of its workgroup, before the
// relaxed atomic that publishes: every wavefront has waited for its own
// stores to reach the L2 before the barrier that precedes this.  The fence
// writes this XCD's L2 back (buffer_wbl2); the explicit wait then holds the
// publishing atomic until that write-back has completed.  The compiler's own
// wait after the write-back is a soft one that its wait-count pass deletes
// when it sees no loads or stores in flight (it does not count the
// write-back): the atomic then reaches the other XCDs before the data, and a
// consumer that is already polling reads the state from before the write.
__device__ __forceinline__ void release_for_workgroup() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
}

// Thread 0 waits for *ctr >= target (relaxed polls, then an agent-scope
// acquire for the workgroup: the producers are on this device).
// On a stall it records (1, job, counter index) in diag[0..2] and returns
// false; it also returns false once another workgroup has recorded one.
// Every waiting workgroup polls, so the words all of them share (the stall
// record and the completed-job count) are read only every kCheckEvery polls:
// reading them on every poll makes those few addresses the hottest in the
// device and slows the polls of the counter a workgroup actually waits on.
constexpr int kStallPolls = 1 << 22;   // polls without progress: a bound independent of the clock
constexpr int kCheckEvery = 32;

__device__ __forceinline__ bool wait_count(int* ctr, int target, int* diag, int job, int index) {
  unsigned long long t0 = wall_clock64();
  int seen = __hip_atomic_load(diag + 3, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  int polls = 0;
  while (__hip_atomic_load(ctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
    if (++polls % kCheckEvery == 0) {
      if (__hip_atomic_load(diag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) return false;
      const int now_done = __hip_atomic_load(diag + 3, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (now_done != seen) {
        seen = now_done;
        t0 = wall_clock64();
        polls = 0;
      } else if (wall_clock64() - t0 > kStallTicks || polls > kStallPolls) {
        if (__hip_atomic_fetch_add(diag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0) {
          __hip_atomic_store(diag + 1, job, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          __hip_atomic_store(diag + 2, index, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        return false;
      }
    }
    __builtin_amdgcn_s_sleep(2);
  }
  acquire_for_workgroup();
  return true;
}

// This wavefront's global stores have completed at the L2 (vector memory
// counter at zero); the memory clobber keeps the compiler from moving stores
// past it.
__device__ __forceinline__ void wait_global_stores() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }

// Counter indices of one problem (layout in launch.hpp; consecutive slices'
// counters are kCounterStride apart).
struct PipeIdx {
  int Ns, K;
  __device__ int coarse(int k, int n) const { return (k * Ns + n - 1) * kCounterStride; }
  __device__ int fine(int k, int n) const { return ((K + 1) * Ns + k * Ns + n - 1) * kCounterStride; }
  __device__ int stage1(int k, int n) const { return ((2 * K + 1) * Ns + k * Ns + n - 1) * kCounterStride; }
  __device__ int stage2(int k, int n) const { return ((3 * K + 2) * Ns + k * Ns + n - 1) * kCounterStride; }
  __device__ int stopped() const { return (4 * K + 3) * Ns * kCounterStride; }
};

// The job's level lies past the level at which its problem stopped (the
// residual reached the tolerance): it publishes its counters without work.
template <typename T>
__device__ __forceinline__ bool past_stop(const PipeJob& jb, const PipeProb<T>& p) {
  if (!(p.tol > 0.0) || jb.k == 0) return false;
  const int st = __hip_atomic_load(&p.cnt[PipeIdx{p.Ns, p.K}.stopped()], __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
  return st > 0 && jb.k > st;
}

// With a tolerance, the job that completes C(k, Ns) reads every residual part
// of level k (level_residual).  The copy jobs of the exact slices m <= k are
// not on the coarse chain that leads to C(k, Ns), so that job also waits for
// their counters (thread 0).
template <typename T>
__device__ __forceinline__ bool wait_level_copies(const PipeProb<T>& p, const PipeIdx& ix, int k, int* diag,
                                                  int jt) {
  if (!(p.tol > 0.0) || k < 1) return true;
  const int last = min(k, p.Ns - 1);
  for (int m = 1; m <= last; ++m)
    if (!wait_count(&p.cnt[ix.coarse(k, m)], 1, diag, jt, ix.coarse(k, m))) return false;
  return true;
}

// Dependencies a job waits for before it starts (thread 0).
template <typename T>
__device__ __forceinline__ bool wait_deps(const PipeJob& jb, const PipeProb<T>& p, int* diag, int jt) {
  const PipeIdx ix{p.Ns, p.K};
  const int k = jb.k, n = jb.n;
  // a stage-2 job starts on U(k, n-1) and waits for the midpoint inside (run_job)
  if (jb.type == kJobStage2) return n == 1 || wait_count(&p.cnt[ix.coarse(k, n - 1)], 1, diag, jt, ix.coarse(k, n - 1));
  if (jb.type == kJobCopy) {
    if (n == k && !wait_count(&p.cnt[ix.fine(k - 1, n)], 1, diag, jt, ix.fine(k - 1, n))) return false;
    if (!wait_count(&p.cnt[ix.coarse(k - 1, n)], 1, diag, jt, ix.coarse(k - 1, n))) return false;
    return n == p.Ns ? wait_level_copies(p, ix, k, diag, jt) : true;
  }
  // a fine job over slices n .. n + g - 1 (g >= 2) needs their inputs U(k, n - 1 .. n + g - 2): the
  // coarse chain publishes in order, so the last one suffices
  const int last = jb.type == kJobFine && jb.g > 1 ? n + jb.g - 2 : n - 1;
  if (last >= 1 && !wait_count(&p.cnt[ix.coarse(k, last)], 1, diag, jt, ix.coarse(k, last))) return false;
  if (jb.type == kJobCoarse && k >= 1) {
    if (!wait_count(&p.cnt[ix.fine(k - 1, n)], 1, diag, jt, ix.fine(k - 1, n))) return false;
    if (!wait_count(&p.cnt[ix.coarse(k - 1, n)], 1, diag, jt, ix.coarse(k - 1, n))) return false;
    if (n == p.Ns && !wait_level_copies(p, ix, k, diag, jt)) return false;
  }
  return true;
}

// Threads per pipeline workgroup: eight wavefronts with up to 256 VGPRs each
// (a job keeps the ETDRK4 state, coefficients and a register DFT live at once).
constexpr int kPipeThreads = 512;
template <typename T, int NX>
constexpr int pipe_slots() {
  return max_slots<T, NX, kPipeThreads>();
}
template <typename T, int NX>
constexpr size_t pipe_lds() {
  return Engine<T, NX, kPipeThreads, pipe_slots<T, NX>()>::lds_bytes();
}
// (slice, mode) items per thread in the pipeline's ETDRK4 fine jobs: two, so
// that a job at N = 1024 (342 modes per slice, 512 threads) steps two slices,
// six transforms per round instead of three; the Strang fine job keeps one.
constexpr int kPipeFineItems = 2;
template <typename T, int NX>
using PipeFineEngine = Engine<T, NX, kPipeThreads, pipe_slots<T, NX>(), 0, kPipeFineItems>;
// Most slices per fine job of the pipeline: ETDRK4 (kind 0) or Strang (kind 1).
template <typename T, int NX>
constexpr int pipe_fine_slices(int kind) {
  return kind == 1 ? Engine<T, NX, kPipeThreads, pipe_slots<T, NX>()>::jmax() : PipeFineEngine<T, NX>::jmax();
}

// Counts a group job of a split step in on counter *ctr (groups jobs count
// in): every wavefront first waits for its stores to reach the L2 (a
// workgroup barrier waits only for LDS), thread 0's release writes them back
// for the other XCDs, then adds 1.  Returns true in the job that arrives
// last, after an acquire that makes every other group's stores visible.
__device__ __forceinline__ bool count_in_last(int* ctr, int groups, int* s_flag) {
  wait_global_stores();
  __syncthreads();
  if (threadIdx.x == 0) {
    release_for_workgroup();
    const int before = __hip_atomic_fetch_add(ctr, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const int last = before == groups - 1;
    if (last) acquire_for_workgroup();
    *s_flag = last;
  }
  __syncthreads();
  return __builtin_amdgcn_readfirstlane(*s_flag) != 0;
}

// The fine slices of a job as an out-of-line call, Strang (KIND 1) or ETDRK4
// (KIND 0): one call per job, and the stepping loop gets a register
// allocation of its own instead of sharing one with every other job type.
// The caller has staged the twiddles.  A kernel for several grid sizes runs
// its ETDRK4 fine jobs inline instead (run_fine_job).
template <typename T, int NX, int JM, int KIND>
__device__ __attribute__((noinline)) void fine_slices_job(unsigned char* smem, const cx<T>* tw, int J,
                                                          const cx<double>* src0, const cx<double>* src1,
                                                          cx<double>* dst, int steps, const cx<double>* coef64,
                                                          const cx<T>* coef, double hf, const Basis<T>* basis) {
  if constexpr (KIND == 1) {
    Engine<T, NX, kPipeThreads, pipe_slots<T, NX>()> en(smem, tw, false);
    strang_job<T, NX, kPipeThreads, pipe_slots<T, NX>(), JM>(en, J, src0, src1, dst, steps, coef64, hf, basis);
  } else {
    PipeFineEngine<T, NX> en(smem, tw, false);
    fine_job<T, NX, kPipeThreads, pipe_slots<T, NX>(), JM>(en, J, src0, src1, dst, steps, coef64, coef, basis);
  }
}

// State of slice `slice` at level lvl in a problem's U, F or G array (Ns + 1
// slices per level, 3 KP coefficients per slice).
__device__ __forceinline__ cx<double>* pipe_state(cx<double>* A, int Ns, size_t st, int lvl, int slice) {
  return A + (size_t(lvl) * (Ns + 1) + slice) * st;
}

// Whether a pipeline kernel runs the ETDRK4 fine jobs of grid size NX inline
// (run_fine_job) rather than as calls (MULTI: the kernel serves several
// sizes; its other jobs are calls).  FP32 only, and up to N = 1024 (several
// sizes) or N = 256 (one size, whose other jobs are inlined too): there the
// inlined job needs little or no scratch.  Larger sizes, FP64, and N = 1024
// beside an inlined coarse path spilled inside the stepping loop, and the
// N = 1024 solve ran slower than with the called job.
template <typename T, int NX, bool MULTI>
constexpr bool pipe_inline_fine() {
  return sizeof(T) == 4 && NX <= (MULTI ? 1024 : 256);
}

// An ETDRK4 fine job (slices n .. n + J - 1 of level k) of grid size NX,
// inlined into the pipeline kernel rather than called.  The stepping loop
// keeps up to 256 VGPRs live; in a called function the calling convention
// makes it save and restore every callee-saved one of them around each job,
// some 200 KiB of scratch traffic each way per job at 512 threads.  A kernel
// saves none.  The engine's thread index is salted with the job number jt, so
// that the job's per-thread values stay inside the job.  Returns the first
// fine counter to publish; npub = J.
template <typename T, int NX>
__device__ __forceinline__ int run_fine_job(unsigned char* smem, const PipeJob& jb, const PipeProb<T>& p,
                                            const void*& staged, int jt, int& npub) {
  using FE = PipeFineEngine<T, NX>;
  constexpr int S = pipe_slots<T, NX>();
  const PipeIdx ix{p.Ns, p.K};
  const int Ns = p.Ns, k = jb.k, n = jb.n;
  const int J = jb.g > 1 ? min(jb.g, pipe_fine_slices<T, NX>(0)) : 1;
  npub = J;
  FE en(smem, p.tw, staged != static_cast<const void*>(p.tw), jt);
  staged = FE::TW_LDS ? static_cast<const void*>(p.tw) : nullptr;
  const size_t st = size_t(3) * FE::KP;
  // slice n reads U(k, n - 1) (U(0, 0) for n = 1), slices n + s read U(k, n + s - 1)
  const cx<double>* src0 = n == 1 ? p.U : pipe_state(p.U, Ns, st, k, n - 1);
  const cx<double>* src1 = pipe_state(p.U, Ns, st, k, n);
  cx<double>* dst = pipe_state(p.F, Ns, st, k, n);
  if (J == 1)
    fine_job<T, NX, kPipeThreads, S, 1>(en, 1, src0, src1, dst, p.steps, p.coef64, p.coef, p.basis);
  else
    fine_job<T, NX, kPipeThreads, S, 0>(en, J, src0, src1, dst, p.steps, p.coef64, p.coef, p.basis);
  return ix.fine(k, n);
}

// Runs an ETDRK4 fine job of grid size nx inline when the kernel does so for
// that size; returns its first counter, or kNotRun.
constexpr int kNotRun = -2;
template <typename T, bool MULTI, int NX, int... REST>
__device__ __forceinline__ int dispatch_fine(int nx, unsigned char* smem, const PipeJob& jb, const PipeProb<T>& p,
                                             const void*& staged, int jt, int& npub) {
  if constexpr (pipe_inline_fine<T, NX, MULTI>())
    if (nx == NX) return run_fine_job<T, NX>(smem, jb, p, staged, jt, npub);
  if constexpr (sizeof...(REST) > 0)
    return dispatch_fine<T, MULTI, REST...>(nx, smem, jb, p, staged, jt, npub);
  else
    return kNotRun;
}

// Runs job jb of problem p (grid size NX) in this workgroup.  Returns the
// counter index to publish when the job's results are complete, or -1.
// `staged` tracks the twiddle table held in LDS across jobs.  KFINE: the
// kernel runs the ETDRK4 fine jobs of this size itself (run_fine_job), so jb
// is never one.
template <typename T, int NX, bool KFINE>
__device__ __forceinline__ int run_job(unsigned char* smem, const PipeJob& jb, const PipeProb<T>& p,
                                       const void*& staged, int* diag, int jt, int* s_flag, bool skip, int& npub) {
  constexpr int NT = kPipeThreads;
  constexpr int S = pipe_slots<T, NX>();
  using E_ = Engine<T, NX, NT, S>;
  constexpr int MPT = E_::MPT;
  const PipeIdx ix{p.Ns, p.K};
  const int Ns = p.Ns, k = jb.k, n = jb.n;
  // a fine job steps J consecutive slices together and publishes their J counters
  const int J = jb.type == kJobFine && jb.g > 1 ? min(jb.g, pipe_fine_slices<T, NX>(p.fine_kind)) : 1;
  npub = J;
  if (skip) {
    // past the stopped level: publish only (group jobs still count in so
    // that the last one publishes: stage 1 its extra count, stage 2 the step)
    if (jb.type == kJobFine) return ix.fine(k, n);
    if (jb.type != kJobStage1 && jb.type != kJobStage2) return ix.coarse(k, n);
    const int c = jb.type == kJobStage1 ? ix.stage1(k, n) : ix.stage2(k, n);
    if (threadIdx.x == 0) {
      const int before = __hip_atomic_fetch_add(&p.cnt[c], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      *s_flag = before == p.groups - 1;
    }
    __syncthreads();
    if (!__builtin_amdgcn_readfirstlane(*s_flag)) return -1;
    return jb.type == kJobStage1 ? ix.stage1(k, n) : ix.coarse(k, n);
  }
  const bool stage = staged != static_cast<const void*>(p.tw);
  E_ en(smem, p.tw, stage);
  staged = E_::TW_LDS ? static_cast<const void*>(p.tw) : nullptr;
  const size_t st = size_t(3) * E_::KP;
  auto state = [&](cx<double>* A, int lvl, int slice) { return pipe_state(A, Ns, st, lvl, slice); };
  const cx<double>* uprev = n == 1 ? state(p.U, 0, 0) : state(p.U, k, n - 1);
  // Completing C(k, Ns) completes level k: with a tolerance, its residual
  // decides whether the problem stops here (levels complete in order).
  auto level_done = [&]() {
    if (p.tol > 0.0 && k >= 1 && n == Ns) {
      const double r = level_residual<T, NX, NT, S>(en, p.part + size_t(k - 1) * Ns, Ns);
      if (threadIdx.x == 0 && r <= p.tol) {
        int zero = 0;
        __hip_atomic_compare_exchange_strong(&p.cnt[ix.stopped()], &zero, k, __ATOMIC_RELAXED,
                                             __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
    }
    return ix.coarse(k, n);
  };
  if (jb.type == kJobFine) {
    // slice n reads uprev, slices n + s (s >= 1) read U(k, n + s - 1), stored in order from U(k, n)
    const cx<double>* src1 = state(p.U, k, n);
    cx<double>* dst = state(p.F, k, n);
    bool done = false;
    if constexpr (!KFINE) {
      if (p.fine_kind == 0) {
        if (J == 1)
          fine_slices_job<T, NX, 1, 0>(smem, p.tw, 1, uprev, src1, dst, p.steps, p.coef64, p.coef, p.hf, p.basis);
        else
          fine_slices_job<T, NX, 0, 0>(smem, p.tw, J, uprev, src1, dst, p.steps, p.coef64, p.coef, p.hf, p.basis);
        done = true;
      }
    }
    if (!done) {
      if (J == 1)
        fine_slices_job<T, NX, 1, 1>(smem, p.tw, 1, uprev, src1, dst, p.steps, p.coef64, p.coef, p.hf, p.basis);
      else
        fine_slices_job<T, NX, 0, 1>(smem, p.tw, J, uprev, src1, dst, p.steps, p.coef64, p.coef, p.hf, p.basis);
    }
    return ix.fine(k, n);
  }
  if (jb.type == kJobCopy) {
    copy_job<T, NX, NT, S>(en, n < k ? state(p.U, k - 1, n) : state(p.F, k - 1, n), state(p.U, k, n),
                           state(p.G, k - 1, n), state(p.G, k, n), state(p.U, k - 1, n),
                           p.part + size_t(k - 1) * Ns + (n - 1));
    return level_done();
  }
  if (jb.type == kJobCoarse && p.coarse_kind == 1) {
    if (k == 0)
      strang_coarse_job<T, NX, NT, S>(en, p.ccoef64, p.hc, p.basis, uprev, state(p.U, 0, n), state(p.G, 0, n),
                                      nullptr, nullptr, nullptr, nullptr);
    else
      strang_coarse_job<T, NX, NT, S>(en, p.ccoef64, p.hc, p.basis, uprev, state(p.U, k, n), state(p.G, k, n),
                                      state(p.G, k - 1, n), state(p.F, k - 1, n), state(p.U, k - 1, n),
                                      p.part + size_t(k - 1) * Ns + (n - 1));
    return level_done();
  }
  if (jb.type == kJobCoarse) {
    if (k == 0)
      coarse_job<T, NX, NT, S>(en, p.ct, p.basis, uprev, state(p.U, 0, n), state(p.G, 0, n), nullptr, nullptr,
                               nullptr, nullptr);
    else
      coarse_job<T, NX, NT, S>(en, p.ct, p.basis, uprev, state(p.U, k, n), state(p.G, k, n),
                               state(p.G, k - 1, n), state(p.F, k - 1, n), state(p.U, k - 1, n),
                               p.part + size_t(k - 1) * Ns + (n - 1));
    return level_done();
  }
  // split step: the stage-1 group sums of level k live at P1 + k (groups + 1) st,
  // followed by the step's midpoint state; the stage-2 sums at P2 + k groups st
  const size_t lvl1 = size_t(k) * (p.groups + 1) * st;
  const size_t lvl = size_t(k) * p.groups * st;
  cx<T>* Y = p.P1 + lvl1 + size_t(p.groups) * st;
  cx<T> w[MPT][3];
  CoarseRegs<T, MPT> cr;
  if (jb.type == kJobStage1) {
    stage_job<T, NX, NT, S>(en, p.ct, p.basis, uprev, 1, jb.g, nullptr, p.P1 + lvl1 + jb.g * st, w, cr,
                            [] { return true; });
    // the last group to arrive forms y for the stage-2 jobs and publishes
    if (!count_in_last(&p.cnt[ix.stage1(k, n)], p.groups, s_flag)) return -1;
    stage_mid<T, NX, NT, S>(en, p.ct, p.P1 + lvl1, p.groups, w, Y);
    return ix.stage1(k, n);
  }
  // wait for the midpoint (every stage-1 group and y): thread 0 for the
  // workgroup, after the job has formed w from uprev
  auto wait_y = [&] {
    if (threadIdx.x == 0) *s_flag = wait_count(&p.cnt[ix.stage1(k, n)], p.groups + 1, diag, jt, ix.stage1(k, n));
    __syncthreads();
    return __builtin_amdgcn_readfirstlane(*s_flag) != 0;
  };
  if (!stage_job<T, NX, NT, S>(en, p.ct, p.basis, uprev, 2, jb.g, Y, p.P2 + lvl + jb.g * st, w, cr, wait_y))
    return -1;
  // Count this group in; the last group to arrive finishes the step.  Every
  // wavefront first waits for its stores of the group sum to reach the L2
  // (a workgroup barrier waits only for LDS); thread 0's release then writes
  // them back for the other XCDs.
  wait_global_stores();
  __syncthreads();
  if (threadIdx.x == 0) {
    release_for_workgroup();
    const int before = __hip_atomic_fetch_add(&p.cnt[ix.stage2(k, n)], 1, __ATOMIC_RELAXED,
                                              __HIP_MEMORY_SCOPE_AGENT);
    int flag = 0;
    if (before == p.groups - 1) {
      acquire_for_workgroup();
      bool ok = true;
      if (k >= 1) {
        ok = wait_count(&p.cnt[ix.fine(k - 1, n)], 1, diag, jt, ix.fine(k - 1, n));
        if (ok) ok = wait_count(&p.cnt[ix.coarse(k - 1, n)], 1, diag, jt, ix.coarse(k - 1, n));
      }
      if (ok && n == Ns) ok = wait_level_copies(p, ix, k, diag, jt);
      flag = ok ? 1 : 0;
    }
    *s_flag = flag;
  }
  __syncthreads();
  const int finish = __builtin_amdgcn_readfirstlane(*s_flag);
  if (!finish) return -1;
  cx<T> g[MPT][3];
  stage_finish<T, NX, NT, S>(en, p.ct, p.P2 + lvl, p.groups, w, cr, g);
  if (k == 0)
    coarse_correct<T, NX, NT, S>(en, g, state(p.U, 0, n), state(p.G, 0, n), nullptr, nullptr, nullptr, nullptr);
  else
    coarse_correct<T, NX, NT, S>(en, g, state(p.U, k, n), state(p.G, k, n), state(p.G, k - 1, n),
                                 state(p.F, k - 1, n), state(p.U, k - 1, n), p.part + size_t(k - 1) * Ns + (n - 1));
  return level_done();
}

// What a job hands back to the kernel's scheduling loop.
struct JobOut {
  int pub;                 // first counter index to publish, or -1
  int npub;                // counters it publishes
  const void* staged;      // twiddle table left in LDS
};

// A job of grid size NX as an out-of-line call, for kernels that serve
// several grid sizes: each size's job code gets a register allocation of its
// own instead of one shared by every size (shared, the coarse steps of the
// larger sizes spilled).  One call per job; a job runs for microseconds to
// milliseconds.
template <typename T, int NX>
__device__ __attribute__((noinline)) JobOut run_job_call(unsigned char* smem, PipeJob jb, const PipeProb<T>* p,
                                                         const void* staged, int* diag, int jt, int* s_flag,
                                                         bool skip) {
  JobOut o;
  o.staged = staged;
  o.npub = 1;
  o.pub = run_job<T, NX, pipe_inline_fine<T, NX, true>()>(smem, jb, *p, o.staged, diag, jt, s_flag, skip, o.npub);
  return o;
}

// CALL: the job runs as a call (run_job_call), in a kernel for several sizes.
template <typename T, bool CALL, int NX, int... REST>
__device__ __forceinline__ int dispatch_job(int nx, unsigned char* smem, const PipeJob& jb, const PipeProb<T>& p,
                                            const void*& staged, int* diag, int jt, int* s_flag, bool skip,
                                            int& npub) {
  if (nx == NX) {
    if constexpr (CALL) {
      const JobOut o = run_job_call<T, NX>(smem, jb, &p, staged, diag, jt, s_flag, skip);
      staged = o.staged;
      npub = o.npub;
      return o.pub;
    } else {
      return run_job<T, NX, pipe_inline_fine<T, NX, false>()>(smem, jb, p, staged, diag, jt, s_flag, skip, npub);
    }
  }
  if constexpr (sizeof...(REST) > 0)
    return dispatch_job<T, CALL, REST...>(nx, smem, jb, p, staged, diag, jt, s_flag, skip, npub);
  else
    return -1;
}

// The persistent solve over the grid sizes NXS (one, or every supported size
// for a batch of problems of several sizes).
template <typename T, int... NXS>
__global__ void __launch_bounds__(kPipeThreads) k_pipeline(const PipeJob* __restrict__ jobs, int njobs,
                                                           const PipeProb<T>* __restrict__ probs, int* ticket,
                                                           int* abort, int* progress, unsigned long long* trace) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ int s_job, s_ok, s_flag, s_skip;
  // Thread 0's scheduling work (publish the previous job's counter, take a
  // ticket, wait on the new job's dependencies) is one region at the top of
  // the body, between the end-of-job barrier and the hand-out barrier; the
  // body ends with a barrier and nothing thread-specific.  Thread-0 regions on
  // both sides of the back-edge would form a single divergent region across
  // it, which the compiler may turn into a loop the other lanes never leave.
  // The values read back from LDS are made uniform with readfirstlane.
  int pub = -1;                 // first counter index of the job finished last
  int npub = 1;                 // counters it publishes (consecutive slices, kCounterStride apart)
  int* pub_cnt = nullptr;
  const void* staged = nullptr;
  for (;;) {
    if (threadIdx.x == 0) {
      if (pub >= 0) {
        // every wavefront's stores of the job reached the L2 before the barrier
        release_for_workgroup();
        for (int i = 0; i < npub; ++i)
          __hip_atomic_fetch_add(&pub_cnt[pub + i * kCounterStride], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_fetch_add(abort + 3, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (progress) {
          progress[2 * blockIdx.x] += 1;
          progress[2 * blockIdx.x + 1] = pub;
        }
      }
      const int jt = __hip_atomic_fetch_add(ticket, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      bool ok = true, skip = false;
      if (jt < njobs) {
        const PipeJob jb = jobs[jt];
        skip = past_stop(jb, probs[jb.prob]);
        if (!skip) ok = wait_deps(jb, probs[jb.prob], abort, jt);
      }
      s_job = jt;
      s_ok = ok;
      s_skip = skip;
    }
    __syncthreads();
    const int j = __builtin_amdgcn_readfirstlane(s_job);
    const int ok = __builtin_amdgcn_readfirstlane(s_ok);
    if (j >= njobs || !ok) break;
    if (trace && threadIdx.x == 0) {
      trace[3 * j] = wall_clock64();
      trace[3 * j + 2] = blockIdx.x;
    }
    const PipeJob jb = jobs[j];
    const PipeProb<T>& p = probs[jb.prob];
    const int nx = __builtin_amdgcn_readfirstlane(p.nx);
    const bool skip = __builtin_amdgcn_readfirstlane(s_skip) != 0;
    int np = 1;
    // ETDRK4 fine jobs of the sizes pipe_inline_fine names run inline, the
    // other jobs through dispatch_job (as calls in a kernel for several sizes)
    constexpr bool kMulti = sizeof...(NXS) > 1;
    int r = kNotRun;
    if (!skip && jb.type == kJobFine && __builtin_amdgcn_readfirstlane(p.fine_kind) == 0)
      r = dispatch_fine<T, kMulti, NXS...>(nx, smem_raw, jb, p, staged, j, np);
    if (r == kNotRun) r = dispatch_job<T, kMulti, NXS...>(nx, smem_raw, jb, p, staged, abort, j, &s_flag, skip, np);
    pub = __builtin_amdgcn_readfirstlane(r);
    npub = __builtin_amdgcn_readfirstlane(np);
    pub_cnt = p.cnt;
    // Every wavefront waits for its stores of the job's results to reach the
    // L2 before the barrier after which thread 0 publishes the job's counters
    // (the barrier alone waits only for LDS); thread 0's release atomic then
    // writes them back to the memory the other XCDs read.
    wait_global_stores();
    __syncthreads();
    if (trace && threadIdx.x == 0) trace[3 * j + 1] = wall_clock64();
  }
}

template <typename T, int... NXS>
inline hipError_t pipeline_launch(size_t lds, const PipeJob* jobs, int njobs, const void* probs, int* ticket,
                                  int* abort, int* progress, unsigned long long* trace, int grid, hipStream_t s) {
  prep_lds(k_pipeline<T, NXS...>, lds);
  hipLaunchKernelGGL((k_pipeline<T, NXS...>), dim3(grid), dim3(kPipeThreads), lds, s, jobs, njobs,
                     static_cast<const PipeProb<T>*>(probs), ticket, abort, progress, trace);
  return hipGetLastError();
}

template <typename T>
inline size_t pipeline_lds_t(int nx, int nx_max) {
  const int sizes[6] = {64, 128, 256, 512, 1024, 2048};
  const size_t lds[6] = {pipe_lds<T, 64>(), pipe_lds<T, 128>(), pipe_lds<T, 256>(),
                         pipe_lds<T, 512>(), pipe_lds<T, 1024>(), pipe_lds<T, 2048>()};
  size_t out = 0;
  for (int i = 0; i < 6; ++i)
    if (nx > 0 ? sizes[i] == nx : sizes[i] <= nx_max) out = lds[i] > out ? lds[i] : out;
  return out;
}

template <typename T, int... NXS>
inline int pipeline_occupancy(size_t lds) {
  prep_lds(k_pipeline<T, NXS...>, lds);
  int per_cu = 0, dev = 0, cus = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(k_pipeline<T, NXS...>),
                                                   kPipeThreads, lds) != hipSuccess ||
      hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
    (void)hipGetLastError();
    return 0;
  }
  return per_cu * cus;
}

}  // namespace ap
