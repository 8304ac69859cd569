/*
 * aparareal.h -- C ABI of the MI355X (gfx950) asymptotic parareal library.
 *
 * Problem (Haut & Wingate, Sec. 1, eq. full eqn; Sec. 6.1, eq. RSW equations):
 *     du/dt + (1/eps) L u = N(u) + D u,   u = (v1, v2, h) periodic on [0, 2 pi),
 *     L = [[0, -1, F^{-1/2} d/dx], [1, 0, 0], [F^{-1/2} d/dx, 0, 0]],
 *     D = -nu d^4/dx^4 (hyperviscosity, damping),
 *     N(u) = -(v1 dv1/dx, v1 dv2/dx, d(h v1)/dx).
 * Fourier pseudo-spectral discretisation on x_j = 2 pi j / N with the 2/3 rule
 * (retained wavenumbers |k| <= floor(N/3)); every input state is projected onto
 * that band first.
 *
 * Conventions for every call below:
 *   - Arrays are DEVICE pointers (HIP global memory, e.g. torch CUDA tensors)
 *     unless marked host.  Physical states are float64, row-major
 *     [batch][3][N] with fields in the order (v1, v2, h) and x_j = 2 pi j / N.
 *   - Work is enqueued on `stream` (a hipStream_t passed as void*, NULL = the
 *     default stream); outputs are valid once that stream has completed.
 *     Calls return after enqueueing; host-side argument errors are reported
 *     before anything is enqueued.
 *   - The caller owns every array it passes.  The library owns the context
 *     (coefficient tables, device scratch) and the server.
 *   - Return value: AP_OK (0) or a negative AP_E* code; the thread-local
 *     message of the last failure is aparareal_last_error().
 *   - precision: AP_PREC_FP32 runs the propagators (FFTs, nonlinear term,
 *     exponential integrator, time average) in FP32 with FP64 inputs/outputs
 *     and FP64 parareal correction; AP_PREC_FP64 runs everything in FP64.
 *   - A context is not thread-safe; use one context per host thread.
 */
#ifndef APARAREAL_H
#define APARAREAL_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  AP_OK = 0,
  AP_PENDING = 1,     /* serving: request not finished yet                     */
  AP_EINVAL = -1,     /* bad argument (size, parameter, NULL pointer)          */
  AP_ENOMEM = -2,     /* device allocation failed / request exceeds budget     */
  AP_EDEVICE = -3,    /* a HIP runtime call failed                             */
  AP_ENOTFOUND = -4,  /* unknown serving ticket                                */
  AP_ENUMERIC = -5,   /* non-finite state or residual                          */
  AP_EBUSY = -6       /* server shutting down                                  */
};

enum { AP_PREC_FP32 = 0, AP_PREC_FP64 = 1 };

typedef struct ap_ctx ap_ctx;

/* Message of the last failed call on this host thread ("" if none).          */
const char* aparareal_last_error(void);

/* Create a context for grid size N (power of two, 64 <= N <= 2048), small
 * parameter eps > 0, F > 0 (the Froude-type constant of Sec. 6.1) and
 * hyperviscosity nu >= 0 on the current HIP device.  NULL on error.          */
ap_ctx* aparareal_create(int N, double eps, double F, double nu);

/* Release the context and its device memory (synchronises the device).      */
int aparareal_destroy(ap_ctx* ctx);

/* Dealiased nonlinear term N(u) (Sec. 6.1, operator table; sign taken from
 * the RSW equations): U_in, N_out physical [batch][3][N].                     */
int aparareal_nonlinear(ap_ctx* ctx, const double* U_in, double* N_out, int batch,
                        int precision, void* stream);

/* Fine propagator (ETDRK4 of Cox & Matthews, the fine integrator of Sec. 6.2):
 * `steps` exponential RK4 steps of length dT/steps applied to every state of
 * the batch at once (the parallel "parfor" over slices of Alg. 4).
 * U_in, U_out physical [batch][3][N]; U_out may not alias U_in.               */
int aparareal_fine_batch(ap_ctx* ctx, const double* U_in, double* U_out, int batch,
                         double dT, int steps, int precision, void* stream);

/* aparareal_fine_batch for callers that cannot allocate memory: code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * Same arguments, kernels and results (bitwise) as aparareal_fine_batch, but
 * every scratch byte (the coefficient tables of dT/steps and the modal input
 * and output states) lives in one 64 MiB array per device that the library
 * holds until the process ends; the call makes no hipMalloc, hipFree or other
 * allocating call, on the device or the host.  The tables are copied from a
 * pageable host buffer of the context with hipMemcpyAsync, so the call is not
 * capturable as it stands.  Limit: 2 * batch * 3 * (N/3 + 1) * 16 bytes plus
 * the tables (576 * (N/3 + 1) bytes, rounded to 256) within 64 MiB, e.g.
 * 8122 states at N = 256 or 1017 at N = 2048; a larger batch returns AP_EINVAL
 * before anything is enqueued.  The context's device must be current.  Every
 * call on one device shares that device's array: calls on one stream run in
 * order, calls that overlap on one GPU (other streams, other contexts or
 * threads) race on it.                                                        */
int aparareal_fine_batch_noalloc(ap_ctx* ctx, const double* U_in, double* U_out, int batch,
                                 double dT, int steps, int precision, void* stream);

/* Strang-splitting propagator (Alg. 3): `steps` steps of length h = dT/steps,
 * each a half step of the exact linear flow exp((h/2)(-L/eps + D)), a
 * midpoint step of the nonlinear flow v <- v + h N(v + (h/2) N(v)), and a
 * second half step; for every state of the batch at once.  It is the fine
 * solver of Alg. 3 and, with steps = 1, the coarse solver of standard
 * parareal.  U_in, U_out physical [batch][3][N]; U_out may not alias U_in.   */
int aparareal_strang_batch(ap_ctx* ctx, const double* U_in, double* U_out, int batch,
                           double dT, int steps, int precision, void* stream);

/* Kernel-weighted time average of the nonlinear term (Sec. 2, eq. numerical
 * average; Alg. 1): Nbar(u) = (1/M) sum_{m<M} rho(m/M) exp(s_m L) N(exp(-s_m L) u),
 * s_m = m T0 / M (fast time), rho the smooth bump of Sec. 2.
 * U_in, Nbar_out physical [batch][3][N]; M >= 2, T0 > 0.                      */
int aparareal_average(ap_ctx* ctx, const double* U_in, double* Nbar_out, int batch,
                      double T0, int M_avg, int precision, void* stream);

/* Asymptotic coarse step G (Alg. 2): half dissipative step, explicit midpoint
 * step of the averaged nonlinear flow, half dissipative step, rotation by
 * exp(-(dT/eps) L).  T0 <= 0 selects T0 = dT/eps (average over one coarse
 * step, Sec. 4).  U_in, U_out physical [batch][3][N].                         */
int aparareal_coarse(ap_ctx* ctx, const double* U_in, double* U_out, int batch,
                     double dT, int M_avg, double T0, int precision, void* stream);

typedef struct {
  double T;          /* final time; slices of length dT = T / slices             */
  int slices;        /* Ns >= 1                                                   */
  int K;             /* parareal iterations after the coarse initial guess >= 0  */
  double dt_fine;    /* requested fine step; fine steps per slice = ceil(dT/dt)  */
  int M_avg;         /* averaging samples M >= 2                                 */
  double T0;         /* fast-time averaging window; <= 0 selects dT/eps          */
  double tol;        /* > 0: stop after the first iteration k with r^k <= tol     */
                     /* (decided on the device); <= 0: run exactly K iterations  */
  int precision;     /* AP_PREC_FP32 or AP_PREC_FP64                              */
} ap_solve_params;

/* Parareal solve (Sec. 3, eq. HMM parareal iteration; Alg. 4):
 *   U_n^0 = G(U_{n-1}^0);  U_n^k = Fine(U_{n-1}^{k-1}) + (G(U_{n-1}^k) - G(U_{n-1}^{k-1}))
 * with the correction evaluated in FP64 and G(U^{k-1}) reused from the previous
 * sweep.  The iterations run as one pipelined persistent launch (iteration
 * k+1 starts on a slice as soon as its inputs exist); the values are those of
 * the iteration-by-iteration order.  Slices n <= k, which iteration k makes
 * exact (they equal the serial fine solution), are copied instead of
 * recomputed (AP_OPT_SKIP).  With tol > 0 the job that completes iteration k
 * computes r^k on the device; once r^k <= tol the later iterations' jobs end
 * without work, U_out holds U^k and the later resid entries are -1 (no host
 * synchronisation; AP_OPT_SWEEPS = 1 instead runs the iterations one by one
 * with a host check of each residual, the same results).
 * u0 physical [3][N]; U_out physical [slices+1][3][N] holds U_0..U_Ns after
 * the last iteration run; resid (device, float64 [K]) receives
 * r^k = max_n ||U_n^k - U_n^{k-1}||_2 / ||U_n^k||_2 over the 3N grid values.  */
int aparareal_solve(ap_ctx* ctx, const double* u0, const ap_solve_params* params,
                    double* U_out, double* resid, void* stream);

/* Many independent problems in one persistent launch (the slices of every
 * problem are the batch of one launch; Alg. 4 per problem).  Each item names
 * its own context (grid size, eps, F, nu; a context may appear only once),
 * initial state, parameters (each problem stops on its own tolerance; the
 * precision must be the same for all items) and outputs, with the meaning and
 * layout of aparareal_solve.  Each problem's results equal those of aparareal_solve on
 * its own.  The first item's context holds the launch's job list and
 * counters; every context keeps its problem's states.                       */
typedef struct {
  ap_ctx* ctx;
  const double* u0;          /* device [3][N]                                     */
  ap_solve_params params;
  double* U_out;             /* device [slices+1][3][N]                           */
  double* resid;             /* device [K]                                        */
} ap_batch_item;
int aparareal_solve_batch(const ap_batch_item* items, int count, void* stream);

/* Execution options of a context (none changes the method; AP_OPT_GROUP
 * changes the summation order of the time average, hence rounding):
 *   AP_OPT_SPLIT  -1 (default): a coarse step of a pipelined solve runs on
 *                 several workgroups (one per sample group, for each of its
 *                 two averages) when the average has two groups or more;
 *                 0: one workgroup per coarse step; 1: always split.
 *   AP_OPT_GROUP  samples per group of the time average (the sum runs over
 *                 each group in sample order, then over the groups in order);
 *                 0 (default) = by grid size, or the size aparareal_autotune
 *                 chose.  Reading returns the size used.
 *   AP_OPT_GRID   workgroups of a persistent launch; 0 (default) = as many as
 *                 are resident on the device at once.
 *   AP_OPT_GRAPH  1: a pipelined solve (or batch whose first item names this
 *                 context) is captured into a hipGraph on its first call and
 *                 replayed by later calls with the same arguments, device
 *                 addresses and shapes (inputs are read at replay time); the
 *                 graph holds kernels and device copies only.  With kernel
 *                 timing on, the pipeline class then times the whole replay.
 *                 0 (default): launches are enqueued one by one.
 *   AP_OPT_SKIP   1 (default): slices made exact by iteration k are copied
 *                 (values unchanged); 0: every coarse step and fine slice of
 *                 every iteration is computed.
 *   AP_OPT_SWEEPS 1: aparareal_solve with tol > 0 runs the iterations one by
 *                 one (a fine batch and a serial coarse sweep each) with a
 *                 host check of the residual; 0 (default): pipelined.
 *                 ETDRK4 fine slices and asymptotic coarse steps only.
 *   AP_OPT_FINE   fine solver of the pipelined solve: 0 (default) ETDRK4,
 *                 1 Strang steps (Alg. 3, aparareal_strang_batch).
 *   AP_OPT_COARSE coarse solver: 0 (default) the asymptotic step (Alg. 2);
 *                 1 one Strang step of length dT, i.e. standard parareal
 *                 on the full equation (the paper's comparison, Sec. 6.2);
 *                 M_avg and T0 are then unused.
 *   AP_OPT_FINE_GROUP  slices one fine job of a pipelined solve steps
 *                 together (consecutive slices of one iteration; each rounds
 *                 as it would alone, so values do not change).  0 (default):
 *                 automatic, 1 while the slices of the solve or batch fit the
 *                 resident workgroups, else the most the grid size allows
 *                 (16, 10, 5, 2, 1, 1 for N = 64 .. 2048); n >= 1: at most n.
 *                 A group starts when its last slice's input is ready, so
 *                 grouping trades latency for throughput.
 *   AP_OPT_FINE_SHAPE  configuration of aparareal_fine_batch: workgroup shape
 *                 (threads and slices per workgroup; three are compiled per
 *                 precision and grid size) and FFT plan (aparareal_fft_plan;
 *                 two for N >= 256): -1 (default) the configuration
 *                 aparareal_autotune_fine chose for this device, grid size
 *                 and precision (in this context or, earlier, in the tuning
 *                 cache), else 0; c = shape + 3 plan sets that one
 *                 (AP_EINVAL if it is not compiled for this N).  The shape
 *                 does not change results; plan 1 rounds differently at
 *                 N = 1024 (other radices), identically elsewhere.
 *   AP_OPT_HANDOFF_NS  scheduling weight of a dependency between two jobs of
 *                 a pipelined launch this context owns, in ns (default 6000):
 *                 the host orders the jobs by a simulation of the launch in
 *                 which a job may start this long after the jobs it waits
 *                 for; aparareal_autotune may choose another value.  Job
 *                 order only: results are unchanged.                         */
enum {
  AP_OPT_SPLIT = 0, AP_OPT_GROUP = 1, AP_OPT_GRID = 2, AP_OPT_GRAPH = 3, AP_OPT_SKIP = 4, AP_OPT_SWEEPS = 5,
  AP_OPT_FINE = 6, AP_OPT_COARSE = 7, AP_OPT_FINE_GROUP = 8, AP_OPT_FINE_SHAPE = 9, AP_OPT_HANDOFF_NS = 10
};
int aparareal_set_option(ap_ctx* ctx, int option, int value);
int aparareal_get_option(ap_ctx* ctx, int option, int* value);

/* Autotuner of the pipelined schedule for the problems of `items` (one item:
 * a single solve; several: a batch as in aparareal_solve_batch, with the same
 * argument rules).  Candidates: whole coarse steps (AP_OPT_SPLIT 0) with the
 * default group size, and split steps (AP_OPT_SPLIT 1) with group sizes of
 * 1, 3/2, 2 and 3 times the grid-size default (one multiple for all items;
 * a context whose AP_OPT_GROUP is set keeps that size).  For each candidate
 * it runs the solve, records every job's duration on the device clock,
 * re-orders the jobs with the measured durations per problem and job type
 * (twice), and times three solves; with the fastest candidate it then times
 * the job order built with half and 5/3 of the first context's
 * AP_OPT_HANDOFF_NS.  It keeps the fastest candidate, its measured durations
 * and the weight in the contexts, so that later solves of the same shape use
 * them.  The outputs receive the results of the last solve run.
 * *best_ms (host, may be NULL) receives the best solve time.  The mapping and
 * the job order leave results unchanged; the chosen group size changes the
 * summation order of the average (rounding only), and later solves equal
 * solves with AP_OPT_SPLIT and AP_OPT_GROUP set to the values read back.    */
int aparareal_autotune(const ap_batch_item* items, int count, void* stream, double* best_ms);

/* Autotuner of the fine batch (the parareal fine sweep over independent
 * states): times every configuration of aparareal_fine_batch compiled for
 * this grid size (AP_FINE_CONFIGS slots: configuration c is workgroup shape
 * c % 3 with FFT plan c / 3, see aparareal_fft_plan; plan 1 exists for
 * N >= 256) in this precision on the caller's states (one warm-up and three
 * timed launches each, HIP events on `stream`; the call synchronises), keeps
 * the fastest in the context, and records it in the tuning cache, a text file
 * read by every later context of this device kind, grid size and precision:
 * $APARAREAL_TUNE_CACHE, else $XDG_CACHE_HOME/aparareal/tune.txt, else
 * $HOME/.cache/aparareal/tune.txt (a write that fails is ignored).  U_in
 * physical [batch][3][N], unchanged.  shape_ms (host, AP_FINE_CONFIGS doubles,
 * may be NULL) receives the mean launch time of each configuration (-1 for
 * one not compiled at this N), *best (may be NULL) the chosen one.  The
 * workgroup shape does not change results; the FFT plan changes the rounding
 * at N = 1024 only (other radices).                                          */
enum { AP_FINE_CONFIGS = 6 };
int aparareal_autotune_fine(ap_ctx* ctx, const double* U_in, int batch, double dT, int steps, int precision,
                            void* stream, double* shape_ms, int* best);

/* The configuration the context's fine batches use in this precision: its
 * index (0 .. AP_FINE_CONFIGS - 1: workgroup shape index % 3, FFT plan
 * index / 3), threads per workgroup and slices per workgroup (outputs may be
 * NULL).                                                                       */
int aparareal_fine_shape(ap_ctx* ctx, int precision, int* shape, int* threads, int* slices);

/* The wave-local FFT of length N/2 (Sec. 6.2's pseudo-spectral evaluation of
 * N: each real field of length N as a complex transform of half the length)
 * in plan `plan` (0: the plan every kernel uses; 1: the fine batch's
 * alternative, N >= 256): its Stockham passes' radices (radices[0 ..
 * *passes - 1], host int[4]) and how many exchanges between passes are row
 * swaps in registers instead of LDS round trips (*reg_exchanges).  Host only;
 * AP_EINVAL for an N or a plan that does not exist.                          */
int aparareal_fft_plan(int N, int plan, int* radices, int* passes, int* reg_exchanges);

/* Measured rates of the current device that the hot path is priced against
 * (diagnostics): FP32 and FP64 vector FMA throughput in TFLOP/s (16
 * independent FMA chains per lane, 16 workgroups of 256 threads per CU; FP32
 * without packed instructions, as the library is built) and LDS read
 * bandwidth in TB/s (conflict-free 64-bit reads by every lane).  Allocates
 * and frees an 8-16 MiB scratch buffer and synchronises `stream`.  Outputs
 * are host doubles.                                                          */
int aparareal_measure_peaks(void* stream, double* fp32_tflops, double* fp64_tflops, double* lds_tbps);

/* Kernel timing (diagnostics, no effect on results).  While enabled, the
 * library brackets each of its own kernel launches with a pair of HIP events
 * recorded on the launch stream and accumulates the elapsed time per kernel
 * class.  aparareal_profile(ctx, 1) resets the counters and enables;
 * aparareal_profile(ctx, 0) disables.  aparareal_profile_read waits for the
 * recorded events (host synchronisation) and returns the number of launches
 * and their total milliseconds for one class.                                */
enum {
  AP_K_FINE = 0,        /* fine ETDRK4 batch                                     */
  AP_K_SWEEP = 1,       /* serial coarse sweep with parareal correction          */
  AP_K_TO_MODAL = 2,    /* physical -> modal boundary transform                  */
  AP_K_TO_PHYSICAL = 3, /* modal -> physical boundary transform                  */
  AP_K_RESID = 4,       /* residual reduction                                    */
  AP_K_NONLINEAR = 5,
  AP_K_AVERAGE = 6,
  AP_K_COARSE = 7,
  AP_K_PIPELINE = 8,    /* persistent pipelined parareal iteration (all jobs)    */
  AP_K_CLASSES = 9
};
int aparareal_profile(ap_ctx* ctx, int enable);
int aparareal_profile_read(ap_ctx* ctx, int kernel_class, int* launches, double* total_ms);

/* Order in which the pipelined solve hands out its jobs (host only, no device
 * needed; for inspection and tests), for a problem of grid size N with
 * parameters p, split / group as AP_OPT_SPLIT / AP_OPT_GROUP, and fine jobs of
 * up to fine_group slices (1..64, capped by the grid size's maximum for
 * p->precision).  Writes up to max_jobs (type, k, n, g) quadruples to the
 * host array `out` (may be NULL): type 0 = coarse step C(k,n) in one
 * workgroup, k = 0..K; 1 = fine slices F(k,n .. n+g-1) = Fine(U_{n-1+i}^k),
 * k = 0..K-1, n > k (g = 1 for a single slice); 2 / 3 = first / second
 * average of a split coarse step C(k,n) for sample group g; 4 = copy of the
 * exact slice n <= k at level k >= 1 (slice skipping).  Jobs are ordered by
 * their estimated ready times, and every job comes after the jobs it depends
 * on.
 * Returns the job count or AP_EINVAL.                                        */
int aparareal_pipeline_schedule(int N, const ap_solve_params* p, int split, int group, int fine_group, int* out,
                                int max_jobs);

/* The hand-out order of a batched launch (as aparareal_solve_batch) of
 * `count` problems of grid sizes N[i] and parameters p[i] (host arrays),
 * split / group / fine_group as above for every problem.  cost (host, may be
 * NULL): per problem four job durations in us that replace the analytic
 * estimates as aparareal_autotune's measurements do: fine step, stage-1 job,
 * stage-2 job, whole coarse step (0 keeps the estimate).  Writes up to
 * max_jobs (prob, type, k, n, g) quintuples to `out` (may be NULL).
 * Returns the job count or AP_EINVAL.                                        */
int aparareal_pipeline_schedule_batch(int count, const int* N, const ap_solve_params* p, int split, int group,
                                      int fine_group, const double* cost, int* out, int max_jobs);

/* Stall record of the context's last pipelined solve (waits for it): host
 * info[3] = (stalled, job index, flag index).  A stall means a job waited on
 * a dependency while no job of the launch completed for 1 s; the launch then ends early and the
 * solve's residuals are NaN.  It does not occur in correct operation.        */
int aparareal_pipeline_status(ap_ctx* ctx, int* info);

/* Per-job timeline of pipelined solves (diagnostics).  enable = 1 / 0 turns
 * recording on / off for the following solves (out may be NULL); enable = -1
 * reads the last launch this context owned into host `out` [8 * max_jobs]:
 * per job in hand-out order (problem, type, k, n, g, start, end, workgroup)
 * with start/end in ticks of the device's constant-rate clock (100 MHz on
 * MI355X).  Returns the number of jobs written (reading waits for the solve). */
int aparareal_pipeline_trace(ap_ctx* ctx, int enable, long long* out, int max_jobs);

/* ---------------------------------------------------------------- serving ---
 * A request loop over parareal solves (Alg. 4 per request).  Requests are
 * admitted in arrival order while their HBM footprint fits the budget and
 * fewer than max_slots run; admitted requests are batched (one persistent
 * launch per batch, as aparareal_solve_batch) and up to four batches run at
 * once on separate streams, so requests that arrive while others are on the
 * device start as soon as memory and slots free up, and their work overlaps.
 * Each request's states stay in device memory for its whole solve; its
 * coarse steps run whole (one workgroup each, AP_OPT_SPLIT 0), since a batch
 * already fills the device with independent jobs.  A request's result does
 * not depend on what it was batched with, and equals aparareal_solve's.
 * One worker thread owns the device work; submit, poll and stats may be
 * called from any thread.                                                   */
typedef struct ap_server ap_server;

/* hbm_budget_bytes: device memory the admitted requests may hold at once
 * (footprint per request: its states at all K+1 iteration levels, tables,
 * job list and buffers); max_slots >= 1: requests running at once.  NULL on
 * error.  Uses the current HIP device.                                      */
ap_server* aparareal_serve_create(size_t hbm_budget_bytes, int max_slots);

/* Queue one solve of the problem (N, eps, F, nu) from u0 (HOST [3][N],
 * copied before returning) with `params` (as for aparareal_solve).  *ticket receives the request's id.  AP_ENOMEM if the request
 * alone exceeds the budget, AP_EINVAL on bad arguments, AP_EBUSY while the
 * server shuts down.                                                        */
int aparareal_serve_submit(ap_server* server, int N, double eps, double F, double nu, const double* u0,
                           const ap_solve_params* params, unsigned long long* ticket);

/* AP_PENDING while the request is queued or running.  Once it has finished:
 * copies U (HOST [slices+1][3][N]) and resid (HOST [K]) if not NULL, sets
 * *latency_s (submit to completion, seconds) if not NULL, releases the
 * ticket and returns AP_OK, or the request's error code (then the ticket is
 * released too).  AP_ENOTFOUND for an unknown or released ticket.          */
int aparareal_serve_poll(ap_server* server, unsigned long long ticket, double* U_out, double* resid,
                         double* latency_s);

/* Counters (host out[7]): completed, failed, queued, running, batched
 * launches, device bytes held by running requests, peak of the latter.     */
int aparareal_serve_stats(ap_server* server, unsigned long long* out);

/* Finish every queued and running request, then release the server.       */
int aparareal_serve_destroy(ap_server* server);

#ifdef __cplusplus
}
#endif

#endif /* APARAREAL_H */
