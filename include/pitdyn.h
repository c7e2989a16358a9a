/*
 * pitdyn -- Parareal for 2.5D kinematic dynamos on AMD Instinct MI355X.
 *
 * C ABI of libpitdyn.so.  The library integrates the dimensionless induction
 * equation dB/dt = curl(u x B) + Rm^-1 lap B (Clarke, Davies, Ruprecht &
 * Tobias, arXiv:1902.00387, Section 1, eq. induction-dimensionless-1) for
 * B = b(x, y, t) exp(i kz z) on the 2pi-periodic square (Section 1, 2.5D
 * ansatz; Section 4, Fourier collocation with N x N modes), with a prescribed
 * flow (Section 2: Roberts flow, Section 2.1; Galloway-Proctor CP flow,
 * Section 2.2), and runs the Parareal iteration of Section 3
 * (eq. parareal) with the defect of eq. error.
 *
 * Field layout ("full layout"): complex128 coefficients as interleaved
 * (re, im) doubles, [nfields][3][N][N] = [field][component x,y,z][ky index]
 * [kx index], index m standing for wavenumber m if m < N/2 else m - N, so that
 * b(x, y) = sum_k b_k exp(i (kx x + ky y)).  Every coefficient outside the
 * square 2/3 box |kx|, |ky| <= floor((N - 1)/3) must be zero (dealiasing
 * rule); a nonzero one is rejected with PD_EINVAL.
 *
 * Time stepping: explicit curl(u x b), implicit diffusion -|k|^2/Rm
 * (Section 4), by the second-order semi-implicit backward difference
 * formula (SBDF2) started in every slice with one SBDF1 step (Section 4:
 * multistep methods restart in every slice).  Coarse propagator: same
 * scheme on an N_C grid with step dt_coarse (Section 3.2: coarsening in
 * space and time; Section 4: Fourier re-sampling between the grids).
 *
 * Conventions for every call:
 *  - returns a pd_status; no C++ exception crosses the ABI;
 *    pd_last_error(ctx) gives a message for the last failure on ctx;
 *  - host pointers are read or written only during the call, caller owned;
 *  - device pointers ("_dev") are borrowed for the call; work is queued on
 *    the given HIP stream (hipStream_t passed as void*; NULL is HIP's null
 *    stream) and the call returns after the work completes on that stream;
 *    calls without a stream argument use the context's stream;
 *  - a context is not thread safe; use one per host thread.
 */
#ifndef PITDYN_H
#define PITDYN_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pd_ctx pd_ctx;

typedef enum {
  PD_OK = 0,
  PD_NOT_CONVERGED = 1, /* Parareal stopped at max_iter with sigma > tol  */
  PD_EINVAL = -1,       /* invalid argument or field outside the 2/3 box  */
  PD_ENOMEM = -2,       /* device allocation failed                       */
  PD_EHIP = -3,         /* HIP runtime error (message in pd_last_error)   */
  PD_ESTATE = -4,       /* call out of order (e.g. no problem set)        */
  PD_EUNSTABLE = -5     /* non-finite state (unstable step size)          */
} pd_status;

typedef enum {
  PD_FLOW_NONE = 0,    /* u = 0: pure diffusion                           */
  PD_FLOW_ROBERTS = 1, /* u = (cos y, sin x, sin y + cos x), Section 2.1 */
  PD_FLOW_GP = 2       /* Galloway-Proctor CP flow, Section 2.2, with the  */
                       /* paper's (y, z, x) relabelled as (x, y, z):       */
                       /* u = A (cos(y + sin t), sin(x + cos t),           */
                       /*        cos(x + cos t) + sin(y + sin t)),         */
                       /* A = sqrt(3/2), t absolute time                   */
} pd_flow;

typedef enum {
  PD_PATH_AUTO = -1,   /* library chooses                                 */
  PD_PATH_MULTI = 0,   /* two launches per step over all fields and tiles */
  PD_PATH_SINGLE = 1,  /* one workgroup per field runs every step         */
  PD_PATH_MULTI2 = 2   /* two-launch path with the batch halved over two
                          streams, half a step apart, so column-phase and
                          row-phase launches overlap                     */
} pd_path;

typedef enum {
  PD_COARSE_AUTO = 0,  /* convolution form for SBDF2 with N_coarse <= 64, else
                          the multi-launch form                              */
  PD_COARSE_FFT = 1,   /* same pseudo-spectral kernels as the fine propagator,
                          the whole sweep in one workgroup                   */
  PD_COARSE_CONV = 2,  /* explicit term as the exact spectral convolution with
                          the flow's four Fourier modes (|k| = 1); equals the
                          pseudo-spectral value to rounding since nothing
                          aliases on the 2/3 box; N_coarse <= 64             */
  PD_COARSE_MULTI = 3  /* host-driven: per slice the multi-launch fine-step
                          kernels on the coarse grid (batch of one)          */
} pd_coarse_form;

/* Time steppers (Section 4: IMEX, explicit advection and stretching, implicit
   diffusion).  Both restart from the slice's start value in every slice. */
typedef enum {
  PD_SCHEME_SBDF2 = 0,  /* one SBDF1 step, then SBDF2 (multistep, restarted) */
  PD_SCHEME_RK443 = 1,  /* ARS(4,4,3) IMEX Runge-Kutta, the paper's RK443:
                           four explicit evaluations a step, third order */
  PD_SCHEME_RK222 = 2,  /* ARS(2,2,2) (RK222): two evaluations, second order */
  PD_SCHEME_RK111 = 3   /* ARS(1,1,1) (RK111), forward-backward Euler */
} pd_scheme;

/* Number type of a context's fields and kernels.  The C ABI always takes and
   returns complex128 fields; with PD_C64 the library rounds them to
   complex64 on entry and computes the fine and coarse propagators, the
   Parareal correction and the slice states in FP32 (defect and norm sums in
   FP64), halving the bytes every step moves.  Set with pd_set_precision. */
typedef enum {
  PD_C128 = 0, /* complex128 (default) */
  PD_C64 = 1   /* complex64 */
} pd_prec;

#define PD_MAX_ITER 256

typedef struct {
  int k_con;                   /* first k with sigma_k <= tol, -1 if none  */
  int iters;                   /* Parareal iterations run (fine sweeps)    */
  double sigma[PD_MAX_ITER];   /* sigma_k, k = 1..iters (eq. error)        */
  double t_coarse0_s;          /* initial coarse run (GPU time)            */
  double t_fine_s;             /* all fine sweeps (GPU time)               */
  double t_coarse_s;           /* all correction sweeps (GPU time)         */
  double t_total_s;            /* wall clock of the whole call             */
  /* R_f / R_c and the speed-up estimate of eq. speed_up, from the times
     above (Section 3.1): a fine sweep runs every slice at once, so its mean
     time stands for R_f, one slice of F; a coarse sweep runs the slices one
     after another, so its mean time over n_slices stands for R_c;
     model_speedup = [(1 + k/P) R_c/R_f + k/P]^-1 with k = k_con (iters if
     not converged).  Pipelined runs overlap their sweeps, so their summed
     times overstate R_f and R_c.  0 when no sweep was timed. */
  double Rf_over_Rc;
  double model_speedup;
} pd_report;

/* Context on HIP device `hip_device` with its own stream. */
pd_status pd_create(pd_ctx** out, int hip_device);
void pd_destroy(pd_ctx* ctx);
/* Message of the last failure on ctx ("" if none); valid until the next call. */
const char* pd_last_error(const pd_ctx* ctx);
/* Queue subsequent work of pd_parareal / host-pointer calls on this stream
   (borrowed; NULL restores the context's own stream). */
pd_status pd_set_stream(pd_ctx* ctx, void* hip_stream);

/* Problem: flow, Rm > 0, kz (any real), N in {16, 32, 64, 128, 256, 512}
   (Section 4: N x N Fourier modes).  Frees slice buffers of an earlier problem. */
pd_status pd_set_problem(pd_ctx* ctx, pd_flow flow, double Rm, double kz, int N);

/* Number type of the context (PD_C128 default, PD_C64).  Drops the time grid
   and slice states (call pd_set_time again).  With PD_C64: SBDF2 steppers
   only; coarse sweep in the convolution (N_coarse <= 64) or multi-launch
   form; one launch shape per grid (pd_autotune is PD_EINVAL); the learned
   coarse propagator, checkpoint/resume (pd_get_coarse_values,
   pd_set_slices) and pd_steps_dev_noalloc are complex128 only (PD_EINVAL). */
pd_status pd_set_precision(pd_ctx* ctx, pd_prec prec);

/* Parareal time grid (Section 3): [0, T] cut into n_slices slices of length
   dT = T/n_slices; fine step dt_fine, coarse step dt_coarse on an N_coarse
   grid (0 = same as N, else a power of two in [16, N]).  dT/dt_fine and
   dT/dt_coarse must be integers to 1e-9 relative.  Allocates the slice buffers
   ((4 n_slices + 2) fields of 3 (2K+1)^2 complex values plus n_slices row
   buffers of 3 (2K+1) N values, used in place by both transform phases). */
pd_status pd_set_time(pd_ctx* ctx, double T, int n_slices, double dt_fine, double dt_coarse,
                      int N_coarse);

/* Choose how batched fine propagation is launched (testing and tuning). */
pd_status pd_set_path(pd_ctx* ctx, pd_path path);
/* Choose how pd_parareal's serial coarse sweep evaluates the explicit term
   (one workgroup runs the whole sweep either way). */
pd_status pd_set_coarse_form(pd_ctx* ctx, pd_coarse_form form);
/* Steppers of the fine and the coarse propagator (default SBDF2 for both;
   applies to pd_fine_dev / pd_coarse_dev / pd_steps_dev / pd_step_* and
   pd_parareal).  The convolution form of the coarse sweep steps SBDF2 only,
   so a Runge-Kutta coarse propagator runs the FFT form (PD_EINVAL together
   with PD_COARSE_CONV).  Batched instances (pd_batch_*) step SBDF2. */
pd_status pd_set_scheme(pd_ctx* ctx, pd_scheme fine, pd_scheme coarse);

/* Initial field U_0, full layout [3][N][N], host or device memory. */
pd_status pd_set_initial(pd_ctx* ctx, const double* b0);
pd_status pd_set_initial_dev(pd_ctx* ctx, const void* d_b0, void* hip_stream);

/* Seeded initial field (the paper's random initial perturbation, Section 4;
   amplitude and spectral extent are this library's choice): for each
   component and every mode inside the 2/3 box with kx^2 + ky^2 <= kmax^2,
   re and im = amp x a pair of normal deviates, every other mode zero; then
   made solenoidal, b <- b - k (k.b)/|k|^2 with k = (kx, ky, kz).  The
   deviates come from Philox4x32-10 (Salmon et al., SC 2011) keyed by `seed`
   with counter (kx mod 2^32, ky mod 2^32, component, 0), turned into two
   53-bit uniforms u1 = (j1 + 1) 2^-53, u2 = j2 2^-53 (j = (w_a >> 5) 2^26 +
   (w_b >> 6) from words 0,1 and 2,3) and then into re = r cos(2 pi u2),
   im = r sin(2 pi u2), r = sqrt(-2 ln u1) (Box-Muller), in plain IEEE double
   arithmetic with the C library's log, sin and cos: the same bits as any
   implementation of that recipe on the same host.
   pd_seed_field writes the field for grid N and kz to out ([3][N][N]
   complex, interleaved; host memory, caller owned; no device work);
   PD_EINVAL for an invalid N, null out or non-finite arguments.
   pd_seed_initial makes it the context's initial field U_0 (as
   pd_set_initial; needs pd_set_time). */
pd_status pd_seed_field(int N, double kz, uint64_t seed, double amp, double kmax, double* out);
pd_status pd_seed_initial(pd_ctx* ctx, uint64_t seed, double amp, double kmax);

/* Fine propagator F over one slice for `batch` independent fields:
   out[f] = F(in[f]) from time t0[f] (host array) to t0[f] + dT with dt_fine
   (n_f = dT/dt_fine steps; the fine propagator of Section 3).  in and out: device,
   full layout [batch][3][N][N]; they may alias.  Needs pd_set_time. */
pd_status pd_fine_dev(pd_ctx* ctx, const double* t0, int batch, const void* d_in, void* d_out,
                      void* hip_stream);
/* Coarse propagator G over one slice: restrict to the N_coarse box, n_c =
   dT/dt_coarse steps on the N_coarse grid, zero-pad back (Section 4,
   Fourier re-sampling).  Same arguments as pd_fine_dev. */
pd_status pd_coarse_dev(pd_ctx* ctx, const double* t0, int batch, const void* d_in, void* d_out,
                        void* hip_stream);
/* F and G over one slice on host arrays: in, out [batch][3][N][N] complex
   (interleaved re, im; may alias), t0[batch] host.  The same propagators as
   pd_fine_dev / pd_coarse_dev, staged through device memory on the context's
   stream. */
pd_status pd_step_fine(pd_ctx* ctx, const double* t0, int batch, const double* in, double* out);
pd_status pd_step_coarse(pd_ctx* ctx, const double* t0, int batch, const double* in, double* out);
/* Any number of steps of size dt on the fine grid from t0[f] (no slice
   length needed): out = n_steps SBDF steps (first one SBDF1). */
pd_status pd_steps_dev(pd_ctx* ctx, const double* t0, int batch, double dt, int n_steps,
                       const void* d_in, void* d_out, void* hip_stream);

/* For callers that cannot allocate device memory (code under HIP graph
   capture, tight serving loops, harnesses that forbid hipMalloc): the same
   propagation as pd_steps_dev (same kernels and results, arguments and
   errors), with its whole workspace -- compact state, SBDF history, the two
   row buffers, the start times, the box-check flag and, for the Runge-Kutta
   steppers, the stage sums -- in one static device array of 64 MiB per GPU,
   held from library load to process end.  The caller passes inputs and
   outputs; the call allocates nothing.  The workspace needs 96 M (M + N)
   bytes a field (M = 2 floor((N-1)/3) + 1; 192 M^2 more with a Runge-Kutta
   stepper) plus 8 a field and a few hundred bytes; a batch that does not
   fit is PD_EINVAL with the sizes in pd_last_error (with SBDF2 at most 2
   fields at N = 512, 9 at 256, 38 at 128, 151 at 64).
   Every call on a GPU shares that GPU's workspace, which keeps the last
   call's contents: calls that overlap on one GPU (from several threads or
   contexts, or on several streams) race and must not be issued. */
pd_status pd_steps_dev_noalloc(pd_ctx* ctx, const double* t0, int batch, double dt, int n_steps,
                               const void* d_in, void* d_out, void* hip_stream);

/* Parareal (Section 3): initial coarse run, then iterations
   U^k_{n+1} = F(U^{k-1}_n) + (G(U^k_n) - G(U^{k-1}_n)) until
   sigma_k = |U^k_P - U^{k-1}_P|_2 / |U^k_P|_2 <= tol or k = max_iter
   (max_iter <= PD_MAX_ITER; tol = 0 runs exactly max_iter iterations).  Slices
   already converged (n < k - 1 in iteration k) are not recomputed: their
   results are unchanged bitwise.  `rep` may be NULL.  Returns PD_OK,
   PD_NOT_CONVERGED, or PD_EUNSTABLE if a defect sum is not finite. */
pd_status pd_parareal(pd_ctx* ctx, double tol, int max_iter, pd_report* rep);
/* Continue the last pd_parareal (or pd_parareal_continue) of this context
   after the k iterations it completed, from the state it left on the device
   (U^k and, for the plain coarse propagator, G(U^k_n)), as pd_set_slices
   would with that state and k, but without copies: iterations k+1 ..
   max_iter (absolute; max_iter > k) until sigma <= tol.  The iterates, the
   defects and k_con are bitwise those of one uninterrupted call; rep numbers
   iterations absolutely and times only this call.  Lets a long solve run in
   bounded pieces.  PD_ESTATE when there is nothing to continue: no run yet,
   or one of pd_set_problem, pd_set_time, pd_set_precision, pd_set_initial,
   pd_set_slices, pd_set_scheme, pd_set_coarse from the learned to the plain
   propagator, pd_lg_add_parareal_samples since, or the last run ended in
   PD_EUNSTABLE.  Switching from the plain to the learned propagator between
   calls is allowed (its difference form needs only U^k): iterations up to k
   with G, the following ones with the learned one. */
pd_status pd_parareal_continue(pd_ctx* ctx, double tol, int max_iter, pd_report* rep);

/* Order of the work inside pd_parareal with the plain coarse propagator.
   chunks >= 2 (default 2, speculate 2): pipelined -- the serial coarse sweep runs on a stream of its
   own in `chunks` runs of consecutive slices, and the fine sweep of a run of
   slices (on one of two fine streams) starts as soon as the coarse sweep has
   produced its start values, so the fine sweeps of iteration k + 1 overlap
   the coarse sweep of iteration k.  They start before the defect of
   iteration k is known: speculate = 1 every run, 0 all but the last run,
   2 every run unless sigma_{k-1}^2 / sigma_{k-2} <= tol predicts that
   iteration k converges (then none).  When the iteration stops at k, the
   call still waits for fine sweeps already started and discards them.
   chunks 0 or 1: every fine sweep, then the coarse sweep, on the context's
   stream.  Both orders give bitwise the same iterates,
   defects and k_con; the timings in pd_report add kernel times per stream
   (they overlap when pipelined).  The learned coarse propagator (difference
   form) is pipelined the same way, its serial sweep run by run. */
pd_status pd_set_pipeline(pd_ctx* ctx, int chunks, int speculate);

/* Temporal blocking of the batched fine propagator F (Section 3: the fine
   solves of the slices are independent, so their order is free).  group > 0:
   fields are taken in consecutive groups of `group`; each group runs all its
   fine steps before the next group on its stream starts, and the groups are
   dealt round-robin to `streams` streams (1..3: the context's stream and the
   two streams of the pipelined schedule, idle outside it), so a group's
   state, history and row buffer stay in the device's last-level cache
   across its steps instead of streaming through HBM at every step.
   group = 0: off (every step runs over the whole batch); group = -1
   (default): groups of 4 fields on 3 streams at 512^2, of 16 fields on 3
   streams at 256^2, off on smaller grids.  Applies to the multi-launch path (fine sweeps of pd_parareal,
   pd_fine_dev / pd_steps_dev batches, pd_fine_sweep_steps, pd_profile_fine);
   in the pipelined schedule each run of slices is blocked on its own fine
   stream in groups holding about as many fields in flight.  Results are
   bitwise the same as unblocked.  PD_EINVAL for group < -1, or group > 0
   with streams outside [1, 3]. */
pd_status pd_set_fine_blocking(pd_ctx* ctx, int group, int streams);
/* The blocking in effect for the context's slice batch: fields a group (0:
   unblocked) and streams.  PD_ESTATE before pd_set_time. */
pd_status pd_get_fine_blocking(pd_ctx* ctx, int* group, int* streams);

/* Checkpoint and resume.  After k iterations of pd_parareal the whole state
   of the iteration is the slice states U^k_n (pd_get_slices) and, for the
   plain coarse propagator, the coarse values G(U^k_n), n = 0..P-1
   (pd_get_coarse_values, full layout [P][3][N][N]).  pd_set_slices loads
   such a state (U: [P+1][3][N][N]; Gold may be NULL when the learned coarse
   propagator is selected, which needs none); the next pd_parareal then skips
   the initial coarse run and goes on with iteration k + 1 up to max_iter
   (> k), giving bitwise the results of the uninterrupted run.  Fields with
   nonzero coefficients outside the 2/3 box are PD_EINVAL.  pd_set_initial
   cancels a pending resume. */
pd_status pd_get_coarse_values(const pd_ctx* ctx, double* out);
pd_status pd_set_slices(pd_ctx* ctx, const double* U, const double* Gold, int k);

/* Measurement helper: times the fine propagator on the context's slice
   buffers (inputs: the current slice states U_0..U_{P-1}; the results are
   discarded and U is left unchanged).  ms[2] = mean time per fine step of
   one whole fine sweep over all slices as pd_parareal launches it; on the
   multi-launch path ms[0] / ms[1] = mean duration of the column-phase /
   row-phase (SBDF2) kernel over `reps` back-to-back launches on the
   context's stream (0 on the single-workgroup path).  HIP events. */
pd_status pd_profile_fine(pd_ctx* ctx, int reps, double* ms);

/* The batched fine propagator F (Section 3: the fine solves of all slices run
   in parallel) one step at a time, for measurement: runs fine steps
   [step0, step0 + n_steps) of the fine sweep over all n_slices slices on the
   context's working slice buffers, the launches pd_parareal makes (one
   column-phase and one row-phase kernel per step, over the whole batch or,
   with fine blocking in effect, over each group of fields, each group
   running all n_steps steps before the next on its stream; SBDF2 fine
   stepper only, else PD_EINVAL).  step0 = 0 starts the sweep from the current slice
   states U_0..U_{P-1} (U itself is not changed); step0 > 0 continues a sweep
   that the previous call on this context left at step0 (else PD_ESTATE);
   step0 + n_steps <= dT/dt_fine.  Any other call that runs the fine
   propagator on the slices ends the stepwise sweep.  ms (may be NULL):
   ms[0] / ms[1] = summed durations of the column-phase / row-phase kernels
   (-1 when blocked: the groups' kernels overlap), ms[2] = duration of the
   whole n_steps, in milliseconds, from HIP events on the context's stream.
   Returns after the work completes. */
pd_status pd_fine_sweep_steps(pd_ctx* ctx, int step0, int n_steps, double* ms);

/* Working states of the fine propagator for slices [first, first + count),
   full layout [count][3][N][N] in device memory: after pd_fine_sweep_steps
   the slices' states after the steps run so far; after pd_parareal F(U_n) of
   the last fine sweep (for the slices it ran). */
pd_status pd_get_fine_states_dev(const pd_ctx* ctx, int first, int count, void* d_out,
                                 void* hip_stream);

/* Launch-shape autotuner for the fine step's two kernels.  The row-phase
   kernel has variants in values a lane (8 or 4) and waves a workgroup; the
   column-phase kernel in values a lane and columns a workgroup (which sets
   its LDS tile).  pd_autotune times every variant of both on this context's
   slice batch (reps back-to-back launches each, after one warm-up round; the
   inputs are the current slice states, which are left unchanged), selects the
   fastest of each for this context, and returns their indices in
   chosen[0] (rows), chosen[1] (columns) and their mean launch times in ms[0..1]
   (either may be NULL).  With those shapes it then times the fine sweep
   (12 steps of every slice) whole-batch and in the blocked orders of
   pd_set_fine_blocking (groups of 1 to 32 fields on 2 or 3 streams) and keeps
   the fastest as this context's blocking (pd_get_fine_blocking; a later
   pd_set_fine_blocking overrides it).  The choice belongs to this context (it applies to
   its fine propagator calls, sweeps and pd_parareal until the next
   pd_set_problem); other contexts keep theirs.  With cache_path non-NULL the choice is first looked
   up in that JSON file (key "<gfx arch>|hip<runtime version>|<N>|<n_slices>",
   value [rows, cols, group, streams]; ms = 0 on a hit) and stored there
   after timing.  Variants give identical results bitwise only
   with equal values a lane; all agree with the oracle to the parity bar. */
pd_status pd_autotune(pd_ctx* ctx, int reps, const char* cache_path, int* chosen, double* ms);
/* Variant table: v = -1 puts the number of variants of `kind` (0 rows,
   1 columns) for grid N in *a; v >= 0 describes variant v (rows: *a values a
   lane, *b waves a workgroup, negative for the form that loads a row's state
   and history with the row, 3 for the form with one row a workgroup and its
   three components on three waves; columns: *a values a lane, *b columns a
   workgroup, negative for the persistent form). */
pd_status pd_variant_info(int N, int kind, int v, int* a, int* b);
/* Select the process-wide default launch-shape variants for grid N (0, 0 =
   defaults), used by contexts and batches that were not autotuned. */
pd_status pd_select_variant(int N, int rows_v, int cols_v);

/* Slice-boundary states U_n, n = 0..n_slices, full layout [P+1][3][N][N]. */
pd_status pd_get_slices(const pd_ctx* ctx, double* out);
pd_status pd_get_slices_dev(const pd_ctx* ctx, void* d_out, void* hip_stream);

/* |U_n|_2 for n = 0..n_slices (host array of n_slices + 1 doubles). */
pd_status pd_slice_norms(const pd_ctx* ctx, double* norms);
/* Amplitude growth rate: least-squares slope of ln|U_n|_2 against t_n over
   n = ceil(P/2) .. P of the current iterate (the paper's Table 1 reports
   growth rates without naming an estimator; this is the reading used). */
pd_status pd_growth_rate(const pd_ctx* ctx, double* gamma);

/* ---- Learned coarse propagator --------------------------------------------
 * The Parareal coarse propagator G (Section 3) may be replaced by
 *   G_learned(D) = G(D) + |D| Net(D/|D|, G(D)/|D|; t_n),
 * G the plain coarse step of this context and Net a small linear spectral
 * neural operator on the fine 2/3 box (lift of the 12 real inputs a mode to
 * 32 channels; `layers` residual layers mixing channels over the mode and its
 * four neighbours with weights V_{l,0,s} + cos t_n V_{l,1,s} + sin t_n V_{l,2,s}
 * and per-mode channel gains; projection to 3 complex values a mode).  It is
 * trained on pairs (D, F(D) - G(D)) that the library's own fine and coarse
 * propagators generate, with BF16 matrix-core (MFMA, FP32 accumulate)
 * forward and backward kernels and Adam on FP32 master weights.  Parareal
 * then runs in difference form U^k_{n+1} = F(U^{k-1}_n) + G_learned(U^k_n -
 * U^{k-1}_n), the same iteration for a linear coarse propagator; G_learned(0)
 * = 0, so converged slices stay bitwise equal to F.  The state belongs to the
 * context and is dropped by pd_set_problem / pd_set_time. */

/* Create the network (layers in [1, 8]) with seeded initial weights. */
pd_status pd_lg_init(pd_ctx* ctx, int layers, uint64_t seed);
/* Add n training samples: device fields D (full layout [n][3][N][N]) and
   slice start times t0 (host); the library computes F(D) and G(D). */
pd_status pd_lg_add_samples(pd_ctx* ctx, int n, const double* t0, const void* d_D,
                            void* hip_stream);
/* Add the fields the coarse propagator sees in a plain-G Parareal run from
   the context's initial field: U^0_n (n < P) of the initial coarse run and
   U^k_n - U^{k-1}_n (k <= n < P) after each of `iters` iterations, each with
   its slice start time; *n_stored (may be null) receives the number of
   stored samples afterwards, the new ones last.  Leaves the context's slice
   states at that run's last iterate (set the initial field again before
   pd_parareal).  iters must be in [0, n_slices). */
pd_status pd_lg_add_parareal_samples(pd_ctx* ctx, int iters, int* n_stored);
/* `steps` Adam steps (learning rate lr) on batches of `batch` distinct
   samples from the stored range [first, first + count), drawn with a seeded
   splitmix64 stream; loss = sum |c - r|^2 / sum |r|^2 with
   r = (F(D) - G(D))/|D|; losses[steps] (may be NULL) receives each step's
   batch loss. */
pd_status pd_lg_train(pd_ctx* ctx, int first, int count, int steps, int batch, double lr,
                      uint64_t seed, double* losses);
/* Add n training samples given directly as network inputs and targets (host
   arrays: features x[n][Q][12], targets r[n][Q][6], slice start times t[n];
   Q = (2K+1)^2 box modes, the order and scaling pd_lg_sample reports).
   *n_stored (may be NULL) receives the number of stored samples. */
pd_status pd_lg_add_feature_samples(pd_ctx* ctx, int n, const float* x, const float* r,
                                    const double* t, int* n_stored);
/* Operand type of the network's matrix-core products: 0 (default) BF16,
   the FP32 activations and weights rounded to nearest even at the operand
   (v_mfma_f32_16x16x16_bf16); 1 FP32 operands unrounded
   (v_mfma_f32_16x16x4_f32), a test mode that isolates the kernels' own
   arithmetic from BF16 rounding.  Both accumulate in FP32.  Applies to every
   later forward, gradient, training and learned-sweep call on ctx. */
pd_status pd_lg_set_operands(pd_ctx* ctx, int fp32);
/* Loss over stored samples [first, first + count). */
pd_status pd_lg_loss(pd_ctx* ctx, int first, int count, double* loss);
/* Gradient of the loss over samples [first, first + count) with respect to
   the flat parameter vector (float[n] as pd_lg_params), and the loss. */
pd_status pd_lg_gradients(pd_ctx* ctx, int first, int count, float* grads, double* loss);
/* Flat FP32 parameters W_in[12][32] | V[L][3][5][32][32] | gamma[L][Q][32] |
   W_out[32][6] (Q = (2K+1)^2): with out NULL *n receives the count. */
pd_status pd_lg_params(pd_ctx* ctx, float* out, size_t* n);
pd_status pd_lg_set_params(pd_ctx* ctx, const float* in, size_t n);
/* Stored sample i: features x[Q][12], targets r[Q][6], slice time t. */
pd_status pd_lg_sample(pd_ctx* ctx, int i, float* x, float* r, double* t);
/* Network output c[Q][6] on stored sample i. */
pd_status pd_lg_forward_sample(pd_ctx* ctx, int i, float* out);
/* Weight the training loss per box mode by w_m = exp(-beta |k_m|^2 dT / Rm),
   the damping diffusion alone applies to mode m over beta slices, so that
   the network spends its accuracy on the modes that persist from slice to
   slice (loss = sum w |c - r|^2 / sum w |r|^2).  beta = 0 (the default):
   uniform weights. */
pd_status pd_lg_set_loss_decay(pd_ctx* ctx, double beta);
/* Use the learned (1) or plain (0) coarse propagator in pd_parareal. */
pd_status pd_set_coarse(pd_ctx* ctx, int learned);
/* Save the network parameters to a file (8-byte magic "PDLGNET1", int32 N,
   box width, layers, channels, uint64 count, FP32 values in the order of
   pd_lg_params), or load such a file into a context with the same N (the
   network is created with the file's layer count; stored samples and the
   optimizer state are dropped).  PD_EINVAL on a file that does not match. */
pd_status pd_lg_save(const pd_ctx* ctx, const char* path);
pd_status pd_lg_load(pd_ctx* ctx, const char* path);

/* ---- Many independent problems in one batch -------------------------------
 * Parareal (Section 3) for many (flow, Rm, kz, N) instances of uneven size at
 * once on one GPU.  Instances of equal (flow, N, fine steps per slice) share
 * one batched fine sweep a Parareal iteration; the serial coarse sweeps of all
 * instances run concurrently (one workgroup each, convolution form: the
 * coarse box is held in LDS when N_coarse <= 64 and in global memory above);
 * one iteration of the whole batch is captured once in a HIP graph and
 * replayed.  Each instance stops when its own defect reaches tol. */
typedef struct pd_batch pd_batch;

pd_status pd_batch_create(pd_batch** out, int hip_device);
void pd_batch_destroy(pd_batch* b);
const char* pd_batch_last_error(const pd_batch* b);
/* Add one instance: the arguments of pd_set_problem and pd_set_time plus its
   initial field (host, full layout [3][N][N], copied).  *id receives its
   index.  At most 4096 instances; at most 65535 slices of one grid size. */
pd_status pd_batch_add(pd_batch* b, pd_flow flow, double Rm, double kz, int N, double T,
                       int n_slices, double dt_fine, double dt_coarse, int N_coarse,
                       const double* b0, int* id);
/* Run Parareal on every instance from its initial field until its sigma <=
   tol or max_iter iterations (tol = 0: exactly max_iter).  use_graph != 0
   replays one captured HIP graph per iteration; 0 launches eagerly (same
   kernels, same results).  PD_NOT_CONVERGED if some instance did not reach
   tol; PD_EUNSTABLE if some instance went non-finite. */
pd_status pd_batch_run(pd_batch* b, double tol, int max_iter, int use_graph);
/* Report of one instance (k_con, sigma history; t_total_s is the whole
   batch's wall clock) and its growth rate (as pd_growth_rate; gamma may be
   NULL). */
pd_status pd_batch_result(const pd_batch* b, int id, pd_report* rep, double* gamma);
/* Slice states U_n of one instance, full layout [P+1][3][N][N], host. */
pd_status pd_batch_get_slices(const pd_batch* b, int id, double* out);
/* Wall-clock seconds of the last pd_batch_run. */
pd_status pd_batch_time(const pd_batch* b, double* seconds);

#ifdef __cplusplus
}
#endif
#endif /* PITDYN_H */
