/*
 * wavepacket.h -- C ABI of libwavepacket, a split-operator solver of the
 * time-dependent Schroedinger equation for one AMD Instinct MI355X (gfx950).
 *
 * Method: Dion, Hashemloo, Rahali, "Program for quantum wave-packet dynamics
 * with time-dependent potentials", Comput. Phys. Commun.  Section 2.1 gives
 * the Hamiltonian H = P^2/2m + V(x,t) (eqs. tdse, hamiltonian), the
 * short-time propagator (eq. short-time), its split form (eq. splitop), the
 * grid (eqs. grid, Deltax), the FFT diagonalisation of the kinetic operator
 * (eq. ft) and the momentum grid; Section 3.2 the user interface this ABI
 * replaces (struct `parameters`, `potential`, `initialize_wf`, `norm`,
 * `expectation1D`, `integrate3D`); Table 3 the observables.
 *
 * One time step, in the default order, is
 *     psi <- exp(-i V(x,t_n+1) dt/2hbar) F^-1 exp(-i hbar|k|^2 dt/2m) F
 *            exp(-i V(x,t_n) dt/2hbar) psi,        t_n = t0 + n dt,
 * the Strang splitting with the potential integral of eq. short-time taken by
 * the trapezoid rule.  Consecutive equal-time potential halves are merged on
 * the device; the result equals the unmerged product up to rounding.
 *
 * Conventions shared by every entry point
 *   - Grid: axis d has n[d] >= 2 points (see wp_create for the supported
 *     lengths) on the half-open interval [lo[d], hi[d]) with spacing
 *     (hi-lo)/n and x_i = lo + i*spacing.  DFT bin m holds the wavenumber
 *     2 pi m'/(hi-lo) with m' = m for 2m < n and m - n otherwise.
 *     1D problems lie along x and 2D problems in the xy-plane (Section 2.2);
 *     unused axes have n = 1.  Boundaries are periodic.
 *   - State psi: row-major [n0][n1][n2] (last axis contiguous), interleaved
 *     (re, im).  WP_C128 stores two doubles per point, WP_C64 and WP_C64X
 *     two floats.  In device memory the planes of the first axis start
 *     wp_state_pitch points apart: n1*n2, except on 3D grids whose lengths
 *     are all powers of two, where 16 unused points follow every plane (so
 *     that a first-axis line does not meet the memory at one power-of-two
 *     stride).  Host buffers are always contiguous.
 *     The FP32 path keeps phase arguments, coordinates, time and every
 *     reduction in FP64 and multiplies by FP64-accurate factors.
 *   - Streams: all device work of a handle is ordered on the HIP stream
 *     given at creation (NULL = the default stream).  Calls marked
 *     "synchronises" wait for that stream before returning.
 *   - Ownership: host buffers passed in are read or written during the call
 *     only and stay owned by the caller.  Device buffers are owned by the
 *     library unless bound with wp_bind_state.
 *   - Errors: functions return a wp_status and never abort the process (the
 *     paper's `abort` of Section 3.2 has no counterpart).  On failure the
 *     handle keeps its previous state and wp_last_error describes the cause.
 *   - Threads: a handle is not thread-safe; distinct handles are independent.
 */
#ifndef WAVEPACKET_H
#define WAVEPACKET_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  WP_OK = 0,
  WP_EINVAL = -1,       /* invalid argument or descriptor                     */
  WP_ENOMEM = -2,       /* device or host allocation failed                   */
  WP_EDEVICE = -3,      /* a HIP call failed                                  */
  WP_EUNSUPPORTED = -4, /* valid input outside what this build implements     */
  WP_ESTATE = -5        /* call not allowed in the handle's current state     */
} wp_status;

/* WP_C64: FP32 state; FFT additions in FP32, every multiply by a twiddle or
 *   phase factor done with the FP64 factor and rounded once.
 * WP_C64X: FP32 state; all arithmetic of a pass in FP64, rounded to FP32
 *   when the pass stores the state.
 * WP_C128: FP64 state and arithmetic. */
typedef enum { WP_C64 = 1, WP_C128 = 2, WP_C64X = 3 } wp_precision;

/* Operator order of a step.  WP_ORDER_VKV is the default described above.
 * WP_ORDER_KVK is eq. splitop as printed: kinetic half step, potential at the
 * midpoint t_n + dt/2 over a full step, kinetic half step. */
typedef enum { WP_ORDER_VKV = 0, WP_ORDER_KVK = 1 } wp_order;

/* Scalar waveform f(t). */
typedef enum {
  WP_WAVE_CONST = 0,     /* A0                                                 */
  WP_WAVE_SIN = 1,       /* A0 + A1 sin(omega t + phase)                       */
  WP_WAVE_COS = 2,       /* A0 + A1 cos(omega t + phase)                       */
  WP_WAVE_GAUSS_COS = 3, /* A0 + A1 exp(-((t - tc)/tau)^2) cos(omega t + phase) */
  WP_WAVE_SIN2_COS = 4   /* A0 + A1 sin^2(pi (t-ti)/(tf-ti)) cos(omega t+phase) */
                         /* on ti <= t <= tf, A0 elsewhere (the pulse of        */
                         /* Section 4.1)                                        */
} wp_wave_kind;

typedef enum {
  WP_V0_NONE = 0,
  WP_V0_SOFTCORE = 1, /* -Z / sqrt(r^2 + eps2), r^2 over the used axes; par = {Z, eps2} */
  WP_V0_MORSE = 2     /* D (1 - exp(-a (x - xe)))^2 along x (Section 4.1); par = {D, a, xe} */
} wp_v0_kind;

typedef struct {
  int32_t kind; /* wp_wave_kind */
  double A0, A1, omega, phase, tc, tau, ti, tf;
} wp_waveform;

/* Grid and physical constants (the grid, mass, dt and hbar fields of the
 * paper's struct `parameters`, Section 3.2.1).  dt may be negative. */
typedef struct {
  int32_t ndim; /* 1, 2 or 3 */
  int32_t prec; /* wp_precision of the device state */
  uint64_t n[3];
  double lo[3], hi[3];
  double mass, hbar, dt;
} wp_grid_desc;

/* Potential family evaluated on the device at every step (replaces the user
 * function `potential`, Section 3.2.3):
 *   V(x,t) = c(t) + sum_d [a_d(t) x_d + b_d(t) x_d^2] + s(t) V0(x).
 * Terms on unused axes are ignored.  This family holds every potential of
 * Section 4 (Morse plus linear dipole coupling; the Paul trap quadrupole). */
typedef struct {
  wp_waveform a[3], b[3], c, s;
  int32_t v0_kind; /* wp_v0_kind */
  double v0_par[4];
} wp_potential_desc;

typedef struct wp_sim wp_sim;

/* Bit mask of wp_observables; out[i] belongs to bit i. */
enum {
  WP_OBS_NORM = 1u << 0,   /* sqrt(<psi|psi>)               (`norm`)          */
  WP_OBS_X = 1u << 1,      /* <psi|x|psi>, not normalised    (`expectation1D`) */
  WP_OBS_Y = 1u << 2,
  WP_OBS_Z = 1u << 3,
  WP_OBS_X2 = 1u << 4,     /* <psi|x^2|psi>                                    */
  WP_OBS_Y2 = 1u << 5,
  WP_OBS_Z2 = 1u << 6,
  WP_OBS_ENERGY = 1u << 7, /* <psi|K + V(t)|psi>, K spectral (Table 3 energy)  */
  WP_OBS_ALL = 0xffu,
  WP_OBS_SX = 1u << 8,     /* width <x^2> - <x>^2 (Table 3 sx; unnormalised)   */
  WP_OBS_SY = 1u << 9,
  WP_OBS_SZ = 1u << 10,
  WP_OBS_AUTOCORR = 1u << 11, /* |<psi_ref|psi>|^2 (Table 3 autocorrelation);
                                 needs wp_store_reference                     */
  WP_OBS_ALL_EXT = 0xfffu
};

/* Device bytes of the state for this grid (n0 * pitch * 8 or 16, pitch as
 * wp_state_pitch reports it).  WP_EINVAL for an invalid descriptor. */
wp_status wp_state_bytes(const wp_grid_desc *grid, uint64_t *bytes);

/* Points between the starts of consecutive first-axis planes of the state
 * in device memory (*pitch >= n1*n2; point (i0, i1, i2) is at
 * i0*pitch + i1*n2 + i2).  The points after each plane's n1*n2 are never
 * read or written.  WP_EINVAL for an invalid descriptor or NULL. */
wp_status wp_state_pitch(const wp_grid_desc *grid, uint64_t *pitch);

/* Device bytes wp_create allocates for this grid in total, state included
 * (state, per-axis kinetic and twiddle tables).  An energy request later
 * adds one more state-sized scratch buffer.  Used for admission by HBM
 * budget (the memory estimate of Section 3.5). */
wp_status wp_workspace_bytes(const wp_grid_desc *grid, uint64_t *bytes);

/* Create a solver on the current HIP device for the grid and potential (the
 * set-up of `initialize_potential`, Section 3.2.2).  `stream` is a
 * hipStream_t or NULL.  The state is zero and the time 0 until a set_state
 * call; the state buffer itself is allocated on first use unless one is
 * bound with wp_bind_state (if it does not fit in device memory, that first
 * call returns WP_ENOMEM and the handle stays valid: bind memory or
 * destroy it).  Axis lengths: powers of two (the fast
 * kernels), or on grids where some length is not a power of two, lengths
 * with prime factors 2, 3, 5 and 7 only (the sizes Section 3.2.1 advises
 * for nx, ny, nz of struct `parameters`),
 * transformed by mixed-radix kernels in FP64 arithmetic.  Errors: WP_EINVAL
 * (bad descriptor: ndim not in 1..3, n < 2 on a used axis, n != 1 on an
 * unused axis, hi <= lo, mass <= 0, hbar <= 0, dt = 0 or not finite,
 * unknown kinds), WP_EUNSUPPORTED (a length this build does not transform:
 * powers of two above 2^20 points in 1D, where grids above 8192 points are
 * transformed as [n1][n2] with twiddles in between, or above 4096 per axis
 * in 2D/3D; other lengths with a prime factor above 7 or above 4096
 * points), WP_ENOMEM, WP_EDEVICE.  On success *out owns all device
 * buffers. */
wp_status wp_create(const wp_grid_desc *grid, const wp_potential_desc *pot, void *stream,
                    wp_sim **out);

/* Release every library-owned buffer.  Waits for the handle's stream. */
wp_status wp_destroy(wp_sim *sim);

/* Use caller-owned device memory `dev_psi` (at least wp_state_bytes, 16-byte
 * aligned; planes wp_state_pitch points apart) as the state from now on;
 * work queued afterwards uses it.  A
 * state buffer the library allocated before is freed after waiting for the
 * handle's stream (only then does the call synchronise).  The caller keeps
 * ownership and must keep the memory alive until wp_destroy.  The content
 * is not changed.  Errors: WP_EINVAL (NULL, too small or misaligned). */
wp_status wp_bind_state(wp_sim *sim, void *dev_psi, uint64_t bytes);

/* Device pointer of the current state (library-owned or bound), laid out
 * with the plane pitch of wp_state_pitch. */
void *wp_state_ptr(wp_sim *sim);

/* Copy a host state (row-major, complex128, n0*n1*n2 points) to the device,
 * converting to the handle's precision, and set the time origin: after this
 * call the state is psi(t0) and the step counter is 0 (the role of
 * `initialize_wf`, Section 3.2.4).  An FP32 state is converted on the
 * device, through a staging buffer of at most 64 MiB that the call
 * allocates and frees.  Synchronises.  Errors: WP_EINVAL (NULL, t0 not
 * finite), WP_ENOMEM, WP_EDEVICE. */
wp_status wp_set_state(wp_sim *sim, const double *host_psi_c128, double t0);

/* Set psi(t0) to the Gaussian of Section 4.2,
 *   prod_d (2/pi)^(1/4) sigma_d^(-1/2) exp(-(x_d-c_d)^2/sigma_d^2 + i k_d (x_d-c_d)),
 * renormalised to unit discrete norm (k_d = p_d0/hbar).  Arrays hold one
 * entry per axis (3 entries; unused axes ignored).  sigma_d must be > 0.
 * Asynchronous on the handle's stream (the arrays may be reused on return). */
wp_status wp_set_state_gaussian(wp_sim *sim, const double center[3], const double sigma[3],
                                const double k[3], double t0);

/* Advance the state by nsteps steps of dt (Algorithm 1's inner loop with
 * merged equal-time potential halves).  Asynchronous on the handle's stream;
 * nsteps = 0 is a no-op.  The step counter advances by nsteps. */
wp_status wp_propagate(wp_sim *sim, uint64_t nsteps);

/* Select the operator order used by later wp_propagate calls (default
 * WP_ORDER_VKV).  WP_EINVAL for an unknown order. */
wp_status wp_set_order(wp_sim *sim, int32_t order);

/* Copy the state at the current time to host memory as interleaved
 * complex128 (as_prec = WP_C128) or complex64 (WP_C64; WP_C64X is not a
 * valid output format), row-major, n0*n1*n2 points.  In the other
 * precision than the stored state's the conversion runs on the device,
 * through a staging buffer of at most 64 MiB that the call allocates and
 * frees.  Synchronises.  Errors: WP_EINVAL, WP_ENOMEM, WP_EDEVICE. */
wp_status wp_get_state(wp_sim *sim, void *host_out, int32_t as_prec);

/* FP64 observables of the current state at the current time (Table 3 and
 * the `norm` / `expectation1D` utilities of Section 3.2.6): writes out[i]
 * for bit i of the WP_OBS_* mask, for every i up to the highest bit set
 * (8 values for masks within WP_OBS_ALL, 12 with the width or
 * autocorrelation bits); entries not in `mask` are 0.  Integrals use the
 * rectangle rule over the periodic cell.  Deterministic (fixed reduction
 * order).  Synchronises.  WP_ESTATE: WP_OBS_AUTOCORR without a stored
 * reference. */
wp_status wp_observables(wp_sim *sim, uint32_t mask, double *out);

/* Propagate nsteps steps (as wp_propagate) and return the observables of
 * the final state in out (as wp_observables(sim, mask, out) would): the
 * algorithm's observables every nprint steps (Algorithm 1, Section 3.2.6).
 * Norm, <x_d>, <x_d^2> and the widths are accumulated in FP64 by the pass
 * that ends the propagation, from the values it stores, with no further
 * read of the state, on power-of-two 2D and 3D grids in the WP_ORDER_VKV
 * order; other masks, orders and grids run wp_propagate and then
 * wp_observables.  Sums in a fixed order (deterministic; equal to
 * wp_observables up to the order of summation).  Allocates one buffer of
 * 64 bytes per workgroup of that pass on first use.  Synchronises.
 * WP_EINVAL: NULL out or nsteps not in 1..2^40; otherwise the errors of
 * wp_propagate and wp_observables. */
wp_status wp_propagate_observe(wp_sim *sim, uint64_t nsteps, uint32_t mask, double *out);

/* For callers that cannot allocate device memory (tight serving loops and
 * harnesses that forbid hipMalloc/hipFree after set-up): wp_propagate_observe
 * without any allocation.  The closing pass writes its moment rows (8
 * doubles per workgroup) to a fixed array of WP_NOALLOC_MOMENT_ROWS rows
 * (4 MiB) that the library's code object holds on every device it runs on
 * until the process ends, instead of a buffer allocated on first use; the
 * slabs of a 3D step run on the handle's stream alone while its second
 * stream has not been created by an earlier propagation.  Results equal
 * wp_propagate_observe's bit for bit.  Only the fused case: a power-of-two
 * 2D or 3D grid in the WP_ORDER_VKV order and a mask within norm, <x_d>,
 * <x_d^2> and the widths.  All calls on one device share that array: calls
 * that overlap in time on one device (different host threads, or handles
 * on different streams without ordering between them) race and must be
 * serialised by the caller.  Synchronises.  Errors: WP_EINVAL (NULL out,
 * nsteps not in 1..2^40), WP_EUNSUPPORTED (another grid, order or mask;
 * a closing pass of more than WP_NOALLOC_MOMENT_ROWS workgroups, e.g. a
 * first axis of 512 points with more than 2^20 lines across it in FP32),
 * WP_ESTATE (no state set or bound yet: allocating it is not allowed
 * here), WP_EDEVICE. */
#define WP_NOALLOC_MOMENT_ROWS 65536
wp_status wp_propagate_observe_noalloc(wp_sim *sim, uint64_t nsteps, uint32_t mask, double *out);

/* Keep a device copy of the current state as the reference of
 * WP_OBS_AUTOCORR (the initial wave function the autocorrelation of
 * Table 3 compares with; Section 3.5 counts its memory).  Allocates one more
 * state-sized buffer on first use; ordered on the handle's stream. */
wp_status wp_store_reference(wp_sim *sim);

/* <phi|psi> = sum conj(phi) psi dV over the grid (`integrate3D` of Section
 * 3.2.6 with f1 = phi, f2 = the current state; the projection onto a
 * given state of Section 3.2.5).  dev_phi: device memory holding the n0*n1*n2
 * points contiguously in row-major order (no plane padding), WP_C64
 * (complex64) or WP_C128 (complex128) per phi_prec, caller-owned and only
 * read.  out[0], out[1]: real and imaginary part.
 * FP64 deterministic reduction.  Synchronises.  WP_EINVAL: NULL pointer or
 * bad precision. */
wp_status wp_inner(wp_sim *sim, const void *dev_phi, int32_t phi_prec, double *out);

/* Kernel classes of a propagation, for wp_profile_propagate. */
enum {
  WP_PASS_SOLVE1D = 0,  /* whole 1D solve in one workgroup                    */
  WP_PASS_AXIS0 = 1,    /* first axis: inverse FFT, potential phase, FFT       */
  WP_PASS_MID_FWD = 2,  /* middle axis (3D): forward FFT                       */
  WP_PASS_LAST = 3,     /* last axis: FFT, kinetic phase, inverse FFT          */
  WP_PASS_MID_INV = 4,  /* middle axis (3D): inverse FFT                       */
  WP_PASS_EDGE = 5,     /* first-axis pass opening or closing a propagation    */
  WP_PASS_COEF = 6,     /* waveform values of the potential for a run of steps */
  WP_PASS_KINDS = 7
};

/* Same work as wp_propagate(sim, nsteps) (the state advances identically),
 * timing every kernel launch of the classes in `kinds` (bit k for class k;
 * 0xffffffff for all) with a HIP event pair attached to that dispatch
 * (hipExtLaunchKernel: the events take the kernel's own start and end
 * times, and nothing is enqueued between kernels); other launches run as in
 * wp_propagate.  On return ms[k] holds the summed device time
 * (milliseconds) and count[k] the number of timed launches of class k, for
 * k < WP_PASS_KINDS (arrays of at least WP_PASS_KINDS entries,
 * caller-owned).  Synchronises.  nsteps must be in 1..100000 (WP_EINVAL
 * otherwise). */
wp_status wp_profile_propagate(wp_sim *sim, uint64_t nsteps, uint32_t kinds, double *ms, uint64_t *count);

/* Device time of one line-pass class of a 2D/3D (or split 1D) step: the
 * pass of class `kind` (WP_PASS_AXIS0, _MID_FWD, _LAST, _MID_INV or _EDGE,
 * as launched by wp_propagate at the current step) is launched `reps` times
 * back to back on the handle's stream between one event pair; *ms receives
 * the average per launch.  Measurement only: the state is transformed
 * `reps` times and is not a solution afterwards (the step counter is
 * unchanged).  Synchronises.  WP_EINVAL: reps not in 1..10000, a kind the
 * grid does not have (e.g. a middle axis in 2D, any pass of a 1D grid
 * solved in one workgroup). */
wp_status wp_time_pass(wp_sim *sim, int32_t kind, uint32_t reps, double *ms);

/* ---- Autotuner -------------------------------------------------------
 * Every line pass exists in up to WP_TUNE_VARIANTS compiled shapes
 * (variant bit 0: 8 instead of 16 values per thread in FP32 passes; bit 1:
 * 256-thread workgroups, three per CU, instead of 512-thread ones, two per
 * CU; variants beyond 0 exist for line lengths 64..1024 and pass kinds F,
 * V, K; FP64 passes have variants 0 and 2).  A process-wide table holds the
 * variant per (batched, precision, log2 line length, strided layout, pass
 * kind: 0 FFT, 1 potential, 2 kinetic, 3/4 split 1D potential/kinetic);
 * entries never tuned run variant 0.  Results do not depend on the variant
 * (the same arithmetic in the same order), only the speed does. */
#define WP_TUNE_VARIANTS 4
#define WP_TUNE_SLAB_CHOICES 8

/* Tune the handle's line passes ([0] potential pass of the first axis, [1]
 * middle-axis FFT (3D), [2] kinetic pass of the last axis) on a device copy
 * of the state (the state itself is unchanged; one state-sized scratch
 * buffer is allocated on first use): first every variant of each class over
 * `reps` back-to-back launches on the whole grid, the fastest stored in the
 * table; on 3D power-of-two grids then whole steps with 1, 2, 4, ... x slabs
 * (see wp_set_slabs), the fastest count kept for this handle; last, for each
 * class in turn, whole steps with each of its variants (the others at their
 * chosen ones), the fastest stored.  ms, if not NULL, receives 3 x
 * WP_TUNE_VARIANTS milliseconds per step of that last round (class-major)
 * followed by WP_TUNE_SLAB_CHOICES milliseconds per step for 2^0 .. 2^7
 * slabs (NaN where not tried).  Passes built afterwards by any handle use
 * the table; a 1D grid solved in one workgroup and mixed-length grids have
 * nothing to tune (WP_OK).  Synchronises.  WP_EINVAL: reps not in
 * 1..10000. */
wp_status wp_autotune(wp_sim *sim, uint32_t reps, double *ms);

/* 3D power-of-two grids: run the middle passes of a step (forward FFT of
 * the middle axis, kinetic pass of the last axis, inverse FFT of the
 * middle axis) on `count` slabs of consecutive x planes, so that a slab
 * stays in the GPU's memory-side cache between its three passes and only
 * the first pass reads it from HBM.  With more than one slab, even slabs
 * run on the handle's stream and odd ones on a second stream the library
 * creates for the handle (default priority), forked from and joined back
 * to the handle's stream by events around the middle of every step, so
 * that work queued on the handle's stream still sees the whole step.  The
 * arithmetic is the same (results are bit-identical for every count).
 * count: a power of two up to n0; 1 for other grids.  The default keeps
 * slabs at most 128 MiB (two in flight fit the cache).  WP_EINVAL
 * otherwise. */
wp_status wp_set_slabs(wp_sim *sim, uint32_t count);
/* The handle's slab count (0 for a NULL handle). */
uint32_t wp_get_slabs(const wp_sim *sim);

/* The table entry for one pass shape (see above); *tune receives 0 for
 * shapes never tuned. */
wp_status wp_tune_get(int32_t batched, int32_t prec, int32_t lg_n, int32_t strided, int32_t kind,
                      int32_t *tune);
/* Set a table entry (for example from a saved tuning run).  WP_EINVAL for
 * a value out of range.  Takes effect for passes built afterwards. */
wp_status wp_tune_set(int32_t batched, int32_t prec, int32_t lg_n, int32_t strided, int32_t kind,
                      int32_t tune);
/* Forget every table entry. */
void wp_tune_clear(void);

/* ---- batches: many independent solves advanced together -------------- */

typedef struct wp_batch wp_batch;

/* Group `count` existing handles so that wp_batch_propagate advances all of
 * them with shared launches: every pass of a step is one launch per class of
 * solves with the same precision, line length and layout, each workgroup
 * taking one tile of one solve (the per-solve work of Algorithm 1, many
 * solves at once).  Solves may differ in size, dimension, potential,
 * precision, dt and start time; all must use WP_ORDER_VKV and be on the
 * current device.  The batch refers to the handles (it does not own them):
 * they must outlive it, and while it exists they should be advanced only
 * through it.  Work is ordered on `stream` (hipStream_t or NULL).  Each
 * member's result equals its own wp_propagate result (same kernels, same
 * reduction order).  Members on grids with a length that is not a power of
 * two are not grouped: each takes the launches wp_propagate would make,
 * within the batch's work.  The batch's work is ordered on `stream` only:
 * work queued on members' own streams must be complete or on the same
 * stream.  Errors: WP_EINVAL (count 0, NULL, a member in K-V-K order),
 * WP_ENOMEM, WP_EDEVICE. */
wp_status wp_batch_create(wp_sim *const *sims, uint32_t count, void *stream, wp_batch **out);

/* Capture runs of k steady steps (1 <= k <= 64) of the 2D/3D members in a
 * HIP graph and replay it; k = 0 launches directly.  Default 0.  The graph
 * refreshes the waveform values from device step counters, so replays need
 * no host updates.  Results do not depend on k. */
wp_status wp_batch_set_graph_steps(wp_batch *b, uint32_t k);

/* Advance every member by nsteps (asynchronous on the batch's stream).  Each
 * member's state, step counter and time advance exactly as with
 * wp_propagate(member, nsteps), bit for bit. */
wp_status wp_batch_propagate(wp_batch *b, uint64_t nsteps);

/* Tune the batched kernels: every pass group of the batch (same
 * precision, line length, layout and kind) is timed in each variant over
 * `reps` back-to-back launches on the members' states, which are saved to
 * per-member scratch buffers (allocated on first use) and restored; the
 * fastest variants go into the table (batched entries) and the batch's
 * block maps are rebuilt for them (a captured graph is captured again at
 * the next propagation).  Synchronises the batch's stream.  WP_EINVAL: reps
 * not in 1..10000. */
wp_status wp_batch_autotune(wp_batch *b, uint32_t reps);

/* Release the batch's own device buffers and graphs (members untouched).
 * Waits for the batch's stream. */
wp_status wp_batch_destroy(wp_batch *b);

/* Description of the last error on the batch ("" when none). */
const char *wp_batch_last_error(const wp_batch *b);

/* Current time t0 + steps*dt and step counter. */
wp_status wp_get_time(wp_sim *sim, double *t, uint64_t *step);

/* Wait for all work queued by this handle. */
wp_status wp_synchronize(wp_sim *sim);

/* Human-readable description of the last error on this handle (never NULL;
 * "" when none).  Valid until the next call on the handle. */
const char *wp_last_error(const wp_sim *sim);

/* Library version string. */
const char *wp_version(void);

#ifdef __cplusplus
}
#endif
#endif
