/*
 * osht.h -- C ABI of the MI355X implementation of the forward and inverse
 * spherical harmonic transform on the optimal-dimensionality L^2-sample
 * scheme of Khalid, Kennedy & McEwen (IEEE TSP 2014).
 *
 * Geometry (Sec. III-A): L iso-latitude rings; ring k (k = 0..L-1) sits at
 * colatitude theta_k = pi n_k / (2L-1), n_k an odd integer numerator
 * (Eq. equiangular_set), and carries 2k+1 samples at phi_j = 2 pi j/(2k+1).
 * The sample vector of one map therefore has exactly L^2 entries
 * (Eq. number_samples_sum), as does the coefficient vector.
 *
 * Array layouts (all arrays are complex128, interleaved re/im doubles):
 *   samples       f[b * L*L + k*k + j]          ring-major, j = 0..2k
 *   coefficients  flm[b * L*L + l*l + l + m]     l-major, 0 <= l < L, |m| <= l
 * b = 0..batch-1 indexes maps.  For spin s, coefficients with l < |s| do not
 * exist: inputs must hold zeros there and outputs are written as zeros.
 *
 * Ownership: a plan owns all of its device memory (placement, Legendre
 * blocks, factorised per-order inverses, workspace) on the HIP device that
 * was current at osht_plan_create.  Transform entry points take caller-owned
 * DEVICE pointers, enqueue work on the given stream and return without
 * synchronising.  Calls on one plan must not overlap in time (the plan's
 * workspace is shared by all of its calls): serialise them on one stream.
 *
 * Errors: every entry point returns OSHT_OK (0) or a negative OSHT_E* code;
 * osht_strerror() gives a message.  Argument errors are detected on the host
 * before any work is enqueued.
 */
#ifndef OSHT_H
#define OSHT_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------------ codes */
#define OSHT_OK            0
#define OSHT_EINVAL       -1  /* bad argument (L, spin, batch, pointer, aliasing) */
#define OSHT_ENOMEM       -2  /* device or host allocation failed */
#define OSHT_EHIP         -3  /* a HIP runtime call failed */
#define OSHT_ESINGULAR    -4  /* a per-order system P_m failed its inversion check */
#define OSHT_ENOTSUP      -5  /* combination of flags not supported */
#define OSHT_EIO          -6  /* placement cache file unreadable or malformed */
#define OSHT_ENONFINITE   -7  /* a transform output held NaN or Inf (OSHT_CHECK_FINITE plans) */

/* ------------------------------------------------------------------ flags */
/* arithmetic of the order-wise apply (Procedure 1 step solve and alias
 * evaluation, Procedure 2 step evaluation, and their adjoints).  The
 * Legendre/Wigner recursion, the inversion of every P_m, the ring DFTs, the
 * alias gathers and every buffer the caller sees stay FP64 in all modes. */
#define OSHT_PREC_FP64        0x0u   /* FP64 throughout */
#define OSHT_PREC_FP32        0x1u   /* A_m built and checked in FP64, stored rounded to FP32 and
                                        applied on FP32 matrix cores (inverse and inverse adjoint):
                                        FP32 accumulation over 16-term k-slices summed in FP64,
                                        right-hand side rounded to FP32 as it is read.  The forward
                                        sweep stays FP64 (its descending-order alias chain amplifies
                                        rounding). */
#define OSHT_PREC_FP32_FWD    0x2u   /* OSHT_PREC_FP32, and the forward's coefficient rows P_m^{-1}
                                        also on FP32 matrix cores; its alias rows A_m^top P_m^{-1}
                                        stay FP64 */
#define OSHT_PREC_I8X6        0x3u   /* inverse apply as exact int8 matrix-core products of 6-digit splits
                                        of A_m (per-ring power-of-two scale) and of the coefficients
                                        (per-column scale), digits of 7 bits: about 2e-10 relative to
                                        max |f| (FP32 operands give ~1e-7), int32 accumulation, scaled and
                                        summed in FP64; the forward as OSHT_PREC_FP32_FWD.  The inverse
                                        adjoint reads FP64 A_m. */
#define OSHT_PREC_I8X8        0x4u   /* as OSHT_PREC_I8X6 with 8 digits (~1e-14, FP64 grade) and the
                                        forward in FP64 */
#define OSHT_PREC_FWD32       0x5u   /* the inverse (and both adjoints) in FP64; the forward's
                                        coefficient rows P_m^{-1} on FP32 matrix cores as in
                                        OSHT_PREC_FP32_FWD, its alias rows in FP64 */
#define OSHT_PREC_MASK        0x0fu
/* colatitude placement (Sec. III-D) */
#define OSHT_THETA_GREEDY       0x00u  /* condition-number-minimising greedy */
#define OSHT_THETA_ALTERNATING  0x10u  /* Eq. sampling_latitude */
#define OSHT_THETA_MASK         0xf0u
/* autotune the forward sweep's block shape (levels per block, columns per
 * delta-solve workgroup) by timing candidates on this device at plan time;
 * the choice is cached in theta_cache_dir as "tune_fwd_<arch>_L<L>_s<s>_p<prec>.txt"
 * when that directory is given */
#define OSHT_TUNE               0x100u
/* run the forward (and forward adjoint) of a spin != 0 plan even when the
 * plan-time self-check found it unstable (see osht_info_t.fwd_check_err);
 * without this flag such calls return OSHT_ENOTSUP */
#define OSHT_SPIN_FWD_FORCE     0x200u
/* every transform of the plan scans its output for NaN / Inf on the device
 * and records a hit in a sticky per-plan status read by osht_plan_status
 * (one extra read of the output, 16 bytes per entry per map; off by
 * default) */
#define OSHT_CHECK_FINITE       0x400u

typedef struct osht_plan osht_plan_t;

typedef struct {
  int32_t  L;
  int32_t  spin;
  uint32_t flags;
  int32_t  fwd_unstable;    /* 1: spin != 0 plan whose forward failed the self-check below
                               (forward calls return OSHT_ENOTSUP unless OSHT_SPIN_FWD_FORCE) */
  int64_t  nsamples;        /* L*L per map */
  int64_t  ncoeffs;         /* L*L per map */
  int64_t  device_bytes;    /* device memory held by the plan */
  double   max_kappa;       /* max over m of the 1-norm condition estimate of P_m */
  double   max_inv_residual;/* max over m of |I - X_m P_m|_max of the stored inverses */
  double   fwd_check_err;   /* plan-time self-check of the forward, in FP64: max |forward(inverse(a)) - a|
                               / max |a| for one fixed pseudo-random band-limited a (entries uniform in
                               [-1, 1] + i[-1, 1], zero for l < |s|).  The forward is exact on band-limited
                               samples, so this measures how the order-by-order chain of Procedure 1
                               amplifies rounding on this plan: ~1e-14 for spin 0 at L <= 512; for spin
                               +-2 it grows from ~1e-11 at L = 8 to O(1) at L = 16 (the spin forward is
                               unstable on this placement).  A spin != 0 plan with a value above 1e-8, or
                               with max_inv_residual above 1e-10, is marked fwd_unstable. */
} osht_info_t;

/*
 * Colatitude placement, computed on the host, no GPU needed.
 * Greedy (Sec. III-D): theta_{L-1} is the member of Theta farthest from the
 * poles; for m = L-2 down to 0, theta_m is the unused member of Theta that
 * minimises cond_2(P_m) (Eq. Y_matrix built from rings m..L-1 and degrees
 * m..L-1); candidates within a relative 1e-12 of the minimum are tied and
 * the smallest numerator wins.
 *   numerators_out: host array of L int32, receives n_k (ring k).
 *   kappa_out:      host array of L doubles or NULL; receives cond_2(P_m).
 * Returns OSHT_EINVAL for L < 1 or a NULL output array.
 */
int osht_theta_greedy(int L, int32_t* numerators_out, double* kappa_out);
/*
 * The same greedy (Sec. III-D) computed on the current HIP device: per order,
 * the candidate rows, S = B^T B (rocBLAS dgemm), its tridiagonal reduction and
 * Q^T r for every candidate (rocSOLVER dsytrd / dormtr), and one secular
 * solve per candidate in a kernel; the choice and its tie rule as above.
 * rocBLAS and rocSOLVER are opened at the first call.  Synchronous; uses the
 * null stream; allocates about 6 L^2 doubles of device memory for the call.
 *   numerators_out / kappa_out: host arrays as for osht_theta_greedy.
 * Returns OSHT_EINVAL for bad arguments, OSHT_ENOTSUP when rocBLAS or
 * rocSOLVER cannot be opened, OSHT_ENOMEM / OSHT_EHIP on device failures.
 * osht_plan_create uses it when the placement cache has no file for L (and
 * the host greedy when the libraries cannot be opened).
 * Currently switched off: returns OSHT_ENOTSUP (an unexplained GPU memory
 * fault is under investigation); plans use the host greedy.
 */
int osht_theta_greedy_device(int L, int32_t* numerators_out, double* kappa_out);
/* Eq. sampling_latitude: even k take 2L-1-k, odd k take k. */
int osht_theta_alternating(int L, int32_t* numerators_out);

/*
 * Build a plan for band-limit L (1 <= L <= 4096) and spin s (|s| < L).
 * theta_cache_dir (nullable): directory holding placement files named
 * "theta_greedy_L<L>.txt" (one numerator per line, '#' lines ignored);
 * read if present, otherwise the greedy is run on the host and the file is
 * written there (write failures are ignored).
 * On the current HIP device: evaluates the Legendre (or Wigner) blocks
 * A_m[k, i] = sY_{l0+i}^m(theta_k, 0) in FP64 with adaptive rescaling
 * (Sec. III-F, III-G), inverts every P_m (rows k >= |m| of A_m; the least
 * squares pseudo-inverse when |m| < |s|) in FP64 on the GPU by Newton-Schulz
 * iteration, keeping each order's iterate with the smallest residual.
 * Spin 0: every m must reach |I - X_m P_m|_max <= 1e-10, else the plan is
 * refused with OSHT_ESINGULAR (the placement makes some P_m numerically
 * singular, e.g. the alternating placement from L = 128 up).  Spin != 0: the
 * inverses serve only the forward, so a larger residual marks the plan
 * fwd_unstable instead.  Then runs the forward self-check described at
 * osht_info_t.fwd_check_err (one inverse and one forward of a single map).
 * Synchronous: returns once the plan is ready.  *out receives the plan.
 */
int osht_plan_create(int L, int spin, uint32_t flags, const char* theta_cache_dir,
                     osht_plan_t** out);
/* Frees everything the plan owns. NULL is accepted. */
int osht_plan_destroy(osht_plan_t* plan);
int osht_plan_info(const osht_plan_t* plan, osht_info_t* out);
/* Copies the L ring numerators n_k (theta_k = pi n_k/(2L-1)) to host memory. */
int osht_plan_theta(const osht_plan_t* plan, int32_t* numerators_host);

/*
 * Inverse SHT (Eq. f_inverse_SHT, Procedure 2): samples from coefficients.
 *   flm: device, batch * L*L complex128 (read)
 *   f:   device, batch * L*L complex128 (written); must not overlap flm.
 * batch >= 1.  Asynchronous on stream, except that a call with a larger
 * batch than any earlier call on the plan first synchronizes the device while
 * it grows the plan's workspace and rewrites its descriptor tables (the same
 * holds for every transform entry point).
 */
int osht_inverse(const osht_plan_t* plan, const void* flm, void* f, int64_t batch,
                 hipStream_t stream);

/*
 * Inverse SHT that allocates no device memory, for callers that cannot
 * allocate: code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc.  Same arguments, layouts, stream semantics and
 * results (bit for bit) as osht_inverse on the same plan, but its per-call
 * workspace (GEMM tables, slot buffers, ring bins) is a 256 MiB static
 * device array of the library, one copy per GPU, held until the process
 * ends, instead of the plan's workspace.  It needs 80 * L^2 * batch bytes
 * plus a few tables for spin 0 (about the same for spin != 0): batch up to
 * 3 at L = 1024, 12 at L = 512, 51 at L = 256; larger requests return
 * OSHT_EINVAL with nothing enqueued, and OSHT_PREC_I8X6 / _I8X8 plans
 * OSHT_ENOTSUP.  Never calls hipMalloc or hipFree.
 * All calls on one GPU share its array, which keeps the last call's
 * contents: calls that overlap in time on one GPU (on any plans or streams)
 * race; serialise them.
 */
int osht_inverse_noalloc(const osht_plan_t* plan, const void* flm, void* f, int64_t batch,
                         hipStream_t stream);

/*
 * Forward SHT (Procedure 1): coefficients from samples, removing the
 * aliases of orders |m'| > |m| in descending |m| before the order-m systems
 * P_m f_m = g_m are solved (Eq. gtof_inverse, Eq. signal_update).
 *   f:   device, batch * L*L complex128 (read)
 *   flm: device, batch * L*L complex128 (written); must not overlap f.
 * Returns OSHT_ENOTSUP, with nothing enqueued, on a plan marked fwd_unstable
 * (spin != 0 above L ~ 9 on the greedy placement) unless the plan was
 * created with OSHT_SPIN_FWD_FORCE; the same holds for osht_forward_adjoint
 * and for forward jobs of osht_batch_run.
 */
int osht_forward(const osht_plan_t* plan, const void* f, void* flm, int64_t batch,
                 hipStream_t stream);

/*
 * Real maps (spin 0 only; other plans return OSHT_ENOTSUP).  A map with real
 * samples has coefficients with f_{l,-m} = (-1)^m conj(f_{l,m}) (the
 * harmonics' conjugation rule, Eq. yellm:conj of the appendix on spherical
 * harmonics); two such maps are carried by one complex transform, so a batch
 * of real maps costs half as many complex transforms.
 *   osht_forward_real: f device, batch * L*L float64 (read) ->
 *     flm device, batch * L*L complex128, the full layout including m < 0
 *     (written).  Equals osht_forward of the same samples.
 *   osht_inverse_real: flm device, batch * L*L complex128 (read) ->
 *     f device, batch * L*L float64 (written): the real part of
 *     osht_inverse(flm), which is the whole of it when flm has the symmetry
 *     above.
 * In and out must not overlap.  Asynchronous on stream, with the workspace
 * rule of osht_inverse for a batch of ceil(batch/2) complex maps.  Not
 * accepted by osht_batch_run.
 */
int osht_forward_real(const osht_plan_t* plan, const void* f, void* flm, int64_t batch,
                      hipStream_t stream);
int osht_inverse_real(const osht_plan_t* plan, const void* flm, void* f, int64_t batch,
                      hipStream_t stream);

/*
 * Adjoints: exact conjugate transposes of osht_inverse and osht_forward with respect to
 * the Euclidean inner product on C^{L^2} (samples and coefficients alike).
 *   inverse_adjoint: f_bar (samples)     -> flm_bar (coefficients)
 *   forward_adjoint: flm_bar (coefficients) -> f_bar (samples)
 * Same layouts, ownership and stream semantics as the transforms.
 */
int osht_inverse_adjoint(const osht_plan_t* plan, const void* f_bar, void* flm_bar,
                         int64_t batch, hipStream_t stream);
int osht_forward_adjoint(const osht_plan_t* plan, const void* flm_bar, void* f_bar,
                         int64_t batch, hipStream_t stream);

/*
 * Batch scheduler.  Runs a list of transforms of possibly different plans
 * (uneven L and spin) as one unit on `stream`: jobs of the same plan run in
 * list order on one internal stream (they share the plan's workspace), jobs
 * of different plans run concurrently on up to 8 internal streams forked
 * from and joined back into `stream`.  Each job's buffers follow the
 * conventions of the single-transform calls (device, complex128,
 * [batch][L*L], no overlap of in and out).  All jobs of one plan must use
 * the same batch, and every plan must live on the current device.
 *   graph_inout == NULL: the jobs are issued directly.
 *   *graph_inout == NULL: the jobs are captured into a HIP graph, which is
 *     launched and returned in *graph_inout (owned by the caller; free it
 *     with osht_graph_destroy).
 *   *graph_inout != NULL: if the job list equals the captured one (same
 *     plans, directions, pointers and batches) the graph is relaunched;
 *     otherwise it is replaced by a new capture.
 * Asynchronous; the caller must not destroy a plan while a graph that
 * references it may still be launched.  Kernel timing is off inside graphs.
 */
#define OSHT_DIR_INVERSE          0
#define OSHT_DIR_FORWARD          1
#define OSHT_DIR_INVERSE_ADJOINT  2
#define OSHT_DIR_FORWARD_ADJOINT  3

typedef struct {
  const osht_plan_t* plan;
  int32_t direction;   /* OSHT_DIR_* */
  int32_t reserved;    /* 0 */
  const void* in;
  void* out;
  int64_t batch;
} osht_job_t;

typedef struct osht_graph osht_graph_t;

int osht_batch_run(const osht_job_t* jobs, int njobs, hipStream_t stream, osht_graph_t** graph_inout);
/* Frees a graph returned by osht_batch_run (NULL accepted). */
int osht_graph_destroy(osht_graph_t* graph);

/*
 * Kernel timing.  With profiling enabled on a plan, each launch of the
 * library's hot kernels made by that plan (or, when only_name is not NULL,
 * each launch with that name only) is bracketed by a pair of HIP events
 * recorded on the launch stream; osht_plan_kernel_time waits for the
 * pending events of one kernel name and returns the number of launches and
 * their summed duration in milliseconds since profiling was (re)enabled.
 * Names: "apply_inverse", "apply_forward", "apply_forward_correction",
 * "apply_inverse_adjoint", "apply_forward_adjoint" (order-wise GEMMs),
 * "ring_analysis", "ring_synthesis" (ring DFTs, one launch per direction up
 * to 4096 points), "fold", "gather_forward", "delta_solve", "coef_to_slots"
 * and "slots_to_coef" (coefficient transposes), "split_digits" (the int8
 * right-hand-side split of OSHT_PREC_I8X6 / _I8X8 plans).
 * Unknown names return zero launches.  Enabling resets all counters.
 * only_name is copied; NULL times every name.
 */
int osht_plan_set_profiling(osht_plan_t* plan, int enable, const char* only_name);
int osht_plan_kernel_time(osht_plan_t* plan, const char* name, int64_t* launches,
                          double* total_ms);

/*
 * Sticky output status of an OSHT_CHECK_FINITE plan: waits for the device
 * to finish the work enqueued so far (hipDeviceSynchronize), stores OSHT_OK
 * or OSHT_ENONFINITE in *status (the latter when any transform output since
 * the last call held a NaN or an Inf) and clears the record.  On plans
 * without the flag *status is always OSHT_OK.  Must not be called while a
 * stream capture is in progress.
 */
int osht_plan_status(osht_plan_t* plan, int32_t* status);

/* Human-readable message for a return code (static storage). */
const char* osht_strerror(int code);
/* Detail of the last error raised on the calling thread (thread-local
 * storage, valid until the next call on that thread). */
const char* osht_last_error_message(void);

#ifdef __cplusplus
}
#endif

#endif /* OSHT_H */
