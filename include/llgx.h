/*
 * llgx — explicit finite-difference LLG micromagnetics with polynomial
 * extrapolation of the demagnetizing field, for AMD Instinct MI355X (gfx950).
 *
 * Method: S. Lepadatu, "Speeding up explicit numerical evaluation methods for
 * micromagnetic simulations using demagnetizing field polynomial
 * extrapolation", arXiv:2107.06729.  Section and equation numbers below refer
 * to that paper.
 *
 * Conventions shared by every call
 *   - Every call returns llgx_status: LLGX_OK (0) or a negative error code.
 *     Nothing throws across the ABI.  llgx_last_error() gives a message.
 *   - Units are SI: cell sizes in m, Ms and fields in A/m, A in J/m, K in
 *     J/m^3, gamma in m/(A s), times in s.  M is in A/m as in Eq. (1).
 *   - Vector fields (M, H, dM/dt) are device arrays in structure-of-arrays
 *     layout [3][nz][ny][nx], x fastest, of the handle's precision
 *     (double for LLGX_F64, float for LLGX_F32), contiguous, no padding.
 *   - Pointers named *_dev are device pointers owned by the caller; the
 *     library never frees them and reads/writes them only during the call's
 *     enqueued work.  Pointers named *_host are host memory.
 *   - All device work is enqueued on the HIP stream given to llgx_create.
 *     Calls that return host scalars (llgx_step, llgx_self_tensor, ...)
 *     synchronise that stream.
 *   - A handle is not thread safe: one host thread per handle.
 */
#ifndef LLGX_H
#define LLGX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t llgx_status;
#define LLGX_OK 0
#define LLGX_E_ARG (-1)         /* bad size, parameter or null pointer        */
#define LLGX_E_STATE (-2)       /* call not valid in the handle's state       */
#define LLGX_E_HIP (-3)         /* HIP runtime failure (message has details)  */
#define LLGX_E_NONFINITE (-4)   /* NaN/Inf in the error norm of a step        */
#define LLGX_E_OOM (-5)         /* device allocation failed                   */
#define LLGX_E_UNSUPPORTED (-6) /* valid request the library does not provide */

#define LLGX_F64 0 /* fields, FFTs and stages in double                       */
#define LLGX_F32 1 /* fields, FFTs and stages in float (error norm in double) */

#define LLGX_SPEC_NATIVE 0 /* FFT intermediates stored in the working precision */
#define LLGX_SPEC_BF16 1   /* FFT intermediates stored as bfloat16 (F32 only)  */
#define LLGX_SPEC_F16 2    /* FFT intermediates stored as float16 (F32 only)   */

/* Explicit methods named in Sec. II (coefficients from refs. [26]-[31]). */
#define LLGX_RK4 0    /* classic 4th order, fixed step                        */
#define LLGX_RKF45 1  /* Fehlberg, 4th order propagated, 5th order estimate   */
#define LLGX_RKCK45 2 /* Cash-Karp, 4th order propagated, 5th order estimate  */
#define LLGX_RKDP54 3 /* Dormand-Prince, 5th propagated, 4th estimate, FSAL   */
#define LLGX_HEUN 4   /* adaptive Heun, 2nd propagated, 1st estimate          */
#define LLGX_RK23 5   /* Bogacki-Shampine, 3rd propagated, 2nd estimate, FSAL */
#define LLGX_RKF56 6  /* Fehlberg, 5th propagated, 6th estimate, 8 stages     */
#define LLGX_ABM2 7   /* Adams-Bashforth-Moulton 2nd order PECE (ref. [32]):
                         variable-step AB2 predictor, trapezoidal corrector,
                         Milne error estimate; per step one Eq. (6) field at
                         the predicted state and one exact Eq. (2) at the
                         corrected state (the next step's start node).
                         Single handles only (not batches).                 */

#define LLGX_EXTRAP_FULL (-1)    /* exact Eq. (2) at every stage              */
#define LLGX_EXTRAP_MATCHED (-2) /* Eq. (6) with p = the propagated order n    */

/* Problem of Sec. II: mesh, cell, material, applied field (Eq. (1)). */
typedef struct {
    int32_t nx, ny, nz;  /* cells per axis, each >= 1                        */
    double dx, dy, dz;   /* cell size (m), > 0                               */
    double Ms;           /* saturation magnetization (A/m), > 0              */
    double A;            /* exchange stiffness (J/m), >= 0                   */
    double K;            /* uniaxial anisotropy constant (J/m^3)             */
    double easy[3];      /* anisotropy axis (normalised by the library)      */
    double alpha;        /* Gilbert damping, >= 0                            */
    double gamma;        /* gyromagnetic ratio of Eq. (1), m/(A s), > 0      */
    double Ha[3];        /* applied field (A/m), constant for t >= 0         */
} llgx_problem;

/* Stepping of Eq. (3)-(4) with the controller of Eq. (5) and the
 * extrapolation of Eq. (6).  llgx_stepper_defaults() fills the constants the
 * paper fixes after Eq. (5): h_min 1 fs, h_max 3 ps, c_min 0.01, c_max 2,
 * e_max 1e-5. */
typedef struct {
    int32_t method;        /* LLGX_RK4 ...                                     */
    int32_t extrap;        /* LLGX_EXTRAP_FULL, LLGX_EXTRAP_MATCHED or p 0..5  */
    int32_t adaptive;      /* 1: Eq. (5) controller (embedded pairs only)      */
    int32_t renormalize;   /* 1: rescale |M| to Ms after every accepted step   */
    int32_t exponent_mode; /* Eq. (5) exponent: 0 -> 1/(min(n,n^)+1), 1 -> 1/(n+1) */
    int32_t report_dmdt;   /* 1: llgx_step fills info->max_dmdt (one more pass
                              over dM/dt and a synchronisation per step)     */
    double h;              /* step (fixed) or first trial step (adaptive), s   */
    double h_min, h_max, c_min, c_max, e_max;
} llgx_stepper;

typedef struct {
    double t;              /* time after the step                               */
    double h_used;         /* accepted step                                     */
    double h_next;         /* next step proposed by Eq. (5) (= h if fixed)      */
    double err;            /* e of Sec. II: max over cells |h sum (c-c^) F|/Ms  */
    int32_t rejected;      /* rejected attempts before acceptance               */
    int32_t exact_evals;   /* Eq. (2) evaluations in this step                  */
    int32_t extrap_evals;  /* Eq. (6) evaluations in this step                  */
    int32_t forced;        /* 1 if accepted at h_min with err > e_max           */
    double max_dmdt;       /* max over cells of |dM/dt| / Ms (1/s) at the state
                              the step started from: the first stage's
                              derivative, Eq. (1) with the exact field of
                              Eq. (2); a diagnostic (e.g. a relaxation test),
                              not part of the paper's method.  Filled by
                              llgx_step when the stepper's report_dmdt is set,
                              else -1 */
} llgx_step_info;

typedef struct llgx_ctx* llgx_handle;

/* Message of the last error on h (owned by h, valid until the next call on
 * it); with h == NULL the message of the last failed llgx_create. */
const char* llgx_last_error(llgx_handle h);

/* Fill s with the Sec. II controller constants, method RK4, full demag,
 * h = 1e-13 s, fixed step, no renormalisation. */
void llgx_stepper_defaults(llgx_stepper* s);

/* Create a handle for problem p (copied).  precision: LLGX_F64/LLGX_F32;
 * spectral: LLGX_SPEC_* (16-bit storage requires LLGX_F32).  hip_stream: the
 * hipStream_t all work is enqueued on (NULL = default stream).  Allocates
 * the device workspace (state, stage buffers, extrapolation history, FFT
 * buffers, k-space kernel).  Errors: LLGX_E_ARG, LLGX_E_OOM, LLGX_E_HIP. */
llgx_status llgx_create(const llgx_problem* p, int32_t precision, int32_t spectral,
                        void* hip_stream, llgx_handle* out);
void llgx_destroy(llgx_handle h);

/* Sec. II, Eq. (2) and ref. [24]: compute the demagnetizing tensor N for
 * all cell offsets on the GPU in double precision (exact Newell form near,
 * moment expansion far), transform it with the library's FFT passes in
 * double, and store the real k-space kernel in the working precision.
 * Idempotent.  Must precede any field or step call (else LLGX_E_STATE). */
llgx_status llgx_precompute_demag(llgx_handle h);

/* Use a caller-supplied real-space tensor instead of llgx_precompute_demag.
 * N_host: double[6][2nz-1][2ny-1][2nx-1], components (xx,yy,zz,xy,xz,yz),
 * index [c][dz+nz-1][dy+ny-1][dx+nx-1] for offset (dx,dy,dz) in cells; it
 * must be even under (dx,dy,dz) -> -(dx,dy,dz).  The self term N00 used by
 * Eq. (6) is read from offset 0. */
llgx_status llgx_set_demag_tensor(llgx_handle h, const double* N_host);

/* Copy the real-space tensor computed by llgx_precompute_demag for offsets
 * 0..n-1 per axis: double[6][nz][ny][nx] (host). */
llgx_status llgx_get_demag_tensor(llgx_handle h, double* N_host);

/* N00 of Eq. (6): diagonal of the self term N(0). Synchronises. */
llgx_status llgx_self_tensor(llgx_handle h, double n00[3]);

/* Current magnetization (copied; the history of Eq. (6) is invalidated and
 * priming restarts; t is kept).  A cell with M = 0 is empty (no magnetic
 * material, as between the particles of the array in Sec. III): it stays
 * zero, and its magnetic neighbours see a free surface there (the exchange
 * term treats it as a missing neighbour); renormalisation leaves it empty.
 * The library notes on the stream whether any cell is empty, so meshes
 * without empty cells skip that test. */
llgx_status llgx_set_m(llgx_handle h, const void* M_dev);
llgx_status llgx_get_m(llgx_handle h, void* M_dev);

/* One exact evaluation of Eq. (2): H_dev = -sum_r N(r - r0) M(r). */
llgx_status llgx_demag(llgx_handle h, const void* M_dev, void* H_dev);
/* Effective field H_a + H_d + H_ex + H_an at M (terms named under Eq. (1)). */
llgx_status llgx_heff(llgx_handle h, const void* M_dev, void* H_dev);
/* F(t, M) of Eq. (1) in explicit Landau-Lifshitz form, exact demag. */
llgx_status llgx_rhs(llgx_handle h, const void* M_dev, void* F_dev);

/* ---- Field evaluation that allocates nothing ---------------------------
 * For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.
 * llgx_demag_noalloc computes exactly what llgx_demag computes (the same
 * kernels and launch variants, so the same bits), but its FFT spectra and
 * its empty-cell flag live in a static device array of the library of
 * LLGX_NOALLOC_SCRATCH_BYTES, one per GPU the library runs on, held until
 * the process ends (not in the handle's workspace).  The call allocates and
 * frees nothing, issues no hipMemset, and enqueues kernels only.
 * The mesh must fit: 256 + round_up(SA, 256) + SB bytes, with
 *   SA = 3 nz ny SX c, SB = 3 nz Py SX c (0 when ny = 1),
 *   Px/Py = next power of two >= 2 nx - 1 / 2 ny - 1 (1 for nx/ny = 1),
 *   SX = round_up(Px/2 + 1, 16), c = bytes per stored complex value
 *   (16 FP64, 8 FP32, 4 with 16-bit spectra); e.g. FP32 256x256x16 needs
 *   80.2 MB.  A larger mesh gives LLGX_E_ARG and enqueues nothing.
 * Every call on one GPU uses that GPU's one array: calls whose work overlaps
 * on a GPU (other streams, other host threads) race and must be ordered by
 * the caller.  The array keeps the last call's contents; the flag is cleared
 * by a kernel at every call and the spectra are fully rewritten before they
 * are read (their padding columns, never read into a result, are left).
 * Errors as llgx_demag (LLGX_E_STATE before llgx_precompute_demag). */
#define LLGX_NOALLOC_SCRATCH_BYTES (128u << 20)
llgx_status llgx_demag_noalloc(llgx_handle h, const void* M_dev, void* H_dev);

/* One accepted step of Eq. (3)-(4) from the handle's (t, M).  With
 * s->adaptive the Eq. (5) controller repeats rejected attempts and the next
 * call starts from info->h_next; otherwise s->h is used.  A change of method
 * or extrap between calls restarts priming.  Synchronises once per attempt
 * when adaptive (to read e), and once more with s->report_dmdt and info
 * given (to read max_dmdt); else not at all.  Errors: LLGX_E_ARG,
 * LLGX_E_STATE, LLGX_E_NONFINITE, LLGX_E_HIP. */
llgx_status llgx_step(llgx_handle h, const llgx_stepper* s, llgx_step_info* info);

/* nsteps fixed steps (s->adaptive must be 0) with no host synchronisation;
 * with use_graph the steady-state steps are captured into HIP graphs (per
 * history phase; 8 consecutive steps per graph while at least 8 remain,
 * else one) and replayed, bitwise the same as eager steps.  info (the last
 * step's) may be NULL; its max_dmdt is -1. */
llgx_status llgx_run_fixed(llgx_handle h, const llgx_stepper* s, int64_t nsteps, int32_t use_graph,
                           llgx_step_info* info);

/* Step until t_end, recording the mesh-averaged M every sample_dt into
 * mavg_host (double[cap][3]); adaptive steps are shortened to land on sample
 * times.  *nsamples receives the count written (including t = start). */
llgx_status llgx_run(llgx_handle h, const llgx_stepper* s, double t_end, double sample_dt,
                     double* mavg_host, int64_t cap, int64_t* nsamples);

/* Per-kernel timing.  With profiling enabled, every kernel the handle
 * launches eagerly is bracketed by HIP events on the handle's stream (graph
 * replay is disabled meanwhile).  llgx_profile_read synchronises, returns the
 * summed milliseconds and launch counts per kernel kind since the last read,
 * and resets them. */
#define LLGX_K_XFWD 0    /* stage combination + forward real-to-complex x pass */
#define LLGX_K_YFWD 1    /* forward y pass                                    */
#define LLGX_K_ZMUL 2    /* z forward, k-space tensor product, z inverse      */
#define LLGX_K_YINV 3    /* inverse y pass                                    */
#define LLGX_K_XINV 4    /* inverse x pass fused with H_eff and the LLG RHS   */
#define LLGX_K_COMBINE 5 /* stage input M_k = M0 + h sum b F (Eq. 4)          */
#define LLGX_K_EXTRAP 6  /* Eq. (6) sub-step field + H_eff + LLG RHS          */
#define LLGX_K_FINAL 7   /* Eq. (3) update and error-norm partials (fused with
                            the last sub-step when it is extrapolated)       */
#define LLGX_K_EPOLY 8   /* Eq. (6) fields for every distinct sub-step time   */
#define LLGX_K_OTHER 9   /* reductions, renormalisation                       */
#define LLGX_K_COUNT 10
llgx_status llgx_profile(llgx_handle h, int32_t enable);
llgx_status llgx_profile_read(llgx_handle h, double ms[LLGX_K_COUNT], int64_t launches[LLGX_K_COUNT]);

/* ---- Launch variants and the autotuner ----------------------------------
 * Each FFT pass of an exact evaluation (kinds LLGX_K_XFWD .. LLGX_K_XINV
 * above, indices 0..4 of the arrays below) can be launched in a few variants
 * -- tile widths and rows per workgroup -- that give bit-identical results
 * and differ only in speed.  Variant 0 is the default.
 *
 * llgx_autotune: times every variant of every pass (reps back-to-back
 * launches each, between HIP events on the handle's stream, in three rounds
 * that take the variants in turn; a variant's time is its fastest round),
 * keeps the fastest, and remembers the choice for the rest of the process
 * under the key (precision, spectral storage, mesh, sample count), so handles
 * created later with that key start with it.  us_out (may be NULL) receives
 * the chosen variants' fastest-round microseconds per launch (0 for a pass
 * the mesh does not need).  Needs llgx_precompute_demag and llgx_set_m (LLGX_E_STATE);
 * uses only the spectral workspace and the stage scratch array, so the
 * stepping state is unchanged.  Synchronises.
 * llgx_time_passes: the same measurement for the current variants only.
 * llgx_get_variants / llgx_set_variants: read or force the choice
 * (LLGX_E_ARG for an index out of range).
 * llgx_variant_counts: number of variants of each pass (n[5], host memory);
 * no handle needed, never fails for a non-null n.
 * llgx_tune_export: the process-wide table as JSON lines
 *   {"key": "f32/native/256x256x16/1", "variant": [v0..v4], "us": [t0..t4]}
 * with the same size protocol as llgx_save_state (buf NULL: size only,
 * including the terminating NUL).  llgx_tune_import: adds such lines to the
 * table (LLGX_E_ARG on a malformed line or a variant out of range; nothing
 * is added then).  Handles created afterwards pick the imported choices. */
llgx_status llgx_autotune(llgx_handle h, int32_t reps, double us_out[5]);
llgx_status llgx_time_passes(llgx_handle h, int32_t reps, double us_out[5]);
llgx_status llgx_get_variants(llgx_handle h, int32_t v[5]);
llgx_status llgx_variant_counts(int32_t n[5]);
llgx_status llgx_set_variants(llgx_handle h, const int32_t v[5]);
llgx_status llgx_tune_export(char* buf, size_t cap, size_t* used);
llgx_status llgx_tune_import(const char* text);

/* ---- Checkpoint / resume ------------------------------------------------
 * The whole stepping state of a handle -- t, the controller's next h, M, the
 * Eq. (6) history (the stage-1 fields of the previous accepted iterations and
 * their start times), the FSAL stage field when valid, the ABM2 start
 * derivative, its stored field and the previous derivative and step, the
 * method and order the history belongs to, and the counters -- as one host
 * byte image, so a
 * run resumed from it continues exactly as the uninterrupted run (no new
 * priming iterations, Sec. III).  The image holds arrays in the handle's
 * working precision and fits only a handle of the same mesh, sample count
 * and precision; the problem's material parameters are not part of it.
 *
 * llgx_save_state: with host_buf NULL, *used receives the size needed and
 * nothing is copied; otherwise cap must be at least that size (LLGX_E_ARG if
 * not).  Synchronises the handle's stream.  LLGX_E_STATE before llgx_set_m.
 * llgx_load_state: len must equal the image size; a foreign, corrupt or
 * mismatched image gives LLGX_E_ARG and leaves the handle unchanged.
 * Synchronises.  The caller owns host_buf in both calls. */
llgx_status llgx_save_state(llgx_handle h, void* host_buf, size_t cap, size_t* used);
llgx_status llgx_load_state(llgx_handle h, const void* host_buf, size_t len);

/* ---- Batches of independent samples -------------------------------------
 * n samples of possibly different meshes and applied fields (parameter and
 * field sweeps) stepped together.  Samples whose problems are equal except
 * for Ha share one set of kernels: every launch covers all of them (FFT
 * passes over all their rows, per-sample applied fields).  With use_graph,
 * one steady-state step of all samples is captured into a HIP graph (one per
 * history phase) and replayed.  All samples share the stepper and the
 * time: adaptive steps (llgx_batch_step) take one h for all.  spectral: the spectra's storage, as for
 * llgx_create (16-bit storage requires LLGX_F32).  llgx_batch_set_m on any
 * sample restarts priming of its group.  Per-sample M is [3][nz][ny][nx] of
 * the batch precision. */
typedef struct llgx_batch_s* llgx_batch;
llgx_status llgx_batch_create(int32_t n, const llgx_problem* problems, int32_t precision, int32_t spectral,
                              void* hip_stream, llgx_batch* out);
void llgx_batch_destroy(llgx_batch b);
const char* llgx_batch_last_error(llgx_batch b);
llgx_status llgx_batch_precompute_demag(llgx_batch b);
llgx_status llgx_batch_set_m(llgx_batch b, int32_t i, const void* M_dev);
llgx_status llgx_batch_get_m(llgx_batch b, int32_t i, void* M_dev);
llgx_status llgx_batch_run_fixed(llgx_batch b, const llgx_stepper* s, int64_t nsteps, int32_t use_graph);
/* One accepted step of every sample (Eq. (3)-(6)) with one h for all.  With
 * s->adaptive the error norm e of an attempt is the largest over all samples
 * and the Eq. (5) controller accepts or rejects it for all of them together
 * (info->err is that e; a rejected attempt reuses every group's stage 1).
 * Fixed steps take s->h.  Eager launches, one host synchronisation per
 * adaptive attempt.  info may be NULL; its evaluation counts are those of
 * the first group; max_dmdt is -1.  ABM2: LLGX_E_UNSUPPORTED. */
llgx_status llgx_batch_step(llgx_batch b, const llgx_stepper* s, llgx_step_info* info);
/* Autotune every mesh group of the batch (llgx_autotune on each). */
llgx_status llgx_batch_autotune(llgx_batch b, int32_t reps);
llgx_status llgx_batch_info(llgx_batch b, int32_t* ngroups, int64_t* total_cells, double* t);

/* How a captured batched step launches its work (the parametric sweeps of
 * Sec. IV: many small, uneven meshes at once).
 *   LLGX_BATCH_JOBS: each pass of the step (Eq. (6) extrapolation, stage
 *     inputs of Eq. (4), Eq. (3) update; x forward, y forward, z pass,
 *     y inverse, x inverse with the fused right-hand side once per FFT
 *     length among the groups) is one launch over a job table of
 *     (mesh group, tile) entries of its groups, one workgroup per job (up to
 *     4 groups a launch; more take one launch per 4).  The launches of one
 *     pass for different FFT lengths run side by side on forked streams.
 *     The job tables live in device memory the batch allocates when it
 *     captures a step and frees in llgx_batch_destroy.  Steps that have no
 *     job-table form (16-bit spectra, padded lengths above 1024 along x,
 *     512 along y or 64 along z) are captured as with LLGX_BATCH_STREAMS.
 *   LLGX_BATCH_STREAMS (default): each group's own launches, on streams
 *     forked from the batch stream inside the captured graph, so the
 *     kernels of different meshes overlap, and a small mesh's step does not
 *     wait at every pass for the large ones (the faster of the two on the
 *     64-sample sweep of four meshes).
 * Both give each sample the bits it gets when stepped alone.  Changing the
 * mode synchronises the batch stream and drops the captured graphs.
 * LLGX_E_ARG for an unknown mode.
 * llgx_batch_launch_info: whether the graph captured last uses job tables
 * (1) or forked streams (0), and its job-table launches per step (-1 when
 * forked); when a step falls back to forked streams, llgx_batch_last_error
 * says why. */
#define LLGX_BATCH_JOBS 0
#define LLGX_BATCH_STREAMS 1
llgx_status llgx_batch_set_launch(llgx_batch b, int32_t mode);
llgx_status llgx_batch_launch_info(llgx_batch b, int32_t* job_table, int32_t* kernels_per_step);

/* Time, proposed next step and counters of the handle. */
llgx_status llgx_get_time(llgx_handle h, double* t, double* h_next);
llgx_status llgx_set_time(llgx_handle h, double t);
llgx_status llgx_counters(llgx_handle h, int64_t out[5]); /* exact, extrap, accepted, rejected, forced */

#ifdef __cplusplus
}
#endif

#endif /* LLGX_H */
