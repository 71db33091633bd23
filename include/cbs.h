/*
 * cbs.h -- C ABI of the MI355X (gfx950) iterative Born solver for the
 * first-order acoustic Helmholtz system with heterogeneous sound speed,
 * density and absorption (arXiv 2507.16087).
 *
 * Problem (Sec. 2.1, eq. Helmholtz-system, row-scaled as eq. HH1stOrderSH and
 * staggered as App. B.1):
 *     rhobar_eta (i w + gamma_eta) u_eta + d/dx_eta p(x + dx/2 e_eta) = rhobar_eta s_u_eta
 *     (i w + gamma) q p + sum_eta d/dx_eta u_eta(x - dx/2 e_eta)        = q s_p
 * with q = (1 - 2 i alpha c / w) / (rho c^2) (complex sound speed,
 * eq. complex_sound_speed), rhobar_eta the two-point average of rho along
 * eta, gamma >= 0 the absorbing-layer rate, and spectral derivatives on a
 * periodic grid.  The iteration is Algorithm 1 (eq. BornAlt with the split
 * L + V of eqs. LV and C and the staggered (L+I)^{-1} of App. B.1).
 *
 * Conventions shared by every entry point
 *  - Grid: ndim in {1, 2, 3}; n[eta] cells per axis, C order, last axis
 *    contiguous.  Each n[eta] must be of the form 2^a 3^b with
 *    4 <= n[eta] <= 512 (4, 6, 8, 9, 12, 16, 18, 24, 27, ..., 384, 432, 486,
 *    512: one compiled FFT plan per length, a whole pencil in one
 *    work-group), else CBS_E_UNSUPPORTED.  Cell centres sit at integer
 *    multiples of dx; u_eta sits half a cell further along eta.
 *  - Units: SI.  alpha in Np/m, omega in rad/s.
 *  - Media c, rho, alpha: real float64 arrays of prod(n) cells.  c > 0,
 *    rho > 0, alpha >= 0, all finite, else CBS_E_INVALID.
 *  - Sources and fields: interleaved complex128 (re, im) arrays.  Pressure
 *    arrays hold prod(n) values; velocity arrays hold ndim planes of prod(n)
 *    values, plane eta being u_eta at the staggered points.
 *  - Time convention: the system carries +i omega with damping gamma >= 0,
 *    so outgoing waves are exp(-i k r).
 *  - Absorbing layer: inside the grid, pml_cells wide on every face, rate
 *    gamma = pml_gamma_max * sum_eta r_eta^2 where r_eta in [0, 1] is the
 *    periodic distance into the layer over (pml_cells + 1/2).
 *  - Pointers: ptr_kind CBS_PTR_HOST (pageable host memory) or
 *    CBS_PTR_DEVICE (device memory of the current HIP device).  Workspaces
 *    are always device memory.
 *  - Ownership: the caller owns every buffer passed in, including the
 *    workspace; the library keeps no pointer past a call.  A medium handle
 *    owns only its own device tables, released by cbs_destroy_medium.
 *  - Streams: hip_stream is a hipStream_t (NULL = default stream).  All
 *    device work of a call is ordered on that stream; solve calls return
 *    after their results are complete (they poll convergence scalars).
 *  - Errors: status codes only.  On CBS_E_* outputs are untouched.  On
 *    CBS_NOT_CONVERGED the outputs hold the last iterate.
 *  - Threading: a medium is immutable after creation except through
 *    cbs_set_scalars, which must not overlap any other call on the same
 *    medium; concurrent calls on one medium must use different
 *    workspaces and streams (the first solves tune the pass plans once,
 *    under a lock).  Per-pass timing (cbs_pass_timing*) is a measurement aid
 *    for one thread at a time.
 */
#ifndef CBS_H
#define CBS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct cbs_medium_s *cbs_medium;

typedef enum {
    CBS_OK = 0,
    CBS_NOT_CONVERGED = 1,   /* iteration cap reached; outputs hold last iterate */
    CBS_E_INVALID = -1,      /* bad argument or medium value                     */
    CBS_E_UNSUPPORTED = -2,  /* grid size or option not supported               */
    CBS_E_NOMEM = -3,        /* device allocation failed / workspace too small   */
    CBS_E_DEVICE = -4,       /* HIP runtime error                                */
    CBS_E_DIVERGED = -5      /* iterate became non-finite or grew without bound  */
} cbs_status;

typedef enum {
    CBS_FP64 = 0,            /* every iteration in complex128                     */
    CBS_FP32_REFINED = 1     /* complex64 inner iterations, FP64 residual and
                                accumulation (iterative refinement)               */
} cbs_precision;

enum { CBS_PTR_HOST = 0, CBS_PTR_DEVICE = 1 };

/* CBS_RHS_PHYSICAL: s_p, s_u are the sources of the first-order system; the
 * library forms the row-scaled right-hand side q s_p and rhobar_eta s_u_eta.
 * CBS_RHS_EQUATION: s_p, s_u are already the right-hand side of the
 * row-scaled system (used for adjoint solves of misfit gradients). */
enum { CBS_RHS_PHYSICAL = 0, CBS_RHS_EQUATION = 1 };

/* Stop rules.  CBS_STOP_UPDATE: Algorithm 1's relative update
 * |x_{k+1} - x_k| / |x_k| <= tol, tested from the second iteration on.
 * CBS_STOP_RESIDUAL: scaled true residual |y - (L+V) x| / |y| <= tol,
 * evaluated in FP64 every check_every iterations.  The refined precision
 * always stops on the residual. */
enum { CBS_STOP_UPDATE = 0, CBS_STOP_RESIDUAL = 1 };

typedef struct {
    int32_t ndim;            /* 1, 2 or 3                                           */
    int64_t n[3];            /* cells per axis (unused axes ignored)                */
    double dx;               /* grid spacing [m]                                    */
    double omega;            /* angular frequency [rad/s]                           */
    int32_t pml_cells;       /* absorbing layer width in cells, 0 <= 2 pml < n      */
    double pml_gamma_max;    /* layer rate scale [1/s]; <= 0 selects omega          */
    double beta;             /* scale factor of eq. C, 0 < beta < 1 (0 -> 0.95)     */
    double nu;               /* step of eq. BornAlt, 0 < nu <= 1 (0 -> 0.9)         */
    int32_t shift_rule;      /* 0: centre of the minimum enclosing circle of each
                                diagonal's values; 1: component-wise median          */
    int32_t collocated;      /* 0: staggered velocities (App. B.1, default);
                                1: collocated grid (App. B first matrix): every
                                field at the cell centres, rho and gamma unshifted,
                                derivative symbol i k with the Nyquist bin zeroed    */
} cbs_grid;

typedef struct {
    double tol;              /* stopping tolerance (see stop rules)                 */
    int64_t max_iter;        /* cap on CBS iterations (inner iterations in total
                                for the refined precision)                           */
    int32_t prec;            /* cbs_precision                                       */
    int32_t check_every;     /* iterations between host checks (0 -> 32)            */
    double inner_tol;        /* refined: inner relative-update tolerance (0 -> 1e-3)*/
    int32_t rhs_kind;        /* CBS_RHS_PHYSICAL or CBS_RHS_EQUATION                */
    int32_t ptr_kind;        /* pointer kind of sources and outputs                 */
    int32_t stop_rule;       /* CBS_STOP_UPDATE or CBS_STOP_RESIDUAL (FP64 only)    */
    int32_t max_outer;       /* refined: cap on outer steps (0 -> 10000)            */
    int32_t max_inner;       /* refined: cap on iterations per inner run (0 -> 256);
                                a stationary iteration restarted on its residual
                                loses nothing, so short inner runs only add FP64
                                residual checks and bound the overshoot           */
} cbs_solve_opts;

typedef struct {
    int64_t iterations;      /* CBS iterations run (FP32 inner ones when refined)   */
    int32_t outer;           /* refinement steps (0 for CBS_FP64)                   */
    int32_t status;          /* the cbs_status returned                             */
    double rel_update;       /* last relative update                                */
    double rel_residual;     /* last FP64 scaled residual, or -1 if not evaluated   */
    double seconds;          /* wall time of the call                               */
    int64_t residual_evals;  /* FP64 true-residual evaluations                      */
} cbs_solve_info;

/* Create a medium (Sec. 2.3.1 preprocessing of Algorithm 1): validates the
 * inputs, forms q, rhobar_eta and the layer rates, chooses the shifts a1, a2,
 * sets lam_j = max|D_j - a_j| / beta (floored at 1e-3 |a_j|) and uploads the
 * compact medium (rhobar, q) in FP64 and FP32 plus per-axis wavenumber,
 * half-cell shift and FFT twiddle tables.  c, rho, alpha: prod(n) float64
 * each, host or device per ptr_kind; read only during the call. */
cbs_status cbs_create_medium(const cbs_grid *grid, const double *c, const double *rho,
                             const double *alpha, int32_t ptr_kind, void *hip_stream,
                             cbs_medium *out);

cbs_status cbs_destroy_medium(cbs_medium m);

/* Scalars of the split (eqs. LV, C): out[0..7] = Re a1, Im a1, Re a2, Im a2,
 * lam1, lam2, beta, nu. */
cbs_status cbs_medium_scalars(cbs_medium m, double out[8]);

/* The same scalars computed on the host alone, without a device or a medium
 * handle (Algorithm 1 preprocessing; shifts per grid->shift_rule: centre of
 * the minimum enclosing circle of each diagonal's values, or their
 * component-wise median; scales per eq. C).  c, rho, alpha: host arrays of
 * prod(n) float64, read only during the call.  out[0..7] as
 * cbs_medium_scalars; a medium created from the same arguments reports the
 * same values.  CBS_E_INVALID / CBS_E_UNSUPPORTED as cbs_create_medium. */
cbs_status cbs_plan_scalars(const cbs_grid *grid, const double *c, const double *rho,
                            const double *alpha, double out[8]);

/* Override the split scalars: in[0..5] = Re a1, Im a1, Re a2, Im a2, lam1,
 * lam2 (lam > 0).  Changes the iteration, not its fixed point. */
cbs_status cbs_set_scalars(cbs_medium m, const double in[6]);

/* Device workspace bytes one solve of this medium needs at this precision;
 * batch is the number of same-medium-shape solves sharing one call (1). */
cbs_status cbs_workspace_bytes(cbs_medium m, int32_t prec, int32_t batch, size_t *bytes);

/* Solve A xi = s_hat (Algorithm 1).  s_p: prod(n) complex128; s_u: ndim x
 * prod(n) complex128 or NULL (zero).  p_out: prod(n) complex128; u_out:
 * ndim x prod(n) complex128 or NULL.  workspace: device buffer of at least
 * cbs_workspace_bytes(m, opts->prec, 1) bytes.  info may be NULL. */
cbs_status cbs_solve(cbs_medium m, const void *s_p, const void *s_u, const cbs_solve_opts *opts,
                     void *p_out, void *u_out, void *workspace, size_t ws_bytes,
                     cbs_solve_info *info, void *hip_stream);

/* Solve the adjoint system A^H xi = rhs (Sec. 2.3: negated differential part,
 * conjugated diagonal), with the same iteration run on conj(B) and the
 * per-wavevector conjugate transpose of (L+I)^{-1}.  Arguments as cbs_solve;
 * rhs_kind is usually CBS_RHS_EQUATION. */
cbs_status cbs_solve_adjoint(cbs_medium m, const void *s_p, const void *s_u,
                             const cbs_solve_opts *opts, void *p_out, void *u_out,
                             void *workspace, size_t ws_bytes, cbs_solve_info *info,
                             void *hip_stream);

/* Scaled residual of given fields: rel = |y - (L+V) x| / |y| with
 * x = C^{1/2} (u, p), y = C^{-1/2} s_hat (eqs. LV, C), in FP64 on the GPU.
 * adjoint selects A^H.  u may be NULL (zero).  r_p / r_u (nullable) receive
 * the physical residual s_hat - A (u, p) (complex128, same layout).
 * workspace: at least cbs_workspace_bytes(m, CBS_FP64, 1) bytes. */
cbs_status cbs_residual(cbs_medium m, const void *s_p, const void *s_u, const void *p,
                        const void *u, int32_t adjoint, int32_t rhs_kind, int32_t ptr_kind,
                        double *rel_residual, void *r_p, void *r_u, void *workspace,
                        size_t ws_bytes, void *hip_stream);

/* Bytes of the device array cbs_residual_noalloc works in (per GPU). */
#define CBS_NOALLOC_SCRATCH_BYTES (64u << 20)

/* cbs_residual without a workspace argument and without any allocation, for
 * callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc).  Arguments, outputs
 * and errors as cbs_residual.  Its kernels work in a file-scope device array
 * of CBS_NOALLOC_SCRATCH_BYTES that each GPU holds from the library's load
 * until the process ends; grids whose residual workspace
 * (cbs_workspace_bytes(m, CBS_FP64, 1)) exceeds it return CBS_E_NOMEM before
 * any device work (about 64^3 cells in 3-D).  It does not tune: it runs the
 * pass plans the medium holds (tuned by an earlier solve or residual call,
 * else the default plans).  Every call on one GPU shares that GPU's array,
 * which keeps the last call's contents; calls that overlap on one GPU (other
 * threads, other streams) race and must be serialised by the caller. */
cbs_status cbs_residual_noalloc(cbs_medium m, const void *s_p, const void *s_u, const void *p,
                                const void *u, int32_t adjoint, int32_t rhs_kind,
                                int32_t ptr_kind, double *rel_residual, void *r_p, void *r_u,
                                void *hip_stream);

/* Misfit gradient with respect to c, rho and alpha (adjoint-state method on
 * the adjoint operator of Sec. 2.3).  Given the physical source (s_p, s_u),
 * the forward solution (p, u) of A xi = s_hat and the adjoint solution
 * (lp, lu) of A^H lambda = g, writes prod(n) float64 values
 *   dJ/dm(x) = Re sum_rows conj(lambda_row) [d s_hat_row/dm(x) - dD_row/dm(x) xi_row]
 * for m in {c, rho, alpha} into g_c, g_rho, g_alpha (each nullable).  s_u and
 * u / lu may be NULL (zero).  All pointers of kind ptr_kind. */
cbs_status cbs_gradient(cbs_medium m, const void *s_p, const void *s_u, const void *p,
                        const void *u, const void *lp, const void *lu, int32_t ptr_kind,
                        double *g_c, double *g_rho, double *g_alpha, void *hip_stream);

/* Slab decomposition of one solve (the Discussion names domain decomposition
 * as the way to spread a solve over several GPUs), run on the current device
 * the way `parts` devices would run it: part g owns the axis-0 planes
 * [g s, (g+1) s) (s = n0 / parts) of the state, the right-hand side, the work
 * array and the medium, and runs the last-axis and axis-1 passes on them;
 * an exchange (the all-to-all of a multi-device run, here a device copy)
 * regroups the work array into axis-1 row groups [h t, (h+1) t)
 * (t = n1 / parts) for the axis-0 pass with the propagator, whose wavenumber
 * tables are offset to the group's rows, and a second exchange regroups it
 * back; one reduction folds every part's norm partial sums.  Every pass is
 * launched per part at the part's own shape.  Same arithmetic per pencil as
 * cbs_solve, so the same iterates; only the order in which the norm partial
 * sums are added differs.  ndim must be 3 and parts (1..64) must divide n0
 * and n1, else CBS_E_UNSUPPORTED.  Forward problem only.  Other
 * arguments, outputs and errors as cbs_solve; workspace: at least
 * cbs_split_workspace_bytes(m, opts->prec, parts) bytes. */
cbs_status cbs_split_workspace_bytes(cbs_medium m, int32_t prec, int32_t parts, size_t *bytes);
cbs_status cbs_solve_split(cbs_medium m, int32_t parts, const void *s_p, const void *s_u,
                           const cbs_solve_opts *opts, void *p_out, void *u_out, void *workspace,
                           size_t ws_bytes, cbs_solve_info *info, void *hip_stream);

/* Per-pass GPU time accounting for measurement: with enable = 1 (which also
 * clears the totals) every pass launch of this medium's solves is bracketed
 * by HIP events on the solve's stream and folded into running totals at each
 * host synchronisation; enable = 0 stops recording. */
cbs_status cbs_pass_timing(cbs_medium m, int32_t enable);

/* Which pass slots cbs_pass_timing brackets with events: bit k set = slot k
 * (the slots of cbs_pass_timing_read; default 0x3f, all six).  Every event
 * pair adds a few microseconds between kernels, so a measurement of one pass
 * can leave the others unbracketed.  CBS_E_INVALID outside [0, 0x3f]. */
cbs_status cbs_pass_timing_slots(cbs_medium m, int32_t slot_mask);

/* Pass plans in use for precision prec (after the first solve tunes them):
 * out[4 i + 0..3] = kind, axis length, columns per work-group and flags of
 * pass i in launch order (kind -1 = unused; kinds 0 contiguous forward, 1
 * contiguous inverse, 2 / 3 strided forward / inverse, 4 axis-0 propagator,
 * 6 the operator alone on the spectrum of a 1-D grid).  Flags:
 *   bit 0     wide radix split (fewer elements per thread);
 *   bits 1-4  variant.  Propagator pass: LDS layout 0 one tile reused field
 *             by field, 1 one region per field with every exchange shared,
 *             2 two regions with fields in pairs, plus 4 for a column tile
 *             without row padding.  Strided passes: 4 = no row padding.
 *             Last-axis inverse pass: prefetch 0 none, 1 x, y and the medium
 *             issued before the transform, 2 x and the medium;
 *   bits 5+   (3-D middle passes) the number of last-axis column blocks the
 *             forward-axis-1, propagator and inverse-axis-1 passes run in,
 *             one block after the other so a block's data is still in the
 *             memory-side cache for its next pass (1 = whole grid).
 * The first solve of each (shape, precision) in a process times the
 * candidate plans and block counts on its workspace and keeps the fastest.
 * Axis lengths other than powers of two and three times powers of two (9, 18, 27, ...)
 * have only variant 0 of each pass (and the unpadded column tile).
 * Environment: CBS_AUTOTUNE=0 keeps the defaults; CBS_PROP_VARIANT (0, 1, 2,
 * 4, 5, 6), CBS_LAST_VARIANT (0, 1, 2), CBS_STRIDED_VARIANT (0, 4) and
 * CBS_COLUMN_BLOCKS (1, 2, 4, 8) pin a choice, tuned or not; CBS_TUNE_FILE
 * names a text file that keeps tuned sets across processes (one line per
 * device architecture, shape, precision and pins; read before tuning, a
 * newly tuned set appended; lines that do not fit their shape are ignored,
 * the others are used without timing them again, so a line edited by hand
 * that a launch refuses makes solves fail with CBS_E_DEVICE).
 * Configurations
 * needing more than 160 KiB of LDS are never launched.  CBS_E_INVALID for a
 * null argument or a prec other than CBS_FP64 and CBS_FP32_REFINED. */
cbs_status cbs_pass_config(cbs_medium m, int32_t prec, int32_t out[20]);

/* Totals so far: ms[g * 6 + k] and launches[g * 6 + k] for group g (0 FP32
 * CBS iteration, 1 FP64 CBS iteration, 2 FP64 residual) and slot k (0..4 the
 * passes in launch order -- contiguous forward, strided forward, axis-0
 * propagator, strided inverse, contiguous inverse; 2-D grids use slots 0, 1
 * and 4, 1-D grids slot 1 for the operator on the spectrum -- and 5 the
 * reduction).  Middle passes run in column blocks count
 * one launch per block. */
cbs_status cbs_pass_timing_read(cbs_medium m, double ms[18], int64_t launches[18]);

/* Streaming-bandwidth probe for measurement: copies `bytes` from src to dst
 * (device pointers, 16-byte aligned, non-overlapping; bytes a non-zero
 * multiple of 16) once to warm up and then reps times on hip_stream (null:
 * the default stream), each work-group one contiguous 16 KiB chunk with
 * nontemporal loads and stores, and writes 2 * bytes / (average copy time)
 * in GB/s to *gbs: the rate a kernel that reads and writes HBM in equal
 * measure reaches on this device, beside which the passes' rates can be
 * read.  Blocks until done.  CBS_E_INVALID for a null, misaligned or
 * overlapping pointer, a bad size or reps < 1; CBS_E_DEVICE for a HIP
 * failure. */
cbs_status cbs_stream_probe(const void *src, void *dst, size_t bytes, int32_t reps, double *gbs,
                            void *hip_stream);

/* ---------------- batched slots (continuous-batching serving) -------------
 * A batch runs same-shape solves side by side: one kernel launch per pass
 * covers every active slot, iterations are captured in a HIP graph per
 * (shape, slot count) and replayed.  Slots are independent: each has its
 * own medium, right-hand side, tolerance, state and stop flag, so a slot's
 * result does not depend on what else is in the batch. */
typedef struct cbs_batch_s *cbs_batch;

/* Create a batch of up to max_slots same-shape slots at precision prec,
 * using the caller's device workspace of cbs_batch_workspace_bytes bytes. */
cbs_status cbs_batch_workspace_bytes(const cbs_grid *grid, int32_t prec, int32_t max_slots,
                                     size_t *bytes);
cbs_status cbs_batch_create(const cbs_grid *grid, int32_t prec, int32_t max_slots,
                            void *workspace, size_t ws_bytes, void *hip_stream, cbs_batch *out);
cbs_status cbs_batch_destroy(cbs_batch b);

/* Start a solve in a free slot; returns its slot index in *slot or
 * CBS_E_NOMEM when every slot is busy.  The medium must have the batch's
 * shape and stay alive until the slot is retired.  Sources as cbs_solve
 * (device or host per opts->ptr_kind). */
cbs_status cbs_batch_submit(cbs_batch b, cbs_medium m, const void *s_p, const void *s_u,
                            const cbs_solve_opts *opts, int32_t *slot);

/* Advance every active slot by up to `iterations` CBS iterations (refined
 * slots also run their outer steps), then poll.  The iterations are captured
 * once per (active slots, starting slots, iterations) as a HIP graph and
 * replayed (CBS_BATCH_GRAPHS=0 in the environment launches them directly);
 * the stream given to cbs_batch_create must therefore not be capturing.  done_mask receives one
 * byte per slot: 1 when that slot has finished (converged, capped or
 * diverged) and awaits retirement. */
cbs_status cbs_batch_step(cbs_batch b, int32_t iterations, uint8_t *done_mask);

/* Copy a finished slot's result (complex128, kind ptr_kind) and free it. */
cbs_status cbs_batch_retire(cbs_batch b, int32_t slot, void *p_out, void *u_out,
                            int32_t ptr_kind, cbs_solve_info *info);

#ifdef __cplusplus
}
#endif
#endif /* CBS_H */
