/*
 * asdsm.h -- C ABI of the MI355X (gfx950) implementation of the Anisotropic Submeshes Domain
 * Splitting Method (ASDSM) for the steady, constant-coefficient advection-diffusion equation
 *
 *     -sum_i alpha_i d^2u/dx_i^2 + sum_i beta_i du/dx_i = s   on (0,1)^d,   u = g on the boundary
 *
 * (eq. (1) of the paper, with one alpha_i and one beta_i per axis).  The fine mesh has
 * N_f = 2^level - 1 interior points per axis (h = 2^-level); the anisotropic submeshes are coarse
 * (H = 2^-coarse_level, N_c = 2^coarse_level - 1 points) along one axis and fine along the others
 * (Section 2.1 eqs. (3)-(5); Section 3.5 for d = 3).  The nesting condition eq. (3),
 * N_f + 1 = n (N_c + 1), holds for every 1 <= coarse_level < level.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - All floating point is IEEE binary64 (double).
 * - Fine-mesh vectors (s, u, r) are device arrays of N_f^d doubles ordered with x_1 fastest
 *   (the ordering of Section 2.2): index = i_1 + N_f*(i_2 + N_f*i_3), 0-based.
 * - Dirichlet data g is a device array of 2*d*N_f^(d-1) doubles: 2*d faces ordered axis j = 1..d
 *   and, per axis, side x_j = 0 then x_j = 1.  Each face holds g at the N_f^(d-1) interior grid
 *   points of the remaining axes, in increasing axis order, lowest axis fastest.  Boundary edges
 *   and corners are never read (the (2d+1)-point stencil does not reach them).
 * - Device pointers must be valid for the plan's HIP device and stay alive until the call returns.
 *   Every call is enqueued on the stream given to asdsm_plan and returns after that stream's work
 *   has completed (calls are blocking).
 * - Return status: 0 = ASDSM_OK, > 0 a warning (the result is valid), < 0 an error (outputs are
 *   unspecified).  asdsm_last_error() returns a thread-local message describing the last error.
 * - Plans are not thread-safe; distinct plans on distinct streams are independent.  No C++
 *   exception crosses this interface.
 */
#ifndef ASDSM_H
#define ASDSM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---- */
#define ASDSM_OK            0
#define ASDSM_STAGNATED     1   /* warning: the stagnation rule stopped the iteration          */
#define ASDSM_MAXITER       2   /* warning: max_iter iterations ran without meeting rtol        */
#define ASDSM_E_ARG        -1   /* invalid argument (d, alpha, beta, level, NULL pointer, ...)  */
#define ASDSM_E_NESTING    -2   /* coarse_level violates 1 <= coarse_level < level (eq. (3))     */
#define ASDSM_E_WORKSPACE  -3   /* workspace missing, too small or misaligned                   */
#define ASDSM_E_NUMERIC    -4   /* non-finite data or a non-finite intermediate                  */
#define ASDSM_E_DEVICE     -5   /* a HIP runtime call failed                                     */
#define ASDSM_E_UNSUPPORTED -6  /* valid by the paper but outside what this build implements    */

/* ---- mesh identifiers for asdsm_mesh_solve: bit j set = axis j+1 is coarse ---- */
#define ASDSM_MESH_FINE     0u

/* ---- phases timed when asdsm_opts.profile != 0 ---- */
#define ASDSM_PHASE_RHS        0   /* right-hand side assembly on the fine mesh and submeshes   */
#define ASDSM_PHASE_TRANSFORM  1   /* mode transforms of the submesh solves (FP64 MFMA)          */
#define ASDSM_PHASE_LINE       2   /* line / small dense solves along coarse axes                */
#define ASDSM_PHASE_SKELETON   3   /* cross points, discrepancy, spline correction, merge       */
#define ASDSM_PHASE_FILLER     4   /* hole right-hand sides, hole solves, fine-vector write     */
#define ASDSM_PHASE_DOTS       5   /* q = A e and the line-search inner products                */
#define ASDSM_PHASE_UPDATE     6   /* u += s e fused with r = b - A u, gather, norm             */
#define ASDSM_PHASE_LEARNED    7   /* learned proposals: features, network, scaling, line search */
#define ASDSM_NPHASE           8

typedef struct asdsm_plan_s *asdsm_plan_t;

/* Options of asdsm_solve (max_iter < 8192).  Stopping rule (the paper's loop condition of Algorithm 4, read as
 * "iterate while not converged and not stagnated"): iterate while ||r_k||_2 > rtol*||b_ff||_2 and
 * k < max_iter and not stagnated; stagnated = ||r_{k+1}||_2 > (1 - stag_eta)*||r_k||_2 for
 * stag_window consecutive iterations (stag_window = 0 disables it).  A zero line-search step leaves
 * u unchanged and counts as one such iteration; the next iteration draws another random choice of
 * the cross points (Algorithm 2 step 3), so it does not end the loop by itself. */
typedef struct {
    int    max_iter;      /* >= 0; 0 returns the initial guess of Algorithm 1                   */
    double rtol;          /* >= 0                                                                */
    int    stag_window;   /* >= 0                                                                */
    double stag_eta;      /* in [0, 1)                                                           */
    int    resume;        /* 0: start from Algorithm 1; 1: u holds the iterate u^(k0) on entry  */
    int64_t k0;           /* iteration counter of the entry iterate (selects the random stream)  */
    double *hist;         /* optional host array, length max_iter+1: ||r_k||_2 per iterate      */
    double *step_hist;    /* optional host array, length max_iter: the line-search step s_k     */
    int    profile;       /* nonzero: time each phase with HIP events (adds synchronisation)    */
    int    eager;         /* nonzero: launch the refinement kernels one by one and check the     */
                          /* stopping rule after every step, instead of replaying a captured    */
                          /* HIP graph of two steps and checking every four steps               */
    int    precision;     /* ASDSM_PREC_FP64 (0, default) or ASDSM_PREC_FP32: the error-phase  */
                          /* submesh solves (Algorithm 1 with the residual as source) run in    */
                          /* FP32 (FP32 MFMA transforms, FP32 line elimination, no refinement   */
                          /* sweeps); the residual, merge, filler and line search stay FP64.    */
                          /* The initial guess is FP64 in both modes.                           */
    int    skeleton;      /* nonzero: skeleton-sparse refinement (Section 3.3, first and last   */
                          /* remarks; d = 3, else ASDSM_E_UNSUPPORTED): after the                */
                          /* initial guess every step computes r, q = A e and the updates only  */
                          /* on the coarse planes (the residual vanishes in the holes,          */
                          /* Proposition 3.2(2)) and e only there and on the hole layers next to */
                          /* them; the holes of u are filled once when the loop ends.  Same     */
                          /* iterates as the fine-mesh loop up to rounding.  In batches the d = 3 */
                          /* members use it and the others the fine-mesh loop; not in learned    */
                          /* solves.                                                             */
} asdsm_opts;

/* values of asdsm_opts.precision */
#define ASDSM_PREC_FP64 0
#define ASDSM_PREC_FP32 1

typedef struct {
    int    status;        /* same as the return value                                            */
    int    iterations;    /* iterations performed by this call                                   */
    double bnorm;         /* ||b_ff||_2                                                          */
    double r0norm;        /* ||r||_2 of the entry iterate                                        */
    double rnorm;         /* ||r||_2 of the returned iterate                                     */
    double phase_ms[ASDSM_NPHASE];      /* accumulated device time per phase (profile only)      */
    int    phase_launches[ASDSM_NPHASE];/* kernel launches per phase (profile only); a kernel    */
                                        /* and the one-block reduction that finishes its sums    */
                                        /* count as one launch                                   */
    double phase_flops[ASDSM_NPHASE];   /* algorithmic floating-point operations per phase       */
                                        /* (profile only; a GEMM counts 2*M*N*K)                 */
    double phase_bytes[ASDSM_NPHASE];   /* algorithmic bytes per phase: every operand read once  */
                                        /* and every result written once (profile only)          */
    double total_ms;      /* device time of the whole call (profile only)                        */
    int    precision;     /* precision the error-phase submesh solves ran in: FP32 is used only  */
                          /* when requested and every anisotropic mesh's transforms are well     */
                          /* enough conditioned (6e-8 * prod cond(V_j) <= 1e-3), else FP64       */
} asdsm_stats;

/* Create a plan (Section 2.1 meshes, Section 2.3 operators, Algorithms 1-4 schedule).
 *   d            : 2, 3 or 4 (dimensions of eq. (1); d = 4 per Section 3.5's construction of the
 *                  submeshes for any d).  Skeleton-sparse refinement is built for d = 3.
 *   alpha, beta  : host arrays of d finite doubles, alpha[j] > 0 (copied).
 *   level        : fine level L, N_f = 2^L - 1, 2 <= L <= 10.
 *   coarse_level : L_c with 1 <= L_c < L (eq. (3)); 0 selects floor(L/2).
 *   seed         : seed of the counter-based random cross-point choice (Algorithm 2 step 3).
 *   hip_stream   : hipStream_t (borrowed, may be NULL for the null stream).
 * The plan owns its small host and device tables (operator spectra, transform matrices, spline
 * matrix); the large work arrays live in a caller-owned workspace (asdsm_set_workspace).
 * A fine axis that fast diagonalisation cannot handle (|cell Peclet| >= 1: complex spectrum; or an
 * eigenvector matrix too ill-conditioned for FP64) is solved along lines by block cyclic reduction
 * (asdsm_line_axes reports which).  For d = 3, an anisotropic mesh with two such fine axes takes
 * both on its line solve: the line along one, and as its block the other fine axis with the coarse
 * axis (N_f N_c points, up to 512), or else, when its coarse axis can be diagonalised, the other
 * fine axis alone per coarse mode, or else that N_f N_c block up to 1024 points; hole boxes with two or three such axes apply the inverse of
 * their operator densely (holes of up to 7^3 points) or, holes of 15^3, solve along one hole axis
 * by block cyclic reduction with the other two as the block.
 * Errors: ASDSM_E_ARG, ASDSM_E_NESTING, ASDSM_E_UNSUPPORTED (two such axes beyond those limits, or
 * in d = 4; hole boxes too large for one workgroup's LDS), ASDSM_E_NUMERIC (a singular block),
 * ASDSM_E_DEVICE. */
int asdsm_plan(asdsm_plan_t *out, int d, const double *alpha, const double *beta, int level,
               int coarse_level, uint64_t seed, void *hip_stream);

/* Bytes of device workspace the plan needs (>= 256-byte aligned base required). */
int asdsm_workspace_size(asdsm_plan_t plan, size_t *bytes);

/* Attach caller-owned device memory (not freed by the library).  ASDSM_E_WORKSPACE if NULL,
 * too small or not 256-byte aligned. */
int asdsm_set_workspace(asdsm_plan_t plan, void *dev, size_t bytes);

/* ASDSM (Algorithm 4): u^(0) = InitialGuess (Algorithm 1, with Skeleton Algorithm 2 and Filler
 * Algorithm 3) unless opts->resume, then refinement steps r = b - A u, error guess on the
 * submeshes, line search s = argmin_{s>=0} ||b - A(u + s e)||, u += s e.
 *   s : device, N_f^d source values at the fine points.
 *   g : device, Dirichlet faces (layout above).
 *   u : device, N_f^d, output iterate (input iterate u^(k0) when opts->resume).
 *   opts : host, may be NULL (defaults: max_iter 50, rtol 1e-10, stag_window 3, stag_eta 1e-3).
 *   stats: host, may be NULL.
 * Returns ASDSM_OK (rtol met), ASDSM_STAGNATED, ASDSM_MAXITER, or an error. */
int asdsm_solve(asdsm_plan_t plan, const double *s, const double *g, double *u,
                const asdsm_opts *opts, asdsm_stats *stats);

/* Fine residual r = b_ff - A_ff u (Algorithm 4 step 3), b_ff = s plus the Dirichlet terms.
 *   r     : device output of N_f^d doubles, may be NULL.
 *   norm2 : host output ||r||_2, may be NULL. */
int asdsm_residual(asdsm_plan_t plan, const double *u, const double *s, const double *g,
                   double *r, double *norm2);

/* Allocation-free variant of asdsm_residual, for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * r = b_ff - A_ff u and ||r||_2, formed in one stencil pass that assembles b_ff on the fly, without
 * the plan's workspace (none need be attached) and without any allocating call.  Its per-block
 * partial sums live in a 16 KiB file-scope device array, one copy per device, resolved when a plan is
 * created on that device; every call on a device shares that copy and overwrites it, so calls that
 * overlap on one device (other streams or threads) race.  Runs on the plan's stream and returns
 * after it has finished.
 *   u, s, g : device, layouts of asdsm_solve (not modified).
 *   r       : device output of N_f^d doubles, may be NULL (then only the norm is formed).
 *   norm2   : host output ||r||_2, may be NULL.
 * Errors: ASDSM_E_ARG (NULL plan, u, s or g), ASDSM_E_UNSUPPORTED (more than 2^31 - 2^19 - 1 fine
 * points: 32-bit indexing), ASDSM_E_DEVICE. */
int asdsm_residual_noalloc(asdsm_plan_t plan, const double *u, const double *s, const double *g,
                           double *r, double *norm2);

/* Direct solve of one mesh system A_S x = rhs with zero Dirichlet data (the submesh solves of
 * Algorithm 1 step 1, eq. (6)).  mesh_mask: bit j set = axis j+1 coarse; ASDSM_MESH_FINE is not
 * accepted; the all-coarse mask is the coarse mesh.  rhs and x are device arrays in the mesh's
 * canonical layout: the fine axes in increasing order, then the coarse axes in increasing order,
 * first listed axis fastest.  rhs and x may not alias. */
int asdsm_mesh_solve(asdsm_plan_t plan, unsigned mesh_mask, const double *rhs, double *x);

/* Autotuner: times the anisotropic-mesh solve (Algorithm 1 steps 1.1/1.2: the FP64 mode
 * transforms and the coarse-axis elimination) with every transform tile shape, `repeats` solves
 * each on reproducible random right-hand sides, and keeps the fastest for this plan (the default,
 * before tuning, picks by problem size).  Needs the workspace; overwrites the plan's mesh buffers.
 *   tile        : host output, may be NULL: the chosen shape (asdsm_tile_name names it).
 *   ms_per_solve: host output, may be NULL: its time per anisotropic solve.
 * Errors: ASDSM_E_ARG (repeats outside 1..1000), ASDSM_E_WORKSPACE, ASDSM_E_DEVICE. */
int asdsm_autotune(asdsm_plan_t plan, int repeats, int *tile, double *ms_per_solve);

/* Static name of a tile shape returned by asdsm_autotune ("auto" for unknown values). */
const char *asdsm_tile_name(int tile);

/* Transform tile shapes of the anisotropic solves (values of asdsm_autotune's `tile`):
 * ASDSM_TILE_AUTO picks by problem size; 1..4 run each fine-axis transform as its own batched GEMM
 * launch with that output tile; ASDSM_TILE_PLANE (d = 3, N_f <= 255) runs both fine-axis transforms
 * of every coarse slab in one launch. */
#define ASDSM_TILE_AUTO   0
#define ASDSM_TILE_32X32  1
#define ASDSM_TILE_64X32  2
#define ASDSM_TILE_32X64  3
#define ASDSM_TILE_64X64  4
#define ASDSM_TILE_PLANE  5

/* Force the transform tile shape of this plan's anisotropic solves (the autotuner's choice is
 * replaced).  Same iterates up to rounding for every shape.
 * Errors: ASDSM_E_ARG (unknown tile), ASDSM_E_UNSUPPORTED (ASDSM_TILE_PLANE with d != 3,
 * N_f > 255 or anisotropic meshes solved with line axes). */
int asdsm_set_tile(asdsm_plan_t plan, int tile);

/* The tile shape the plan's anisotropic solves use now: ASDSM_TILE_PLANE when both fine-axis
 * transforms run in one launch (chosen, or picked by size), else the chosen GEMM shape or
 * ASDSM_TILE_AUTO (GEMM tiles picked per launch by size).  tile: host output.
 * Errors: ASDSM_E_ARG (NULL argument). */
int asdsm_get_tile(asdsm_plan_t plan, int *tile);

/* ---- measured ceilings of the device (for the roofline; the solver never calls these) ----
 * asdsm_probe_mfma_f64: back-to-back v_mfma_f64_16x16x4f64 (eight independent chains per wave, 8
 *   workgroups of 4 waves per CU) for `iters` rounds; *tflops = achieved FP64 matrix rate.
 *   scratch: device buffer of at least asdsm_probe_mfma_scratch_bytes() bytes (caller-owned).
 * asdsm_probe_copy: `reps` streaming copies src -> dst of `bytes` (rounded down to 16), 16-byte
 *   accesses, four in flight per thread; *tbps = (read + written bytes) / time.  src, dst: device, 16-byte aligned, no overlap.
 * Both run on hip_stream (may be NULL), synchronise, and return ASDSM_E_ARG for NULL pointers or
 * non-positive counts, ASDSM_E_DEVICE if a HIP call fails. */
size_t asdsm_probe_mfma_scratch_bytes(void);
int asdsm_probe_mfma_f64(void *scratch, int iters, void *hip_stream, double *tflops);
int asdsm_probe_copy(const void *src, void *dst, size_t bytes, int reps, void *hip_stream, double *tbps);

/* Which fine axis of each mesh is solved by block cyclic reduction along it (a "line axis": its
 * 1D operator has a complex spectrum, |cell Peclet| >= 1, or an eigenvector matrix too
 * ill-conditioned for fast diagonalisation; or line axes save the refinement sweeps).
 *   axis : host output of 2^d ints indexed by mesh mask (bit j set = axis j+1 coarse); entry S is
 *          the 0-based axis solved along lines in mesh M_S, or -1 when every fine axis of M_S is
 *          diagonalised (always -1 for the fine mesh, S = 0).
 *   sweeps: host output of 2^d ints, may be NULL: refinement sweeps of each mesh solve.
 * Errors: ASDSM_E_ARG. */
int asdsm_line_axes(asdsm_plan_t plan, int *axis, int *sweeps);

/* Launch groups of the last asdsm_solve made with opts->profile = 1, by kind (a roofline per
 * kernel rather than per phase).  A kind is one kernel (its name, e.g. "k_plane2 forward") when
 * each of its groups is a single launch of that kernel, else "phase:<phase name>".
 * asdsm_profile_count: number of kinds (0 when the last call was not profiled), or an error.
 * asdsm_profile_entry: kind i (0 <= i < count): name (host buffer of name_cap bytes, truncated and
 *   NUL-terminated), phase (ASDSM_PHASE_*), ms (device time summed over the groups, from HIP event
 *   pairs on the plan's stream that the kernels themselves stamp), groups, kernel launches, and
 *   the algorithmic flops and bytes of those launches (every operand read once, every result
 *   written once).  Any output pointer may be NULL.  Errors: ASDSM_E_ARG. */
int asdsm_profile_count(asdsm_plan_t plan);
int asdsm_profile_entry(asdsm_plan_t plan, int i, char *name, int name_cap, int *phase, double *ms,
                        int *groups, int *launches, double *flops, double *bytes);

/* Release the plan and its tables (not the workspace).  NULL is ignored. */
void asdsm_destroy(asdsm_plan_t plan);

/* ---- batches of independent problems (any d, sizes and coefficients) ----
 * A batch runs the refinement loops (Algorithm 4) of its member plans together: every replay of
 * one captured HIP graph performs two refinement steps of every member that is still running, as
 * parallel branches; the host reads the members' loop states behind one pair of replays while the
 * next runs, and captures the graph again without the members whose stopping rule has fired.
 * Results are bitwise those of asdsm_solve on each plan with the same options. */
typedef struct asdsm_batch_s *asdsm_batch_t;

/* plans: host array of n distinct plans (1 <= n <= 4096) on one device, each with its workspace
 * attached; they are borrowed and must outlive the batch, and must not be used by another call
 * while a batch call runs.  Errors: ASDSM_E_ARG, ASDSM_E_DEVICE. */
int asdsm_batch_create(asdsm_batch_t *out, const asdsm_plan_t *plans, int n);

/* s, g, u: host arrays of n device pointers, member i in the layouts of asdsm_solve for plan i.
 * opts: shared by all members (may be NULL: the defaults of asdsm_solve); with profile or eager
 * set the members are solved one after the other.  stats: host array of n (may be NULL).
 * Returns the largest member status (0, ASDSM_STAGNATED, ASDSM_MAXITER) or the first error. */
int asdsm_batch_solve(asdsm_batch_t batch, const double *const *s, const double *const *g,
                      double *const *u, const asdsm_opts *opts, asdsm_stats *stats);

/* Release the batch's graph, streams and events (not the plans).  NULL is ignored. */
void asdsm_batch_destroy(asdsm_batch_t batch);

/* Thread-local description of the last error ("" if none). */
const char *asdsm_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* ASDSM_H */
