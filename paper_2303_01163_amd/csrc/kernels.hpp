// Kernel launchers (host side), implemented in the k_*.hip files.
#pragma once

#include <hip/hip_ext.h>

#include "asdsm_internal.hpp"

namespace asdsm {

// Profiling hook.  While a launch group is timed (asdsm_opts.profile), `stop` is set: every launch
// then goes through hipExtLaunchKernelGGL, which stamps the events with the kernel's own start and
// end times; the group's first launch records `start` (and clears it), every launch records `stop`,
// so the pair spans the group's kernels without the host-side launch latency.
struct LaunchEvents {
    hipEvent_t start = nullptr, stop = nullptr;
};
LaunchEvents &launch_events();  // per host thread

#define ASDSM_LAUNCH(KERNEL, GRID, BLOCK, SHMEM, STREAM, ...)                                      \
    do {                                                                                          \
        ::asdsm::LaunchEvents &le_ = ::asdsm::launch_events();                                    \
        if (le_.stop) {                                                                           \
            hipExtLaunchKernelGGL(KERNEL, GRID, BLOCK, SHMEM, STREAM, le_.start, le_.stop, 0,     \
                                  __VA_ARGS__);                                                   \
            le_.start = nullptr;                                                                  \
        } else {                                                                                  \
            hipLaunchKernelGGL(KERNEL, GRID, BLOCK, SHMEM, STREAM, __VA_ARGS__);                  \
        }                                                                                         \
    } while (0)

// Allocation-free residual (k_noalloc.hip): resolve the device's copy of its scratch array (once
// per device, from the plan constructor), and r = b_ff - A_ff u with ||r||_2 on the plan's stream.
int noalloc_setup(int device);
int residual_noalloc(const Plan &p, const double *u, const double *s, const double *g, double *r,
                     double *norm2_host);

// Block cyclic reduction along a submesh's line axis (k_blockcr.hip): per mode of the diagonalised
// fine axes, the line's N = 2^L - 1 positions each hold the mesh's coarse block (NB points).
// Element (mode, i, c) of a box lives at (mode % mext0) ms0 + (mode / mext0) ms1 + i sw + c sc.
// tab holds, per mode and level l = 0..L-1, the row-major NB x NB matrices G_l, P_l, Q_l.
struct CrBox {
    const double *src;   // right-hand sides (may equal dst)
    double *dst;         // solution (dst += solution when accumulating)
    const double *tab;
    long long nmodes;
    long long mext0, ms0, ms1, sw, sc;
};
struct CrJob {
    CrBox box[kMaxD];
    int nbox;
    int N, L, NB;
    int tm;              // modes per workgroup (LDS form); 0: the global-memory form (in place
                         // in dst after copying src there; no accumulation)
    int accum;
    int fast;            // 1: the form with the whole line and all levels' matrices in LDS
    const int *gate;
    // the global-memory form as batched FP64 GEMMs per level (block_cr_gemm), when non-null:
    // scratch of at least NB * 2^(L-1) * nmodes doubles for the box with the most modes
    double *scratch;
    long long scratch_len;
    int shared_tab;      // 1: every mode uses the one table at box[b].tab (GEMM form only)
};
constexpr size_t kCrMaxLds = 64 * 1024;
size_t cr_lds_cap();  // LDS one workgroup may allocate on the current device (>= kCrMaxLds)
size_t cr_lds_bytes(int N, int NB, int tm);
// modes per workgroup of the fast form (want > 0: that count if it is valid), or 0 when the fast
// form does not apply
int cr2_modes_per_group(int N, int L, int NB, long long nmodes, int nbox, int want = 0);
bool cr_lds_supported(int NB);  // block sizes with an LDS-staged kernel
bool launch_block_cr(const CrJob &job, hipStream_t st);

struct BoxPtrs {
    double *p[kMaxD];
};

// The skeleton-sparse update of the previous step (u += s e, r -= s q on the skeleton) carried by
// the forward transform of the next error guess, whose B operand is that residual (mesh b's
// canonical layout, B[k, n] at k + N_f n: k the first fine coordinate, n = second + N_f plane).
// While a step is pending (IterState::pending) every block forms s from the line search's partial
// sums; the tiles stage r - s q as their operand, and nbox * nub update blocks after the tiles (on
// the CUs the tiles leave free) store r - s q as the next residual, add s e to u and leave their
// sums of (r - s q)^2 over owned points at res_out[update block].  With nothing pending the operand
// is r, copied to the next residual.
struct UpdArgs {
    const double *R[kMaxD];     // current residual per box (also the B operand)
    double *Rn[kMaxD];          // next residual
    const double *Q[kMaxD];     // q = A e
    const double *E[kMaxD];     // merged skeleton error guess
    double *U[kMaxD];           // skeleton iterate (in place)
    int mesh[kMaxD];            // mesh (coarse axis) of each box: which shared points it owns
    int nbox, nub;              // boxes, update blocks per box
    Geo geo;
    const double *dots;         // line-search partial sums: (<r, q>, <q, q>) pairs
    int ndots;
    double *scal;               // <r, q>, <q, q> and s recorded by block 0
    const IterState *stt;
    double *res_out;
};
int upd_blocks_per_box(const Geo &g);  // update blocks that cover one mesh's skeleton points

// One batched GEMM C = A * B per entry z (up to 3 boxes), FP64 MFMA; element (i, k) of A at
// A + b*sAb + i*sAi + k*sAk, and likewise for B (k, n) and C (i, n).
struct GemmJob {
    const double *A[kMaxD];
    const double *B[kMaxD];
    double *C[kMaxD];
    int nbox;
    int M, N, K, nbatch;
    int accum;                 // 1: C += A B, 0: C = A B
    int neg;                   // 1: the product enters negated (C -= A B, or C = -A B)
    int any_layout;            // 1: operands with no unit stride are accepted (slow, correct)
    const int *gate;           // return at once when *gate != 0 (may be nullptr)
    long long sAb, sAi, sAk, sBb, sBk, sBn, sCb, sCi, sCn;
    int tile;                  // FP64 tile shape: kTileAuto or one of kGemmTiles (autotuner)
    // non-null for box b: each output tile's block stores the sum of squares of the C values it
    // wrote at norm_out[b][batch * tiles_per_batch + tile index] (the error-guess norms)
    double *norm_out[kMaxD];
    // 1: one block beyond the tiles applies a pending stopping rule (finalize_pending) while the
    // tiles run; set only on a launch that no other launch of its step precedes
    int fin_on;
    FinArgs fin;
    int upd_on;                // 1: UpdArgs apply (A and B k-fast, one batch)
    UpdArgs upd;
};
int gemm_tiles_per_box(const GemmJob &job);  // output tiles of one box (all batches) as launched

// FP64 transform tile shapes (TM x TN, K chunk), chosen per plan by asdsm_autotune.
// kTilePlane: both fine-axis transforms of a d = 3 anisotropic box in one launch (k_plane2).
enum GemmTile { kTileAuto = 0, kTile32x32 = 1, kTile64x32 = 2, kTile32x64 = 3, kTile64x64 = 4, kTilePlane = 5 };
constexpr int kGemmTiles[] = {kTile32x32, kTile64x32, kTile32x64, kTile64x64, kTilePlane};
const char *gemm_tile_name(int tile);

// Thomas elimination along the coarse (slowest) axis of anisotropic boxes after their fine axes
// have been diagonalised: for each mode, (T_coarse + sigma I) x = f, sigma = sum of fine eigenvalues.
struct LineJob {
    double *X[kMaxD];          // data, in place
    double *scratch[kMaxD];    // same size as X
    const double *mu_a[kMaxD]; // eigenvalues of the first fine axis
    const double *mu_b[kMaxD]; // eigenvalues of the second fine axis (nullptr when d = 2)
    const double *mu_c[kMaxD]; // eigenvalues of the third fine axis (d = 4 only, else nullptr)
    Tri t[kMaxD];              // coarse-axis operator of each box
    int nbox;
    long long nmodes;          // product of the fine extents
    int ext_a;                 // extent of the first fine axis
    int ncoarse;               // points along the coarse axis
    int fp32;                  // 1: X and scratch hold floats (mixed-precision error guesses)
    const int *gate;
};

enum FinMode { kFinRnorm = 0, kFinBnorm = 1, kFinDots = 2, kFinBoxNorms = 3, kFinInit = 4, kFinIter = 5 };
void launch_finalize(const Plan &p, int nblk, int mode, int nbox, hipStream_t st);
void launch_rhs(const Plan &p, unsigned mask, const double *s, const double *gf, double *out,
                bool with_norm, hipStream_t st);
// fin_mode: kFinRnorm (plain), kFinInit (start of the loop), kFinIter (after a refinement step)
void launch_update_residual(const Plan &p, const double *uin, const double *e, double *uout,
                            double *const *gather, int fin_mode, hipStream_t st);
void launch_dots(const Plan &p, hipStream_t st);

bool launch_gemm(const GemmJob &job, hipStream_t st);  // false: unsupported operand layout

// C_c = L X_c R^T for every N_f x N_f slab c (row-major, contiguous slabs) of up to 3 boxes: the two
// fine-axis transforms of a d = 3 anisotropic box in one launch.  L and R are N_f x N_f, row-major.
struct PlaneJob {
    const double *X[kMaxD];
    double *C[kMaxD];
    const double *L[kMaxD];
    const double *R[kMaxD];
    int nbox, Nf, nplanes;
    int accum;                 // 1: C += result
    const int *gate;
    double *norm_partials;     // non-null: one sum of squares of the written C values per block,
                               // at the block's (box, slab, panel) item index
};
constexpr int kPlaneMaxNf = 256;  // largest N_f of k_plane2 (16 row tiles of 16, two per wave)
bool launch_plane2(const PlaneJob &job, hipStream_t st);  // false: N_f too large
void plane_prepare();  // once per process, device current: the kernels' dynamic LDS limit

// Measured ceilings (k_probe.hip): FP64 MFMA rate and streaming-copy rate of the device.
size_t probe_mfma_scratch_bytes();
int probe_mfma_f64(double *scratch, int iters, hipStream_t st, double *tflops);
int probe_copy(const double *src, double *dst, size_t bytes, int reps, hipStream_t st, double *tbps);
// FP32 MFMA variant: A read as double (a_f64) or float, B float, C written as double (c_f64) or
// float; the GemmJob pointers are reinterpreted accordingly.
bool launch_gemm32(const GemmJob &job, bool a_f64, bool c_f64, hipStream_t st);
void launch_line(const LineJob &job, hipStream_t st);
void launch_dense_modes(long long nmodes, int B, const double *inv, const double *in, double *out,
                        int accum, hipStream_t st);
void launch_box_norms(const Plan &p, const double *const *sol, hipStream_t st);

// Residual of a mesh system with zero Dirichlet data, out = f - A_S x, for up to 3 meshes at once
// (refinement sweeps of the submesh solves).
struct BoxResJob {
    const double *f[kMaxD];
    const double *x[kMaxD];
    double *out[kMaxD];
    MeshDesc m[kMaxD];
    int nbox;
    const int *gate;
};
void launch_box_residual(const Plan &p, const BoxResJob &job, hipStream_t st);
// y_i += x_i for up to 3 arrays of n doubles
void launch_axpy(double *const *y, const double *const *x, long long n, int nbox, hipStream_t st);

// deterministic pseudo-random fill in [-1, 1) (counter-based hash of seed and index)
void launch_fill_random(double *x, long long n, uint64_t seed, hipStream_t st);
// sum of squares of up to 3 arrays into scal[kScalEnorm2 + k] (finalised)
void launch_sumsq(const Plan &p, const double *const *x, const long long *n, int nbox, hipStream_t st);

// skeleton: mode 0 = initial guess (extrapolated cross points), 1 = error phase (random choice)
// In the error phase the permutation of the current step is read on the device from
// p.ws.perm_table[p.ws.state->it].
void launch_crosspoints(const Plan &p, int mode, const double *const *res, hipStream_t st);
void launch_merge(const Plan &p, int mode, const double *const *res, hipStream_t st);
// d = 3 with N_c in {7, 15, 31}: the merge forms the cross-point discrepancies itself and
// launch_crosspoints launches nothing
bool merge_forms_discrepancies(const Plan &p);
// d = 4 (k_skel4.hip): the discrepancy families and Boolean-sum remainders, then the merge
void launch_crosspoints4(const Plan &p, int mode, const double *const *res, hipStream_t st);
void launch_merge4(const Plan &p, int mode, const double *const *res, hipStream_t st);
// skel: the merged skeleton values per anisotropic mesh (default: the Y buffers); adj_only: write the
// hole layers next to each coarse plane into the EA buffers instead of the fine tiles (the error
// equation of the skeleton-sparse step: bff must be null, the holes' right-hand side is zero)
bool launch_filler(const Plan &p, const double *bff, double *out, hipStream_t st, double *const *skel = nullptr,
                   bool adj_only = false);
// skeleton-sparse refinement (k_sparse.hip)
void launch_skel_gather(const Plan &p, const double *u, hipStream_t st);
void launch_skel_dots(const Plan &p, hipStream_t st);
void launch_skel_update(const Plan &p, double *const *gather, hipStream_t st);
// k_skel_update leaves the step's stopping rule pending on the device (IterState::pending): the next
// step's first transform GEMM applies it in one extra block (GemmJob::fin_on), and
// launch_finalize_pending applies it on its own (a no-op launch when nothing is pending) wherever
// the loop state is read or no such GEMM follows.
FinArgs pending_fin_args(const Plan &p);
// the line search's partial sums that k_skel_dots leaves ((<r, q>, <q, q>) pairs) and their count
const double *skel_dots_partials(const Plan &p);
int skel_dots_count(const Plan &p);
void launch_finalize_pending(const Plan &p, hipStream_t st);

}  // namespace asdsm
