// Internal declarations shared by the host plan, the driver and the kernel launchers.
//
// Meshes (Section 2.1 eqs. (3)-(5), Section 3.5): a mesh is named by the bitmask S of its coarse
// axes.  S = 0 is the fine mesh, S = {k} the anisotropic submesh coarse along axis k, |S| >= 2 the
// intersection meshes (S = all axes: the coarse mesh).  Inside the library every submesh vector is
// stored in its *canonical layout*: the fine axes first (increasing), then the coarse axes
// (increasing), first listed axis fastest.  The fine mesh keeps the paper's x_1-fastest order.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/asdsm.h"

namespace asdsm {

constexpr int kMaxD = 4;
constexpr int kMaxMeshes = 1 << kMaxD;
constexpr int kDenseMaxBlock = 4096;  // coarse points per mode of an intersection-mesh dense solve
constexpr int kCrMaxBlock = 512;      // coarse points per position of a line solve
// points per position of a line solve over a fine axis with the coarse axis when that coarse axis
// cannot be diagonalised either (host-built tables of 3 L NB^2 doubles)
constexpr int kCrMaxBlock2 = 1024;
constexpr int kHoleDenseMax = 7;      // largest hole edge whose operator is inverted densely

// Canonical layout of mesh M_S.
struct MeshDesc {
    unsigned mask = 0;
    int nd = 0;
    int nfine = 0;                 // canonical positions [0, nfine) are fine axes
    int ax[kMaxD] = {0, 0, 0, 0};     // original axis at each canonical position
    int ext[kMaxD] = {1, 1, 1, 1};    // extent at each canonical position
    long long stride[kMaxD] = {0, 0, 0, 0};
    long long size = 0;            // number of points
    long long nmodes = 1;          // product of the fine extents
    int block = 1;                 // product of the coarse extents
};

// (sub, diag, super) row of alpha/h^2 tridiag(-1,2,-1) + beta/(2h) tridiag(-1,0,1).
struct Tri {
    double a, b, c;
};

// Small per-launch constant block for the stencil / skeleton / filler kernels.
struct Geo {
    int d;
    int Nf;        // fine interior points per axis
    int Nc;        // coarse interior points per axis
    int n;         // H / h (a power of two)
    long long NF;  // Nf^d
    Tri fine[kMaxD];
    Tri coarse[kMaxD];
};

// Per-axis spectral data of a 1D fine-spacing operator of size N (fast diagonalisation).
struct AxisSpectrum {
    int N = 0;
    double r = 1.0;                 // sqrt(sub/super): eigenvectors r^i sin(i m pi/(N+1))
    double cond = 1.0;              // condition number of the eigenvector matrix, r^(N-1)
    std::vector<double> mu;         // eigenvalues, m = 1..N
    std::vector<double> W;          // forward transform  W[m*N + i] = V^{-1}(m, i)
    std::vector<double> V;          // backward transform V[i*N + m] = V(i, m)
};

// Device-resident state of the refinement loop (Algorithm 4 with the stopping rule): the loop can
// run several iterations, or a captured graph of them, without a host round trip; every kernel of a
// refinement step returns at once when `done` is set.
struct IterState {
    int done;          // 1 once the stopping rule has fired (or a non-finite value appeared)
    int status;        // ASDSM_OK / ASDSM_STAGNATED / ASDSM_MAXITER / ASDSM_E_NUMERIC
    int it;            // refinement steps completed by this call
    int stag;          // consecutive steps with ||r_{k+1}|| > (1 - eta) ||r_k||
    int max_iter;
    int stag_window;
    int learned;       // learned proposals accepted (solves with a correction network)
    int pending;       // 1: a skeleton-sparse step has left its residual partial sums for the
                       // stopping rule, which the next step's first transform launch applies
    double rtol;
    double stag_eta;
    double rn_prev;    // ||r|| of the current iterate
    double spare;
    int perm[kMaxD];   // axis permutation of step `it` (Algorithm 2 step 3), kept beside the counter
                       // so that the error-phase kernels read it with one load
};

constexpr int kHistCap = 8192;   // capacity of the device residual / step histories

struct Workspace {
    double *b = nullptr;         // fine right-hand side b_ff
    double *r = nullptr;         // fine residual
    double *e = nullptr;         // merged error guess (fine)
    double *u2 = nullptr;        // second iterate buffer (ping-pong with the caller's u)
    double *X[kMaxMeshes] = {};  // mesh buffers (canonical), per mask
    double *Y[kMaxMeshes] = {};  // transform scratch, per mask
    double *Z[kMaxMeshes] = {};  // saved right-hand side (refinement sweeps), per mask
    double *W[kMaxMeshes] = {};  // accumulated solution (refinement sweeps), per mask
    double *lines[kMaxD] = {};   // cross-point discrepancies of each anisotropic mesh
    float *F1[kMaxD] = {};       // FP32 transform scratch of each anisotropic mesh (mixed
    float *F2[kMaxD] = {};       // precision error guesses)
    // skeleton-sparse refinement (d = 3), per anisotropic mesh in its canonical layout: u, r and
    // q = A e on the skeleton, and the error guess on the hole layers next to each plane (2 sides)
    double *SU[kMaxD] = {}, *SR[kMaxD] = {}, *SQ[kMaxD] = {}, *EA[kMaxD] = {};
    // with the update fused into the next forward transform: the second residual buffer (the
    // transform reads one and writes the other) and the merged error guess, which must outlive the
    // transform's output in Y
    double *SR2[kMaxD] = {}, *SE[kMaxD] = {};
    // back-substitution results of the line solves whose block is too large for the LDS forms
    // (block_cr_gemm), and its length in doubles
    double *crs = nullptr;
    long long crs_len = 0;
    // hole right-hand sides and solutions of the hole line solve (Plan::hole_cr): per hole nh^3
    // values, the line axis slowest and the block (the other two axes, the lower fastest) fastest
    double *HB = nullptr;
    IterState *state = nullptr;  // refinement-loop state
    double *hist = nullptr;      // ||r_k||, k = 0..it
    double *step_hist = nullptr; // s_hat_k
    int *perm_table = nullptr;   // axis permutation of every step of this call (kMaxD ints each)
    double *partials = nullptr;  // per-block partial sums
    double *scal = nullptr;      // device scalars (see kScal*)
};

// Device scalar slots.
enum ScalarSlot {
    kScalRnorm2 = 0,   // ||r||^2
    kScalBnorm2 = 1,   // ||b||^2
    kScalRQ = 2,       // <r, q>
    kScalQQ = 3,       // <q, q>
    kScalStep = 4,     // s_hat
    kScalEnorm2 = 5,   // ||e_k||^2, k = 0..d-1  (slots 5..8)
    kScalInvNorm = 9,  // 1/||e_k|| or 1 (slots 9..12)
    kScalFlags = 13,   // non-finite flag accumulator
    kScalNoalloc = 14, // host mirror only: ||r||^2 of asdsm_residual_noalloc
    kScalCount = 16
};

// Arguments of a deferred stopping rule (a skeleton-sparse step's, applied by a later launch).
struct FinArgs {
    const double *partials;  // the step's per-block sums of ||r||^2 over owned skeleton points
    int nblk;
    double *scal;
    IterState *stt;
    double *hist, *step_hist;
    const int *perm_table;
};

struct Plan {
    int d = 0, level = 0, clevel = 0;
    int Nf = 0, Nc = 0, n = 0;
    double h = 0, H = 0;
    double alpha[kMaxD] = {}, beta[kMaxD] = {};
    uint64_t seed = 0;
    uint64_t serial = 0;  // unique per plan object (never 0)
    // bumped whenever something that captured launches depend on changes (the workspace layout, the
    // transform tile, the sweep counts); a captured graph is replayed only while it matches
    uint64_t generation = 1;
    hipStream_t stream = nullptr;
    int device = 0;
    Geo geo{};

    MeshDesc mesh[kMaxMeshes];
    AxisSpectrum fine_spec[kMaxD];   // size N_f, used by the anisotropic / intersection meshes
    AxisSpectrum hole_spec[kMaxD];   // size n-1, used by the hole boxes
    int hole_line_axis = 0;          // the hole axis solved by line elimination
    std::vector<double> Sp;          // N_f x N_c spline matrix, row major
    std::vector<double> dense_inv[kMaxMeshes];  // per-mode inverses for |S| >= 2
    double fdm_cond[kMaxMeshes] = {};  // product of the eigenvector condition numbers of the
                                       // transformed axes of each mesh
    // line axes: canonical position of the fine axis of each mesh that is solved by block cyclic
    // reduction (together with the coarse block) instead of being transformed, or -1
    int line_pos[kMaxMeshes] = {-1, -1, -1, -1, -1, -1, -1, -1, -1, -1, -1, -1, -1, -1, -1, -1};
    bool line_aniso = false;           // the anisotropic meshes use line axes
    // d = 3 anisotropic mesh whose two fine axes both defeat fast diagonalisation: its line axis is
    // canonical position 0 and the block holds the other fine axis with the coarse axis (N_f N_c
    // points, no mode axes); solved by the GEMM form of the block cyclic reduction
    bool line_block2[kMaxMeshes] = {};
    // d = 3 anisotropic mesh whose two fine axes both defeat fast diagonalisation while its coarse
    // axis does not: that axis is diagonalised (coarse_spec), and per coarse mode the line solve
    // runs along canonical position 0 with the other fine axis (N_f points) as its block
    bool line_cmodes[kMaxMeshes] = {};
    AxisSpectrum coarse_spec[kMaxD];  // size N_c, for the meshes with line_cmodes
    double *dWc[kMaxD] = {}, *dVc[kMaxD] = {};
    // holes of up to 7^3 points with two or more axes that defeat fast diagonalisation: the hole
    // operator's inverse, applied densely by the generic filler (host copy while the plan is
    // built; device copy in the table allocation)
    bool hole_dense = false;
    std::vector<double> hole_inv;
    double *dhinv = nullptr;
    // d = 3 holes of 15^3 points with two or more such axes: block cyclic reduction along the hole
    // line axis with the other two axes (225 points, the lower axis fastest) as its block, one table
    // (per level G, P, Q) shared by every hole, run as batched GEMMs over the holes (hole_cr_tab:
    // host copy while the plan is built)
    bool hole_cr = false;
    int hole_cr_L = 0;
    std::vector<double> hole_cr_tab;
    double *dhcr = nullptr;
    int cr_tm = 0;                     // modes per workgroup of their line solve (0: by size)
    std::vector<double> cr_tab[kMaxMeshes];  // host copies while the plan is built
    double *dcr[kMaxMeshes] = {};      // per mode and level: G, P, Q (device)
    int sweeps[kMaxMeshes] = {};       // refinement sweeps of each mesh solve (calibrated)
    int sweeps_prior[kMaxMeshes] = {}; // a-priori counts from the condition numbers

    // device copies of the tables (one allocation owned by the plan)
    void *dtab = nullptr;
    size_t dtab_bytes = 0;
    double *dW[kMaxD] = {}, *dV[kMaxD] = {}, *dmu[kMaxD] = {};
    double *dWh[kMaxD] = {}, *dVh[kMaxD] = {}, *dmuh[kMaxD] = {};
    // FP32 copies of the fine-axis transforms (mixed-precision error guesses)
    std::vector<float> W32[kMaxD], V32[kMaxD];
    float *dW32[kMaxD] = {}, *dV32[kMaxD] = {};
    bool prec32 = false;             // this call's error guesses run in FP32
    bool sparse = false;             // this call's refinement runs on the skeleton only
    int tile_aniso = 0;              // FP64 transform tile of the anisotropic solves (0: auto)
    // error phase with the plane kernel: its backward launch leaves per-block sums of squares of the
    // solutions here (norm_nblk per mesh) for the cross-point and merge kernels; else nullptr
    double *norm_partials = nullptr;
    int norm_nblk = 0;
    bool fp32_ok = false;            // every anisotropic mesh: 6e-8 * prod cond(V_j) <= 1e-3
    double *dSp = nullptr;
    double *ddense[kMaxMeshes] = {};

    // caller workspace
    void *ws_base = nullptr;
    size_t ws_bytes = 0;
    Workspace ws;
    size_t ws_need = 0;
    int max_blocks = 0;              // partial-sum capacity

    // pinned host mirror of the device scalars and of the loop state
    double *hscal = nullptr;
    IterState *hstate = nullptr;
    IterState *hstate_ring[2] = {nullptr, nullptr};  // pinned slots of the pipelined graph loop
    hipEvent_t loop_ev[2] = {nullptr, nullptr};
    int *hperm = nullptr;        // pinned staging of the permutation table

    // refinement kernels return early when *gate != 0 (nullptr outside the refinement loop)
    const int *gate = nullptr;
    // a skeleton-sparse step is being launched whose first launch, a transform GEMM, applies the
    // previous step's stopping rule (pending on the device); cleared by the launch that carries it
    bool fin_carry = false;
    // skeleton-sparse loop with the update fused into the next step's forward transform (set per
    // solve): the merged error guess lives in SE, the residual alternates between SR (sr_par 0) and
    // SR2 (1); upd_carry marks the step whose forward transform is still to be launched, and
    // fin_res_nblk > 0 the residual partial sums that the carried stopping rule then reads
    bool upd_fused = false;
    bool upd_carry = false;
    int sr_par = 0;
    int fin_res_nblk = 0;

    // captured refinement graph (two steps: u -> u2 -> u), rebuilt when the iterate pointer changes
    hipStream_t capture_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    const double *graph_u = nullptr;
    uint64_t graph_gen = 0;          // generation the graph was captured at
    bool graph_prec32 = false;
    bool graph_sparse = false;
    // learned proposals (a correction network bound to this plan) for this call, and the network
    // and acceptance factor of the captured graph
    struct Net *learn_net = nullptr;
    double learn_factor = 4.0;
    uint64_t graph_net_serial = 0;      // 0: the graph holds plain steps
    const void *graph_net_ws = nullptr;
    double graph_factor = 0.0;

    // profiling: a pair of events around every timed launch group, read after the call's final
    // synchronisation (launches stay queued back to back, so the pair brackets the kernels alone)
    struct PhaseRec {
        int phase, launches;
        double flops, bytes;
        bool launched;
        const char *tag;   // kernel of a single-kernel launch group (string literal), or nullptr
    };
    // per launch-group kind of the last profiled call: device time, groups, launches, work
    struct KernelRec {
        std::string name;
        int phase;
        double ms;
        int groups, launches;
        double flops, bytes;
    };
    std::vector<KernelRec> kern_recs;
    bool profiling = false;
    bool prof_failed = false;
    std::vector<hipEvent_t> ev_pool;
    std::vector<PhaseRec> ev_recs;
    double phase_ms[ASDSM_NPHASE] = {};
    int phase_launches[ASDSM_NPHASE] = {};
    double phase_flops[ASDSM_NPHASE] = {};
    double phase_bytes[ASDSM_NPHASE] = {};
};

// block size and mode count of the line solve of mesh s (line_pos[s] >= 0)
inline int cr_block(const Plan &p, unsigned s) {
    if (p.line_cmodes[s]) return p.mesh[s].ext[1];
    return p.line_block2[s] ? p.mesh[s].ext[1] * p.mesh[s].block : p.mesh[s].block;
}
inline long long cr_modes(const Plan &p, unsigned s) {
    if (p.line_cmodes[s]) return p.mesh[s].block;
    return p.line_block2[s] ? 1 : p.mesh[s].nmodes / p.mesh[s].ext[p.line_pos[s]];
}

// the merged skeleton values of anisotropic mesh k (the merge's output)
inline double *merged_buf(const Plan &p, int k) { return p.upd_fused ? p.ws.SE[k] : p.ws.Y[1u << k]; }
// the skeleton residual of anisotropic mesh k that the next operation reads
inline double *sr_cur(const Plan &p, int k) { return p.sr_par ? p.ws.SR2[k] : p.ws.SR[k]; }
inline double *sr_next(const Plan &p, int k) { return p.sr_par ? p.ws.SR[k] : p.ws.SR2[k]; }
// the residual partial sums of the fused update (behind the other users of the partials area)
inline double *fused_res_partials(const Plan &p) { return p.ws.partials + 3 * (size_t)p.max_blocks; }

// ---- host plan construction (plan.cpp)
int build_plan(Plan &p, int d, const double *alpha, const double *beta, int level,
               int coarse_level, uint64_t seed, hipStream_t stream);
void layout_workspace(Plan &p, char *base, bool assign);
void release_plan(Plan &p);
MeshDesc make_mesh(int d, int Nf, int Nc, unsigned mask);

// counter-based permutation of the axes for iteration k
void axis_permutation(uint64_t seed, int64_t k, int d, int perm[kMaxD]);

// ---- error reporting
void set_error(const std::string &msg);
int fail(int code, const std::string &msg);

}  // namespace asdsm

struct asdsm_plan_s {
    asdsm::Plan p;
};
