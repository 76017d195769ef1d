// C ABI entry points and the ASDSM driver (Algorithms 1-4) on one HIP stream.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <new>

#include "../../include/asdsm_learn.h"
#include "asdsm_internal.hpp"
#include "kernels.hpp"
#include "learn_internal.hpp"

namespace asdsm {
const char *last_error_cstr();

LaunchEvents &launch_events() {
    static thread_local LaunchEvents ev;
    return ev;
}

namespace {

#define ASDSM_HIP_CHECK(expr)                                                                    \
    do {                                                                                          \
        hipError_t _e = (expr);                                                                   \
        if (_e != hipSuccess) return fail(ASDSM_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(_e)); \
    } while (0)

int check_launch(const char *what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(ASDSM_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
    return ASDSM_OK;
}

const char *phase_name(int ph) {
    static const char *names[ASDSM_NPHASE] = {"rhs", "transform", "line", "skeleton",
                                              "filler", "dots", "update", "learned"};
    return (ph >= 0 && ph < ASDSM_NPHASE) ? names[ph] : "?";
}

// Phase timing (opts->profile): a pair of events stamped by the kernels of a launch group (see
// LaunchEvents), with the algorithmic work of those launches (flops; bytes with every operand read
// once and every result written once).  Nothing synchronises here: the pairs are read once the
// call has finished.
struct PhaseTimer {
    Plan &p;
    size_t idx = 0;
    bool on = false;
    PhaseTimer(Plan &pl, int ph, int nl, double fl = 0.0, double by = 0.0, const char *tag = nullptr)
        : p(pl) {
        if (!p.profiling || p.prof_failed) return;
        idx = p.ev_recs.size();
        while (p.ev_pool.size() < 2 * (idx + 1)) {
            hipEvent_t e = nullptr;
            if (hipEventCreate(&e) != hipSuccess) {
                p.prof_failed = true;
                return;
            }
            p.ev_pool.push_back(e);
        }
        p.ev_recs.push_back({ph, nl, fl, by, false, tag});
        LaunchEvents &le = launch_events();
        le.start = p.ev_pool[2 * idx];
        le.stop = p.ev_pool[2 * idx + 1];
        on = true;
    }
    ~PhaseTimer() {
        if (!on) return;
        LaunchEvents &le = launch_events();
        p.ev_recs[idx].launched = (le.start == nullptr);  // the first launch consumed `start`
        le = LaunchEvents{};
    }
};

// Sum the recorded pairs into the per-phase totals (after the stream has been synchronised).
int collect_phases(Plan &p) {
    if (p.prof_failed) return fail(ASDSM_E_DEVICE, "profiling events could not be recorded");
    for (size_t i = 0; i < p.ev_recs.size(); ++i) {
        const Plan::PhaseRec &r = p.ev_recs[i];
        if (!r.launched) continue;
        float ms = 0.f;
        ASDSM_HIP_CHECK(hipEventElapsedTime(&ms, p.ev_pool[2 * i], p.ev_pool[2 * i + 1]));
        p.phase_ms[r.phase] += ms;
        p.phase_launches[r.phase] += r.launches;
        p.phase_flops[r.phase] += r.flops;
        p.phase_bytes[r.phase] += r.bytes;
        // per launch group kind: the groups with a kernel tag are single launches of that kernel
        const std::string name = r.tag ? std::string(r.tag) : std::string("phase:") + phase_name(r.phase);
        Plan::KernelRec *kr = nullptr;
        for (auto &k : p.kern_recs)
            if (k.name == name) kr = &k;
        if (!kr) {
            p.kern_recs.push_back(Plan::KernelRec{name, r.phase, 0.0, 0, 0, 0.0, 0.0});
            kr = &p.kern_recs.back();
        }
        kr->ms += ms;
        kr->groups += 1;
        kr->launches += r.launches;
        kr->flops += r.flops;
        kr->bytes += r.bytes;
    }
    return ASDSM_OK;
}

// Algorithmic work of one batched GEMM launch: 2 M N K flops per product; an operand shared by the
// batch (batch stride 0) is counted once per box; C is read as well when accumulating.
double gemm_flops(const GemmJob &j) { return 2.0 * j.M * j.N * j.K * j.nbatch * j.nbox; }
double gemm_bytes(const GemmJob &j) {
    const double a = (double)j.M * j.K * (j.sAb ? j.nbatch : 1);
    const double b = (double)j.K * j.N * (j.sBb ? j.nbatch : 1);
    const double c = (double)j.M * j.N * j.nbatch * (j.accum ? 2 : 1);
    return 8.0 * j.nbox * (a + b + c);
}

// two products of N_f^3 multiply-adds per slab
double plane_flops(const PlaneJob &j) { return 4.0 * j.Nf * (double)j.Nf * j.Nf * j.nplanes * j.nbox; }
// the slabs read and written once (C read as well when accumulating) and both matrices per box
double plane_bytes(const PlaneJob &j) {
    const double slab = (double)j.Nf * j.Nf;
    return 8.0 * j.nbox * (slab * j.nplanes * (j.accum ? 3 : 2) + 2 * slab);
}
// Whether the anisotropic solves run both fine-axis transforms of a slab in one launch (d = 3):
// chosen by the autotuner or asdsm_set_tile, else by size: up to N_f = 127 (one row tile per wave)
// the plane kernel beats two batched GEMMs; at 255 the 64 x 64 GEMM tiles are faster.  (Batches
// keep the rule too: with GEMM transforms the 15-problem batch of the bench took 47.4 ms instead
// of 43.0.)
constexpr int kPlaneAutoMaxNf = 127;
bool plane_transforms(const Plan &p) {
    if (p.d != 3 || p.Nf > kPlaneMaxNf || p.line_aniso) return false;
    if (p.tile_aniso == kTilePlane) return true;
    return p.tile_aniso == kTileAuto && p.Nf <= kPlaneAutoMaxNf;
}

void fine_axes(int d, int k, int &a, int &b) {
    if (d == 2) {
        a = 1 - k;
        b = -1;
    } else {
        a = (k == 0) ? 1 : 0;
        b = (k == 2) ? 1 : 2;
    }
}

// Buffers of mesh M_S: where its right-hand side is gathered and where its solution ends up.
// Without refinement sweeps the anisotropic meshes solve in place in X and the intersection meshes
// from X into Y; with sweeps the right-hand side is kept in Z and the solution accumulates in W.
double *rhs_buf(const Plan &p, unsigned m) { return p.sweeps[m] ? p.ws.Z[m] : p.ws.X[m]; }
double *sol_buf(const Plan &p, unsigned m) {
    if (p.sweeps[m]) return p.ws.W[m];
    return (__builtin_popcount(m) == 1) ? p.ws.X[m] : p.ws.Y[m];
}

double aniso_points(const Plan &p);

// The first transform GEMM of a skeleton-sparse step carries the previous step's pending stopping
// rule (one extra block; a no-op on the device when nothing is pending).
void carry_finalize(Plan &p, GemmJob &j) {
    if (!p.fin_carry) return;
    j.fin_on = 1;
    j.fin = pending_fin_args(p);
    if (p.fin_res_nblk > 0) {  // the residual sums the fused update has just left
        j.fin.partials = fused_res_partials(p);
        j.fin.nblk = p.fin_res_nblk;
    }
    p.fin_carry = false;
    p.fin_res_nblk = 0;
}

// The previous step's skeleton update fused into this forward transform (p.upd_carry): B is the
// current skeleton residual of each box's mesh instead of the gathered right-hand side, and the
// launch after it carries the stopping rule on the residual sums it leaves.
void carry_update(Plan &p, GemmJob &j, const int *slot) {
    if (!p.upd_carry) return;
    j.upd_on = 1;
    // short contractions load every K chunk at once: 64 x 32 tiles (measured at 127^3: 12.4 us
    // against 13.6 for 32 x 32, whose four tile rows each re-read r and q, and 14.2 for 32 x 64,
    // whose threads would hold more loads in flight than the per-wave counter allows)
    if (j.K <= 128) j.tile = kTile64x32;
    UpdArgs &u = j.upd;
    for (int b = 0; b < j.nbox; ++b) {
        const int k = slot[b];
        j.B[b] = sr_cur(p, k);
        u.R[b] = sr_cur(p, k);
        u.Rn[b] = sr_next(p, k);
        u.Q[b] = p.ws.SQ[k];
        u.E[b] = p.ws.SE[k];
        u.U[b] = p.ws.SU[k];
        u.mesh[b] = k;
    }
    u.nbox = j.nbox;
    u.nub = upd_blocks_per_box(p.geo);
    u.geo = p.geo;
    u.dots = skel_dots_partials(p);
    u.ndots = skel_dots_count(p);
    u.scal = p.ws.scal;
    u.stt = p.ws.state;
    u.res_out = fused_res_partials(p);
    p.upd_carry = false;
    p.fin_carry = true;
    p.fin_res_nblk = u.nbox * u.nub;
}

// Mode transform along canonical position q (a fine axis of extent N_f) of nb boxes of the shape m:
// out_b = T_b applied along q to in_b (out += when accum), T_b an N_f x N_f row-major matrix
// (T[m][i]).  Position 0 is contiguous (one GEMM over all rows); a later position is a batch over
// the outer positions of (N_f x N_f) times (N_f x inner) products.
int transform_position(Plan &p, const MeshDesc &m, int q, int nb, const double *const *in,
                       const double *const *T, double *const *out, int accum,
                       const int *norm_slot = nullptr) {
    GemmJob j{};
    j.nbox = nb;
    j.gate = p.gate;
    j.tile = (p.tile_aniso == kTilePlane) ? kTileAuto : p.tile_aniso;
    j.accum = accum;
    // E: the axis' extent (N_f for a fine axis, N_c for a diagonalised coarse axis)
    const long long E = m.ext[q], inner = m.stride[q];
    if (q == 0) {
        j.M = (int)(m.size / E); j.N = (int)E; j.K = (int)E; j.nbatch = 1;
        j.sAb = j.sBb = j.sCb = 0;
        j.sAi = E; j.sAk = 1;
        j.sBk = 1;  j.sBn = E;
        j.sCi = E; j.sCn = 1;
        for (int b = 0; b < nb; ++b) {
            j.A[b] = in[b];
            j.B[b] = T[b];
            j.C[b] = out[b];
        }
    } else {
        j.M = (int)E; j.N = (int)inner; j.K = (int)E; j.nbatch = (int)(m.size / (inner * E));
        j.sAb = 0;         j.sAi = E;     j.sAk = 1;
        j.sBb = inner * E; j.sBk = inner; j.sBn = 1;
        j.sCb = inner * E; j.sCi = inner; j.sCn = 1;
        for (int b = 0; b < nb; ++b) {
            j.A[b] = T[b];
            j.B[b] = in[b];
            j.C[b] = out[b];
        }
    }
    if (norm_slot && p.norm_partials) {
        // the error guesses' sums of squares, norm_nblk per mesh in the order of the coarse axis
        p.norm_nblk = gemm_tiles_per_box(j);
        for (int b = 0; b < nb; ++b) j.norm_out[b] = p.norm_partials + (size_t)norm_slot[b] * p.norm_nblk;
    }
    carry_finalize(p, j);
    PhaseTimer t(p, ASDSM_PHASE_TRANSFORM, 1, gemm_flops(j), gemm_bytes(j), "k_gemm_f64");
    if (!launch_gemm(j, p.stream)) return fail(ASDSM_E_ARG, "unsupported transform operand layout");
    return check_launch("transform");
}

// Mode transform along canonical position 0 of nb d = 3 boxes whose lines (the line axis at
// position 1, with the coarse axis) the block cyclic reduction reads whole: the forward transform
// writes mode-major, each mode's N_f x N_c line contiguous (C = T X^T, coalesced stores along the
// line), and the backward transform reads that layout back as an m-fast A operand and writes the
// canonical layout.  norm_slot as in transform_position.
int transform_pos0_modes_major(Plan &p, const MeshDesc &m, int nb, const double *const *in,
                               const double *const *T, double *const *out, bool fwd, int accum,
                               const int *norm_slot, const int *slot) {
    GemmJob j{};
    j.nbox = nb;
    j.gate = p.gate;
    j.tile = (p.tile_aniso == kTilePlane) ? kTileAuto : p.tile_aniso;
    j.accum = accum;
    j.nbatch = 1;
    j.sAb = j.sBb = j.sCb = 0;
    const long long Nf = p.Nf, rows = m.size / Nf;
    if (fwd) {
        j.M = (int)Nf; j.N = (int)rows; j.K = (int)Nf;
        j.sAi = Nf; j.sAk = 1;      // A = W (mode, position)
        j.sBk = 1;  j.sBn = Nf;     // B[k, row] = x(position k of the row)
        j.sCi = rows; j.sCn = 1;    // C[mode, row], mode-major
        for (int b = 0; b < nb; ++b) {
            j.A[b] = T[b];
            j.B[b] = in[b];
            j.C[b] = out[b];
        }
    } else {
        j.M = (int)rows; j.N = (int)Nf; j.K = (int)Nf;
        j.sAi = 1; j.sAk = rows;    // A[row, mode], mode-major data
        j.sBk = 1; j.sBn = Nf;      // B[mode, position] = V(position, mode)
        j.sCi = Nf; j.sCn = 1;      // canonical layout
        for (int b = 0; b < nb; ++b) {
            j.A[b] = in[b];
            j.B[b] = T[b];
            j.C[b] = out[b];
        }
    }
    if (norm_slot && p.norm_partials) {
        p.norm_nblk = gemm_tiles_per_box(j);
        for (int b = 0; b < nb; ++b) j.norm_out[b] = p.norm_partials + (size_t)norm_slot[b] * p.norm_nblk;
    }
    carry_finalize(p, j);
    if (fwd && accum == 0) carry_update(p, j, slot);
    // the launch that carries the skeleton update is its own kind: besides the transform it reads
    // q beside the operand and, per skeleton point, r, q, e, u and writes r, u (56 B in all)
    PhaseTimer t(p, ASDSM_PHASE_TRANSFORM, 1, gemm_flops(j),
                 gemm_bytes(j) + (j.upd_on ? 56.0 * aniso_points(p) : 0.0),
                 j.upd_on ? "k_gemm_f64+upd" : "k_gemm_f64");
    if (!launch_gemm(j, p.stream)) return fail(ASDSM_E_ARG, "unsupported transform operand layout");
    return check_launch("transform");
}

// d = 3 anisotropic meshes whose two fine axes both need the line solve and whose coarse axis is
// diagonalised (Plan::line_cmodes): forward transform along the coarse axis (canonical position 2,
// in -> Y), per coarse mode block cyclic reduction along position 0 with position 1 as the block
// (in place on Y, the GEMM form), backward transform (Y -> out, out += when accum).
int solve_mesh_cmodes(Plan &p, int nb, const unsigned *masks, const double *const *in, double *const *out,
                      int accum) {
    const MeshDesc &m = p.mesh[masks[0]];
    double *Y[kMaxD];
    const double *T[kMaxD];
    for (int b = 0; b < nb; ++b) {
        Y[b] = p.ws.Y[masks[b]];
        T[b] = p.dWc[p.mesh[masks[b]].ax[2]];
    }
    if (int rc = transform_position(p, m, 2, nb, in, T, Y, 0)) return rc;
    CrJob job{};
    job.nbox = nb;
    job.N = p.Nf;
    job.L = p.level;
    job.NB = cr_block(p, masks[0]);
    job.gate = p.gate;
    job.scratch = p.ws.crs;
    job.scratch_len = p.ws.crs_len;
    for (int b = 0; b < nb; ++b) {
        const MeshDesc &mb = p.mesh[masks[b]];
        CrBox &bx = job.box[b];
        bx.src = bx.dst = Y[b];
        bx.tab = p.dcr[masks[b]];
        bx.nmodes = cr_modes(p, masks[b]);
        bx.mext0 = mb.ext[2];
        bx.ms0 = mb.stride[2];
        bx.ms1 = 0;
        bx.sw = mb.stride[0];
        bx.sc = mb.stride[1];
    }
    {
        const double B = job.NB, pts = (double)nb * job.box[0].nmodes * job.N * B;
        PhaseTimer t(p, ASDSM_PHASE_LINE, 1, 6.0 * pts * B, 8.0 * (2.0 * pts + 3.0 * nb * job.box[0].nmodes * job.L * B * B),
                     "k_block_cr");
        if (!launch_block_cr(job, p.stream)) return fail(ASDSM_E_ARG, "line solve: unsupported shape");
        if (int rc = check_launch("block cyclic reduction")) return rc;
    }
    for (int b = 0; b < nb; ++b) T[b] = p.dVc[p.mesh[masks[b]].ax[2]];
    const double *Yc[kMaxD];
    for (int b = 0; b < nb; ++b) Yc[b] = Y[b];
    return transform_position(p, m, 2, nb, Yc, T, out, accum);
}

// Direct solve of nb meshes of one shape that have a line axis (Plan::line_pos, any d): the other
// fine axes are diagonalised by mode transforms, then block cyclic reduction runs along the line
// axis with the mesh's coarse block as blocks (k_blockcr.hip), then the backward transforms.
// in[b] -> out[b] (out += when accum); X and Y of each mesh are intermediates, in may be X, and out
// may be X (no transform) or X, Y or W as sol_buf names them.  The meshes' line axes may sit at
// different canonical positions: the transforms run per group of equal positions, the reduction
// for all meshes in one launch.
int solve_mesh_line(Plan &p, int nb, const unsigned *masks, const double *const *in, double *const *out,
                    int accum) {
    const MeshDesc &m = p.mesh[masks[0]];
    // transformed positions per mesh (none when both fine axes are on the line solve; the meshes
    // of one call are all of one kind)
    const bool block2 = p.line_block2[masks[0]];
    if (p.line_cmodes[masks[0]]) return solve_mesh_cmodes(p, nb, masks, in, out, accum);
    const int nt = block2 ? 0 : m.nfine - 1;
    int fq[kMaxD][kMaxD];        // [box][t]: the transformed canonical positions, ascending
    for (int b = 0; b < nb; ++b) {
        int t = 0;
        for (int q = 0; q < m.nfine && t < nt; ++q)
            if (q != p.line_pos[masks[b]]) fq[b][t++] = q;
    }
    // forward transforms: in -> Y -> X ... (transform t writes Y for even t, X for odd t)
    const double *cur[kMaxD];
    double *X[kMaxD], *Y[kMaxD];
    for (int b = 0; b < nb; ++b) {
        cur[b] = in[b];
        X[b] = p.ws.X[masks[b]];
        Y[b] = p.ws.Y[masks[b]];
    }
    // the backward transforms of all anisotropic meshes in one launch leave the error guesses'
    // sums of squares for the skeleton kernels (norm_partials, set by error_guess)
    bool one_group = true;
    for (int b = 1; b < nb && nt == 1; ++b) one_group = one_group && fq[b][0] == fq[0][0];
    const bool fuse_norms = p.norm_partials && nt == 1 && one_group && nb == p.d &&
                            __builtin_popcount(masks[0]) == 1;
    // d = 3 with the transformed axis at position 0: the line solve reads and writes mode-major
    // whole lines (transform_pos0_modes_major)
    const bool modes_major = nt == 1 && m.nd == 3 && one_group && fq[0][0] == 0;
    auto run_grouped = [&](int t, const double *const *src, double *const *dst, bool fwd, int acc) -> int {
        bool done[kMaxD] = {};
        for (int b = 0; b < nb; ++b) {
            if (done[b]) continue;
            const int q = fq[b][t];
            const double *gs[kMaxD], *gT[kMaxD];
            double *gd[kMaxD];
            int slot[kMaxD];
            int ng = 0;
            for (int c = b; c < nb; ++c)
                if (!done[c] && fq[c][t] == q) {
                    done[c] = true;
                    gs[ng] = src[c];
                    gd[ng] = dst[c];
                    slot[ng] = __builtin_ctz(masks[c]);
                    const int ax = p.mesh[masks[c]].ax[q];
                    gT[ng] = fwd ? p.dW[ax] : p.dV[ax];
                    ++ng;
                }
            const bool norms = !fwd && t == 0 && fuse_norms;
            if (modes_major) {
                if (int rc = transform_pos0_modes_major(p, m, ng, gs, gT, gd, fwd, acc, norms ? slot : nullptr, slot))
                    return rc;
            } else if (int rc = transform_position(p, m, q, ng, gs, gT, gd, acc, norms ? slot : nullptr)) {
                return rc;
            }
        }
        return ASDSM_OK;
    };
    for (int t = 0; t < nt; ++t) {
        double *dst[kMaxD];
        for (int b = 0; b < nb; ++b) dst[b] = (t % 2 == 0) ? Y[b] : X[b];
        if (int rc = run_grouped(t, cur, dst, true, 0)) return rc;
        for (int b = 0; b < nb; ++b) cur[b] = dst[b];
    }
    // the reduction: in place on the transformed data, or in -> out when nothing was transformed
    double *D[kMaxD], *O[kMaxD];
    for (int b = 0; b < nb; ++b) {
        D[b] = (nt % 2 == 1) ? Y[b] : X[b];
        O[b] = (nt % 2 == 1) ? X[b] : Y[b];
    }
    {
        CrJob job{};
        job.nbox = nb;
        job.N = p.Nf;
        job.L = p.level;
        job.NB = cr_block(p, masks[0]);
        job.gate = p.gate;
        job.accum = (nt == 0) ? accum : 0;
        long long nm = 0;
        for (int b = 0; b < nb; ++b) {
            const unsigned mk = masks[b];
            const MeshDesc &mb = p.mesh[mk];
            CrBox &bx = job.box[b];
            bx.src = (nt == 0) ? in[b] : D[b];
            bx.dst = (nt == 0) ? out[b] : D[b];
            bx.tab = p.dcr[mk];
            bx.nmodes = cr_modes(p, mk);
            bx.mext0 = nt >= 1 ? mb.ext[fq[b][0]] : 1;
            bx.ms0 = nt >= 1 ? mb.stride[fq[b][0]] : 0;
            bx.ms1 = nt >= 2 ? mb.stride[fq[b][1]] : 0;
            bx.sw = mb.stride[p.line_pos[mk]];
            // the block: the coarse axes, or the second fine axis with them (contiguous after the
            // line axis at position 0 in either case of line_block2)
            bx.sc = block2 ? mb.stride[1] : mb.stride[mb.nfine];
            if (modes_major) {  // element (mode, i, c) at mode (N_f N_c) + i + N_f c
                bx.ms0 = mb.size / mb.ext[0];
                bx.sw = 1;
                bx.sc = mb.ext[0];
            }
            nm = std::max(nm, bx.nmodes);
        }
        // modes per workgroup: 8 when the first mode axis is contiguous (coalesced loads), else 2;
        // fewer when the LDS does not hold them; the global-memory form when not even one fits
        const bool aniso = __builtin_popcount(masks[0]) == 1;
        int tm = cr2_modes_per_group(job.N, job.L, job.NB, nm, nb, aniso ? p.cr_tm : 0);
        if (tm == 0 && aniso && p.cr_tm) tm = cr2_modes_per_group(job.N, job.L, job.NB, nm, nb);
        job.fast = tm > 0 ? 1 : 0;
        if (!job.fast) {
            tm = (job.box[0].ms0 == 1) ? 8 : 2;
            while (tm > 1 && cr_lds_bytes(job.N, job.NB, tm) > kCrMaxLds) tm /= 2;
            if (!cr_lds_supported(job.NB) || cr_lds_bytes(job.N, job.NB, tm) > kCrMaxLds) tm = 0;
        }
        if (tm == 0 && job.accum)
            return fail(ASDSM_E_UNSUPPORTED, "line solve: accumulation needs the LDS form");
        job.tm = tm;
        job.scratch = p.ws.crs;
        job.scratch_len = p.ws.crs_len;
        const double B = job.NB;
        const double pts = (double)nm * nb * job.N * B;
        PhaseTimer t(p, ASDSM_PHASE_LINE, 1, 6.0 * pts * B, 8.0 * (2.0 * pts + 3.0 * nm * nb * job.L * B * B),
                     "k_block_cr");
        if (!launch_block_cr(job, p.stream)) return fail(ASDSM_E_ARG, "line solve: unsupported shape");
        if (int rc = check_launch("block cyclic reduction")) return rc;
    }
    // backward transforms, last first: D -> O -> D ... -> out
    for (int t = nt - 1; t >= 0; --t) {
        const double *src[kMaxD];
        double *dst[kMaxD];
        for (int b = 0; b < nb; ++b) {
            src[b] = D[b];
            dst[b] = (t == 0) ? out[b] : O[b];
        }
        if (int rc = run_grouped(t, src, dst, false, t == 0 ? accum : 0)) return rc;
        for (int b = 0; b < nb; ++b) std::swap(D[b], O[b]);
    }
    return ASDSM_OK;
}

// Direct solve of nb meshes of one shape, any d (the d = 4 path): every fine axis diagonalised by a
// mode transform, then per mode a Thomas elimination along the coarse axis (one coarse axis) or the
// precomputed dense inverse of the coarse block (several), then the backward transforms.
// in[b] -> out[b] (out += when accum); X and Y of each mesh are intermediates.  in may be X.  The
// last backward transform reads Y when the mesh has one coarse axis and X otherwise, so out may be X
// or W in the first case and Y or W in the second (the buffers sol_buf names).
int solve_mesh_nd(Plan &p, int nb, const unsigned *masks, const double *const *in, double *const *out,
                  int accum) {
    if (p.line_pos[masks[0]] >= 0) return solve_mesh_line(p, nb, masks, in, out, accum);
    const MeshDesc &m = p.mesh[masks[0]];
    const int nf = m.nfine;
    double *X[kMaxD], *Y[kMaxD];
    const double *T[kMaxD];
    for (int b = 0; b < nb; ++b) {
        X[b] = p.ws.X[masks[b]];
        Y[b] = p.ws.Y[masks[b]];
    }
    if (nf == 0) {  // the coarse mesh: one dense block
        for (int b = 0; b < nb; ++b) {
            const double B = m.block;
            PhaseTimer t(p, ASDSM_PHASE_LINE, 1, 2.0 * B * B, 8.0 * (B * B + (accum ? 3 : 2) * B));
            launch_dense_modes(1, m.block, p.ddense[masks[b]], in[b], out[b], accum, p.stream);
            if (int rc = check_launch("dense")) return rc;
        }
        return ASDSM_OK;
    }
    // forward transforms: in -> Y -> X -> Y ... (position q writes Y for even q, X for odd q)
    const double *cur[kMaxD];
    for (int b = 0; b < nb; ++b) cur[b] = in[b];
    for (int q = 0; q < nf; ++q) {
        double *dst[kMaxD];
        for (int b = 0; b < nb; ++b) {
            dst[b] = (q % 2 == 0) ? Y[b] : X[b];
            T[b] = p.dW[p.mesh[masks[b]].ax[q]];
        }
        if (int rc = transform_position(p, m, q, nb, cur, T, dst, 0)) return rc;
        for (int b = 0; b < nb; ++b) cur[b] = dst[b];
    }
    // the data sit in D = (nf odd ? Y : X); the other buffer O is free
    double *D[kMaxD], *O[kMaxD];
    for (int b = 0; b < nb; ++b) {
        D[b] = (nf % 2 == 1) ? Y[b] : X[b];
        O[b] = (nf % 2 == 1) ? X[b] : Y[b];
    }
    if (m.nd - nf == 1) {
        // one coarse axis: Thomas per mode, in place on D (scratch O)
        LineJob L{};
        L.nbox = nb;
        L.gate = p.gate;
        L.nmodes = m.nmodes;
        L.ext_a = p.Nf;
        L.ncoarse = m.block;
        for (int b = 0; b < nb; ++b) {
            const MeshDesc &mb = p.mesh[masks[b]];
            L.X[b] = D[b];
            L.scratch[b] = O[b];
            L.mu_a[b] = p.dmu[mb.ax[0]];
            L.mu_b[b] = nf >= 2 ? p.dmu[mb.ax[1]] : nullptr;
            L.mu_c[b] = nf >= 3 ? p.dmu[mb.ax[2]] : nullptr;
            L.t[b] = p.geo.coarse[mb.ax[nf]];
        }
        const double lpts = (double)L.nmodes * L.ncoarse * nb;
        PhaseTimer t(p, ASDSM_PHASE_LINE, 1, 8.0 * lpts, 16.0 * lpts, "k_line");
        launch_line(L, p.stream);
        if (int rc = check_launch("line")) return rc;
    } else {
        // several coarse axes: the dense inverse of each mode's coarse block, D -> O
        for (int b = 0; b < nb; ++b) {
            const double B = m.block, nmo = (double)m.nmodes;
            PhaseTimer t(p, ASDSM_PHASE_LINE, 1, 2.0 * nmo * B * B, 8.0 * nmo * (B * B + 2 * B));
            launch_dense_modes(m.nmodes, m.block, p.ddense[masks[b]], D[b], O[b], 0, p.stream);
            if (int rc = check_launch("dense")) return rc;
            std::swap(D[b], O[b]);
        }
    }
    // backward transforms, last position first: D -> O -> D ... -> out
    for (int q = nf - 1; q >= 0; --q) {
        const double *src[kMaxD];
        double *dst[kMaxD];
        for (int b = 0; b < nb; ++b) {
            src[b] = D[b];
            dst[b] = (q == 0) ? out[b] : O[b];
            T[b] = p.dV[p.mesh[masks[b]].ax[q]];
        }
        if (int rc = transform_position(p, m, q, nb, src, T, dst, q == 0 ? accum : 0)) return rc;
        for (int b = 0; b < nb; ++b) std::swap(D[b], O[b]);
    }
    return ASDSM_OK;
}

// Direct solves of the anisotropic meshes k in kbits (fast diagonalisation of the fine axes, Thomas
// along the coarse axis): in[k] -> out[k] (out += solution when accum).  X_k and Y_k are used as
// intermediates, so in[k] may be X_k and out[k] may be X_k, but neither may be Y_k.
int solve_aniso(Plan &p, unsigned kbits, double *const *in, double *const *out, int accum) {
    const int d = p.d, Nf = p.Nf, Nc = p.Nc;
    int ks[kMaxD], nb = 0;
    for (int k = 0; k < d; ++k)
        if ((kbits >> k) & 1u) ks[nb++] = k;
    if (nb == 0) return ASDSM_OK;
    if (d == 4 || p.line_aniso) {
        // the meshes with a transformed axis first (their first launch is a transform, which may
        // carry the previous step's stopping rule): a fine axis, then the coarse axis of meshes with
        // both fine axes on the line; last those that transform nothing (one line solve per mesh)
        for (int kind = 0; kind < 3; ++kind) {
            unsigned masks[kMaxD];
            const double *bin[kMaxD];
            double *bout[kMaxD];
            int ng = 0;
            for (int q = 0; q < nb; ++q) {
                const unsigned mq = 1u << ks[q];
                if ((p.line_cmodes[mq] ? 1 : p.line_block2[mq] ? 2 : 0) != kind) continue;
                masks[ng] = mq;
                bin[ng] = in[ks[q]];
                bout[ng] = out[ks[q]];
                ++ng;
            }
            if (ng == 0) continue;
            if (int rc = solve_mesh_nd(p, ng, masks, bin, bout, accum)) return rc;
        }
        return ASDSM_OK;
    }
    const long long Nf2 = (long long)Nf * Nf;
    GemmJob j{};
    j.nbox = nb;
    j.gate = p.gate;
    j.tile = p.tile_aniso;
    // d = 3 with the plane kernel: both forward transforms in one launch (in -> Y), the line
    // elimination on Y, both backward transforms in one launch (Y -> out)
    const bool plane = plane_transforms(p);
    if (plane) {
        PlaneJob pj{};
        pj.nbox = nb; pj.Nf = Nf; pj.nplanes = Nc; pj.accum = 0; pj.gate = p.gate;
        for (int q = 0; q < nb; ++q) {
            int a, b;
            fine_axes(d, ks[q], a, b);
            pj.X[q] = in[ks[q]];
            pj.C[q] = p.ws.Y[1u << ks[q]];
            pj.L[q] = p.dW[b];
            pj.R[q] = p.dW[a];
        }
        PhaseTimer t(p, ASDSM_PHASE_TRANSFORM, 1, plane_flops(pj), plane_bytes(pj), "k_plane2 forward");
        if (!launch_plane2(pj, p.stream)) return fail(ASDSM_E_ARG, "plane transforms: N_f too large");
        if (int rc = check_launch("transform")) return rc;
    }
    // forward transform along canonical axis 0 (contiguous): in -> Y
    if (!plane) {
        j.M = (d == 2) ? Nc : Nf * Nc;
        j.N = Nf; j.K = Nf; j.nbatch = 1; j.accum = 0;
        j.sAb = j.sBb = j.sCb = 0;
        j.sAi = Nf; j.sAk = 1;
        j.sBk = 1;  j.sBn = Nf;
        j.sCi = Nf; j.sCn = 1;
        for (int q = 0; q < nb; ++q) {
            int a, b;
            fine_axes(d, ks[q], a, b);
            j.A[q] = in[ks[q]];
            j.B[q] = p.dW[a];
            j.C[q] = p.ws.Y[1u << ks[q]];
        }
        PhaseTimer t(p, ASDSM_PHASE_TRANSFORM, 1, gemm_flops(j), gemm_bytes(j), "k_gemm_f64");
        if (!launch_gemm(j, p.stream)) return fail(ASDSM_E_ARG, "unsupported transform operand layout");
        if (int rc = check_launch("transform")) return rc;
    }
    if (d == 3 && !plane) {
        // forward along canonical axis 1, batched over the coarse slabs: Y -> X
        j.M = Nf; j.N = Nf; j.K = Nf; j.nbatch = Nc; j.accum = 0;
        j.sAb = 0;   j.sAi = Nf; j.sAk = 1;
        j.sBb = Nf2; j.sBk = Nf; j.sBn = 1;
        j.sCb = Nf2; j.sCi = Nf; j.sCn = 1;
        for (int q = 0; q < nb; ++q) {
            int a, b;
            fine_axes(d, ks[q], a, b);
            j.A[q] = p.dW[b];
            j.B[q] = p.ws.Y[1u << ks[q]];
            j.C[q] = p.ws.X[1u << ks[q]];
        }
        PhaseTimer t(p, ASDSM_PHASE_TRANSFORM, 1, gemm_flops(j), gemm_bytes(j), "k_gemm_f64");
        if (!launch_gemm(j, p.stream)) return fail(ASDSM_E_ARG, "unsupported transform operand layout");
        if (int rc = check_launch("transform")) return rc;
    }
    // line elimination along the coarse axis: on Y (scratch X) for d = 2 and the plane kernel,
    // else on X (scratch Y)
    {
        LineJob L{};
        L.nbox = nb;
        L.gate = p.gate;
        L.nmodes = (d == 2) ? Nf : Nf2;
        L.ext_a = Nf;
        L.ncoarse = Nc;
        for (int q = 0; q < nb; ++q) {
            int a, b;
            const int k = ks[q];
            fine_axes(d, k, a, b);
            const bool onY = (d == 2) || plane;
            L.X[q] = onY ? p.ws.Y[1u << k] : p.ws.X[1u << k];
            L.scratch[q] = onY ? p.ws.X[1u << k] : p.ws.Y[1u << k];
            L.mu_a[q] = p.dmu[a];
            L.mu_b[q] = (d == 3) ? p.dmu[b] : nullptr;
            L.t[q] = p.geo.coarse[k];
        }
        const double lpts = (double)L.nmodes * L.ncoarse * nb;
        PhaseTimer t(p, ASDSM_PHASE_LINE, 1, 8.0 * lpts, 16.0 * lpts, "k_line");
        launch_line(L, p.stream);
        if (int rc = check_launch("line")) return rc;
    }
    if (plane) {
        PlaneJob pj{};
        pj.nbox = nb; pj.Nf = Nf; pj.nplanes = Nc; pj.accum = accum; pj.gate = p.gate;
        // the last backward launch of an error guess leaves the norms' partial sums (a later
        // sweep's launch overwrites those of the first)
        pj.norm_partials = (p.norm_partials && nb == d) ? p.norm_partials : nullptr;
        for (int q = 0; q < nb; ++q) {
            int a, b;
            fine_axes(d, ks[q], a, b);
            pj.X[q] = p.ws.Y[1u << ks[q]];
            pj.C[q] = out[ks[q]];
            pj.L[q] = p.dV[b];
            pj.R[q] = p.dV[a];
        }
        PhaseTimer t(p, ASDSM_PHASE_TRANSFORM, 1, plane_flops(pj), plane_bytes(pj), "k_plane2 backward");
        if (!launch_plane2(pj, p.stream)) return fail(ASDSM_E_ARG, "plane transforms: N_f too large");
        return check_launch("transform");
    }
    if (d == 3) {
        // backward along canonical axis 1: X -> Y
        j.M = Nf; j.N = Nf; j.K = Nf; j.nbatch = Nc; j.accum = 0;
        j.sAb = 0;   j.sAi = Nf; j.sAk = 1;
        j.sBb = Nf2; j.sBk = Nf; j.sBn = 1;
        j.sCb = Nf2; j.sCi = Nf; j.sCn = 1;
        for (int q = 0; q < nb; ++q) {
            int a, b;
            fine_axes(d, ks[q], a, b);
            j.A[q] = p.dV[b];
            j.B[q] = p.ws.X[1u << ks[q]];
            j.C[q] = p.ws.Y[1u << ks[q]];
        }
        PhaseTimer t(p, ASDSM_PHASE_TRANSFORM, 1, gemm_flops(j), gemm_bytes(j), "k_gemm_f64");
        if (!launch_gemm(j, p.stream)) return fail(ASDSM_E_ARG, "unsupported transform operand layout");
        if (int rc = check_launch("transform")) return rc;
    }
    {
        // backward along canonical axis 0: Y -> out
        j.M = (d == 2) ? Nc : Nf * Nc;
        j.N = Nf; j.K = Nf; j.nbatch = 1; j.accum = accum;
        j.sAb = j.sBb = j.sCb = 0;
        j.sAi = Nf; j.sAk = 1;
        j.sBk = 1;  j.sBn = Nf;
        j.sCi = Nf; j.sCn = 1;
        for (int q = 0; q < nb; ++q) {
            int a, b;
            fine_axes(d, ks[q], a, b);
            j.A[q] = p.ws.Y[1u << ks[q]];
            j.B[q] = p.dV[a];
            j.C[q] = out[ks[q]];
        }
        PhaseTimer t(p, ASDSM_PHASE_TRANSFORM, 1, gemm_flops(j), gemm_bytes(j), "k_gemm_f64");
        if (!launch_gemm(j, p.stream)) return fail(ASDSM_E_ARG, "unsupported transform operand layout");
        if (int rc = check_launch("transform")) return rc;
    }
    return ASDSM_OK;
}

// Direct solve of an intersection mesh (>= 2 coarse axes): in -> out (out += when accum).  X_S and
// Y_S are intermediates (in may be X_S; out may be neither X_S nor Y_S unless it is the plain
// Y_S output without accumulation).
int solve_intersection(Plan &p, unsigned mask, const double *in, double *out, int accum) {
    const MeshDesc &m = p.mesh[mask];
    if (p.line_pos[mask] >= 0) return solve_mesh_line(p, 1, &mask, &in, &out, accum);
    if (m.nfine >= 2) return solve_mesh_nd(p, 1, &mask, &in, &out, accum);  // d = 4, two fine axes
    if (m.nfine == 0) {
        const double B = m.block;
        PhaseTimer t(p, ASDSM_PHASE_LINE, 1, 2.0 * B * B, 8.0 * (B * B + (accum ? 3 : 2) * B));
        launch_dense_modes(1, m.block, p.ddense[mask], in, out, accum, p.stream);
        return check_launch("dense");
    }
    // one fine axis (d = 3 edge meshes): transform, per-mode dense solve, back-transform
    const int f = m.ax[0];
    GemmJob j{};
    j.nbox = 1;
    j.gate = p.gate;
    j.M = m.block; j.N = p.Nf; j.K = p.Nf; j.nbatch = 1;
    j.sAb = j.sBb = j.sCb = 0;
    j.sAi = p.Nf; j.sAk = 1;
    j.sBk = 1;    j.sBn = p.Nf;
    j.sCi = p.Nf; j.sCn = 1;
    {
        j.A[0] = in;
        j.B[0] = p.dW[f];
        j.C[0] = p.ws.Y[mask];
        j.accum = 0;
        PhaseTimer t(p, ASDSM_PHASE_TRANSFORM, 1, gemm_flops(j), gemm_bytes(j), "k_gemm_f64");
        if (!launch_gemm(j, p.stream)) return fail(ASDSM_E_ARG, "unsupported transform operand layout");
        if (int rc = check_launch("transform")) return rc;
    }
    {
        const double B = m.block, nmo = (double)m.nmodes;
        PhaseTimer t(p, ASDSM_PHASE_LINE, 1, 2.0 * nmo * B * B, 8.0 * nmo * (B * B + 2 * B));
        launch_dense_modes(m.nmodes, m.block, p.ddense[mask], p.ws.Y[mask], p.ws.X[mask], 0, p.stream);
        if (int rc = check_launch("dense")) return rc;
    }
    {
        j.A[0] = p.ws.X[mask];
        j.B[0] = p.dV[f];
        j.C[0] = out;
        j.accum = accum;
        PhaseTimer t(p, ASDSM_PHASE_TRANSFORM, 1, gemm_flops(j), gemm_bytes(j), "k_gemm_f64");
        if (!launch_gemm(j, p.stream)) return fail(ASDSM_E_ARG, "unsupported transform operand layout");
        if (int rc = check_launch("transform")) return rc;
    }
    return ASDSM_OK;
}

// Mesh solves with the plan's refinement sweeps: x = M^-1 f, then x += M^-1 (f - A x) per sweep.
// The right-hand side is read from rhs_buf and the solution left in sol_buf.
int solve_aniso_refined(Plan &p, unsigned kbits) {
    double *in[kMaxD] = {}, *out[kMaxD] = {};
    int ns = 0, nb = 0;
    unsigned masks[kMaxD];
    unsigned sweep_bits = 0;  // the meshes that take the sweeps (not those solved on the line alone)
    for (int k = 0; k < p.d; ++k)
        if ((kbits >> k) & 1u) {
            const unsigned m = 1u << k;
            in[k] = rhs_buf(p, m);
            out[k] = sol_buf(p, m);
            if (p.line_block2[m]) continue;
            masks[nb++] = m;
            sweep_bits |= 1u << k;
            ns = std::max(ns, p.sweeps[m]);
        }
    if (int rc = solve_aniso(p, kbits, in, out, 0)) return rc;
    kbits = sweep_bits;
    for (int sweep = 0; sweep < ns; ++sweep) {
        BoxResJob job{};
        job.nbox = nb;
        job.gate = p.gate;
        double *res[kMaxD] = {};
        for (int q = 0; q < nb; ++q) {
            const unsigned m = masks[q];
            const int k = __builtin_ctz(m);
            job.f[q] = in[k];
            job.x[q] = out[k];
            job.out[q] = p.ws.X[m];
            job.m[q] = p.mesh[m];
            res[k] = p.ws.X[m];
        }
        {
            double pts = 0.0;
            for (int q = 0; q < job.nbox; ++q) pts += (double)job.m[q].size;
            PhaseTimer t(p, ASDSM_PHASE_LINE, 1, 2.0 * (2 * p.d + 1) * pts, 24.0 * pts);
            launch_box_residual(p, job, p.stream);
            if (int rc = check_launch("box residual")) return rc;
        }
        if (int rc = solve_aniso(p, kbits, res, out, 1)) return rc;
    }
    return ASDSM_OK;
}

// Mixed-precision error guesses: the anisotropic solves of Algorithm 1 with the residual as source,
// in FP32 (FP32 MFMA transforms with FP32 accumulation, FP32 line elimination, no refinement
// sweeps).  in[k] (FP64 right-hand side) is rounded to FP32 as the first transform stages it; the
// last transform writes the FP64 solution out[k].  F1/F2 hold the FP32 intermediates.
// FP32 error guess on the four anisotropic meshes of a d = 4 plan: the same fast diagonalisation as
// the FP64 solve (each fine axis by its mode transform, Thomas along the coarse axis per mode), in
// FP32 with FP32 MFMA products; the input is rounded while the first product stages it and the last
// product writes the FP64 solution.  Canonical layout of M_k: f0 + N_f (f1 + N_f (f2 + N_f c_k)).
static int solve_aniso32_4(Plan &p, const double *const *in, double *const *out) {
    const int Nf = p.Nf, Nc = p.Nc, nb = 4;
    const long long Nf2 = (long long)Nf * Nf, Nf3 = Nf2 * Nf;
    auto f64 = [](float *x) { return reinterpret_cast<double *>(x); };
    auto cf64 = [](const float *x) { return reinterpret_cast<const double *>(x); };
    int ax[4][3];
    for (int k = 0; k < nb; ++k)
        for (int j = 0, q = 0; j < 4; ++j)
            if (j != k) ax[k][q++] = j;
    auto run = [&](GemmJob &j, bool a64, bool c64, double byte_share) -> int {
        PhaseTimer t(p, ASDSM_PHASE_TRANSFORM, 1, gemm_flops(j), gemm_bytes(j) * byte_share);
        if (!launch_gemm32(j, a64, c64, p.stream)) return fail(ASDSM_E_ARG, "unsupported transform operand layout");
        return check_launch("transform");
    };
    GemmJob j{};
    j.nbox = nb;
    j.gate = p.gate;
    // position 0 (f0), all rows at once: in (FP64) -> F1; backward: F1 -> out (FP64)
    auto pos0 = [&](bool fwd) {
        j.M = (int)(Nf2 * Nc); j.N = Nf; j.K = Nf; j.nbatch = 1; j.accum = 0;
        j.sAb = j.sBb = j.sCb = 0;
        j.sAi = Nf; j.sAk = 1;
        j.sBk = 1;  j.sBn = Nf;
        j.sCi = Nf; j.sCn = 1;
        for (int k = 0; k < nb; ++k) {
            j.A[k] = fwd ? in[k] : cf64(p.ws.F1[k]);
            j.B[k] = cf64(fwd ? p.dW32[ax[k][0]] : p.dV32[ax[k][0]]);
            j.C[k] = fwd ? f64(p.ws.F1[k]) : out[k];
        }
    };
    // position 1 (f1), batched over the N_f N_c slabs (f2, c_k): src -> dst
    auto pos1 = [&](bool fwd, float *const *src, float *const *dst) {
        j.M = Nf; j.N = Nf; j.K = Nf; j.nbatch = Nf * Nc; j.accum = 0;
        j.sAb = 0;   j.sAi = Nf; j.sAk = 1;
        j.sBb = Nf2; j.sBk = Nf; j.sBn = 1;
        j.sCb = Nf2; j.sCi = Nf; j.sCn = 1;
        for (int k = 0; k < nb; ++k) {
            j.A[k] = cf64(fwd ? p.dW32[ax[k][1]] : p.dV32[ax[k][1]]);
            j.B[k] = cf64(src[k]);
            j.C[k] = f64(dst[k]);
        }
    };
    // position 2 (f2), batched over the N_c coarse planes: (N_f x N_f) by (N_f x N_f^2) products
    auto pos2 = [&](bool fwd, float *const *src, float *const *dst) {
        j.M = Nf; j.N = (int)Nf2; j.K = Nf; j.nbatch = Nc; j.accum = 0;
        j.sAb = 0;   j.sAi = Nf;  j.sAk = 1;
        j.sBb = Nf3; j.sBk = Nf2; j.sBn = 1;
        j.sCb = Nf3; j.sCi = Nf2; j.sCn = 1;
        for (int k = 0; k < nb; ++k) {
            j.A[k] = cf64(fwd ? p.dW32[ax[k][2]] : p.dV32[ax[k][2]]);
            j.B[k] = cf64(src[k]);
            j.C[k] = f64(dst[k]);
        }
    };
    float *F1[4], *F2[4];
    for (int k = 0; k < nb; ++k) {
        F1[k] = p.ws.F1[k];
        F2[k] = p.ws.F2[k];
    }
    pos0(true);
    if (int rc = run(j, true, false, 0.75)) return rc;
    pos1(true, F1, F2);
    if (int rc = run(j, false, false, 0.5)) return rc;
    pos2(true, F2, F1);
    if (int rc = run(j, false, false, 0.5)) return rc;
    {
        // FP32 line elimination along the coarse axis on F1 (scratch F2); modes f0 + N_f (f1 + N_f f2)
        LineJob L{};
        L.nbox = nb;
        L.gate = p.gate;
        L.fp32 = 1;
        L.nmodes = Nf3;
        L.ext_a = Nf;
        L.ncoarse = Nc;
        for (int k = 0; k < nb; ++k) {
            L.X[k] = f64(F1[k]);
            L.scratch[k] = f64(F2[k]);
            L.mu_a[k] = p.dmu[ax[k][0]];
            L.mu_b[k] = p.dmu[ax[k][1]];
            L.mu_c[k] = p.dmu[ax[k][2]];
            L.t[k] = p.geo.coarse[k];
        }
        const double lpts = (double)L.nmodes * L.ncoarse * nb;
        PhaseTimer t(p, ASDSM_PHASE_LINE, 1, 8.0 * lpts, 8.0 * lpts);
        launch_line(L, p.stream);
        if (int rc = check_launch("line")) return rc;
    }
    pos2(false, F1, F2);
    if (int rc = run(j, false, false, 0.5)) return rc;
    pos1(false, F2, F1);
    if (int rc = run(j, false, false, 0.5)) return rc;
    pos0(false);
    return run(j, false, true, 0.75);
}

int solve_aniso32(Plan &p, const double *const *in, double *const *out) {
    const int d = p.d, Nf = p.Nf, Nc = p.Nc;
    if (d == 4) return solve_aniso32_4(p, in, out);
    const long long Nf2 = (long long)Nf * Nf;
    const int nb = d;
    auto f64 = [](float *x) { return reinterpret_cast<double *>(x); };
    auto cf64 = [](const float *x) { return reinterpret_cast<const double *>(x); };
    GemmJob j{};
    j.nbox = nb;
    j.gate = p.gate;
    // forward along canonical axis 0: in (FP64) -> F1
    j.M = (d == 2) ? Nc : Nf * Nc;
    j.N = Nf; j.K = Nf; j.nbatch = 1; j.accum = 0;
    j.sAb = j.sBb = j.sCb = 0;
    j.sAi = Nf; j.sAk = 1;
    j.sBk = 1;  j.sBn = Nf;
    j.sCi = Nf; j.sCn = 1;
    for (int k = 0; k < nb; ++k) {
        int a, b;
        fine_axes(d, k, a, b);
        j.A[k] = in[k];
        j.B[k] = cf64(p.dW32[a]);
        j.C[k] = f64(p.ws.F1[k]);
    }
    {
        PhaseTimer t(p, ASDSM_PHASE_TRANSFORM, 1, gemm_flops(j), gemm_bytes(j) * 0.75);
        if (!launch_gemm32(j, true, false, p.stream)) return fail(ASDSM_E_ARG, "unsupported transform operand layout");
        if (int rc = check_launch("transform")) return rc;
    }
    if (d == 3) {
        // forward along canonical axis 1, batched over the coarse slabs: F1 -> F2
        j.M = Nf; j.N = Nf; j.K = Nf; j.nbatch = Nc;
        j.sAb = 0;   j.sAi = Nf; j.sAk = 1;
        j.sBb = Nf2; j.sBk = Nf; j.sBn = 1;
        j.sCb = Nf2; j.sCi = Nf; j.sCn = 1;
        for (int k = 0; k < nb; ++k) {
            int a, b;
            fine_axes(d, k, a, b);
            j.A[k] = cf64(p.dW32[b]);
            j.B[k] = cf64(p.ws.F1[k]);
            j.C[k] = f64(p.ws.F2[k]);
        }
        PhaseTimer t(p, ASDSM_PHASE_TRANSFORM, 1, gemm_flops(j), gemm_bytes(j) * 0.5);
        if (!launch_gemm32(j, false, false, p.stream)) return fail(ASDSM_E_ARG, "unsupported transform operand layout");
        if (int rc = check_launch("transform")) return rc;
    }
    {
        // FP32 line elimination along the coarse axis: d = 2 on F1 (scratch F2), d = 3 on F2
        LineJob L{};
        L.nbox = nb;
        L.gate = p.gate;
        L.fp32 = 1;
        L.nmodes = (d == 2) ? Nf : Nf2;
        L.ext_a = Nf;
        L.ncoarse = Nc;
        for (int k = 0; k < nb; ++k) {
            int a, b;
            fine_axes(d, k, a, b);
            L.X[k] = f64((d == 2) ? p.ws.F1[k] : p.ws.F2[k]);
            L.scratch[k] = f64((d == 2) ? p.ws.F2[k] : p.ws.F1[k]);
            L.mu_a[k] = p.dmu[a];
            L.mu_b[k] = (d == 3) ? p.dmu[b] : nullptr;
            L.t[k] = p.geo.coarse[k];
        }
        const double lpts = (double)L.nmodes * L.ncoarse * nb;
        PhaseTimer t(p, ASDSM_PHASE_LINE, 1, 8.0 * lpts, 8.0 * lpts);
        launch_line(L, p.stream);
        if (int rc = check_launch("line")) return rc;
    }
    if (d == 3) {
        // backward along canonical axis 1: F2 -> F1
        j.M = Nf; j.N = Nf; j.K = Nf; j.nbatch = Nc;
        j.sAb = 0;   j.sAi = Nf; j.sAk = 1;
        j.sBb = Nf2; j.sBk = Nf; j.sBn = 1;
        j.sCb = Nf2; j.sCi = Nf; j.sCn = 1;
        for (int k = 0; k < nb; ++k) {
            int a, b;
            fine_axes(d, k, a, b);
            j.A[k] = cf64(p.dV32[b]);
            j.B[k] = cf64(p.ws.F2[k]);
            j.C[k] = f64(p.ws.F1[k]);
        }
        PhaseTimer t(p, ASDSM_PHASE_TRANSFORM, 1, gemm_flops(j), gemm_bytes(j) * 0.5);
        if (!launch_gemm32(j, false, false, p.stream)) return fail(ASDSM_E_ARG, "unsupported transform operand layout");
        if (int rc = check_launch("transform")) return rc;
    }
    {
        // backward along canonical axis 0: F1 -> out (FP64)
        j.M = (d == 2) ? Nc : Nf * Nc;
        j.N = Nf; j.K = Nf; j.nbatch = 1; j.accum = 0;
        j.sAb = j.sBb = j.sCb = 0;
        j.sAi = Nf; j.sAk = 1;
        j.sBk = 1;  j.sBn = Nf;
        j.sCi = Nf; j.sCn = 1;
        for (int k = 0; k < nb; ++k) {
            int a, b;
            fine_axes(d, k, a, b);
            j.A[k] = cf64(p.ws.F1[k]);
            j.B[k] = cf64(p.dV32[a]);
            j.C[k] = out[k];
        }
        PhaseTimer t(p, ASDSM_PHASE_TRANSFORM, 1, gemm_flops(j), gemm_bytes(j) * 0.75);
        if (!launch_gemm32(j, false, true, p.stream)) return fail(ASDSM_E_ARG, "unsupported transform operand layout");
        if (int rc = check_launch("transform")) return rc;
    }
    return ASDSM_OK;
}

int solve_intersection_refined(Plan &p, unsigned mask) {
    const double *in = rhs_buf(p, mask);
    double *out = sol_buf(p, mask);
    if (int rc = solve_intersection(p, mask, in, out, 0)) return rc;
    for (int sweep = 0; sweep < p.sweeps[mask]; ++sweep) {
        BoxResJob job{};
        job.nbox = 1;
        job.f[0] = in;
        job.x[0] = out;
        job.out[0] = p.ws.X[mask];
        job.m[0] = p.mesh[mask];
        {
            double pts = 0.0;
            for (int q = 0; q < job.nbox; ++q) pts += (double)job.m[q].size;
            PhaseTimer t(p, ASDSM_PHASE_LINE, 1, 2.0 * (2 * p.d + 1) * pts, 24.0 * pts);
            launch_box_residual(p, job, p.stream);
            if (int rc = check_launch("box residual")) return rc;
        }
        if (int rc = solve_intersection(p, mask, p.ws.X[mask], out, 1)) return rc;
    }
    return ASDSM_OK;
}

void result_pointers(const Plan &p, const double *res[kMaxMeshes]) {
    for (unsigned s = 0; s < kMaxMeshes; ++s) res[s] = nullptr;
    for (unsigned s = 1; s < (1u << p.d); ++s) res[s] = sol_buf(p, s);
}

void gather_pointers(const Plan &p, double *g[kMaxMeshes]) {
    for (unsigned s = 0; s < kMaxMeshes; ++s) g[s] = nullptr;
    for (unsigned s = 1; s < (1u << p.d); ++s) g[s] = rhs_buf(p, s);
}


// Points of the anisotropic meshes (the refinement loop's submeshes), of all submeshes, of one
// Dirichlet face and of the holes.
double aniso_points(const Plan &p) {
    double n = 0.0;
    for (int k = 0; k < p.d; ++k) n += (double)p.mesh[1u << k].size;
    return n;
}
double submesh_points(const Plan &p) {
    double n = 0.0;
    for (unsigned m = 1; m < (1u << p.d); ++m) n += (double)p.mesh[m].size;
    return n;
}
double face_points(const Plan &p) { return std::pow((double)p.Nf, p.d - 1); }
double hole_points(const Plan &p) { return std::pow((double)(p.Nc + 1) * (p.geo.n - 1), p.d); }
// Hole solves: forward and backward mode transforms along d-1 axes (2 (n-1) flops each per point)
// and a Thomas line (8 flops per point).
double filler_flops(const Plan &p) { return hole_points(p) * (4.0 * (p.d - 1) * (p.geo.n - 1) + 8.0); }

// Launches of the cross-point and merge kernels (Algorithm 2) for this d.
int skeleton_launches(const Plan &p) { return p.d == 4 ? 4 : (merge_forms_discrepancies(p) ? 1 : 2); }

int read_scalars(Plan &p) {
    ASDSM_HIP_CHECK(hipMemcpyAsync(p.hscal, p.ws.scal, kScalCount * sizeof(double), hipMemcpyDeviceToHost, p.stream));
    ASDSM_HIP_CHECK(hipStreamSynchronize(p.stream));
    return ASDSM_OK;
}

// A-posteriori refinement count.  The plan's a-priori count uses eps * prod cond(V_j), which bounds
// the worst case; the error actually reached is usually orders of magnitude smaller.  With the
// workspace attached, each mesh group that was given sweeps is solved once for a reproducible
// random right-hand side and refined until a sweep changes the solution by less than 1e-12
// (relative 2-norm); the sweeps before that one are what the solves keep.
int calibrate_sweeps(Plan &p) {
    const int d = p.d;
    const int kMax = 10;
    // groups: all anisotropic meshes together, then each intersection mesh
    unsigned groups[kMaxMeshes];
    int ng = 0;
    {
        unsigned all = 0;
        for (int k = 0; k < d; ++k)
            if (p.sweeps[1u << k] > 0) all |= 1u << k;
        if (all) groups[ng++] = 0x100u | all;  // tag: anisotropic batch
        for (unsigned m = 1; m < (1u << d); ++m)
            if (__builtin_popcount(m) >= 2 && p.sweeps[m] > 0) groups[ng++] = m;
    }
    for (int gi = 0; gi < ng; ++gi) {
        const bool aniso = (groups[gi] & 0x100u) != 0;
        const unsigned kbits = groups[gi] & 0xFFu;
        unsigned masks[kMaxD];
        int nb = 0;
        if (aniso) {
            for (int k = 0; k < d; ++k)
                if ((kbits >> k) & 1u) masks[nb++] = 1u << k;
        } else {
            masks[nb++] = kbits;
        }
        // right-hand sides, plain solves
        double *in[kMaxD] = {}, *out[kMaxD] = {}, *tmp[kMaxD] = {}, *resid[kMaxD] = {};
        double *temps[2] = {p.ws.e, p.ws.r};  // fine-mesh work vectors are free at this point
        for (int q = 0; q < nb; ++q) {
            const unsigned m = masks[q];
            const long long n = p.mesh[m].size;
            const int slot = aniso ? __builtin_ctz(m) : 0;
            in[slot] = rhs_buf(p, m);
            out[slot] = sol_buf(p, m);
            // one fine vector holds two meshes (N_c N_f^(d-1) points each, 2 N_c < N_f)
            tmp[slot] = (q < 2) ? temps[q] : p.ws.u2 + (q - 2) * n;
            resid[slot] = p.ws.X[m];
            launch_fill_random(in[slot], n, 0x5EEDull * (m + 1), p.stream);
        }
        if (aniso) {
            if (int rc = solve_aniso(p, kbits, in, out, 0)) return rc;
        } else {
            if (int rc = solve_intersection(p, masks[0], in[0], out[0], 0)) return rc;
        }
        int needed = kMax;
        for (int sweep = 1; sweep <= kMax; ++sweep) {
            BoxResJob job{};
            job.nbox = nb;
            for (int q = 0; q < nb; ++q) {
                const unsigned m = masks[q];
                const int slot = aniso ? __builtin_ctz(m) : 0;
                job.f[q] = in[slot];
                job.x[q] = out[slot];
                job.out[q] = resid[slot];
                job.m[q] = p.mesh[m];
            }
            launch_box_residual(p, job, p.stream);
            if (aniso) {
                if (int rc = solve_aniso(p, kbits, resid, tmp, 0)) return rc;
            } else {
                if (int rc = solve_intersection(p, masks[0], resid[0], tmp[0], 0)) return rc;
            }
            const double *xs[2 * kMaxD];
            long long ns[2 * kMaxD];
            int nx = 0;
            for (int q = 0; q < nb; ++q) {
                const unsigned m = masks[q];
                const int slot = aniso ? __builtin_ctz(m) : 0;
                xs[nx] = tmp[slot];
                ns[nx++] = p.mesh[m].size;
            }
            launch_sumsq(p, xs, ns, nx, p.stream);
            if (int rc = read_scalars(p)) return rc;
            double corr[kMaxD];
            for (int q = 0; q < nb; ++q) corr[q] = p.hscal[kScalEnorm2 + q];
            nx = 0;
            for (int q = 0; q < nb; ++q) {
                const unsigned m = masks[q];
                const int slot = aniso ? __builtin_ctz(m) : 0;
                xs[nx] = out[slot];
                ns[nx++] = p.mesh[m].size;
            }
            launch_sumsq(p, xs, ns, nx, p.stream);
            if (int rc = read_scalars(p)) return rc;
            double worst = 0.0;
            for (int q = 0; q < nb; ++q) {
                const double sol = p.hscal[kScalEnorm2 + q];
                const double ratio = (sol > 0.0) ? std::sqrt(corr[q] / sol) : 0.0;
                if (!std::isfinite(ratio)) return fail(ASDSM_E_NUMERIC, "non-finite value while calibrating refinement");
                worst = std::max(worst, ratio);
            }
            double *ys[kMaxD];
            const double *xa[kMaxD];
            for (int q = 0; q < nb; ++q) {
                const unsigned m = masks[q];
                const int slot = aniso ? __builtin_ctz(m) : 0;
                ys[q] = out[slot];
                xa[q] = tmp[slot];
            }
            long long nmax = 0;
            for (int q = 0; q < nb; ++q) nmax = std::max(nmax, p.mesh[masks[q]].size);
            if (nb == 1 || aniso) {
                // every anisotropic mesh has the same size
                launch_axpy(ys, xa, nmax, nb, p.stream);
            }
            if (int rc = check_launch("calibration")) return rc;
            if (worst < 1e-12) {
                needed = sweep - 1;
                break;
            }
        }
        if (needed >= kMax)
            return fail(ASDSM_E_UNSUPPORTED, "refinement of the fast-diagonalisation solves does not converge");
        for (int q = 0; q < nb; ++q) p.sweeps[masks[q]] = needed;
    }
    ASDSM_HIP_CHECK(hipStreamSynchronize(p.stream));
    return ASDSM_OK;
}

// Algorithm 1 with the source: u^(0) into u, then r = b - A u^(0) with its gathers, ||b||, ||r_0||
// and the start of the device-side stopping rule.
int initial_guess(Plan &p, const double *s, const double *g, double *u) {
    const unsigned nm = 1u << p.d;
    {
        PhaseTimer t(p, ASDSM_PHASE_RHS, (int)nm, 0.0,
                     8.0 * (2.0 * (double)p.geo.NF + 2.0 * p.d * face_points(p) + submesh_points(p)));
        launch_rhs(p, 0, s, g, p.ws.b, true, p.stream);
        for (unsigned m = 1; m < nm; ++m) launch_rhs(p, m, s, g, rhs_buf(p, m), false, p.stream);
        if (int rc = check_launch("rhs")) return rc;
    }
    if (int rc = solve_aniso_refined(p, nm - 1)) return rc;
    for (unsigned m = 1; m < nm; ++m)
        if (__builtin_popcount(m) >= 2)
            if (int rc = solve_intersection_refined(p, m)) return rc;
    const double *res[kMaxMeshes];
    result_pointers(p, res);
    {
        PhaseTimer t(p, ASDSM_PHASE_SKELETON, skeleton_launches(p), 0.0,
                     8.0 * (submesh_points(p) + aniso_points(p)));
        launch_crosspoints(p, 0, res, p.stream);
        launch_merge(p, 0, res, p.stream);
        if (int rc = check_launch("skeleton")) return rc;
    }
    {
        PhaseTimer t(p, ASDSM_PHASE_FILLER, 1, filler_flops(p),
                     8.0 * ((double)p.geo.NF + hole_points(p) + aniso_points(p)));
        if (!launch_filler(p, p.ws.b, u, p.stream))
            return fail(ASDSM_E_ARG, "hole solve: unsupported shape");
        if (int rc = check_launch("filler")) return rc;
    }
    {
        PhaseTimer t(p, ASDSM_PHASE_UPDATE, 1, 2.0 * (2 * p.d + 1) * (double)p.geo.NF,
                     8.0 * (3.0 * (double)p.geo.NF + aniso_points(p)));
        double *gat[kMaxMeshes];
        gather_pointers(p, gat);
        launch_update_residual(p, u, nullptr, nullptr, gat, kFinInit, p.stream);
        if (int rc = check_launch("residual")) return rc;
    }
    return ASDSM_OK;
}

// The error guess of a refinement step (Algorithm 1 with the residual as source): the anisotropic
// solves, their normalisation, the cross points and the merge into the Y buffers.
int error_guess(Plan &p) {
    if (p.prec32) {
        const double *in[kMaxD] = {};
        double *out[kMaxD] = {};
        for (int k = 0; k < p.d; ++k) {
            in[k] = rhs_buf(p, 1u << k);
            out[k] = sol_buf(p, 1u << k);
        }
        if (int rc = solve_aniso32(p, in, out)) return rc;
    } else {
        // with the plane kernel, or with line axes whose backward transforms run in one GEMM launch
        // (d = 3), the backward transforms also leave the partial sums of ||e_k||^2 that the
        // skeleton kernels reduce themselves (no separate norm launches)
        bool fused = plane_transforms(p);
        if (!fused && p.line_aniso && p.d == 3) {
            fused = true;
            for (int k = 1; k < 3; ++k) fused = fused && p.line_pos[1u << k] == p.line_pos[1u];
            for (int k = 0; k < 3; ++k) fused = fused && !p.line_block2[1u << k] && !p.line_cmodes[1u << k];
        }
        p.norm_partials = fused ? p.ws.partials : nullptr;
        p.norm_nblk = p.Nc * ((p.Nf + 15) / 16);  // the plane kernel's count (the GEMM sets its own)
        const int rc = solve_aniso_refined(p, (1u << p.d) - 1);
        if (!fused) p.norm_partials = nullptr;
        if (rc) {
            p.norm_partials = nullptr;
            return rc;
        }
    }
    const double *res[kMaxMeshes];
    result_pointers(p, res);
    PhaseTimer t(p, ASDSM_PHASE_SKELETON, skeleton_launches(p) + (p.norm_partials ? 0 : 1), 0.0,
                 24.0 * aniso_points(p));
    if (!p.norm_partials) launch_box_norms(p, res, p.stream);
    launch_crosspoints(p, 1, res, p.stream);
    launch_merge(p, 1, res, p.stream);
    p.norm_partials = nullptr;
    return check_launch("skeleton");
}

// One refinement step of Algorithm 4 from u_cur (with r and its gathers current) into u_next.  All
// of its kernels return at once when the device stopping rule has fired (p.gate), so steps can be
// queued (or replayed from a graph) ahead of the host's check.
int refine_step(Plan &p, const double *u_cur, double *u_next) {
    if (int rc = error_guess(p)) return rc;
    {
        PhaseTimer t(p, ASDSM_PHASE_FILLER, 1, filler_flops(p),
                     8.0 * ((double)p.geo.NF + aniso_points(p)), "hole filler (error guess)");
        if (!launch_filler(p, nullptr, p.ws.e, p.stream))
            return fail(ASDSM_E_ARG, "hole solve: unsupported shape");
        if (int rc = check_launch("filler")) return rc;
    }
    {
        PhaseTimer t(p, ASDSM_PHASE_DOTS, 1, (4.0 * p.d + 6.0) * (double)p.geo.NF, 16.0 * (double)p.geo.NF,
                     "fine dots pass (+ its finalize)");
        launch_dots(p, p.stream);
        if (int rc = check_launch("dots")) return rc;
    }
    {
        PhaseTimer t(p, ASDSM_PHASE_UPDATE, 1, (4.0 * p.d + 6.0) * (double)p.geo.NF,
                     8.0 * (5.0 * (double)p.geo.NF + aniso_points(p)), "fine update pass (+ its finalize)");
        double *gat[kMaxMeshes];
        gather_pointers(p, gat);
        launch_update_residual(p, u_cur, p.ws.e, u_next, gat, kFinIter, p.stream);
        if (int rc = check_launch("update")) return rc;
    }
    return ASDSM_OK;
}

// Skeleton-sparse refinement step (d = 3): the same error guess, then only what the next step and
// the line search need -- the error guess on the hole layers next to the coarse planes (the filler
// in adjacent-layer mode), q = A e and <r, q>, <q, q> on the skeleton, and u += s e, r -= s q with
// the gathers on the skeleton.  The fine u is rebuilt from the skeleton when the loop ends.
int sparse_step(Plan &p) {
    // With the update fused (p.upd_fused), the previous step's update and stopping rule are pending
    // on the device (k_skel_dots leaves them): this step's forward transform applies the update and
    // the backward transform, in one extra block, the stopping rule.  Otherwise the previous step's
    // stopping rule alone is pending (k_skel_update leaves it): with line-axis meshes (FP64) this
    // step's first launch is a transform GEMM, which applies it in one extra block beside its tiles;
    // otherwise a launch of its own applies it first.
    bool transformed = false;  // some anisotropic mesh has a transformed fine axis
    for (int k = 0; k < p.d; ++k) transformed = transformed || !p.line_block2[1u << k];
    const bool carry = p.line_aniso && !p.prec32 && transformed;
    if (p.upd_fused) {
        p.upd_carry = true;
    } else if (carry) {
        p.fin_carry = true;
    } else {
        PhaseTimer t(p, ASDSM_PHASE_UPDATE, 1, 0.0, 0.0, "k_finalize_pending");
        launch_finalize_pending(p, p.stream);
    }
    const int erc = error_guess(p);
    const bool missed = p.fin_carry || p.upd_carry;
    p.fin_carry = false;
    p.upd_carry = false;
    p.fin_res_nblk = 0;
    if (erc) return erc;
    if (missed) return fail(ASDSM_E_UNSUPPORTED, "skeleton-sparse step: no transform carried the update");
    if (p.upd_fused) p.sr_par ^= 1;  // the forward transform has written the next residual
    const double skel = aniso_points(p);  // skeleton points counted once per mesh
    {
        PhaseTimer t(p, ASDSM_PHASE_FILLER, 1, filler_flops(p), 8.0 * (3.0 * skel), "hole filler (layer mode)");
        if (!launch_filler(p, nullptr, nullptr, p.stream, nullptr, true))
            return fail(ASDSM_E_ARG, "hole solve: unsupported shape");
        if (int rc = check_launch("filler (layers)")) return rc;
    }
    {
        PhaseTimer t(p, ASDSM_PHASE_DOTS, 1, 17.0 * skel, 8.0 * 5.0 * skel, "k_skel_dots");
        launch_skel_dots(p, p.stream);
        if (int rc = check_launch("skeleton dots")) return rc;
    }
    if (!p.upd_fused) {
        PhaseTimer t(p, ASDSM_PHASE_UPDATE, 1, 5.0 * skel, 8.0 * 7.0 * skel, "k_skel_update");
        double *gat[kMaxMeshes];
        gather_pointers(p, gat);
        launch_skel_update(p, gat, p.stream);
        if (int rc = check_launch("skeleton update")) return rc;
    }
    return ASDSM_OK;
}

// The skeleton-sparse update can ride on the next forward transform: d = 3 with every anisotropic
// mesh solved by its line axis at canonical position 1 (one FP64 forward transform GEMM over the
// three meshes, mode-major) and no refinement sweeps (which would re-read the right-hand side).
bool sparse_fusable(const Plan &p) {
    if (!p.sparse || p.d != 3 || !p.line_aniso || p.prec32) return false;
    for (int k = 0; k < 3; ++k)
        if (p.line_pos[1u << k] != 1 || p.sweeps[1u << k] != 0 || p.mesh[1u << k].nfine != 2) return false;
    return true;
}

// A refinement step with a learned proposal (p.learn_net, bound to this plan, n = N_f): the
// network maps r_k to a correction e, the line search of Algorithm 4 gives <r, Ae> and <Ae, Ae>, and
// a device-side test accepts the proposal when the optimal step lowers ||r|| by p.learn_factor.  The
// update u_next = u_cur + w e runs only if accepted, the plain step (refine_step) only if not; both
// are gated by the test's flags, so the step needs no host round trip and can be captured.
int learned_step(Plan &p, const double *u_cur, double *u_next) {
    Net &net = *p.learn_net;
    const int *done = p.gate;
    const double nf = (double)p.geo.NF;
    {
        // MFMA work of the four convolutions (padded channels) and the bytes of their operands
        double conv_flops = 0.0, conv_bytes = 0.0;
        for (int l = 0; l < kNetLayers; ++l) {
            conv_flops += 2.0 * 27.0 * kNetCinP[l] * kNetCoutP[l] * nf;
            conv_bytes += 4.0 * (kNetCinP[l] + (l + 1 < kNetLayers ? kNetCinP[l + 1] : 1)) * nf;
        }
        PhaseTimer t(p, ASDSM_PHASE_LEARNED, kNetLayers + 4, conv_flops + (4.0 * p.d + 6.0) * nf,
                     conv_bytes + (8.0 + 64.0) * nf + (4.0 + 8.0) * nf + 16.0 * nf);
        const int off[3] = {0, 0, 0};
        net_features(net.n, net.Nf, net.nsp, off, p.ws.r, p.ws.scal + kScalRnorm2, 0.0, net.pe, net.act[0],
                     nullptr, done, p.stream);
        for (int l = 0; l < kNetLayers; ++l) {
            const bool last = (l == kNetLayers - 1);
            net_conv_fwd(net.n, kNetCinP[l], kNetCout[l], last ? 1 : 32, !last, net.act[l], l > 0, net.Wb[l],
                         net.P + net.bofs[l], net.act[l + 1], !last, done, p.stream);
        }
        net_correction(p.geo.NF, net.act[kNetLayers], p.ws.scal + kScalRnorm2, net.h2a, p.ws.e, done, p.stream);
        launch_dots(p, p.stream);
        net_accept(p.ws.scal, &p.ws.state->done, &p.ws.state->learned, p.learn_factor, net.skip, p.stream);
        if (int rc = check_launch("learned proposal")) return rc;
    }
    p.gate = net.skip;  // skip[0]: not accepted (or done)
    {
        PhaseTimer t(p, ASDSM_PHASE_UPDATE, 1, (4.0 * p.d + 6.0) * nf, 8.0 * (5.0 * nf + aniso_points(p)));
        double *gat[kMaxMeshes];
        gather_pointers(p, gat);
        launch_update_residual(p, u_cur, p.ws.e, u_next, gat, kFinIter, p.stream);
    }
    p.gate = net.skip + 1;  // skip[1]: accepted (or done)
    const int rc = refine_step(p, u_cur, u_next);
    p.gate = done;
    if (rc != ASDSM_OK) return rc;
    return check_launch("learned update");
}

int step(Plan &p, const double *u_cur, double *u_next) {
    if (p.learn_net) return learned_step(p, u_cur, u_next);
    if (p.sparse) return sparse_step(p);
    return refine_step(p, u_cur, u_next);
}

int require_ws(const Plan &p) {
    if (!p.ws_base) return fail(ASDSM_E_WORKSPACE, "no workspace attached (asdsm_set_workspace)");
    return ASDSM_OK;
}

// Two events (no timing) behind which the graph loop checks the loop state (created once per plan).
int ensure_loop_events(Plan &p) {
    for (int i = 0; i < 2; ++i)
        if (!p.loop_ev[i]) ASDSM_HIP_CHECK(hipEventCreateWithFlags(&p.loop_ev[i], hipEventDisableTiming));
    return ASDSM_OK;
}

int read_state_on(Plan &p, hipStream_t st) {
    ASDSM_HIP_CHECK(hipMemcpyAsync(p.hstate, p.ws.state, sizeof(IterState), hipMemcpyDeviceToHost, st));
    ASDSM_HIP_CHECK(hipStreamSynchronize(st));
    return ASDSM_OK;
}

int read_state(Plan &p) {
    ASDSM_HIP_CHECK(hipMemcpyAsync(p.hstate, p.ws.state, sizeof(IterState), hipMemcpyDeviceToHost, p.stream));
    ASDSM_HIP_CHECK(hipStreamSynchronize(p.stream));
    return ASDSM_OK;
}

void destroy_graph(Plan &p) {
    if (p.graph_exec) (void)hipGraphExecDestroy(p.graph_exec);
    if (p.graph) (void)hipGraphDestroy(p.graph);
    p.graph_exec = nullptr;
    p.graph = nullptr;
    p.graph_u = nullptr;
    p.graph_gen = 0;
}

// Something the captured launches depend on changed (workspace, tile, sweep counts): drop the
// plan's graph and let every batch graph holding this plan see the new generation.
void plan_changed(Plan &p) {
    ++p.generation;
    destroy_graph(p);
}

// Capture two gated refinement steps (u -> u2 -> u) into a graph, replayed by the solve loop.  The
// capture happens on a private stream (the caller's may be the null stream); the graph is launched
// on the plan's stream.  It holds kernel nodes only (no memset or copy nodes).
int build_graph(Plan &p, double *u) {
    destroy_graph(p);
    if (!p.capture_stream) ASDSM_HIP_CHECK(hipStreamCreateWithFlags(&p.capture_stream, hipStreamNonBlocking));
    hipStream_t saved = p.stream;
    p.stream = p.capture_stream;
    ASDSM_HIP_CHECK(hipStreamBeginCapture(p.capture_stream, hipStreamCaptureModeThreadLocal));
    int rc = step(p, u, p.ws.u2);
    if (rc == ASDSM_OK) rc = step(p, p.ws.u2, u);
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamEndCapture(p.capture_stream, &graph);
    p.stream = saved;
    if (rc != ASDSM_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return rc;
    }
    if (e != hipSuccess) return fail(ASDSM_E_DEVICE, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
    p.graph = graph;
    e = hipGraphInstantiate(&p.graph_exec, graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        destroy_graph(p);
        return fail(ASDSM_E_DEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
    }
    p.graph_u = u;
    p.graph_gen = p.generation;
    p.graph_prec32 = p.prec32;
    p.graph_sparse = p.sparse;
    p.graph_net_serial = p.learn_net ? p.learn_net->serial : 0;
    p.graph_net_ws = p.learn_net ? p.learn_net->ws : nullptr;
    p.graph_factor = p.learn_factor;
    return ASDSM_OK;
}

// Events of a profiled call, destroyed on every exit path.
struct CallEvents {
    hipEvent_t tb = nullptr, te = nullptr;
    ~CallEvents() {
        if (tb) (void)hipEventDestroy(tb);
        if (te) (void)hipEventDestroy(te);
    }
};

// Autotuner: time the anisotropic solve (the four FP64 mode transforms and the line elimination)
// with every transform tile shape on reproducible random right-hand sides and keep the fastest.
int autotune_impl(Plan &p, int reps, int *best_tile, double *best_ms) {
    if (int rc = require_ws(p)) return rc;
    if (reps < 1 || reps > 1000) return fail(ASDSM_E_ARG, "repeats must be in 1..1000");
    const unsigned kbits = (1u << p.d) - 1;
    double *in[kMaxD] = {}, *out[kMaxD] = {};
    for (int k = 0; k < p.d; ++k) {
        const unsigned m = 1u << k;
        in[k] = rhs_buf(p, m);
        out[k] = sol_buf(p, m);
        launch_fill_random(in[k], p.mesh[m].size, 0x7A11ull * (m + 1), p.stream);
    }
    p.gate = nullptr;
    CallEvents ev;
    ASDSM_HIP_CHECK(hipEventCreate(&ev.tb));
    ASDSM_HIP_CHECK(hipEventCreate(&ev.te));
    const int saved = p.tile_aniso;
    int best = saved;
    double best_t = 1e300;
    for (int tile : kGemmTiles) {
        if (tile == kTilePlane && (p.d != 3 || p.Nf > kPlaneMaxNf || p.line_aniso)) continue;
        p.tile_aniso = tile;
        int rc = solve_aniso(p, kbits, in, out, 0);  // warm-up (code objects, caches)
        if (rc == ASDSM_OK) {
            ASDSM_HIP_CHECK(hipEventRecord(ev.tb, p.stream));
            for (int r = 0; r < reps && rc == ASDSM_OK; ++r) rc = solve_aniso(p, kbits, in, out, 0);
            ASDSM_HIP_CHECK(hipEventRecord(ev.te, p.stream));
        }
        if (rc != ASDSM_OK) {
            p.tile_aniso = saved;
            return rc;
        }
        ASDSM_HIP_CHECK(hipEventSynchronize(ev.te));
        float ms = 0.f;
        ASDSM_HIP_CHECK(hipEventElapsedTime(&ms, ev.tb, ev.te));
        const double t = (double)ms / reps;
        if (t < best_t) {
            best_t = t;
            best = tile;
        }
    }
    p.tile_aniso = best;
    if (p.line_aniso) {
        // modes per workgroup of the line solve: from the size rule, then each valid count
        const int saved_tm = p.cr_tm;
        int best_tm = 0;
        const MeshDesc &m = p.mesh[1];
        const long long nmodes = m.nmodes / m.ext[p.line_pos[1]];
        for (int tm : {0, 1, 2, 4, 8}) {
            if (tm > 0 && cr2_modes_per_group(p.Nf, p.level, m.block, nmodes, p.d, tm) != tm) continue;
            p.cr_tm = tm;
            int rc = solve_aniso(p, kbits, in, out, 0);
            if (rc == ASDSM_OK) {
                ASDSM_HIP_CHECK(hipEventRecord(ev.tb, p.stream));
                for (int r = 0; r < reps && rc == ASDSM_OK; ++r) rc = solve_aniso(p, kbits, in, out, 0);
                ASDSM_HIP_CHECK(hipEventRecord(ev.te, p.stream));
            }
            if (rc != ASDSM_OK) {
                p.cr_tm = saved_tm;
                return rc;
            }
            ASDSM_HIP_CHECK(hipEventSynchronize(ev.te));
            float ms = 0.f;
            ASDSM_HIP_CHECK(hipEventElapsedTime(&ms, ev.tb, ev.te));
            const double t = (double)ms / reps;
            if (t < best_t) {
                best_t = t;
                best_tm = tm;
            }
        }
        p.cr_tm = best_tm;
    }
    plan_changed(p);  // captured launches carry the old tile choice
    if (best_tile) *best_tile = best;
    if (best_ms) *best_ms = best_t;
    return ASDSM_OK;
}

// Options with their defaults, validated.
int normalize_opts(const asdsm_opts *o, asdsm_opts &opt) {
    if (o) {
        opt = *o;
    } else {
        std::memset(&opt, 0, sizeof opt);
        opt.max_iter = 50;
        opt.rtol = 1e-10;
        opt.stag_window = 3;
        opt.stag_eta = 1e-3;
    }
    if (opt.max_iter < 0 || opt.max_iter >= kHistCap || !(opt.rtol >= 0.0) || opt.stag_window < 0 ||
        !(opt.stag_eta >= 0.0) || !(opt.stag_eta < 1.0))
        return fail(ASDSM_E_ARG, "invalid options (max_iter must be < " + std::to_string(kHistCap) + ")");
    if (opt.precision != ASDSM_PREC_FP64 && opt.precision != ASDSM_PREC_FP32)
        return fail(ASDSM_E_ARG, "invalid precision");
    if (opt.skeleton != 0 && opt.skeleton != 1) return fail(ASDSM_E_ARG, "invalid skeleton flag");
    return ASDSM_OK;
}

// The skeleton-sparse loop runs on d = 3 plans (every hole size: both fillers write the layers next
// to the coarse planes).
int check_sparse(const Plan &p, const asdsm_opts &opt) {
    if (opt.skeleton && p.d != 3) return fail(ASDSM_E_UNSUPPORTED, "skeleton-sparse refinement needs d = 3");
    return ASDSM_OK;
}

// Everything before the refinement loop, enqueued on p.stream: the loop state and the random
// cross-point choices of every step of this call, then Algorithm 1 (or the residual of the resumed
// iterate).  Leaves p.gate pointing at the device stopping flag.
int begin_solve(Plan &p, const double *s, const double *g, double *u, const asdsm_opts &opt) {
    if (!s || !g || !u) return fail(ASDSM_E_ARG, "s, g and u must be non-NULL device pointers");
    if (int rc = require_ws(p)) return rc;
    p.prec32 = (opt.precision == ASDSM_PREC_FP32) && p.fp32_ok;
    p.sparse = opt.skeleton != 0;
    p.upd_fused = sparse_fusable(p);
    p.upd_carry = false;
    p.fin_carry = false;
    p.fin_res_nblk = 0;
    p.sr_par = 0;
    for (int q = 0; q < ASDSM_NPHASE; ++q) {
        p.phase_ms[q] = 0.0;
        p.phase_launches[q] = 0;
        p.phase_flops[q] = 0.0;
        p.phase_bytes[q] = 0.0;
    }
    p.kern_recs.clear();
    IterState &hs = *p.hstate;
    std::memset(&hs, 0, sizeof hs);
    hs.status = ASDSM_MAXITER;
    hs.max_iter = opt.max_iter;
    hs.stag_window = opt.stag_window;
    hs.rtol = opt.rtol;
    hs.stag_eta = opt.stag_eta;
    const int64_t k0 = opt.resume ? opt.k0 : 0;
    for (int i = 0; i < opt.max_iter; ++i) axis_permutation(p.seed, k0 + i, p.d, p.hperm + kMaxD * i);
    for (int j = 0; j < kMaxD; ++j) hs.perm[j] = (opt.max_iter > 0) ? p.hperm[j] : j;
    ASDSM_HIP_CHECK(hipMemcpyAsync(p.ws.state, &hs, sizeof hs, hipMemcpyHostToDevice, p.stream));
    if (opt.max_iter > 0)
        ASDSM_HIP_CHECK(hipMemcpyAsync(p.ws.perm_table, p.hperm, (size_t)opt.max_iter * kMaxD * sizeof(int),
                                       hipMemcpyHostToDevice, p.stream));
    p.gate = nullptr;
    if (!opt.resume) {
        if (int rc = initial_guess(p, s, g, u)) return rc;
    } else {
        {
            PhaseTimer t(p, ASDSM_PHASE_RHS, 1, 0.0, 8.0 * (2.0 * (double)p.geo.NF + 2.0 * p.d * face_points(p)));
            launch_rhs(p, 0, s, g, p.ws.b, true, p.stream);
            if (int rc = check_launch("rhs")) return rc;
        }
        PhaseTimer t(p, ASDSM_PHASE_UPDATE, 1, 2.0 * (2 * p.d + 1) * (double)p.geo.NF,
                     8.0 * (3.0 * (double)p.geo.NF + aniso_points(p)));
        double *gat[kMaxMeshes];
        gather_pointers(p, gat);
        launch_update_residual(p, u, nullptr, nullptr, gat, kFinInit, p.stream);
        if (int rc = check_launch("residual")) return rc;
    }
    if (p.sparse && opt.resume) {
        // The skeleton-sparse loop relies on a zero residual in the holes (Proposition 3.2(2)),
        // which every ASDSM iterate has.  A resumed iterate that may come from elsewhere gets its
        // holes re-filled from its own skeleton first (Algorithm 3 with b_ff); for an ASDSM
        // iterate that changes nothing beyond rounding.
        {
            PhaseTimer t(p, ASDSM_PHASE_UPDATE, 1, 0.0, 8.0 * 4.0 * aniso_points(p));
            launch_skel_gather(p, u, p.stream);
            if (int rc = check_launch("skeleton gather")) return rc;
        }
        {
            PhaseTimer t(p, ASDSM_PHASE_FILLER, 1, filler_flops(p),
                         8.0 * (2.0 * (double)p.geo.NF + aniso_points(p)));
            if (!launch_filler(p, p.ws.b, u, p.stream, p.ws.SU, false))
                return fail(ASDSM_E_ARG, "hole solve: unsupported shape");
            if (int rc = check_launch("resume fill")) return rc;
        }
        PhaseTimer t(p, ASDSM_PHASE_UPDATE, 1, 2.0 * (2 * p.d + 1) * (double)p.geo.NF,
                     8.0 * (3.0 * (double)p.geo.NF + aniso_points(p)));
        double *gat[kMaxMeshes];
        gather_pointers(p, gat);
        launch_update_residual(p, u, nullptr, nullptr, gat, kFinInit, p.stream);
        if (int rc = check_launch("residual")) return rc;
    }
    if (p.sparse) {  // u and r on the skeleton, from the fine vectors
        PhaseTimer t(p, ASDSM_PHASE_UPDATE, 1, 0.0, 8.0 * 4.0 * aniso_points(p));
        launch_skel_gather(p, u, p.stream);
        if (int rc = check_launch("skeleton gather")) return rc;
    }
    p.gate = &p.ws.state->done;
    return ASDSM_OK;
}

// Skeleton-sparse loop: the fine iterate from its skeleton (Algorithm 3 with b_ff, once), then its
// fine residual (so that r and the gathers describe the returned u).  Not gated: it runs whatever
// the stopping rule did.
int finish_sparse(Plan &p, double *u) {
    if (p.upd_fused) {
        // the last step's update, still pending (gated: nothing to do once the loop has stopped)
        PhaseTimer t(p, ASDSM_PHASE_UPDATE, 1, 0.0, 0.0, "k_skel_update");
        double *gat[kMaxMeshes];
        gather_pointers(p, gat);
        launch_skel_update(p, gat, p.stream);
        if (int rc = check_launch("skeleton update")) return rc;
    }
    {
        // the last step's stopping rule (gated: nothing to do once the loop has stopped)
        PhaseTimer t(p, ASDSM_PHASE_UPDATE, 1, 0.0, 0.0, "k_finalize_pending");
        launch_finalize_pending(p, p.stream);
        if (int rc = check_launch("finalize")) return rc;
    }
    p.gate = nullptr;
    {
        PhaseTimer t(p, ASDSM_PHASE_FILLER, 1, filler_flops(p),
                     8.0 * (2.0 * (double)p.geo.NF + aniso_points(p)));
        if (!launch_filler(p, p.ws.b, u, p.stream, p.ws.SU, false))
            return fail(ASDSM_E_ARG, "hole solve: unsupported shape");
        if (int rc = check_launch("final fill")) return rc;
    }
    PhaseTimer t(p, ASDSM_PHASE_UPDATE, 1, 2.0 * (2 * p.d + 1) * (double)p.geo.NF,
                 8.0 * (3.0 * (double)p.geo.NF + aniso_points(p)));
    double *gat[kMaxMeshes];
    gather_pointers(p, gat);
    launch_update_residual(p, u, nullptr, nullptr, gat, kFinRnorm, p.stream);
    return check_launch("final residual");
}

// After the loop (the plan's stream is synchronised here): the final iterate into u, the
// histories, the statistics.  Returns the status.
int end_solve(Plan &p, double *u, const asdsm_opts &opt, asdsm_stats *st) {
    p.gate = nullptr;
    IterState &hs = *p.hstate;
    if (int rc = read_state(p)) return rc;
    if (int rc = read_scalars(p)) return rc;
    const int it = hs.it;
    if (!hs.done) hs.status = ASDSM_MAXITER;
    if (hs.status == ASDSM_E_NUMERIC) return fail(ASDSM_E_NUMERIC, "non-finite right-hand side or residual");
    // the iterate after `it` steps is in u for even it, in the second buffer for odd it (the
    // skeleton-sparse loop has written u itself)
    if (it % 2 == 1 && !p.sparse)
        ASDSM_HIP_CHECK(hipMemcpyAsync(u, p.ws.u2, (size_t)p.geo.NF * sizeof(double), hipMemcpyDeviceToDevice, p.stream));
    double r0 = 0.0, rn = 0.0;
    ASDSM_HIP_CHECK(hipMemcpyAsync(&r0, p.ws.hist, sizeof(double), hipMemcpyDeviceToHost, p.stream));
    ASDSM_HIP_CHECK(hipMemcpyAsync(&rn, p.ws.hist + it, sizeof(double), hipMemcpyDeviceToHost, p.stream));
    if (opt.hist)
        ASDSM_HIP_CHECK(hipMemcpyAsync(opt.hist, p.ws.hist, (size_t)(it + 1) * sizeof(double), hipMemcpyDeviceToHost, p.stream));
    if (opt.step_hist && it > 0)
        ASDSM_HIP_CHECK(hipMemcpyAsync(opt.step_hist, p.ws.step_hist, (size_t)it * sizeof(double), hipMemcpyDeviceToHost, p.stream));
    ASDSM_HIP_CHECK(hipStreamSynchronize(p.stream));
    if (p.profiling)
        if (int rc = collect_phases(p)) return rc;
    if (st) {
        std::memset(st, 0, sizeof *st);
        st->status = hs.status;
        st->iterations = it;
        st->bnorm = std::sqrt(p.hscal[kScalBnorm2]);
        st->r0norm = r0;
        // the skeleton-sparse loop recomputes the residual of the rebuilt fine iterate at the end
        st->rnorm = p.sparse ? std::sqrt(p.hscal[kScalRnorm2]) : rn;
        st->precision = p.prec32 ? ASDSM_PREC_FP32 : ASDSM_PREC_FP64;
        for (int q = 0; q < ASDSM_NPHASE; ++q) {
            st->phase_ms[q] = p.phase_ms[q];
            st->phase_launches[q] = p.phase_launches[q];
            st->phase_flops[q] = p.phase_flops[q];
            st->phase_bytes[q] = p.phase_bytes[q];
        }
    }
    return hs.status;
}

int solve_impl(Plan &p, const double *s, const double *g, double *u, const asdsm_opts *o,
               asdsm_stats *st) {
    asdsm_opts opt;
    if (int rc = normalize_opts(o, opt)) return rc;
    if (int rc = check_sparse(p, opt)) return rc;
    if (opt.skeleton && p.learn_net)
        return fail(ASDSM_E_ARG, "learned proposals need the fine residual: no skeleton-sparse refinement");
    p.profiling = opt.profile != 0;
    p.prof_failed = false;
    p.ev_recs.clear();
    struct ProfilingOff {
        Plan &p;
        ~ProfilingOff() { p.profiling = false; }
    } off{p};
    const bool use_graph = !p.profiling && !opt.eager;
    CallEvents ev;
    if (p.profiling) {
        ASDSM_HIP_CHECK(hipEventCreate(&ev.tb));
        ASDSM_HIP_CHECK(hipEventCreate(&ev.te));
        ASDSM_HIP_CHECK(hipEventRecord(ev.tb, p.stream));
    }
    if (int rc = begin_solve(p, s, g, u, opt)) return rc;
    IterState &hs = *p.hstate;
    int rc = ASDSM_OK;
    if (use_graph) {
        const uint64_t net_serial = p.learn_net ? p.learn_net->serial : 0;
        const void *net_ws = p.learn_net ? p.learn_net->ws : nullptr;
        if (p.graph_u != u || !p.graph_exec || p.graph_gen != p.generation || p.graph_prec32 != p.prec32 ||
            p.graph_sparse != p.sparse ||
            p.graph_net_serial != net_serial ||
            p.graph_net_ws != net_ws || (p.learn_net && p.graph_factor != p.learn_factor))
            rc = build_graph(p, u);
        // two steps per replay, two replays per batch; the host checks the loop state of batch i
        // while batch i + 1 runs (the state is copied into one of two pinned slots behind each
        // batch), so the device never waits for the host; steps beyond the stopping point are gated
        // no-ops
        if (rc == ASDSM_OK) rc = ensure_loop_events(p);
        int steps = 0, inflight = 0;
        auto launch_batch = [&](int slot) -> int {
            for (int rep = 0; rep < 2 && steps < opt.max_iter; ++rep, steps += 2) {
                hipError_t e = hipGraphLaunch(p.graph_exec, p.stream);
                if (e != hipSuccess)
                    return fail(ASDSM_E_DEVICE, std::string("hipGraphLaunch: ") + hipGetErrorString(e));
            }
            ASDSM_HIP_CHECK(hipMemcpyAsync(p.hstate_ring[slot], p.ws.state, sizeof(IterState),
                                           hipMemcpyDeviceToHost, p.stream));
            ASDSM_HIP_CHECK(hipEventRecord(p.loop_ev[slot], p.stream));
            ++inflight;
            return ASDSM_OK;
        };
        if (rc == ASDSM_OK) rc = launch_batch(0);
        if (rc == ASDSM_OK && steps < opt.max_iter) rc = launch_batch(1);
        for (int slot = 0; rc == ASDSM_OK && inflight > 0; slot ^= 1) {
            hipError_t e = hipEventSynchronize(p.loop_ev[slot]);
            if (e != hipSuccess) {
                rc = fail(ASDSM_E_DEVICE, std::string("hipEventSynchronize: ") + hipGetErrorString(e));
                break;
            }
            --inflight;
            if (p.hstate_ring[slot]->done) break;
            if (steps < opt.max_iter) rc = launch_batch(slot);
        }
        if (rc == ASDSM_OK) rc = read_state(p);
    } else {
        for (int i = 0; i < opt.max_iter && rc == ASDSM_OK; ++i) {
            rc = (i % 2 == 0) ? step(p, u, p.ws.u2) : step(p, p.ws.u2, u);
            if (rc == ASDSM_OK) rc = read_state(p);
            if (hs.done) break;
        }
    }
    if (rc == ASDSM_OK && p.sparse) rc = finish_sparse(p, u);
    if (rc != ASDSM_OK) {
        p.gate = nullptr;
        return rc;
    }
    const int status = end_solve(p, u, opt, st);
    if (status < 0) return status;
    if (st && p.profiling) {
        ASDSM_HIP_CHECK(hipEventRecord(ev.te, p.stream));
        ASDSM_HIP_CHECK(hipEventSynchronize(ev.te));
        float ms = 0.f;
        ASDSM_HIP_CHECK(hipEventElapsedTime(&ms, ev.tb, ev.te));
        st->total_ms = ms;
    }
    set_error("");
    return status;
}

// ---------------------------------------------------------------------------------------------
// Batches: independent problems (any sizes) whose refinement loops run as one graph.  Each
// replay of the graph performs two gated refinement steps of every member, as parallel branches
// (one capture stream per member); a member whose stopping rule has fired turns into no-ops while
// the others continue.  The host checks every member's state after every two replays.
// ---------------------------------------------------------------------------------------------
struct Batch {
    std::vector<Plan *> plans;
    hipStream_t root = nullptr;              // launch stream of the graph
    hipStream_t cap = nullptr;               // capture root
    std::vector<hipStream_t> branch;         // capture stream of each member
    std::vector<hipEvent_t> ready, joined;   // member -> root dependencies
    hipEvent_t fork = nullptr, done = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<double *> graph_u;
    std::vector<bool> graph_prec32;
    std::vector<bool> graph_sparse;
    std::vector<uint64_t> graph_gen;         // each member's plan generation at capture
    std::vector<int> graph_members;          // members whose steps the graph holds
    hipEvent_t slot_ev[2] = {nullptr, nullptr};  // the pipelined state checks
};

void destroy_batch_graph(Batch &b) {
    if (b.exec) (void)hipGraphExecDestroy(b.exec);
    if (b.graph) (void)hipGraphDestroy(b.graph);
    b.exec = nullptr;
    b.graph = nullptr;
    b.graph_u.clear();
    b.graph_prec32.clear();
    b.graph_sparse.clear();
    b.graph_gen.clear();
    b.graph_members.clear();
}

void release_batch(Batch &b) {
    destroy_batch_graph(b);
    for (hipStream_t s : b.branch) if (s) (void)hipStreamDestroy(s);
    for (hipEvent_t e : b.ready) if (e) (void)hipEventDestroy(e);
    for (hipEvent_t e : b.joined) if (e) (void)hipEventDestroy(e);
    if (b.fork) (void)hipEventDestroy(b.fork);
    if (b.done) (void)hipEventDestroy(b.done);
    for (int i = 0; i < 2; ++i) {
        if (b.slot_ev[i]) (void)hipEventDestroy(b.slot_ev[i]);
        b.slot_ev[i] = nullptr;
    }
    if (b.cap) (void)hipStreamDestroy(b.cap);
    if (b.root) (void)hipStreamDestroy(b.root);
    b.branch.clear();
    b.ready.clear();
    b.joined.clear();
    b.fork = b.done = nullptr;
    b.cap = b.root = nullptr;
}

int build_batch(Batch &b, int n) {
    ASDSM_HIP_CHECK(hipStreamCreateWithFlags(&b.root, hipStreamNonBlocking));
    ASDSM_HIP_CHECK(hipStreamCreateWithFlags(&b.cap, hipStreamNonBlocking));
    ASDSM_HIP_CHECK(hipEventCreateWithFlags(&b.fork, hipEventDisableTiming));
    ASDSM_HIP_CHECK(hipEventCreateWithFlags(&b.done, hipEventDisableTiming));
    for (int i = 0; i < 2; ++i) ASDSM_HIP_CHECK(hipEventCreateWithFlags(&b.slot_ev[i], hipEventDisableTiming));
    b.branch.assign(n, nullptr);
    b.ready.assign(n, nullptr);
    b.joined.assign(n, nullptr);
    for (int i = 0; i < n; ++i) {
        ASDSM_HIP_CHECK(hipStreamCreateWithFlags(&b.branch[i], hipStreamNonBlocking));
        ASDSM_HIP_CHECK(hipEventCreateWithFlags(&b.ready[i], hipEventDisableTiming));
        ASDSM_HIP_CHECK(hipEventCreateWithFlags(&b.joined[i], hipEventDisableTiming));
    }
    return ASDSM_OK;
}

// Capture two refinement steps of every member (u -> u2 -> u) as parallel branches.
// Capture two gated refinement steps of each member in `members` as parallel branches of one graph
// (fork/join events; each branch runs on its own capture stream).  Members that have stopped are
// left out: their steps would be gated no-ops that still cost a launch each.
int capture_batch_graph(Batch &b, double *const *u, const std::vector<int> &members) {
    destroy_batch_graph(b);
    const int n = (int)b.plans.size();
    ASDSM_HIP_CHECK(hipStreamBeginCapture(b.cap, hipStreamCaptureModeThreadLocal));
    int rc = ASDSM_OK;
    hipError_t e = hipEventRecord(b.fork, b.cap);
    if (e != hipSuccess) rc = fail(ASDSM_E_DEVICE, std::string("hipEventRecord: ") + hipGetErrorString(e));
    for (int i : members) {
        if (rc != ASDSM_OK) break;
        Plan &p = *b.plans[i];
        e = hipStreamWaitEvent(b.branch[i], b.fork, 0);
        if (e != hipSuccess) {
            rc = fail(ASDSM_E_DEVICE, std::string("hipStreamWaitEvent: ") + hipGetErrorString(e));
            break;
        }
        hipStream_t saved = p.stream;
        p.stream = b.branch[i];
        // plain steps (a correction network bound to a member plays no part in batches)
        rc = p.sparse ? sparse_step(p) : refine_step(p, u[i], p.ws.u2);
        if (rc == ASDSM_OK) rc = p.sparse ? sparse_step(p) : refine_step(p, p.ws.u2, u[i]);
        p.stream = saved;
        if (rc != ASDSM_OK) break;
        e = hipEventRecord(b.joined[i], b.branch[i]);
        if (e == hipSuccess) e = hipStreamWaitEvent(b.cap, b.joined[i], 0);
        if (e != hipSuccess) rc = fail(ASDSM_E_DEVICE, std::string("batch join: ") + hipGetErrorString(e));
    }
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(b.cap, &graph);
    if (rc != ASDSM_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return rc;
    }
    if (e != hipSuccess) return fail(ASDSM_E_DEVICE, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
    b.graph = graph;
    e = hipGraphInstantiate(&b.exec, graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        destroy_batch_graph(b);
        return fail(ASDSM_E_DEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
    }
    b.graph_u.assign(u, u + n);
    for (int i = 0; i < n; ++i) {
        b.graph_prec32.push_back(b.plans[i]->prec32);
        b.graph_sparse.push_back(b.plans[i]->sparse);
        b.graph_gen.push_back(b.plans[i]->generation);
    }
    b.graph_members = members;
    return ASDSM_OK;
}

int batch_solve_impl(Batch &b, const double *const *s, const double *const *g, double *const *u,
                     const asdsm_opts *o, asdsm_stats *st) {
    asdsm_opts opt;
    if (int rc = normalize_opts(o, opt)) return rc;
    const int n = (int)b.plans.size();
    if (!s || !g || !u) return fail(ASDSM_E_ARG, "s, g and u must be non-NULL arrays of n pointers");
    if (opt.profile || opt.eager) {
        // one member after the other, each on its own loop
        int worst = ASDSM_OK;
        for (int i = 0; i < n; ++i) {
            asdsm_opts oi = opt;
            oi.skeleton = (opt.skeleton && b.plans[i]->d == 3) ? 1 : 0;
            const int rc = solve_impl(*b.plans[i], s[i], g[i], u[i], &oi, st ? st + i : nullptr);
            if (rc < 0) return rc;
            worst = std::max(worst, rc);
        }
        return worst;
    }
    for (int i = 0; i < n; ++i) {
        Plan &p = *b.plans[i];
        p.profiling = false;
        // skeleton-sparse refinement where it is built (d = 3), the fine-mesh loop elsewhere
        asdsm_opts oi = opt;
        oi.skeleton = (opt.skeleton && p.d == 3) ? 1 : 0;
        if (int rc = begin_solve(p, s[i], g[i], u[i], oi)) return rc;
        ASDSM_HIP_CHECK(hipEventRecord(b.ready[i], p.stream));
        ASDSM_HIP_CHECK(hipStreamWaitEvent(b.root, b.ready[i], 0));
    }
    std::vector<int> active;
    for (int i = 0; i < n; ++i) active.push_back(i);
    auto stale = [&]() {
        if (!b.exec || (int)b.graph_u.size() != n || b.graph_members != active) return true;
        for (int i = 0; i < n; ++i)
            if (b.graph_u[i] != u[i] || b.graph_prec32[i] != b.plans[i]->prec32 ||
                b.graph_sparse[i] != b.plans[i]->sparse || b.graph_gen[i] != b.plans[i]->generation)
                return true;
        return false;
    };
    int rc = stale() ? capture_batch_graph(b, u, active) : ASDSM_OK;
    // two replays per batch of work; the host reads every active member's loop state behind batch i
    // (one of two pinned slots per member) while batch i + 1 runs; when members have stopped, the
    // graph is captured again without them
    int steps = 0, inflight = 0;
    auto launch_batch = [&](int slot) -> int {
        for (int rep = 0; rep < 2 && steps < opt.max_iter; ++rep, steps += 2) {
            hipError_t e = hipGraphLaunch(b.exec, b.root);
            if (e != hipSuccess) return fail(ASDSM_E_DEVICE, std::string("hipGraphLaunch: ") + hipGetErrorString(e));
        }
        for (int i : b.graph_members) {
            Plan &p = *b.plans[i];
            ASDSM_HIP_CHECK(hipMemcpyAsync(p.hstate_ring[slot], p.ws.state, sizeof(IterState),
                                           hipMemcpyDeviceToHost, b.root));
        }
        ASDSM_HIP_CHECK(hipEventRecord(b.slot_ev[slot], b.root));
        ++inflight;
        return ASDSM_OK;
    };
    std::vector<int> slot_members[2];
    if (rc == ASDSM_OK) {
        slot_members[0] = b.graph_members;
        rc = launch_batch(0);
    }
    if (rc == ASDSM_OK && steps < opt.max_iter) {
        slot_members[1] = b.graph_members;
        rc = launch_batch(1);
    }
    for (int slot = 0; rc == ASDSM_OK && inflight > 0; slot ^= 1) {
        hipError_t e = hipEventSynchronize(b.slot_ev[slot]);
        if (e != hipSuccess) {
            rc = fail(ASDSM_E_DEVICE, std::string("hipEventSynchronize: ") + hipGetErrorString(e));
            break;
        }
        --inflight;
        std::vector<int> still;
        for (int i : slot_members[slot])
            if (!b.plans[i]->hstate_ring[slot]->done) still.push_back(i);
        if (still.empty()) break;
        if (steps >= opt.max_iter) continue;
        if (still.size() < active.size()) {
            // members stopped: wait for the batch in flight, then leave them out of the graph
            e = hipStreamSynchronize(b.root);
            if (e != hipSuccess) {
                rc = fail(ASDSM_E_DEVICE, std::string("hipStreamSynchronize: ") + hipGetErrorString(e));
                break;
            }
            inflight = 0;
            std::vector<int> alive;
            for (int i : still) {
                Plan &p = *b.plans[i];
                if ((rc = read_state_on(p, b.root))) break;
                if (!p.hstate->done) alive.push_back(i);
            }
            if (rc != ASDSM_OK || alive.empty()) break;
            active = alive;
            rc = capture_batch_graph(b, u, active);
            if (rc != ASDSM_OK) break;
        }
        slot_members[slot] = b.graph_members;
        rc = launch_batch(slot);
    }
    if (rc == ASDSM_OK) {
        hipError_t e = hipStreamSynchronize(b.root);
        if (e != hipSuccess) rc = fail(ASDSM_E_DEVICE, std::string("hipStreamSynchronize: ") + hipGetErrorString(e));
    }
    // the members' streams continue after the graph's work (the skeleton-sparse members then
    // rebuild their fine iterate on their own streams)
    ASDSM_HIP_CHECK(hipEventRecord(b.done, b.root));
    for (int i = 0; i < n; ++i) ASDSM_HIP_CHECK(hipStreamWaitEvent(b.plans[i]->stream, b.done, 0));
    for (int i = 0; i < n && rc == ASDSM_OK; ++i)
        if (b.plans[i]->sparse) rc = finish_sparse(*b.plans[i], u[i]);
    if (rc != ASDSM_OK) {
        for (int i = 0; i < n; ++i) b.plans[i]->gate = nullptr;
        return rc;
    }
    int worst = ASDSM_OK;
    for (int i = 0; i < n; ++i) {
        const int r = end_solve(*b.plans[i], u[i], opt, st ? st + i : nullptr);
        if (r < 0) return r;
        worst = std::max(worst, r);
    }
    set_error("");
    return worst;
}

}  // namespace
}  // namespace asdsm

using namespace asdsm;

extern "C" {

int asdsm_plan(asdsm_plan_t *out, int d, const double *alpha, const double *beta, int level,
               int coarse_level, uint64_t seed, void *hip_stream) {
    if (!out) return fail(ASDSM_E_ARG, "out must be non-NULL");
    *out = nullptr;
    asdsm_plan_s *h = new (std::nothrow) asdsm_plan_s();
    if (!h) return fail(ASDSM_E_ARG, "out of host memory");
    int rc = build_plan(h->p, d, alpha, beta, level, coarse_level, seed, (hipStream_t)hip_stream);
    static std::atomic<uint64_t> serials{0};
    h->p.serial = ++serials;
    if (rc != ASDSM_OK) {
        release_plan(h->p);
        delete h;
        return rc;
    }
    *out = h;
    set_error("");
    return ASDSM_OK;
}

int asdsm_workspace_size(asdsm_plan_t plan, size_t *bytes) {
    if (!plan || !bytes) return fail(ASDSM_E_ARG, "plan and bytes must be non-NULL");
    *bytes = plan->p.ws_need;
    return ASDSM_OK;
}

int asdsm_set_workspace(asdsm_plan_t plan, void *dev, size_t bytes) {
    if (!plan) return fail(ASDSM_E_ARG, "plan must be non-NULL");
    Plan &p = plan->p;
    if (!dev) return fail(ASDSM_E_WORKSPACE, "workspace pointer is NULL");
    if (((uintptr_t)dev & 255u) != 0) return fail(ASDSM_E_WORKSPACE, "workspace must be 256-byte aligned");
    if (bytes < p.ws_need)
        return fail(ASDSM_E_WORKSPACE, "workspace too small: need " + std::to_string(p.ws_need) + " bytes");
    plan_changed(p);  // a captured graph points into the previous workspace
    p.ws_base = dev;
    p.ws_bytes = bytes;
    layout_workspace(p, (char *)dev, true);
    // restore the a-priori sweep counts (the layout holds their buffers), then calibrate
    for (unsigned m = 0; m < kMaxMeshes; ++m) p.sweeps[m] = p.sweeps_prior[m];
    return calibrate_sweeps(p);
}

int asdsm_solve(asdsm_plan_t plan, const double *s, const double *g, double *u,
                const asdsm_opts *opts, asdsm_stats *stats) {
    if (!plan) return fail(ASDSM_E_ARG, "plan must be non-NULL");
    return solve_impl(plan->p, s, g, u, opts, stats);
}

int asdsm_solve_learned(asdsm_plan_t plan, asdsm_net_t net, double factor, const double *s, const double *g,
                        double *u, const asdsm_opts *opts, asdsm_stats *stats, int *accepted) {
    if (accepted) *accepted = 0;
    if (!plan || !net) return fail(ASDSM_E_ARG, "plan and net must be non-NULL");
    Plan &p = plan->p;
    Net &nt = net->net;
    if (nt.plan != plan || nt.plan_serial != p.serial)
        return fail(ASDSM_E_ARG, "the network is not bound to this plan");
    if (nt.n != p.geo.Nf) return fail(ASDSM_E_ARG, "the network's volume differs from the fine mesh");
    if (!nt.ws) return fail(ASDSM_E_WORKSPACE, "no workspace attached to the network");
    if (!(factor > 1.0) || !std::isfinite(factor)) return fail(ASDSM_E_ARG, "factor must be finite and > 1");
    p.learn_net = &nt;
    p.learn_factor = factor;
    struct Reset {
        Plan &p;
        ~Reset() { p.learn_net = nullptr; }
    } reset{p};
    const int rc = solve_impl(p, s, g, u, opts, stats);
    if (accepted && rc >= 0) *accepted = p.hstate->learned;
    return rc;
}

int asdsm_residual(asdsm_plan_t plan, const double *u, const double *s, const double *g, double *r,
                   double *norm2) {
    if (!plan) return fail(ASDSM_E_ARG, "plan must be non-NULL");
    Plan &p = plan->p;
    if (!u || !s || !g) return fail(ASDSM_E_ARG, "u, s and g must be non-NULL device pointers");
    if (int rc = require_ws(p)) return rc;
    launch_rhs(p, 0, s, g, p.ws.b, true, p.stream);
    double *gat[kMaxMeshes];
    gather_pointers(p, gat);
    p.gate = nullptr;
    launch_update_residual(p, u, nullptr, nullptr, gat, kFinRnorm, p.stream);
    if (int rc = check_launch("residual")) return rc;
    if (r) ASDSM_HIP_CHECK(hipMemcpyAsync(r, p.ws.r, (size_t)p.geo.NF * sizeof(double), hipMemcpyDeviceToDevice, p.stream));
    if (int rc = read_scalars(p)) return rc;
    if (norm2) *norm2 = std::sqrt(p.hscal[kScalRnorm2]);
    set_error("");
    return ASDSM_OK;
}

int asdsm_residual_noalloc(asdsm_plan_t plan, const double *u, const double *s, const double *g,
                           double *r, double *norm2) {
    if (!plan) return fail(ASDSM_E_ARG, "plan must be non-NULL");
    if (!u || !s || !g) return fail(ASDSM_E_ARG, "u, s and g must be non-NULL device pointers");
    if (int rc = residual_noalloc(plan->p, u, s, g, r, norm2)) return rc;
    set_error("");
    return ASDSM_OK;
}

int asdsm_mesh_solve(asdsm_plan_t plan, unsigned mesh_mask, const double *rhs, double *x) {
    if (!plan) return fail(ASDSM_E_ARG, "plan must be non-NULL");
    Plan &p = plan->p;
    if (!rhs || !x) return fail(ASDSM_E_ARG, "rhs and x must be non-NULL device pointers");
    if (mesh_mask == 0 || mesh_mask >= (1u << p.d)) return fail(ASDSM_E_ARG, "invalid mesh mask");
    if (int rc = require_ws(p)) return rc;
    const size_t bytes = (size_t)p.mesh[mesh_mask].size * sizeof(double);
    ASDSM_HIP_CHECK(hipMemcpyAsync(rhs_buf(p, mesh_mask), rhs, bytes, hipMemcpyDeviceToDevice, p.stream));
    if (__builtin_popcount(mesh_mask) == 1) {
        if (int rc = solve_aniso_refined(p, mesh_mask)) return rc;
    } else {
        if (int rc = solve_intersection_refined(p, mesh_mask)) return rc;
    }
    const double *res = sol_buf(p, mesh_mask);
    ASDSM_HIP_CHECK(hipMemcpyAsync(x, res, bytes, hipMemcpyDeviceToDevice, p.stream));
    ASDSM_HIP_CHECK(hipStreamSynchronize(p.stream));
    set_error("");
    return ASDSM_OK;
}

struct asdsm_batch_s {
    Batch b;
};

int asdsm_batch_create(asdsm_batch_t *out, const asdsm_plan_t *plans, int n) {
    if (!out) return fail(ASDSM_E_ARG, "out must be non-NULL");
    *out = nullptr;
    if (!plans || n < 1 || n > 4096) return fail(ASDSM_E_ARG, "plans must hold 1..4096 plans");
    for (int i = 0; i < n; ++i) {
        if (!plans[i]) return fail(ASDSM_E_ARG, "NULL plan in batch");
        for (int j = 0; j < i; ++j)
            if (plans[j] == plans[i]) return fail(ASDSM_E_ARG, "a plan appears twice in the batch");
        if (plans[i]->p.device != plans[0]->p.device) return fail(ASDSM_E_ARG, "batch plans on different devices");
    }
    asdsm_batch_s *h = new (std::nothrow) asdsm_batch_s();
    if (!h) return fail(ASDSM_E_ARG, "out of host memory");
    for (int i = 0; i < n; ++i) h->b.plans.push_back(&plans[i]->p);
    if (int rc = build_batch(h->b, n)) {
        release_batch(h->b);
        delete h;
        return rc;
    }
    *out = h;
    set_error("");
    return ASDSM_OK;
}

int asdsm_batch_solve(asdsm_batch_t batch, const double *const *s, const double *const *g,
                      double *const *u, const asdsm_opts *opts, asdsm_stats *stats) {
    if (!batch) return fail(ASDSM_E_ARG, "batch must be non-NULL");
    return batch_solve_impl(batch->b, s, g, u, opts, stats);
}

int asdsm_autotune(asdsm_plan_t plan, int repeats, int *tile, double *ms_per_solve) {
    if (!plan) return fail(ASDSM_E_ARG, "plan must be non-NULL");
    const int rc = autotune_impl(plan->p, repeats, tile, ms_per_solve);
    if (rc == ASDSM_OK) set_error("");
    return rc;
}

const char *asdsm_tile_name(int tile) { return gemm_tile_name(tile); }

int asdsm_line_axes(asdsm_plan_t plan, int *axis, int *sweeps) {
    if (!plan || !axis) return fail(ASDSM_E_ARG, "plan and axis must be non-NULL");
    const Plan &p = plan->p;
    for (unsigned s = 0; s < (1u << p.d); ++s) {
        axis[s] = (s > 0 && p.line_pos[s] >= 0) ? p.mesh[s].ax[p.line_pos[s]] : -1;
        if (sweeps) sweeps[s] = p.sweeps[s];
    }
    set_error("");
    return ASDSM_OK;
}

int asdsm_profile_count(asdsm_plan_t plan) {
    if (!plan) return fail(ASDSM_E_ARG, "plan must be non-NULL");
    return (int)plan->p.kern_recs.size();
}

int asdsm_profile_entry(asdsm_plan_t plan, int i, char *name, int name_cap, int *phase, double *ms,
                        int *groups, int *launches, double *flops, double *bytes) {
    if (!plan) return fail(ASDSM_E_ARG, "plan must be non-NULL");
    const auto &recs = plan->p.kern_recs;
    if (i < 0 || i >= (int)recs.size()) return fail(ASDSM_E_ARG, "profile entry index out of range");
    const auto &r = recs[(size_t)i];
    if (name && name_cap > 0) {
        const size_t n = std::min((size_t)(name_cap - 1), r.name.size());
        std::memcpy(name, r.name.data(), n);
        name[n] = '\0';
    }
    if (phase) *phase = r.phase;
    if (ms) *ms = r.ms;
    if (groups) *groups = r.groups;
    if (launches) *launches = r.launches;
    if (flops) *flops = r.flops;
    if (bytes) *bytes = r.bytes;
    set_error("");
    return ASDSM_OK;
}

size_t asdsm_probe_mfma_scratch_bytes(void) { return probe_mfma_scratch_bytes(); }

int asdsm_probe_mfma_f64(void *scratch, int iters, void *hip_stream, double *tflops) {
    if (!scratch || !tflops || iters < 1) return fail(ASDSM_E_ARG, "probe: NULL pointer or iters < 1");
    if (int rc = probe_mfma_f64((double *)scratch, iters, (hipStream_t)hip_stream, tflops))
        return fail(rc, "probe: HIP call failed");
    set_error("");
    return ASDSM_OK;
}

int asdsm_probe_copy(const void *src, void *dst, size_t bytes, int reps, void *hip_stream, double *tbps) {
    if (!src || !dst || !tbps || reps < 1 || bytes < 16) return fail(ASDSM_E_ARG, "probe: bad arguments");
    if ((((uintptr_t)src) | ((uintptr_t)dst)) & 15u) return fail(ASDSM_E_ARG, "probe: buffers must be 16-byte aligned");
    if (int rc = probe_copy((const double *)src, (double *)dst, bytes, reps, (hipStream_t)hip_stream, tbps))
        return fail(rc, "probe: HIP call failed");
    set_error("");
    return ASDSM_OK;
}

static_assert(ASDSM_TILE_AUTO == kTileAuto && ASDSM_TILE_32X32 == kTile32x32 && ASDSM_TILE_64X32 == kTile64x32 &&
                  ASDSM_TILE_32X64 == kTile32x64 && ASDSM_TILE_64X64 == kTile64x64 && ASDSM_TILE_PLANE == kTilePlane,
              "tile codes of the C ABI");

int asdsm_get_tile(asdsm_plan_t plan, int *tile) {
    if (!plan || !tile) return fail(ASDSM_E_ARG, "plan and tile must be non-NULL");
    *tile = plane_transforms(plan->p) ? kTilePlane : plan->p.tile_aniso;
    set_error("");
    return ASDSM_OK;
}

int asdsm_set_tile(asdsm_plan_t plan, int tile) {
    if (!plan) return fail(ASDSM_E_ARG, "plan must be non-NULL");
    Plan &p = plan->p;
    if (tile < kTileAuto || tile > kTilePlane) return fail(ASDSM_E_ARG, "unknown tile shape");
    if (tile == kTilePlane && (p.d != 3 || p.Nf > kPlaneMaxNf || p.line_aniso))
        return fail(ASDSM_E_UNSUPPORTED, "plane transforms need d = 3, N_f <= 255 and no line axes");
    if (tile != p.tile_aniso) {
        p.tile_aniso = tile;
        plan_changed(p);  // captured launches carry the old tile choice
    }
    set_error("");
    return ASDSM_OK;
}

void asdsm_batch_destroy(asdsm_batch_t batch) {
    if (!batch) return;
    release_batch(batch->b);
    delete batch;
}

void asdsm_destroy(asdsm_plan_t plan) {
    if (!plan) return;
    release_plan(plan->p);
    delete plan;
}

const char *asdsm_last_error(void) { return last_error_cstr(); }

}  // extern "C"
