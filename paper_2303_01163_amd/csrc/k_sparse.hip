// Skeleton-sparse refinement (d = 3).  After the filler (Algorithm 3) every hole equation holds, so
// the fine residual r = b - A u vanishes off the coarse planes (Proposition 3.2(2)), and so does
// q = A e for the homogeneous error guess e.  A refinement step therefore needs r, q and u only on
// the skeleton (the points of the anisotropic meshes M_k) and e only on the skeleton and on the
// hole layers next to it (the stencil's neighbours across a coarse plane); the holes of u are
// filled once, when the loop ends (Section 3.3, first and last remarks: compute only the non-zero
// residual entries, keep only the skeleton and the elements next to it).  The skeleton lives in the
// anisotropic meshes' canonical layouts -- point (a, b) of plane c of M_k at a + N_f b + N_f^2 c,
// a and b the fine coordinates of the two other axes in
// increasing order -- and the layers next to plane c on side s (s = 0: one below, s = 1: one above
// along axis k) at the same offset plus s N_c N_f^2.  A point on several planes is stored in each
// of their meshes with identical values; sums count it once, in the mesh of its lowest coarse axis.
#include <algorithm>

#include "device_common.hpp"
#include "kernels.hpp"
#include "skel_common.hpp"

namespace asdsm {

struct SkelPtrs {
    double *p[kMaxD];
};

// U_k = u and R_k = r on every skeleton point (from the fine vectors after the initial guess).
__global__ __launch_bounds__(256) void k_skel_gather(Geo g, const double *__restrict__ u, const double *__restrict__ r,
                                                     SkelPtrs U, SkelPtrs R, const int *gate) {
    if (gate && *gate) return;
    const int per = g.Nc * g.Nf * g.Nf;
    const int k = blockIdx.y;
    double *__restrict__ Uk = (k == 0) ? U.p[0] : (k == 1) ? U.p[1] : U.p[2];
    double *__restrict__ Rk = (k == 0) ? R.p[0] : (k == 1) ? R.p[1] : R.p[2];
    const long long sy = g.Nf, sz = (long long)g.Nf * g.Nf;
    for (int idx = blockIdx.x * 256 + threadIdx.x; idx < per; idx += gridDim.x * 256) {
        int x0, x1, x2;
        bool own;
        if (k == 0) skel_point<0>(g, idx, x0, x1, x2, own);
        else if (k == 1) skel_point<1>(g, idx, x0, x1, x2, own);
        else skel_point<2>(g, idx, x0, x1, x2, own);
        const long long f = x0 + sy * x1 + sz * x2;
        Uk[idx] = u[f];
        Rk[idx] = r[f];
    }
}

// q = A e on the skeleton points of M_K, from E_K (the merged skeleton values of the error guess)
// and EA_K (the hole layers on both sides of each plane), summed over the axes in the fixed order
// of the fine-mesh pass (centre, axis 0 -, +, axis 1 -, +, axis 2 -, +) so that the copies of a
// point in several meshes agree bit for bit; partial sums of <r, q> and <q, q> over owned points.
template <int K>
__device__ __forceinline__ void skel_dots_mesh(const Geo &g, const double *__restrict__ E, const double *__restrict__ EA,
                                               const double *__restrict__ R, double *__restrict__ Q, double &rq,
                                               double &qq, int tile, int ntile, int gv) {
    constexpr int PPT = 4;  // points per thread whose loads are in flight together
    const int Nf = g.Nf;
    const int per = g.Nc * Nf * Nf;
    const int stride = ntile * 256;
    const double bsum = g.fine[0].b + g.fine[1].b + g.fine[2].b;
    for (int base = tile * 256 + threadIdx.x; base < per; base += PPT * stride) {
        // every operand of the thread's points first (branch-free: a neighbour outside the plane
        // reads the point itself and is dropped below), then the sums in point order
        double ec[PPT], am[PPT], ap[PPT], bm[PPT], bp[PPT], cm[PPT], cp[PPT], rr[PPT];
        unsigned inside[PPT];
#pragma unroll
        for (int t = 0; t < PPT; ++t) {
            const int idx = base + t * stride;
            const int i = idx < per ? idx : 0;
            const unsigned row = (unsigned)i / (unsigned)Nf;
            const int a = i - (int)row * Nf, b = (int)(row % (unsigned)Nf);
            inside[t] = (a > 0 ? 1u : 0u) | (a < Nf - 1 ? 2u : 0u) | (b > 0 ? 4u : 0u) | (b < Nf - 1 ? 8u : 0u);
            ec[t] = E[i];
            am[t] = E[a > 0 ? i - 1 : i];
            ap[t] = E[a < Nf - 1 ? i + 1 : i];
            bm[t] = E[b > 0 ? i - Nf : i];
            bp[t] = E[b < Nf - 1 ? i + Nf : i];
            cm[t] = EA[i];
            cp[t] = EA[i + per];
            rr[t] = R[i];
        }
#pragma unroll
        for (int t = 0; t < PPT; ++t) {
            const int idx = base + t * stride;
            if (idx >= per) break;
            int x0, x1, x2;
            bool own;
            skel_point<K>(g, idx, x0, x1, x2, own);
            // neighbours within the plane (fine axes a, b) and across it (layers)
            const double vam = (inside[t] & 1u) ? am[t] : 0.0, vap = (inside[t] & 2u) ? ap[t] : 0.0;
            const double vbm = (inside[t] & 4u) ? bm[t] : 0.0, vbp = (inside[t] & 8u) ? bp[t] : 0.0;
            double q = bsum * ec[t];
            if (K == 0) {
                q += g.fine[0].a * cm[t]; q += g.fine[0].c * cp[t];
                q += g.fine[1].a * vam; q += g.fine[1].c * vap;
                q += g.fine[2].a * vbm; q += g.fine[2].c * vbp;
            } else if (K == 1) {
                q += g.fine[0].a * vam; q += g.fine[0].c * vap;
                q += g.fine[1].a * cm[t]; q += g.fine[1].c * cp[t];
                q += g.fine[2].a * vbm; q += g.fine[2].c * vbp;
            } else {
                q += g.fine[0].a * vam; q += g.fine[0].c * vap;
                q += g.fine[1].a * vbm; q += g.fine[1].c * vbp;
                q += g.fine[2].a * cm[t]; q += g.fine[2].c * cp[t];
            }
            if (flag_clear(gv)) Q[idx] = q;  // the stopping flag, tested after the first loads
            if (own) {
                rq += rr[t] * q;
                qq += q * q;
            }
        }
    }
}

// Grid (tiles, 3): blockIdx.y selects the mesh.  Partial sums per block at blockIdx.x + tiles * y;
// mark (non-null): the update and stopping rule of this step are left pending.
__global__ __launch_bounds__(256) void k_skel_dots(Geo g, SkelPtrs E, SkelPtrs EA, SkelPtrs R, SkelPtrs Q,
                                                   double *partials, IterState *mark, const int *gate) {
    // the stopping flag is read with the operands; a gated launch writes nothing
    const int gv = gate_value(gate);
    double rq = 0.0, qq = 0.0;
    const int k = blockIdx.y;
    if (k == 0) skel_dots_mesh<0>(g, E.p[0], EA.p[0], R.p[0], Q.p[0], rq, qq, blockIdx.x, gridDim.x, gv);
    else if (k == 1) skel_dots_mesh<1>(g, E.p[1], EA.p[1], R.p[1], Q.p[1], rq, qq, blockIdx.x, gridDim.x, gv);
    else skel_dots_mesh<2>(g, E.p[2], EA.p[2], R.p[2], Q.p[2], rq, qq, blockIdx.x, gridDim.x, gv);
    const bool live = flag_clear(gv);
    double vals[2] = {rq, qq};
    if (live) block_partials<256, 2>(vals, partials, blockIdx.x + (size_t)gridDim.x * blockIdx.y);  // block-uniform
    // the update this line search defines is left to the next forward transform (mark non-null)
    if (mark && live && blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) mark->pending = 1;
}

// u += s e and r -= s q on the skeleton (Algorithm 4 step 7 and the residual it implies), the
// projections of r onto the anisotropic meshes for the next error guess (steps 4.1/4.2: r
// restricted to M_k is R_k itself), and partial sums of ||r||^2 over owned points.  The step
// s = max(0, <r,q>/<q,q>) (step 6) is formed by every block from k_skel_dots' partial sums in one
// fixed order, so all blocks agree bit for bit; block 0 records <r,q>, <q,q> and s in scal and marks
// the step's stopping rule pending (FinArgs, applied by the next launch that carries it).
__global__ __launch_bounds__(256) void k_skel_update(Geo g, double *__restrict__ scal, const double *__restrict__ dots,
                                                     int ndots, SkelPtrs U, SkelPtrs E, SkelPtrs R, SkelPtrs Q,
                                                     SkelPtrs G, double *partials, IterState *stt,
                                                     const int *gate) {
    // the stopping flag, the operands of this thread's first point and the partial sums are all
    // loaded before the first barrier; a gated launch writes nothing
    const int gv = gate_value(gate);
    const int per = g.Nc * g.Nf * g.Nf;
    const int k = blockIdx.y;
    double *__restrict__ Uk = (k == 0) ? U.p[0] : (k == 1) ? U.p[1] : U.p[2];
    const double *__restrict__ Ek = (k == 0) ? E.p[0] : (k == 1) ? E.p[1] : E.p[2];
    double *__restrict__ Rk = (k == 0) ? R.p[0] : (k == 1) ? R.p[1] : R.p[2];
    const double *__restrict__ Qk = (k == 0) ? Q.p[0] : (k == 1) ? Q.p[1] : Q.p[2];
    double *__restrict__ Gk = (k == 0) ? G.p[0] : (k == 1) ? G.p[1] : G.p[2];
    const int idx0 = blockIdx.x * 256 + threadIdx.x;
    const int i0 = idx0 < per ? idx0 : 0;
    const double u0 = Uk[i0], e0 = Ek[i0], r0 = Rk[i0], q0 = Qk[i0];
    __shared__ double sh[4], sstep;
    bool live;
    {
        double a0 = 0.0, a1 = 0.0;
        for (int b = threadIdx.x; b < ndots; b += 256) {
            a0 += dots[2 * b];
            a1 += dots[2 * b + 1];
        }
        const double rq = block_sum<256>(a0, sh);
        const double qq = block_sum<256>(a1, sh);
        live = flag_clear(gv);
        if (threadIdx.x == 0) {
            const double st = (qq > 0.0) ? rq / qq : 0.0;
            sstep = (st > 0.0) ? st : 0.0;
            if (live && blockIdx.x == 0 && blockIdx.y == 0) {
                scal[kScalRQ] = rq;
                scal[kScalQQ] = qq;
                scal[kScalStep] = sstep;
                stt->pending = 1;  // the stopping rule on these partial sums is left to a later launch
            }
        }
        __syncthreads();
    }
    if (!live) return;  // block-uniform
    const double s = sstep;
    double acc = 0.0;
    auto update = [&](int idx, double uv, double ev, double rv, double qv) {
        int x0, x1, x2;
        bool own;
        if (k == 0) skel_point<0>(g, idx, x0, x1, x2, own);
        else if (k == 1) skel_point<1>(g, idx, x0, x1, x2, own);
        else skel_point<2>(g, idx, x0, x1, x2, own);
        Uk[idx] = uv + s * ev;
        const double rr = rv - s * qv;
        Rk[idx] = rr;
        Gk[idx] = rr;
        if (own) acc += rr * rr;
    };
    if (idx0 < per) update(idx0, u0, e0, r0, q0);
    for (int idx = idx0 + gridDim.x * 256; idx < per; idx += gridDim.x * 256) update(idx, Uk[idx], Ek[idx], Rk[idx], Qk[idx]);
    double vals[1] = {acc};
    block_partials<256, 1>(vals, partials, blockIdx.x + (size_t)gridDim.x * blockIdx.y);
}

// ---------------------------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------------------------
static SkelPtrs skel_ptrs(double *const *v) {
    SkelPtrs s;
    for (int k = 0; k < kMaxD; ++k) s.p[k] = v[k];
    return s;
}

static int skel_tiles(const Plan &p) {
    const long long per = (long long)p.Nc * p.Nf * p.Nf;
    long long t = (per + 255) / 256;
    const long long cap = 1024;  // per mesh (grid-stride beyond); three meshes' partials fit easily
    if (t > cap) t = cap;
    return (int)(t < 1 ? 1 : t);
}

// k_skel_dots runs on at most 3 x 128 blocks: every block of k_skel_update sums their partials.
static int dots_tiles(const Plan &p) { return std::min(skel_tiles(p), 128); }
// the dots partials sit behind the update's own partials (one value per block) in the workspace
static double *dots_partials(const Plan &p) { return p.ws.partials + 2 * (size_t)p.max_blocks; }

const double *skel_dots_partials(const Plan &p) { return dots_partials(p); }
int skel_dots_count(const Plan &p) { return 3 * dots_tiles(p); }

void launch_skel_gather(const Plan &p, const double *u, hipStream_t st) {
    const int tiles = skel_tiles(p);
    ASDSM_LAUNCH(k_skel_gather, dim3((unsigned)tiles, 3), dim3(256), 0, st, p.geo, u, p.ws.r, skel_ptrs(p.ws.SU),
                 skel_ptrs(p.ws.SR), p.gate);
}

void launch_skel_dots(const Plan &p, hipStream_t st) {
    const int tiles = dots_tiles(p);
    double *E[kMaxD] = {merged_buf(p, 0), merged_buf(p, 1), merged_buf(p, 2)};
    double *R[kMaxD] = {sr_cur(p, 0), sr_cur(p, 1), sr_cur(p, 2)};
    ASDSM_LAUNCH(k_skel_dots, dim3((unsigned)tiles, 3), dim3(256), 0, st, p.geo, skel_ptrs(E), skel_ptrs(p.ws.EA),
                 skel_ptrs(R), skel_ptrs(p.ws.SQ), dots_partials(p), p.upd_fused ? p.ws.state : nullptr, p.gate);
}

void launch_skel_update(const Plan &p, double *const *gather, hipStream_t st) {
    const int tiles = skel_tiles(p);
    double *E[kMaxD] = {merged_buf(p, 0), merged_buf(p, 1), merged_buf(p, 2)};
    double *R[kMaxD] = {sr_cur(p, 0), sr_cur(p, 1), sr_cur(p, 2)};
    double *G[kMaxD] = {gather[1], gather[2], gather[4]};
    ASDSM_LAUNCH(k_skel_update, dim3((unsigned)tiles, 3), dim3(256), 0, st, p.geo, p.ws.scal, dots_partials(p),
                 3 * dots_tiles(p), skel_ptrs(p.ws.SU), skel_ptrs(E), skel_ptrs(R), skel_ptrs(p.ws.SQ),
                 skel_ptrs(G), p.ws.partials, p.ws.state, p.gate);
}

// The stopping rule of the last skeleton-sparse step, left pending by k_skel_update.
FinArgs pending_fin_args(const Plan &p) {
    FinArgs f;
    f.partials = p.ws.partials;
    f.nblk = 3 * skel_tiles(p);
    f.scal = p.ws.scal;
    f.stt = p.ws.state;
    f.hist = p.ws.hist;
    f.step_hist = p.ws.step_hist;
    f.perm_table = p.ws.perm_table;
    return f;
}

__global__ __launch_bounds__(256) void k_finalize_pending(FinArgs f, const int *gate) {
    finalize_pending(f, !(gate && *gate));
}

void launch_finalize_pending(const Plan &p, hipStream_t st) {
    ASDSM_LAUNCH(k_finalize_pending, dim3(1), dim3(256), 0, st, pending_fin_args(p), p.gate);
}

}  // namespace asdsm
