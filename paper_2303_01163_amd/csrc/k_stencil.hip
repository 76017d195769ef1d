// HBM-bound fine-mesh passes:
//   * right-hand side assembly on the fine mesh and on any submesh (source injection plus the
//     Dirichlet terms with the mesh's own spacing, Section 2.3);
//   * the fused iterate update and fine residual  u' = u + s e,  r = b - A u'  (Algorithm 4 steps
//     7 and 3), which also gathers r onto every anisotropic submesh (steps 4.1/4.2) and reduces
//     ||r||^2;
//   * the line-search products q = A e, <r,q>, <q,q> and the clamped step
//     s = max(0, <r,q>/<q,q>) (Algorithm 4 step 6).
// Thread layout of the stencil passes: a block is 4 waves; a wave covers 64 consecutive x_1 points
// of one fine row (rows = the N_f^(d-1) lines along x_1), so loads and stores are row-coalesced.
#include "device_common.hpp"
#include "kernels.hpp"

namespace asdsm {

// ---------------------------------------------------------------------------------------------
// Right-hand side on mesh M_S (canonical layout).  For the fine mesh also reduces ||b||^2.
// ---------------------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_rhs(Geo g, MeshDesc m, const double *__restrict__ s,
                                             const double *__restrict__ gf,
                                             double *__restrict__ out, double *partials,
                                             int with_norm) {
    const int d = g.d;
    const long long faceN = (d == 2) ? g.Nf : (long long)g.Nf * g.Nf;
    double acc = 0.0;
    for (long long idx = (long long)blockIdx.x * 256 + threadIdx.x; idx < m.size;
         idx += (long long)gridDim.x * 256) {
        int i[kMaxD] = {0, 0, 0};
        int cpos[kMaxD] = {0, 0, 0};
        long long rem = idx;
        for (int q = 0; q < d; ++q) {
            const int pos = (int)(rem % m.ext[q]);
            rem /= m.ext[q];
            const int j = m.ax[q];
            if (q < m.nfine) {
                i[j] = pos;
                cpos[j] = -1;
            } else {
                i[j] = (pos + 1) * g.n - 1;
                cpos[j] = pos;
            }
        }
        long long f = i[0] + (long long)g.Nf * (i[1] + (long long)g.Nf * (d == 3 ? i[2] : 0));
        double v = s[f];
        for (int j = 0; j < d; ++j) {
            const bool coarse = (m.mask >> j) & 1u;
            const Tri t = coarse ? g.coarse[j] : g.fine[j];
            const bool lo = coarse ? (cpos[j] == 0) : (i[j] == 0);
            const bool hi = coarse ? (cpos[j] == g.Nc - 1) : (i[j] == g.Nf - 1);
            if (!lo && !hi) continue;
            // face index over the other axes, increasing order, lowest fastest
            long long fidx = 0, mul = 1;
            for (int o = 0; o < d; ++o) {
                if (o == j) continue;
                fidx += (long long)i[o] * mul;
                mul *= g.Nf;
            }
            if (lo) v -= t.a * gf[(long long)(2 * j) * faceN + fidx];
            if (hi) v -= t.c * gf[(long long)(2 * j + 1) * faceN + fidx];
        }
        out[idx] = v;
        acc += v * v;
    }
    if (with_norm) {
        double vals[1] = {acc};
        block_partials<256, 1>(vals, partials, blockIdx.x);
    }
}

// ---------------------------------------------------------------------------------------------
// Fused update + residual + gather.  e == nullptr: plain residual of uin (no update, uout unused).
// ---------------------------------------------------------------------------------------------
template <int D>
__global__ __launch_bounds__(256) void k_update_residual(
    Geo g, const double *__restrict__ uin, const double *__restrict__ e,
    const double *__restrict__ scal, const double *__restrict__ b, double *__restrict__ uout,
    double *__restrict__ r, BoxPtrs boxes, double *partials, const int *gate) {
    if (gate && *gate) return;
    const int Nf = g.Nf, n = g.n;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    const int i0 = blockIdx.y * 64 + tx;
    const int nrows = (int)(g.NF / Nf);
    const double s = e ? scal[kScalStep] : 0.0;
    const int sy = Nf, sz = Nf * Nf;
    const double bsum = g.fine[0].b + g.fine[1].b + (D == 3 ? g.fine[2].b : 0.0);
    double acc = 0.0;
    const int stride = gridDim.x * 4;
    // two rows per thread per pass, so the loads of both are in flight together
    for (int row0 = blockIdx.x * 4 + ty; row0 < nrows; row0 += 2 * stride) {
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const int row = row0 + q * stride;
            if (i0 >= Nf || row >= nrows) continue;
            const int i1 = row % Nf;
            const int i2 = (D == 3) ? row / Nf : 0;
            const int p = i0 + Nf * row;
            auto val = [&](int qq) -> double { return e ? uin[qq] + s * e[qq] : uin[qq]; };
            const double uc = val(p);
            double au = bsum * uc;
            if (i0 > 0) au += g.fine[0].a * val(p - 1);
            if (i0 < Nf - 1) au += g.fine[0].c * val(p + 1);
            if (i1 > 0) au += g.fine[1].a * val(p - sy);
            if (i1 < Nf - 1) au += g.fine[1].c * val(p + sy);
            if (D == 3) {
                if (i2 > 0) au += g.fine[2].a * val(p - sz);
                if (i2 < Nf - 1) au += g.fine[2].c * val(p + sz);
            }
            const double rr = b[p] - au;
            r[p] = rr;
            if (e) uout[p] = uc;
            acc += rr * rr;
            // gather onto the anisotropic submeshes (canonical layouts)
            if (D == 2) {
                if (on_coarse(i0, n)) boxes.p[0][i1 + Nf * coarse_of(i0, n)] = rr;
                if (on_coarse(i1, n)) boxes.p[1][i0 + Nf * coarse_of(i1, n)] = rr;
            } else {
                if (on_coarse(i0, n)) boxes.p[0][i1 + sy * i2 + sz * coarse_of(i0, n)] = rr;
                if (on_coarse(i1, n)) boxes.p[1][i0 + sy * i2 + sz * coarse_of(i1, n)] = rr;
                if (on_coarse(i2, n)) boxes.p[2][i0 + sy * i1 + sz * coarse_of(i2, n)] = rr;
            }
        }
    }
    double vals[1] = {acc};
    block_partials<256, 1>(vals, partials, blockIdx.x + (size_t)gridDim.x * blockIdx.y);
}

// ---------------------------------------------------------------------------------------------
// Line search: q = A e (zero Dirichlet data), <r,q>, <q,q>, s = max(0, <r,q>/<q,q>) (0 if q = 0).
// ---------------------------------------------------------------------------------------------
template <int D>
__global__ __launch_bounds__(256) void k_dots(Geo g, const double *__restrict__ e,
                                              const double *__restrict__ r, double *partials,
                                              const int *gate) {
    if (gate && *gate) return;
    const int Nf = g.Nf;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    const int i0 = blockIdx.y * 64 + tx;
    const int nrows = (int)(g.NF / Nf);
    const int sy = Nf, sz = Nf * Nf;
    const double bsum = g.fine[0].b + g.fine[1].b + (D == 3 ? g.fine[2].b : 0.0);
    double rq = 0.0, qq = 0.0;
    const int stride = gridDim.x * 4;
    for (int row0 = blockIdx.x * 4 + ty; row0 < nrows; row0 += 2 * stride) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int row = row0 + h * stride;
            if (i0 >= Nf || row >= nrows) continue;
            const int i1 = row % Nf;
            const int i2 = (D == 3) ? row / Nf : 0;
            const int p = i0 + Nf * row;
            double q = bsum * e[p];
            if (i0 > 0) q += g.fine[0].a * e[p - 1];
            if (i0 < Nf - 1) q += g.fine[0].c * e[p + 1];
            if (i1 > 0) q += g.fine[1].a * e[p - sy];
            if (i1 < Nf - 1) q += g.fine[1].c * e[p + sy];
            if (D == 3) {
                if (i2 > 0) q += g.fine[2].a * e[p - sz];
                if (i2 < Nf - 1) q += g.fine[2].c * e[p + sz];
            }
            rq += r[p] * q;
            qq += q * q;
        }
    }
    double vals[2] = {rq, qq};
    block_partials<256, 2>(vals, partials, blockIdx.x + (size_t)gridDim.x * blockIdx.y);
}

// ---------------------------------------------------------------------------------------------
// Totals of the per-block partial sums, in block order (deterministic), and what derives from them.
// ---------------------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_finalize(const double *__restrict__ partials, int nblk,
                                                  int mode, int nbox, double *scal, IterState *stt,
                                                  double *hist, double *step_hist, const int *gate) {
    if (gate && *gate) return;
    __shared__ double sh[4];
    const int tid = threadIdx.x;
    if (mode == kFinDots) {
        double a0 = 0.0, a1 = 0.0;
        for (int b = tid; b < nblk; b += 256) {
            a0 += partials[2 * b];
            a1 += partials[2 * b + 1];
        }
        const double rq = block_sum<256>(a0, sh);
        const double qq = block_sum<256>(a1, sh);
        if (tid == 0) {
            scal[kScalRQ] = rq;
            scal[kScalQQ] = qq;
            const double st = (qq > 0.0) ? rq / qq : 0.0;
            scal[kScalStep] = (st > 0.0) ? st : 0.0;
        }
    } else if (mode == kFinBoxNorms) {
        for (int k = 0; k < nbox; ++k) {
            double a = 0.0;
            for (int b = tid; b < nblk; b += 256) a += partials[(size_t)k * nblk + b];
            const double t = block_sum<256>(a, sh);
            if (tid == 0) {
                scal[kScalEnorm2 + k] = t;
                scal[kScalInvNorm + k] = (t > 0.0) ? 1.0 / sqrt(t) : 1.0;
            }
        }
    } else {
        double a = 0.0;
        for (int b = tid; b < nblk; b += 256) a += partials[b];
        const double t = block_sum<256>(a, sh);
        if (tid != 0) return;
        if (mode == kFinBnorm) {
            scal[kScalBnorm2] = t;
            return;
        }
        scal[kScalRnorm2] = t;
        if (mode == kFinRnorm) return;
        // stopping rule of the refinement loop
        const double rn = sqrt(t);
        const double bn = sqrt(scal[kScalBnorm2]);
        if (mode == kFinInit) {
            stt->it = 0;
            stt->stag = 0;
            stt->rn_prev = rn;
            hist[0] = rn;
            if (!isfinite(rn) || !isfinite(bn)) {
                stt->done = 1;
                stt->status = ASDSM_E_NUMERIC;
            } else if ((bn > 0.0 && rn <= stt->rtol * bn) || (bn == 0.0 && rn == 0.0)) {
                stt->done = 1;
                stt->status = ASDSM_OK;
            } else if (stt->max_iter <= 0) {
                stt->done = 1;
                stt->status = ASDSM_MAXITER;
            }
            return;
        }
        // kFinIter: one refinement step has just produced u_{k+1} and r_{k+1}
        const double shat = scal[kScalStep];
        const int it = stt->it + 1;
        stt->it = it;
        if (it < kHistCap) hist[it] = rn;
        if (it - 1 < kHistCap) step_hist[it - 1] = shat;
        if (!isfinite(rn) || !isfinite(shat)) {
            stt->done = 1;
            stt->status = ASDSM_E_NUMERIC;
            return;
        }
        stt->stag = (rn > (1.0 - stt->stag_eta) * stt->rn_prev) ? stt->stag + 1 : 0;
        stt->rn_prev = rn;
        if (shat == 0.0 || (stt->stag_window > 0 && stt->stag >= stt->stag_window)) {
            stt->done = 1;
            stt->status = ASDSM_STAGNATED;
        } else if ((bn > 0.0 && rn <= stt->rtol * bn) || (bn == 0.0 && rn == 0.0)) {
            stt->done = 1;
            stt->status = ASDSM_OK;
        } else if (it >= stt->max_iter) {
            stt->done = 1;
            stt->status = ASDSM_MAXITER;
        }
    }
}

void launch_finalize(const Plan &p, int nblk, int mode, int nbox, hipStream_t st) {
    ASDSM_LAUNCH(k_finalize, dim3(1), dim3(256), 0, st, p.ws.partials, nblk, mode, nbox, p.ws.scal,
                       p.ws.state, p.ws.hist, p.ws.step_hist, p.gate);
}

// ---------------------------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------------------------
static void stencil_grid(const Geo &g, dim3 &grid) {
    const long long nrows = g.NF / g.Nf;
    const int xch = (g.Nf + 63) / 64;
    long long rgs = (nrows + 3) / 4;
    long long cap = 2048 / xch;
    if (cap < 1) cap = 1;
    grid = dim3((unsigned)(rgs < cap ? rgs : cap), (unsigned)xch, 1);
}

int stencil_blocks(const Geo &g) {
    dim3 gr;
    stencil_grid(g, gr);
    return (int)(gr.x * gr.y);
}

void launch_rhs(const Plan &p, unsigned mask, const double *s, const double *gf, double *out,
                bool with_norm, hipStream_t st) {
    const MeshDesc &m = p.mesh[mask];
    long long blocks = (m.size + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    ASDSM_LAUNCH(k_rhs, dim3((unsigned)blocks), dim3(256), 0, st, p.geo, m, s, gf, out,
                       p.ws.partials, with_norm ? 1 : 0);
    if (with_norm) launch_finalize(p, (int)blocks, kFinBnorm, 1, st);
}

void launch_update_residual(const Plan &p, const double *uin, const double *e, double *uout,
                            double *const *gather, int fin_mode, hipStream_t st) {
    dim3 grid;
    stencil_grid(p.geo, grid);
    BoxPtrs bx;
    for (int k = 0; k < kMaxD; ++k) bx.p[k] = (k < p.d) ? gather[1u << k] : nullptr;
    if (p.d == 2)
        ASDSM_LAUNCH((k_update_residual<2>), grid, dim3(256), 0, st, p.geo, uin, e, p.ws.scal,
                           p.ws.b, uout, p.ws.r, bx, p.ws.partials, p.gate);
    else
        ASDSM_LAUNCH((k_update_residual<3>), grid, dim3(256), 0, st, p.geo, uin, e, p.ws.scal,
                           p.ws.b, uout, p.ws.r, bx, p.ws.partials, p.gate);
    launch_finalize(p, (int)(grid.x * grid.y), fin_mode, 1, st);
}

void launch_dots(const Plan &p, hipStream_t st) {
    dim3 grid;
    stencil_grid(p.geo, grid);
    if (p.d == 2)
        ASDSM_LAUNCH((k_dots<2>), grid, dim3(256), 0, st, p.geo, p.ws.e, p.ws.r, p.ws.partials, p.gate);
    else
        ASDSM_LAUNCH((k_dots<3>), grid, dim3(256), 0, st, p.geo, p.ws.e, p.ws.r, p.ws.partials, p.gate);
    launch_finalize(p, (int)(grid.x * grid.y), kFinDots, 1, st);
}

}  // namespace asdsm
