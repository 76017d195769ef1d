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
    long long faceN = 1;  // N_f^(d-1) points per face
    for (int j = 1; j < d; ++j) faceN *= g.Nf;
    double acc = 0.0;
    for (long long idx = (long long)blockIdx.x * 256 + threadIdx.x; idx < m.size;
         idx += (long long)gridDim.x * 256) {
        // fine coordinates i[] and coarse indices cpos[] (-1 on fine axes) of the point; written
        // through compile-time indices only (a run-time index would put the arrays in scratch)
        int i[kMaxD] = {0, 0, 0, 0};
        int cpos[kMaxD] = {0, 0, 0, 0};
        long long rem = idx;
        for (int q = 0; q < d; ++q) {
            const int eq = axis_sel(m.ext, q);
            const int pos = (int)(rem % eq);
            rem /= eq;
            const int j = axis_sel(m.ax, q);
            const bool fine = q < m.nfine;
#pragma unroll
            for (int jj = 0; jj < kMaxD; ++jj)
                if (jj == j) {
                    i[jj] = fine ? pos : (pos + 1) * g.n - 1;
                    cpos[jj] = fine ? -1 : pos;
                }
        }
        long long f = i[0] + (long long)g.Nf * (i[1] + (long long)g.Nf * (i[2] + (long long)g.Nf * i[3]));
        double v = s[f];
#pragma unroll
        for (int j = 0; j < kMaxD; ++j) {
            if (j >= d) break;
            const bool coarse = (m.mask >> j) & 1u;
            const Tri t = coarse ? g.coarse[j] : g.fine[j];
            const bool lo = coarse ? (cpos[j] == 0) : (i[j] == 0);
            const bool hi = coarse ? (cpos[j] == g.Nc - 1) : (i[j] == g.Nf - 1);
            if (!lo && !hi) continue;
            // face index over the other axes, increasing order, lowest fastest
            long long fidx = 0, mul = 1;
#pragma unroll
            for (int o = 0; o < kMaxD; ++o) {
                if (o == j || o >= d) continue;
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
    const int sy = Nf, sz = Nf * Nf, sw = Nf * Nf * Nf;
    const double bsum = g.fine[0].b + g.fine[1].b + (D >= 3 ? g.fine[2].b : 0.0) + (D == 4 ? g.fine[3].b : 0.0);
    double acc = 0.0;
    const int stride = gridDim.x * 4;
    // two rows per thread per pass, so the loads of both are in flight together
    for (int row0 = blockIdx.x * 4 + ty; row0 < nrows; row0 += 2 * stride) {
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const int row = row0 + q * stride;
            if (i0 >= Nf || row >= nrows) continue;
            const int i1 = row % Nf;
            const int i2 = (D == 3) ? row / Nf : (D == 4) ? (row / Nf) % Nf : 0;
            const int i3 = (D == 4) ? row / sz : 0;
            const int p = i0 + Nf * row;
            auto val = [&](int qq) -> double { return e ? uin[qq] + s * e[qq] : uin[qq]; };
            const double uc = val(p);
            double au = bsum * uc;
            if (i0 > 0) au += g.fine[0].a * val(p - 1);
            if (i0 < Nf - 1) au += g.fine[0].c * val(p + 1);
            if (i1 > 0) au += g.fine[1].a * val(p - sy);
            if (i1 < Nf - 1) au += g.fine[1].c * val(p + sy);
            if (D >= 3) {
                if (i2 > 0) au += g.fine[2].a * val(p - sz);
                if (i2 < Nf - 1) au += g.fine[2].c * val(p + sz);
            }
            if (D == 4) {
                if (i3 > 0) au += g.fine[3].a * val(p - sw);
                if (i3 < Nf - 1) au += g.fine[3].c * val(p + sw);
            }
            const double rr = b[p] - au;
            r[p] = rr;
            if (e) uout[p] = uc;
            acc += rr * rr;
            // gather onto the anisotropic submeshes (canonical layouts)
            if (D == 2) {
                if (on_coarse(i0, n)) boxes.p[0][i1 + Nf * coarse_of(i0, n)] = rr;
                if (on_coarse(i1, n)) boxes.p[1][i0 + Nf * coarse_of(i1, n)] = rr;
            } else if (D == 3) {
                if (on_coarse(i0, n)) boxes.p[0][i1 + sy * i2 + sz * coarse_of(i0, n)] = rr;
                if (on_coarse(i1, n)) boxes.p[1][i0 + sy * i2 + sz * coarse_of(i1, n)] = rr;
                if (on_coarse(i2, n)) boxes.p[2][i0 + sy * i1 + sz * coarse_of(i2, n)] = rr;
            } else {
                const long long w = sw;
                if (on_coarse(i0, n)) boxes.p[0][i1 + sy * i2 + sz * i3 + w * coarse_of(i0, n)] = rr;
                if (on_coarse(i1, n)) boxes.p[1][i0 + sy * i2 + sz * i3 + w * coarse_of(i1, n)] = rr;
                if (on_coarse(i2, n)) boxes.p[2][i0 + sy * i1 + sz * i3 + w * coarse_of(i2, n)] = rr;
                if (on_coarse(i3, n)) boxes.p[3][i0 + sy * i1 + sz * i2 + w * coarse_of(i3, n)] = rr;
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
    const int sy = Nf, sz = Nf * Nf, sw = Nf * Nf * Nf;
    const double bsum = g.fine[0].b + g.fine[1].b + (D >= 3 ? g.fine[2].b : 0.0) + (D == 4 ? g.fine[3].b : 0.0);
    double rq = 0.0, qq = 0.0;
    const int stride = gridDim.x * 4;
    for (int row0 = blockIdx.x * 4 + ty; row0 < nrows; row0 += 2 * stride) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int row = row0 + h * stride;
            if (i0 >= Nf || row >= nrows) continue;
            const int i1 = row % Nf;
            const int i2 = (D == 3) ? row / Nf : (D == 4) ? (row / Nf) % Nf : 0;
            const int i3 = (D == 4) ? row / sz : 0;
            const int p = i0 + Nf * row;
            double q = bsum * e[p];
            if (i0 > 0) q += g.fine[0].a * e[p - 1];
            if (i0 < Nf - 1) q += g.fine[0].c * e[p + 1];
            if (i1 > 0) q += g.fine[1].a * e[p - sy];
            if (i1 < Nf - 1) q += g.fine[1].c * e[p + sy];
            if (D >= 3) {
                if (i2 > 0) q += g.fine[2].a * e[p - sz];
                if (i2 < Nf - 1) q += g.fine[2].c * e[p + sz];
            }
            if (D == 4) {
                if (i3 > 0) q += g.fine[3].a * e[p - sw];
                if (i3 < Nf - 1) q += g.fine[3].c * e[p + sw];
            }
            rq += r[p] * q;
            qq += q * q;
        }
    }
    double vals[2] = {rq, qq};
    block_partials<256, 2>(vals, partials, blockIdx.x + (size_t)gridDim.x * blockIdx.y);
}

// ---------------------------------------------------------------------------------------------
// d = 3 versions of the two passes: z-marching column tiles.  A block owns a tile of 64 (x_1) x
// ROWS (x_2) columns and a chunk of ZC planes along x_3; tiles are ordered (z chunk, x_2 tile, x_1
// tile) and each XCD takes one contiguous range of them, so neighbouring tiles share an L2.  Every
// value is read from memory once per tile: the x_3 neighbours stay in registers as the tile marches
// along x_3; the current plane (with a one-point halo loaded by the first 128 + 2 ROWS threads)
// sits in LDS for the x_1 / x_2 neighbours; the next plane's loads are issued one step ahead.
// Neighbours outside the domain enter as zeros (the Dirichlet data live in b).
// ---------------------------------------------------------------------------------------------
struct Tile3 {
    int xtn, ytn, zcn, wn;  // wn: N_f at d = 4 (one x_4 index per tile), 1 at d = 3
};

// d = 4 runs the same tiles over x_1..x_3 for every x_4 index w, with w fastest in the tile order:
// the x_4 neighbours of a tile are the tiles running beside it on the same XCD, so those loads
// (the only ones not covered by the registers and the LDS plane) are served by its L2.
__device__ __forceinline__ bool tile3_of(const Tile3 &t, int &xt, int &yt, int &zc, int &w) {
    const int total = t.xtn * t.ytn * t.zcn * t.wn;
    const int per = (total + 7) / 8;
    const int q = blockIdx.x >> 3;
    int tile = (blockIdx.x & 7) * per + q;
    if (q >= per || tile >= total) return false;
    w = tile % t.wn;
    tile /= t.wn;
    xt = tile % t.xtn;
    yt = (tile / t.xtn) % t.ytn;
    zc = tile / (t.xtn * t.ytn);
    return true;
}

template <int D, int ROWS, int ZC>
__global__ __launch_bounds__(64 * ROWS) void k_update_residual3(
    Geo g, Tile3 tl, const double *__restrict__ uin, const double *__restrict__ e,
    const double *__restrict__ scal, const double *__restrict__ b, double *__restrict__ uout,
    double *__restrict__ r, BoxPtrs boxes, double *partials, const int *gate) {
    if (gate && *gate) return;
    __shared__ double pl[2][ROWS + 2][66];
    const int Nf = g.Nf, n = g.n;
    double acc = 0.0;
    int xt, yt, zc, w;
    if (tile3_of(tl, xt, yt, zc, w)) {
        const double s = e ? scal[kScalStep] : 0.0;
        const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
        const int i0 = xt * 64 + tx, i1 = yt * ROWS + ty;
        const bool act = i0 < Nf && i1 < Nf;
        const int sy = Nf, sz = Nf * Nf, sw = Nf * Nf * Nf;
        const int base = min(i0, Nf - 1) + sy * min(i1, Nf - 1) + (D == 4 ? sw * w : 0);
        const int z0 = zc * ZC, z1 = min(Nf, z0 + ZC);
        const bool wlo = D == 4 && act && w > 0, whi = D == 4 && act && w < Nf - 1;
        // halo of the plane tile: row below, row above, column left, column right
        const int h = threadIdx.x;
        int hx = -1, hy = -1, hlx = 0, hly = 0;
        if (h < 64) {
            hx = xt * 64 + h; hy = yt * ROWS - 1; hlx = h + 1; hly = 0;
        } else if (h < 128) {
            hx = xt * 64 + h - 64; hy = yt * ROWS + ROWS; hlx = h - 63; hly = ROWS + 1;
        } else if (h < 128 + ROWS) {
            hx = xt * 64 - 1; hy = yt * ROWS + (h - 128); hlx = 0; hly = h - 127;
        } else if (h < 128 + 2 * ROWS) {
            hx = xt * 64 + 64; hy = yt * ROWS + (h - 128 - ROWS); hlx = 65; hly = h - 127 - ROWS;
        }
        const bool hload = h < 128 + 2 * ROWS;
        const bool hval = hx >= 0 && hx < Nf && hy >= 0 && hy < Nf;
        const int hbase = hval ? hx + sy * hy + (D == 4 ? sw * w : 0) : 0;
        auto ldu = [&](bool ok, int q) -> double { return ok ? uin[q] : 0.0; };
        auto lde = [&](bool ok, int q) -> double { return (ok && e) ? e[q] : 0.0; };
        double vprev = 0.0, vcur = 0.0, hcur = 0.0;
        if (act && z0 > 0) vprev = ldu(true, base + (z0 - 1) * sz) + s * lde(true, base + (z0 - 1) * sz);
        if (act) vcur = ldu(true, base + z0 * sz) + s * lde(true, base + z0 * sz);
        if (hval) hcur = ldu(true, hbase + z0 * sz) + s * lde(true, hbase + z0 * sz);
        const bool ok1 = act && z0 + 1 < Nf, hok1 = hval && z0 + 1 < z1;
        double u1 = ldu(ok1, base + (z0 + 1) * sz), e1 = lde(ok1, base + (z0 + 1) * sz);
        double hu1 = ldu(hok1, hbase + (z0 + 1) * sz), he1 = lde(hok1, hbase + (z0 + 1) * sz);
        double b1 = act ? b[base + z0 * sz] : 0.0;
        // x_4 neighbours of the current plane (d = 4), loaded one plane ahead
        double wl = 0.0, wh = 0.0;
        if (D == 4) {
            wl = ldu(wlo, base + z0 * sz - sw) + s * lde(wlo, base + z0 * sz - sw);
            wh = ldu(whi, base + z0 * sz + sw) + s * lde(whi, base + z0 * sz + sw);
        }
        int buf = 0;
        pl[0][ty + 1][tx + 1] = vcur;
        if (hload) pl[0][hly][hlx] = hcur;
        __syncthreads();
        const bool g0 = on_coarse(i0, n), g1 = on_coarse(i1, n);
        const int k0 = coarse_of(i0, n), k1 = coarse_of(i1, n);
        const double bsum = g.fine[0].b + g.fine[1].b + g.fine[2].b + (D == 4 ? g.fine[3].b : 0.0);
        for (int z = z0; z < z1; ++z) {
            const int p = base + z * sz;
            double wl1 = 0.0, wh1 = 0.0;
            if (D == 4) {
                const bool nz = z + 1 < z1;
                wl1 = ldu(wlo && nz, p + sz - sw) + s * lde(wlo && nz, p + sz - sw);
                wh1 = ldu(whi && nz, p + sz + sw) + s * lde(whi && nz, p + sz + sw);
            }
            const bool ok2 = act && z + 2 < Nf, hok2 = hval && z + 2 < z1;
            const double u2 = ldu(ok2, p + 2 * sz), e2 = lde(ok2, p + 2 * sz);
            const double hu2 = ldu(hok2, hbase + (z + 2) * sz), he2 = lde(hok2, hbase + (z + 2) * sz);
            const double b2 = (act && z + 1 < z1) ? b[p + sz] : 0.0;
            const double vnext = u1 + s * e1;
            const double hnext = hu1 + s * he1;
            double au = bsum * vcur;
            au += g.fine[0].a * pl[buf][ty + 1][tx];
            au += g.fine[0].c * pl[buf][ty + 1][tx + 2];
            au += g.fine[1].a * pl[buf][ty][tx + 1];
            au += g.fine[1].c * pl[buf][ty + 2][tx + 1];
            au += g.fine[2].a * vprev;
            au += g.fine[2].c * vnext;
            if (D == 4) {
                au += g.fine[3].a * wl;
                au += g.fine[3].c * wh;
            }
            const double rr = b1 - au;
            if (act) {
                r[p] = rr;
                if (e) uout[p] = vcur;
                acc += rr * rr;
                // gather onto the anisotropic submeshes (canonical layouts)
                if (D == 3) {
                    if (g0) boxes.p[0][i1 + sy * z + sz * k0] = rr;
                    if (g1) boxes.p[1][i0 + sy * z + sz * k1] = rr;
                    if (on_coarse(z, n)) boxes.p[2][i0 + sy * i1 + sz * coarse_of(z, n)] = rr;
                } else {
                    if (g0) boxes.p[0][i1 + sy * z + sz * w + sw * k0] = rr;
                    if (g1) boxes.p[1][i0 + sy * z + sz * w + sw * k1] = rr;
                    if (on_coarse(z, n)) boxes.p[2][i0 + sy * i1 + sz * w + sw * coarse_of(z, n)] = rr;
                    if (on_coarse(w, n)) boxes.p[3][i0 + sy * i1 + sz * z + sw * coarse_of(w, n)] = rr;
                }
            }
            wl = wl1;
            wh = wh1;
            vprev = vcur;
            vcur = vnext;
            u1 = u2; e1 = e2; hu1 = hu2; he1 = he2; b1 = b2;
            buf ^= 1;
            pl[buf][ty + 1][tx + 1] = vcur;
            if (hload) pl[buf][hly][hlx] = hnext;
            __syncthreads();
        }
    }
    double vals[1] = {acc};
    block_partials<64 * ROWS, 1>(vals, partials, blockIdx.x);
}

// Line-search products q = A e, <r, q>, <q, q> with the same z-marching tiles as the update pass:
// the current plane of e with its one-point halo in LDS (double-buffered), the x_3 neighbours in
// registers, and the next plane's e, halo and r loaded one step ahead.
template <int D, int ROWS, int ZC>
__global__ __launch_bounds__(64 * ROWS) void k_dots3(Geo g, Tile3 tl, const double *__restrict__ e,
                                                     const double *__restrict__ r, double *partials,
                                                     const int *gate) {
    if (gate && *gate) return;
    __shared__ double pl[2][ROWS + 2][66];
    const int Nf = g.Nf;
    double rq = 0.0, qq = 0.0;
    int xt, yt, zc, w;
    if (tile3_of(tl, xt, yt, zc, w)) {
        const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
        const int i0 = xt * 64 + tx, i1 = yt * ROWS + ty;
        const bool act = i0 < Nf && i1 < Nf;
        const int sy = Nf, sz = Nf * Nf, sw = Nf * Nf * Nf;
        const int base = min(i0, Nf - 1) + sy * min(i1, Nf - 1) + (D == 4 ? sw * w : 0);
        const int z0 = zc * ZC, z1 = min(Nf, z0 + ZC);
        const bool wlo = D == 4 && act && w > 0, whi = D == 4 && act && w < Nf - 1;
        // halo of the plane tile: row below, row above, column left, column right
        const int h = threadIdx.x;
        int hx = -1, hy = -1, hlx = 0, hly = 0;
        if (h < 64) {
            hx = xt * 64 + h; hy = yt * ROWS - 1; hlx = h + 1; hly = 0;
        } else if (h < 128) {
            hx = xt * 64 + h - 64; hy = yt * ROWS + ROWS; hlx = h - 63; hly = ROWS + 1;
        } else if (h < 128 + ROWS) {
            hx = xt * 64 - 1; hy = yt * ROWS + (h - 128); hlx = 0; hly = h - 127;
        } else if (h < 128 + 2 * ROWS) {
            hx = xt * 64 + 64; hy = yt * ROWS + (h - 128 - ROWS); hlx = 65; hly = h - 127 - ROWS;
        }
        const bool hload = h < 128 + 2 * ROWS;
        const bool hval = hx >= 0 && hx < Nf && hy >= 0 && hy < Nf;
        const int hbase = hval ? hx + sy * hy + (D == 4 ? sw * w : 0) : 0;
        double vprev = (act && z0 > 0) ? e[base + (z0 - 1) * sz] : 0.0;
        double vcur = act ? e[base + z0 * sz] : 0.0;
        const double hcur = hval ? e[hbase + z0 * sz] : 0.0;
        double v1 = (act && z0 + 1 < Nf) ? e[base + (z0 + 1) * sz] : 0.0;
        double hv1 = (hval && z0 + 1 < z1) ? e[hbase + (z0 + 1) * sz] : 0.0;
        double r1 = act ? r[base + z0 * sz] : 0.0;
        double wl = wlo ? e[base + z0 * sz - sw] : 0.0, wh = whi ? e[base + z0 * sz + sw] : 0.0;
        int buf = 0;
        pl[0][ty + 1][tx + 1] = vcur;
        if (hload) pl[0][hly][hlx] = hcur;
        __syncthreads();
        const double bsum = g.fine[0].b + g.fine[1].b + g.fine[2].b + (D == 4 ? g.fine[3].b : 0.0);
        for (int z = z0; z < z1; ++z) {
            const int p = base + z * sz;
            const bool nz = z + 1 < z1;
            const double wl1 = (wlo && nz) ? e[p + sz - sw] : 0.0;
            const double wh1 = (whi && nz) ? e[p + sz + sw] : 0.0;
            // one step ahead: e two planes up (the next plane's upper neighbour), its halo, next r
            const double v2 = (act && z + 2 < Nf) ? e[p + 2 * sz] : 0.0;
            const double hv2 = (hval && z + 2 < z1) ? e[hbase + (z + 2) * sz] : 0.0;
            const double r2 = (act && z + 1 < z1) ? r[p + sz] : 0.0;
            double q = bsum * vcur;
            q += g.fine[0].a * pl[buf][ty + 1][tx];
            q += g.fine[0].c * pl[buf][ty + 1][tx + 2];
            q += g.fine[1].a * pl[buf][ty][tx + 1];
            q += g.fine[1].c * pl[buf][ty + 2][tx + 1];
            q += g.fine[2].a * vprev;
            q += g.fine[2].c * v1;
            if (D == 4) {
                q += g.fine[3].a * wl;
                q += g.fine[3].c * wh;
            }
            wl = wl1;
            wh = wh1;
            if (act) {
                rq += r1 * q;
                qq += q * q;
            }
            vprev = vcur;
            vcur = v1;
            v1 = v2;
            const double hnext = hv1;
            hv1 = hv2;
            r1 = r2;
            buf ^= 1;
            pl[buf][ty + 1][tx + 1] = vcur;
            if (hload) pl[buf][hly][hlx] = hnext;
            __syncthreads();
        }
    }
    double vals[2] = {rq, qq};
    block_partials<64 * ROWS, 2>(vals, partials, blockIdx.x);
}

// ---------------------------------------------------------------------------------------------
// Totals of the per-block partial sums, in block order (deterministic), and what derives from them.
// ---------------------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_finalize(const double *__restrict__ partials, int nblk,
                                                  int mode, int nbox, double *scal, IterState *stt,
                                                  double *hist, double *step_hist, const int *perm_table,
                                                  const int *gate) {
    // the stopping flag is read with the partial sums and tested before anything is written
    const int gv = gate_value(gate);
    __shared__ double sh[4];
    const int tid = threadIdx.x;
    if (mode == kFinDots) {
        double a0 = 0.0, a1 = 0.0;
        // unrolled: the loads of several trips in flight, the additions in the same order
#pragma unroll 8
        for (int b = tid; b < nblk; b += 256) {
            a0 += partials[2 * b];
            a1 += partials[2 * b + 1];
        }
        const double rq = block_sum<256>(a0, sh);
        const double qq = block_sum<256>(a1, sh);
        if (tid == 0 && flag_clear(gv)) {
            scal[kScalRQ] = rq;
            scal[kScalQQ] = qq;
            const double st = (qq > 0.0) ? rq / qq : 0.0;
            scal[kScalStep] = (st > 0.0) ? st : 0.0;
        }
    } else if (mode == kFinBoxNorms) {
        for (int k = 0; k < nbox; ++k) {
            double a = 0.0;
#pragma unroll 8
            for (int b = tid; b < nblk; b += 256) a += partials[(size_t)k * nblk + b];
            const double t = block_sum<256>(a, sh);
            if (tid == 0 && flag_clear(gv)) {
                scal[kScalEnorm2 + k] = t;
                scal[kScalInvNorm + k] = (t > 0.0) ? 1.0 / sqrt(t) : 1.0;
            }
        }
    } else {
        double a = 0.0;
#pragma unroll 8
        for (int b = tid; b < nblk; b += 256) a += partials[b];
        const double t = block_sum<256>(a, sh);
        if (tid != 0 || !flag_clear(gv)) return;
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
        finalize_step(t, scal, stt, hist, step_hist, perm_table);
    }
}

void launch_finalize(const Plan &p, int nblk, int mode, int nbox, hipStream_t st) {
    ASDSM_LAUNCH(k_finalize, dim3(1), dim3(256), 0, st, p.ws.partials, nblk, mode, nbox, p.ws.scal,
                       p.ws.state, p.ws.hist, p.ws.step_hist, p.ws.perm_table, p.gate);
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

void launch_rhs(const Plan &p, unsigned mask, const double *s, const double *gf, double *out,
                bool with_norm, hipStream_t st) {
    const MeshDesc &m = p.mesh[mask];
    long long blocks = (m.size + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    ASDSM_LAUNCH(k_rhs, dim3((unsigned)blocks), dim3(256), 0, st, p.geo, m, s, gf, out,
                       p.ws.partials, with_norm ? 1 : 0);
    if (with_norm) launch_finalize(p, (int)blocks, kFinBnorm, 1, st);
}

static Tile3 tile3(const Geo &g, int rows, int zc, int &blocks) {
    Tile3 t;
    t.xtn = (g.Nf + 63) / 64;
    t.ytn = (g.Nf + rows - 1) / rows;
    t.zcn = (g.Nf + zc - 1) / zc;
    t.wn = (g.d == 4) ? g.Nf : 1;
    const long long total = (long long)t.xtn * t.ytn * t.zcn * t.wn;
    blocks = (int)(8 * ((total + 7) / 8));
    return t;
}

void launch_update_residual(const Plan &p, const double *uin, const double *e, double *uout,
                            double *const *gather, int fin_mode, hipStream_t st) {
    BoxPtrs bx;
    for (int k = 0; k < kMaxD; ++k) bx.p[k] = (k < p.d) ? gather[1u << k] : nullptr;
    int blocks = 0;
    if (p.d == 4) {
        const Tile3 t = tile3(p.geo, 8, 8, blocks);
        if (blocks <= p.max_blocks) {
            ASDSM_LAUNCH((k_update_residual3<4, 8, 8>), dim3(blocks), dim3(512), 0, st, p.geo, t, uin, e,
                         p.ws.scal, p.ws.b, uout, p.ws.r, bx, p.ws.partials, p.gate);
            launch_finalize(p, blocks, fin_mode, 1, st);
            return;
        }
    }
    if (p.d == 2 || p.d == 4) {
        dim3 grid;
        stencil_grid(p.geo, grid);
        if (p.d == 2)
            ASDSM_LAUNCH((k_update_residual<2>), grid, dim3(256), 0, st, p.geo, uin, e, p.ws.scal,
                         p.ws.b, uout, p.ws.r, bx, p.ws.partials, p.gate);
        else
            ASDSM_LAUNCH((k_update_residual<4>), grid, dim3(256), 0, st, p.geo, uin, e, p.ws.scal,
                         p.ws.b, uout, p.ws.r, bx, p.ws.partials, p.gate);
        launch_finalize(p, (int)(grid.x * grid.y), fin_mode, 1, st);
        return;
    }
    if (p.Nf >= 255) {
        const Tile3 t = tile3(p.geo, 16, 16, blocks);
        ASDSM_LAUNCH((k_update_residual3<3, 16, 16>), dim3(blocks), dim3(1024), 0, st, p.geo, t, uin, e,
                     p.ws.scal, p.ws.b, uout, p.ws.r, bx, p.ws.partials, p.gate);
    } else {
        const Tile3 t = tile3(p.geo, 8, 8, blocks);
        ASDSM_LAUNCH((k_update_residual3<3, 8, 8>), dim3(blocks), dim3(512), 0, st, p.geo, t, uin, e,
                     p.ws.scal, p.ws.b, uout, p.ws.r, bx, p.ws.partials, p.gate);
    }
    launch_finalize(p, blocks, fin_mode, 1, st);
}

void launch_dots(const Plan &p, hipStream_t st) {
    int blocks = 0;
    if (p.d == 4) {
        const Tile3 t = tile3(p.geo, 8, 8, blocks);
        if (2 * blocks <= p.max_blocks) {
            ASDSM_LAUNCH((k_dots3<4, 8, 8>), dim3(blocks), dim3(512), 0, st, p.geo, t, p.ws.e, p.ws.r,
                         p.ws.partials, p.gate);
            launch_finalize(p, blocks, kFinDots, 1, st);
            return;
        }
    }
    if (p.d == 2 || p.d == 4) {
        dim3 grid;
        stencil_grid(p.geo, grid);
        if (p.d == 2)
            ASDSM_LAUNCH((k_dots<2>), grid, dim3(256), 0, st, p.geo, p.ws.e, p.ws.r, p.ws.partials, p.gate);
        else
            ASDSM_LAUNCH((k_dots<4>), grid, dim3(256), 0, st, p.geo, p.ws.e, p.ws.r, p.ws.partials, p.gate);
        launch_finalize(p, (int)(grid.x * grid.y), kFinDots, 1, st);
        return;
    }
    if (p.geo.Nf >= 255) {
        const Tile3 t = tile3(p.geo, 16, 16, blocks);
        ASDSM_LAUNCH((k_dots3<3, 16, 16>), dim3(blocks), dim3(1024), 0, st, p.geo, t, p.ws.e, p.ws.r,
                     p.ws.partials, p.gate);
    } else {
        const Tile3 t = tile3(p.geo, 8, 8, blocks);
        ASDSM_LAUNCH((k_dots3<3, 8, 8>), dim3(blocks), dim3(512), 0, st, p.geo, t, p.ws.e, p.ws.r,
                     p.ws.partials, p.gate);
    }
    launch_finalize(p, blocks, kFinDots, 1, st);
}

}  // namespace asdsm
