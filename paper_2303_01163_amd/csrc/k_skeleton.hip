// Skeleton builder (Algorithm 2) and filler (Algorithm 3).
//
// Cross points (points of an anisotropic mesh M_k that also lie on another mesh) take
//   * in the initial guess: uhat = (sum_{j in S(p)} u_j(p) - u_{S(p)}(p)) / (|S(p)| - 1), the
//     extrapolation that combines the anisotropic solutions with the solution on the intersection
//     mesh M_{S(p)} (for d = 2 this is P u_fc + P u_cf - u_cc);
//   * in the error phase: the value of the first mesh of this iteration's random axis permutation
//     that contains the point (one random choice per iteration), after normalisation.
// The discrepancy delta_k = uhat - u_k on the cross points of M_k is extended over M_k by the cubic
// not-a-knot spline with zero end values along each fine axis (Boolean sum for two fine axes) and
// added; the merged skeleton value is the corrected u_k on points of one mesh only and uhat on cross
// points (step 6).  The merged values are written per anisotropic mesh (canonical layout); the
// filler reads them as Dirichlet data of the holes and writes whole fine tiles.
#include <algorithm>

#include "device_common.hpp"
#include "kernels.hpp"

namespace asdsm {

struct SkelArgs {
    const double *res[kMaxMeshes];  // solution on each mesh (canonical layout)
    MeshDesc mesh[kMaxMeshes];
    double *lines[kMaxD];           // discrepancy lines per anisotropic mesh
    double *skel[kMaxD];            // merged skeleton values per anisotropic mesh (output)
    const double *Sp;               // N_f x N_c spline matrix
    const double *scal;             // normalisation factors (error phase)
    int mode;                       // 0 initial guess, 1 error phase
    const IterState *state;
    const int *gate;
    // error phase with the plane kernel: per-block partial sums of squares of each anisotropic
    // solution (norm_nblk per mesh, mesh-major), from which every block forms the normalisation
    // itself; nullptr: the factors are in scal (k_box_norms)
    const double *norm_partials;
    int norm_nblk;
};

// A fine point as three coordinates (x2 = 0 for d = 2).  The helpers below index only with
// compile-time constants or selects, so nothing lands in scratch memory.
struct Pt {
    int x0, x1, x2;
};

// Point of anisotropic mesh M_k: coordinate c on the coarse axis k, u and v on its fine axes
// (increasing order).
__device__ __forceinline__ Pt mesh_pt(int k, int d, int u, int v, int c) {
    if (d == 2) return (k == 0) ? Pt{c, u, 0} : Pt{u, c, 0};
    if (k == 0) return Pt{c, u, v};
    if (k == 1) return Pt{u, c, v};
    return Pt{u, v, c};
}

__device__ __forceinline__ unsigned coarse_set(const Pt &p, int d, int n) {
    unsigned S = 0;
    if (on_coarse(p.x0, n)) S |= 1u;
    if (on_coarse(p.x1, n)) S |= 2u;
    if (d == 3 && on_coarse(p.x2, n)) S |= 4u;
    return S;
}

// Offset of a point of M_j (coarse axis j) in its canonical layout (fine axes a < b, then j).
__device__ __forceinline__ long long aniso_offset(const Geo &g, int j, const Pt &p) {
    const long long Nf = g.Nf;
    if (g.d == 2) return (j == 0) ? p.x1 + Nf * coarse_of(p.x0, g.n) : p.x0 + Nf * coarse_of(p.x1, g.n);
    if (j == 0) return p.x1 + Nf * (p.x2 + Nf * coarse_of(p.x0, g.n));
    if (j == 1) return p.x0 + Nf * (p.x2 + Nf * coarse_of(p.x1, g.n));
    return p.x0 + Nf * (p.x1 + Nf * coarse_of(p.x2, g.n));
}

// Offset of a point of the intersection mesh M_S (|S| >= 2) in its canonical layout: the fine axis
// (if any) first, then the coarse axes in increasing order.
__device__ __forceinline__ long long inter_offset(const Geo &g, unsigned S, const Pt &p) {
    const long long Nf = g.Nf, Nc = g.Nc;
    const int n = g.n;
    const long long c0 = coarse_of(p.x0, n), c1 = coarse_of(p.x1, n);
    if (g.d == 2) return c0 + Nc * c1;
    const long long c2 = coarse_of(p.x2, n);
    if (S == 7u) return c0 + Nc * (c1 + Nc * c2);
    if (S == 6u) return p.x0 + Nf * (c1 + Nc * c2);  // fine x_1
    if (S == 5u) return p.x1 + Nf * (c0 + Nc * c2);  // fine x_2
    return p.x2 + Nf * (c0 + Nc * c1);               // S = 3, fine x_3
}

// Per-launch values of the error phase, read once per block before the point loop: this step's
// axis permutation and the normalisation factors 1/||e_k||.  Must be called by every thread of the
// block (the factors may come from a block reduction).
struct XChoice {
    int p0, p1, p2;
    double inv0, inv1, inv2;
};

__device__ __forceinline__ XChoice load_choice(const SkelArgs &a, const Geo &g) {
    XChoice c{0, 1, 2, 1.0, 1.0, 1.0};
    if (a.mode == 1) {
        const int *perm = a.state->perm;
        c.p0 = perm[0];
        c.p1 = perm[1];
        c.p2 = (g.d == 3) ? perm[2] : 2;
        if (a.norm_partials) {
            // the three sums in one pass: their loads are issued together, one reduction in a
            // fixed order (every block of every launch gets the same values)
            __shared__ double sh[3][16];
            const int nb = a.norm_nblk;
            const bool three = (g.d == 3);
            double v0 = 0.0, v1 = 0.0, v2 = 0.0;
            for (int b = threadIdx.x; b < nb; b += blockDim.x) {
                v0 += a.norm_partials[b];
                v1 += a.norm_partials[(size_t)nb + b];
                if (three) v2 += a.norm_partials[2 * (size_t)nb + b];
            }
            for (int off = 32; off > 0; off >>= 1) {
                v0 += __shfl_down(v0, off, 64);
                v1 += __shfl_down(v1, off, 64);
                v2 += __shfl_down(v2, off, 64);
            }
            if ((threadIdx.x & 63) == 0) {
                sh[0][threadIdx.x >> 6] = v0;
                sh[1][threadIdx.x >> 6] = v1;
                sh[2][threadIdx.x >> 6] = v2;
            }
            __syncthreads();
            double t0 = 0.0, t1 = 0.0, t2 = 0.0;
            for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
                t0 += sh[0][w];
                t1 += sh[1][w];
                t2 += sh[2][w];
            }
            c.inv0 = (t0 > 0.0) ? 1.0 / sqrt(t0) : 1.0;
            c.inv1 = (t1 > 0.0) ? 1.0 / sqrt(t1) : 1.0;
            c.inv2 = three ? ((t2 > 0.0) ? 1.0 / sqrt(t2) : 1.0) : 1.0;
        } else {
            c.inv0 = a.scal[kScalInvNorm + 0];
            c.inv1 = a.scal[kScalInvNorm + 1];
            c.inv2 = (g.d == 3) ? a.scal[kScalInvNorm + 2] : 1.0;
        }
    }
    return c;
}

__device__ __forceinline__ double inv_of(const XChoice c, int k) { return k == 0 ? c.inv0 : (k == 1 ? c.inv1 : c.inv2); }

__device__ __forceinline__ double crosspoint_value(const SkelArgs &a, const Geo &g, const Pt &p,
                                                  unsigned S, const XChoice ch) {
    if (a.mode == 0) {
        double sum = 0.0;
        int cnt = 0;
        if (S & 1u) { sum += a.res[1][aniso_offset(g, 0, p)]; ++cnt; }
        if (S & 2u) { sum += a.res[2][aniso_offset(g, 1, p)]; ++cnt; }
        if (S & 4u) { sum += a.res[4][aniso_offset(g, 2, p)]; ++cnt; }
        // the intersection mesh's solution by integer arithmetic on the four pointers: a chain of
        // selects among the argument struct's fields becomes one load at a computed offset, which
        // copies the struct to scratch memory
        const unsigned long long r3 = (unsigned long long)a.res[3], r5 = (unsigned long long)a.res[5],
                                 r6 = (unsigned long long)a.res[6], r7 = (unsigned long long)a.res[7];
        const double *rs = (const double *)((S == 3u) * r3 + (S == 5u) * r5 + (S == 6u) * r6 + (S == 7u) * r7);
        sum -= rs[inter_offset(g, S, p)];
        return sum / (double)(cnt - 1);
    }
    // the first axis of this step's permutation that contains the point
    int j = ch.p0;
    if (!((S >> j) & 1u)) j = ch.p1;
    if (!((S >> j) & 1u)) j = ch.p2;
    const double inv = inv_of(ch, j);
    const double *rj = (j == 0) ? a.res[1] : (j == 1) ? a.res[2] : a.res[4];
    return inv * rj[aniso_offset(g, j, p)];
}

// Error phase, in two halves so that the loads can be issued before this step's choice is known:
// the solutions of the anisotropic meshes that contain a cross point (0 for the others), then the
// value of the first axis of the permutation among them, normalised.
struct XCand {
    double v0, v1, v2;
};

__device__ __forceinline__ XCand cross_candidates(const SkelArgs &a, const Geo &g, const Pt &p, unsigned S) {
    // every lane issues all three loads, with offset 0 for a mesh that does not hold the point:
    // no branches and no use of the values here, so they stay in flight with the caller's other
    // loads; cross_pick only ever takes the value of a mesh that holds the point
    return XCand{a.res[1][(S & 1u) ? aniso_offset(g, 0, p) : 0], a.res[2][(S & 2u) ? aniso_offset(g, 1, p) : 0],
                 a.res[4][(S & 4u) ? aniso_offset(g, 2, p) : 0]};
}

__device__ __forceinline__ double cross_pick(const XChoice ch, unsigned S, const XCand c) {
    int j = ch.p0;
    if (!((S >> j) & 1u)) j = ch.p1;
    if (!((S >> j) & 1u)) j = ch.p2;
    return inv_of(ch, j) * ((j == 0) ? c.v0 : (j == 1) ? c.v1 : c.v2);
}

__device__ __forceinline__ void fine_axes_of(int k, int d, int &a, int &b) {
    if (d == 2) {
        a = 1 - k;
        b = -1;
    } else {
        a = (k == 0) ? 1 : 0;
        b = (k == 2) ? 1 : 2;
    }
}

// d = 2: delta_k on the cross points of each anisotropic mesh, lines[k][ck*Nc + ca].
__global__ __launch_bounds__(256) void k_crosspoints(Geo g, SkelArgs a) {
    if (a.gate && *a.gate) return;
    const XChoice ch = load_choice(a, g);
    const int k = blockIdx.y;
    const int Nf = g.Nf, Nc = g.Nc, n = g.n;
    const double scale_k = (a.mode == 0) ? 1.0 : inv_of(ch, k);
    const long long total = (long long)Nc * Nc;
    const double *__restrict__ Xk = (k == 0) ? a.res[1] : a.res[2];
    for (long long t = (long long)blockIdx.x * 256 + threadIdx.x; t < total; t += (long long)gridDim.x * 256) {
        const int ca = (int)(t % Nc), ck = (int)(t / Nc);
        const int u = (ca + 1) * n - 1;
        const Pt p = mesh_pt(k, 2, u, 0, (ck + 1) * n - 1);
        const double uh = crosspoint_value(a, g, p, coarse_set(p, 2, n), ch);
        a.lines[k][t] = uh - scale_k * Xk[(long long)u + (long long)Nf * ck];
    }
}

// d = 3 layout of the discrepancy lines of M_k: part A [ck][ca][ib] (Nc*Nc*Nf), part B
// [ck][ia][cb] (Nc*Nf*Nc), then part R [ck][ca][ib] = A[ck][ca][ib] - sum_cb Sp[ib][cb]
// A[ck][ca][C[cb]], so that the Boolean sum P_a delta + P_b delta - P_a P_b delta = P_a R + P_b delta
// costs O(N_c) per point.
// d = 3: the discrepancies of part A row by row -- one block per (c_k, c_a) row of N_f values, kept
// in LDS -- together with that row's Boolean-sum remainder R (below), and part B by the remaining
// blocks: one launch where k_crosspoints and k_lines_residual take two.
__global__ __launch_bounds__(256) void k_crosspoints3(Geo g, SkelArgs a, int nrowblk) {
    // the stopping flag is read with the first loads and tested once they have arrived; a gated
    // launch writes nothing
    const int gv = gate_value(a.gate);
    __shared__ double row[1024];  // N_f <= 1023
    const int k = blockIdx.y;
    const int Nf = g.Nf, Nc = g.Nc, n = g.n;
    const long long nA = (long long)Nc * Nc * Nf;
    const double *__restrict__ Xk = (k == 0) ? a.res[1] : (k == 1) ? a.res[2] : a.res[4];
    double *__restrict__ lk = (k == 0) ? a.lines[0] : (k == 1) ? a.lines[1] : a.lines[2];
    const bool err = a.mode == 1;
    // the loads of one discrepancy: M_k's own value and, in the error phase, the candidates
    struct Ld {
        double x;
        XCand c;
    };
    auto fetch = [&](int u, int v, int ck) -> Ld {
        Ld l;
        l.x = Xk[(long long)u + (long long)Nf * (v + (long long)Nf * ck)];
        l.c = XCand{0.0, 0.0, 0.0};
        if (err) {
            const Pt p = mesh_pt(k, 3, u, v, (ck + 1) * n - 1);
            l.c = cross_candidates(a, g, p, coarse_set(p, 3, n));
        }
        return l;
    };
    auto delta = [&](int u, int v, int ck, const Ld &l, const XChoice &ch, double scale_k) -> double {
        const Pt p = mesh_pt(k, 3, u, v, (ck + 1) * n - 1);
        const unsigned S = coarse_set(p, 3, n);
        const double uh = err ? cross_pick(ch, S, l.c) : crosspoint_value(a, g, p, S, ch);
        return uh - scale_k * l.x;
    };
    // this block's first row (part A) or first entry (part B) is loaded before the choice
    constexpr int KP = 4;  // entries of a row per thread (N_f <= 1023)
    const bool partA = (int)blockIdx.x < nrowblk;
    Ld pre[KP];
    if (partA) {
        const int rw = blockIdx.x;  // < N_c^2: nrowblk <= N_c^2
        const int u = (rw % Nc + 1) * n - 1, ck = rw / Nc;
#pragma unroll
        for (int j = 0; j < KP; ++j) {
            const int ib = threadIdx.x + 256 * j;
            if (ib < Nf) pre[j] = fetch(u, ib, ck);
        }
    } else {
        const long long w = (long long)(blockIdx.x - nrowblk) * 256 + threadIdx.x;
        if (w < nA) pre[0] = fetch((int)((w / Nc) % Nf), ((int)(w % Nc) + 1) * n - 1, (int)(w / ((long long)Nc * Nf)));
    }
    const XChoice ch = load_choice(a, g);
    if (!flag_clear(gv)) return;  // block-uniform
    const double scale_k = (a.mode == 0) ? 1.0 : inv_of(ch, k);
    if (partA) {
        bool first = true;
        for (int rw = blockIdx.x; rw < Nc * Nc; rw += nrowblk, first = false) {
            const int ca = rw % Nc, ck = rw / Nc;
            const int u = (ca + 1) * n - 1;
            double *__restrict__ A = lk + (long long)rw * Nf;
            double *__restrict__ R = lk + 2 * nA + (long long)rw * Nf;
#pragma unroll
            for (int j = 0; j < KP; ++j) {
                const int ib = threadIdx.x + 256 * j;
                if (ib < Nf) {
                    const double dv = delta(u, ib, ck, first ? pre[j] : fetch(u, ib, ck), ch, scale_k);
                    A[ib] = dv;
                    row[ib] = dv;
                }
            }
            __syncthreads();
            for (int ib = threadIdx.x; ib < Nf; ib += 256) {
                double v = 0.0;
                if (!on_coarse(ib, n)) {
                    v = row[ib];
                    for (int cb = 0; cb < Nc; ++cb) v -= a.Sp[(long long)ib * Nc + cb] * row[(cb + 1) * n - 1];
                }
                R[ib] = v;
            }
            __syncthreads();
        }
        return;
    }
    // part B: [ck][ia][cb]
    bool first = true;
    for (long long w = (long long)(blockIdx.x - nrowblk) * 256 + threadIdx.x; w < nA;
         w += (long long)(gridDim.x - nrowblk) * 256, first = false) {
        const int cb = (int)(w % Nc);
        const int u = (int)((w / Nc) % Nf);
        const int ck = (int)(w / ((long long)Nc * Nf));
        const int v = (cb + 1) * n - 1;
        lk[nA + w] = delta(u, v, ck, first ? pre[0] : fetch(u, v, ck), ch, scale_k);
    }
}

__global__ __launch_bounds__(256) void k_merge(Geo g, SkelArgs a) {
    if (a.gate && *a.gate) return;
    const XChoice ch = load_choice(a, g);
    const int k = blockIdx.y;
    const int d = g.d, Nf = g.Nf, Nc = g.Nc, n = g.n;
    int fa, fb;
    fine_axes_of(k, d, fa, fb);
    const unsigned mk = 1u << k;
    const MeshDesc &m = a.mesh[mk];
    const double scale_k = (a.mode == 0) ? 1.0 : inv_of(ch, k);
    const double *__restrict__ X = a.res[mk];
    double *__restrict__ out = a.skel[k];
    const double *__restrict__ L = a.lines[k];
    const double *__restrict__ Sp = a.Sp;
    const long long nA = (long long)Nc * Nc * Nf;
    for (long long idx = (long long)blockIdx.x * 256 + threadIdx.x; idx < m.size; idx += (long long)gridDim.x * 256) {
        const int ia = (int)(idx % Nf);
        int ib = 0, ck;
        if (d == 2) {
            ck = (int)(idx / Nf);
        } else {
            ib = (int)((idx / Nf) % Nf);
            ck = (int)(idx / ((long long)Nf * Nf));
        }
        const Pt p = mesh_pt(k, d, ia, ib, (ck + 1) * n - 1);
        const unsigned S = coarse_set(p, d, n);
        double v;
        if (S != mk) {
            v = crosspoint_value(a, g, p, S, ch);
        } else if (d == 2) {
            double corr = 0.0;
            for (int ca = 0; ca < Nc; ++ca) corr += Sp[(long long)ia * Nc + ca] * L[(long long)ck * Nc + ca];
            v = scale_k * X[idx] + corr;
        } else {
            const double *__restrict__ R = L + 2 * nA;
            const double *__restrict__ B = L + nA;
            double c1 = 0.0, c2 = 0.0;
            for (int ca = 0; ca < Nc; ++ca)
                c1 += Sp[(long long)ia * Nc + ca] * R[((long long)ck * Nc + ca) * Nf + ib];
            for (int cb = 0; cb < Nc; ++cb)
                c2 += Sp[(long long)ib * Nc + cb] * B[((long long)ck * Nf + ia) * Nc + cb];
            v = scale_k * X[idx] + (c1 + c2);
        }
        out[idx] = v;
    }
}

// d = 3 merge by tiles, with the discrepancies of the tile formed in place: block (64 values of
// i_a x 8 values of i_b, coarse plane c_k, mesh k), two points per thread.  The Boolean-sum
// correction of the plane is two rank-N_c products, Sp R_ck + B_ck Sp^T, with A, B and R as in
// k_crosspoints3; instead of reading them from a launch of their own, the block forms the
// discrepancies it needs -- A at its 8 rows i_b and at the N_c coarse rows for every c_a, B at its
// 64 values of i_a for every c_b -- and the R of its rows from them, in LDS, with the arithmetic
// of k_crosspoints3 (the same values bit for bit).  Their loads, the tile's own values and the
// cross-point candidates are all issued before this step's choice is read.  Cross points take the
// value of crosspoint_value as in k_merge.
template <int NC>
__global__ __launch_bounds__(256) void k_merge3(Geo g, SkelArgs a) {
    // the stopping flag is read with the first loads and tested once they have arrived
    const int gv = gate_value(a.gate);
    constexpr int RB = 8;
    constexpr int NA = NC * (RB + NC);  // A: [c_a][the 8 rows, then the N_c coarse rows]
    constexpr int ND = NA + 64 * NC;    // then B: [i_a][c_b]
    constexpr int DPT = (ND + 255) / 256;
    __shared__ double sSa[64 * NC], sSb[RB][NC], sA[NC][RB + NC], sB[64][NC + 1], sR[NC][RB];
    const int Nf = g.Nf, n = g.n;
    const int k = blockIdx.z, ck = blockIdx.y;
    const int xtn = (Nf + 63) / 64;
    const int ia0 = (blockIdx.x % xtn) * 64, ib0 = (blockIdx.x / xtn) * RB;
    const unsigned mk = 1u << k;
    // per-mesh pointers chosen by selects (a dynamic index into the argument struct would be
    // copied to scratch memory)
    double *sk = (k == 0) ? a.skel[0] : (k == 1) ? a.skel[1] : a.skel[2];
    const double *__restrict__ Sp = a.Sp;
    const double *__restrict__ X = (k == 0) ? a.res[1] : (k == 1) ? a.res[2] : a.res[4];
    const int t = threadIdx.x, tx = t & 63, ty = t >> 6;
    const int nrow = min(64, Nf - ia0);  // i_a rows of this tile
    const bool err = a.mode == 1;
    // the spline rows of the tile into registers first (stored to LDS after the choice, so that
    // every load of the block, the choice's included, is in flight at once; a load followed by its
    // store in one loop would wait for each load in turn)
    constexpr int SPT = (64 * NC + 255) / 256;
    double spa[SPT];
#pragma unroll
    for (int j = 0; j < SPT; ++j) {
        const int q = t + 256 * j;
        spa[j] = Sp[(long long)ia0 * NC + (q < nrow * NC ? q : 0)];
    }
    const bool sbt = t < NC * RB;
    const double spb = Sp[sbt ? (long long)min(ib0 + t % RB, Nf - 1) * NC + t / RB : 0];
    // discrepancy d of the block at (u, v) of plane c_k: d < NA is A at c_a = d / (RB + NC), column
    // w = d % (RB + NC) (row i_b = ib0 + w for w < RB, else coarse row w - RB); else B at
    // i_a = ia0 + (d - NA) / N_c, c_b = (d - NA) % N_c (rows past N_f - 1 clamped, never used)
    auto dpoint = [&](int d, int &u, int &v) {
        if (d < NA) {
            const int ca = d / (RB + NC), w = d - ca * (RB + NC);
            u = (ca + 1) * n - 1;
            v = (w < RB) ? min(ib0 + w, Nf - 1) : (w - RB + 1) * n - 1;
        } else {
            const int e = d - NA, ia = e / NC, cb = e - ia * NC;
            u = min(ia0 + ia, Nf - 1);
            v = (cb + 1) * n - 1;
        }
    };
    double dx[DPT];
    XCand dc[DPT];
#pragma unroll
    for (int j = 0; j < DPT; ++j) {
        // a lane past the block's last discrepancy loads that one's operands (discarded later)
        const int d = min(t + 256 * j, ND - 1);
        int u, v;
        dpoint(d, u, v);
        dx[j] = X[(long long)u + (long long)Nf * (v + (long long)Nf * ck)];
        dc[j] = XCand{0.0, 0.0, 0.0};
        if (err) {  // launch-uniform
            const Pt p = mesh_pt(k, 3, u, v, (ck + 1) * n - 1);
            dc[j] = cross_candidates(a, g, p, coarse_set(p, 3, n));
        }
    }
    const int ia = ia0 + tx;
    const int iac = min(ia, Nf - 1);
    auto ld = [&](int j) -> double {
        const int ibc = min(ib0 + j, Nf - 1);
        return X[(long long)iac + (long long)Nf * ibc + (long long)Nf * Nf * ck];
    };
    const double xa = ld(ty), xb = ld(ty + 4);
    // cross points of the error phase among the tile's own points: the candidates
    XCand cand[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int ib = min(ib0 + ty + 4 * h, Nf - 1);
        const Pt p = mesh_pt(k, 3, iac, ib, (ck + 1) * n - 1);
        const unsigned S = coarse_set(p, 3, n);
        cand[h] = XCand{0.0, 0.0, 0.0};
        if (err) cand[h] = cross_candidates(a, g, p, S);  // launch-uniform; used at cross points only
    }
    const XChoice ch = load_choice(a, g);
    if (!flag_clear(gv)) return;  // block-uniform
#pragma unroll
    for (int j = 0; j < SPT; ++j) {
        const int q = t + 256 * j;
        if (q < nrow * NC) sSa[q] = spa[j];
    }
    if (sbt) sSb[t % RB][t / RB] = spb;
    const double scale_k = (a.mode == 0) ? 1.0 : inv_of(ch, k);
    // the discrepancies (cross-point value minus the scaled solution of M_k) into LDS
#pragma unroll
    for (int j = 0; j < DPT; ++j) {
        const int d = t + 256 * j;
        if (d < ND) {
            int u, v;
            dpoint(d, u, v);
            const Pt p = mesh_pt(k, 3, u, v, (ck + 1) * n - 1);
            const unsigned S = coarse_set(p, 3, n);
            const double uh = err ? cross_pick(ch, S, dc[j]) : crosspoint_value(a, g, p, S, ch);
            const double dv = uh - scale_k * dx[j];
            if (d < NA) {
                const int ca = d / (RB + NC);
                sA[ca][d - ca * (RB + NC)] = dv;
            } else {
                const int e = d - NA, ib = e / NC;
                sB[ib][e - ib * NC] = dv;
            }
        }
    }
    __syncthreads();
    // R of the tile's rows: 0 on a coarse row, else A minus the spline of the row's coarse values
    if (t < NC * RB) {
        const int ca = t / RB, j = t % RB;
        double v = 0.0;
        if (!on_coarse(ib0 + j, n)) {
            v = sA[ca][j];
            for (int cb = 0; cb < NC; ++cb) v -= sSb[j][cb] * sA[ca][RB + cb];
        }
        sR[ca][j] = v;
    }
    __syncthreads();
    if (ia >= Nf) return;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int j = ty + 4 * h, ib = ib0 + j;
        const double x = h ? xb : xa;
        if (ib >= Nf) break;
        const Pt p = mesh_pt(k, 3, ia, ib, (ck + 1) * n - 1);
        const unsigned S = coarse_set(p, 3, n);
        double v;
        if (S != mk) {
            v = err ? cross_pick(ch, S, cand[h]) : crosspoint_value(a, g, p, S, ch);
        } else {
            double c1 = 0.0, c2 = 0.0;
#pragma unroll
            for (int c = 0; c < NC; ++c) c1 += sSa[tx * NC + c] * sR[c][j];
#pragma unroll
            for (int c = 0; c < NC; ++c) c2 += sSb[j][c] * sB[tx][c];
            v = scale_k * x + (c1 + c2);
        }
        sk[(long long)ia + (long long)Nf * ib + (long long)Nf * Nf * ck] = v;
    }
}

// k_merge3 forms its own discrepancies for these coarse sizes
bool merge_forms_discrepancies(const Plan &p) { return p.d == 3 && (p.Nc == 7 || p.Nc == 15 || p.Nc == 31); }

static SkelArgs skel_args(const Plan &p, int mode, const double *const *res) {
    SkelArgs a;
    for (unsigned s = 0; s < kMaxMeshes; ++s) {
        a.res[s] = (s < (1u << p.d)) ? res[s] : nullptr;
        a.mesh[s] = (s < (1u << p.d)) ? p.mesh[s] : MeshDesc();
    }
    for (int k = 0; k < kMaxD; ++k) {
        a.lines[k] = (k < p.d) ? p.ws.lines[k] : nullptr;
        a.skel[k] = (k < p.d) ? merged_buf(p, k) : nullptr;
    }
    a.state = p.ws.state;
    a.gate = p.gate;
    a.Sp = p.dSp;
    a.scal = p.ws.scal;
    a.mode = mode;
    a.norm_partials = (mode == 1) ? p.norm_partials : nullptr;
    a.norm_nblk = p.norm_nblk;
    return a;
}

void launch_crosspoints(const Plan &p, int mode, const double *const *res, hipStream_t st) {
    if (p.d == 4) {
        launch_crosspoints4(p, mode, res, st);
        return;
    }
    if (merge_forms_discrepancies(p)) return;
    SkelArgs a = skel_args(p, mode, res);
    if (p.d == 3) {
        const int nrow = std::min(p.Nc * p.Nc, 512);
        long long nb = ((long long)p.Nc * p.Nc * p.Nf + 255) / 256;
        if (nb > 1024) nb = 1024;
        ASDSM_LAUNCH(k_crosspoints3, dim3((unsigned)(nrow + nb), 3, 1), dim3(256), 0, st, p.geo, a, nrow);
        return;
    }
    const long long total = (long long)p.Nc * p.Nc;
    long long blocks = (total + 255) / 256;
    if (blocks > 1024) blocks = 1024;
    ASDSM_LAUNCH(k_crosspoints, dim3((unsigned)blocks, p.d, 1), dim3(256), 0, st, p.geo, a);
}

void launch_merge(const Plan &p, int mode, const double *const *res, hipStream_t st) {
    if (p.d == 4) {
        launch_merge4(p, mode, res, st);
        return;
    }
    SkelArgs a = skel_args(p, mode, res);
    if (merge_forms_discrepancies(p)) {
        const unsigned tiles = (unsigned)(((p.Nf + 63) / 64) * ((p.Nf + 7) / 8));
        const dim3 grid(tiles, (unsigned)p.Nc, 3);
        if (p.Nc == 7)
            ASDSM_LAUNCH((k_merge3<7>), grid, dim3(256), 0, st, p.geo, a);
        else if (p.Nc == 15)
            ASDSM_LAUNCH((k_merge3<15>), grid, dim3(256), 0, st, p.geo, a);
        else
            ASDSM_LAUNCH((k_merge3<31>), grid, dim3(256), 0, st, p.geo, a);
        return;
    }
    long long blocks = (p.mesh[1].size + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    ASDSM_LAUNCH(k_merge, dim3((unsigned)blocks, p.d, 1), dim3(256), 0, st, p.geo, a);
}

// ---------------------------------------------------------------------------------------------
// Filler (Algorithm 3): one workgroup per hole tile.  The tile of hole (t_1..t_d) covers the fine
// indices n t_j .. n t_j + n - 1 on every axis: the (n-1)^d hole plus the skeleton planes above it.
// Hole right-hand side: (b_ff in the initial guess, 0 in the error phase) minus the stencil
// coupling to the merged skeleton values on the hole faces, i.e. P_h b - P_h A u~.  All holes share
// one matrix (a diagonal block of A_ff, Remark 2.5): its d-1 transform axes are diagonalised with
// LDS-resident (n-1) x (n-1) matrices and the remaining axis is eliminated line by line.
// ---------------------------------------------------------------------------------------------
struct FillArgs {
    const double *skel[kMaxD];
    MeshDesc mk[kMaxD];
    const double *W[kMaxD];
    const double *V[kMaxD];
    const double *mu[kMaxD];
    int line_axis;
    int ntr;
    int tr[kMaxD];
    const double *bff;
    double *out;
    double *adj[kMaxD];  // adjacent-layer mode (k_filler_mfma3): the layers next to each coarse plane
    int adj_only;        // 1: write only those layers (skeleton-sparse refinement), not the fine tile
    const int *gate;
    // non-null (k_filler, d = 3): the hole operator's inverse, column by column ((n-1)^3 squared),
    // applied densely instead of the transforms and the line elimination
    const double *hinv;
    // hole line solve in global memory (k_filler, d = 3): phase 1 stores each hole's right-hand
    // side at hbuf (hole-major, the line axis slowest, the lower other axis fastest) and ends;
    // phase 2 takes the hole values from there; 0: the solve in LDS
    int hphase;
    double *hbuf;
};

template <int D, int NH>
__global__ __launch_bounds__(256) void k_filler(Geo g, FillArgs a) {
    if (a.gate && *a.gate) return;
    extern __shared__ double lds[];
    // NH > 0: hole edge length known at compile time (constant-divisor index arithmetic)
    const int nh = (NH > 0) ? NH : g.n - 1;
    const int n = nh + 1, Nf = g.Nf, Nc = g.Nc;
    int npts = 1, st[kMaxD] = {1, 1, 1, 1};
    for (int j = 0; j < D; ++j) {
        st[j] = npts;
        npts *= nh;
    }
    double *bufA = lds;
    double *bufB = lds + npts;
    double *mat = lds + 2 * npts;  // per transform axis: W (nh*nh), V (nh*nh), mu (nh)
    const int tid = threadIdx.x;
    for (int q = 0; q < a.ntr; ++q) {
        const int j = a.tr[q];
        double *Wq = mat + q * (2 * nh * nh + nh);
        for (int e = tid; e < nh * nh; e += 256) {
            Wq[e] = a.W[j][e];
            Wq[nh * nh + e] = a.V[j][e];
        }
        for (int e = tid; e < nh; e += 256) Wq[2 * nh * nh + e] = a.mu[j][e];
    }
    int tt[kMaxD] = {0, 0, 0, 0};
    {
        int rem = blockIdx.x;
        for (int j = 0; j < D; ++j) {
            tt[j] = rem % (Nc + 1);
            rem /= (Nc + 1);
        }
    }
    // offset of hole point o in hbuf (phases 1 and 2, D = 3)
    auto hoff = [&](int o) -> long long {
        const int l0 = o % nh, l1 = (o / nh) % nh, l2 = o / (nh * nh);
        const int la = a.line_axis;
        const int ll = (la == 0) ? l0 : (la == 1) ? l1 : l2;
        const int c0 = (la == 0) ? l1 : l0, c1 = (la == 2) ? l1 : l2;
        return (long long)blockIdx.x * npts + (long long)ll * (nh * nh) + c0 + nh * c1;
    };
    // 1) hole right-hand side (phase 2 reads the solved holes from hbuf where it writes the tile)
    for (int o = tid; o < npts && a.hphase != 2; o += 256) {
        int l[kMaxD] = {0, 0, 0, 0}, i[kMaxD] = {0, 0, 0, 0};
        int rem = o;
        for (int j = 0; j < D; ++j) {
            l[j] = rem % nh;
            rem /= nh;
            i[j] = n * tt[j] + l[j];
        }
        long long f = i[0] + (long long)Nf * (i[1] + (long long)Nf * (i[2] + (long long)Nf * i[3]));
        double v = a.bff ? a.bff[f] : 0.0;
        for (int j = 0; j < D; ++j) {
            if (l[j] == 0 && tt[j] > 0) {
                int q[kMaxD] = {i[0], i[1], i[2], i[3]};
                q[j] -= 1;
                v -= g.fine[j].a * a.skel[j][canon_offset(a.mk[j], q, n)];
            }
            if (l[j] == nh - 1 && tt[j] < Nc) {
                int q[kMaxD] = {i[0], i[1], i[2], i[3]};
                q[j] += 1;
                v -= g.fine[j].c * a.skel[j][canon_offset(a.mk[j], q, n)];
            }
        }
        if (D == 3 && a.hphase == 1) a.hbuf[hoff(o)] = v;
        else bufA[o] = v;
    }
    if (a.hphase == 1) return;
    __syncthreads();
    double *cur = bufA, *oth = bufB;
    if (a.hinv) {
        // 2') x = A_hole^-1 f, the inverse read column by column (consecutive threads read
        // consecutive rows of a column)
        for (int o = tid; o < npts; o += 256) {
            double acc = 0.0;
            for (int q = 0; q < npts; ++q) acc += a.hinv[(size_t)q * npts + o] * cur[q];
            oth[o] = acc;
        }
        __syncthreads();
        cur = bufB;
        oth = bufA;
    }
    // 2) forward transforms
    for (int q = 0; q < a.ntr; ++q) {
        const int j = a.tr[q];
        const double *Wq = mat + q * (2 * nh * nh + nh);
        for (int o = tid; o < npts; o += 256) {
            const int sj = axis_sel(st, j);
            const int m = (o / sj) % nh;
            const int base = o - m * sj;
            double acc = 0.0;
            for (int l = 0; l < nh; ++l) acc += Wq[m * nh + l] * cur[base + l * sj];
            oth[o] = acc;
        }
        __syncthreads();
        double *t = cur;
        cur = oth;
        oth = t;
    }
    // 3) line elimination along the line axis, one thread per line
    if (!a.hinv && a.hphase == 0) {
        const int L = a.line_axis;
        const int nlines = npts / nh;
        const Tri t = g.fine[L];
        for (int ln = tid; ln < nlines; ln += 256) {
            // coordinates of the other axes
            int rem = ln, base = 0;
            double sigma = 0.0;
            for (int j = 0; j < D; ++j) {
                if (j == L) continue;
                const int c = rem % nh;
                rem /= nh;
                base += c * st[j];
                for (int q = 0; q < a.ntr; ++q)
                    if (a.tr[q] == j) sigma += mat[q * (2 * nh * nh + nh) + 2 * nh * nh + c];
            }
            const int sL = axis_sel(st, L);
            const double diag = t.b + sigma;
            double den = diag;
            double cp = t.c / den;
            double dp = cur[base] / den;
            oth[base] = cp;
            cur[base] = dp;
            for (int c = 1; c < nh; ++c) {
                den = diag - t.a * cp;
                dp = (cur[base + c * sL] - t.a * dp) / den;
                cp = t.c / den;
                oth[base + c * sL] = cp;
                cur[base + c * sL] = dp;
            }
            double x = dp;
            for (int c = nh - 2; c >= 0; --c) {
                x = cur[base + c * sL] - oth[base + c * sL] * x;
                cur[base + c * sL] = x;
            }
        }
        __syncthreads();
    }
    // 4) backward transforms
    for (int q = a.ntr - 1; q >= 0; --q) {
        const int j = a.tr[q];
        const double *Vq = mat + q * (2 * nh * nh + nh) + nh * nh;
        for (int o = tid; o < npts; o += 256) {
            const int sj = axis_sel(st, j);
            const int ii = (o / sj) % nh;
            const int base = o - ii * sj;
            double acc = 0.0;
            for (int m = 0; m < nh; ++m) acc += Vq[ii * nh + m] * cur[base + m * sj];
            oth[o] = acc;
        }
        __syncthreads();
        double *t = cur;
        cur = oth;
        oth = t;
    }
    // 5) write the whole tile (hole values and the skeleton planes above it), x_1 fastest
    int ntile = 1;
    for (int j = 0; j < D; ++j) ntile *= n;
    for (int o = tid; o < ntile; o += 256) {
        int l[kMaxD] = {0, 0, 0, 0}, i[kMaxD] = {0, 0, 0, 0};
        int rem = o;
        bool inside = true, hole = true;
        for (int j = 0; j < D; ++j) {
            l[j] = rem % n;
            rem /= n;
            i[j] = n * tt[j] + l[j];
            if (i[j] >= Nf) inside = false;
            if (l[j] == n - 1) hole = false;
        }
        if (!inside) continue;
        double v;
        if (hole) {
            int lo = 0;
            for (int j = 0; j < D; ++j) lo += l[j] * st[j];
            v = (D == 3 && a.hphase == 2) ? a.hbuf[hoff(lo)] : cur[lo];
        } else {
            int j = 0;
            while (l[j] != n - 1) ++j;
            v = a.skel[j][canon_offset(a.mk[j], i, n)];
        }
        if (D == 3 && a.adj_only) {
            // adjacent-layer mode (see k_filler_mfma3): the first and last hole layer along each axis
            const long long lay = (long long)Nc * Nf * Nf;
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                const int ga = (j == 0) ? i[1] : i[0], gb = (j == 2) ? i[1] : i[2];
                const int lj = (j == 0) ? l[0] : (j == 1) ? l[1] : l[2];
                const int tj = (j == 0) ? tt[0] : (j == 1) ? tt[1] : tt[2];
                double *dst = (j == 0) ? a.adj[0] : (j == 1) ? a.adj[1] : a.adj[2];
                const long long inplane = ga + (long long)Nf * gb;
                if (lj == 0 && tj > 0) dst[lay + inplane + (long long)Nf * Nf * (tj - 1)] = v;
                if (lj == nh - 1 && tj < Nc) dst[inplane + (long long)Nf * Nf * tj] = v;
            }
            continue;
        }
        const long long f = i[0] + (long long)Nf * (i[1] + (long long)Nf * (i[2] + (long long)Nf * i[3]));
        a.out[f] = v;
    }
}

// ---------------------------------------------------------------------------------------------
// Filler for d = 3, 4 with small holes (n - 1 = NH in {1, 3, 7}), the same hole solve as k_filler
// with every size known at compile time.  The hole sits in one LDS buffer (no second buffer):
// each transform and the line elimination go line by line in place -- a lane loads a line of NH
// values into registers, maps it and stores it back -- so twice as many holes fit on a CU.  The
// global loads of the right-hand side and of the skeleton values written with the tile are issued
// together (fully unrolled loops of constant length) instead of one wait per loop trip.
// ---------------------------------------------------------------------------------------------
constexpr int ipow_c(int b, int e) { return e == 0 ? 1 : b * ipow_c(b, e - 1); }

// Offset in the canonical layout of M_{j} (fine axes in increasing order, then coarse axis j) of
// the point with fine coordinates i[] off axis j and coarse index cj on axis j.
template <int D, int J>
__device__ __forceinline__ long long skel_offset(const int (&i)[D], int cj, int Nf) {
    long long off = cj, mul = 1;
    for (int q = 0; q < D - 1; ++q) mul *= Nf;
    off *= mul;
    long long s = 1;
#pragma unroll
    for (int q = 0; q < D; ++q) {
        if (q == J) continue;
        off += (long long)i[q] * s;
        s *= Nf;
    }
    return off;
}

// Transform of every line along axis J of the hole buffer by the NH x NH matrix M (out, in).  A
// lane holds all its lines at once (NR of them), so each matrix entry is read once per lane; the
// entries are read at wave-uniform addresses from global memory (scalar loads into SGPR operands),
// which leaves the LDS bandwidth to the hole values.
template <int D, int NH, int J>
__device__ __forceinline__ void hole_lines_map(double *buf, const double *__restrict__ M) {
    constexpr int N = ipow_c(NH, D), NL = N / NH, SJ = ipow_c(NH, J), NR = (NL + 255) / 256;
    // read-only for the kernel's lifetime: the constant address space makes the loads scalar
    const __attribute__((address_space(4))) double *Mc = (const __attribute__((address_space(4))) double *)M;
    double x[NR][NH];
    int base[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        const int ln = min((int)threadIdx.x + 256 * r, NL - 1);
        base[r] = ln % SJ + (ln / SJ) * SJ * NH;
#pragma unroll
        for (int l = 0; l < NH; ++l) x[r][l] = buf[base[r] + l * SJ];
    }
    __syncthreads();  // lanes whose second line is clamped read a line another lane rewrites
#pragma unroll
    for (int m = 0; m < NH; ++m) {
        double acc[NR];
#pragma unroll
        for (int r = 0; r < NR; ++r) acc[r] = 0.0;
#pragma unroll
        for (int l = 0; l < NH; ++l) {
            const double w = Mc[m * NH + l];
#pragma unroll
            for (int r = 0; r < NR; ++r) acc[r] += w * x[r][l];
        }
#pragma unroll
        for (int r = 0; r < NR; ++r)
            if ((int)threadIdx.x + 256 * r < NL) buf[base[r] + m * SJ] = acc[r];
    }
}

// Tridiagonal solve of every line along axis J (the line axis) with the diagonal shifted by the
// eigenvalues of the transformed axes at the line's modes.
template <int D, int NH, int J>
__device__ __forceinline__ void hole_lines_solve(double *buf, const FillArgs &a, Tri t) {
    constexpr int N = ipow_c(NH, D), NL = N / NH, SJ = ipow_c(NH, J), NR = (NL + 255) / 256;
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        const int ln = (int)threadIdx.x + 256 * r;
        if (ln >= NL) continue;
        const int base = ln % SJ + (ln / SJ) * SJ * NH;
        double sigma = 0.0;
#pragma unroll
        for (int q = 0; q < D; ++q) {
            if (q == J) continue;
            sigma += a.mu[q][(base / ipow_c(NH, q)) % NH];
        }
        const double diag = t.b + sigma;
        double x[NH], cp[NH];
#pragma unroll
        for (int l = 0; l < NH; ++l) x[l] = buf[base + l * SJ];
        double inv = 1.0 / diag;
        cp[0] = t.c * inv;
        x[0] *= inv;
#pragma unroll
        for (int c = 1; c < NH; ++c) {
            inv = 1.0 / (diag - t.a * cp[c - 1]);
            cp[c] = t.c * inv;
            x[c] = (x[c] - t.a * x[c - 1]) * inv;
        }
#pragma unroll
        for (int c = NH - 2; c >= 0; --c) x[c] -= cp[c] * x[c + 1];
#pragma unroll
        for (int l = 0; l < NH; ++l) buf[base + l * SJ] = x[l];
    }
}

template <int D, int NH>
__device__ __forceinline__ void hole_map_axis(double *buf, const double *__restrict__ M, int j) {
    switch (j) {
        case 0: hole_lines_map<D, NH, 0>(buf, M); break;
        case 1: hole_lines_map<D, NH, 1>(buf, M); break;
        case 2: hole_lines_map<D, NH, 2>(buf, M); break;
        default: if constexpr (D == 4) hole_lines_map<D, NH, 3>(buf, M); break;
    }
}

template <int D, int NH>
__global__ __launch_bounds__(256) void k_filler_lines(Geo g, FillArgs a) {
    if (a.gate && *a.gate) return;
    constexpr int n = NH + 1, N = ipow_c(NH, D), NT = ipow_c(n, D);
    constexpr int K1 = (N + 255) / 256, K5 = (NT + 255) / 256;
    __shared__ double buf[N];
    const int Nf = g.Nf, Nc = g.Nc, tid = threadIdx.x;
    // the matrices of axis j, through selects (a dynamic index into the argument struct would be
    // copied to scratch)
    auto pick = [&](const double *const *m, int j) -> const double * {
        return j == 0 ? m[0] : (j == 1 ? m[1] : (j == 2 ? m[2] : m[D - 1]));
    };
    int tt[D];
    {
        int rem = blockIdx.x;
#pragma unroll
        for (int j = 0; j < D; ++j) {
            tt[j] = rem % (Nc + 1);
            rem /= (Nc + 1);
        }
    }
    long long fs[D];
    fs[0] = 1;
#pragma unroll
    for (int j = 1; j < D; ++j) fs[j] = fs[j - 1] * Nf;
    // 1) hole right-hand side: b_ff (initial guess) minus the coupling to the skeleton faces, in
    // batches of KA points per lane
    constexpr int KA = K1 < 5 ? K1 : 5;
#pragma unroll 1
    for (int kc = 0; kc < K1; kc += KA) {
        double v[KA];
#pragma unroll
        for (int k = 0; k < KA; ++k) {
            const int o = tid + 256 * (kc + k);
            v[k] = 0.0;
            if (o < N) {
                int i[D];
                long long f = 0;
                int rem = o;
#pragma unroll
                for (int j = 0; j < D; ++j) {
                    i[j] = n * tt[j] + rem % NH;
                    rem /= NH;
                    f += i[j] * fs[j];
                }
                double s = a.bff ? a.bff[f] : 0.0;
#pragma unroll
                for (int j = 0; j < D; ++j) {
                    const int l = i[j] - n * tt[j];
                    const double *sk = a.skel[j];
                    long long off = -1;
                    double cf = 0.0;
                    if (l == 0 && tt[j] > 0) {
                        cf = g.fine[j].a;
                        off = (j == 0) ? skel_offset<D, 0>(i, tt[j] - 1, Nf)
                            : (j == 1) ? skel_offset<D, 1>(i, tt[j] - 1, Nf)
                            : (j == 2) ? skel_offset<D, 2>(i, tt[j] - 1, Nf)
                                       : skel_offset<D, D - 1>(i, tt[j] - 1, Nf);
                    }
                    if (l == NH - 1 && tt[j] < Nc) {
                        // NH = 1: both faces of the same point; the upper one is added below
                        if (off >= 0) s -= cf * sk[off];
                        cf = g.fine[j].c;
                        off = (j == 0) ? skel_offset<D, 0>(i, tt[j], Nf)
                            : (j == 1) ? skel_offset<D, 1>(i, tt[j], Nf)
                            : (j == 2) ? skel_offset<D, 2>(i, tt[j], Nf)
                                       : skel_offset<D, D - 1>(i, tt[j], Nf);
                    }
                    if (off >= 0) s -= cf * sk[off];
                }
                v[k] = s;
            }
        }
#pragma unroll
        for (int k = 0; k < KA; ++k)
            if (tid + 256 * (kc + k) < N) buf[tid + 256 * (kc + k)] = v[k];
    }
    __syncthreads();
    // 2) forward transforms, 3) line elimination, 4) backward transforms
    for (int q = 0; q < a.ntr; ++q) {
        hole_map_axis<D, NH>(buf, pick(a.W, a.tr[q]), a.tr[q]);
        __syncthreads();
    }
    switch (a.line_axis) {
        case 0: hole_lines_solve<D, NH, 0>(buf, a, g.fine[0]); break;
        case 1: hole_lines_solve<D, NH, 1>(buf, a, g.fine[1]); break;
        case 2: hole_lines_solve<D, NH, 2>(buf, a, g.fine[2]); break;
        default: if constexpr (D == 4) hole_lines_solve<D, NH, 3>(buf, a, g.fine[3]); break;
    }
    __syncthreads();
    for (int q = a.ntr - 1; q >= 0; --q) {
        hole_map_axis<D, NH>(buf, pick(a.V, a.tr[q]), a.tr[q]);
        __syncthreads();
    }
    // 5) the whole tile: hole values and the skeleton planes above it (merged values), in batches
    // of KB points per lane whose loads are in flight together
    constexpr int KB = K5 < 8 ? K5 : 8;
#pragma unroll 1
    for (int kc = 0; kc < K5; kc += KB) {
        double w[KB];
        long long fo[KB];
#pragma unroll
        for (int k = 0; k < KB; ++k) {
            const int o = tid + 256 * (kc + k);
            w[k] = 0.0;
            fo[k] = -1;
            if (o < NT) {
                int i[D], l[D];
                bool inside = true, hole = true;
                long long f = 0;
                int lo = 0, rem = o;
#pragma unroll
                for (int j = 0; j < D; ++j) {
                    l[j] = rem % n;
                    rem /= n;
                    i[j] = n * tt[j] + l[j];
                    inside = inside && i[j] < Nf;
                    hole = hole && l[j] < NH;
                    f += i[j] * fs[j];
                    lo += l[j] * ipow_c(NH, j);
                }
                if (inside) {
                    fo[k] = f;
                    if (hole) {
                        w[k] = buf[lo];
                    } else {
                        // the first axis whose coordinate lies on a coarse plane
                        if (l[0] == NH) w[k] = a.skel[0][skel_offset<D, 0>(i, tt[0], Nf)];
                        else if (l[1] == NH) w[k] = a.skel[1][skel_offset<D, 1>(i, tt[1], Nf)];
                        else if (D == 3 || l[2] == NH) w[k] = a.skel[2][skel_offset<D, 2>(i, tt[2], Nf)];
                        else w[k] = a.skel[D - 1][skel_offset<D, D - 1>(i, tt[D - 1], Nf)];
                    }
                }
            }
        }
#pragma unroll
        for (int k = 0; k < KB; ++k)
            if (fo[k] >= 0) a.out[fo[k]] = w[k];
    }
}

// ---------------------------------------------------------------------------------------------
// Filler for d = 3 with 15^3 holes (n = 16) on MFMA: line axis L (eliminated by Thomas), the two
// other axes j0 < j1 diagonalised.  The hole is padded to 16^3 in one LDS buffer with strides
// (1, 17, 289): for every axis the 16 rows of an MFMA operand fragment and the 16 columns of a
// result fragment fall in distinct banks.  Wave w owns the slabs l_L = w, w + 4, w + 8 and w + 12
// (slab 15 is padding that no step reads).  A transform along a diagonalised axis j is, per slab,
// the GEMM of its 16 lines along j (rows: the third coordinate) by the 16 x 16 matrix W_j^T (pad
// row and column zero), 4 v_mfma_f64_16x16x4f64; it never leaves the slab, so the two transforms
// of each side run without a workgroup barrier.
//
// Global traffic per hole is the face values, the four 15 x 15 transform matrices (read once per
// block into LDS) and two eigenvalues per line; the line factors are formed in registers while
// the face values are in flight, and the first barrier orders LDS only.
// ---------------------------------------------------------------------------------------------
constexpr int kFS1 = 17, kFS2 = 289, kFBuf = 16 * kFS2;
constexpr int kFMat = 16 * 17;  // one transform matrix in LDS: T[m][k] at m * 17 + k, zero beyond 15

__host__ __device__ constexpr int fstride(int j) { return j == 0 ? 1 : (j == 1 ? kFS1 : kFS2); }

// In-slab transform along axis J of the slabs of one wave (L the slab axis, P the third axis):
// A rows l_P, K and the result columns along J; B[k][m] = T[m][k] from the LDS copy of T.  The
// four slabs' accumulator chains are interleaved.  The slabs are private to the wave, whose LDS
// instructions execute in order; the wavefront-scope fences keep the compiler from moving a lane's
// writes above another lane's reads of the same slab.
template <int J, int L>
__device__ __forceinline__ void slab_transform(double *buf, const double *T, int lane, int wave) {
    constexpr int P = 3 - J - L;
    constexpr int Sp = fstride(P), Ss = fstride(L), Sj = fstride(J);
    double b[4], x[4][4];
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) b[ks] = T[(lane & 15) * 17 + 4 * ks + (lane >> 4)];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const int s = wave + 4 * t;
#pragma unroll
        for (int ks = 0; ks < 4; ++ks)
            x[t][ks] = (s < 15) ? buf[(lane & 15) * Sp + s * Ss + (4 * ks + (lane >> 4)) * Sj] : 0.0;
    }
    double4_t acc[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) acc[t] = double4_t{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int ks = 0; ks < 4; ++ks)
#pragma unroll
        for (int t = 0; t < 4; ++t) acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(x[t][ks], b[ks], acc[t], 0, 0, 0);
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const int s = wave + 4 * t;
        if (s < 15) {
#pragma unroll
            for (int v = 0; v < 4; ++v) buf[((lane >> 4) + 4 * v) * Sp + s * Ss + (lane & 15) * Sj] = acc[t][v];
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
}

// Face values in LDS: face f = 2 j + side (side 0 below the hole, on coarse plane t_j - 1; side 1
// above it, on plane t_j), entry (la, lb) at f * 256 + la + 16 lb, la and lb the hole-local
// coordinates of the two other axes in increasing order; zero where the face is the domain boundary.
__device__ __forceinline__ int face_at(int f, int la, int lb) { return f * 256 + la + 16 * lb; }

// The hole's right-hand side at (l0, l1, l2) < 15 from v = b_ff there (or 0): minus, axis by axis,
// the coupling to the face value below (coefficient a_j) or above (c_j) a point of the first or
// last layer.
__device__ __forceinline__ double hole_rhs(const Geo &g, const double *fa, int l0, int l1, int l2,
                                           double v) {
    constexpr int last = 14;
    if (l0 == 0) v -= g.fine[0].a * fa[face_at(0, l1, l2)];
    else if (l0 == last) v -= g.fine[0].c * fa[face_at(1, l1, l2)];
    if (l1 == 0) v -= g.fine[1].a * fa[face_at(2, l0, l2)];
    else if (l1 == last) v -= g.fine[1].c * fa[face_at(3, l0, l2)];
    if (l2 == 0) v -= g.fine[2].a * fa[face_at(4, l0, l1)];
    else if (l2 == last) v -= g.fine[2].c * fa[face_at(5, l0, l1)];
    return v;
}

// LAYERS: adjacent-layer mode (skeleton-sparse refinement; the hole's right-hand side is zero).
template <int L, bool LAYERS>
__global__ __launch_bounds__(256, 2) void k_filler_mfma3(Geo g, FillArgs a) {
    // the stopping flag is read with the other loads and tested after the first barrier
    const int gv = gate_value(a.gate);
    __shared__ double buf[kFBuf];
    __shared__ double fa[6 * 256];
    __shared__ double mats[4 * kFMat];  // W_j0, W_j1, V_j1, V_j0
    constexpr int nh = 15, n = 16;
    constexpr int j0 = (L == 0) ? 1 : 0, j1 = (L == 2) ? 1 : 2;
    const int Nf = g.Nf, Nc = g.Nc;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    int tt[3];
    {
        int rem = blockIdx.x;
        for (int j = 0; j < 3; ++j) {
            tt[j] = rem % (Nc + 1);
            rem /= (Nc + 1);
        }
    }
    // Face bases: the merged skeleton values next to the hole lie on coarse planes of the anisotropic
    // meshes; in M_j's canonical layout (fine axes a < b, coarse axis j) the point with hole-local
    // coordinates (l_a, l_b) on plane c is at 16 t_a + l_a + Nf (16 t_b + l_b) + Nf^2 c.
    int lo_base[3], hi_base[3];
    const int Nf2 = Nf * Nf;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        const int fa_ = (j == 0) ? 1 : 0, fb_ = (j == 2) ? 1 : 2;
        const int base = n * tt[fa_] + Nf * (n * tt[fb_]);
        lo_base[j] = (tt[j] > 0) ? base + Nf2 * (tt[j] - 1) : -1;
        hi_base[j] = (tt[j] < Nc) ? base + Nf2 * tt[j] : -1;
    }
    const int f0 = n * tt[0] + Nf * (n * tt[1]) + Nf2 * (n * tt[2]);  // fine index of the tile origin
    // 1) the loads.  Every lane issues every load (a lane without a value reads an in-bounds
    // stand-in and discards it), so the compiler waits for exactly the ones needed next.  First the
    // two eigenvalues of this thread's line (mode pair m_j0 = tid % 15, m_j1 = tid / 15), then the
    // face values around the tile (16 x 16 per face, the last row and column being points on two
    // planes, used only by the output), b_ff at this thread's points (x_1 fastest), and the
    // transform matrices.
    const bool thomas = tid < nh * nh;
    const int m0 = thomas ? tid % nh : 0, m1 = thomas ? tid / nh : 0;
    const double mu0 = a.mu[j0][m0], mu1 = a.mu[j1][m1];
    const int la = tid & 15, lb = tid >> 4;
    // (the raw values; the stand-ins are zeroed where the values are stored, below the line factors)
    double fvals[6];
    bool fin[6];
#pragma unroll
    for (int f = 0; f < 6; ++f) {
        const int j = f >> 1, fa_ = (j == 0) ? 1 : 0, fb_ = (j == 2) ? 1 : 2;
        const int bse = (f & 1) ? hi_base[j] : lo_base[j];
        fin[f] = bse >= 0 && n * tt[fa_] + la < Nf && n * tt[fb_] + lb < Nf;
        fvals[f] = a.skel[j][fin[f] ? bse + la + Nf * lb : 0];
    }
    double bv[16];
    const bool has_b = !LAYERS && a.bff;
    const double *bsrc = has_b ? a.bff : a.mu[j0];  // an in-bounds stand-in when there is no b_ff
    const bool bin = has_b && la < nh && lb < nh;
#pragma unroll
    for (int k = 0; k < 16; ++k) bv[k] = (k < nh) ? bsrc[bin ? f0 + la + Nf * lb + Nf2 * k : 0] : 0.0;
    double mv[4];  // element e = tid + 256 q of the four matrices, padded to 16 x 17
    const bool min_ = (tid >> 4) < nh && (tid & 15) < nh;  // the same (m, k) for every q
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const double *T = (q == 0) ? a.W[j0] : (q == 1) ? a.W[j1] : (q == 2) ? a.V[j1] : a.V[j0];
        mv[q] = T[min_ ? (tid >> 4) * nh + (tid & 15) : 0];
    }
    // the line factors of Thomas along L for this mode pair, while the loads are in flight:
    // pivots p_0 = b_L + mu_j0 + mu_j1, p_c = p_0 - a_L c_L / p_(c-1); hinv_c = 1 / p_c
    const double sub = g.fine[L].a, sup = g.fine[L].c;
    double hinv[nh];
    {
        const double diag = g.fine[L].b + (mu0 + mu1);
        double cp = 0.0;
#pragma unroll
        for (int c = 0; c < nh; ++c) {
            const double den = (c == 0) ? diag : diag - sub * cp;
            hinv[c] = 1.0 / den;
            cp = sup * hinv[c];
        }
        // keep the chain here, in the shadow of the loads, rather than next to its use, and keep
        // the uses of the loaded values below it (the chain waits for the eigenvalues only)
#pragma unroll
        for (int c = 0; c < nh; ++c) asm volatile("" ::"v"(hinv[c]));
        __builtin_amdgcn_sched_barrier(0);
    }
    // 2) the hole's right-hand side: b_ff (or 0, and 0 in the padding) everywhere, then each point
    // of the first or last layer along some axis completed by one thread, that of its lowest such
    // axis' face at its two other coordinates (axis by axis, as hole_rhs subtracts)
#pragma unroll
    for (int k = 0; k < 16; ++k) buf[la + kFS1 * lb + kFS2 * k] = bin ? bv[k] : 0.0;
#pragma unroll
    for (int f = 0; f < 6; ++f) fa[face_at(f, la, lb)] = fin[f] ? fvals[f] : 0.0;
#pragma unroll
    for (int q = 0; q < 4; ++q) mats[q * kFMat + (tid >> 4) * 17 + (tid & 15)] = min_ ? mv[q] : 0.0;
    lds_barrier();
    if (!flag_clear(gv)) return;  // block-uniform
    if (la < nh && lb < nh) {
#pragma unroll
        for (int f = 0; f < 6; ++f) {
            const int j = f >> 1;
            const int lj = (f & 1) ? nh - 1 : 0;
            const int l0 = (j == 0) ? lj : la;
            const int l1 = (j == 1) ? lj : (j == 0 ? la : lb);
            const int l2 = (j == 2) ? lj : lb;
            const bool lower = (j >= 1 && (l0 == 0 || l0 == nh - 1)) || (j == 2 && (l1 == 0 || l1 == nh - 1));
            if (lower) continue;
            double *pt = buf + l0 + kFS1 * l1 + kFS2 * l2;
            *pt = hole_rhs(g, fa, l0, l1, l2, *pt);
        }
    }
    lds_barrier();
    // 3) forward transforms (slab-private)
    slab_transform<j0, L>(buf, mats, lane, wave);
    slab_transform<j1, L>(buf, mats + kFMat, lane, wave);
    __syncthreads();
    // 4) Thomas along the line axis for the 225 lines of modes (m_j0, m_j1)
    if (thomas) {
        constexpr int sL = fstride(L);
        const int base = m0 * fstride(j0) + m1 * fstride(j1);
        double f[nh];
#pragma unroll
        for (int c = 0; c < nh; ++c) f[c] = buf[base + c * sL];
        f[0] = f[0] * hinv[0];
#pragma unroll
        for (int c = 1; c < nh; ++c) f[c] = (f[c] - sub * f[c - 1]) * hinv[c];
#pragma unroll
        for (int c = nh - 2; c >= 0; --c) f[c] -= (sup * hinv[c]) * f[c + 1];
#pragma unroll
        for (int c = 0; c < nh; ++c) buf[base + c * sL] = f[c];
    }
    __syncthreads();
    // 5) backward transforms (slab-private)
    slab_transform<j1, L>(buf, mats + 2 * kFMat, lane, wave);
    slab_transform<j0, L>(buf, mats + 3 * kFMat, lane, wave);
    __syncthreads();
    // 6) write the whole tile (hole values and the skeleton planes above it), x_1 fastest; or, in
    // adjacent-layer mode, only the tile points next to a coarse plane across it (the first and last
    // hole layer along each axis, skeleton points of other planes included) into that plane's layer
    // buffer: side 1 (above) of plane t_j - 1 for l_j = 0, side 0 (below) of plane t_j for
    // l_j = nh - 1, at the canonical offset of the two other fine coordinates.  Tile points on a
    // coarse plane come from the face values.
    auto tile_value = [&](int l0, int l1, int l2) -> double {
        if (l0 < nh && l1 < nh && l2 < nh) return buf[l0 + kFS1 * l1 + kFS2 * l2];
        if (l0 == nh) return fa[face_at(1, l1, l2)];
        if (l1 == nh) return fa[face_at(3, l0, l2)];
        return fa[face_at(5, l0, l1)];
    };
    if (!LAYERS) {
#pragma unroll 4
        for (int o = tid; o < 4096; o += 256) {
            const int l0 = o & 15, l1 = (o >> 4) & 15, l2 = o >> 8;
            if (n * tt[0] + l0 >= Nf || n * tt[1] + l1 >= Nf || n * tt[2] + l2 >= Nf) continue;
            a.out[f0 + l0 + Nf * l1 + Nf2 * l2] = tile_value(l0, l1, l2);
        }
        return;
    }
    const long long lay = (long long)Nc * Nf2;  // one side's layers of one mesh
#pragma unroll
    for (int face = 0; face < 6; ++face) {
        const int j = face >> 1, side = face & 1;  // side 0: layer l_j = 0 (above plane t_j - 1)
        if (side == 0 ? tt[j] == 0 : tt[j] == Nc) continue;
        const int lj = side == 0 ? 0 : nh - 1;
        const int l0 = (j == 0) ? lj : la;
        const int l1 = (j == 1) ? lj : (j == 0 ? la : lb);
        const int l2 = (j == 2) ? lj : lb;
        const int g0 = n * tt[0] + l0, g1 = n * tt[1] + l1, g2 = n * tt[2] + l2;
        if (g0 >= Nf || g1 >= Nf || g2 >= Nf) continue;
        const double v = tile_value(l0, l1, l2);
        // fine coordinates of the two other axes, increasing order
        const int ga = (j == 0) ? g1 : g0, gb = (j == 2) ? g1 : g2;
        double *dst = a.adj[j];
        const long long plane = side == 0 ? tt[j] - 1 : tt[j];
        dst[(side == 0 ? lay : 0) + ga + (long long)Nf * gb + (long long)Nf2 * plane] = v;
    }
}

bool launch_filler(const Plan &p, const double *bff, double *out, hipStream_t st, double *const *skel,
                   bool adj_only) {
    FillArgs a;
    const int d = p.d, nh = p.n - 1;
    for (int j = 0; j < kMaxD; ++j) {
        a.skel[j] = (j < d) ? (skel ? skel[j] : merged_buf(p, j)) : nullptr;
        a.adj[j] = (j < d && adj_only) ? p.ws.EA[j] : nullptr;
        a.mk[j] = (j < d) ? p.mesh[1u << j] : MeshDesc();
        a.W[j] = (j < d) ? p.dWh[j] : nullptr;
        a.V[j] = (j < d) ? p.dVh[j] : nullptr;
        a.mu[j] = (j < d) ? p.dmuh[j] : nullptr;
        a.tr[j] = 0;
    }
    a.line_axis = p.hole_line_axis;
    a.ntr = 0;
    for (int j = 0; j < d; ++j)
        if (j != p.hole_line_axis) a.tr[a.ntr++] = j;
    a.bff = bff;
    a.out = out;
    a.adj_only = adj_only ? 1 : 0;
    a.gate = p.gate;
    a.hinv = nullptr;
    a.hphase = 0;
    a.hbuf = nullptr;
    if (p.hole_dense || p.hole_cr) a.ntr = 0;
    if (p.hole_dense) {  // d = 3, holes of up to 7^3: the dense inverse in the generic filler
        a.hinv = p.dhinv;
        a.ntr = 0;
    }
    int npts = 1;
    for (int j = 0; j < d; ++j) npts *= nh;
    const size_t lds = (size_t)(2 * npts + a.ntr * (2 * nh * nh + nh)) * sizeof(double);
    int tiles = 1;
    for (int j = 0; j < d; ++j) tiles *= (p.Nc + 1);
    const dim3 grid(tiles), blk(256);
    if (p.hole_dense) {
        const size_t ldsd = (size_t)2 * npts * sizeof(double);
        switch (nh) {
            case 1: ASDSM_LAUNCH((k_filler<3, 1>), grid, blk, ldsd, st, p.geo, a); break;
            case 3: ASDSM_LAUNCH((k_filler<3, 3>), grid, blk, ldsd, st, p.geo, a); break;
            default: ASDSM_LAUNCH((k_filler<3, 7>), grid, blk, ldsd, st, p.geo, a); break;
        }
        return true;
    }
    if (p.hole_cr) {
        // d = 3, holes of 15^3: right-hand sides to HB, block cyclic reduction over all holes in
        // place (one shared table, the GEMM form), the tiles from HB
        if (d != 3 || nh != 15 || !p.ws.HB) return false;
        a.hbuf = p.ws.HB;
        a.hphase = 1;
        ASDSM_LAUNCH((k_filler<3, 15>), grid, blk, 0, st, p.geo, a);
        CrJob job{};
        job.nbox = 1;
        job.N = nh;
        job.L = p.hole_cr_L;
        job.NB = nh * nh;
        job.gate = p.gate;
        job.scratch = p.ws.crs;
        job.scratch_len = p.ws.crs_len;
        job.shared_tab = 1;
        CrBox &bx = job.box[0];
        bx.src = bx.dst = p.ws.HB;
        bx.tab = p.dhcr;
        bx.nmodes = tiles;
        bx.mext0 = tiles;
        bx.ms0 = npts;
        bx.ms1 = (long long)tiles * npts;
        bx.sw = nh * nh;
        bx.sc = 1;
        if (!launch_block_cr(job, st)) return false;
        a.hphase = 2;
        ASDSM_LAUNCH((k_filler<3, 15>), grid, blk, 0, st, p.geo, a);
        return true;
    }
    if (d == 3 && nh == 15) {
#define ASDSM_FILL3(LL)                                                                   \
    do {                                                                                  \
        if (adj_only) ASDSM_LAUNCH((k_filler_mfma3<LL, true>), grid, blk, 0, st, p.geo, a); \
        else ASDSM_LAUNCH((k_filler_mfma3<LL, false>), grid, blk, 0, st, p.geo, a);         \
    } while (0)
        if (p.hole_line_axis == 0) ASDSM_FILL3(0);
        else if (p.hole_line_axis == 1) ASDSM_FILL3(1);
        else ASDSM_FILL3(2);
#undef ASDSM_FILL3
        return true;
    }
    if (!adj_only && (d == 3 || d == 4) && (nh == 1 || nh == 3 || nh == 7)) {
#define ASDSM_FILL_LINES(DD, NHV) ASDSM_LAUNCH((k_filler_lines<DD, NHV>), grid, blk, 0, st, p.geo, a)
        if (d == 3) {
            if (nh == 1) ASDSM_FILL_LINES(3, 1);
            else if (nh == 3) ASDSM_FILL_LINES(3, 3);
            else ASDSM_FILL_LINES(3, 7);
        } else {
            if (nh == 1) ASDSM_FILL_LINES(4, 1);
            else if (nh == 3) ASDSM_FILL_LINES(4, 3);
            else ASDSM_FILL_LINES(4, 7);
        }
#undef ASDSM_FILL_LINES
        return true;
    }
#define ASDSM_FILL(DD, NHV) ASDSM_LAUNCH((k_filler<DD, NHV>), grid, blk, lds, st, p.geo, a)
    if (d == 2) {
        switch (nh) {
            case 1: ASDSM_FILL(2, 1); break;
            case 3: ASDSM_FILL(2, 3); break;
            case 7: ASDSM_FILL(2, 7); break;
            case 15: ASDSM_FILL(2, 15); break;
            case 31: ASDSM_FILL(2, 31); break;
            default: ASDSM_FILL(2, 0); break;
        }
    } else if (d == 3) {
        switch (nh) {
            case 1: ASDSM_FILL(3, 1); break;
            case 3: ASDSM_FILL(3, 3); break;
            case 7: ASDSM_FILL(3, 7); break;
            case 15: ASDSM_FILL(3, 15); break;
            default: ASDSM_FILL(3, 0); break;
        }
    } else {
        switch (nh) {
            case 1: ASDSM_FILL(4, 1); break;
            case 3: ASDSM_FILL(4, 3); break;
            case 7: ASDSM_FILL(4, 7); break;
            default: ASDSM_FILL(4, 0); break;
        }
    }
#undef ASDSM_FILL
    return true;
}

}  // namespace asdsm
