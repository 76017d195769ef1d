// Skeleton builder (Algorithm 2) for d = 4.
//
// Each anisotropic mesh M_k has three fine axes f0 < f1 < f2 and its coarse axis k.  Its cross
// points are the points with a fine coordinate on a coarse plane: three families of planes, family
// j holding the points with coordinate f_j on a coarse plane.  The cross-point value uhat (initial
// guess: the extrapolation over the meshes that contain the point and their intersection mesh;
// error phase: this step's random axis choice) gives the discrepancy delta = uhat - u_k on every
// family, which the Boolean sum I - (I - P_0)(I - P_1)(I - P_2) of the three spline extensions
// (P_j: cubic not-a-knot spline with zero ends along f_j, from the values on family j) carries over
// the rest of M_k.  It is evaluated as
//     B_12 = P_2 delta + P_1 R_12,        R_12 = delta - P_2 delta            on family 1,
//     B    = B_12 + P_0 R_0,              R_0  = delta - B_12                 on family 0,
// so a point costs three sums of N_c terms.  Layouts per mesh (F = N_c^2 N_f^2 values each):
//     family 0 / R_0  : i1 + N_f (i2 + N_f (c0 + N_c ck))
//     family 1 / R_12 : i0 + N_f (i2 + N_f (c1 + N_c ck))
//     family 2        : i0 + N_f (i1 + N_f (c2 + N_c ck))
// with i_j the fine coordinate along f_j, c_j the coarse index of a coordinate on a coarse plane and
// ck the coarse plane of M_k; buffer order: family 0, 1, 2, R_12, R_0.
#include <algorithm>

#include "device_common.hpp"
#include "kernels.hpp"

namespace asdsm {

struct Skel4Args {
    const double *res[kMaxMeshes];  // solution on each mesh (canonical layout)
    double *lines[kMaxD];           // discrepancy families and remainders per anisotropic mesh
    double *skel[kMaxD];            // merged skeleton values per anisotropic mesh (output)
    const double *Sp;               // N_f x N_c spline matrix
    const double *scal;             // normalisation factors (error phase)
    int mode;                       // 0 initial guess, 1 error phase
    const IterState *state;
    const int *gate;
};

__device__ __forceinline__ int c4(const int4 &p, int j) { return j == 0 ? p.x : j == 1 ? p.y : j == 2 ? p.z : p.w; }

// The fine point of M_k with fine coordinates (i0, i1, i2) along its fine axes and coarse plane ck.
__device__ __forceinline__ int4 pt4(int k, int i0, int i1, int i2, int ck, int n) {
    const int c = (ck + 1) * n - 1;
    if (k == 0) return int4{c, i0, i1, i2};
    if (k == 1) return int4{i0, c, i1, i2};
    if (k == 2) return int4{i0, i1, c, i2};
    return int4{i0, i1, i2, c};
}

__device__ __forceinline__ unsigned cset4(const int4 &p, int n) {
    return (on_coarse(p.x, n) ? 1u : 0u) | (on_coarse(p.y, n) ? 2u : 0u) | (on_coarse(p.z, n) ? 4u : 0u) |
           (on_coarse(p.w, n) ? 8u : 0u);
}

// Canonical offset of p on M_S: the fine axes (not in S) first, then the coarse axes of S, each
// group in increasing order, first listed fastest.
__device__ __forceinline__ long long off4(unsigned S, const int4 &p, int Nf, int Nc, int n) {
    long long off = 0, mul = 1;
#pragma unroll
    for (int j = 0; j < 4; ++j)
        if (!((S >> j) & 1u)) {
            off += (long long)c4(p, j) * mul;
            mul *= Nf;
        }
#pragma unroll
    for (int j = 0; j < 4; ++j)
        if ((S >> j) & 1u) {
            off += (long long)coarse_of(c4(p, j), n) * mul;
            mul *= Nc;
        }
    return off;
}

// res[S] through selects (a dynamic index into the argument struct would be copied to scratch)
__device__ __forceinline__ const double *pick4(const Skel4Args &a, unsigned S) {
    const double *r = a.res[0];
#pragma unroll
    for (unsigned q = 1; q < 16; ++q) r = (S == q) ? a.res[q] : r;
    return r;
}

struct Perm4 {
    int p0, p1, p2, p3;
};

__device__ __forceinline__ Perm4 load_perm4(const Skel4Args &a) {
    Perm4 c{0, 1, 2, 3};
    if (a.mode == 1) {
        const int *perm = a.state->perm;
        c = Perm4{perm[0], perm[1], perm[2], perm[3]};
    }
    return c;
}

// uhat at a cross point p (coarse set S, |S| >= 2)
__device__ __forceinline__ double xval4(const Skel4Args &a, const int4 &p, unsigned S, int Nf, int Nc, int n,
                                        const Perm4 &pm) {
    if (a.mode == 0) {
        double sum = 0.0;
        int cnt = 0;
#pragma unroll
        for (int j = 0; j < 4; ++j)
            if ((S >> j) & 1u) {
                sum += a.res[1u << j][off4(1u << j, p, Nf, Nc, n)];
                ++cnt;
            }
        sum -= pick4(a, S)[off4(S, p, Nf, Nc, n)];
        return sum / (double)(cnt - 1);
    }
    int j = pm.p0;
    if (!((S >> j) & 1u)) j = pm.p1;
    if (!((S >> j) & 1u)) j = pm.p2;
    if (!((S >> j) & 1u)) j = pm.p3;
    const unsigned mj = 1u << j;
    return a.scal[kScalInvNorm + j] * pick4(a, mj)[off4(mj, p, Nf, Nc, n)];
}

// Block index with each XCD owning one contiguous range of the (row-ordered) blocks: the hardware
// deals the blocks of a launch to the eight XCDs in turn, so consecutive rows would otherwise land
// on different XCDs and every XCD's L2 would fetch all of the (small, much re-read) family arrays.
// The launchers round gridDim.x up to a multiple of 8, which makes this a permutation.
__device__ __forceinline__ int xcd_block() {
    const int per = (int)gridDim.x >> 3;
    return (int)(blockIdx.x & 7) * per + (int)(blockIdx.x >> 3);
}

__device__ __forceinline__ const double *res_k(const Skel4Args &a, int k) {
    return (k == 0) ? a.res[1] : (k == 1) ? a.res[2] : (k == 2) ? a.res[4] : a.res[8];
}
__device__ __forceinline__ double *lines_k(const Skel4Args &a, int k) {
    return (k == 0) ? a.lines[0] : (k == 1) ? a.lines[1] : (k == 2) ? a.lines[2] : a.lines[3];
}

// delta on the three plane families of every M_k.  Grid (blocks, 4): one wave per row of N_f
// values along the family's first free axis; the row's (family, second free coordinate, coarse
// indices) are wave-uniform 32-bit values.
__global__ __launch_bounds__(256) void k_cross4(Geo g, Skel4Args a) {
    if (a.gate && *a.gate) return;
    const Perm4 pm = load_perm4(a);
    const int k = blockIdx.y;
    const int Nf = g.Nf, Nc = g.Nc, n = g.n;
    const long long F = (long long)Nc * Nc * Nf * Nf;
    const int rows_fam = Nf * Nc * Nc, nrows = 3 * rows_fam;
    const double scale_k = (a.mode == 0) ? 1.0 : a.scal[kScalInvNorm + k];
    const double *__restrict__ Xk = res_k(a, k);
    double *__restrict__ L = lines_k(a, k);
    double *__restrict__ out = (k == 0) ? a.skel[0] : (k == 1) ? a.skel[1] : (k == 2) ? a.skel[2] : a.skel[3];
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    for (int row0 = xcd_block() * 4 + ty; row0 < nrows; row0 += gridDim.x * 4) {
        const int row = __builtin_amdgcn_readfirstlane(row0);
        const int fam = row / rows_fam, rw = row - fam * rows_fam;
        const int v = rw % Nf, q = rw / Nf, cf = q % Nc, ck = q / Nc;
        const int C = (cf + 1) * n - 1;
        double *__restrict__ dst = L + fam * F + (long long)Nf * rw;
        for (int u = tx; u < Nf; u += 64) {
            const int i0 = fam == 0 ? C : u;
            const int i1 = fam == 0 ? u : (fam == 1 ? C : v);
            const int i2 = fam == 2 ? C : v;
            const int4 p = pt4(k, i0, i1, i2, ck, n);
            const double uh = xval4(a, p, cset4(p, n), Nf, Nc, n, pm);
            const long long idx = i0 + Nf * (i1 + (long long)Nf * (i2 + (long long)Nf * ck));
            dst[u] = uh - scale_k * Xk[idx];
            // the merged value of a cross point is uhat itself: written here, skipped by k_merge4
            // (a point on two or three families gets the same value from each)
            out[idx] = uh;
        }
    }
}

// R_12 on family 1: delta - P_2 delta (zero where f2 is on a coarse plane).  One wave per row of
// N_f values along f0, as in k_cross4.
__global__ __launch_bounds__(256) void k_rem12(Geo g, Skel4Args a) {
    if (a.gate && *a.gate) return;
    const int k = blockIdx.y;
    const int Nf = g.Nf, Nc = g.Nc, n = g.n;
    const long long F = (long long)Nc * Nc * Nf * Nf;
    const int nrows = Nf * Nc * Nc;
    double *__restrict__ L = lines_k(a, k);
    const double *__restrict__ Sp = a.Sp;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    for (int row0 = xcd_block() * 4 + ty; row0 < nrows; row0 += gridDim.x * 4) {
        const int row = __builtin_amdgcn_readfirstlane(row0);
        const int i2 = row % Nf, q = row / Nf, c1 = q % Nc, ck = q / Nc;
        const int i1 = (c1 + 1) * n - 1;
        const double *__restrict__ D1 = L + F + (long long)Nf * row;
        const double *__restrict__ D2 = L + 2 * F + (long long)Nf * i1 + (long long)Nf * Nf * Nc * ck;
        double *__restrict__ R12 = L + 3 * F + (long long)Nf * row;
        const bool live = !on_coarse(i2, n);
        for (int i0 = tx; i0 < Nf; i0 += 64) {
            double v = 0.0;
            if (live) {
                v = D1[i0];
                for (int c2 = 0; c2 < Nc; ++c2) v -= Sp[i2 * Nc + c2] * D2[i0 + (long long)Nf * Nf * c2];
            }
            R12[i0] = v;
        }
    }
}

// R_0 on family 0: delta - (P_2 delta + P_1 R_12) (zero where f1 or f2 is on a coarse plane).  One
// wave per row of N_f values along f1.
__global__ __launch_bounds__(256) void k_rem0(Geo g, Skel4Args a) {
    if (a.gate && *a.gate) return;
    const int k = blockIdx.y;
    const int Nf = g.Nf, Nc = g.Nc, n = g.n;
    const long long F = (long long)Nc * Nc * Nf * Nf;
    const int nrows = Nf * Nc * Nc;
    double *__restrict__ L = lines_k(a, k);
    const double *__restrict__ Sp = a.Sp;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    for (int row0 = xcd_block() * 4 + ty; row0 < nrows; row0 += gridDim.x * 4) {
        const int row = __builtin_amdgcn_readfirstlane(row0);
        const int i2 = row % Nf, q = row / Nf, c0 = q % Nc, ck = q / Nc;
        const int i0 = (c0 + 1) * n - 1;
        const long long cb = (long long)Nf * Nf * Nc * ck;
        const double *__restrict__ D0 = L + (long long)Nf * row;
        const double *__restrict__ D2 = L + 2 * F + cb + i0;
        const double *__restrict__ R12 = L + 3 * F + cb + i0 + (long long)Nf * i2;
        double *__restrict__ R0 = L + 4 * F + (long long)Nf * row;
        const bool live2 = !on_coarse(i2, n);
        for (int i1 = tx; i1 < Nf; i1 += 64) {
            double v = 0.0;
            if (live2 && !on_coarse(i1, n)) {
                double b = 0.0;
                for (int c2 = 0; c2 < Nc; ++c2)
                    b += Sp[i2 * Nc + c2] * D2[(long long)Nf * (i1 + (long long)Nf * c2)];
                for (int c1 = 0; c1 < Nc; ++c1) b += Sp[i1 * Nc + c1] * R12[(long long)Nf * Nf * c1];
                v = D0[i1] - b;
            }
            R0[i1] = v;
        }
    }
}

// Merged skeleton values of every M_k off the cross points: u_k + B delta (Algorithm 2 steps 5 and
// 6; the cross points' uhat is written by k_cross4).  Grid (blocks, 4): one wave per row of N_f points along f0, so the row's other
// coordinates (i1, i2, ck) are 32-bit and uniform in the wave; NC > 0 fixes N_c at compile time
// and the three N_c-term sums are unrolled (all their loads in flight together).
template <int NC>
__global__ __launch_bounds__(256) void k_merge4(Geo g, Skel4Args a) {
    if (a.gate && *a.gate) return;
    const int k = blockIdx.y;
    const int Nf = g.Nf, Nc = (NC > 0) ? NC : g.Nc, n = g.n;
    const long long Nf2 = (long long)Nf * Nf, F = (long long)Nc * Nc * Nf2;
    const int nrows = Nf * Nf * Nc;
    const unsigned mk = 1u << k;
    const double scale_k = (a.mode == 0) ? 1.0 : a.scal[kScalInvNorm + k];
    const double *__restrict__ X = res_k(a, k);
    const double *__restrict__ L = lines_k(a, k);
    const double *__restrict__ Sp = a.Sp;
    double *__restrict__ out = (k == 0) ? a.skel[0] : (k == 1) ? a.skel[1] : (k == 2) ? a.skel[2] : a.skel[3];
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    for (int row0 = xcd_block() * 4 + ty; row0 < nrows; row0 += gridDim.x * 4) {
        // the row is the same for the whole wave: make that visible (scalar address arithmetic)
        const int row = __builtin_amdgcn_readfirstlane(row0);
        const int i1 = row % Nf, q = row / Nf, i2 = q % Nf, ck = q / Nf;
        const long long cb = Nf2 * Nc * ck;
        const double *__restrict__ D2 = L + 2 * F + cb + (long long)Nf * i1;
        const double *__restrict__ R12 = L + 3 * F + cb + (long long)Nf * i2;
        const double *__restrict__ R0 = L + 4 * F + cb + i1 + (long long)Nf * i2;
        for (int i0 = tx; i0 < Nf; i0 += 64) {
            const long long idx = i0 + (long long)Nf * row;
            const int4 p = pt4(k, i0, i1, i2, ck, n);
            if (cset4(p, n) != mk) continue;  // cross point: uhat, written by k_cross4
            double c2s = 0.0, c1s = 0.0, c0s = 0.0;
#pragma unroll(NC > 0 ? NC : 1)
            for (int c = 0; c < Nc; ++c) {
                c2s += Sp[i2 * Nc + c] * D2[i0 + Nf2 * c];
                c1s += Sp[i1 * Nc + c] * R12[i0 + Nf2 * c];
                c0s += Sp[i0 * Nc + c] * R0[Nf2 * c];
            }
            out[idx] = scale_k * X[idx] + (c2s + c1s + c0s);
        }
    }
}

static Skel4Args skel4_args(const Plan &p, int mode, const double *const *res) {
    Skel4Args a;
    for (unsigned s = 0; s < kMaxMeshes; ++s) a.res[s] = (s < (1u << p.d)) ? res[s] : nullptr;
    for (int k = 0; k < kMaxD; ++k) {
        a.lines[k] = (k < p.d) ? p.ws.lines[k] : nullptr;
        a.skel[k] = (k < p.d) ? p.ws.Y[1u << k] : nullptr;
    }
    a.state = p.ws.state;
    a.gate = p.gate;
    a.Sp = p.dSp;
    a.scal = p.ws.scal;
    a.mode = mode;
    return a;
}

static unsigned blocks_for(long long n, long long cap) {
    long long b = (n + 255) / 256;
    if (b > cap) b = cap;
    if (b < 1) b = 1;
    return (unsigned)((b + 7) / 8 * 8);  // a multiple of 8 (see xcd_block)
}

void launch_crosspoints4(const Plan &p, int mode, const double *const *res, hipStream_t st) {
    const Skel4Args a = skel4_args(p, mode, res);
    const long long F = (long long)p.Nc * p.Nc * p.Nf * p.Nf;
    const long long rows = F / p.Nf;  // rows of N_f values per family
    ASDSM_LAUNCH(k_cross4, dim3(blocks_for(3 * rows * 64, 8192), 4, 1), dim3(256), 0, st, p.geo, a);
    ASDSM_LAUNCH(k_rem12, dim3(blocks_for(rows * 64, 8192), 4, 1), dim3(256), 0, st, p.geo, a);
    ASDSM_LAUNCH(k_rem0, dim3(blocks_for(rows * 64, 8192), 4, 1), dim3(256), 0, st, p.geo, a);
}

void launch_merge4(const Plan &p, int mode, const double *const *res, hipStream_t st) {
    const Skel4Args a = skel4_args(p, mode, res);
    long long rows = (long long)p.Nf * p.Nf * p.Nc;
    const dim3 grid(blocks_for(rows * 64, 8192), 4, 1);
    switch (p.Nc) {
        case 3: ASDSM_LAUNCH((k_merge4<3>), grid, dim3(256), 0, st, p.geo, a); break;
        case 7: ASDSM_LAUNCH((k_merge4<7>), grid, dim3(256), 0, st, p.geo, a); break;
        case 15: ASDSM_LAUNCH((k_merge4<15>), grid, dim3(256), 0, st, p.geo, a); break;
        default: ASDSM_LAUNCH((k_merge4<0>), grid, dim3(256), 0, st, p.geo, a); break;
    }
}

}  // namespace asdsm
