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
    const int *perm_table;          // error phase: permutation of step it at perm_table[kMaxD*it]
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
        const int *perm = a.perm_table + kMaxD * a.state->it;
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

__device__ __forceinline__ const double *res_k(const Skel4Args &a, int k) {
    return (k == 0) ? a.res[1] : (k == 1) ? a.res[2] : (k == 2) ? a.res[4] : a.res[8];
}
__device__ __forceinline__ double *lines_k(const Skel4Args &a, int k) {
    return (k == 0) ? a.lines[0] : (k == 1) ? a.lines[1] : (k == 2) ? a.lines[2] : a.lines[3];
}

// delta on the three plane families of every M_k.  Grid (blocks, 4).
__global__ __launch_bounds__(256) void k_cross4(Geo g, Skel4Args a) {
    if (a.gate && *a.gate) return;
    const Perm4 pm = load_perm4(a);
    const int k = blockIdx.y;
    const int Nf = g.Nf, Nc = g.Nc, n = g.n;
    const long long F = (long long)Nc * Nc * Nf * Nf, Nf2 = (long long)Nf * Nf;
    const double scale_k = (a.mode == 0) ? 1.0 : a.scal[kScalInvNorm + k];
    const double *__restrict__ Xk = res_k(a, k);
    double *__restrict__ L = lines_k(a, k);
    for (long long t = (long long)blockIdx.x * 256 + threadIdx.x; t < 3 * F; t += (long long)gridDim.x * 256) {
        const int fam = (int)(t / F);
        const long long r = t - fam * F;
        const int u = (int)(r % Nf), v = (int)((r / Nf) % Nf);
        const int cf = (int)((r / Nf2) % Nc), ck = (int)(r / (Nf2 * Nc));
        const int C = (cf + 1) * n - 1;
        const int i0 = fam == 0 ? C : u;
        const int i1 = fam == 0 ? u : (fam == 1 ? C : v);
        const int i2 = fam == 2 ? C : v;
        const int4 p = pt4(k, i0, i1, i2, ck, n);
        const double uh = xval4(a, p, cset4(p, n), Nf, Nc, n, pm);
        L[t] = uh - scale_k * Xk[i0 + Nf * (i1 + (long long)Nf * (i2 + (long long)Nf * ck))];
    }
}

// R_12 on family 1: delta - P_2 delta (zero where f2 is on a coarse plane).
__global__ __launch_bounds__(256) void k_rem12(Geo g, Skel4Args a) {
    if (a.gate && *a.gate) return;
    const int k = blockIdx.y;
    const int Nf = g.Nf, Nc = g.Nc, n = g.n;
    const long long F = (long long)Nc * Nc * Nf * Nf, Nf2 = (long long)Nf * Nf;
    double *__restrict__ L = lines_k(a, k);
    const double *__restrict__ D1 = L + F;
    const double *__restrict__ D2 = L + 2 * F;
    double *__restrict__ R12 = L + 3 * F;
    const double *__restrict__ Sp = a.Sp;
    for (long long t = (long long)blockIdx.x * 256 + threadIdx.x; t < F; t += (long long)gridDim.x * 256) {
        const int i0 = (int)(t % Nf), i2 = (int)((t / Nf) % Nf);
        const int c1 = (int)((t / Nf2) % Nc), ck = (int)(t / (Nf2 * Nc));
        double v = 0.0;
        if (!on_coarse(i2, n)) {
            const int i1 = (c1 + 1) * n - 1;
            v = D1[t];
            for (int c2 = 0; c2 < Nc; ++c2)
                v -= Sp[(long long)i2 * Nc + c2] * D2[i0 + Nf * (i1 + (long long)Nf * (c2 + (long long)Nc * ck))];
        }
        R12[t] = v;
    }
}

// R_0 on family 0: delta - (P_2 delta + P_1 R_12) (zero where f1 or f2 is on a coarse plane).
__global__ __launch_bounds__(256) void k_rem0(Geo g, Skel4Args a) {
    if (a.gate && *a.gate) return;
    const int k = blockIdx.y;
    const int Nf = g.Nf, Nc = g.Nc, n = g.n;
    const long long F = (long long)Nc * Nc * Nf * Nf, Nf2 = (long long)Nf * Nf;
    double *__restrict__ L = lines_k(a, k);
    const double *__restrict__ D0 = L;
    const double *__restrict__ D2 = L + 2 * F;
    const double *__restrict__ R12 = L + 3 * F;
    double *__restrict__ R0 = L + 4 * F;
    const double *__restrict__ Sp = a.Sp;
    for (long long t = (long long)blockIdx.x * 256 + threadIdx.x; t < F; t += (long long)gridDim.x * 256) {
        const int i1 = (int)(t % Nf), i2 = (int)((t / Nf) % Nf);
        const int c0 = (int)((t / Nf2) % Nc), ck = (int)(t / (Nf2 * Nc));
        double v = 0.0;
        if (!on_coarse(i1, n) && !on_coarse(i2, n)) {
            const int i0 = (c0 + 1) * n - 1;
            double b = 0.0;
            for (int c2 = 0; c2 < Nc; ++c2)
                b += Sp[(long long)i2 * Nc + c2] * D2[i0 + Nf * (i1 + (long long)Nf * (c2 + (long long)Nc * ck))];
            for (int c1 = 0; c1 < Nc; ++c1)
                b += Sp[(long long)i1 * Nc + c1] * R12[i0 + Nf * (i2 + (long long)Nf * (c1 + (long long)Nc * ck))];
            v = D0[t] - b;
        }
        R0[t] = v;
    }
}

// Merged skeleton values of every M_k: uhat on cross points, u_k + B delta elsewhere (Algorithm 2
// steps 5 and 6).
__global__ __launch_bounds__(256) void k_merge4(Geo g, Skel4Args a) {
    if (a.gate && *a.gate) return;
    const Perm4 pm = load_perm4(a);
    const int k = blockIdx.y;
    const int Nf = g.Nf, Nc = g.Nc, n = g.n;
    const long long F = (long long)Nc * Nc * Nf * Nf, Nf2 = (long long)Nf * Nf;
    const long long size = Nf2 * Nf * Nc;
    const unsigned mk = 1u << k;
    const double scale_k = (a.mode == 0) ? 1.0 : a.scal[kScalInvNorm + k];
    const double *__restrict__ X = res_k(a, k);
    const double *__restrict__ L = lines_k(a, k);
    const double *__restrict__ D2 = L + 2 * F;
    const double *__restrict__ R12 = L + 3 * F;
    const double *__restrict__ R0 = L + 4 * F;
    double *__restrict__ out = (k == 0) ? a.skel[0] : (k == 1) ? a.skel[1] : (k == 2) ? a.skel[2] : a.skel[3];
    const double *__restrict__ Sp = a.Sp;
    for (long long idx = (long long)blockIdx.x * 256 + threadIdx.x; idx < size; idx += (long long)gridDim.x * 256) {
        const int i0 = (int)(idx % Nf), i1 = (int)((idx / Nf) % Nf), i2 = (int)((idx / Nf2) % Nf);
        const int ck = (int)(idx / (Nf2 * Nf));
        const int4 p = pt4(k, i0, i1, i2, ck, n);
        const unsigned S = cset4(p, n);
        double v;
        if (S != mk) {
            v = xval4(a, p, S, Nf, Nc, n, pm);
        } else {
            double c2s = 0.0, c1s = 0.0, c0s = 0.0;
            for (int c = 0; c < Nc; ++c) {
                const long long base = (long long)Nf * Nf * (c + (long long)Nc * ck);
                c2s += Sp[(long long)i2 * Nc + c] * D2[i0 + (long long)Nf * i1 + base];
                c1s += Sp[(long long)i1 * Nc + c] * R12[i0 + (long long)Nf * i2 + base];
                c0s += Sp[(long long)i0 * Nc + c] * R0[i1 + (long long)Nf * i2 + base];
            }
            v = scale_k * X[idx] + (c2s + c1s + c0s);
        }
        out[idx] = v;
    }
}

static Skel4Args skel4_args(const Plan &p, int mode, const double *const *res) {
    Skel4Args a;
    for (unsigned s = 0; s < kMaxMeshes; ++s) a.res[s] = (s < (1u << p.d)) ? res[s] : nullptr;
    for (int k = 0; k < kMaxD; ++k) {
        a.lines[k] = (k < p.d) ? p.ws.lines[k] : nullptr;
        a.skel[k] = (k < p.d) ? p.ws.Y[1u << k] : nullptr;
    }
    a.perm_table = p.ws.perm_table;
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
    return (unsigned)(b < 1 ? 1 : b);
}

void launch_crosspoints4(const Plan &p, int mode, const double *const *res, hipStream_t st) {
    const Skel4Args a = skel4_args(p, mode, res);
    const long long F = (long long)p.Nc * p.Nc * p.Nf * p.Nf;
    ASDSM_LAUNCH(k_cross4, dim3(blocks_for(3 * F, 1024), 4, 1), dim3(256), 0, st, p.geo, a);
    ASDSM_LAUNCH(k_rem12, dim3(blocks_for(F, 1024), 4, 1), dim3(256), 0, st, p.geo, a);
    ASDSM_LAUNCH(k_rem0, dim3(blocks_for(F, 1024), 4, 1), dim3(256), 0, st, p.geo, a);
}

void launch_merge4(const Plan &p, int mode, const double *const *res, hipStream_t st) {
    const Skel4Args a = skel4_args(p, mode, res);
    ASDSM_LAUNCH(k_merge4, dim3(blocks_for(p.mesh[1].size, 4096), 4, 1), dim3(256), 0, st, p.geo, a);
}

}  // namespace asdsm
