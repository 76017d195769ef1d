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
    int perm[kMaxD];
};

__device__ __forceinline__ double crosspoint_value(const SkelArgs &a, const Geo &g, const int *i,
                                                  unsigned S) {
    if (a.mode == 0) {
        double sum = 0.0;
        int cnt = 0;
        for (int j = 0; j < g.d; ++j)
            if ((S >> j) & 1u) {
                const unsigned mj = 1u << j;
                sum += a.res[mj][canon_offset(a.mesh[mj], i, g.n)];
                ++cnt;
            }
        sum -= a.res[S][canon_offset(a.mesh[S], i, g.n)];
        return sum / (double)(cnt - 1);
    }
    for (int q = 0; q < g.d; ++q) {
        const int j = a.perm[q];
        if ((S >> j) & 1u) {
            const unsigned mj = 1u << j;
            return a.scal[kScalInvNorm + j] * a.res[mj][canon_offset(a.mesh[mj], i, g.n)];
        }
    }
    return 0.0;  // unreachable: S has >= 2 axes
}

__device__ __forceinline__ unsigned coarse_set(const int *i, int d, int n) {
    unsigned S = 0;
    for (int j = 0; j < d; ++j)
        if (on_coarse(i[j], n)) S |= 1u << j;
    return S;
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

// delta_k on the cross-point lines of each anisotropic mesh.
// d = 2: lines[k][ck*Nc + ca].
// d = 3: part A [ck][ca][ib] (Nc*Nc*Nf), part B [ck][ia][cb] (Nc*Nf*Nc), then part R (filled later).
__global__ __launch_bounds__(256) void k_crosspoints(Geo g, SkelArgs a) {
    const int k = blockIdx.y;
    const int d = g.d, Nf = g.Nf, Nc = g.Nc, n = g.n;
    int fa, fb;
    fine_axes_of(k, d, fa, fb);
    const unsigned mk = 1u << k;
    const double scale_k = (a.mode == 0) ? 1.0 : a.scal[kScalInvNorm + k];
    const long long nA = (d == 2) ? (long long)Nc * Nc : (long long)Nc * Nc * Nf;
    const long long total = (d == 2) ? nA : 2 * nA;
    for (long long t = (long long)blockIdx.x * 256 + threadIdx.x; t < total; t += (long long)gridDim.x * 256) {
        int i[kMaxD] = {0, 0, 0};
        if (d == 2) {
            const int ca = (int)(t % Nc), ck = (int)(t / Nc);
            i[k] = (ck + 1) * n - 1;
            i[fa] = (ca + 1) * n - 1;
        } else if (t < nA) {
            const int ib = (int)(t % Nf);
            const int ca = (int)((t / Nf) % Nc);
            const int ck = (int)(t / ((long long)Nf * Nc));
            i[k] = (ck + 1) * n - 1;
            i[fa] = (ca + 1) * n - 1;
            i[fb] = ib;
        } else {
            const long long u = t - nA;
            const int cb = (int)(u % Nc);
            const int ia = (int)((u / Nc) % Nf);
            const int ck = (int)(u / ((long long)Nc * Nf));
            i[k] = (ck + 1) * n - 1;
            i[fa] = ia;
            i[fb] = (cb + 1) * n - 1;
        }
        const unsigned S = coarse_set(i, d, n);
        const double uh = crosspoint_value(a, g, i, S);
        const double uk = scale_k * a.res[mk][canon_offset(a.mesh[mk], i, n)];
        a.lines[k][t] = uh - uk;
    }
}

// d = 3 only: R[ck][ca][ib] = A[ck][ca][ib] - sum_cb Sp[ib][cb] A[ck][ca][C[cb]], so that the Boolean
// sum P_a delta + P_b delta - P_a P_b delta = P_a R + P_b delta costs O(N_c) per point.
__global__ __launch_bounds__(256) void k_lines_residual(Geo g, SkelArgs a) {
    const int k = blockIdx.y;
    const int Nf = g.Nf, Nc = g.Nc, n = g.n;
    const long long nA = (long long)Nc * Nc * Nf;
    const double *__restrict__ A = a.lines[k];
    double *__restrict__ R = a.lines[k] + 2 * nA;
    for (long long t = (long long)blockIdx.x * 256 + threadIdx.x; t < nA; t += (long long)gridDim.x * 256) {
        const int ib = (int)(t % Nf);
        const long long rowbase = t - ib;  // (ck*Nc + ca)*Nf
        double v = A[t];
        if (on_coarse(ib, n)) {
            R[t] = 0.0;
            continue;
        }
        for (int cb = 0; cb < Nc; ++cb) v -= a.Sp[(long long)ib * Nc + cb] * A[rowbase + (cb + 1) * n - 1];
        R[t] = v;
    }
}

__global__ __launch_bounds__(256) void k_merge(Geo g, SkelArgs a) {
    const int k = blockIdx.y;
    const int d = g.d, Nf = g.Nf, Nc = g.Nc, n = g.n;
    int fa, fb;
    fine_axes_of(k, d, fa, fb);
    const unsigned mk = 1u << k;
    const MeshDesc &m = a.mesh[mk];
    const double scale_k = (a.mode == 0) ? 1.0 : a.scal[kScalInvNorm + k];
    const double *__restrict__ X = a.res[mk];
    double *__restrict__ out = a.skel[k];
    const double *__restrict__ L = a.lines[k];
    const double *__restrict__ Sp = a.Sp;
    const long long nA = (long long)Nc * Nc * Nf;
    for (long long idx = (long long)blockIdx.x * 256 + threadIdx.x; idx < m.size; idx += (long long)gridDim.x * 256) {
        int i[kMaxD] = {0, 0, 0};
        const int ia = (int)(idx % Nf);
        i[fa] = ia;
        int ib = 0, ck;
        if (d == 2) {
            ck = (int)(idx / Nf);
        } else {
            ib = (int)((idx / Nf) % Nf);
            ck = (int)(idx / ((long long)Nf * Nf));
            i[fb] = ib;
        }
        i[k] = (ck + 1) * n - 1;
        const unsigned S = coarse_set(i, d, n);
        double v;
        if (S != mk) {
            v = crosspoint_value(a, g, i, S);
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

static SkelArgs skel_args(const Plan &p, int mode, const int *perm, const double *const *res) {
    SkelArgs a;
    for (unsigned s = 0; s < kMaxMeshes; ++s) {
        a.res[s] = (s < (1u << p.d)) ? res[s] : nullptr;
        a.mesh[s] = (s < (1u << p.d)) ? p.mesh[s] : MeshDesc();
    }
    for (int k = 0; k < kMaxD; ++k) {
        a.lines[k] = (k < p.d) ? p.ws.lines[k] : nullptr;
        a.skel[k] = (k < p.d) ? p.ws.Y[1u << k] : nullptr;
        a.perm[k] = (perm && k < p.d) ? perm[k] : k;
    }
    a.Sp = p.dSp;
    a.scal = p.ws.scal;
    a.mode = mode;
    return a;
}

void launch_crosspoints(const Plan &p, int mode, const int *perm, const double *const *res,
                        hipStream_t st) {
    SkelArgs a = skel_args(p, mode, perm, res);
    const long long nA = (p.d == 2) ? (long long)p.Nc * p.Nc : (long long)p.Nc * p.Nc * p.Nf;
    const long long total = (p.d == 2) ? nA : 2 * nA;
    long long blocks = (total + 255) / 256;
    if (blocks > 1024) blocks = 1024;
    hipLaunchKernelGGL(k_crosspoints, dim3((unsigned)blocks, p.d, 1), dim3(256), 0, st, p.geo, a);
    if (p.d == 3) {
        long long b2 = (nA + 255) / 256;
        if (b2 > 1024) b2 = 1024;
        hipLaunchKernelGGL(k_lines_residual, dim3((unsigned)b2, p.d, 1), dim3(256), 0, st, p.geo, a);
    }
}

void launch_merge(const Plan &p, int mode, const int *perm, const double *const *res,
                  hipStream_t st) {
    SkelArgs a = skel_args(p, mode, perm, res);
    long long blocks = (p.mesh[1].size + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_merge, dim3((unsigned)blocks, p.d, 1), dim3(256), 0, st, p.geo, a);
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
};

template <int D, int NH>
__global__ __launch_bounds__(256) void k_filler(Geo g, FillArgs a) {
    extern __shared__ double lds[];
    // NH > 0: hole edge length known at compile time (constant-divisor index arithmetic)
    const int nh = (NH > 0) ? NH : g.n - 1;
    const int n = nh + 1, Nf = g.Nf, Nc = g.Nc;
    int npts = 1, st[kMaxD] = {1, 1, 1};
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
    int tt[kMaxD] = {0, 0, 0};
    {
        int rem = blockIdx.x;
        for (int j = 0; j < D; ++j) {
            tt[j] = rem % (Nc + 1);
            rem /= (Nc + 1);
        }
    }
    // 1) hole right-hand side
    for (int o = tid; o < npts; o += 256) {
        int l[kMaxD] = {0, 0, 0}, i[kMaxD] = {0, 0, 0};
        int rem = o;
        for (int j = 0; j < D; ++j) {
            l[j] = rem % nh;
            rem /= nh;
            i[j] = n * tt[j] + l[j];
        }
        long long f = i[0] + (long long)Nf * (i[1] + (long long)Nf * (D == 3 ? i[2] : 0));
        double v = a.bff ? a.bff[f] : 0.0;
        for (int j = 0; j < D; ++j) {
            if (l[j] == 0 && tt[j] > 0) {
                int q[kMaxD] = {i[0], i[1], i[2]};
                q[j] -= 1;
                v -= g.fine[j].a * a.skel[j][canon_offset(a.mk[j], q, n)];
            }
            if (l[j] == nh - 1 && tt[j] < Nc) {
                int q[kMaxD] = {i[0], i[1], i[2]};
                q[j] += 1;
                v -= g.fine[j].c * a.skel[j][canon_offset(a.mk[j], q, n)];
            }
        }
        bufA[o] = v;
    }
    __syncthreads();
    double *cur = bufA, *oth = bufB;
    // 2) forward transforms
    for (int q = 0; q < a.ntr; ++q) {
        const int j = a.tr[q];
        const double *Wq = mat + q * (2 * nh * nh + nh);
        for (int o = tid; o < npts; o += 256) {
            const int m = (o / st[j]) % nh;
            const int base = o - m * st[j];
            double acc = 0.0;
            for (int l = 0; l < nh; ++l) acc += Wq[m * nh + l] * cur[base + l * st[j]];
            oth[o] = acc;
        }
        __syncthreads();
        double *t = cur;
        cur = oth;
        oth = t;
    }
    // 3) line elimination along the line axis, one thread per line
    {
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
            const int sL = st[L];
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
            const int ii = (o / st[j]) % nh;
            const int base = o - ii * st[j];
            double acc = 0.0;
            for (int m = 0; m < nh; ++m) acc += Vq[ii * nh + m] * cur[base + m * st[j]];
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
        int l[kMaxD] = {0, 0, 0}, i[kMaxD] = {0, 0, 0};
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
            v = cur[lo];
        } else {
            int j = 0;
            while (l[j] != n - 1) ++j;
            v = a.skel[j][canon_offset(a.mk[j], i, n)];
        }
        const long long f = i[0] + (long long)Nf * (i[1] + (long long)Nf * (D == 3 ? i[2] : 0));
        a.out[f] = v;
    }
}

void launch_filler(const Plan &p, const double *bff, double *out, hipStream_t st) {
    FillArgs a;
    const int d = p.d, nh = p.n - 1;
    for (int j = 0; j < kMaxD; ++j) {
        a.skel[j] = (j < d) ? p.ws.Y[1u << j] : nullptr;
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
    int npts = 1;
    for (int j = 0; j < d; ++j) npts *= nh;
    const size_t lds = (size_t)(2 * npts + a.ntr * (2 * nh * nh + nh)) * sizeof(double);
    int tiles = 1;
    for (int j = 0; j < d; ++j) tiles *= (p.Nc + 1);
    const dim3 grid(tiles), blk(256);
#define ASDSM_FILL(DD, NHV) hipLaunchKernelGGL((k_filler<DD, NHV>), grid, blk, lds, st, p.geo, a)
    if (d == 2) {
        switch (nh) {
            case 1: ASDSM_FILL(2, 1); break;
            case 3: ASDSM_FILL(2, 3); break;
            case 7: ASDSM_FILL(2, 7); break;
            case 15: ASDSM_FILL(2, 15); break;
            case 31: ASDSM_FILL(2, 31); break;
            default: ASDSM_FILL(2, 0); break;
        }
    } else {
        switch (nh) {
            case 1: ASDSM_FILL(3, 1); break;
            case 3: ASDSM_FILL(3, 3); break;
            case 7: ASDSM_FILL(3, 7); break;
            case 15: ASDSM_FILL(3, 15); break;
            default: ASDSM_FILL(3, 0); break;
        }
    }
#undef ASDSM_FILL
}

}  // namespace asdsm
