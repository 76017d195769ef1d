// Tensor-product submesh solvers (Algorithm 1 steps 1.1-1.3 and the error phase).
//
// The operator of a box is a Kronecker sum of 1D tridiagonal Toeplitz operators (Section 2.3).
// Every fine axis (|cell Peclet| < 1) is diagonalised: its mode transforms V^-1 and V are dense
// N_f x N_f contractions executed as FP64 MFMA GEMMs (v_mfma_f64_16x16x4f64).  What remains per mode
// is a problem on the coarse axes only:
//   * one coarse axis (the anisotropic meshes): a tridiagonal system, solved by Thomas elimination
//     (each thread owns one mode; the coarse line is short);
//   * two or more coarse axes (intersection meshes, coarse mesh): a small dense system whose
//     inverse is precomputed per mode on the host (LU with partial pivoting) and applied here.
#include "device_common.hpp"
#include "kernels.hpp"

namespace asdsm {

// ---------------------------------------------------------------------------------------------
// Batched FP64 GEMM on MFMA.  Block = 4 waves, block tile 32 x 32, each wave one 16 x 16 MFMA tile.
// The A (32 x 64) and B (64 x 32) panels of each K chunk are staged in LDS with fully coalesced
// loads (a wave reads 64 consecutive doubles along the contiguous index of the operand), so every
// cache line is fetched once per block; MFMA operands are then read from padded, conflict-free LDS.
// Operand layout of v_mfma_f64_16x16x4f64 (lane l, 0..63):
//   A: row l%16, k l/16;  B: k l/16, col l%16;  D[v]: row l/16 + 4v, col l%16.
// ---------------------------------------------------------------------------------------------
constexpr int GKC = 64;  // K chunk

__global__ __launch_bounds__(256) void k_gemm_f64(GemmJob job) {
    __shared__ double sA[32][GKC + 1];
    __shared__ double sB[GKC][32 + 1];
    const int box = blockIdx.z / job.nbatch;
    const int bat = blockIdx.z % job.nbatch;
    const double *__restrict__ A = job.A[box] + (long long)bat * job.sAb;
    const double *__restrict__ B = job.B[box] + (long long)bat * job.sBb;
    const int m0 = blockIdx.y * 32, n0 = blockIdx.x * 32;
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int wm = w & 1, wn = w >> 1;
    const bool a_kfast = (job.sAk == 1);
    const bool b_kfast = (job.sBk == 1);
    double4_t acc = {0.0, 0.0, 0.0, 0.0};
    for (int k0 = 0; k0 < job.K; k0 += GKC) {
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int e = t + 256 * j;  // 0 .. 2047
            int ii, kk;
            if (a_kfast) { ii = e >> 6; kk = e & 63; } else { kk = e >> 5; ii = e & 31; }
            const int gi = m0 + ii, gk = k0 + kk;
            sA[ii][kk] = (gi < job.M && gk < job.K) ? A[(long long)gi * job.sAi + (long long)gk * job.sAk] : 0.0;
            int nn;
            if (b_kfast) { nn = e >> 6; kk = e & 63; } else { kk = e >> 5; nn = e & 31; }
            const int gn = n0 + nn, gk2 = k0 + kk;
            sB[kk][nn] = (gn < job.N && gk2 < job.K) ? B[(long long)gk2 * job.sBk + (long long)gn * job.sBn] : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < GKC; kk += 4) {
            const double a = sA[wm * 16 + (lane & 15)][kk + (lane >> 4)];
            const double b = sB[kk + (lane >> 4)][wn * 16 + (lane & 15)];
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
        }
        __syncthreads();
    }
    double *__restrict__ C = job.C[box] + (long long)bat * job.sCb;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int gi = m0 + wm * 16 + (lane >> 4) + 4 * v;
        const int gn = n0 + wn * 16 + (lane & 15);
        if (gi < job.M && gn < job.N) {
            double *c = C + (long long)gi * job.sCi + (long long)gn * job.sCn;
            *c = job.accum ? *c + acc[v] : acc[v];
        }
    }
}

void launch_gemm(const GemmJob &job, hipStream_t st) {
    dim3 grid((job.N + 31) / 32, (job.M + 31) / 32, job.nbox * job.nbatch);
    hipLaunchKernelGGL(k_gemm_f64, grid, dim3(256), 0, st, job);
}

// ---------------------------------------------------------------------------------------------
// Thomas elimination along the coarse axis, one thread per mode, boxes along blockIdx.y.  Lines of
// up to NCR points stay in registers (loads issued together); longer lines use the scratch array.
// ---------------------------------------------------------------------------------------------
template <int NCR>
__global__ __launch_bounds__(256) void k_line(LineJob job) {
    const int box = blockIdx.y;
    const long long m = (long long)blockIdx.x * 256 + threadIdx.x;
    if (m >= job.nmodes) return;
    double *__restrict__ X = job.X[box];
    double *__restrict__ S = job.scratch[box];
    const Tri t = job.t[box];
    const int ma = (int)(m % job.ext_a);
    const long long mb = m / job.ext_a;
    double sigma = job.mu_a[box][ma];
    if (job.mu_b[box]) sigma += job.mu_b[box][mb];
    const long long st = job.nmodes;
    const double diag = t.b + sigma;
    const int nc = job.ncoarse;
    if (NCR > 0) {
        double f[NCR > 0 ? NCR : 1], cp[NCR > 0 ? NCR : 1];
#pragma unroll
        for (int c = 0; c < NCR; ++c)
            if (c < nc) f[c] = X[m + st * c];
        double den = diag;
        cp[0] = t.c / den;
        f[0] = f[0] / den;
#pragma unroll
        for (int c = 1; c < NCR; ++c)
            if (c < nc) {
                den = diag - t.a * cp[c - 1];
                f[c] = (f[c] - t.a * f[c - 1]) / den;
                cp[c] = t.c / den;
            }
#pragma unroll
        for (int c = NCR - 2; c >= 0; --c)
            if (c < nc - 1) f[c] = f[c] - cp[c] * f[c + 1];
#pragma unroll
        for (int c = 0; c < NCR; ++c)
            if (c < nc) X[m + st * c] = f[c];
        return;
    }
    double den = diag;
    double cq = t.c / den;
    double dp = X[m] / den;
    S[m] = cq;
    X[m] = dp;
    for (int c = 1; c < nc; ++c) {
        den = diag - t.a * cq;
        const double fc = X[m + st * c];
        dp = (fc - t.a * dp) / den;
        cq = t.c / den;
        S[m + st * c] = cq;
        X[m + st * c] = dp;
    }
    double x = dp;
    for (int c = nc - 2; c >= 0; --c) {
        x = X[m + st * c] - S[m + st * c] * x;
        X[m + st * c] = x;
    }
}

void launch_line(const LineJob &job, hipStream_t st) {
    dim3 grid((unsigned)((job.nmodes + 255) / 256), job.nbox, 1);
    if (job.ncoarse <= 7)
        hipLaunchKernelGGL(k_line<7>, grid, dim3(256), 0, st, job);
    else if (job.ncoarse <= 15)
        hipLaunchKernelGGL(k_line<15>, grid, dim3(256), 0, st, job);
    else if (job.ncoarse <= 31)
        hipLaunchKernelGGL(k_line<31>, grid, dim3(256), 0, st, job);
    else
        hipLaunchKernelGGL(k_line<0>, grid, dim3(256), 0, st, job);
}

// ---------------------------------------------------------------------------------------------
// Per-mode dense solve: out[m + nmodes*e] = sum_e' inv[m][e][e'] in[m + nmodes*e'].
// ---------------------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_dense_modes(long long nmodes, int B,
                                                     const double *__restrict__ inv,
                                                     const double *__restrict__ in,
                                                     double *__restrict__ out, int accum) {
    const long long t = (long long)blockIdx.x * 256 + threadIdx.x;
    if (t >= nmodes * B) return;
    const long long m = t % nmodes;
    const int row = (int)(t / nmodes);
    const double *__restrict__ Mi = inv + (m * B + row) * (long long)B;
    double acc = 0.0;
    for (int e = 0; e < B; ++e) acc += Mi[e] * in[m + nmodes * e];
    out[m + nmodes * row] = accum ? out[m + nmodes * row] + acc : acc;
}

void launch_dense_modes(long long nmodes, int B, const double *inv, const double *in, double *out,
                        int accum, hipStream_t st) {
    const long long n = nmodes * B;
    hipLaunchKernelGGL(k_dense_modes, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, nmodes, B,
                       inv, in, out, accum);
}

// ---------------------------------------------------------------------------------------------
// ||e_k||^2 of each anisotropic box and the normalisation factor 1/||e_k|| (Algorithm 1 steps
// 2.1/2.2; a zero vector is left unscaled).
// ---------------------------------------------------------------------------------------------
constexpr int kNormBlocks = 128;

__global__ __launch_bounds__(256) void k_box_norms(BoxPtrs X, long long size, double *partials) {
    const int k = blockIdx.y;
    const double *__restrict__ x = X.p[k];
    double acc = 0.0;
    for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < size; i += (long long)gridDim.x * 256)
        acc += x[i] * x[i];
    double vals[1] = {acc};
    block_partials<256, 1>(vals, partials + (size_t)k * kNormBlocks, blockIdx.x);
}

void launch_box_norms(const Plan &p, const double *const *sol, hipStream_t st) {
    BoxPtrs bx;
    for (int k = 0; k < kMaxD; ++k) bx.p[k] = (k < p.d) ? const_cast<double *>(sol[1u << k]) : nullptr;
    const long long size = p.mesh[1].size;
    hipLaunchKernelGGL(k_box_norms, dim3(kNormBlocks, p.d, 1), dim3(256), 0, st, bx, size, p.ws.partials);
    launch_finalize(p, kNormBlocks, kFinBoxNorms, p.d, st);
}

// ---------------------------------------------------------------------------------------------
// Mesh residual out = f - A_S x (zero Dirichlet data) in the canonical layout of M_S.
// ---------------------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_box_residual(Geo g, BoxResJob job) {
    const int box = blockIdx.y;
    const MeshDesc &m = job.m[box];
    const double *__restrict__ f = job.f[box];
    const double *__restrict__ x = job.x[box];
    double *__restrict__ out = job.out[box];
    for (long long idx = (long long)blockIdx.x * 256 + threadIdx.x; idx < m.size; idx += (long long)gridDim.x * 256) {
        const double xc = x[idx];
        double ax = 0.0;
        long long rem = idx;
        for (int q = 0; q < m.nd; ++q) {
            const int pos = (int)(rem % m.ext[q]);
            rem /= m.ext[q];
            const int j = m.ax[q];
            const Tri t = (q < m.nfine) ? g.fine[j] : g.coarse[j];
            ax += t.b * xc;
            if (pos > 0) ax += t.a * x[idx - m.stride[q]];
            if (pos < m.ext[q] - 1) ax += t.c * x[idx + m.stride[q]];
        }
        out[idx] = f[idx] - ax;
    }
}

void launch_box_residual(const Plan &p, const BoxResJob &job, hipStream_t st) {
    long long mx = 0;
    for (int q = 0; q < job.nbox; ++q) mx = job.m[q].size > mx ? job.m[q].size : mx;
    long long blocks = (mx + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_box_residual, dim3((unsigned)blocks, job.nbox, 1), dim3(256), 0, st, p.geo, job);
}

struct AxpyJob {
    double *y[kMaxD];
    const double *x[kMaxD];
};

__global__ __launch_bounds__(256) void k_axpy(AxpyJob job, long long n) {
    double *__restrict__ y = job.y[blockIdx.y];
    const double *__restrict__ x = job.x[blockIdx.y];
    for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long long)gridDim.x * 256) y[i] += x[i];
}

void launch_axpy(double *const *y, const double *const *x, long long n, int nbox, hipStream_t st) {
    AxpyJob job{};
    for (int q = 0; q < nbox; ++q) {
        job.y[q] = y[q];
        job.x[q] = x[q];
    }
    long long blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_axpy, dim3((unsigned)blocks, nbox, 1), dim3(256), 0, st, job, n);
}

// ---------------------------------------------------------------------------------------------
// Calibration helpers: a reproducible random right-hand side and sums of squares.
// ---------------------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_fill_random(double *x, long long n, unsigned long long seed) {
    for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long long)gridDim.x * 256) {
        unsigned long long z = seed + 0x9E3779B97F4A7C15ull * (unsigned long long)(i + 1);
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        z = z ^ (z >> 31);
        x[i] = (double)(z >> 11) * (2.0 / 9007199254740992.0) - 1.0;
    }
}

void launch_fill_random(double *x, long long n, uint64_t seed, hipStream_t st) {
    long long blocks = (n + 255) / 256;
    if (blocks > 2048) blocks = 2048;
    hipLaunchKernelGGL(k_fill_random, dim3((unsigned)blocks), dim3(256), 0, st, x, n, (unsigned long long)seed);
}

struct SumsqJob {
    const double *x[kMaxD];
    long long n[kMaxD];
};

__global__ __launch_bounds__(256) void k_sumsq(SumsqJob job, double *partials) {
    const int k = blockIdx.y;
    const double *__restrict__ x = job.x[k];
    double acc = 0.0;
    for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < job.n[k]; i += (long long)gridDim.x * 256)
        acc += x[i] * x[i];
    double vals[1] = {acc};
    block_partials<256, 1>(vals, partials + (size_t)k * kNormBlocks, blockIdx.x);
}

void launch_sumsq(const Plan &p, const double *const *x, const long long *n, int nbox, hipStream_t st) {
    SumsqJob job{};
    for (int k = 0; k < nbox; ++k) {
        job.x[k] = x[k];
        job.n[k] = n[k];
    }
    hipLaunchKernelGGL(k_sumsq, dim3(kNormBlocks, nbox, 1), dim3(256), 0, st, job, p.ws.partials);
    launch_finalize(p, kNormBlocks, kFinBoxNorms, nbox, st);
}

}  // namespace asdsm
