// Block cyclic reduction along the line axis of a submesh (Section 2.3 operators, Algorithm 1's
// submesh solves), for fine axes that fast diagonalisation cannot handle: |cell Peclet| >= 1
// (complex spectrum) or an eigenvector matrix too ill-conditioned for FP64.
//
// The submesh's other fine axes are diagonalised first (mode transforms, k_gemm_f64), so every mode
// of them leaves an independent system along the line axis w.  Its unknowns at position i are the
// points of the coarse block (all coarse axes, flattened), x_i in R^NB:
//     a_w x_{i-1} + B x_i + c_w x_{i+1} = f_i,   B = T_block + (b_w + sigma_mode) I,
// with T_block the Kronecker sum of the coarse axes' operators.  The line has N = 2^L - 1 positions,
// so odd-even (cyclic) reduction closes without boundary cases: level l keeps the equations at
// multiples of 2^(l+1) and eliminates the odd multiples of 2^l,
//     f_i <- f_i - P_l f_(i-s) - Q_l f_(i+s)               (forward, s = 2^l)
//     x_i  = G_l f_i - P_l x_(i-s) - Q_l x_(i+s)            (back substitution)
// with G_l = B_l^-1, P_l = G_l A_l, Q_l = G_l C_l and the reduced blocks of every level precomputed
// per mode on the host (all blocks are functions of T_block, so they commute).  2 (L - 1) + 1
// dependent levels instead of 2 N for block Thomas; every level is a batch of independent NB x NB
// matrix-vector products.
//
// One workgroup holds `tm` consecutive modes: the kept equations of level 0 (half the line) and the
// current level's matrices are staged in LDS; a thread owns one (mode, equation) row-block at a
// time, so every level is updated in place without hazards.
#include <algorithm>
#include <atomic>

#include "device_common.hpp"
#include "kernels.hpp"

namespace asdsm {

namespace {

// Row r of G f - P x1 - Q x2 (f[r] - ... when G is nullptr), NB x NB row-major matrices.  The
// operands are in registers (compile-time indices), the row index is a run-time value, so the rows
// can be produced one at a time without holding the whole result.
template <int NB>
__device__ __forceinline__ double cr_row(int r, const double *__restrict__ G, const double *__restrict__ P,
                                         const double *__restrict__ Q, const double (&f)[NB],
                                         const double (&x1)[NB], const double (&x2)[NB]) {
    double acc = 0.0;
    if (G) {
#pragma unroll
        for (int c = 0; c < NB; ++c) acc += G[r * NB + c] * f[c];
    } else {
#pragma unroll
        for (int c = 0; c < NB; ++c)
            if (c == r) acc = f[c];
    }
#pragma unroll
    for (int c = 0; c < NB; ++c) acc -= P[r * NB + c] * x1[c];
#pragma unroll
    for (int c = 0; c < NB; ++c) acc -= Q[r * NB + c] * x2[c];
    return acc;
}

template <int NB>
__global__ __launch_bounds__(256) void k_block_cr(CrJob job) {
    if (job.gate && *job.gate) return;
    extern __shared__ double lds[];
    const int box = blockIdx.y;
    const CrBox &bx = job.box[box];
    const long long mode0 = (long long)blockIdx.x * job.tm;
    if (mode0 >= bx.nmodes) return;
    const int tm = (int)((bx.nmodes - mode0) < job.tm ? (bx.nmodes - mode0) : job.tm);
    const int N = job.N, L = job.L;
    const int Nk = (N - 1) / 2;                       // kept equations of level 0 (1-based i = 2j)
    double *S = lds;                                  // [tm][Nk][NB]
    double *M = lds + (size_t)job.tm * Nk * NB;       // [tm][3][NB*NB] matrices of the level
    const double *src = bx.src;  // may be dst (in place): no restrict
    double *dst = bx.dst;
    const int tid = threadIdx.x;
    constexpr int MM = NB * NB;
    // global offset of (mode, position i0 (0-based), coarse c)
    auto goff = [&](long long mode, int i0) -> long long {
        const long long m0 = mode % bx.mext0, m1 = mode / bx.mext0;
        return m0 * bx.ms0 + m1 * bx.ms1 + (long long)i0 * bx.sw;
    };
    auto load_mats = [&](int l) {
        for (int e = tid; e < tm * 3 * MM; e += 256) {
            const int ml = e / (3 * MM), rem = e - ml * 3 * MM;
            M[(size_t)ml * 3 * MM + rem] = bx.tab[((size_t)(mode0 + ml) * L + l) * 3 * MM + rem];
        }
    };
    // task order: modes fastest when they are contiguous in memory, else the line position
    const bool modes_fast = bx.ms0 == 1;

    // ---- level 0, forward: S[j] = f_2j - P0 f_(2j-1) - Q0 f_(2j+1) (1-based), read from src
    load_mats(0);
    __syncthreads();
    for (int t = tid; t < tm * Nk; t += 256) {
        const int ml = modes_fast ? t % tm : t / Nk;
        const int j = modes_fast ? t / tm : t % Nk;  // 0-based kept index: i = 2(j+1), 0-based 2j+1
        const long long base = goff(mode0 + ml, 2 * j + 1);
        double f[NB], x1[NB], x2[NB];
#pragma unroll
        for (int c = 0; c < NB; ++c) {
            f[c] = src[base + c * bx.sc];
            x1[c] = src[base - bx.sw + c * bx.sc];
            x2[c] = src[base + bx.sw + c * bx.sc];
        }
        const double *Mm = M + (size_t)ml * 3 * MM;
        double *sj = S + ((size_t)ml * Nk + j) * NB;
#pragma unroll 1
        for (int r = 0; r < NB; ++r) sj[r] = cr_row<NB>(r, nullptr, Mm + MM, Mm + 2 * MM, f, x1, x2);
    }
    __syncthreads();
    // ---- levels 1 .. L-2, forward, on the kept equations (even i, stored at j = i/2 - 1)
    for (int l = 1; l <= L - 2; ++l) {
        load_mats(l);
        __syncthreads();
        const int step = 1 << l;              // neighbour distance in i; in j-units step/2
        const int nkeep = (1 << (L - l - 1)) - 1;
        for (int t = tid; t < tm * nkeep; t += 256) {
            const int ml = t % tm, q = t / tm;
            const int i = (q + 1) * 2 * step;  // 1-based kept index of this level
            const int j = i / 2 - 1, h = step / 2;
            double *Sm = S + (size_t)ml * Nk * NB;
            double f[NB], x1[NB], x2[NB];
#pragma unroll
            for (int c = 0; c < NB; ++c) {
                f[c] = Sm[j * NB + c];
                x1[c] = Sm[(j - h) * NB + c];
                x2[c] = Sm[(j + h) * NB + c];
            }
            const double *Mm = M + (size_t)ml * 3 * MM;
#pragma unroll 1
            for (int r = 0; r < NB; ++r) Sm[j * NB + r] = cr_row<NB>(r, nullptr, Mm + MM, Mm + 2 * MM, f, x1, x2);
        }
        __syncthreads();
    }
    // ---- the last equation (i = 2^(L-1)): x = G f
    load_mats(L - 1);
    __syncthreads();
    if (L >= 2) {
        for (int ml = tid; ml < tm; ml += 256) {
            const int j = (1 << (L - 2)) - 1;
            double *Sm = S + (size_t)ml * Nk * NB;
            double f[NB], z[NB];
#pragma unroll
            for (int c = 0; c < NB; ++c) {
                f[c] = Sm[j * NB + c];
                z[c] = 0.0;
            }
            const double *Mm = M + (size_t)ml * 3 * MM;
#pragma unroll 1
            for (int r = 0; r < NB; ++r) Sm[j * NB + r] = cr_row<NB>(r, Mm, Mm + MM, Mm + 2 * MM, f, z, z);
        }
    }
    __syncthreads();
    // ---- back substitution, levels L-2 .. 1, in LDS
    for (int l = L - 2; l >= 1; --l) {
        load_mats(l);
        __syncthreads();
        const int step = 1 << l;
        const int nel = 1 << (L - l - 1);     // eliminated equations of this level
        for (int t = tid; t < tm * nel; t += 256) {
            const int ml = t % tm, q = t / tm;
            const int i = (2 * q + 1) * step;  // 1-based
            const int j = i / 2 - 1, h = step / 2;
            double *Sm = S + (size_t)ml * Nk * NB;
            double f[NB], x1[NB], x2[NB];
            const bool has1 = i - step >= 1, has2 = i + step <= N;
#pragma unroll
            for (int c = 0; c < NB; ++c) {
                f[c] = Sm[j * NB + c];
                x1[c] = has1 ? Sm[(j - h) * NB + c] : 0.0;
                x2[c] = has2 ? Sm[(j + h) * NB + c] : 0.0;
            }
            const double *Mm = M + (size_t)ml * 3 * MM;
#pragma unroll 1
            for (int r = 0; r < NB; ++r) Sm[j * NB + r] = cr_row<NB>(r, Mm, Mm + MM, Mm + 2 * MM, f, x1, x2);
        }
        __syncthreads();
    }
    // ---- level 0 back substitution: odd i from src (their level-0 right-hand sides) and the kept
    // neighbours; every position written to dst (added when accumulating)
    load_mats(0);
    __syncthreads();
    for (int t = tid; t < tm * N; t += 256) {
        const int ml = modes_fast ? t % tm : t / N;
        const int i0 = modes_fast ? t / tm : t % N;  // 0-based position; 1-based i = i0 + 1
        const long long base = goff(mode0 + ml, i0);
        const double *Sm = S + (size_t)ml * Nk * NB;
        const int acc = job.accum;
        if ((i0 & 1) == 1) {  // even 1-based i: kept, solved in LDS
            const int j = (i0 + 1) / 2 - 1;
#pragma unroll 1
            for (int r = 0; r < NB; ++r) {
                const long long a = base + r * bx.sc;
                const double v = Sm[j * NB + r];
                dst[a] = acc ? dst[a] + v : v;
            }
        } else {
            // kept neighbours: 1-based i-1 = i0 at j = i0/2 - 1, i+1 = i0 + 2 at j = i0/2; the whole
            // right-hand side row-block is read before any of it is overwritten (src may be dst)
            double f[NB], x1[NB], x2[NB];
            const bool has1 = i0 >= 1, has2 = i0 + 1 < N;
#pragma unroll
            for (int c = 0; c < NB; ++c) {
                f[c] = src[base + c * bx.sc];
                x1[c] = has1 ? Sm[(i0 / 2 - 1) * NB + c] : 0.0;
                x2[c] = has2 ? Sm[(i0 / 2) * NB + c] : 0.0;
            }
            const double *Mm = M + (size_t)ml * 3 * MM;
#pragma unroll 1
            for (int r = 0; r < NB; ++r) {
                const long long a = base + r * bx.sc;
                const double v = cr_row<NB>(r, Mm, Mm + MM, Mm + 2 * MM, f, x1, x2);
                dst[a] = acc ? dst[a] + v : v;
            }
        }
    }
}

// The fast form: the whole line of `tm` modes and every level's matrices of those modes staged in
// LDS once (one burst of global loads, the matrices of consecutive modes being contiguous), then
// the 2 (L - 1) + 1 levels run from LDS.  Thread (mode, row r, group e) produces row r of the
// equations q = e, e + E, ... of a level (E = 256 / (tm RB) groups, RB = NB rounded up to a power
// of two), so a level costs about (equations / E) * 2 NB multiply-adds per thread.  Forward
// reduction writes only the thread's own row of a kept equation and reads eliminated neighbours,
// so it runs in place; back substitution reads a whole row-block of the equation it overwrites, so
// its results are held in registers until a barrier.  The solved line is copied to dst at the end.
constexpr int kCrMaxPerThread = 16;
constexpr int kCrLd = 5;  // staging loads per thread and array in flight together (k_block_cr2)

template <int NB, int RB>
__global__ __launch_bounds__(256) void k_block_cr2(CrJob job) {
    // the stopping flag is read with the first loads and tested once they have arrived
    const int gv = gate_value(job.gate);
    extern __shared__ double lds[];
    const int box = blockIdx.y;
    const CrBox &bx = job.box[box];
    const long long mode0 = (long long)blockIdx.x * job.tm;
    if (mode0 >= bx.nmodes) return;
    const int tmw = job.tm;                                  // modes per workgroup (layout)
    const int tm = (int)((bx.nmodes - mode0) < tmw ? (bx.nmodes - mode0) : tmw);
    const int N = job.N, L = job.L, tid = threadIdx.x;
    constexpr int MM = NB * NB;
    double *D = lds;                                         // [tmw][N][NB]
    double *Mt = lds + (size_t)tmw * N * NB;                 // [tmw][L][3][MM]
    __shared__ long long mbase[8];                           // offset of each mode's line
    if (tid < tm) {
        const long long mode = mode0 + tid;
        mbase[tid] = (mode % bx.mext0) * bx.ms0 + (mode / bx.mext0) * bx.ms1;
    }
    lds_barrier();  // the offsets (nothing is in flight yet)
    const int mats = tm * L * 3 * MM;
    const double *tsrc = bx.tab + (size_t)mode0 * L * 3 * MM;
    const bool modes_fast = bx.ms0 == 1;
    const long long sw = bx.sw, sc = bx.sc;
    // element t of the coalesced order: modes fastest when they are contiguous, else the line
    auto elem = [&](int t, int &ml, int &i, int &c) {
        if (modes_fast) {
            ml = t % tm;
            const int rest = t / tm;
            i = rest % N;
            c = rest / N;
        } else {
            i = t % N;
            const int rest = t / N;
            ml = rest % tm;
            c = rest / tm;
        }
    };
    // the matrices and the lines in rounds of kCrLd values of each per thread: every load of a
    // round is in flight before the first LDS store (a lane beyond the end reads element 0 and
    // drops it), so the staging waits for memory once per round instead of once per value
    const int nline = tm * N * NB;
    for (int r0 = 0; r0 < mats || r0 < nline; r0 += 256 * kCrLd) {
        double tv[kCrLd], lv[kCrLd];
        int li[kCrLd];
#pragma unroll
        for (int u = 0; u < kCrLd; ++u) {
            const int e = r0 + u * 256 + tid;
            tv[u] = tsrc[e < mats ? e : 0];
            int ml, i, c;
            elem(e < nline ? e : 0, ml, i, c);
            li[u] = (ml * N + i) * NB + c;
            lv[u] = bx.src[mbase[ml] + i * sw + c * sc];
        }
#pragma unroll
        for (int u = 0; u < kCrLd; ++u) {
            const int e = r0 + u * 256 + tid;
            if (e < mats) Mt[e] = tv[u];
            if (e < nline) D[li[u]] = lv[u];
        }
    }
    __syncthreads();
    if (!flag_clear(gv)) return;  // block-uniform
    const int E = 256 / (tmw * RB);
    const int ml = tid / (RB * E), rem = tid % (RB * E), r = rem % RB, eg = rem / RB;
    const bool act = ml < tm && r < NB;
    double *Dm = D + (size_t)(ml < tm ? ml : 0) * N * NB;
    const double *Mm = Mt + (size_t)(ml < tm ? ml : 0) * L * 3 * MM;
    // ---- forward reduction, levels 0 .. L-2: f_i[r] -= P[r,:] f_(i-s) + Q[r,:] f_(i+s)
    for (int l = 0; l <= L - 2; ++l) {
        const int step = 1 << l, nkeep = (1 << (L - l - 1)) - 1;
        if (act) {
            double pr[NB], qr[NB];
            const double *P = Mm + ((size_t)l * 3 + 1) * MM + r * NB, *Q = P + MM;
#pragma unroll
            for (int c = 0; c < NB; ++c) {
                pr[c] = P[c];
                qr[c] = Q[c];
            }
            for (int q = eg; q < nkeep; q += E) {
                const int i0 = (q + 1) * 2 * step - 1;   // 0-based
                const double *a = Dm + (size_t)(i0 - step) * NB, *b = Dm + (size_t)(i0 + step) * NB;
                // two independent chains (the P and the Q products) shorten the dependent FMAs
                double s1 = 0.0, s2 = 0.0;
#pragma unroll
                for (int c = 0; c < NB; ++c) {
                    s1 += pr[c] * a[c];
                    s2 += qr[c] * b[c];
                }
                Dm[(size_t)i0 * NB + r] = Dm[(size_t)i0 * NB + r] - (s1 + s2);
            }
        }
        __syncthreads();
    }
    // ---- back substitution, levels L-1 .. 0: x_i[r] = G[r,:] f_i - P[r,:] x_(i-s) - Q[r,:] x_(i+s)
    for (int l = L - 1; l >= 0; --l) {
        const int step = 1 << l, nel = 1 << (L - l - 1);
        double res[kCrMaxPerThread];
        if (act) {
            double gr[NB], pr[NB], qr[NB];
            const double *G = Mm + ((size_t)l * 3) * MM + r * NB, *P = G + MM, *Q = G + 2 * MM;
#pragma unroll
            for (int c = 0; c < NB; ++c) {
                gr[c] = G[c];
                pr[c] = P[c];
                qr[c] = Q[c];
            }
#pragma unroll
            for (int k = 0; k < kCrMaxPerThread; ++k) {
                const int q = eg + k * E;
                if (q >= nel) break;
                const int i = (2 * q + 1) * step;        // 1-based
                const double *f = Dm + (size_t)(i - 1) * NB;
                // three independent chains (G, P and Q products)
                double s0 = 0.0, s1 = 0.0, s2 = 0.0;
#pragma unroll
                for (int c = 0; c < NB; ++c) s0 += gr[c] * f[c];
                if (i - step >= 1) {
                    const double *a = Dm + (size_t)(i - 1 - step) * NB;
#pragma unroll
                    for (int c = 0; c < NB; ++c) s1 += pr[c] * a[c];
                }
                if (i + step <= N) {
                    const double *b = Dm + (size_t)(i - 1 + step) * NB;
#pragma unroll
                    for (int c = 0; c < NB; ++c) s2 += qr[c] * b[c];
                }
                res[k] = s0 - (s1 + s2);
            }
        }
        __syncthreads();
        if (act) {
#pragma unroll
            for (int k = 0; k < kCrMaxPerThread; ++k) {
                const int q = eg + k * E;
                if (q >= nel) break;
                const int i = (2 * q + 1) * step;
                Dm[(size_t)(i - 1) * NB + r] = res[k];
            }
        }
        __syncthreads();
    }
    // ---- the solved line to dst (added when accumulating), in the load's coalesced order
    const int acc = job.accum;
    for (int t = tid; t < tm * N * NB; t += 256) {
        int mlw, i, c;
        elem(t, mlw, i, c);
        const long long a = mbase[mlw] + i * sw + c * sc;
        const double v = D[(mlw * N + i) * NB + c];
        bx.dst[a] = acc ? bx.dst[a] + v : v;
    }
}

// Any block size (intersection meshes of the initial guess, whose coarse block holds N_c^|S|
// points): one workgroup per mode, the line solved in place in dst (canonical layout) after src is
// copied there; one (equation, row) pair per task.  Back substitution reads a whole row-block of the
// equation it writes, so each chunk of tasks is computed into registers, then written after a
// barrier.  No accumulation (the host never asks for it here).
constexpr int kCrChunk = 16;

__global__ __launch_bounds__(256) void k_block_cr_global(CrJob job) {
    if (job.gate && *job.gate) return;
    const int box = blockIdx.y;
    const CrBox &bx = job.box[box];
    const long long mode = blockIdx.x;
    if (mode >= bx.nmodes) return;
    const int N = job.N, L = job.L, NB = job.NB, tid = threadIdx.x;
    const long long MM = (long long)NB * NB;
    const double *tabm = bx.tab + (size_t)mode * L * 3 * MM;
    const long long m0 = mode % bx.mext0, m1 = mode / bx.mext0;
    const long long gbase = m0 * bx.ms0 + m1 * bx.ms1;
    double *W = bx.dst + gbase;  // element (i, c) at W[i sw + c sc]
    const long long sw = bx.sw, sc = bx.sc;
    if (bx.src != bx.dst) {
        const double *S = bx.src + gbase;
        for (int e = tid; e < N * NB; e += 256) {
            const int i0 = e / NB, c = e - i0 * NB;
            W[i0 * sw + c * sc] = S[i0 * sw + c * sc];
        }
        __syncthreads();
    }
    // forward: a kept equation's row r depends on its own row r and the eliminated neighbours only
    for (int l = 0; l <= L - 2; ++l) {
        const double *P = tabm + ((size_t)l * 3 + 1) * MM, *Q = tabm + ((size_t)l * 3 + 2) * MM;
        const int step = 1 << l, nkeep = (1 << (L - l - 1)) - 1;
        for (int t = tid; t < nkeep * NB; t += 256) {
            const int q = t / NB, r = t - q * NB;
            const long long i0 = (long long)(q + 1) * 2 * step - 1;
            double acc = W[i0 * sw + r * sc];
            for (int c = 0; c < NB; ++c)
                acc -= P[r * NB + c] * W[(i0 - step) * sw + c * sc] + Q[r * NB + c] * W[(i0 + step) * sw + c * sc];
            W[i0 * sw + r * sc] = acc;
        }
        __syncthreads();
    }
    // back substitution from the last level down: x_i = G f_i - P x_(i-s) - Q x_(i+s).  Chunks hold
    // whole equations, so no task reads a row-block that another task of its chunk has overwritten.
    const int eq_chunk = (256 * kCrChunk) / NB;
    for (int l = L - 1; l >= 0; --l) {
        const double *G = tabm + ((size_t)l * 3) * MM;
        const double *P = G + MM, *Q = G + 2 * MM;
        const int step = 1 << l, nel = 1 << (L - l - 1);
        for (int q0 = 0; q0 < nel; q0 += eq_chunk) {
            const int ntask = (nel - q0 < eq_chunk ? nel - q0 : eq_chunk) * NB;
            double res[kCrChunk];
#pragma unroll
            for (int u = 0; u < kCrChunk; ++u) {
                const int t = u * 256 + tid;
                res[u] = 0.0;
                if (t >= ntask) continue;
                const int q = q0 + t / NB, r = t % NB;
                const long long i = (long long)(2 * q + 1) * step;  // 1-based
                const bool has1 = i - step >= 1, has2 = i + step <= N;
                double acc = 0.0;
                for (int c = 0; c < NB; ++c) {
                    acc += G[r * NB + c] * W[(i - 1) * sw + c * sc];
                    if (has1) acc -= P[r * NB + c] * W[(i - 1 - step) * sw + c * sc];
                    if (has2) acc -= Q[r * NB + c] * W[(i - 1 + step) * sw + c * sc];
                }
                res[u] = acc;
            }
            __syncthreads();
#pragma unroll
            for (int u = 0; u < kCrChunk; ++u) {
                const int t = u * 256 + tid;
                if (t >= ntask) continue;
                const int q = q0 + t / NB, r = t % NB;
                const long long i = (long long)(2 * q + 1) * step;
                W[(i - 1) * sw + r * sc] = res[u];
            }
            __syncthreads();
        }
    }
}

// dst = src over n doubles (the line solve in place in dst)
__global__ __launch_bounds__(256) void k_cr_copy(const double *__restrict__ src, double *__restrict__ dst, long long n,
                                                 const int *gate) {
    if (!gate_open(gate)) return;
    for (long long e = (long long)blockIdx.x * 256 + threadIdx.x; e < n; e += (long long)gridDim.x * 256) dst[e] = src[e];
}

// The back substitution's results T (per mode NB x nel, row r of equation q at r + NB q) into the
// line at the equations' positions (2q + 1) s - 1.
__global__ __launch_bounds__(256) void k_cr_scatter(const double *__restrict__ T, double *__restrict__ W, int NB, int nel,
                                                    long long tstride, long long mstride, long long sw, long long sc,
                                                    int s, long long nmodes, const int *gate) {
    if (!gate_open(gate)) return;
    const long long per = (long long)NB * nel, tot = per * nmodes;
    for (long long e = (long long)blockIdx.x * 256 + threadIdx.x; e < tot; e += (long long)gridDim.x * 256) {
        const long long mode = e / per, rem = e - mode * per;
        const int q = (int)(rem / NB), r = (int)(rem - (long long)q * NB);
        W[mode * mstride + ((long long)(2 * q + 1) * s - 1) * sw + r * sc] = T[mode * tstride + rem];
    }
}

}  // namespace

// The global-memory form as FP64 GEMMs: at each level every kept (forward) or solved (back)
// equation of every mode applies the same level matrices of its mode, so a level is a batched
// product over the modes, with the equations as columns (strided in the line).  Forward: f_i -=
// P f_(i-s) and f_i -= Q f_(i+s) in place (the columns read and written are disjoint).  Back:
// T = G f_i, T -= P x_(i-s) (all but the first equation), T -= Q x_(i+s) (all but the last), then T
// into the line.  One mode axis (all modes at a common stride) is required; false otherwise.
static bool block_cr_gemm(const CrJob &job, hipStream_t st) {
    const int N = job.N, L = job.L, NB = job.NB;
    const long long MM = (long long)NB * NB;
    for (int b = 0; b < job.nbox; ++b) {
        const CrBox &bx = job.box[b];
        if (!(bx.nmodes <= bx.mext0 || bx.ms1 == bx.mext0 * bx.ms0)) return false;
        if ((long long)NB * (1ll << (L - 1)) * bx.nmodes > job.scratch_len) return false;
    }
    for (int b = 0; b < job.nbox; ++b) {
        const CrBox &bx = job.box[b];
        double *W = bx.dst;
        const long long ms = bx.nmodes > 1 ? bx.ms0 : 0, sw = bx.sw, sc = bx.sc;
        if (bx.src != bx.dst) {
            // the box's lines span [0, extent) of its canonical layout
            const long long n = (bx.nmodes - 1) * ms + (N - 1) * sw + (NB - 1) * sc + 1;
            ASDSM_LAUNCH(k_cr_copy, dim3((unsigned)std::min<long long>((n + 255) / 256, 4096)), dim3(256), 0, st,
                         bx.src, W, n, job.gate);
        }
        GemmJob g{};
        g.nbox = 1;
        g.gate = job.gate;
        g.tile = kTileAuto;
        g.any_layout = 1;
        g.M = NB;
        g.K = NB;
        g.sAb = 0;
        g.sAi = NB;
        g.sAk = 1;
        g.sBk = sc;
        g.sCi = sc;
        const long long tstride = (long long)NB << (L - 1);
        // columns and batches of a level's product: per-mode tables batch over the modes with the
        // level's equations as columns; one table for every mode (shared_tab) batches over the
        // equations with the modes as columns, so that each product has many columns
        const bool shared = job.shared_tab != 0;
        auto cols = [&](GemmJob &t, int neq, long long b_eq, long long c_eq, long long c_mode) {
            if (shared) {
                t.N = (int)bx.nmodes;
                t.sBn = ms;
                t.sCn = c_mode;
                t.nbatch = neq;
                t.sBb = b_eq;
                t.sCb = c_eq;
            } else {
                t.N = neq;
                t.sBn = b_eq;
                t.sCn = c_eq;
                t.nbatch = (int)bx.nmodes;
                t.sAb = (long long)L * 3 * MM;
                t.sBb = ms;
                t.sCb = c_mode;
            }
        };
        for (int l = 0; l <= L - 2; ++l) {  // forward reduction
            const int s = 1 << l, nkeep = (1 << (L - l - 1)) - 1;
            cols(g, nkeep, 2ll * s * sw, 2ll * s * sw, ms);
            g.accum = 1;
            g.neg = 1;
            g.C[0] = W + (2ll * s - 1) * sw;
            g.A[0] = bx.tab + ((long long)l * 3 + 1) * MM;  // P
            g.B[0] = W + ((long long)s - 1) * sw;
            if (!launch_gemm(g, st)) return false;
            g.A[0] = bx.tab + ((long long)l * 3 + 2) * MM;  // Q
            g.B[0] = W + (3ll * s - 1) * sw;
            if (!launch_gemm(g, st)) return false;
        }
        for (int l = L - 1; l >= 0; --l) {  // back substitution
            const int s = 1 << l, nel = 1 << (L - l - 1);
            GemmJob t = g;
            t.sCi = 1;
            cols(t, nel, 2ll * s * sw, NB, tstride);
            t.accum = 0;
            t.neg = 0;
            t.A[0] = bx.tab + (long long)l * 3 * MM;  // G
            t.B[0] = W + ((long long)s - 1) * sw;
            t.C[0] = job.scratch;
            if (!launch_gemm(t, st)) return false;
            if (nel >= 2) {
                cols(t, nel - 1, 2ll * s * sw, NB, tstride);
                t.accum = 1;
                t.neg = 1;
                t.A[0] = bx.tab + ((long long)l * 3 + 1) * MM;  // P x_(i-s), equations 1 .. nel-1
                t.B[0] = W + (2ll * s - 1) * sw;
                t.C[0] = job.scratch + NB;
                if (!launch_gemm(t, st)) return false;
                t.A[0] = bx.tab + ((long long)l * 3 + 2) * MM;  // Q x_(i+s), equations 0 .. nel-2
                t.C[0] = job.scratch;
                if (!launch_gemm(t, st)) return false;
            }
            const long long tot = (long long)NB * nel * bx.nmodes;
            ASDSM_LAUNCH(k_cr_scatter, dim3((unsigned)std::min<long long>((tot + 255) / 256, 4096)), dim3(256), 0, st,
                         job.scratch, W, NB, nel, tstride, ms, sw, sc, s, bx.nmodes, job.gate);
        }
    }
    return true;
}

size_t cr_lds_bytes(int N, int NB, int tm) {
    const int Nk = (N - 1) / 2;
    return 8ull * ((size_t)tm * Nk * NB + (size_t)tm * 3 * NB * NB);
}

// LDS of the fast form: the whole line and all levels' matrices of tm modes
size_t cr2_lds_bytes(int N, int L, int NB, int tm) {
    return 8ull * (size_t)tm * ((size_t)N * NB + (size_t)L * 3 * NB * NB);
}

static int cr_rb(int NB) {
    int rb = 1;
    while (rb < NB) rb *= 2;
    return rb;
}

// modes per workgroup of the fast form, or 0 when it does not apply: 256 threads hold tm * RB rows
// with at least one equation group, the back substitution's per-thread results fit the register
// array, and the LDS holds the lines and matrices
// LDS one workgroup may allocate on the current device (CDNA4: 160 KiB), cached per device
size_t cr_lds_cap() {
    static std::atomic<int> cache[64];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return kCrMaxLds;
    int v = cache[dev].load(std::memory_order_relaxed);
    if (v == 0) {
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess || v <= 0)
            v = (int)kCrMaxLds;
        v = std::min(v, 160 * 1024);
        cache[dev].store(v, std::memory_order_relaxed);
    }
    return (size_t)std::max(v, (int)kCrMaxLds);
}

int cr2_modes_per_group(int N, int L, int NB, long long nmodes, int nbox, int want) {
    if (!(NB == 1 || NB == 3 || NB == 7 || NB == 9 || NB == 15)) return 0;
    const int rb = cr_rb(NB);
    // 64 KiB first; the rest of the workgroup LDS only when not even one mode fits that (255 fine
    // positions with 15-point blocks: 72 KiB per mode), since more LDS per group leaves fewer
    // groups per CU
    const size_t caps[2] = {kCrMaxLds, cr_lds_cap()};
    for (const size_t cap : caps) {
        auto valid = [&](int tm) {
            if (tm < 1 || tm > 8 || (tm & (tm - 1)) || tm * rb > 256) return false;
            const int E = 256 / (tm * rb);
            return (1 << (L - 1)) <= E * kCrMaxPerThread && cr2_lds_bytes(N, L, NB, tm) <= cap;
        };
        if (!valid(1) && !valid(2) && !valid(4) && !valid(8)) continue;
        if (want > 0) return valid(want) ? want : 0;
        for (int tm = 8; tm >= 1; tm /= 2) {
            if (!valid(tm)) continue;
            // fewer modes per group while that still leaves under one group per CU; beyond 64 KiB,
            // also while two groups would not fit one CU's LDS
            if (tm > 1 && (nmodes * nbox + tm - 1) / tm < 256 && cr2_lds_bytes(N, L, NB, tm / 2) <= cap) continue;
            if (tm > 1 && cap > kCrMaxLds && 2 * cr2_lds_bytes(N, L, NB, tm) > cap) continue;
            return tm;
        }
        return 0;
    }
    return 0;
}

bool cr_lds_supported(int NB) { return NB == 1 || NB == 3 || NB == 7 || NB == 9 || NB == 15; }

bool launch_block_cr(const CrJob &job, hipStream_t st) {
    if (job.shared_tab)  // only the GEMM form indexes one table for all modes
        return job.tm == 0 && !job.fast && !job.accum && job.scratch && block_cr_gemm(job, st);
    long long maxm = 0;
    for (int b = 0; b < job.nbox; ++b) maxm = std::max(maxm, job.box[b].nmodes);
    if (job.fast) {
        const dim3 grid((unsigned)((maxm + job.tm - 1) / job.tm), (unsigned)job.nbox);
        const size_t lds = cr2_lds_bytes(job.N, job.L, job.NB, job.tm);
        if (lds > cr_lds_cap()) return false;
        switch (job.NB) {
            case 1: ASDSM_LAUNCH((k_block_cr2<1, 1>), grid, dim3(256), lds, st, job); return true;
            case 3: ASDSM_LAUNCH((k_block_cr2<3, 4>), grid, dim3(256), lds, st, job); return true;
            case 7: ASDSM_LAUNCH((k_block_cr2<7, 8>), grid, dim3(256), lds, st, job); return true;
            case 9: ASDSM_LAUNCH((k_block_cr2<9, 16>), grid, dim3(256), lds, st, job); return true;
            case 15: ASDSM_LAUNCH((k_block_cr2<15, 16>), grid, dim3(256), lds, st, job); return true;
            default: return false;
        }
    }
    if (job.tm == 0) {  // the global-memory form, in place in dst
        if (job.scratch && !job.accum && block_cr_gemm(job, st)) return true;
        ASDSM_LAUNCH(k_block_cr_global, dim3((unsigned)maxm, (unsigned)job.nbox), dim3(256), 0, st, job);
        return true;
    }
    const dim3 grid((unsigned)((maxm + job.tm - 1) / job.tm), (unsigned)job.nbox);
    const size_t lds = cr_lds_bytes(job.N, job.NB, job.tm);
    if (lds > kCrMaxLds) return false;
    switch (job.NB) {
        case 1: ASDSM_LAUNCH((k_block_cr<1>), grid, dim3(256), lds, st, job); return true;
        case 3: ASDSM_LAUNCH((k_block_cr<3>), grid, dim3(256), lds, st, job); return true;
        case 7: ASDSM_LAUNCH((k_block_cr<7>), grid, dim3(256), lds, st, job); return true;
        case 9: ASDSM_LAUNCH((k_block_cr<9>), grid, dim3(256), lds, st, job); return true;
        case 15: ASDSM_LAUNCH((k_block_cr<15>), grid, dim3(256), lds, st, job); return true;
        default: return false;
    }
}

}  // namespace asdsm
