// Host-side plan: validation, mesh geometry, 1D operator spectra, transform matrices, spline
// matrix, dense per-mode inverses of the intersection meshes, workspace layout.
//
// Paper references: meshes and nesting condition, Section 2.1 eqs. (3)-(5); discretisation,
// Section 2.3; the submesh family for d = 3, Section 3.5; the spline of the cross-point
// discrepancy, Algorithm 2 step 5 (cubic with zero end values; here the not-a-knot end rule).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <limits>
#include <mutex>
#include <thread>

#include "asdsm_internal.hpp"
#include "kernels.hpp"

namespace asdsm {

static thread_local std::string g_last_error;

void set_error(const std::string &msg) { g_last_error = msg; }
int fail(int code, const std::string &msg) {
    g_last_error = msg;
    return code;
}
const char *last_error_cstr() { return g_last_error.c_str(); }

static Tri op1d(double alpha, double beta, double h) {
    Tri t;
    t.a = -alpha / (h * h) - beta / (2.0 * h);
    t.b = 2.0 * alpha / (h * h);
    t.c = -alpha / (h * h) + beta / (2.0 * h);
    return t;
}

MeshDesc make_mesh(int d, int Nf, int Nc, unsigned mask) {
    MeshDesc m;
    m.mask = mask;
    m.nd = d;
    int p = 0;
    for (int j = 0; j < d; ++j)
        if (!(mask & (1u << j))) {
            m.ax[p] = j;
            m.ext[p] = Nf;
            ++p;
        }
    m.nfine = p;
    for (int j = 0; j < d; ++j)
        if (mask & (1u << j)) {
            m.ax[p] = j;
            m.ext[p] = Nc;
            ++p;
        }
    long long s = 1;
    for (int q = 0; q < d; ++q) {
        m.stride[q] = s;
        s *= m.ext[q];
    }
    m.size = s;
    m.nmodes = 1;
    for (int q = 0; q < m.nfine; ++q) m.nmodes *= m.ext[q];
    m.block = (int)(m.size / m.nmodes);
    return m;
}

// Eigen-decomposition of tridiag(a, b, c) of size N with a*c > 0 (|cell Peclet| < 1):
// eigenvectors v_i = r^i sin(i m pi/(N+1)), r = sqrt(a/c), eigenvalues b - 2 sqrt(ac) cos(m pi/(N+1)).
// The eigenvector matrix V = D Q with Q the orthonormal sine matrix (Q = Q^T = Q^-1) and
// D = diag(r^(i - c0)), c0 = (N+1)/2 (centred to keep the scaling symmetric); V^-1 = Q D^-1.
static void spectrum(const Tri &t, int N, AxisSpectrum &s) {
    s.N = N;
    if (N == 1) {  // a 1 x 1 operator, whatever its off-diagonal coefficients
        s.r = 1.0;
        s.mu.assign(1, t.b);
        s.W.assign(1, 1.0);
        s.V.assign(1, 1.0);
        s.cond = 1.0;
        return;
    }
    s.r = std::sqrt(t.a / t.c);
    const double sq = std::sqrt(t.a * t.c);
    const double PI = M_PI;
    const int M2 = 2 * (N + 1);
    std::vector<double> sn(M2);
    for (int k = 0; k < M2; ++k) sn[k] = std::sin(PI * (double)k / (double)(N + 1));
    const double nrm = std::sqrt(2.0 / (double)(N + 1));
    s.mu.assign(N, 0.0);
    for (int m = 0; m < N; ++m) s.mu[m] = t.b - 2.0 * sq * std::cos(PI * (double)(m + 1) / (double)(N + 1));
    const double c0 = 0.5 * (double)(N + 1);
    std::vector<double> dpow(N);
    for (int i = 0; i < N; ++i) dpow[i] = std::pow(s.r, (double)(i + 1) - c0);
    s.W.assign((size_t)N * N, 0.0);
    s.V.assign((size_t)N * N, 0.0);
    for (int i = 0; i < N; ++i)
        for (int m = 0; m < N; ++m) {
            const double q = nrm * sn[((long long)(i + 1) * (m + 1)) % M2];
            s.W[(size_t)m * N + i] = q / dpow[i];
            s.V[(size_t)i * N + m] = dpow[i] * q;
        }
    s.cond = std::pow(std::max(s.r, 1.0 / s.r), (double)(N - 1));
}

// Dense LU with partial pivoting (row major), in place.  Returns false on a zero pivot.
static bool lu_factor(int n, std::vector<double> &A, std::vector<int> &piv) {
    piv.resize(n);
    for (int k = 0; k < n; ++k) {
        int p = k;
        double best = std::fabs(A[(size_t)k * n + k]);
        for (int i = k + 1; i < n; ++i) {
            double v = std::fabs(A[(size_t)i * n + k]);
            if (v > best) {
                best = v;
                p = i;
            }
        }
        piv[k] = p;
        if (best == 0.0) return false;
        if (p != k)
            for (int j = 0; j < n; ++j) std::swap(A[(size_t)k * n + j], A[(size_t)p * n + j]);
        const double inv = 1.0 / A[(size_t)k * n + k];
        for (int i = k + 1; i < n; ++i) {
            double l = A[(size_t)i * n + k] * inv;
            A[(size_t)i * n + k] = l;
            if (l != 0.0)
                for (int j = k + 1; j < n; ++j) A[(size_t)i * n + j] -= l * A[(size_t)k * n + j];
        }
    }
    return true;
}

static void lu_solve(int n, const std::vector<double> &LU, const std::vector<int> &piv, double *x) {
    for (int k = 0; k < n; ++k) {
        if (piv[k] != k) std::swap(x[k], x[piv[k]]);
    }
    for (int i = 1; i < n; ++i) {
        double s = x[i];
        for (int j = 0; j < i; ++j) s -= LU[(size_t)i * n + j] * x[j];
        x[i] = s;
    }
    for (int i = n - 1; i >= 0; --i) {
        double s = x[i];
        for (int j = i + 1; j < n; ++j) s -= LU[(size_t)i * n + j] * x[j];
        x[i] = s / LU[(size_t)i * n + i];
    }
}

// Cubic not-a-knot spline through the uniform knots t*H, t = 0..Nc+1, with zero values at both
// ends, evaluated at the fine points (i+1) h: returns Sp (Nf x Nc, row major) such that the spline
// through the knot values y_1..y_Nc is Sp y.  Built from the second-derivative ("moment")
// equations M_{t-1} + 4 M_t + M_{t+1} = 6 (y_{t+1} - 2 y_t + y_{t-1}) / H^2 at the interior knots and
// the not-a-knot rows M_0 - 2 M_1 + M_2 = 0, M_{Nc-1} - 2 M_Nc + M_{Nc+1} = 0.  With one interior
// knot the spline is the parabola through the three knots.
static void build_spline(int Nf, int Nc, int n, double h, double H, std::vector<double> &Sp) {
    Sp.assign((size_t)Nf * Nc, 0.0);
    if (Nc == 1) {
        for (int i = 0; i < Nf; ++i) {
            double x = (double)(i + 1) * h;
            Sp[i] = ((i + 1) % n == 0) ? 1.0 : 4.0 * x * (1.0 - x);
        }
        return;
    }
    const int K = Nc + 2;
    std::vector<double> A((size_t)K * K, 0.0);
    A[0 * K + 0] = 1.0;
    A[0 * K + 1] = -2.0;
    A[0 * K + 2] = 1.0;
    for (int t = 1; t <= Nc; ++t) {
        A[(size_t)t * K + t - 1] = 1.0;
        A[(size_t)t * K + t] = 4.0;
        A[(size_t)t * K + t + 1] = 1.0;
    }
    A[(size_t)(K - 1) * K + (K - 3)] = 1.0;
    A[(size_t)(K - 1) * K + (K - 2)] = -2.0;
    A[(size_t)(K - 1) * K + (K - 1)] = 1.0;
    std::vector<int> piv;
    lu_factor(K, A, piv);
    std::vector<double> y(K), M(K);
    for (int c = 0; c < Nc; ++c) {
        std::fill(y.begin(), y.end(), 0.0);
        y[c + 1] = 1.0;
        std::fill(M.begin(), M.end(), 0.0);
        for (int t = 1; t <= Nc; ++t) M[t] = 6.0 * (y[t + 1] - 2.0 * y[t] + y[t - 1]) / (H * H);
        lu_solve(K, A, piv, M.data());
        for (int i = 0; i < Nf; ++i) {
            if ((i + 1) % n == 0) {
                Sp[(size_t)i * Nc + c] = ((i + 1) / n - 1 == c) ? 1.0 : 0.0;
                continue;
            }
            const double x = (double)(i + 1) * h;
            int t = (i + 1) / n;                 // interval [t H, (t+1) H]
            const double xl = (double)t * H, xr = (double)(t + 1) * H;
            const double dl = x - xl, dr = xr - x;
            const double v = M[t] * dr * dr * dr / (6.0 * H) + M[t + 1] * dl * dl * dl / (6.0 * H) +
                             (y[t] - M[t] * H * H / 6.0) * dr / H +
                             (y[t + 1] - M[t + 1] * H * H / 6.0) * dl / H;
            Sp[(size_t)i * Nc + c] = v;
        }
    }
}

// Inverse of an n x n matrix (row major, overwritten by its LU factors) by LU with partial pivoting,
// written column by column: inv[j*n + i] = (A^-1)(i, j).  The row extents of the (pivot-widened)
// band are tracked so that elimination and substitution skip the zeros outside it; the n right-hand
// sides of the substitutions are split over threads by column range.
static bool dense_inverse(int n, std::vector<double> &A, double *inv) {
    std::vector<int> lo(n), hi(n), perm(n);
    for (int i = 0; i < n; ++i) {
        int l = i, h = i;
        for (int j = 0; j < n; ++j)
            if (A[(size_t)i * n + j] != 0.0) {
                l = std::min(l, j);
                h = std::max(h, j);
            }
        lo[i] = l;
        hi[i] = h;
        perm[i] = i;
    }
    for (int k = 0; k < n; ++k) {
        int p = k;
        double best = 0.0;
        for (int i = k; i < n; ++i)
            if (lo[i] <= k) {
                const double v = std::fabs(A[(size_t)i * n + k]);
                if (v > best) {
                    best = v;
                    p = i;
                }
            }
        if (best == 0.0) return false;
        if (p != k) {
            const int a = std::min(lo[k], lo[p]), b = std::max(hi[k], hi[p]);
            for (int j = a; j <= b; ++j) std::swap(A[(size_t)k * n + j], A[(size_t)p * n + j]);
            std::swap(lo[k], lo[p]);
            std::swap(hi[k], hi[p]);
            std::swap(perm[k], perm[p]);
        }
        const double piv = A[(size_t)k * n + k];
        for (int i = k + 1; i < n; ++i) {
            if (lo[i] > k) continue;
            const double l = A[(size_t)i * n + k] / piv;
            A[(size_t)i * n + k] = l;
            if (l == 0.0) continue;
            for (int j = k + 1; j <= hi[k]; ++j) A[(size_t)i * n + j] -= l * A[(size_t)k * n + j];
            hi[i] = std::max(hi[i], hi[k]);
        }
    }
    // X = A^-1 (row major): X starts as P, then L and U substitutions row by row
    std::vector<double> X((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i) X[(size_t)i * n + perm[i]] = 1.0;
    auto substitute = [&](int c0, int c1) {
        for (int i = 0; i < n; ++i) {
            double *xi = X.data() + (size_t)i * n;
            for (int k = lo[i]; k < i; ++k) {
                const double l = A[(size_t)i * n + k];
                if (l == 0.0) continue;
                const double *xk = X.data() + (size_t)k * n;
                for (int j = c0; j < c1; ++j) xi[j] -= l * xk[j];
            }
        }
        for (int i = n - 1; i >= 0; --i) {
            double *xi = X.data() + (size_t)i * n;
            for (int k = i + 1; k <= hi[i]; ++k) {
                const double u = A[(size_t)i * n + k];
                if (u == 0.0) continue;
                const double *xk = X.data() + (size_t)k * n;
                for (int j = c0; j < c1; ++j) xi[j] -= u * xk[j];
            }
            const double d = 1.0 / A[(size_t)i * n + i];
            for (int j = c0; j < c1; ++j) xi[j] *= d;
        }
    };
    int nt = 1;
    if (n >= 512) nt = std::max(1, std::min(16, (int)std::thread::hardware_concurrency()));
    if (nt == 1) {
        substitute(0, n);
    } else {
        std::vector<std::thread> pool;
        const int chunk = (n + nt - 1) / nt;
        for (int t = 0; t < nt; ++t) {
            const int c0 = t * chunk, c1 = std::min(n, c0 + chunk);
            if (c0 < c1) pool.emplace_back(substitute, c0, c1);
        }
        for (std::thread &th : pool) th.join();
    }
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) inv[(size_t)j * n + i] = X[(size_t)i * n + j];
    return true;
}

// Per-mode inverses for a mesh with >= 2 coarse axes: after the fine axes are diagonalised, mode m
// couples only the coarse points through (Kronecker sum of the coarse-axis operators) + sigma_m I,
// sigma_m = sum of the fine-axis eigenvalues of the mode.
static bool build_dense_inverse(Plan &p, unsigned mask) {
    const MeshDesc &m = p.mesh[mask];
    const int B = m.block;
    std::vector<double> &out = p.dense_inv[mask];
    out.assign((size_t)m.nmodes * B * B, 0.0);
    // Kronecker-sum matrix of the coarse axes on B points (coarse canonical order, first fastest)
    std::vector<double> Kc((size_t)B * B, 0.0);
    long long cs = 1;
    for (int q = m.nfine; q < m.nd; ++q) {
        const Tri t = p.geo.coarse[m.ax[q]];
        const int e = m.ext[q];
        for (int idx = 0; idx < B; ++idx) {
            int pos = (int)((idx / cs) % e);
            Kc[(size_t)idx * B + idx] += t.b;
            if (pos > 0) Kc[(size_t)idx * B + (idx - cs)] += t.a;
            if (pos < e - 1) Kc[(size_t)idx * B + (idx + cs)] += t.c;
        }
        cs *= e;
    }
    // modes are independent: small blocks (many modes) are spread over host threads; large blocks
    // thread their own substitutions
    auto run = [&](long long m0, long long m1, bool *ok) {
        std::vector<double> A((size_t)B * B);
        for (long long mode = m0; mode < m1; ++mode) {
            double sigma = 0.0;
            long long rem = mode;
            for (int q = 0; q < m.nfine; ++q) {
                int mq = (int)(rem % m.ext[q]);
                rem /= m.ext[q];
                sigma += p.fine_spec[m.ax[q]].mu[mq];
            }
            A = Kc;
            for (int i = 0; i < B; ++i) A[(size_t)i * B + i] += sigma;
            if (!dense_inverse(B, A, out.data() + (size_t)mode * B * B)) {
                *ok = false;
                return;
            }
        }
    };
    int nt = 1;
    if (B < 512 && m.nmodes >= 16 && (double)m.nmodes * B * B * B > 1e7)
        nt = std::max(1, std::min(16, (int)std::thread::hardware_concurrency()));
    if (nt == 1) {
        bool ok = true;
        run(0, m.nmodes, &ok);
        return ok;
    }
    std::vector<std::thread> pool;
    std::vector<char> oks(nt, 1);
    const long long chunk = (m.nmodes + nt - 1) / nt;
    for (int t = 0; t < nt; ++t) {
        const long long m0 = t * chunk, m1 = std::min<long long>(m.nmodes, m0 + chunk);
        if (m0 < m1) pool.emplace_back([&, t, m0, m1] {
            bool ok = true;
            run(m0, m1, &ok);
            oks[t] = ok;
        });
    }
    for (std::thread &th : pool) th.join();
    for (char o : oks)
        if (!o) return false;
    return true;
}

// Row-major products and inverse of small dense NB x NB matrices (CR tables).
static void matmul(int n, const double *A, const double *B, double *C) {
    auto rows = [&](int i0, int i1) {
        for (int i = i0; i < i1; ++i)
            for (int j = 0; j < n; ++j) {
                double acc = 0.0;
                for (int k = 0; k < n; ++k) acc += A[(size_t)i * n + k] * B[(size_t)k * n + j];
                C[(size_t)i * n + j] = acc;
            }
    };
    // large blocks (the line solves whose block holds a fine axis): rows over host threads, each
    // row accumulated along B's rows (contiguous loads)
    auto rows_by_k = [&](int i0, int i1) {
        for (int i = i0; i < i1; ++i) {
            double *ci = C + (size_t)i * n;
            std::fill(ci, ci + n, 0.0);
            for (int k = 0; k < n; ++k) {
                const double a = A[(size_t)i * n + k];
                const double *bk = B + (size_t)k * n;
                for (int j = 0; j < n; ++j) ci[j] += a * bk[j];
            }
        }
    };
    const int nt = (n >= 128) ? std::max(1, std::min(16, (int)std::thread::hardware_concurrency())) : 1;
    if (nt == 1) {
        rows(0, n);
        return;
    }
    std::vector<std::thread> pool;
    const int chunk = (n + nt - 1) / nt;
    for (int t = 0; t < nt; ++t) {
        const int i0 = t * chunk, i1 = std::min(n, i0 + chunk);
        if (i0 < i1) pool.emplace_back(rows_by_k, i0, i1);
    }
    for (std::thread &th : pool) th.join();
}

// The level tables of one system of block cyclic reduction: B_0 = Kc + (b_w + sigma) I, A_0 = a_w I,
// C_0 = c_w I; per level G, P, Q (row major) into dst, L * 3 * NB^2 doubles.  False on a singular
// block.
static bool cr_level_tables(int NB, int L, const std::vector<double> &Kc, Tri tw, double sigma, double *dst0) {
    const size_t MM = (size_t)NB * NB;
    std::vector<double> B(Kc), A(MM, 0.0), C(MM, 0.0), G(MM), T1(MM), T2(MM), LU(MM), inv(MM);
    for (int i = 0; i < NB; ++i) {
        B[(size_t)i * NB + i] += tw.b + sigma;
        A[(size_t)i * NB + i] = tw.a;
        C[(size_t)i * NB + i] = tw.c;
    }
    for (int l = 0; l < L; ++l) {
        LU = B;
        if (!dense_inverse(NB, LU, inv.data())) return false;
        for (int i = 0; i < NB; ++i)  // dense_inverse writes column by column
            for (int j = 0; j < NB; ++j) G[(size_t)i * NB + j] = inv[(size_t)j * NB + i];
        double *dst = dst0 + (size_t)l * 3 * MM;
        std::copy(G.begin(), G.end(), dst);
        matmul(NB, G.data(), A.data(), dst + MM);
        matmul(NB, G.data(), C.data(), dst + 2 * MM);
        if (l == L - 1) break;
        // B -= A G C + C G A;  A = -A G A;  C = -C G C
        matmul(NB, A.data(), dst + 2 * MM, T1.data());   // A (G C)
        matmul(NB, C.data(), dst + MM, T2.data());       // C (G A)
        for (size_t e = 0; e < MM; ++e) B[e] -= T1[e] + T2[e];
        matmul(NB, A.data(), dst + MM, T1.data());       // A G A
        matmul(NB, C.data(), dst + 2 * MM, T2.data());   // C G C
        for (size_t e = 0; e < MM; ++e) {
            A[e] = -T1[e];
            C[e] = -T2[e];
        }
    }
    return true;
}

// Reduced blocks of block cyclic reduction along the line axis of mesh `mask` (k_blockcr.hip): per
// mode of the other fine axes, B_0 = T_block + (b_w + sigma) I, A_0 = a_w I, C_0 = c_w I and per
// level G_l = B_l^-1, P_l = G_l A_l, Q_l = G_l C_l, then B_(l+1) = B_l - A_l G_l C_l - C_l G_l A_l,
// A_(l+1) = -A_l G_l A_l, C_(l+1) = -C_l G_l C_l (elimination of the odd equations of the level).
// Stored per mode and level as G, P, Q, row major.
static bool build_cr_tables(Plan &p, unsigned mask) {
    const MeshDesc &m = p.mesh[mask];
    const int lp = p.line_pos[mask];
    const int NB = cr_block(p, mask), L = p.level;
    const size_t MM = (size_t)NB * NB;
    const long long nmodes = cr_modes(p, mask);
    const Tri tw = p.geo.fine[m.ax[lp]];
    // Kronecker-sum matrix of the block's axes (canonical order, first fastest): the coarse axes,
    // preceded by the second fine axis when both fine axes are on the line solve (line_block2)
    const bool cmodes = p.line_cmodes[mask];
    const int qb = (p.line_block2[mask] || cmodes) ? 1 : m.nfine;  // first canonical position of the block
    const int qe = cmodes ? 2 : m.nd;                                // one past its last
    std::vector<double> Kc(MM, 0.0);
    long long cs = 1;
    for (int q = qb; q < qe; ++q) {
        const Tri t = (q < m.nfine) ? p.geo.fine[m.ax[q]] : p.geo.coarse[m.ax[q]];
        const int e = m.ext[q];
        for (int idx = 0; idx < NB; ++idx) {
            const int pos = (int)((idx / cs) % e);
            Kc[(size_t)idx * NB + idx] += t.b;
            if (pos > 0) Kc[(size_t)idx * NB + (idx - cs)] += t.a;
            if (pos < e - 1) Kc[(size_t)idx * NB + (idx + cs)] += t.c;
        }
        cs *= e;
    }
    int fq[kMaxD], nfq = 0;  // fine positions other than the line axis and the block (the mode axes)
    for (int q = 0; q < std::min(m.nfine, qb); ++q)
        if (q != lp) fq[nfq++] = q;
    std::vector<double> &out = p.cr_tab[mask];
    out.assign((size_t)nmodes * L * 3 * MM, 0.0);
    auto run = [&](long long m0, long long m1, bool *ok) {
        for (long long mode = m0; mode < m1; ++mode) {
            double sigma = 0.0;
            long long rem = mode;
            for (int t = 0; t < nfq; ++t) {
                const int mq = (int)(rem % m.ext[fq[t]]);
                rem /= m.ext[fq[t]];
                sigma += p.fine_spec[m.ax[fq[t]]].mu[mq];
            }
            if (cmodes) sigma += p.coarse_spec[m.ax[2]].mu[mode];  // the diagonalised coarse axis
            if (!cr_level_tables(NB, L, Kc, tw, sigma, out.data() + (size_t)mode * L * 3 * MM)) {
                *ok = false;
                return;
            }
        }
    };
    int nt = 1;
    if (nmodes >= 16 && (double)nmodes * L * MM * NB > 1e7)
        nt = std::max(1, std::min(16, (int)std::thread::hardware_concurrency()));
    std::vector<char> oks(nt, 1);
    std::vector<std::thread> pool;
    const long long chunk = (nmodes + nt - 1) / nt;
    for (int t = 0; t < nt; ++t) {
        const long long a = t * chunk, b = std::min<long long>(nmodes, a + chunk);
        if (a >= b) continue;
        if (nt == 1) {
            bool ok = true;
            run(a, b, &ok);
            oks[t] = ok;
        } else {
            pool.emplace_back([&, t, a, b] {
                bool ok = true;
                run(a, b, &ok);
                oks[t] = ok;
            });
        }
    }
    for (std::thread &th : pool) th.join();
    for (char o : oks)
        if (!o) return false;
    return true;
}

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

void layout_workspace(Plan &p, char *base, bool assign) {
    size_t off = 0;
    auto take = [&](size_t bytes) -> char * {
        char *ptr = base ? base + off : nullptr;
        off = align256(off + bytes);
        return ptr;
    };
    const size_t NF = (size_t)p.geo.NF;
    Workspace w;
    w.b = (double *)take(NF * 8);
    w.r = (double *)take(NF * 8);
    w.e = (double *)take(NF * 8);
    w.u2 = (double *)take(NF * 8);
    const unsigned nm = 1u << p.d;
    for (unsigned s = 1; s < nm; ++s) {
        w.X[s] = (double *)take((size_t)p.mesh[s].size * 8);
        w.Y[s] = (double *)take((size_t)p.mesh[s].size * 8);
        if (p.sweeps[s] > 0) {
            w.Z[s] = (double *)take((size_t)p.mesh[s].size * 8);
            w.W[s] = (double *)take((size_t)p.mesh[s].size * 8);
        }
    }
    {
        // line solves with blocks the LDS forms do not take: NB x 2^(L-1) per mode of the mesh
        long long need = 0;
        for (unsigned s = 1; s < nm; ++s) {
            if (p.line_pos[s] < 0 || cr_lds_supported(cr_block(p, s))) continue;
            need = std::max(need, (long long)cr_block(p, s) * (1ll << (p.level - 1)) * cr_modes(p, s));
        }
        long long holes = 1;
        for (int j = 0; j < p.d; ++j) holes *= p.Nc + 1;
        const long long nh = p.n - 1;
        if (p.hole_cr) need = std::max(need, nh * nh * (1ll << (p.hole_cr_L - 1)) * holes);
        w.crs_len = need;
        w.crs = need ? (double *)take((size_t)need * 8) : nullptr;
        if (p.hole_cr) w.HB = (double *)take((size_t)(holes * nh * nh * nh) * 8);
    }
    // cross-point discrepancies of each anisotropic mesh: d=2: Nc*Nc; d=3: parts A, B, R of
    // Nc*Nc*Nf values each; d=4: three plane families and two Boolean-sum remainders of
    // Nc*Nc*Nf*Nf values each
    const size_t nl = (p.d == 2)   ? (size_t)p.Nc * p.Nc
                      : (p.d == 3) ? (size_t)3 * p.Nc * p.Nc * p.Nf
                                   : (size_t)5 * p.Nc * p.Nc * p.Nf * p.Nf;
    for (int k = 0; k < p.d; ++k) w.lines[k] = (double *)take(nl * 8);
    for (int k = 0; k < p.d; ++k) {
        w.F1[k] = (float *)take((size_t)p.mesh[1u << k].size * 4);
        w.F2[k] = (float *)take((size_t)p.mesh[1u << k].size * 4);
    }
    if (p.d == 3) {
        for (int k = 0; k < 3; ++k) {
            const size_t sz = (size_t)p.mesh[1u << k].size;
            w.SU[k] = (double *)take(sz * 8);
            w.SR[k] = (double *)take(sz * 8);
            w.SQ[k] = (double *)take(sz * 8);
            w.EA[k] = (double *)take(2 * sz * 8);
            w.SR2[k] = (double *)take(sz * 8);
            w.SE[k] = (double *)take(sz * 8);
        }
    }
    w.state = (IterState *)take(sizeof(IterState));
    w.hist = (double *)take((size_t)kHistCap * 8);
    w.step_hist = (double *)take((size_t)kHistCap * 8);
    w.perm_table = (int *)take((size_t)kHistCap * kMaxD * sizeof(int));
    w.partials = (double *)take((size_t)p.max_blocks * 4 * 8);
    w.scal = (double *)take(kScalCount * 8);
    p.ws_need = off;
    if (assign) p.ws = w;
}

void axis_permutation(uint64_t seed, int64_t k, int d, int perm[kMaxD]) {
    const uint64_t golden = 0x9E3779B97F4A7C15ull;
    uint64_t state = seed ^ ((uint64_t)(k + 1) * golden);
    for (int i = 0; i < d; ++i) perm[i] = i;
    for (int i = d - 1; i >= 1; --i) {
        state += golden;
        uint64_t z = state;
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        z = z ^ (z >> 31);
        int j = (int)(z % (uint64_t)(i + 1));
        std::swap(perm[i], perm[j]);
    }
}

int build_plan(Plan &p, int d, const double *alpha, const double *beta, int level,
               int coarse_level, uint64_t seed, hipStream_t stream) {
    if (d < 2 || d > kMaxD) return fail(ASDSM_E_ARG, "d must be 2, 3 or 4");
    if (!alpha || !beta) return fail(ASDSM_E_ARG, "alpha and beta must be non-NULL");
    if (level < 2 || level > 10) return fail(ASDSM_E_ARG, "level must be in [2, 10]");
    if (coarse_level == 0) coarse_level = level / 2;
    if (coarse_level < 1 || coarse_level >= level)
        return fail(ASDSM_E_NESTING, "coarse_level must satisfy 1 <= coarse_level < level (eq. (3))");
    for (int j = 0; j < d; ++j) {
        if (!std::isfinite(alpha[j]) || !(alpha[j] > 0.0))
            return fail(ASDSM_E_ARG, "alpha[" + std::to_string(j) + "] must be finite and > 0");
        if (!std::isfinite(beta[j]))
            return fail(ASDSM_E_ARG, "beta[" + std::to_string(j) + "] must be finite");
    }
    p.d = d;
    p.level = level;
    p.clevel = coarse_level;
    p.Nf = (1 << level) - 1;
    p.Nc = (1 << coarse_level) - 1;
    p.n = 1 << (level - coarse_level);
    p.h = 1.0 / (double)(p.Nf + 1);
    p.H = 1.0 / (double)(p.Nc + 1);
    p.seed = seed;
    p.stream = stream;
    for (int j = 0; j < d; ++j) {
        p.alpha[j] = alpha[j];
        p.beta[j] = beta[j];
    }
    // hole boxes are solved inside one workgroup's LDS: two (n-1)^d buffers plus, per transform
    // axis, two (n-1)^2 matrices and n-1 eigenvalues; keep it within 64 KiB
    {
        const long long nh = p.n - 1;
        long long pts = 1;
        for (int j = 0; j < d; ++j) pts *= nh;
        const long long lds = (2 * pts + (long long)(d - 1) * (2 * nh * nh + nh)) * 8;
        if (lds > 64 * 1024)
            return fail(ASDSM_E_UNSUPPORTED, "hole boxes of (n-1)^d points exceed the LDS budget; "
                                             "raise coarse_level");
    }
    Geo &g = p.geo;
    g.d = d;
    g.Nf = p.Nf;
    g.Nc = p.Nc;
    g.n = p.n;
    g.NF = 1;
    for (int j = 0; j < d; ++j) g.NF *= p.Nf;
    for (int j = 0; j < kMaxD; ++j) {
        g.fine[j] = (j < d) ? op1d(alpha[j], beta[j], p.h) : Tri{0, 0, 0};
        g.coarse[j] = (j < d) ? op1d(alpha[j], beta[j], p.H) : Tri{0, 0, 0};
    }
    // Per fine axis: fast diagonalisation needs a real spectrum (|beta h / (2 alpha)| < 1) and is
    // accurate to about eps * cond(V) with cond(V) = r^(N-1), V = D Q the eigenvector matrix.  An axis
    // with a complex spectrum gets cond = inf; such axes are solved by line elimination instead.
    const double kInf = std::numeric_limits<double>::infinity();
    double cond_f[kMaxD], cond_h[kMaxD];
    for (int j = 0; j < d; ++j) {
        const double P = std::fabs(beta[j] * p.h / (2.0 * alpha[j]));
        if (P < 1.0) {
            spectrum(g.fine[j], p.Nf, p.fine_spec[j]);
            cond_f[j] = p.fine_spec[j].cond;
        } else {
            cond_f[j] = kInf;
        }
        if (P < 1.0 || p.n - 1 == 1) {
            spectrum(g.fine[j], p.n - 1, p.hole_spec[j]);
            cond_h[j] = p.hole_spec[j].cond;
        } else {
            cond_h[j] = kInf;
        }
    }
    // hole line axis: the worst-conditioned axis is eliminated, the others are transformed
    p.hole_line_axis = 0;
    for (int j = 1; j < d; ++j)
        if (cond_h[j] > cond_h[p.hole_line_axis]) p.hole_line_axis = j;
    {
        double ch = 1.0;
        for (int j = 0; j < d; ++j)
            if (j != p.hole_line_axis) ch *= cond_h[j];
        if (!(2.2e-16 * ch <= 1e-12)) {
            // two or more such axes: holes of up to kHoleDenseMax^3 points (d = 3) take the hole
            // operator's inverse, applied densely; holes of 15^3 the hole line solve
            if (d != 3 || (p.n - 1 > kHoleDenseMax && p.n - 1 != 15))
                return fail(ASDSM_E_UNSUPPORTED, "hole boxes: more than one axis too ill-conditioned for "
                                                 "fast diagonalisation (|cell Peclet| near or above 1)");
            if (p.n - 1 <= kHoleDenseMax) p.hole_dense = true;
            else p.hole_cr = true;
        }
    }
    if (p.hole_cr) {
        // block cyclic reduction along the hole line axis: the block operator is the Kronecker sum
        // of the other two axes' fine-spacing operators on nh^2 points (the lower axis fastest)
        const int nh = p.n - 1, NB = nh * nh, la = p.hole_line_axis;
        const int ax0 = (la == 0) ? 1 : 0, ax1 = (la == 2) ? 1 : 2;
        std::vector<double> Kc((size_t)NB * NB, 0.0);
        for (int o = 0; o < NB; ++o) {
            const int c0 = o % nh, c1 = o / nh;
            const Tri t0 = g.fine[ax0], t1 = g.fine[ax1];
            Kc[(size_t)o * NB + o] = t0.b + t1.b;
            if (c0 > 0) Kc[(size_t)o * NB + o - 1] = t0.a;
            if (c0 < nh - 1) Kc[(size_t)o * NB + o + 1] = t0.c;
            if (c1 > 0) Kc[(size_t)o * NB + o - nh] = t1.a;
            if (c1 < nh - 1) Kc[(size_t)o * NB + o + nh] = t1.c;
        }
        p.hole_cr_L = 4;  // nh = 2^4 - 1
        p.hole_cr_tab.assign((size_t)p.hole_cr_L * 3 * NB * NB, 0.0);
        if (!cr_level_tables(NB, p.hole_cr_L, Kc, g.fine[la], 0.0, p.hole_cr_tab.data()))
            return fail(ASDSM_E_NUMERIC, "singular reduced block of the hole line solve");
    }
    if (p.hole_dense) {
        // the hole operator: the Kronecker sum of the three fine-spacing 1D operators on (n-1)^3
        // points (x_1 fastest); its inverse, column by column
        const int nh = p.n - 1, np = nh * nh * nh;
        std::vector<double> A((size_t)np * np, 0.0);
        const int st[3] = {1, nh, nh * nh};
        for (int o = 0; o < np; ++o) {
            const int l[3] = {o % nh, (o / nh) % nh, o / (nh * nh)};
            for (int j = 0; j < 3; ++j) {
                const Tri t = g.fine[j];
                A[(size_t)o * np + o] += t.b;
                if (l[j] > 0) A[(size_t)o * np + o - st[j]] += t.a;
                if (l[j] < nh - 1) A[(size_t)o * np + o + st[j]] += t.c;
            }
        }
        p.hole_inv.assign((size_t)np * np, 0.0);
        if (!dense_inverse(np, A, p.hole_inv.data())) return fail(ASDSM_E_NUMERIC, "singular hole operator");
    }
    build_spline(p.Nf, p.Nc, p.n, p.h, p.H, p.Sp);
    for (unsigned s = 0; s < (1u << d); ++s) p.mesh[s] = make_mesh(d, p.Nf, p.Nc, s);
    // Refinement sweeps x <- x + M^-1 (f - A x) around a solve accurate to delta = eps * prod cond
    // over its transformed axes, each gaining -log10(delta) digits, so that the result reaches
    // ~1e-14; none where delta <= 2e-11; impossible (-1) from delta >= 0.05.
    auto sweeps_for = [](double c) -> int {
        const double delta = 2.2e-16 * c;
        if (delta <= 2e-11) return 0;
        if (!(delta < 0.05)) return -1;
        return std::max(1, (int)std::ceil(std::log(1e-14) / std::log(delta)) - 1);
    };
    auto worse = [](int a, int b) { return a < 0 || (b >= 0 && a > b); };  // a needs more than b
    // Anisotropic meshes: either every fine axis is transformed and the coarse axis eliminated
    // (Thomas), or the worst fine axis of each becomes its line axis, solved together with the
    // coarse axis by block cyclic reduction, and the others are transformed.  Line axes are used
    // when the transforms alone cannot reach the accuracy, or need more sweeps.
    int swA = 0, swB = 0;
    int lineq[kMaxD];
    double condB[kMaxD];
    bool block2 = false;
    for (int k = 0; k < d; ++k) {
        const MeshDesc &m = p.mesh[1u << k];
        double cA = 1.0;
        int wq = 0;
        for (int q = 0; q < m.nfine; ++q) {
            cA *= cond_f[m.ax[q]];
            if (cond_f[m.ax[q]] > cond_f[m.ax[wq]]) wq = q;
        }
        double cB = 1.0;
        for (int q = 0; q < m.nfine; ++q)
            if (q != wq) cB *= cond_f[m.ax[q]];
        lineq[k] = wq;
        condB[k] = cB;
        const int a = sweeps_for(cA), b = sweeps_for(cB);
        if (worse(a, swA)) swA = a;
        if (b < 0) {
            // both fine axes defeat fast diagonalisation (d = 3): a mesh whose block of the second
            // fine axis with the coarse axis (N_f N_c points) fits the line solve takes both on it;
            // else, if the coarse axis can be diagonalised without refinement, each of its modes
            // leaves a line solve with the second fine axis as the block; else blocks of up to
            // kCrMaxBlock2 points
            if (d != 3)
                return fail(ASDSM_E_UNSUPPORTED, "a d = 4 submesh has two fine axes that fast diagonalisation "
                                                 "cannot handle (|cell Peclet| near or above 1 on two axes)");
            if ((long long)p.Nf * m.block <= kCrMaxBlock) {
                p.line_block2[1u << k] = true;
            } else {
                const Tri tc = g.coarse[k];
                const bool real = std::fabs(beta[k] * p.H / (2.0 * alpha[k])) < 1.0;
                if (real) spectrum(tc, p.Nc, p.coarse_spec[k]);
                if (real && sweeps_for(p.coarse_spec[k].cond) == 0)
                    p.line_cmodes[1u << k] = true;
                else if ((long long)p.Nf * m.block <= kCrMaxBlock2)
                    p.line_block2[1u << k] = true;
                else
                    return fail(ASDSM_E_UNSUPPORTED, "a submesh has two fine axes that fast diagonalisation "
                                                     "cannot handle (|cell Peclet| near or above 1 on two axes), "
                                                     "more than " + std::to_string(kCrMaxBlock2) +
                                                     " points per line position, and a coarse axis that "
                                                     "cannot be diagonalised either");
            }
            block2 = true;
            continue;
        }
        if (worse(b, swB)) swB = b;
    }
    p.line_aniso = block2 || worse(swA, swB);
    for (unsigned s = 0; s < kMaxMeshes; ++s) p.line_pos[s] = -1;
    for (int k = 0; k < d; ++k) {
        const unsigned m = 1u << k;
        if (p.line_block2[m] || p.line_cmodes[m]) {
            p.line_pos[m] = 0;
            p.fdm_cond[m] = p.line_cmodes[m] ? p.coarse_spec[k].cond : 1.0;
            p.sweeps[m] = 0;
        } else if (p.line_aniso) {
            p.line_pos[m] = lineq[k];
            p.fdm_cond[m] = condB[k];
            p.sweeps[m] = swB;
        } else {
            double c = 1.0;
            for (int q = 0; q < p.mesh[m].nfine; ++q) c *= cond_f[p.mesh[m].ax[q]];
            p.fdm_cond[m] = c;
            p.sweeps[m] = swA;  // the anisotropic meshes are solved together: the largest count
        }
    }
    // FP32 error guesses: transformed fine axes only, if the conditioning allows
    p.fp32_ok = !p.line_aniso;
    for (int k = 0; k < d && p.fp32_ok; ++k)
        if (6e-8 * p.fdm_cond[1u << k] > 1e-3) p.fp32_ok = false;
    // Intersection meshes: transforms of the fine axes and per-mode dense inverses of the coarse
    // block, unless a fine axis cannot be transformed: then it is the line axis (block cyclic
    // reduction with the coarse block as blocks).
    {
        double bytes = 0.0;
        for (unsigned s = 1; s < (1u << d); ++s) {
            if (__builtin_popcount(s) < 2) continue;
            const MeshDesc &m = p.mesh[s];
            double cA = 1.0;
            int wq = 0;
            for (int q = 0; q < m.nfine; ++q) {
                cA *= cond_f[m.ax[q]];
                if (cond_f[m.ax[q]] > cond_f[m.ax[wq]]) wq = q;
            }
            int sw = sweeps_for(cA);
            if (sw >= 0) {
                p.fdm_cond[s] = cA;
                p.sweeps[s] = sw;
                if (m.block > kDenseMaxBlock)
                    return fail(ASDSM_E_UNSUPPORTED, "intersection mesh with more than " +
                                                         std::to_string(kDenseMaxBlock) +
                                                         " coarse points per mode");
                bytes += 8.0 * (double)m.nmodes * m.block * m.block;
                continue;
            }
            double cB = 1.0;
            for (int q = 0; q < m.nfine; ++q)
                if (q != wq) cB *= cond_f[m.ax[q]];
            sw = sweeps_for(cB);
            if (sw < 0)
                return fail(ASDSM_E_UNSUPPORTED, "an intersection mesh has two fine axes that fast "
                                                 "diagonalisation cannot handle");
            if (m.block > kCrMaxBlock)
                return fail(ASDSM_E_UNSUPPORTED, "intersection mesh with a line axis and more than " +
                                                     std::to_string(kCrMaxBlock) + " coarse points");
            p.line_pos[s] = wq;
            p.fdm_cond[s] = cB;
            p.sweeps[s] = sw;
        }
        if (bytes > 2048.0 * 1024 * 1024)
            return fail(ASDSM_E_UNSUPPORTED, "intersection-mesh inverses exceed 2 GiB");
    }
    for (unsigned s = 1; s < (1u << d); ++s) {
        if (p.line_pos[s] >= 0) {
            if (!build_cr_tables(p, s)) return fail(ASDSM_E_NUMERIC, "singular block in the line solve");
        } else if (__builtin_popcount(s) >= 2) {
            if (!build_dense_inverse(p, s))
                return fail(ASDSM_E_NUMERIC, "singular intersection-mesh operator");
        }
    }
    for (unsigned m = 0; m < kMaxMeshes; ++m) p.sweeps_prior[m] = p.sweeps[m];
    // partial-sum capacity: the largest grid used by a reducing kernel
    p.max_blocks = 1 << 16;
    layout_workspace(p, nullptr, false);

    // device tables
    hipError_t err = hipGetDevice(&p.device);
    {
        static std::once_flag plane_once;
        std::call_once(plane_once, plane_prepare);
    }
    if (err != hipSuccess) return fail(ASDSM_E_DEVICE, std::string("hipGetDevice: ") + hipGetErrorString(err));
    if (int rc = noalloc_setup(p.device)) return rc;
    size_t off = 0;
    struct Item {
        size_t off;
        const void *data;
        size_t bytes;
    };
    std::vector<Item> items;
    auto add = [&](const std::vector<double> &v) {
        items.push_back({off, v.data(), v.size() * 8});
        size_t o = off;
        off = align256(off + v.size() * 8);
        return o;
    };
    auto add32 = [&](const std::vector<float> &v) {
        items.push_back({off, v.data(), v.size() * 4});
        size_t o = off;
        off = align256(off + v.size() * 4);
        return o;
    };
    size_t oW32[kMaxD] = {}, oV32[kMaxD] = {};
    for (int j = 0; j < d; ++j) {
        p.W32[j].assign(p.fine_spec[j].W.begin(), p.fine_spec[j].W.end());
        p.V32[j].assign(p.fine_spec[j].V.begin(), p.fine_spec[j].V.end());
        oW32[j] = add32(p.W32[j]);
        oV32[j] = add32(p.V32[j]);
    }
    size_t oW[kMaxD], oV[kMaxD], oM[kMaxD], oWh[kMaxD], oVh[kMaxD], oMh[kMaxD], oD[kMaxMeshes];
    for (int j = 0; j < d; ++j) {
        oW[j] = add(p.fine_spec[j].W);
        oV[j] = add(p.fine_spec[j].V);
        oM[j] = add(p.fine_spec[j].mu);
        oWh[j] = add(p.hole_spec[j].W);
        oVh[j] = add(p.hole_spec[j].V);
        oMh[j] = add(p.hole_spec[j].mu);
    }
    size_t oS = add(p.Sp);
    size_t oCR[kMaxMeshes] = {};
    for (unsigned s = 1; s < (1u << d); ++s) {
        if (p.line_pos[s] >= 0) oCR[s] = add(p.cr_tab[s]);
        else if (__builtin_popcount(s) >= 2) oD[s] = add(p.dense_inv[s]);
    }
    const size_t oH = p.hole_dense ? add(p.hole_inv) : 0;
    const size_t oHC = p.hole_cr ? add(p.hole_cr_tab) : 0;
    size_t oWc[kMaxD] = {}, oVc[kMaxD] = {};
    for (int k = 0; k < d; ++k)
        if (p.line_cmodes[1u << k]) {
            oWc[k] = add(p.coarse_spec[k].W);
            oVc[k] = add(p.coarse_spec[k].V);
        }
    p.dtab_bytes = off;
    err = hipMalloc(&p.dtab, p.dtab_bytes);
    if (err != hipSuccess) return fail(ASDSM_E_DEVICE, std::string("hipMalloc(tables): ") + hipGetErrorString(err));
    std::vector<char> host(p.dtab_bytes, 0);
    for (auto &it : items) std::memcpy(host.data() + it.off, it.data, it.bytes);
    err = hipMemcpy(p.dtab, host.data(), p.dtab_bytes, hipMemcpyHostToDevice);
    if (err != hipSuccess) return fail(ASDSM_E_DEVICE, std::string("hipMemcpy(tables): ") + hipGetErrorString(err));
    // the per-mode inverses live on the device only (up to 2 GiB)
    for (unsigned s = 0; s < kMaxMeshes; ++s) std::vector<double>().swap(p.dense_inv[s]);
    char *base = (char *)p.dtab;
    for (int j = 0; j < d; ++j) {
        p.dW[j] = (double *)(base + oW[j]);
        p.dV[j] = (double *)(base + oV[j]);
        p.dmu[j] = (double *)(base + oM[j]);
        p.dWh[j] = (double *)(base + oWh[j]);
        p.dVh[j] = (double *)(base + oVh[j]);
        p.dmuh[j] = (double *)(base + oMh[j]);
    }
    p.dSp = (double *)(base + oS);
    for (int j = 0; j < d; ++j) {
        p.dW32[j] = (float *)(base + oW32[j]);
        p.dV32[j] = (float *)(base + oV32[j]);
    }
    for (unsigned s = 1; s < (1u << d); ++s) {
        if (p.line_pos[s] >= 0) p.dcr[s] = (double *)(base + oCR[s]);
        else if (__builtin_popcount(s) >= 2) p.ddense[s] = (double *)(base + oD[s]);
    }
    for (unsigned s = 0; s < kMaxMeshes; ++s) std::vector<double>().swap(p.cr_tab[s]);
    if (p.hole_dense) p.dhinv = (double *)(base + oH);
    if (p.hole_cr) p.dhcr = (double *)(base + oHC);
    for (int k = 0; k < d; ++k)
        if (p.line_cmodes[1u << k]) {
            p.dWc[k] = (double *)(base + oWc[k]);
            p.dVc[k] = (double *)(base + oVc[k]);
        }
    std::vector<double>().swap(p.hole_inv);
    std::vector<double>().swap(p.hole_cr_tab);
    err = hipHostMalloc((void **)&p.hscal, kScalCount * sizeof(double), hipHostMallocDefault);
    if (err == hipSuccess) err = hipHostMalloc((void **)&p.hstate, sizeof(IterState), hipHostMallocDefault);
    if (err == hipSuccess)
        err = hipHostMalloc((void **)&p.hperm, (size_t)kHistCap * kMaxD * sizeof(int), hipHostMallocDefault);
    for (int i = 0; i < 2 && err == hipSuccess; ++i)
        err = hipHostMalloc((void **)&p.hstate_ring[i], sizeof(IterState), hipHostMallocDefault);
    if (err != hipSuccess) return fail(ASDSM_E_DEVICE, std::string("hipHostMalloc: ") + hipGetErrorString(err));
    return ASDSM_OK;
}

void release_plan(Plan &p) {
    if (p.graph_exec) (void)hipGraphExecDestroy(p.graph_exec);
    if (p.graph) (void)hipGraphDestroy(p.graph);
    if (p.capture_stream) (void)hipStreamDestroy(p.capture_stream);
    p.graph_exec = nullptr;
    p.graph = nullptr;
    p.capture_stream = nullptr;
    if (p.dtab) (void)hipFree(p.dtab);
    if (p.hscal) (void)hipHostFree(p.hscal);
    if (p.hstate) (void)hipHostFree(p.hstate);
    if (p.hperm) (void)hipHostFree(p.hperm);
    for (int i = 0; i < 2; ++i) {
        if (p.hstate_ring[i]) (void)hipHostFree(p.hstate_ring[i]);
        if (p.loop_ev[i]) (void)hipEventDestroy(p.loop_ev[i]);
        p.hstate_ring[i] = nullptr;
        p.loop_ev[i] = nullptr;
    }
    p.hstate = nullptr;
    p.hperm = nullptr;
    for (hipEvent_t e : p.ev_pool) (void)hipEventDestroy(e);
    p.ev_pool.clear();
    p.ev_recs.clear();
    p.dtab = nullptr;
    p.hscal = nullptr;
}

}  // namespace asdsm
