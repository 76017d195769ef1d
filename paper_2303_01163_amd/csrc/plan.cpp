// Host-side plan: validation, mesh geometry, 1D operator spectra, transform matrices, spline
// matrix, dense per-mode inverses of the intersection meshes, workspace layout.
//
// Paper references: meshes and nesting condition, Section 2.1 eqs. (3)-(5); discretisation,
// Section 2.3; the submesh family for d = 3, Section 3.5; the spline of the cross-point
// discrepancy, Algorithm 2 step 5 (cubic with zero end values; here the not-a-knot end rule).
#include <algorithm>
#include <cmath>
#include <cstring>
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
    // fast diagonalisation needs real spectra on the fine axes: |beta h / (2 alpha)| < 1
    for (int j = 0; j < d; ++j) {
        const double P = std::fabs(beta[j] * p.h / (2.0 * alpha[j]));
        if (!(P < 1.0))
            return fail(ASDSM_E_UNSUPPORTED, "cell Peclet number >= 1 on fine axis " +
                                                 std::to_string(j) + " (complex spectrum)");
        spectrum(g.fine[j], p.Nf, p.fine_spec[j]);
        spectrum(g.fine[j], p.n - 1, p.hole_spec[j]);
    }
    // hole line axis: the worst-conditioned axis is eliminated, the others are transformed
    p.hole_line_axis = 0;
    for (int j = 1; j < d; ++j)
        if (p.hole_spec[j].cond > p.hole_spec[p.hole_line_axis].cond) p.hole_line_axis = j;
    build_spline(p.Nf, p.Nc, p.n, p.h, p.H, p.Sp);
    for (unsigned s = 0; s < (1u << d); ++s) p.mesh[s] = make_mesh(d, p.Nf, p.Nc, s);
    // intersection meshes: per-mode dense inverses of at most kDenseMaxBlock coarse points, at most
    // 2 GiB in total (d = 4 at 63^4 with N_c = 7 needs 0.74 GB)
    {
        double bytes = 0.0;
        for (unsigned s = 1; s < (1u << d); ++s)
            if (__builtin_popcount(s) >= 2) {
                const MeshDesc &m = p.mesh[s];
                if (m.block > kDenseMaxBlock)
                    return fail(ASDSM_E_UNSUPPORTED, "intersection mesh with more than " +
                                                         std::to_string(kDenseMaxBlock) +
                                                         " coarse points per mode");
                bytes += 8.0 * (double)m.nmodes * m.block * m.block;
            }
        if (bytes > 2048.0 * 1024 * 1024)
            return fail(ASDSM_E_UNSUPPORTED, "intersection-mesh inverses exceed 2 GiB");
    }
    for (unsigned s = 1; s < (1u << d); ++s) {
        if (__builtin_popcount(s) >= 2) {
            if (!build_dense_inverse(p, s))
                return fail(ASDSM_E_NUMERIC, "singular intersection-mesh operator");
        }
    }
    // Fast diagonalisation of a fine axis uses the eigenvector matrix V = D Q with
    // cond(V) = r^(N-1), so a mesh solve is accurate to about eps * prod cond(V_j) over its
    // transformed axes.  Where that exceeds 2e-11 the direct solve becomes the preconditioner of
    // FP64 refinement sweeps x <- x + M^-1 (f - A x), each gaining -log10(eps * prod cond) digits;
    // the count is fixed here so that the result reaches ~1e-14.
    p.fp32_ok = true;  // FP32 error guesses: every d, if the conditioning below allows
    for (unsigned s = 1; s < (1u << d); ++s) {
        double c = 1.0;
        for (int q = 0; q < p.mesh[s].nfine; ++q) c *= p.fine_spec[p.mesh[s].ax[q]].cond;
        p.fdm_cond[s] = c;
        if (__builtin_popcount(s) == 1 && 6e-8 * c > 1e-3) p.fp32_ok = false;
        const double delta = 2.2e-16 * c;
        if (delta <= 2e-11) {
            p.sweeps[s] = 0;
        } else if (delta >= 0.05) {
            return fail(ASDSM_E_UNSUPPORTED,
                        "fine-axis eigenvector matrices too ill-conditioned for fast diagonalisation "
                        "(|cell Peclet| close to 1 on two axes)");
        } else {
            p.sweeps[s] = (int)std::ceil(std::log(1e-14) / std::log(delta)) - 1;
            if (p.sweeps[s] < 1) p.sweeps[s] = 1;
        }
    }
    {
        // the anisotropic meshes are solved together: they share the largest sweep count
        int smax = 0;
        for (int k = 0; k < d; ++k) smax = std::max(smax, p.sweeps[1u << k]);
        for (int k = 0; k < d; ++k) p.sweeps[1u << k] = smax;
        for (unsigned m = 0; m < kMaxMeshes; ++m) p.sweeps_prior[m] = p.sweeps[m];
    }
    {
        double ch = 1.0;
        for (int j = 0; j < d; ++j)
            if (j != p.hole_line_axis) ch *= p.hole_spec[j].cond;
        if (2.2e-16 * ch > 1e-12)
            return fail(ASDSM_E_UNSUPPORTED, "hole-box transforms too ill-conditioned");
    }
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
    // hole line factors: Thomas along the line axis for every mode pair of the transformed axes
    size_t oHI = 0, oHC = 0;
    if (d == 3) {
        const int nh = p.n - 1, L = p.hole_line_axis;
        int tr[2], nt = 0;
        for (int j = 0; j < d; ++j)
            if (j != L) tr[nt++] = j;
        const Tri t = p.geo.fine[L];
        p.hole_inv.assign((size_t)nh * nh * nh, 0.0);
        p.hole_cp.assign((size_t)nh * nh * nh, 0.0);
        for (int m1 = 0; m1 < nh; ++m1)
            for (int m0 = 0; m0 < nh; ++m0) {
                const size_t q = (size_t)m0 + (size_t)nh * m1;
                const double diag = t.b + (p.hole_spec[tr[0]].mu[m0] + p.hole_spec[tr[1]].mu[m1]);
                double cp = 0.0;
                for (int c = 0; c < nh; ++c) {
                    const double den = (c == 0) ? diag : diag - t.a * cp;
                    cp = t.c / den;
                    p.hole_inv[(size_t)c * nh * nh + q] = 1.0 / den;
                    p.hole_cp[(size_t)c * nh * nh + q] = cp;
                }
            }
        oHI = add(p.hole_inv);
        oHC = add(p.hole_cp);
    }
    size_t oS = add(p.Sp);
    for (unsigned s = 1; s < (1u << d); ++s)
        if (__builtin_popcount(s) >= 2) oD[s] = add(p.dense_inv[s]);
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
    if (d == 3) {
        p.dhole_inv = (double *)(base + oHI);
        p.dhole_cp = (double *)(base + oHC);
    }
    for (unsigned s = 1; s < (1u << d); ++s)
        if (__builtin_popcount(s) >= 2) p.ddense[s] = (double *)(base + oD[s]);
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
