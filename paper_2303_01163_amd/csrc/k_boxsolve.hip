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
#include "skel_common.hpp"

namespace asdsm {

// ---------------------------------------------------------------------------------------------
// Batched FP64 GEMM on MFMA (v_mfma_f64_16x16x4f64) for the mode transforms.  Block = 4 waves, tile
// TM x TN, each wave one (TM/2) x (TN/2) quadrant of (TM/32) x (TN/32) MFMA tiles with independent
// accumulators.  K runs in chunks of KC staged in two LDS buffers: while the waves multiply chunk c,
// the loads of chunk c+1 are already in flight in registers, and one barrier per chunk separates
// the two buffers' uses.  Panels are loaded along the contiguous index of each operand (A is k-fast
// in every transform; B is k-fast or n-fast, template BKF).  Consecutive block ids go to consecutive
// XCDs; block b takes tile (b % 8) * per + b / 8 of the (z, tile y, tile x) order, so each XCD owns
// one contiguous range of tiles (tiles sharing an operand panel reuse its L2) and every XCD gets
// the same number of tiles.
// Operand layout of v_mfma_f64_16x16x4f64 (lane l, 0..63):
//   A: row l%16, k l/16;  B: k l/16, col l%16;  D[v]: row l/16 + 4v, col l%16.
// ---------------------------------------------------------------------------------------------
constexpr int kGemmPrefetch = 4;  // chunks whose loads k_gemm_f64 issues together
constexpr int kUpdPoints = 4;     // skeleton points per thread of an update block

// The line search's partial sums of the pending update, (<r,q>, <q,q>) pairs: thread t holds pairs t
// and t + 256 (zero beyond u.ndots <= 512), loaded at the start of the block so that they arrive
// with its other operands.
struct UpdDots {
    double v[4];
};
__device__ __forceinline__ UpdDots upd_load_dots(const UpdArgs &u) {
    UpdDots d;
#pragma unroll
    for (int it = 0; it < 2; ++it) {
        const int b = (int)threadIdx.x + 256 * it;
        const int bi = b < u.ndots ? b : 0;
        d.v[2 * it] = u.dots[2 * bi];
        d.v[2 * it + 1] = u.dots[2 * bi + 1];
    }
    return d;
}

// The step s = max(0, <r,q>/<q,q>), formed by every block from the same partial sums in the same
// order as k_skel_update (block_sum's: wave shuffles, then the waves in turn; all blocks agree bit
// for bit), then the flags (gv the stopping flag, pv the pending flag, both loaded earlier); block 0
// records <r,q>, <q,q> and s.  Its barriers order LDS only, so the block's operand loads stay in
// flight while the step is formed.
__device__ __forceinline__ void upd_step(const UpdArgs &u, const UpdDots &d, int gv, int pv, double &s, bool &pend,
                                         bool &live) {
    __shared__ double shu[8], s_sh;
    // the partial sums are taken here, not where they were loaded (the compiler would otherwise
    // wait for them there, before the block's other loads are issued)
    double v[4] = {d.v[0], d.v[1], d.v[2], d.v[3]};
    asm volatile("" : "+v"(v[0]), "+v"(v[1]), "+v"(v[2]), "+v"(v[3]));
    double a0 = 0.0, a1 = 0.0;
#pragma unroll
    for (int it = 0; it < 2; ++it) {
        const bool in = (int)threadIdx.x + 256 * it < u.ndots;
        a0 += in ? v[2 * it] : 0.0;
        a1 += in ? v[2 * it + 1] : 0.0;
    }
    for (int off = 32; off > 0; off >>= 1) {
        a0 += __shfl_down(a0, off, 64);
        a1 += __shfl_down(a1, off, 64);
    }
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) {
        shu[wid] = a0;
        shu[4 + wid] = a1;
    }
    lds_barrier();
    live = flag_clear(gv);
    pend = live && !flag_clear(pv);
    if (threadIdx.x == 0) {
        double rq = 0.0, qq = 0.0;
        for (int w = 0; w < 4; ++w) rq += shu[w];
        for (int w = 0; w < 4; ++w) qq += shu[4 + w];
        const double st = (qq > 0.0) ? rq / qq : 0.0;
        s_sh = (st > 0.0) ? st : 0.0;
        if (pend && blockIdx.x == 0) {
            u.scal[kScalRQ] = rq;
            u.scal[kScalQQ] = qq;
            u.scal[kScalStep] = s_sh;
        }
    }
    lds_barrier();
    s = s_sh;
}

// Update block xb of the fused launch (u.nub per box, box-major): the skeleton update on its
// points (skel_update_points) and, while a step is pending, its sum of r_next^2 at res_out[xb].
__device__ __forceinline__ void upd_block(const UpdArgs &u, int xb, int gv) {
    const int box = xb / u.nub, blk = xb - box * u.nub;
    if (box >= u.nbox) return;  // block-uniform
    const int pv = flag_load(&u.stt->pending);
    const UpdDots dd = upd_load_dots(u);
    const double *R = u.R[box];
    double *Rn = u.Rn[box];
    const double *Q = u.Q[box];
    const double *E = u.E[box];
    double *U = u.U[box];
    auto ready = [&](double &s, bool &pend, bool &live) { upd_step(u, dd, gv, pv, s, pend, live); };
    bool pend = false, live = false;
    double acc = 0.0;
    skel_update_points<kUpdPoints>(u.geo, u.mesh[box], blk, u.nub, R, Rn, Q, E, U, ready, pend, live, acc);
    if (pend && live) {  // block-uniform
        __shared__ double shr[4];
        const double tot = block_sum<256>(acc, shr);
        if (threadIdx.x == 0) u.res_out[xb] = tot;
    }
}

template <int TM, int TN, int KC, bool BKF, bool AKF, bool UPD = false>
__global__ __launch_bounds__(256) void k_gemm_f64(GemmJob job) {
    // the stopping flag is read with the first panel loads and tested once they have arrived
    const int gv = gate_value(job.gate);
    bool live = true;
    constexpr int MI = TM / 32, NI = TN / 32;            // MFMA tiles per wave along m and n
    constexpr int LA = TM * KC / 256, LB = KC * TN / 256;  // panel elements per thread
    __shared__ double sA[2][TM][KC + 1];
    __shared__ double sB[2][KC][TN + 1];
    const int tx = (job.N + TN - 1) / TN, ty = (job.M + TM - 1) / TM;
    const int per_z = tx * ty;
    const int total = per_z * job.nbox * job.nbatch;
    const int per = (total + 7) / 8;
    const int tile = (blockIdx.x & 7) * per + (blockIdx.x >> 3);
    if ((int)(blockIdx.x >> 3) >= per || tile >= total) {  // padding (block-uniform)
        // the blocks after the tiles, concurrently with them: the skeleton update (UPD), or a
        // pending stopping rule
        const int xb = (int)blockIdx.x - 8 * per;
        if (UPD && xb >= 0) upd_block(job.upd, xb, gv);
        else if (job.fin_on && xb == 0) finalize_pending(job.fin, gate_open(job.gate));
        return;
    }
    const int z = tile / per_z;
    const int rem = tile - z * per_z;
    const int by = rem / tx, bx = rem - by * tx;
    const int box = z / job.nbatch, bat = z - box * job.nbatch;
    const double *__restrict__ A = job.A[box] + (long long)bat * job.sAb;
    const double *__restrict__ B = job.B[box] + (long long)bat * job.sBb;
    const int m0 = by * TM, n0 = bx * TN;
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int wm = w & 1, wn = w >> 1;
    const int sAi = (int)job.sAi, sAk = (int)job.sAk, sBk = (int)job.sBk, sBn = (int)job.sBn;
    // panel element j of this thread: A (k-fast) row t/KC + (256/KC) j, k t%KC; A (m-fast) row
    // t%TM, k t/TM + (256/TM) j; B (k-fast) col t/KC + (256/KC) j, k t%KC; B (n-fast) k
    // t/TN + (256/TN) j, col t%TN
    const int ar = AKF ? t / KC : t % TM, ak = AKF ? t % KC : t / TM;
    const int bn0 = BKF ? (t / KC) : (t % TN), bk0 = BKF ? (t % KC) : (t / TN);
    double ra[LA], rb[LB];
    const int nch = (job.K + KC - 1) / KC;
    // fused skeleton update (UPD): the pending flag is read with the operands (nothing else in this
    // launch writes it), and q is loaded beside each B element (the current residual r)
    const int pv = UPD ? flag_load(&job.upd.stt->pending) : 0;
    UpdDots dd{};
    if (UPD) dd = upd_load_dots(job.upd);
    bool pend = false;
    const double *__restrict__ uQ = UPD ? job.upd.Q[box] : nullptr;
    double qb[LB];
    double s_upd = 0.0;
    // B element j of chunk c becomes r - s q (r while nothing is pending)
    auto stage_b = [&](int c, int j, double r, double q) -> double {
        const int n = n0 + (BKF ? bn0 + (256 / KC) * j : bn0);
        const int kb = c * KC + (BKF ? bk0 : bk0 + (256 / TN) * j);
        const bool in = n < job.N && kb < job.K;
        const double b = pend ? r - s_upd * q : r;
        return in ? b : 0.0;
    };
    // the step and the flags, once the operands are in flight
    auto form_step = [&]() {
        upd_step(job.upd, dd, gv, pv, s_upd, pend, live);
    };
    auto gload = [&](int c) {
        const int k0 = c * KC;
#pragma unroll
        for (int j = 0; j < LA; ++j) {
            const int row = m0 + ar + (AKF ? (256 / KC) * j : 0);
            const int k = k0 + ak + (AKF ? 0 : (256 / TM) * j);
            ra[j] = (row < job.M && k < job.K) ? (AKF ? A[row * sAi + k] : A[row + k * sAk]) : 0.0;
        }
#pragma unroll
        for (int j = 0; j < LB; ++j) {
            const int n = n0 + (BKF ? bn0 + (256 / KC) * j : bn0);
            const int kb = k0 + (BKF ? bk0 : bk0 + (256 / TN) * j);
            const bool in = n < job.N && kb < job.K;
            const int bi = in ? kb * sBk + n * sBn : 0;
            rb[j] = in ? B[bi] : 0.0;
            if (UPD) qb[j] = uQ[bi];
        }
    };
    auto lstore = [&](int buf, int c) {
        if (UPD && c >= 0) {  // c < 0: already staged
#pragma unroll
            for (int j = 0; j < LB; ++j) rb[j] = stage_b(c, j, rb[j], qb[j]);
        }
#pragma unroll
        for (int j = 0; j < LA; ++j) {
            if (AKF)
                sA[buf][ar + (256 / KC) * j][ak] = ra[j];
            else
                sA[buf][ar][ak + (256 / TM) * j] = ra[j];
        }
#pragma unroll
        for (int j = 0; j < LB; ++j) {
            if (BKF)
                sB[buf][bk0][bn0 + (256 / KC) * j] = rb[j];
            else
                sB[buf][bk0 + (256 / TN) * j][bn0] = rb[j];
        }
    };
    double4_t acc[MI][NI];
#pragma unroll
    for (int a = 0; a < MI; ++a)
#pragma unroll
        for (int b = 0; b < NI; ++b) acc[a][b] = {0.0, 0.0, 0.0, 0.0};
    auto mma = [&](int buf) {
#pragma unroll
        for (int kk = 0; kk < KC; kk += 4) {
            const int kq = kk + (lane >> 4);
            double av[MI], bv[NI];
#pragma unroll
            for (int a = 0; a < MI; ++a) av[a] = sA[buf][wm * (TM / 2) + a * 16 + (lane & 15)][kq];
#pragma unroll
            for (int b = 0; b < NI; ++b) bv[b] = sB[buf][kq][wn * (TN / 2) + b * 16 + (lane & 15)];
#pragma unroll
            for (int a = 0; a < MI; ++a)
#pragma unroll
                for (int b = 0; b < NI; ++b)
                    acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a], bv[b], acc[a][b], 0, 0, 0);
        }
    };
    if (nch <= kGemmPrefetch) {
        // short contractions (the mode transforms, K = N_f <= kGemmPrefetch * KC): every chunk's
        // loads are issued at once into registers, so the block waits for memory once; the chunks
        // then pass through the two LDS buffers in turn
        // (every lane loads every element, an out-of-range one from the operand's first element,
        // and zeroes it: straight-line loads, all in flight together)
        double pa[kGemmPrefetch][LA], pb[kGemmPrefetch][LB];
        double pq[UPD ? kGemmPrefetch : 1][LB];
#pragma unroll
        for (int c = 0; c < kGemmPrefetch; ++c) {
            const int k0 = c * KC;
#pragma unroll
            for (int j = 0; j < LA; ++j) {
                const int row = m0 + ar + (AKF ? (256 / KC) * j : 0);
                const int k = k0 + ak + (AKF ? 0 : (256 / TM) * j);
                const bool in = row < job.M && k < job.K;
                const double x = A[in ? (AKF ? row * sAi + k : row + k * sAk) : 0];
                pa[c][j] = in ? x : 0.0;
            }
#pragma unroll
            for (int j = 0; j < LB; ++j) {
                const int nn = n0 + (BKF ? bn0 + (256 / KC) * j : bn0);
                const int kb = k0 + (BKF ? bk0 : bk0 + (256 / TN) * j);
                const bool in = nn < job.N && kb < job.K;
                const int bi = in ? kb * sBk + nn * sBn : 0;
                const double x = B[bi];
                pb[c][j] = in ? x : 0.0;
                if (UPD) pq[c][j] = uQ[bi];
            }
        }
        if (UPD) {
            form_step();
#pragma unroll
            for (int c = 0; c < kGemmPrefetch; ++c)
#pragma unroll
                for (int j = 0; j < LB; ++j)
                    if (c < nch) pb[c][j] = stage_b(c, j, pb[c][j], pq[c][j]);
        }
        auto put = [&](int c) {
#pragma unroll
            for (int j = 0; j < LA; ++j) ra[j] = pa[c][j];
#pragma unroll
            for (int j = 0; j < LB; ++j) rb[j] = pb[c][j];
            lstore(c & 1, -1);
        };
        put(0);
        __syncthreads();
        if (!UPD) live = flag_clear(gv);
        if (!live) return;  // block-uniform
#pragma unroll
        for (int c = 0; c < kGemmPrefetch; ++c) {
            if (c < nch) {
                mma(c & 1);
                if (c + 1 < nch) put(c + 1);
                __syncthreads();
            }
        }
    } else {
        gload(0);
        if (UPD) form_step();
        lstore(0, 0);
        __syncthreads();
        if (!UPD) live = flag_clear(gv);
        if (!live) return;  // block-uniform
        for (int c = 0; c < nch; ++c) {
            const int buf = c & 1;
            if (c + 1 < nch) gload(c + 1);
            mma(buf);
            if (c + 1 < nch) lstore(buf ^ 1, c + 1);
            __syncthreads();
        }
    }
    double *__restrict__ C = job.C[box] + (long long)bat * job.sCb;
    double ss = 0.0;  // sum of squares of the values this thread writes (norm_out only)
#pragma unroll
    for (int a = 0; a < MI; ++a)
#pragma unroll
        for (int b = 0; b < NI; ++b)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int gi = m0 + wm * (TM / 2) + a * 16 + (lane >> 4) + 4 * v;
                const int gn = n0 + wn * (TN / 2) + b * 16 + (lane & 15);
                if (gi < job.M && gn < job.N) {
                    double *cp = C + (long long)gi * job.sCi + (long long)gn * job.sCn;
                    const double pr = job.neg ? -acc[a][b][v] : acc[a][b][v];
                    const double val = job.accum ? *cp + pr : pr;
                    *cp = val;
                    ss += val * val;
                }
            }
    if (job.norm_out[box]) {  // block-uniform
        __shared__ double sh[4];
        const double tot = block_sum<256>(ss, sh);
        if (t == 0) job.norm_out[box][bat * per_z + rem] = tot;
    }
}

template <int TM, int TN, int KC>
static void launch_gemm_tile(const GemmJob &job, hipStream_t st) {
    const long long tx = (job.N + TN - 1) / TN, ty = (job.M + TM - 1) / TM;
    const long long total = tx * ty * job.nbox * job.nbatch;
    const long long extra = job.upd_on ? (long long)job.upd.nbox * job.upd.nub : (job.fin_on ? 1 : 0);
    const dim3 grid((unsigned)(8 * ((total + 7) / 8) + extra));
    const bool akf = job.sAk == 1;
    if (job.upd_on) {  // checked by launch_gemm: A and B k-fast
        ASDSM_LAUNCH((k_gemm_f64<TM, TN, KC, true, true, true>), grid, dim3(256), 0, st, job);
        return;
    }
    if (job.sBk == 1) {
        if (akf) ASDSM_LAUNCH((k_gemm_f64<TM, TN, KC, true, true>), grid, dim3(256), 0, st, job);
        else ASDSM_LAUNCH((k_gemm_f64<TM, TN, KC, true, false>), grid, dim3(256), 0, st, job);
    } else {
        if (akf) ASDSM_LAUNCH((k_gemm_f64<TM, TN, KC, false, true>), grid, dim3(256), 0, st, job);
        else ASDSM_LAUNCH((k_gemm_f64<TM, TN, KC, false, false>), grid, dim3(256), 0, st, job);
    }
}

const char *gemm_tile_name(int tile) {
    switch (tile) {
        case kTile32x32: return "32x32 k32";
        case kTile64x32: return "64x32 k32";
        case kTile32x64: return "32x64 k32";
        case kTile64x64: return "64x64 k16";
        case kTilePlane: return "plane panels 16";
        default: return "auto";
    }
}

static int gemm_pick_tile(const GemmJob &job) {
    int tile = job.tile;
    if (tile == kTileAuto) {
        // 64 x 64 tiles once there are enough of them to fill the chip twice, else 32 x 32
        const long long t64 = ((job.N + 63) / 64) * ((job.M + 63) / 64) * job.nbox * job.nbatch;
        tile = (t64 >= 512) ? kTile64x64 : kTile32x32;
    }
    return tile;
}

int gemm_tiles_per_box(const GemmJob &job) {
    int tm = 32, tn = 32;
    switch (gemm_pick_tile(job)) {
        case kTile64x32: tm = 64; break;
        case kTile32x64: tn = 64; break;
        case kTile64x64: tm = tn = 64; break;
        default: break;
    }
    return ((job.N + tn - 1) / tn) * ((job.M + tm - 1) / tm) * job.nbatch;
}

int upd_blocks_per_box(const Geo &g) {
    const long long per = (long long)g.Nc * g.Nf * g.Nf;
    return (int)((per + 256 * kUpdPoints - 1) / (256 * kUpdPoints));
}

bool launch_gemm(const GemmJob &job, hipStream_t st) {
    // operand layouts of the mode transforms: A k-fast or m-fast, B k-fast or n-fast (any other
    // strides only when asked for: the kernel indexes them correctly, with uncoalesced panels)
    if (!job.any_layout && ((job.sAk != 1 && job.sAi != 1) || (job.sBk != 1 && job.sBn != 1))) return false;
    // the fused skeleton update: k-fast operands, one batch, no accumulation or norms, no carried
    // stopping rule (that reads what this launch writes)
    if (job.upd_on && (job.sAk != 1 || job.sBk != 1 || job.nbatch != 1 || job.accum || job.fin_on ||
                       job.upd.ndots > 512))
        return false;
    for (int b = 0; b < job.nbox && job.upd_on; ++b)
        if (job.norm_out[b]) return false;
    const int tile = gemm_pick_tile(job);
    switch (tile) {
        case kTile64x32: launch_gemm_tile<64, 32, 32>(job, st); break;
        case kTile32x64: launch_gemm_tile<32, 64, 32>(job, st); break;
        case kTile64x64: launch_gemm_tile<64, 64, 16>(job, st); break;
        default: launch_gemm_tile<32, 32, 32>(job, st); break;
    }
    return true;
}

// ---------------------------------------------------------------------------------------------
// Both fine-axis transforms of a d = 3 anisotropic box in one launch.  Each slab of constant coarse
// index is an N_f x N_f matrix X_c (row = second fine axis, column = first fine axis, contiguous
// rows) and becomes C_c = L X_c R^T (forward: L = W_b, R = W_a; backward: L = V_b, R = V_a).  One
// block (8 waves) owns a 16-column panel [m0, m0 + 16) of one slab, and the two products split
// without recomputation:
//     T = X_c R[m0:m0+16, :]^T  (N_f x 16, kept in LDS),   C_c[:, m0:m0+16] = L T.
// Wave w owns row tiles w, w + 8, ... (16 rows) of both products.  A row tile of the A operand
// (X_c or L) is staged through the wave's own LDS area in chunks of KC columns: sixteen row
// segments of KC contiguous doubles, one coalesced load per row, the next chunk's loads in flight
// in registers while the current chunk is multiplied; the MFMA fragments are then read from LDS.
// R's panel and T are LDS-resident for the whole block.  Consecutive block ids go to consecutive
// XCDs and each XCD takes a contiguous range of (box, slab, panel) items, so the panels of one slab
// share that XCD's L2 copy of X_c.  Indices past the row ends or the last row are clamped into the
// data: the B operand (R's panel, T) is zero there, and rows of T past N_f are set to zero.
// Operand layout of v_mfma_f64_16x16x4f64 (lane l): A row l%16, k l/16; B k l/16, col l%16;
// D[v] row l/16 + 4v, col l%16.
// ---------------------------------------------------------------------------------------------
template <int NT>
struct PlaneLds {
    static constexpr int KP = 16 * NT;                 // contraction length padded to whole tiles
    static constexpr int KC = KP < 64 ? KP : 64;       // staged columns per chunk
    static constexpr int PITCH = KC + 4;               // row pitch of a staged tile (doubles)
    static constexpr int STAGE = 16 * PITCH;           // one wave's staging area
    static constexpr size_t BYTES = (size_t)(2 * KP * 16 + 8 * STAGE) * sizeof(double);
};

template <int NT>
__global__ __launch_bounds__(512) void k_plane2(PlaneJob job) {
    if (job.gate && *job.gate) return;
    using S = PlaneLds<NT>;
    constexpr int KP = S::KP, KC = S::KC, NCH = KP / KC, RT = (NT + 7) / 8;
    extern __shared__ double smem[];
    double(*sR)[16] = reinterpret_cast<double(*)[16]>(smem);            // sR[k][n] = R[m0 + n][k]
    double(*sT)[16] = reinterpret_cast<double(*)[16]>(smem + KP * 16);  // T
    const int Nf = job.Nf;
    const int np = (Nf + 15) >> 4;
    const int total = job.nbox * job.nplanes * np;
    const int per = (total + 7) / 8;
    const int item = (blockIdx.x & 7) * per + (blockIdx.x >> 3);
    if ((int)(blockIdx.x >> 3) >= per || item >= total) return;  // padding (block-uniform)
    const int pan = item % np;
    const int zc = item / np;
    const int box = zc / job.nplanes, c = zc - box * job.nplanes;
    const long long slab = (long long)c * Nf * Nf;
    const double *__restrict__ X = job.X[box] + slab;
    double *__restrict__ C = job.C[box] + slab;
    const double *__restrict__ L = job.L[box];
    const double *__restrict__ R = job.R[box];
    const int m0 = pan * 16;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int ln = lane & 15, lg = lane >> 4;
    double *__restrict__ sA = smem + 2 * KP * 16 + w * S::STAGE;  // this wave's staging area
    // R's panel, n fastest across threads (contiguous LDS writes); indices clamped, values selected
#pragma unroll
    for (int e0 = 0; e0 < 16 * KP; e0 += 512) {
        const int e = e0 + tid, n = e & 15, k = e >> 4;
        const bool ok = m0 + n < Nf && k < Nf;
        sR[k][n] = R[(long long)(m0 + n < Nf ? m0 + n : Nf - 1) * Nf + (k < Nf ? k : Nf - 1)] * (ok ? 1.0 : 0.0);
    }
    // chunk ch of row tile rt of matrix A into registers: row r of the tile, column ch*KC + lane
    // (lanes past KC idle when KC < 64)
    double xr[16];
    auto fetch = [&](const double *__restrict__ A, int rt, int ch) {
        const int col = ch * KC + lane;
        const int cc = col < Nf ? col : Nf - 1;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int row = rt * 16 + r;
            xr[r] = A[(long long)(row < Nf ? row : 0) * Nf + cc];
        }
    };
    auto stage = [&]() {
        if (lane < KC) {
#pragma unroll
            for (int r = 0; r < 16; ++r) sA[r * S::PITCH + lane] = xr[r];
        }
    };
    auto mfma_chunk = [&](double4_t &acc, const double (*sB)[16], int ch) {
#pragma unroll
        for (int q = 0; q < KC / 4; ++q)
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(sA[ln * S::PITCH + 4 * q + lg], sB[ch * KC + 4 * q + lg][ln],
                                                       acc, 0, 0, 0);
    };
    // one product over this wave's row tiles: A (global, staged) times B (LDS); every wave runs the
    // same number of chunk steps, so the block barriers are uniform
    auto product = [&](const double *__restrict__ A, const double (*sB)[16], auto &&epilogue) {
#pragma unroll
        for (int i = 0; i < RT; ++i) {
            const int rt = w + 8 * i;
            double4_t acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int ch = 0; ch < NCH; ++ch) {
                __syncthreads();  // the previous chunk's fragment reads are done
                stage();
                __syncthreads();  // the staged chunk is visible
                // next loads in flight during the MFMAs: the next chunk, or the next tile's first
                if (ch + 1 < NCH)
                    fetch(A, rt < NT ? rt : 0, ch + 1);
                else if (i + 1 < RT)
                    fetch(A, rt + 8 < NT ? rt + 8 : 0, 0);
                if (rt < NT) mfma_chunk(acc, sB, ch);
            }
            if (rt < NT) epilogue(rt, acc);
        }
    };
    // T = X_c R_panel^T; rows of T past N_f are zero
    fetch(X, w < NT ? w : 0, 0);
    product(X, sR, [&](int rt, const double4_t &acc) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int tr = rt * 16 + lg + 4 * v;
            sT[tr][ln] = tr < Nf ? acc[v] : 0.0;
        }
    });
    // C_c[:, m0:m0+16] = L T (the first chunk of L is fetched before the barrier that publishes T,
    // which the first chunk step of the product provides)
    fetch(L, w < NT ? w : 0, 0);
    const int col = m0 + ln;
    double ss = 0.0;  // sum of squares of the values this thread writes
    product(L, sT, [&](int rt, const double4_t &acc) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int orow = rt * 16 + lg + 4 * v;
            if (orow < Nf && col < Nf) {
                double *cp = C + (long long)orow * Nf + col;
                const double val = job.accum ? *cp + acc[v] : acc[v];
                *cp = val;
                ss += val * val;
            }
        }
    });
    if (job.norm_partials) {
        __shared__ double sh[8];
        const double t = block_sum<512>(ss, sh);
        if (tid == 0) job.norm_partials[item] = t;
    }
}

template <int NT>
static void plane_prepare_one() {
    (void)hipFuncSetAttribute((const void *)k_plane2<NT>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)PlaneLds<NT>::BYTES);
}

void plane_prepare() {
    // the staging areas take the kernels past 64 KB of dynamic LDS
    plane_prepare_one<2>();
    plane_prepare_one<4>();
    plane_prepare_one<8>();
    plane_prepare_one<16>();
}

bool launch_plane2(const PlaneJob &job, hipStream_t st) {
    const int nt = (job.Nf + 15) / 16;
    const long long total = (long long)job.nbox * job.nplanes * nt;
    const dim3 grid((unsigned)(8 * ((total + 7) / 8))), blk(512);
    if (nt <= 2) ASDSM_LAUNCH((k_plane2<2>), grid, blk, PlaneLds<2>::BYTES, st, job);
    else if (nt <= 4) ASDSM_LAUNCH((k_plane2<4>), grid, blk, PlaneLds<4>::BYTES, st, job);
    else if (nt <= 8) ASDSM_LAUNCH((k_plane2<8>), grid, blk, PlaneLds<8>::BYTES, st, job);
    else if (nt <= 16) ASDSM_LAUNCH((k_plane2<16>), grid, blk, PlaneLds<16>::BYTES, st, job);
    else return false;
    return true;
}

// FP32 variant for the mixed-precision error guesses (v_mfma_f32_16x16x4f32, FP32 accumulation):
// the same tiling and double buffering; A is read as TA (double: the FP64 right-hand side is
// rounded to FP32 while it is staged), B is FP32, C is written as TC (double: the solution goes
// back to the FP64 buffers).  The GemmJob pointers are reinterpreted accordingly.
// Output layout of the FP32 16x16x4 MFMA: D[v] at row 4 (l/16) + v, col l%16.
template <int TM, int TN, int KC, bool BKF, typename TA, typename TC>
__global__ __launch_bounds__(256) void k_gemm_f32(GemmJob job) {
    if (job.gate && *job.gate) return;
    constexpr bool AKF = true;  // the FP32 transforms take k-fast A operands only
    constexpr int MI = TM / 32, NI = TN / 32;
    constexpr int LA = TM * KC / 256, LB = KC * TN / 256;
    __shared__ float sA[2][TM][KC + 1];
    __shared__ float sB[2][KC][TN + 1];
    const int tx = (job.N + TN - 1) / TN, ty = (job.M + TM - 1) / TM;
    const int per_z = tx * ty;
    const int total = per_z * job.nbox * job.nbatch;
    const int per = (total + 7) / 8;
    const int tile = (blockIdx.x & 7) * per + (blockIdx.x >> 3);
    if ((int)(blockIdx.x >> 3) >= per || tile >= total) return;
    const int z = tile / per_z;
    const int rem = tile - z * per_z;
    const int by = rem / tx, bx = rem - by * tx;
    const int box = z / job.nbatch, bat = z - box * job.nbatch;
    const TA *__restrict__ A = reinterpret_cast<const TA *>(job.A[box]) + (long long)bat * job.sAb;
    const float *__restrict__ B = reinterpret_cast<const float *>(job.B[box]) + (long long)bat * job.sBb;
    const int m0 = by * TM, n0 = bx * TN;
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int wm = w & 1, wn = w >> 1;
    const int sAi = (int)job.sAi, sBk = (int)job.sBk, sBn = (int)job.sBn;
    const int ar = t / KC, ak = t % KC;
    const int bn0 = BKF ? (t / KC) : (t % TN), bk0 = BKF ? (t % KC) : (t / TN);
    float ra[LA], rb[LB];
    const int nch = (job.K + KC - 1) / KC;
    auto gload = [&](int c) {
        const int k0 = c * KC;
#pragma unroll
        for (int j = 0; j < LA; ++j) {
            const int row = m0 + ar + (256 / KC) * j, k = k0 + ak;
            ra[j] = (row < job.M && k < job.K) ? (float)A[row * sAi + k] : 0.f;
        }
#pragma unroll
        for (int j = 0; j < LB; ++j) {
            const int n = n0 + (BKF ? bn0 + (256 / KC) * j : bn0);
            const int kb = k0 + (BKF ? bk0 : bk0 + (256 / TN) * j);
            rb[j] = (n < job.N && kb < job.K) ? B[kb * sBk + n * sBn] : 0.f;
        }
    };
    auto lstore = [&](int buf) {
#pragma unroll
        for (int j = 0; j < LA; ++j) {
            if (AKF)
                sA[buf][ar + (256 / KC) * j][ak] = ra[j];
            else
                sA[buf][ar][ak + (256 / TM) * j] = ra[j];
        }
#pragma unroll
        for (int j = 0; j < LB; ++j) {
            if (BKF)
                sB[buf][bk0][bn0 + (256 / KC) * j] = rb[j];
            else
                sB[buf][bk0 + (256 / TN) * j][bn0] = rb[j];
        }
    };
    float4_t acc[MI][NI];
#pragma unroll
    for (int a = 0; a < MI; ++a)
#pragma unroll
        for (int b = 0; b < NI; ++b) acc[a][b] = {0.f, 0.f, 0.f, 0.f};
    gload(0);
    lstore(0);
    __syncthreads();
    for (int c = 0; c < nch; ++c) {
        const int buf = c & 1;
        if (c + 1 < nch) gload(c + 1);
#pragma unroll
        for (int kk = 0; kk < KC; kk += 4) {
            const int kq = kk + (lane >> 4);
            float av[MI], bv[NI];
#pragma unroll
            for (int a = 0; a < MI; ++a) av[a] = sA[buf][wm * (TM / 2) + a * 16 + (lane & 15)][kq];
#pragma unroll
            for (int b = 0; b < NI; ++b) bv[b] = sB[buf][kq][wn * (TN / 2) + b * 16 + (lane & 15)];
#pragma unroll
            for (int a = 0; a < MI; ++a)
#pragma unroll
                for (int b = 0; b < NI; ++b)
                    acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[a], bv[b], acc[a][b], 0, 0, 0);
        }
        if (c + 1 < nch) lstore(buf ^ 1);
        __syncthreads();
    }
    TC *__restrict__ C = reinterpret_cast<TC *>(job.C[box]) + (long long)bat * job.sCb;
#pragma unroll
    for (int a = 0; a < MI; ++a)
#pragma unroll
        for (int b = 0; b < NI; ++b)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int gi = m0 + wm * (TM / 2) + a * 16 + 4 * (lane >> 4) + v;
                const int gn = n0 + wn * (TN / 2) + b * 16 + (lane & 15);
                if (gi < job.M && gn < job.N) {
                    TC *cp = C + (long long)gi * job.sCi + (long long)gn * job.sCn;
                    *cp = job.accum ? (TC)(*cp + acc[a][b][v]) : (TC)acc[a][b][v];
                }
            }
}

template <int TM, int TN, int KC, typename TA, typename TC>
static void launch_gemm32_tile(const GemmJob &job, hipStream_t st) {
    const long long tx = (job.N + TN - 1) / TN, ty = (job.M + TM - 1) / TM;
    const long long total = tx * ty * job.nbox * job.nbatch;
    const dim3 grid((unsigned)(8 * ((total + 7) / 8)));
    if (job.sBk == 1)
        ASDSM_LAUNCH((k_gemm_f32<TM, TN, KC, true, TA, TC>), grid, dim3(256), 0, st, job);
    else
        ASDSM_LAUNCH((k_gemm_f32<TM, TN, KC, false, TA, TC>), grid, dim3(256), 0, st, job);
}

template <typename TA, typename TC>
static void launch_gemm32_io(const GemmJob &job, hipStream_t st) {
    const long long t64 = ((job.N + 63) / 64) * ((job.M + 63) / 64) * job.nbox * job.nbatch;
    if (t64 >= 512)
        launch_gemm32_tile<64, 64, 32, TA, TC>(job, st);
    else
        launch_gemm32_tile<32, 32, 32, TA, TC>(job, st);
}

bool launch_gemm32(const GemmJob &job, bool a_f64, bool c_f64, hipStream_t st) {
    if (job.sAk != 1 || (job.sBk != 1 && job.sBn != 1)) return false;
    if (a_f64 && c_f64) launch_gemm32_io<double, double>(job, st);
    else if (a_f64) launch_gemm32_io<double, float>(job, st);
    else if (c_f64) launch_gemm32_io<float, double>(job, st);
    else launch_gemm32_io<float, float>(job, st);
    return true;
}

// ---------------------------------------------------------------------------------------------
// Thomas elimination along the coarse axis, one thread per mode, boxes along blockIdx.y.  Lines of
// up to NCR points stay in registers (loads issued together); longer lines use the scratch array.
// ---------------------------------------------------------------------------------------------
template <int NCR, typename T>
__global__ __launch_bounds__(256) void k_line(LineJob job) {
    if (job.gate && *job.gate) return;
    const int box = blockIdx.y;
    const long long m = (long long)blockIdx.x * 256 + threadIdx.x;
    if (m >= job.nmodes) return;
    T *__restrict__ X = reinterpret_cast<T *>(job.X[box]);
    T *__restrict__ S = reinterpret_cast<T *>(job.scratch[box]);
    const Tri t64 = job.t[box];
    const T ta = (T)t64.a, tc = (T)t64.c;
    const int ma = (int)(m % job.ext_a);
    long long mb = m / job.ext_a;
    double sigma = job.mu_a[box][ma];
    if (job.mu_c[box]) {  // three fine axes of extent ext_a (d = 4)
        sigma += job.mu_c[box][mb / job.ext_a];
        mb %= job.ext_a;
    }
    if (job.mu_b[box]) sigma += job.mu_b[box][mb];
    const long long st = job.nmodes;
    const T diag = (T)(t64.b + sigma);
    const int nc = job.ncoarse;
    if (NCR > 0) {
        T f[NCR > 0 ? NCR : 1], cp[NCR > 0 ? NCR : 1];
#pragma unroll
        for (int c = 0; c < NCR; ++c)
            if (c < nc) f[c] = X[m + st * c];
        T den = diag;
        cp[0] = tc / den;
        f[0] = f[0] / den;
#pragma unroll
        for (int c = 1; c < NCR; ++c)
            if (c < nc) {
                den = diag - ta * cp[c - 1];
                f[c] = (f[c] - ta * f[c - 1]) / den;
                cp[c] = tc / den;
            }
#pragma unroll
        for (int c = NCR - 2; c >= 0; --c)
            if (c < nc - 1) f[c] = f[c] - cp[c] * f[c + 1];
#pragma unroll
        for (int c = 0; c < NCR; ++c)
            if (c < nc) X[m + st * c] = f[c];
        return;
    }
    T den = diag;
    T cq = tc / den;
    T dp = X[m] / den;
    S[m] = cq;
    X[m] = dp;
    for (int c = 1; c < nc; ++c) {
        den = diag - ta * cq;
        const T fc = X[m + st * c];
        dp = (fc - ta * dp) / den;
        cq = tc / den;
        S[m + st * c] = cq;
        X[m + st * c] = dp;
    }
    T x = dp;
    for (int c = nc - 2; c >= 0; --c) {
        x = X[m + st * c] - S[m + st * c] * x;
        X[m + st * c] = x;
    }
}

void launch_line(const LineJob &job, hipStream_t st) {
    dim3 grid((unsigned)((job.nmodes + 255) / 256), job.nbox, 1);
    if (job.fp32) {
        if (job.ncoarse <= 7)
            ASDSM_LAUNCH((k_line<7, float>), grid, dim3(256), 0, st, job);
        else if (job.ncoarse <= 15)
            ASDSM_LAUNCH((k_line<15, float>), grid, dim3(256), 0, st, job);
        else if (job.ncoarse <= 31)
            ASDSM_LAUNCH((k_line<31, float>), grid, dim3(256), 0, st, job);
        else
            ASDSM_LAUNCH((k_line<0, float>), grid, dim3(256), 0, st, job);
        return;
    }
    if (job.ncoarse <= 7)
        ASDSM_LAUNCH((k_line<7, double>), grid, dim3(256), 0, st, job);
    else if (job.ncoarse <= 15)
        ASDSM_LAUNCH((k_line<15, double>), grid, dim3(256), 0, st, job);
    else if (job.ncoarse <= 31)
        ASDSM_LAUNCH((k_line<31, double>), grid, dim3(256), 0, st, job);
    else
        ASDSM_LAUNCH((k_line<0, double>), grid, dim3(256), 0, st, job);
}

// ---------------------------------------------------------------------------------------------
// Per-mode dense solve: out[m + nmodes*r] = sum_e inv_m(r, e) in[m + nmodes*e], the inverse of mode
// m stored column by column (inv[(m*B + e)*B + r]) so that a wave reads 64 consecutive rows.  Block
// (row chunk of 64, mode): the mode's input vector is staged in LDS, the four waves split the sum
// over e and combine their partial sums through LDS.
// ---------------------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_dense_modes(long long nmodes, int B,
                                                     const double *__restrict__ inv,
                                                     const double *__restrict__ in,
                                                     double *__restrict__ out, int accum) {
    __shared__ double x[kDenseMaxBlock];
    __shared__ double part[4][64];
    const long long m = blockIdx.y;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    for (int e = threadIdx.x; e < B; e += 256) x[e] = in[m + nmodes * e];
    __syncthreads();
    const int r = blockIdx.x * 64 + lane;
    const int per = (B + 3) / 4;
    const int e0 = w * per, e1 = min(B, e0 + per);
    double acc = 0.0;
    if (r < B) {
        const double *__restrict__ col = inv + ((size_t)m * B) * B + r;
        for (int e = e0; e < e1; ++e) acc += col[(size_t)e * B] * x[e];
    }
    part[w][lane] = acc;
    __syncthreads();
    if (w == 0 && r < B) {
        const double v = ((part[0][lane] + part[1][lane]) + part[2][lane]) + part[3][lane];
        double *o = out + m + nmodes * r;
        *o = accum ? *o + v : v;
    }
}

void launch_dense_modes(long long nmodes, int B, const double *inv, const double *in, double *out,
                        int accum, hipStream_t st) {
    dim3 grid((unsigned)((B + 63) / 64), (unsigned)nmodes);
    ASDSM_LAUNCH(k_dense_modes, grid, dim3(256), 0, st, nmodes, B, inv, in, out, accum);
}

// ---------------------------------------------------------------------------------------------
// ||e_k||^2 of each anisotropic box and the normalisation factor 1/||e_k|| (Algorithm 1 steps
// 2.1/2.2; a zero vector is left unscaled).
// ---------------------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_box_norms(BoxPtrs X, long long size, double *partials,
                                                   const int *gate) {
    if (gate && *gate) return;
    const int k = blockIdx.y;
    const double *__restrict__ x = X.p[k];
    double acc = 0.0;
    // unrolled: the loads of several trips in flight, the additions in order
#pragma unroll 8
    for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < size; i += (long long)gridDim.x * 256)
        acc += x[i] * x[i];
    double vals[1] = {acc};
    block_partials<256, 1>(vals, partials + (size_t)k * gridDim.x, blockIdx.x);
}

void launch_box_norms(const Plan &p, const double *const *sol, hipStream_t st) {
    BoxPtrs bx;
    for (int k = 0; k < kMaxD; ++k) bx.p[k] = (k < p.d) ? const_cast<double *>(sol[1u << k]) : nullptr;
    const long long size = p.mesh[1].size;
    // about 16 values per thread, 128 to 1024 blocks per mesh
    const int nblk = (int)std::min<long long>(1024, std::max<long long>(128, (size + 4095) / 4096));
    ASDSM_LAUNCH(k_box_norms, dim3(nblk, p.d, 1), dim3(256), 0, st, bx, size, p.ws.partials, p.gate);
    launch_finalize(p, nblk, kFinBoxNorms, p.d, st);
}

// ---------------------------------------------------------------------------------------------
// Mesh residual out = f - A_S x (zero Dirichlet data) in the canonical layout of M_S.
// ---------------------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_box_residual(Geo g, BoxResJob job) {
    if (job.gate && *job.gate) return;
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
    ASDSM_LAUNCH(k_box_residual, dim3((unsigned)blocks, job.nbox, 1), dim3(256), 0, st, p.geo, job);
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
    ASDSM_LAUNCH(k_axpy, dim3((unsigned)blocks, nbox, 1), dim3(256), 0, st, job, n);
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
    ASDSM_LAUNCH(k_fill_random, dim3((unsigned)blocks), dim3(256), 0, st, x, n, (unsigned long long)seed);
}

constexpr int kNormBlocks = 128;

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
    ASDSM_LAUNCH(k_sumsq, dim3(kNormBlocks, nbox, 1), dim3(256), 0, st, job, p.ws.partials);
    launch_finalize(p, kNormBlocks, kFinBoxNorms, nbox, st);
}

}  // namespace asdsm
