// Learned correction network (a small 3D convolutional net proposing refinement corrections):
// conv3d 3x3x3 with zero padding, BF16 operands on MFMA with FP32 accumulation, fused bias and
// ReLU; its backward passes (data: the same kernel on spatially flipped, channel-transposed
// weights; weights: FP32 sums over voxel tiles reduced in a fixed order); MSE loss; Adam.
//
// Layouts.  A volume of n^3 voxels, v = x + n (y + n z).  Activations are FP32, channels last,
// padded to 16 or 32 channels: act[v * CP + c].  Weights: FP32 master and BF16 copy, as
// w[co][tap][ci] (tap = (dz+1)*9 + (dy+1)*3 + (dx+1)), co and ci padded like the activations.
// Operand layout of v_mfma_f32_16x16x16bf16_1k (lane l): A[l%16][4(l/16)+t], B[4(l/16)+t][l%16],
// t = 0..3; D[v] at row 4(l/16)+v, col l%16.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "device_common.hpp"
#include "kernels.hpp"
#include "learn_internal.hpp"

namespace asdsm {

typedef short short4_t __attribute__((ext_vector_type(4)));

// FP32 -> BF16 with round-to-nearest-even (finite inputs).
__device__ __forceinline__ unsigned short to_bf16(float x) {
    const unsigned u = __float_as_uint(x);
    const unsigned r = u + 0x7FFFu + ((u >> 16) & 1u);
    return (unsigned short)(r >> 16);
}


// ---------------------------------------------------------------------------------------------
// Forward convolution, z-marching.  A block (8 waves) owns a 64 (x) by 4 (y) column of output
// voxels over a chunk of zc planes.  Wave w covers the 16 x-voxels 16 (w % 4) .. +15 and one N tile
// of 16 output channels: with COT = 2 tiles, tile w / 4 for all 4 rows; with COT = 1, rows
// 2 (w / 4) and 2 (w / 4) + 1.  The layer's BF16 weights sit in LDS for the whole block, as
// w[tap][co][ci]; the input (FP32 in memory, rounded to BF16 when staged) passes through a ring of
// three LDS planes of 6 x 66 voxels with their halo, the plane two steps ahead being fetched into
// registers while the current plane is computed.  For each (dz, dx) a wave reads the A fragments
// of its input rows once and uses each for up to three output rows (dy).  CIN = 32:
// v_mfma_f32_16x16x32_bf16, one instruction per tap; CIN = 16: v_mfma_f32_16x16x16bf16_1k.
// out[v*cop + co] = bias[co] + sum, ReLU when RELU, for co < cout.  The staged planes' channel
// stride is padded by 8 BF16 values (aligned 16-byte fragments without bank conflicts).
// Operand layouts (lane l): 16x16x32: A[l%16][8(l/16)+t], B[8(l/16)+t][l%16], t < 8;
// 16x16x16: A[l%16][4(l/16)+t], B[4(l/16)+t][l%16], t < 4; both D[v] at row 4(l/16)+v, col l%16.
// ---------------------------------------------------------------------------------------------
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));

constexpr int kConvThreads = 512;

template <int CIN, int COT>
struct ConvLds {
    static constexpr int CS = CIN + 8;                 // staged plane channel stride (BF16 values)
    static constexpr int PLANE = 6 * 66 * CS;          // one staged input plane
    static constexpr int WSZ = 27 * COT * 16 * CIN;    // the weights, unpadded
    static constexpr int LOADS = 6 * 66 * CIN / 4;     // float4 loads per plane
    static constexpr int PER_THREAD = (LOADS + kConvThreads - 1) / kConvThreads;
    static constexpr size_t BYTES = 2 * (size_t)(3 * PLANE + WSZ);
};

// One MFMA step of the convolution: K = 32 (16x16x32, 8 values per lane) or 16 (16x16x16, 4).
template <int CIN>
using ConvFrag = typename std::conditional<CIN == 32, bf16x8_t, short4_t>::type;

template <int CIN>
__device__ __forceinline__ float4_t conv_mfma(const ConvFrag<CIN> &a, const ConvFrag<CIN> &b, float4_t c) {
    if constexpr (CIN == 32)
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
    else
        return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

// XB: the input is stored as BF16 (else FP32, rounded when staged); OB: the output is stored as
// BF16 (round to nearest even, else FP32).
template <int CIN, int COT, bool RELU, bool XB, bool OB>
__global__ __launch_bounds__(kConvThreads) void k_conv_fwd(int n, int zc, const void *__restrict__ xv,
                                                           const unsigned short *__restrict__ w,
                                                           const float *__restrict__ bias, int cout, int cop,
                                                           void *__restrict__ outv, const int *gate) {
    static_assert(CIN == 16 || CIN == 32, "16 or 32 input channels");
    static_assert(COT == 1 || COT == 2, "16 or 32 output channels");
    if (gate && *gate) return;
    using Lds = ConvLds<CIN, COT>;
    using Frag = ConvFrag<CIN>;
    constexpr int CS = Lds::CS, CO = COT * 16, NT = kConvThreads;
    constexpr int ROWS = (COT == 2) ? 4 : 2;  // output rows per wave
    extern __shared__ __attribute__((aligned(16))) unsigned short lds[];
    unsigned short *sw = lds;                       // [27][CO][CIN]
    unsigned short *sp = lds + Lds::WSZ;            // [3][6][66][CS]
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int mt = wave & 3;                                   // M tile (16 x-voxels)
    const int ct = (COT == 2) ? (wave >> 2) : 0;               // N tile
    const int r0 = (COT == 2) ? 0 : 2 * (wave >> 2);           // first output row
    const int xtn = (n + 63) / 64, ytn = (n + 3) / 4;
    const int b = blockIdx.x;
    const int xt = b % xtn, yt = (b / xtn) % ytn, zt = b / (xtn * ytn);
    const int x0 = xt * 64, y0 = yt * 4, z0 = zt * zc;
    const int z1 = min(z0 + zc, n);
    // weights: global w[co][tap][ci] -> LDS [tap][co][ci], each row's four fragment chunks (KL
    // values) permuted by (co >> SH) & 3 so that the 16 rows one fragment read touches fall in
    // distinct banks
    constexpr int KL = (CIN == 32) ? 8 : 4;  // K values per lane and instruction
    constexpr int SH = (CIN == 32) ? 2 : 3;  // rows per bank cycle: 4 (64-byte rows) or 8 (32-byte)
    for (int q = t; q < 27 * CO * (CIN / 4); q += NT) {
        const int c4 = q % (CIN / 4), tap = (q / (CIN / 4)) % 27, co = q / (27 * (CIN / 4));
        const short4_t v = *reinterpret_cast<const short4_t *>(w + ((long long)co * 27 + tap) * CIN + 4 * c4);
        const int chunk = (4 * c4) / KL, within = (4 * c4) % KL;
        const int phys = (chunk ^ ((co >> SH) & 3)) * KL + within;
        *reinterpret_cast<short4_t *>(sw + (tap * CO + co) * CIN + phys) = v;
    }
    // input plane gz (zero outside the volume) into registers / into a ring slot
    using Pre = typename std::conditional<XB, short4_t, float4_t>::type;
    Pre pre[Lds::PER_THREAD];
    auto fetch = [&](int gz) {
#pragma unroll
        for (int j = 0; j < Lds::PER_THREAD; ++j) {
            const int q = t + NT * j;
            const int c4 = q % (CIN / 4), xi = (q / (CIN / 4)) % 66, yi = q / (66 * (CIN / 4));
            const int gx = x0 - 1 + xi, gy = y0 - 1 + yi;
            const bool in = q < Lds::LOADS && gz >= 0 && gz < n && gx >= 0 && gx < n && gy >= 0 && gy < n;
            const long long off = ((long long)gx + (long long)n * (gy + (long long)n * gz)) * CIN + 4 * c4;
            if constexpr (XB)
                pre[j] = in ? *reinterpret_cast<const short4_t *>(static_cast<const unsigned short *>(xv) + off)
                            : short4_t{0, 0, 0, 0};
            else
                pre[j] = in ? *reinterpret_cast<const float4_t *>(static_cast<const float *>(xv) + off)
                            : float4_t{0.f, 0.f, 0.f, 0.f};
        }
    };
    auto store = [&](int slot) {
#pragma unroll
        for (int j = 0; j < Lds::PER_THREAD; ++j) {
            const int q = t + NT * j;
            if (q < Lds::LOADS) {
                const int c4 = q % (CIN / 4), xi = (q / (CIN / 4)) % 66, yi = q / (66 * (CIN / 4));
                short4_t v;
                if constexpr (XB) {
                    v = pre[j];
                } else {
#pragma unroll
                    for (int e = 0; e < 4; ++e) v[e] = (short)to_bf16(pre[j][e]);
                }
                *reinterpret_cast<short4_t *>(sp + ((slot * 6 + yi) * 66 + xi) * CS + 4 * c4) = v;
            }
        }
    };
    fetch(z0 - 1);
    store((z0 + 2) % 3);
    fetch(z0);
    store(z0 % 3);
    fetch(z0 + 1);
    store((z0 + 1) % 3);
    __syncthreads();
    for (int z = z0; z < z1; ++z) {
        if (z + 1 < z1) fetch(z + 2);  // in flight during the compute of plane z
        float4_t acc[ROWS];
#pragma unroll
        for (int r = 0; r < ROWS; ++r) acc[r] = {0.f, 0.f, 0.f, 0.f};
        // nine (dz, dx) groups, software-pipelined: the fragments of group g + 1 are read from LDS
        // while the MFMAs of group g run
        const int cob = 16 * ct + (lane & 15);
        const int pa_off = (r0 * 66 + 16 * mt + (lane & 15)) * CS + KL * (lane >> 4);
        const unsigned short *pb0 = sw + cob * CIN + KL * ((lane >> 4) ^ ((cob >> SH) & 3));
        auto load = [&](int grp, Frag (&af)[ROWS + 2], Frag (&bf)[3]) {
            const int dz = grp / 3, dx = grp % 3;
            const unsigned short *pa = sp + ((z + dz + 2) % 3) * Lds::PLANE + pa_off + dx * CS;
            const unsigned short *pb = pb0 + (dz * 9 + dx) * CO * CIN;
#pragma unroll
            for (int yi = 0; yi < ROWS + 2; ++yi) af[yi] = *reinterpret_cast<const Frag *>(pa + yi * 66 * CS);
#pragma unroll
            for (int dy = 0; dy < 3; ++dy) bf[dy] = *reinterpret_cast<const Frag *>(pb + dy * 3 * CO * CIN);
        };
        auto compute = [&](const Frag (&af)[ROWS + 2], const Frag (&bf)[3]) {
#pragma unroll
            for (int dy = 0; dy < 3; ++dy)
#pragma unroll
                for (int r = 0; r < ROWS; ++r) acc[r] = conv_mfma<CIN>(af[r + dy], bf[dy], acc[r]);
        };
        Frag fa0[ROWS + 2], fb0[3], fa1[ROWS + 2], fb1[3];
        load(0, fa0, fb0);
#pragma unroll
        for (int grp = 0; grp < 9; ++grp) {
            // scheduling barriers keep the next group's LDS reads ahead of this group's MFMAs
            if (grp % 2 == 0) {
                if (grp + 1 < 9) load(grp + 1, fa1, fb1);
                __builtin_amdgcn_sched_barrier(0);
                compute(fa0, fb0);
            } else {
                if (grp + 1 < 9) load(grp + 1, fa0, fb0);
                __builtin_amdgcn_sched_barrier(0);
                compute(fa1, fb1);
            }
            __builtin_amdgcn_sched_barrier(0);
        }
        // epilogue: D[v] of row r is voxel x0 + 16 mt + 4 (lane / 16) + v of row y0 + r0 + r,
        // channel 16 ct + lane % 16
        const int co = 16 * ct + (lane & 15);
        if (co < cout) {
            const float bv = bias ? bias[co] : 0.f;
#pragma unroll
            for (int r = 0; r < ROWS; ++r) {
                const int yv = y0 + r0 + r;
                if (yv >= n) continue;
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int xv = x0 + 16 * mt + 4 * (lane >> 4) + v;
                    if (xv >= n) continue;
                    float rr = acc[r][v] + bv;
                    if (RELU) rr = fmaxf(rr, 0.f);
                    const long long o = ((long long)xv + (long long)n * (yv + (long long)n * z)) * cop + co;
                    if constexpr (OB)
                        static_cast<unsigned short *>(outv)[o] = to_bf16(rr);
                    else
                        static_cast<float *>(outv)[o] = rr;
                }
            }
        }
        __syncthreads();               // every wave is done with slot (z - 1) % 3
        if (z + 1 < z1) store((z + 2) % 3);
        __syncthreads();
    }
}

// Backward weights and biases: dw[co][tap][ci] = sum_v g[v][co] bf16(x[v + off(tap)][ci]) and
// db[co] = sum_v g[v][co] -- the gradient of the convolution as computed, whose operands x are the
// BF16-rounded activations -- a contraction over voxels on v_mfma_f32_16x16x4f32 (FP32 products of
// the FP32 gradient and the exactly widened BF16 activation, FP32 sums).  A work item is a run of
// yc consecutive x-rows (64 voxels each) at fixed x tile and z; block b takes items b,
// b + gridDim.x, ... in order.  Along the run the input rows pass through an LDS ring of four
// y-slots, each holding the three planes z - 1, z, z + 1 of one row with its x halo (BF16), the row
// two steps ahead being fetched into registers while the current row is computed, so every input
// row is read once per item instead of nine times.  Wave w owns the 16 x 16 channel tile pair w % P
// (P = COUT/16 * CIN/16) for all 27 taps (27 accumulators) and, when P < 4, the voxel slice w / P of
// each row (KS = 4 / P slices).  Every (block, slice) writes its own partial gradient -- the
// weights, then COUT biases, the layout of the parameter vector -- and k_reduce_blocks sums them in
// a fixed order, so the result does not depend on scheduling.  g = upstream gradient (channels
// cop_g), x = layer input (CIN channels).
template <int CIN>
struct WgradLds {
    static constexpr int XS = CIN + 2;                          // staged voxel stride (BF16 values)
    static constexpr int SLOT = 3 * 66 * XS;                    // one y-slot: 3 planes x 66 voxels
    static constexpr int LOADS = 3 * 66 * CIN / 4;              // float4 loads per staged row
    static constexpr int PER_THREAD = (LOADS + 255) / 256;
};

template <int CIN, int COUT, bool XB>
__global__ __launch_bounds__(256) void k_conv_wgrad(int n, int yc, const float *__restrict__ g, int cop_g,
                                                    const void *__restrict__ xv,
                                                    float *__restrict__ partial) {
    constexpr int NCI = CIN / 16, P = (COUT / 16) * NCI, KS = 4 / P, KV = 64 / KS;
    constexpr int NW = COUT * 27 * CIN;
    static_assert(P * KS == 4, "four waves cover the channel tiles");
    using Lds = WgradLds<CIN>;
    constexpr int XS = Lds::XS;
    __shared__ float sg[64][COUT + 1];
    __shared__ unsigned short sx[4 * Lds::SLOT];  // [slot][plane][66][XS]
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int pair = wave % P, slice = wave / P;
    const int cot = pair / NCI, cit = pair % NCI;
    const int xtn = (n + 63) / 64, ycn = (n + yc - 1) / yc;
    const int nitems = xtn * n * ycn;
    float4_t acc[27];
#pragma unroll
    for (int tp = 0; tp < 27; ++tp) acc[tp] = {0.f, 0.f, 0.f, 0.f};
    float bacc = 0.f;  // bias sum of channel `lane` over this slice's voxels (first wave of a slice)
    using Pre = typename std::conditional<XB, short4_t, float4_t>::type;
    Pre pre[Lds::PER_THREAD];
    for (int item = blockIdx.x; item < nitems; item += gridDim.x) {
        const int xt = item % xtn, z = (item / xtn) % n, ych = item / (xtn * n);
        const int x0 = xt * 64, y0 = ych * yc, y1 = min(y0 + yc, n);
        // row yy (planes z - 1 .. z + 1, x halo) into registers, zero outside the volume
        auto fetch = [&](int yy) {
#pragma unroll
            for (int j = 0; j < Lds::PER_THREAD; ++j) {
                const int q = t + 256 * j;  // float4 index
                const int c4 = q % (CIN / 4), xi = (q / (CIN / 4)) % 66, pz = q / (66 * (CIN / 4));
                const int xx = x0 - 1 + xi, zz = z - 1 + pz;
                const bool in = q < Lds::LOADS && yy >= 0 && yy < n && zz >= 0 && zz < n && xx >= 0 && xx < n;
                const long long off = ((long long)xx + (long long)n * (yy + (long long)n * zz)) * CIN + 4 * c4;
                if constexpr (XB)
                    pre[j] = in ? *reinterpret_cast<const short4_t *>(static_cast<const unsigned short *>(xv) + off)
                                : short4_t{0, 0, 0, 0};
                else
                    pre[j] = in ? *reinterpret_cast<const float4_t *>(static_cast<const float *>(xv) + off)
                                : float4_t{0.f, 0.f, 0.f, 0.f};
            }
        };
        auto store = [&](int yy) {
            unsigned short *dst = sx + (yy & 3) * Lds::SLOT;
#pragma unroll
            for (int j = 0; j < Lds::PER_THREAD; ++j) {
                const int q = t + 256 * j;
                if (q < Lds::LOADS) {
                    const int c4 = q % (CIN / 4), xi = (q / (CIN / 4)) % 66, pz = q / (66 * (CIN / 4));
                    unsigned short *p = dst + (pz * 66 + xi) * XS + 4 * c4;
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        if constexpr (XB)
                            p[e] = (unsigned short)pre[j][e];
                        else
                            p[e] = to_bf16(pre[j][e]);
                    }
                }
            }
        };
        __syncthreads();  // the previous item's readers of the ring and of sg are done
        fetch(y0 - 1);
        store(y0 - 1);
        fetch(y0);
        store(y0);
        fetch(y0 + 1);
        store(y0 + 1);
        for (int y = y0; y < y1; ++y) {
            if (y + 1 < y1) fetch(y + 2);  // in flight during the compute of row y
            for (int q = t; q < 64 * COUT; q += 256) {
                const int vv = q / COUT, co = q % COUT;
                const int xv = x0 + vv;
                sg[vv][co] = (xv < n) ? g[((long long)xv + (long long)n * (y + (long long)n * z)) * cop_g + co] : 0.f;
            }
            __syncthreads();
            if (pair == 0 && lane < COUT)
                for (int vv = slice * KV; vv < slice * KV + KV; ++vv) bacc += sg[vv][lane];
#pragma unroll
            for (int dzy = 0; dzy < 9; ++dzy) {
                const unsigned short *row = sx + ((y + dzy % 3 - 1) & 3) * Lds::SLOT + (dzy / 3) * 66 * XS;
                for (int k0 = slice * KV; k0 < slice * KV + KV; k0 += 4) {
                    const int vv = k0 + (lane >> 4);
                    const float a = sg[vv][cot * 16 + (lane & 15)];
                    const unsigned short *px = row + vv * XS + cit * 16 + (lane & 15);
#pragma unroll
                    for (int dx = 0; dx < 3; ++dx) {
                        const float bv = __uint_as_float((unsigned)px[dx * XS] << 16);
                        acc[dzy * 3 + dx] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, bv, acc[dzy * 3 + dx], 0, 0, 0);
                    }
                }
            }
            __syncthreads();  // done with sg and with the slot of row y - 1
            if (y + 1 < y1) store(y + 2);
        }
    }
    float *dst = partial + ((size_t)blockIdx.x * KS + slice) * (NW + COUT);
    const int ci = cit * 16 + (lane & 15);
#pragma unroll
    for (int tp = 0; tp < 27; ++tp)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int co = cot * 16 + 4 * (lane >> 4) + v;
            dst[((size_t)co * 27 + tp) * CIN + ci] = acc[tp][v];
        }
    if (pair == 0 && lane < COUT) dst[NW + lane] = bacc;
}

// out[i] = sum_b partial[b * len + i] for i < len: 64 columns per block, the rows split over four
// thread groups (rows b = grp, grp + 4, ...), each summing with eight independent partial sums so
// that eight loads are in flight; all sums are combined in a fixed order.
__global__ __launch_bounds__(256) void k_reduce_blocks(const float *__restrict__ partial, int nblk, int len,
                                                       float *__restrict__ out) {
    __shared__ float sh[4][64];
    const int col = blockIdx.x * 64 + (threadIdx.x & 63), grp = threadIdx.x >> 6;
    float s = 0.f;
    if (col < len) {
        const float *p = partial + col;
        float a[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        int b = grp;
        for (; b + 28 < nblk; b += 32) {
#pragma unroll
            for (int j = 0; j < 8; ++j) a[j] += p[(size_t)(b + 4 * j) * len];
        }
        for (int j = 0; b < nblk; b += 4, ++j) a[j & 7] += p[(size_t)b * len];
        s = ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
    }
    sh[grp][threadIdx.x & 63] = s;
    __syncthreads();
    if (grp == 0 && col < len) out[col] = ((sh[0][threadIdx.x] + sh[1][threadIdx.x]) + sh[2][threadIdx.x]) + sh[3][threadIdx.x];
}

// Transposed, flipped BF16 weights for the data gradient: wt[ci][tap][co] = w[co][26 - tap][ci].
__global__ __launch_bounds__(256) void k_flip_weights(const float *__restrict__ w, int cout_p, int cin_p,
                                                      unsigned short *__restrict__ wt) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    const int total = cout_p * 27 * cin_p;
    if (i >= total) return;
    const int co = i % cout_p;  // fastest index of wt
    const int tap = (i / cout_p) % 27;
    const int ci = i / (cout_p * 27);
    wt[i] = to_bf16(w[((long long)co * 27 + (26 - tap)) * cin_p + ci]);
}

__global__ __launch_bounds__(256) void k_to_bf16(const float *__restrict__ a, unsigned short *__restrict__ b,
                                                 int len) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < len) b[i] = to_bf16(a[i]);
}

// g[v*cop + c] *= (y[v*cop + c] > 0) for the first cout channels (ReLU backward), zero elsewhere;
// y is a BF16 activation (positive exactly when its FP32 value was).
__global__ __launch_bounds__(256) void k_relu_mask(long long nvox, int cop, int cout,
                                                   const unsigned short *__restrict__ y, float *__restrict__ g) {
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i >= nvox * cop) return;
    const int c = (int)(i % cop);
    const float yv = __uint_as_float((unsigned)y[i] << 16);
    g[i] = (c < cout && yv > 0.f) ? g[i] : 0.f;
}

// Loss of the output o against t through a 7-point stencil K (coefficients of the centre and of
// the x-, x+, y-, y+, z-, z+ neighbours, zero outside the volume): rho = t - K o, loss = mean rho^2.
// K = identity gives the mean squared error.  First pass: rho and per-block sums of rho^2.
__device__ __forceinline__ float stencil_at(int n, const float *__restrict__ f, const NetStencil &K, int x, int y,
                                            int z) {
    const long long v = (long long)x + (long long)n * (y + (long long)n * z);
    const long long nn = (long long)n * n;
    float a = K.c[0] * f[v];
    if (x > 0) a += K.c[1] * f[v - 1];
    if (x < n - 1) a += K.c[2] * f[v + 1];
    if (y > 0) a += K.c[3] * f[v - n];
    if (y < n - 1) a += K.c[4] * f[v + n];
    if (z > 0) a += K.c[5] * f[v - nn];
    if (z < n - 1) a += K.c[6] * f[v + nn];
    return a;
}

__global__ __launch_bounds__(256) void k_stencil_res(int n, const float *__restrict__ o, const float *__restrict__ t,
                                                     NetStencil K, float *__restrict__ rho,
                                                     double *__restrict__ partial) {
    __shared__ double sh[4];
    const long long nv = (long long)n * n * n;
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    double e2 = 0.0;
    if (i < nv) {
        const int x = (int)(i % n), y = (int)((i / n) % n), z = (int)(i / ((long long)n * n));
        const float e = t[i] - stencil_at(n, o, K, x, y, z);
        rho[i] = e;
        e2 = (double)e * e;
    }
    const double s = block_sum<256>(e2, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

// Second pass: gradient of the loss with respect to o, -(2/N) K^T rho (KT = the transposed stencil),
// into channel 0 of a 16-channel buffer (channels 1..15 zero) for the backward pass of the last layer.
__global__ __launch_bounds__(256) void k_stencil_grad(int n, const float *__restrict__ rho, NetStencil KT,
                                                      float scale, float *__restrict__ d16) {
    const long long nv = (long long)n * n * n;
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i >= nv) return;
    const int x = (int)(i % n), y = (int)((i / n) % n), z = (int)(i / ((long long)n * n));
    float4_t *dst = reinterpret_cast<float4_t *>(d16 + i * 16);
    dst[0] = {scale * stencil_at(n, rho, KT, x, y, z), 0.f, 0.f, 0.f};
    dst[1] = {0.f, 0.f, 0.f, 0.f};
    dst[2] = {0.f, 0.f, 0.f, 0.f};
    dst[3] = {0.f, 0.f, 0.f, 0.f};
}

// Input of the learned correction for the window [o0, o0 + n)^3 (per axis offsets) of the fine grid:
// channel 0 r / sigma with sigma^2 = ||r||^2 / N_f^3 (||r||^2 read from *rn2, or rn2_value when rn2
// is null), channels 1..3 the
// coarse-plane indicators of axes 0..2 (fine index i, 0-based, lies on a coarse plane when
// (i + 1) % nsp == 0), channels 4..6 the cell Peclet numbers of axes 0..2, channels 7..15 zero.
// rhat (optional) receives channel 0 contiguously.
__global__ __launch_bounds__(256) void k_net_features(int n, int Nf, int nsp, int o0, int o1, int o2,
                                                      const double *__restrict__ r, const double *__restrict__ rn2,
                                                      double rn2_value, float pe0, float pe1, float pe2,
                                                      float *__restrict__ in16,
                                                      float *__restrict__ rhat, const int *gate) {
    if (gate && *gate) return;
    const long long nv = (long long)n * n * n;
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i >= nv) return;
    const int x = (int)(i % n), y = (int)((i / n) % n), z = (int)(i / ((long long)n * n));
    const int gx = x + o0, gy = y + o1, gz = z + o2;
    const double nf3 = (double)Nf * Nf * Nf;
    const double sig2 = (rn2 ? *rn2 : rn2_value) / nf3;
    const double inv = sig2 > 0.0 ? 1.0 / sqrt(sig2) : 0.0;
    const float rv = (float)(r[(long long)gx + (long long)Nf * (gy + (long long)Nf * gz)] * inv);
    float4_t *dst = reinterpret_cast<float4_t *>(in16 + i * 16);
    dst[0] = {rv, ((gx + 1) % nsp == 0) ? 1.f : 0.f, ((gy + 1) % nsp == 0) ? 1.f : 0.f, ((gz + 1) % nsp == 0) ? 1.f : 0.f};
    dst[1] = {pe0, pe1, pe2, 0.f};
    dst[2] = {0.f, 0.f, 0.f, 0.f};
    dst[3] = {0.f, 0.f, 0.f, 0.f};
    if (rhat) rhat[i] = rv;
}

// Correction proposed by the network in the solver's units: e = o * sigma * h^2 / mean(alpha)
// (sigma as in k_net_features), FP64, over the whole fine grid (the network's volume).
__global__ __launch_bounds__(256) void k_net_correction(long long nv, const float *__restrict__ o,
                                                        const double *__restrict__ rn2, double h2a,
                                                        double *__restrict__ e, const int *gate) {
    if (gate && *gate) return;
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i >= nv) return;
    const double sig2 = *rn2 / (double)nv;
    e[i] = (double)o[i] * (sqrt(sig2) * h2a);
}

// Acceptance test of a learned proposal e with <r, Ae> = rq and <Ae, Ae> = qq: with the optimal step
// rq / qq the new residual has ||r||^2 - rq^2 / qq; the proposal is taken when that is at most
// ||r||^2 / factor^2 (factor2 = factor^2).  Writes skip[0] = 1 when the learned update is not to be
// applied and skip[1] = 1 when the plain step is not to be taken (both once the loop is done), and
// counts accepted proposals.  Runs whatever the state: its flags gate the rest of the step.
__global__ void k_learned_accept(const double *__restrict__ scal, int *__restrict__ done, int *__restrict__ accepted,
                                 double factor2, int *__restrict__ skip) {
    if (threadIdx.x != 0) return;
    const int dn = *done;
    bool ok = false;
    if (!dn) {
        const double rr = scal[kScalRnorm2], rq = scal[kScalRQ], qq = scal[kScalQQ];
        ok = qq > 0.0 && rq > 0.0 && isfinite(rq) && isfinite(qq) && (rr - rq * (rq / qq)) * factor2 <= rr;
        if (ok) *accepted += 1;
    }
    skip[0] = (dn || !ok) ? 1 : 0;
    skip[1] = (dn || ok) ? 1 : 0;
}

__global__ __launch_bounds__(256) void k_adam(int len, float *__restrict__ w, const float *__restrict__ g,
                                              float *__restrict__ m, float *__restrict__ v, float lr, float b1,
                                              float b2, float eps, float c1, float c2) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= len) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    w[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// ---------------------------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------------------------
static unsigned blocks_of(int n) { return (unsigned)(((n + 63) / 64) * n * n); }

unsigned net_reduce_blocks(int n) {
    const unsigned nb = blocks_of(n);
    return nb < (unsigned)kNetMaxReduceBlocks ? nb : (unsigned)kNetMaxReduceBlocks;
}

template <int CIN, int COT, bool RELU, bool XB, bool OB>
static void conv_launch(int n, const void *x, const unsigned short *w, const float *bias, int cout, int cop,
                        void *out, const int *gate, hipStream_t st) {
    // z chunks: enough blocks to cover the chip twice where the volume allows, at least 4 planes each
    const int xy = ((n + 63) / 64) * ((n + 3) / 4);
    int zc = 16;
    while (zc > 4 && (long long)xy * ((n + zc - 1) / zc) < 512) zc /= 2;
    const int blocks = xy * ((n + zc - 1) / zc);
    const size_t lds = ConvLds<CIN, COT>::BYTES;
    ASDSM_LAUNCH((k_conv_fwd<CIN, COT, RELU, XB, OB>), dim3((unsigned)blocks), dim3(kConvThreads), lds, st, n, zc, x,
                 w, bias, cout, cop, out, gate);
}

template <int CIN, int COT, bool RELU, bool XB, bool OB>
static void conv_prepare_one() {
    (void)hipFuncSetAttribute((const void *)k_conv_fwd<CIN, COT, RELU, XB, OB>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)ConvLds<CIN, COT>::BYTES);
}

void net_conv_prepare() {
    // the kernels use more than 64 KB of dynamic LDS
    conv_prepare_one<16, 2, true, false, true>();
    conv_prepare_one<32, 2, true, true, true>();
    conv_prepare_one<32, 1, false, true, false>();
    conv_prepare_one<16, 2, false, false, false>();
    conv_prepare_one<32, 2, false, false, false>();
}

// The combinations the network uses: forward layers (first: FP32 input, BF16 output; hidden: BF16 in
// and out; last: BF16 in, FP32 out) and the data gradients (FP32 in and out, no ReLU).
void net_conv_fwd(int n, int cin_p, int cout, int cop, bool relu, const void *x, bool x_bf16, const unsigned short *w,
                  const float *bias, void *out, bool out_bf16, const int *gate, hipStream_t st) {
    const int cot = (cout + 15) / 16;
    if (cin_p == 16 && cot == 2 && relu && !x_bf16 && out_bf16)
        conv_launch<16, 2, true, false, true>(n, x, w, bias, cout, cop, out, gate, st);
    else if (cin_p == 32 && cot == 2 && relu && x_bf16 && out_bf16)
        conv_launch<32, 2, true, true, true>(n, x, w, bias, cout, cop, out, gate, st);
    else if (cin_p == 32 && cot == 1 && !relu && x_bf16 && !out_bf16)
        conv_launch<32, 1, false, true, false>(n, x, w, bias, cout, cop, out, gate, st);
    else if (cin_p == 16 && cot == 2 && !relu && !x_bf16 && !out_bf16)
        conv_launch<16, 2, false, false, false>(n, x, w, bias, cout, cop, out, gate, st);
    else if (cin_p == 32 && cot == 2 && !relu && !x_bf16 && !out_bf16)
        conv_launch<32, 2, false, false, false>(n, x, w, bias, cout, cop, out, gate, st);
}

static int wgrad_rows(int n) {
    // rows per work item: about two items per block where the volume allows
    const long long cols = (long long)((n + 63) / 64) * n;
    int yc = 8;
    while (yc < n && cols * ((n + yc - 1) / yc) > 2LL * kNetMaxReduceBlocks) yc *= 2;
    return yc < n ? yc : n;
}

void net_conv_wgrad(int n, int cin_p, int cout_p, const float *g, int cop_g, const void *x, bool x_bf16,
                    float *partial, float *dwb, hipStream_t st) {
    const int yc = wgrad_rows(n);
    const long long items = (long long)((n + 63) / 64) * n * ((n + yc - 1) / yc);
    const unsigned nb = (unsigned)(items < kNetMaxReduceBlocks ? items : kNetMaxReduceBlocks);
    // the first layer's input is the FP32 network input, the others' the BF16 activations
    if (cin_p == 16 && cout_p == 32 && !x_bf16)
        ASDSM_LAUNCH((k_conv_wgrad<16, 32, false>), dim3(nb), dim3(256), 0, st, n, yc, g, cop_g, x, partial);
    else if (cin_p == 32 && cout_p == 32 && x_bf16)
        ASDSM_LAUNCH((k_conv_wgrad<32, 32, true>), dim3(nb), dim3(256), 0, st, n, yc, g, cop_g, x, partial);
    else if (cin_p == 32 && cout_p == 16 && x_bf16)
        ASDSM_LAUNCH((k_conv_wgrad<32, 16, true>), dim3(nb), dim3(256), 0, st, n, yc, g, cop_g, x, partial);
    const int len = cout_p * 27 * cin_p + cout_p;            // weights, then biases
    const int slices = 4 / ((cout_p / 16) * (cin_p / 16));  // partial gradients per block
    ASDSM_LAUNCH(k_reduce_blocks, dim3((len + 63) / 64), dim3(256), 0, st, partial, (int)nb * slices, len, dwb);
}

void net_flip(const float *w, int cout_p, int cin_p, unsigned short *wt, hipStream_t st) {
    const int total = cout_p * 27 * cin_p;
    ASDSM_LAUNCH(k_flip_weights, dim3((total + 255) / 256), dim3(256), 0, st, w, cout_p, cin_p, wt);
}

void net_to_bf16(const float *a, unsigned short *b, int len, hipStream_t st) {
    ASDSM_LAUNCH(k_to_bf16, dim3((len + 255) / 256), dim3(256), 0, st, a, b, len);
}

void net_relu_mask(long long nvox, int cop, int cout, const unsigned short *y, float *g, hipStream_t st) {
    ASDSM_LAUNCH(k_relu_mask, dim3((unsigned)((nvox * cop + 255) / 256)), dim3(256), 0, st, nvox, cop, cout, y, g);
}

void net_stencil_loss(int n, const float *o, const float *t, const NetStencil &K, const NetStencil &KT, float *rho,
                      float *d16, double *partial, hipStream_t st) {
    const long long nv = (long long)n * n * n;
    const dim3 grid((unsigned)((nv + 255) / 256));
    ASDSM_LAUNCH(k_stencil_res, grid, dim3(256), 0, st, n, o, t, K, rho, partial);
    ASDSM_LAUNCH(k_stencil_grad, grid, dim3(256), 0, st, n, rho, KT, (float)(-2.0 / (double)nv), d16);
}

void net_features(int n, int Nf, int nsp, const int off[3], const double *r, const double *rn2, double rn2_value,
                  const float pe[3], float *in16, float *rhat, const int *gate, hipStream_t st) {
    const long long nv = (long long)n * n * n;
    ASDSM_LAUNCH(k_net_features, dim3((unsigned)((nv + 255) / 256)), dim3(256), 0, st, n, Nf, nsp, off[0], off[1],
                 off[2], r, rn2, rn2_value, pe[0], pe[1], pe[2], in16, rhat, gate);
}

void net_correction(long long nv, const float *o, const double *rn2, double h2a, double *e, const int *gate,
                    hipStream_t st) {
    ASDSM_LAUNCH(k_net_correction, dim3((unsigned)((nv + 255) / 256)), dim3(256), 0, st, nv, o, rn2, h2a, e, gate);
}

void net_accept(const double *scal, int *done, int *accepted, double factor, int *skip, hipStream_t st) {
    ASDSM_LAUNCH(k_learned_accept, dim3(1), dim3(64), 0, st, scal, done, accepted, factor * factor, skip);
}

void net_adam(int len, float *w, const float *g, float *m, float *v, float lr, float b1, float b2, float eps,
              float c1, float c2, hipStream_t st) {
    ASDSM_LAUNCH(k_adam, dim3((len + 255) / 256), dim3(256), 0, st, len, w, g, m, v, lr, b1, b2, eps, c1, c2);
}

}  // namespace asdsm
