// Allocation-free fine residual: r = b_ff - A_ff u and ||r||_2 (Algorithm 4 step 3, b_ff = s plus
// the Dirichlet terms of Section 2.3) without the plan's workspace.  The right-hand side is formed
// inside the stencil pass, and the per-block partial sums of ||r||^2 go to a file-scope device
// array, so asdsm_residual_noalloc needs no device memory beyond its inputs and outputs and calls
// no allocating routine.  Every call on a device shares that device's copy of the array: calls that
// overlap on one device race.
#include <climits>
#include <cmath>
#include <mutex>

#include "device_common.hpp"
#include "kernels.hpp"

namespace asdsm {

namespace {
constexpr int kNoallocBlocks = 2048;             // grid of the residual pass (grid-stride loop)
constexpr int kNoallocSlots = kNoallocBlocks + 8; // partial sums, then the total at kNoallocBlocks
constexpr int kNoallocMaxDevices = 64;
}  // namespace

// 16.1 KiB per device, held until the process ends.  In host code this name is a stand-in, not a
// device address: kernels receive the address hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) double scratch[kNoallocSlots];

namespace {
std::mutex g_scratch_mu;
double *g_scratch_ptr[kNoallocMaxDevices] = {};

// b = s + Dirichlet terms, then r = b - A u, in the operation order of the plan's right-hand side
// assembly (axis by axis, low side before high side) and stencil (centre, then each axis' low and
// high neighbour); per-block sums of r^2 in partials[blockIdx.x].
template <int D>
__global__ __launch_bounds__(256) void k_residual_direct(Geo g, const double *__restrict__ u,
                                                         const double *__restrict__ s,
                                                         const double *__restrict__ gf,
                                                         double *__restrict__ r,
                                                         double *__restrict__ partials) {
    const int Nf = g.Nf;
    const int NF = (int)g.NF;
    int faceN = 1;
    for (int j = 1; j < D; ++j) faceN *= Nf;
    const int sy = Nf, sz = Nf * Nf, sw = Nf * Nf * Nf;
    const double bsum = g.fine[0].b + g.fine[1].b + (D >= 3 ? g.fine[2].b : 0.0) + (D == 4 ? g.fine[3].b : 0.0);
    double acc = 0.0;
    for (int p = blockIdx.x * 256 + threadIdx.x; p < NF; p += gridDim.x * 256) {
        int i[kMaxD] = {0, 0, 0, 0};
        int rem = p;
        i[0] = rem % Nf;
        rem /= Nf;
        i[1] = rem % Nf;
        rem /= Nf;
        if (D >= 3) {
            i[2] = rem % Nf;
            rem /= Nf;
        }
        if (D == 4) i[3] = rem;
        double b = s[p];
#pragma unroll
        for (int j = 0; j < D; ++j) {
            const bool lo = i[j] == 0, hi = i[j] == Nf - 1;
            if (!lo && !hi) continue;
            int fidx = 0, mul = 1;
#pragma unroll
            for (int o = 0; o < D; ++o) {
                if (o == j) continue;
                fidx += i[o] * mul;
                mul *= Nf;
            }
            if (lo) b -= g.fine[j].a * gf[(2 * j) * faceN + fidx];
            if (hi) b -= g.fine[j].c * gf[(2 * j + 1) * faceN + fidx];
        }
        double au = bsum * u[p];
        if (i[0] > 0) au += g.fine[0].a * u[p - 1];
        if (i[0] < Nf - 1) au += g.fine[0].c * u[p + 1];
        if (i[1] > 0) au += g.fine[1].a * u[p - sy];
        if (i[1] < Nf - 1) au += g.fine[1].c * u[p + sy];
        if (D >= 3) {
            if (i[2] > 0) au += g.fine[2].a * u[p - sz];
            if (i[2] < Nf - 1) au += g.fine[2].c * u[p + sz];
        }
        if (D == 4) {
            if (i[3] > 0) au += g.fine[3].a * u[p - sw];
            if (i[3] < Nf - 1) au += g.fine[3].c * u[p + sw];
        }
        const double rr = b - au;
        if (r) r[p] = rr;
        acc += rr * rr;
    }
    double vals[1] = {acc};
    block_partials<256, 1>(vals, partials, blockIdx.x);
}

// One block: the total of nblk partial sums in a fixed order, stored at partials[kNoallocBlocks].
__global__ __launch_bounds__(256) void k_noalloc_total(double *partials, int nblk) {
    __shared__ double sh[4];
    double a = 0.0;
    for (int b = threadIdx.x; b < nblk; b += 256) a += partials[b];
    const double t = block_sum<256>(a, sh);
    if (threadIdx.x == 0) partials[kNoallocBlocks] = t;
}
}  // namespace

// Resolve this device's copy of `scratch` (the plan constructor calls this with the plan's device
// current; once per device).
int noalloc_setup(int device) {
    if (device < 0 || device >= kNoallocMaxDevices)
        return fail(ASDSM_E_DEVICE, "device ordinal beyond the allocation-free entry point's table");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_ptr[device]) return ASDSM_OK;
    void *ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
        return fail(ASDSM_E_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[device] = (double *)ptr;
    return ASDSM_OK;
}

int residual_noalloc(const Plan &p, const double *u, const double *s, const double *g, double *r,
                     double *norm2_host) {
    // 32-bit point indices, including the grid-stride loop's last increment
    if (p.geo.NF > (long long)INT_MAX - (long long)kNoallocBlocks * 256)
        return fail(ASDSM_E_UNSUPPORTED, "asdsm_residual_noalloc: more than 2^31 - 2^19 - 1 fine points");
    double *part = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_scratch_mu);
        if (p.device >= 0 && p.device < kNoallocMaxDevices) part = g_scratch_ptr[p.device];
    }
    if (!part) return fail(ASDSM_E_DEVICE, "asdsm_residual_noalloc: scratch not resolved on the plan's device");
    long long blocks = (p.geo.NF + 255) / 256;
    if (blocks > kNoallocBlocks) blocks = kNoallocBlocks;
    const dim3 grid((unsigned)blocks), block(256);
    switch (p.d) {
        case 2: hipLaunchKernelGGL(k_residual_direct<2>, grid, block, 0, p.stream, p.geo, u, s, g, r, part); break;
        case 3: hipLaunchKernelGGL(k_residual_direct<3>, grid, block, 0, p.stream, p.geo, u, s, g, r, part); break;
        default: hipLaunchKernelGGL(k_residual_direct<4>, grid, block, 0, p.stream, p.geo, u, s, g, r, part); break;
    }
    hipLaunchKernelGGL(k_noalloc_total, dim3(1), dim3(256), 0, p.stream, part, (int)blocks);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(ASDSM_E_DEVICE, std::string("residual_noalloc launch: ") + hipGetErrorString(e));
    if (norm2_host) {
        // the plan's pinned scalar mirror (allocated with the plan) receives the total
        e = hipMemcpyAsync(p.hscal + kScalNoalloc, part + kNoallocBlocks, sizeof(double),
                           hipMemcpyDeviceToHost, p.stream);
        if (e != hipSuccess) return fail(ASDSM_E_DEVICE, std::string("residual_noalloc copy: ") + hipGetErrorString(e));
    }
    e = hipStreamSynchronize(p.stream);
    if (e != hipSuccess) return fail(ASDSM_E_DEVICE, std::string("residual_noalloc: ") + hipGetErrorString(e));
    if (norm2_host) *norm2_host = std::sqrt(p.hscal[kScalNoalloc]);
    return ASDSM_OK;
}

}  // namespace asdsm
