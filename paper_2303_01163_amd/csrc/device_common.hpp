// Device helpers shared by the kernels: index maps between the fine mesh and the canonical
// submesh layouts, deterministic block reductions and the last-block finalisation pattern.
#pragma once

#include <hip/hip_runtime.h>

#include "asdsm_internal.hpp"

namespace asdsm {

typedef double double4_t __attribute__((ext_vector_type(4)));

// A fine index i (0-based) lies on a coarse line iff i+1 is a multiple of n (n a power of two).
__device__ __forceinline__ bool on_coarse(int i, int n) { return ((i + 1) & (n - 1)) == 0; }
__device__ __forceinline__ int coarse_of(int i, int n) { return (i + 1) / n - 1; }

// Canonical offset of the fine point i[] inside mesh M_S (the point must lie on M_S).
__device__ __forceinline__ long long canon_offset(const MeshDesc &m, const int *i, int n) {
    long long off = 0;
    for (int q = 0; q < m.nd; ++q) {
        const int j = m.ax[q];
        const int pos = (q < m.nfine) ? i[j] : coarse_of(i[j], n);
        off += (long long)pos * m.stride[q];
    }
    return off;
}

// Wave64 + LDS tree sum with a fixed order (deterministic for a fixed launch shape).
template <int NT>
__device__ __forceinline__ double block_sum(double v, double *sh) {
    static_assert(NT % 64 == 0, "block must be whole waves");
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) sh[wid] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0) {
        for (int w = 0; w < NT / 64; ++w) t += sh[w];
    }
    return t;  // valid in thread 0
}

__device__ __forceinline__ double load_coherent(const double *p) {
    unsigned long long bits = __hip_atomic_load((const unsigned long long *)p, __ATOMIC_RELAXED,
                                                __HIP_MEMORY_SCOPE_AGENT);
    return __longlong_as_double((long long)bits);
}

// Each block stores NV partial sums; the last block to arrive sums all partials in block order and
// calls fin(totals) with thread 0.  The ticket counter is returned to zero by the last block.
template <int NT, int NV, typename Fin>
__device__ __forceinline__ void reduce_and_finalize_slice(const double (&v)[NV], double *partials,
                                                          unsigned *counter, unsigned bid,
                                                          unsigned nblk, Fin fin) {
    __shared__ double sh[NT / 64];
    __shared__ bool last;
    double tot[NV];
    for (int q = 0; q < NV; ++q) tot[q] = block_sum<NT>(v[q], sh);
    if (threadIdx.x == 0) {
        for (int q = 0; q < NV; ++q) partials[(size_t)bid * NV + q] = tot[q];
        __threadfence();
        const unsigned ticket = atomicAdd(counter, 1u);
        last = (ticket == nblk - 1);
    }
    __syncthreads();
    if (!last) return;
    __threadfence();
    double acc[NV];
    for (int q = 0; q < NV; ++q) acc[q] = 0.0;
    for (unsigned b = threadIdx.x; b < nblk; b += NT)
        for (int q = 0; q < NV; ++q) acc[q] += load_coherent(partials + (size_t)b * NV + q);
    double res[NV];
    for (int q = 0; q < NV; ++q) res[q] = block_sum<NT>(acc[q], sh);
    if (threadIdx.x == 0) {
        fin(res);
        *counter = 0u;
    }
}

template <int NT, int NV, typename Fin>
__device__ __forceinline__ void reduce_and_finalize(const double (&v)[NV], double *partials,
                                                    unsigned *counter, Fin fin) {
    const unsigned nblk = gridDim.x * gridDim.y * gridDim.z;
    const unsigned bid = blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z);
    reduce_and_finalize_slice<NT, NV>(v, partials, counter, bid, nblk, fin);
}

}  // namespace asdsm
