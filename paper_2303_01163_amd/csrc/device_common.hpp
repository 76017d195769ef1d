// Device helpers shared by the kernels: index maps between the fine mesh and the canonical
// submesh layouts, deterministic block reductions and the last-block finalisation pattern.
#pragma once

#include <hip/hip_runtime.h>

#include "asdsm_internal.hpp"

namespace asdsm {

typedef double double4_t __attribute__((ext_vector_type(4)));
typedef float float4_t __attribute__((ext_vector_type(4)));

// A fine index i (0-based) lies on a coarse line iff i+1 is a multiple of n (n a power of two).
__device__ __forceinline__ bool on_coarse(int i, int n) { return ((i + 1) & (n - 1)) == 0; }
// Its coarse index, (i + 1) / n - 1, by a shift: a division by the run-time n costs tens of
// instructions, and the index maps of the skeleton kernels take several per point.
__device__ __forceinline__ int coarse_of(int i, int n) { return ((i + 1) >> __builtin_ctz((unsigned)n)) - 1; }

// Element j (a run-time axis) of a per-axis array of kMaxD ints, through selects: a dynamic index
// into a local array would place the array in scratch memory.
__device__ __forceinline__ int axis_sel(const int *v, int j) {
    return j == 0 ? v[0] : (j == 1 ? v[1] : (j == 2 ? v[2] : v[3]));
}

// Canonical offset of the fine point i[] (kMaxD entries) inside mesh M_S (the point must lie on M_S).
__device__ __forceinline__ long long canon_offset(const MeshDesc &m, const int *i, int n) {
    long long off = 0;
    for (int q = 0; q < m.nd; ++q) {
        const int ij = axis_sel(i, m.ax[q]);
        const int pos = (q < m.nfine) ? ij : coarse_of(ij, n);
        off += (long long)pos * m.stride[q];
    }
    return off;
}

// A flag read with a vector load (device-scope relaxed atomic): the kernels that test it late issue
// it with their operand loads; a plain load of a uniform address becomes a scalar load, which is
// waited for together with the kernel arguments, before any other load is issued.
__device__ __forceinline__ int flag_load(const int *f) {
    return __hip_atomic_load(f, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// The stopping flag of the refinement loop (nullptr: none).  No branch on the pointer either: a
// null gate reads a zero of its own, so the test of the value can wait until it is needed.
static __device__ int g_gate_open = 0;
__device__ __forceinline__ int gate_value(const int *gate) { return flag_load(gate ? gate : &g_gate_open); }
__device__ __forceinline__ bool gate_open(const int *gate) { return gate_value(gate) == 0; }
// The test of a flag value where it stands: the compiler would otherwise place the comparison (and
// the wait for the load) where the value was loaded, ahead of the kernel's other loads.
__device__ __forceinline__ bool flag_clear(int v) {
    asm volatile("" : "+v"(v));
    return v == 0;
}

// Workgroup barrier that orders LDS accesses only: global loads in flight stay in flight.
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
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

// Each block stores its NV partial sums (fixed in-block order) at partials[bid*NV + q].  The totals
// are formed by k_finalize in a separate launch, so no fence or atomic is needed here: on a
// multi-XCD device an agent-scope release fence per block would write back the L2 every time.
template <int NT, int NV>
__device__ __forceinline__ void block_partials(const double (&v)[NV], double *partials, size_t bid) {
    __shared__ double sh[NT / 64];
    double tot[NV];
    for (int q = 0; q < NV; ++q) tot[q] = block_sum<NT>(v[q], sh);
    if (threadIdx.x == 0)
        for (int q = 0; q < NV; ++q) partials[bid * NV + q] = tot[q];
}

// The stopping rule after one refinement step has produced r_{k+1} (thread 0; t = ||r_{k+1}||^2,
// s_hat in scal): step count, the next step's axis permutation, the histories, stagnation, and
// the done flag with the status.
__device__ __forceinline__ void finalize_step(double t, double *scal, IterState *stt, double *hist,
                                              double *step_hist, const int *perm_table) {
    scal[kScalRnorm2] = t;
    const double rn = sqrt(t);
    const double bn = sqrt(scal[kScalBnorm2]);
    const double shat = scal[kScalStep];
    const int it = stt->it + 1;
    stt->it = it;
    // the next step's axis permutation (the table holds max_iter < kHistCap entries)
    if (it < stt->max_iter)
        for (int j = 0; j < kMaxD; ++j) stt->perm[j] = perm_table[kMaxD * it + j];
    if (it < kHistCap) hist[it] = rn;
    if (it - 1 < kHistCap) step_hist[it - 1] = shat;
    if (!isfinite(rn) || !isfinite(shat)) {
        stt->done = 1;
        stt->status = ASDSM_E_NUMERIC;
        return;
    }
    stt->stag = (rn > (1.0 - stt->stag_eta) * stt->rn_prev) ? stt->stag + 1 : 0;
    stt->rn_prev = rn;
    // a zero step leaves u unchanged and counts towards the window like any step that does
    // not reduce ||r|| enough; the next step draws another cross-point choice
    if (stt->stag_window > 0 && stt->stag >= stt->stag_window) {
        stt->done = 1;
        stt->status = ASDSM_STAGNATED;
    } else if ((bn > 0.0 && rn <= stt->rtol * bn) || (bn == 0.0 && rn == 0.0)) {
        stt->done = 1;
        stt->status = ASDSM_OK;
    } else if (it >= stt->max_iter) {
        stt->done = 1;
        stt->status = ASDSM_MAXITER;
    }
}

// One 256-thread block applies the pending stopping rule, if any: the partial sums in the fixed
// order of k_finalize, then finalize_step; clears the pending flag.  Does nothing once the loop
// has stopped (live false) or when no step is pending.
__device__ __forceinline__ void finalize_pending(const FinArgs &f, bool live) {
    __shared__ double sh[4];
    if (!live || !f.stt->pending) return;  // block-uniform
    double a = 0.0;
#pragma unroll 8
    for (int b = threadIdx.x; b < f.nblk; b += 256) a += f.partials[b];
    const double t = block_sum<256>(a, sh);
    if (threadIdx.x != 0) return;
    f.stt->pending = 0;
    finalize_step(t, f.scal, f.stt, f.hist, f.step_hist, f.perm_table);
}

}  // namespace asdsm
