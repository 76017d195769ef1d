// Skeleton points of the anisotropic meshes (d = 3, skeleton-sparse refinement): index maps and the
// per-point update shared by k_skel_update and the forward transform that carries the update.
// Point (a, b) of plane c of M_k sits at a + N_f b + N_f^2 c, a and b the fine coordinates of the
// two other axes in increasing order; a point on several planes is stored in each of their meshes
// and counted once, in the mesh of its lowest coarse axis.
#pragma once

#include "device_common.hpp"

namespace asdsm {

// Fine index and ownership of point idx of M_K (N_c N_f^2 < 2^31 points: 32-bit arithmetic).
template <int K>
__device__ __forceinline__ void skel_point(const Geo &g, int idx, int &x0, int &x1, int &x2, bool &owner) {
    const int Nf = g.Nf, n = g.n;
    const unsigned row = (unsigned)idx / (unsigned)Nf;
    const int a = idx - (int)row * Nf;
    const int c = (int)(row / (unsigned)Nf);
    const int b = (int)row - c * Nf;
    const int cf = (c + 1) * n - 1;
    if (K == 0) { x0 = cf; x1 = a; x2 = b; owner = true; }
    if (K == 1) { x0 = a; x1 = cf; x2 = b; owner = !on_coarse(a, n); }
    if (K == 2) { x0 = a; x1 = b; x2 = cf; owner = !on_coarse(a, n) && !on_coarse(b, n); }
}

// Whether point idx of M_k (k at run time) is the copy that sums count (skel_point's owner).
__device__ __forceinline__ bool skel_owner(const Geo &g, int idx, int k) {
    const unsigned row = (unsigned)idx / (unsigned)g.Nf;
    const int a = idx - (int)row * g.Nf;
    const int b = (int)(row % (unsigned)g.Nf);
    return k == 0 || (!on_coarse(a, g.n) && (k == 1 || !on_coarse(b, g.n)));
}

// The update of the skeleton-sparse loop on the points of M_k that thread threadIdx.x of update
// block blk (of nblk per mesh) owns, PPT of them at a stride of nblk * 256 (the launch covers
// every point): r_next = r - s q (r while nothing is pending), and while a step is pending
// u += s e and the sum of r_next^2 over owned points into acc.  All operands of the thread's points
// are loaded before the step s is formed (ready() forms it and tests the flags, which it also
// returns), so their latency overlaps the reduction of the line search's partial sums.
template <int PPT, class Ready>
__device__ __forceinline__ void skel_update_points(const Geo &g, int k, int blk, int nblk, const double *__restrict__ R,
                                                   double *__restrict__ Rn, const double *__restrict__ Q,
                                                   const double *__restrict__ E, double *__restrict__ U,
                                                   Ready ready, bool &pend, bool &live, double &acc) {
    const int per = g.Nc * g.Nf * g.Nf;
    int idx[PPT];
    double r[PPT], q[PPT], e[PPT], u[PPT];
#pragma unroll
    for (int t = 0; t < PPT; ++t) {
        idx[t] = blk * 256 + (int)threadIdx.x + t * nblk * 256;
        const int i = idx[t] < per ? idx[t] : 0;
        r[t] = R[i];
        q[t] = Q[i];
        e[t] = E[i];
        u[t] = U[i];
    }
    double s;
    ready(s, pend, live);  // block-uniform flags
    if (!live) return;
#pragma unroll
    for (int t = 0; t < PPT; ++t) {
        if (idx[t] >= per) continue;
        const double b = pend ? r[t] - s * q[t] : r[t];
        Rn[idx[t]] = b;
        if (pend) {
            U[idx[t]] = u[t] + s * e[t];
            if (skel_owner(g, idx[t], k)) acc += b * b;
        }
    }
}

}  // namespace asdsm
