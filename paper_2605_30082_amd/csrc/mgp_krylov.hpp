// Vector kernels of the flexible conjugate-gradient variant (one V-cycle as
// the preconditioner B, one previous search direction kept):
//   z = B r
//   d = z - ((z, q_prev) / (d_prev, q_prev)) d_prev      (d = z first)
//   q = L d,  alpha = (d, r) / (d, q),  x += alpha d,  r -= alpha q
// Scalars that depend on reductions of the same iteration (gamma, alpha) are
// read from the device scalar slots inside the kernels, so an iteration needs
// one host synchronisation (for the stopping test) like a V-cycle.  All block
// partial sums use the fixed grid of kReduceBlocks blocks: the reductions are
// deterministic.
#pragma once

#include "mgp_kernels.hpp"

namespace mgp {

// out[blockIdx.x] = sum of v over the block
__device__ inline void block_partial(double v, double* out)
{
    v = block_sum(v);
    if (threadIdx.x == 0) out[blockIdx.x] = v;
}

// partials of (z, q); z is the preconditioner output (FP64, or FP32 in mixed mode)
template <typename TZ>
__global__ void k_fcg_dot(const TZ* __restrict__ z, const double* __restrict__ q, long n,
                          double* __restrict__ partials)
{
    double acc = 0.0;
    for (long c = (long)blockIdx.x * kBlock + threadIdx.x; c < n; c += (long)gridDim.x * kBlock)
        acc += (double)z[c] * q[c];
    block_partial(acc, partials);
}

// d = z - gamma d with gamma = scal[zq_slot] / dq_prev (first: d = z)
template <typename TZ>
__global__ void k_fcg_direction(const TZ* __restrict__ z, double* __restrict__ d, long n,
                                const double* __restrict__ scal, int zq_slot, double dq_prev, int first)
{
    const double gamma = first ? 0.0 : scal[zq_slot] / dq_prev;
    for (long c = (long)blockIdx.x * kBlock + threadIdx.x; c < n; c += (long)gridDim.x * kBlock)
        d[c] = first ? (double)z[c] : (double)z[c] - gamma * d[c];
}

// q = L d, with partials of (d, q) in partials[0, gridDim) and of (d, r) in
// partials[gridDim, 2 gridDim)
__global__ void k_fcg_apply(const double* __restrict__ bx, const double* __restrict__ by,
                            const double* __restrict__ bz, Dims d, double inv_h2, const double* __restrict__ dv,
                            const double* __restrict__ r, double* __restrict__ q, double* __restrict__ partials)
{
    const long n = (long)d.nx * d.ny * d.nz;
    double dq = 0.0, dr = 0.0;
    for (long c = (long)blockIdx.x * kBlock + threadIdx.x; c < n; c += (long)gridDim.x * kBlock) {
        int i, j, k;
        cell_of(c, d, i, j, k);
        double dg, of;
        stencil(bx, by, bz, dv, d, i, j, k, c, dg, of);
        const double qc = (of - dg * dv[c]) * inv_h2;
        q[c] = qc;
        dq += dv[c] * qc;
        dr += dv[c] * r[c];
    }
    block_partial(dq, partials);
    block_partial(dr, partials + gridDim.x);
}

// alpha = scal[dr_slot] / scal[dq_slot]; x += alpha d; r -= alpha q;
// r32 = (float) r (when non-null); partials of ||r||^2
__global__ void k_fcg_update(double* __restrict__ x, double* __restrict__ r, const double* __restrict__ dv,
                             const double* __restrict__ q, long n, const double* __restrict__ scal, int dr_slot,
                             int dq_slot, float* __restrict__ r32, double* __restrict__ partials)
{
    const double alpha = scal[dr_slot] / scal[dq_slot];
    double acc = 0.0;
    for (long c = (long)blockIdx.x * kBlock + threadIdx.x; c < n; c += (long)gridDim.x * kBlock) {
        x[c] += alpha * dv[c];
        const double rc = r[c] - alpha * q[c];
        r[c] = rc;
        if (r32) r32[c] = (float)rc;
        acc += rc * rc;
    }
    block_partial(acc, partials);
}

}  // namespace mgp
