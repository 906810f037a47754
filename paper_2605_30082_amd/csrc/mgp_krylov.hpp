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
#include "mgp_resid.hpp"

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

// The direction update and q = L d in one tiled pass (the tiling of k_resid:
// 64 x 32 tiles marching in z, one LDS plane per step): while a plane of d is
// staged into LDS it is formed as z - gamma d_prev (gamma = scal[zq_slot] /
// dq_prev; first: d = z), with its 1-cell ring recomputed rather than
// exchanged.  Each thread writes d and q for its pair and accumulates (d, q)
// into partials[0, gridDim) and (d, r) into partials[gridDim, 2 gridDim).
// RHO: coefficients formed from the cell density rho (staged like d), as in
// the density-fed instances of k_resid.
template <typename TZ, bool RHO = false>
__global__ void __launch_bounds__(kResNT)
k_fcg_dir_apply(const double* __restrict__ bx, const double* __restrict__ by, const double* __restrict__ bz,
                const TZ* __restrict__ zv, const double* __restrict__ dprev, const double* __restrict__ r, Dims d,
                double inv_h2, const double* __restrict__ scal, int zq_slot, double dq_prev, int first, int zc,
                int ntx, int nty, double* __restrict__ dout, double* __restrict__ q, double* __restrict__ partials,
                const double* __restrict__ rho = nullptr)
{
    using T = double;
    using T2 = double2;
    __shared__ T slot[4 * kResPlane];
    __shared__ T rslot[RHO ? 4 * kResPlane : 1];
    __shared__ double ws[kResNT / 64];

    const int nb = (int)gridDim.x, bid = (int)blockIdx.x;
    const int q8 = nb / 8, r8 = nb % 8, xcd = bid % 8;
    const int logical = xcd * q8 + (xcd < r8 ? xcd : r8) + bid / 8;
    const int tx = logical % ntx, ty = (logical / ntx) % nty, tz = logical / (ntx * nty);
    const int x0 = tx * 64, y0 = ty * kResTY, z0 = tz * zc;
    const int z1 = min(z0 + zc, d.nz);
    const double gamma = first ? 0.0 : scal[zq_slot] / dq_prev;

    const int t = (int)threadIdx.x;
    const int row = t >> 5, k = t & 31;
    const int y = y0 + row, xp = x0 + 2 * k;
    const bool mine = y < d.ny && xp < d.nx;
    const int yc = min(y, d.ny - 1), xc = min(xp, d.nx - 2);

    const unsigned psz = (unsigned)((long)d.nx * d.ny * sizeof(T));
    const unsigned pszz = (unsigned)((long)d.nx * d.ny * sizeof(TZ));
    const unsigned pfx = (unsigned)((long)(d.nx + 2) * d.ny * sizeof(T));
    const unsigned pfy = (unsigned)((long)d.nx * (d.ny + 1) * sizeof(T));
    const unsigned rowb = (unsigned)(d.nx * sizeof(T));
    const long ncell = (long)d.nx * d.ny * d.nz;
    const auto r_r = make_rsrc(r, (unsigned)(ncell * sizeof(T)));
    const auto r_bx = make_rsrc(bx, (unsigned)(n_fx(d) * sizeof(T)));
    const auto r_by = make_rsrc(by, (unsigned)(n_fy(d) * sizeof(T)));
    const auto r_bz = make_rsrc(bz, (unsigned)(n_fz(d) * sizeof(T)));
    const auto r_z = make_rsrc(zv, (unsigned)(ncell * sizeof(TZ)));
    const auto r_dp = make_rsrc(dprev, first ? 0u : (unsigned)(ncell * sizeof(T)));
    const auto r_rho = make_rsrc(RHO ? (const void*)rho : (const void*)zv, RHO ? (unsigned)(ncell * sizeof(T)) : 0u);
    const auto r_null = make_rsrc(zv, 0u);

    const unsigned oc = (unsigned)(yc * d.nx + xc) * sizeof(T);
    const unsigned ofx = (unsigned)(yc * (d.nx + 2) + xc) * sizeof(T);
    unsigned loff[kResLoads], loffz[kResLoads];
    int lidx[kResLoads];
#pragma unroll
    for (int j = 0; j < kResLoads; ++j) {
        const int f = t + j * kResNT;
        loff[j] = loffz[j] = kOutside;
        lidx[j] = -1;
        if (f < 66 * kResEY) {
            const int ey = f / 66, ex = f - ey * 66;
            const int gx = x0 - 1 + ex, gy = y0 - 1 + ey;
            lidx[j] = ey * kResEX + ex + 1;
            if (gx >= 0 && gx < d.nx && gy >= 0 && gy < d.ny) {
                loff[j] = (unsigned)(gy * d.nx + gx) * sizeof(T);
                loffz[j] = (unsigned)(gy * d.nx + gx) * sizeof(TZ);
            }
        }
    }
    auto cplane = [&](int zz) { return (unsigned)min(max(zz, 0), d.nz - 1); };
    // plane of d = z - gamma d_prev (0 outside the domain)
    auto load_plane = [&](int zz, T* v) {
        const bool in = zz >= 0 && zz < d.nz;
        const auto rz = in ? r_z : r_null;
        const auto rd = in ? r_dp : r_null;
#pragma unroll
        for (int j = 0; j < kResLoads; ++j)
            v[j] = (T)bload1<TZ>(rz, loffz[j], cplane(zz) * pszz) - gamma * bload1<T>(rd, loff[j], cplane(zz) * psz);
    };
    auto store_plane = [&](int zz, const T* v) {
        T* sl = slot + (zz & 3) * kResPlane;
#pragma unroll
        for (int j = 0; j < kResLoads; ++j)
            if (lidx[j] >= 0) sl[lidx[j]] = v[j];
    };
    auto load_rho = [&](int zz, T* w) {
        if constexpr (RHO) rho_plane_load<T>(r_rho, r_null, loff, zz, d.nz, psz, w);
    };
    auto store_rho = [&](int zz, const T* w) {
        if constexpr (RHO) {
            T* sl = rslot + (zz & 3) * kResPlane;
#pragma unroll
            for (int j = 0; j < kResLoads; ++j)
                if (lidx[j] >= 0) sl[lidx[j]] = w[j];
        }
    };
    struct Coef {
        T2 r, bx, by, byu, bzh;
        T bxn;
    };
    auto load_coef = [&](int zz, Coef& C) {
        const unsigned zp = cplane(zz);
        C.r = bload2<T>(r_r, oc, zp * psz);
        if constexpr (RHO) return;
        C.bx = bload2<T>(r_bx, ofx, zp * pfx);
        C.bxn = bload1<T>(r_bx, ofx, zp * pfx + 2u * sizeof(T));
        C.by = bload2<T>(r_by, oc, zp * pfy);
        C.byu = bload2<T>(r_by, oc, zp * pfy + rowb);
        C.bzh = bload2<T>(r_bz, oc, (unsigned)min(max(zz + 1, 0), d.nz) * psz);
    };

    T v[kResLoads], w[RHO ? kResLoads : 1];
    load_plane(z0 - 1, v);
    store_plane(z0 - 1, v);
    load_rho(z0 - 1, w);
    store_rho(z0 - 1, w);
    load_plane(z0, v);
    store_plane(z0, v);
    load_rho(z0, w);
    store_rho(z0, w);
    load_plane(z0 + 1, v);
    load_rho(z0 + 1, w);
    Coef C, Cn;
    load_coef(z0, C);
    T2 bzl;
    if constexpr (!RHO) bzl = bload2<T>(r_bz, oc, (unsigned)min(max(z0, 0), d.nz) * psz);
    double dq = 0.0, dr = 0.0;
    const int li = (row + 1) * kResEX + (xp - x0) + 2;

    for (int s = z0; s < z1; ++s) {
        store_plane(s + 1, v);
        load_plane(s + 2, v);
        store_rho(s + 1, w);
        load_rho(s + 2, w);
        load_coef(s + 1, Cn);
        lds_barrier();
        const T* S0 = slot + (s & 3) * kResPlane;
        const T* Sm = slot + ((s - 1) & 3) * kResPlane;
        const T* Sp = slot + ((s + 1) & 3) * kResPlane;
        if constexpr (RHO) {
            const T* R0 = rslot + (s & 3) * kResPlane;
            if (s == z0) {
                const T2 rd = *reinterpret_cast<const T2*>(rslot + ((s - 1) & 3) * kResPlane + li);
                const T2 rc = *reinterpret_cast<const T2*>(R0 + li);
                bzl.x = (T)2 / (rd.x + rc.x);
                bzl.y = (T)2 / (rd.y + rc.y);
            }
            rho_pair_faces<T, T2>(R0, rslot + ((s + 1) & 3) * kResPlane, li, C.bx, C.bxn, C.by, C.byu, C.bzh);
        }
        const T2 c = *reinterpret_cast<const T2*>(S0 + li);
        const T w = S0[li - 1], ea = S0[li + 2];
        const T2 sn = *reinterpret_cast<const T2*>(S0 + li - kResEX);
        const T2 nn = *reinterpret_cast<const T2*>(S0 + li + kResEX);
        const T2 dn = *reinterpret_cast<const T2*>(Sm + li);
        const T2 up = *reinterpret_cast<const T2*>(Sp + li);
        T dg0 = C.bx.x, of0 = C.bx.x * w;
        dg0 += C.bx.y; of0 += C.bx.y * c.y;
        dg0 += C.by.x; of0 += C.by.x * sn.x;
        dg0 += C.byu.x; of0 += C.byu.x * nn.x;
        dg0 += bzl.x; of0 += bzl.x * dn.x;
        dg0 += C.bzh.x; of0 += C.bzh.x * up.x;
        T dg1 = C.bx.y, of1 = C.bx.y * c.x;
        dg1 += C.bxn; of1 += C.bxn * ea;
        dg1 += C.by.y; of1 += C.by.y * sn.y;
        dg1 += C.byu.y; of1 += C.byu.y * nn.y;
        dg1 += bzl.y; of1 += bzl.y * dn.y;
        dg1 += C.bzh.y; of1 += C.bzh.y * up.y;
        if (mine) {
            T2 qq;
            qq.x = (of0 - dg0 * c.x) * inv_h2;
            qq.y = (of1 - dg1 * c.y) * inv_h2;
            const long cell = (long)s * d.nx * d.ny + (long)y * d.nx + xp;
            *reinterpret_cast<T2*>(dout + cell) = c;
            *reinterpret_cast<T2*>(q + cell) = qq;
            dq += c.x * qq.x + c.y * qq.y;
            dr += c.x * C.r.x + c.y * C.r.y;
        }
        bzl = C.bzh;
        C = Cn;
    }
    const double t0 = block_sum_n<kResNT>(dq, ws);
    __syncthreads();
    const double t1 = block_sum_n<kResNT>(dr, ws);
    if (threadIdx.x == 0) {
        partials[blockIdx.x] = t0;
        partials[gridDim.x + blockIdx.x] = t1;
    }
}

}  // namespace mgp
