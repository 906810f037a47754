// Residual-type stencil passes r = b - L x on one level, marching in z:
//   RES_NORM      partial sums of ||r||^2 (FP64 convergence test)
//   RES_RESTRICT  coarse rhs = mean of the 8 children of r (multigrid restriction)
//   RES_OUTER     mixed-precision outer step: q = p + e (e FP32; p NULL reads as
//                 zeros), r = b - L q, p_out = q, r32 = (float) r, partial sums of ||r||^2
// A block owns a 64 x 32 tile of (x, y) and a chunk of z (tall tiles: the 1-cell
// ring of x re-read by neighbouring tiles is 1/16 of a tile row count, not 1/4).  Each thread owns a
// pair of x-adjacent cells of one row.  Per z-step s it writes plane s+1 of x
// (tile plus a 1-cell ring) into one of four LDS slots, issues the loads of
// the next plane, and after a single barrier forms the residual of its pair on
// plane s from LDS (neighbours) and registers (coefficients).  All global loads
// are buffer loads with loop-invariant resources, a wave-uniform plane offset
// and a 32-bit lane offset.
#pragma once

#include "mgp_buffer.hpp"

namespace mgp {

enum { RES_NORM = 0, RES_RESTRICT = 1, RES_OUTER = 2 };

constexpr int kResTY = 32;                  // tile rows
constexpr int kResNT = 32 * kResTY;         // threads per block
constexpr int kResEX = 68;                  // LDS row: x0-2 .. x0+65 (pairs stay 2-aligned)
constexpr int kResEY = kResTY + 2;          // LDS rows: y0-1 .. y0+TY
constexpr int kResPlane = kResEX * kResEY;
constexpr int kResLoads = (66 * kResEY + kResNT - 1) / kResNT;  // x0-1 .. x0+64 of each row

// Density-fed coefficients (passes over the finest grid of a density context):
// density planes are staged in LDS on the iterate's footprint with +inf at
// cells outside the domain, and a pair's face coefficients are formed as the
// correctly rounded 2/(rho_L + rho_R) that defines the face arrays, so a wall
// coefficient comes out as 2/inf = 0 without a branch.
template <typename T>
__device__ inline void rho_plane_load(__amdgpu_buffer_rsrc_t r_rho, __amdgpu_buffer_rsrc_t r_null, const unsigned* loff,
                                      int z, int nz, unsigned psz, T* w)
{
    const bool zv = z >= 0 && z < nz;
    const auto r = zv ? r_rho : r_null;
    const unsigned so = (unsigned)min(max(z, 0), nz - 1) * psz;
#pragma unroll
    for (int j = 0; j < kResLoads; ++j) {
        const T a = bload1<T>(r, loff[j], so);
        w[j] = (zv && loff[j] != kOutside) ? a : (T)__builtin_huge_val();
    }
}

// Faces of the cell pair at LDS index li (even cell) of density plane R0: x faces
// below, between and above the pair, y faces below and above, z faces above
// (densities of the plane above in Rp).
template <typename T, typename T2>
__device__ inline void rho_pair_faces(const T* R0, const T* Rp, int li, T2& bx, T& bxn, T2& by, T2& byu, T2& bzh)
{
    const T2 rc = *reinterpret_cast<const T2*>(R0 + li);
    const T2 rs = *reinterpret_cast<const T2*>(R0 + li - kResEX);
    const T2 rn = *reinterpret_cast<const T2*>(R0 + li + kResEX);
    const T2 ru = *reinterpret_cast<const T2*>(Rp + li);
    bx.x = (T)2 / (R0[li - 1] + rc.x);
    bx.y = (T)2 / (rc.x + rc.y);
    bxn = (T)2 / (rc.y + R0[li + 2]);
    by.x = (T)2 / (rs.x + rc.x);
    by.y = (T)2 / (rs.y + rc.y);
    byu.x = (T)2 / (rc.x + rn.x);
    byu.y = (T)2 / (rc.y + rn.y);
    bzh.x = (T)2 / (rc.x + ru.x);
    bzh.y = (T)2 / (rc.y + ru.y);
}

// Block partial of a double over the block (result valid in thread 0).
template <int NT>
__device__ inline double block_sum_n(double v, double* ws)
{
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    v = wave_sum(v);
    if (lane == 0) ws[wid] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < NT / 64; ++w) s += ws[w];
    return s;
}

// T: arithmetic type of x, b and the coefficients (RES_OUTER: double, with e float).
// RHO: the coefficients are not read from the face arrays but formed from the
// cell density rho as 2/(rho_L + rho_R), the same correctly rounded quotient
// that defines the stored faces, so the results are identical while 8 bytes
// per cell replace 24.  rho is staged in LDS like x, with +inf outside the
// domain, which makes every wall coefficient 2/inf = 0 without a branch.
template <typename T, int MODE, bool RHO = false>
__global__ void __launch_bounds__(kResNT)
k_resid(const T* __restrict__ bx, const T* __restrict__ by, const T* __restrict__ bz, const T* __restrict__ bb,
        const T* __restrict__ x, const float* __restrict__ e, Dims d, T inv_h2, int zc, int ntx, int nty,
        T* __restrict__ xout, float* __restrict__ r32, T* __restrict__ coarse, double* __restrict__ partials,
        const T* __restrict__ rho = nullptr)
{
    using T2 = typename Vec2<T>::type;
    __shared__ T slot[4 * kResPlane];
    __shared__ T rslot[RHO ? 4 * kResPlane : 1];
    __shared__ double ws[kResNT / 64];

    const int nb = (int)gridDim.x, bid = (int)blockIdx.x;
    const int q8 = nb / 8, r8 = nb % 8, xcd = bid % 8;
    const int logical = xcd * q8 + (xcd < r8 ? xcd : r8) + bid / 8;
    const int tx = logical % ntx, ty = (logical / ntx) % nty, tz = logical / (ntx * nty);
    const int x0 = tx * 64, y0 = ty * kResTY, z0 = tz * zc;
    const int z1 = min(z0 + zc, d.nz);

    const int t = (int)threadIdx.x;
    const int row = t >> 5, k = t & 31;
    const int y = y0 + row, xp = x0 + 2 * k;
    const bool mine = y < d.ny && xp < d.nx;
    const int yc = min(y, d.ny - 1), xc = min(xp, d.nx - 2);

    const unsigned psz = (unsigned)((long)d.nx * d.ny * sizeof(T));
    const unsigned pfx = (unsigned)((long)(d.nx + 2) * d.ny * sizeof(T));
    const unsigned pfy = (unsigned)((long)d.nx * (d.ny + 1) * sizeof(T));
    const unsigned rowb = (unsigned)(d.nx * sizeof(T));
    const long ncell = (long)d.nx * d.ny * d.nz;
    const auto r_b = make_rsrc(bb, (unsigned)(ncell * sizeof(T)));
    const auto r_bx = make_rsrc(bx, (unsigned)(n_fx(d) * sizeof(T)));
    const auto r_by = make_rsrc(by, (unsigned)(n_fy(d) * sizeof(T)));
    const auto r_bz = make_rsrc(bz, (unsigned)(n_fz(d) * sizeof(T)));
    const auto r_x = make_rsrc(x, x ? (unsigned)(ncell * sizeof(T)) : 0u);  // x NULL: an iterate of zeros
    const auto r_e = make_rsrc(e ? (const void*)e : (const void*)x, e ? (unsigned)(ncell * sizeof(float)) : 0u);
    const auto r_rho = make_rsrc(RHO ? (const void*)rho : (const void*)x, RHO ? (unsigned)(ncell * sizeof(T)) : 0u);
    const auto r_null = make_rsrc(x, 0u);

    // lane offsets of the pair
    const unsigned oc = (unsigned)(yc * d.nx + xc) * sizeof(T);        // cell / y-face / z-face layouts
    const unsigned ofx = (unsigned)(yc * (d.nx + 2) + xc) * sizeof(T); // x-face layout
    // E1 plane loads: x0-1 .. x0+64 (66) by y0-1 .. y0+TY
    unsigned loff[kResLoads];
    unsigned loffe[kResLoads];
    int lidx[kResLoads];
#pragma unroll
    for (int j = 0; j < kResLoads; ++j) {
        const int f = t + j * kResNT;
        loff[j] = loffe[j] = kOutside;
        lidx[j] = -1;
        if (f < 66 * kResEY) {
            const int ey = f / 66, ex = f - ey * 66;
            const int gx = x0 - 1 + ex, gy = y0 - 1 + ey;
            lidx[j] = ey * kResEX + ex + 1;
            if (gx >= 0 && gx < d.nx && gy >= 0 && gy < d.ny) {
                loff[j] = (unsigned)(gy * d.nx + gx) * sizeof(T);
                loffe[j] = (unsigned)(gy * d.nx + gx) * sizeof(float);
            }
        }
    }
    auto cplane = [&](int z) { return (unsigned)min(max(z, 0), d.nz - 1); };
    auto load_plane = [&](int z, T* v) {
        const bool zv = z >= 0 && z < d.nz;
        const auto r = zv ? r_x : r_null;
        const unsigned so = cplane(z) * psz;
        if constexpr (MODE == RES_OUTER) {
            const auto re = zv ? r_e : r_null;
            const unsigned soe = cplane(z) * (unsigned)((long)d.nx * d.ny * sizeof(float));
#pragma unroll
            for (int j = 0; j < kResLoads; ++j)
                v[j] = bload1<T>(r, loff[j], so) + (T)bload1<float>(re, loffe[j], soe);
        } else {
#pragma unroll
            for (int j = 0; j < kResLoads; ++j) v[j] = bload1<T>(r, loff[j], so);
        }
    };
    auto store_plane = [&](int z, const T* v) {
        T* s = slot + (z & 3) * kResPlane;
#pragma unroll
        for (int j = 0; j < kResLoads; ++j)
            if (lidx[j] >= 0) s[lidx[j]] = v[j];
    };
    // density planes (RHO), staged like x
    auto load_rho = [&](int z, T* w) {
        if constexpr (RHO) rho_plane_load<T>(r_rho, r_null, loff, z, d.nz, psz, w);
    };
    auto store_rho = [&](int z, const T* w) {
        if constexpr (RHO) {
            T* s = rslot + (z & 3) * kResPlane;
#pragma unroll
            for (int j = 0; j < kResLoads; ++j)
                if (lidx[j] >= 0) s[lidx[j]] = w[j];
        }
    };
    struct Coef {
        T2 b, bx, by, byu, bzh;
        T bxn;
    };
    auto load_coef = [&](int z, Coef& C) {
        const unsigned zc_ = cplane(z);
        C.b = bload2<T>(r_b, oc, zc_ * psz);
        if constexpr (RHO) return;
        C.bx = bload2<T>(r_bx, ofx, zc_ * pfx);
        C.bxn = bload1<T>(r_bx, ofx, zc_ * pfx + 2u * sizeof(T));
        C.by = bload2<T>(r_by, oc, zc_ * pfy);
        C.byu = bload2<T>(r_by, oc, zc_ * pfy + rowb);
        C.bzh = bload2<T>(r_bz, oc, (unsigned)min(max(z + 1, 0), d.nz) * psz);
    };

    // prologue
    const int sbeg = z0;
    T v[kResLoads], w[RHO ? kResLoads : 1];
    load_plane(sbeg - 1, v);
    store_plane(sbeg - 1, v);
    load_rho(sbeg - 1, w);
    store_rho(sbeg - 1, w);
    load_plane(sbeg, v);
    store_plane(sbeg, v);
    load_rho(sbeg, w);
    store_rho(sbeg, w);
    load_plane(sbeg + 1, v);
    load_rho(sbeg + 1, w);
    Coef C, Cn;
    load_coef(sbeg, C);
    T2 bzl;
    if constexpr (!RHO) bzl = bload2<T>(r_bz, oc, (unsigned)min(max(sbeg, 0), d.nz) * psz);
    double acc = 0.0;
    T racc = (T)0;
    const int li = (row + 1) * kResEX + (xp - x0) + 2;  // LDS index of the pair's even cell

    for (int s = sbeg; s < z1; ++s) {
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
            // coefficients of the pair's faces from the densities around it; the
            // lower z faces are carried from the step below
            const T* R0 = rslot + (s & 3) * kResPlane;
            if (s == sbeg) {
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
        // cell 0 (even x): west w, east c.y; cell 1: west c.x, east ea.  The
        // products accumulate through explicit fmas in this order (contraction
        // may fuse either product of a two-product sum; the FP32 pre-smoothing +
        // restriction kernel rounds its residuals exactly like this)
        T dg0 = C.bx.x, of0 = C.bx.x * w;
        dg0 += C.bx.y; of0 = fma(C.bx.y, c.y, of0);
        dg0 += C.by.x; of0 = fma(C.by.x, sn.x, of0);
        dg0 += C.byu.x; of0 = fma(C.byu.x, nn.x, of0);
        dg0 += bzl.x; of0 = fma(bzl.x, dn.x, of0);
        dg0 += C.bzh.x; of0 = fma(C.bzh.x, up.x, of0);
        T dg1 = C.bx.y, of1 = C.bx.y * c.x;
        dg1 += C.bxn; of1 = fma(C.bxn, ea, of1);
        dg1 += C.by.y; of1 = fma(C.by.y, sn.y, of1);
        dg1 += C.byu.y; of1 = fma(C.byu.y, nn.y, of1);
        dg1 += bzl.y; of1 = fma(bzl.y, dn.y, of1);
        dg1 += C.bzh.y; of1 = fma(C.bzh.y, up.y, of1);
        const T r0 = mine ? C.b.x - (of0 - dg0 * c.x) * inv_h2 : (T)0;
        const T r1 = mine ? C.b.y - (of1 - dg1 * c.y) * inv_h2 : (T)0;
        const long cell = (long)s * d.nx * d.ny + (long)y * d.nx + xp;
        if constexpr (MODE == RES_NORM) {
            acc += (double)r0 * r0 + (double)r1 * r1;
        } else if constexpr (MODE == RES_OUTER) {
            acc += (double)r0 * r0 + (double)r1 * r1;
            if (mine) {
                *reinterpret_cast<T2*>(xout + cell) = c;
                float2 rr;
                rr.x = (float)r0;
                rr.y = (float)r1;
                *reinterpret_cast<float2*>(r32 + cell) = rr;
            }
        } else {  // RES_RESTRICT: sum the 2x2 children of this plane, then 2 planes
            T sum = r0 + r1;
            sum += __shfl_xor(sum, 32, 64);  // rows 2j and 2j+1 sit in one wave
            racc += sum;
            if (s & 1) {
                if (mine && (row & 1) == 0) {
                    const int cnx = d.nx / 2, cny = d.ny / 2;
                    coarse[((long)(s >> 1) * cny + (y >> 1)) * cnx + (xp >> 1)] = racc * (T)0.125;
                }
                racc = (T)0;
            }
        }
        bzl = C.bzh;
        C = Cn;
    }
    if constexpr (MODE != RES_RESTRICT) {
        const double tot = block_sum_n<kResNT>(acc, ws);
        if (threadIdx.x == 0) partials[blockIdx.x] = tot;
    }
}

struct ResGeom {
    int ntx, nty, zc, nzc, blocks;
};

// Tiling of a level for k_resid; chunks start and end on even planes.
inline ResGeom res_geom(const Dims& d)
{
    ResGeom g;
    g.ntx = (d.nx + 63) / 64;
    g.nty = (d.ny + kResTY - 1) / kResTY;
    const int tiles = g.ntx * g.nty;
    // about 256 blocks, one per compute unit, each a long chunk (each chunk
    // re-reads two planes and restarts its pipeline; at 512^3 the outer update
    // took 1.14 / 1.10 / 1.07 / 1.05 / 1.70 ms with 2048 / 1024 / 512 / 256 /
    // 128 blocks)
    int nzc = (256 + tiles - 1) / tiles;
    int zc = (d.nz + nzc - 1) / nzc;
    // at least 8 planes unless that leaves fewer than 1024 blocks: small grids
    // take short chunks (at 64^3 / 128^3 chunks of 2 took 5.9 / 10.0 against
    // 13.5 / 13.6 us with 8)
    const int z8 = zc < 8 ? 8 : zc;
    if ((long)tiles * ((d.nz + z8 - 1) / z8) >= 1024) zc = z8;
    if (zc < 2) zc = 2;
    zc += zc & 1;
    if (zc >= d.nz) zc = d.nz;
    g.zc = zc;
    g.nzc = (d.nz + zc - 1) / zc;
    g.blocks = tiles * g.nzc;
    return g;
}

// Levels that k_resid handles: at least 64 cells wide and 8 deep in y, even
// extents (restriction needs even ny and nz too), arrays below 2^31 bytes.
inline bool res_tiled_ok(const Dims& d, size_t elem)
{
    const long big = n_fx(d) > n_fz(d) ? n_fx(d) : n_fz(d);
    return d.nx >= 64 && d.ny >= 8 && (d.nx % 2) == 0 && (d.ny % 2) == 0 && (d.nz % 2) == 0 &&
           big * (long)elem < (1L << 31);
}

}  // namespace mgp
