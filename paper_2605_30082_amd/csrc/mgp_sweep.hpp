// Red-black Gauss-Seidel sweep kernels.
//
// One full sweep maps `in` to `out`: every cell of the first colour is set from
// its neighbours in `in` (they all have the other colour), then every cell of
// the second colour is set from its (already updated) first-colour neighbours:
//   first colour  : out_c = (sum_f beta_f in_nb  - h^2 b_c) / sum_f beta_f
//   second colour : out_c = (sum_f beta_f out_nb - h^2 b_c) / sum_f beta_f
// Colour of cell (x,y,z) = (x+y+z) & 1; order 0 runs colour 0 (red) first,
// order 1 colour 1 (black) first.  Old values of a colour are never read, so
// one pass over the grid suffices when the second-colour update of plane z-1
// trails the first-colour update of plane z.
//
// k_sweep_fused does exactly that in one launch: a block owns a 64 x TY tile
// of (x, y) and marches through a chunk of z.  Per z-step s it
//   1. writes the prefetched plane s+1 of `in` (tile plus a 2-cell ring) to an
//      LDS slot and issues global loads for the next plane's data;
//   2. updates the first-colour cells of plane s on the tile plus a 1-cell ring
//      (the ring is recomputed here so that no block waits for another);
//   3. updates the second-colour cells of plane s-1 on the tile, and stores the
//      finished cell pairs of plane s-1 with one vector store per thread.
// Each thread owns a pair of x-adjacent cells of one row: in every plane one
// cell of the pair has the first colour and the other the second, so no lane
// idles, and the pair is stored with one 2-element store.  The coefficients of
// the pair are fetched with 2-element buffer loads one plane ahead; ring cells
// (tile edge + 1) fetch their own coefficients in the lanes that own them.
#pragma once

#include "mgp_buffer.hpp"

namespace mgp {

// Algorithmic HBM bytes of one full sweep per cell: read p, b and the three
// low-face coefficients, write p.
template <typename T>
constexpr double sweep_bytes_per_cell()
{
    return 6.0 * sizeof(T);
}

template <int TY>
struct FusedGeom {
    static constexpr int TX = 64;          // tile width (cells)
    static constexpr int EX = TX + 4;      // LDS plane: x0-2 .. x0+TX+1
    static constexpr int EY = TY + 4;      //            y0-2 .. y0+TY+1
    static constexpr int HX = EX / 2;      // cells of one parity per LDS row
    static constexpr int NT = 32 * TY;     // threads: 32 pairs x TY rows
    static constexpr int NW = NT / 64;     // waves
    static constexpr int PLANE = EX * EY;
    static constexpr int NLOAD = (PLANE + NT - 1) / NT;
    static constexpr int NRING = TX + 2 + TY;  // first-colour ring cells per plane
    // LDS position of E2 coordinates (ex, ey): each row keeps its even-x cells,
    // then its odd-x cells, so that the stride-2 accesses of one colour are
    // consecutive in LDS.
    __device__ static int idx(int ex, int ey) { return ey * EX + (ex & 1) * HX + (ex >> 1); }
};

// Launch contract: nx even and >= 64, every array below 2^31 bytes.
// NORM: also accumulate ||b - L in||^2 of the *input* iterate (its partial per
// block goes to partials[blockIdx.x]); the input is read before any update,
// so the sweep that starts a V-cycle yields the residual norm of the previous
// cycle's result.  Per step s the residual of plane s+1 is formed before the
// first colour of plane s is updated: plane s and plane s+1 (with its ring)
// are still the input in LDS, plane s+2 comes from a pair load one step ahead,
// and plane s+1's coefficients from a register set loaded a step earlier.
template <typename T, int TY, bool NORM = false>
__global__ void __launch_bounds__(32 * TY)
k_sweep_fused(const T* __restrict__ bx, const T* __restrict__ by, const T* __restrict__ bz, const T* __restrict__ bb,
        const T* __restrict__ in, T* __restrict__ out, Dims d, T h2, int c0, int zero_in, int zc, int ntx, int nty,
        double* __restrict__ partials = nullptr)
{
    using G = FusedGeom<TY>;
    using T2 = typename Vec2<T>::type;
    __shared__ T slot[4 * G::PLANE];
    const int nb = (int)gridDim.x, bid = (int)blockIdx.x;
    const int q8 = nb / 8, r8 = nb % 8, xcd = bid % 8;
    const int logical = xcd * q8 + (xcd < r8 ? xcd : r8) + bid / 8;
    const int tx = logical % ntx, ty = (logical / ntx) % nty, tz = logical / (ntx * nty);
    const int x0 = tx * G::TX, y0 = ty * TY, z0 = tz * zc;
    const int z1 = min(z0 + zc, d.nz);
    const int t = (int)threadIdx.x;
    const int k = t & 31, row = t >> 5;
    const int y = y0 + row, xp = x0 + 2 * k;
    const bool mine = (y < d.ny) && (xp < d.nx);
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
    const auto r_in = make_rsrc(in, (unsigned)(ncell * sizeof(T)));
    const auto r_null = make_rsrc(in, 0u);
    const unsigned oc = (unsigned)(yc * d.nx + xc) * sizeof(T);
    const unsigned ofx = (unsigned)(yc * (d.nx + 2) + xc) * sizeof(T);

    // E2 plane loads
    unsigned loff[G::NLOAD];
    int lidx[G::NLOAD];
#pragma unroll
    for (int j = 0; j < G::NLOAD; ++j) {
        const int e = t + j * G::NT;
        loff[j] = kOutside;
        lidx[j] = -1;
        if (e < G::PLANE) {
            const int ey = e / G::EX, ex = e - ey * G::EX;
            const int gx = x0 - 2 + ex, gy = y0 - 2 + ey;
            lidx[j] = G::idx(ex, ey);
            if (gx >= 0 && gx < d.nx && gy >= 0 && gy < d.ny) loff[j] = (unsigned)(gy * d.nx + gx) * sizeof(T);
        }
    }
    auto cpl = [&](int z) { return (unsigned)min(max(z, 0), d.nz - 1); };
    auto load_plane = [&](int z, T* v) {
        const bool zv = !zero_in && z >= 0 && z < d.nz;
        const auto r = zv ? r_in : r_null;
        const unsigned so = cpl(z) * psz;
#pragma unroll
        for (int j = 0; j < G::NLOAD; ++j) v[j] = bload1<T>(r, loff[j], so);
    };
    auto store_plane = [&](int z, const T* v) {
        T* s = slot + (z & 3) * G::PLANE;
#pragma unroll
        for (int j = 0; j < G::NLOAD; ++j)
            if (lidx[j] >= 0) s[lidx[j]] = v[j];
    };
    struct Coef {
        T2 b, bx, by, byu, bzh;
        T bxn;
    };
    auto load_coef = [&](int z, Coef& C) {
        const unsigned zc_ = cpl(z);
        C.b = bload2<T>(r_b, oc, zc_ * psz);
        C.bx = bload2<T>(r_bx, ofx, zc_ * pfx);
        C.bxn = bload1<T>(r_bx, ofx, zc_ * pfx + 2u * sizeof(T));
        C.by = bload2<T>(r_by, oc, zc_ * pfy);
        C.byu = bload2<T>(r_by, oc, zc_ * pfy + rowb);
        C.bzh = bload2<T>(r_bz, oc, (unsigned)min(max(z + 1, 0), d.nz) * psz);
    };
    // ring
    const int rq = (t & 63) * G::NW + (t >> 6);
    const bool ring = rq < G::NRING;
    struct Ring {
        T b, bxl, bxh, byl, byh, bzl, bzh;
    };
    auto ring_pos = [&](int z, int& gx, int& gy) {
        const int q = rq;
        if (q < 33) {
            gy = y0 - 1;
            gx = x0 - 1 + ((x0 - 1 + gy + z + c0) & 1) + 2 * q;
        } else if (q < 66) {
            gy = y0 + TY;
            gx = x0 - 1 + ((x0 - 1 + gy + z + c0) & 1) + 2 * (q - 33);
        } else {
            gy = y0 + (q - 66);
            gx = ((x0 - 1 + gy + z + c0) & 1) == 0 ? x0 - 1 : x0 + G::TX;
        }
    };
    auto ring_valid = [&](int z) -> bool {
        if (!ring || z < 0 || z >= d.nz) return false;
        int gx, gy;
        ring_pos(z, gx, gy);
        return gx >= 0 && gx < d.nx && gy >= 0 && gy < d.ny;
    };
    auto load_ring = [&](int z, Ring& R) {
        if (ring_valid(z)) {
            int gx, gy;
            ring_pos(z, gx, gy);
            const unsigned c = (unsigned)(gy * d.nx + gx) * sizeof(T);
            const unsigned f = (unsigned)(gy * (d.nx + 2) + gx) * sizeof(T);
            R.b = bload1<T>(r_b, c, (unsigned)z * psz);
            R.bxl = bload1<T>(r_bx, f, (unsigned)z * pfx);
            R.bxh = bload1<T>(r_bx, f, (unsigned)z * pfx + sizeof(T));
            R.byl = bload1<T>(r_by, c, (unsigned)z * pfy);
            R.byh = bload1<T>(r_by, c, (unsigned)z * pfy + rowb);
            R.bzl = bload1<T>(r_bz, c, (unsigned)z * psz);
            R.bzh = bload1<T>(r_bz, c, (unsigned)(z + 1) * psz);
        }
    };
    auto lds = [&](const T* S, int gx, int gy) -> T { return S[G::idx(gx - (x0 - 2), gy - (y0 - 2))]; };
    auto relax = [&](T bxl, T bxh, T byl, T byh, T bzl, T bzh, T pw, T pe, T ps, T pn, T pd, T pu, T b) -> T {
        T dg = bxl, of = bxl * pw;
        dg += bxh; of += bxh * pe;
        dg += byl; of += byl * ps;
        dg += byh; of += byh * pn;
        dg += bzl; of += bzl * pd;
        dg += bzh; of += bzh * pu;
        return quot(of - h2 * b, dg);
    };

    const int sbeg = z0 - 1;
    T v[G::NLOAD];
    load_plane(sbeg - 1, v);
    store_plane(sbeg - 1, v);
    load_plane(sbeg, v);
    store_plane(sbeg, v);
    load_plane(sbeg + 1, v);
    Coef Cp, C, Cn, Cnn;
    load_coef(sbeg - 1, Cp);
    load_coef(sbeg, C);
    if constexpr (NORM) load_coef(sbeg + 1, Cn);
    // NORM: the pair's own input values of plane s+2, one step ahead
    auto load_pair = [&](int z) -> T2 {
        const bool zv = !zero_in && z >= 0 && z < d.nz;
        return bload2<T>(zv ? r_in : r_null, oc, cpl(z) * psz);
    };
    T2 p2 = {}, p2n = {};
    if constexpr (NORM) p2 = load_pair(sbeg + 2);
    double acc = 0.0;
    T2 zlo_p = bload2<T>(r_bz, oc, (unsigned)min(max(sbeg - 1, 0), d.nz) * psz);  // bz of plane sbeg-1
    Ring R, Rn;
    load_ring(sbeg, R);
    T a_prev2 = (T)0, a_prev = (T)0;

    for (int s = sbeg; s <= z1; ++s) {
        store_plane(s + 1, v);
        load_plane(s + 2, v);
        if constexpr (NORM) {
            p2n = load_pair(s + 3);
            load_coef(s + 2, Cnn);
        } else {
            load_coef(s + 1, Cn);
        }
        load_ring(s + 1, Rn);
        lds_barrier();
        const T* Sm = slot + ((s - 1) & 3) * G::PLANE;
        T* S0 = slot + (s & 3) * G::PLANE;
        const T* Sp = slot + ((s + 1) & 3) * G::PLANE;
        if constexpr (NORM) {
            // residual of the input on plane s+1 (planes s, s+1 in LDS, s+2 in p2)
            if (mine && s + 1 >= z0 && s + 1 < z1) {
                const int ex = xp - (x0 - 2), ey = y - (y0 - 2);
                const T cx = Sp[G::idx(ex, ey)], cy = Sp[G::idx(ex + 1, ey)];
                const T w = Sp[G::idx(ex - 1, ey)], ea = Sp[G::idx(ex + 2, ey)];
                const T s0 = Sp[G::idx(ex, ey - 1)], s1 = Sp[G::idx(ex + 1, ey - 1)];
                const T n0 = Sp[G::idx(ex, ey + 1)], n1 = Sp[G::idx(ex + 1, ey + 1)];
                const T d0 = S0[G::idx(ex, ey)], d1 = S0[G::idx(ex + 1, ey)];
                const T inv_h2 = (T)1 / h2;
                T dg0 = Cn.bx.x, of0 = Cn.bx.x * w;
                dg0 += Cn.bx.y; of0 += Cn.bx.y * cy;
                dg0 += Cn.by.x; of0 += Cn.by.x * s0;
                dg0 += Cn.byu.x; of0 += Cn.byu.x * n0;
                dg0 += C.bzh.x; of0 += C.bzh.x * d0;
                dg0 += Cn.bzh.x; of0 += Cn.bzh.x * p2.x;
                T dg1 = Cn.bx.y, of1 = Cn.bx.y * cx;
                dg1 += Cn.bxn; of1 += Cn.bxn * ea;
                dg1 += Cn.by.y; of1 += Cn.by.y * s1;
                dg1 += Cn.byu.y; of1 += Cn.byu.y * n1;
                dg1 += C.bzh.y; of1 += C.bzh.y * d1;
                dg1 += Cn.bzh.y; of1 += Cn.bzh.y * p2.y;
                const T r0 = Cn.b.x - (of0 - dg0 * cx) * inv_h2;
                const T r1 = Cn.b.y - (of1 - dg1 * cy) * inv_h2;
                acc += (double)r0 * r0 + (double)r1 * r1;
            }
        }
        const bool splane = s >= 0 && s < d.nz;
        const int odd = (xp + y + s + c0) & 1;
        const int xa = xp + odd;
        T a_cur = (T)0;
        if (mine && splane) {
            const T b = odd ? C.b.y : C.b.x;
            const T bxl = odd ? C.bx.y : C.bx.x;
            const T bxh = odd ? C.bxn : C.bx.y;
            const T byl = odd ? C.by.y : C.by.x;
            const T byh = odd ? C.byu.y : C.byu.x;
            const T bzl = odd ? Cp.bzh.y : Cp.bzh.x;
            const T bzh = odd ? C.bzh.y : C.bzh.x;
            a_cur = relax(bxl, bxh, byl, byh, bzl, bzh, lds(S0, xa - 1, y), lds(S0, xa + 1, y), lds(S0, xa, y - 1),
                          lds(S0, xa, y + 1), lds(Sm, xa, y), lds(Sp, xa, y), b);
            S0[G::idx(xa - (x0 - 2), y - (y0 - 2))] = a_cur;
        }
        if (ring_valid(s)) {
            int gx, gy;
            ring_pos(s, gx, gy);
            const T vv = relax(R.bxl, R.bxh, R.byl, R.byh, R.bzl, R.bzh, lds(S0, gx - 1, gy), lds(S0, gx + 1, gy),
                               lds(S0, gx, gy - 1), lds(S0, gx, gy + 1), lds(Sm, gx, gy), lds(Sp, gx, gy), R.b);
            S0[G::idx(gx - (x0 - 2), gy - (y0 - 2))] = vv;
        }
        lds_barrier();
        const int zb = s - 1;
        if (mine && zb >= z0 && zb < z1) {
            const T b = odd ? Cp.b.y : Cp.b.x;
            const T bxl = odd ? Cp.bx.y : Cp.bx.x;
            const T bxh = odd ? Cp.bxn : Cp.bx.y;
            const T byl = odd ? Cp.by.y : Cp.by.x;
            const T byh = odd ? Cp.byu.y : Cp.byu.x;
            const T bzl = odd ? zlo_p.y : zlo_p.x;
            const T bzh = odd ? Cp.bzh.y : Cp.bzh.x;
            const T bv = relax(bxl, bxh, byl, byh, bzl, bzh, lds(Sm, xa - 1, y), lds(Sm, xa + 1, y),
                               lds(Sm, xa, y - 1), lds(Sm, xa, y + 1), a_prev2, a_cur, b);
            T2 o;
            o.x = odd ? a_prev : bv;
            o.y = odd ? bv : a_prev;
            *reinterpret_cast<T2*>(out + (long)zb * d.nx * d.ny + (long)y * d.nx + xp) = o;
        }
        a_prev2 = a_prev;
        a_prev = a_cur;
        zlo_p = Cp.bzh;
        Cp = C;
        C = Cn;
        if constexpr (NORM) {
            Cn = Cnn;
            p2 = p2n;
        }
        R = Rn;
    }
    if constexpr (NORM) {
        __shared__ double ws[G::NW];
        const double v0 = wave_sum(acc);
        if ((t & 63) == 0) ws[t >> 6] = v0;
        __syncthreads();
        if (t == 0) {
            double tot = 0.0;
            for (int w = 0; w < G::NW; ++w) tot += ws[w];
            partials[blockIdx.x] = tot;
        }
    }
}
// Launch of the fused kernel with TY-row tiles; z is split into chunks so that
// the grid holds about 2048 blocks (at least 16 planes per chunk).
struct FusedLaunch {
    int ntx, nty, zc, blocks;
};

template <int TY>
inline FusedLaunch fused_geom(const Dims& d)
{
    FusedLaunch g;
    g.ntx = (d.nx + 63) / 64;
    g.nty = (d.ny + TY - 1) / TY;
    const int tiles = g.ntx * g.nty;
    int nzc = (2048 + tiles - 1) / tiles;
    int zc = (d.nz + nzc - 1) / nzc;
    if (zc < 16) zc = 16;
    if (zc >= d.nz) zc = d.nz;
    g.zc = zc;
    g.blocks = tiles * ((d.nz + zc - 1) / zc);
    return g;
}

// ev0/ev1 (nullable): events that take the kernel's start and end timestamps.
template <typename T, int TY>
hipError_t launch_fused(const T* bx, const T* by, const T* bz, Dims d, T h2, const T* b, const T* in, T* out,
                        int c0, bool zero_in, hipStream_t s, double* norm_partials = nullptr,
                        int* norm_blocks = nullptr, hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr)
{
    const FusedLaunch g = fused_geom<TY>(d);
    const int ntx = g.ntx, nty = g.nty, zc = g.zc, tiles = ntx * nty, nzc = g.blocks / tiles;
    const int zi = zero_in ? 1 : 0;
    if (norm_partials) *norm_blocks = tiles * nzc;
    if (norm_partials)
        hipExtLaunchKernelGGL(k_sweep_fused<T, TY, true>, dim3(tiles * nzc), dim3(32 * TY), 0, s, ev0, ev1, 0, bx, by,
                              bz, b, in, out, d, h2, c0, zi, zc, ntx, nty, norm_partials);
    else
        hipExtLaunchKernelGGL(k_sweep_fused<T, TY, false>, dim3(tiles * nzc), dim3(32 * TY), 0, s, ev0, ev1, 0, bx,
                              by, bz, b, in, out, d, h2, c0, zi, zc, ntx, nty, (double*)nullptr);
    return hipGetLastError();
}

// One full sweep: out = GS(in) with colour order (red, black) for order 0 and
// (black, red) for order 1; `in` is only read (treated as 0 with zero_in).
// Grids at least 64 cells wide use the fused single-pass kernel (FP32 with
// 64 x 8 tiles; FP64 with 64 x 16 tiles, which halve the ring share at its
// lower occupancy); smaller ones run the two half-sweeps as two launches.
inline bool sweep_is_fused(const Dims& d, size_t elem)
{
    const long big = n_fx(d) > n_fz(d) ? n_fx(d) : n_fz(d);
    return d.nx >= 64 && (d.nx % 2) == 0 && d.ny >= 8 && big * (long)elem < (1L << 31);
}

template <typename T>
hipError_t launch_sweep(const T* bx, const T* by, const T* bz, Dims d, T h2, const T* b, const T* in, T* out,
                        int order, bool zero_in, hipStream_t s, hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr)
{
    const int c0 = order == 0 ? 0 : 1;
    if (sweep_is_fused(d, sizeof(T))) {
        if constexpr (sizeof(T) == 8)
            return launch_fused<T, 16>(bx, by, bz, d, h2, b, in, out, c0, zero_in, s, nullptr, nullptr, ev0, ev1);
        else return launch_fused<T, 8>(bx, by, bz, d, h2, b, in, out, c0, zero_in, s, nullptr, nullptr, ev0, ev1);
    }
    const dim3 blk(64, 4, 1);
    const dim3 grd((unsigned)(((d.nx + 1) / 2 + 63) / 64), (unsigned)((d.ny + 3) / 4), (unsigned)d.nz);
    k_half_sweep<T><<<grd, blk, 0, s>>>(bx, by, bz, d, h2, b, in, out, c0, zero_in ? 1 : 0);
    k_half_sweep<T><<<grd, blk, 0, s>>>(bx, by, bz, d, h2, b, out, out, 1 - c0, 0);
    return hipGetLastError();
}

}  // namespace mgp
