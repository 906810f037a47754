// The pre-smoothing of a V-cycle level from a zero iterate (two red-black
// sweeps) fused with the residual + restriction that follows it: one pass over
// memory writes the smoothed iterate x and the coarse right-hand side
// mean-of-8-children(b - L x).
//
// The sweeps are the stages A1, B1, A2, B2 of the two-sweep kernel (see
// mgp_sweep2.hpp), each ring one cell wider, so that the final x is known on
// the tile plus a one-cell ring:
//   phase 1: A1 on plane s (tile + 4 ring), A2 on plane s-3 (+2 ring)
//   phase 2: B1 on plane s-1 (+3 ring), B2 on plane s-4 (+1 ring; the tile
//            part is written to memory), residual of the B-cells of plane s-4,
//            residual of the A-cells of plane s-5.
// From a zero iterate A1 reads no neighbour: each A-cell becomes -h^2 b / diag.
// A B-cell's six neighbours are A-cells, final after A2, so its residual is
// formed from the sums its B2 relaxation has just built.  An A-cell of plane
// s-5 needs the cell above it, at the same (x, y) in plane s-4: the B-cell
// this thread has just relaxed, so that term comes from a register.  Both residuals are evaluated as the
// residual pass (k_resid, RES_RESTRICT) evaluates them: same neighbour values,
// same order of terms, same expression, so the coarse right-hand side equals
// that of the separate passes bit for bit.  The children are summed as there:
// the pair, then the two rows (through a small LDS buffer, since rows of the
// 72-cell-wide plane do not fall on wave halves), then the two planes.
//
// The coefficients of a plane stay in registers from their load (two steps
// ahead) until its B2 stage; the six values of its A-cell are then moved
// aside for the A-cells' residual one step later (seven sets, seven LDS
// planes; the z loop is unrolled seven times).
#pragma once

#include <type_traits>

#include "mgp_sweep2.hpp"

namespace mgp {

// Launch contract: nx even and >= 64, ny even and >= TY, nz even, zc even,
// every array below 2^31 bytes, grid = ntx * nty * ceil(nz / zc) blocks of
// Sweep2Geom<64, TY>::NT threads; coarse has the (nx/2, ny/2, nz/2) layout.
template <int TY>
__global__ void __launch_bounds__((Sweep2Geom<64, TY>::NT))
k_sweep2_restrict(const float* __restrict__ bx, const float* __restrict__ by, const float* __restrict__ bz,
                  const float* __restrict__ bb, float* __restrict__ out, float* __restrict__ coarse, Dims d, float h2,
                  float inv_h2, int c0, int zc, int ntx, int nty)
{
    using G = Sweep2Geom<64, TY>;
    using T = float;
    using T2 = float2;
    constexpr int NS = 7;  // LDS planes s-6 .. s, coefficient sets of planes s-4 .. s+2
    __shared__ T slot[NS * G::PLANE];
    __shared__ T rbuf[(TY / 2) * 32];  // odd tile rows' pair sums of one plane

    const int nb = (int)gridDim.x, bid = (int)blockIdx.x;
    const int q8 = nb / 8, r8 = nb % 8, xcd = bid % 8;
    const int logical = xcd * q8 + (xcd < r8 ? xcd : r8) + bid / 8;
    const int tx = logical % ntx, ty = (logical / ntx) % nty, tz = logical / (ntx * nty);
    const int x0 = tx * 64, y0 = ty * TY, z0 = tz * zc;
    const int z1 = min(z0 + zc, d.nz);
    const int t = (int)threadIdx.x;
    const bool active = t < G::NP;
    const int pxi = active ? t % G::HX : 0, pyi = active ? t / G::HX : 0;
    const int gx0 = x0 - 4 + 2 * pxi, gy = y0 - 4 + pyi;
    const bool inside = active && gx0 >= 0 && gx0 < d.nx && gy >= 0 && gy < d.ny;

    for (int i = t; i < NS * G::PLANE; i += G::NT) slot[i] = (T)0;

    const unsigned psz = (unsigned)((long)d.nx * d.ny * sizeof(T));
    const unsigned pfx = (unsigned)((long)(d.nx + 2) * d.ny * sizeof(T));
    const unsigned pfy = (unsigned)((long)d.nx * (d.ny + 1) * sizeof(T));
    const unsigned rowb = (unsigned)(d.nx * sizeof(T));
    const long ncell = (long)d.nx * d.ny * d.nz;
    const auto r_b = make_rsrc(bb, (unsigned)(ncell * sizeof(T)));
    const auto r_bx = make_rsrc(bx, (unsigned)(n_fx(d) * sizeof(T)));
    const auto r_by = make_rsrc(by, (unsigned)(n_fy(d) * sizeof(T)));
    const auto r_bz = make_rsrc(bz, (unsigned)(n_fz(d) * sizeof(T)));
    const unsigned oc = inside ? (unsigned)(gy * d.nx + gx0) * sizeof(T) : kOutside;
    const auto r_out = make_rsrc(out, (unsigned)(ncell * sizeof(T)));
    const long ccell = (long)(d.nx / 2) * (d.ny / 2) * (d.nz / 2);
    const auto r_coarse = make_rsrc(coarse, (unsigned)(ccell * sizeof(T)));
    // lane offset of the pair's coarse cell within a coarse plane (even rows write)
    const unsigned occ = (unsigned)(((gy >> 1) * (d.nx / 2) + (gx0 >> 1)) * sizeof(T));
    const unsigned cpsz = (unsigned)((long)(d.nx / 2) * (d.ny / 2) * sizeof(T));
    const unsigned ofx = inside ? (unsigned)(gy * (d.nx + 2) + gx0) * sizeof(T) : kOutside;
    const int le = G::idx(2 * pxi, pyi), lo = G::idx(2 * pxi + 1, pyi);

    auto cpl = [&](int z) { return (unsigned)min(max(z, 0), d.nz - 1); };
    auto plane = [&](int K, int dz) -> T* { return slot + ((K + dz + 8 * NS) % NS) * G::PLANE; };
    struct Coef {
        T2 bz, b, bx, by, byu;
        T bxn;
    };
    auto load_coef = [&](int z, Coef& C) {
        const unsigned zz = cpl(z);
        C.bz = bload2<T>(r_bz, oc, (unsigned)min(max(z, 0), d.nz) * psz);
        C.b = bload2<T>(r_b, oc, zz * psz);
        C.bx = bload2<T>(r_bx, ofx, zz * pfx);
        C.bxn = bload1<T>(r_bx, ofx, zz * pfx + 2u * sizeof(T));
        C.by = bload2<T>(r_by, oc, zz * pfy);
        C.byu = bload2<T>(r_by, oc, zz * pfy + rowb);
    };

    // bit 2r + o of `ring`: cell o of the pair lies in the tile + r ring and in the domain
    int ring = 0;
    for (int r = 0; r <= 4; ++r)
        for (int o = 0; o <= 1; ++o) {
            const int gx = gx0 + o;
            const bool in_r = inside && gx >= x0 - r && gx < x0 + 64 + r && gx < d.nx && gy >= y0 - r &&
                              gy < y0 + TY + r;
            ring |= (in_r ? 1 : 0) << (2 * r + o);
        }
    const int gyp = gy & 1;
    const bool core = active && pxi >= 2 && pxi < 2 + 32 && pyi >= 4 && pyi < 4 + TY && gy < d.ny && gx0 < d.nx;
    const bool odd_row = ((pyi - 4) & 1) != 0;
    const int rb = ((pyi - 4) >> 1) * 32 + (pxi - 2);  // rbuf entry of a core pair

    // The six coefficients and the rhs of the colour-`col` cell of the pair on
    // plane z (C: set of plane z, Cup: set of plane z + 1), its LDS index, the
    // LDS index of its lower x-neighbour, and whether the stage at ring r covers it.
    struct Cell {
        T bxl, bxh, byl, byh, bzl, bzh, b;
        int li, xm;
        bool ok;
    };
    auto cell = [&](int z, int col, int r, const Coef& C, const Coef& Cup) -> Cell {
        Cell e;
        const int odd = gyp ^ ((z + col) & 1);
        e.ok = z >= 0 && z < d.nz && ((ring >> (2 * r + odd)) & 1);
        e.li = odd ? lo : le;
        e.xm = odd ? le : lo - 1;
        e.bxl = odd ? C.bx.y : C.bx.x;
        e.bxh = odd ? C.bxn : C.bx.y;
        e.byl = odd ? C.by.y : C.by.x;
        e.byh = odd ? C.byu.y : C.byu.x;
        e.bzl = odd ? C.bz.y : C.bz.x;
        e.bzh = odd ? Cup.bz.y : Cup.bz.x;
        e.b = odd ? C.b.y : C.b.x;
        return e;
    };
    // Gauss-Seidel update of a cell from LDS planes Pm, P0, Pp (z-1, z, z+1);
    // `of` and `dg` are the neighbour and diagonal sums (the terms, order and
    // rounding of the two-sweep kernel and of the residual pass: explicit fmas,
    // since contraction may fuse either product of a two-product sum)
    auto relax = [&](const Cell& e, const T* Pm, const T* P0, const T* Pp, T& of, T& dg) -> T {
        dg = e.bxl;
        of = e.bxl * P0[e.xm];
        dg += e.bxh;
        of = fma(e.bxh, P0[e.xm + 1], of);
        dg += e.byl;
        of = fma(e.byl, P0[e.li - G::RS], of);
        dg += e.byh;
        of = fma(e.byh, P0[e.li + G::RS], of);
        dg += e.bzl;
        of = fma(e.bzl, Pm[e.li], of);
        dg += e.bzh;
        of = fma(e.bzh, Pp[e.li], of);
        return quot(of - h2 * e.b, dg);
    };

    const int cA = c0, cB = 1 - c0;
    const int sbeg = z0 - 4, send = z1 + 5;
    T rB_prev = (T)0, p_own = (T)0, racc = (T)0;
    // the A-cell's coefficients of plane s-5, taken out of its set before the set
    // is reloaded (the upper z-face comes from the set of plane s-4)
    struct ACoef {
        T bxl, bxh, byl, byh, bzl, b;
    } ac{};

    // One z-step at unroll position K = (s - sbeg) mod 7; set(z) = R[(z - sbeg) mod 7].
    auto step = [&](auto Kc, int s, Coef& Ln, const Coef& Cp1, const Coef& Cs, const Coef& Cm1, const Coef& Cm2,
                    const Coef& Cm3, const Coef& Cm4) {
        constexpr int K = decltype(Kc)::value;
        load_coef(s + 2, Ln);
        lds_barrier();
        // phase 1 -------------------------------------------------------------
        {
            // rows of plane s-6: the pair sums of the odd row came through rbuf
            const int zr = s - 6;
            if (core && !odd_row && zr >= z0 && zr < z1) {
                racc += p_own + rbuf[rb];
                if (zr & 1) {
                    bstore1f(r_coarse, racc * (T)0.125, occ, (unsigned)(zr >> 1) * cpsz);
                    racc = (T)0;
                }
            }
        }
        if (s <= z1 + 3) {
            // A1 from the zero iterate: the neighbour sum is 0
            const Cell e = cell(s, cA, 4, Cs, Cp1);
            if (e.ok) {
                T dg = e.bxl;
                dg += e.bxh;
                dg += e.byl;
                dg += e.byh;
                dg += e.bzl;
                dg += e.bzh;
                const T of = (T)0;
                plane(K, 0)[e.li] = quot(of - h2 * e.b, dg);
            }
        }
        if (s - 3 >= z0 - 2 && s - 3 <= z1 + 1) {
            const Cell e = cell(s - 3, cA, 2, Cm3, Cm2);
            if (e.ok) {
                T of, dg;
                plane(K, -3)[e.li] = relax(e, plane(K, -4), plane(K, -3), plane(K, -2), of, dg);
            }
        }
        lds_barrier();
        // phase 2 -------------------------------------------------------------
        if (s - 1 >= z0 - 3 && s - 1 <= z1 + 2) {
            const Cell e = cell(s - 1, cB, 3, Cm1, Cs);
            if (e.ok) {
                T of, dg;
                plane(K, -1)[e.li] = relax(e, plane(K, -2), plane(K, -1), plane(K, 0), of, dg);
            }
        }
        const int zb = s - 4;
        T bv = (T)0, rB = (T)0;
        if (zb >= z0 - 1 && zb <= z1) {
            const Cell e = cell(zb, cB, 1, Cm4, Cm3);
            if (e.ok) {
                T of, dg;
                bv = relax(e, plane(K, -5), plane(K, -4), plane(K, -3), of, dg);
                plane(K, -4)[e.li] = bv;
                rB = e.b - (of - dg * bv) * inv_h2;
            }
            if (core && zb >= z0 && zb < z1) {
                const bool bodd = e.li == lo;
                const T av = plane(K, -4)[bodd ? le : lo];
                T2 o;
                o.x = bodd ? av : bv;
                o.y = bodd ? bv : av;
                bstore2(r_out, o, oc, (unsigned)zb * psz);
            }
        }
        // A-cell of plane s-5 (planes s-6, s-5 are final and untouched in this
        // phase); the cell above it is the B-cell relaxed just now
        const int za = s - 5;
        const int odd5 = gyp ^ ((za + cA) & 1);
        if (core && za >= z0 && za < z1) {
            const int li = odd5 ? lo : le, xm = odd5 ? le : lo - 1;
            const T bzh = odd5 ? Cm4.bz.y : Cm4.bz.x;
            const T* P0 = plane(K, -5);
            const T* Pm = plane(K, -6);
            T dg = ac.bxl;
            T of = ac.bxl * P0[xm];
            dg += ac.bxh;
            of = fma(ac.bxh, P0[xm + 1], of);
            dg += ac.byl;
            of = fma(ac.byl, P0[li - G::RS], of);
            dg += ac.byh;
            of = fma(ac.byh, P0[li + G::RS], of);
            dg += ac.bzl;
            of = fma(ac.bzl, Pm[li], of);
            dg += bzh;
            of = fma(bzh, bv, of);
            const T rA = ac.b - (of - dg * P0[li]) * inv_h2;
            const T pr = rA + rB_prev;
            if (odd_row) rbuf[rb] = pr;
            else p_own = pr;
        }
        // the A-cell of plane s-4 is the other cell of the pair
        ac.bxl = odd5 ? Cm4.bx.x : Cm4.bx.y;
        ac.bxh = odd5 ? Cm4.bx.y : Cm4.bxn;
        ac.byl = odd5 ? Cm4.by.x : Cm4.by.y;
        ac.byh = odd5 ? Cm4.byu.x : Cm4.byu.y;
        ac.bzl = odd5 ? Cm4.bz.x : Cm4.bz.y;
        ac.b = odd5 ? Cm4.b.x : Cm4.b.y;
        rB_prev = rB;
    };

    Coef R0, R1, R2, R3, R4, R5, R6;
    load_coef(sbeg, R0);
    load_coef(sbeg + 1, R1);
    R2 = R3 = R4 = R5 = R6 = R0;
    using I0 = std::integral_constant<int, 0>;
    using I1 = std::integral_constant<int, 1>;
    using I2 = std::integral_constant<int, 2>;
    using I3 = std::integral_constant<int, 3>;
    using I4 = std::integral_constant<int, 4>;
    using I5 = std::integral_constant<int, 5>;
    using I6 = std::integral_constant<int, 6>;
    // step(K, s, Ln = set(s+2), set(s+1), set(s), set(s-1), ..., set(s-4))
    for (int s = sbeg; s <= send; s += 7) {
        step(I0{}, s, R2, R1, R0, R6, R5, R4, R3);
        if (s + 1 > send) break;
        step(I1{}, s + 1, R3, R2, R1, R0, R6, R5, R4);
        if (s + 2 > send) break;
        step(I2{}, s + 2, R4, R3, R2, R1, R0, R6, R5);
        if (s + 3 > send) break;
        step(I3{}, s + 3, R5, R4, R3, R2, R1, R0, R6);
        if (s + 4 > send) break;
        step(I4{}, s + 4, R6, R5, R4, R3, R2, R1, R0);
        if (s + 5 > send) break;
        step(I5{}, s + 5, R0, R6, R5, R4, R3, R2, R1);
        if (s + 6 > send) break;
        step(I6{}, s + 6, R1, R0, R6, R5, R4, R3, R2);
    }
}

// z chunks as for the two-sweep kernel (about 256 blocks), but even: the
// restriction pairs planes 2k, 2k+1 inside a chunk.
template <int TY>
inline Sweep2Launch sweep2r_geom(const Dims& d)
{
    Sweep2Launch g = sweep2_geom<64, TY>(d);
    g.zc += g.zc & 1;
    if (g.zc > d.nz) g.zc = d.nz;
    g.blocks = g.ntx * g.nty * ((d.nz + g.zc - 1) / g.zc);
    return g;
}

constexpr int kSweep2rTY = 16;

// Grids the fused pre-smoothing + restriction serves: those of the 64-wide
// two-sweep launch that also have even extents for the restriction.
inline bool sweep2r_ok(const Dims& d)
{
    return sweep2_ok(d, sizeof(float)) && sweep2_wide(d) && d.ny >= kSweep2rTY && (d.ny % 2) == 0 &&
           (d.nz % 2) == 0;
}

// out = two sweeps (order 0: red first) of L x = b from x = 0; coarse = mean
// of the 8 children of b - L out.
inline hipError_t launch_sweep2_restrict(const float* bx, const float* by, const float* bz, Dims d, float h2,
                                         float inv_h2, const float* b, float* out, float* coarse, int order,
                                         hipStream_t s, hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr)
{
    const Sweep2Launch g = sweep2r_geom<kSweep2rTY>(d);
    hipExtLaunchKernelGGL(k_sweep2_restrict<kSweep2rTY>, dim3(g.blocks), dim3(Sweep2Geom<64, kSweep2rTY>::NT), 0, s,
                          ev0, ev1, 0, bx, by, bz, b, out, coarse, d, h2, inv_h2, order == 0 ? 0 : 1, g.zc, g.ntx,
                          g.nty);
    return hipGetLastError();
}

}  // namespace mgp
