// Two red-black Gauss-Seidel sweeps in one pass over memory (temporal blocking).
//
// Two full sweeps with colour order (A, B) are four half-sweeps A1, B1, A2, B2:
//   A1: A-cells from `in`;  B1: B-cells from A1;  A2: A-cells from B1;
//   B2: B-cells from A2.    out = (A2 on A-cells, B2 on B-cells).
// A half-sweep of a cell reads only its six face neighbours, which have the
// other colour, so a stage on plane z needs the previous stage on planes
// z-1, z, z+1.  A block that owns a TX x TY tile of (x, y) marches a chunk of
// z with the stages staggered in z, per step s (two LDS barriers):
//   phase 1: A1 on plane s   (tile + 3-cell ring)  and  A2 on plane s-3 (tile + 1-cell ring)
//   phase 2: B1 on plane s-1 (tile + 2-cell ring)  and  B2 on plane s-4 (tile)
// The two stages of a phase touch disjoint planes and states: A2(s-3) needs
// B1 up to plane s-2 (done a step earlier), B2(s-4) needs A2 up to s-3 (done
// in phase 1), and B1(s-1) still finds plane s-2's A-cells in state A1.  The rings
// shrink by one cell per stage, so every value a tile cell needs is computed
// inside the block: no block waits for another.  Every plane holds the newest
// value of each of its cells in one LDS slot (7 slots cover planes s-5..s+1;
// plane s+1 goes into the slot of plane s-6); stage order within a step
// guarantees that each read sees the state it needs (e.g. B1(s-1) reads
// A-cells of s-2 before A2 overwrites them in the same step).
//
// Each thread owns one pair of x-adjacent cells of the tile + 4-cell ring
// (TX / 2 + 4 pairs per row, TY + 8 rows): in every plane one cell of the pair is an
// A-cell and the other a B-cell.  The coefficients of the pair's cells are
// loaded once per plane, two steps before first full use, and kept in
// registers for the steps during which the four stages visit that plane.  The
// previous iterate is read once and the result written once: the memory
// traffic of one sweep for two sweeps of work, plus the ring re-reads.
#pragma once

#include <type_traits>

#include "mgp_buffer.hpp"

namespace mgp {

template <int TX_, int TY, int E = 4>
struct Sweep2Geom {
    static constexpr int TX = TX_;             // tile width (cells): 64, or 32 for 32-wide grids
    static constexpr int EX = TX + 8;          // LDS plane: x0-4 .. x0+TX+3
    static constexpr int EY = TY + 8;          //            y0-4 .. y0+TY+3
    static constexpr int HX = EX / 2;          // pairs per row
    static constexpr int NP = HX * EY;         // pairs per plane = working threads
    static constexpr int NT = (NP + 63) / 64 * 64;
    // LDS row stride and offset of a row's odd-x cells.  64-wide FP32 tiles: a
    // wave spans rows of 36 pairs; with RS +- HO = 36 (mod 32), the next row's
    // cells of one colour start in the bank after the previous row's last, and
    // 2 RS = 8 (mod 64): fewer bank conflicts than the packed 72 / 36 layout
    // (measured: 0.864 against 0.879 ms per 512^3 launch).  32-wide tiles (rows
    // of 20 pairs): the same rule, RS - HO = 20 + 4.  FP64 (E = 8, a value
    // takes two banks, 16 lanes cover the 32 banks): consecutive rows of a
    // wave read opposite halves (a stage relaxes the even cells of one row and
    // the odd cells of the next), so a group of 16 lanes that holds the last k
    // pairs of one row and the first 16 - k of the next is free of conflicts
    // when RS + HO = RS - HO = 4 (mod 16): RS = 84, HO = 48.
    static constexpr int RS = E == 8 ? 84 : (TX == 64 ? 100 : 56);
    static constexpr int HO = E == 8 ? 48 : (TX == 64 ? 64 : 32);
    static_assert(RS >= HO + HX, "a row's odd-x cells must not reach the next row");
    static constexpr int PLANE = RS * EY;
    static constexpr int SLOTS = 7;         // planes s-5 .. s+1 of step s
    // LDS position of plane coordinates (ex, ey): each row keeps its even-x
    // cells, then its odd-x cells (one colour of a row is contiguous).
    __device__ static int idx(int ex, int ey) { return ey * RS + (ex & 1) * HO + (ex >> 1); }
};

// Post-smoothing right after a coarse-grid correction can take the correction
// with it (PRO, coarse dims cd = d / 2): the iterate is then read as
// in + P ec, P the trilinear prolongation, so the separate prolongation pass
// (read in, write in) goes away.  The value is the one k_prolong_tiled writes:
// pro_lerp along x, then y, then z.  Fine plane z lies between coarse planes
// (z - 1) / 2 and (z + 1) / 2 (clamped).  Each step the block loads its patch
// of one coarse plane (one value per thread), stores the patch of the plane
// that enters next into one of three LDS slots a step later, and each pair
// interpolates its x and y values from LDS; the correction is added when the
// fine plane goes to LDS, a step after its load.  No load result passes through
// a conditional assignment: a copy made where a branch merges would wait for
// the load, and with it for every load in flight, in the step that issues it.
//
// FP64: the coefficients of seven planes would not fit the registers of 14
// waves, so the FP64 instance takes 64 x 8 tiles (9 waves) and keeps the
// y-face coefficients in LDS planes beside the iterate (written once per plane
// from a load one step ahead, like the iterate; the upper face of a cell is the
// lower face of the cell above it); the other coefficients stay in registers.
//
// Launch contract: nx even and >= TX, ny >= TY, every array below 2^31 bytes,
// grid = ntx * nty * ceil(nz / zc) blocks of Sweep2Geom<TX, TY, sizeof(T)>::NT
// threads; PRO: nx, ny, nz even, ec the d / 2 grid, zero_in 0.
template <typename T, int TX, int TY, bool PRO>
__global__ void __launch_bounds__((Sweep2Geom<TX, TY, sizeof(T)>::NT))
k_sweep2_fused(const T* __restrict__ bx, const T* __restrict__ by, const T* __restrict__ bz,
               const T* __restrict__ bb, const T* __restrict__ in, T* __restrict__ out, Dims d, T h2, int c0,
               int zero_in, int zc, int ntx, int nty, const T* __restrict__ ec, Dims cd)
{
    using G = Sweep2Geom<TX, TY, sizeof(T)>;
    using T2 = typename Vec2<T>::type;
    constexpr bool BYL = sizeof(T) == 8;  // y-face coefficients in LDS planes
    using Fz = std::integral_constant<bool, false>;  // step flavour with the z tests
    __shared__ T slot[G::SLOTS * G::PLANE];
    __shared__ T yslot[BYL ? G::SLOTS * G::PLANE : 1];
    const int nb = (int)gridDim.x, bid = (int)blockIdx.x;
    const int q8 = nb / 8, r8 = nb % 8, xcd = bid % 8;
    const int logical = xcd * q8 + (xcd < r8 ? xcd : r8) + bid / 8;
    const int tx = logical % ntx, ty = (logical / ntx) % nty, tz = logical / (ntx * nty);
    const int x0 = tx * G::TX, y0 = ty * TY, z0 = tz * zc;
    const int z1 = min(z0 + zc, d.nz);
    const int t = (int)threadIdx.x;
    const bool active = t < G::NP;
    const int pxi = active ? t % G::HX : 0, pyi = active ? t / G::HX : 0;
    const int gx0 = x0 - 4 + 2 * pxi, gy = y0 - 4 + pyi;
    const bool inside = active && gx0 >= 0 && gx0 < d.nx && gy >= 0 && gy < d.ny;
    // rows y0-4 and y0+TY+3 only supply neighbour values: no coefficients
    const bool coef_row = inside && pyi >= 1 && pyi <= G::EY - 2;

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
    const auto r_out = make_rsrc(out, (unsigned)(ncell * sizeof(T)));
    const unsigned oin = inside ? (unsigned)(gy * d.nx + gx0) * sizeof(T) : kOutside;
    const unsigned oc = coef_row ? (unsigned)(gy * d.nx + gx0) * sizeof(T) : kOutside;
    const unsigned ofx = coef_row ? (unsigned)(gy * (d.nx + 2) + gx0) * sizeof(T) : kOutside;
    // (LDS y-faces) the lower y-face of every row but the first: the last row's
    // is the upper face of the row below it
    const unsigned oby = (inside && pyi >= 1) ? (unsigned)(gy * d.nx + gx0) * sizeof(T) : kOutside;
    const int le = G::idx(2 * pxi, pyi), lo = G::idx(2 * pxi + 1, pyi);

    auto cpl = [&](int z) { return (unsigned)min(max(z, 0), d.nz - 1); };
    const auto r_e = make_rsrc(ec, PRO ? (unsigned)((long)cd.nx * cd.ny * cd.nz * sizeof(T)) : 0u);
    const unsigned cpb = (unsigned)((long)cd.nx * cd.ny * sizeof(T));
    // A coarse plane goes through LDS as the block's patch of it: columns
    // x0/2 - 3 .. x0/2 + TX/2 + 2 and rows y0/2 - 3 .. y0/2 + TY/2 + 2, each
    // coordinate clamped to the grid (so the patch holds the clamped
    // neighbours the prolongation takes at the walls), one value per thread.
    // Fine plane z lies between coarse planes hu(z) - 1 and hu(z) (clamped),
    // hu(z) = floor((z + 1) / 2), which moves up at odd z; plane c lives in
    // LDS slot c mod 3 from before its first use to after its last.
    constexpr int CPX = TX / 2 + 6, CPY = TY / 2 + 6, CPN = CPX * CPY;
    static_assert(CPN <= G::NT, "one patch value per thread");
    __shared__ T cslot[PRO ? 3 * CPN : 1];
    const unsigned ocp = [&] {
        if (t >= CPN) return kOutside;
        const int ci = min(max(x0 / 2 - 3 + t % CPX, 0), cd.nx - 1);
        const int cj = min(max(y0 / 2 - 3 + t / CPX, 0), cd.ny - 1);
        return (unsigned)(cj * cd.nx + ci) * (unsigned)sizeof(T);
    }();
    auto hu_of = [](int z) { return (z + 1) >> 1; };
    auto cbase = [&](int c) { return cslot + ((c + 3) % 3) * CPN; };  // c >= -3
    // (the plane offset is wave-uniform; said so, or the compiler loops over lanes)
    auto patch_load = [&](int c) {
        const unsigned so = (unsigned)__builtin_amdgcn_readfirstlane(min(max(c, 0), cd.nz - 1)) * cpb;
        return bload1<T>(r_e, ocp, so);
    };
    auto patch_store = [&](int c, T q) {
        if (t < CPN) cbase(c)[t] = q;
    };
    // patch positions of the pair's coarse cell (I, J) and of (I, Jn), Jn the
    // coarse row on the pair's side; I - 1 and I + 1 lie beside them
    const int pm0 = ((gy >> 1) - (y0 / 2 - 3)) * CPX + ((gx0 >> 1) - (x0 / 2 - 3));
    const int dpm = (gy & 1) ? CPX : -CPX;  // pm1 = pm0 + dpm
    // x- and y-interpolated correction of coarse plane c for the pair's two cells
    auto coarse_xy = [&](int c) -> T2 {
        const T* C = cbase(c);
        const int pm1 = pm0 + dpm;
        const T m0 = C[pm0], m1 = C[pm1];
        const T a0 = pro_lerp(m0, C[pm0 - 1]), a1 = pro_lerp(m0, C[pm0 + 1]);
        const T b0 = pro_lerp(m1, C[pm1 - 1]), b1 = pro_lerp(m1, C[pm1 + 1]);
        T2 p;
        p.x = pro_lerp(a0, b0);
        p.y = pro_lerp(a1, b1);
        return p;
    };
    // The step that stores fine plane z to LDS stores the patch of plane
    // hu(z + 1) when it is a new one (z even), loaded a step earlier, and loads
    // that of hu(z + 2): every step loads (half of the loads repeat a plane),
    // so no load result passes through a conditional assignment, which would
    // make the compiler wait for it, and with it for every load in flight, in
    // the step that issues it.
    T Qn;
    auto patch_step = [&](int z) {
        if (!(z & 1)) patch_store(hu_of(z + 1), Qn);
        Qn = patch_load(hu_of(z + 2));
    };
    // FP32 keeps the interpolated values of planes hu(z) - 1 and hu(z) of the
    // plane z last stored in registers (W0, W1; a step reads one plane from
    // LDS); FP64 has no registers to spare for them and reads both planes at
    // each use.
    constexpr bool WIN = sizeof(T) == 4;
    T2 W0, W1;
    auto move_window = [&](int z) {
        const T2 n = coarse_xy(hu_of(z));
        const bool up = (z & 1) != 0;
        W0.x = up ? W1.x : W0.x;
        W0.y = up ? W1.y : W0.y;
        W1 = n;
    };
    // the iterate of fine plane z with the correction added: fine plane 2K
    // takes coarse planes K and K-1, plane 2K+1 K and K+1 (clamped)
    auto corrected = [&](auto fullc, int z, T2 v) -> T2 {
        if constexpr (PRO) {
            if constexpr (WIN) move_window(z);
            if (inside && (decltype(fullc)::value || (z >= 0 && z < d.nz))) {
                T2 hi, lo;
                if constexpr (WIN) {
                    hi = W1;
                    lo = W0;
                } else {
                    hi = coarse_xy(hu_of(z));
                    lo = coarse_xy(hu_of(z) - 1);
                }
                const bool odd = (z & 1) != 0;
                const T2 n = odd ? lo : hi, f = odd ? hi : lo;
                v.x = v.x + pro_lerp(n.x, f.x);
                v.y = v.y + pro_lerp(n.y, f.y);
            }
        }
        return v;
    };
    auto load_in = [&](auto fullc, int z) -> T2 {
        if constexpr (decltype(fullc)::value) {
            if (PRO || !zero_in) return bload2<T>(r_in, oin, (unsigned)z * psz);
        }
        const bool zv = !(PRO ? false : zero_in) && z >= 0 && z < d.nz;
        return bload2<T>(r_in, zv ? oin : kOutside, cpl(z) * psz);
    };
    // LDS plane of z-step position K (0..6) and plane offset dz from the step's
    // plane s: the loop is unrolled seven times, so slot numbers are constants
    auto plane = [&](int K, int dz) -> T* { return slot + ((K + dz + 7 * 7) % 7) * G::PLANE; };
    auto yplane = [&](int K, int dz) -> T* { return yslot + ((K + dz + 7 * 7) % 7) * G::PLANE; };
    auto store_in = [&](T* P, T2 v) {
        if (active) {
            P[le] = v.x;
            P[lo] = v.y;
        }
    };
    // coefficients of the pair in one plane: lower z-faces (loaded first: the
    // stage one plane down needs them as its upper faces one step earlier than
    // the rest), rhs, x-faces (3), y-faces below and above
    struct CoefY {
        T2 by, byu;
    };
    struct Coef : std::conditional_t<BYL, Vec2<T>, CoefY> {
        T2 bz, b, bx;
        T bxn;
    };
    auto load_coef = [&](int z, Coef& C) {
        const unsigned zz = cpl(z);
        // z-faces have nz + 1 planes: plane nz is the top wall (0)
        C.bz = bload2<T>(r_bz, oc, (unsigned)min(max(z, 0), d.nz) * psz);
        C.b = bload2<T>(r_b, oc, zz * psz);
        C.bx = bload2<T>(r_bx, ofx, zz * pfx);
        C.bxn = bload1<T>(r_bx, ofx, zz * pfx + 2u * sizeof(T));
        if constexpr (!BYL) {
            C.by = bload2<T>(r_by, oc, zz * pfy);
            C.byu = bload2<T>(r_by, oc, zz * pfy + rowb);
        }
    };
    auto load_y = [&](int z) -> T2 { return bload2<T>(r_by, oby, cpl(z) * pfy); };

    // Which cell of the pair a stage relaxes, and whether it lies in the
    // stage's ring: bit 2r + o of `ring` says cell o (0 even x, 1 odd x) of
    // this thread's pair is in the tile + r ring and in the domain.
    int ring = 0;
    for (int r = 0; r <= 3; ++r)
        for (int o = 0; o <= 1; ++o) {
            const int gx = gx0 + o;
            const bool in_r = inside && gx >= x0 - r && gx < x0 + G::TX + r && gx < d.nx && gy >= y0 - r &&
                              gy < y0 + TY + r;
            ring |= (in_r ? 1 : 0) << (2 * r + o);
        }
    const int gyp = gy & 1;  // the pair starts at even x: cell parity is (gy + z) & 1 plus the cell index

    // Half-sweep of the colour-`col` cell of the pair on plane z (LDS planes
    // Pm, P0, Pp hold z-1, z, z+1), if that cell lies in the tile + r ring and
    // in the domain; the value goes to `v`, its LDS index to `li`.
    auto relax = [&](auto fullc, int z, int col, int r, const T* Pm, const T* P0, const T* Pp, const T* Y0,
                     const Coef& C, const Coef& Cup, bool& ok, int& li, T& v) {
        const int odd = gyp ^ ((z + col) & 1);
        ok = (decltype(fullc)::value || (z >= 0 && z < d.nz)) && ((ring >> (2 * r + odd)) & 1);
        li = odd ? lo : le;
        if (!ok) return;
        // x-neighbours: (even cell) odd cells x-1, x+1 = lo-1, lo; (odd cell) even cells le, le+1
        const int xm = odd ? le : lo - 1;
        const T bxl = odd ? C.bx.y : C.bx.x;
        const T bxh = odd ? C.bxn : C.bx.y;
        T byl, byh;
        if constexpr (BYL) {
            byl = Y0[li];
            byh = Y0[li + G::RS];
        } else {
            byl = odd ? C.by.y : C.by.x;
            byh = odd ? C.byu.y : C.byu.x;
        }
        const T bzl = odd ? C.bz.y : C.bz.x;
        const T bzh = odd ? Cup.bz.y : Cup.bz.x;
        const T b = odd ? C.b.y : C.b.x;
        // the products accumulate through explicit fmas in this order (the
        // pre-smoothing + restriction kernel and the residual pass round alike)
        T dg = bxl, of = bxl * P0[xm];
        dg += bxh; of = fma(bxh, P0[xm + 1], of);
        dg += byl; of = fma(byl, P0[li - G::RS], of);
        dg += byh; of = fma(byh, P0[li + G::RS], of);
        dg += bzl; of = fma(bzl, Pm[li], of);
        dg += bzh; of = fma(bzh, Pp[li], of);
        v = quot(of - h2 * b, dg);
    };

    const int cA = c0, cB = 1 - c0;
    const int sbeg = z0 - 3, send = z1 + 3;
    const bool core = active && pxi >= 2 && pxi < 2 + G::HX - 4 && pyi >= 4 && pyi < 4 + TY && gy < d.ny &&
                      gx0 < d.nx;

    // One z-step at unroll position K = (s - sbeg) mod 7.  The coefficients of
    // plane z live in set R[(z - sbeg) mod 7]: a step loads plane s+2's set
    // (two steps before its first full use) into the set of plane s-5, which no
    // stage needs any more, so the seven sets rotate by name.  A stage on plane
    // z takes its upper z-faces from the set of plane z+1.  The iterate of
    // plane s+2 is loaded first in the step and written to LDS at the next step.
    T2 v, yv;
    auto step = [&](auto Kc, auto fullc, int s, Coef& Ln, const Coef& Cp1, const Coef& Cs, const Coef& Cm1,
                    const Coef& Cm2, const Coef& Cm3, const Coef& Cm4) {
        constexpr int K = decltype(Kc)::value;
        constexpr bool FULL = decltype(fullc)::value;
        if constexpr (PRO) patch_step(s + 1);
        store_in(plane(K, 1), corrected(fullc, s + 1, v));
        if constexpr (BYL) store_in(yplane(K, 1), yv);
        v = load_in(fullc, s + 2);
        if constexpr (BYL) yv = load_y(s + 2);
        load_coef(s + 2, Ln);
        lds_barrier();
        // phase 1: A1 on plane s and A2 on plane s-3 (disjoint planes and states)
        if (FULL || s <= z1 + 2) {
            bool ok;
            int li;
            T a = (T)0;
            relax(fullc, s, cA, 3, plane(K, -1), plane(K, 0), plane(K, 1), yplane(K, 0), Cs, Cp1, ok, li, a);
            if (ok) plane(K, 0)[li] = a;
        }
        if (FULL || (s - 3 >= z0 - 1 && s - 3 <= z1)) {
            bool ok;
            int li;
            T a = (T)0;
            relax(fullc, s - 3, cA, 1, plane(K, -4), plane(K, -3), plane(K, -2), yplane(K, -3), Cm3, Cm2, ok, li, a);
            if (ok) plane(K, -3)[li] = a;
        }
        lds_barrier();
        // phase 2: B1 on plane s-1 and B2 on plane s-4 (B2 written to memory)
        if (FULL || (s - 1 >= z0 - 2 && s - 1 <= z1 + 1)) {
            bool ok;
            int li;
            T bv = (T)0;
            relax(fullc, s - 1, cB, 2, plane(K, -2), plane(K, -1), plane(K, 0), yplane(K, -1), Cm1, Cs, ok, li, bv);
            if (ok) plane(K, -1)[li] = bv;
        }
        const int zb = s - 4;
        if ((FULL || zb >= z0) && core) {
            bool ok;
            int li;
            T bv = (T)0;
            relax(fullc, zb, cB, 0, plane(K, -5), plane(K, -4), plane(K, -3), yplane(K, -4), Cm4, Cm3, ok, li, bv);
            const bool bodd = li == lo;
            const T av = plane(K, -4)[bodd ? le : lo];
            T2 o;
            o.x = bodd ? av : bv;
            o.y = bodd ? bv : av;
            bstore2(r_out, o, oin, (unsigned)zb * psz);
        }
    };

    if constexpr (PRO) {
        // the planes the prologue and the first step read; then the window of
        // plane sbeg - 2 (moved to sbeg - 1 by the first use)
        for (int c = hu_of(sbeg - 1) - 1; c <= hu_of(sbeg + 1); ++c) patch_store(c, patch_load(c));
        lds_barrier();
        if constexpr (WIN) {
            // planes hu - 1, hu of plane sbeg - 2: h - 1, h (sbeg - 1 even) or h - 2, h - 1
            // (sbeg - 1 odd: the first move drops W0, set to h - 1 here)
            const int h = hu_of(sbeg - 1);
            W0 = coarse_xy(h - 1);
            W1 = ((sbeg - 1) & 1) ? W0 : coarse_xy(h);
        }
    }
    store_in(plane(0, -1), corrected(Fz{}, sbeg - 1, load_in(Fz{}, sbeg - 1)));
    store_in(plane(0, 0), corrected(Fz{}, sbeg, load_in(Fz{}, sbeg)));
    v = load_in(Fz{}, sbeg + 1);
    if constexpr (BYL) {
        store_in(yplane(0, 0), load_y(sbeg));
        yv = load_y(sbeg + 1);
    }
    if constexpr (PRO) {
        Qn = patch_load(hu_of(sbeg + 2));
        lds_barrier();  // the reads above before the first step's patch store
    }
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
    // step(K, full, s, Ln = set(s+2), set(s+1), set(s), set(s-1), set(s-2), set(s-3), set(s-4)).
    // Steps s in [z0 + 4, min(z1 + 2, nz - 3)] touch planes s-5 .. s+2 all
    // inside the grid and run every stage: they take the "full" instance,
    // without the z tests and the branches around the stages.
    const int flo = z0 + 4, fhi = min(z1 + 2, d.nz - 3);
    using Ft = std::integral_constant<bool, true>;
    auto seven = [&](auto fullc, int s) {
        step(I0{}, fullc, s, R2, R1, R0, R6, R5, R4, R3);
        step(I1{}, fullc, s + 1, R3, R2, R1, R0, R6, R5, R4);
        step(I2{}, fullc, s + 2, R4, R3, R2, R1, R0, R6, R5);
        step(I3{}, fullc, s + 3, R5, R4, R3, R2, R1, R0, R6);
        step(I4{}, fullc, s + 4, R6, R5, R4, R3, R2, R1, R0);
        step(I5{}, fullc, s + 5, R0, R6, R5, R4, R3, R2, R1);
        step(I6{}, fullc, s + 6, R1, R0, R6, R5, R4, R3, R2);
    };
    int s = sbeg;
    for (; s < flo && s + 6 <= send; s += 7) seven(Fz{}, s);
    for (; s + 6 <= fhi; s += 7) seven(Ft{}, s);
    for (; s <= send; s += 7) {
        step(I0{}, Fz{}, s, R2, R1, R0, R6, R5, R4, R3);
        if (s + 1 > send) break;
        step(I1{}, Fz{}, s + 1, R3, R2, R1, R0, R6, R5, R4);
        if (s + 2 > send) break;
        step(I2{}, Fz{}, s + 2, R4, R3, R2, R1, R0, R6, R5);
        if (s + 3 > send) break;
        step(I3{}, Fz{}, s + 3, R5, R4, R3, R2, R1, R0, R6);
        if (s + 4 > send) break;
        step(I4{}, Fz{}, s + 4, R6, R5, R4, R3, R2, R1, R0);
        if (s + 5 > send) break;
        step(I5{}, Fz{}, s + 5, R0, R6, R5, R4, R3, R2, R1);
        if (s + 6 > send) break;
        step(I6{}, Fz{}, s + 6, R1, R0, R6, R5, R4, R3, R2);
    }
}

// Blocks of the two-sweep kernel: z is cut into chunks so that the grid holds
// about 256 blocks, one per compute unit (one block of 14 waves fills a CU).
// Measured on 128^3..512^3 grids, fewer and longer chunks beat more and
// shorter ones down to one block per CU; a chunk re-walks 7 planes of stage
// lag, so grids too small to fill the chip (64^3: 4 tiles) take chunks of
// down to 2 planes, which run 14.5 against 22.8 us with 8-plane chunks.
struct Sweep2Launch {
    int ntx, nty, zc, blocks;
};

template <int TX, int TY>
inline Sweep2Launch sweep2_geom(const Dims& d)
{
    Sweep2Launch g;
    g.ntx = (d.nx + TX - 1) / TX;
    g.nty = (d.ny + TY - 1) / TY;
    const int tiles = g.ntx * g.nty;
    int nzc = (256 + tiles - 1) / tiles;
    int zc = (d.nz + nzc - 1) / nzc;
    if (zc < 2) zc = 2;
    if (zc > d.nz) zc = d.nz;
    g.zc = zc;
    g.blocks = tiles * ((d.nz + zc - 1) / zc);
    return g;
}

// Tile rows of the two-sweep launches: 16 in FP32, 8 in FP64.
template <typename T>
constexpr int sweep2_ty() { return sizeof(T) == 8 ? 8 : 16; }

// Grids the two-sweep kernel serves: FP32 at least 32 cells wide (even; 64-wide
// tiles from 64 cells on) and 16 rows; FP64 at least 64 cells wide (even) and
// 8 rows; arrays below 2^31 bytes.
inline bool sweep2_ok(const Dims& d, size_t elem)
{
    const long big = n_fx(d) > n_fz(d) ? n_fx(d) : n_fz(d);
    if (big * (long)elem >= (1L << 31) || (d.nx % 2) != 0) return false;
    if (elem == 4) return d.nx >= 32 && d.ny >= 16;
    return elem == 8 && d.nx >= 64 && d.ny >= 8;
}

// the launches with 64-wide tiles (the timed ones)
inline bool sweep2_wide(const Dims& d) { return d.nx >= 64; }

// ev0/ev1 (nullable): events that take the kernel's start and end timestamps.
// ec (nullable): coarse correction to prolongate into `in` on the fly (grid d
// must then have even extents and ec the d / 2 grid; zero_in false).
template <typename T>
hipError_t launch_sweep2(const T* bx, const T* by, const T* bz, Dims d, T h2, const T* b, const T* in, T* out,
                         int order, bool zero_in, hipStream_t s, hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr,
                         const T* ec = nullptr)
{
    constexpr int TY = sweep2_ty<T>();
    const Dims cd{d.nx / 2, d.ny / 2, d.nz / 2};
    const int c0 = order == 0 ? 0 : 1, zi = zero_in ? 1 : 0;
    if (sweep2_wide(d)) {
        const Sweep2Launch g = sweep2_geom<64, TY>(d);
        auto k = ec ? k_sweep2_fused<T, 64, TY, true> : k_sweep2_fused<T, 64, TY, false>;
        hipExtLaunchKernelGGL(k, dim3(g.blocks), dim3(Sweep2Geom<64, TY, sizeof(T)>::NT), 0, s, ev0, ev1, 0, bx, by,
                              bz, b, in, out, d, h2, c0, zi, g.zc, g.ntx, g.nty, ec, cd);
    } else if constexpr (sizeof(T) == 4) {
        const Sweep2Launch g = sweep2_geom<32, TY>(d);
        auto k = ec ? k_sweep2_fused<T, 32, TY, true> : k_sweep2_fused<T, 32, TY, false>;
        hipExtLaunchKernelGGL(k, dim3(g.blocks), dim3(Sweep2Geom<32, TY>::NT), 0, s, ev0, ev1, 0, bx, by, bz, b, in,
                              out, d, h2, c0, zi, g.zc, g.ntx, g.nty, ec, cd);
    } else {
        return hipErrorInvalidValue;  // FP64 pairs only on 64-wide grids (sweep2_ok)
    }
    return hipGetLastError();
}

}  // namespace mgp
