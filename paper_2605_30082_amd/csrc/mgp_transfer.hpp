// Prolongation + correction x_fine += P e_coarse, marching in coarse z.
//
// P is cell-centred trilinear interpolation: per axis a fine cell takes 3/4 of
// its parent and 1/4 of the parent's neighbour on its side, the parent itself
// standing in for a neighbour beyond a wall.  A block owns a 64 x 32 fine tile
// (a 32 x 16 coarse tile) and a chunk of coarse planes.  Per coarse plane K it
// stages coarse plane K+1 (tile plus a 1-cell ring, read at clamped
// coordinates so that the wall rule needs no branch) into one of four LDS
// slots, then each thread updates its fine cell pair in fine planes 2K and 2K+1
// from 12 coarse values.
#pragma once

#include "mgp_buffer.hpp"

namespace mgp {

constexpr int kProTY = 32;                // fine rows per tile
constexpr int kProNT = 32 * kProTY;       // threads: one fine pair each
constexpr int kProCX = 34;                // coarse LDS row: X0-1 .. X0+32
constexpr int kProCY = kProTY / 2 + 2;    // coarse LDS rows: Y0-1 .. Y0+16
constexpr int kProPlane = kProCX * kProCY;
constexpr int kProLoads = (kProPlane + kProNT - 1) / kProNT;

template <typename T>
__global__ void __launch_bounds__(kProNT)
k_prolong_tiled(Dims f, Dims c, const T* __restrict__ e, T* __restrict__ x, int kc, int ntx, int nty)
{
    using T2 = typename Vec2<T>::type;
    __shared__ T slot[4 * kProPlane];

    const int nb = (int)gridDim.x, bid = (int)blockIdx.x;
    const int q8 = nb / 8, r8 = nb % 8, xcd = bid % 8;
    const int logical = xcd * q8 + (xcd < r8 ? xcd : r8) + bid / 8;
    const int tx = logical % ntx, ty = (logical / ntx) % nty, tz = logical / (ntx * nty);
    const int x0 = tx * 64, y0 = ty * kProTY;   // fine tile origin
    const int X0 = x0 / 2, Y0 = y0 / 2;         // coarse tile origin
    const int K0 = tz * kc, K1 = min(K0 + kc, c.nz);

    const int t = (int)threadIdx.x;
    const int row = t >> 5, k = t & 31;
    const int y = y0 + row, xp = x0 + 2 * k;
    const bool mine = y < f.ny && xp < f.nx;

    const long csz = (long)c.nx * c.ny;
    const auto r_e = make_rsrc(e, (unsigned)(csz * c.nz * sizeof(T)));
    // coarse plane loads at clamped coordinates
    unsigned coff[kProLoads];
    int cidx[kProLoads];
#pragma unroll
    for (int j = 0; j < kProLoads; ++j) {
        const int q = t + j * kProNT;
        coff[j] = 0;
        cidx[j] = -1;
        if (q < kProPlane) {
            const int ey = q / kProCX, ex = q - ey * kProCX;
            const int gx = min(max(X0 - 1 + ex, 0), c.nx - 1), gy = min(max(Y0 - 1 + ey, 0), c.ny - 1);
            cidx[j] = q;
            coff[j] = (unsigned)(gy * c.nx + gx) * sizeof(T);
        }
    }
    const unsigned cpb = (unsigned)(csz * sizeof(T));
    auto load_c = [&](int K, T* v) {
        const unsigned so = (unsigned)min(max(K, 0), c.nz - 1) * cpb;
#pragma unroll
        for (int j = 0; j < kProLoads; ++j) v[j] = bload1<T>(r_e, coff[j], so);
    };
    auto store_c = [&](int K, const T* v) {
        T* s = slot + (K & 3) * kProPlane;
#pragma unroll
        for (int j = 0; j < kProLoads; ++j)
            if (cidx[j] >= 0) s[cidx[j]] = v[j];
    };
    // fine pair in two planes
    const int yc = min(y, f.ny - 1), xc = min(xp, f.nx - 2);
    const long fsz = (long)f.nx * f.ny;
    const auto r_x = make_rsrc(x, (unsigned)(fsz * f.nz * sizeof(T)));
    const unsigned fo = (unsigned)(yc * f.nx + xc) * sizeof(T);
    const unsigned fpb = (unsigned)(fsz * sizeof(T));
    auto load_f = [&](int K, T2& a, T2& b) {  // fine planes 2K, 2K+1
        const int z0 = min(2 * K, f.nz - 1), z1 = min(2 * K + 1, f.nz - 1);
        a = bload2<T>(r_x, fo, (unsigned)z0 * fpb);
        b = bload2<T>(r_x, fo, (unsigned)z1 * fpb);
    };

    // LDS coordinates of the parent and its neighbours
    const int I = xp >> 1;                   // parent (both cells of the pair)
    const int lx = I - X0 + 1;               // LDS column of the parent
    const int J = y >> 1;
    const int ly0 = J - Y0 + 1;              // parent row
    const int ly1 = ly0 + ((y & 1) ? 1 : -1);  // row neighbour on this cell's side

    // prologue
    T v[kProLoads];
    load_c(K0 - 1, v);
    store_c(K0 - 1, v);
    load_c(K0, v);
    store_c(K0, v);
    load_c(K0 + 1, v);
    T2 fa, fb;
    load_f(K0, fa, fb);

    for (int K = K0; K < K1; ++K) {
        store_c(K + 1, v);
        load_c(K + 2, v);
        T2 na, nbv;
        load_f(K + 1, na, nbv);
        lds_barrier();
        const T* Sm = slot + ((K - 1) & 3) * kProPlane;
        const T* S0 = slot + (K & 3) * kProPlane;
        const T* Sp = slot + ((K + 1) & 3) * kProPlane;
        // x-interpolated rows (cell 0 takes I-1, cell 1 takes I+1), then y, then z
        auto xrow = [&](const T* S, int ly, T& c0, T& c1) {
            const T* r = S + ly * kProCX + lx;
            const T m = r[0];
            c0 = pro_lerp(m, r[-1]);
            c1 = pro_lerp(m, r[1]);
        };
        T a0, a1, b0, b1;
        xrow(S0, ly0, a0, a1);
        xrow(S0, ly1, b0, b1);
        const T p0 = pro_lerp(a0, b0), p1 = pro_lerp(a1, b1);   // plane K
        xrow(Sm, ly0, a0, a1);
        xrow(Sm, ly1, b0, b1);
        const T m0 = pro_lerp(a0, b0), m1 = pro_lerp(a1, b1);   // plane K-1 (clamped)
        xrow(Sp, ly0, a0, a1);
        xrow(Sp, ly1, b0, b1);
        const T u0 = pro_lerp(a0, b0), u1 = pro_lerp(a1, b1);   // plane K+1 (clamped)
        if (mine) {
            const long base = (long)y * f.nx + xp;
            T2 o;
            o.x = fa.x + pro_lerp(p0, m0);
            o.y = fa.y + pro_lerp(p1, m1);
            *reinterpret_cast<T2*>(x + (long)(2 * K) * fsz + base) = o;
            o.x = fb.x + pro_lerp(p0, u0);
            o.y = fb.y + pro_lerp(p1, u1);
            *reinterpret_cast<T2*>(x + (long)(2 * K + 1) * fsz + base) = o;
        }
        fa = na;
        fb = nbv;
    }
}

struct ProGeom {
    int ntx, nty, kc, nkc, blocks;
};

inline ProGeom pro_geom(const Dims& f, const Dims& c)
{
    ProGeom g;
    g.ntx = (f.nx + 63) / 64;
    g.nty = (f.ny + kProTY - 1) / kProTY;
    const int tiles = g.ntx * g.nty;
    int nkc = (2048 + tiles - 1) / tiles;
    int kc = (c.nz + nkc - 1) / nkc;
    if (kc < 4) kc = 4;
    if (kc >= c.nz) kc = c.nz;
    g.kc = kc;
    g.nkc = (c.nz + kc - 1) / kc;
    g.blocks = tiles * g.nkc;
    return g;
}

// fine levels that k_prolong_tiled handles (even extents, 64 wide, 8 deep)
inline bool pro_tiled_ok(const Dims& f, size_t elem)
{
    return f.nx >= 64 && f.ny >= 8 && (f.nx % 2) == 0 && (f.ny % 2) == 0 && (f.nz % 2) == 0 &&
           (long)f.nx * f.ny * f.nz * (long)elem < (1L << 31);
}

}  // namespace mgp
