// Face arrays computed from values of the two cells on either side of every
// face, in one pass over the cells: the face gradient of the adjoint
// (lambda, p), and the coefficients 2/(rho_L + rho_R) from a cell density or
// from the VOF fractions the density is formed from.
//
// Each thread owns one (x, y) column of a chunk of z-planes and marches it
// upwards.  Per plane it reads its own cell, the cell before it in x (the same
// cache lines as its neighbours' cells) and the cell before it in y (a row the
// block has just read: 64 x 16 columns per block, so only one row in 16 comes
// from another block), and keeps the cell below from the previous plane in
// registers; it writes the lower x-, y- and z-face of its cell (plus the upper
// wall of the last column, row or plane).  Every cell array is read from memory
// once, where a pass per face array reads each of them three times.  The face
// values are the same expressions of the same two cells as one thread per face
// evaluates them, so the results are identical bit for bit.  Optionally the
// same pass writes FP32 copies of the faces (the mixed-precision V-cycle's
// coefficients, (float) of each value) and a copy of the cell values.
#pragma once

#include "mgp_kernels.hpp"

namespace mgp {

constexpr int kMarchTX = 64, kMarchTY = 16;  // block: 64 x 16 columns
constexpr long kMarchBlocks = 4096;          // chunks of z cut for about this many tiles

// (lambda, p) of a cell; the face value is (lambda_R - lambda_L)(p_R - p_L)/h^2
struct FaceGradOp {
    const double* lam;
    const double* p;
    double inv_h2;
    using V = double2;
    static constexpr bool kBad = false;
    __device__ V load(long c) const { return double2{lam[c], p[c]}; }
    __device__ double face(V a, V b) const { return (b.x - a.x) * (b.y - a.y) * inv_h2; }
    __device__ bool bad(double, V, V) const { return false; }
    __device__ void copy(long, V) const {}
};

// a cell density; the face value is 2/(rho_L + rho_R), correctly rounded; with
// BAD a count of interior faces whose coefficient or either density is not
// finite and > 0
// finest grid of a density context: with BAD a count of interior faces whose coefficient or
// either density is not finite and > 0; rho_copy (nullable) receives the densities read
template <bool BAD>
struct DensityFaceOp {
    const double* rho;
    double* rho_copy;
    using V = double;
    static constexpr bool kBad = BAD;
    __device__ V load(long c) const { return rho[c]; }
    __device__ double face(V a, V b) const { return 2.0 / (a + b); }
    __device__ bool bad(double v, V a, V b) const { return bad_coeff(v) || bad_coeff(a) || bad_coeff(b); }
    __device__ void copy(long c, V v) const
    {
        if (rho_copy) rho_copy[c] = v;
    }
};

// the density rho_d f_d + rho_f f_f + rho_g max(0, 1 - f_d - f_f) of a cell,
// formed from its VOF fractions, then as DensityFaceOp
struct VofFaceOp {
    const double* fd;
    const double* ff;
    double rd, rf, rg;
    using V = double;
    static constexpr bool kBad = false;
    __device__ V load(long c) const { return cell_density(fd[c], ff[c], rd, rf, rg); }
    __device__ double face(V a, V b) const { return 2.0 / (a + b); }
    __device__ bool bad(double, V, V) const { return false; }
    __device__ void copy(long, V) const {}
};

// rx: length of an x-face row (nx + 1 public, nx + 2 internal with one padding
// entry, written 0).  Block tiles are (tx, ty, tz) = 64 x 16 columns x zc planes,
// visited grid-stride; with Op::kBad, partials[blockIdx.x] = the block's count.
// fx, fy, fz (nullable, all or none): FP32 copies of the faces, same layouts.
template <typename Op>
__global__ void __launch_bounds__(kMarchTX* kMarchTY)
k_faces_march(Op op, Dims d, int rx, int zc, int ntx, int nty, long ntiles, double* __restrict__ gx,
              double* __restrict__ gy, double* __restrict__ gz, double* __restrict__ partials,
              float* __restrict__ fx = nullptr, float* __restrict__ fy = nullptr, float* __restrict__ fz = nullptr)
{
    using V = typename Op::V;
    const bool f32 = fx != nullptr;
    const long sy = d.nx, sz = (long)d.nx * d.ny;
    double bad = 0.0;
    // XCD-aware order: the hardware deals blocks round-robin to the 8 XCDs, so
    // consecutive block ids are remapped to consecutive tiles of one XCD; a
    // tile's left neighbour (whose cache line its first column's x-1 read
    // touches) and the row of tiles below then share its L2
    const int nb = (int)gridDim.x, bid = (int)blockIdx.x;
    const int q8 = nb / 8, r8 = nb % 8, xcd = bid % 8;
    const long logical = (long)xcd * q8 + (xcd < r8 ? xcd : r8) + bid / 8;
    for (long tile = logical; tile < ntiles; tile += nb) {
        const int tx = (int)(tile % ntx);
        const long rest = tile / ntx;
        const int ty = (int)(rest % nty);
        const int tz = (int)(rest / nty);
        const int i = tx * kMarchTX + (int)(threadIdx.x % kMarchTX);
        const int j = ty * kMarchTY + (int)(threadIdx.x / kMarchTX);
        const int k0 = tz * zc, k1 = min(k0 + zc, d.nz);
        if (i >= d.nx || j >= d.ny) continue;
        V below{};
        if (k0 > 0) below = op.load(((long)(k0 - 1) * d.ny + j) * sy + i);
        // the three cells of plane k are loaded one plane ahead, before the
        // stores of the plane below, so that loads stay in flight across them
        long c = ((long)k0 * d.ny + j) * sy + i;
        V v{}, vx{}, vy{};
        if (k0 < k1) {
            v = op.load(c);
            if (i > 0) vx = op.load(c - 1);
            if (j > 0) vy = op.load(c - sy);
        }
        for (int k = k0; k < k1; ++k, c += sz) {
            V nv{}, nvx{}, nvy{};
            if (k + 1 < k1) {
                nv = op.load(c + sz);
                if (i > 0) nvx = op.load(c + sz - 1);
                if (j > 0) nvy = op.load(c + sz - sy);
            }
            const long fxr = ((long)k * d.ny + j) * rx;
            double g = 0.0;
            if (i > 0) {
                g = op.face(vx, v);
                if (Op::kBad) bad += op.bad(g, vx, v) ? 1.0 : 0.0;
            }
            gx[fxr + i] = g;
            if (f32) fx[fxr + i] = (float)g;
            if (i == d.nx - 1)
                for (int e = d.nx; e < rx; ++e) {
                    gx[fxr + e] = 0.0;
                    if (f32) fx[fxr + e] = 0.0f;
                }
            const long fyr = ((long)k * (d.ny + 1) + j) * sy;
            g = 0.0;
            if (j > 0) {
                g = op.face(vy, v);
                if (Op::kBad) bad += op.bad(g, vy, v) ? 1.0 : 0.0;
            }
            gy[fyr + i] = g;
            if (f32) fy[fyr + i] = (float)g;
            if (j == d.ny - 1) {
                gy[fyr + sy + i] = 0.0;
                if (f32) fy[fyr + sy + i] = 0.0f;
            }
            g = 0.0;
            if (k > 0) {
                g = op.face(below, v);
                if (Op::kBad) bad += op.bad(g, below, v) ? 1.0 : 0.0;
            }
            gz[c] = g;
            if (f32) fz[c] = (float)g;
            op.copy(c, v);
            below = v;
            v = nv;
            vx = nvx;
            vy = nvy;
        }
        if (k1 == d.nz) {
            gz[(long)d.nz * sz + (long)j * sy + i] = 0.0;
            if (f32) fz[(long)d.nz * sz + (long)j * sy + i] = 0.0f;
        }
    }
    if (Op::kBad) {
        __shared__ double ws[kMarchTX * kMarchTY / 64];
        const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
        bad = wave_sum(bad);
        if (lane == 0) ws[wid] = bad;
        __syncthreads();
        if (threadIdx.x == 0) {
            double s = 0.0;
            for (int w = 0; w < kMarchTX * kMarchTY / 64; ++w) s += ws[w];
            partials[blockIdx.x] = s;
        }
    }
}

struct MarchGeom {
    int ntx, nty, zc, blocks;
    long ntiles;
};

// z chunks for about kMarchBlocks tiles; at most max_blocks blocks (the
// partials a launch with a count may write)
inline MarchGeom march_geom(const Dims& d, long max_blocks)
{
    MarchGeom g;
    g.ntx = (d.nx + kMarchTX - 1) / kMarchTX;
    g.nty = (d.ny + kMarchTY - 1) / kMarchTY;
    const long cols = (long)g.ntx * g.nty;
    long nzc = (kMarchBlocks + cols - 1) / cols;
    if (nzc > d.nz) nzc = d.nz;
    if (nzc < 1) nzc = 1;
    g.zc = (int)((d.nz + nzc - 1) / nzc);
    nzc = (d.nz + g.zc - 1) / g.zc;
    g.ntiles = cols * nzc;
    g.blocks = (int)(g.ntiles < max_blocks ? g.ntiles : max_blocks);
    return g;
}

}  // namespace mgp
