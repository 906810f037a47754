// The coarse end of a V-cycle in one launch.
//
// Below a few thousand cells a level's kernels are far shorter than a launch:
// the pre-sweeps, residual + restriction, prolongation + correction and
// post-sweeps of the 16^3, 8^3 ... grids would cost a dozen launches per level
// for microseconds of work.  Here one workgroup runs the V-cycle's recursion
// below and including the first such level, down to the exact coarsest-grid
// solve and back up, separating the steps with workgroup barriers instead of
// kernel boundaries.
//
// The iterate and the rhs of every level live in LDS for the whole V-cycle (at
// most 2 x 4682 values; the first level's copied in at the start), in FP32 the
// face coefficients too; otherwise only the coarsest inverse (and in FP64 the
// faces) are read from memory, and only the first level's result is written
// back.  A Gauss-Seidel half-sweep reads only cells of the other colour, so
// the sweeps run in place: the same values as the out-of-place sweeps of the
// per-level kernels.  The prolongation and the coarse solve are the per-level
// kernels' device functions (prolong_value_at, coarse_apply_block); the sweeps and
// the restriction compute the same expressions in the same order, with the
// wall terms written as +0 instead of skipped (tail_stencil), so both paths
// give identical results bit for bit.
#pragma once

#include "mgp_kernels.hpp"

namespace mgp {

constexpr int kTailNT = 1024;      // threads of the one workgroup
constexpr long kTailCells = 4096;  // largest grid the tail takes (16^3)
constexpr int kTailLds = 4682;     // cells of a 4096-cell level and all its coarser ones
// cells per thread whose loads are issued together (FP64: 2, within 128 VGPRs)
template <typename T>
constexpr int tail_batch() { return sizeof(T) == 8 ? 2 : 4; }
constexpr int kTailMaxLevels = 16;
constexpr int kTailFaceLds = 24576;  // FP32 face coefficients kept in LDS (96 KB)

// One level as the tail kernel sees it (a table in device memory, built at
// setup): its face arrays and sizes.  Its iterate and rhs live in the kernel's
// LDS instead of the level buffers of the per-level path.
template <typename T>
struct TailLevel {
    const T* bx;
    const T* by;
    const T* bz;
    Dims d;
    T h2;      // h^2 (sweeps)
    T inv_h2;  // 1 / h^2 (residual)
};

// Index arithmetic of the tail's loops (cell index -> coordinates): by shifts
// and masks when every tail level's x and y sizes are powers of two (P2; the
// tail is VALU-bound, and the divisions took about a quarter of its time),
// else by division.
template <bool P2>
__device__ inline void tail_divmod(int q, int n, int& quot, int& rem)
{
    if constexpr (P2) {
        quot = q >> __builtin_ctz((unsigned)n);
        rem = q & (n - 1);
    } else {
        quot = q / n;
        rem = q - quot * n;
    }
}

template <bool P2>
__device__ inline void tail_cell_of(int q, const Dims d, int& i, int& j, int& k)
{
    int row;
    tail_divmod<P2>(q, d.nx, row, i);
    tail_divmod<P2>(row, d.ny, k, j);
}

// The per-level kernels' stencil without its wall branches.  Wall faces are
// stored zeros at every level, so a wall term adds +0 to the diagonal and
// 0 * x to the off-diagonal sum: the same sums as skipping it, term by term in
// the same order (the neighbour index is clamped into the level, where every
// value is finite).  Indices in int: a level here has at most kTailCells cells.
template <typename T>
__device__ inline void tail_stencil(const T* fx, const T* fy, const T* fz, const T* x, const Dims d, int i, int j,
                                    int k, int c, int n, T& diag, T& off)
{
    const int sy = d.nx, sz = d.nx * d.ny;
    const int ix = (k * d.ny + j) * (d.nx + 2) + i, iy = (k * (d.ny + 1) + j) * d.nx + i;
    T dg = 0, of = 0, f;
    f = fx[ix];          dg += f; of += f * x[max(c - 1, 0)];
    f = fx[ix + 1];      dg += f; of += f * x[min(c + 1, n - 1)];
    f = fy[iy];          dg += f; of += f * x[max(c - sy, 0)];
    f = fy[iy + d.nx];   dg += f; of += f * x[min(c + sy, n - 1)];
    f = fz[c];           dg += f; of += f * x[max(c - sz, 0)];
    f = fz[c + sz];      dg += f; of += f * x[min(c + sz, n - 1)];
    diag = dg;
    off = of;
}

// half_sweep_value with tail_stencil
template <typename T>
__device__ inline T tail_half_sweep_value(const T* fx, const T* fy, const T* fz, const Dims d, int n, T h2,
                                          const T* b, const T* src, int zero_src, int i, int j, int k)
{
    const int c = (k * d.ny + j) * d.nx + i;
    T dg, of;
    if (zero_src) {
        const int ix = (k * d.ny + j) * (d.nx + 2) + i, iy = (k * (d.ny + 1) + j) * d.nx + i;
        dg = 0;
        dg += fx[ix];
        dg += fx[ix + 1];
        dg += fy[iy];
        dg += fy[iy + d.nx];
        dg += fz[c];
        dg += fz[c + d.nx * d.ny];
        of = 0;
    } else {
        tail_stencil<T>(fx, fy, fz, src, d, i, j, k, c, n, dg, of);
    }
    T v;
    if (dg > (T)0) v = (of - h2 * b[c]) / dg;
    else v = zero_src ? (T)0 : src[c];
    return v;
}

// k_residual_restrict's coarse value (children added z, then y, then x) with
// tail_stencil
template <typename T>
__device__ inline T tail_restrict_cell(const T* fx, const T* fy, const T* fz, const Dims f, T inv_h2, const T* b,
                                       const T* x, int I, int J, int K)
{
    const int n = f.nx * f.ny * f.nz;
    T s = 0;
    for (int cz = 0; cz < 2; ++cz)
        for (int cy = 0; cy < 2; ++cy)
            for (int cx = 0; cx < 2; ++cx) {
                const int i = 2 * I + cx, j = 2 * J + cy, k = 2 * K + cz;
                const int c = (k * f.ny + j) * f.nx + i;
                T dg, of;
                tail_stencil<T>(fx, fy, fz, x, f, i, j, k, c, n, dg, of);
                s += b[c] - (of - dg * x[c]) * inv_h2;
            }
    return s * (T)0.125;
}

// One sweep of x (in LDS) in place: colour c0 (treating x as 0 if zero_in),
// then the other colour.  fx, fy, fz: the level's faces (LDS or memory).
template <typename T, bool P2>
__device__ void tail_sweep(const T* fx, const T* fy, const T* fz, const Dims d, T h2, const T* b, T* x, int c0,
                           int zero_in)
{
    const int hx = (d.nx + 1) / 2;
    const int cnt = hx * d.ny * d.nz;
    constexpr int kTailBatch = tail_batch<T>();
    for (int h = 0; h < 2; ++h) {
        const int colour = h == 0 ? c0 : 1 - c0;
        const int zs = h == 0 ? zero_in : 0;
        for (int q0 = 0; q0 < cnt; q0 += kTailBatch * kTailNT) {
            T v[kTailBatch];
            int c[kTailBatch];
#pragma unroll
            for (int u = 0; u < kTailBatch; ++u) {
                const int q = q0 + u * kTailNT + (int)threadIdx.x;
                int r, m, k, j;
                tail_divmod<P2>(q, hx, r, m);
                tail_divmod<P2>(r, d.ny, k, j);
                const int i = 2 * m + ((j + k + colour) & 1);
                c[u] = -1;
                if (q < cnt && i < d.nx) {
                    c[u] = (k * d.ny + j) * d.nx + i;
                    v[u] = tail_half_sweep_value<T>(fx, fy, fz, d, d.nx * d.ny * d.nz, h2, b, x, zs, i, j, k);
                }
            }
#pragma unroll
            for (int u = 0; u < kTailBatch; ++u)
                if (c[u] >= 0) x[c[u]] = v[u];
        }
        __syncthreads();
    }
}

// V-cycle from level l0 down to the coarsest level nl-1 and back.  x0: level
// l0's iterate (read unless zero_init says it counts as 0); b0: its rhs;
// pre_done: pre-sweeps already run on level l0.  The result goes to x0, or to
// t0 when the sweeps on level l0 are odd in number (where the per-level path,
// which sweeps from one buffer into the other, leaves it).
// FLDS (FP32 only): the face coefficients of levels l0..nl-2 are copied to LDS
// first (at most kTailFaceLds values together), so that no step after the
// start reads memory except the coarsest inverse; a template flag, so that
// every face read is an LDS read by construction.
// P2: every level's x and y sizes are powers of two (index arithmetic by shifts).
// Launch: one block of kTailNT threads; levels l0..nl-1 at most kTailCells
// cells each and kTailLds together, the coarsest at most 64, nl - l0 at most
// kTailMaxLevels.
template <typename T, bool FLDS, bool P2>
__global__ void __launch_bounds__(kTailNT)
k_vcycle_tail(const TailLevel<T>* __restrict__ tab, int l0, int nl, const double* __restrict__ G,
              T* x0, T* t0, const T* __restrict__ b0, int pre, int post, int zero_init, int pre_done)
{
    static_assert(!FLDS || sizeof(T) == 4, "faces in LDS for FP32 only");
    __shared__ T xs[kTailLds];  // iterate of each level
    __shared__ T bs[kTailLds];  // rhs of each level (the first one's copied in)
    __shared__ T fs[FLDS ? kTailFaceLds : 1];  // faces of the swept levels
    __shared__ double rs[64];
    constexpr int kTailBatch = tail_batch<T>();
    const int tid = (int)threadIdx.x;
    const int nlv = nl - l0;
    // level parameters stay in scalar registers (uniform loads from the table)
    const TailLevel<T>* lv = tab + l0;
    auto ncell = [&](int k) { return lv[k].d.nx * lv[k].d.ny * lv[k].d.nz; };
    auto off = [&](int k) {
        int o = 0;
        for (int m = 0; m < k; ++m) o += ncell(m);
        return o;
    };
    auto nfaces = [&](int k) { return (int)(n_fx(lv[k].d) + n_fy(lv[k].d) + n_fz(lv[k].d)); };
    auto foff = [&](int k) {
        int o = 0;
        for (int m = 0; m < k; ++m) o += nfaces(m);
        return o;
    };
    // every iterate value a stencil may read (also at a clamped wall index) is finite
    for (int q = tid; q < off(nlv); q += kTailNT) xs[q] = (T)0;
    if (!(zero_init && pre_done == 0))
        for (int q = tid; q < ncell(0); q += kTailNT) xs[q] = x0[q];
    for (int q = tid; q < ncell(0); q += kTailNT) bs[q] = b0[q];
    if constexpr (FLDS) {
        {
            for (int k = 0; k < nlv - 1; ++k) {
                T* F = fs + foff(k);
                const int a = (int)n_fx(lv[k].d), c = (int)n_fy(lv[k].d), e = (int)n_fz(lv[k].d);
                for (int q = tid; q < a; q += kTailNT) F[q] = lv[k].bx[q];
                for (int q = tid; q < c; q += kTailNT) F[a + q] = lv[k].by[q];
                for (int q = tid; q < e; q += kTailNT) F[a + c + q] = lv[k].bz[q];
            }
        }
    }
    __syncthreads();
    // the faces of level k, from LDS or from memory
    auto faces = [&](int k, const T*& fx, const T*& fy, const T*& fz) {
        if constexpr (FLDS) {
            fx = fs + foff(k);
            fy = fx + n_fx(lv[k].d);
            fz = fy + n_fy(lv[k].d);
        } else {
            fx = lv[k].bx;
            fy = lv[k].by;
            fz = lv[k].bz;
        }
    };

    for (int k = 0; k < nlv - 1; ++k) {
        const TailLevel<T>& L = lv[k];
        const T *fx, *fy, *fz;
        faces(k, fx, fy, fz);
        T* x = xs + off(k);
        const T* b = bs + off(k);
        const int zi = k == 0 ? zero_init : 1;
        const int done = k == 0 ? pre_done : 0;
        if (zi && pre == 0) {
            for (int q = tid; q < ncell(k); q += kTailNT) x[q] = (T)0;
            __syncthreads();
        }
        for (int s = 0; s < pre - done; ++s)
            tail_sweep<T, P2>(fx, fy, fz, L.d, L.h2, b, x, 0, zi && done == 0 && s == 0);
        const Dims cd = lv[k + 1].d;
        T* bc = bs + off(k + 1);
        for (int q = tid; q < ncell(k + 1); q += kTailNT) {
            int I, J, K;
            tail_cell_of<P2>(q, cd, I, J, K);
            bc[q] = tail_restrict_cell<T>(fx, fy, fz, L.d, L.inv_h2, b, x, I, J, K);
        }
        __syncthreads();
    }
    coarse_apply_block<T>(G, ncell(nlv - 1), bs + off(nlv - 1), xs + off(nlv - 1), rs);
    __syncthreads();
    for (int k = nlv - 2; k >= 0; --k) {
        const TailLevel<T>& L = lv[k];
        const T *fx, *fy, *fz;
        faces(k, fx, fy, fz);
        T* x = xs + off(k);
        const T* e = xs + off(k + 1);
        const T* b = bs + off(k);
        const Dims cd = lv[k + 1].d;
        for (int q0 = 0; q0 < ncell(k); q0 += kTailBatch * kTailNT) {
            T v[kTailBatch];
#pragma unroll
            for (int u = 0; u < kTailBatch; ++u) {
                const int q = q0 + u * kTailNT + tid;
                if (q < ncell(k)) {
                    int i, j, kk;
                    tail_cell_of<P2>(q, L.d, i, j, kk);
                    v[u] = x[q] + prolong_value_at<T, int>(cd, e, i, j, kk);
                }
            }
#pragma unroll
            for (int u = 0; u < kTailBatch; ++u) {
                const int q = q0 + u * kTailNT + tid;
                if (q < ncell(k)) x[q] = v[u];
            }
        }
        __syncthreads();
        for (int s = 0; s < post; ++s) tail_sweep<T, P2>(fx, fy, fz, L.d, L.h2, b, x, 1, 0);
    }
    T* out = (((pre - pre_done) + post) & 1) ? t0 : x0;
    for (int q = tid; q < ncell(0); q += kTailNT) out[q] = xs[q];
}

}  // namespace mgp
