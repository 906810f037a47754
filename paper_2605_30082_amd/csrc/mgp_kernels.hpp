// Device kernels of the multigrid pressure-Poisson solver (gfx950).
//
// Internal layouts of a level with nx*ny*nz cells (x fastest):
//   cell arrays   T[nz][ny][nx]
//   x-faces       T[nz][ny][nx+2]  entry x = face between cells x-1 and x;
//                                  x = 0 and x = nx are walls (stored 0), x = nx+1
//                                  is padding (0) that keeps rows of even length
//   y-faces       T[nz][ny+1][nx]  rows 0 and ny are walls (0)
//   z-faces       T[nz+1][ny][nx]  planes 0 and nz are walls (0)
// Both faces of every cell are plain loads (walls are real zeros), so the
// stencil kernels need no branch for a wall coefficient.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mgp {

constexpr int kBlock = 256;          // threads per block of the generic kernels
constexpr int kReduceBlocks = 1024;  // fixed partial count -> deterministic reductions

struct Dims {
    int nx, ny, nz;
};

__host__ __device__ inline long fx_index(const Dims& d, int x, int y, int z)
{
    return ((long)z * d.ny + y) * (d.nx + 2) + x;
}
__host__ __device__ inline long fy_index(const Dims& d, int x, int y, int z)
{
    return ((long)z * (d.ny + 1) + y) * d.nx + x;
}
__host__ __device__ inline long fz_index(const Dims& d, int x, int y, int z)
{
    return ((long)z * d.ny + y) * d.nx + x;
}
__host__ __device__ inline long n_fx(const Dims& d) { return (long)d.nz * d.ny * (d.nx + 2); }
__host__ __device__ inline long n_fy(const Dims& d) { return (long)d.nz * (d.ny + 1) * d.nx; }
__host__ __device__ inline long n_fz(const Dims& d) { return (long)(d.nz + 1) * d.ny * d.nx; }

// ---------------------------------------------------------------------------
// reductions: fixed-shape block partials, then one block sums them in order
// ---------------------------------------------------------------------------

__device__ inline double wave_sum(double v)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    return v;
}

// Sum over the block; the result is valid in thread 0.  blockDim.x == kBlock.
__device__ inline double block_sum(double v)
{
    __shared__ double ws[kBlock / 64];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    v = wave_sum(v);
    if (lane == 0) ws[wid] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0) {
        for (int w = 0; w < kBlock / 64; ++w) s += ws[w];
    }
    __syncthreads();
    return s;
}

// out[slot] = sum of partials[0..count)
__global__ void k_reduce_final(const double* __restrict__ partials, int count, double* __restrict__ out,
                               int slot)
{
    double v = 0.0;
    for (int t = threadIdx.x; t < count; t += kBlock) v += partials[t];
    v = block_sum(v);
    if (threadIdx.x == 0) out[slot] = v;
}

// The reductions over a whole array run a fixed grid (kReduceBlocks), so each
// thread walks many elements: it loads kReduceUnroll of them before adding
// any (that many loads in flight instead of one), in the order of the plain
// grid-stride loop, so the sums do not depend on the unrolling.
constexpr int kReduceUnroll = 8;

template <typename T>
__global__ void k_sum(const T* __restrict__ x, long n, double* __restrict__ partials)
{
    constexpr int U = kReduceUnroll;
    const long stride = (long)gridDim.x * kBlock;
    double v = 0.0;
    long c = (long)blockIdx.x * kBlock + threadIdx.x;
    for (; c + (U - 1) * stride < n; c += U * stride) {
        T a[U];
        for (int u = 0; u < U; ++u) a[u] = x[c + u * stride];
        for (int u = 0; u < U; ++u) v += (double)a[u];
    }
    for (; c < n; c += stride) v += (double)x[c];
    v = block_sum(v);
    if (threadIdx.x == 0) partials[blockIdx.x] = v;
}

// y = x - scal[slot] * scale (and, with F32, y32 = y rounded to FP32), partial
// sums of y^2
template <bool F32>
__global__ void k_sub_scalar_norm(const double* __restrict__ x, long n, const double* __restrict__ scal,
                                  int slot, double scale, double* __restrict__ y, float* __restrict__ y32,
                                  double* __restrict__ partials)
{
    constexpr int U = kReduceUnroll;
    const long stride = (long)gridDim.x * kBlock;
    const double mu = scal[slot] * scale;
    double v = 0.0;
    auto put = [&](long i, double xi) {
        const double t = xi - mu;
        y[i] = t;
        if constexpr (F32) y32[i] = (float)t;
        v += t * t;
    };
    long c = (long)blockIdx.x * kBlock + threadIdx.x;
    for (; c + (U - 1) * stride < n; c += U * stride) {
        double a[U];
        for (int u = 0; u < U; ++u) a[u] = x[c + u * stride];
        for (int u = 0; u < U; ++u) put(c + u * stride, a[u]);
    }
    for (; c < n; c += stride) put(c, x[c]);
    v = block_sum(v);
    if (threadIdx.x == 0) partials[blockIdx.x] = v;
}

// x -= scal[slot] * scale
__global__ void k_sub_scalar(double* __restrict__ x, long n, const double* __restrict__ scal, int slot,
                             double scale)
{
    const double mu = scal[slot] * scale;
    for (long c = (long)blockIdx.x * kBlock + threadIdx.x; c < n; c += (long)gridDim.x * kBlock)
        x[c] -= mu;
}

template <typename T>
__global__ void k_fill(T* __restrict__ x, long n, T v)
{
    for (long c = (long)blockIdx.x * kBlock + threadIdx.x; c < n; c += (long)gridDim.x * kBlock) x[c] = v;
}

template <typename S, typename D>
__global__ void k_convert(const S* __restrict__ x, long n, D* __restrict__ y)
{
    for (long c = (long)blockIdx.x * kBlock + threadIdx.x; c < n; c += (long)gridDim.x * kBlock)
        y[c] = (D)x[c];
}

// ---------------------------------------------------------------------------
// face coefficients: import, validation, coarsening
// ---------------------------------------------------------------------------

__device__ inline void cell_of(long c, const Dims d, int& i, int& j, int& k)
{
    const unsigned cc = (unsigned)c;
    const unsigned row = cc / (unsigned)d.nx;
    i = (int)(cc - row * (unsigned)d.nx);
    k = (int)(row / (unsigned)d.ny);
    j = (int)(row - (unsigned)k * (unsigned)d.ny);
}

__device__ inline bool bad_coeff(double v)
{
    return !(v > 0.0) || !(v < INFINITY);  // NaN, <= 0 or +Inf
}

// public face layouts -> internal layouts (walls and padding written as 0);
// partial count of interior entries that are not finite and > 0
__global__ void k_import_faces(const double* __restrict__ pbx, const double* __restrict__ pby,
                               const double* __restrict__ pbz, Dims d, double* __restrict__ bx,
                               double* __restrict__ by, double* __restrict__ bz,
                               double* __restrict__ partials, float* __restrict__ fbx = nullptr,
                               float* __restrict__ fby = nullptr, float* __restrict__ fbz = nullptr)
{
    const bool f32 = fbx != nullptr;  // also the FP32 copies (all three or none)
    const long nx_ = n_fx(d), ny_ = n_fy(d), nz_ = n_fz(d);
    const long total = nx_ + ny_ + nz_;
    double bad = 0.0;
    for (long f = (long)blockIdx.x * kBlock + threadIdx.x; f < total; f += (long)gridDim.x * kBlock) {
        if (f < nx_) {
            const int x = (int)(f % (d.nx + 2));
            const long row = f / (d.nx + 2);
            double v = 0.0;
            if (x >= 1 && x <= d.nx - 1) {
                v = pbx[row * (d.nx + 1) + x];
                bad += bad_coeff(v) ? 1.0 : 0.0;
            }
            bx[f] = v;
            if (f32) fbx[f] = (float)v;
        } else if (f < nx_ + ny_) {
            const long g = f - nx_;
            const int y = (int)((g / d.nx) % (d.ny + 1));
            double v = 0.0;
            if (y >= 1 && y <= d.ny - 1) {
                v = pby[g];
                bad += bad_coeff(v) ? 1.0 : 0.0;
            }
            by[g] = v;
            if (f32) fby[g] = (float)v;
        } else {
            const long g = f - nx_ - ny_;
            const int z = (int)(g / ((long)d.ny * d.nx));
            double v = 0.0;
            if (z >= 1 && z <= d.nz - 1) {
                v = pbz[g];
                bad += bad_coeff(v) ? 1.0 : 0.0;
            }
            bz[g] = v;
            if (f32) fbz[g] = (float)v;
        }
    }
    bad = block_sum(bad);
    if (threadIdx.x == 0) partials[blockIdx.x] = bad;
}

// internal face layouts of a level -> public face layouts
template <typename T>
__global__ void k_export_faces(const T* __restrict__ bx, const T* __restrict__ by, const T* __restrict__ bz,
                               Dims d, double* __restrict__ pbx, double* __restrict__ pby,
                               double* __restrict__ pbz)
{
    const long nfx = (long)d.nz * d.ny * (d.nx + 1);
    const long nfy = n_fy(d), nfz = n_fz(d);
    const long total = nfx + nfy + nfz;
    for (long f = (long)blockIdx.x * kBlock + threadIdx.x; f < total; f += (long)gridDim.x * kBlock) {
        if (f < nfx) {
            const int x = (int)(f % (d.nx + 1));
            const long row = f / (d.nx + 1);
            pbx[f] = (double)bx[row * (d.nx + 2) + x];
        } else if (f < nfx + nfy) {
            pby[f - nfx] = (double)by[f - nfx];
        } else {
            pbz[f - nfx - nfy] = (double)bz[f - nfx - nfy];
        }
    }
}

// coarse face = mean of the 4 fine faces that tile it (walls stay 0)
__global__ void k_coarsen_faces(const double* __restrict__ fbx, const double* __restrict__ fby,
                                const double* __restrict__ fbz, Dims f, Dims c, double* __restrict__ cbx,
                                double* __restrict__ cby, double* __restrict__ cbz, float* __restrict__ sbx = nullptr,
                                float* __restrict__ sby = nullptr, float* __restrict__ sbz = nullptr)
{
    const bool f32 = sbx != nullptr;  // also the FP32 copies (all three or none)
    const long nx_ = n_fx(c), ny_ = n_fy(c), nz_ = n_fz(c);
    const long total = nx_ + ny_ + nz_;
    for (long g = (long)blockIdx.x * kBlock + threadIdx.x; g < total; g += (long)gridDim.x * kBlock) {
        if (g < nx_) {
            const int X = (int)(g % (c.nx + 2));
            const long row = g / (c.nx + 2);
            const int Y = (int)(row % c.ny), Z = (int)(row / c.ny);
            double v = 0.0;
            if (X >= 1 && X <= c.nx - 1)
                v = (fbx[fx_index(f, 2 * X, 2 * Y, 2 * Z)] + fbx[fx_index(f, 2 * X, 2 * Y + 1, 2 * Z)] +
                     fbx[fx_index(f, 2 * X, 2 * Y, 2 * Z + 1)] + fbx[fx_index(f, 2 * X, 2 * Y + 1, 2 * Z + 1)]) / 4.0;
            cbx[g] = v;
            if (f32) sbx[g] = (float)v;
        } else if (g < nx_ + ny_) {
            const long h = g - nx_;
            const int X = (int)(h % c.nx);
            const long row = h / c.nx;
            const int Y = (int)(row % (c.ny + 1)), Z = (int)(row / (c.ny + 1));
            double v = 0.0;
            if (Y >= 1 && Y <= c.ny - 1)
                v = (fby[fy_index(f, 2 * X, 2 * Y, 2 * Z)] + fby[fy_index(f, 2 * X + 1, 2 * Y, 2 * Z)] +
                     fby[fy_index(f, 2 * X, 2 * Y, 2 * Z + 1)] + fby[fy_index(f, 2 * X + 1, 2 * Y, 2 * Z + 1)]) / 4.0;
            cby[h] = v;
            if (f32) sby[h] = (float)v;
        } else {
            const long h = g - nx_ - ny_;
            const int X = (int)(h % c.nx);
            const long row = h / c.nx;
            const int Y = (int)(row % c.ny), Z = (int)(row / c.ny);
            double v = 0.0;
            if (Z >= 1 && Z <= c.nz - 1)
                v = (fbz[fz_index(f, 2 * X, 2 * Y, 2 * Z)] + fbz[fz_index(f, 2 * X + 1, 2 * Y, 2 * Z)] +
                     fbz[fz_index(f, 2 * X, 2 * Y + 1, 2 * Z)] + fbz[fz_index(f, 2 * X + 1, 2 * Y + 1, 2 * Z)]) / 4.0;
            cbz[h] = v;
            if (f32) sbz[h] = (float)v;
        }
    }
}

// ---------------------------------------------------------------------------
// exact coarsest-grid inverse (setup, one block)
// ---------------------------------------------------------------------------

constexpr int kCoarseMax = 64;    // cells of the coarsest grid at most
constexpr int kCoarseNT = 1024;   // threads of the coarse-inverse block

// Builds the bordered matrix M = [[L, 1], [1^T, 0]] (m = n+1) of the coarsest
// level next to an identity, reduces it by Gauss-Jordan elimination with
// partial pivoting, and stores G = top-left n x n block of M^-1: for any r,
// G r is the zero-mean solution of L e = r - mean(r).  The m x 2m system lives
// in LDS (at most 65 x 130 doubles); the pivot of a column is the first row of
// largest magnitude, found by one wave.  status[0] = 0 on success, 1 if
// singular.  Launch: one block of kCoarseNT threads, n <= kCoarseMax.
__global__ void __launch_bounds__(kCoarseNT)
k_coarse_inverse(const double* __restrict__ bx, const double* __restrict__ by, const double* __restrict__ bz, Dims d,
                 double h, double* __restrict__ G, double* __restrict__ status)
{
    const int n = d.nx * d.ny * d.nz, m = n + 1, w = 2 * m;
    const double h2 = h * h;
    __shared__ double work[(kCoarseMax + 1) * 2 * (kCoarseMax + 1)];
    __shared__ int piv_row;
    __shared__ int singular;
    for (int t = threadIdx.x; t < m * w; t += blockDim.x) work[t] = 0.0;
    if (threadIdx.x == 0) singular = 0;
    __syncthreads();
    for (int c = threadIdx.x; c < m; c += blockDim.x) {
        double* row = work + c * w;
        row[m + c] = 1.0;
        if (c == n) {
            for (int t = 0; t < n; ++t) row[t] = 1.0;
            continue;
        }
        const int i = c % d.nx, j = (c / d.nx) % d.ny, k = c / (d.nx * d.ny);
        const int sy = d.nx, sz = d.nx * d.ny;
        double diag = 0.0, bf;
        if (i > 0)        { bf = bx[fx_index(d, i, j, k)];     row[c - 1] += bf / h2;  diag -= bf / h2; }
        if (i < d.nx - 1) { bf = bx[fx_index(d, i + 1, j, k)]; row[c + 1] += bf / h2;  diag -= bf / h2; }
        if (j > 0)        { bf = by[fy_index(d, i, j, k)];     row[c - sy] += bf / h2; diag -= bf / h2; }
        if (j < d.ny - 1) { bf = by[fy_index(d, i, j + 1, k)]; row[c + sy] += bf / h2; diag -= bf / h2; }
        if (k > 0)        { bf = bz[fz_index(d, i, j, k)];     row[c - sz] += bf / h2; diag -= bf / h2; }
        if (k < d.nz - 1) { bf = bz[fz_index(d, i, j, k + 1)]; row[c + sz] += bf / h2; diag -= bf / h2; }
        row[c] += diag;
        row[n] = 1.0;
    }
    __syncthreads();
    for (int col = 0; col < m; ++col) {
        if (threadIdx.x < 64) {
            // first row of largest |a| among rows col..m-1 (two rows per lane, then the wave)
            const int lane = threadIdx.x;
            double best = -1.0;
            int p = m;
            for (int r = col + lane; r < m; r += 64) {
                const double a = fabs(work[r * w + col]);
                if (r == col || a > best) {  // row col stands first, as in a serial search
                    best = a;
                    p = r;
                }
            }
            for (int off = 32; off > 0; off >>= 1) {
                const double ob = __shfl_down(best, off, 64);
                const int op = __shfl_down(p, off, 64);
                if (ob > best || (ob == best && op < p)) {
                    best = ob;
                    p = op;
                }
            }
            if (lane == 0) {
                piv_row = p;
                if (best == 0.0) singular = 1;
            }
        }
        __syncthreads();
        if (singular) break;
        const int p = piv_row;
        if (p != col) {
            for (int t = threadIdx.x; t < w; t += blockDim.x) {
                const double a = work[col * w + t];
                work[col * w + t] = work[p * w + t];
                work[p * w + t] = a;
            }
        }
        __syncthreads();
        const double inv = 1.0 / work[col * w + col];
        __syncthreads();
        for (int t = threadIdx.x; t < w; t += blockDim.x) work[col * w + t] *= inv;
        __syncthreads();
        // eliminate column `col` from every other row; the pivot row is read-only
        // here (element e = r w + t, its row and column stepped without division)
        {
            const int dr = (int)blockDim.x / w, dt = (int)blockDim.x % w;
            int r = (int)threadIdx.x / w, t = (int)threadIdx.x % w;
            for (; r < m; r += dr, t += dt) {
                if (t >= w) {
                    t -= w;
                    ++r;
                    if (r >= m) break;
                }
                if (r == col || t == col) continue;
                const double f = work[r * w + col];
                work[r * w + t] -= f * work[col * w + t];
            }
        }
        __syncthreads();
        for (int r = threadIdx.x; r < m; r += blockDim.x)
            if (r != col) work[r * w + col] = 0.0;
        __syncthreads();
    }
    for (int e = threadIdx.x; e < n * n; e += blockDim.x) {
        const int r = e / n, t = e % n;
        G[e] = work[r * w + m + t];
    }
    if (threadIdx.x == 0) status[0] = singular ? 1.0 : 0.0;
}

// e = G r on the coarsest level (n <= 64 cells), accumulated in FP64, by the
// first n threads of a block; rs: 64 doubles of LDS
template <typename T>
__device__ inline void coarse_apply_block(const double* __restrict__ G, int n, const T* __restrict__ r,
                                          T* __restrict__ e, double* rs)
{
    const int t = threadIdx.x;
    if (t < n) rs[t] = (double)r[t];
    __syncthreads();
    if (t < n) {
        double s = 0.0;
        for (int j = 0; j < n; ++j) s += G[(long)t * n + j] * rs[j];
        e[t] = (T)s;
    }
}

template <typename T>
__global__ void k_coarse_apply(const double* __restrict__ G, int n, const T* __restrict__ r, T* __restrict__ e)
{
    __shared__ double rs[64];
    coarse_apply_block<T>(G, n, r, e, rs);
}

// ---------------------------------------------------------------------------
// stencil helpers
// ---------------------------------------------------------------------------

// Face and cell indices in an index type I: long in general, int where a
// level is known to be small (the single-workgroup launch); same values.
template <typename I>
__device__ inline I fx_at(const Dims& d, int x, int y, int z)
{
    return ((I)z * d.ny + y) * (d.nx + 2) + x;
}
template <typename I>
__device__ inline I fy_at(const Dims& d, int x, int y, int z)
{
    return ((I)z * (d.ny + 1) + y) * d.nx + x;
}
template <typename I>
__device__ inline I fz_at(const Dims& d, int x, int y, int z)
{
    return ((I)z * d.ny + y) * d.nx + x;
}

// diag = sum of coupled face coefficients, off = sum beta_f * x_neighbour
template <typename T, typename X, typename I = long>
__device__ inline void stencil(const T* __restrict__ bx, const T* __restrict__ by, const T* __restrict__ bz,
                               const X* x, const Dims d, int i, int j, int k, I c, T& diag, T& off)
{
    const I sy = d.nx, sz = (I)d.nx * d.ny;
    T dg = 0, of = 0, f;
    if (i > 0)        { f = bx[fx_at<I>(d, i, j, k)];     dg += f; of += f * (T)x[c - 1]; }
    if (i < d.nx - 1) { f = bx[fx_at<I>(d, i + 1, j, k)]; dg += f; of += f * (T)x[c + 1]; }
    if (j > 0)        { f = by[fy_at<I>(d, i, j, k)];     dg += f; of += f * (T)x[c - sy]; }
    if (j < d.ny - 1) { f = by[fy_at<I>(d, i, j + 1, k)]; dg += f; of += f * (T)x[c + sy]; }
    if (k > 0)        { f = bz[fz_at<I>(d, i, j, k)];     dg += f; of += f * (T)x[c - sz]; }
    if (k < d.nz - 1) { f = bz[fz_at<I>(d, i, j, k + 1)]; dg += f; of += f * (T)x[c + sz]; }
    diag = dg;
    off = of;
}

// ---------------------------------------------------------------------------
// reference-shaped kernels: apply, residual norm, half-sweeps, transfers
// ---------------------------------------------------------------------------

// y = L x
__global__ void k_apply(const double* __restrict__ bx, const double* __restrict__ by,
                        const double* __restrict__ bz, Dims d, double inv_h2, const double* __restrict__ x,
                        double* __restrict__ y)
{
    const long n = (long)d.nx * d.ny * d.nz;
    for (long c = (long)blockIdx.x * kBlock + threadIdx.x; c < n; c += (long)gridDim.x * kBlock) {
        int i, j, k;
        cell_of(c, d, i, j, k);
        double dg, of;
        stencil(bx, by, bz, x, d, i, j, k, c, dg, of);
        y[c] = (of - dg * x[c]) * inv_h2;
    }
}

// partials of ||b - L p||^2 (optionally storing r)
__global__ void k_residual_norm(const double* __restrict__ bx, const double* __restrict__ by,
                                const double* __restrict__ bz, Dims d, double inv_h2,
                                const double* __restrict__ b, const double* __restrict__ p,
                                double* __restrict__ r_out, double* __restrict__ partials)
{
    const long n = (long)d.nx * d.ny * d.nz;
    double acc = 0.0;
    for (long c = (long)blockIdx.x * kBlock + threadIdx.x; c < n; c += (long)gridDim.x * kBlock) {
        int i, j, k;
        cell_of(c, d, i, j, k);
        double dg, of;
        stencil(bx, by, bz, p, d, i, j, k, c, dg, of);
        const double r = b[c] - (of - dg * p[c]) * inv_h2;
        if (r_out) r_out[c] = r;
        acc += r * r;
    }
    acc = block_sum(acc);
    if (threadIdx.x == 0) partials[blockIdx.x] = acc;
}

// One Gauss-Seidel half-sweep over colour `colour` ((i+j+k)&1 == colour):
//   dst_c = (sum beta_f src_nb - h^2 b_c) / sum beta_f
// src holds the other colour (it may alias dst).  With zero_src the other
// colour is taken as 0.  A cell with no coupled face copies its old value.
// Launch: grid (ceil(ceil(nx/2)/64), ceil(ny/4), nz), block (64, 4).
template <typename T, typename I = long>
__device__ inline T half_sweep_value(const T* __restrict__ bx, const T* __restrict__ by, const T* __restrict__ bz,
                                     const Dims d, T h2, const T* __restrict__ b, const T* src, int zero_src, int i,
                                     int j, int k)
{
    const I c = ((I)k * d.ny + j) * d.nx + i;
    T dg, of;
    if (zero_src) {
        dg = 0;
        if (i > 0) dg += bx[fx_at<I>(d, i, j, k)];
        if (i < d.nx - 1) dg += bx[fx_at<I>(d, i + 1, j, k)];
        if (j > 0) dg += by[fy_at<I>(d, i, j, k)];
        if (j < d.ny - 1) dg += by[fy_at<I>(d, i, j + 1, k)];
        if (k > 0) dg += bz[fz_at<I>(d, i, j, k)];
        if (k < d.nz - 1) dg += bz[fz_at<I>(d, i, j, k + 1)];
        of = 0;
    } else {
        stencil<T, T, I>(bx, by, bz, src, d, i, j, k, c, dg, of);
    }
    T v;
    if (dg > (T)0) v = (of - h2 * b[c]) / dg;
    else v = zero_src ? (T)0 : src[c];
    return v;
}

template <typename T>
__device__ inline void half_sweep_cell(const T* __restrict__ bx, const T* __restrict__ by,
                                       const T* __restrict__ bz, const Dims d, T h2, const T* __restrict__ b,
                                       const T* src, T* dst, int zero_src, int i, int j, int k)
{
    dst[((long)k * d.ny + j) * d.nx + i] = half_sweep_value<T>(bx, by, bz, d, h2, b, src, zero_src, i, j, k);
}

template <typename T>
__global__ void k_half_sweep(const T* __restrict__ bx, const T* __restrict__ by, const T* __restrict__ bz,
                             Dims d, T h2, const T* __restrict__ b, const T* src, T* dst, int colour,
                             int zero_src)
{
    const int m = blockIdx.x * 64 + threadIdx.x;
    const int j = blockIdx.y * 4 + threadIdx.y;
    const int k = blockIdx.z;
    if (j >= d.ny) return;
    const int i = 2 * m + ((j + k + colour) & 1);
    if (i >= d.nx) return;
    half_sweep_cell<T>(bx, by, bz, d, h2, b, src, dst, zero_src, i, j, k);
}


// b_coarse = mean over the 8 children of (b - L x) (fine dims f, coarse dims
// cd), the eight children of a coarse cell on eight threads of a block: each
// forms one child's residual, and the first of the eight adds them one after
// another, z, then y, then x (the order of the single-workgroup tail).  The
// levels this serves are small, and one thread per coarse cell working
// through its children in turn left most of the chip idle.  Launch: blocks of
// kBlock threads, any grid.
template <typename T>
__global__ void __launch_bounds__(kBlock)
k_residual_restrict(const T* __restrict__ bx, const T* __restrict__ by, const T* __restrict__ bz, Dims f, Dims cd,
                    T inv_h2, const T* __restrict__ b, const T* __restrict__ x, T* __restrict__ bc)
{
    constexpr int kCells = kBlock / 8;  // coarse cells per block and pass
    __shared__ T rs[kBlock];
    const long n = (long)cd.nx * cd.ny * cd.nz;
    const int t = (int)threadIdx.x, ch = t & 7;
    const int cx = ch & 1, cy = (ch >> 1) & 1, cz = ch >> 2;
    for (long C0 = (long)blockIdx.x * kCells; C0 < n; C0 += (long)gridDim.x * kCells) {
        const long C = C0 + (t >> 3);
        T r = 0;
        if (C < n) {
            int I, J, K;
            cell_of(C, cd, I, J, K);
            const int i = 2 * I + cx, j = 2 * J + cy, k = 2 * K + cz;
            const long c = ((long)k * f.ny + j) * f.nx + i;
            T dg, of;
            stencil<T, T, long>(bx, by, bz, x, f, i, j, k, c, dg, of);
            r = b[c] - (of - dg * x[c]) * inv_h2;
        }
        rs[t] = r;
        __syncthreads();
        if (ch == 0 && C < n) {
            T s = 0;
            for (int q = 0; q < 8; ++q) s += rs[t + q];
            bc[C] = s * (T)0.125;
        }
        __syncthreads();
    }
}

// One axis of the trilinear prolongation: 3/4 of the parent, 1/4 of the
// parent's neighbour on the fine cell's side, rounded once (side / 4 is exact,
// so the explicit fma gives the correctly rounded sum whatever the compiler
// contracts elsewhere).  Every prolongation path uses it, x first, then y, then
// z, so they all give the same values.
template <typename T>
__device__ __forceinline__ T pro_lerp(T parent, T side)
{
    if constexpr (sizeof(T) == 4) return __builtin_fmaf(0.75f, parent, 0.25f * side);
    else return __builtin_fma(0.75, parent, 0.25 * side);
}

// x_fine += trilinear prolongation of the coarse correction e: the value at
// fine cell (i, j, k)
template <typename T, typename IX = long>
__device__ inline T prolong_value_at(const Dims cd, const T* __restrict__ e, int i, int j, int k)
{
    const int I0 = i >> 1, J0 = j >> 1, K0 = k >> 1;
    int I1 = (i & 1) ? I0 + 1 : I0 - 1;
    int J1 = (j & 1) ? J0 + 1 : J0 - 1;
    int K1 = (k & 1) ? K0 + 1 : K0 - 1;
    I1 = I1 < 0 ? 0 : (I1 > cd.nx - 1 ? cd.nx - 1 : I1);
    J1 = J1 < 0 ? 0 : (J1 > cd.ny - 1 ? cd.ny - 1 : J1);
    K1 = K1 < 0 ? 0 : (K1 > cd.nz - 1 ? cd.nz - 1 : K1);
    const IX sy = cd.nx, sz = (IX)cd.nx * cd.ny;
    auto E = [&](int a, int bb, int cc) { return e[(IX)cc * sz + (IX)bb * sy + a]; };
    // x-direction first, then y, then z
    const T e00 = pro_lerp(E(I0, J0, K0), E(I1, J0, K0));
    const T e10 = pro_lerp(E(I0, J1, K0), E(I1, J1, K0));
    const T e01 = pro_lerp(E(I0, J0, K1), E(I1, J0, K1));
    const T e11 = pro_lerp(E(I0, J1, K1), E(I1, J1, K1));
    const T f0 = pro_lerp(e00, e10);
    const T f1 = pro_lerp(e01, e11);
    return pro_lerp(f0, f1);
}

// the same at fine cell index c
template <typename T, typename IX = long>
__device__ inline T prolong_value(const Dims f, const Dims cd, const T* __restrict__ e, IX c)
{
    int i, j, k;
    cell_of(c, f, i, j, k);
    return prolong_value_at<T, IX>(cd, e, i, j, k);
}

template <typename T>
__device__ inline void prolong_cell(const Dims f, const Dims cd, const T* __restrict__ e, T* __restrict__ x, long c)
{
    x[c] += prolong_value<T>(f, cd, e, c);
}

template <typename T>
__global__ void k_prolong_correct(Dims f, Dims cd, const T* __restrict__ e, T* __restrict__ x)
{
    const long n = (long)f.nx * f.ny * f.nz;
    for (long c = (long)blockIdx.x * kBlock + threadIdx.x; c < n; c += (long)gridDim.x * kBlock)
        prolong_cell<T>(f, cd, e, x, c);
}

// Mixed-precision outer step (FP64):
//   q = p + e (e FP32), r = b - L q, r32 = (float) r, partials of ||r||^2.
// q is written to p_out (must not alias p_in).
__global__ void k_outer_update(const double* __restrict__ bx, const double* __restrict__ by,
                               const double* __restrict__ bz, Dims d, double inv_h2,
                               const double* __restrict__ b, const double* __restrict__ p_in,
                               const float* __restrict__ e, int zero_e, double* __restrict__ p_out,
                               float* __restrict__ r32, double* __restrict__ partials)
{
    const long n = (long)d.nx * d.ny * d.nz;
    const long sy = d.nx, sz = (long)d.nx * d.ny;
    double acc = 0.0;
    for (long c = (long)blockIdx.x * kBlock + threadIdx.x; c < n; c += (long)gridDim.x * kBlock) {
        int i, j, k;
        cell_of(c, d, i, j, k);
        auto Q = [&](long t) { return zero_e ? p_in[t] : p_in[t] + (double)e[t]; };
        double dg = 0.0, of = 0.0, f;
        if (i > 0)        { f = bx[fx_index(d, i, j, k)];     dg += f; of += f * Q(c - 1); }
        if (i < d.nx - 1) { f = bx[fx_index(d, i + 1, j, k)]; dg += f; of += f * Q(c + 1); }
        if (j > 0)        { f = by[fy_index(d, i, j, k)];     dg += f; of += f * Q(c - sy); }
        if (j < d.ny - 1) { f = by[fy_index(d, i, j + 1, k)]; dg += f; of += f * Q(c + sy); }
        if (k > 0)        { f = bz[fz_index(d, i, j, k)];     dg += f; of += f * Q(c - sz); }
        if (k < d.nz - 1) { f = bz[fz_index(d, i, j, k + 1)]; dg += f; of += f * Q(c + sz); }
        const double qc = Q(c);
        const double r = b[c] - (of - dg * qc) * inv_h2;
        p_out[c] = qc;
        r32[c] = (float)r;
        acc += r * r;
    }
    acc = block_sum(acc);
    if (threadIdx.x == 0) partials[blockIdx.x] = acc;
}

// ---------------------------------------------------------------------------
// inputs of the solve (contraction off: each product rounds, as written)
// ---------------------------------------------------------------------------

__device__ inline double cell_density(double fd, double ff, double rd, double rf, double rg)
{
#pragma clang fp contract(off)
    double fg = 1.0 - fd - ff;
    fg = fg < 0.0 ? 0.0 : fg;
    return rd * fd + rf * ff + rg * fg;
}

// rho = sum_i rho_i f_i per cell
__global__ void k_density_from_vof(const double* __restrict__ fd, const double* __restrict__ ff, long n,
                                   double rd, double rf, double rg, double* __restrict__ rho)
{
    for (long i = (long)blockIdx.x * kBlock + threadIdx.x; i < n; i += (long)gridDim.x * kBlock)
        rho[i] = cell_density(fd[i], ff[i], rd, rf, rg);
}

__global__ void k_divergence(const double* __restrict__ u, const double* __restrict__ v,
                             const double* __restrict__ w, Dims d, double h, double dt, double* __restrict__ b)
{
#pragma clang fp contract(off)
    const long n = (long)d.nx * d.ny * d.nz;
    for (long c = (long)blockIdx.x * kBlock + threadIdx.x; c < n; c += (long)gridDim.x * kBlock) {
        int i, j, k;
        cell_of(c, d, i, j, k);
        const long fx = ((long)k * d.ny + j) * (d.nx + 1) + i;
        const long fy = ((long)k * (d.ny + 1) + j) * d.nx + i;
        const long fz = c;
        const long sz = (long)d.nx * d.ny;
        const double s = (u[fx + 1] - u[fx]) + (v[fy + d.nx] - v[fy]) + (w[fz + sz] - w[fz]);
        b[c] = s / h / dt;
    }
}

// dL/df_drop and dL/df_film per cell from dL/dbeta on the faces (public
// layouts), gathered over the cell's interior faces:
//   dL/drho_c = sum_f dL/dbeta_f * (-2 / (rho_c + rho_nb)^2)
//   dL/df     = dL/drho_c * (rho_phase - rho_gas), rho_gas dropped where the
//               gas fraction 1 - f_drop - f_film is clamped (negative).
__global__ void k_vof_grad(const double* __restrict__ fd, const double* __restrict__ ff, Dims d, double rd,
                           double rf, double rg, const double* __restrict__ gx, const double* __restrict__ gy,
                           const double* __restrict__ gz, double* __restrict__ g_drop, double* __restrict__ g_film)
{
#pragma clang fp contract(off)
    const long n = (long)d.nx * d.ny * d.nz;
    const long sz = (long)d.nx * d.ny;
    for (long c = (long)blockIdx.x * kBlock + threadIdx.x; c < n; c += (long)gridDim.x * kBlock) {
        int i, j, k;
        cell_of(c, d, i, j, k);
        const double rc = cell_density(fd[c], ff[c], rd, rf, rg);
        const long fx = ((long)k * d.ny + j) * (d.nx + 1) + i;
        const long fy = ((long)k * (d.ny + 1) + j) * d.nx + i;
        double acc = 0.0;
        auto face = [&](long nb, double g) {
            const double s = rc + cell_density(fd[nb], ff[nb], rd, rf, rg);
            acc += g * (-2.0 / (s * s));
        };
        if (i > 0) face(c - 1, gx[fx]);
        if (i < d.nx - 1) face(c + 1, gx[fx + 1]);
        if (j > 0) face(c - d.nx, gy[fy]);
        if (j < d.ny - 1) face(c + d.nx, gy[fy + d.nx]);
        if (k > 0) face(c - sz, gz[c]);
        if (k < d.nz - 1) face(c + sz, gz[c + sz]);
        const double gas = (1.0 - fd[c] - ff[c] < 0.0) ? 0.0 : rg;
        g_drop[c] = acc * (rd - gas);
        g_film[c] = acc * (rf - gas);
    }
}

// dL/drho_c = sum over the cell's interior faces f of dL/dbeta_f * (-2 / (rho_c + rho_nb)^2),
// the derivative of beta_f = 2/(rho_L + rho_R); g in the public face layouts.
__global__ void k_density_grad(const double* __restrict__ rho, Dims d, const double* __restrict__ gx,
                               const double* __restrict__ gy, const double* __restrict__ gz,
                               double* __restrict__ grho)
{
#pragma clang fp contract(off)
    const long n = (long)d.nx * d.ny * d.nz;
    const long sz = (long)d.nx * d.ny;
    for (long c = (long)blockIdx.x * kBlock + threadIdx.x; c < n; c += (long)gridDim.x * kBlock) {
        int i, j, k;
        cell_of(c, d, i, j, k);
        const double rc = rho[c];
        const long fx = ((long)k * d.ny + j) * (d.nx + 1) + i;
        const long fy = ((long)k * (d.ny + 1) + j) * d.nx + i;
        double acc = 0.0;
        auto face = [&](long nb, double g) {
            const double s = rc + rho[nb];
            acc += g * (-2.0 / (s * s));
        };
        if (i > 0) face(c - 1, gx[fx]);
        if (i < d.nx - 1) face(c + 1, gx[fx + 1]);
        if (j > 0) face(c - d.nx, gy[fy]);
        if (j < d.ny - 1) face(c + d.nx, gy[fy + d.nx]);
        if (k > 0) face(c - sz, gz[c]);
        if (k < d.nz - 1) face(c + sz, gz[c + sz]);
        grho[c] = acc;
    }
}

// u_f -= dt * beta_f * (p_R - p_L) / h on interior faces of the public face
// layouts (evaluated left to right, no contraction); one thread per face.
__global__ void k_velocity_correct(const double* __restrict__ bx, const double* __restrict__ by,
                                   const double* __restrict__ bz, const double* __restrict__ p, Dims d, double h,
                                   double dt, double* __restrict__ u, double* __restrict__ v, double* __restrict__ w)
{
#pragma clang fp contract(off)
    const long nfx = (long)d.nz * d.ny * (d.nx + 1);
    const long nfy = (long)d.nz * (d.ny + 1) * d.nx;
    const long nfz = (long)(d.nz + 1) * d.ny * d.nx;
    const long sz = (long)d.nx * d.ny;
    for (long f = (long)blockIdx.x * kBlock + threadIdx.x; f < nfx + nfy + nfz; f += (long)gridDim.x * kBlock) {
        if (f < nfx) {
            const int i = (int)(f % (d.nx + 1));
            const long row = f / (d.nx + 1);
            if (i == 0 || i == d.nx) continue;
            const long c = row * d.nx + i;
            u[f] = u[f] - dt * bx[f] * (p[c] - p[c - 1]) / h;
        } else if (f < nfx + nfy) {
            const long g = f - nfx;
            const int i = (int)(g % d.nx);
            const long r = g / d.nx;
            const int j = (int)(r % (d.ny + 1));
            const long k = r / (d.ny + 1);
            if (j == 0 || j == d.ny) continue;
            const long c = (k * d.ny + j) * d.nx + i;
            v[g] = v[g] - dt * by[g] * (p[c] - p[c - d.nx]) / h;
        } else {
            const long g = f - nfx - nfy;
            const long k = g / sz;
            if (k == 0 || k == d.nz) continue;
            w[g] = w[g] - dt * bz[g] * (p[g] - p[g - sz]) / h;
        }
    }
}

}  // namespace mgp
