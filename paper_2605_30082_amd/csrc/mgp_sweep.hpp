// Red-black Gauss-Seidel sweep launchers.
#pragma once

#include "mgp_kernels.hpp"

namespace mgp {

// Algorithmic HBM bytes of one full sweep per cell: read p, b and the three
// low-face coefficients, write p.
template <typename T>
constexpr double sweep_bytes_per_cell()
{
    return 6.0 * sizeof(T);
}

// One full sweep: out = GS(in) with colour order (red, black) for order 0 and
// (black, red) for order 1; `in` is only read (treated as 0 with zero_in).
template <typename T>
hipError_t launch_sweep(const T* bx, const T* by, const T* bz, Dims d, T h2, const T* b, const T* in, T* out,
                        int order, bool zero_in, hipStream_t s)
{
    const int c0 = order == 0 ? 0 : 1;
    const dim3 blk(64, 4, 1);
    const dim3 grd((unsigned)(((d.nx + 1) / 2 + 63) / 64), (unsigned)((d.ny + 3) / 4), (unsigned)d.nz);
    k_half_sweep<T><<<grd, blk, 0, s>>>(bx, by, bz, d, h2, b, in, out, c0, zero_in ? 1 : 0);
    k_half_sweep<T><<<grd, blk, 0, s>>>(bx, by, bz, d, h2, b, out, out, 1 - c0, 0);
    return hipGetLastError();
}

}  // namespace mgp
