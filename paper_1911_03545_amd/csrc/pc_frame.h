// pc_frame.h -- the column-local float32 frames shared by the gridding and
// the pair sweep (device code only).
//
// On 3-D grids the float32 x and y coordinates of a point are stored relative
// to the centre of its own column, z relative to the domain origin, all
// scaled by g.fscale:
//     X = fl32((x - cx) * s),  Y = fl32((y - cy) * s),  Z = fl32((z - lo_z) * s).
// The sweep places the i point of a work item in the frame of the item's j
// column (plus the item's periodic offset), so a float32 difference carries
// rounding errors proportional to the column width instead of the box size.
#pragma once
#include <hip/hip_runtime.h>

#include "pc_common.h"

namespace pc {

// Centre of column index k along axis a (0: x, 1: y): lo + (k + 1/2) width,
// every operation rounded once (no contraction), so that the gridding and the
// sweep compute the same value.
__device__ __forceinline__ double col_centre(double lo, double width, int k)
{
    return __dadd_rn(lo, __dmul_rn(__dadd_rn((double)k, 0.5), width));
}

// Column (ix, iy) of a cell id (cells of catalogue c are c * ncell ..).
__device__ __forceinline__ void cell_column(int cell, int nx, int ny, int nz, int *ix, int *iy)
{
    const int lcol = (cell / nz) % (nx * ny);
    *ix = lcol / ny;
    *iy = lcol % ny;
}

}  // namespace pc
