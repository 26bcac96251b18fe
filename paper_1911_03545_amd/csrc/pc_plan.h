// pc_plan.h -- host planner interface (grid, bands, bin description).
#pragma once
#include <stddef.h>

#include <vector>

#include "pc_common.h"

namespace pc {

struct HostBins {
    pc_bins hdr;
    pc_bins_layout lay;
    std::vector<char> buf;   // pc_bins and its band arrays, ready to upload
    size_t upload = 0;       // bytes of buf; the table (lay.tbl ..) is built on the device
    int ne = 0;              // r / rp edges
    int nq = 0;              // pi edges (1 when unused)
};

int plan_grid(const double lo[3], const double hi[3], double boxsize, double reach_xy,
              double reach_z, int slices_per_reach, pc_grid *g, int xy_refine = 1,
              bool zball = false);
// angular grid of unit vectors (overrides n, ncell, zreach and the slice
// fields of a grid planned on the vectors' bounding box)
int plan_sky_grid(double chord_reach, double zlo, double zhi, int slices, int ra_refine,
                  pc_grid *g, std::vector<pc_band> *bands);
int fp32_bands(const double *edges_sq, int nedges, int ndim, double scale, float *lo,
               float *hi);
// per-axis rounding bounds of the two float32 coordinates (ndim values)
int fp32_bands_axes(const double *edges_sq, int nedges, int ndim, const double *axis_eps,
                    double scale, float *lo, float *hi);
// rounding bound of one column-local axis: coordinates at most a_max and
// b_max from the frame origin, each rounded once from binary64
double frame_eps(double a_max, double b_max, double scale);
// `priv`: size the lookup table for the private-histogram (batched) sweep
int fp32_scale(int metric, const double *edges, int nb, double coord_scale, bool priv,
               double *c);
// axis_eps (optional, x y z): per-axis rounding bounds (else box-frame 6 u S);
// fscale: the float32 coordinate scale (bands are moved into it)
int build_bins(int metric, bool fp32, const double *edges, int nb, double pimax, int npi,
               double coord_scale, const double *axis_eps, double fscale, bool priv,
               HostBins *out);

}  // namespace pc
