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
// per-axis rounding bounds of the two float32 coordinates (ndim values);
// xy_mag > 0 (ndim 2 or 3): the float32 sweep expands x and y as |a|^2 +
// |b|^2 - 2 a.b, with xy_mag = xy_expand_mag of the coordinates' maxima
int fp32_bands_axes(const double *edges_sq, int nedges, int ndim, const double *axis_eps,
                    double scale, float *lo, float *hi, double xy_mag = 0.0);
// magnitude term of the expanded x and y of squared r (ndim 3) or rp (ndim
// 2): a_max = the lane's largest |x|, |y| in the j column's frame, b_max = the
// j point's
double xy_expand_mag(const double a_max[2], const double b_max[2], int ndim);
// per-pair narrowing of the expanded r (ndim 3) and rp (ndim 2) bands in
// coordinates scaled by fscale: a pair whose own magnitude term is m (scaled) may take its band
// narrowed by K (M - m) on each side; both constants rounded down
void xy_pair_margin(double xy_mag, double fscale, float *K, float *M);
// rounding bound of one column-local axis: coordinates at most a_max and
// b_max from the frame origin, each rounded once from binary64
double frame_eps(double a_max, double b_max, double scale);
// `priv`: size the lookup table for the private-histogram (batched) sweep
// (axis_eps and xy_mag, when given: the sweep's own top band also fits)
int fp32_scale(int metric, const double *edges, int nb, double coord_scale, bool priv,
               const double *axis_eps, double xy_mag, double *c);
// axis_eps (optional, x y z): per-axis rounding bounds (else box-frame 6 u S);
// fscale: the float32 coordinate scale (bands are moved into it)
int build_bins(int metric, bool fp32, const double *edges, int nb, double pimax, int npi,
               double coord_scale, const double *axis_eps, double fscale, bool priv,
               double xy_mag, HostBins *out);

}  // namespace pc
