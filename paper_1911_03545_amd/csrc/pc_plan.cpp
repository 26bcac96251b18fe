// pc_plan.cpp -- host-side planning: cell grid, float32 decision bands and the
// bin lookup table.  No device work happens here.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "../../include/paircount.h"
#include "pc_common.h"
#include "pc_fixed.h"
#include "pc_plan.h"

namespace pc {

namespace {

const double kU32 = 0x1p-24;   // float32 unit roundoff
const double kU64 = 0x1p-53;   // binary64 unit roundoff
const double kSafety = 1.25;   // multiplies every derived bound

float float_down(double v)
{
    float f = (float)v;
    if ((double)f > v)
        f = nextafterf(f, -INFINITY);
    return f;
}

float float_up(double v)
{
    float f = (float)v;
    if ((double)f < v)
        f = nextafterf(f, INFINITY);
    return f;
}

uint32_t fbits(float f)
{
    uint32_t u;
    memcpy(&u, &f, 4);
    return u;
}

float bits_f(uint32_t u)
{
    float f;
    memcpy(&f, &u, 4);
    return f;
}

}  // namespace

int plan_grid_k(const double lo_in[3], const double hi_in[3], double boxsize,
                double reach_xy, double reach_z, int slices_per_reach,
                pc_grid *g, int k, bool zball);

// Cell grid of section "Partitioning the particles on a grid".
//
// Transverse columns (x, y) are at least `reach_xy` wide, so two points within
// the reach are at most one column apart (the 27/9-neighbour argument).  The
// width carries a relative margin of 2^-28 plus 2^-40 of the extent: cell
// assignment t = fl(fl(x - lo) * fl(n / extent)) is monotone in x and its
// rounding moves a cell boundary by far less than that margin, so two points
// two columns apart are always separated by more than the reach.  The plain
// rule n = floor(extent / reach) of the paper gives a width exactly equal to
// the reach when the ratio is an integer, where rounding could hide a pair.
//
// Along z (the line of sight) the grid is finer: slices of about
// reach_z / slices_per_reach, of which `zreach` are searched on each side of a
// block.  zreach = floor(reach_z / width_z (1 + 2^-28) + 2^-28) + 1 covers
// every point within reach_z of any point of the block.
//
// With xy_refine = k > 1 ("Sub-dividing the cells") the columns are at least
// reach_xy / k wide and a block pairs with the (2k + 1)^2 columns around its
// own; a periodic axis needs 2k + 1 columns, else k is lowered.  When the
// reach is a 3-D ball (`zball`: r, angular chords, on-sky pairs) the z window
// of a column at offset (ox, oy) shrinks to sqrt(reach^2 - d^2), d the
// smallest transverse distance between the two columns ((|o| - 1) column
// widths per axis, less a margin of 2^-30 of the extent); columns no pair can
// reach are skipped.
int plan_grid(const double lo_in[3], const double hi_in[3], double boxsize,
              double reach_xy, double reach_z, int slices_per_reach,
              pc_grid *g, int xy_refine, bool zball)
{
    int k = std::min(std::max(xy_refine, 1), PC_MAX_XYK);
    for (;; k--) {
        const int rc = plan_grid_k(lo_in, hi_in, boxsize, reach_xy, reach_z, slices_per_reach,
                                   g, k, zball);
        if (rc != CF_EUNSUPPORTED || k == 1)
            return rc;
    }
}

int plan_grid_k(const double lo_in[3], const double hi_in[3], double boxsize,
                double reach_xy, double reach_z, int slices_per_reach,
                pc_grid *g, int k, bool zball)
{
    memset(g, 0, sizeof(*g));
    g->fscale = 1.0;
    g->zq_inv = 0.0;
    if (!(reach_xy > 0.0) || !(reach_z > 0.0) || !isfinite(reach_xy) ||
        !isfinite(reach_z))
        return CF_EINVAL;
    if (slices_per_reach <= 0)
        slices_per_reach = 16;
    const bool periodic = boxsize > 0.0;
    if (std::isnan(boxsize) || (periodic && !isfinite(boxsize)))
        return CF_EINVAL;
    g->periodic = periodic ? 1 : 0;
    g->boxsize = periodic ? boxsize : 0.0;
    for (int a = 0; a < 3; a++) {
        if (periodic) {
            g->lo[a] = 0.0;
            g->extent[a] = boxsize;
        } else {
            if (!isfinite(lo_in[a]) || !isfinite(hi_in[a]) || hi_in[a] < lo_in[a])
                return CF_EINVAL;
            g->lo[a] = lo_in[a];
            g->extent[a] = hi_in[a] - lo_in[a];
        }
    }
    const int max_cols = 1024;
    for (int a = 0; a < 2; a++) {
        const double ext = g->extent[a];
        const double need = reach_xy / k * (1.0 + 0x1p-28) + ext * 0x1p-40;
        double nd = ext > 0.0 ? floor(ext / need) : 1.0;
        int n = (int)std::min(std::max(nd, 1.0), (double)max_cols);
        while (n > 1 && ext / n < need)
            n--;
        if (periodic && n < 2 * k + 1)
            return CF_EUNSUPPORTED;
        g->n[a] = n;
        g->inv_w[a] = ext > 0.0 ? (double)n / ext : 0.0;
        g->width[a] = ext / n;
    }
    {
        const double ext = g->extent[2];
        if (periodic && !(3.0 * reach_z * (1.0 + 0x1p-28) <= ext))
            return CF_EUNSUPPORTED;
        const double target = reach_z / slices_per_reach;
        double nd = ext > 0.0 ? floor(ext / target) : 1.0;
        const double max_slices = 4096.0;
        int n = (int)std::min(std::max(nd, 1.0), max_slices);
        // keep the total cell count modest
        const int64_t ncol = (int64_t)g->n[0] * g->n[1];
        while (n > 1 && ncol * n > (int64_t(1) << 26))
            n = (n + 1) / 2;
        g->n[2] = n;
        g->inv_w[2] = ext > 0.0 ? (double)n / ext : 0.0;
        g->width[2] = ext / n;
        const double r = reach_z * g->inv_w[2];
        int zr = (int)floor(r * (1.0 + 0x1p-28) + 0x1p-28) + 1;
        g->zreach = std::min(zr, n);
    }
    g->ncell = (int64_t)g->n[0] * g->n[1] * g->n[2];
    g->xyk = k;
    for (int a = 0; a <= PC_MAX_XYK; a++)
        for (int b = 0; b <= PC_MAX_XYK; b++) {
            const double dx = std::max(0.0, (a - 1) * g->width[0] - g->extent[0] * 0x1p-30);
            const double dy = std::max(0.0, (b - 1) * g->width[1] - g->extent[1] * 0x1p-30);
            const double d2 = dx * dx + dy * dy;
            int zr = g->zreach;
            if (a > k || b > k || d2 >= reach_xy * reach_xy * (1.0 + 0x1p-30)) {
                zr = -1;
            } else if (zball && d2 > 0.0) {
                const double rz = sqrt(std::max(0.0, reach_z * reach_z * (1.0 + 0x1p-30) - d2));
                const double r = rz * g->inv_w[2];
                zr = std::min((int)floor(r * (1.0 + 0x1p-28) + 0x1p-28) + 1, g->zreach);
            }
            g->zro[a][b] = (int16_t)zr;
        }
    return CF_OK;
}

// Angular grid of section "Partitioning the particles on a grid: angular
// correlation functions": declination bands at least one angular reach high
// (two points further apart in declination are further apart on the sky), each
// split into right-ascension cells whose reach follows from the haversine
// relation (the section's angular-distance equation): for two points in
// bands b, b' whose cos(dec) is at least c_b, c_b', sin(dRA / 2) <=
// sin(theta / 2) / sqrt(c_b c_b').  With c_b = c_b' this is the paper's
// right-ascension binning equation; the product form is tighter across bands.
// Cells are 1 / ra_refine of the band's own reach wide ("Sub-dividing the
// cells").  Inside a band, `slices` declination slices give the window search.
//
// Inputs are unit vectors whose squared norm is within 2^-20 of 1 (the
// gridding kernel checks it), so their directions are within 2^-20 of the
// vectors and a chord below `chord_reach` between vectors means an angle
// below 2 asin((chord_reach + 2^-19) / 2) between directions.  Every derived
// reach carries a relative margin of 2^-20 and an absolute one of 2^-40
// radians, far above the rounding of the device's atan2 and of the cell
// arithmetic.  zlo, zhi bound the z components (declination range).
int plan_sky_grid(double chord_reach, double zlo, double zhi, int slices, int ra_refine,
                  pc_grid *g, std::vector<pc_band> *bands)
{
    if (!(chord_reach > 0.0) || !isfinite(chord_reach) || !isfinite(zlo) || !isfinite(zhi) ||
        zhi < zlo)
        return CF_EINVAL;
    if (slices <= 0)
        slices = 16;
    slices = std::min(slices, 4096);
    if (ra_refine <= 0)
        ra_refine = 1;
    const double cc = chord_reach * (1.0 + 0x1p-40) + 0x1p-19;
    const double theta = (cc >= 2.0 ? M_PI : 2.0 * asin(0.5 * cc)) * (1.0 + 0x1p-20) + 0x1p-40;
    // bands are a little higher than the reach, so that a declination window
    // of the reach never spans more than the neighbouring band
    const double hmin = theta * (1.0 + 0x1p-20);
    const double za = std::max(-1.0, zlo - 0x1p-18), zb = std::min(1.0, zhi + 0x1p-18);
    const double dlo = std::max(-M_PI_2, asin(za) - 0x1p-30);
    const double dhi = std::min(M_PI_2, asin(zb) + 0x1p-30);
    const double span = dhi - dlo;
    int nb = (int)std::min(std::max(floor(span / hmin), 1.0), (double)PC_MAX_BANDS);
    while (nb > 1 && span / nb < hmin)
        nb--;
    const double h = std::max(span / nb, hmin);

    // lower bound of cos(dec) over each band (its edge furthest from the
    // equator, widened by the margin)
    std::vector<double> cmin(nb);
    for (int b = 0; b < nb; b++) {
        const double d0 = dlo + b * h, d1 = dlo + (b + 1) * h;
        const double m = std::min(M_PI_2, std::max(fabs(d0), fabs(d1)) + 0x1p-30);
        cmin[b] = std::max(0.0, cos(m));
    }
    const double s2 = sin(0.5 * std::min(theta, M_PI));
    auto reach_ra = [&](int b, int b2) {
        if (b2 < 0 || b2 >= nb)
            return 8.0;
        const double den = sqrt(cmin[b] * cmin[b2]);
        if (!(den > 0.0) || s2 >= den)
            return 8.0;
        const double d = 2.0 * asin(s2 / den) * (1.0 + 0x1p-20) + 0x1p-40;
        return d >= M_PI ? 8.0 : d;
    };
    bands->assign(nb, pc_band{});
    std::vector<int> nra(nb);
    for (int b = 0; b < nb; b++) {
        const double d = reach_ra(b, b);
        const double want = d >= M_PI ? 1.0 : floor(2.0 * M_PI * ra_refine / d);
        nra[b] = (int)std::min(std::max(want, 1.0), (double)PC_MAX_RA);
    }
    // keep the column count bounded (coarser cells stay correct)
    auto total = [&]() {
        int64_t t = 0;
        for (int b = 0; b < nb; b++)
            t += nra[b];
        return t;
    };
    while (total() > PC_MAX_SKY_COLS)
        for (int b = 0; b < nb; b++)
            nra[b] = std::max(1, nra[b] / 2);
    const int64_t ncol = total();
    while (slices > 1 && ncol * slices > (int64_t(1) << 26))
        slices = (slices + 1) / 2;
    int32_t col0 = 0;
    for (int b = 0; b < nb; b++) {
        pc_band &B = (*bands)[b];
        B.col0 = col0;
        B.nra = nra[b];
        B.ra_scale = nra[b] / (2.0 * M_PI);
        for (int d = 0; d < 3; d++)
            B.dra[d] = reach_ra(b, b - 1 + d);
        col0 += nra[b];
    }
    g->n[0] = 1;
    g->n[1] = (int32_t)ncol;
    g->n[2] = slices;
    g->ncell = ncol * slices;
    g->nband = nb;
    g->dec_lo = dlo;
    g->inv_hs = slices / h;
    g->inv_w[0] = 0.0;
    g->inv_w[1] = 0.0;
    g->inv_w[2] = g->inv_hs;
    g->width[0] = h;
    g->width[1] = 0.0;
    g->sky_reach = theta;
    g->width[2] = h / slices;
    const double r = theta * g->inv_hs;
    const int zr = (int)floor(r * (1.0 + 0x1p-28) + 0x1p-28) + 1;
    g->zreach = std::min(zr, slices);
    g->bands = nullptr;
    g->xyk = 1;
    for (int a = 0; a <= PC_MAX_XYK; a++)
        for (int b = 0; b <= PC_MAX_XYK; b++)
            g->zro[a][b] = (int16_t)g->zreach;
    return CF_OK;
}

// Float32 decision bands.  The float32 sweep evaluates, per axis, the float32
// difference d32 = fl32(A - X_j) of two float32 coordinates whose rounding
// errors (from the binary64 values, and any offset added on the way) sum to
// at most eps_a, and then s32 with one multiply and fused multiply-adds.
// With u = 2^-24 and U = 2^-53:
//   |d32 - d| <= dl_a = eps_a (1 + u) + u (|d| + eps_a) + 2 U S
// for the exact wrapped difference d (S bounds every coordinate and periodic
// offset; the 2 U S term covers the binary64 differences).  Summing ndim
// squares (Cauchy-Schwarz on the cross terms),
//   |s32 - s| <= 2 sqrt(s) sqrt(sum dl_a^2) + sum dl_a^2 + (ndim + 1) u s'
// and the binary64 definition differs from the exact s by at most
// (ndim + 1) U s'.  The band of edge E is [E - B(E), E + B(E)] rounded
// outward to float32, with B the sum of both bounds times kSafety.  Because
// B grows slower than s, a float32 value below the band proves s64 < E and
// one above proves s64 > E.
//
// Expanded x and y (xy_mag > 0): the sweep forms
//   t0 = fl(dz dz + Bj), t1 = fl(-2 a_x b_x + t0), t2 = fl(-2 a_y b_y + t1),
//   s32 = fl(t2 + A)
// with Bj = fl(b_y b_y + fl(b_x b_x)) stored per point and A = fl(a_y a_y +
// fl(a_x a_x)) per lane (-2 a is exact), whose exact value at the rounded
// coordinates is the same sum of squared differences.  With
// |Bj - |b|^2| <= 2u |b|^2, |A - |a|^2| <= 2u |a|^2, |dz^2 - dz*^2| <= 2u s',
// |t0| <= s' + |b|^2, |t1| <= |t0| + 2|a_x b_x|, |t2| <= |t1| + 2|a_y b_y|
// (to first order), the arithmetic part of the bound becomes
//   u (6 s' + 5 |b|^2 + 2 |a|^2 + 4 (|a_x b_x| + |a_y b_y|)) (1 + 2^-20),
// the magnitudes taken at their maxima (xy_mag, xy_expand_mag) in place of
// (ndim + 1) u s'; the coordinate part stays as above (it also covers the
// rounding of x and y differences, which the expanded form does not make).
// rp^2 (ndim 2) is formed as t0 = fl(A + Bj), t1 = fl(-2 a_x b_x + t0), s32 =
// fl(-2 a_y b_y + t1) (each instruction then reads one scalar operand), with
// |t0| <= |a|^2 + |b|^2 and |t1| <= |t0| + 2|a_x b_x|: the arithmetic part is
// u (s' + 4 |a|^2 + 4 |b|^2 + 2 |a_x b_x|) to first order, within
// u (6 s' + xy_mag) for xy_mag = 4 |a|^2 + 4 |b|^2 + 2 (|a_x b_x| + |a_y b_y|).
double xy_expand_mag(const double a_max[2], const double b_max[2], int ndim)
{
    const double g = 1.0 + 0x1p-16;   // points a rounding outside their column
    const double ax = a_max[0] * g, ay = a_max[1] * g, bx = b_max[0] * g, by = b_max[1] * g;
    const double A = ax * ax + ay * ay, B = bx * bx + by * by, P = ax * bx + ay * by;
    return ndim == 2 ? 4.0 * A + 4.0 * B + 2.0 * P : 5.0 * B + 2.0 * A + 4.0 * P;
}

// The bound above holds for each pair with its own magnitudes, m = 5 |b|^2
// + 2 |a|^2 + 4 (|a_x b_x| + |a_y b_y|) (rp: 4 |a|^2 + 4 |b|^2 + 2 (|a_x b_x|
// + |a_y b_y|)), in place of xy_mag; every band
// holds kSafety u (1 + 2^-20) xy_mag of it, so a pair may narrow both sides
// of its band by kSafety u (1 + 2^-20) (xy_mag - m).  In the scaled
// coordinates the band (scaled by c^2 and rounded outward) narrows by K (M -
// m) with M = c^2 xy_mag, m from the float32 |a|^2 and |b|^2 the sweep holds
// (each within 2u of the exact value) and |a_x b_x| + |a_y b_y| <= |a| |b|.
void xy_pair_margin(double xy_mag, double fscale, float *K, float *M)
{
    *K = float_down(kSafety * kU32 * (1.0 + 0x1p-20) * (1.0 - 0x1p-40));
    *M = float_down(xy_mag * fscale * fscale * (1.0 - 0x1p-40));
}

int fp32_bands_axes(const double *edges_sq, int nedges, int ndim, const double *axis_eps,
                    double scale, float *lo, float *hi, double xy_mag)
{
    if (!(xy_mag >= 0.0) || !isfinite(xy_mag) || (xy_mag > 0.0 && ndim < 2))
        return CF_EINVAL;
    if (nedges < 1 || ndim < 1 || ndim > 3 || !(scale >= 0.0) || !isfinite(scale))
        return CF_EINVAL;
    double eps[3];
    for (int a = 0; a < ndim; a++) {
        if (!(axis_eps[a] >= 0.0) || !isfinite(axis_eps[a]))
            return CF_EINVAL;
        eps[a] = axis_eps[a];
    }
    const double d64 = 2.0 * kU64 * scale;
    for (int k = 0; k < nedges; k++) {
        const double E = edges_sq[k];
        if (!isfinite(E) || E < 0.0 || E > 1e30)
            return CF_EINVAL;
        if (E == 0.0) {
            lo[k] = -1.0f;
            hi[k] = -1.0f;
            continue;
        }
        double B;
        if (ndim == 1) {
            // an unsquared line-of-sight edge compared with |dz|
            B = eps[0] * (1.0 + kU32) + kU32 * (E + eps[0]) + d64;
        } else {
            const double r = sqrt(E);
            double sum2 = 0.0;
            for (int a = 0; a < ndim; a++) {
                const double dl = eps[a] * (1.0 + kU32) + kU32 * (r + eps[a]) + d64;
                sum2 += dl * dl;
            }
            const double s_hi = E + 2.0 * r * sqrt(sum2) + sum2;
            const double arith = xy_mag > 0.0
                                     ? kU32 * (6.0 * s_hi + xy_mag) * (1.0 + 0x1p-20)
                                     : (ndim + 1) * kU32 * s_hi;
            B = 2.0 * r * sqrt(sum2) + sum2 + arith + (ndim + 1) * kU64 * s_hi;
        }
        B = B * kSafety + 1e-300;
        lo[k] = float_down(E - B);
        hi[k] = float_up(E + B);
    }
    return CF_OK;
}

// Box-frame coordinates (every axis): X = fl32(x - lo), the lane's A =
// fl32(X_i + fl32(D)) and the difference: eps = 6 u S covers the roundings
// of X_i, X_j, D and A.
int fp32_bands(const double *edges_sq, int nedges, int ndim, double scale, float *lo,
               float *hi)
{
    const double e = 6.0 * kU32 * scale;
    const double e3[3] = {e, e, e};
    return fp32_bands_axes(edges_sq, nedges, ndim, e3, scale, lo, hi);
}

// Rounding bound of one axis of the column-local frames (pc_frame.h): the
// lane's coordinate (i point plus offset, in the frame of the j column, at
// most `a_max` from its origin) and the j coordinate (at most `b_max`) are
// each rounded once from binary64 values, so their errors sum to at most
// u (a_max + b_max), plus the binary64 roundings of forming them (a few U
// times the box scale); a relative 2^-20 covers points a rounding outside
// their column.
double frame_eps(double a_max, double b_max, double scale)
{
    return kU32 * (a_max + b_max) * (1.0 + 0x1p-20) + 8.0 * kU64 * scale;
}

// Binary64 path: the float32 value fl32(s64) is compared against the edge
// rounded down and up; only values inside [down, up] need the exact compare.
static void fp64_bands(const double *edges_sq, int nedges, float *lo, float *hi)
{
    for (int k = 0; k < nedges; k++) {
        const double E = edges_sq[k];
        if (E == 0.0) {
            lo[k] = -1.0f;
            hi[k] = -1.0f;
        } else {
            lo[k] = float_down(E);
            hi[k] = float_up(E);
        }
    }
}

// Cells of a lookup table: byte entries up to 125 bins, else 16-bit entries,
// each filling the same LDS space (a smaller one for the private-histogram
// sweep of batched calls).
static int table_cells(int nb, bool priv)
{
    if (priv)
        return nb > PC_TBL8_MAX_BINS ? PC_TBL_PRIV_BYTES / 2 : PC_TBL_PRIV_BYTES;
    return nb > PC_TBL8_MAX_BINS ? PC_TBL16_MAX : PC_TBL8_MAX;
}

// The float32 path of the shared-histogram sweeps with byte entries keys its
// table by rounding: key = round(min(s, 1) * 32767) (one instruction), over
// PC_TBL_PK_CELLS cells; the private-histogram and 16-bit tables keep the
// linear key floor(min(s, cells - 1)).
static bool rounding_key(int nb, bool priv) { return !priv && nb <= PC_TBL8_MAX_BINS; }

// The largest scaled value the float32 key keeps apart from "above every
// edge": below the last cell of either key.
static double key_top(int nb, bool priv)
{
    return rounding_key(nb, priv) ? 32766.0 / 32767.0 : (double)(table_cells(nb, priv) - 1);
}

// Table geometry of the binary64 path: key = sat(bits(s) - base) >> sh over
// float bit patterns (monotone for s >= 0).  The table starts one cell below
// the first band that matters, so every value below it shares cell 0; `sh`
// is the smallest shift that fits [base, s_top] into `cap` cells, plus one
// extra last cell "above every edge" for clamped keys.
static void log_table_geometry(const float *lo, const float *hi, int nedges, float s_top,
                               uint32_t cap, uint32_t *n_out, int *shift, uint32_t *base_out)
{
    const uint32_t top = fbits(std::max(s_top, 0.0f));
    // first band that is not the empty band of a zero edge
    uint32_t first = top;
    for (int k = 0; k < nedges; k++)
        if (hi[k] >= 0.0f) {
            first = fbits(std::max(lo[k], 0.0f));
            break;
        }
    int sh = 0;
    uint32_t base = 0;
    for (;; sh++) {
        const uint32_t step = 1u << sh;
        base = first > step ? first - step : 0u;
        if (((top - base) >> sh) + 2 <= cap)
            break;
    }
    *n_out = ((top - base) >> sh) + 2;
    *shift = sh;
    *base_out = base;
}

static size_t align8(size_t v) { return (v + 7) & ~(size_t)7; }

// Pack pc_bins and its arrays for one call.  `edges` are linear (r, rp or
// chord) edges, squared here as fl(e * e).  For rppi the pi edges are
// q_p = p * fl(pimax / npi) (p < npi) and q_npi = pimax.
// Scale c of the float32 path's coordinates (every float32 coordinate is
// fl32(c (x - origin))).  c puts the top band just below the key's top
// (key_top: cells - 1 for the linear key, just below 1 for the rounding
// key), so that nearly every value above the top band -- most candidate
// pairs -- lands in the one last cell: its table reads are then a broadcast
// of a single LDS address.  c need not be a power of two: every float32
// coordinate is rounded once from its binary64 scaled value either way, and
// the decision bands are scaled by c^2 and rounded outward.
int fp32_scale(int metric, const double *edges, int nb, double coord_scale, bool priv,
               const double *axis_eps, double xy_mag, double *c_out)
{
    const double E = edges[nb] * edges[nb];
    float lo, hi;
    const int ndim = (metric == PC_METRIC_RPPI) ? 2 : 3;
    int rc = fp32_bands(&E, 1, ndim, coord_scale, &lo, &hi);
    if (rc)
        return rc;
    if (axis_eps) {
        // the top band the sweep will use, when it is the wider one
        float lo2, hi2;
        if ((rc = fp32_bands_axes(&E, 1, ndim, axis_eps, coord_scale, &lo2, &hi2, xy_mag)))
            return rc;
        hi = std::max(hi, hi2);
    }
    if (!(hi > 0.0f) || !std::isfinite(hi))
        return CF_EINVAL;
    double c = std::sqrt(key_top(nb, priv) * (1.0 - 0x1p-16) / (double)hi);
    // keep every scaled coordinate and offset a normal float32 of moderate size
    while (c > 0x1p-60 && (2.0 * coord_scale + 1.0) * c > 0x1p100)
        c *= 0.5;
    if (!(c > 0.0) || !std::isfinite(c))
        return CF_EINVAL;
    *c_out = c;
    return CF_OK;
}

int build_bins(int metric, bool fp32, const double *edges, int nb, double pimax,
               int npi, double coord_scale, const double *axis_eps, double fscale, bool priv,
               double xy_mag, HostBins *out)
{
    if (!fp32)
        fscale = 1.0;
    if (nb < 1 || nb + 1 > PC_MAX_EDGES)
        return CF_EINVAL;
    if (metric == PC_METRIC_RPPI) {
        if (npi < 1 || npi > PC_MAX_NPI || !(pimax > 0.0) || !isfinite(pimax))
            return CF_EINVAL;
    } else {
        npi = 1;
    }
    if ((int64_t)nb * npi > PC_MAX_BINS_TOTAL)
        return CF_EINVAL;
    const int ne = nb + 1;
    std::vector<double> E(ne);
    for (int k = 0; k < ne; k++)
        E[k] = edges[k] * edges[k];
    std::vector<float> lo(ne), hi(ne);
    int rc;
    const int ndim = (metric == PC_METRIC_RPPI) ? 2 : 3;
    if (fp32) {
        const double e = 6.0 * kU32 * coord_scale;
        const double e3[3] = {e, e, e};
        rc = fp32_bands_axes(E.data(), ne, ndim, axis_eps ? axis_eps : e3, coord_scale,
                             lo.data(), hi.data(), axis_eps ? xy_mag : 0.0);
        if (rc)
            return rc;
    } else {
        fp64_bands(E.data(), ne, lo.data(), hi.data());
    }
    const int nq = (metric == PC_METRIC_RPPI) ? npi + 1 : 1;
    std::vector<double> q(nq, 0.0);
    std::vector<float> plo(nq, -1.0f), phi(nq, -1.0f);
    if (metric == PC_METRIC_RPPI) {
        const double dpi = pimax / (double)npi;
        for (int p = 0; p < npi; p++)
            q[p] = (double)p * dpi;
        q[npi] = pimax;
        for (int p = 0; p < npi; p++)
            if (!(q[p] < q[p + 1]))
                return CF_EINVAL;
        if (fp32) {
            rc = fp32_bands(q.data(), nq, 1, coord_scale, plo.data(), phi.data());
            if (rc)
                return rc;
        } else {
            fp64_bands(q.data(), nq, plo.data(), phi.data());
        }
    }
    // float32 path: move the float bands into the scaled coordinates (c^2
    // for squared separations, c for the line of sight), rounded outward
    if (fp32) {
        const double c2 = fscale * fscale;
        for (int k = 0; k < ne; k++) {
            if (hi[k] < 0.0f)   // the empty band of a zero edge
                continue;
            lo[k] = float_down((double)lo[k] * c2);
            hi[k] = float_up((double)hi[k] * c2);
            if (!std::isfinite(lo[k]) || !std::isfinite(hi[k]) ||
                std::fpclassify(lo[k]) == FP_SUBNORMAL || std::fpclassify(hi[k]) == FP_SUBNORMAL)
                return CF_EINVAL;
        }
        for (int p = 0; p < nq; p++) {
            if (phi[p] < 0.0f)
                continue;
            plo[p] = float_down((double)plo[p] * fscale);
            phi[p] = float_up((double)phi[p] * fscale);
        }
        // bottoms and tops that never decrease (a band only ever widens,
        // which sends more values to the binary64 recheck): the sweep then
        // finds the band of a value by a binary search over the tops
        for (int k = ne - 2; k >= 0; k--)
            lo[k] = std::min(lo[k], lo[k + 1]);
        for (int k = 1; k < ne; k++)
            hi[k] = std::max(hi[k], hi[k - 1]);
    }
    int shift = 0;
    uint32_t base = 0, tbl_n = 0;
    const bool wide = nb > PC_TBL8_MAX_BINS;
    const bool rppi = metric == PC_METRIC_RPPI;
    const bool pk = fp32 && rounding_key(nb, priv);
    if (fp32) {
        tbl_n = pk ? (uint32_t)PC_TBL_PK_CELLS : (uint32_t)table_cells(nb, priv);
        if (!((double)hi[nb] < key_top(nb, priv)))
            return CF_EINVAL;
    } else {
        log_table_geometry(lo.data(), hi.data(), ne, hi[nb], (uint32_t)table_cells(nb, priv),
                           &tbl_n, &shift, &base);
    }
    bool ordered = true;
    for (int k = 1; k < ne; k++)
        ordered = ordered && hi[k] >= hi[k - 1];
    // suffix minimum of the band bottoms (the table kernel stops its scan
    // once every later band starts above the cell)
    std::vector<float> lo_min(ne);
    float m_run = INFINITY;
    for (int k = ne - 1; k >= 0; k--) {
        m_run = std::min(m_run, lo[k]);
        lo_min[k] = m_run;
    }
    pc_bins h;
    memset(&h, 0, sizeof(h));
    h.nb = nb;
    h.npi = npi;
    h.tbl_shift = shift;
    h.tbl_n = (int32_t)tbl_n;
    h.tbl_wide = wide ? 1 : 0;
    h.tbl_base = base;
    h.e0_zero = (E[0] == 0.0) ? 1 : 0;
    h.s_top = hi[nb];
    h.pi_top = (metric == PC_METRIC_RPPI) ? phi[npi] : 0.0f;
    h.inv_dpi = (metric == PC_METRIC_RPPI) ? (float)((double)npi / pimax) : 0.0f;
    h.fscale_log2 = 0;
    if (metric == PC_METRIC_RPPI && !fp32) {
        // (the float32 pass bins pi in fixed point and needs no margin)
        // error of rounding the binary64 |dz| to float32, in units of the pi
        // bin width, plus the float32 product and the binary64 edges' offset
        // from p * dpi
        const double dpi = pimax / (double)npi;
        const double dz_err = kU32 * pimax;
        const double tau = kSafety * (dz_err / dpi + 3.0 * kU32 * npi + 4.0 * kU64 * npi) + 0x1p-22;
        if (!(tau < 0.25))
            return CF_EINVAL;
        h.pi_tau = (float)tau;
    }
    h.E_top = E[nb];
    h.pimax = (metric == PC_METRIC_RPPI) ? pimax : 0.0;
    h.row_w = rppi ? npi + 2 : 1;
    h.col0 = rppi ? 1 : 0;
    h.tbl_linear = fp32 ? (pk ? 2 : 1) : 0;
    h.tbl_out_zero = rppi ? 1 : 0;
    h.tbl_ordered = ordered ? 1 : 0;

    pc_bins_layout L;
    size_t off = align8(sizeof(pc_bins));
    L.lo = off;  off = align8(off + sizeof(float) * ne);
    L.hi = off;  off = align8(off + sizeof(float) * ne);
    L.lo_min = off; off = align8(off + sizeof(float) * ne);
    L.E = off;   off = align8(off + sizeof(double) * ne);
    L.plo = off; off = align8(off + sizeof(float) * nq);
    L.phi = off; off = align8(off + sizeof(float) * nq);
    L.q = off;   off = align8(off + sizeof(double) * nq);
    const size_t esz = wide ? sizeof(uint16_t) : sizeof(uint8_t);
    L.tbl = off; off = align8(off + esz * tbl_n);
    L.total = off;

    out->hdr = h;
    out->lay = L;
    // the table region is filled on the device (launch_build_table); only
    // the header and band arrays travel
    out->upload = L.tbl;
    out->buf.assign(L.tbl, 0);
    char *b = out->buf.data();
    memcpy(b, &h, sizeof(h));
    memcpy(b + L.lo, lo.data(), sizeof(float) * ne);
    memcpy(b + L.hi, hi.data(), sizeof(float) * ne);
    memcpy(b + L.lo_min, lo_min.data(), sizeof(float) * ne);
    memcpy(b + L.E, E.data(), sizeof(double) * ne);
    memcpy(b + L.plo, plo.data(), sizeof(float) * nq);
    memcpy(b + L.phi, phi.data(), sizeof(float) * nq);
    memcpy(b + L.q, q.data(), sizeof(double) * nq);
    out->nq = nq;
    out->ne = ne;
    return CF_OK;
}

}  // namespace pc

extern "C" cf_status cf_plan_grid(const double lo[3], const double hi[3],
                                  double boxsize, double reach_xy, double reach_z,
                                  int32_t slices_per_reach, cf_grid_plan *out)
{
    return cf_plan_grid_ex(lo, hi, boxsize, reach_xy, reach_z, slices_per_reach, 1, 0, out,
                           nullptr, nullptr);
}

extern "C" cf_status cf_plan_grid_ex(const double lo[3], const double hi[3], double boxsize,
                                     double reach_xy, double reach_z, int32_t slices_per_reach,
                                     int32_t xy_refine, int32_t ball, cf_grid_plan *out,
                                     int16_t *zro, int32_t *k_used)
{
    if (!out)
        return CF_EINVAL;
    double zl[3] = {0, 0, 0}, zh[3] = {0, 0, 0};
    if (std::isnan(boxsize) || (boxsize <= 0.0 && (!lo || !hi)))
        return CF_EINVAL;
    if (xy_refine < 1 || xy_refine > PC_MAX_XYK)
        return CF_EINVAL;
    pc_grid g;
    int rc = pc::plan_grid(lo ? lo : zl, hi ? hi : zh, boxsize, reach_xy, reach_z,
                           slices_per_reach, &g, xy_refine, ball != 0);
    if (rc)
        return (cf_status)rc;
    memset(out, 0, sizeof(*out));
    for (int a = 0; a < 3; a++) {
        out->lo[a] = g.lo[a];
        out->extent[a] = g.extent[a];
        out->inv_width[a] = g.inv_w[a];
        out->width[a] = g.width[a];
        out->n[a] = g.n[a];
    }
    out->zreach = g.zreach;
    out->periodic = g.periodic;
    out->boxsize = g.boxsize;
    out->ncell = g.ncell;
    if (zro)
        for (int a = 0; a <= PC_MAX_XYK; a++)
            for (int b = 0; b <= PC_MAX_XYK; b++)
                zro[a * (PC_MAX_XYK + 1) + b] = g.zro[a][b];
    if (k_used)
        *k_used = g.xyk;
    return CF_OK;
}

static_assert(sizeof(cf_sky_band) == sizeof(pc_band), "cf_sky_band mirrors pc_band");

extern "C" cf_status cf_plan_sky_grid(double chord_reach, double zlo, double zhi,
                                      int32_t slices, int32_t ra_refine, cf_sky_plan *out,
                                      cf_sky_band *bands, int32_t max_bands)
{
    if (!out || !bands)
        return CF_EINVAL;
    pc_grid g;
    memset(&g, 0, sizeof(g));
    std::vector<pc_band> b;
    int rc = pc::plan_sky_grid(chord_reach, zlo, zhi, slices, ra_refine, &g, &b);
    if (rc)
        return (cf_status)rc;
    if ((int64_t)b.size() > max_bands)
        return CF_EINVAL;
    memset(out, 0, sizeof(*out));
    out->nband = g.nband;
    out->ncol = g.n[1];
    out->slices = g.n[2];
    out->zreach = g.zreach;
    out->dec_lo = g.dec_lo;
    out->band_height = g.width[0];
    out->inv_slice = g.inv_hs;
    out->theta_reach = g.sky_reach;
    for (size_t k = 0; k < b.size(); k++) {
        bands[k].col0 = b[k].col0;
        bands[k].nra = b[k].nra;
        bands[k].ra_scale = b[k].ra_scale;
        for (int d = 0; d < 3; d++)
            bands[k].dra[d] = b[k].dra[d];
    }
    return CF_OK;
}

extern "C" cf_status cf_fp32_bands(const double *edges_sq, int32_t nedges, int32_t ndim,
                                   double coord_scale, float *lo, float *hi)
{
    if (!edges_sq || !lo || !hi)
        return CF_EINVAL;
    return (cf_status)pc::fp32_bands(edges_sq, nedges, ndim, coord_scale, lo, hi);
}

extern "C" cf_status cf_fp32_bands_axes(const double *edges_sq, int32_t nedges, int32_t ndim,
                                        const double *axis_eps, double coord_scale,
                                        float *lo, float *hi)
{
    if (!edges_sq || !axis_eps || !lo || !hi)
        return CF_EINVAL;
    return (cf_status)pc::fp32_bands_axes(edges_sq, nedges, ndim, axis_eps, coord_scale, lo,
                                          hi);
}

extern "C" cf_status cf_fp32_bands_xy(const double *edges_sq, int32_t nedges, int32_t ndim,
                                      const double *axis_eps, const double *xy_max,
                                      double coord_scale, float *lo, float *hi)
{
    if (!edges_sq || !axis_eps || !xy_max || !lo || !hi || (ndim != 2 && ndim != 3))
        return CF_EINVAL;
    for (int k = 0; k < 4; k++)
        if (!(xy_max[k] >= 0.0) || !std::isfinite(xy_max[k]))
            return CF_EINVAL;
    const double mag = pc::xy_expand_mag(xy_max, xy_max + 2, ndim);
    return (cf_status)pc::fp32_bands_axes(edges_sq, nedges, ndim, axis_eps, coord_scale, lo, hi,
                                          mag > 0.0 ? mag : 0x1p-1000);
}

extern "C" cf_status cf_fp32_pair_margin(const double *xy_max, int32_t ndim, double fscale,
                                         float *K, float *M)
{
    if (!xy_max || !K || !M || (ndim != 2 && ndim != 3) || !(fscale > 0.0) ||
        !std::isfinite(fscale))
        return CF_EINVAL;
    for (int k = 0; k < 4; k++)
        if (!(xy_max[k] >= 0.0) || !std::isfinite(xy_max[k]))
            return CF_EINVAL;
    pc::xy_pair_margin(pc::xy_expand_mag(xy_max, xy_max + 2, ndim), fscale, K, M);
    return CF_OK;
}

// Host twin of the fixed-point weight sums (pc_fixed.h): the same limb split,
// limb sums and 192-bit assembly as the sweep and its merges, in one thread.
extern "C" cf_status cf_fixed_sum(const double *p, int64_t n, int32_t q, double *out)
{
    if (!out || n < 0 || (n > 0 && !p) || q < -1022 || q > 900)
        return CF_EINVAL;
    unsigned long long acc[3] = {0ull, 0ull, 0ull};
    unsigned long long s0 = 0, s1 = 0, s2 = 0;
    int64_t pending = 0;
    for (int64_t k = 0; k < n; k++) {
        const double P = ldexp(p[k], -q);
        if (!(fabs(P) < 0x1p94) || P != floor(P))
            return CF_EINVAL;
        unsigned long long l0, l1, l2;
        pc::fixed_limbs(P, l0, l1, l2);
        s0 += l0;
        s1 += l1;
        s2 += l2;
        // merge before 2^31 limbs could overflow the int64 sums, as the
        // sweep's flush bound does
        if (++pending == 0x7fffffff || k + 1 == n) {
            unsigned long long v[3];
            pc::fixed_words((long long)s0, (long long)s1, (long long)s2, v);
            pc::fixed_add(acc, v);
            s0 = s1 = s2 = 0;
            pending = 0;
        }
    }
    *out = pc::fixed_to_double(acc, q);
    return CF_OK;
}
