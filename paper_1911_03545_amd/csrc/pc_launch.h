// pc_launch.h -- host-callable launchers of the gfx950 kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pc_common.h"
#include "pc_fixed.h"

namespace pc {

// flags raised by the input kernels
#define PC_FLAG_NONFINITE 1u
#define PC_FLAG_RANGE 2u
#define PC_FLAG_WEIGHT 4u
#define PC_FLAG_RADEC 8u
#define PC_FLAG_ITEMS 16u
#define PC_FLAG_UNIT 32u      // angular grid: a vector whose squared norm is not within 2^-20 of 1
#define PC_FLAG_WFIXED 64u    // fixed-point weight sums: no grid holds every pair weight

struct SweepArgs {
    const pc_item *items;
    int32_t n_items;              // items, or the item capacity when n_items_dev is set
    const int32_t *n_items_dev;   // device item count (replayed calls), or NULL
    int32_t *counter;      // PC_STREAMS item counters, PC_STREAM_STRIDE apart, zeroed
    const float *X1, *Y1, *Z1, *X2, *Y2, *Z2;    // float32 (x, y column-local when xy_local)
    const double *x1, *y1, *z1, *x2, *y2, *z2;   // binary64, input values
    const double *w1, *w2;
    double L;
    float Lf32;            // periodic length in the scaled float32 coordinates
    pc_bins B;
    const float *lo, *hi, *plo, *phi;
    const double *E, *q;
    const uint16_t *tbl;
    unsigned long long *g_hist;
    double *g_whist;
    // fixed-point weight sums (pc_fixed.h): the LDS weight area holds three
    // uint64 limb sums per slot, wlimb slots apart; g_wfix three words per bin
    int32_t wfixed;
    int32_t wlimb;
    const pc_wfixed *wfx;
    unsigned long long *g_wfix;
    double *g_rhist;       // sums of separation x pair weight (mean separation), or NULL
    int32_t ravg;          // 0: no mean separation; 1: distance sqrt(s);
                           // 2: angle in degrees of a squared chord s
    int32_t wtype;         // pair weight: 0 product, 1 sum
    double sep_scale;      // float32 pass: length per float32 coordinate unit (1 / fscale)
    unsigned *rq_count;   // float32 pass: pairs re-evaluated in binary64
    // a wave merges its LDS replicas into the global bins before its pending
    // pair evaluations since the last merge would exceed flush_at (so no
    // uint32 LDS counter can wrap); flush_count counts those merges
    unsigned long long flush_at;
    unsigned *flush_count;
    // float32 sweeps of 3-D grids: x and y of side 2 are column-local
    // (pc_frame.h); each lane's point is placed in the frame of the item's j
    // column, found from the cell id of the item's first j point
    int32_t xy_local;
    // float32 DD(r) and DD(rp, pi) of 3-D grids: x and y expanded as |a|^2 +
    // |b|^2 - 2 a.b, with P2 = (x, y, z, |b|^2) of every sorted point of side
    // 2 in float32 (z: the rp/pi path's fixed-point bits)
    int32_t xy_exp;
    const float4 *P2;
    // the expanded bands hold the magnitude term xy_M (scaled coordinates)
    // times xy_K; a pair whose own magnitude term m is smaller may narrow
    // both sides of its band by xy_K (xy_M - m) (both rounded down)
    float xy_K, xy_M;
    int32_t gnx, gny, gnz;
    double glo[3];
    double gw[2];
    double fscale;
    const int32_t *cs2;   // cell id of every sorted point of side 2
    const int32_t *icell; // cell id of every item's first j point
    int32_t priv;       // per-wave private replicas, flushed per catalogue (batches)
    int32_t copies;     // LDS histogram replicas per wave (power of two; 64 = one per
                        // lane with unconditional updates, 1-D unweighted only)
    int32_t nbt;        // bins in total (nb * npi)
    int32_t slots;      // slots per replica: (nb + 2) * npi
    int32_t rep_stride; // distance between replicas (slots rounded up to odd)
    // dynamic LDS layout (bytes)
    int32_t o_tbl, o_lo, o_hi, o_E, o_q, o_hist, o_whist, o_rhist;
    int32_t hist_stride;   // uint32 slots of all replicas (one set per workgroup)
    int32_t whist_stride;  // double slots of all replicas
    int32_t lds_bytes;
};

// fill the lookup table of a bin description (B.tbl_n cells) on the device
hipError_t launch_build_table(hipStream_t s, const pc_bins &B, int nedges, const float *lo,
                              const float *hi, const float *lo_min, void *tbl);
// zero `bytes` (a multiple of 4) of device memory with a kernel
hipError_t launch_zero(hipStream_t s, void *p, size_t bytes);
// zero `count` (at most PC_ZERO_MAX) such regions with one launch
#define PC_ZERO_MAX 6
hipError_t launch_zero_multi(hipStream_t s, int count, void *const *ptrs, const size_t *bytes);
// unit vectors of RA/DEC in degrees, times the distance column when `dist`
// is not NULL (on-sky positions)
hipError_t launch_radec(hipStream_t s, int64_t n, const void *ra, const void *dec,
                        const void *dist, int f32, double d2r, double *x, double *y, double *z,
                        unsigned *flags);
hipError_t launch_minmax(hipStream_t s, int64_t n, const void *x, const void *y,
                         const void *z, int f32, double *part, int nparts, unsigned *flags);
hipError_t launch_minmax_final(hipStream_t s, const double *part, int nparts, double *out6);
// cell and in-cell rank of every point of a side's catalogues, plus a
// 32-byte (x, y, z, w) record per point in input order (rec: ntot records)
hipError_t launch_cell_index(hipStream_t s, int ncat, const pc_cat *cats, int64_t ntot,
                             const pc_grid &g, unsigned *cnt, int32_t *cell_of, int32_t *rank_of,
                             void *rec, unsigned *flags);
// exclusive scan of n int32 values into out[0..n] (out[n] = total); `tmp`
// needs scan_tmp_elems(n) int32.
size_t scan_tmp_elems(int64_t n);
hipError_t scan_exclusive(hipStream_t s, const int32_t *in, int64_t n, int32_t *out,
                          int32_t *tmp);
// place every point at start[cell] + rank: a permutation scatter of source
// indices into `perm` (ntot int32), then a gather in sorted order.  P
// (optional; the expanded float32 sweeps): the float32 x, y, z and
// fl(y y + fl(x x)) of every sorted point side by side, written with Z in
// place of X and Y.
hipError_t launch_scatter(hipStream_t s, int64_t ntot, const pc_grid &g, const int32_t *cell_of,
                          const int32_t *rank_of, const void *rec, const int32_t *start,
                          int32_t *perm, float *X, float *Y, float *Z, double *xd, double *yd,
                          double *zd, double *wd, float4 *P, int32_t *cell_sorted);
// the gather half of launch_scatter (perm already known; with cell_of NULL
// the cell ids of the sorted points are left as they are)
hipError_t launch_gather(hipStream_t s, int64_t ntot, const pc_grid &g, const int32_t *perm,
                         const int32_t *cell_of, const void *rec, float *X, float *Y, float *Z,
                         double *xd, double *yd, double *zd, double *wd, float4 *P,
                         int32_t *cell_sorted);
// Two-level counting sort without global atomics (columns in LDS per chunk of
// `chunk` points, then z slices in LDS per column) followed by the gather
// into the sorted arrays: start (ncat * ncell + 1), cell_sorted, X, Y, Z, xd,
// yd, zd and (optional) wd, like launch_cell_index + scan + launch_scatter.
// Needs ncolc and g.n[2] at most PC_SORT2_MAX_BINS; `lay` holds 3 (ncat + 1)
// ints, wcnt m ints, woff m + 1 ints (m = sum over catalogues of ncolc *
// chunks), tmp scan_tmp_elems(m) ints; scratch: colrec ntot 32-byte records
// (column order), rank_slice ntot int pairs, perm, cell_of and rank_of ntot
// ints each.
#define PC_SORT2_MAX_BINS 16384
hipError_t launch_sort2(hipStream_t s, int ncat, const pc_cat *cats, int64_t ntot,
                        const pc_grid &g, int32_t chunk, int32_t ncolc, int32_t n_chunks,
                        int64_t m, int32_t *lay, int32_t *wcnt, int32_t *woff, int32_t *tmp,
                        int32_t *cell_of, int32_t *rank_of, void *colrec, void *rank_slice,
                        int32_t *perm, int32_t *start, int32_t *cell_sorted, float *X, float *Y,
                        float *Z, double *xd, double *yd, double *zd, double *wd, float4 *P,
                        unsigned *flags);
hipError_t launch_block_count(hipStream_t s, int32_t ncol, int32_t nz, const int32_t *start,
                              int32_t *bcnt);
hipError_t launch_block_emit(hipStream_t s, int32_t ncol, int32_t nz, const int32_t *start,
                             const int32_t *boff, pc_block *blocks);
hipError_t launch_item_count(hipStream_t s, int32_t nblocks, const int32_t *nblocks_dev,
                             const pc_block *blocks, const pc_grid &g, const int32_t *start2,
                             const int32_t *cell1_sorted, int autocorr, int chunk,
                             int32_t *icnt, unsigned long long *cand);
// icell (optional, with cell2_sorted): the cell id of every item's first j
// point, beside the items (the float32 sweep of 3-D grids reads it one item
// ahead, with the item, to place its lanes in the j column's frame)
hipError_t launch_item_emit(hipStream_t s, int32_t nblocks, const int32_t *nblocks_dev,
                            const pc_block *blocks, const pc_grid &g, const int32_t *start2,
                            const int32_t *cell1_sorted, int autocorr, int chunk,
                            const int32_t *ioff, pc_item *items, int32_t cap, unsigned *flags,
                            const int32_t *cell2_sorted, int32_t *icell);
// wmode: 0 unweighted, 1 weight sums, 2 weight and mean-separation sums
hipError_t launch_sweep(hipStream_t s, int metric, bool fp32, int wmode, const SweepArgs &a,
                        int nwg);
// per-catalogue sum of the self-pair weights (w^2, or 2w for summed pair
// weights) over the cell-ordered weights of a side
hipError_t launch_wsq(hipStream_t s, int32_t ncat, int64_t ncell, const int32_t *start,
                      const double *w, int wtype, double *out);
// Fixed-point weight sums: atomic maxima over the nonzero weights of one
// side (side 0 or 1) into fx (zeroed first), then the grid and its checks
// (PC_FLAG_WFIXED when the weights do not fit), then the self-pair sums
// (three words per catalogue, zeroed first).
hipError_t launch_wfixed_scan(hipStream_t s, int64_t n, const double *w, int side,
                              pc_wfixed *fx);
hipError_t launch_wfixed_plan(hipStream_t s, int wtype, int two_sided, pc_wfixed *fx,
                              unsigned *flags);
hipError_t launch_wsq_fixed(hipStream_t s, int32_t ncat, int64_t ncell, const int32_t *start,
                            const double *w, int wtype, const pc_wfixed *fx,
                            unsigned long long *out);
// counts (and weight sums, mean separations) of every catalogue: doubling
// and self-pairs of autocorrelations; the mean separation is the separation
// sum over the weight sum
// (it also copies the device work-item and block counts to `sizes_out`)
hipError_t launch_finalize(hipStream_t s, int32_t ncat, int32_t nbt, int autocorr, int e0_zero,
                           const pc_cat *cats, const unsigned long long *g_hist,
                           const double *g_whist, const double *g_rhist, const double *wsq,
                           const unsigned long long *g_wfix,
                           const unsigned long long *wsq_fix, const pc_wfixed *wfx,
                           unsigned long long *out_counts, double *out_wsum,
                           double *out_ravg, const int32_t *n_items_dev,
                           const int32_t *n_blocks_dev, int32_t *sizes_out);
// resident sweep workgroups per CU for a dynamic LDS size
// waves per sweep workgroup
int sweep_waves();
// (exp: the float32 r sweep with x and y expanded)
hipError_t sweep_occupancy(int metric, bool fp32, int wmode, bool t16, bool unc, bool priv,
                           bool exp, int lds_bytes, int *per_cu);
// device address and size of the fixed scratch of the no-allocation entry
// point on `device`, which must be the current device (looked up once per
// device, then cached)
hipError_t noalloc_scratch(int device, void **ptr, size_t *bytes);

}  // namespace pc
