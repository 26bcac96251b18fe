// pc_grid.hip -- input staging, gridding (cell index + counting sort) and the
// work-list kernels for gfx950.
//
// Gridding follows section "Partitioning the particles on a grid" (cell index
// of each point from the bounding box and the cell count per axis) and
// section "Improving cache locality" (points copied into contiguous per-cell
// arrays), done as a parallel counting sort: an atomic histogram of cell ids,
// an exclusive scan, and a scatter into structure-of-arrays buffers.
//
// The work list follows sections "Associating pairs of cells" and "Symmetry
// considerations for autocorrelations": for each block of up to 64 points of
// one x/y column, the neighbouring columns (periodic indices wrapped with a
// stored offset of +-L) and, inside each, the contiguous run of z slices that
// can hold a partner within the line-of-sight reach.
#include <hip/hip_runtime.h>

#include "pc_common.h"
#include "pc_frame.h"
#include "pc_launch.h"

namespace pc {
namespace {

constexpr int kThreads = 256;

__device__ __forceinline__ double ld(const void *p, int f32, int64_t i)
{
    return f32 ? (double)static_cast<const float *>(p)[i] : static_cast<const double *>(p)[i];
}

int grid_for(int64_t n, int threads = kThreads, int cap = 8192)
{
    int64_t g = (n + threads - 1) / threads;
    if (g < 1)
        g = 1;
    if (g > cap)
        g = cap;
    return (int)g;
}

// Zero n 32-bit words (a kernel rather than a memset node, so that the
// call's device work can be captured into a graph and replayed).
__global__ void k_zero(uint32_t *p, int64_t n)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0u;
}

// Several regions cleared by one launch (blockIdx.y selects the region).
struct ZeroSet {
    uint32_t *p[PC_ZERO_MAX];
    int64_t n[PC_ZERO_MAX];
};

__global__ void k_zero_multi(ZeroSet z)
{
    uint32_t *p = z.p[blockIdx.y];
    const int64_t n = z.n[blockIdx.y];
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0u;
}

// Unit vectors of RA/DEC (degrees; d2r = fl(pi) / 180), or, with a distance
// column, the positions D u of on-sky catalogues.
__global__ void k_radec(int64_t n, const void *ra, const void *dec, const void *dist, int f32,
                        double d2r, double *x, double *y, double *z, unsigned *flags)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const double a = ld(ra, f32, i), d = ld(dec, f32, i);
        if (!(a >= 0.0 && a <= 360.0 && d >= -90.0 && d <= 90.0))
            atomicOr(flags, PC_FLAG_RADEC);
        const double ar = a * d2r, dr = d * d2r;
        const double cd = cos(dr);
        double ux = cd * cos(ar), uy = cd * sin(ar), uz = sin(dr);
        if (dist) {
            const double D = ld(dist, f32, i);
            if (!(D >= 0.0) || !isfinite(D))
                atomicOr(flags, PC_FLAG_NONFINITE);
            ux = D * ux;
            uy = D * uy;
            uz = D * uz;
        }
        x[i] = ux;
        y[i] = uy;
        z[i] = uz;
    }
}

__global__ void k_minmax(int64_t n, const void *x, const void *y, const void *z, int f32,
                         double *part, unsigned *flags)
{
    double mn[3] = {INFINITY, INFINITY, INFINITY};
    double mx[3] = {-INFINITY, -INFINITY, -INFINITY};
    bool bad = false;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const double c[3] = {ld(x, f32, i), ld(y, f32, i), ld(z, f32, i)};
        for (int a = 0; a < 3; a++) {
            if (!isfinite(c[a]))
                bad = true;
            else {
                mn[a] = fmin(mn[a], c[a]);
                mx[a] = fmax(mx[a], c[a]);
            }
        }
    }
    if (bad)
        atomicOr(flags, PC_FLAG_NONFINITE);
    __shared__ double sm[6][kThreads];
    for (int a = 0; a < 3; a++) {
        sm[a][threadIdx.x] = mn[a];
        sm[3 + a][threadIdx.x] = mx[a];
    }
    __syncthreads();
    for (int st = kThreads / 2; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st)
            for (int a = 0; a < 3; a++) {
                sm[a][threadIdx.x] = fmin(sm[a][threadIdx.x], sm[a][threadIdx.x + st]);
                sm[3 + a][threadIdx.x] =
                    fmax(sm[3 + a][threadIdx.x], sm[3 + a][threadIdx.x + st]);
            }
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int a = 0; a < 6; a++)
            part[blockIdx.x * 6 + a] = sm[a][0];
}

__global__ void k_minmax_final(const double *part, int nparts, double *out6)
{
    // one wavefront: each lane folds a strided share of the partials, then
    // the lanes are combined with shuffles (fmin / fmax are exact, so the
    // order does not change the result)
    double r[6] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY};
    for (int p = threadIdx.x; p < nparts; p += blockDim.x)
        for (int a = 0; a < 3; a++) {
            r[a] = fmin(r[a], part[p * 6 + a]);
            r[3 + a] = fmax(r[3 + a], part[p * 6 + 3 + a]);
        }
    for (int off = 32; off > 0; off >>= 1)
        for (int a = 0; a < 3; a++) {
            r[a] = fmin(r[a], __shfl_xor(r[a], off, 64));
            r[3 + a] = fmax(r[3 + a], __shfl_xor(r[3 + a], off, 64));
        }
    if (threadIdx.x == 0)
        for (int a = 0; a < 6; a++)
            out6[a] = r[a];
}

// Cell coordinate: t = fl(fl(x - lo) * inv_w) is monotone in x; NaN and
// negative values go to cell 0 and values at or past the far face to n - 1.
__device__ __forceinline__ int cell_coord(double d, double inv, int n)
{
    const double t = d * inv;
    if (!(t > 0.0))
        return 0;
    if (t >= (double)(n - 1))
        return n - 1;
    return (int)t;
}

// Column and slice of a point; non-finite coordinates and coordinates outside
// a periodic box raise flags.  Angular grid: the declination slice and the
// right-ascension cell of the vector's direction (atan2 of its components,
// so the vector need not be exactly unit; its squared norm is checked to lie
// within 2^-20 of 1, the bound the grid's reach was planned for).
template <bool SKY>
__device__ __forceinline__ int2 point_cell(const pc_grid &g, const double c[3], unsigned &fl)
{
    for (int a = 0; a < 3; a++) {
        if (!isfinite(c[a]))
            fl |= PC_FLAG_NONFINITE;
        else if (g.periodic && (c[a] < 0.0 || c[a] > g.boxsize))
            fl |= PC_FLAG_RANGE;
    }
    if constexpr (SKY) {
        const double rho2 = c[0] * c[0] + c[1] * c[1];
        const double r2 = rho2 + c[2] * c[2];
        if (!(fabs(r2 - 1.0) <= 0x1p-20))
            fl |= PC_FLAG_UNIT;
        const double dec = atan2(c[2], sqrt(rho2));
        double ra = atan2(c[1], c[0]);
        if (ra < 0.0)
            ra += 2.0 * M_PI;
        const int S = g.n[2];
        const int gs = cell_coord(dec - g.dec_lo, g.inv_hs, g.nband * S);
        const int b = gs / S;
        const pc_band &B = g.bands[b];
        return make_int2(B.col0 + cell_coord(ra, B.ra_scale, B.nra), gs - b * S);
    } else {
    const int ix = cell_coord(c[0] - g.lo[0], g.inv_w[0], g.n[0]);
    const int iy = cell_coord(c[1] - g.lo[1], g.inv_w[1], g.n[1]);
    const int iz = cell_coord(c[2] - g.lo[2], g.inv_w[2], g.n[2]);
    return make_int2(ix * g.n[1] + iy, iz);
    }
}

// Catalogue of flattened index i: the last catalogue starting at or before
// i (empty catalogues share their start with the next one, which wins).
__device__ __forceinline__ int find_cat(const pc_cat *cats, int ncat, int64_t i)
{
    int lo = 0, hi = ncat - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (cats[mid].off <= i)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

// Cell of every point of every catalogue of a side (catalogue c owns cells
// c * ncell .. (c + 1) * ncell - 1) and its rank inside the cell; input
// checks (finite, inside the periodic box, finite weights) raise flags.
// It also writes each point as one 32-byte record (x, y, z, w) in input
// order, so that the gather after the sort reads one line per point.
template <bool SKY>
__global__ void k_cell_index(int ncat, const pc_cat *cats, int64_t ntot, pc_grid g,
                             unsigned *cnt, int32_t *cell_of, int32_t *rank_of, double4 *rec,
                             unsigned *flags)
{
    unsigned fl = 0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < ntot;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int ci = ncat == 1 ? 0 : find_cat(cats, ncat, i);
        const pc_cat &k = cats[ci];
        const int64_t j = i - k.off;
        const double c[3] = {ld(k.x, k.f32, j), ld(k.y, k.f32, j), ld(k.z, k.f32, j)};
        const int2 cs = point_cell<SKY>(g, c, fl);
        // unit weights without weights (the mean-separation sums use them)
        const double w = k.w ? ld(k.w, k.wf32, j) : 1.0;
        if (!isfinite(w))
            fl |= PC_FLAG_WEIGHT;
        const int cell = (int)(ci * g.ncell) + cs.x * g.n[2] + cs.y;
        cell_of[i] = cell;
        rec[i] = make_double4(c[0], c[1], c[2], w);
        rank_of[i] = (int32_t)atomicAdd(&cnt[cell], 1u);
    }
    if (fl)
        atomicOr(flags, fl);
}

// ---- exclusive scan (int32), 1024 values per workgroup -------------------
constexpr int kScanPer = 4;
constexpr int kScanBlock = kThreads * kScanPer;
// block totals a k_scan_apply_parts block sums itself (up to 2048 values of
// loads per block, instead of one more scan launch)
constexpr int kScanPartsInline = 2048;

__device__ int block_exclusive(int v, int *total)
{
    __shared__ int sm[kThreads];
    sm[threadIdx.x] = v;
    __syncthreads();
    for (int off = 1; off < kThreads; off <<= 1) {
        int t = (int)threadIdx.x >= off ? sm[threadIdx.x - off] : 0;
        __syncthreads();
        sm[threadIdx.x] += t;
        __syncthreads();
    }
    const int incl = sm[threadIdx.x];
    *total = sm[kThreads - 1];
    __syncthreads();
    return incl - v;
}

__global__ void k_scan_reduce(const int32_t *in, int64_t n, int32_t *part)
{
    const int64_t base = (int64_t)blockIdx.x * kScanBlock + threadIdx.x * kScanPer;
    int s = 0;
    for (int k = 0; k < kScanPer; k++)
        if (base + k < n)
            s += in[base + k];
    int total;
    block_exclusive(s, &total);
    if (threadIdx.x == 0)
        part[blockIdx.x] = total;
}

// Like k_scan_apply below, with the block's offset summed from the block
// totals `part` (nparts of them, at most a few thousand) by the block itself,
// so a scan of up to kScanBlock * nparts values takes two launches.
__global__ void k_scan_apply_parts(const int32_t *in, int64_t n, const int32_t *part,
                                   int32_t *out)
{
    int pre = 0;
    for (int k = threadIdx.x; k < (int)blockIdx.x; k += kThreads)
        pre += part[k];
    int total;
    block_exclusive(pre, &total);
    const int64_t base = (int64_t)blockIdx.x * kScanBlock + threadIdx.x * kScanPer;
    int v[kScanPer];
    int s = 0;
    for (int k = 0; k < kScanPer; k++) {
        v[k] = (base + k < n) ? in[base + k] : 0;
        s += v[k];
    }
    int tot2;
    int run = block_exclusive(s, &tot2) + total;
    for (int k = 0; k < kScanPer; k++) {
        if (base + k < n)
            out[base + k] = run;
        run += v[k];
    }
    const int64_t end = (int64_t)(blockIdx.x + 1) * kScanBlock;
    if (threadIdx.x == kThreads - 1 && end >= n)
        out[n] = run;
}

// out[i] = exclusive prefix + offset[block]; the workgroup holding the end
// also writes out[n].
__global__ void k_scan_apply(const int32_t *in, int64_t n, const int32_t *offs, int32_t *out)
{
    const int64_t base = (int64_t)blockIdx.x * kScanBlock + threadIdx.x * kScanPer;
    int v[kScanPer];
    int s = 0;
    for (int k = 0; k < kScanPer; k++) {
        v[k] = (base + k < n) ? in[base + k] : 0;
        s += v[k];
    }
    int total;
    int run = block_exclusive(s, &total) + (offs ? offs[blockIdx.x] : 0);
    for (int k = 0; k < kScanPer; k++) {
        if (base + k < n)
            out[base + k] = run;
        run += v[k];
    }
    const int64_t end = (int64_t)(blockIdx.x + 1) * kScanBlock;
    if (threadIdx.x == kThreads - 1 && end >= n)
        out[n] = run;
}

// ---- two-level counting sort (no global atomics) --------------------------
// Level 1 groups the points by column: a workgroup takes a chunk of one
// catalogue's points, counts them per column in LDS (the LDS atomic gives a
// point its rank among the chunk's points of that column) and writes the
// chunk's column counts into a [catalogue][column][chunk] matrix, whose
// exclusive scan is every (chunk, column) run's place in column order.
// Level 2 sorts each column's points by z slice in LDS and writes the final
// cell order (`perm`) and the cell starts.  Layout per catalogue k (computed
// on the device): lay[3k] = first chunk index, lay[3k+1] = chunks, lay[3k+2]
// = first matrix entry.
__global__ void k_grid_layout(int ncat, const pc_cat *cats, int32_t chunk, int32_t ncolc,
                              int32_t *lay)
{
    if (threadIdx.x != 0 || blockIdx.x != 0)
        return;
    int64_t wg = 0, mb = 0;
    for (int k = 0; k < ncat; k++) {
        const int64_t nw = (cats[k].n + chunk - 1) / chunk;
        lay[3 * k] = (int32_t)wg;
        lay[3 * k + 1] = (int32_t)nw;
        lay[3 * k + 2] = (int32_t)mb;
        wg += nw;
        mb += nw * ncolc;
    }
    lay[3 * ncat] = (int32_t)wg;
    lay[3 * ncat + 1] = 0;
    lay[3 * ncat + 2] = (int32_t)mb;
}

// Level 1, counting: one workgroup per chunk, LDS histogram of ncolc columns.
// Each thread loads kHistPer points before it bins them, so that their loads
// are in flight together.
constexpr int kHistPer = 8;
template <bool SKY>
__global__ __launch_bounds__(kThreads) void k_cell_hist(int ncat, const pc_cat *cats,
                                                        const int32_t *lay, pc_grid g,
                                                        int32_t chunk, int32_t ncolc,
                                                        int32_t *__restrict__ cell_of,
                                                        int32_t *__restrict__ rank_of,
                                                        int32_t *__restrict__ wcnt,
                                                        unsigned *flags)
{
    extern __shared__ unsigned hist[];
    const int w = blockIdx.x;
    int k = 0, hi = ncat - 1;   // the last catalogue whose first chunk is <= w
    while (k < hi) {
        const int mid = (k + hi + 1) >> 1;
        if (lay[3 * mid] <= w)
            k = mid;
        else
            hi = mid - 1;
    }
    const pc_cat &ct = cats[k];
    const int wl = w - lay[3 * k], nw = lay[3 * k + 1], mb = lay[3 * k + 2];
    const int64_t i0 = ct.off + (int64_t)wl * chunk;
    const int64_t i1 = min(ct.off + ct.n, i0 + chunk);
    for (int c = threadIdx.x; c < ncolc; c += blockDim.x)
        hist[c] = 0u;
    __syncthreads();
    unsigned fl = 0;
    for (int64_t base = i0 + threadIdx.x; base < i1; base += (int64_t)kHistPer * blockDim.x) {
        double c[kHistPer][3];
#pragma unroll
        for (int p = 0; p < kHistPer; p++) {
            const int64_t i = base + (int64_t)p * blockDim.x;
            const int64_t j = (i < i1 ? i : i0) - ct.off;
            c[p][0] = ld(ct.x, ct.f32, j);
            c[p][1] = ld(ct.y, ct.f32, j);
            c[p][2] = ld(ct.z, ct.f32, j);
        }
#pragma unroll
        for (int p = 0; p < kHistPer; p++) {
            const int64_t i = base + (int64_t)p * blockDim.x;
            if (i >= i1)
                break;
            const int2 cs = point_cell<SKY>(g, c[p], fl);
            const int col = cs.x;
            cell_of[i] = (int)((int64_t)k * g.ncell) + col * g.n[2] + cs.y;
            rank_of[i] = (int32_t)atomicAdd(&hist[col], 1u);
        }
    }
    __syncthreads();
    for (int c = threadIdx.x; c < ncolc; c += blockDim.x)
        wcnt[mb + (int64_t)c * nw + wl] = (int32_t)hist[c];
    if (fl)
        atomicOr(flags, fl);
}

// Level 1, placement with a chunk-local sort (chunks of kLocalChunk points,
// at most kThreads columns): one workgroup per chunk first places its
// records in LDS in (column, rank) order, then writes each column's run of
// records contiguously to its column-ordered place; the same result as
// k_col_scatter with writes in runs instead of one 32-byte record per lane
// anywhere in the output.
// It also writes each point's slice (recomputed from its record with the
// cell arithmetic of k_cell_hist) beside it, so the slice sort's counting pass
// reads 8 bytes per point instead of the record.
constexpr int kLocalChunk = 2048;
template <bool SKY>
__global__ __launch_bounds__(kThreads) void k_col_scatter_local(
    int ncat, const pc_cat *cats, const int32_t *lay, pc_grid g, int32_t ncolc,
    const int32_t *__restrict__ cell_of, const int32_t *__restrict__ rank_of,
    const int32_t *__restrict__ wcnt, const int32_t *__restrict__ woff,
    double4 *__restrict__ colrec, int2 *__restrict__ rank_slice, unsigned *flags)
{
    const int nz = g.n[2];
    __shared__ double4 s_rec[kLocalChunk];
    __shared__ int s_pos[kLocalChunk];
    __shared__ int s_loc[kThreads];
    __shared__ int s_glob[kThreads];
    const int w = blockIdx.x;
    int k = 0, hi = ncat - 1;   // the last catalogue whose first chunk is <= w
    while (k < hi) {
        const int mid = (k + hi + 1) >> 1;
        if (lay[3 * mid] <= w)
            k = mid;
        else
            hi = mid - 1;
    }
    const pc_cat &ct = cats[k];
    const int wl = w - lay[3 * k], nw = lay[3 * k + 1], mb = lay[3 * k + 2];
    const int64_t i0 = ct.off + (int64_t)wl * kLocalChunk;
    const int n = (int)min((int64_t)kLocalChunk, ct.off + ct.n - i0);
    // this chunk's count and output place per column, and the local prefix
    const int c = threadIdx.x;
    const int cnt = c < ncolc ? wcnt[mb + (int64_t)c * nw + wl] : 0;
    if (c < ncolc)
        s_glob[c] = woff[mb + (int64_t)c * nw + wl];
    int total;
    const int ex = block_exclusive(cnt, &total);
    if (c < ncolc)
        s_loc[c] = ex;
    __syncthreads();
    unsigned fl = 0;
    for (int p = threadIdx.x; p < n; p += kThreads) {
        const int64_t i = i0 + p;
        const int64_t j = i - ct.off;
        const double wt = ct.w ? ld(ct.w, ct.wf32, j) : 1.0;
        if (!isfinite(wt))
            fl |= PC_FLAG_WEIGHT;
        const int col = (int)((uint32_t)cell_of[i] / (uint32_t)nz) - k * ncolc;
        const int r = rank_of[i];
        const int slot = s_loc[col] + r;
        s_rec[slot] = make_double4(ld(ct.x, ct.f32, j), ld(ct.y, ct.f32, j), ld(ct.z, ct.f32, j),
                                   wt);
        s_pos[slot] = s_glob[col] + r;
    }
    __syncthreads();
    unsigned fl2 = 0;   // (flags were raised by k_cell_hist)
    for (int q = threadIdx.x; q < n; q += kThreads) {
        const double4 r = s_rec[q];
        const double c3[3] = {r.x, r.y, r.z};
        const int d = s_pos[q];
        colrec[d] = r;
        rank_slice[d] = make_int2(0, point_cell<SKY>(g, c3, fl2).y);
    }
    if (fl)
        atomicOr(flags, fl);
}

// Level 1, placement: every point, as one 32-byte record (x, y, z, w) read
// from the input columns, to its column-ordered place, so that level 2
// streams through its column.  Non-finite weights raise a flag here.
__global__ __launch_bounds__(kThreads) void k_col_scatter(
    int64_t ntot, int ncat, const pc_cat *cats, const int32_t *lay, int32_t nz, int32_t chunk,
    int32_t ncolc, const int32_t *__restrict__ cell_of, const int32_t *__restrict__ rank_of,
    const int32_t *__restrict__ woff, double4 *__restrict__ colrec, unsigned *flags)
{
    unsigned fl = 0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < ntot;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int k = ncat == 1 ? 0 : find_cat(cats, ncat, i);
        const pc_cat &ct = cats[k];
        const int64_t j = i - ct.off;
        const double x = ld(ct.x, ct.f32, j), y = ld(ct.y, ct.f32, j), z = ld(ct.z, ct.f32, j);
        // unit weights without weights (the mean-separation sums use them)
        const double wt = ct.w ? ld(ct.w, ct.wf32, j) : 1.0;
        if (!isfinite(wt))
            fl |= PC_FLAG_WEIGHT;
        const int wl = (int)((uint32_t)j / (uint32_t)chunk);
        const int cz = (int)((uint32_t)cell_of[i] / (uint32_t)nz);
        const int64_t m = lay[3 * k + 2] + (int64_t)(cz - k * ncolc) * lay[3 * k + 1] + wl;
        colrec[(int64_t)woff[m] + rank_of[i]] = make_double4(x, y, z, wt);
    }
    if (fl)
        atomicOr(flags, fl);
}

// Exclusive prefix of v over a workgroup of NT threads (NT a multiple of the
// wave size, at most 64 waves), with the workgroup's total.
template <int NT>
__device__ int block_exclusive_waves(int v, int *total)
{
    constexpr int NWV = NT / PC_WAVE;
    __shared__ int wsum[NWV];
    const int lane = threadIdx.x & (PC_WAVE - 1), wv = threadIdx.x / PC_WAVE;
    int x = v;
    for (int off = 1; off < PC_WAVE; off <<= 1) {
        const int t = __shfl_up(x, off, PC_WAVE);
        if (lane >= off)
            x += t;
    }
    if (lane == PC_WAVE - 1)
        wsum[wv] = x;
    __syncthreads();
    if (wv == 0) {
        int y = lane < NWV ? wsum[lane] : 0;
        for (int off = 1; off < NWV; off <<= 1) {
            const int t = __shfl_up(y, off, PC_WAVE);
            if (lane >= off)
                y += t;
        }
        if (lane < NWV)
            wsum[lane] = y;
    }
    __syncthreads();
    const int before = wv ? wsum[wv - 1] : 0;
    *total = wsum[NWV - 1];
    __syncthreads();
    return before + x - v;
}

// One point to its sorted place d: the float32 coordinates of the bulk
// sweep (x and y relative to the centre of the point's own column on 3-D
// grids, z relative to the domain origin, all scaled by g.fscale; z as fixed
// point on the float32 rp/pi path) and the binary64 values.
__device__ __forceinline__ void store_sorted(const pc_grid &g, const double4 &r, int cell,
                                             int64_t d, float *X, float *Y, float *Z,
                                             double *xd, double *yd, double *zd, double *wd,
                                             float4 *P)
{
    float fx, fy, fz;
    if (g.xy_local) {
        int ix, iy;
        cell_column(cell, g.n[0], g.n[1], g.n[2], &ix, &iy);
        fx = (float)((r.x - col_centre(g.lo[0], g.width[0], ix)) * g.fscale);
        fy = (float)((r.y - col_centre(g.lo[1], g.width[1], iy)) * g.fscale);
    } else {
        fx = (float)((r.x - g.lo[0]) * g.fscale);
        fy = (float)((r.y - g.lo[1]) * g.fscale);
    }
    if (g.zq_shift > 0)
        fz = __uint_as_float((uint32_t)llrint((r.z - g.lo[2]) * g.zq_inv) + PC_ZQ_BIAS);
    else
        fz = (float)((r.z - g.lo[2]) * g.fscale);
    // the expanded form's j points: x, y, z and |b|^2 = fl(y y + fl(x x)),
    // rounded as the sweep's bound assumes, side by side; its lanes read
    // binary64 x and y, and z from Z (the rp/pi lane its fixed-point z), so
    // X and Y are then not written
    if (P) {
        P[d] = make_float4(fx, fy, fz, __fmaf_rn(fy, fy, __fmul_rn(fx, fx)));
    } else {
        X[d] = fx;
        Y[d] = fy;
    }
    Z[d] = fz;
    xd[d] = r.x;
    yd[d] = r.y;
    zd[d] = r.z;
    if (wd)
        wd[d] = r.w;
}

// Level 2: one workgroup per column sorts the column's points by z slice
// (LDS counts and prefix) and writes the column's cell starts, the cell of
// every sorted place and `perm`, the column-ordered index of the point that
// goes there (k_gather then reads the records in sorted order).  The slice
// of a point is recomputed from its record with the same arithmetic as its
// cell in k_cell_hist (point_cell), so it is the same value.
constexpr int kSliceThreads = 1024;
constexpr int kSlicePer = 4;
// GIVEN: the placement already wrote the slices into rank_slice.
template <bool SKY, bool GIVEN>
__global__ __launch_bounds__(kSliceThreads) void k_slice_sort(
    int ncat, const int32_t *lay, int32_t ncolc, pc_grid g, const int32_t *__restrict__ woff,
    const double4 *__restrict__ colrec, int2 *__restrict__ rank_slice, int32_t *start,
    int32_t *__restrict__ perm, int32_t *__restrict__ cell_sorted)
{
    extern __shared__ unsigned sh[];
    const int nz = g.n[2];
    const int64_t colall = blockIdx.x;
    const int k = (int)(colall / ncolc), col = (int)(colall % ncolc);
    const int nw = lay[3 * k + 1], mb = lay[3 * k + 2];
    const int cs = woff[mb + (int64_t)col * nw];
    const int ce = woff[mb + (int64_t)(col + 1) * nw];
    const int64_t cell0 = colall * nz;
    for (int z = threadIdx.x; z < nz; z += blockDim.x)
        sh[z] = 0u;
    __syncthreads();
    unsigned fl = 0;   // (the flags were raised by k_cell_hist already)
    for (int base = cs + (int)threadIdx.x; base < ce; base += kSlicePer * kSliceThreads) {
        int sl[kSlicePer];
        if constexpr (GIVEN) {
#pragma unroll
            for (int p = 0; p < kSlicePer; p++) {
                const int q = base + p * kSliceThreads;
                sl[p] = rank_slice[q < ce ? q : cs].y;
            }
        } else {
            double4 r[kSlicePer];
#pragma unroll
            for (int p = 0; p < kSlicePer; p++) {
                const int q = base + p * kSliceThreads;
                r[p] = colrec[q < ce ? q : cs];
            }
#pragma unroll
            for (int p = 0; p < kSlicePer; p++) {
                const double c[3] = {r[p].x, r[p].y, r[p].z};
                sl[p] = point_cell<SKY>(g, c, fl).y;
            }
        }
#pragma unroll
        for (int p = 0; p < kSlicePer; p++) {
            const int q = base + p * kSliceThreads;
            if (q >= ce)
                break;
            rank_slice[q] = make_int2((int)atomicAdd(&sh[sl[p]], 1u), sl[p]);
        }
    }
    __syncthreads();
    int carry = 0;
    for (int base = 0; base < nz; base += kSliceThreads) {
        const int z = base + (int)threadIdx.x;
        const int v = z < nz ? (int)sh[z] : 0;
        int total;
        const int ex = block_exclusive_waves<kSliceThreads>(v, &total);
        if (z < nz)
            sh[z] = (unsigned)(carry + ex);
        carry += total;
        __syncthreads();
    }
    for (int z = threadIdx.x; z < nz; z += blockDim.x)
        start[cell0 + z] = cs + (int)sh[z];
    if (colall == (int64_t)ncat * ncolc - 1 && threadIdx.x == 0)
        start[cell0 + nz] = ce;
    for (int base = cs + (int)threadIdx.x; base < ce; base += kSlicePer * kSliceThreads) {
        int2 rs[kSlicePer];
#pragma unroll
        for (int p = 0; p < kSlicePer; p++) {
            const int q = base + p * kSliceThreads;
            rs[p] = rank_slice[q < ce ? q : cs];
        }
#pragma unroll
        for (int p = 0; p < kSlicePer; p++) {
            const int q = base + p * kSliceThreads;
            if (q >= ce)
                break;
            const int d = cs + (int)sh[rs[p].y] + rs[p].x;
            perm[d] = q;
            cell_sorted[d] = (int)(cell0 + rs[p].y);
        }
    }
}

// ---- scatter into per-cell contiguous structure-of-arrays ----------------
// Counting-sort placement in two steps.  Writing every column of a point to
// its sorted place would scatter eight small writes per point over the whole
// output; instead only the 4-byte source index goes to the sorted place
// (k_perm), and k_gather walks the sorted order, reads the point's columns
// (random reads, no partial-line writes) and writes every output column
// contiguously.
__global__ void k_perm(int64_t ntot, const int32_t *cell_of, const int32_t *rank_of,
                       const int32_t *start, int32_t *perm)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < ntot;
         i += (int64_t)gridDim.x * blockDim.x)
        perm[(int64_t)start[cell_of[i]] + rank_of[i]] = (int32_t)i;
}

// Workgroups are dealt round-robin to the 8 XCDs (workgroup b to XCD b % 8);
// the launch remaps b so that each XCD walks one contiguous eighth of the
// sorted order, and the records a column's places read (after the two-level
// sort: one column-ordered range) are fetched into one XCD's L2.
constexpr int kXcds = 8;
__global__ void k_gather(int64_t ntot, pc_grid g, const int32_t *perm, const int32_t *cell_of,
                         const double4 *rec, float *X, float *Y, float *Z, double *xd, double *yd,
                         double *zd, double *wd, float4 *P, int32_t *cell_sorted)
{
    const int per = (int)(gridDim.x / kXcds);   // gridDim.x is a multiple of kXcds
    const int lb = (int)(blockIdx.x % kXcds) * per + (int)(blockIdx.x / kXcds);
    for (int64_t d = lb * (int64_t)blockDim.x + threadIdx.x; d < ntot;
         d += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = perm[d];
        const double4 r = rec[i];
        const int cell = cell_of ? cell_of[i] : cell_sorted[d];
        store_sorted(g, r, cell, d, X, Y, Z, xd, yd, zd, wd, P);
        if (cell_of)
            cell_sorted[d] = cell;
    }
}

// ---- blocks of up to 64 points per column --------------------------------
__global__ void k_block_count(int32_t ncol, int32_t nz, const int32_t *start, int32_t *bcnt)
{
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < ncol; c += gridDim.x * blockDim.x) {
        const int a = start[(int64_t)c * nz], b = start[(int64_t)(c + 1) * nz];
        bcnt[c] = (b - a + PC_BLOCK_I - 1) / PC_BLOCK_I;
    }
}

__global__ void k_block_emit(int32_t ncol, int32_t nz, const int32_t *start,
                             const int32_t *boff, pc_block *blocks)
{
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < ncol; c += gridDim.x * blockDim.x) {
        const int a = start[(int64_t)c * nz], b = start[(int64_t)(c + 1) * nz];
        int o = boff[c];
        for (int i0 = a; i0 < b; i0 += PC_BLOCK_I, o++) {
            pc_block blk;
            blk.col = c;
            blk.i0 = i0;
            blk.ni = min(PC_BLOCK_I, b - i0);
            blk.pad = 0;
            blocks[o] = blk;
        }
    }
}

// ---- segments of one block ------------------------------------------------
struct SegCtx {
    pc_grid g;
    const int32_t *start2;
    const int32_t *cell1_sorted;
    int autocorr;
};

// Calls f(j0, j1, dcode, tri) for every run of second-catalogue points the
// block must be paired with.  dcode packs the periodic offset codes
// (x | y << 2 | z << 4).
//
// Autocorrelation visits each unordered pair once: the block's own column
// forward along the sorted order (the triangle j > i inside the block, then
// later points up to zreach slices beyond the block's last slice, then the
// periodic wrap past the top face), and the forward half of the column
// offsets within xyk ((0, +1..), then (+1.., any)), each over its z window.
// Cross-correlation visits all (2 xyk + 1)^2 columns.  With 2 xyk + 1 columns
// or more on a periodic axis every offset names a distinct column, so the
// forward half meets each pair of columns once.
// Angular grid: the block's own cell and the right-ascension cells of its
// own and the two neighbouring declination bands that come within the
// right-ascension reach of the block's cell (its east and west edges
// projected onto the target band, widened by the reach, then every target
// cell met, each once even where the range wraps round).  Declination slices
// outside zreach of the block's slices are skipped.  Autocorrelation visits
// only cells after the block's own (a cell pair from its lower-numbered
// cell), and the own cell forward along the sorted order.
template <class F>
__device__ void sky_segments(const SegCtx &c, const pc_block &b, F &&f)
{
    const int S = c.g.n[2], zr = c.g.zreach, nband = c.g.nband;
    const int ncolc = c.g.n[1];
    const int lcol = b.col % ncolc;
    const int cbase = b.col - lcol;
    int band = 0, hi = nband - 1;   // the last band whose first column is <= lcol
    while (band < hi) {
        const int mid = (band + hi + 1) >> 1;
        if (c.g.bands[mid].col0 <= lcol)
            band = mid;
        else
            hi = mid - 1;
    }
    const pc_band &B = c.g.bands[band];
    const int a = lcol - B.col0;
    const int sa = c.cell1_sorted[b.i0] % S;
    const int sb = c.cell1_sorted[b.i0 + b.ni - 1] % S;
    if (c.autocorr) {
        if (b.ni > 1)
            f(b.i0 + 1, b.i0 + b.ni, 0u, 1);
        const int jend = c.start2[(int64_t)b.col * S + min(sb + zr, S - 1) + 1];
        if (jend > b.i0 + b.ni)
            f(b.i0 + b.ni, jend, 0u, 0);
    }
    for (int d = c.autocorr ? 0 : -1; d <= 1; d++) {
        const int b2 = band + d;
        if (b2 < 0 || b2 >= nband)
            continue;
        const int a0 = max(sa - zr - d * S, 0), a1 = min(sb + zr - d * S, S - 1);
        if (a0 > a1)
            continue;
        const pc_band &C = c.g.bands[b2];
        const double D = d < 0 ? B.dra[0] : (d == 0 ? B.dra[1] : B.dra[2]);
        int k0 = 0, k1 = C.nra - 1;
        if (D < M_PI) {
            const double x0 = ((double)a / B.ra_scale - D) * C.ra_scale;
            const double x1 = ((double)(a + 1) / B.ra_scale + D) * C.ra_scale;
            const int f0 = (int)floor(x0), f1 = (int)floor(x1);
            if (f1 - f0 + 1 < C.nra) {
                k0 = f0;
                k1 = f1;
            }
        }
        for (int k = k0; k <= k1; k++) {
            int a2 = k % C.nra;
            if (a2 < 0)
                a2 += C.nra;
            const int col2 = cbase + C.col0 + a2;
            if (c.autocorr && col2 <= b.col)
                continue;
            const int64_t base = (int64_t)col2 * S;
            f(c.start2[base + a0], c.start2[base + a1 + 1], 0u, 0);
        }
    }
}

// KX > 0: the x/y refinement is KX (a compile-time constant, so the loops
// over neighbour columns unroll and their cell-start loads are in flight
// together); 0: read it from the grid.
template <int KX, class F>
__device__ __forceinline__ void grid_segments(const SegCtx &c, const pc_block &b, F &&f)
{
    const int nx = c.g.n[0], ny = c.g.n[1], nz = c.g.n[2];
    // columns are numbered across catalogues: catalogue k owns columns
    // k * nx * ny ..; neighbours stay inside the block's own catalogue
    const int lcol = b.col % (nx * ny);
    const int cbase = b.col - lcol;
    const int ix = lcol / ny, iy = lcol % ny;
    const int sa = c.cell1_sorted[b.i0] % nz;
    const int sb = c.cell1_sorted[b.i0 + b.ni - 1] % nz;
    const int zr = c.g.zreach;
    const bool per = c.g.periodic != 0;

    auto zwin = [&](int ccol, unsigned dxy, int zw) {
        const int64_t base = (int64_t)ccol * nz;
        const int lo_s = sa - zw, hi_s = sb + zw;
        const int a0 = max(lo_s, 0), a1 = min(hi_s, nz - 1);
        if (a0 <= a1)
            f(c.start2[base + a0], c.start2[base + a1 + 1], dxy, 0);
        if (per) {
            if (lo_s < 0) {
                const int w0 = max(lo_s + nz, 0);
                f(c.start2[base + w0], c.start2[base + nz], dxy | (PC_D_PLUS << 4), 0);
            }
            if (hi_s >= nz) {
                const int w1 = min(hi_s - nz, nz - 1);
                f(c.start2[base], c.start2[base + w1 + 1], dxy | (PC_D_MINUS << 4), 0);
            }
        }
    };
    auto column = [&](int ox, int oy) {
        const int zw = c.g.zro[ox < 0 ? -ox : ox][oy < 0 ? -oy : oy];
        if (zw < 0)
            return;
        int jx = ix + ox, jy = iy + oy;
        unsigned code = 0;
        if (jx < 0 || jx >= nx) {
            if (!per)
                return;
            code |= (jx < 0) ? PC_D_PLUS : PC_D_MINUS;
            jx = (jx < 0) ? jx + nx : jx - nx;
        }
        if (jy < 0 || jy >= ny) {
            if (!per)
                return;
            code |= ((jy < 0) ? PC_D_PLUS : PC_D_MINUS) << 2;
            jy = (jy < 0) ? jy + ny : jy - ny;
        }
        zwin(cbase + jx * ny + jy, code, zw);
    };

    const int k = KX > 0 ? KX : c.g.xyk;
    if (c.autocorr) {
        // the block against itself (its triangle, j < i0 + ni) and its column
        // forward up to the reach: one contiguous segment flagged as holding
        // the triangle (the sweep masks only the chunks that reach into it)
        const int64_t base = (int64_t)b.col * nz;
        const int hi_s = sb + zr;
        const int jend = max(c.start2[base + min(hi_s, nz - 1) + 1], b.i0 + b.ni);
        if (jend > b.i0 + 1)
            f(b.i0 + 1, jend, 0u, 1);
        if (per && hi_s >= nz) {
            const int w1 = min(hi_s - nz, nz - 1);
            f(c.start2[base], c.start2[base + w1 + 1], PC_D_MINUS << 4, 0);
        }
        // the forward half of the offsets: (0, 1..k), then (1..k, -k..k)
        for (int oy = 1; oy <= k; oy++)
            column(0, oy);
        for (int ox = 1; ox <= k; ox++)
            for (int oy = -k; oy <= k; oy++)
                column(ox, oy);
    } else {
        for (int ox = -k; ox <= k; ox++)
            for (int oy = -k; oy <= k; oy++)
                column(ox, oy);
    }
}

template <bool SKY, class F>
__device__ void for_each_segment(const SegCtx &c, const pc_block &b, F &&f)
{
    if constexpr (SKY) {
        sky_segments(c, b, f);
    } else {
        if (c.g.xyk == 1)
            grid_segments<1>(c, b, f);
        else
            grid_segments<0>(c, b, f);
    }
}

template <bool SKY>
__global__ void k_item_count(int32_t nblocks, const int32_t *nblocks_dev,
                             const pc_block *blocks, SegCtx c, int chunk, int32_t *icnt,
                             unsigned long long *cand)
{
    const int nb = nblocks_dev ? *nblocks_dev : nblocks;
    unsigned long long my = 0;
    for (int bi = blockIdx.x * blockDim.x + threadIdx.x; bi < nb;
         bi += gridDim.x * blockDim.x) {
        const pc_block b = blocks[bi];
        int total = 0;
        for_each_segment<SKY>(c, b, [&](int j0, int j1, unsigned, int tri) {
            if (j1 <= j0)
                return;
            total += (j1 - j0 + chunk - 1) / chunk;
            // a triangle segment: the block's unique pairs with itself, then
            // every j beyond the block (j1 >= i0 + ni)
            my += tri ? (unsigned long long)b.ni * (b.ni - 1) / 2 +
                            (unsigned long long)b.ni * (unsigned long long)(j1 - b.i0 - b.ni)
                      : (unsigned long long)b.ni * (unsigned long long)(j1 - j0);
        });
        icnt[bi] = total;
    }
    // one atomic per wave: a per-thread add to the one counter serialises
    // every block of the work list at one L2 address
    for (int off = PC_WAVE / 2; off > 0; off >>= 1)
        my += __shfl_xor(my, off);
    if ((threadIdx.x & (PC_WAVE - 1)) == 0 && my)
        atomicAdd(cand, my);
}

// Items beyond `cap` are not written; the flag PC_FLAG_ITEMS reports them
// (a replayed call whose inputs now need more items than it was built for).
template <bool SKY>
__global__ void k_item_emit(int32_t nblocks, const int32_t *nblocks_dev, const pc_block *blocks,
                            SegCtx c, int chunk, const int32_t *ioff, pc_item *items, int32_t cap,
                            unsigned *flags, const int32_t *cs2, int32_t *icell)
{
    const int nb = nblocks_dev ? *nblocks_dev : nblocks;
    for (int bi = blockIdx.x * blockDim.x + threadIdx.x; bi < nb;
         bi += gridDim.x * blockDim.x) {
        const pc_block b = blocks[bi];
        const int cat = b.col / (c.g.n[0] * c.g.n[1]);
        int o = ioff[bi];
        for_each_segment<SKY>(c, b, [&](int j0, int j1, unsigned dcode, int tri) {
            for (int j = j0; j < j1; j += chunk) {
                pc_item it;
                it.i0 = b.i0;
                it.j0 = j;
                it.j1 = min(j + chunk, j1);
                it.meta = (unsigned)(b.ni - 1) | (dcode << 6) | ((unsigned)tri << 12) |
                          ((unsigned)cat << 13);
                if (o < cap) {
                    items[o] = it;
                    if (icell)
                        icell[o] = cs2[j];
                }
                o++;
            }
        });
        if (o > cap)
            atomicOr(flags, PC_FLAG_ITEMS);
    }
}

// ---- lookup table of the decision bands -------------------------------------
// One thread per table cell [c_lo, c_hi]: linear cells [k, k + 1) (the last
// cell takes everything above) or float-bit cells of the binary64 path (the
// extra last cell is "above every edge").  Entry = number of bands wholly
// below the cell (the histogram row), flagged when one band (flag | edge) or
// several bands meet the cell; with out_zero, cells wholly above every edge
// hold 0 like those below.  Band tops hi[] never decrease when `ordered`; the
// scan over meeting bands stops once every later band starts above the cell
// (lo_min is the suffix minimum of lo).
__global__ void k_build_table(pc_bins B, int nedges, const float *lo, const float *hi,
                              const float *lo_min, void *tbl)
{
    const bool wide = B.tbl_wide != 0;
    for (int key = blockIdx.x * blockDim.x + threadIdx.x; key < B.tbl_n;
         key += gridDim.x * blockDim.x) {
        unsigned e;
        if (!B.tbl_linear && key == B.tbl_n - 1) {
            e = B.tbl_out_zero ? 0u : (unsigned)nedges;
        } else {
            float c_lo, c_hi;
            if (B.tbl_linear == 2) {
                // values whose rounded key is `key`: (key -+ 1/2) / 32767, the
                // bounds widened outward by a float32 ulp (the conversion
                // rounds the exact product, and no float32 value gives an
                // exact tie); the last cell takes everything above
                const double q = 1.0 / 32767.0;
                c_lo = key == 0 ? 0.0f : nextafterf((float)(((double)key - 0.5) * q), 0.0f);
                c_hi = key + 1 < B.tbl_n
                           ? nextafterf((float)(((double)key + 0.5) * q), INFINITY)
                           : INFINITY;
            } else if (B.tbl_linear) {
                c_lo = (float)key;
                c_hi = key + 1 < B.tbl_n ? nextafterf((float)(key + 1), 0.0f) : INFINITY;
            } else {
                const unsigned cell0 = B.tbl_base + ((unsigned)key << B.tbl_shift);
                const unsigned lo_b = key == 0 ? 0u : cell0;
                const unsigned hi_b = cell0 + ((1u << B.tbl_shift) - 1u);
                c_lo = __uint_as_float(lo_b);
                c_hi = __uint_as_float(min(hi_b, 0x7f7fffffu));
            }
            int below = 0, inter = 0, which = -1;
            if (B.tbl_ordered) {
                int a = 0, b = nedges;   // first band with hi >= c_lo
                while (a < b) {
                    const int m = (a + b) >> 1;
                    if (hi[m] < c_lo)
                        a = m + 1;
                    else
                        b = m;
                }
                below = a;
                for (int k = a; k < nedges && lo_min[k] <= c_hi; k++)
                    if (lo[k] <= c_hi) {
                        inter++;
                        which = k;
                    }
            } else {
                for (int k = 0; k < nedges; k++) {
                    if (hi[k] < c_lo)
                        below++;
                    else if (lo[k] <= c_hi) {
                        inter++;
                        which = k;
                    }
                }
            }
            if (B.tbl_out_zero && inter == 0 && below == nedges)
                below = 0;
            if (inter == 0)
                e = (unsigned)below;
            else if (inter == 1 && which == below)
                e = (unsigned)below | (wide ? PC_TBL_BAND : PC_TBL8_BAND);
            else
                e = wide ? PC_TBL_MULTI : PC_TBL8_MULTI;
        }
        if (wide)
            static_cast<uint16_t *>(tbl)[key] = (uint16_t)e;
        else
            static_cast<uint8_t *>(tbl)[key] = (uint8_t)e;
    }
}

}  // namespace

hipError_t launch_zero_multi(hipStream_t s, int count, void *const *ptrs, const size_t *bytes)
{
    if (count < 1 || count > PC_ZERO_MAX)
        return hipErrorInvalidValue;
    ZeroSet z;
    int64_t most = 0;
    for (int k = 0; k < count; k++) {
        z.p[k] = static_cast<uint32_t *>(ptrs[k]);
        z.n[k] = (int64_t)(bytes[k] / 4);
        most = std::max(most, z.n[k]);
    }
    if (most <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_zero_multi, dim3(grid_for(most, kThreads, 512), count), dim3(kThreads),
                       0, s, z);
    return hipGetLastError();
}

hipError_t launch_zero(hipStream_t s, void *p, size_t bytes)
{
    const int64_t n = (int64_t)(bytes / 4);
    if (n <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_zero, dim3(grid_for(n, kThreads, 2048)), dim3(kThreads), 0, s,
                       static_cast<uint32_t *>(p), n);
    return hipGetLastError();
}

hipError_t launch_radec(hipStream_t s, int64_t n, const void *ra, const void *dec,
                        const void *dist, int f32, double d2r, double *x, double *y, double *z,
                        unsigned *flags)
{
    hipLaunchKernelGGL(k_radec, dim3(grid_for(n)), dim3(kThreads), 0, s, n, ra, dec, dist, f32,
                       d2r, x, y, z, flags);
    return hipGetLastError();
}

hipError_t launch_minmax(hipStream_t s, int64_t n, const void *x, const void *y, const void *z,
                         int f32, double *part, int nparts, unsigned *flags)
{
    hipLaunchKernelGGL(k_minmax, dim3(nparts), dim3(kThreads), 0, s, n, x, y, z, f32, part,
                       flags);
    return hipGetLastError();
}

hipError_t launch_minmax_final(hipStream_t s, const double *part, int nparts, double *out6)
{
    hipLaunchKernelGGL(k_minmax_final, dim3(1), dim3(64), 0, s, part, nparts, out6);
    return hipGetLastError();
}

hipError_t launch_cell_index(hipStream_t s, int ncat, const pc_cat *cats, int64_t ntot,
                             const pc_grid &g, unsigned *cnt, int32_t *cell_of, int32_t *rank_of,
                             void *rec, unsigned *flags)
{
    hipLaunchKernelGGL(g.nband > 0 ? k_cell_index<true> : k_cell_index<false>,
                       dim3(grid_for(ntot)), dim3(kThreads), 0, s, ncat, cats, ntot, g, cnt, cell_of, rank_of, static_cast<double4 *>(rec), flags);
    return hipGetLastError();
}

size_t scan_tmp_elems(int64_t n)
{
    size_t total = 0;
    while (n > kScanBlock) {
        const int64_t nb = (n + kScanBlock - 1) / kScanBlock;
        total += (size_t)nb + (size_t)nb + 1;
        n = nb;
    }
    return total + 1;
}

hipError_t scan_exclusive(hipStream_t s, const int32_t *in, int64_t n, int32_t *out,
                          int32_t *tmp)
{
    if (n <= kScanBlock) {
        hipLaunchKernelGGL(k_scan_apply, dim3(1), dim3(kThreads), 0, s, in, n,
                           (const int32_t *)nullptr, out);
        return hipGetLastError();
    }
    const int64_t nb = (n + kScanBlock - 1) / kScanBlock;
    int32_t *part = tmp;
    int32_t *part_scan = tmp + nb;
    hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)nb), dim3(kThreads), 0, s, in, n, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    if (nb <= kScanPartsInline) {
        // each block sums the totals before it itself: no scan of the totals
        hipLaunchKernelGGL(k_scan_apply_parts, dim3((unsigned)nb), dim3(kThreads), 0, s, in, n,
                           (const int32_t *)part, out);
        return hipGetLastError();
    }
    e = scan_exclusive(s, part, nb, part_scan, tmp + 2 * nb + 1);
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)nb), dim3(kThreads), 0, s, in, n,
                       (const int32_t *)part_scan, out);
    return hipGetLastError();
}

hipError_t launch_scatter(hipStream_t s, int64_t ntot, const pc_grid &g, const int32_t *cell_of,
                          const int32_t *rank_of, const void *rec, const int32_t *start,
                          int32_t *perm, float *X, float *Y, float *Z, double *xd, double *yd,
                          double *zd, double *wd, float4 *P, int32_t *cell_sorted)
{
    hipLaunchKernelGGL(k_perm, dim3(grid_for(ntot)), dim3(kThreads), 0, s, ntot, cell_of, rank_of,
                       start, perm);
    return launch_gather(s, ntot, g, perm, cell_of, rec, X, Y, Z, xd, yd, zd, wd, P, cell_sorted);
}

hipError_t launch_gather(hipStream_t s, int64_t ntot, const pc_grid &g, const int32_t *perm,
                         const int32_t *cell_of, const void *rec, float *X, float *Y, float *Z,
                         double *xd, double *yd, double *zd, double *wd, float4 *P,
                         int32_t *cell_sorted)
{
    const int gw = (grid_for(ntot) + kXcds - 1) / kXcds * kXcds;
    hipLaunchKernelGGL(k_gather, dim3(gw), dim3(kThreads), 0, s, ntot, g, perm,
                       cell_of, static_cast<const double4 *>(rec), X, Y, Z, xd, yd, zd, wd, P,
                       cell_sorted);
    return hipGetLastError();
}

hipError_t launch_sort2(hipStream_t s, int ncat, const pc_cat *cats, int64_t ntot,
                        const pc_grid &g, int32_t chunk, int32_t ncolc, int32_t n_chunks,
                        int64_t m, int32_t *lay, int32_t *wcnt, int32_t *woff, int32_t *tmp,
                        int32_t *cell_of, int32_t *rank_of, void *colrec, void *rank_slice,
                        int32_t *perm, int32_t *start, int32_t *cell_sorted, float *X, float *Y,
                        float *Z, double *xd, double *yd, double *zd, double *wd, float4 *P,
                        unsigned *flags)
{
    double4 *cr = static_cast<double4 *>(colrec);
    hipLaunchKernelGGL(k_grid_layout, dim3(1), dim3(64), 0, s, ncat, cats, chunk, ncolc, lay);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    if (n_chunks > 0)
        hipLaunchKernelGGL(g.nband > 0 ? k_cell_hist<true> : k_cell_hist<false>,
                           dim3((unsigned)n_chunks), dim3(kThreads),
                           sizeof(unsigned) * (size_t)ncolc, s, ncat, cats, lay, g, chunk, ncolc,
                           cell_of, rank_of, wcnt, flags);
    if ((e = hipGetLastError()) != hipSuccess)
        return e;
    if ((e = scan_exclusive(s, wcnt, m, woff, tmp)) != hipSuccess)
        return e;
    const bool local = ntot > 0 && chunk == kLocalChunk && ncolc <= kThreads && n_chunks > 0;
    int2 *rs = static_cast<int2 *>(rank_slice);
    if (local)
        hipLaunchKernelGGL(g.nband > 0 ? k_col_scatter_local<true> : k_col_scatter_local<false>,
                           dim3((unsigned)n_chunks), dim3(kThreads), 0, s, ncat, cats, lay, g,
                           ncolc, cell_of, rank_of, wcnt, woff, cr, rs, flags);
    else if (ntot > 0)
        hipLaunchKernelGGL(k_col_scatter, dim3(grid_for(ntot)), dim3(kThreads), 0, s, ntot, ncat,
                           cats, lay, g.n[2], chunk, ncolc, cell_of, rank_of, woff, cr, flags);
    if ((e = hipGetLastError()) != hipSuccess)
        return e;
    hipLaunchKernelGGL(g.nband > 0 ? (local ? k_slice_sort<true, true> : k_slice_sort<true, false>)
                                   : (local ? k_slice_sort<false, true>
                                            : k_slice_sort<false, false>),
                       dim3((unsigned)((int64_t)ncat * ncolc)), dim3(kSliceThreads),
                       sizeof(unsigned) * (size_t)g.n[2], s, ncat, lay, ncolc, g, woff, cr,
                       static_cast<int2 *>(rank_slice), start, perm, cell_sorted);
    if ((e = hipGetLastError()) != hipSuccess)
        return e;
    return launch_gather(s, ntot, g, perm, nullptr, colrec, X, Y, Z, xd, yd, zd, wd, P,
                         cell_sorted);
}

hipError_t launch_block_count(hipStream_t s, int32_t ncol, int32_t nz, const int32_t *start,
                              int32_t *bcnt)
{
    hipLaunchKernelGGL(k_block_count, dim3(grid_for(ncol)), dim3(kThreads), 0, s, ncol, nz,
                       start, bcnt);
    return hipGetLastError();
}

hipError_t launch_block_emit(hipStream_t s, int32_t ncol, int32_t nz, const int32_t *start,
                             const int32_t *boff, pc_block *blocks)
{
    hipLaunchKernelGGL(k_block_emit, dim3(grid_for(ncol, 64)), dim3(64), 0, s, ncol, nz, start,
                       boff, blocks);
    return hipGetLastError();
}

hipError_t launch_item_count(hipStream_t s, int32_t nblocks, const int32_t *nblocks_dev,
                             const pc_block *blocks, const pc_grid &g, const int32_t *start2,
                             const int32_t *cell1_sorted, int autocorr, int chunk,
                             int32_t *icnt, unsigned long long *cand)
{
    SegCtx c{g, start2, cell1_sorted, autocorr};
    hipLaunchKernelGGL(g.nband > 0 ? k_item_count<true> : k_item_count<false>,
                       dim3(grid_for(nblocks, 128)), dim3(128), 0, s, nblocks,
                       nblocks_dev, blocks, c, chunk, icnt, cand);
    return hipGetLastError();
}

hipError_t launch_item_emit(hipStream_t s, int32_t nblocks, const int32_t *nblocks_dev,
                            const pc_block *blocks, const pc_grid &g, const int32_t *start2,
                            const int32_t *cell1_sorted, int autocorr, int chunk,
                            const int32_t *ioff, pc_item *items, int32_t cap, unsigned *flags,
                            const int32_t *cell2_sorted, int32_t *icell)
{
    SegCtx c{g, start2, cell1_sorted, autocorr};
    hipLaunchKernelGGL(g.nband > 0 ? k_item_emit<true> : k_item_emit<false>,
                       dim3(grid_for(nblocks, 128)), dim3(128), 0, s, nblocks,
                       nblocks_dev, blocks, c, chunk, ioff, items, cap, flags, cell2_sorted,
                       icell);
    return hipGetLastError();
}

hipError_t launch_build_table(hipStream_t s, const pc_bins &B, int nedges, const float *lo,
                              const float *hi, const float *lo_min, void *tbl)
{
    hipLaunchKernelGGL(k_build_table, dim3(grid_for(B.tbl_n)), dim3(kThreads), 0, s, B, nedges,
                       lo, hi, lo_min, tbl);
    return hipGetLastError();
}

}  // namespace pc
