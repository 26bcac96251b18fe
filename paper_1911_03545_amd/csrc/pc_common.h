// pc_common.h -- layouts shared by the host planner and the gfx950 kernels.
#pragma once
#include <stdint.h>

#define PC_WAVE 64
#define PC_BLOCK_I 64          // i points per work item: one per lane
#ifndef PC_TBL8_MAX
#define PC_TBL8_MAX 40960      // byte lookup-table entries (up to 125 bins)
#endif
#ifndef PC_TBL16_MAX
#define PC_TBL16_MAX 20480     // 16-bit lookup-table entries (more bins)
#endif
#define PC_TBL8_MAX_BINS 125
// cells of the float32 path's rounding-key table: key = round(s * 32767) for
// a scaled s in [0, 1] (one v_cvt_pknorm_i16_f32: clamp, scale, round to
// nearest); used with byte entries by the shared-histogram sweeps
#define PC_TBL_PK_CELLS 32768
// lookup-table bytes of the private-histogram (batched) sweep
#define PC_TBL_PRIV_BYTES 16384
// The sweep's work items are dealt to PC_STREAMS streams (contiguous item
// ranges), each with its own counter PC_STREAM_STRIDE ints apart, so that
// item fetches spread over many addresses instead of serialising on one.
#define PC_STREAMS 64
#define PC_STREAM_STRIDE 64
#define PC_MAX_EDGES 1025      // r / rp / theta edges
#define PC_MAX_NPI 1024
#define PC_MAX_BINS_TOTAL 4096 // r bins, or nrp * npi
#define PC_MAX_HIST_WAVE 4096  // uint32 LDS counters per wave (bins * copies)
// fixed device scratch of the no-allocation entry point (per GPU), and the
// devices whose scratch address the library can keep
#define PC_NOALLOC_SCRATCH_BYTES (128ull << 20)
#define PC_NOALLOC_MAX_DEVICES 64

// Lookup-table entries.  A plain entry is the histogram slot of every value
// in the table cell: the number of edges whose band lies wholly below the
// cell (bin + 1; 0 and nb + 1 mean out of range).  16-bit entries flag a cell
// met by exactly one band with PC_TBL_BAND | edge, by several bands with
// PC_TBL_MULTI; byte entries use 0x80 | edge and 0xFF.
#define PC_TBL_BAND 0x8000u
#define PC_TBL_MULTI 0x4000u
#define PC_TBL_MASK 0x3FFFu
#define PC_TBL8_BAND 0x80u
#define PC_TBL8_MULTI 0xFFu
#define PC_TBL8_MASK 0x7Fu

// Periodic offset codes, two bits per axis: 0 -> 0, 1 -> +L, 2 -> -L.
#define PC_D_ZERO 0u
#define PC_D_PLUS 1u
#define PC_D_MINUS 2u

// R: 3-D r (and theta as chords); RPPI: rp and pi with z as the line of
// sight; MOCKS: rp and pi with the line of sight through the pair midpoint
enum { PC_METRIC_R = 0, PC_METRIC_RPPI = 1, PC_METRIC_MOCKS = 2 };

// A declination band of the angular grid: its right-ascension cells are the
// columns col0 .. col0 + nra - 1, each 2 pi / nra wide.  dra[d] bounds the
// right-ascension difference (radians, taken round the circle) of two unit
// vectors within the angular reach when one lies in this band and the other
// in band b - 1 + d; a value >= pi means any difference.
struct pc_band {
    int32_t col0;
    int32_t nra;
    double ra_scale;   // nra / (2 pi)
    double dra[3];
};

#define PC_MAX_XYK 4
#define PC_MAX_BANDS 1024
#define PC_MAX_RA 4096
#define PC_MAX_SKY_COLS (1 << 20)

// Cell grid: x/y columns of width >= the transverse reach, z slices.
// Cell id = (ix * ny + iy) * nz + iz, so columns are contiguous runs of cells
// ordered by z.
//
// The angular grid (nband > 0, unit vectors only) keeps this layout with
// n = {1, columns, slices per band}: a column is one right-ascension cell of
// one declination band, and a slice a declination interval inside the band.
struct pc_grid {
    double lo[3];
    double extent[3];
    double inv_w[3];
    double width[3];
    int32_t n[3];
    int32_t zreach;
    int32_t periodic;
    int32_t zq_shift;    // > 0: float32 rp/pi path stores z as fixed point (below)
    double boxsize;
    int64_t ncell;
    double fscale;       // scale applied to the float32 coordinates
    // fixed-point z of the float32 rp/pi path: Zq = round((z - lo_z) * zq_inv)
    // + 2^30 as uint32 bits, one pi bin = 2^zq_shift quanta
    double zq_inv;
    // x/y refinement: columns at least reach / xyk wide, so a pair within
    // the reach is at most xyk columns apart per axis; zro[|ox|][|oy|] is the
    // z window (slices each side) of the column at that offset, narrowed by
    // the offset's smallest transverse distance when the reach is a 3-D
    // ball, -1 where no pair of the two columns can be within reach
    int32_t xyk;
    int16_t zro[PC_MAX_XYK + 1][PC_MAX_XYK + 1];
    // float32 path on a 3-D grid: x and y stored relative to the centre of
    // each point's column (column-local frames), else relative to lo
    int32_t xy_local;
    // angular grid: declination bands of nband * n[2] slices, slice index
    // floor((dec - dec_lo) * inv_hs); bands is a device table of nband entries
    int32_t nband;
    double dec_lo;
    double inv_hs;
    double sky_reach;   // angular reach with its margins (radians)
    const pc_band *bands;
};

// A block: up to 64 consecutive sorted points of one column (one per lane).
struct pc_block {
    int32_t col;
    int32_t i0;
    int32_t ni;
    int32_t pad;
};

// A work item: the block's points i0 .. i0+ni-1 against sorted points
// j0 .. j1-1 of the second catalogue, with one periodic offset.
struct pc_item {
    int32_t i0;
    int32_t j0;
    int32_t j1;
    uint32_t meta;   // [0,6) ni-1, [6,12) offset codes x|y<<2|z<<4, [12] triangle
};
#define PC_META_NI(m) (((m) & 63u) + 1)
#define PC_META_DCODE(m) (((m) >> 6) & 63u)
#define PC_META_TRI(m) (((m) >> 12) & 1u)
#define PC_META_CAT(m) ((m) >> 13)
#define PC_MAX_CATS (1 << 19)

// One catalogue of a (possibly batched) side, as seen by the device kernels:
// device pointers of its columns, its size and its first index in the
// concatenation of the side's catalogues.
struct pc_cat {
    const void *x, *y, *z, *w;
    int64_t n;
    int64_t off;
    int32_t f32, wf32;
};

// Bin description uploaded once per call; float bands are [lo_k, hi_k].
struct pc_bins {
    int32_t nb;          // r / rp bins
    int32_t npi;         // pi bins (1 for r and theta)
    int32_t tbl_shift;   // key = sat(float_bits(s) - tbl_base) >> tbl_shift
    int32_t tbl_n;       // used table entries
    int32_t e0_zero;     // first r / rp edge is exactly zero
    int32_t tbl_wide;    // 0: byte entries, 1: 16-bit entries
    uint32_t tbl_base;   // float bit pattern subtracted before the shift
    int32_t fscale_log2; // unused (0)
    float s_top;         // float32 prefilter: candidate only if s32 <= s_top
    float pi_top;        // rppi: candidate only if pi32 <= pi_top
    float inv_dpi;       // rppi: npi / pimax in float32
    float pi_tau;        // rppi: margin of the fractional part of |dz| * inv_dpi
    double E_top;        // binary64 cut: s64 < E_top
    double pimax;        // binary64 cut: pi64 < pimax
    // histogram slot of (row, col) = row * row_w + col: row = rp bin + 1
    // (0 and nb + 1 out of range), col = pi bin + col0; r: row_w 1, col0 0;
    // rppi: row_w npi + 2, col0 1 (columns 0 and npi + 1 out of range)
    int32_t row_w;
    int32_t col0;
    // lookup-table construction (done on the device): 1: linear cells
    // [k, k+1) (float32 path, key = floor(min(s, cells - 1))); 2: rounding
    // cells [(k - 1/2) / 32767, (k + 1/2) / 32767) (float32 path, key =
    // round(min(s, 1) * 32767)); 0: float-bit cells (binary64 path);
    // out_zero: cells wholly out of range hold 0; ordered: band tops never
    // decrease
    int32_t tbl_linear;
    int32_t tbl_out_zero;
    int32_t tbl_ordered;
    // rp/pi float32 path with fixed-point z (zq_shift > 0): pi bin =
    // |dq| >> zq_shift, undecided within PC_ZQ_MARGIN quanta of a bin edge;
    // zq_L is the periodic length in quanta (the per-item z offset)
    int32_t zq_shift;
    uint32_t zq_L;
    int32_t pad3;
};
#define PC_ZQ_MARGIN 2
#define PC_ZQ_BIAS 0x40000000u

// Offsets (bytes) of the arrays packed after pc_bins in one device buffer.
struct pc_bins_layout {
    size_t lo, hi, lo_min, E, plo, phi, q, tbl, total;
};
