// pc_sweep.hip -- the pair sweep, the binary64 recheck and the finalize step.
//
// The sweep evaluates the loop body of Code 1 for every pair of a work item:
// the separation (Appendix A; the periodic offset is applied once per work
// item as in Code 4 instead of a per-pair wrap), the squared-edge bin search
// (section "Finding and updating the histogram bins") and the histogram
// update into a wave-private LDS histogram merged into global uint64 bins
// (the thread-private histograms of the OpenMP section, one per wavefront).
//
// Execution model: persistent workgroups of four independent wavefronts.
// Each wavefront pulls work items from a global counter; lane l holds point
// i0 + l of the item's block in registers while the second catalogue's points
// j0 .. j1-1 arrive as wave-uniform scalar loads, so each VALU instruction
// evaluates 64 pairs that share one j.
//
// Bin search: an LDS lookup table keyed by the squared separation gives, for
// most values, the histogram slot directly: slot = bin + 1, with slot 0 and
// slot nb + 1 catching separations below the first and above the last edge.
// Keys: the float bit pattern (monotone for non-negative values) on the
// binary64 path; on the float32 path round(min(s, 1) * 32767) (one
// v_cvt_pknorm_i16_f32) or the linear floor(min(s, cells - 1)) of the
// private-histogram and 16-bit tables.  Table cells that meet an edge's
// decision band are flagged and resolved on a rare slow path.
//
// Two precisions:
//  * binary64: dx = fl(x_i - x_j) (+ offset), s = ((dx*dx + dy*dy) + dz*dz),
//    one rounding per operation -- the definition itself; flagged cells are
//    resolved by an exact binary64 comparison with the edge.
//  * float32: differences of float32 coordinates (x and y in the frame of
//    the item's j column on 3-D grids, pc_frame.h) and fused multiply-adds; a
//    value inside an edge's proven error band is not decided in float32 but
//    re-evaluated from the binary64 coordinates inline (exact_slot).
#include <hip/hip_runtime.h>

#include "pc_common.h"
#include "pc_fixed.h"
#include "pc_frame.h"
#include "pc_launch.h"

namespace pc {
namespace {

// LDS (address space 3) and read-only, wave-uniform global data read through
// the scalar cache (address space 4).
#define LDS __attribute__((address_space(3)))
#define KCONST __attribute__((address_space(4)))
typedef const LDS float *lds_f32p;
typedef const LDS double *lds_f64p;
typedef LDS unsigned *lds_u32p;
typedef LDS double *lds_f64wp;
typedef LDS unsigned long long *lds_u64p;
typedef const KCONST float *kf32p;
typedef const KCONST double *kf64p;

// LDS atomics on the workgroup's histogram replicas
__device__ __forceinline__ void lds_add(LDS unsigned *p, unsigned v)
{
    __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ void lds_add(LDS double *p, double v)
{
    __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ unsigned lds_take(LDS unsigned *p)
{
    return __hip_atomic_exchange(p, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ double lds_take(LDS double *p)
{
    return __hip_atomic_exchange(p, 0.0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ void lds_add(LDS unsigned long long *p, unsigned long long v)
{
    __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ unsigned long long lds_take(LDS unsigned long long *p)
{
    return __hip_atomic_exchange(p, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

#ifndef PC_SWEEP_THREADS
#define PC_SWEEP_THREADS 512
#endif
constexpr int kSweepThreads = PC_SWEEP_THREADS;
constexpr int kTblBytes = PC_TBL8_MAX > 2 * PC_TBL16_MAX ? PC_TBL8_MAX : 2 * PC_TBL16_MAX;
// table of the private-histogram sweep, which leaves LDS to per-wave histograms
constexpr int kTblBytesPriv = PC_TBL_PRIV_BYTES;
constexpr int kWaves = kSweepThreads / PC_WAVE;
constexpr unsigned kSlow = PC_TBL_BAND | PC_TBL_MULTI;

__device__ __forceinline__ double dval(unsigned code, double L)
{
    return code == PC_D_PLUS ? L : (code == PC_D_MINUS ? -L : 0.0);
}

// Separation of one pair in binary64, exactly as the definition: one rounding
// per operation, the periodic offset added after the difference (adding 0.0
// is exact).
template <int M>
__device__ __forceinline__ void exact_sep(double xi, double yi, double zi, double xj, double yj,
                                          double zj, unsigned dcode, double L, double *s,
                                          double *pz)
{
    double dx = __dsub_rn(xi, xj), dy = __dsub_rn(yi, yj), dz = __dsub_rn(zi, zj);
    dx = __dadd_rn(dx, dval(dcode & 3u, L));
    dy = __dadd_rn(dy, dval((dcode >> 2) & 3u, L));
    dz = __dadd_rn(dz, dval((dcode >> 4) & 3u, L));
    if (M == PC_METRIC_R) {
        *s = __dadd_rn(__dadd_rn(__dmul_rn(dx, dx), __dmul_rn(dy, dy)), __dmul_rn(dz, dz));
        *pz = 0.0;
    } else {
        *s = __dadd_rn(__dmul_rn(dx, dx), __dmul_rn(dy, dy));
        *pz = fabs(dz);
    }
}

// Number of entries of a[0..n-1] (increasing) that are <= v.
template <class P>
__device__ __forceinline__ int count_le(P a, int n, double v)
{
    int lo = 0, hi = n;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (v >= a[mid])
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo;
}

// Exact output bin of a binary64 separation, or -1 when out of range.
template <int M, class P>
__device__ __forceinline__ int exact_bin(double s, double pz, P E, int nb, P q, int npi,
                                         double pimax)
{
    if (!(s >= E[0] && s < E[nb]))
        return -1;
    const int k = count_le(E, nb + 1, s) - 1;
    if (M == PC_METRIC_R)
        return k;
    if (!(pz < pimax))
        return -1;
    return k * npi + (count_le(q, npi, pz) - 1);
}

struct Lds {
    const LDS unsigned char *tbl;   // byte or 16-bit entries
    lds_f32p lo, hi;  // r / rp bands, followed (rppi) by the pi bands
    lds_f64p E, q;
    lds_u32p hist;    // this wave's histogram replicas
    lds_f64wp whist;
};

// Weight of a pair (section 2.1's weight_func): 0 product, 1 sum.
__device__ __forceinline__ double pair_weight(int wtype, double a, double b)
{
    return wtype == 1 ? a + b : a * b;
}

// A lane's side of the pair weight as one fused multiply-add,
// w_ij = fma(a, w_j, b): (w_i, 0) for products, (1, w_i) for sums.  Either
// form rounds once, so it equals w_i * w_j or w_i + w_j.  With fixed-point
// weight sums (pc_fixed.h) both parts carry the grid's scale 2^-Q, which
// commutes with the rounding, so fma gives the integer P = w_ij 2^-Q; `u`
// (2^Q, else 1) scales it back for the mean-separation sums.
struct LaneW {
    double a, b, u;
};

__device__ __forceinline__ LaneW lane_weight(const SweepArgs &a, double wi)
{
    double sc = 1.0, u = 1.0;
    if (a.wfixed) {
        sc = a.wfx->scale;
        u = a.wfx->unscale;
    }
    return a.wtype == 1 ? LaneW{sc, wi * sc, u} : LaneW{wi * sc, 0.0, u};
}

// Exact fixed-point add of a scaled pair weight P (an integer, |P| < 2^94):
// its three signed limbs (magnitudes below 2^32) go to three int64 LDS sums,
// wlimb slots apart.  A slot receives at most 2^31 adds between merges (the
// flush bound), so every limb sum stays below 2^63 in magnitude.
__device__ __forceinline__ void add_fixed(const SweepArgs &a, lds_f64wp whb, int slot, double P)
{
    unsigned long long l0, l1, l2;
    fixed_limbs(P, l0, l1, l2);
    lds_u64p u = (lds_u64p)whb + slot;
    lds_add(u, l0);
    lds_add(u + a.wlimb, l1);
    lds_add(u + 2 * a.wlimb, l2);
}

// Separation reported by the mean-separation output, from the squared
// separation s: the distance (kind 1) or the angle in degrees of a squared
// chord (kind 2).  Binary64 pass: from the binary64 s.
__device__ __forceinline__ double sep_value(int kind, double s)
{
    const double c = sqrt(s);
    return kind == 1 ? c : (2.0 * asin(0.5 * c)) * (180.0 / M_PI);
}

// Float32 pass: from the float32 s of the scaled coordinates (one float32
// unit is `scale` in length).
__device__ __forceinline__ double sep_value_f32(int kind, float s, double scale)
{
    // (scale need not be a power of two: the product is taken in binary64)
    const double c = (double)sqrtf(s) * scale;
    if (kind == 1)
        return c;
    return (double)(2.0f * asinf(0.5f * (float)c)) * (180.0 / M_PI);
}

// Pair weight and (W == 2) mean-separation sums of one pair in range.  The
// separation sums live in a second set of replicas with the layout of the
// weight sums, (o_rhist - o_whist) / 8 doubles further on.
template <int W>
__device__ __forceinline__ void add_weight_f32(const SweepArgs &a, lds_f64wp whb, int slot,
                                               LaneW wi, double wj, float s, int kind)
{
    const double wp = fma(wi.a, wj, wi.b);
    if (a.wfixed)
        add_fixed(a, whb, slot, wp);
    else
        lds_add(&whb[slot], wp);
    if (W == 2)
        lds_add(&whb[slot + ((a.o_rhist - a.o_whist) >> 3)],
                (wp * wi.u) * sep_value_f32(kind, s, a.sep_scale));
}

template <int W>
__device__ __forceinline__ void add_weight_f64(const SweepArgs &a, lds_f64wp whb, int slot,
                                               LaneW wi, double wj, double s, int kind)
{
    const double wp = fma(wi.a, wj, wi.b);
    if (a.wfixed)
        add_fixed(a, whb, slot, wp);
    else
        lds_add(&whb[slot], wp);
    if (W == 2)
        lds_add(&whb[slot + ((a.o_rhist - a.o_whist) >> 3)], (wp * wi.u) * sep_value(kind, s));
}

// Table entry of a value (float bits already reduced to the key).
// Table entries as signed values: flagged cells read negative (byte entries
// sign-extend 0x80 | edge, 16-bit entries have 0x8000 or 0x4000 set and are
// tested separately).
template <bool T16>
__device__ __forceinline__ int tbl_entry(const Lds &L, unsigned key)
{
    if (T16)
        return (int)((const LDS uint16_t *)L.tbl)[key];
    return (int)((const LDS signed char *)L.tbl)[key];
}

template <bool T16>
__device__ __forceinline__ bool is_slow(int e)
{
    return T16 ? (e & (int)(PC_TBL_BAND | PC_TBL_MULTI)) != 0 : e < 0;
}

template <bool T16>
__device__ __forceinline__ bool is_multi(int e)
{
    return T16 ? (e & (int)PC_TBL_MULTI) != 0 : (e & 0xFF) == (int)PC_TBL8_MULTI;
}

template <bool T16>
__device__ __forceinline__ int band_edge(int e)
{
    return T16 ? (e & (int)PC_TBL_MASK) : (e & (int)PC_TBL8_MASK);
}

// Table key of a value, clamped to the extra last entry, which places every
// value beyond the table above all edges.
__device__ __forceinline__ unsigned tbl_key(float s, unsigned base, int sh, unsigned last)
{
    return min(__builtin_elementwise_sub_sat(__float_as_uint(s), base) >> sh, last);
}

// Key of the float32 path's linear table: floor(s) for s below the last
// cell, the last cell for everything above (coordinates are scaled so that
// the top band lies below the last cell).  s is a sum of squares, or +inf
// for an inactive lane, never negative or NaN, so its bit pattern orders
// like its value and an integer min clamps it in one instruction.
__device__ __forceinline__ unsigned tbl_key_linear(float s, float kmax)
{
    return (unsigned)__uint_as_float(min(__float_as_uint(s), __float_as_uint(kmax)));
}

// Key of the float32 path: the rounding key round(min(s, 1) * 32767) of the
// shared-histogram sweeps' byte tables in one v_cvt_pknorm_i16_f32 (s >= 0
// here, and the high half, the conversion of 0.0, is zero), else the linear
// key.
template <bool PK>
__device__ __forceinline__ unsigned tbl_key_f32(float s, float kmax)
{
    if constexpr (PK)
        return __builtin_bit_cast(unsigned, __builtin_amdgcn_cvt_pknorm_i16(s, 0.0f));
    else
        return tbl_key_linear(s, kmax);
}

// Value that the key sends to the last cell ("above every edge").
template <bool PK>
__device__ __forceinline__ float key_top_value(const SweepArgs &a)
{
    return PK ? 1.0f : (float)(a.B.tbl_n - 1);
}

// Number of bands wholly below s (bin + 1), or -1 when s lies inside a band.
// Band bottoms and tops never decrease (the planner widens bands where they
// would), so the first band whose top reaches s is the only one that can
// hold it: a binary search over the tops and one test of that band's bottom.
__device__ __forceinline__ int band_scan(float s, lds_f32p lo, lds_f32p hi, int nedges)
{
    int a = 0, b = nedges;
    while (a < b) {
        const int m = (a + b) >> 1;
        if (s > hi[m])
            a = m + 1;
        else
            b = m;
    }
    return (a < nedges && s >= lo[a]) ? -1 : a;
}

// Float32 slot of a value in a flagged table cell: the number of bands
// wholly below it (bin + 1), or -1 when the value lies inside a band.
template <bool T16>
__device__ __forceinline__ int slow_slot(float s, int e, lds_f32p lo, lds_f32p hi,
                                         int nedges)
{
    if (!is_multi<T16>(e)) {
        const int c = band_edge<T16>(e);
        if (s > hi[c])
            return c + 1;
        if (s < lo[c])
            return c;
        return -1;
    }
    return band_scan(s, lo, hi, nedges);
}

// Binary64 slot of a value in a flagged cell: exact comparison with the edges.
template <bool T16>
__device__ __forceinline__ int slow_slot_exact(double s, int e, lds_f64p E, int nedges)
{
    if (!is_multi<T16>(e)) {
        const int c = band_edge<T16>(e);
        return (s >= E[c]) ? c + 1 : c;
    }
    return count_le(E, nedges, s);
}

// Exact histogram row and column of a pair the float32 pass could not
// decide: the binary64 separation of the definition from the binary64 copies
// of both points (the second point is wave-uniform and comes through the
// scalar cache), binned against the exact edges.  row = rp bin + 1 and col =
// pi bin + col0, or both 0 when out of range.
template <int M>
__device__ __forceinline__ void exact_rowcol(const SweepArgs &a, const Lds &L, int i, int j,
                                             unsigned dcode, int &row, int &col)
{
    const kf64p x2 = (kf64p)a.x2, y2 = (kf64p)a.y2, z2 = (kf64p)a.z2;
    double s, pz;
    exact_sep<M>(a.x1[i], a.y1[i], a.z1[i], x2[j], y2[j], z2[j], dcode, a.L, &s, &pz);
    const int b = exact_bin<M>(s, pz, L.E, a.B.nb, L.q, a.B.npi, a.B.pimax);
    if (b < 0) {
        row = 0;
        col = 0;
    } else if (M == PC_METRIC_R) {
        row = b + 1;
        col = 0;
    } else {
        row = b / a.B.npi + 1;
        col = b % a.B.npi + a.B.col0;
    }
}

// Histogram slot of exact_rowcol (0, a catch-all, when out of range).
template <int M>
__device__ __forceinline__ int exact_slot(const SweepArgs &a, const Lds &L, int i, int j,
                                       unsigned dcode)
{
    int row, col;
    exact_rowcol<M>(a, L, i, j, dcode, row, col);
    return row * a.B.row_w + col;
}

// A lane's point as the float32 item loop reads it: binary64 x and y (3-D
// grids with column-local frames) or float32 X and Y, z as the item needs it,
// and the weight.  Consecutive items of a wave mostly share their block, so
// the sweep loads this once per block rather than once per item.
struct LanePt {
    double x, y, z, w;
    float X, Y, Z;
};

// Binary64 slot of an r pair whose lane point (binary64) is at hand.
__device__ __forceinline__ int exact_slot_r_at(const SweepArgs &a, const Lds &L, double xi,
                                               double yi, double zi, int j, unsigned dcode)
{
    const kf64p x2 = (kf64p)a.x2, y2 = (kf64p)a.y2, z2 = (kf64p)a.z2;
    double s, pz;
    exact_sep<PC_METRIC_R>(xi, yi, zi, x2[j], y2[j], z2[j], dcode, a.L, &s, &pz);
    return exact_bin<PC_METRIC_R>(s, pz, L.E, a.B.nb, L.q, 1, 0.0) + 1;
}

// An expanded r (NDIM 3) or rp (NDIM 2) pair whose float32 value lies inside
// its edge's band: the band holds the rounding term of the largest magnitudes
// a lane and a j point can have; narrowed by the pair's own term, from the
// lane's A = |a|^2 and the j point's |b|^2, it often decides the pair without
// the binary64 recheck.  -1 when the value stays inside the narrowed band, or
// the cell holds several bands.  Every float32 rounding errs towards a
// narrower narrowing: m is rounded up, the narrowing and the differences
// below down.
template <bool T16, int NDIM = 3>
__device__ __forceinline__ int tight_slot(const SweepArgs &a, const Lds &L, float s, int e,
                                          float A, int j)
{
    if (is_multi<T16>(e))
        return -1;
    const int c = band_edge<T16>(e);
    const float q = ((kf32p)a.P2)[4 * j + 3];
    // r: m >= 5 |b|^2 + 2 |a|^2 + 4 |a| |b|, as 4 |a| |b| <= 6 |b|^2 + (2/3)
    // |a|^2; rp: m >= 4 |b|^2 + 4 |a|^2 + 2 |a| |b|, as 2 |a| |b| <= 3 |b|^2 +
    // (1/3) |a|^2; (1 + 2^-18) covers the roundings of A, |b|^2 and of m
    const float m = (NDIM == 3 ? fmaf(11.0f, q, 2.75f * A) : fmaf(7.0f, q, 4.375f * A)) *
                    (1.0f + 0x1p-18f);
    const float D = a.xy_K * (a.xy_M - m) * (1.0f - 0x1p-18f);
    if (s - L.hi[c] > -D)
        return c + 1;
    if (L.lo[c] - s > -D)
        return c;
    return -1;
}

// ---- float32 chunk: CH pairs sharing lane i ------------------------------
// Three phases so that the CH table reads are in flight together: (1)
// separations, candidate masks and table keys, (2) table reads, (3) slot
// resolution and histogram updates.
// UNC: every lane adds to its own histogram replica (out-of-range values land
// in the catch-all slots), which needs no candidate branch; used for the
// unweighted 1-D statistics.
// MASK: the item's last, partial chunk; pairs k >= rem are padding (their
// loads repeat the item's last point) and are sent out of range.
// EXP: x and y expanded, s = fl(fl(fl(fl(dz dz + |b|^2) - 2 a_x b_x) -
// 2 a_y b_y) + |a|^2) with qs = |b|^2 of the j points, ax and ay holding
// -2 a_x and -2 a_y, and A = |a|^2: four instructions instead of six, with
// the rounding bound the planner's expanded bands assume.
template <int M, int W, bool TRI, bool T16, bool UNC, bool PK, int CH, bool MASK = false,
          bool EXP = false>
__device__ __forceinline__ void chunk_f32(const SweepArgs &a, const Lds &L, lds_u32p hb,
                                          lds_f64wp whb, float ax, float ay, float az, float A,
                                          LaneW wi, int i, const LanePt &lp, const float *xs,
                                          const float *ys, const float *zs, const float *qs,
                                          const double *ws, int j, unsigned dcode,
                                          unsigned &rechecks, int rem = CH)
{
    static_assert(M == PC_METRIC_R, "float32 rp/pi pairs take the fixed-point chunk");
    float s[CH];
    bool c[CH];
    unsigned key[CH];
    int e[CH];
    const float kmax = key_top_value<PK>(a);
#pragma unroll
    for (int k = 0; k < CH; k++) {
        if constexpr (EXP) {
            const float dz = az - zs[k];
            float t = fmaf(dz, dz, qs[k]);
            t = fmaf(ax, xs[k], t);
            t = fmaf(ay, ys[k], t);
            s[k] = t + A;
        } else {
            const float dx = ax - xs[k], dy = ay - ys[k], dz = az - zs[k];
            s[k] = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
        }
        c[k] = s[k] <= a.B.s_top;
        if (TRI) {
            c[k] = c[k] && (j + k > i);
            // pairs j <= i of the block's own triangle (the lane's own point
            // among them, s = 0) go to the catch-all above every edge rather
            // than to the crowded low cells, which would take the slow path
            if (!(j + k > i))
                s[k] = kmax;
        }
        if (MASK && k >= rem) {
            c[k] = false;
            s[k] = kmax;
        }
        key[k] = tbl_key_f32<PK>(s[k], kmax);
    }
    // every lane reads (no exec-mask changes), so the CH reads stay in flight;
    // byte entries of the unconditional path are read unsigned (a flagged
    // cell has bit 7 set)
    constexpr bool U8 = UNC && !T16;
#pragma unroll
    for (int k = 0; k < CH; k++)
        e[k] = U8 ? (int)((const LDS unsigned char *)L.tbl)[key[k]] : tbl_entry<T16>(L, key[k]);
    if constexpr (U8) {
        // keep the entries as the zero-extended words the or below takes
        // (otherwise one is read sign-extended for the per-pair tests and
        // masked back for the or: one instruction more per chunk)
#pragma unroll
        for (int k = 0; k < CH; k++)
            asm volatile("" : "+v"(e[k]));
    }
    if (UNC) {
        // M == PC_METRIC_R, unweighted.  One test for the whole chunk: the
        // slow flags of all CH entries are or-ed together, so the per-pair
        // band resolution only runs for chunks that need it.
        unsigned any = 0;
#pragma unroll
        for (int k = 0; k < CH; k++)
            any |= (unsigned)e[k];
        if (__builtin_expect(U8 ? any >= PC_TBL8_BAND : is_slow<T16>((int)any), 0)) {
#pragma unroll
            for (int k = 0; k < CH; k++) {
                if (U8 ? (unsigned)e[k] >= PC_TBL8_BAND : is_slow<T16>(e[k])) {
                    int slot = slow_slot<T16>(s[k], e[k], L.lo, L.hi, a.B.nb + 1);
                    if constexpr (EXP) {
                        if (slot < 0)
                            slot = tight_slot<T16>(a, L, s[k], e[k], A, j + k);
                    }
                    if (slot < 0) {
                        // (the expanded form runs on 3-D grids, whose lane
                        // point holds the binary64 coordinates)
                        slot = EXP ? exact_slot_r_at(a, L, lp.x, lp.y, lp.z, j + k, dcode)
                                   : exact_slot<M>(a, L, i, j + k, dcode);
                        rechecks++;
                    }
                    e[k] = slot;
                }
            }
        }
#pragma unroll
        for (int k = 0; k < CH; k++)
            lds_add(&hb[e[k] * PC_WAVE], 1u);
        return;
    }
#pragma unroll
    for (int k = 0; k < CH; k++) {
        if (!c[k])
            continue;
        int slot = e[k];
        if (__builtin_expect(is_slow<T16>(e[k]), 0)) {
            slot = slow_slot<T16>(s[k], e[k], L.lo, L.hi, a.B.nb + 1);
            if constexpr (EXP) {
                if (slot < 0)
                    slot = tight_slot<T16>(a, L, s[k], e[k], A, j + k);
            }
            if (slot < 0) {
                slot = EXP ? exact_slot_r_at(a, L, lp.x, lp.y, lp.z, j + k, dcode)
                           : exact_slot<M>(a, L, i, j + k, dcode);
                rechecks++;
            }
        }
        lds_add(&hb[slot], 1u);
        if (W)
            add_weight_f32<W>(a, whb, slot, wi, ws[k], s[k], a.ravg);
    }
}

// Fast pi bin of |dz| for the binary64 chunk: t = |dz| * npi / pimax in
// float32; the bin floor(t) is taken only when the fractional part of t keeps
// clear of both integers by the margin tau (covering the rounding of |dz| to
// float32, of the product and the offset of the binary64 edges q_p from
// p * pimax / npi).  Returns -1 otherwise.
__device__ __forceinline__ int pi_fast(float pz, float inv_dpi, float tau, int npi)
{
    const float t = pz * inv_dpi;
    const float fl = floorf(t);
    const float fr = t - fl;
    const int k = (int)fl;
    return (fr > tau && fr < 1.0f - tau && k < npi) ? k : -1;
}

// ---- binary64 chunk ------------------------------------------------------
template <int M, int W, bool TRI, bool OFS, bool T16, bool UNC, int CH, bool MASK = false>
__device__ __forceinline__ void chunk_f64(const SweepArgs &a, const Lds &L, lds_u32p hb,
                                          lds_f64wp whb, double xi, double yi, double zi,
                                          double Dx, double Dy, double Dz, LaneW wi, int i,
                                          const double *xs, const double *ys, const double *zs,
                                          const double *ws, int j, int rem = CH)
{
    double s[CH], pz[CH];
    bool c[CH];
    unsigned key[CH];
    int e[CH];
#pragma unroll
    for (int k = 0; k < CH; k++) {
        double dx = __dsub_rn(xi, xs[k]), dy = __dsub_rn(yi, ys[k]), dz = __dsub_rn(zi, zs[k]);
        if (OFS) {
            dx = __dadd_rn(dx, Dx);
            dy = __dadd_rn(dy, Dy);
            dz = __dadd_rn(dz, Dz);
        }
        if (M == PC_METRIC_R) {
            s[k] = __dadd_rn(__dadd_rn(__dmul_rn(dx, dx), __dmul_rn(dy, dy)), __dmul_rn(dz, dz));
            c[k] = s[k] < a.B.E_top;
        } else if (M == PC_METRIC_RPPI) {
            s[k] = __dadd_rn(__dmul_rn(dx, dx), __dmul_rn(dy, dy));
            pz[k] = fabs(dz);
            c[k] = (s[k] < a.B.E_top) && (pz[k] < a.B.pimax);
        } else {
            // on-sky: the line of sight L = v1 + v2 through the pair's
            // midpoint; pi = |s.L| / |L|, rp^2 = s.s - pi^2 (Appendix A),
            // every operation rounded as written
            const double ss = __dadd_rn(__dadd_rn(__dmul_rn(dx, dx), __dmul_rn(dy, dy)),
                                        __dmul_rn(dz, dz));
            // A pair in range has s.s below rp_max^2 + pimax^2 up to a few
            // roundings (if pi < pimax then rp^2 >= s.s - pimax^2 - O(u)),
            // so with the relative margin 2^-30 a slot where no lane is
            // below the limit skips the division and square root.
            const double lim = (a.B.E_top + a.B.pimax * a.B.pimax) * (1.0 + 0x1p-30);
            if (__any(ss < lim)) {
                const double lx = __dadd_rn(xi, xs[k]), ly = __dadd_rn(yi, ys[k]),
                             lz = __dadd_rn(zi, zs[k]);
                const double sl = __dadd_rn(__dadd_rn(__dmul_rn(dx, lx), __dmul_rn(dy, ly)),
                                            __dmul_rn(dz, lz));
                const double ll = __dadd_rn(__dadd_rn(__dmul_rn(lx, lx), __dmul_rn(ly, ly)),
                                            __dmul_rn(lz, lz));
                pz[k] = ll > 0.0 ? __ddiv_rn(fabs(sl), __dsqrt_rn(ll)) : 0.0;
                s[k] = fmax(__dsub_rn(ss, __dmul_rn(pz[k], pz[k])), 0.0);
                c[k] = (s[k] < a.B.E_top) && (pz[k] < a.B.pimax);
            } else {
                pz[k] = 1.0e300;
                s[k] = 1.0e300;
                c[k] = false;
            }
        }
        if (TRI)
            c[k] = c[k] && (j + k > i);
        if (MASK && k >= rem) {
            c[k] = false;
            s[k] = 1.0e300;
        }
        key[k] = tbl_key(__double2float_rn(s[k]), a.B.tbl_base, a.B.tbl_shift,
                         (unsigned)a.B.tbl_n - 1u);
    }
#pragma unroll
    for (int k = 0; k < CH; k++)
        e[k] = tbl_entry<T16>(L, key[k]);
    if (UNC) {
#pragma unroll
        for (int k = 0; k < CH; k++) {
            int slot = e[k];
            if (is_slow<T16>(slot))
                slot = slow_slot_exact<T16>(s[k], slot, L.E, a.B.nb + 1);
            if (TRI && !(j + k > i))
                slot = 0;
            lds_add(&hb[slot * PC_WAVE], 1u);
        }
        return;
    }
#pragma unroll
    for (int k = 0; k < CH; k++) {
        if (!c[k])
            continue;
        int slot = e[k];
        if (is_slow<T16>(e[k]))
            slot = slow_slot_exact<T16>(s[k], e[k], L.E, a.B.nb + 1);
        if (M != PC_METRIC_R) {
            const int npi = a.B.npi;
            int kp = pi_fast(__double2float_rn(pz[k]), a.B.inv_dpi, a.B.pi_tau, npi);
            if (kp < 0)
                kp = count_le(L.q, npi, pz[k]) - 1;
            slot = slot * a.B.row_w + kp + a.B.col0;
        }
        lds_add(&hb[slot], 1u);
        if (W)
            add_weight_f64<W>(a, whb, slot, wi, ws[k], s[k],
                              M != PC_METRIC_R ? 1 : a.ravg);
    }
}

// ---- float32 rp/pi chunk with fixed-point z ---------------------------------
// z is stored as fixed point with one pi bin = 2^sh quanta, so the pi bin of a
// pair is the integer |dq| >> sh, exact except within PC_ZQ_MARGIN quanta of a
// bin edge (quantisation and the rounding of the periodic length stay below
// 1.5 quanta).  rp comes from the float32 table (0 for cells wholly out of
// range).  Pairs on a flagged rp cell or near a pi edge are settled against
// the float32 rp bands and, when still undecided, in binary64.
//
// The chunk works with u = |dq| + PC_ZQ_MARGIN (one v_sad_u32): a pair is
// near a pi edge iff (u mod 2^sh) < 2 * PC_ZQ_MARGIN, and otherwise u >> sh
// equals |dq| >> sh, since subtracting the margin then stays inside the bin.
__device__ __forceinline__ unsigned absdiff_plus(unsigned a, unsigned b, unsigned c)
{
    return (max(a, b) - min(a, b)) + c;
}

// EXP: rp^2 expanded, fl(fl(fl(|a|^2 + |b|^2) - 2 a_x b_x) - 2 a_y b_y) with
// ax, ay holding -2 a_x, -2 a_y and qs = |b|^2 (the order that gives every
// instruction one scalar operand: three instructions for rp^2).
template <int W, bool TRI, bool T16, bool PK, int CH, bool MASK = false, bool EXP = false>
__device__ __forceinline__ void chunk_f32_rppi_q(const SweepArgs &a, const Lds &L, lds_u32p hb,
                                                 lds_f64wp whb, float ax, float ay, float A,
                                                 unsigned azq, LaneW wi, int i,
                                                 const float *xs, const float *ys,
                                                 const float *zs, const float *qs,
                                                 const double *ws, int j, unsigned dcode,
                                                 unsigned &rechecks, int rem = CH)
{
    const float kmax = key_top_value<PK>(a);
    const int sh = a.B.zq_shift;
    const unsigned mask = (1u << sh) - 1u;
    const unsigned npi = (unsigned)a.B.npi;
    float s[CH];
    unsigned u[CH], key[CH], near[CH];
    int er[CH];
    unsigned nmin = mask;
#pragma unroll
    for (int k = 0; k < CH; k++) {
        if constexpr (EXP) {
            const float t = fmaf(ax, xs[k], A + qs[k]);
            s[k] = fmaf(ay, ys[k], t);
        } else {
            const float dx = ax - xs[k], dy = ay - ys[k];
            s[k] = fmaf(dy, dy, dx * dx);
        }
        u[k] = absdiff_plus(azq, __float_as_uint(zs[k]), PC_ZQ_MARGIN);
        // the block's own triangle (j <= i) and the padding of a partial
        // chunk: out of range in rp, mid-bin in pi (never undecided)
        if ((TRI && !(j + k > i)) || (MASK && k >= rem)) {
            s[k] = kmax;
            u[k] = 1u << (sh - 1);
        }
        // s >= 0, so the bit patterns order like the values (no NaN here)
        key[k] = tbl_key_f32<PK>(s[k], kmax);
        near[k] = u[k] & mask;
        nmin = min(nmin, near[k]);
    }
#pragma unroll
    for (int k = 0; k < CH; k++)
        er[k] = tbl_entry<T16>(L, key[k]);
    int flag = 0;
#pragma unroll
    for (int k = 0; k < CH; k++)
        flag |= T16 ? ((er[k] << 16) | (er[k] << 17)) : er[k];
    const int nb = a.B.nb;
    if (__builtin_expect((flag < 0) | (nmin < 2u * PC_ZQ_MARGIN), 0)) {
#pragma unroll
        for (int k = 0; k < CH; k++) {
            const bool sr = is_slow<T16>(er[k]);
            const bool sp = near[k] < 2u * PC_ZQ_MARGIN;
            if (sr || sp) {
                int row = er[k];
                if (sr) {
                    row = slow_slot<T16>(s[k], er[k], L.lo, L.hi, nb + 1);
                    if constexpr (EXP) {
                        if (row < 0)
                            row = tight_slot<T16, 2>(a, L, s[k], er[k], A, j + k);
                    }
                    if (row == nb + 1)
                        row = 0;
                }
                // |dq| < 2 * margin lies well inside pi bin 0 (u >> sh is 0)
                if (row != 0 && (row < 0 || (sp && u[k] >= 3u * PC_ZQ_MARGIN))) {
                    int col;
                    exact_rowcol<PC_METRIC_RPPI>(a, L, i, j + k, dcode, row, col);
                    rechecks++;
                    // a pi bin below |dz| / dpi <= 2^(29 - sh) shifts without
                    // overflow; out of range gives row 0, which is not counted
                    u[k] = col > 0 ? (unsigned)(col - 1) << sh : 0u;
                }
                er[k] = row;
            }
        }
    }
    // kp < npi iff u < npi << sh (every u fits when that shift overflows);
    // the slot is one 24-bit multiply-add of row and column, and its byte
    // address one shift-add (the + 1 rides in the LDS instruction's offset)
    const unsigned ulim = npi > (0xFFFFFFFFu >> sh) ? 0xFFFFFFFFu : npi << sh;
    const unsigned rw = (unsigned)a.B.row_w;
#pragma unroll
    for (int k = 0; k < CH; k++) {
        if ((er[k] > 0) & (u[k] < ulim)) {
            unsigned slot = __umul24((unsigned)er[k], rw) + (u[k] >> sh);
            // (opaque here, or the compiler scales both terms of the sum
            // separately: two instructions more)
            asm("" : "+v"(slot));
            lds_add(&hb[slot + 1u], 1u);
            if (W)
                add_weight_f32<W>(a, whb, (int)(slot + 1u), wi, ws[k], s[k], 1);
        }
    }
}

// ---- item loops ----------------------------------------------------------
// The float32 rp/pi pairs of one item (z in fixed point), as r_loop.
template <int W, bool TRI, bool T16, bool PK, int CH, bool EXP>
__device__ __forceinline__ void rppi_loop(const SweepArgs &a, const Lds &L, lds_u32p hb,
                                          lds_f64wp whb, float ax, float ay, float A,
                                          unsigned azq, LaneW wi, int i, int j0, int j1,
                                          unsigned dcode, unsigned &rechecks)
{
    const kf32p X2 = (kf32p)a.X2, Y2 = (kf32p)a.Y2, Z2 = (kf32p)a.Z2;
    typedef float v4f __attribute__((ext_vector_type(4)));
    const KCONST v4f *P2 = (const KCONST v4f *)a.P2;   // (x, y, z bits, |b|^2) per point
    const kf64p w2 = (kf64p)a.w2;
    int j = j0;
    for (; j + CH <= j1; j += CH) {
        float xs[CH], ys[CH], zs[CH], qs[CH];
        double ws[CH];
#pragma unroll
        for (int k = 0; k < CH; k++) {
            if constexpr (EXP) {
                const v4f p = P2[j + k];
                xs[k] = p.x;
                ys[k] = p.y;
                zs[k] = p.z;
                qs[k] = p.w;
            } else {
                xs[k] = X2[j + k];
                ys[k] = Y2[j + k];
                zs[k] = Z2[j + k];
                qs[k] = 0.0f;
            }
            ws[k] = W ? w2[j + k] : 0.0;
        }
        chunk_f32_rppi_q<W, TRI, T16, PK, CH, false, EXP>(a, L, hb, whb, ax, ay, A, azq, wi, i,
                                                          xs, ys, zs, qs, ws, j, dcode,
                                                          rechecks);
    }
    if (j < j1) {
        const int rem = j1 - j;
        float xs[CH], ys[CH], zs[CH], qs[CH];
        double ws[CH];
#pragma unroll
        for (int k = 0; k < CH; k++) {
            const int jk = j + min(k, rem - 1);
            if constexpr (EXP) {
                const v4f p = P2[jk];
                xs[k] = p.x;
                ys[k] = p.y;
                zs[k] = p.z;
                qs[k] = p.w;
            } else {
                xs[k] = X2[jk];
                ys[k] = Y2[jk];
                zs[k] = Z2[jk];
                qs[k] = 0.0f;
            }
            ws[k] = W ? w2[jk] : 0.0;
        }
        chunk_f32_rppi_q<W, TRI, T16, PK, CH, true, EXP>(a, L, hb, whb, ax, ay, A, azq, wi, i,
                                                         xs, ys, zs, qs, ws, j, dcode, rechecks,
                                                         rem);
    }
}

// The float32 r pairs of one item: chunks of CH j points, then the partial
// last chunk padded with the item's last point.  Second-catalogue points are
// wave-uniform and read through the scalar cache (the arrays are not written
// during the sweep); the expanded form reads them as (x, y, z, |b|^2) side
// by side, two 64-byte scalar loads per chunk from one base address.
template <int W, bool TRI, bool T16, bool UNC, bool PK, int CH, bool EXP>
__device__ __forceinline__ void r_loop(const SweepArgs &a, const Lds &L, lds_u32p hb,
                                       lds_f64wp whb, float ax, float ay, float az, float A,
                                       LaneW wi, int i, const LanePt &lp, int j0, int j1,
                                       unsigned dcode, unsigned &rechecks)
{
    const kf32p X2 = (kf32p)a.X2, Y2 = (kf32p)a.Y2, Z2 = (kf32p)a.Z2;
    typedef float v4f __attribute__((ext_vector_type(4)));
    const KCONST v4f *P2 = (const KCONST v4f *)a.P2;   // (x, y, z, |b|^2) per point
    const kf64p w2 = (kf64p)a.w2;
    int j = j0;
    for (; j + CH <= j1; j += CH) {
        float xs[CH], ys[CH], zs[CH], qs[CH];
        double ws[CH];
#pragma unroll
        for (int k = 0; k < CH; k++) {
            if constexpr (EXP) {
                const v4f p = P2[j + k];
                xs[k] = p.x;
                ys[k] = p.y;
                zs[k] = p.z;
                qs[k] = p.w;
            } else {
                xs[k] = X2[j + k];
                ys[k] = Y2[j + k];
                zs[k] = Z2[j + k];
                qs[k] = 0.0f;
            }
            ws[k] = W ? w2[j + k] : 0.0;
        }
        chunk_f32<PC_METRIC_R, W, TRI, T16, UNC, PK, CH, false, EXP>(
            a, L, hb, whb, ax, ay, az, A, wi, i, lp, xs, ys, zs, qs, ws, j, dcode, rechecks);
    }
    if (j < j1) {
        const int rem = j1 - j;
        float xs[CH], ys[CH], zs[CH], qs[CH];
        double ws[CH];
#pragma unroll
        for (int k = 0; k < CH; k++) {
            const int jk = j + min(k, rem - 1);
            if constexpr (EXP) {
                const v4f p = P2[jk];
                xs[k] = p.x;
                ys[k] = p.y;
                zs[k] = p.z;
                qs[k] = p.w;
            } else {
                xs[k] = X2[jk];
                ys[k] = Y2[jk];
                zs[k] = Z2[jk];
                qs[k] = 0.0f;
            }
            ws[k] = W ? w2[jk] : 0.0;
        }
        chunk_f32<PC_METRIC_R, W, TRI, T16, UNC, PK, CH, true, EXP>(
            a, L, hb, whb, ax, ay, az, A, wi, i, lp, xs, ys, zs, qs, ws, j, dcode, rechecks,
            rem);
    }
}

template <int M, int W>
__device__ __forceinline__ LanePt load_lane(const SweepArgs &a, int i, bool act)
{
    LanePt p = {0.0, 0.0, 0.0, 0.0, 0.0f, 0.0f, 0.0f};
    if (!act)
        return p;
    if (a.xy_local) {
        p.x = a.x1[i];
        p.y = a.y1[i];
        if (M == PC_METRIC_R)
            p.z = a.z1[i];
    } else {
        p.X = a.X1[i];
        p.Y = a.Y1[i];
        if (M == PC_METRIC_R)
            p.Z = a.Z1[i];
    }
    if (M != PC_METRIC_R)
        p.Z = a.Z1[i];
    if (W)
        p.w = a.w1[i];
    return p;
}

// CACHED: the caller holds the lane's point (lpc); otherwise it is loaded here.
// EXP: r pairs with x and y expanded (float32 DD(r) of 3-D grids).
template <int M, int W, bool TRI, bool T16, bool UNC, bool PK, bool CACHED, bool EXP>
__device__ __forceinline__ void item_f32(const SweepArgs &a, const Lds &L, lds_u32p hb,
                                         lds_f64wp whb, int i, bool act, const LanePt &lpc,
                                         int j0, int j1, unsigned dcode, unsigned &rechecks,
                                         int jx, int jy)
{
    const LanePt lp = CACHED ? lpc : load_lane<M, W>(a, i, act);
    const float Lf = a.Lf32;
    const unsigned cx = dcode & 3u, cy = (dcode >> 2) & 3u, cz = (dcode >> 4) & 3u;
    const float Dx = cx == PC_D_PLUS ? Lf : (cx == PC_D_MINUS ? -Lf : 0.0f);
    const float Dy = cy == PC_D_PLUS ? Lf : (cy == PC_D_MINUS ? -Lf : 0.0f);
    const float Dz = cz == PC_D_PLUS ? Lf : (cz == PC_D_MINUS ? -Lf : 0.0f);
    // inactive lanes sit far away: their separations overflow to +inf
    float ax, ay;
    if (a.xy_local) {
        // the lane's point (shifted by the item's periodic offset) in the
        // frame of the j column, from its binary64 coordinates, rounded once
        ax = act ? (float)((lp.x + dval(cx, a.L) - col_centre(a.glo[0], a.gw[0], jx)) *
                           a.fscale)
                 : 3.0e30f;
        ay = act ? (float)((lp.y + dval(cy, a.L) - col_centre(a.glo[1], a.gw[1], jy)) *
                           a.fscale)
                 : 3.0e30f;
    } else {
        ax = act ? lp.X + Dx : 3.0e30f;
        ay = act ? lp.Y + Dy : 3.0e30f;
    }
    const LaneW wi = lane_weight(a, (W && act) ? lp.w : 0.0);
    // second-catalogue points are wave-uniform: read them through the scalar
    // cache (the arrays are not written during the sweep)
    const kf32p X2 = (kf32p)a.X2, Y2 = (kf32p)a.Y2, Z2 = (kf32p)a.Z2;
    const kf64p w2 = (kf64p)a.w2;
    constexpr int CH = W ? 4 : 8;
    int j = j0;
    if constexpr (M == PC_METRIC_RPPI) {
        // z in fixed point: the periodic z offset is a whole number of quanta
        const unsigned Dq = cz == PC_D_PLUS ? a.B.zq_L : (cz == PC_D_MINUS ? 0u - a.B.zq_L : 0u);
        const unsigned azq = __float_as_uint(lp.Z) + Dq;
        if constexpr (EXP) {
            const float A = act ? __fmaf_rn(ay, ay, __fmul_rn(ax, ax)) : 0.0f;
            const float ex = act ? -2.0f * ax : 0.0f, ey = act ? -2.0f * ay : 0.0f;
            // (an inactive lane: s = 0 + 0 + 0 would be in range, so its
            // weight-free catch-all is forced through A = +inf)
            rppi_loop<W, TRI, T16, PK, CH, true>(a, L, hb, whb, ex, ey, act ? A : INFINITY, azq,
                                                 wi, i, j0, j1, dcode, rechecks);
        } else {
            rppi_loop<W, TRI, T16, PK, CH, false>(a, L, hb, whb, ax, ay, 0.0f, azq, wi, i, j0,
                                                  j1, dcode, rechecks);
        }
        return;
    } else {
        float az;
        if (a.xy_local)
            az = act ? (float)((lp.z + dval(cz, a.L) - a.glo[2]) * a.fscale) : 3.0e30f;
        else
            az = act ? lp.Z + Dz : 3.0e30f;
        if constexpr (EXP) {
            // -2 a and |a|^2 = fl(a_y a_y + fl(a_x a_x)) of the lane; an
            // inactive lane keeps its far z, so s overflows to +inf
            const float A = act ? __fmaf_rn(ay, ay, __fmul_rn(ax, ax)) : 0.0f;
            const float ex = act ? -2.0f * ax : 0.0f, ey = act ? -2.0f * ay : 0.0f;
            r_loop<W, TRI, T16, UNC, PK, CH, true>(a, L, hb, whb, ex, ey, az, A, wi, i, lp, j0,
                                                   j1, dcode, rechecks);
        } else {
            r_loop<W, TRI, T16, UNC, PK, CH, false>(a, L, hb, whb, ax, ay, az, 0.0f, wi, i, lp,
                                                    j0, j1, dcode, rechecks);
        }
    }
}

template <int M, int W, bool TRI, bool OFS, bool T16, bool UNC>
__device__ __forceinline__ void item_f64(const SweepArgs &a, const Lds &L, lds_u32p hb,
                                         lds_f64wp whb, int i, bool act, int j0, int j1,
                                         unsigned dcode)
{
    const double Dx = dval(dcode & 3u, a.L), Dy = dval((dcode >> 2) & 3u, a.L),
                 Dz = dval((dcode >> 4) & 3u, a.L);
    const double xi = act ? a.x1[i] : 1.0e300;
    const double yi = act ? a.y1[i] : 1.0e300;
    const double zi = act ? a.z1[i] : 1.0e300;
    const LaneW wi = lane_weight(a, (W && act) ? a.w1[i] : 0.0);
    const kf64p x2 = (kf64p)a.x2, y2 = (kf64p)a.y2, z2 = (kf64p)a.z2, w2 = (kf64p)a.w2;
    constexpr int CH = W ? 4 : 8;
    int j = j0;
    for (; j + CH <= j1; j += CH) {
        double xs[CH], ys[CH], zs[CH], ws[CH];
#pragma unroll
        for (int k = 0; k < CH; k++) {
            xs[k] = x2[j + k];
            ys[k] = y2[j + k];
            zs[k] = z2[j + k];
            ws[k] = W ? w2[j + k] : 0.0;
        }
        chunk_f64<M, W, TRI, OFS, T16, UNC, CH>(a, L, hb, whb, xi, yi, zi, Dx, Dy, Dz, wi, i, xs,
                                                ys, zs, ws, j);
    }
    if (j < j1) {
        // the partial last chunk, padded with the item's last point
        const int rem = j1 - j;
        double xs[CH], ys[CH], zs[CH], ws[CH];
#pragma unroll
        for (int k = 0; k < CH; k++) {
            const int jk = j + min(k, rem - 1);
            xs[k] = x2[jk];
            ys[k] = y2[jk];
            zs[k] = z2[jk];
            ws[k] = W ? w2[jk] : 0.0;
        }
        chunk_f64<M, W, TRI, OFS, T16, UNC, CH, true>(a, L, hb, whb, xi, yi, zi, Dx, Dy, Dz, wi,
                                                      i, xs, ys, zs, ws, j, rem);
    }
}

// End of the triangle-masked part of an item [j0, j1) whose block ends at
// iend: the chunks (CH pairs each, as item_f32 and item_f64 take them) up to
// the first chunk boundary at or past iend.
template <int W>
__device__ __forceinline__ int tri_end(int j0, int j1, int iend)
{
    constexpr int CH = W ? 4 : 8;
    const int n = max(iend - j0, 0);
    return min(j1, j0 + (n + CH - 1) / CH * CH);
}

// Take the next work item for this wave from stream s, moving on to the
// following streams once it is exhausted.  Stream s owns the contiguous
// items [s n / S, (s + 1) n / S), so a wave's consecutive items are
// neighbours (same catalogue, nearby cells).  Returns n_items when every
// stream is exhausted.  On a stream that last gave the wave an item, lane 0
// increments the counter at once (one round trip per item; the one increment
// past the end is harmless, as every take compares with the length).  On the
// streams it moves on to (`probe`), it reads the counter first and only
// increments it while items remain, so exhausted streams cost one load each.
__device__ __forceinline__ int wave_fetch(int *ctrs, int n_items, int lane, int &s, bool &probe)
{
    for (int tries = 0; tries < PC_STREAMS; tries++) {
        const int first = (int)(((long long)n_items * s) / PC_STREAMS);
        const int len = (int)(((long long)n_items * (s + 1)) / PC_STREAMS) - first;
        int v = len;
        if (lane == 0) {
            int *c = ctrs + s * PC_STREAM_STRIDE;
            if (!probe || __hip_atomic_load(c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < len)
                v = atomicAdd(c, 1);
        }
        v = __builtin_amdgcn_readfirstlane(v);
        if (v < len) {
            probe = false;
            return first + v;
        }
        s = (s + 1) & (PC_STREAMS - 1);
        probe = true;
    }
    return n_items;
}

// Merge histogram replicas into the global bins of catalogue `cat` and clear
// them.  Output bin b = k * npi + p lives in slot (k + 1) * row_w + p + col0;
// every other slot is an out-of-range catch-all and is only cleared.  Called
// by threads t = first, first + step, ...; slots are taken with atomic
// exchanges, so other waves may keep adding to shared replicas meanwhile.
// Word of slot `slot` of count replica r.  One replica per lane (UNC: the
// unconditional sweeps) interleaves the replicas, slot * 64 + lane, so the 64
// lanes of a wave always add to 64 different banks whatever their slots;
// fewer replicas keep each replica's slots together, rep_stride apart.
template <bool UNC>
__device__ __forceinline__ int count_index(const SweepArgs &a, int r, int slot)
{
    return UNC ? slot * PC_WAVE + r : r * a.rep_stride + slot;
}

template <bool UNC>
__device__ __forceinline__ void flush_hist(const SweepArgs &a, const Lds &L, int first, int step,
                                           bool W, unsigned cat)
{
    const int npi = a.B.npi, rw = a.B.row_w, c0 = a.B.col0;
    unsigned long long *gh = a.g_hist + (size_t)cat * a.nbt;
    double *gw = W ? a.g_whist + (size_t)cat * a.nbt : nullptr;
    // mean-separation sums: a second set of replicas after the weight sums
    const bool R = W && a.ravg;
    const int roff = (a.o_rhist - a.o_whist) >> 3;
    double *gr = R ? a.g_rhist + (size_t)cat * a.nbt : nullptr;
    // fixed-point weight sums: three uint64 limb sums per slot
    const bool F = W && a.wfixed;
    const lds_u64p fx = F ? (lds_u64p)L.whist : (lds_u64p) nullptr;
    unsigned long long *gf = F ? a.g_wfix + 3 * (size_t)cat * a.nbt : nullptr;
    for (int b = first; b < a.nbt; b += step) {
        const int slot = (b / npi + 1) * rw + b % npi + c0;
        unsigned long long c = 0;
        double w = 0.0, rs = 0.0;
        unsigned long long f0 = 0, f1 = 0, f2 = 0;
        for (int r = 0; r < a.copies; r++) {
            c += lds_take(&L.hist[count_index<UNC>(a, r, slot)]);
            if (F) {
                const int o = r * a.rep_stride + slot;
                f0 += lds_take(&fx[o]);
                f1 += lds_take(&fx[o + a.wlimb]);
                f2 += lds_take(&fx[o + 2 * a.wlimb]);
            } else if (W) {
                w += lds_take(&L.whist[r * a.rep_stride + slot]);
            }
            if (R)
                rs += lds_take(&L.whist[r * a.rep_stride + slot + roff]);
        }
        if (c)
            atomicAdd(&gh[b], c);
        if (F) {
            if (f0 | f1 | f2) {
                unsigned long long v[3];
                fixed_words((long long)f0, (long long)f1, (long long)f2, v);
                fixed_atomic_add(gf + 3 * (size_t)b, v);
            }
        } else if (W && w != 0.0) {
            atomicAdd(&gw[b], w);
        }
        if (R && rs != 0.0)
            atomicAdd(&gr[b], rs);
    }
    for (int t = first; t < a.copies * a.slots; t += step) {
        const int r = t / a.slots, sl = t % a.slots;
        const int row = sl / rw, col = sl % rw - c0;
        if (row >= 1 && row <= a.B.nb && col >= 0 && col < npi)
            continue;
        lds_take(&L.hist[count_index<UNC>(a, r, sl)]);
        if (F) {
            const int o = r * a.rep_stride + sl;
            lds_take(&fx[o]);
            lds_take(&fx[o + a.wlimb]);
            lds_take(&fx[o + 2 * a.wlimb]);
        } else if (W) {
            lds_take(&L.whist[r * a.rep_stride + sl]);
        }
        if (R)
            lds_take(&L.whist[r * a.rep_stride + sl + roff]);
    }
}

// PRIV: every wave owns its histogram replicas and flushes them whenever the
// catalogue of its work items changes (batched calls); otherwise the
// workgroup's waves share one set of replicas for a single catalogue.
// EXP: the float32 r sweep with x and y expanded (its own kernel, so the
// differences form's arrays hold no registers in its loop).
template <int M, bool P32, int W, bool T16, bool UNC, bool PRIV, bool EXP>
__device__ __forceinline__ void sweep_body(const SweepArgs &a)
{
    // the lookup table has a fixed place so its address folds into the
    // LDS instructions; the rest of the layout is dynamic
    // (the rounding-key byte table of float32 shared-histogram sweeps is
    // smaller, which leaves room for a fourth workgroup per CU)
    __shared__ __align__(16) unsigned char
        s_tbl[PRIV ? kTblBytesPriv : ((P32 && !T16) ? PC_TBL_PK_CELLS : kTblBytes)];
    extern __shared__ __align__(16) unsigned char smem[];
    LDS unsigned char *sm = (LDS unsigned char *)smem;
    {
        const int tid = threadIdx.x;
        if (T16) {
            LDS uint16_t *tbl = (LDS uint16_t *)(LDS unsigned char *)s_tbl;
            const uint16_t *src = (const uint16_t *)a.tbl;
            for (int k = tid; k < a.B.tbl_n; k += kSweepThreads)
                tbl[k] = src[k];
        } else {
            LDS unsigned char *tbl = (LDS unsigned char *)s_tbl;
            const unsigned char *src = (const unsigned char *)a.tbl;
            for (int k = tid; k < a.B.tbl_n; k += kSweepThreads)
                tbl[k] = src[k];
        }
        // float bands: the r / rp edges, then (rppi) the pi edges
        const int ne = a.B.nb + 1, nq = (M != PC_METRIC_R) ? a.B.npi + 1 : 0;
        LDS float *lo = (LDS float *)(sm + a.o_lo);
        LDS float *hi = (LDS float *)(sm + a.o_hi);
        for (int k = tid; k < ne; k += kSweepThreads) {
            lo[k] = a.lo[k];
            hi[k] = a.hi[k];
        }
        for (int k = tid; k < nq; k += kSweepThreads) {
            lo[ne + k] = a.plo[k];
            hi[ne + k] = a.phi[k];
        }
        LDS double *E = (LDS double *)(sm + a.o_E);
        for (int k = tid; k < ne; k += kSweepThreads)
            E[k] = a.E[k];
        LDS double *q = (LDS double *)(sm + a.o_q);
        for (int k = tid; k < nq; k += kSweepThreads)
            q[k] = a.q[k];
        constexpr int sets = PRIV ? kWaves : 1;
        LDS unsigned *hist = (LDS unsigned *)(sm + a.o_hist);
        for (int k = tid; k < sets * a.hist_stride; k += kSweepThreads)
            hist[k] = 0u;
        if (W) {
            // weight sums (binary64, or three uint64 limb sums), then (mean
            // separation) the separation sums: the rest of the layout
            LDS unsigned long long *wh = (LDS unsigned long long *)(sm + a.o_whist);
            const int nw = (a.lds_bytes - a.o_whist) >> 3;
            for (int k = tid; k < nw; k += kSweepThreads)
                wh[k] = 0ull;
        }
    }
    __syncthreads();

    const int lane = threadIdx.x & (PC_WAVE - 1);
    Lds L;
    L.tbl = (const LDS unsigned char *)s_tbl;
    L.lo = (lds_f32p)(sm + a.o_lo);
    L.hi = (lds_f32p)(sm + a.o_hi);
    L.E = (lds_f64p)(sm + a.o_E);
    L.q = (lds_f64p)(sm + a.o_q);
    // one set of replicas shared by the workgroup's waves, or one per wave
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / PC_WAVE));
    L.hist = (lds_u32p)(sm + a.o_hist) + (PRIV ? wave * a.hist_stride : 0);
    L.whist = W ? (lds_f64wp)(sm + a.o_whist) + (PRIV ? wave * a.whist_stride : 0)
                : (lds_f64wp) nullptr;
    // this lane's replica
    const int rep = lane & (a.copies - 1);
    lds_u32p hb = L.hist + (UNC ? rep : rep * a.rep_stride);   // (count_index)
    lds_f64wp whb = W ? L.whist + rep * a.rep_stride : (lds_f64wp) nullptr;

    // Pairs this wave added since its last flush.  A shared slot holds at
    // most the adds since the most recent flush by any wave, i.e. at most the
    // sum of every wave's pending count, so a per-wave bound of 2^31 / waves
    // keeps the uint32 slots from wrapping; private slots take 2^31.  The
    // host passes that bound, or a smaller one (a test hook).
    unsigned long long pending = 0;
    const unsigned long long flush_at = a.flush_at;
    unsigned cur_cat = 0;

    unsigned rechecks = 0;   // pairs this lane settled in binary64
    // wave-uniform (kept in a scalar register, so every item field and j
    // index derived from it stays scalar)
    int stream = __builtin_amdgcn_readfirstlane(
        (int)((blockIdx.x * kWaves + wave) & (PC_STREAMS - 1)));
    int n_items = a.n_items;
    if (a.n_items_dev)
        n_items = min(n_items, __builtin_amdgcn_readfirstlane(*(const volatile int32_t *)a.n_items_dev));
    bool probe = false;
    // the float32 loop's lane point, kept while consecutive items share a block
    int lp_i0 = -1, lp_ni = -1;
    LanePt lp = {0.0, 0.0, 0.0, 0.0, 0.0f, 0.0f, 0.0f};
    int next = wave_fetch(a.counter, n_items, lane, stream, probe);
    pc_item nit = {};
    // (3-D grids: the cell of the next item's first j point, read with the
    // item so that its column is known when the item starts)
    const KCONST int32_t *icell = (const KCONST int32_t *)a.icell;
    int ncell = 0;
    if (P32 && next < n_items) {
        nit = a.items[next];
        if (a.xy_local)
            ncell = icell[next];
    }
    // Unweighted float32 r sweeps of one catalogue also start the take of the
    // item after the next one before running an item (one atomic increment
    // on the wave's stream, `pend`), read its result only at the next item
    // (the round trip overlaps the item's work), and keep the lane's point
    // while consecutive items share a block.  (The registers these hold
    // across items cost the weighted, rp/pi and private-histogram sweeps more
    // occupancy than they save.)
    constexpr bool PIPE = P32 && W == 0 && !PRIV && M == PC_METRIC_R;
    // the take one item ahead alone also pays in the batched sweeps, whose
    // items are short (measured 1.3% on 48 mock catalogues; the other
    // weighted and rp/pi sweeps measured 2-3% slower with it)
    constexpr bool AHEAD = PIPE || (P32 && PRIV);
    int pv = 0;
    bool pend = false;
    while (next < n_items) {
        // float32 sweeps load the following item's descriptor while this
        // item runs (measured slower for the binary64 sweep, which keeps the
        // load after the take)
        const int cur = next;
        const pc_item it = P32 ? nit : a.items[cur];
        const int jcell = ncell;
        if (AHEAD && pend) {
            pend = false;
            const int first = (int)(((long long)n_items * stream) / PC_STREAMS);
            const int len = (int)(((long long)n_items * (stream + 1)) / PC_STREAMS) - first;
            const int v = __builtin_amdgcn_readfirstlane(pv);
            if (v < len) {
                next = first + v;
            } else {
                stream = (stream + 1) & (PC_STREAMS - 1);
                probe = true;
                next = wave_fetch(a.counter, n_items, lane, stream, probe);
            }
        } else {
            next = wave_fetch(a.counter, n_items, lane, stream, probe);
        }
        if (P32 && next < n_items) {
            nit = a.items[next];
            if (a.xy_local)
                ncell = icell[next];
        }
        if (AHEAD && next < n_items && !probe) {
            if (lane == 0)
                pv = atomicAdd(a.counter + stream * PC_STREAM_STRIDE, 1);
            pend = true;
        }
        const int ni = (int)PC_META_NI(it.meta);
        const unsigned dcode = PC_META_DCODE(it.meta);
        const bool tri = PC_META_TRI(it.meta) != 0;
        const unsigned long long work = (unsigned long long)ni * (unsigned)(it.j1 - it.j0);
        if (PRIV) {
            const unsigned cat = PC_META_CAT(it.meta);
            if (cat != cur_cat) {
                if (pending)
                    flush_hist<UNC>(a, L, lane, PC_WAVE, W, cur_cat);
                pending = 0;
                cur_cat = cat;
            }
        }
        if (pending + work > flush_at) {
            flush_hist<UNC>(a, L, lane, PC_WAVE, W, cur_cat);
            pending = 0;
            if (lane == 0)
                atomicAdd(a.flush_count, 1u);
        }
        pending += work;
        const bool act = lane < ni;
        const int i = it.i0 + (act ? lane : 0);
        if constexpr (P32) {
            // the item's j column (every j point of an item lies in one column)
            int jx = 0, jy = 0;
            if (a.xy_local)
                cell_column(__builtin_amdgcn_readfirstlane(jcell), a.gnx, a.gny, a.gnz, &jx, &jy);
            constexpr bool PK = !PRIV && !T16;
            if (PIPE && (it.i0 != lp_i0 || ni != lp_ni)) {
                lp = load_lane<M, W>(a, i, act);
                lp_i0 = it.i0;
                lp_ni = ni;
            }
            // an item that holds (part of) the block's triangle masks its
            // chunks up to the block's end (rounded up to whole chunks: the
            // mask passes every j >= i0 + ni) and runs the rest unmasked
            const int tm = tri ? tri_end<W>(it.j0, it.j1, it.i0 + ni) : it.j0;
            if (tm > it.j0)
                item_f32<M, W, true, T16, UNC, PK, PIPE, EXP>(a, L, hb, whb, i, act, lp, it.j0, tm,
                                                         dcode, rechecks, jx, jy);
            if (it.j1 > tm)
                item_f32<M, W, false, T16, UNC, PK, PIPE, EXP>(a, L, hb, whb, i, act, lp, tm,
                                                          it.j1, dcode, rechecks, jx, jy);
        } else {
            const int tm = tri ? tri_end<W>(it.j0, it.j1, it.i0 + ni) : it.j0;
            if (tm > it.j0)
                item_f64<M, W, true, false, T16, UNC>(a, L, hb, whb, i, act, it.j0, tm, dcode);
            if (it.j1 > tm) {
                if (dcode == 0u)
                    item_f64<M, W, false, false, T16, UNC>(a, L, hb, whb, i, act, tm, it.j1,
                                                           dcode);
                else
                    item_f64<M, W, false, true, T16, UNC>(a, L, hb, whb, i, act, tm, it.j1,
                                                          dcode);
            }
        }
    }
    // the result of a take still in flight (past the last item) is waited
    // for, not left outstanding (a counter value is never negative)
    if (AHEAD && pend && __builtin_amdgcn_readfirstlane(pv) < 0)
        rechecks++;
    if (PRIV) {
        flush_hist<UNC>(a, L, lane, PC_WAVE, W, cur_cat);
    } else {
        __syncthreads();
        flush_hist<UNC>(a, L, (int)threadIdx.x, kSweepThreads, W, 0u);
    }
    if (P32) {
        // one atomic per wave for the recheck statistic
        unsigned tot = rechecks;
        for (int off = PC_WAVE / 2; off > 0; off >>= 1)
            tot += __shfl_xor(tot, off);
        if (lane == 0 && tot)
            atomicAdd(a.rq_count, tot);
    }
}

template <int M, bool P32, int W, bool T16, bool UNC, bool PRIV, bool EXP = false>
__global__ __launch_bounds__(kSweepThreads) void k_sweep(SweepArgs a)
{
    sweep_body<M, P32, W, T16, UNC, PRIV, EXP>(a);
}

// The unweighted float32 r sweeps with one histogram replica per lane: their
// LDS (the 32 KiB byte table and 64 small replicas) fits four workgroups per
// CU, so their registers are held to 64 per lane (eight waves per SIMD).
template <int M, bool P32, int W, bool T16, bool UNC, bool PRIV, bool EXP = false>
__global__ __launch_bounds__(kSweepThreads, 8) void k_sweep_o8(SweepArgs a)
{
    sweep_body<M, P32, W, T16, UNC, PRIV, EXP>(a);
}

// Sum of the self-pair weights of every catalogue of a side (w^2 for
// product pair weights, w + w for summed ones): the weights are in cell
// order, so catalogue c owns [start[c * ncell], start[(c + 1) * ncell]).
// blockIdx.y is the catalogue.
__global__ void k_wsq(int64_t ncell, const int32_t *start, const double *w, int wtype,
                      double *out)
{
    const int c = blockIdx.y;
    const int64_t a = start[c * ncell], b = start[(c + 1) * ncell];
    double s = 0.0;
    for (int64_t i = a + blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < b;
         i += (int64_t)gridDim.x * blockDim.x)
        s += pair_weight(wtype, w[i], w[i]);
    __shared__ double sm[256];
    sm[threadIdx.x] = s;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st)
            sm[threadIdx.x] += sm[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0 && sm[0] != 0.0)
        atomicAdd(&out[c], sm[0]);
}

// ---- fixed-point weight sums (pc_fixed.h) ---------------------------------
// Lowest set bit of a nonzero, finite |w| (bits without the sign): w is a
// multiple of 2^low.
__device__ __forceinline__ int low_bit_exp(unsigned long long bits)
{
    const int e = (int)(bits >> 52);
    unsigned long long m = bits & ((1ull << 52) - 1ull);
    if (e)
        m |= 1ull << 52;
    const int base = e ? e - 1075 : -1074;
    return base + __ffsll((long long)m) - 1;
}

// Atomic maxima over the nonzero weights of one side: 2100 - low(w), |w|,
// and the complement of |w| (whose maximum gives the minimum).
__global__ void k_wfixed_scan(int64_t n, const double *w, int side, pc_wfixed *fx)
{
    unsigned key = 0;
    unsigned long long mx = 0, nmn = 0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const unsigned long long b = __double_as_longlong(w[i]) & ~(1ull << 63);
        if (b == 0)
            continue;
        key = max(key, (unsigned)(2100 - low_bit_exp(b)));
        mx = max(mx, b);
        nmn = max(nmn, ~b);
    }
    for (int off = PC_WAVE / 2; off > 0; off >>= 1) {
        key = max(key, (unsigned)__shfl_xor((int)key, off));
        mx = max(mx, (unsigned long long)__shfl_xor((long long)mx, off));
        nmn = max(nmn, (unsigned long long)__shfl_xor((long long)nmn, off));
    }
    if ((threadIdx.x & (PC_WAVE - 1)) == 0 && key) {
        atomicMax(&fx->lowkey[side], key);
        atomicMax(&fx->maxbits[side], mx);
        atomicMax(&fx->notmin[side], nmn);
    }
}

// The grid 2^Q of the call and its checks (one thread).  two_sided: side 1
// was scanned separately (cross-correlations); otherwise side 2 is side 1.
__global__ void k_wfixed_plan(int wtype, int two_sided, pc_wfixed *fx, unsigned *flags)
{
    if (threadIdx.x != 0 || blockIdx.x != 0)
        return;
    const int s2 = two_sided ? 1 : 0;
    const bool any1 = fx->lowkey[0] != 0, any2 = fx->lowkey[s2] != 0;
    int q = 0;
    double pmax = 0.0;   // bound on max |pair weight|
    const double mx1 = any1 ? __longlong_as_double((long long)fx->maxbits[0]) : 0.0;
    const double mx2 = any2 ? __longlong_as_double((long long)fx->maxbits[s2]) : 0.0;
    const double mn1 = any1 ? __longlong_as_double((long long)~fx->notmin[0]) : 0.0;
    const double mn2 = any2 ? __longlong_as_double((long long)~fx->notmin[s2]) : 0.0;
    const int low1 = 2100 - (int)fx->lowkey[0], low2 = 2100 - (int)fx->lowkey[s2];
    bool ok = true;
    if (wtype == 1) {
        if (any1 || any2) {
            q = any1 ? (any2 ? min(low1, low2) : low1) : low2;
            pmax = mx1 + mx2;
        }
    } else if (any1 && any2) {
        q = low1 + low2;
        // a product is also a multiple of its own ulp, at least that of the
        // smallest product fl(min1 * min2) when that is normal
        const double pmin = mn1 * mn2;
        if (pmin >= 0x1p-1022) {
            int e;
            frexp(pmin, &e);   // pmin in [2^(e-1), 2^e)
            q = max(q, e - 1 - 52);
        }
        pmax = mx1 * mx2;
    }
    // every scaled pair weight below 2^94 (a margin over the 2^95 of the
    // limbs for the rounding of pmax), every scaled lane weight a normal
    // finite number, and every nonzero result normal
    if (q < -1022 || q > 900)
        ok = false;
    if (ok && !(ldexp(pmax, -q) < 0x1p94))
        ok = false;
    if (ok && (any1 || any2)) {
        const double big = fmax(mx1, mx2), small = any1 && any2 ? fmin(mn1, mn2) : (any1 ? mn1 : mn2);
        if (!(ldexp(big, -q) < 0x1p1000) || !(ldexp(small, -q) >= 0x1p-1000))
            ok = false;
    }
    fx->q = ok ? q : 0;
    fx->scale = ok ? ldexp(1.0, -q) : 0.0;
    fx->unscale = ok ? ldexp(1.0, q) : 0.0;
    fx->ok = ok ? 1 : 0;
    if (!ok)
        atomicOr(flags, PC_FLAG_WFIXED);
}

// Self-pair weights of every catalogue in fixed point (k_wsq's sums, exact):
// 192-bit totals, three words per catalogue.
__global__ void k_wsq_fixed(int64_t ncell, const int32_t *start, const double *w, int wtype,
                            const pc_wfixed *fx, unsigned long long *out)
{
    const int c = blockIdx.y;
    const int64_t a = start[c * ncell], b = start[(c + 1) * ncell];
    const double sc = fx->scale;
    unsigned long long s0 = 0, s1 = 0, s2 = 0;
    for (int64_t i = a + blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < b;
         i += (int64_t)gridDim.x * blockDim.x) {
        const double P = wtype == 1 ? fma(sc, w[i], w[i] * sc) : fma(w[i] * sc, w[i], 0.0);
        unsigned long long l0, l1, l2;
        fixed_limbs(P, l0, l1, l2);
        s0 += l0;
        s1 += l1;
        s2 += l2;
    }
    __shared__ unsigned long long sm[3][256];
    sm[0][threadIdx.x] = s0;
    sm[1][threadIdx.x] = s1;
    sm[2][threadIdx.x] = s2;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st)
            for (int k = 0; k < 3; k++)
                sm[k][threadIdx.x] += sm[k][threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        unsigned long long v[3];
        fixed_words((long long)sm[0][0], (long long)sm[1][0], (long long)sm[2][0], v);
        fixed_atomic_add(out + 3 * (size_t)c, v);
    }
}

// Appendix B: autocorrelation counts are doubled (ordered pairs) and the
// N self-pairs of each catalogue join its bin 0 when the first edge is zero
// (with their weights, and separation 0).  The mean separation is the
// separation sum over the weight sum (doubling cancels).  Fixed-point weight
// sums (g_wfix, wsq_fix: three words per bin or catalogue) are doubled and
// completed in 192-bit integers and rounded to binary64 once.
__global__ void k_finalize(int32_t ncat, int32_t nbt, int autocorr, int e0_zero,
                           const pc_cat *cats, const unsigned long long *g_hist,
                           const double *g_whist, const double *g_rhist, const double *wsq,
                           const unsigned long long *g_wfix,
                           const unsigned long long *wsq_fix, const pc_wfixed *wfx,
                           unsigned long long *out_counts, double *out_wsum, double *out_ravg,
                           const int32_t *n_items_dev, const int32_t *n_blocks_dev,
                           int32_t *sizes_out)
{
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        sizes_out[0] = *n_items_dev;
        sizes_out[1] = *n_blocks_dev;
    }
    const int64_t total = (int64_t)ncat * nbt;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int c = (int)(t / nbt), b = (int)(t % nbt);
        unsigned long long v = g_hist[t];
        double w = g_whist ? g_whist[t] : 0.0;
        if (autocorr) {
            v *= 2ull;
            w *= 2.0;
            if (e0_zero && b == 0) {
                v += (unsigned long long)cats[c].n;
                if (wsq)
                    w += wsq[c];
            }
        }
        if (g_wfix) {
            unsigned long long f[3] = {g_wfix[3 * t], g_wfix[3 * t + 1], g_wfix[3 * t + 2]};
            if (autocorr) {
                f[2] = (f[2] << 1) | (f[1] >> 63);
                f[1] = (f[1] << 1) | (f[0] >> 63);
                f[0] <<= 1;
                if (e0_zero && b == 0 && wsq_fix) {
                    const unsigned long long d[3] = {wsq_fix[3 * c], wsq_fix[3 * c + 1],
                                                     wsq_fix[3 * c + 2]};
                    fixed_add(f, d);
                }
            }
            w = fixed_to_double(f, wfx->q);
        }
        out_counts[t] = v;
        if (out_wsum)
            out_wsum[t] = w;
        if (out_ravg) {
            const double r = autocorr ? 2.0 * g_rhist[t] : g_rhist[t];
            out_ravg[t] = w != 0.0 ? r / w : 0.0;
        }
    }
}

template <int M, bool P32, int W, bool EXP>
const void *sweep_fn(bool t16, bool unc, bool priv)
{
    if (priv)
        return t16 ? (const void *)&k_sweep<M, P32, W, true, false, true, EXP>
                   : (const void *)&k_sweep<M, P32, W, false, false, true, EXP>;
    if (t16)
        return (const void *)&k_sweep<M, P32, W, true, false, false, EXP>;
    if constexpr (M == PC_METRIC_R && W == 0) {
        if (unc) {
            if constexpr (P32)
                return (const void *)&k_sweep_o8<M, P32, W, false, true, false, EXP>;
            else
                return (const void *)&k_sweep<M, P32, W, false, true, false, EXP>;
        }
    }
    return (const void *)&k_sweep<M, P32, W, false, false, false, EXP>;
}

template <int M, bool P32>
const void *sweep_fn_w(int wmode, bool t16, bool unc, bool priv, bool exp)
{
    if (wmode == 2)
        return sweep_fn<M, P32, 2, false>(t16, unc, priv);
    if constexpr ((M == PC_METRIC_R || M == PC_METRIC_RPPI) && P32) {
        if (exp)
            return wmode == 1 ? sweep_fn<M, P32, 1, true>(t16, unc, priv)
                              : sweep_fn<M, P32, 0, true>(t16, unc, priv);
    }
    if (wmode == 1)
        return sweep_fn<M, P32, 1, false>(t16, unc, priv);
    return sweep_fn<M, P32, 0, false>(t16, unc, priv);
}

// wmode: 0 unweighted, 1 weight sums, 2 weight and mean-separation sums;
// exp: the float32 r sweep with x and y expanded (wmode 0 or 1).  On-sky
// pairs have binary64 kernels only.
const void *sweep_ptr(int metric, bool fp32, int wmode, bool t16, bool unc, bool priv,
                      bool exp)
{
    if (metric == PC_METRIC_MOCKS)
        return sweep_fn_w<PC_METRIC_MOCKS, false>(wmode, t16, unc, priv, false);
    if (metric == PC_METRIC_R)
        return fp32 ? sweep_fn_w<PC_METRIC_R, true>(wmode, t16, unc, priv, exp)
                    : sweep_fn_w<PC_METRIC_R, false>(wmode, t16, unc, priv, false);
    return fp32 ? sweep_fn_w<PC_METRIC_RPPI, true>(wmode, t16, unc, priv, exp)
                : sweep_fn_w<PC_METRIC_RPPI, false>(wmode, t16, unc, priv, false);
}

}  // namespace

hipError_t launch_sweep(hipStream_t s, int metric, bool fp32, int wmode, const SweepArgs &a,
                        int nwg)
{
    SweepArgs copy = a;
    void *args[] = {&copy};
    const void *fn = sweep_ptr(metric, fp32, wmode, a.B.tbl_wide != 0, a.copies == PC_WAVE,
                               a.priv != 0, a.xy_exp != 0);
    if (a.lds_bytes > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                           a.lds_bytes);
        if (e != hipSuccess)
            return e;
    }
    return hipLaunchKernel(fn, dim3(nwg), dim3(kSweepThreads), args, (size_t)a.lds_bytes, s);
}

int sweep_waves() { return kWaves; }

hipError_t sweep_occupancy(int metric, bool fp32, int wmode, bool t16, bool unc, bool priv,
                           bool exp, int lds_bytes, int *per_cu)
{
    const void *fn = sweep_ptr(metric, fp32, wmode, t16, unc, priv, exp);
    if (lds_bytes > 64 * 1024) {
        hipError_t e =
            hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, lds_bytes);
        if (e != hipSuccess)
            return e;
    }
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, fn, kSweepThreads,
                                                        (size_t)lds_bytes);
}

hipError_t launch_wsq(hipStream_t s, int32_t ncat, int64_t ncell, const int32_t *start,
                      const double *w, int wtype, double *out)
{
    hipLaunchKernelGGL(k_wsq, dim3(64, (unsigned)ncat), dim3(256), 0, s, ncell, start, w, wtype,
                       out);
    return hipGetLastError();
}

hipError_t launch_finalize(hipStream_t s, int32_t ncat, int32_t nbt, int autocorr, int e0_zero,
                           const pc_cat *cats, const unsigned long long *g_hist,
                           const double *g_whist, const double *g_rhist, const double *wsq,
                           const unsigned long long *g_wfix,
                           const unsigned long long *wsq_fix, const pc_wfixed *wfx,
                           unsigned long long *out_counts, double *out_wsum,
                           double *out_ravg, const int32_t *n_items_dev,
                           const int32_t *n_blocks_dev, int32_t *sizes_out)
{
    const int64_t total = (int64_t)ncat * nbt;
    int64_t g = (total + 255) / 256;
    g = g < 1 ? 1 : (g > 4096 ? 4096 : g);
    hipLaunchKernelGGL(k_finalize, dim3((unsigned)g), dim3(256), 0, s, ncat, nbt, autocorr,
                       e0_zero, cats, g_hist, g_whist, g_rhist, wsq, g_wfix, wsq_fix, wfx,
                       out_counts, out_wsum, out_ravg, n_items_dev, n_blocks_dev, sizes_out);
    return hipGetLastError();
}

hipError_t launch_wfixed_scan(hipStream_t s, int64_t n, const double *w, int side,
                              pc_wfixed *fx)
{
    if (n <= 0)
        return hipSuccess;
    int64_t g = (n + 255) / 256;
    g = g > 1024 ? 1024 : g;
    hipLaunchKernelGGL(k_wfixed_scan, dim3((unsigned)g), dim3(256), 0, s, n, w, side, fx);
    return hipGetLastError();
}

hipError_t launch_wfixed_plan(hipStream_t s, int wtype, int two_sided, pc_wfixed *fx,
                              unsigned *flags)
{
    hipLaunchKernelGGL(k_wfixed_plan, dim3(1), dim3(64), 0, s, wtype, two_sided, fx, flags);
    return hipGetLastError();
}

hipError_t launch_wsq_fixed(hipStream_t s, int32_t ncat, int64_t ncell, const int32_t *start,
                            const double *w, int wtype, const pc_wfixed *fx,
                            unsigned long long *out)
{
    hipLaunchKernelGGL(k_wsq_fixed, dim3(64, (unsigned)ncat), dim3(256), 0, s, ncell, start, w,
                       wtype, fx, out);
    return hipGetLastError();
}

}  // namespace pc
