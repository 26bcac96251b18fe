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
// Bin search: a lookup table indexed by the float32 bit pattern of the
// squared separation (monotone for non-negative values) gives, for most
// values, the histogram slot directly: slot = bin + 1, with slot 0 and slot
// nb + 1 catching separations below the first and above the last edge.  Table
// cells that meet an edge's decision band are flagged and resolved on a rare
// slow path.
//
// Two precisions:
//  * binary64: dx = fl(x_i - x_j) (+ offset), s = ((dx*dx + dy*dy) + dz*dz),
//    one rounding per operation -- the definition itself; flagged cells are
//    resolved by an exact binary64 comparison with the edge.
//  * float32: differences of box-frame float32 coordinates and fused
//    multiply-adds; a value inside an edge's error band is not decided but
//    queued for the binary64 recheck kernel.
#include <hip/hip_runtime.h>

#include "pc_common.h"
#include "pc_launch.h"

namespace pc {
namespace {

// LDS (address space 3) and read-only, wave-uniform global data read through
// the scalar cache (address space 4).
#define LDS __attribute__((address_space(3)))
#define KCONST __attribute__((address_space(4)))
typedef const LDS uint16_t *lds_u16p;
typedef const LDS float *lds_f32p;
typedef const LDS double *lds_f64p;
typedef LDS unsigned *lds_u32p;
typedef LDS double *lds_f64wp;
typedef const KCONST float *kf32p;
typedef const KCONST double *kf64p;

// LDS atomics on wave-private replicas
__device__ __forceinline__ void lds_add(LDS unsigned *p, unsigned v)
{
    __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
}
__device__ __forceinline__ void lds_add(LDS double *p, double v)
{
    __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
}

constexpr int kSweepThreads = 256;
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
    lds_u16p tbl;
    lds_f32p lo, hi;  // r / rp bands, followed (rppi) by the pi bands
    lds_f64p E, q;
    lds_u32p hist;    // this wave's histogram replicas
    lds_f64wp whist;
};

// Float32 slot of a value in a flagged table cell (or of any value when e
// carries PC_TBL_MULTI): number of bands wholly below it, i.e. bin + 1, or
// -1 when the value lies inside a band.
__device__ __forceinline__ int slow_slot(float s, unsigned e, lds_f32p lo, lds_f32p hi,
                                         int nedges)
{
    if (e & PC_TBL_BAND) {
        const int c = (int)(e & PC_TBL_MASK);
        if (s > hi[c])
            return c + 1;
        if (s < lo[c])
            return c;
        return -1;
    }
    int below = 0;
    for (int k = 0; k < nedges; k++) {
        if (s > hi[k])
            below++;
        else if (s >= lo[k])
            return -1;
    }
    return below;
}

// Binary64 slot of a value in a flagged cell: exact comparison with the edges.
__device__ __forceinline__ int slow_slot_exact(double s, unsigned e, lds_f64p E, int nedges)
{
    if (e & PC_TBL_BAND) {
        const int c = (int)(e & PC_TBL_MASK);
        return (s >= E[c]) ? c + 1 : c;
    }
    return count_le(E, nedges, s);
}

__device__ __forceinline__ void push_recheck(const SweepArgs &a, int i, int j, unsigned dcode)
{
    const unsigned slot = atomicAdd(a.rq_count, 1u);
    if (slot < a.rq_cap)
        a.rq[slot] = make_uint4((unsigned)i, (unsigned)j, dcode, 0u);
}

// Float32 pi bin of |dz|: t = |dz| * npi / pimax; the bin floor(t) is taken
// only when the fractional part of t keeps clear of both integers by the
// margin tau (covering the error of |dz|, of the product and the offset of
// the binary64 edges q_p from p * pimax / npi).  Returns -1 otherwise.
__device__ __forceinline__ int pi_fast(float pz, float inv_dpi, float tau, int npi)
{
    const float t = pz * inv_dpi;
    const float fl = floorf(t);
    const float fr = t - fl;
    const int k = (int)fl;
    return (fr > tau && fr < 1.0f - tau && k < npi) ? k : -1;
}

// ---- float32 pair -------------------------------------------------------
template <int M, bool W, bool TRI>
__device__ __forceinline__ void pair_f32(const SweepArgs &a, const Lds &L, lds_u32p hb,
                                         lds_f64wp whb, float ax, float ay, float az, double wi,
                                         int i, float xj, float yj, float zj, double wj, int j,
                                         unsigned dcode)
{
    const float dx = ax - xj, dy = ay - yj, dz = az - zj;
    if (M == PC_METRIC_R) {
        const float s = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
        bool cand = s <= a.B.s_top;
        if (TRI)
            cand = cand && (j > i);
        if (cand) {
            int slot = (int)L.tbl[__float_as_uint(s) >> a.B.tbl_shift];
            if ((unsigned)slot & kSlow) {
                slot = slow_slot(s, (unsigned)slot, L.lo, L.hi, a.B.nb + 1);
                if (slot < 0) {
                    push_recheck(a, i, j, dcode);
                    slot = 0;
                }
            }
            lds_add(&hb[slot], 1u);
            if (W)
                lds_add(&whb[slot], wi * wj);
        }
    } else {
        const float rp = fmaf(dy, dy, dx * dx);
        const float pz = fabsf(dz);
        bool cand = (rp <= a.B.s_top) && (pz <= a.B.pi_top);
        if (TRI)
            cand = cand && (j > i);
        if (cand) {
            const int npi = a.B.npi;
            int row = (int)L.tbl[__float_as_uint(rp) >> a.B.tbl_shift];
            int k = pi_fast(pz, a.B.inv_dpi, a.B.pi_tau, npi);
            int slot;
            if (((unsigned)row & kSlow) || k < 0) {
                if ((unsigned)row & kSlow)
                    row = slow_slot(rp, (unsigned)row, L.lo, L.hi, a.B.nb + 1);
                int ps = k + 1;
                if (k < 0)
                    ps = slow_slot(pz, PC_TBL_MULTI, L.lo + a.B.nb + 1, L.hi + a.B.nb + 1,
                                   npi + 1);
                // row / ps: bands below (bin + 1), or -1 when inside a band
                if (row == 0 || row == a.B.nb + 1 || ps == 0 || ps == npi + 1) {
                    slot = 0;   // definitely out of range
                } else if (row < 0 || ps < 0) {
                    push_recheck(a, i, j, dcode);
                    slot = 0;
                } else {
                    slot = row * npi + (ps - 1);
                }
            } else {
                slot = row * npi + k;
            }
            lds_add(&hb[slot], 1u);
            if (W)
                lds_add(&whb[slot], wi * wj);
        }
    }
}

// ---- binary64 pair ------------------------------------------------------
template <int M, bool W, bool TRI, bool OFS>
__device__ __forceinline__ void pair_f64(const SweepArgs &a, const Lds &L, lds_u32p hb,
                                         lds_f64wp whb, double xi, double yi, double zi,
                                         double Dx, double Dy, double Dz, double wi, int i,
                                         double xj, double yj, double zj, double wj, int j)
{
    double dx = __dsub_rn(xi, xj), dy = __dsub_rn(yi, yj), dz = __dsub_rn(zi, zj);
    if (OFS) {
        dx = __dadd_rn(dx, Dx);
        dy = __dadd_rn(dy, Dy);
        dz = __dadd_rn(dz, Dz);
    }
    if (M == PC_METRIC_R) {
        const double s =
            __dadd_rn(__dadd_rn(__dmul_rn(dx, dx), __dmul_rn(dy, dy)), __dmul_rn(dz, dz));
        bool cand = s < a.B.E_top;
        if (TRI)
            cand = cand && (j > i);
        if (cand) {
            int slot = (int)L.tbl[__float_as_uint(__double2float_rn(s)) >> a.B.tbl_shift];
            if ((unsigned)slot & kSlow)
                slot = slow_slot_exact(s, (unsigned)slot, L.E, a.B.nb + 1);
            lds_add(&hb[slot], 1u);
            if (W)
                lds_add(&whb[slot], wi * wj);
        }
    } else {
        const double rp = __dadd_rn(__dmul_rn(dx, dx), __dmul_rn(dy, dy));
        const double pz = fabs(dz);
        bool cand = (rp < a.B.E_top) && (pz < a.B.pimax);
        if (TRI)
            cand = cand && (j > i);
        if (cand) {
            const int npi = a.B.npi;
            int row = (int)L.tbl[__float_as_uint(__double2float_rn(rp)) >> a.B.tbl_shift];
            int k = pi_fast(__double2float_rn(pz), a.B.inv_dpi, a.B.pi_tau, npi);
            if ((unsigned)row & kSlow)
                row = slow_slot_exact(rp, (unsigned)row, L.E, a.B.nb + 1);
            if (k < 0)
                k = count_le(L.q, npi, pz) - 1;
            lds_add(&hb[row * npi + k], 1u);
            if (W)
                lds_add(&whb[row * npi + k], wi * wj);
        }
    }
}

// ---- item loops ----------------------------------------------------------
template <int M, bool W, bool TRI>
__device__ __forceinline__ void item_f32(const SweepArgs &a, const Lds &L, lds_u32p hb,
                                         lds_f64wp whb, int i, bool act, int j0, int j1,
                                         unsigned dcode)
{
    const float Lf = (float)a.L;
    const unsigned cx = dcode & 3u, cy = (dcode >> 2) & 3u, cz = (dcode >> 4) & 3u;
    const float Dx = cx == PC_D_PLUS ? Lf : (cx == PC_D_MINUS ? -Lf : 0.0f);
    const float Dy = cy == PC_D_PLUS ? Lf : (cy == PC_D_MINUS ? -Lf : 0.0f);
    const float Dz = cz == PC_D_PLUS ? Lf : (cz == PC_D_MINUS ? -Lf : 0.0f);
    // inactive lanes sit far away: their separations overflow to +inf
    const float ax = act ? a.X1[i] + Dx : 3.0e30f;
    const float ay = act ? a.Y1[i] + Dy : 3.0e30f;
    const float az = act ? a.Z1[i] + Dz : 3.0e30f;
    const double wi = (W && act) ? a.w1[i] : 0.0;
    // second-catalogue points are wave-uniform: read them through the scalar
    // cache (the arrays are not written during the sweep)
    const kf32p X2 = (kf32p)a.X2, Y2 = (kf32p)a.Y2, Z2 = (kf32p)a.Z2;
    const kf64p w2 = (kf64p)a.w2;
    constexpr int CH = W ? 4 : 8;
    int j = j0;
    for (; j + CH <= j1; j += CH) {
        float xs[CH], ys[CH], zs[CH];
        double ws[CH];
#pragma unroll
        for (int k = 0; k < CH; k++) {
            xs[k] = X2[j + k];
            ys[k] = Y2[j + k];
            zs[k] = Z2[j + k];
            ws[k] = W ? w2[j + k] : 0.0;
        }
#pragma unroll
        for (int k = 0; k < CH; k++)
            pair_f32<M, W, TRI>(a, L, hb, whb, ax, ay, az, wi, i, xs[k], ys[k], zs[k], ws[k],
                                j + k, dcode);
    }
    for (; j < j1; j++)
        pair_f32<M, W, TRI>(a, L, hb, whb, ax, ay, az, wi, i, X2[j], Y2[j], Z2[j],
                            W ? w2[j] : 0.0, j, dcode);
}

template <int M, bool W, bool TRI, bool OFS>
__device__ __forceinline__ void item_f64(const SweepArgs &a, const Lds &L, lds_u32p hb,
                                         lds_f64wp whb, int i, bool act, int j0, int j1,
                                         unsigned dcode)
{
    const double Dx = dval(dcode & 3u, a.L), Dy = dval((dcode >> 2) & 3u, a.L),
                 Dz = dval((dcode >> 4) & 3u, a.L);
    const double xi = act ? a.x1[i] : 1.0e300;
    const double yi = act ? a.y1[i] : 1.0e300;
    const double zi = act ? a.z1[i] : 1.0e300;
    const double wi = (W && act) ? a.w1[i] : 0.0;
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
#pragma unroll
        for (int k = 0; k < CH; k++)
            pair_f64<M, W, TRI, OFS>(a, L, hb, whb, xi, yi, zi, Dx, Dy, Dz, wi, i, xs[k], ys[k],
                                     zs[k], ws[k], j + k);
    }
    for (; j < j1; j++)
        pair_f64<M, W, TRI, OFS>(a, L, hb, whb, xi, yi, zi, Dx, Dy, Dz, wi, i, x2[j], y2[j],
                                 z2[j], W ? w2[j] : 0.0, j);
}

__device__ __forceinline__ int wave_fetch(int *counter, int lane)
{
    int v = 0;
    if (lane == 0)
        v = atomicAdd(counter, 1);
    return __builtin_amdgcn_readfirstlane(v);
}

// Merge this wave's replicas into the global bins and clear them.  Output bin
// b = k * npi + p lives in slot (k + 1) * npi + p; rows 0 and nb + 1 are the
// out-of-range catch-alls and are only cleared.
__device__ __forceinline__ void flush_hist(const SweepArgs &a, const Lds &L, int lane, bool W)
{
    __builtin_amdgcn_wave_barrier();
    const int npi = a.B.npi;
    for (int b = lane; b < a.nbt; b += PC_WAVE) {
        const int slot = b + npi;
        unsigned long long c = 0;
        double w = 0.0;
        for (int r = 0; r < a.copies; r++) {
            c += L.hist[r * a.slots + slot];
            L.hist[r * a.slots + slot] = 0u;
            if (W) {
                w += L.whist[r * a.slots + slot];
                L.whist[r * a.slots + slot] = 0.0;
            }
        }
        if (c)
            atomicAdd(&a.g_hist[b], c);
        if (W && w != 0.0)
            atomicAdd(&a.g_whist[b], w);
    }
    for (int t = lane; t < a.copies * npi; t += PC_WAVE) {
        const int r = t / npi, p = t % npi;
        L.hist[r * a.slots + p] = 0u;
        L.hist[r * a.slots + (a.B.nb + 1) * npi + p] = 0u;
        if (W) {
            L.whist[r * a.slots + p] = 0.0;
            L.whist[r * a.slots + (a.B.nb + 1) * npi + p] = 0.0;
        }
    }
    __builtin_amdgcn_wave_barrier();
}

template <int M, bool P32, bool W>
__global__ __launch_bounds__(kSweepThreads) void k_sweep(SweepArgs a)
{
    extern __shared__ __align__(16) unsigned char smem[];
    LDS unsigned char *sm = (LDS unsigned char *)smem;
    {
        const int tid = threadIdx.x;
        LDS uint16_t *tbl = (LDS uint16_t *)(sm + a.o_tbl);
        for (int k = tid; k < a.B.tbl_n; k += kSweepThreads)
            tbl[k] = a.tbl[k];
        // float bands: the r / rp edges, then (rppi) the pi edges
        const int ne = a.B.nb + 1, nq = (M == PC_METRIC_RPPI) ? a.B.npi + 1 : 0;
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
        LDS unsigned *hist = (LDS unsigned *)(sm + a.o_hist);
        for (int k = tid; k < kWaves * a.hist_stride; k += kSweepThreads)
            hist[k] = 0u;
        if (W) {
            LDS double *wh = (LDS double *)(sm + a.o_whist);
            for (int k = tid; k < kWaves * a.whist_stride; k += kSweepThreads)
                wh[k] = 0.0;
        }
    }
    __syncthreads();

    const int lane = threadIdx.x & (PC_WAVE - 1);
    const int wave = threadIdx.x / PC_WAVE;
    Lds L;
    L.tbl = (lds_u16p)(sm + a.o_tbl);
    L.lo = (lds_f32p)(sm + a.o_lo);
    L.hi = (lds_f32p)(sm + a.o_hi);
    L.E = (lds_f64p)(sm + a.o_E);
    L.q = (lds_f64p)(sm + a.o_q);
    L.hist = (lds_u32p)(sm + a.o_hist) + wave * a.hist_stride;
    L.whist = W ? (lds_f64wp)(sm + a.o_whist) + wave * a.whist_stride : (lds_f64wp) nullptr;
    // this lane's replica
    const int rep = lane & (a.copies - 1);
    lds_u32p hb = L.hist + rep * a.slots;
    lds_f64wp whb = W ? L.whist + rep * a.slots : (lds_f64wp) nullptr;

    // pairs added to this wave's uint32 replicas since the last flush
    unsigned long long pending = 0;
    const unsigned long long flush_at = 0x7fffffffull;

    int next = wave_fetch(a.counter, lane);
    while (next < a.n_items) {
        const int cur = next;
        next = wave_fetch(a.counter, lane);
        const pc_item it = a.items[cur];
        const int ni = (int)PC_META_NI(it.meta);
        const unsigned dcode = PC_META_DCODE(it.meta);
        const bool tri = PC_META_TRI(it.meta) != 0;
        const unsigned long long work = (unsigned long long)ni * (unsigned)(it.j1 - it.j0);
        if (pending + work > flush_at) {
            flush_hist(a, L, lane, W);
            pending = 0;
        }
        pending += work;
        const bool act = lane < ni;
        const int i = it.i0 + (act ? lane : 0);
        if (P32) {
            if (tri)
                item_f32<M, W, true>(a, L, hb, whb, i, act, it.j0, it.j1, dcode);
            else
                item_f32<M, W, false>(a, L, hb, whb, i, act, it.j0, it.j1, dcode);
        } else {
            if (tri)
                item_f64<M, W, true, false>(a, L, hb, whb, i, act, it.j0, it.j1, dcode);
            else if (dcode == 0u)
                item_f64<M, W, false, false>(a, L, hb, whb, i, act, it.j0, it.j1, dcode);
            else
                item_f64<M, W, false, true>(a, L, hb, whb, i, act, it.j0, it.j1, dcode);
        }
    }
    flush_hist(a, L, lane, W);
}

// ---- binary64 recheck of queued pairs ------------------------------------
template <int M, bool W>
__global__ __launch_bounds__(256) void k_recheck(SweepArgs a)
{
    const unsigned n = min(*a.rq_count, a.rq_cap);
    for (unsigned t = blockIdx.x * blockDim.x + threadIdx.x; t < n; t += gridDim.x * blockDim.x) {
        const uint4 e = a.rq[t];
        const int i = (int)e.x, j = (int)e.y;
        double s, pz;
        exact_sep<M>(a.x1[i], a.y1[i], a.z1[i], a.x2[j], a.y2[j], a.z2[j], e.z, a.L, &s, &pz);
        const int b = exact_bin<M>(s, pz, a.E, a.B.nb, a.q, a.B.npi, a.B.pimax);
        if (b >= 0) {
            atomicAdd(&a.g_hist[b], 1ull);
            if (W)
                atomicAdd(&a.g_whist[b], a.w1[i] * a.w2[j]);
        }
    }
}

__global__ void k_wsq(int64_t n, const double *w, double *out)
{
    double s = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        s += w[i] * w[i];
    __shared__ double sm[256];
    sm[threadIdx.x] = s;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st)
            sm[threadIdx.x] += sm[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        atomicAdd(out, sm[0]);
}

// Appendix B: autocorrelation counts are doubled (ordered pairs) and the N
// self-pairs join bin 0 when the first edge is zero.
__global__ void k_finalize(int32_t nbt, int autocorr, int e0_zero, int64_t n1,
                           const unsigned long long *g_hist, const double *g_whist,
                           const double *wsq, unsigned long long *out_counts, double *out_wsum)
{
    for (int b = blockIdx.x * blockDim.x + threadIdx.x; b < nbt; b += gridDim.x * blockDim.x) {
        unsigned long long c = g_hist[b];
        double w = g_whist ? g_whist[b] : 0.0;
        if (autocorr) {
            c *= 2ull;
            w *= 2.0;
            if (e0_zero && b == 0) {
                c += (unsigned long long)n1;
                if (wsq)
                    w += *wsq;
            }
        }
        out_counts[b] = c;
        if (out_wsum)
            out_wsum[b] = w;
    }
}

template <int M, bool P32, bool W>
const void *sweep_fn()
{
    return (const void *)&k_sweep<M, P32, W>;
}

const void *sweep_ptr(int metric, bool fp32, bool weighted)
{
    if (metric == PC_METRIC_R) {
        if (fp32)
            return weighted ? sweep_fn<PC_METRIC_R, true, true>()
                            : sweep_fn<PC_METRIC_R, true, false>();
        return weighted ? sweep_fn<PC_METRIC_R, false, true>()
                        : sweep_fn<PC_METRIC_R, false, false>();
    }
    if (fp32)
        return weighted ? sweep_fn<PC_METRIC_RPPI, true, true>()
                        : sweep_fn<PC_METRIC_RPPI, true, false>();
    return weighted ? sweep_fn<PC_METRIC_RPPI, false, true>()
                    : sweep_fn<PC_METRIC_RPPI, false, false>();
}

}  // namespace

hipError_t launch_sweep(hipStream_t s, int metric, bool fp32, bool weighted, const SweepArgs &a,
                        int nwg)
{
    SweepArgs copy = a;
    void *args[] = {&copy};
    const void *fn = sweep_ptr(metric, fp32, weighted);
    if (a.lds_bytes > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                           a.lds_bytes);
        if (e != hipSuccess)
            return e;
    }
    return hipLaunchKernel(fn, dim3(nwg), dim3(kSweepThreads), args, (size_t)a.lds_bytes, s);
}

hipError_t sweep_occupancy(int metric, bool fp32, bool weighted, int lds_bytes, int *per_cu)
{
    if (lds_bytes > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute(sweep_ptr(metric, fp32, weighted),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, lds_bytes);
        if (e != hipSuccess)
            return e;
    }
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, sweep_ptr(metric, fp32, weighted),
                                                        kSweepThreads, (size_t)lds_bytes);
}

hipError_t launch_recheck(hipStream_t s, int metric, bool weighted, const SweepArgs &a)
{
    const int grid = 1024;
    if (metric == PC_METRIC_R) {
        if (weighted)
            hipLaunchKernelGGL((k_recheck<PC_METRIC_R, true>), dim3(grid), dim3(256), 0, s, a);
        else
            hipLaunchKernelGGL((k_recheck<PC_METRIC_R, false>), dim3(grid), dim3(256), 0, s, a);
    } else {
        if (weighted)
            hipLaunchKernelGGL((k_recheck<PC_METRIC_RPPI, true>), dim3(grid), dim3(256), 0, s, a);
        else
            hipLaunchKernelGGL((k_recheck<PC_METRIC_RPPI, false>), dim3(grid), dim3(256), 0, s, a);
    }
    return hipGetLastError();
}

hipError_t launch_wsq(hipStream_t s, int64_t n, const double *w, double *out)
{
    int64_t g = (n + 255) / 256;
    g = g < 1 ? 1 : (g > 1024 ? 1024 : g);
    hipLaunchKernelGGL(k_wsq, dim3((unsigned)g), dim3(256), 0, s, n, w, out);
    return hipGetLastError();
}

hipError_t launch_finalize(hipStream_t s, int32_t nbt, int autocorr, int e0_zero, int64_t n1,
                           const unsigned long long *g_hist, const double *g_whist,
                           const double *wsq, unsigned long long *out_counts, double *out_wsum)
{
    const int g = (nbt + 255) / 256;
    hipLaunchKernelGGL(k_finalize, dim3(g), dim3(256), 0, s, nbt, autocorr, e0_zero, n1, g_hist,
                       g_whist, wsq, out_counts, out_wsum);
    return hipGetLastError();
}

}  // namespace pc
