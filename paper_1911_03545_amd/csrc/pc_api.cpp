// pc_api.cpp -- the C ABI: contexts, argument validation and the per-call
// pipeline (stage -> bounding box -> plan -> grid -> work list -> sweep with
// inline binary64 recheck -> finalize -> copy-out), all enqueued on the context's stream.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <vector>

#include "../../include/paircount.h"
#include "pc_common.h"
#include "pc_launch.h"
#include "pc_plan.h"

namespace {

struct DevBuf {
    void *p = nullptr;
    size_t cap = 0;
};

enum BufId {
    B_IN1X, B_IN1Y, B_IN1Z, B_IN1W, B_IN2X, B_IN2Y, B_IN2Z, B_IN2W,
    B_CNT, B_START1, B_START2, B_CELLOF, B_RANKOF,
    B_X1, B_Y1, B_Z1, B_XD1, B_YD1, B_ZD1, B_WD1, B_CS1,
    B_X2, B_Y2, B_Z2, B_XD2, B_YD2, B_ZD2, B_WD2, B_CS2,
    B_SCANTMP, B_BCNT, B_BOFF, B_BLOCKS, B_ICNT, B_IOFF, B_ITEMS,
    B_BINS, B_MISC, B_HIST, B_WHIST, B_OUTC, B_OUTW, B_PART, B_CTRS,
    B_COUNT
};

// byte offsets inside the B_MISC buffer
enum {
    M_FLAGS = 0,        // unsigned
    M_RQCOUNT = 16,     // unsigned
    M_CAND = 32,        // u64
    M_WSQ = 40,         // double
    M_OUT6 = 64,        // 6 doubles
    M_SIZE = 256
};

}  // namespace

// failure message of the last cf_create (no context exists to hold it)
static thread_local std::string g_create_error;

struct cf_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    std::string err;
    cf_stats stats;
    DevBuf buf[B_COUNT];
    void *pinned = nullptr;
    size_t pinned_cap = 0;
    hipEvent_t ev[8] = {};
    int num_cu = 256;
};

namespace {

cf_status fail(cf_ctx *c, cf_status st, const char *fmt, ...)
{
    char msg[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(msg, sizeof(msg), fmt, ap);
    va_end(ap);
    if (c)
        c->err = msg;
    return st;
}

#define HIPCHK(expr)                                                                     \
    do {                                                                                 \
        hipError_t e_ = (expr);                                                          \
        if (e_ != hipSuccess)                                                            \
            return fail(c, e_ == hipErrorOutOfMemory ? CF_ENOMEM : CF_EDEVICE,           \
                        "%s: %s (%s:%d)", #expr, hipGetErrorString(e_), __FILE__, __LINE__); \
    } while (0)

cf_status ensure(cf_ctx *c, BufId id, size_t bytes)
{
    bytes = std::max<size_t>(bytes, 256);
    DevBuf &b = c->buf[id];
    if (b.cap >= bytes)
        return CF_OK;
    if (b.p) {
        HIPCHK(hipStreamSynchronize(c->stream));
        HIPCHK(hipFree(b.p));
        b.p = nullptr;
        b.cap = 0;
    }
    size_t want = bytes + bytes / 4;
    hipError_t e = hipMalloc(&b.p, want);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(c, CF_ENOMEM, "hipMalloc(%zu) failed: %s", want, hipGetErrorString(e));
    }
    b.cap = want;
    return CF_OK;
}

cf_status ensure_pinned(cf_ctx *c, size_t bytes)
{
    if (c->pinned_cap >= bytes)
        return CF_OK;
    if (c->pinned) {
        HIPCHK(hipStreamSynchronize(c->stream));
        HIPCHK(hipHostFree(c->pinned));
        c->pinned = nullptr;
        c->pinned_cap = 0;
    }
    size_t want = std::max<size_t>(bytes, 1 << 16);
    hipError_t e = hipHostMalloc(&c->pinned, want, hipHostMallocDefault);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(c, CF_ENOMEM, "hipHostMalloc(%zu) failed", want);
    }
    c->pinned_cap = want;
    return CF_OK;
}

template <class T>
T *dptr(cf_ctx *c, BufId id)
{
    return static_cast<T *>(c->buf[id].p);
}

char *misc(cf_ctx *c) { return static_cast<char *>(c->buf[B_MISC].p); }

size_t dsize(int dtype) { return dtype == CF_F32 ? 4 : 8; }

cf_status check_catalog(cf_ctx *c, const cf_catalog *d, const char *name, bool theta,
                        bool unit_vectors)
{
    if (!d)
        return fail(c, CF_EINVAL, "%s is NULL", name);
    if (d->n < 0)
        return fail(c, CF_EINVAL, "%s.n < 0", name);
    if (d->dtype != CF_F32 && d->dtype != CF_F64)
        return fail(c, CF_EINVAL, "%s.dtype must be CF_F32 or CF_F64", name);
    if (d->mem != CF_MEM_HOST && d->mem != CF_MEM_DEVICE)
        return fail(c, CF_EINVAL, "%s.mem must be CF_MEM_HOST or CF_MEM_DEVICE", name);
    if (d->reserved != 0)
        return fail(c, CF_EINVAL, "%s.reserved must be 0", name);
    const bool need_z = !theta || unit_vectors;
    if (d->n > 0 && (!d->x || !d->y || (need_z && !d->z)))
        return fail(c, CF_EINVAL, "%s has NULL coordinate arrays", name);
    if (d->w && d->wdtype != CF_F32 && d->wdtype != CF_F64)
        return fail(c, CF_EINVAL, "%s.wdtype must be CF_F32 or CF_F64", name);
    return CF_OK;
}

cf_status check_edges(cf_ctx *c, const double *e, int32_t nb, bool allow_zero_first)
{
    if (!e)
        return fail(c, CF_EINVAL, "edges is NULL");
    if (nb < 1)
        return fail(c, CF_EINVAL, "nbins must be >= 1");
    if (nb + 1 > PC_MAX_EDGES)
        return fail(c, CF_EINVAL, "too many bins (max %d)", PC_MAX_EDGES - 1);
    for (int k = 0; k <= nb; k++)
        if (!isfinite(e[k]) || e[k] < 0.0)
            return fail(c, CF_EINVAL, "edge %d is negative or not finite", k);
    for (int k = 0; k < nb; k++)
        if (!(e[k] < e[k + 1]))
            return fail(c, CF_EINVAL, "edges must be strictly increasing (edge %d)", k);
    (void)allow_zero_first;
    return CF_OK;
}

// Stage one coordinate/weight array on the device; returns the device view.
cf_status stage(cf_ctx *c, const void *src, int dtype, int64_t n, int mem, BufId id,
                const void **out)
{
    if (mem == CF_MEM_DEVICE || n == 0) {
        *out = src;
        return CF_OK;
    }
    const size_t bytes = dsize(dtype) * (size_t)n;
    cf_status st = ensure(c, id, bytes);
    if (st)
        return st;
    HIPCHK(hipMemcpyAsync(c->buf[id].p, src, bytes, hipMemcpyHostToDevice, c->stream));
    *out = c->buf[id].p;
    return CF_OK;
}

struct Side {
    int64_t n = 0;
    const void *x = nullptr, *y = nullptr, *z = nullptr, *w = nullptr;
    int f32 = 0, wf32 = 0;
};

void record(cf_ctx *c, bool on, int k)
{
    if (on)
        (void)hipEventRecord(c->ev[k], c->stream);
}

float elapsed(cf_ctx *c, int a, int b)
{
    float ms = 0.0f;
    if (hipEventElapsedTime(&ms, c->ev[a], c->ev[b]) != hipSuccess) {
        (void)hipGetLastError();
        return 0.0f;
    }
    return ms;
}

// Grid one catalogue: cell index -> scan -> scatter.
cf_status grid_side(cf_ctx *c, const Side &s, const pc_grid &g, BufId start, BufId X, BufId Y,
                    BufId Z, BufId XD, BufId YD, BufId ZD, BufId WD, BufId CS)
{
    const int64_t n = s.n;
    cf_status st;
    if ((st = ensure(c, B_CNT, sizeof(int32_t) * (size_t)g.ncell)) ||
        (st = ensure(c, start, sizeof(int32_t) * (size_t)(g.ncell + 1))) ||
        (st = ensure(c, B_CELLOF, sizeof(int32_t) * (size_t)n)) ||
        (st = ensure(c, B_RANKOF, sizeof(int32_t) * (size_t)n)) ||
        (st = ensure(c, B_SCANTMP, sizeof(int32_t) * pc::scan_tmp_elems(g.ncell))) ||
        (st = ensure(c, X, sizeof(float) * (size_t)n)) ||
        (st = ensure(c, Y, sizeof(float) * (size_t)n)) ||
        (st = ensure(c, Z, sizeof(float) * (size_t)n)) ||
        (st = ensure(c, XD, sizeof(double) * (size_t)n)) ||
        (st = ensure(c, YD, sizeof(double) * (size_t)n)) ||
        (st = ensure(c, ZD, sizeof(double) * (size_t)n)) ||
        (st = ensure(c, CS, sizeof(int32_t) * (size_t)n)))
        return st;
    if (s.w && (st = ensure(c, WD, sizeof(double) * (size_t)n)))
        return st;
    unsigned *flags = (unsigned *)(misc(c) + M_FLAGS);
    HIPCHK(hipMemsetAsync(c->buf[B_CNT].p, 0, sizeof(int32_t) * (size_t)g.ncell, c->stream));
    HIPCHK(pc::launch_cell_index(c->stream, n, s.x, s.y, s.z, s.f32, g, dptr<unsigned>(c, B_CNT),
                                 dptr<int32_t>(c, B_CELLOF), dptr<int32_t>(c, B_RANKOF), flags));
    HIPCHK(pc::scan_exclusive(c->stream, dptr<int32_t>(c, B_CNT), g.ncell, dptr<int32_t>(c, start),
                              dptr<int32_t>(c, B_SCANTMP)));
    HIPCHK(pc::launch_scatter(c->stream, n, s.x, s.y, s.z, s.f32, s.w, s.wf32, g,
                              dptr<int32_t>(c, B_CELLOF), dptr<int32_t>(c, B_RANKOF),
                              dptr<int32_t>(c, start), dptr<float>(c, X), dptr<float>(c, Y),
                              dptr<float>(c, Z), dptr<double>(c, XD), dptr<double>(c, YD),
                              dptr<double>(c, ZD), s.w ? dptr<double>(c, WD) : nullptr,
                              dptr<int32_t>(c, CS)));
    return CF_OK;
}

int pow2_floor(int v)
{
    int p = 1;
    while (p * 2 <= v)
        p *= 2;
    return p;
}

cf_status run(cf_ctx *c, int metric, bool theta, const cf_catalog *d1, const cf_catalog *d2,
              const double *edges, int32_t nb, double pimax, int32_t npi, double boxsize,
              cf_precision prec, uint64_t *counts, double *wsum, const cf_options *opt_in)
{
    if (!c)
        return CF_EINVAL;
    c->err.clear();
    memset(&c->stats, 0, sizeof(c->stats));
    cf_options opt;
    cf_default_options(&opt);
    if (opt_in) {
        if (opt_in->struct_size != (int32_t)sizeof(cf_options))
            return fail(c, CF_EINVAL, "cf_options.struct_size mismatch");
        opt = *opt_in;
    }
    const bool unit_vec = theta && opt.theta_unit_vectors;
    cf_status st;
    if ((st = check_catalog(c, d1, "d1", theta, unit_vec)))
        return st;
    const bool autocorr = (d2 == nullptr);
    if (!autocorr && (st = check_catalog(c, d2, "d2", theta, unit_vec)))
        return st;
    if (!autocorr && ((d1->w == nullptr) != (d2->w == nullptr)))
        return fail(c, CF_EINVAL, "weights must be given for both catalogues or neither");
    if (!counts)
        return fail(c, CF_EINVAL, "counts is NULL");
    if (prec != CF_PREC_FP64 && prec != CF_PREC_FP32_RECHECK)
        return fail(c, CF_EINVAL, "unknown precision mode");
    if ((st = check_edges(c, edges, nb, true)))
        return st;
    if (metric == PC_METRIC_RPPI) {
        if (npi < 1 || npi > PC_MAX_NPI)
            return fail(c, CF_EINVAL, "npi must be in [1, %d]", PC_MAX_NPI);
        if (!(pimax > 0.0) || !isfinite(pimax))
            return fail(c, CF_EINVAL, "pimax must be positive and finite");
    } else {
        npi = 1;
    }
    const bool weighted = d1->w != nullptr;
    const int64_t nbt = (int64_t)nb * npi;
    if (nbt > (weighted ? PC_MAX_BINS_TOTAL / 2 : PC_MAX_BINS_TOTAL))
        return fail(c, CF_EINVAL, "too many output bins (%lld)", (long long)nbt);
    if (!isfinite(boxsize) && boxsize > 0.0)
        return fail(c, CF_EINVAL, "boxsize must be finite");
    if (theta && boxsize > 0.0)
        return fail(c, CF_EINVAL, "angular counts are never periodic");

    // theta: chord edges c_k = 2 sin(theta_k / 2) on the host
    std::vector<double> lin(edges, edges + nb + 1);
    if (theta) {
        const double d2r = M_PI / 180.0;
        for (int k = 0; k <= nb; k++) {
            if (edges[k] > 180.0)
                return fail(c, CF_ERANGE, "theta edge %d above 180 degrees", k);
            lin[k] = 2.0 * sin(0.5 * (edges[k] * d2r));
        }
        for (int k = 0; k < nb; k++)
            if (!(lin[k] < lin[k + 1]))
                return fail(c, CF_EINVAL, "theta edges give non-increasing chords");
    }
    const double reach_xy = lin[nb];
    const double reach_z = (metric == PC_METRIC_RPPI) ? pimax : lin[nb];
    const int64_t n1 = d1->n, n2 = autocorr ? d1->n : d2->n;
    if (n1 + (autocorr ? 0 : n2) > (int64_t)0x7fffff00)
        return fail(c, CF_EINVAL, "too many points for one call (limit 2^31 - 256)");

    HIPCHK(hipSetDevice(c->device));
    const bool timing = opt.collect_timing != 0;
    record(c, timing, 0);

    cf_status st2;
    if ((st2 = ensure(c, B_MISC, M_SIZE)))
        return st2;
    HIPCHK(hipMemsetAsync(c->buf[B_MISC].p, 0, M_SIZE, c->stream));

    const bool empty = (n1 == 0) || (!autocorr && n2 == 0);
    if (empty) {
        if (opt.output_on_device) {
            HIPCHK(hipMemsetAsync(counts, 0, sizeof(uint64_t) * nbt, c->stream));
            if (wsum)
                HIPCHK(hipMemsetAsync(wsum, 0, sizeof(double) * nbt, c->stream));
            HIPCHK(hipStreamSynchronize(c->stream));
        } else {
            memset(counts, 0, sizeof(uint64_t) * nbt);
            if (wsum)
                memset(wsum, 0, sizeof(double) * nbt);
        }
        return CF_OK;
    }

    // ---- stage inputs ----------------------------------------------------
    Side s1, s2;
    const cf_catalog *cats[2] = {d1, autocorr ? d1 : d2};
    Side *sides[2] = {&s1, &s2};
    const BufId inb[2][4] = {{B_IN1X, B_IN1Y, B_IN1Z, B_IN1W}, {B_IN2X, B_IN2Y, B_IN2Z, B_IN2W}};
    unsigned *flags = (unsigned *)(misc(c) + M_FLAGS);
    for (int k = 0; k < (autocorr ? 1 : 2); k++) {
        const cf_catalog *d = cats[k];
        Side &s = *sides[k];
        s.n = d->n;
        if (theta && !unit_vec) {
            const void *ra, *dec;
            if ((st2 = stage(c, d->x, d->dtype, d->n, d->mem, inb[k][0], &ra)) ||
                (st2 = stage(c, d->y, d->dtype, d->n, d->mem, inb[k][1], &dec)))
                return st2;
            // unit vectors go to the z slot and two fresh slots
            if ((st2 = ensure(c, inb[k][2], sizeof(double) * 3 * (size_t)d->n)))
                return st2;
            double *v = dptr<double>(c, inb[k][2]);
            HIPCHK(pc::launch_radec(c->stream, d->n, ra, dec, d->dtype == CF_F32, M_PI / 180.0,
                                    v, v + d->n, v + 2 * d->n, flags));
            s.x = v;
            s.y = v + d->n;
            s.z = v + 2 * d->n;
            s.f32 = 0;
        } else {
            if ((st2 = stage(c, d->x, d->dtype, d->n, d->mem, inb[k][0], &s.x)) ||
                (st2 = stage(c, d->y, d->dtype, d->n, d->mem, inb[k][1], &s.y)) ||
                (st2 = stage(c, d->z, d->dtype, d->n, d->mem, inb[k][2], &s.z)))
                return st2;
            s.f32 = d->dtype == CF_F32;
        }
        if (d->w) {
            if ((st2 = stage(c, d->w, d->wdtype, d->n, d->mem, inb[k][3], &s.w)))
                return st2;
            s.wf32 = d->wdtype == CF_F32;
            HIPCHK(pc::launch_check_weights(c->stream, d->n, s.w, s.wf32, flags));
        }
    }
    if (autocorr)
        s2 = s1;

    // ---- bounding box ------------------------------------------------------
    double lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
    const bool periodic = boxsize > 0.0;
    if (!periodic) {
        const int nparts = 256;
        if ((st2 = ensure(c, B_PART, sizeof(double) * 6 * 2 * nparts)))
            return st2;
        double *part = dptr<double>(c, B_PART);
        HIPCHK(pc::launch_minmax(c->stream, s1.n, s1.x, s1.y, s1.z, s1.f32, part, nparts, flags));
        int np = nparts;
        if (!autocorr) {
            HIPCHK(pc::launch_minmax(c->stream, s2.n, s2.x, s2.y, s2.z, s2.f32, part + 6 * nparts,
                                     nparts, flags));
            np = 2 * nparts;
        }
        double *out6 = (double *)(misc(c) + M_OUT6);
        HIPCHK(pc::launch_minmax_final(c->stream, part, np, out6));
        if ((st2 = ensure_pinned(c, 256)))
            return st2;
        HIPCHK(hipMemcpyAsync(c->pinned, misc(c), M_SIZE, hipMemcpyDeviceToHost, c->stream));
        HIPCHK(hipStreamSynchronize(c->stream));
        const char *hm = (const char *)c->pinned;
        unsigned hflags;
        memcpy(&hflags, hm + M_FLAGS, 4);
        if (hflags & PC_FLAG_RADEC)
            return fail(c, CF_ERANGE, "RA must lie in [0, 360] and DEC in [-90, 90]");
        if (hflags & PC_FLAG_NONFINITE)
            return fail(c, CF_EINVAL, "non-finite coordinate");
        if (hflags & PC_FLAG_WEIGHT)
            return fail(c, CF_EINVAL, "non-finite weight");
        double o6[6];
        memcpy(o6, hm + M_OUT6, sizeof(o6));
        for (int a = 0; a < 3; a++) {
            lo[a] = o6[a];
            hi[a] = o6[3 + a];
        }
    }

    // ---- plan ------------------------------------------------------------
    pc_grid g;
    int rc = pc::plan_grid(lo, hi, boxsize, reach_xy, reach_z, opt.slices_per_reach, &g);
    if (rc == CF_EUNSUPPORTED)
        return fail(c, CF_EUNSUPPORTED,
                    "periodic box needs every reach (r, rp, pi) at most boxsize/3");
    if (rc)
        return fail(c, (cf_status)rc, "grid planning failed");
    double scale = periodic ? boxsize : 0.0;
    for (int a = 0; a < 3; a++)
        scale = std::max(scale, g.extent[a]);
    const bool fp32 = prec == CF_PREC_FP32_RECHECK;
    int fscale_log2 = 0;
    if (fp32 && (rc = pc::fp32_scale_log2(metric, lin.data(), nb, scale, &fscale_log2)))
        return fail(c, (cf_status)rc, "float32 scaling failed");
    g.fscale = std::ldexp(1.0, fscale_log2);
    record(c, timing, 1);

    // ---- grid ------------------------------------------------------------
    if ((st2 = grid_side(c, s1, g, B_START1, B_X1, B_Y1, B_Z1, B_XD1, B_YD1, B_ZD1, B_WD1, B_CS1)))
        return st2;
    if (!autocorr &&
        (st2 = grid_side(c, s2, g, B_START2, B_X2, B_Y2, B_Z2, B_XD2, B_YD2, B_ZD2, B_WD2, B_CS2)))
        return st2;
    // the bin description is built on the host while the gridding kernels run
    pc::HostBins hb;
    rc = pc::build_bins(metric, fp32, lin.data(), nb, pimax, npi, scale, fscale_log2, &hb);
    if (rc)
        return fail(c, (cf_status)rc, "bin description failed");
    if ((st2 = ensure(c, B_BINS, hb.buf.size())))
        return st2;
    if ((st2 = ensure_pinned(c, std::max<size_t>(hb.buf.size(), 256))))
        return st2;
    // pinned staging keeps the upload asynchronous; no copy that reads or
    // writes the pinned buffer is pending here (the last one was followed by
    // a synchronisation)
    memcpy(c->pinned, hb.buf.data(), hb.buf.size());
    HIPCHK(hipMemcpyAsync(c->buf[B_BINS].p, c->pinned, hb.buf.size(), hipMemcpyHostToDevice,
                          c->stream));
    record(c, timing, 2);

    // ---- work list ---------------------------------------------------------
    const int32_t ncol = g.n[0] * g.n[1];
    const int64_t maxblocks = n1 / PC_BLOCK_I + ncol + 1;
    const int chunk = opt.chunk > 0 ? std::min(opt.chunk, 1 << 20) : 2048;
    if ((st2 = ensure(c, B_BCNT, sizeof(int32_t) * (size_t)ncol)) ||
        (st2 = ensure(c, B_BOFF, sizeof(int32_t) * (size_t)(ncol + 1))) ||
        (st2 = ensure(c, B_BLOCKS, sizeof(pc_block) * (size_t)maxblocks)) ||
        (st2 = ensure(c, B_ICNT, sizeof(int32_t) * (size_t)maxblocks)) ||
        (st2 = ensure(c, B_IOFF, sizeof(int32_t) * (size_t)(maxblocks + 1))) ||
        (st2 = ensure(c, B_SCANTMP, sizeof(int32_t) * pc::scan_tmp_elems(std::max<int64_t>(
                                        std::max<int64_t>(maxblocks, ncol), g.ncell)))))
        return st2;
    const int32_t *start1 = dptr<int32_t>(c, B_START1);
    const int32_t *start2 = autocorr ? start1 : dptr<int32_t>(c, B_START2);
    HIPCHK(pc::launch_block_count(c->stream, ncol, g.n[2], start1, dptr<int32_t>(c, B_BCNT)));
    HIPCHK(pc::scan_exclusive(c->stream, dptr<int32_t>(c, B_BCNT), ncol, dptr<int32_t>(c, B_BOFF),
                              dptr<int32_t>(c, B_SCANTMP)));
    HIPCHK(pc::launch_block_emit(c->stream, ncol, g.n[2], start1, dptr<int32_t>(c, B_BOFF),
                                 dptr<pc_block>(c, B_BLOCKS)));
    const int32_t *nblocks_dev = dptr<int32_t>(c, B_BOFF) + ncol;
    HIPCHK(hipMemsetAsync(c->buf[B_ICNT].p, 0, sizeof(int32_t) * (size_t)maxblocks, c->stream));
    unsigned long long *cand = (unsigned long long *)(misc(c) + M_CAND);
    HIPCHK(pc::launch_item_count(c->stream, (int32_t)maxblocks, nblocks_dev,
                                 dptr<pc_block>(c, B_BLOCKS), g, start2, dptr<int32_t>(c, B_CS1),
                                 autocorr ? 1 : 0, chunk, dptr<int32_t>(c, B_ICNT), cand));
    HIPCHK(pc::scan_exclusive(c->stream, dptr<int32_t>(c, B_ICNT), maxblocks,
                              dptr<int32_t>(c, B_IOFF), dptr<int32_t>(c, B_SCANTMP)));
    // item count to the host (sizes the item array and the sweep launch)
    int32_t hcounts[2];
    HIPCHK(hipMemcpyAsync(c->pinned, dptr<int32_t>(c, B_IOFF) + maxblocks, sizeof(int32_t),
                          hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipMemcpyAsync((char *)c->pinned + 8, nblocks_dev, sizeof(int32_t),
                          hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    memcpy(&hcounts[0], c->pinned, 4);
    memcpy(&hcounts[1], (char *)c->pinned + 8, 4);
    const int32_t n_items = hcounts[0];
    if (n_items < 0)
        return fail(c, CF_EOVERFLOW, "work-item count overflow");
    if ((st2 = ensure(c, B_ITEMS, sizeof(pc_item) * (size_t)std::max(n_items, 1))))
        return st2;
    HIPCHK(pc::launch_item_emit(c->stream, (int32_t)maxblocks, nblocks_dev,
                                dptr<pc_block>(c, B_BLOCKS), g, start2, dptr<int32_t>(c, B_CS1),
                                autocorr ? 1 : 0, chunk, dptr<int32_t>(c, B_IOFF),
                                dptr<pc_item>(c, B_ITEMS)));
    record(c, timing, 3);

    // ---- sweep -------------------------------------------------------------
    if ((st2 = ensure(c, B_HIST, sizeof(unsigned long long) * nbt)) ||
        (st2 = ensure(c, B_WHIST, sizeof(double) * nbt)) ||
        (st2 = ensure(c, B_OUTC, sizeof(unsigned long long) * nbt)) ||
        (st2 = ensure(c, B_OUTW, sizeof(double) * nbt)) ||
        (st2 = ensure(c, B_CTRS, sizeof(int32_t) * PC_STREAMS * PC_STREAM_STRIDE)))
        return st2;
    HIPCHK(hipMemsetAsync(c->buf[B_CTRS].p, 0, sizeof(int32_t) * PC_STREAMS * PC_STREAM_STRIDE,
                          c->stream));
    HIPCHK(hipMemsetAsync(c->buf[B_HIST].p, 0, sizeof(unsigned long long) * nbt, c->stream));
    HIPCHK(hipMemsetAsync(c->buf[B_WHIST].p, 0, sizeof(double) * nbt, c->stream));
    const char *bb = (const char *)c->buf[B_BINS].p;
    pc::SweepArgs a;
    memset(&a, 0, sizeof(a));
    a.items = dptr<pc_item>(c, B_ITEMS);
    a.n_items = n_items;
    a.counter = dptr<int32_t>(c, B_CTRS);
    a.X1 = dptr<float>(c, B_X1);
    a.Y1 = dptr<float>(c, B_Y1);
    a.Z1 = dptr<float>(c, B_Z1);
    a.x1 = dptr<double>(c, B_XD1);
    a.y1 = dptr<double>(c, B_YD1);
    a.z1 = dptr<double>(c, B_ZD1);
    a.w1 = weighted ? dptr<double>(c, B_WD1) : nullptr;
    if (autocorr) {
        a.X2 = a.X1; a.Y2 = a.Y1; a.Z2 = a.Z1;
        a.x2 = a.x1; a.y2 = a.y1; a.z2 = a.z1;
        a.w2 = a.w1;
    } else {
        a.X2 = dptr<float>(c, B_X2);
        a.Y2 = dptr<float>(c, B_Y2);
        a.Z2 = dptr<float>(c, B_Z2);
        a.x2 = dptr<double>(c, B_XD2);
        a.y2 = dptr<double>(c, B_YD2);
        a.z2 = dptr<double>(c, B_ZD2);
        a.w2 = weighted ? dptr<double>(c, B_WD2) : nullptr;
    }
    a.L = periodic ? boxsize : 0.0;
    a.Lf32 = (float)(a.L * g.fscale);
    a.B = hb.hdr;
    a.lo = (const float *)(bb + hb.lay.lo);
    a.hi = (const float *)(bb + hb.lay.hi);
    a.E = (const double *)(bb + hb.lay.E);
    a.plo = (const float *)(bb + hb.lay.plo);
    a.phi = (const float *)(bb + hb.lay.phi);
    a.q = (const double *)(bb + hb.lay.q);
    a.tbl = (const uint16_t *)(bb + hb.lay.tbl);
    a.g_hist = dptr<unsigned long long>(c, B_HIST);
    a.g_whist = weighted ? dptr<double>(c, B_WHIST) : nullptr;
    a.rq_count = (unsigned *)(misc(c) + M_RQCOUNT);
    a.nbt = (int32_t)nbt;
    a.slots = (int32_t)((nb + 2) * npi);
    // Histogram replicas: one per lane (unconditional updates, no candidate
    // branch) for unweighted 1-D counts with few bins, else a few shared ones.
    const bool unc_ok = metric == PC_METRIC_R && !weighted && !hb.hdr.tbl_wide &&
                        PC_WAVE * (a.slots | 1) <= PC_MAX_HIST_WAVE;
    int copies;
    if (opt.hist_copies > 0)
        copies = pow2_floor(std::min(opt.hist_copies, PC_WAVE));
    else
        copies = unc_ok ? PC_WAVE
                        : pow2_floor((int)std::max<int64_t>(1, std::min<int64_t>(16, 512 / nbt)));
    if (copies == PC_WAVE && !unc_ok)
        copies = PC_WAVE / 2;
    while (copies > 1 && copies * (a.slots | 1) > PC_MAX_HIST_WAVE)
        copies /= 2;
    a.copies = copies;
    // dynamic LDS layout
    int off = 0;
    auto take = [&](int bytes) {
        const int o = off;
        off += (bytes + 15) & ~15;
        return o;
    };
    const int ne = nb + 1, nq = hb.nq;
    a.o_tbl = 0;   // the kernel keeps the table in a static LDS array
    a.o_lo = take(4 * (ne + nq));
    a.o_hi = take(4 * (ne + nq));
    a.o_E = take(8 * ne);
    a.o_q = take(8 * nq);
    // replica stride: odd, so the 64 lanes' copies of one slot spread over banks
    a.rep_stride = a.slots | 1;
    a.hist_stride = (int32_t)(copies * a.rep_stride);
    a.o_hist = take(4 * a.hist_stride);   // shared by the workgroup's waves
    a.whist_stride = weighted ? (int32_t)(copies * a.rep_stride) : 0;
    a.o_whist = take(weighted ? 8 * a.whist_stride : 0);
    a.lds_bytes = off;
    // static LDS of the sweep: the lookup table
    if (off + (PC_TBL8_MAX > 2 * PC_TBL16_MAX ? PC_TBL8_MAX : 2 * PC_TBL16_MAX) > 160 * 1024)
        return fail(c, CF_EINVAL, "bin configuration needs too much LDS (%d bytes)", off);

    int per_cu = 0;
    HIPCHK(pc::sweep_occupancy(metric, fp32, weighted, hb.hdr.tbl_wide != 0,
                               copies == PC_WAVE, off, &per_cu));
    per_cu = std::max(per_cu, 1);
    const int waves = pc::sweep_waves();
    int nwg = (int)std::min<int64_t>((n_items + waves - 1) / waves, (int64_t)c->num_cu * per_cu);
    nwg = std::max(nwg, 1);
    c->stats.sweep_workgroups = nwg;
    c->stats.hist_copies = copies;
    double *wsq = nullptr;
    if (weighted && autocorr && hb.hdr.e0_zero)
        wsq = (double *)(misc(c) + M_WSQ);
    unsigned long long *outc = opt.output_on_device ? (unsigned long long *)counts
                                                    : dptr<unsigned long long>(c, B_OUTC);
    double *outw = wsum ? (opt.output_on_device ? wsum : dptr<double>(c, B_OUTW)) : nullptr;
    const size_t need = M_SIZE + (sizeof(uint64_t) + sizeof(double)) * (size_t)nbt;
    if ((st2 = ensure_pinned(c, need)))
        return st2;
    char *hp = (char *)c->pinned;
    record(c, timing, 4);
    if (n_items > 0)
        HIPCHK(pc::launch_sweep(c->stream, metric, fp32, weighted, a, nwg));
    record(c, timing, 5);
    // ---- finalize ------------------------------------------------------------
    if (wsq) {
        HIPCHK(hipMemsetAsync(wsq, 0, sizeof(double), c->stream));
        HIPCHK(pc::launch_wsq(c->stream, n1, dptr<double>(c, B_WD1), wsq));
    }
    HIPCHK(pc::launch_finalize(c->stream, (int32_t)nbt, autocorr ? 1 : 0, hb.hdr.e0_zero, n1,
                               a.g_hist, a.g_whist, wsq, outc, outw));
    HIPCHK(hipMemcpyAsync(hp, misc(c), M_SIZE, hipMemcpyDeviceToHost, c->stream));
    if (!opt.output_on_device) {
        HIPCHK(hipMemcpyAsync(hp + M_SIZE, outc, sizeof(uint64_t) * nbt, hipMemcpyDeviceToHost,
                              c->stream));
        if (outw)
            HIPCHK(hipMemcpyAsync(hp + M_SIZE + sizeof(uint64_t) * nbt, outw,
                                  sizeof(double) * nbt, hipMemcpyDeviceToHost, c->stream));
    }
    record(c, timing, 6);
    HIPCHK(hipStreamSynchronize(c->stream));
    unsigned rqn = 0;
    memcpy(&rqn, hp + M_RQCOUNT, 4);

    unsigned hflags;
    memcpy(&hflags, hp + M_FLAGS, 4);
    if (hflags & PC_FLAG_RADEC)
        return fail(c, CF_ERANGE, "RA must lie in [0, 360] and DEC in [-90, 90]");
    if (hflags & PC_FLAG_NONFINITE)
        return fail(c, CF_EINVAL, "non-finite coordinate");
    if (hflags & PC_FLAG_RANGE)
        return fail(c, CF_ERANGE, "periodic coordinate outside [0, boxsize]");
    if (hflags & PC_FLAG_WEIGHT)
        return fail(c, CF_EINVAL, "non-finite weight");
    if (!opt.output_on_device) {
        memcpy(counts, hp + M_SIZE, sizeof(uint64_t) * nbt);
        if (wsum)
            memcpy(wsum, hp + M_SIZE + sizeof(uint64_t) * nbt, sizeof(double) * nbt);
    }
    unsigned long long cnd;
    memcpy(&cnd, hp + M_CAND, 8);
    cf_stats &S = c->stats;
    for (int k = 0; k < 3; k++) {
        S.grid[k] = g.n[k];
        S.cell_width[k] = g.width[k];
    }
    S.zreach = g.zreach;
    S.n_blocks = hcounts[1];
    S.n_items = n_items;
    S.candidate_pairs = cnd;
    S.rechecks = (uint64_t)rqn;
    if (timing) {
        S.t_prepare_ms = elapsed(c, 0, 1);
        S.t_grid_ms = elapsed(c, 1, 2);
        S.t_worklist_ms = elapsed(c, 2, 3);
        S.t_sweep_ms = elapsed(c, 4, 5);
        S.t_finalize_ms = elapsed(c, 5, 6);
        S.t_total_ms = elapsed(c, 0, 6);
    }
    return CF_OK;
}

}  // namespace

extern "C" {

void cf_default_options(cf_options *opt)
{
    if (!opt)
        return;
    memset(opt, 0, sizeof(*opt));
    opt->struct_size = (int32_t)sizeof(cf_options);
    opt->slices_per_reach = 16;
    opt->chunk = 2048;
}

cf_status cf_create(int device, void *hip_stream, cf_ctx **out)
{
    if (!out)
        return CF_EINVAL;
    *out = nullptr;
    int ndev = 0;
    hipError_t e = hipGetDeviceCount(&ndev);
    if (e != hipSuccess || ndev <= 0) {
        g_create_error = std::string("hipGetDeviceCount: ") + hipGetErrorString(e) +
                         " (devices: " + std::to_string(ndev) + ")";
        (void)hipGetLastError();
        return CF_EDEVICE;
    }
    if (device < 0 || device >= ndev) {
        g_create_error = "device index out of range";
        return CF_EINVAL;
    }
    e = hipSetDevice(device);
    if (e != hipSuccess) {
        g_create_error = std::string("hipSetDevice: ") + hipGetErrorString(e);
        return CF_EDEVICE;
    }
    cf_ctx *c = new cf_ctx();
    c->device = device;
    c->stream = (hipStream_t)hip_stream;
    memset(&c->stats, 0, sizeof(c->stats));
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) == hipSuccess && prop.multiProcessorCount > 0)
        c->num_cu = prop.multiProcessorCount;
    for (auto &ev : c->ev) {
        e = hipEventCreate(&ev);
        if (e != hipSuccess) {
            g_create_error = std::string("hipEventCreate: ") + hipGetErrorString(e);
            cf_destroy(c);
            return CF_EDEVICE;
        }
    }
    g_create_error.clear();
    *out = c;
    return CF_OK;
}

cf_status cf_destroy(cf_ctx *c)
{
    if (!c)
        return CF_EINVAL;
    (void)hipSetDevice(c->device);
    (void)hipStreamSynchronize(c->stream);
    for (auto &b : c->buf)
        if (b.p)
            (void)hipFree(b.p);
    if (c->pinned)
        (void)hipHostFree(c->pinned);
    for (auto &ev : c->ev)
        if (ev)
            (void)hipEventDestroy(ev);
    delete c;
    return CF_OK;
}

const char *cf_last_error(const cf_ctx *c)
{
    if (!c)
        return g_create_error.empty() ? "no context" : g_create_error.c_str();
    return c->err.c_str();
}

cf_status cf_get_stats(const cf_ctx *c, cf_stats *out)
{
    if (!c || !out)
        return CF_EINVAL;
    *out = c->stats;
    return CF_OK;
}

cf_status count_pairs_r_ex(cf_ctx *c, const cf_catalog *d1, const cf_catalog *d2,
                           const double *edges, int32_t nbins, double boxsize, cf_precision prec,
                           uint64_t *counts, double *wsum, const cf_options *opt)
{
    return run(c, PC_METRIC_R, false, d1, d2, edges, nbins, 0.0, 1, boxsize, prec, counts, wsum,
               opt);
}

cf_status count_pairs_r(cf_ctx *c, const cf_catalog *d1, const cf_catalog *d2,
                        const double *edges, int32_t nbins, double boxsize, cf_precision prec,
                        uint64_t *counts, double *wsum)
{
    return count_pairs_r_ex(c, d1, d2, edges, nbins, boxsize, prec, counts, wsum, nullptr);
}

cf_status count_pairs_rppi_ex(cf_ctx *c, const cf_catalog *d1, const cf_catalog *d2,
                              const double *rp_edges, int32_t nrp, double pimax, int32_t npi,
                              double boxsize, cf_precision prec, uint64_t *counts, double *wsum,
                              const cf_options *opt)
{
    return run(c, PC_METRIC_RPPI, false, d1, d2, rp_edges, nrp, pimax, npi, boxsize, prec, counts,
               wsum, opt);
}

cf_status count_pairs_rppi(cf_ctx *c, const cf_catalog *d1, const cf_catalog *d2,
                           const double *rp_edges, int32_t nrp, double pimax, int32_t npi,
                           double boxsize, cf_precision prec, uint64_t *counts, double *wsum)
{
    return count_pairs_rppi_ex(c, d1, d2, rp_edges, nrp, pimax, npi, boxsize, prec, counts, wsum,
                               nullptr);
}

cf_status count_pairs_theta_ex(cf_ctx *c, const cf_catalog *d1, const cf_catalog *d2,
                               const double *theta_edges_deg, int32_t nbins, cf_precision prec,
                               uint64_t *counts, double *wsum, const cf_options *opt)
{
    return run(c, PC_METRIC_R, true, d1, d2, theta_edges_deg, nbins, 0.0, 1, 0.0, prec, counts,
               wsum, opt);
}

cf_status count_pairs_theta(cf_ctx *c, const cf_catalog *d1, const cf_catalog *d2,
                            const double *theta_edges_deg, int32_t nbins, cf_precision prec,
                            uint64_t *counts, double *wsum)
{
    return count_pairs_theta_ex(c, d1, d2, theta_edges_deg, nbins, prec, counts, wsum, nullptr);
}

}  // extern "C"
