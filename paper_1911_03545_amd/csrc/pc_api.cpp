// pc_api.cpp -- the C ABI: contexts, argument validation and the per-call
// pipeline (stage -> bounding box -> plan -> grid -> work list -> sweep with
// inline binary64 recheck -> finalize -> copy-out), all enqueued on the context's stream.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <map>
#include <string>
#include <thread>
#include <vector>

#include "../../include/paircount.h"
#include "pc_common.h"
#include "pc_launch.h"
#include "pc_plan.h"

namespace {

struct DevBuf {
    void *p = nullptr;
    size_t cap = 0;
    bool user = false;   // came from the registered allocator
};

enum BufId {
    B_IN1X, B_IN1Y, B_IN1Z, B_IN1W, B_IN2X, B_IN2Y, B_IN2Z, B_IN2W,
    B_CNT, B_START1, B_START2, B_CELLOF, B_RANKOF, B_PERM, B_REC, B_WOFF, B_LAY, B_COLS,
    B_X1, B_Y1, B_Z1, B_XD1, B_YD1, B_ZD1, B_WD1, B_CS1,
    B_X2, B_Y2, B_Z2, B_XD2, B_YD2, B_ZD2, B_WD2, B_CS2, B_Q1, B_Q2,
    B_SCANTMP, B_BCNT, B_BOFF, B_BLOCKS, B_ICNT, B_IOFF, B_ITEMS, B_ICELL,
    B_BINS, B_BANDS, B_MISC, B_HIST, B_WHIST, B_OUTC, B_OUTW, B_RHIST, B_OUTR, B_PART, B_CTRS, B_CATS1, B_CATS2, B_UV1, B_UV2, B_WSQ,
    B_COUNT
};

// byte offsets inside the B_MISC buffer
enum {
    M_FLAGS = 0,        // unsigned
    M_RQCOUNT = 16,     // unsigned
    M_CAND = 32,        // u64
    M_SIZES = 40,       // 2 int32: work items, blocks (copied by the finalize kernel)
    M_FLUSH = 48,       // unsigned: mid-sweep histogram flushes
    M_OUT6 = 64,        // 6 doubles
    M_WFIX = 128,       // pc_wfixed: grid of the fixed-point weight sums
    M_SIZE = 256
};
static_assert(M_WFIX + sizeof(pc::pc_wfixed) <= M_SIZE, "misc layout");

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
    // graph replay of repeated identical calls (cf_options.use_graph)
    int32_t last_items = 0;          // work items of the last eager call
    std::vector<char> last_shape;    // shape of the last eager call (see run)
    // sweep workgroups per CU by kernel variant and LDS size
    std::map<std::vector<int64_t>, int> occupancy;
    std::vector<char> gkey;          // signature of the cached graph
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    hipStream_t cap_stream = nullptr;
    void *gpin = nullptr;            // pinned staging owned by the graph
    size_t gpin_cap = 0;
    size_t g_misc = 0, g_out = 0, g_nout = 0;
    bool g_wsum = false;
    bool g_ravg = false;
    cf_stats gstats;
    // autotuned choices per workload class
    struct Tuned {
        int32_t slices_per_reach, chunk, angular_grid, xy_refine;
    };
    std::map<std::vector<int64_t>, Tuned> tuned;
    // registered scratch allocator (cf_set_allocator); NULL: hipMalloc
    cf_alloc_fn alloc = nullptr;
    cf_free_fn free_ = nullptr;
    void *alloc_user = nullptr;
    // fixed device scratch of count_pairs_r_noalloc (shared by every context
    // on the device); while `arena` is set, ensure() carves buffers out of it
    // from arena_off on instead of allocating
    char *scratch = nullptr;
    size_t scratch_cap = 0;
    bool arena = false;
    size_t arena_off = 0;
    // small inputs the last eager call left on the device (the catalogue
    // descriptors, the bin description with its table): the bytes and the
    // buffer they went to.  An identical repeat skips its copy (and the table
    // build); a buffer (re)allocation, a graph capture or replay clears them.
    struct Upload {
        std::vector<char> bytes;
        const void *p = nullptr;
    };
    Upload up_cats1, up_bins;
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

void drop_graph(cf_ctx *c);

// Give a scratch buffer back to whichever allocator made it.
hipError_t release(cf_ctx *c, DevBuf &b)
{
    hipError_t e = hipSuccess;
    if (b.p) {
        if (b.user)
            c->free_(b.p, c->alloc_user);
        else
            e = hipFree(b.p);
    }
    b.p = nullptr;
    b.cap = 0;
    b.user = false;
    return e;
}

bool upload_fresh(const cf_ctx::Upload &u, const void *dev, const void *src, size_t n)
{
    return u.p == dev && u.bytes.size() == n && memcmp(u.bytes.data(), src, n) == 0;
}

void upload_keep(cf_ctx::Upload &u, const void *dev, const void *src, size_t n)
{
    u.p = dev;
    u.bytes.assign(static_cast<const char *>(src), static_cast<const char *>(src) + n);
}

void uploads_clear(cf_ctx *c)
{
    c->up_cats1 = cf_ctx::Upload{};
    c->up_bins = cf_ctx::Upload{};
}

cf_status ensure(cf_ctx *c, BufId id, size_t bytes)
{
    bytes = std::max<size_t>(bytes, 256);
    DevBuf &b = c->buf[id];
    if (b.cap >= bytes)
        return CF_OK;
    if (c->arena) {
        // no-allocation call: the next 256-byte aligned piece of the fixed
        // scratch (a buffer that grows within a call leaves its old piece),
        // with the same quarter of headroom as an allocated buffer so that
        // both paths see identical capacities; the last MiB stays unused
        const size_t off = (c->arena_off + 255) & ~(size_t)255;
        const size_t want = bytes + bytes / 4;
        if (off + want + (1u << 20) > c->scratch_cap)
            return fail(c, CF_EINVAL,
                        "the call needs more than the %zu bytes of fixed scratch of "
                        "count_pairs_r_noalloc (%zu in use, %zu more asked); use "
                        "count_pairs_r_ex", c->scratch_cap, off, want);
        b.p = c->scratch + off;
        b.cap = want;
        b.user = false;
        c->arena_off = off + want;
        return CF_OK;
    }
    // a recorded graph holds the addresses of these buffers
    drop_graph(c);
    uploads_clear(c);
    if (b.p) {
        HIPCHK(hipStreamSynchronize(c->stream));
        HIPCHK(release(c, b));
    }
    size_t want = bytes + bytes / 4;
    if (c->alloc) {
        b.p = c->alloc(want, c->alloc_user);
        if (!b.p)
            return fail(c, CF_ENOMEM, "registered allocator returned NULL for %zu bytes", want);
        if (reinterpret_cast<uintptr_t>(b.p) % 256 != 0) {
            c->free_(b.p, c->alloc_user);
            b.p = nullptr;
            return fail(c, CF_EINVAL, "registered allocator returned memory not 256-byte aligned");
        }
        b.user = true;
    } else {
        hipError_t e = hipMalloc(&b.p, want);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            b.p = nullptr;
            return fail(c, CF_ENOMEM, "hipMalloc(%zu) failed: %s", want, hipGetErrorString(e));
        }
    }
    b.cap = want;
    return CF_OK;
}

cf_status ensure_pinned(cf_ctx *c, size_t bytes)
{
    if (c->pinned_cap >= bytes)
        return CF_OK;
    if (c->arena)
        return fail(c, CF_EINVAL,
                    "the call needs %zu bytes of host staging, more than the %zu bytes "
                    "pinned when the context was created", bytes, c->pinned_cap);
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

int pow2_floor(int v)
{
    int p = 1;
    while (p * 2 <= v)
        p *= 2;
    return p;
}

// One side of a call (the first or second catalogue argument): its
// catalogues as device views, in the order of the call.
struct SideData {
    int ncat = 0;
    int64_t ntot = 0;
    std::vector<pc_cat> cats;
};

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

// Stage the catalogues of one side on the device: host columns are copied
// into one concatenated buffer per column, device columns are used in place,
// RA/DEC become unit vectors.
// radec: x, y are RA, DEC in degrees, converted on the device to unit
// vectors, or (sky) to positions D u with the distance D in z.
// RA/DEC (and distance) of one catalogue to unit vectors (positions) on the
// host with the C library's sin and cos: v = (cos d cos a, cos d sin a, sin d)
// with a, d in radians (degrees times pi/180), times the distance for on-sky
// pairs, split over host threads.  The vectors go to vx, vy, vz on the
// device.
cf_status radec_on_host(cf_ctx *c, const cf_catalog &cat, bool sky, double *vx, double *vy,
                        double *vz)
{
    const size_t n = (size_t)cat.n;
    std::vector<double> in((sky ? 3 : 2) * n), out(3 * n);
    auto fetch = [&](const void *src, int dtype, double *dst) -> cf_status {
        const size_t bytes = dsize(dtype) * n;
        std::vector<char> tmp;
        const void *h = src;
        if (cat.mem == CF_MEM_DEVICE) {
            tmp.resize(bytes);
            HIPCHK(hipMemcpyAsync(tmp.data(), src, bytes, hipMemcpyDeviceToHost, c->stream));
            HIPCHK(hipStreamSynchronize(c->stream));
            h = tmp.data();
        }
        if (dtype == CF_F32)
            for (size_t i = 0; i < n; i++)
                dst[i] = static_cast<const float *>(h)[i];
        else
            memcpy(dst, h, bytes);
        return CF_OK;
    };
    cf_status st;
    if ((st = fetch(cat.x, cat.dtype, in.data())) ||
        (st = fetch(cat.y, cat.dtype, in.data() + n)) ||
        (sky && (st = fetch(cat.z, cat.dtype, in.data() + 2 * n))))
        return st;
    const double d2r = M_PI / 180.0;
    // bad[0]: RA/DEC out of range, bad[1]: bad distance (per thread slice)
    auto convert = [&](size_t i0, size_t i1, int *bad) {
        for (size_t i = i0; i < i1; i++) {
            const double a = in[i], d = in[n + i];
            if (!(a >= 0.0 && a <= 360.0 && d >= -90.0 && d <= 90.0)) {
                bad[0] = 1;
                return;
            }
            const double ar = a * d2r, dr = d * d2r;
            const double cd = cos(dr);
            double ux = cd * cos(ar), uy = cd * sin(ar), uz = sin(dr);
            if (sky) {
                const double D = in[2 * n + i];
                if (!(D >= 0.0) || !std::isfinite(D)) {
                    bad[1] = 1;
                    return;
                }
                ux = D * ux;
                uy = D * uy;
                uz = D * uz;
            }
            out[i] = ux;
            out[n + i] = uy;
            out[2 * n + i] = uz;
        }
    };
    // the conversion is independent per point: split it over host threads
    // (at most 16, at least 64 Ki points each)
    const unsigned hw = std::max(1u, std::thread::hardware_concurrency());
    const size_t nthr = std::max<size_t>(1, std::min<size_t>({(size_t)hw, 16, n / 65536}));
    std::vector<int> bad(2 * nthr, 0);
    std::vector<std::thread> pool;
    for (size_t t = 1; t < nthr; t++)
        pool.emplace_back(convert, n * t / nthr, n * (t + 1) / nthr, &bad[2 * t]);
    convert(0, n / nthr, &bad[0]);
    for (auto &th : pool)
        th.join();
    for (size_t t = 0; t < nthr; t++) {
        if (bad[2 * t])
            return fail(c, CF_ERANGE, "RA must lie in [0, 360] and DEC in [-90, 90]");
        if (bad[2 * t + 1])
            return fail(c, CF_EINVAL, "distances must be finite and non-negative");
    }
    HIPCHK(hipMemcpyAsync(vx, out.data(), sizeof(double) * n, hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipMemcpyAsync(vy, out.data() + n, sizeof(double) * n, hipMemcpyHostToDevice,
                          c->stream));
    HIPCHK(hipMemcpyAsync(vz, out.data() + 2 * n, sizeof(double) * n, hipMemcpyHostToDevice,
                          c->stream));
    // `out` is released on return
    HIPCHK(hipStreamSynchronize(c->stream));
    return CF_OK;
}

cf_status stage_side(cf_ctx *c, const cf_catalog *d, int ncat, bool radec, bool sky, int side,
                     SideData &s, unsigned *flags, bool host_radec)
{
    static const BufId inb[2][4] = {{B_IN1X, B_IN1Y, B_IN1Z, B_IN1W},
                                    {B_IN2X, B_IN2Y, B_IN2Z, B_IN2W}};
    s.ncat = ncat;
    s.cats.assign(ncat, pc_cat{});
    s.ntot = 0;
    for (int i = 0; i < ncat; i++) {
        s.cats[i].n = d[i].n;
        s.cats[i].off = s.ntot;
        s.ntot += d[i].n;
    }
    // host bytes of each column
    size_t need[4] = {0, 0, 0, 0};
    for (int i = 0; i < ncat; i++) {
        if (d[i].mem != CF_MEM_HOST || d[i].n == 0)
            continue;
        const size_t b = align256(dsize(d[i].dtype) * (size_t)d[i].n);
        need[0] += b;
        need[1] += b;
        if (!radec || sky)
            need[2] += b;
        if (d[i].w)
            need[3] += align256(dsize(d[i].wdtype) * (size_t)d[i].n);
    }
    cf_status st;
    for (int k = 0; k < 4; k++)
        if (need[k] && (st = ensure(c, inb[side][k], need[k])))
            return st;
    // unit vectors of RA/DEC input go to a separate buffer (3 ntot doubles)
    const BufId uvb = side == 0 ? B_UV1 : B_UV2;
    if (radec && (st = ensure(c, uvb, sizeof(double) * 3 * (size_t)std::max<int64_t>(s.ntot, 1))))
        return st;
    size_t hoff[4] = {0, 0, 0, 0};
    auto place = [&](int k, const void *src, int dtype, const cf_catalog &cat) -> const void * {
        if (cat.mem == CF_MEM_DEVICE || cat.n == 0)
            return src;
        char *dst = static_cast<char *>(c->buf[inb[side][k]].p) + hoff[k];
        const size_t bytes = dsize(dtype) * (size_t)cat.n;
        hoff[k] += align256(bytes);
        if (hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, c->stream) != hipSuccess)
            return nullptr;
        return dst;
    };
    for (int i = 0; i < ncat; i++) {
        const cf_catalog &cat = d[i];
        pc_cat &o = s.cats[i];
        // RA/DEC converted on the host are read where they are
        const bool hconv = radec && host_radec;
        const void *x = hconv ? cat.x : place(0, cat.x, cat.dtype, cat);
        const void *y = hconv ? cat.y : place(1, cat.y, cat.dtype, cat);
        const void *z = ((radec && !sky) || hconv) ? nullptr : place(2, cat.z, cat.dtype, cat);
        const void *w = cat.w ? place(3, cat.w, cat.wdtype, cat) : nullptr;
        if (cat.n > 0 &&
            (!x || !y || ((!radec || sky) && !hconv && !z) || (cat.w && !w)))
            return fail(c, CF_EDEVICE, "host-to-device copy of catalogue %d failed", i);
        if (radec) {
            double *v = dptr<double>(c, uvb);
            double *vx = v + o.off, *vy = v + s.ntot + o.off, *vz = v + 2 * s.ntot + o.off;
            if (cat.n > 0 && hconv) {
                if ((st = radec_on_host(c, cat, sky, vx, vy, vz)))
                    return st;
            } else if (cat.n > 0) {
                HIPCHK(pc::launch_radec(c->stream, cat.n, x, y, sky ? z : nullptr,
                                        cat.dtype == CF_F32, M_PI / 180.0, vx, vy, vz, flags));
            }
            o.x = vx;
            o.y = vy;
            o.z = vz;
            o.f32 = 0;
        } else {
            o.x = x;
            o.y = y;
            o.z = z;
            o.f32 = cat.dtype == CF_F32;
        }
        o.w = w;
        o.wf32 = cat.w ? (cat.wdtype == CF_F32) : 0;
    }
    return CF_OK;
}

// Grid the catalogues of one side: cell index -> scan -> scatter.  Cells of
// catalogue k are k * ncell .. (k + 1) * ncell - 1, so the sorted arrays hold
// the catalogues one after the other, each in cell order.
// Q (or B_COUNT: none): (x, y, z, |b|^2) in float32 of every sorted point,
// side by side, for sweeps that expand x and y (with Z; X and Y not written)
cf_status grid_side(cf_ctx *c, const SideData &s, const pc_cat *cats_dev, bool weighted,
                    const pc_grid &g, BufId start, BufId X, BufId Y, BufId Z, BufId XD, BufId YD,
                    BufId ZD, BufId WD, BufId CS, BufId Q, unsigned *flags)
{
    const int64_t n = s.ntot;
    const int64_t ncells = (int64_t)s.ncat * g.ncell;
    cf_status st;
    if ((st = ensure(c, B_CNT, sizeof(int32_t) * (size_t)ncells)) ||
        (st = ensure(c, start, sizeof(int32_t) * (size_t)(ncells + 1))) ||
        (st = ensure(c, B_CELLOF, sizeof(int32_t) * (size_t)n)) ||
        (st = ensure(c, B_RANKOF, sizeof(int32_t) * (size_t)n)) ||
        (st = ensure(c, B_PERM, sizeof(int32_t) * (size_t)n)) ||
        (st = ensure(c, B_REC, 32 * (size_t)n)) ||
        (st = ensure(c, B_SCANTMP, sizeof(int32_t) * pc::scan_tmp_elems(ncells))) ||
        (st = ensure(c, X, sizeof(float) * (size_t)n)) ||
        (st = ensure(c, Y, sizeof(float) * (size_t)n)) ||
        (st = ensure(c, Z, sizeof(float) * (size_t)n)) ||
        (st = ensure(c, XD, sizeof(double) * (size_t)n)) ||
        (st = ensure(c, YD, sizeof(double) * (size_t)n)) ||
        (st = ensure(c, ZD, sizeof(double) * (size_t)n)) ||
        (st = ensure(c, CS, sizeof(int32_t) * (size_t)n)))
        return st;
    if (weighted && (st = ensure(c, WD, sizeof(double) * (size_t)n)))
        return st;
    if (Q != B_COUNT && (st = ensure(c, Q, 4 * sizeof(float) * (size_t)n)))
        return st;
    float4 *qd = Q != B_COUNT ? static_cast<float4 *>(c->buf[Q].p) : nullptr;
    // Two-level counting sort when the columns of a catalogue and the z
    // slices of a column fit an LDS histogram: chunks of at least 2048
    // points (and 8 per column, bounding the count matrix by n / 8 + ...)
    const int32_t ncolc = g.n[0] * g.n[1];
    const int32_t nz = g.n[2];
    const int64_t chunk = ((std::max<int64_t>(2048, 8 * (int64_t)ncolc) + 255) / 256) * 256;
    int64_t nchunks = 0;
    for (const pc_cat &k : s.cats)
        nchunks += (k.n + chunk - 1) / chunk;
    const int64_t m = nchunks * ncolc;
    if (ncolc <= PC_SORT2_MAX_BINS && nz <= PC_SORT2_MAX_BINS && m < 0x7ffffff0 &&
        nchunks < 0x7fffffff && (int64_t)s.ncat * ncolc < 0x7fffffff && chunk < 0x7fffffff) {
        if ((st = ensure(c, B_CNT, sizeof(int32_t) * (size_t)std::max<int64_t>(m, 1))) ||
            (st = ensure(c, B_WOFF, sizeof(int32_t) * (size_t)(m + 1))) ||
            (st = ensure(c, B_LAY, sizeof(int32_t) * 3 * (size_t)(s.ncat + 1))) ||
            (st = ensure(c, B_COLS, 2 * sizeof(int32_t) * (size_t)std::max<int64_t>(n, 1))) ||
            (st = ensure(c, B_SCANTMP, sizeof(int32_t) * pc::scan_tmp_elems(m))))
            return st;
        // (the record buffer holds the column-ordered records here)
        HIPCHK(pc::launch_sort2(c->stream, s.ncat, cats_dev, n, g, (int32_t)chunk, ncolc,
                                (int32_t)nchunks, m, dptr<int32_t>(c, B_LAY),
                                dptr<int32_t>(c, B_CNT), dptr<int32_t>(c, B_WOFF),
                                dptr<int32_t>(c, B_SCANTMP), dptr<int32_t>(c, B_CELLOF),
                                dptr<int32_t>(c, B_RANKOF), c->buf[B_REC].p, c->buf[B_COLS].p,
                                dptr<int32_t>(c, B_PERM), dptr<int32_t>(c, start),
                                dptr<int32_t>(c, CS), dptr<float>(c, X), dptr<float>(c, Y),
                                dptr<float>(c, Z), dptr<double>(c, XD), dptr<double>(c, YD),
                                dptr<double>(c, ZD), weighted ? dptr<double>(c, WD) : nullptr,
                                qd, flags));
        return CF_OK;
    }
    HIPCHK(pc::launch_zero(c->stream, c->buf[B_CNT].p, sizeof(int32_t) * (size_t)ncells));
    HIPCHK(pc::launch_cell_index(c->stream, s.ncat, cats_dev, n, g, dptr<unsigned>(c, B_CNT),
                                 dptr<int32_t>(c, B_CELLOF), dptr<int32_t>(c, B_RANKOF),
                                 c->buf[B_REC].p, flags));
    HIPCHK(pc::scan_exclusive(c->stream, dptr<int32_t>(c, B_CNT), ncells, dptr<int32_t>(c, start),
                              dptr<int32_t>(c, B_SCANTMP)));
    HIPCHK(pc::launch_scatter(c->stream, n, g, dptr<int32_t>(c, B_CELLOF),
                              dptr<int32_t>(c, B_RANKOF), c->buf[B_REC].p,
                              dptr<int32_t>(c, start), dptr<int32_t>(c, B_PERM),
                              dptr<float>(c, X), dptr<float>(c, Y), dptr<float>(c, Z),
                              dptr<double>(c, XD), dptr<double>(c, YD), dptr<double>(c, ZD),
                              weighted ? dptr<double>(c, WD) : nullptr, qd,
                              dptr<int32_t>(c, CS)));
    return CF_OK;
}

// The counting call behind every entry point.  d1 holds ncat catalogues
// (ncat > 1 only for batched autocorrelations); d2 is NULL for an
// autocorrelation.  counts / wsum hold ncat * nbins * npi values.
// How run() executes: eagerly (with host synchronisations), or as the
// synchronisation-free sequence recorded into a graph, with a fixed
// work-item capacity and its own pinned staging.
void key_add(std::vector<char> &k, const void *p, size_t n)
{
    k.insert(k.end(), static_cast<const char *>(p), static_cast<const char *>(p) + n);
}

// Work-item capacity for a call that does not read the count first: the
// last count plus a quarter plus 1024, or 0 when that would not fit int32.
int32_t item_margin(int32_t last)
{
    const int64_t cap = (int64_t)last + last / 4 + 1024;
    return cap <= (int64_t)0x7fffffff ? (int32_t)cap : 0;
}

struct RunCtl {
    bool capture = false;
    bool no_async = false;  // eager call: read the work-item count before the sweep
    int32_t item_cap = 0;
    char *pin = nullptr;
    size_t pin_cap = 0;
    size_t pin_need = 0;   // out: pinned bytes the call needs
    size_t p_misc = 0, p_out = 0;   // out: regions of the pinned staging
};

cf_status run(cf_ctx *c, RunCtl &ctl, int metric, bool theta, const cf_catalog *d1,
              int32_t ncat, const cf_catalog *d2, const double *edges, int32_t nb, double pimax,
              int32_t npi, double boxsize, cf_precision prec, uint64_t *counts, double *wsum,
              const cf_options *opt_in)
{
    if (!c)
        return CF_EINVAL;
    c->err.clear();
    if (!ctl.capture)
        memset(&c->stats, 0, sizeof(c->stats));
    cf_options opt;
    cf_default_options(&opt);
    if (opt_in) {
        if (opt_in->struct_size != (int32_t)sizeof(cf_options))
            return fail(c, CF_EINVAL, "cf_options.struct_size mismatch");
        opt = *opt_in;
    }
    // on-sky (rp, pi): RA, DEC and distance, or Cartesian positions with
    // theta_unit_vectors; theta: RA, DEC, or unit vectors
    const bool sky = metric == PC_METRIC_MOCKS;
    const bool unit_vec = (theta || sky) && opt.theta_unit_vectors;
    cf_status st;
    if (ncat < 1 || ncat > PC_MAX_CATS)
        return fail(c, CF_EINVAL, "number of catalogues must be in [1, %d]", PC_MAX_CATS);
    if (!d1)
        return fail(c, CF_EINVAL, "d1 is NULL");
    for (int i = 0; i < ncat; i++) {
        char name[32];
        snprintf(name, sizeof(name), ncat > 1 ? "catalogue %d" : "d1", i);
        if ((st = check_catalog(c, &d1[i], name, theta, unit_vec)))
            return st;
        if ((d1[i].w == nullptr) != (d1[0].w == nullptr))
            return fail(c, CF_EINVAL, "weights must be given for every catalogue or none");
    }
    const bool autocorr = (d2 == nullptr);
    if (!autocorr && ncat != 1)
        return fail(c, CF_EINVAL, "cross-correlations take one catalogue per side");
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
    if (metric != PC_METRIC_R) {
        if (npi < 1 || npi > PC_MAX_NPI)
            return fail(c, CF_EINVAL, "npi must be in [1, %d]", PC_MAX_NPI);
        if (!(pimax > 0.0) || !isfinite(pimax))
            return fail(c, CF_EINVAL, "pimax must be positive and finite");
    } else {
        npi = 1;
    }
    const bool user_w = d1->w != nullptr;
    if (opt.weight_type != CF_WEIGHT_PRODUCT && opt.weight_type != CF_WEIGHT_SUM)
        return fail(c, CF_EINVAL, "unknown weight_type %d", opt.weight_type);
    if (opt.weight_type != CF_WEIGHT_PRODUCT && !user_w)
        return fail(c, CF_EINVAL, "summed pair weights need weights");
    const bool want_ravg = opt.ravg != nullptr;
    if (opt.separation_form < 0 || opt.separation_form > 2)
        return fail(c, CF_EINVAL, "separation_form must be 0, 1 or 2");
    // the sweep carries weights when the caller gives them or asks for the
    // mean separation (unit weights then, whose sums are the counts)
    const bool weighted = user_w || want_ravg;
    // exact fixed-point weight sums (unit weights, for the mean separation
    // alone, sum exactly in binary64 anyway)
    const bool wfixed = user_w && opt.deterministic_weights != 0;
    const int64_t nbt = (int64_t)nb * npi;
    if (nbt > PC_MAX_BINS_TOTAL / (want_ravg ? 3 : (weighted ? 2 : 1)))
        return fail(c, CF_EINVAL, "too many output bins (%lld)", (long long)nbt);
    if (isnan(boxsize) || (!isfinite(boxsize) && boxsize > 0.0))
        return fail(c, CF_EINVAL, "boxsize must be finite (or <= 0 for no wrap)");
    if (theta && boxsize > 0.0)
        return fail(c, CF_EINVAL, "angular counts are never periodic");
    if (sky && boxsize > 0.0)
        return fail(c, CF_EINVAL, "on-sky counts are never periodic");
    if (opt.angular_grid < -1 || opt.angular_grid > 64)
        return fail(c, CF_EINVAL, "angular_grid must be in [-1, 64]");
    if (opt.angular_grid != 0 && !theta)
        return fail(c, CF_EINVAL, "angular_grid applies to angular counts only");
    // angular counts default to the angular grid with 16 right-ascension
    // cells per reach; -1 selects 3-D cells on the unit vectors
    if (theta && opt.angular_grid == 0)
        opt.angular_grid = 16;
    if (opt.angular_grid < 0)
        opt.angular_grid = 0;
    const bool sky_grid = theta && opt.angular_grid > 0;
    if (opt.flush_pairs < 0)
        return fail(c, CF_EINVAL, "flush_pairs must be >= 0");
    if (opt.xy_refine < 0 || opt.xy_refine > PC_MAX_XYK)
        return fail(c, CF_EINVAL, "xy_refine must be in [0, %d]", PC_MAX_XYK);
    if (opt.xy_refine == 0)
        opt.xy_refine = 1;
    if (opt.slices_per_reach <= 0)
        opt.slices_per_reach = 32;

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
    // on-sky pairs: the line of sight varies, so every axis must reach the
    // largest 3-D separation sqrt(rp_max^2 + pimax^2) (kept a little wider
    // than its rounding)
    const double reach_sky = std::sqrt(lin[nb] * lin[nb] + pimax * pimax) * (1.0 + 0x1p-30);
    const double reach_xy = sky ? reach_sky : lin[nb];
    const double reach_z = sky ? reach_sky : (metric == PC_METRIC_RPPI) ? pimax : lin[nb];
    int64_t n1 = 0;
    for (int i = 0; i < ncat; i++)
        n1 += d1[i].n;
    const int64_t n2 = autocorr ? n1 : d2->n;
    if (n1 + (autocorr ? 0 : n2) > (int64_t)0x7fffff00)
        return fail(c, CF_EINVAL, "too many points for one call (limit 2^31 - 256)");
    const size_t nout = (size_t)ncat * (size_t)nbt;

    HIPCHK(hipSetDevice(c->device));
    const bool timing = opt.collect_timing != 0 && !ctl.capture;
    record(c, timing, 0);

    cf_status st2;
    if ((st2 = ensure(c, B_MISC, M_SIZE)))
        return st2;
    HIPCHK(pc::launch_zero(c->stream, c->buf[B_MISC].p, M_SIZE));

    const bool empty = (n1 == 0) || (!autocorr && n2 == 0);
    if (empty) {
        if (opt.output_on_device) {
            HIPCHK(hipMemsetAsync(counts, 0, sizeof(uint64_t) * nout, c->stream));
            if (wsum)
                HIPCHK(hipMemsetAsync(wsum, 0, sizeof(double) * nout, c->stream));
            if (want_ravg)
                HIPCHK(hipMemsetAsync(opt.ravg, 0, sizeof(double) * nout, c->stream));
            HIPCHK(hipStreamSynchronize(c->stream));
        } else {
            memset(counts, 0, sizeof(uint64_t) * nout);
            if (wsum)
                memset(wsum, 0, sizeof(double) * nout);
            if (want_ravg)
                memset(opt.ravg, 0, sizeof(double) * nout);
        }
        return CF_OK;
    }

    // pinned staging: [misc | side-1 catalogues | side-2 catalogue | bins |
    // outputs]; every region has its own place, so no host write waits for a
    // pending copy of another
    const size_t p_misc = 0;
    const size_t p_cats1 = align256(M_SIZE);
    const size_t p_cats2 = p_cats1 + align256(sizeof(pc_cat) * (size_t)ncat);
    const size_t p_bins = p_cats2 + align256(sizeof(pc_cat));
    const size_t bins_cap = 256 * 1024 + 64 * (size_t)(nb + npi + 2);
    const size_t p_sky = p_bins + bins_cap;
    const size_t p_out = p_sky + (sky_grid ? align256(sizeof(pc_band) * PC_MAX_BANDS) : 0);
    ctl.pin_need = p_out + (sizeof(uint64_t) + 2 * sizeof(double)) * nout;
    ctl.p_misc = p_misc;
    ctl.p_out = p_out;
    char *pin;
    if (ctl.capture) {
        if (ctl.pin_cap < ctl.pin_need)
            return fail(c, CF_EINVAL, "graph staging too small");
        pin = ctl.pin;
    } else {
        if ((st2 = ensure_pinned(c, ctl.pin_need)))
            return st2;
        pin = static_cast<char *>(c->pinned);
    }

    // ---- stage inputs ----------------------------------------------------
    unsigned *flags = (unsigned *)(misc(c) + M_FLAGS);
    const bool radec = (theta || sky) && !unit_vec;
    SideData s1, s2;
    if ((st2 = stage_side(c, d1, ncat, radec, sky, 0, s1, flags, opt.radec_on_device == 0)))
        return st2;
    if (!autocorr &&
        (st2 = stage_side(c, d2, 1, radec, sky, 1, s2, flags, opt.radec_on_device == 0)))
        return st2;
    if ((st2 = ensure(c, B_CATS1, sizeof(pc_cat) * (size_t)ncat)) ||
        (st2 = ensure(c, B_CATS2, sizeof(pc_cat))))
        return st2;
    // (eager calls of the context's own buffers keep their uploads; a graph
    // capture records every copy, and a no-allocation call's buffers are
    // shared by every context on the device)
    const bool keep_uploads = !ctl.capture && !c->arena;
    const size_t cats1_bytes = sizeof(pc_cat) * (size_t)ncat;
    if (!(keep_uploads &&
          upload_fresh(c->up_cats1, c->buf[B_CATS1].p, s1.cats.data(), cats1_bytes))) {
        memcpy(pin + p_cats1, s1.cats.data(), cats1_bytes);
        HIPCHK(hipMemcpyAsync(c->buf[B_CATS1].p, pin + p_cats1, cats1_bytes,
                              hipMemcpyHostToDevice, c->stream));
        if (keep_uploads)
            upload_keep(c->up_cats1, c->buf[B_CATS1].p, s1.cats.data(), cats1_bytes);
        else
            c->up_cats1 = cf_ctx::Upload{};
    }
    if (!autocorr) {
        memcpy(pin + p_cats2, s2.cats.data(), sizeof(pc_cat));
        HIPCHK(hipMemcpyAsync(c->buf[B_CATS2].p, pin + p_cats2, sizeof(pc_cat),
                              hipMemcpyHostToDevice, c->stream));
    }
    const pc_cat *cats1_dev = dptr<pc_cat>(c, B_CATS1);
    const pc_cat *cats2_dev = autocorr ? cats1_dev : dptr<pc_cat>(c, B_CATS2);

    // ---- bounding box ------------------------------------------------------
    double lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
    const bool periodic = boxsize > 0.0;
    if (!periodic && ctl.capture)
        return fail(c, CF_EINVAL, "graph replay needs a periodic box");
    if (!periodic) {
        std::vector<const pc_cat *> all;
        for (auto &k : s1.cats)
            if (k.n > 0)
                all.push_back(&k);
        if (!autocorr && s2.cats[0].n > 0)
            all.push_back(&s2.cats[0]);
        const int nparts = all.size() > 4 ? 32 : 256;
        if ((st2 = ensure(c, B_PART, sizeof(double) * 6 * nparts * all.size())))
            return st2;
        double *part = dptr<double>(c, B_PART);
        for (size_t k = 0; k < all.size(); k++)
            HIPCHK(pc::launch_minmax(c->stream, all[k]->n, all[k]->x, all[k]->y, all[k]->z,
                                     all[k]->f32, part + 6 * nparts * k, nparts, flags));
        double *out6 = (double *)(misc(c) + M_OUT6);
        HIPCHK(pc::launch_minmax_final(c->stream, part, nparts * (int)all.size(), out6));
        HIPCHK(hipMemcpyAsync(pin + p_misc, misc(c), M_SIZE, hipMemcpyDeviceToHost, c->stream));
        HIPCHK(hipStreamSynchronize(c->stream));
        const char *hm = pin + p_misc;
        unsigned hflags;
        memcpy(&hflags, hm + M_FLAGS, 4);
        if (hflags & PC_FLAG_RADEC)
            return fail(c, CF_ERANGE, "RA must lie in [0, 360] and DEC in [-90, 90]");
        if (hflags & PC_FLAG_NONFINITE)
            return fail(c, CF_EINVAL, "non-finite coordinate");
        const double *o6 = (const double *)(hm + M_OUT6);
        for (int a = 0; a < 3; a++) {
            lo[a] = o6[a];
            hi[a] = o6[3 + a];
        }
    }

    // ---- plan ------------------------------------------------------------
    pc_grid g;
    // r, angular chords and on-sky pairs are bounded by a 3-D ball
    int rc = pc::plan_grid(lo, hi, boxsize, reach_xy, reach_z, opt.slices_per_reach, &g,
                           opt.xy_refine, metric != PC_METRIC_RPPI);
    if (rc == CF_EUNSUPPORTED)
        return fail(c, CF_EUNSUPPORTED,
                    "periodic box needs every reach (r, rp, pi) at most boxsize/3");
    if (rc)
        return fail(c, (cf_status)rc, "grid planning failed");
    if (sky_grid) {
        // declination bands and right-ascension cells on the unit vectors
        std::vector<pc_band> bands;
        rc = pc::plan_sky_grid(lin[nb], lo[2], hi[2], opt.slices_per_reach, opt.angular_grid,
                               &g, &bands);
        if (rc)
            return fail(c, (cf_status)rc, "angular grid planning failed");
        const size_t bytes = sizeof(pc_band) * bands.size();
        if ((st2 = ensure(c, B_BANDS, bytes)))
            return st2;
        memcpy(pin + p_sky, bands.data(), bytes);
        HIPCHK(hipMemcpyAsync(c->buf[B_BANDS].p, pin + p_sky, bytes, hipMemcpyHostToDevice,
                              c->stream));
        g.bands = dptr<pc_band>(c, B_BANDS);
    }
    if ((int64_t)ncat * g.ncell + 1 > (int64_t)0x7fffffff)
        return fail(c, CF_EINVAL, "too many cells for this batch; use fewer z slices");
    double scale = periodic ? boxsize : 0.0;
    for (int a = 0; a < 3; a++)
        scale = std::max(scale, g.extent[a]);
    // on-sky pairs are evaluated in binary64 in either mode (same counts):
    // the definition has a division and a square root per pair, and the
    // vector binary64 rate equals the non-packed float32 rate here
    bool fp32 = prec == CF_PREC_FP32_RECHECK && !sky;
    // float32 rp/pi path: z as fixed point with one pi bin = 2^k quanta, k
    // as large as keeps every biased value (and the periodic offset) below
    // 2^31.  When a bin would get fewer than 2^4 quanta the call sweeps in
    // binary64 instead, which gives the same counts.
    if (fp32 && metric == PC_METRIC_RPPI) {
        const double dpi = pimax / (double)npi;
        const double span = periodic ? boxsize : g.extent[2];
        int k = 24;
        while (k >= 4 && std::ldexp(span / dpi, k) > 0x1p29)
            k--;
        if (k >= 4) {
            g.zq_shift = k;
            g.zq_inv = std::ldexp(1.0, k) / dpi;
        } else {
            fp32 = false;
        }
    }
    // float32 sweeps of 3-D grids keep x and y in column-local frames, so
    // their rounding scales with the column width instead of the box
    g.xy_local = (fp32 && !sky_grid) ? 1 : 0;
    // their rounding bounds: the lane's x (y) lies within k + 1/2 column
    // widths of the j column's centre, the j point within half a width; z
    // (box frame) within scale + reach_z and scale
    const double axis_eps[3] = {
        pc::frame_eps((g.xyk + 0.5) * g.width[0], 0.5 * g.width[0], scale),
        pc::frame_eps((g.xyk + 0.5) * g.width[1], 0.5 * g.width[1], scale),
        pc::frame_eps(scale + reach_z, scale, scale)};
    // Float32 DD(r) (and chords) and DD(rp, pi) of 3-D grids without the
    // mean separation: x and y expanded as |a|^2 + |b|^2 - 2 a.b, one
    // instruction fewer per pair.  By default only while its absolute
    // rounding term widens the band of the smallest nonzero edge by at most
    // an eighth of that edge (the sweep narrows each pair's band by its own
    // magnitudes before a binary64 recheck, which keeps the rechecks of the
    // crowded small rp edges in check).  (The float32 mean separation takes
    // the square root of s and keeps the differences.)
    double xy_mag = 0.0;
    if (fp32 && g.xy_local && (metric == PC_METRIC_R || metric == PC_METRIC_RPPI) && !sky &&
        !want_ravg && opt.separation_form != 1) {
        const double am[2] = {(g.xyk + 0.5) * g.width[0], (g.xyk + 0.5) * g.width[1]};
        const double bm[2] = {0.5 * g.width[0], 0.5 * g.width[1]};
        const double mag = pc::xy_expand_mag(am, bm, metric == PC_METRIC_RPPI ? 2 : 3);
        double emin = INFINITY;
        for (int k = 0; k <= nb; k++)
            if (lin[k] > 0.0)
                emin = std::min(emin, lin[k] * lin[k]);
        if (opt.separation_form == 2 || 1.25 * 0x1p-24 * mag <= 0.125 * emin)
            xy_mag = mag;
    }
    // batches: private per-wave histograms, flushed per catalogue
    const bool priv = ncat > 1;
    double fscale = 1.0;
    if (fp32 && (rc = pc::fp32_scale(metric, lin.data(), nb, scale, priv,
                                     g.xy_local ? axis_eps : nullptr, xy_mag, &fscale)))
        return fail(c, (cf_status)rc, "float32 scaling failed");
    g.fscale = fscale;
    record(c, timing, 1);

    // ---- work-list and sweep buffers, cleared by one kernel ahead of the
    // gridding (the host issues it while nothing else waits on it) ----------
    const int32_t ncol = g.n[0] * g.n[1] * ncat;   // columns of every catalogue
    const int64_t maxblocks = n1 / PC_BLOCK_I + ncol + 1;
    const int chunk = opt.chunk > 0 ? std::min(opt.chunk, 1 << 20) : 2048;
    if ((st2 = ensure(c, B_BCNT, sizeof(int32_t) * (size_t)ncol)) ||
        (st2 = ensure(c, B_BOFF, sizeof(int32_t) * (size_t)(ncol + 1))) ||
        (st2 = ensure(c, B_BLOCKS, sizeof(pc_block) * (size_t)maxblocks)) ||
        (st2 = ensure(c, B_ICNT, sizeof(int32_t) * (size_t)maxblocks)) ||
        (st2 = ensure(c, B_IOFF, sizeof(int32_t) * (size_t)(maxblocks + 1))) ||
        (st2 = ensure(c, B_SCANTMP, sizeof(int32_t) * pc::scan_tmp_elems(std::max<int64_t>(
                                        std::max<int64_t>(maxblocks, ncol),
                                        (int64_t)ncat * g.ncell)))) ||
        (st2 = ensure(c, B_HIST, sizeof(unsigned long long) * nout)) ||
        (st2 = ensure(c, B_WHIST, (wfixed ? 24 : 8) * nout)) ||
        (st2 = ensure(c, B_OUTC, sizeof(unsigned long long) * nout)) ||
        (st2 = ensure(c, B_OUTW, sizeof(double) * nout)) ||
        (want_ravg && (st2 = ensure(c, B_RHIST, sizeof(double) * nout))) ||
        (want_ravg && (st2 = ensure(c, B_OUTR, sizeof(double) * nout))) ||
        (st2 = ensure(c, B_WSQ, (wfixed ? 24 : 8) * (size_t)ncat)) ||
        (st2 = ensure(c, B_CTRS, sizeof(int32_t) * PC_STREAMS * PC_STREAM_STRIDE)))
        return st2;
    {
        void *zp[PC_ZERO_MAX];
        size_t zb[PC_ZERO_MAX];
        int nz = 0;
        zp[nz] = c->buf[B_ICNT].p;
        zb[nz++] = sizeof(int32_t) * (size_t)maxblocks;
        zp[nz] = c->buf[B_CTRS].p;
        zb[nz++] = sizeof(int32_t) * PC_STREAMS * PC_STREAM_STRIDE;
        zp[nz] = c->buf[B_HIST].p;
        zb[nz++] = sizeof(unsigned long long) * nout;
        if (weighted) {
            zp[nz] = c->buf[B_WHIST].p;
            zb[nz++] = (wfixed ? 24 : 8) * nout;
        }
        if (want_ravg) {
            zp[nz] = c->buf[B_RHIST].p;
            zb[nz++] = sizeof(double) * nout;
        }
        HIPCHK(pc::launch_zero_multi(c->stream, nz, zp, zb));
    }

    // ---- grid ------------------------------------------------------------
    // (|b|^2 for the expanded form: on the j side only)
    if ((st2 = grid_side(c, s1, cats1_dev, weighted, g, B_START1, B_X1, B_Y1, B_Z1, B_XD1, B_YD1,
                         B_ZD1, B_WD1, B_CS1, (xy_mag > 0.0 && autocorr) ? B_Q1 : B_COUNT,
                         flags)))
        return st2;
    if (!autocorr &&
        (st2 = grid_side(c, s2, cats2_dev, weighted, g, B_START2, B_X2, B_Y2, B_Z2, B_XD2,
                         B_YD2, B_ZD2, B_WD2, B_CS2, xy_mag > 0.0 ? B_Q2 : B_COUNT, flags)))
        return st2;
    // fixed-point weight sums: the grid 2^Q of this call's pair weights
    pc::pc_wfixed *wfx = wfixed ? (pc::pc_wfixed *)(misc(c) + M_WFIX) : nullptr;
    if (wfixed) {
        HIPCHK(pc::launch_wfixed_scan(c->stream, s1.ntot, dptr<double>(c, B_WD1), 0, wfx));
        if (!autocorr)
            HIPCHK(pc::launch_wfixed_scan(c->stream, s2.ntot, dptr<double>(c, B_WD2), 1, wfx));
        HIPCHK(pc::launch_wfixed_plan(c->stream, opt.weight_type, autocorr ? 0 : 1, wfx, flags));
    }
    // the bin description is built on the host while the gridding kernels run
    pc::HostBins hb;
    // on-sky pairs bin (rp, pi) like the Cartesian statistic
    rc = pc::build_bins(sky ? PC_METRIC_RPPI : metric, fp32, lin.data(), nb, pimax, npi, scale,
                        g.xy_local ? axis_eps : nullptr, fscale, priv, xy_mag, &hb);
    if (rc)
        return fail(c, (cf_status)rc, "bin description failed");
    if (g.zq_shift > 0) {
        hb.hdr.zq_shift = g.zq_shift;
        hb.hdr.zq_L = periodic ? (uint32_t)llrint(boxsize * g.zq_inv) : 0u;
        memcpy(hb.buf.data(), &hb.hdr, sizeof(hb.hdr));
    }
    if (hb.buf.size() > bins_cap)
        return fail(c, CF_EINVAL, "bin description too large");
    if ((st2 = ensure(c, B_BINS, hb.lay.total)))
        return st2;
    if (!(keep_uploads &&
          upload_fresh(c->up_bins, c->buf[B_BINS].p, hb.buf.data(), hb.buf.size()))) {
        memcpy(pin + p_bins, hb.buf.data(), hb.buf.size());
        HIPCHK(hipMemcpyAsync(c->buf[B_BINS].p, pin + p_bins, hb.buf.size(),
                              hipMemcpyHostToDevice, c->stream));
        char *bd = static_cast<char *>(c->buf[B_BINS].p);
        HIPCHK(pc::launch_build_table(c->stream, hb.hdr, nb + 1,
                                      (const float *)(bd + hb.lay.lo),
                                      (const float *)(bd + hb.lay.hi),
                                      (const float *)(bd + hb.lay.lo_min), bd + hb.lay.tbl));
        if (keep_uploads)
            upload_keep(c->up_bins, c->buf[B_BINS].p, hb.buf.data(), hb.buf.size());
        else
            c->up_bins = cf_ctx::Upload{};
    }
    record(c, timing, 2);

    // ---- work list ---------------------------------------------------------
    const int32_t *start1 = dptr<int32_t>(c, B_START1);
    const int32_t *start2 = autocorr ? start1 : dptr<int32_t>(c, B_START2);
    HIPCHK(pc::launch_block_count(c->stream, ncol, g.n[2], start1, dptr<int32_t>(c, B_BCNT)));
    HIPCHK(pc::scan_exclusive(c->stream, dptr<int32_t>(c, B_BCNT), ncol, dptr<int32_t>(c, B_BOFF),
                              dptr<int32_t>(c, B_SCANTMP)));
    HIPCHK(pc::launch_block_emit(c->stream, ncol, g.n[2], start1, dptr<int32_t>(c, B_BOFF),
                                 dptr<pc_block>(c, B_BLOCKS)));
    const int32_t *nblocks_dev = dptr<int32_t>(c, B_BOFF) + ncol;
    unsigned long long *cand = (unsigned long long *)(misc(c) + M_CAND);
    HIPCHK(pc::launch_item_count(c->stream, (int32_t)maxblocks, nblocks_dev,
                                 dptr<pc_block>(c, B_BLOCKS), g, start2, dptr<int32_t>(c, B_CS1),
                                 autocorr ? 1 : 0, chunk, dptr<int32_t>(c, B_ICNT), cand));
    HIPCHK(pc::scan_exclusive(c->stream, dptr<int32_t>(c, B_ICNT), maxblocks,
                              dptr<int32_t>(c, B_IOFF), dptr<int32_t>(c, B_SCANTMP)));
    // Item count to the host (sizes the item array and the sweep launch);
    // a recorded call instead takes a fixed capacity and leaves the count
    // on the device, where the emit kernel and the sweep read it.
    // A repeat of the previous eager call's shape (same statistic, sizes,
    // bins, box, options and grid) also leaves the count on the device:
    // the items array is sized from the last count with a margin, and a
    // call whose work list overflows it raises PC_FLAG_ITEMS and is redone
    // with the count read first.  This saves a host round trip per call.
    std::vector<char> shape;
    {
        const int64_t sh[] = {metric, theta ? 1 : 0, ncat, autocorr ? 1 : 0, n1, n2, nb, npi,
                              (int64_t)prec, opt.slices_per_reach, chunk, g.n[0], g.n[1],
                              g.n[2], weighted ? 1 : 0, opt.angular_grid, g.xyk};
        key_add(shape, sh, sizeof(sh));
        key_add(shape, &boxsize, sizeof(boxsize));
        key_add(shape, &pimax, sizeof(pimax));
    }
    const bool async_items = !ctl.capture && !ctl.no_async && c->last_items > 0 &&
                             item_margin(c->last_items) > 0 && shape == c->last_shape;
    int32_t hcounts[2] = {0, 0};
    int32_t n_items;
    if (ctl.capture) {
        n_items = ctl.item_cap;
    } else if (async_items) {
        n_items = item_margin(c->last_items);
    } else {
        HIPCHK(hipMemcpyAsync(pin + p_misc, dptr<int32_t>(c, B_IOFF) + maxblocks,
                              sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
        HIPCHK(hipMemcpyAsync(pin + p_misc + 8, nblocks_dev, sizeof(int32_t),
                              hipMemcpyDeviceToHost, c->stream));
        HIPCHK(hipStreamSynchronize(c->stream));
        memcpy(&hcounts[0], pin + p_misc, 4);
        memcpy(&hcounts[1], pin + p_misc + 8, 4);
        n_items = hcounts[0];
        if (n_items < 0)
            return fail(c, CF_EOVERFLOW, "work-item count overflow");
        c->last_items = n_items;
    }
    if ((st2 = ensure(c, B_ITEMS, sizeof(pc_item) * (size_t)std::max(n_items, 1))) ||
        (g.xy_local && (st2 = ensure(c, B_ICELL, sizeof(int32_t) * (size_t)std::max(n_items, 1)))))
        return st2;
    // (the float32 sweep of 3-D grids takes each item's j column from the
    // cell of its first j point, written beside the items)
    const int32_t *cs2_dev = dptr<int32_t>(c, autocorr ? B_CS1 : B_CS2);
    HIPCHK(pc::launch_item_emit(c->stream, (int32_t)maxblocks, nblocks_dev,
                                dptr<pc_block>(c, B_BLOCKS), g, start2, dptr<int32_t>(c, B_CS1),
                                autocorr ? 1 : 0, chunk, dptr<int32_t>(c, B_IOFF),
                                dptr<pc_item>(c, B_ITEMS), n_items, flags, cs2_dev,
                                g.xy_local ? dptr<int32_t>(c, B_ICELL) : nullptr));
    record(c, timing, 3);

    // ---- sweep -------------------------------------------------------------
    const char *bb = (const char *)c->buf[B_BINS].p;
    pc::SweepArgs a;
    memset(&a, 0, sizeof(a));
    a.items = dptr<pc_item>(c, B_ITEMS);
    a.n_items = n_items;
    a.n_items_dev = (ctl.capture || async_items) ? dptr<int32_t>(c, B_IOFF) + maxblocks : nullptr;
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
    a.g_whist = (weighted && !wfixed) ? dptr<double>(c, B_WHIST) : nullptr;
    a.wfixed = wfixed ? 1 : 0;
    a.wfx = wfx;
    a.g_wfix = wfixed ? dptr<unsigned long long>(c, B_WHIST) : nullptr;
    a.g_rhist = want_ravg ? dptr<double>(c, B_RHIST) : nullptr;
    a.ravg = want_ravg ? (theta ? 2 : 1) : 0;
    a.wtype = opt.weight_type;
    a.sep_scale = 1.0 / g.fscale;
    a.rq_count = (unsigned *)(misc(c) + M_RQCOUNT);
    a.flush_count = (unsigned *)(misc(c) + M_FLUSH);
    a.xy_local = g.xy_local;
    a.xy_exp = xy_mag > 0.0 ? 1 : 0;
    a.xy_K = 0.0f;
    a.xy_M = 0.0f;
    if (xy_mag > 0.0)
        pc::xy_pair_margin(xy_mag, g.fscale, &a.xy_K, &a.xy_M);
    a.P2 = xy_mag > 0.0 ? static_cast<const float4 *>(c->buf[autocorr ? B_Q1 : B_Q2].p)
                        : nullptr;
    a.gnx = g.n[0];
    a.gny = g.n[1];
    a.gnz = g.n[2];
    for (int k = 0; k < 3; k++)
        a.glo[k] = g.lo[k];
    a.gw[0] = g.width[0];
    a.gw[1] = g.width[1];
    a.fscale = g.fscale;
    a.cs2 = autocorr ? dptr<int32_t>(c, B_CS1) : dptr<int32_t>(c, B_CS2);
    a.icell = g.xy_local ? dptr<int32_t>(c, B_ICELL) : nullptr;
    a.nbt = (int32_t)nbt;
    a.slots = (int32_t)((nb + 2) * hb.hdr.row_w);
    a.priv = priv ? 1 : 0;
    // replica stride: odd, so the lanes' copies of one slot spread over banks
    a.rep_stride = a.slots | 1;
    // Histogram replicas: one per lane (unconditional updates, no candidate
    // branch) for unweighted 1-D counts with few bins, else a few shared ones
    // (at least two where they fit: one set shared by a workgroup's waves
    // measured 8% (counts) to 14% (weighted sums) slower on 1000 rp/pi bins);
    // private per-wave sets must fit eight waves into a modest LDS budget.
    const bool unc_ok = !priv && metric == PC_METRIC_R && !weighted && !hb.hdr.tbl_wide &&
                        PC_WAVE * a.rep_stride <= PC_MAX_HIST_WAVE;
    int copies;
    if (opt.hist_copies > 0)
        copies = pow2_floor(std::min(opt.hist_copies, PC_WAVE));
    else
        copies = unc_ok ? PC_WAVE
                        : pow2_floor((int)std::max<int64_t>(2, std::min<int64_t>(16, 512 / nbt)));
    if (copies == PC_WAVE && !unc_ok)
        copies = PC_WAVE / 2;
    while (copies > 1 && copies * a.rep_stride > PC_MAX_HIST_WAVE)
        copies /= 2;
    const int waves = pc::sweep_waves();
    // private replicas take up to 2^31 adds per slot; shared ones are bounded
    // by the sum of the waves' pending counts
    a.flush_at = priv ? 0x7fffffffull : 0x7fffffffull / (unsigned)waves;
    if (opt.flush_pairs > 0)
        a.flush_at = std::min<unsigned long long>(a.flush_at, (unsigned long long)opt.flush_pairs);
    const int slot_bytes = 4 + (weighted ? (wfixed ? 24 : 8) : 0) + (want_ravg ? 8 : 0);
    while (priv && copies > 1 && waves * copies * a.rep_stride * slot_bytes > 28 * 1024)
        copies /= 2;
    // fixed-point sums take three times the weight area: fewer shared copies
    // where they would crowd the LDS
    while (wfixed && !priv && copies > 1 && copies * a.rep_stride * slot_bytes > 64 * 1024)
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
    const int sets = priv ? waves : 1;
    a.hist_stride = (int32_t)(copies * a.rep_stride);
    a.o_hist = take(4 * sets * a.hist_stride);
    a.whist_stride = weighted ? (int32_t)(copies * a.rep_stride) : 0;
    a.wlimb = wfixed ? sets * a.whist_stride : 0;
    a.o_whist = take(weighted ? 8 * (wfixed ? 3 : 1) * sets * a.whist_stride : 0);
    a.o_rhist = take(want_ravg ? 8 * sets * a.whist_stride : 0);
    a.lds_bytes = off;
    // static LDS of the sweep: the lookup table
    const int tbl_bytes = priv ? PC_TBL_PRIV_BYTES
                               : (fp32 && !hb.hdr.tbl_wide)
                                     ? PC_TBL_PK_CELLS
                                     : (PC_TBL8_MAX > 2 * PC_TBL16_MAX ? PC_TBL8_MAX
                                                                       : 2 * PC_TBL16_MAX);
    if (off + tbl_bytes > 160 * 1024)
        return fail(c, CF_EINVAL, "bin configuration needs too much LDS (%d bytes)", off);

    int per_cu = 0;
    const int wmode = weighted ? (want_ravg ? 2 : 1) : 0;
    {
        const std::vector<int64_t> ok = {metric, fp32 ? 1 : 0, wmode, hb.hdr.tbl_wide != 0 ? 1 : 0,
                                         copies == PC_WAVE ? 1 : 0, priv ? 1 : 0, off,
                                         xy_mag > 0.0 ? 1 : 0};
        auto it = c->occupancy.find(ok);
        if (it != c->occupancy.end()) {
            per_cu = it->second;
        } else {
            HIPCHK(pc::sweep_occupancy(metric, fp32, wmode, hb.hdr.tbl_wide != 0,
                                       copies == PC_WAVE, priv, xy_mag > 0.0, off, &per_cu));
            c->occupancy[ok] = per_cu;
        }
    }
    per_cu = std::max(per_cu, 1);
    int nwg = (ctl.capture || async_items)
                  ? c->num_cu * per_cu
                  : (int)std::min<int64_t>((n_items + waves - 1) / waves,
                                           (int64_t)c->num_cu * per_cu);
    nwg = std::max(nwg, 1);
    c->stats.sweep_workgroups = nwg;
    c->stats.hist_copies = copies;
    double *wsq = nullptr;
    unsigned long long *wsq_fix = nullptr;
    if (weighted && autocorr && hb.hdr.e0_zero) {
        if (wfixed)
            wsq_fix = dptr<unsigned long long>(c, B_WSQ);
        else
            wsq = dptr<double>(c, B_WSQ);
    }
    unsigned long long *outc = opt.output_on_device ? (unsigned long long *)counts
                                                    : dptr<unsigned long long>(c, B_OUTC);
    double *outw = (wsum && user_w) ? (opt.output_on_device ? wsum : dptr<double>(c, B_OUTW))
                                    : nullptr;
    record(c, timing, 4);
    if (n_items > 0)
        HIPCHK(pc::launch_sweep(c->stream, metric, fp32, wmode, a, nwg));
    record(c, timing, 5);
    // ---- finalize ------------------------------------------------------------
    if (wsq) {
        HIPCHK(pc::launch_zero(c->stream, wsq, sizeof(double) * (size_t)ncat));
        HIPCHK(pc::launch_wsq(c->stream, ncat, g.ncell, start1, dptr<double>(c, B_WD1),
                              opt.weight_type, wsq));
    }
    if (wsq_fix) {
        HIPCHK(pc::launch_zero(c->stream, wsq_fix, 24 * (size_t)ncat));
        HIPCHK(pc::launch_wsq_fixed(c->stream, ncat, g.ncell, start1, dptr<double>(c, B_WD1),
                                    opt.weight_type, wfx, wsq_fix));
    }
    double *outr = want_ravg ? (opt.output_on_device ? opt.ravg : dptr<double>(c, B_OUTR))
                             : nullptr;
    // without weights the weight sums are zero
    if (wsum && !user_w && opt.output_on_device)
        HIPCHK(pc::launch_zero(c->stream, wsum, sizeof(double) * nout));
    HIPCHK(pc::launch_finalize(c->stream, ncat, (int32_t)nbt, autocorr ? 1 : 0, hb.hdr.e0_zero,
                               cats1_dev, a.g_hist, a.g_whist, a.g_rhist, wsq, a.g_wfix,
                               wsq_fix, wfx, outc, outw, outr,
                               dptr<int32_t>(c, B_IOFF) + maxblocks, nblocks_dev,
                               (int32_t *)(misc(c) + M_SIZES)));
    char *hp = pin + p_out;
    HIPCHK(hipMemcpyAsync(pin + p_misc, misc(c), M_SIZE, hipMemcpyDeviceToHost, c->stream));
    if (!opt.output_on_device) {
        HIPCHK(hipMemcpyAsync(hp, outc, sizeof(uint64_t) * nout, hipMemcpyDeviceToHost,
                              c->stream));
        if (outw)
            HIPCHK(hipMemcpyAsync(hp + sizeof(uint64_t) * nout, outw, sizeof(double) * nout,
                                  hipMemcpyDeviceToHost, c->stream));
        if (outr)
            HIPCHK(hipMemcpyAsync(hp + (sizeof(uint64_t) + sizeof(double)) * nout, outr,
                                  sizeof(double) * nout, hipMemcpyDeviceToHost, c->stream));
    }
    record(c, timing, 6);
    if (ctl.capture)
        return CF_OK;
    HIPCHK(hipStreamSynchronize(c->stream));
    const char *hm = pin + p_misc;
    unsigned rqn = 0;
    memcpy(&rqn, hm + M_RQCOUNT, 4);
    unsigned hflags;
    memcpy(&hflags, hm + M_FLAGS, 4);
    if (hflags & PC_FLAG_RADEC)
        return fail(c, CF_ERANGE, "RA must lie in [0, 360] and DEC in [-90, 90]");
    if (hflags & PC_FLAG_NONFINITE)
        return fail(c, CF_EINVAL, "non-finite coordinate");
    if (hflags & PC_FLAG_RANGE)
        return fail(c, CF_ERANGE, "periodic coordinate outside [0, boxsize]");
    if (hflags & PC_FLAG_WEIGHT)
        return fail(c, CF_EINVAL, "non-finite weight");
    if (hflags & PC_FLAG_UNIT)
        return fail(c, CF_EINVAL,
                    "the angular grid needs unit vectors (squared norm within 2^-20 of 1)");
    if (hflags & PC_FLAG_WFIXED)
        return fail(c, CF_EINVAL,
                    "deterministic_weights: the weights span too wide a range for exact "
                    "fixed-point sums (every pair weight must be a multiple of one power of "
                    "two 2^Q, Q >= -1022, and below 2^(Q + 94))");
    int32_t sizes[2];
    memcpy(sizes, hm + M_SIZES, sizeof(sizes));
    if (async_items && (hflags & PC_FLAG_ITEMS)) {
        // the work list outgrew the capacity taken from the last call: redo
        // the call with the count read first
        c->last_items = 0;
        RunCtl again = ctl;
        again.no_async = true;
        const cf_status st3 = run(c, again, metric, theta, d1, ncat, d2, edges, nb, pimax, npi,
                                  boxsize, prec, counts, wsum, opt_in);
        ctl.pin_need = again.pin_need;
        ctl.p_misc = again.p_misc;
        ctl.p_out = again.p_out;
        return st3;
    }
    c->last_items = sizes[0];
    c->last_shape = std::move(shape);
    hcounts[0] = sizes[0];
    hcounts[1] = sizes[1];
    if (!opt.output_on_device) {
        memcpy(counts, hp, sizeof(uint64_t) * nout);
        if (wsum && user_w)
            memcpy(wsum, hp + sizeof(uint64_t) * nout, sizeof(double) * nout);
        else if (wsum)
            memset(wsum, 0, sizeof(double) * nout);
        if (want_ravg)
            memcpy(opt.ravg, hp + (sizeof(uint64_t) + sizeof(double)) * nout,
                   sizeof(double) * nout);
    }
    unsigned long long cnd;
    memcpy(&cnd, hm + M_CAND, 8);
    unsigned nflush = 0;
    memcpy(&nflush, hm + M_FLUSH, 4);
    cf_stats &S = c->stats;
    S.flushes = nflush;
    for (int k = 0; k < 3; k++) {
        S.grid[k] = g.n[k];
        S.cell_width[k] = g.width[k];
    }
    if (sky_grid)
        S.grid[0] = g.nband;
    S.zreach = g.zreach;
    S.slices_per_reach = opt.slices_per_reach;
    S.angular_grid = opt.angular_grid;
    S.xy_refine = sky_grid ? 0 : g.xyk;
    S.separation_form = fp32 ? (xy_mag > 0.0 ? 2 : 1) : 0;
    S.chunk = chunk;
    S.n_blocks = hcounts[1];
    S.n_items = hcounts[0];
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

// ---- graph replay of repeated identical calls --------------------------


// Everything a recorded call depends on: the catalogue views (pointers and
// sizes, not the data), bins, box, precision, options and device outputs.
std::vector<char> call_key(int metric, bool theta, const cf_catalog *d1, int32_t ncat,
                           const cf_catalog *d2, const double *edges, int32_t nb, double pimax,
                           int32_t npi, double boxsize, cf_precision prec, uint64_t *counts,
                           double *wsum, const cf_options &opt)
{
    std::vector<char> k;
    const int32_t head[5] = {metric, theta ? 1 : 0, ncat, d2 ? 1 : 0, (int32_t)prec};
    key_add(k, head, sizeof(head));
    key_add(k, d1, sizeof(cf_catalog) * (size_t)ncat);
    if (d2)
        key_add(k, d2, sizeof(cf_catalog));
    key_add(k, &nb, sizeof(nb));
    key_add(k, edges, sizeof(double) * (size_t)(nb + 1));
    key_add(k, &pimax, sizeof(pimax));
    key_add(k, &npi, sizeof(npi));
    key_add(k, &boxsize, sizeof(boxsize));
    // host output arrays may change between replays (the results are copied
    // out after each); device outputs are part of the graph
    cf_options o = opt;
    if (!opt.output_on_device)
        o.ravg = nullptr;
    key_add(k, &o, sizeof(o));
    const bool has_w = wsum != nullptr, has_r = opt.ravg != nullptr;
    key_add(k, &has_w, sizeof(has_w));
    key_add(k, &has_r, sizeof(has_r));
    if (opt.output_on_device) {
        key_add(k, &counts, sizeof(counts));
        key_add(k, &wsum, sizeof(wsum));
    }
    return k;
}

void drop_graph(cf_ctx *c)
{
    uploads_clear(c);
    if (c->gexec)
        (void)hipGraphExecDestroy(c->gexec);
    if (c->graph)
        (void)hipGraphDestroy(c->graph);
    c->gexec = nullptr;
    c->graph = nullptr;
    c->gkey.clear();
}

// Replay the cached graph.  Returns CF_OK with the outputs filled, a
// failure status, or CF_EOVERFLOW when the inputs now need more work items
// than the graph holds (the caller then runs eagerly and records anew).
cf_status replay(cf_ctx *c, uint64_t *counts, double *wsum, const cf_options &opt)
{
    HIPCHK(hipSetDevice(c->device));
    // the graph writes its own uploads into the same buffers
    uploads_clear(c);
    HIPCHK(hipGraphLaunch(c->gexec, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    const char *pin = static_cast<const char *>(c->gpin);
    const char *hm = pin + c->g_misc;
    unsigned hflags;
    memcpy(&hflags, hm + M_FLAGS, 4);
    if (hflags & PC_FLAG_ITEMS)
        return CF_EOVERFLOW;
    if (hflags & PC_FLAG_NONFINITE)
        return fail(c, CF_EINVAL, "non-finite coordinate");
    if (hflags & PC_FLAG_RANGE)
        return fail(c, CF_ERANGE, "periodic coordinate outside [0, boxsize]");
    if (hflags & PC_FLAG_WEIGHT)
        return fail(c, CF_EINVAL, "non-finite weight");
    if (hflags & PC_FLAG_WFIXED)
        return fail(c, CF_EINVAL, "deterministic_weights: the weights span too wide a range");
    if (!opt.output_on_device) {
        memcpy(counts, pin + c->g_out, sizeof(uint64_t) * c->g_nout);
        if (wsum && c->g_wsum)
            memcpy(wsum, pin + c->g_out + sizeof(uint64_t) * c->g_nout,
                   sizeof(double) * c->g_nout);
        else if (wsum)
            memset(wsum, 0, sizeof(double) * c->g_nout);
        if (opt.ravg && c->g_ravg)
            memcpy(opt.ravg, pin + c->g_out + (sizeof(uint64_t) + sizeof(double)) * c->g_nout,
                   sizeof(double) * c->g_nout);
    }
    c->stats = c->gstats;
    c->stats.replayed = 1;
    unsigned rqn = 0;
    unsigned long long cnd = 0;
    memcpy(&rqn, hm + M_RQCOUNT, 4);
    memcpy(&cnd, hm + M_CAND, 8);
    c->stats.rechecks = rqn;
    c->stats.candidate_pairs = cnd;
    unsigned nflush = 0;
    memcpy(&nflush, hm + M_FLUSH, 4);
    c->stats.flushes = nflush;
    return CF_OK;
}

// Record the call's device work into a graph (after an eager run of the same
// call has sized every buffer).  Failure only means no graph is kept.
void record_graph(cf_ctx *c, std::vector<char> &&key, const RunCtl &eager, int metric,
                  bool theta, const cf_catalog *d1, int32_t ncat, const cf_catalog *d2,
                  const double *edges, int32_t nb, double pimax, int32_t npi, double boxsize,
                  cf_precision prec, uint64_t *counts, double *wsum, const cf_options *opt)
{
    drop_graph(c);
    if (!c->cap_stream && hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking) !=
                              hipSuccess) {
        (void)hipGetLastError();
        c->cap_stream = nullptr;
        return;
    }
    if (c->gpin_cap < eager.pin_need) {
        if (c->gpin)
            (void)hipHostFree(c->gpin);
        c->gpin = nullptr;
        c->gpin_cap = 0;
        if (hipHostMalloc(&c->gpin, eager.pin_need, hipHostMallocDefault) != hipSuccess) {
            (void)hipGetLastError();
            c->gpin = nullptr;
            return;
        }
        c->gpin_cap = eager.pin_need;
    }
    RunCtl ctl;
    ctl.capture = true;
    ctl.item_cap = item_margin(c->last_items);
    if (ctl.item_cap <= 0)
        return;
    ctl.pin = static_cast<char *>(c->gpin);
    ctl.pin_cap = c->gpin_cap;
    if (ensure(c, B_ITEMS, sizeof(pc_item) * (size_t)ctl.item_cap) != CF_OK ||
        ensure(c, B_ICELL, sizeof(int32_t) * (size_t)ctl.item_cap) != CF_OK)
        return;
    const cf_stats keep = c->stats;
    const std::string keep_err = c->err;
    hipStream_t user = c->stream;
    c->stream = c->cap_stream;
    hipGraph_t graph = nullptr;
    cf_status st = CF_EDEVICE;
    if (hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeRelaxed) == hipSuccess) {
        st = run(c, ctl, metric, theta, d1, ncat, d2, edges, nb, pimax, npi, boxsize, prec,
                 counts, wsum, opt);
        if (hipStreamEndCapture(c->cap_stream, &graph) != hipSuccess)
            st = CF_EDEVICE;
    }
    c->stream = user;
    c->stats = keep;
    c->err = keep_err;
    hipGraphExec_t exec = nullptr;
    if (st == CF_OK && graph &&
        hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) == hipSuccess) {
        c->graph = graph;
        c->gexec = exec;
        c->gkey = std::move(key);
        c->g_misc = ctl.p_misc;
        c->g_out = ctl.p_out;
        c->g_nout = (size_t)ncat * (size_t)nb * (size_t)(metric != PC_METRIC_R ? npi : 1);
        c->g_wsum = wsum != nullptr && d1->w != nullptr;
        c->g_ravg = opt && opt->ravg != nullptr;
        c->gstats = keep;
        return;
    }
    (void)hipGetLastError();
    if (graph)
        (void)hipGraphDestroy(graph);
}

// Entry of every counting call: eager, or (cf_options.use_graph) a replay of
// the graph recorded for the same call.
// Workload class of a call for the tuning cache: metric, precision,
// weights, auto/cross, bins, and the orders of magnitude of the points per
// catalogue, of the catalogue count and of the mean number of neighbours
// within the reach (points per catalogue x reach volume / domain volume).
std::vector<int64_t> tune_key(int metric, bool theta, const cf_catalog *d1, int32_t ncat,
                              const cf_catalog *d2, const double *edges, int32_t nb,
                              double pimax, int32_t npi, double boxsize, cf_precision prec)
{
    double n = 0.0;
    for (int i = 0; i < ncat; i++)
        n += (double)d1[i].n;
    n /= ncat;
    const double r = edges[nb];
    const double rz = metric == PC_METRIC_RPPI ? pimax : r;
    const double vol = boxsize > 0.0 ? boxsize * boxsize * boxsize : 0.0;
    const double neigh = vol > 0.0 ? n * r * r * rz / vol : 0.0;
    auto mag = [](double v) { return (int64_t)std::floor(std::log2(std::max(v, 1.0))); };
    return {metric, theta ? 1 : 0, (int64_t)prec, d1->w ? 1 : 0, d2 ? 1 : 0, nb, npi,
            mag(n), mag((double)ncat), mag(neigh * 1e3)};
}

cf_status count(cf_ctx *c, int metric, bool theta, const cf_catalog *d1, int32_t ncat,
                const cf_catalog *d2, const double *edges, int32_t nb, double pimax, int32_t npi,
                double boxsize, cf_precision prec, uint64_t *counts, double *wsum,
                const cf_options *opt_in)
{
    // autotuning: pick slices_per_reach and chunk (and, for angular counts,
    // the right-ascension refinement of the angular grid, else the x/y
    // refinement of the 3-D grid) by timing whole calls on the live input
    // (coordinate descent), once per workload class
    cf_options tuned_opt;
    const cf_options *opt = opt_in;
    if (c && opt_in && opt_in->struct_size == (int32_t)sizeof(cf_options) && opt_in->autotune &&
        d1 && edges && nb >= 1 && ncat >= 1 && !opt_in->output_on_device) {
        tuned_opt = *opt_in;
        tuned_opt.autotune = 0;
        tuned_opt.collect_timing = 0;
        std::vector<int64_t> tk =
            tune_key(metric, theta, d1, ncat, d2, edges, nb, pimax, npi, boxsize, prec);
        tk.push_back(opt_in->angular_grid);
        tk.push_back(opt_in->xy_refine);
        auto it = c->tuned.find(tk);
        if (it == c->tuned.end()) {
            RunCtl probe;
            // the angular grid of angular counts is tuned too when left at
            // its default
            const bool tune_ang = theta && opt_in->angular_grid == 0;
            int32_t best_ang = tune_ang ? 16 : opt_in->angular_grid;
            int32_t best_spr = 32, best_chunk = 2048;
            // x/y refinement of a 3-D grid, when left at its default
            const bool tune_xy = opt_in->xy_refine == 0 && !(theta && best_ang >= 0);
            int32_t best_xy = tune_xy ? 1 : opt_in->xy_refine;
            auto time_call = [&](int32_t spr, int32_t chunk, int32_t ang,
                                 double *ms) -> cf_status {
                cf_options o = tuned_opt;
                o.use_graph = 0;
                o.slices_per_reach = spr;
                o.chunk = chunk;
                o.angular_grid = ang;
                o.xy_refine = best_xy;
                const auto t0 = std::chrono::steady_clock::now();
                cf_status st = run(c, probe, metric, theta, d1, ncat, d2, edges, nb, pimax, npi,
                                   boxsize, prec, counts, wsum, &o);
                *ms = std::chrono::duration<double, std::milli>(
                          std::chrono::steady_clock::now() - t0).count();
                return st;
            };
            double best = 0.0;
            cf_status st = time_call(best_spr, best_chunk, best_ang, &best);   // warms buffers
            if (st != CF_OK)
                return st;
            if ((st = time_call(best_spr, best_chunk, best_ang, &best)))
                return st;
            for (int32_t spr : {2, 4, 8, 16, 32}) {
                if (spr == best_spr)
                    continue;
                double ms;
                if ((st = time_call(spr, best_chunk, best_ang, &ms)))
                    return st;
                if (ms < best) {
                    best = ms;
                    best_spr = spr;
                }
            }
            for (int32_t chunk : {512, 1024, 4096, 8192}) {
                double ms;
                if ((st = time_call(best_spr, chunk, best_ang, &ms)))
                    return st;
                if (ms < best) {
                    best = ms;
                    best_chunk = chunk;
                }
            }
            if (tune_ang)
                for (int32_t ang : {8, 32}) {
                    double ms;
                    if ((st = time_call(best_spr, best_chunk, ang, &ms)))
                        return st;
                    if (ms < best) {
                        best = ms;
                        best_ang = ang;
                    }
                }
            if (tune_xy) {
                best_xy = 2;
                double ms;
                if ((st = time_call(best_spr, best_chunk, best_ang, &ms)))
                    return st;
                if (ms < best)
                    best = ms;
                else
                    best_xy = 1;
            }
            it = c->tuned.emplace(tk, cf_ctx::Tuned{best_spr, best_chunk, best_ang, best_xy})
                     .first;
        }
        tuned_opt.slices_per_reach = it->second.slices_per_reach;
        tuned_opt.chunk = it->second.chunk;
        tuned_opt.angular_grid = it->second.angular_grid;
        tuned_opt.xy_refine = it->second.xy_refine;
        tuned_opt.collect_timing = opt_in->collect_timing;
        opt = &tuned_opt;
    }
    RunCtl eager;
    const bool want_graph = c && opt && opt->struct_size == (int32_t)sizeof(cf_options) &&
                            opt->use_graph && d1 && edges && nb >= 1 && ncat >= 1;
    if (!want_graph)
        return run(c, eager, metric, theta, d1, ncat, d2, edges, nb, pimax, npi, boxsize, prec,
                   counts, wsum, opt);
    std::vector<char> key = call_key(metric, theta, d1, ncat, d2, edges, nb, pimax, npi,
                                     boxsize, prec, counts, wsum, *opt);
    if (c->gexec && key == c->gkey) {
        c->err.clear();
        cf_status st = replay(c, counts, wsum, *opt);
        if (st != CF_EOVERFLOW)
            return st;
        drop_graph(c);
    }
    cf_status st = run(c, eager, metric, theta, d1, ncat, d2, edges, nb, pimax, npi, boxsize,
                       prec, counts, wsum, opt);
    if (st != CF_OK)
        return st;
    bool ok = boxsize > 0.0 && !theta && c->last_items > 0;
    for (int i = 0; i < ncat && ok; i++)
        ok = d1[i].mem == CF_MEM_DEVICE;
    if (d2)
        ok = ok && d2->mem == CF_MEM_DEVICE;
    if (ok)
        record_graph(c, std::move(key), eager, metric, theta, d1, ncat, d2, edges, nb, pimax,
                     npi, boxsize, prec, counts, wsum, opt);
    return CF_OK;
}

// Host staging pinned at context creation: enough for every single-catalogue
// DD(r) call (the staging of run() is about 256 KiB plus 24 bytes per bin).
constexpr size_t kNoallocPinned = 1u << 20;

// Device bytes a no-allocation DD(r) call needs at least: per point of each
// side the gridded copies (float32 and binary64 coordinates, binary64
// weights), the 32-byte gather records, the counting-sort and cell-id
// scratch, and staged host columns; plus a margin for the bins, blocks and
// counters.  The work list is sized on the device and checked when taken.
size_t noalloc_need(const cf_catalog *d1, const cf_catalog *d2)
{
    size_t need = 1u << 20;
    for (const cf_catalog *d : {d1, d2}) {
        if (!d || d->n <= 0)
            continue;
        const size_t n = (size_t)d->n;
        size_t per = 12 + 24 + 32 + 4 * 3 + 8 + 4 + 1;   // X..Z, x..z, rec, sort, cols, ids, blocks
        if (d->w)
            per += 8 + (d->mem == CF_MEM_HOST ? dsize(d->wdtype) : 0);
        if (d->mem == CF_MEM_HOST)
            per += 3 * dsize(d->dtype);
        need += n * per;
    }
    return need + need / 4;   // the headroom of every buffer
}

}  // namespace

extern "C" {

cf_status count_pairs_r_noalloc(cf_ctx *c, const cf_catalog *d1, const cf_catalog *d2,
                                const double *edges, int32_t nbins, double boxsize,
                                cf_precision prec, uint64_t *counts, double *wsum,
                                const cf_options *opt)
{
    if (!c)
        return CF_EINVAL;
    c->err.clear();
    if (!c->scratch)
        return fail(c, CF_EDEVICE, "no fixed scratch on this device");
    if (opt && opt->struct_size == (int32_t)sizeof(cf_options) &&
        (opt->use_graph || opt->autotune))
        return fail(c, CF_EINVAL,
                    "use_graph and autotune allocate; count_pairs_r_noalloc takes neither");
    if (d1 && d1->n >= 0 && (!d2 || d2->n >= 0)) {
        const size_t need = noalloc_need(d1, d2);
        if (need > c->scratch_cap)
            return fail(c, CF_EINVAL,
                        "count_pairs_r_noalloc: %lld + %lld points need about %zu MiB of "
                        "scratch, more than its fixed %zu MiB; use count_pairs_r_ex",
                        (long long)d1->n, (long long)(d2 ? d2->n : 0), need >> 20,
                        c->scratch_cap >> 20);
    }
    // run the ordinary pipeline on a buffer table carved from the fixed
    // scratch; the context's own buffers and work-list history stay as they
    // were for its other calls
    DevBuf saved[B_COUNT];
    for (int k = 0; k < B_COUNT; k++) {
        saved[k] = c->buf[k];
        c->buf[k] = DevBuf{};
    }
    const int32_t saved_items = c->last_items;
    std::vector<char> saved_shape;
    saved_shape.swap(c->last_shape);
    c->arena = true;
    c->arena_off = 0;
    RunCtl ctl;
    ctl.no_async = true;
    const cf_status st = run(c, ctl, PC_METRIC_R, false, d1, 1, d2, edges, nbins, 0.0, 1,
                             boxsize, prec, counts, wsum, opt);
    c->arena = false;
    for (int k = 0; k < B_COUNT; k++)
        c->buf[k] = saved[k];
    c->last_items = saved_items;
    c->last_shape.swap(saved_shape);
    return st;
}

void cf_default_options(cf_options *opt)
{
    if (!opt)
        return;
    memset(opt, 0, sizeof(*opt));
    opt->struct_size = (int32_t)sizeof(cf_options);
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
    // set-up of the no-allocation entry point: the device address of this
    // device's fixed scratch (looked up with the device current) and host
    // staging pinned now, so that such a call allocates nothing
    void *sp = nullptr;
    size_t sbytes = 0;
    e = pc::noalloc_scratch(device, &sp, &sbytes);
    if (e != hipSuccess) {
        g_create_error = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
        (void)hipGetLastError();
        cf_destroy(c);
        return CF_EDEVICE;
    }
    c->scratch = static_cast<char *>(sp);
    c->scratch_cap = sbytes;
    if (ensure_pinned(c, kNoallocPinned) != CF_OK) {
        g_create_error = c->err;
        cf_destroy(c);
        return CF_ENOMEM;
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
        (void)release(c, b);
    if (c->pinned)
        (void)hipHostFree(c->pinned);
    drop_graph(c);
    if (c->gpin)
        (void)hipHostFree(c->gpin);
    if (c->cap_stream)
        (void)hipStreamDestroy(c->cap_stream);
    for (auto &ev : c->ev)
        if (ev)
            (void)hipEventDestroy(ev);
    delete c;
    return CF_OK;
}

cf_status cf_set_allocator(cf_ctx *c, cf_alloc_fn alloc, cf_free_fn free_, void *user)
{
    if (!c)
        return CF_EINVAL;
    if ((alloc == nullptr) != (free_ == nullptr))
        return fail(c, CF_EINVAL, "give both an allocation and a release function, or neither");
    HIPCHK(hipSetDevice(c->device));
    HIPCHK(hipStreamSynchronize(c->stream));
    // buffers from the previous allocator go back to it; a recorded graph
    // held their addresses
    drop_graph(c);
    for (auto &b : c->buf)
        HIPCHK(release(c, b));
    c->last_items = 0;
    c->last_shape.clear();
    c->alloc = alloc;
    c->free_ = free_;
    c->alloc_user = user;
    c->err.clear();
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
    return count(c, PC_METRIC_R, false, d1, 1, d2, edges, nbins, 0.0, 1, boxsize, prec, counts,
               wsum, opt);
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
    return count(c, PC_METRIC_RPPI, false, d1, 1, d2, rp_edges, nrp, pimax, npi, boxsize, prec,
               counts, wsum, opt);
}

cf_status count_pairs_rppi(cf_ctx *c, const cf_catalog *d1, const cf_catalog *d2,
                           const double *rp_edges, int32_t nrp, double pimax, int32_t npi,
                           double boxsize, cf_precision prec, uint64_t *counts, double *wsum)
{
    return count_pairs_rppi_ex(c, d1, d2, rp_edges, nrp, pimax, npi, boxsize, prec, counts, wsum,
                               nullptr);
}

cf_status count_pairs_rppi_mocks_ex(cf_ctx *c, const cf_catalog *d1, const cf_catalog *d2,
                                    const double *rp_edges, int32_t nrp, double pimax,
                                    int32_t npi, cf_precision prec, uint64_t *counts,
                                    double *wsum, const cf_options *opt)
{
    return count(c, PC_METRIC_MOCKS, false, d1, 1, d2, rp_edges, nrp, pimax, npi, 0.0, prec,
                 counts, wsum, opt);
}

cf_status count_pairs_rppi_mocks(cf_ctx *c, const cf_catalog *d1, const cf_catalog *d2,
                                 const double *rp_edges, int32_t nrp, double pimax,
                                 int32_t npi, cf_precision prec, uint64_t *counts,
                                 double *wsum)
{
    return count_pairs_rppi_mocks_ex(c, d1, d2, rp_edges, nrp, pimax, npi, prec, counts, wsum,
                                     nullptr);
}

cf_status count_pairs_rppi_batch_ex(cf_ctx *c, const cf_catalog *cats, int32_t ncat,
                                    const double *rp_edges, int32_t nrp, double pimax,
                                    int32_t npi, double boxsize, cf_precision prec,
                                    uint64_t *counts, double *wsum, const cf_options *opt)
{
    return count(c, PC_METRIC_RPPI, false, cats, ncat, nullptr, rp_edges, nrp, pimax, npi, boxsize,
               prec, counts, wsum, opt);
}

cf_status count_pairs_rppi_batch(cf_ctx *c, const cf_catalog *cats, int32_t ncat,
                                 const double *rp_edges, int32_t nrp, double pimax, int32_t npi,
                                 double boxsize, cf_precision prec, uint64_t *counts,
                                 double *wsum)
{
    return count_pairs_rppi_batch_ex(c, cats, ncat, rp_edges, nrp, pimax, npi, boxsize, prec,
                                     counts, wsum, nullptr);
}

cf_status count_pairs_theta_ex(cf_ctx *c, const cf_catalog *d1, const cf_catalog *d2,
                               const double *theta_edges_deg, int32_t nbins, cf_precision prec,
                               uint64_t *counts, double *wsum, const cf_options *opt)
{
    return count(c, PC_METRIC_R, true, d1, 1, d2, theta_edges_deg, nbins, 0.0, 1, 0.0, prec, counts,
               wsum, opt);
}

cf_status count_pairs_theta(cf_ctx *c, const cf_catalog *d1, const cf_catalog *d2,
                            const double *theta_edges_deg, int32_t nbins, cf_precision prec,
                            uint64_t *counts, double *wsum)
{
    return count_pairs_theta_ex(c, d1, d2, theta_edges_deg, nbins, prec, counts, wsum, nullptr);
}

}  // extern "C"
