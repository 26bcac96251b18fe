/*
 * paircount.h -- C ABI of the MI355X (gfx950) binned pair counter.
 *
 * Binned pair counting of Sinha & Garrison, "Corrfunc" (arXiv:1911.03545):
 * the brute-force definition of Code 1 (section "How to compute a correlation
 * function") evaluated with the paper's cell-list method (sections
 * "Partitioning the particles on a grid", "Associating pairs of cells",
 * "Symmetry considerations for autocorrelations").  Separations follow
 * Appendix A, periodic wrapping follows Code 3, the pair convention follows
 * Appendix B.
 *
 * Conventions shared by every counting call
 * -----------------------------------------
 *  * Positions are structure-of-arrays (x[], y[], z[]), float32 or float64,
 *    promoted exactly to binary64.  Weights are optional, float32 or float64.
 *  * Bin edges e_0 < e_1 < ... < e_nb (e_0 >= 0) are compared in squared
 *    form: a pair lies in bin k iff fl(e_k*e_k) <= s < fl(e_{k+1}*e_{k+1}),
 *    with s evaluated in binary64 in the order ((dx*dx + dy*dy) + dz*dz),
 *    dx = x_i - x_j, and for periodic boxes the wrap of Code 3
 *    (dx > L/2 -> dx - L; dx <= -L/2 -> dx + L).  Integer counts are
 *    bit-exact with that definition in both precision modes.
 *  * counts[] are ordered-pair counts (uint64).  An autocorrelation (d2 ==
 *    NULL) equals the cross-correlation of d1 with itself, i.e. it includes
 *    the N self-pairs in bin 0 when e_0 == 0 (Appendix B).
 *  * wsum[] (optional) is sum over the same pairs of the pair weight
 *    (w_i * w_j, or w_i + w_j with cf_options.weight_type) accumulated in
 *    binary64; its order of accumulation is not fixed, so it matches the
 *    exact sum to a relative error of about 1e-13 rather than bit-exactly.
 *  * cf_options.ravg (optional) receives the mean separation per bin.  The
 *    binary64 mode sums sqrt(s) (theta: 2 asin(sqrt(s) / 2) in degrees) in
 *    binary64 like wsum.  The float32 mode sums the separation of the
 *    float32 evaluation, whose error is bounded by a few float32 roundings
 *    of the coordinates (relative to the domain origin) and of the result.
 *  * boxsize > 0 selects a periodic cube [0, boxsize]^3 (every coordinate
 *    must lie in the closed interval); boxsize <= 0 selects a non-periodic
 *    domain bounded by the bounding box of both catalogues; NaN or +inf is
 *    CF_EINVAL.
 *  * Precision: CF_PREC_FP64 evaluates every pair in binary64 exactly as
 *    above.  CF_PREC_FP32_RECHECK evaluates pairs in float32 and decides only
 *    the pairs that a proven error bound places away from every squared edge;
 *    the remaining pairs are re-evaluated in binary64 inside the same sweep.
 *    Both give identical counts.
 *
 * Memory and streams
 * ------------------
 *  Inputs are borrowed for the duration of the call and never retained.
 *  They may be host or device memory (cf_catalog.mem).  Outputs are host
 *  memory unless cf_options.output_on_device is set.  Work runs on the
 *  context's HIP stream; every counting call returns only after its results
 *  are in the output arrays.  A context is not thread safe.
 *
 * Errors
 * ------
 *  Every function returns a cf_status; on error the outputs are unspecified
 *  and cf_last_error() describes the failure.  No call aborts the process.
 */
#ifndef PAIRCOUNT_H
#define PAIRCOUNT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    CF_OK = 0,
    CF_EINVAL = -1,       /* bad argument: NULL pointer, nbins < 1, edges not
                             increasing or negative, NaN/Inf, npi < 1,
                             pimax <= 0, weights on one catalogue only,
                             unsupported dtype, too many points or bins     */
    CF_ERANGE = -2,       /* periodic coordinate outside [0, boxsize];
                             RA outside [0,360], DEC outside [-90,90];
                             theta edge above 180 degrees                   */
    CF_ENOMEM = -3,       /* device or pinned-host allocation failed        */
    CF_EDEVICE = -4,      /* HIP runtime error                              */
    CF_EUNSUPPORTED = -5, /* periodic reach above boxsize/3                 */
    CF_EOVERFLOW = -6     /* a count would exceed 2^64 - 1                  */
} cf_status;

typedef enum { CF_F32 = 1, CF_F64 = 2 } cf_dtype;
typedef enum { CF_MEM_HOST = 0, CF_MEM_DEVICE = 1 } cf_mem;
typedef enum { CF_PREC_FP64 = 0, CF_PREC_FP32_RECHECK = 1 } cf_precision;

/* A borrowed view of one catalogue.  For count_pairs_theta x holds RA and y
   holds DEC in degrees and z is unused, unless cf_options.theta_unit_vectors
   is set, in which case x, y, z are unit vectors.  For count_pairs_rppi_mocks
   x, y are RA, DEC in degrees and z the line-of-sight distance, unless
   cf_options.theta_unit_vectors is set, in which case x, y, z are Cartesian
   positions (distance times unit vector). */
typedef struct cf_catalog {
    int64_t n;          /* number of points, >= 0                          */
    int32_t dtype;      /* cf_dtype of x, y, z                             */
    int32_t wdtype;     /* cf_dtype of w (ignored when w == NULL)          */
    int32_t mem;        /* cf_mem: where x, y, z and w live                */
    int32_t reserved;   /* must be 0                                       */
    const void *x;
    const void *y;
    const void *z;
    const void *w;      /* NULL: unweighted                                */
} cf_catalog;

/* Tuning and output options; zero-initialise and set struct_size, or call
   cf_default_options.  Zero fields take the defaults. */
typedef struct cf_options {
    int32_t struct_size;        /* sizeof(cf_options)                          */
    int32_t slices_per_reach;   /* z slices per line-of-sight reach (0: 32;
                                   declination slices per band on the angular
                                   grid)                                       */
    int32_t chunk;              /* max j points per work item (default 2048)   */
    int32_t output_on_device;   /* counts / wsum are device pointers           */
    int32_t theta_unit_vectors; /* theta input is unit vectors, not RA/DEC;
                                   on-sky (mocks) input is Cartesian positions,
                                   not RA/DEC/distance                         */
    int32_t collect_timing;     /* time phases with HIP events (cf_stats)      */
    int32_t hist_copies;        /* LDS histogram replicas per wave (0: auto)   */
    int32_t use_graph;          /* replay repeated identical calls from a HIP
                                   graph (periodic, device-resident inputs)    */
    int32_t autotune;           /* time slices_per_reach and chunk candidates
                                   (and, when left at 0, angular_grid 8 / 32
                                   for angular counts or xy_refine 2 for 3-D
                                   grids) on the first call of a workload class
                                   and reuse the fastest (cached per context)  */
    int32_t weight_type;        /* cf_weight: weight of a pair from the weights
                                   of its two points (needs weights unless
                                   CF_WEIGHT_PRODUCT)                          */
    int32_t angular_grid;       /* angular counts only: the cell layout.  0
                                   (default): the paper's angular grid
                                   (section "Partitioning the particles on a
                                   grid: angular correlation functions") with
                                   16 right-ascension cells per reach.  n in
                                   1..64: declination bands one angular reach
                                   high, cut into right-ascension cells 1/n of
                                   the band's right-ascension reach wide, with
                                   slices_per_reach declination slices per
                                   band.  -1: 3-D cells on the unit vectors
                                   (chord reach).  Counts are identical either
                                   way.  The angular grid needs unit vectors
                                   (squared norm within 2^-20 of 1, else
                                   CF_EINVAL), which RA/DEC input always
                                   gives.  Other statistics need 0.            */
    int32_t xy_refine;          /* 3-D grids: columns at least reach/k wide in
                                   x and y (section "Sub-dividing the cells"),
                                   k in 1..4 (0: 1); a block then pairs with
                                   the (2k+1)^2 columns around its own, each
                                   over a z window narrowed by the columns'
                                   transverse distance when the reach is a
                                   ball.  Lowered when a periodic box has fewer
                                   than 2k+1 columns.                           */
    int32_t radec_on_device;    /* RA/DEC (and distance) input: 0 (default)
                                   converts to unit vectors (positions) on the
                                   host with the C library's sin and cos, in
                                   parallel threads, the formula and library
                                   of a host reference, so counts are
                                   reproducible against it bit for bit
                                   (device-resident input is copied to the
                                   host and back); 1 converts on the device, a
                                   faster mode whose math library may differ
                                   from the host's in the last bit of a
                                   vector, which can move a pair lying within
                                   an ulp of an edge into the next bin.       */
    int32_t flush_pairs;        /* > 0: merge a wave's LDS histogram replicas
                                   into the global bins whenever its pending
                                   pair evaluations would exceed this many (at
                                   most the default, which keeps the uint32
                                   LDS counters from wrapping); a test hook
                                   for the overflow guard of section "Finding
                                   and updating the histogram bins".  0: the
                                   default bound.                              */
    int32_t deterministic_weights; /* 1: sum the pair weights (section 2.1,
                                   weight_func) in exact fixed point instead of
                                   binary64 atomics: wsum is then the exact sum
                                   of the binary64 pair weights, rounded once
                                   (ties to even), identical in every run and
                                   on every device.  Every pair weight must be
                                   a multiple of one power of two 2^Q (found
                                   from the weights: the lowest set bits of
                                   their significands, and for products the
                                   ulp of the smallest product) with |w_ij| <
                                   2^(Q + 94) and Q >= -1022, else CF_EINVAL:
                                   products of weights that span less than
                                   2^23 in magnitude (float32 values) or 2^20
                                   (any binary64 values) fit; sums span far
                                   wider ranges.
                                   The self-pair weights (first edge zero) are
                                   summed the same way; the mean separation's
                                   numerator stays a binary64 sum.  0: binary64
                                   atomics (the default; sums then agree with
                                   the exact sum to about 1e-12 relative).     */
    int32_t separation_form;    /* float32 DD(r), DD(rp, pi) (also batched)
                                   and theta-as-chord sweeps of 3-D grids (no
                                   mean separation): how the squared
                                   separation (rp^2) is formed.  1: from the
                                   coordinate differences dx^2 + dy^2 + dz^2;
                                   2: x and y expanded as |a|^2 + |b|^2 -
                                   2 a.b (|b|^2 stored per point by the
                                   gridding, -2 a and |a|^2 per lane), one
                                   instruction fewer per pair, with a larger
                                   absolute rounding bound (about u times 17
                                   squared column widths, folded into the
                                   decision bands, so results stay exact; a
                                   pair inside a band is first tested
                                   against the band narrowed by its own
                                   magnitudes, then rechecked in binary64);
                                   0 (default): 2 when that bound widens the
                                   band of the smallest nonzero edge by at
                                   most an eighth of its value, else 1.  Other
                                   statistics and the binary64 mode ignore
                                   it.  cf_stats.separation_form reports the
                                   form used.                                  */
    double *ravg;               /* optional output, same layout and memory kind
                                   as counts: the mean separation of the pairs
                                   in each bin (r, rp, or theta in degrees),
                                   weighted by the pair weights when weights
                                   are given; 0 for a bin with no weight.  The
                                   paper's average separation output, which
                                   costs a square root (theta: also an arc
                                   sine) per pair in range; NULL skips it.     */
} cf_options;

/* Pair weight (section 2.1, weight_func): the product w_i * w_j (the usual
   choice) or the sum w_i + w_j, each one rounded binary64 operation. */
typedef enum { CF_WEIGHT_PRODUCT = 0, CF_WEIGHT_SUM = 1 } cf_weight;

/* Statistics of the last counting call on a context. */
typedef struct cf_stats {
    int32_t grid[3];            /* x columns, y columns, z slices (angular
                                   grid: declination bands, right-ascension
                                   cells of all bands, slices per band)        */
    int32_t zreach;             /* z slices searched on each side              */
    double cell_width[3];       /* x, y column widths and z slice width        */
    int64_t n_blocks;           /* i-blocks of up to 64 points                 */
    int64_t n_items;            /* work items processed by the pair sweep      */
    uint64_t candidate_pairs;   /* pair evaluations performed by the sweep     */
    uint64_t rechecks;          /* FP32 pairs re-evaluated in binary64         */
    int32_t sweep_workgroups;   /* persistent workgroups of the sweep launch   */
    int32_t hist_copies;        /* LDS histogram replicas per wave             */
    float t_prepare_ms;         /* validation, conversion, bounding box        */
    float t_grid_ms;            /* cell index + scan + scatter                 */
    float t_worklist_ms;        /* blocks + work items                         */
    float t_sweep_ms;           /* pair sweep kernel (with binary64 rechecks)  */
    float t_finalize_ms;        /* doubling, self-pairs, copy-out              */
    float t_total_ms;           /* whole call, first to last event             */
    int32_t slices_per_reach;   /* z slices per reach used (after autotuning)  */
    int32_t chunk;              /* max j points per work item used             */
    int32_t replayed;           /* 1 when the call replayed a recorded graph   */
    int32_t angular_grid;       /* angular grid refinement used (0: 3-D cells) */
    int32_t xy_refine;          /* x/y refinement of a 3-D grid (0: angular)   */
    int32_t separation_form;    /* float32 sweep: 1 differences, 2 expanded x
                                   and y (cf_options.separation_form); 0 when
                                   no float32 sweep ran                        */
    uint64_t flushes;           /* mid-sweep merges of LDS histogram replicas
                                   forced by the overflow bound (flush_pairs)  */
} cf_stats;

typedef struct cf_ctx cf_ctx;

/* Create a context on HIP device `device` that enqueues all work on
   `hip_stream` (a hipStream_t; NULL = the null stream).  The stream stays
   owned by the caller and must outlive the context. */
cf_status cf_create(int device, void *hip_stream, cf_ctx **out);
cf_status cf_destroy(cf_ctx *ctx);
/* Device scratch allocator of a context (the gridded arrays, work lists,
   histograms: everything the library keeps on the device between calls).
   alloc(bytes, user) must return `bytes` of device memory on the context's
   device, 256-byte aligned, usable on the context's stream (NULL on failure,
   which the call reports as CF_ENOMEM); free_(ptr, user) takes it back.  The
   library frees a buffer only after synchronising its stream.  Passing NULL
   for both restores hipMalloc / hipFree.  Buffers held when the allocator
   changes go back to the allocator that made them first; cf_destroy returns
   the rest.  Errors: CF_EINVAL when ctx is NULL or exactly one function is
   NULL. */
typedef void *(*cf_alloc_fn)(size_t bytes, void *user);
typedef void (*cf_free_fn)(void *ptr, void *user);
cf_status cf_set_allocator(cf_ctx *ctx, cf_alloc_fn alloc, cf_free_fn free_, void *user);
/* Message of the last failing call on ctx, or with ctx == NULL of the last
   failing cf_create on this thread (never NULL). */
const char *cf_last_error(const cf_ctx *ctx);
cf_status cf_get_stats(const cf_ctx *ctx, cf_stats *out);
void cf_default_options(cf_options *opt);

/* DD(r) -- Table 1 "xi(r)" / "DD": 3-D separations (Appendix A).
   counts[nbins], wsum[nbins] (wsum may be NULL). */
cf_status count_pairs_r(cf_ctx *ctx, const cf_catalog *d1, const cf_catalog *d2,
                        const double *edges, int32_t nbins, double boxsize,
                        cf_precision prec, uint64_t *counts, double *wsum);
cf_status count_pairs_r_ex(cf_ctx *ctx, const cf_catalog *d1, const cf_catalog *d2,
                           const double *edges, int32_t nbins, double boxsize,
                           cf_precision prec, uint64_t *counts, double *wsum,
                           const cf_options *opt);

/* DD(r) without allocation -- for callers that cannot allocate during a
   call: code under HIP stream capture, tight serving loops, harnesses that
   forbid hipMalloc.  The same counts as count_pairs_r_ex (same pipeline and
   kernels), but every device buffer is carved from one fixed device scratch
   array of CF_NOALLOC_SCRATCH_BYTES per GPU, a file-scope array of the
   library that each GPU it runs on holds until the process ends; host
   staging is pinned when the context is created.  The call makes no
   hipMalloc, hipHostMalloc, hipFree or allocator callback.
   Limits: the points of d1 and d2 together need about 115 bytes each (plus
   10 with weights, plus the staged columns of host input) and the work list
   20 bytes per item, all within the scratch: about 1.1e6 points of an
   autocorrelation; beyond that the call returns CF_EINVAL before any device
   work (or, when the work list outgrows the rest, before the sweep) with a
   message naming the limit.  cf_options.use_graph and autotune are rejected
   (CF_EINVAL).  Every call on a GPU shares that GPU's scratch, which keeps
   the last call's contents (each call clears what it needs zeroed): calls
   that overlap on one GPU, from any context or stream, race and must be
   serialised by the caller. */
#define CF_NOALLOC_SCRATCH_BYTES (128ull << 20)
cf_status count_pairs_r_noalloc(cf_ctx *ctx, const cf_catalog *d1, const cf_catalog *d2,
                                const double *edges, int32_t nbins, double boxsize,
                                cf_precision prec, uint64_t *counts, double *wsum,
                                const cf_options *opt);

/* DD(rp, pi) -- Table 1 "DDrppi" / "wp": rp^2 = dx^2 + dy^2 and pi = |dz|
   with z the line of sight (Appendix A).  pi bins are q_p = p * fl(pimax/npi)
   for p < npi and q_npi = pimax, half-open, so pi < pimax; wp(rp) counts are
   the sums over p.  counts[k * npi + p], wsum likewise. */
cf_status count_pairs_rppi(cf_ctx *ctx, const cf_catalog *d1, const cf_catalog *d2,
                           const double *rp_edges, int32_t nrp, double pimax,
                           int32_t npi, double boxsize, cf_precision prec,
                           uint64_t *counts, double *wsum);
cf_status count_pairs_rppi_ex(cf_ctx *ctx, const cf_catalog *d1, const cf_catalog *d2,
                              const double *rp_edges, int32_t nrp, double pimax,
                              int32_t npi, double boxsize, cf_precision prec,
                              uint64_t *counts, double *wsum, const cf_options *opt);

/* Batched DD(rp, pi) autocorrelations -- many catalogues (for example the
   mock catalogues of an MCMC fit, the use case of section "Introduction") with
   the same bins, box and precision, counted in one pass: one gridding over
   all catalogues (catalogue k owns its own cells), one work list and one
   persistent sweep launch whose per-wave histograms are flushed per
   catalogue.  cats[ncat] are borrowed like single catalogues (host or device
   memory, any mix); all have weights or none.  Each catalogue's result
   equals count_pairs_rppi on it alone.  counts[(c * nrp + k) * npi + p] and
   wsum likewise; ncat in [1, 2^19]; the total number of points is limited
   like a single call.  Returns CF_EINVAL when the cells of all catalogues
   together exceed 2^31 (use fewer slices_per_reach). */
cf_status count_pairs_rppi_batch(cf_ctx *ctx, const cf_catalog *cats, int32_t ncat,
                                 const double *rp_edges, int32_t nrp, double pimax,
                                 int32_t npi, double boxsize, cf_precision prec,
                                 uint64_t *counts, double *wsum);
cf_status count_pairs_rppi_batch_ex(cf_ctx *ctx, const cf_catalog *cats, int32_t ncat,
                                    const double *rp_edges, int32_t nrp, double pimax,
                                    int32_t npi, double boxsize, cf_precision prec,
                                    uint64_t *counts, double *wsum, const cf_options *opt);

/* DD(theta) / DR(theta) -- Table 1 "DDtheta_mocks": angular separations
   (Appendix A, spherical volumes) binned through the squared chord of unit
   vectors, |v1 - v2|^2 = 2 - 2 cos(theta), a monotone function of theta.
   Unit vectors v = (cos d cos a, cos d sin a, sin d) with a, d = RA, DEC in
   radians (degrees * fl(pi/180)) are formed on the host (on the device with
   cf_options.radec_on_device); chord edges c_k = 2 sin(theta_k / 2) on the
   host.  theta edges in degrees, at most 180.
   Never periodic.  counts[nbins], wsum[nbins]. */
cf_status count_pairs_theta(cf_ctx *ctx, const cf_catalog *d1, const cf_catalog *d2,
                            const double *theta_edges_deg, int32_t nbins,
                            cf_precision prec, uint64_t *counts, double *wsum);
cf_status count_pairs_theta_ex(cf_ctx *ctx, const cf_catalog *d1, const cf_catalog *d2,
                               const double *theta_edges_deg, int32_t nbins,
                               cf_precision prec, uint64_t *counts, double *wsum,
                               const cf_options *opt);

/* DD(rp, pi) of on-sky catalogues ("mocks"), Appendix A (spherical volumes,
   the convention of Fisher et al. 1994): positions v = D u from RA, DEC
   (degrees) and the line-of-sight distance D, in the units of the bins (the
   paper's CZ input becomes a distance only through a cosmology, which the
   caller applies).  With s = v1 - v2 and L = v1 + v2 (twice the line of
   sight l, which cancels), evaluated in binary64 in this order:
       sl = (sx*Lx + sy*Ly) + sz*Lz,  LL = (Lx*Lx + Ly*Ly) + Lz*Lz,
       ss = (sx*sx + sy*sy) + sz*sz,  pi = |sl| / sqrt(LL) (0 if LL == 0),
       rp^2 = max(ss - pi*pi, 0);
   the pair is in bin (k, p) iff fl(rp_k^2) <= rp^2 < fl(rp_{k+1}^2) and
   q_p <= pi < q_{p+1} (q_p as for count_pairs_rppi).  The cell grid reaches
   sqrt(rp_max^2 + pimax^2) along every axis (section "Partitioning the
   particles on a grid").  Never periodic.  Both precision modes evaluate in
   binary64.  counts[k * npi + p], wsum likewise; cf_options.ravg gives the
   mean rp per bin. */
cf_status count_pairs_rppi_mocks(cf_ctx *ctx, const cf_catalog *d1, const cf_catalog *d2,
                                 const double *rp_edges, int32_t nrp, double pimax,
                                 int32_t npi, cf_precision prec, uint64_t *counts,
                                 double *wsum);
cf_status count_pairs_rppi_mocks_ex(cf_ctx *ctx, const cf_catalog *d1, const cf_catalog *d2,
                                    const double *rp_edges, int32_t nrp, double pimax,
                                    int32_t npi, cf_precision prec, uint64_t *counts,
                                    double *wsum, const cf_options *opt);

/* Grid plan (host only, no device work) -- the cell grid of section
   "Partitioning the particles on a grid": columns of width >= reach_xy in x
   and y (a pair within the reach can only be one column apart), and z
   slices of width extent_z / n_z with zreach slices searched on each side.
   lo/hi: bounding box (ignored when boxsize > 0, which selects [0, boxsize]).
   Returns CF_EUNSUPPORTED when a periodic axis would have fewer than three
   columns, CF_EINVAL on non-finite or non-positive reaches. */
typedef struct cf_grid_plan {
    double lo[3];
    double extent[3];
    double inv_width[3];   /* cells per unit length used for cell assignment */
    double width[3];
    int32_t n[3];          /* x columns, y columns, z slices                 */
    int32_t zreach;
    int32_t periodic;
    int32_t reserved;
    double boxsize;
    int64_t ncell;
} cf_grid_plan;
cf_status cf_plan_grid(const double lo[3], const double hi[3], double boxsize,
                       double reach_xy, double reach_z, int32_t slices_per_reach,
                       cf_grid_plan *out);
/* The same with x/y refinement (cf_options.xy_refine; columns at least
   reach_xy / k wide, k lowered while a periodic axis has fewer than 2k + 1
   columns) and, with `ball` nonzero (the reach is a 3-D ball: r, angular
   chords, on-sky pairs), the z window of each column offset narrowed by the
   offsets' smallest transverse distance.  zro receives 25 values, zro[5 a +
   b] for offsets |ox| = a, |oy| = b (0..4): the z slices searched on each
   side, -1 where no pair of the two columns can be within reach.  *k_used
   receives k. */
cf_status cf_plan_grid_ex(const double lo[3], const double hi[3], double boxsize,
                          double reach_xy, double reach_z, int32_t slices_per_reach,
                          int32_t xy_refine, int32_t ball, cf_grid_plan *out, int16_t *zro,
                          int32_t *k_used);

/* Angular grid plan (host only, no device work) -- see
   cf_options.angular_grid.  chord_reach: the largest chord 2 sin(theta_max/2)
   of the bins; zlo, zhi: range of the unit vectors' z components (the
   declination range).  Band b covers declinations from dec_lo + b *
   band_height; its RA cells are columns col0 .. col0 + nra - 1, cell a
   starting at RA 2 pi a / nra.  dra[d] bounds the right-ascension difference
   (radians, round the circle) of two vectors within the reach, one in band b
   and one in band b - 1 + d; a value >= pi means any.  bands receives nband
   entries (at most max_bands, else CF_EINVAL). */
typedef struct cf_sky_band {
    int32_t col0;
    int32_t nra;
    double ra_scale;       /* nra / (2 pi)                                    */
    double dra[3];
} cf_sky_band;
typedef struct cf_sky_plan {
    int32_t nband;
    int32_t ncol;          /* RA cells of all bands                           */
    int32_t slices;        /* declination slices per band                     */
    int32_t zreach;        /* slices searched on each side                    */
    double dec_lo;         /* radians                                         */
    double band_height;    /* radians, >= the angular reach                   */
    double inv_slice;      /* slices per radian of declination                */
    double theta_reach;    /* angular reach with its margins (radians)        */
} cf_sky_plan;
cf_status cf_plan_sky_grid(double chord_reach, double zlo, double zhi, int32_t slices,
                           int32_t ra_refine, cf_sky_plan *out, cf_sky_band *bands,
                           int32_t max_bands);

/* Float32 decision bands (host only) -- for each squared edge E_k the float32
   interval [lo_k, hi_k] outside which a float32-evaluated separation decides
   the comparison with E_k the same way as the binary64 definition.  `ndim`
   is the number of squared axis differences summed (3 for r and theta, 2 for
   rp^2, 1 for the line-of-sight pi with E_k given unsquared); `coord_scale`
   bounds the magnitude of every coordinate and periodic offset.  A zero edge
   gets the empty band [-1, -1].  Returns CF_EINVAL on bad input. */
cf_status cf_fp32_bands(const double *edges_sq, int32_t nedges, int32_t ndim,
                        double coord_scale, float *lo, float *hi);
/* The same with a rounding bound per axis (axis_eps[ndim]): the largest
   total error of the two float32 coordinates whose difference is taken on
   that axis.  cf_fp32_bands uses 6 u S on every axis (box-frame
   coordinates, u = 2^-24, S = coord_scale); the float32 sweeps of 3-D grids
   hold x and y relative to column centres, so their bound scales with the
   column width.  Per axis dl = eps (1 + u) + u (r + eps) + 2 U S with
   U = 2^-53, r = sqrt(E); then B = (2 r sqrt(sum dl^2) + sum dl^2 +
   (ndim + 1)(u + U) s') * 1.25 with s' = E + 2 r sqrt(sum dl^2) + sum dl^2,
   and the band is [E - B, E + B] rounded outward to float32. */
cf_status cf_fp32_bands_axes(const double *edges_sq, int32_t nedges, int32_t ndim,
                             const double *axis_eps, double coord_scale, float *lo,
                             float *hi);
/* The bands of the expanded form of a 3-D grid's float32 sweep
   (cf_options.separation_form 2), ndim 3 (r): x and y as t0 = fl(dz dz +
   Bj), t1 = fl(-2 a_x b_x + t0), t2 = fl(-2 a_y b_y + t1), s = fl(t2 + A)
   with Bj = fl(b_y b_y + fl(b_x b_x)) and A = fl(a_y a_y + fl(a_x a_x));
   ndim 2 (rp^2): t0 = fl(A + Bj), t1 = fl(-2 a_x b_x + t0), s = fl(-2 a_y
   b_y + t1).  The arithmetic term (ndim + 1) u s' above becomes u (6 s' + M)
   (1 + 2^-20) with M = 5 |b|^2 + 2 |a|^2 + 4 (|a_x b_x| + |a_y b_y|) (ndim
   3) or 4 |a|^2 + 4 |b|^2 + 2 (|a_x b_x| + |a_y b_y|) (ndim 2) at the
   largest magnitudes, given
   as xy_max = {a_x, a_y, b_x, b_y} (the lane's largest |x|, |y| in the j
   column's frame, the j point's); the coordinate term is unchanged.
   axis_eps holds ndim values.  The sweep narrows the band of a pair inside
   it by 1.25 u (1 + 2^-20) (M - m), m the same term at the pair's own
   magnitudes (bounded above from |a|^2 and |b|^2 alone), before it
   rechecks the pair in binary64. */
cf_status cf_fp32_bands_xy(const double *edges_sq, int32_t nedges, int32_t ndim,
                           const double *axis_eps, const double *xy_max, double coord_scale,
                           float *lo, float *hi);

/* Host-only: the two float32 constants of that narrowing as the sweep
   receives them, for coordinates scaled by fscale > 0: *K = 1.25 u (1 +
   2^-20) and *M = fscale^2 times M of the bands above (xy_max and ndim as
   for cf_fp32_bands_xy), each rounded down; a pair narrows its band by
   K (M - m) with m in the scaled coordinates.  CF_EINVAL on a null
   pointer, ndim other than 2 or 3, or a negative or non-finite value. */
cf_status cf_fp32_pair_margin(const double *xy_max, int32_t ndim, double fscale, float *K,
                              float *M);

/* Host-only: the exact sum of n values p[k], each an integer multiple of 2^q
   with |p[k]| < 2^(q + 94), rounded once to binary64 (ties to even), through
   the same fixed-point arithmetic as cf_options.deterministic_weights (three
   signed 32-bit limbs per value, int64 limb sums, a 192-bit total).
   CF_EINVAL for a value off the grid or too large, or q outside
   [-1022, 900].  out: one double. */
cf_status cf_fixed_sum(const double *p, int64_t n, int32_t q, double *out);

#ifdef __cplusplus
}
#endif
#endif /* PAIRCOUNT_H */
