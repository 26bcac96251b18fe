/*
 * paircount_oracle.c -- TEST INFRASTRUCTURE, not part of the library.
 *
 * A plain, slow, obviously correct CPU implementation of binned pair counting
 * as defined in Sinha & Garrison, "Corrfunc -- a suite of blazing fast
 * correlation functions on the CPU" (arXiv:1911.03545).  Only the test suite,
 * the smoke check and the benchmark's CPU-baseline leg load it.  It shares no
 * code, header, table or constant with the GPU library, and the GPU library
 * never calls it.
 *
 * What is computed (the brute-force pair counter of Code 1 in section 2.1,
 * "How to compute a correlation function"):
 *
 *   for every ordered pair (i, j) in D1 x D2:
 *       s = separation(i, j)                      -- distance_metric
 *       skip unless E_0 <= s < E_nb               -- min/max separation cut
 *       k = bin of s                              -- dist_to_bin_index
 *       counts[k] += 1; wsum[k] += w_i * w_j      -- weight_func (product)
 *
 * Precision rules (binary64, round to nearest even, no FMA contraction: the
 * file is compiled with -ffp-contract=off and without -ffast-math):
 *   * inputs are promoted exactly to binary64 by the caller;
 *   * separations are compared in squared form (section "Finding and updating
 *     the histogram bins": bins on r^2 avoid the square root), so the squared
 *     edges are E_k = fl(e_k * e_k) and a pair lies in bin k iff
 *     E_k <= s < E_{k+1} (half-open bins, Code 1's skip test);
 *   * per axis dx = x_i - x_j, then the periodic wrap of Code 3
 *     ("Accounting for periodic boundary conditions"):
 *         if (dx >  L/2) dx -= L;   if (dx <= -L/2) dx += L;
 *   * 3-D separation (Appendix A, eq. for r^2): s = (dx*dx + dy*dy) + dz*dz;
 *   * rp^2 = dx*dx + dy*dy and pi = |dz| with z the line of sight
 *     (Appendix A, Cartesian volumes);
 *   * on-sky (rp, pi) ("mocks", Appendix A, spherical volumes, after Fisher et
 *     al. 1994): positions v = D u with u the unit vector of (RA, DEC) below
 *     and D the line-of-sight distance; s = v1 - v2 and the line of sight
 *     l = (v1 + v2) / 2, evaluated as L = v1 + v2 (the factor 1/2 cancels
 *     exactly in pi):
 *         sl = (sx*Lx + sy*Ly) + sz*Lz,  LL = (Lx*Lx + Ly*Ly) + Lz*Lz,
 *         ss = (sx*sx + sy*sy) + sz*sz,
 *         pi = |sl| / sqrt(LL)   (0 when LL == 0: both points at the observer),
 *         rp^2 = max(ss - pi*pi, 0)   (rounding cannot make it negative);
 *     bins as for the Cartesian (rp, pi) statistic; never periodic;
 *   * angular separations use unit vectors v = (cos d cos a, cos d sin a, sin d)
 *     and the squared chord |v1 - v2|^2 with edges c_k = 2 sin(theta_k / 2);
 *     this is the cos(theta) = v1.v2 relation of Appendix A rewritten as a
 *     monotone function of theta that needs no arccos.
 *
 * Pair weights (section 2.1's weight_func): the product w_i * w_j, or, as a
 * second example of a user weighting scheme, the sum w_i + w_j; each is one
 * rounded binary64 operation per pair.
 *
 * Mean separation per bin (the average separation that the paper computes
 * only on request, since it costs a square root, or an arc function for
 * angles, per pair): the pair-weighted mean sum(sep_ij * w_ij) / sum(w_ij)
 * over the pairs of the bin, with w_ij = 1 without weights (then the
 * denominator is the count).  sep_ij = fl(sqrt(s)) for r and rp; for angles
 * theta_ij = fl(fl(2 * asin(0.5 * fl(sqrt(chord^2)))) * fl(180 / pi)) in
 * degrees, the arc form that stays accurate for small angles.  Self-pairs
 * add their weight (w_i * w_i, or w_i + w_i) to the denominator and zero to
 * the numerator.  Both sums are exactly rounded (below); the mean is their
 * rounded quotient, and 0 for a bin without weight.
 *
 * Pair convention (section "Symmetry considerations for autocorrelations" and
 * Appendix B): an autocorrelation of D must equal the cross-correlation of D
 * with itself, i.e. all N^2 ordered pairs including i == j.  It is computed as
 * the paper describes: unique pairs j > i only, counts doubled, and N
 * self-pairs added to bin 0 when the first edge is exactly zero.  Weighted
 * sums follow the same rule (unique-pair products doubled, w_i^2 added when
 * the first edge is zero).  Weighted sums are the exact real sum of the
 * binary64 products, rounded once, via Shewchuk's non-overlapping expansions
 * (the algorithm behind Python's math.fsum).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORACLE_OK 0
#define ORACLE_EINVAL (-1)
#define ORACLE_ENOMEM (-3)
#define ORACLE_EINTERNAL (-7)

/* ------------------------------------------------------------------------ */
/* Exact summation: a sum is held as a list of non-overlapping partials in   */
/* increasing magnitude (Shewchuk 1997, "Adaptive precision floating-point   */
/* arithmetic"), and rounded to binary64 once at the end with the            */
/* round-half-even correction used by Python's math.fsum.                    */
/* ------------------------------------------------------------------------ */
#define XSUM_MAX 64
typedef struct {
    int n;
    int overflow;
    double p[XSUM_MAX];
} xacc;

static void xacc_add(xacc *a, double x)
{
    int i = 0;
    for (int k = 0; k < a->n; k++) {
        double y = a->p[k];
        if (fabs(x) < fabs(y)) {
            double t = x;
            x = y;
            y = t;
        }
        double hi = x + y;
        double lo = y - (hi - x);
        if (lo != 0.0)
            a->p[i++] = lo;
        x = hi;
    }
    if (i >= XSUM_MAX) {
        a->overflow = 1;
        return;
    }
    a->p[i++] = x;
    a->n = i;
}

static double xacc_value(const xacc *a)
{
    int n = a->n;
    double hi = 0.0;
    if (n > 0) {
        double lo = 0.0;
        n--;
        hi = a->p[n];
        while (n > 0) {
            double x = hi;
            n--;
            double y = a->p[n];
            hi = x + y;
            double yr = hi - x;
            lo = y - yr;
            if (lo != 0.0)
                break;
        }
        /* If the discarded tail pushes past a half-way case, round away. */
        if (n > 0 && ((lo < 0.0 && a->p[n - 1] < 0.0) ||
                      (lo > 0.0 && a->p[n - 1] > 0.0))) {
            double y = lo * 2.0;
            double x = hi + y;
            double yr = x - hi;
            if (y == yr)
                hi = x;
        }
    }
    return hi;
}

static void xacc_merge(xacc *dst, const xacc *src)
{
    for (int k = 0; k < src->n; k++)
        xacc_add(dst, src->p[k]);
    dst->overflow |= src->overflow;
}

/* Exact rounded sum of an array: exported so the tests can pin the
   summation against an independent implementation. */
double oracle_xsum(int64_t n, const double *v)
{
    xacc a;
    a.n = 0;
    a.overflow = 0;
    for (int64_t i = 0; i < n; i++)
        xacc_add(&a, v[i]);
    return xacc_value(&a);
}

/* ------------------------------------------------------------------------ */
/* Separations                                                               */
/* ------------------------------------------------------------------------ */

/* Code 3: minimum-image wrap of one axis difference, for positions in the
   closed interval [0, L]. */
static double wrap_axis(double d, double L, double half)
{
    if (d > half)
        d -= L;
    if (d <= -half)
        d += L;
    return d;
}

static int check_edges(const double *edges, int32_t nbins)
{
    if (nbins < 1 || edges == NULL)
        return ORACLE_EINVAL;
    for (int k = 0; k <= nbins; k++)
        if (!isfinite(edges[k]) || edges[k] < 0.0)
            return ORACLE_EINVAL;
    for (int k = 0; k < nbins; k++)
        if (!(edges[k] < edges[k + 1]))
            return ORACLE_EINVAL;
    return ORACLE_OK;
}

/* pi bins of Appendix A: npi bins of equal width pimax/npi in [0, pimax).
   q_p = p * fl(pimax / npi) for p < npi, and q_npi = pimax exactly, so the
   line-of-sight cut is pi < pimax. */
int oracle_pi_edges(double pimax, int32_t npi, double *q)
{
    if (!(pimax > 0.0) || !isfinite(pimax) || npi < 1)
        return ORACLE_EINVAL;
    double dpi = pimax / (double)npi;
    for (int p = 0; p < npi; p++)
        q[p] = (double)p * dpi;
    q[npi] = pimax;
    for (int p = 0; p < npi; p++)
        if (!(q[p] < q[p + 1]))
            return ORACLE_EINVAL;
    return ORACLE_OK;
}

/* Separation reported in the mean-separation output: the distance sqrt(s)
   (r, rp), or (angle != 0) the angle in degrees of a squared chord s.       */
static double separation_value(int angle, double s)
{
    const double c = sqrt(s);
    if (!angle)
        return c;
    return (2.0 * asin(0.5 * c)) * (180.0 / M_PI);
}

/* Weight of pair (a, b): 0 product, 1 sum.                                 */
static double pair_weight(int wtype, double a, double b)
{
    return wtype == 1 ? a + b : a * b;
}

/* ------------------------------------------------------------------------ */
/* Exactly pruned pair sets (for the full-size reference counts)             */
/* ------------------------------------------------------------------------ */
/* Every summand of a separation is non-negative and rounding is monotone,
   so s = fl(fl(fl(dx*dx) + fl(dy*dy)) + fl(dz*dz)) >= fl(d*d) for each axis
   difference d (likewise rp^2 >= fl(dx*dx), fl(dy*dy); and pi = |dz|).  If
   the wrapped, rounded difference along one axis has |d| >= R, where R is
   the largest edge (pimax for pi), then fl(d*d) >= fl(R*R) and the pair lies
   outside every bin.  The rounded difference is within a few ulps of the
   exact one, so a pair whose exact difference along the axis (and, in a
   periodic box, along its images at +-L) exceeds R + margin, with the margin
   far above those ulps, can be skipped without changing any count.  The
   pruned variant sorts the second catalogue by that axis and visits, for
   each i, only the j whose key lies within R + margin of the key of i or of
   its periodic images; every visited pair goes through the unchanged
   definition below.                                                         */

/* First index of the ascending array k[0..n-1] whose value is >= v.      */
static int64_t first_at_least(const double *k, int64_t n, double v)
{
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        const int64_t mid = lo + (hi - lo) / 2;
        if (k[mid] < v)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo;
}

/* First index whose value is > v.                                         */
static int64_t first_above(const double *k, int64_t n, double v)
{
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        const int64_t mid = lo + (hi - lo) / 2;
        if (k[mid] <= v)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo;
}

/* The ranges of j visited for row i.  key2 == NULL: every j (j > i for an
   autocorrelation), the plain definition.  Otherwise key2 (ascending) holds
   the pruning axis of the second catalogue and ki that of point i; the
   ranges cover every j with |key2[j] - ki| <= reach and, in a periodic box
   of side L > 2 reach (so the three ranges are disjoint), with
   |key2[j] - ki -+ L| <= reach.  Returns the number of ranges (<= 3).      */
static int j_ranges(int64_t i, int autocorr, int64_t n2, const double *key2,
                    double ki, double reach, double L, int64_t *lo,
                    int64_t *hi)
{
    const int64_t jmin = autocorr ? i + 1 : 0;
    if (key2 == NULL) {
        lo[0] = jmin;
        hi[0] = n2;
        return 1;
    }
    int nr = 0;
    const double shift[3] = {0.0, L, -L};
    const int nimg = L > 0.0 ? 3 : 1;
    for (int m = 0; m < nimg; m++) {
        int64_t a = first_at_least(key2, n2, (ki + shift[m]) - reach);
        const int64_t b = first_above(key2, n2, (ki + shift[m]) + reach);
        if (a < jmin)
            a = jmin;
        if (a < b) {
            lo[nr] = a;
            hi[nr] = b;
            nr++;
        }
    }
    return nr;
}

/* One engine for the 1-D (r or chord) and the 2-D (rp, pi) statistics.
   mode 0: s = (dx*dx + dy*dy) + dz*dz, bins k over E
   mode 1: s = dx*dx + dy*dy, pi = |dz|, bins k*npi + p over E x q
   mode 2: s = rp^2 and pi of the on-sky convention, bins as mode 1
   wtype: pair weight (0 product, 1 sum); ravg (optional): mean separation
   per bin, angle != 0 reporting angles from squared chords.
   key2 (optional): the exactly pruned pair set of j_ranges, with key1 and
   key2 the pruning axis of the first and (ascending) second catalogue.      */
static int count_engine(int mode,
                        int64_t n1, const double *x1, const double *y1,
                        const double *z1, const double *w1,
                        int64_t n2, const double *x2, const double *y2,
                        const double *z2, const double *w2,
                        int autocorr, const double *edges, int32_t nbins,
                        const double *q, int32_t npi, double boxsize,
                        uint64_t *counts, double *wsum, int wtype, int angle,
                        double *ravg, int nthreads, const double *key1,
                        const double *key2, double reach)
{
    int rc = check_edges(edges, nbins);
    if (rc)
        return rc;
    if (n1 < 0 || counts == NULL)
        return ORACLE_EINVAL;
    if (autocorr) {
        n2 = n1;
        x2 = x1;
        y2 = y1;
        z2 = z1;
        w2 = w1;
        key2 = key1;
    } else if (n2 < 0) {
        return ORACLE_EINVAL;
    }
    const int weighted = (w1 != NULL);
    if (weighted && w2 == NULL)
        return ORACLE_EINVAL;
    if (wtype != 0 && (wtype != 1 || !weighted))
        return ORACLE_EINVAL;
    const int want_r = (ravg != NULL);
    const int nout = (mode >= 1) ? nbins * npi : nbins;
    const int periodic = boxsize > 0.0;
    if (mode == 2 && periodic)
        return ORACLE_EINVAL;
    const double L = boxsize;
    const double half = 0.5 * boxsize;
    const double pimax = (mode >= 1) ? q[npi] : 0.0;

    double *E = (double *)malloc(sizeof(double) * (size_t)(nbins + 1));
    if (!E)
        return ORACLE_ENOMEM;
    for (int k = 0; k <= nbins; k++)
        E[k] = edges[k] * edges[k];

    memset(counts, 0, sizeof(uint64_t) * (size_t)nout);
    xacc *total = NULL, *rtotal = NULL;
    if (weighted)
        total = (xacc *)calloc((size_t)nout, sizeof(xacc));
    if (want_r)
        rtotal = (xacc *)calloc((size_t)nout, sizeof(xacc));
    if ((weighted && !total) || (want_r && !rtotal)) {
        free(E);
        free(total);
        free(rtotal);
        return ORACLE_ENOMEM;
    }
    int failed = 0;

#ifdef _OPENMP
    if (nthreads <= 0)
        nthreads = omp_get_max_threads();
#pragma omp parallel num_threads(nthreads)
#endif
    {
        uint64_t *c = (uint64_t *)calloc((size_t)nout, sizeof(uint64_t));
        xacc *acc = weighted ? (xacc *)calloc((size_t)nout, sizeof(xacc)) : NULL;
        xacc *racc = want_r ? (xacc *)calloc((size_t)nout, sizeof(xacc)) : NULL;
        int ok = (c != NULL) && (!weighted || acc != NULL) && (!want_r || racc != NULL);
#ifdef _OPENMP
#pragma omp for schedule(dynamic, 16)
#endif
        for (int64_t i = 0; i < n1; i++) {
            if (!ok)
                continue;
            const double xi = x1[i], yi = y1[i], zi = z1[i];
            int64_t rlo[3], rhi[3];
            const int nr = j_ranges(i, autocorr, n2, key2, key2 ? key1[i] : 0.0,
                                    reach, L, rlo, rhi);
            for (int r = 0; r < nr; r++) {
                for (int64_t j = rlo[r]; j < rhi[r]; j++) {
                    double dx = xi - x2[j];
                    double dy = yi - y2[j];
                    double dz = zi - z2[j];
                    if (periodic) {
                        dx = wrap_axis(dx, L, half);
                        dy = wrap_axis(dy, L, half);
                        dz = wrap_axis(dz, L, half);
                    }
                    int bin;
                    double s;
                    if (mode == 0) {
                        s = (dx * dx + dy * dy) + dz * dz;
                        if (s < E[0] || s >= E[nbins])
                            continue;
                        int k = nbins - 1; /* reverse scan over the bins */
                        while (s < E[k])
                            k--;
                        bin = k;
                    } else {
                        double pi;
                        if (mode == 1) {
                            s = dx * dx + dy * dy;
                            pi = fabs(dz);
                        } else {
                            const double lx = xi + x2[j], ly = yi + y2[j], lz = zi + z2[j];
                            const double sl = (dx * lx + dy * ly) + dz * lz;
                            const double ll = (lx * lx + ly * ly) + lz * lz;
                            const double ss = (dx * dx + dy * dy) + dz * dz;
                            pi = ll > 0.0 ? fabs(sl) / sqrt(ll) : 0.0;
                            s = fmax(ss - pi * pi, 0.0);
                        }
                        if (s < E[0] || s >= E[nbins] || pi >= pimax)
                            continue;
                        int k = nbins - 1;
                        while (s < E[k])
                            k--;
                        int p = npi - 1;
                        while (pi < q[p])
                            p--;
                        bin = k * npi + p;
                    }
                    c[bin]++;
                    double prod = 1.0;
                    if (weighted) {
                        prod = pair_weight(wtype, w1[i], w2[j]);
                        /* autocorrelation: the unique pair stands for (i,j) and
                           (j,i); doubling is exact in binary64 */
                        xacc_add(&acc[bin], autocorr ? 2.0 * prod : prod);
                    }
                    if (want_r) {
                        const double rw = separation_value(angle, s) * prod;
                        xacc_add(&racc[bin], autocorr ? 2.0 * rw : rw);
                    }
                }
            }
        }
#ifdef _OPENMP
#pragma omp critical
#endif
        {
            if (!ok) {
                failed = 1;
            } else {
                for (int b = 0; b < nout; b++) {
                    counts[b] += c[b];
                    if (weighted)
                        xacc_merge(&total[b], &acc[b]);
                    if (want_r)
                        xacc_merge(&rtotal[b], &racc[b]);
                }
            }
        }
        free(c);
        free(acc);
        free(racc);
    }
    if (failed) {
        free(E);
        free(total);
        free(rtotal);
        return ORACLE_ENOMEM;
    }

    if (autocorr) {
        for (int b = 0; b < nout; b++)
            counts[b] *= 2u;
        /* Appendix B: self-pairs belong to bin 0 when it starts at zero
           separation (and, for (rp, pi), pi bin 0 always starts at zero). */
        if (E[0] == 0.0) {
            counts[0] += (uint64_t)n1;
            if (weighted)
                for (int64_t i = 0; i < n1; i++)
                    xacc_add(&total[0], pair_weight(wtype, w1[i], w1[i]));
        }
    }
    if (wsum) {
        for (int b = 0; b < nout; b++)
            wsum[b] = weighted ? xacc_value(&total[b]) : 0.0;
    }
    if (weighted) {
        for (int b = 0; b < nout; b++)
            if (total[b].overflow)
                rc = ORACLE_EINTERNAL;
    }
    if (want_r) {
        for (int b = 0; b < nout; b++) {
            const double den = weighted ? xacc_value(&total[b]) : (double)counts[b];
            ravg[b] = den != 0.0 ? xacc_value(&rtotal[b]) / den : 0.0;
            if (rtotal[b].overflow)
                rc = ORACLE_EINTERNAL;
        }
    }
    free(E);
    free(total);
    free(rtotal);
    return rc;
}

/* DD(r): counts[k] over r edges (edges[0..nbins]); boxsize <= 0 means
   non-periodic; autocorr != 0 ignores the second catalogue.  The _ex form
   adds the pair weight type and the optional mean separation per bin. */
int oracle_count_r_ex(int64_t n1, const double *x1, const double *y1,
                      const double *z1, const double *w1,
                      int64_t n2, const double *x2, const double *y2,
                      const double *z2, const double *w2,
                      int autocorr, const double *edges, int32_t nbins,
                      double boxsize, uint64_t *counts, double *wsum,
                      int wtype, double *ravg, int nthreads)
{
    return count_engine(0, n1, x1, y1, z1, w1, n2, x2, y2, z2, w2, autocorr,
                        edges, nbins, NULL, 0, boxsize, counts, wsum, wtype,
                        0, ravg, nthreads, NULL, NULL, 0.0);
}

int oracle_count_r(int64_t n1, const double *x1, const double *y1,
                   const double *z1, const double *w1,
                   int64_t n2, const double *x2, const double *y2,
                   const double *z2, const double *w2,
                   int autocorr, const double *edges, int32_t nbins,
                   double boxsize, uint64_t *counts, double *wsum,
                   int nthreads)
{
    return oracle_count_r_ex(n1, x1, y1, z1, w1, n2, x2, y2, z2, w2, autocorr,
                             edges, nbins, boxsize, counts, wsum, 0, NULL,
                             nthreads);
}

/* DD(rp, pi): counts[k * npi + p]; rp edges rp_edges[0..nrp]; the mean
   separation of the _ex form is the mean rp of each (rp, pi) bin. */
int oracle_count_rppi_ex(int64_t n1, const double *x1, const double *y1,
                         const double *z1, const double *w1,
                         int64_t n2, const double *x2, const double *y2,
                         const double *z2, const double *w2,
                         int autocorr, const double *rp_edges, int32_t nrp,
                         double pimax, int32_t npi, double boxsize,
                         uint64_t *counts, double *wsum, int wtype,
                         double *ravg, int nthreads)
{
    if (npi < 1)
        return ORACLE_EINVAL;
    double *q = (double *)malloc(sizeof(double) * (size_t)(npi + 1));
    if (!q)
        return ORACLE_ENOMEM;
    int rc = oracle_pi_edges(pimax, npi, q);
    if (rc == ORACLE_OK)
        rc = count_engine(1, n1, x1, y1, z1, w1, n2, x2, y2, z2, w2,
                          autocorr, rp_edges, nrp, q, npi, boxsize, counts,
                          wsum, wtype, 0, ravg, nthreads, NULL, NULL, 0.0);
    free(q);
    return rc;
}

int oracle_count_rppi(int64_t n1, const double *x1, const double *y1,
                      const double *z1, const double *w1,
                      int64_t n2, const double *x2, const double *y2,
                      const double *z2, const double *w2,
                      int autocorr, const double *rp_edges, int32_t nrp,
                      double pimax, int32_t npi, double boxsize,
                      uint64_t *counts, double *wsum, int nthreads)
{
    return oracle_count_rppi_ex(n1, x1, y1, z1, w1, n2, x2, y2, z2, w2,
                                autocorr, rp_edges, nrp, pimax, npi, boxsize,
                                counts, wsum, 0, NULL, nthreads);
}

/* DD(rp, pi) of on-sky positions (mocks): Cartesian positions v = D u from
   oracle_sky_to_cartesian; counts[k * npi + p]; the mean separation is the
   mean rp per bin. */
int oracle_count_rppi_mocks(int64_t n1, const double *x1, const double *y1,
                            const double *z1, const double *w1,
                            int64_t n2, const double *x2, const double *y2,
                            const double *z2, const double *w2,
                            int autocorr, const double *rp_edges, int32_t nrp,
                            double pimax, int32_t npi, uint64_t *counts,
                            double *wsum, int wtype, double *ravg,
                            int nthreads)
{
    if (npi < 1)
        return ORACLE_EINVAL;
    double *q = (double *)malloc(sizeof(double) * (size_t)(npi + 1));
    if (!q)
        return ORACLE_ENOMEM;
    int rc = oracle_pi_edges(pimax, npi, q);
    if (rc == ORACLE_OK)
        rc = count_engine(2, n1, x1, y1, z1, w1, n2, x2, y2, z2, w2,
                          autocorr, rp_edges, nrp, q, npi, 0.0, counts,
                          wsum, wtype, 0, ravg, nthreads, NULL, NULL, 0.0);
    free(q);
    return rc;
}

/* RA/DEC in degrees -> unit vectors (binary64, host libm). */
int oracle_radec_to_unit(int64_t n, const double *ra, const double *dec,
                         double *x, double *y, double *z)
{
    const double d2r = M_PI / 180.0;
    for (int64_t i = 0; i < n; i++) {
        if (!(ra[i] >= 0.0 && ra[i] <= 360.0 && dec[i] >= -90.0 &&
              dec[i] <= 90.0))
            return ORACLE_EINVAL;
        double a = ra[i] * d2r;
        double d = dec[i] * d2r;
        double cd = cos(d);
        x[i] = cd * cos(a);
        y[i] = cd * sin(a);
        z[i] = sin(d);
    }
    return ORACLE_OK;
}

/* RA/DEC in degrees and line-of-sight distance D -> positions D u. */
int oracle_sky_to_cartesian(int64_t n, const double *ra, const double *dec,
                            const double *dist, double *x, double *y,
                            double *z)
{
    int rc = oracle_radec_to_unit(n, ra, dec, x, y, z);
    if (rc)
        return rc;
    for (int64_t i = 0; i < n; i++) {
        if (!(dist[i] >= 0.0) || !isfinite(dist[i]))
            return ORACLE_EINVAL;
        x[i] = dist[i] * x[i];
        y[i] = dist[i] * y[i];
        z[i] = dist[i] * z[i];
    }
    return ORACLE_OK;
}

/* Angular edges (degrees) -> chord lengths c = 2 sin(theta / 2). */
int oracle_theta_chord_edges(int32_t nedges, const double *theta_deg,
                             double *chord)
{
    const double d2r = M_PI / 180.0;
    for (int k = 0; k < nedges; k++) {
        if (!(theta_deg[k] >= 0.0 && theta_deg[k] <= 180.0))
            return ORACLE_EINVAL;
        chord[k] = 2.0 * sin(0.5 * (theta_deg[k] * d2r));
    }
    return ORACLE_OK;
}

/* DD(theta) / DR(theta) from RA/DEC in degrees; the mean separation of
   the _ex form is the mean angle in degrees. */
int oracle_count_theta_ex(int64_t n1, const double *ra1, const double *dec1,
                          const double *w1, int64_t n2, const double *ra2,
                          const double *dec2, const double *w2, int autocorr,
                          const double *theta_edges_deg, int32_t nbins,
                          uint64_t *counts, double *wsum, int wtype,
                          double *ravg, int nthreads)
{
    if (n1 < 0 || nbins < 1)
        return ORACLE_EINVAL;
    if (autocorr)
        n2 = 0;
    double *v1 = (double *)malloc(sizeof(double) * 3 * (size_t)(n1 + 1));
    double *v2 = (double *)malloc(sizeof(double) * 3 * (size_t)(n2 + 1));
    double *c = (double *)malloc(sizeof(double) * (size_t)(nbins + 1));
    int rc = ORACLE_ENOMEM;
    if (v1 && v2 && c) {
        rc = oracle_theta_chord_edges(nbins + 1, theta_edges_deg, c);
        if (rc == ORACLE_OK)
            rc = oracle_radec_to_unit(n1, ra1, dec1, v1, v1 + n1, v1 + 2 * n1);
        if (rc == ORACLE_OK && !autocorr)
            rc = oracle_radec_to_unit(n2, ra2, dec2, v2, v2 + n2, v2 + 2 * n2);
        if (rc == ORACLE_OK)
            rc = count_engine(0, n1, v1, v1 + n1, v1 + 2 * n1, w1, n2, v2,
                              v2 + n2, v2 + 2 * n2, w2, autocorr, c, nbins,
                              NULL, 0, 0.0, counts, wsum, wtype, 1, ravg,
                              nthreads, NULL, NULL, 0.0);
    }
    free(v1);
    free(v2);
    free(c);
    return rc;
}

int oracle_count_theta(int64_t n1, const double *ra1, const double *dec1,
                       const double *w1, int64_t n2, const double *ra2,
                       const double *dec2, const double *w2, int autocorr,
                       const double *theta_edges_deg, int32_t nbins,
                       uint64_t *counts, double *wsum, int nthreads)
{
    return oracle_count_theta_ex(n1, ra1, dec1, w1, n2, ra2, dec2, w2,
                                 autocorr, theta_edges_deg, nbins, counts,
                                 wsum, 0, NULL, nthreads);
}

/* ------------------------------------------------------------------------ */
/* Exactly pruned variants (see j_ranges): the same counts and exactly      */
/* rounded sums as the plain functions, for inputs too large to enumerate.  */
/* ------------------------------------------------------------------------ */
typedef struct {
    double key;
    int64_t idx;
} keyed;

static int keyed_cmp(const void *a, const void *b)
{
    const keyed *p = (const keyed *)a, *q = (const keyed *)b;
    if (p->key < q->key)
        return -1;
    if (p->key > q->key)
        return 1;
    return (p->idx > q->idx) - (p->idx < q->idx);
}

/* A copy of a catalogue sorted by coordinate `axis`: columns x, y, z, w
   (w may be NULL) and the key column.  Returns NULL on allocation failure;
   the single block is released with free().                               */
static double *sorted_copy(int64_t n, const double *x, const double *y,
                           const double *z, const double *w, int axis,
                           double **sx, double **sy, double **sz, double **sw,
                           double **sk)
{
    const double *cols[3] = {x, y, z};
    keyed *order = (keyed *)malloc(sizeof(keyed) * (size_t)(n + 1));
    double *blk = (double *)malloc(sizeof(double) * 5 * (size_t)(n + 1));
    if (!order || !blk) {
        free(order);
        free(blk);
        return NULL;
    }
    for (int64_t i = 0; i < n; i++) {
        order[i].key = cols[axis][i];
        order[i].idx = i;
    }
    qsort(order, (size_t)n, sizeof(keyed), keyed_cmp);
    *sx = blk;
    *sy = blk + n;
    *sz = blk + 2 * n;
    *sw = w ? blk + 3 * n : NULL;
    *sk = blk + 4 * n;
    for (int64_t i = 0; i < n; i++) {
        const int64_t o = order[i].idx;
        (*sx)[i] = x[o];
        (*sy)[i] = y[o];
        (*sz)[i] = z[o];
        if (w)
            (*sw)[i] = w[o];
        (*sk)[i] = order[i].key;
    }
    free(order);
    return blk;
}

/* Largest magnitude of a column (the scale of its rounding errors).       */
static double max_abs(int64_t n, const double *v)
{
    double m = 0.0;
    for (int64_t i = 0; i < n; i++)
        if (fabs(v[i]) > m)
            m = fabs(v[i]);
    return m;
}

/* Pruned DD(r) (mode 0) or DD(rp, pi) (mode 1) along axis 0, 1 or 2: the
   reach is the largest edge, or pimax for the line of sight of mode 1.  The
   margin 1e-9 (L, or the coordinate scale without a box) exceeds the error
   of a rounded axis difference by orders of magnitude.  A periodic box must
   exceed 2.5 times the reach with its margin, so that the three key ranges
   of j_ranges are disjoint with room to spare.                             */
static int count_pruned(int mode, int axis, int64_t n1, const double *x1,
                        const double *y1, const double *z1, const double *w1,
                        int64_t n2, const double *x2, const double *y2,
                        const double *z2, const double *w2, int autocorr,
                        const double *edges, int32_t nbins, const double *q,
                        int32_t npi, double boxsize, uint64_t *counts,
                        double *wsum, int wtype, int angle, int nthreads)
{
    if (axis < 0 || axis > 2 || n1 < 0 || (!autocorr && n2 < 0))
        return ORACLE_EINVAL;
    int rc = check_edges(edges, nbins);
    if (rc)
        return rc;
    const double *c1[3] = {x1, y1, z1}, *c2[3] = {x2, y2, z2};
    const double R = (mode == 1 && axis == 2) ? q[npi] : edges[nbins];
    double scale = boxsize > 0.0 ? boxsize : max_abs(n1, c1[axis]);
    if (!autocorr && boxsize <= 0.0 && max_abs(n2, c2[axis]) > scale)
        scale = max_abs(n2, c2[axis]);
    const double reach = R + 1e-9 * (scale + R);
    if (boxsize > 0.0 && !(boxsize > 2.5 * reach))
        return ORACLE_EINVAL;
    double *bx, *by, *bz, *bw, *bk;
    double *blk = sorted_copy(autocorr ? n1 : n2, autocorr ? x1 : x2, autocorr ? y1 : y2,
                              autocorr ? z1 : z2, autocorr ? w1 : w2, axis, &bx, &by,
                              &bz, &bw, &bk);
    if (!blk)
        return ORACLE_ENOMEM;
    if (autocorr)
        rc = count_engine(mode, n1, bx, by, bz, bw, n1, bx, by, bz, bw, 1, edges,
                          nbins, q, npi, boxsize, counts, wsum, wtype, angle, NULL,
                          nthreads, bk, bk, reach);
    else /* the first catalogue keeps its order; its keys are its own column */
        rc = count_engine(mode, n1, x1, y1, z1, w1, n2, bx, by, bz, bw, 0, edges,
                          nbins, q, npi, boxsize, counts, wsum, wtype, angle, NULL,
                          nthreads, c1[axis], bk, reach);
    free(blk);
    return rc;
}

int oracle_count_r_pruned(int axis, int64_t n1, const double *x1, const double *y1,
                          const double *z1, const double *w1, int64_t n2,
                          const double *x2, const double *y2, const double *z2,
                          const double *w2, int autocorr, const double *edges,
                          int32_t nbins, double boxsize, uint64_t *counts,
                          double *wsum, int wtype, int nthreads)
{
    return count_pruned(0, axis, n1, x1, y1, z1, w1, n2, x2, y2, z2, w2, autocorr,
                        edges, nbins, NULL, 0, boxsize, counts, wsum, wtype, 0,
                        nthreads);
}

int oracle_count_rppi_pruned(int axis, int64_t n1, const double *x1,
                             const double *y1, const double *z1, const double *w1,
                             int64_t n2, const double *x2, const double *y2,
                             const double *z2, const double *w2, int autocorr,
                             const double *rp_edges, int32_t nrp, double pimax,
                             int32_t npi, double boxsize, uint64_t *counts,
                             double *wsum, int wtype, int nthreads)
{
    if (npi < 1)
        return ORACLE_EINVAL;
    double *q = (double *)malloc(sizeof(double) * (size_t)(npi + 1));
    if (!q)
        return ORACLE_ENOMEM;
    int rc = oracle_pi_edges(pimax, npi, q);
    if (rc == ORACLE_OK)
        rc = count_pruned(1, axis, n1, x1, y1, z1, w1, n2, x2, y2, z2, w2, autocorr,
                          rp_edges, nrp, q, npi, boxsize, counts, wsum, wtype, 0,
                          nthreads);
    free(q);
    return rc;
}

/* Pruned DD(theta) / DR(theta) of unit vectors (from oracle_radec_to_unit)
   and theta edges in degrees, along one axis of the unit vectors.         */
int oracle_count_theta_uv_pruned(int axis, int64_t n1, const double *x1,
                                 const double *y1, const double *z1,
                                 const double *w1, int64_t n2, const double *x2,
                                 const double *y2, const double *z2,
                                 const double *w2, int autocorr,
                                 const double *theta_edges_deg, int32_t nbins,
                                 uint64_t *counts, double *wsum, int wtype,
                                 int nthreads)
{
    if (nbins < 1)
        return ORACLE_EINVAL;
    double *c = (double *)malloc(sizeof(double) * (size_t)(nbins + 1));
    if (!c)
        return ORACLE_ENOMEM;
    int rc = oracle_theta_chord_edges(nbins + 1, theta_edges_deg, c);
    if (rc == ORACLE_OK)
        rc = count_pruned(0, axis, n1, x1, y1, z1, w1, n2, x2, y2, z2, w2, autocorr,
                          c, nbins, NULL, 0, 0.0, counts, wsum, wtype, 1, nthreads);
    free(c);
    return rc;
}
