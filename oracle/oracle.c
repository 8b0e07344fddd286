/*
 * FP64 reference gridder -- TEST INFRASTRUCTURE ONLY.
 *
 * Only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark may load this file's library.  The product path (the HIP library
 * and its Python binding) never calls it and shares no code with it.
 *
 * What it computes is the gather form of convolution gridding, Eq. (1) of
 * Sec. 2.2: for every cell g of a regular grid,
 *
 *     V[g] = (1 / W_g) * sum_n V[s_n] w(g; s_n),     W_g = sum_n w(g; s_n),
 *
 * with a Gaussian kernel of the angular distance, and the inclusive support
 * test d <= R of the cell-update workflow (Algorithm 1, Sec. 4.1.2).  The
 * paper leaves the kernel, the distance, the grid convention and empty cells
 * open; the readings taken here are:
 *
 *   - w(d) = exp(-d^2 / (2 sigma^2)), sigma = FWHM / sqrt(8 ln 2) (not
 *     normalised: W cancels any constant factor); Eq. 1 leaves w open, and two
 *     other shapes are offered through the *_k entry points:
 *       1: Gauss-tapered sinc, w = sinc(d/b) exp(-(d/a)^2), sinc(x) =
 *          sin(pi x)/(pi x), sinc(0) = 1 (a, b in degrees);
 *       2: elliptical Gaussian, w = exp(-u^2/(2 s_maj^2) - v^2/(2 s_min^2)),
 *          u = d cos(theta - pa), v = d sin(theta - pa), theta the bearing of
 *          the sample from the cell (atan2 of its east and north components,
 *          from north through east), s = FWHM / sqrt(8 ln 2) for the major
 *          (fwhm) and minor (p1) axes, pa = p2 degrees;
 *   - d is the great-circle distance, evaluated through the haversine
 *     h = sin^2(dDec/2) + cos(Dec_p) cos(Dec_n) sin^2(dRA/2); the support test
 *     is h <= h_R with h_R = sin^2(R/2), which is d <= R because h grows with d
 *     on [0, pi]; then d = 2 asin(min(1, sqrt(h)));
 *   - grid: plate carree in coordinate degrees; pixel (i, j) has centre
 *     RA = ra0 + (i - (nx-1)/2) dra, Dec = dec0 + (j - (ny-1)/2) ddec,
 *     flat index p = j*nx + i, output layout [channel][j][i]; or (proj 1) a
 *     patch of a HEALPix RING grid in its equatorial belt (Eq. 1 leaves the
 *     cell set open): cell (i, j) is RING pixel number
 *     2 ns (ns - 1) + 4 ns (r - ns) + (pix0 + i) mod 4 ns of ring r = ring0 - j,
 *     centred where the HEALPix layout puts that pixel (or_healpix_centre);
 *   - a cell with no sample in its support gets V = NaN, count 0, W = 0;
 *   - sums run over the neighbours in ascending original sample index.
 *
 * Everything is plain single-threaded FP64.  The only acceleration is a
 * declination-sorted index: a sample farther than R in declination is farther
 * than R on the sphere, so each cell scans the samples whose declination lies
 * within R (+1e-9 rad) of its own and applies the exact test to each.  A
 * brute-force mode tests every pair instead; both modes run the same per-pair
 * arithmetic, so they must agree bit for bit.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_F64 0
#define OR_F32 1
#define OR_BF16 2
#define OR_F16 3

#define OR_OK 0
#define OR_ERR_ARG 1
#define OR_ERR_NOMEM 3

typedef struct {
    double ra0_deg, dec0_deg; /* map centre */
    double dra_deg, ddec_deg; /* pixel spacing in coordinate degrees */
    int32_t nx, ny;
    int32_t proj;              /* 0 plate carree, 1 HEALPix patch */
    int32_t nside, ring0, pix0; /* HEALPix patch: resolution, ring of row 0, pixel of column 0 */
} or_map;

static const double PI = 3.14159265358979323846;
static const double DEG = 3.14159265358979323846 / 180.0;

/* The RING number of cell (i, j) of a HEALPix patch: the ring-0-based
   numbering runs ring by ring from the north pole; the north cap's rings
   1 .. ns-1 hold 4, 8, ..., 4 (ns-1) pixels, 2 ns (ns - 1) in all, and each
   belt ring holds 4 ns. */
static int64_t or_healpix_cell(const or_map* m, int64_t i, int64_t j) {
    int64_t ns = m->nside, r = m->ring0 - j;
    return 2 * ns * (ns - 1) + 4 * ns * (r - ns) + (m->pix0 + i) % (4 * ns);
}

/* Centre of belt pixel pix at resolution ns (Gorski et al. 2005): its ring r
   and place k in the ring follow from the count above; the belt rings are
   equally spaced in z = sin Dec from 2/3 (ring ns) to -2/3 (ring 3 ns), and
   a ring's 4 ns pixels are equally spaced in RA from 0, or from half a pixel
   on the rings where r - ns is even. */
static void or_healpix_centre(int64_t ns, int64_t pix, double* ra, double* dec) {
    int64_t q = pix - 2 * ns * (ns - 1);
    int64_t r = ns + q / (4 * ns), k = q % (4 * ns);
    double half = ((r - ns) % 2 == 0) ? 0.5 : 0.0;
    *dec = asin((double)(4 * ns - 2 * r) / (double)(3 * ns));
    *ra = ((double)k + half) * (PI / (double)(2 * ns));
}

/* Exact widening of one stored value to FP64. */
static double or_decode(const void* base, int64_t off, int dtype) {
    switch (dtype) {
    case OR_F64:
        return ((const double*)base)[off];
    case OR_F32:
        return (double)((const float*)base)[off];
    case OR_BF16: {
        /* bfloat16 is the upper half of an IEEE binary32 */
        uint32_t bits = (uint32_t)((const uint16_t*)base)[off] << 16;
        float f;
        memcpy(&f, &bits, sizeof f);
        return (double)f;
    }
    case OR_F16: {
        /* IEEE binary16: 1 sign, 5 exponent (bias 15), 10 fraction bits */
        uint16_t h = ((const uint16_t*)base)[off];
        int sign = (h >> 15) & 1, e = (h >> 10) & 31, f = h & 1023;
        double v;
        if (e == 0)
            v = ldexp((double)f, -24); /* subnormal: f * 2^-14 * 2^-10 */
        else if (e == 31)
            v = f ? NAN : INFINITY;
        else
            v = ldexp((double)(1024 + f), e - 25);
        return sign ? -v : v;
    }
    }
    return NAN;
}

static void or_pixel_centre(const or_map* m, int64_t p, double* ra, double* dec) {
    int64_t i = p % m->nx, j = p / m->nx;
    if (m->proj == 1) {
        or_healpix_centre(m->nside, or_healpix_cell(m, i, j), ra, dec);
        return;
    }
    *ra = (m->ra0_deg + ((double)i - (m->nx - 1) / 2.0) * m->dra_deg) * DEG;
    *dec = (m->dec0_deg + ((double)j - (m->ny - 1) / 2.0) * m->ddec_deg) * DEG;
}

/* haversine of the angle between (a1, d1) and (a2, d2), radians */
static double or_haversine(double a1, double d1, double a2, double d2) {
    double sd = sin(0.5 * (d2 - d1));
    double sa = sin(0.5 * (a2 - a1));
    return sd * sd + cos(d1) * cos(d2) * sa * sa;
}

typedef struct {
    double dec;
    int64_t idx;
} or_key;

static int or_cmp_key(const void* x, const void* y) {
    const or_key* a = (const or_key*)x;
    const or_key* b = (const or_key*)y;
    if (a->dec < b->dec) return -1;
    if (a->dec > b->dec) return 1;
    return (a->idx > b->idx) - (a->idx < b->idx);
}

typedef struct {
    int64_t idx;
    double w;
} or_nb;

static int or_cmp_nb(const void* x, const void* y) {
    const or_nb* a = (const or_nb*)x;
    const or_nb* b = (const or_nb*)y;
    return (a->idx > b->idx) - (a->idx < b->idx);
}

typedef struct {
    int64_t n;
    const double* ra_deg;
    const double* dec_deg;
    double* ra; /* radians */
    double* dec;
    or_key* by_dec; /* NULL in brute-force mode */
    double sigma, h_r, r_rad;
    int ktype;                    /* 0 Gaussian, 1 Gauss-sinc, 2 elliptical */
    double ka, kb;                /* Gauss-sinc a and b, radians */
    double smaj, smin, pa;        /* elliptical sigmas and position angle, radians */
    double margin; /* min |h - h_R| / h_R over all pairs tested */
    or_nb* buf;    /* scratch for one cell's neighbours */
    int64_t buf_cap;
} or_ctx;

static void or_ctx_free(or_ctx* c) {
    free(c->ra);
    free(c->dec);
    free(c->by_dec);
    free(c->buf);
}

static int or_ctx_init(or_ctx* c, int64_t n, const double* ra_deg, const double* dec_deg,
                       double fwhm_deg, double support_deg, int brute, int32_t ktype, double p1,
                       double p2) {
    memset(c, 0, sizeof *c);
    if (n < 0 || (n > 0 && (!ra_deg || !dec_deg)) || !(support_deg >= 0) || ktype < 0 ||
        ktype > 2)
        return OR_ERR_ARG;
    if (ktype != 1 && !(fwhm_deg > 0)) return OR_ERR_ARG;
    if (ktype == 1 && !(p1 > 0 && p2 > 0)) return OR_ERR_ARG;
    if (ktype == 2 && !(p1 > 0)) return OR_ERR_ARG;
    c->ktype = ktype;
    c->ka = p1 * DEG;
    c->kb = p2 * DEG;
    c->smaj = fwhm_deg * DEG / sqrt(8.0 * log(2.0));
    c->smin = p1 * DEG / sqrt(8.0 * log(2.0));
    c->pa = p2 * DEG;
    c->n = n;
    c->ra = (double*)malloc(sizeof(double) * (size_t)(n ? n : 1));
    c->dec = (double*)malloc(sizeof(double) * (size_t)(n ? n : 1));
    c->buf_cap = 1024;
    c->buf = (or_nb*)malloc(sizeof(or_nb) * (size_t)c->buf_cap);
    if (!c->ra || !c->dec || !c->buf) return OR_ERR_NOMEM;
    for (int64_t k = 0; k < n; k++) {
        c->ra[k] = ra_deg[k] * DEG;
        c->dec[k] = dec_deg[k] * DEG;
    }
    c->sigma = fwhm_deg * DEG / sqrt(8.0 * log(2.0));
    c->r_rad = support_deg * DEG;
    double s = sin(0.5 * c->r_rad);
    c->h_r = s * s;
    c->margin = INFINITY;
    if (!brute) {
        c->by_dec = (or_key*)malloc(sizeof(or_key) * (size_t)(n ? n : 1));
        if (!c->by_dec) return OR_ERR_NOMEM;
        for (int64_t k = 0; k < n; k++) {
            c->by_dec[k].dec = c->dec[k];
            c->by_dec[k].idx = k;
        }
        qsort(c->by_dec, (size_t)n, sizeof(or_key), or_cmp_key);
    }
    return OR_OK;
}

/* the kernel's weight of a pair at distance d, cell (ra_p, dec_p), sample (ra_n, dec_n) */
static double or_weight(const or_ctx* c, double d, double ra_p, double dec_p, double ra_n,
                        double dec_n) {
    if (c->ktype == 1) {
        double x = PI * d / c->kb;
        double sinc = x == 0.0 ? 1.0 : sin(x) / x;
        return sinc * exp(-(d / c->ka) * (d / c->ka));
    }
    if (c->ktype == 2) {
        double east = cos(dec_n) * sin(ra_n - ra_p);
        double north = cos(dec_p) * sin(dec_n) - sin(dec_p) * cos(dec_n) * cos(ra_n - ra_p);
        double theta = atan2(east, north);
        double u = d * cos(theta - c->pa), v = d * sin(theta - c->pa);
        return exp(-(u * u) / (2.0 * c->smaj * c->smaj) - (v * v) / (2.0 * c->smin * c->smin));
    }
    return exp(-(d * d) / (2.0 * c->sigma * c->sigma));
}

/* one candidate pair: exact inclusive test; appends to the cell's list */
static int or_try(or_ctx* c, double ra_p, double dec_p, int64_t k, int64_t* cnt) {
    double h = or_haversine(ra_p, dec_p, c->ra[k], c->dec[k]);
    if (c->h_r > 0) {
        double mg = fabs(h - c->h_r) / c->h_r;
        if (mg < c->margin) c->margin = mg;
    }
    if (!(h <= c->h_r)) return OR_OK;
    double d = 2.0 * asin(fmin(1.0, sqrt(h)));
    if (*cnt == c->buf_cap) {
        int64_t cap = c->buf_cap * 2;
        or_nb* nb = (or_nb*)realloc(c->buf, sizeof(or_nb) * (size_t)cap);
        if (!nb) return OR_ERR_NOMEM;
        c->buf = nb;
        c->buf_cap = cap;
    }
    c->buf[*cnt].idx = k;
    c->buf[*cnt].w = or_weight(c, d, ra_p, dec_p, c->ra[k], c->dec[k]);
    (*cnt)++;
    return OR_OK;
}

/* neighbours of one cell, ascending original index, with their weights */
static int or_cell(or_ctx* c, double ra_p, double dec_p, int64_t* cnt) {
    *cnt = 0;
    if (!c->by_dec) {
        for (int64_t k = 0; k < c->n; k++) {
            int rc = or_try(c, ra_p, dec_p, k, cnt);
            if (rc) return rc;
        }
        return OR_OK; /* already in index order */
    }
    double lo = dec_p - c->r_rad - 1e-9, hi = dec_p + c->r_rad + 1e-9;
    int64_t a = 0, b = c->n; /* first key with dec >= lo */
    while (a < b) {
        int64_t mid = a + (b - a) / 2;
        if (c->by_dec[mid].dec < lo)
            a = mid + 1;
        else
            b = mid;
    }
    for (int64_t t = a; t < c->n && c->by_dec[t].dec <= hi; t++) {
        int rc = or_try(c, ra_p, dec_p, c->by_dec[t].idx, cnt);
        if (rc) return rc;
    }
    qsort(c->buf, (size_t)*cnt, sizeof(or_nb), or_cmp_nb);
    return OR_OK;
}

static int or_check_map(const or_map* m) {
    if (!m || m->nx <= 0 || m->ny <= 0) return 0;
    if (m->proj == 1) {
        int64_t ns = m->nside;
        return ns >= 1 && m->nx <= 4 * ns && m->pix0 >= 0 && m->pix0 < 4 * ns &&
               m->ring0 - (m->ny - 1) >= ns && m->ring0 <= 3 * ns;
    }
    return m->proj == 0 && m->dra_deg > 0 && m->ddec_deg > 0;
}

/* Centres (radians) of all nx*ny cells, flat index j*nx + i, and for a
   HEALPix patch their RING numbers (ids may be NULL). */
int oracle_cell_centres(const or_map* m, double* ra, double* dec, int64_t* ids) {
    if (!or_check_map(m) || !ra || !dec) return OR_ERR_ARG;
    int64_t ncell = (int64_t)m->nx * m->ny;
    for (int64_t p = 0; p < ncell; p++) {
        or_pixel_centre(m, p, &ra[p], &dec[p]);
        if (ids) ids[p] = m->proj == 1 ? or_healpix_cell(m, p % m->nx, p / m->nx) : -1;
    }
    return OR_OK;
}

/*
 * Grid the selected channels at the selected cells.
 *   values:   [n][ld] of dtype (OR_F64 / OR_F32 / OR_BF16 bits / OR_F16 bits)
 *   chans:    nchan channel indices (each < ld)
 *   pix:      npix flat cell indices p = j*nx + i, or NULL for all nx*ny cells
 *   out:      [nchan][npix] FP64, NaN where the cell has no neighbour
 *   count, W: [npix]; margin: closest call min |h - h_R| / h_R (may be NULL)
 */
int oracle_grid_k(int64_t n, const double* ra_deg, const double* dec_deg, const void* values,
                  int32_t dtype, int64_t ld, const int64_t* chans, int64_t nchan, const or_map* m,
                  double fwhm_deg, double support_deg, int32_t ktype, double p1, double p2,
                  int32_t brute, const int64_t* pix, int64_t npix, double* out, int32_t* count,
                  double* W, double* margin) {
    if (!or_check_map(m) || nchan < 0 || (nchan > 0 && (!values || !chans || !out)) ||
        dtype < OR_F64 || dtype > OR_F16)
        return OR_ERR_ARG;
    int64_t ncell = (int64_t)m->nx * m->ny;
    if (!pix) npix = ncell;
    for (int64_t k = 0; k < nchan; k++)
        if (chans[k] < 0 || chans[k] >= ld) return OR_ERR_ARG;
    or_ctx c;
    int rc = or_ctx_init(&c, n, ra_deg, dec_deg, fwhm_deg, support_deg, brute, ktype, p1, p2);
    if (rc) {
        or_ctx_free(&c);
        return rc;
    }
    for (int64_t q = 0; q < npix; q++) {
        int64_t p = pix ? pix[q] : q;
        if (p < 0 || p >= ncell) {
            or_ctx_free(&c);
            return OR_ERR_ARG;
        }
        double ra_p, dec_p;
        or_pixel_centre(m, p, &ra_p, &dec_p);
        int64_t cnt;
        rc = or_cell(&c, ra_p, dec_p, &cnt);
        if (rc) {
            or_ctx_free(&c);
            return rc;
        }
        double wsum = 0.0;
        for (int64_t t = 0; t < cnt; t++) wsum += c.buf[t].w;
        if (count) count[q] = (int32_t)cnt;
        if (W) W[q] = wsum;
        for (int64_t k = 0; k < nchan; k++) {
            double s = 0.0;
            for (int64_t t = 0; t < cnt; t++)
                s += c.buf[t].w * or_decode(values, c.buf[t].idx * ld + chans[k], dtype);
            out[k * npix + q] = cnt ? s / wsum : NAN;
        }
    }
    if (margin) *margin = c.margin;
    or_ctx_free(&c);
    return OR_OK;
}

/* oracle_grid_k with the Gaussian kernel */
int oracle_grid(int64_t n, const double* ra_deg, const double* dec_deg, const void* values,
                int32_t dtype, int64_t ld, const int64_t* chans, int64_t nchan, const or_map* m,
                double fwhm_deg, double support_deg, int32_t brute, const int64_t* pix,
                int64_t npix, double* out, int32_t* count, double* W, double* margin) {
    return oracle_grid_k(n, ra_deg, dec_deg, values, dtype, ld, chans, nchan, m, fwhm_deg,
                         support_deg, 0, 0.0, 0.0, brute, pix, npix, out, count, W, margin);
}

/*
 * Neighbour lists (CSR) of the selected cells: row_ptr[npix+1], and for the
 * t-th neighbour of row q its original index idx[t] and weight w[t].  Rows are
 * in ascending original index.  Returns the total count through *nnz; idx and
 * w are written only while they fit in cap (pass cap = 0 to size them).
 */
int oracle_neighbours_k(int64_t n, const double* ra_deg, const double* dec_deg,
                        const or_map* m, double fwhm_deg, double support_deg, int32_t ktype,
                        double p1, double p2, int32_t brute, const int64_t* pix, int64_t npix,
                        int64_t* row_ptr, int64_t* idx, double* w, int64_t cap, int64_t* nnz) {
    if (!or_check_map(m) || !row_ptr || !nnz) return OR_ERR_ARG;
    int64_t ncell = (int64_t)m->nx * m->ny;
    if (!pix) npix = ncell;
    or_ctx c;
    int rc = or_ctx_init(&c, n, ra_deg, dec_deg, fwhm_deg, support_deg, brute, ktype, p1, p2);
    if (rc) {
        or_ctx_free(&c);
        return rc;
    }
    int64_t total = 0;
    row_ptr[0] = 0;
    for (int64_t q = 0; q < npix; q++) {
        int64_t p = pix ? pix[q] : q;
        if (p < 0 || p >= ncell) {
            or_ctx_free(&c);
            return OR_ERR_ARG;
        }
        double ra_p, dec_p;
        or_pixel_centre(m, p, &ra_p, &dec_p);
        int64_t cnt;
        rc = or_cell(&c, ra_p, dec_p, &cnt);
        if (rc) {
            or_ctx_free(&c);
            return rc;
        }
        for (int64_t t = 0; t < cnt; t++, total++) {
            if (total < cap) {
                if (idx) idx[total] = c.buf[t].idx;
                if (w) w[total] = c.buf[t].w;
            }
        }
        row_ptr[q + 1] = total;
    }
    *nnz = total;
    or_ctx_free(&c);
    return OR_OK;
}

/* oracle_neighbours_k with the Gaussian kernel */
int oracle_neighbours(int64_t n, const double* ra_deg, const double* dec_deg, const or_map* m,
                      double fwhm_deg, double support_deg, int32_t brute, const int64_t* pix,
                      int64_t npix, int64_t* row_ptr, int64_t* idx, double* w, int64_t cap,
                      int64_t* nnz) {
    return oracle_neighbours_k(n, ra_deg, dec_deg, m, fwhm_deg, support_deg, 0, 0.0, 0.0, brute,
                               pix, npix, row_ptr, idx, w, cap, nnz);
}
