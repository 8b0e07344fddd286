/*
 * libhegrid -- convolution gridding of non-uniformly sampled multi-channel
 * single-dish data onto a regular sky map, on one AMD Instinct MI355X (gfx950).
 *
 * The operation is the gather form of Eq. (1) (Sec. 2.2): every map cell g
 * takes the normalised weighted sum of the samples s_n in its kernel support,
 *
 *     V[g] = (1 / W_g) sum_n V[s_n] w(g; s_n),     W_g = sum_n w(g; s_n),
 *
 * with the inclusive support test d <= R of the cell-update workflow
 * (Algorithm 1, Sec. 4.1.2).  Readings where the paper is open:
 *   - kernel: Gaussian of the great-circle distance d, w = exp(-d^2 / 2 sigma^2),
 *     sigma = FWHM / sqrt(8 ln 2);
 *   - support: d <= R, R = hg_kernel.support_deg, tested in FP64 as
 *     sin^2(dDec/2) + cos(Dec_g) cos(Dec_n) sin^2(dRA/2) <= sin^2(R/2);
 *   - map: plate carree in coordinate degrees; pixel (i, j) is centred at
 *     RA = ra0 + (i - (nx-1)/2) dra, Dec = dec0 + (j - (ny-1)/2) ddec;
 *   - a cell with no sample in its support gets NaN (count 0, W 0).
 *
 * The work is split the way the paper's shared-component design splits it
 * (Sec. 4.3.1): everything that depends only on the sample positions -- sky-cell
 * binning with HEALPix ang2pix in FP64 (Sec. 4.1.1 step 1), the sort and the
 * look-up table (steps 1, 2, 4), and the per-cell neighbour search with its
 * distances and weights (Algorithm 1) -- runs once in hg_grid_setup and stays
 * on the device in an hg_plan; hg_grid_channels then grids any number of
 * channels against that plan, since channels are independent (Sec. 4.2).
 *
 * Conventions: every call returns a status (HG_OK = 0); no C++ exception
 * crosses this interface; hg_last_error() describes the last failure on the
 * calling thread.  Arguments that can be checked on the host are checked
 * before anything is enqueued.  A plan is not thread-safe; distinct plans are
 * independent.  HIP is initialised on the first call that needs the device.
 */
#ifndef HEGRID_H
#define HEGRID_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define HG_OK 0
#define HG_ERR_ARG 1         /* invalid argument                          */
#define HG_ERR_STATE 2       /* call not valid for this plan's state      */
#define HG_ERR_NOMEM 3       /* device allocation failed or over the cap  */
#define HG_ERR_DEVICE 4      /* no usable device / HIP runtime error      */
#define HG_ERR_UNSUPPORTED 5 /* valid request this build does not handle  */
#define HG_ERR_INTERNAL 6    /* bug: an unexpected condition              */

/* value dtypes (hg_grid_channels) */
#define HG_F32 0  /* IEEE binary32 */
#define HG_BF16 1 /* bfloat16 bit patterns */
#define HG_F16 2  /* IEEE binary16 */

/* accumulation form (hg_opts.precision) */
#define HG_PREC_FP32 0      /* FP32 weights x FP32 values, FP32 accumulation     */
#define HG_PREC_MFMA_BF16 1 /* BF16 weights x BF16 values on MFMA, FP32 accumulation;
                               W is the sum of the same BF16-rounded weights        */
#define HG_PREC_MFMA_F16 2  /* as above with FP16 weights and values              */

typedef struct hg_plan hg_plan; /* opaque; owns all device memory it allocates */

typedef struct {
    double ra0_deg, dec0_deg; /* map centre (degrees)                          */
    double dra_deg, ddec_deg; /* pixel spacing in coordinate degrees, > 0      */
    int32_t nx, ny;           /* pixels along RA and Dec, > 0                  */
} hg_map;

typedef struct {
    double fwhm_deg;    /* Gaussian FWHM (degrees), > 0                          */
    double support_deg; /* support radius R (degrees), 0 <= R <= 10, inclusive */
} hg_kernel;

typedef struct {
    int32_t precision;      /* HG_PREC_*; 0 = HG_PREC_FP32.  A BF16 / FP16 plan
                               grids values of that type only                   */
    int32_t nside;          /* HEALPix resolution of the sky cells; 0 = auto    */
    int32_t chunk;          /* tile slots staged per step: 0 (= 32), 8, 16, 24, 32 */
    int32_t reserved;       /* must be 0                                        */
    int64_t device_mem_cap; /* bytes; 0 = none.  Setup fails with HG_ERR_NOMEM
                               before any allocation beyond it                  */
    uint32_t flags;         /* HG_FLAG_*                                        */
    uint32_t reserved2;     /* must be 0                                        */
} hg_opts;

#define HG_FLAG_TIME_CHANNELS 1u /* record HIP events around channel kernels   */

typedef struct {
    int64_t n_samples;   /* samples passed to setup                              */
    int64_t n_used;      /* samples inside the band of rings that can reach the map */
    int64_t nnz;         /* (pixel, sample) pairs in support                      */
    int64_t n_entries;   /* (pixel group, sample) entries the channel kernel reads */
    int64_t n_cells;     /* HEALPix cells in the band                             */
    int64_t total_slots; /* staged sample slots summed over tiles                 */
    int64_t device_bytes;/* device memory held by the plan                        */
    int32_t nside;
    int32_t chunk;
    double setup_ms;      /* wall time of hg_grid_setup                           */
    double last_channels_ms; /* device time of the last hg_grid_channels (timed plans) */
    double total_channels_ms;
    int64_t channels_calls;
} hg_stats;

/*
 * Build a plan: bin, sort, index and search the samples once (Sec. 4.1.1,
 * Algorithm 1, shared component of Sec. 4.3.1).
 *   ra_deg, dec_deg: DEVICE pointers, n FP64 values each (degrees).  Read only;
 *                    the caller keeps ownership.  Non-finite values or
 *                    |Dec| > 90 make setup fail with HG_ERR_ARG.
 *   n:               sample count, 0 <= n < 2^31.
 *   k, m:            kernel and map (host structs, copied).
 *   o:               options (may be NULL for defaults).
 *   hip_stream:      hipStream_t to run on (NULL = the null stream).  Setup
 *                    synchronises this stream before returning.
 *   out:             receives the new plan; *out = NULL on failure.
 */
int hg_grid_setup(const double* ra_deg, const double* dec_deg, int64_t n, const hg_kernel* k,
                  const hg_map* m, const hg_opts* o, void* hip_stream, hg_plan** out);

/*
 * Grid nchan channels against a plan (Eq. 1 for each channel).
 *   values: DEVICE pointer, row-major [n][ld] of dtype; channel c of sample s
 *           at values[s*ld + c]; nchan <= ld (nchan = 0 does nothing; values
 *           may be NULL when the plan has n = 0).  The caller keeps ownership.
 *   out:    DEVICE pointer, FP32 [nchan][ny][nx]; fully overwritten (NaN where
 *           a cell has no neighbour).
 *   Asynchronous on hip_stream: the caller keeps values and out alive until
 *   the stream has passed this point.  With HG_FLAG_TIME_CHANNELS the kernel
 *   time is recorded with HIP events on the same stream.
 */
int hg_grid_channels(hg_plan* p, const void* values, int64_t ld, int32_t nchan, int32_t dtype,
                     float* out, void* hip_stream);

/* Synchronise the device, free everything the plan holds.  NULL is a no-op. */
int hg_grid_finish(hg_plan* p);

/* Plan statistics (host struct).  Synchronises to read channel timings. */
int hg_plan_stats(hg_plan* p, hg_stats* s);

/* Per-pixel neighbour counts, HOST int32 [ny*nx] (flat index j*nx + i). */
int hg_plan_counts(const hg_plan* p, int32_t* host_counts);

/* Per-pixel weight sums W (FP64 sum of the FP32 weights the kernels use),
   HOST double [ny*nx]. */
int hg_plan_weight_sums(const hg_plan* p, double* host_W);

/*
 * Neighbour lists in CSR form, HOST arrays: row_ptr[ny*nx + 1]; for the t-th
 * neighbour of pixel p (ascending original sample index) idx[t] and its FP32
 * weight w[t] (either may be NULL).  *nnz receives the total; idx and w are
 * written only when cap >= *nnz.
 */
int hg_plan_neighbours(const hg_plan* p, int64_t* row_ptr, int64_t* idx, float* w, int64_t cap,
                       int64_t* nnz);

/*
 * HEALPix RING ang2pix in FP64 (the sky-cell binning of Sec. 4.1.1, step 1):
 * pix[i] = RING index at resolution nside (1 <= nside <= 2^14) of
 * (ra_deg[i], dec_deg[i]).  All pointers are DEVICE pointers; asynchronous on
 * hip_stream.
 */
int hg_ang2pix_ring(int32_t nside, const double* ra_deg, const double* dec_deg, int64_t n,
                    int64_t* pix, void* hip_stream);

/* Text of the last failure on this thread ("" if none); valid until the next
   call on the same thread. */
const char* hg_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* HEGRID_H */
