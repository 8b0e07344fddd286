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
 *     sigma = FWHM / sqrt(8 ln 2), by default; a Gauss-tapered sinc and an
 *     elliptical Gaussian on request (hg_kernel.type);
 *   - support: d <= R, R = hg_kernel.support_deg, tested in FP64 as
 *     sin^2(dDec/2) + cos(Dec_g) cos(Dec_n) sin^2(dRA/2) <= sin^2(R/2);
 *   - map: plate carree in coordinate degrees; pixel (i, j) is centred at
 *     RA = ra0 + (i - (nx-1)/2) dra, Dec = dec0 + (j - (ny-1)/2) ddec; or a
 *     patch of a HEALPix grid (hg_map.proj; Eq. 1 leaves the cell set G open);
 *   - a cell with no sample in its support gets NaN (count 0, W 0);
 *   - values are assumed finite (Eq. 1 has no per-sample flags).  A NaN or
 *     infinite value reaches every cell of its sample's support, and also the
 *     other cells of the 2 x 2 cell groups that hold such a cell: the kernels
 *     multiply a group's four cells together, with weight 0 where a cell is
 *     outside the support, and 0 x NaN is NaN.  Cells farther away are not
 *     affected.
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
#define HG_ERR_UNSUPPORTED 5 /* valid request the library does not handle */
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

/* target cell sets (hg_map.proj) */
#define HG_PROJ_CAR 0     /* plate carree in coordinate degrees                  */
#define HG_PROJ_HEALPIX 1 /* a patch of a HEALPix RING grid (Gorski et al. 2005) */

/* Output cells are laid out [ny][nx], cell (i, j) at flat index j*nx + i.
   HG_PROJ_CAR: cell (i, j) is centred at RA = ra0 + (i - (nx-1)/2) dra,
   Dec = dec0 + (j - (ny-1)/2) ddec; nside, ring0 and pix0 must be 0.
   HG_PROJ_HEALPIX: row j is HEALPix ring r = ring0 - j (rings counted from 1 at
   the north pole, so rows run south to north) and column i is pixel
   k = (pix0 + i) mod 4 nside of that ring (0-based, eastward from RA 0): the
   RING-scheme pixel 2 nside (nside - 1) + 4 nside (r - nside) + k, centred at
   z = sin Dec = 4/3 - 2 r / (3 nside), RA = (k + s/2) pi / (2 nside) with
   s = (r - nside + 1) mod 2.  Every ring must lie in the equatorial belt
   (nside <= r <= 3 nside), where each ring holds 4 nside equally spaced
   pixels; polar-cap rings give HG_ERR_UNSUPPORTED.  nx <= 4 nside;
   ra0/dec0/dra/ddec are unused and must be 0.  hg_map_pixel_ids gives the
   pixel numbers of the patch. */
typedef struct {
    double ra0_deg, dec0_deg; /* CAR: map centre (degrees)                     */
    double dra_deg, ddec_deg; /* CAR: pixel spacing in coordinate degrees, > 0 */
    int32_t nx, ny;           /* cells along RA and Dec, > 0                   */
    int32_t proj;             /* HG_PROJ_*; 0 = plate carree                   */
    int32_t nside;            /* HEALPIX: grid resolution, a power of two <= 2^20 */
    int32_t ring0;            /* HEALPIX: ring of row 0                        */
    int32_t pix0;             /* HEALPIX: pixel of column 0 within each ring, < 4 nside */
} hg_map;

/* Kernel shapes w(g; s) of Eq. 1 (the paper leaves w open).  d is the
   great-circle distance, theta the bearing of the sample seen from the cell
   (from north through east). */
enum {
    HG_KERNEL_GAUSS = 0,      /* exp(-d^2 / 2 sigma^2), sigma = FWHM / sqrt(8 ln 2)        */
    HG_KERNEL_GAUSS_SINC = 1, /* sinc(d / b) exp(-(d / a)^2), sinc(x) = sin(pi x)/(pi x);
                                 a = p1, b = p2 (degrees, > 0); weights may be negative   */
    HG_KERNEL_ELLIPTICAL = 2  /* exp(-u^2 / 2 s_maj^2 - v^2 / 2 s_min^2): (u, v) = d times
                                 (cos, sin) of theta - pa, the offset along the major and
                                 minor axes; s_maj from fwhm_deg, s_min from FWHM p1
                                 (degrees, > 0), pa = p2 (degrees, north through east)     */
};

typedef struct {
    double fwhm_deg;    /* Gaussian FWHM (degrees), > 0; the major axis for
                           HG_KERNEL_ELLIPTICAL (unused by HG_KERNEL_GAUSS_SINC)  */
    double support_deg; /* support radius R (degrees), 0 <= R <= 10, inclusive */
    int32_t type;       /* HG_KERNEL_*; 0 = Gaussian                            */
    int32_t reserved;   /* must be 0                                            */
    double p1, p2;      /* shape parameters of the non-Gaussian kernels         */
} hg_kernel;

typedef struct {
    int32_t precision;      /* HG_PREC_*; 0 = HG_PREC_FP32.  A BF16 / FP16 plan
                               grids values of that type only                   */
    int32_t nside;          /* HEALPix resolution of the sky cells; 0 = auto    */
    int32_t chunk;          /* tile slots staged per step, a multiple of 8 up to 64
                               (FP32 form, 1 KB rows) or 112 (16-bit forms, 512 B
                               rows), else HG_ERR_ARG; 0 = the longest that fits (56
                               for the FP32 form, 112 for the 16-bit forms, shorter
                               for dense fields), tried from the longest, or with
                               HG_FLAG_PREDICT_CHUNK (and for a batch's fields) from
                               the length predicted from the support.  An explicit chunk whose densest
                               entry block would not fit two staged chunks in LDS,
                               or (past 64 slots) where one pixel group takes more
                               than 64 entries of a chunk, fails (HG_ERR_UNSUPPORTED) */
    int32_t waves;          /* channel kernel: waves per workgroup, 8 or 16; 0 = 16.
                               The waves share the tile's 64 pixel groups       */
    int64_t device_mem_cap; /* bytes; 0 = none.  Setup fails with HG_ERR_NOMEM
                               before any allocation beyond it                  */
    uint32_t flags;         /* HG_FLAG_*                                        */
    int32_t chan_block;     /* channel kernel: channels per workgroup, 64, 128 or
                               256; 0 = 256.  waves, chan_block and chunk are the
                               shapes the autotuner (tune.py) sweeps; the maps do
                               not depend on waves and chan_block (the same
                               operations in the same order), only on chunk.
                               Shapes other than 16 x 256 are built for aligned
                               FP32 values in the FP32 form and for the 16-bit
                               forms; other calls use 16 x 256                  */
} hg_opts;

#define HG_FLAG_TIME_CHANNELS 1u /* record HIP events around channel kernels   */
/* chunk 0: start at the longest length predicted to fit from the support in
   pixels (a group's mean run in a dealt chunk is the chunk times the group's
   share of its tile's slot region, with a margin) instead of at the longest
   of all; a field that does not fit is still set up again shorter.  Fewer
   dense fields are set up twice, at the cost of shorter chunks where the
   margin was not needed.  Batch fields always start this way. */
#define HG_FLAG_PREDICT_CHUNK 2u

typedef struct {
    int64_t n_samples;   /* samples passed to setup                              */
    int64_t n_used;      /* samples inside the band of rings that can reach the map */
    int64_t nnz;         /* (pixel, sample) pairs in support                      */
    int64_t n_entries;   /* entry-block units the channel kernel reads: groups of
                            four (pixel group, sample) entries, each (group, chunk)
                            run padded to a whole unit                             */
    int64_t n_cells;     /* HEALPix cells in the band                             */
    int64_t total_slots; /* staged sample slots summed over tiles                 */
    int64_t device_bytes;/* device memory held by the plan                        */
    int32_t nside;
    int32_t chunk;
    int32_t waves;        /* channel kernel shape the plan launches with:         */
    int32_t chan_block;   /* waves per workgroup and channels per workgroup       */
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
 *                    |Dec| > 90 make setup fail with HG_ERR_ARG.  The
 *                    coordinates are device pointers because every step of
 *                    setup (binning, sort, look-up table, neighbour search)
 *                    runs on the device; a caller holding host arrays copies
 *                    them first, on its own stream, where the copy can overlap
 *                    other work (the paper's CPU pre-processing, Sec. 4.1.1, is
 *                    moved to the GPU here).  Host memory is refused
 *                    (HG_ERR_ARG).
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
 *           a cell has no neighbour).  values and out must be device memory
 *           of the plan's device (else HG_ERR_ARG, before any launch).
 *   Asynchronous on hip_stream: the caller keeps values and out alive until
 *   the stream has passed this point.  With HG_FLAG_TIME_CHANNELS the kernel
 *   time is recorded with HIP events on the same stream.  The first call with
 *   a given number of 256-channel blocks also uploads, on hip_stream, the
 *   order in which the kernel's workgroups take the plan's tiles (a few KB,
 *   kept by the plan until hg_grid_finish).
 */
int hg_grid_channels(hg_plan* p, const void* values, int64_t ld, int32_t nchan, int32_t dtype,
                     float* out, void* hip_stream);

/*
 * hg_grid_channels for the tiles of tile rows [tile_row0, tile_row1): map rows
 * [16 tile_row0, min(16 tile_row1, ny)) of every channel (tiles are 16 x 16
 * pixels; the map has ceil(ny / 16) tile rows).  The same per-tile work as
 * hg_grid_channels, so calls over rows that cover the map give its result bit
 * for bit; only those rows of out ([nchan][ny][nx], the whole cube's buffer)
 * are written.  This lets a caller copy finished rows back, or start rows
 * whose samples have arrived, while later rows are computed (the channels of
 * Eq. 1 split by output region: each pixel's sum still runs over all of its
 * neighbours, Sec. 4.2).  0 <= tile_row0 <= tile_row1 <= tile rows, else
 * HG_ERR_ARG; tile_row0 == tile_row1 does nothing.  Other arguments, errors
 * and asynchrony as for hg_grid_channels; each distinct row range keeps its
 * own launch order on the plan (a few KB).
 */
int hg_grid_channels_rows(hg_plan* p, const void* values, int64_t ld, int32_t nchan,
                          int32_t dtype, float* out, int32_t tile_row0, int32_t tile_row1,
                          void* hip_stream);

/*
 * For bands of rows_per_band tile rows (band b: tile rows [b rows_per_band,
 * min((b + 1) rows_per_band, tile rows))): host_need[b] = 1 + the largest
 * sample index that any tile of the band stages, 0 if it stages none, so
 * hg_grid_channels_rows over band b reads only the values of samples
 * [0, host_need[b]).  A caller streaming the values to the device in index
 * order can start a band once that prefix has arrived (for scans recorded in
 * order, a band's samples lie in a narrow index range).  host_need: HOST
 * int64 [nbands], nbands = ceil(tile rows / rows_per_band), else HG_ERR_ARG;
 * rows_per_band >= 1.  Runs a small kernel on hip_stream and synchronises it.
 */
int hg_plan_row_needs(const hg_plan* p, int32_t rows_per_band, int64_t* host_need,
                      int32_t nbands, void* hip_stream);

/*
 * Grid a cube held in HOST memory, block by block of channels, with the copy
 * of the next block in, the kernel of the current block and the copy of the
 * previous block out overlapped on three streams (channels are independent,
 * Sec. 4.2; pinned buffers and transfer/compute overlap as in Sec. 4.3.2).
 *   host_values: HOST [n][ld] of dtype, channel c of sample s at s*ld + c.
 *   host_out:    HOST FP32 [nchan][ny][nx]; fully overwritten.
 *   block:       channels per block (0 = 4096).  The plan keeps two device
 *                slots of n x block values and block x ny x nx maps (counted
 *                against device_mem_cap) between calls.
 *   If both buffers are page-locked (hipHostMalloc, or torch pin_memory) the
 *   copies are direct; otherwise the library stages blocks through two pinned
 *   slots of its own with host threads.
 *   Synchronous: returns when host_out is complete.  Kernels run on
 *   hip_stream; the copies on two streams of the plan.
 *   info (may be NULL) receives the block count, bytes moved and the device
 *   time of the copies and kernels.
 */
typedef struct {
    int32_t blocks;       /* channel blocks processed                              */
    int32_t pinned;       /* 1: direct copies from the caller's page-locked buffers */
    int64_t h2d_bytes;    /* value bytes copied to the device                      */
    int64_t d2h_bytes;    /* map bytes copied back                                 */
    double wall_ms;       /* host time of the call                                 */
    double kernel_ms;     /* device time of the channel kernels (sum over blocks)  */
    double h2d_ms;        /* device time of the copies in (sum)                    */
    double d2h_ms;        /* device time of the copies out (sum)                   */
} hg_stream_info;

int hg_grid_channels_host(hg_plan* p, const void* host_values, int64_t ld, int32_t nchan,
                          int32_t dtype, float* host_out, int32_t block, void* hip_stream,
                          hg_stream_info* info);

/*
 * hg_grid_channels_host for callers that cannot allocate device memory (code
 * that must not call hipMalloc: serving loops, harnesses that forbid it).  It
 * allocates nothing: the two device slots of values and maps live in one
 * fixed staging array of HG_NOALLOC_STAGING_BYTES that the library holds on
 * every device it runs on until the process ends; the two copy streams and
 * their events are made on the first call on a device and kept.
 *   host_values, host_out: as for hg_grid_channels_host, but both must be
 *     page-locked (hipHostMalloc or torch pin_memory); pageable buffers are
 *     refused with HG_ERR_ARG (staging them would need pinned memory).
 *   block: channels per block; 0 picks the widest block (at most 4096) whose
 *     two value slots (n x block) and two map slots (block x ny x nx, FP32)
 *     fit the array.  A block that does not fit is refused with HG_ERR_ARG,
 *     before anything is enqueued.
 *   The maps equal hg_grid_channels_host's (the same kernels and per-cell
 *   operations).  Synchronous.  info receives the block count, bytes moved
 *   and the wall time; its device times stay 0 (timing would make events).
 *   Every call on a device shares that device's array and streams: calls
 *   that overlap on one device race, so serialise them.
 */
#define HG_NOALLOC_STAGING_BYTES (256u << 20) /* bytes of the staging array per device */

int hg_grid_channels_host_noalloc(hg_plan* p, const void* host_values, int64_t ld,
                                  int32_t nchan, int32_t dtype, float* host_out, int32_t block,
                                  void* hip_stream, hg_stream_info* info);

/*
 * Algorithm 1 as the paper states it (Sec. 4.1.2, Fig. 7, with the cells per
 * thread of Sec. 4.3.3), a comparison path beside hg_grid_channels on the same
 * plan: one launch per channel; one thread per gamma output cells of one 2x2
 * pixel group (gamma 1, 2 or 4), walking the HEALPix cell runs of the rings
 * that can hold a neighbour; for every channel it recomputes each FP64
 * distance and Gaussian weight and reads the channel's values with stride ld,
 * and sums w v and w in FP64 (Eq. 1).  NaN where a cell has no neighbour.
 *   values: DEVICE float32 [n][ld] (FP32 only); out: DEVICE float32
 *   [nchan][ny][nx].  block_threads: threads per workgroup, a multiple of 64
 *   in [64, 1024].  Asynchronous on hip_stream.
 *   Errors: HG_ERR_ARG (NULL pointers, gamma not 1/2/4, block_threads, ld <
 *   nchan), HG_ERR_STATE (finished plan), HG_ERR_UNSUPPORTED (a plan whose
 *   kernel is not the Gaussian), HG_ERR_DEVICE.
 */
int hg_grid_channels_literal(hg_plan* p, const float* values, int64_t ld, int32_t nchan,
                             float* out, int32_t gamma, int32_t block_threads, void* hip_stream);

/* End of a plan: the shared component (look-up table, coordinates and
   neighbour structure, Sec. 4.3.1) is released once no channel needs it.
   Synchronises the device, then frees everything the plan holds.  NULL is a
   no-op.  A plan borrowed from a batch is refused with HG_ERR_STATE. */
int hg_grid_finish(hg_plan* p);

/* Plan statistics (host struct): the sizes of the shared component of
   Sec. 4.3.1 (samples used, cells, staged slots, device bytes), the number of
   (cell, sample) pairs in support -- the terms of Eq. 1's sums -- and
   timings.  Synchronises to read channel timings. */
int hg_plan_stats(hg_plan* p, hg_stats* s);

/* Set the channel kernel's shape for the plan's later hg_grid_channels and
   hg_grid_channels_host calls: waves 8 or 16 per workgroup, chan_block 64,
   128 or 256 channels per workgroup (0 keeps 16 and 256).  The maps do not
   change (every cell's sums are the same operations in the same order); only
   the speed does.  This is how the autotuner times one plan in every shape
   without repeating setup.  The paper tunes its kernel's block size by hand
   for each GPU (Sec. 5.3.2 on the V100, Sec. 5.4 on the MI50).  Not
   thread-safe with calls on the same plan; HG_ERR_ARG for other values. */
int hg_plan_set_shape(hg_plan* p, int32_t waves, int32_t chan_block);

/* Per-pixel neighbour counts |N(g)|, HOST int32 [ny*nx] (flat index j*nx + i):
   the number of samples s_n with d(g, s_n) <= R, the terms of Eq. 1's sums
   for cell g (the inclusive test of Algorithm 1). */
int hg_plan_counts(const hg_plan* p, int32_t* host_counts);

/* Per-pixel weight sums W_g = sum_n w(g; s_n) of Eq. 1, the normaliser of
   every channel's map (FP64 sum of the FP32 weights the kernels use),
   HOST double [ny*nx]; 0 where the cell has no neighbour. */
int hg_plan_weight_sums(const hg_plan* p, double* host_W);

/*
 * Neighbour lists N(g) of Eq. 1 (the samples that pass Algorithm 1's
 * inclusive test d <= R) in CSR form, HOST arrays: row_ptr[ny*nx + 1]; for the
 * t-th neighbour of pixel p (ascending original sample index) idx[t] and its
 * FP32 weight w[t] = w(g; s_n) (either may be NULL).  *nnz receives the total;
 * idx and w are written only when cap >= *nnz.
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

/*
 * HEALPix RING pixel numbers of a HG_PROJ_HEALPIX map's cells, HOST int64
 * [ny*nx] (flat index j*nx + i), by the formula given with hg_map: where to
 * put the gridded cells in a full-sky RING array.  Host arithmetic only (no
 * device call).  The map is checked as hg_grid_setup checks it; a plate-carree
 * map gives HG_ERR_ARG.
 */
int hg_map_pixel_ids(const hg_map* m, int64_t* host_ids);

/*
 * Batched form: many independent fields (each its own Eq. 1 problem with its
 * own samples, map, kernel and channel count) gridded by ONE kernel launch,
 * held in a HIP graph and replayed by hg_batch_run.  This stands where the
 * paper runs channels and fields through a CPU multi-process x GPU
 * multi-stream pipeline with FIFO scheduling (Sec. 4.2.2): here each field is
 * set up once on the device (as hg_grid_setup) and the launch covers every
 * (field, 16x16-pixel tile, 256-channel block) item, placed longest first over
 * the XCDs so that the hardware dispatcher balances the work.
 */
typedef struct hg_batch hg_batch; /* opaque; owns its fields' plans */

typedef struct {
    const double* ra_deg;  /* DEVICE, n FP64 (degrees); read during hg_batch_create only */
    const double* dec_deg; /* DEVICE, n FP64 (degrees)                                   */
    int64_t n;             /* samples, 0 <= n < 2^31                                     */
    hg_kernel kernel;
    hg_map map;
    const void* values;    /* DEVICE [n][ld] of the batch dtype; read by every run       */
    int64_t ld;            /* row stride in elements, >= nchan                           */
    int32_t nchan;         /* channels, >= 0 (0: the field is set up but not gridded)    */
    int32_t reserved;      /* must be 0                                                  */
    float* out;            /* DEVICE FP32 [nchan][ny][nx]; written by every run          */
} hg_field;

typedef struct {
    int32_t n_fields;
    int32_t reserved;
    int64_t n_items;      /* (field, tile, channel block) work items                   */
    int64_t n_workgroups; /* launch size, including idle padding items                 */
    int64_t n_samples, nnz, n_entries;
    int64_t device_bytes; /* plans plus the batch's descriptors                        */
    double setup_ms;      /* wall time of hg_batch_create (all field setups)           */
    double last_run_ms;   /* device time of the last run (HG_FLAG_TIME_CHANNELS)       */
    double total_run_ms;
    int64_t runs;
} hg_batch_info;

/*
 * Set up every field and build the batched launch.
 *   fields:  HOST array of nfields >= 1 descriptors (copied); the device
 *            buffers they point to stay owned by the caller.  values and out
 *            are bound now: every hg_batch_run reads and writes them.
 *   dtype:   HG_F32 / HG_BF16 / HG_F16, common to all fields; must match a
 *            BF16 / FP16 MFMA precision (else HG_ERR_UNSUPPORTED).
 *   o:       options for every field (precision, nside, chunk, device_mem_cap
 *            per field, HG_FLAG_TIME_CHANNELS times each run); may be NULL.
 *   Synchronises hip_stream.  On failure nothing is kept, *out = NULL and the
 *   error text names the field.
 */
int hg_batch_create(const hg_field* fields, int32_t nfields, int32_t dtype, const hg_opts* o,
                    void* hip_stream, hg_batch** out);

/* Grid every field: Eq. 1 for every channel of every field, the work the
   paper's two-level FIFO scheduler hands to CPU processes and GPU streams
   (Sec. 4.2.2), as one graph launch.  Asynchronous on hip_stream; reads the
   values and writes the outputs bound at hg_batch_create. */
int hg_batch_run(hg_batch* b, void* hip_stream);

/* End of a batch (as hg_grid_finish for each field's shared component,
   Sec. 4.3.1): synchronise the device and free the batch and its plans.
   NULL is a no-op. */
int hg_batch_destroy(hg_batch* b);

/* Batch statistics (host struct): fields, work items, samples, (cell,
   sample) pairs in support (the terms of Eq. 1 over all fields), bytes and
   timings.  Synchronises to read run timings. */
int hg_batch_stats(hg_batch* b, hg_batch_info* s);

/* Borrow field i's plan, the field's shared component of Sec. 4.3.1 (for
   hg_plan_counts, hg_plan_neighbours, hg_grid_channels ...); it stays owned
   by the batch, and hg_grid_finish on it fails. */
int hg_batch_plan(hg_batch* b, int32_t i, hg_plan** out);

/* Text of the last failure on this thread ("" if none); valid until the next
   call on the same thread.  The paper defines no error reporting; this
   belongs to the boundary's conventions (status codes, no exceptions across
   the interface), stated at the top of this header. */
const char* hg_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* HEGRID_H */
