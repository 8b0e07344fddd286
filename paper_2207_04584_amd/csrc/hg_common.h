// Internal declarations of libhegrid: HEALPix RING geometry, the plan's device
// layout and the kernel launchers.  Not part of the public C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <map>
#include <tuple>
#include <string>
#include <utility>
#include <vector>

#include "hegrid.h"

namespace hg {

constexpr double kPi = 3.14159265358979323846;
constexpr double kDeg = 3.14159265358979323846 / 180.0;
// LDS a workgroup can hold on gfx950 (160 KB per compute unit)
constexpr int LDS_BYTES = 160 * 1024;

// Pixel groups (PG): 2 x 2 map pixels that share one neighbour walk and one
// entry list; slot r = 2*(j&1) + (i&1).  Tiles: TILE_PGX x TILE_PGY groups
// (16 x 16 pixels) that share one staged sample list in the channel kernels.
constexpr int PG = 2;
constexpr int TILE_PGX = 8;
constexpr int TILE_PGY = 8;
constexpr int TILE_PGS = TILE_PGX * TILE_PGY;
constexpr uint32_t SLOT_MASK = 0x0FFFFFFFu;  // low 28 bits: tile-local slot
constexpr int SLOT_SHIFT = 28;               // high 4 bits: in-support mask
constexpr int PGOFF_STRIDE = 68;             // uint16 per block: 65 offsets, padded to 136 B
constexpr int MAX_CHUNK = 112;               // tile slots per staged chunk, upper bound

// ---------------------------------------------------------------------------
// HEALPix RING scheme (Gorski et al. 2005; the partition used by the paper's
// look-up table, Sec. 4.1.1).  Rings i = 1 .. 4N-1 from the north pole; ring
// i holds n_i pixels numbered from `first`, centred at z_i, azimuths
// (k + shift/2) 2 pi / n_i for k = 0 .. n_i - 1.
struct Ring {
    int64_t first;
    int64_t n;
    double z;
    int shift;
};

__host__ __device__ inline Ring hp_ring(int64_t N, int64_t i) {
    Ring r;
    if (i < N) {
        r.first = 2 * i * (i - 1);
        r.n = 4 * i;
        r.z = 1.0 - (double)(i * i) / (3.0 * (double)N * (double)N);
        r.shift = 1;
    } else if (i <= 3 * N) {
        r.first = 2 * N * (N - 1) + (i - N) * 4 * N;
        r.n = 4 * N;
        r.z = 4.0 / 3.0 - 2.0 * (double)i / (3.0 * (double)N);
        r.shift = (int)((i - N + 1) & 1);
    } else {
        int64_t k = 4 * N - i;
        r.first = 12 * N * N - 2 * k * (k + 1);
        r.n = 4 * k;
        r.z = -(1.0 - (double)(k * k) / (3.0 * (double)N * (double)N));
        r.shift = 1;
    }
    return r;
}

// Continuous ring coordinate of latitude z: ring centres sit at integers, and a
// pixel of ring i covers latitudes strictly between rings i-1 and i+1.
__host__ __device__ inline double hp_ring_coord(int64_t N, double z) {
    if (z > 2.0 / 3.0) return (double)N * sqrt(3.0 * (1.0 - z));
    if (z < -2.0 / 3.0) return 4.0 * (double)N - (double)N * sqrt(3.0 * (1.0 + z));
    return (double)N * (2.0 - 1.5 * z);
}

__host__ __device__ inline int64_t floor_div2(int64_t a) { return (a >= 0) ? a / 2 : -((1 - a) / 2); }

__host__ __device__ inline int64_t mod_pos(int64_t a, int64_t m) {
    int64_t r = a % m;
    return r < 0 ? r + m : r;
}

// RING index of the pixel containing (z = sin Dec, phi = RA in radians).
// In the equatorial belt (|z| <= 2/3) pixel edges are the lines
// N (phi/(pi/2) + 1/2) -+ (3/4) N z = integer; in the polar caps they are the
// curves t N sqrt(3 (1-|z|)) = integer and (1-t) N sqrt(3 (1-|z|)) = integer,
// t the azimuth fraction within a base pixel.
__host__ __device__ inline int64_t hp_ang2pix(int64_t N, double z, double phi) {
    double twopi = 2.0 * kPi;
    phi = fmod(phi, twopi);
    if (phi < 0.0) phi += twopi;
    double tt = phi / (0.5 * kPi);
    if (tt >= 4.0) tt = 0.0;
    double za = fabs(z);
    if (za <= 2.0 / 3.0) {
        double t1 = (double)N * (0.5 + tt);
        double t2 = (double)N * z * 0.75;
        int64_t jp = (int64_t)floor(t1 - t2);
        int64_t jm = (int64_t)floor(t1 + t2);
        int64_t ir = N + 1 + jp - jm;
        int64_t kshift = 1 - (ir & 1);
        int64_t ip = mod_pos(floor_div2(jp + jm - N + kshift + 1), 4 * N);
        return 2 * N * (N - 1) + (ir - 1) * 4 * N + ip;
    }
    double tp = tt - floor(tt);
    double tmp = (double)N * sqrt(3.0 * (1.0 - za));
    int64_t jp = (int64_t)floor(tp * tmp);
    int64_t jm = (int64_t)floor((1.0 - tp) * tmp);
    int64_t ir = jp + jm + 1;
    int64_t ip = mod_pos((int64_t)floor(tt * (double)ir), 4 * ir);
    return (z > 0.0) ? 2 * ir * (ir - 1) + ip : 12 * N * N - 2 * ir * (ir + 1) + ip;
}

// Pixels of ring r whose azimuth extent (centre -+ pi/n) meets [pa, pb]
// (radians, unwrapped), widened by one pixel each side.  Written as at most two
// pieces of wrapped indices, in ascending order.  Returns the piece count.
__host__ __device__ inline int hp_ring_pieces(const Ring& r, double pa, double pb, int64_t* a0,
                                              int64_t* b0, int64_t* a1, int64_t* b1) {
    double scale = (double)r.n / (2.0 * kPi);
    double off = 0.5 * (double)r.shift;
    int64_t ka = (int64_t)ceil(pa * scale - off - 0.5) - 1;
    int64_t kb = (int64_t)floor(pb * scale - off + 0.5) + 1;
    if (kb - ka + 1 >= r.n) {
        *a0 = 0;
        *b0 = r.n - 1;
        return 1;
    }
    int64_t wa = mod_pos(ka, r.n), wb = mod_pos(kb, r.n);
    if (wa <= wb) {
        *a0 = wa;
        *b0 = wb;
        return 1;
    }
    *a0 = 0;
    *b0 = wb;
    *a1 = wa;
    *b1 = r.n - 1;
    return 2;
}

// Shape of the channel kernel's workgroup: `waves` waves (8 or 16) share one
// tile's 64 pixel groups, and the workgroup grids 64 g channels (g = 1, 2 or
// 4).  The plan's entry blocks do not depend on it, so it is chosen per
// launch; {16, 4} is the default.
struct Shape {
    int32_t waves = 16, g = 4;
};

// ---------------------------------------------------------------------------
// Plan: everything grid_setup leaves on the device for grid_channels.
struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
};
// page-locked host memory from the process-wide pool (runtime.hip)
struct HostBuf {
    void* p = nullptr;
    size_t bytes = 0;
};

// The order in which the channel kernel's workgroups take a plan's (tile,
// channel block) items, for one channel-block count: item b of the launch is
// tile * ncb + cb, or -1 for an idle workgroup (see launch_order).
struct LaunchOrder {
    DevBuf items;               // int64 [n] on the device
    HostBuf host;               // the same in page-locked memory, the upload's source
    hipEvent_t ready = nullptr; // recorded after the upload
    int64_t n = 0;
};

// Rings for host-streamed channel blocks (hg_grid_channels_host): two device
// slots of values and maps, two pinned host slots for callers whose buffers
// are pageable, and the two copy streams.  Kept by the plan across calls.
constexpr int RING_SLOTS = 2;
struct HostRing {
    DevBuf vals[RING_SLOTS], out[RING_SLOTS];
    void* pin_in[RING_SLOTS] = {nullptr, nullptr};
    void* pin_out[RING_SLOTS] = {nullptr, nullptr};
    size_t pin_in_bytes = 0, pin_out_bytes = 0;
    hipStream_t h2d = nullptr, d2h = nullptr;
    hipEvent_t ev_h2d[RING_SLOTS] = {nullptr, nullptr};
    hipEvent_t ev_ker[RING_SLOTS] = {nullptr, nullptr};
    hipEvent_t ev_d2h[RING_SLOTS] = {nullptr, nullptr};
};

struct Plan {
    int device = 0;
    // geometry and kernel constants (row a1)
    hg_map map{};
    hg_kernel kern{};
    hg_opts opts{};
    double sigma = 0, r_rad = 0, h_r = 0;
    int64_t n = 0, n_used = 0;
    int64_t nside = 0;
    int64_t ring_lo = 0, ring_hi = 0;  // band of rings that can hold a neighbour
    int64_t cell_base = 0, n_cells = 0;
    int32_t npgx = 0, npgy = 0, ntx = 0, nty = 0;
    int64_t npg = 0, ntiles = 0, npix = 0;
    int32_t tile_rings = 0, pg_rings = 0;  // max rings per tile / per pixel group
    int32_t chunk = 32;                    // tile slots per staged chunk
    Shape shape;                           // channel kernel shape (hg_opts or default)
    int64_t total_slots = 0, ent_cap = 0, nnz_entries = 0, chunk_ptrs = 0;
    int64_t nnz = 0;  // (pixel, sample) pairs in support
    double setup_ms = 0;
    // device arrays
    DevBuf srt_idx;      // uint32 [n_used]   original index, sorted by (cell, index)
    DevBuf srt_coord;    // double4 [n_used]  (ra, dec, cos dec, -) radians
    DevBuf cell_off;     // uint32 [n_cells+1]
    DevBuf tile_piece;   // int4 [ntiles][tile_rings*2] (pos_a, len, slot0, cell_a)
    DevBuf tile_nslots;  // int64 [ntiles+1] exclusive scan of slots per tile
    DevBuf pg_piece;     // int4 [npg][pg_rings*2]   (pos_a, len, slot0, -)
    DevBuf pg_base;      // int64 [npg+1] entry capacity scan
    DevBuf pg_cnt;       // uint32 [npg] entries used
    DevBuf slot_idx;     // uint32 [total_slots] original index of each tile slot
    DevBuf ent_slot;     // uint32 [ent_cap] slot | mask << 28
    DevBuf ent_w;        // float4 [ent_cap]
    DevBuf cp_base;      // int64 [ntiles+1] chunk-pointer base per tile
    DevBuf chunk_ptr;    // uint32 [chunk_ptrs] entry offset (relative to pg_base)
    // chunk-major entry blocks: block b = (tile t, chunk c), b = tile_blk[t] + c
    int64_t n_blocks = 0;
    int32_t blk_max = 0;  // most units (entries, or groups of four) in one block
    int32_t run_max = 0;  // longest (group, chunk) run of entries if over 64, else 0
    DevBuf tile_blk;     // int64 [ntiles+1] first block of each tile
    std::vector<int64_t> tile_blk_host;       // the same, on the host (launch order costs)
    // launch orders by (channel-block count, first tile row, end tile row)
    std::map<std::tuple<int32_t, int32_t, int32_t>, LaunchOrder> orders;
    DevBuf blk_base;     // int64 [n_blocks+1] first entry of each block
    DevBuf blk_pgoff;    // uint16 [n_blocks][PGOFF_STRIDE] per-group offsets in the block
    DevBuf e2_w;         // float [units][4 pixels][4 entries] weights, block order
    DevBuf e2_s;         // uint4 [units] chunk-local slots of a unit's four entries
    // precision forms: entries in groups of four per pixel group (the MFMA K)
    DevBuf e3_w;         // uint16 [groups][4 pixels][4 entries] BF16 / FP16 weights
    DevBuf e3_s;         // uint4  [groups] chunk-local slots of the four entries
    DevBuf pix_count;    // int32 [npix]
    DevBuf pix_W;        // double [npix]
    DevBuf pix_Wf;       // float [npix] W rounded to FP32 (0 where count = 0)
    DevBuf scratch;      // small device scratch (flags, totals)
    // channel-kernel timing: event pairs recorded around launches, resolved
    // lazily (hg_plan_stats) so that timed calls stay asynchronous
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_pending, ev_free;
    int64_t ch_calls = 0, ch_timed_calls = 0;
    double ch_ms_total = 0, ch_ms_last = 0;
    bool finished = false;
    HostRing ring;
};

// Everything the channel kernel needs to grid one field: the plan's device
// arrays plus the call's values and output (device pointers).
struct FieldDesc {
    const void* values;
    int64_t ld;
    const int64_t* tile_base;
    const uint32_t* slot_idx;
    const int64_t* tile_blk;
    const int64_t* blk_base;
    const uint16_t* blk_pgoff;
    const void* ent_w;
    const void* ent_s;
    const float* pix_Wf;
    const uint32_t* pg_cnt;  // entries per pixel group (the balanced wave assignment)
    float* out;
    int32_t nchan, ncb, npgx, npgy, ntx, nx, ny, chunk, out_vec;
    int32_t ucap;     // LDS capacity in units per staged block (>= the plan's blk_max)
    int32_t nbuf;     // staged chunks resident in LDS (2..4)
    int32_t balance;  // 1: pixel groups dealt to waves by entry count
};

// One work item of the batched launch: (field, tile, channel block); field < 0
// marks a padding item that does nothing.
struct BatchItem {
    int32_t field, cb;
    int64_t tile;
};

struct BatchKernelInfo {
    const void* main;  // k_channels_batch(fields, items): one workgroup per item
    size_t shm;        // dynamic LDS bytes
    int threads;        // threads per workgroup of the main kernel
    int channels_per_block;
};

// Cell centres in radians.  Plate carree: (i, j) at ra0 + (i - (nx-1)/2) dra,
// dec0 + (j - (ny-1)/2) ddec.  HEALPix patch (equatorial belt): row j is ring
// r = ring0 - j at z = 4/3 - 2r/(3 nside); column i is pixel pix0 + i of the
// ring, at RA (pix0 + i + s/2) pi / (2 nside) with s = (r - nside + 1) mod 2,
// left unwrapped past 2 pi (every use of an RA is periodic or wraps it).
__host__ __device__ inline double pix_dec(const hg_map& m, int64_t j) {
    if (m.proj == HG_PROJ_HEALPIX)
        return asin(4.0 / 3.0 - 2.0 * (double)(m.ring0 - j) / (3.0 * (double)m.nside));
    return (m.dec0_deg + ((double)j - (m.ny - 1) / 2.0) * m.ddec_deg) * kDeg;
}
__host__ __device__ inline double pix_ra(const hg_map& m, int64_t i, int64_t j) {
    if (m.proj == HG_PROJ_HEALPIX) {
        const int64_t s = (m.ring0 - j - m.nside + 1) & 1;
        return ((double)(m.pix0 + i) + 0.5 * (double)s) * (kPi / (2.0 * (double)m.nside));
    }
    return (m.ra0_deg + ((double)i - (m.nx - 1) / 2.0) * m.dra_deg) * kDeg;
}
// least and greatest centre RA of column i over all rows (the planner's bounds;
// HEALPix rings alternate by half a pixel)
__host__ __device__ inline double col_ra_lo(const hg_map& m, int64_t i) {
    if (m.proj == HG_PROJ_HEALPIX)
        return (double)(m.pix0 + i) * (kPi / (2.0 * (double)m.nside));
    return pix_ra(m, i, 0);
}
__host__ __device__ inline double col_ra_hi(const hg_map& m, int64_t i) {
    if (m.proj == HG_PROJ_HEALPIX)
        return ((double)(m.pix0 + i) + 0.5) * (kPi / (2.0 * (double)m.nside));
    return pix_ra(m, i, 0);
}

// The launch order of a plan's channel kernel for ncb channel blocks, built
// and uploaded on stream s at its first use (runtime.hip).
// The (tile, channel block) items of tile rows [row0, row1) (row1 < 0: every
// row) in launch order: XCD-aware, cached per plan.
hipError_t launch_order(Plan& P, int32_t ncb, hipStream_t s, const int64_t** items, int64_t* n,
                        int32_t row0 = 0, int32_t row1 = -1);
// per tile: 1 + the largest sample index it stages (0 for an empty tile), on s
hipError_t launch_tile_max_index(const Plan& P, int64_t* tile_need, hipStream_t s);

// kernel launchers (setup.hip, channels.hip, literal.hip)
hipError_t launch_setup(Plan& P, const double* ra_deg, const double* dec_deg, hipStream_t s,
                        std::string& err, int& status);
// the channel phase over tile rows [row0, row1) (row1 < 0: the whole map)
hipError_t launch_channels(Plan& P, const void* values, int64_t ld, int32_t nchan, int32_t dtype,
                           float* out, hipStream_t s, Shape shape, int32_t row0 = 0,
                           int32_t row1 = -1);
// the same launch on a caller-provided item order of nwg positions (device)
hipError_t launch_channels_on(Plan& P, const void* values, int64_t ld, int32_t nchan,
                              int32_t dtype, float* out, hipStream_t s, Shape shape,
                              const int64_t* order, int64_t nwg);
// the same launch with workgroup b on item b (no order buffer)
hipError_t launch_channels_plain_order(Plan& P, const void* values, int64_t ld, int32_t nchan,
                                      int32_t dtype, float* out, hipStream_t s, Shape shape);
hipError_t launch_literal(const Plan& P, const float* values, int64_t ld, int32_t nchan,
                          float* out, int32_t gamma, int32_t block, hipStream_t s);
FieldDesc field_desc(const Plan& P, const void* values, int64_t ld, int32_t nchan, float* out,
                     Shape shape);
bool values_vec(const Plan& P, const void* values, int64_t ld, int32_t dtype);
// the shape a launch really uses: shapes other than the default exist only for
// aligned FP32 values in the FP32 form and for the 16-bit forms
Shape effective_shape(bool m16, int32_t dtype, bool vec, Shape s);
BatchKernelInfo batch_kernel(bool m16, int32_t dtype, bool vec, size_t shm, Shape shape);
size_t field_lds_bytes(const FieldDesc& d, bool m16, Shape shape);
bool channel_lds_fits(bool m16, int chunk, int blk_max);
// the channel kernel holds a run's slots one a lane: runs of at most 64 entries
inline bool channel_runs_fit(int chunk, int run_max) { return chunk <= 64 || run_max <= 64; }
hipError_t launch_ang2pix(int64_t nside, const double* ra_deg, const double* dec_deg, int64_t n,
                          int64_t* pix, hipStream_t s);

void plan_band(Plan& P, double eps);

// host-streamed channel blocks (stream.hip)
int grid_channels_host(Plan& P, const void* host_values, int64_t ld, int32_t nchan, int32_t dtype,
                       float* host_out, int32_t block, hipStream_t s, hg_stream_info* info,
                       std::string& err);
void ring_free(HostRing& R);
// the same through the fixed per-device staging array (no allocation)
int grid_channels_host_noalloc(Plan& P, const void* host_values, int64_t ld, int32_t nchan,
                               int32_t dtype, float* host_out, int32_t block, hipStream_t s,
                               hg_stream_info* info, std::string& err);

// device memory (runtime.hip)
hipError_t dev_alloc(DevBuf& b, size_t bytes);
void dev_free(DevBuf& b);
hipError_t host_alloc(HostBuf& b, size_t bytes);
void host_free(HostBuf& b);

}  // namespace hg
