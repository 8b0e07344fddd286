// Setup path of libhegrid: everything that depends only on the sample
// positions, run once per field (the shared component of Sec. 4.3.1).
//
//   1. sky-cell binning: HEALPix RING ang2pix in FP64      (Sec. 4.1.1, step 1)
//   2. counting sort by (cell, original index)             (steps 1 and 2)
//   3. look-up table: CSR offsets per cell of the band     (step 4)
//   4. tile / pixel-group planner: per ring, the cell range (hence the sample
//      range) that can reach the group                     (Algorithm 1,
//      ring_min..ring_max and pixel_min..pixel_max)
//   5. neighbour gather: exact FP64 support test d <= R and Gaussian weight for
//      every (pixel, candidate) pair                       (Algorithm 1, Eq. 1)
//
// This file is compiled with -ffp-contract=off so that the FP64 support test
// and weight evaluate in the same operation order as a plain C evaluation of
// the same formulas.
#include "hg_common.h"

namespace hg {
namespace {

constexpr uint32_t BAD_KEY = 0xFFFFFFFFu;

// ---------------------------------------------------------------------------
// exclusive scan (reduce -> scan of block sums -> final), out has n + 1 items
constexpr int SCAN_T = 256, SCAN_I = 16, SCAN_B = SCAN_T * SCAN_I;

template <typename T>
__device__ T block_exclusive_scan(T v, T* sh, T& total) {
    int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    T x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        T y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) sh[wid] = x;
    __syncthreads();
    if (threadIdx.x == 0) {
        T acc = 0;
        for (int w = 0; w < SCAN_T / 64; w++) {
            T t = sh[w];
            sh[w] = acc;
            acc += t;
        }
        sh[SCAN_T / 64] = acc;
    }
    __syncthreads();
    T res = x - v + sh[wid];
    total = sh[SCAN_T / 64];
    __syncthreads();
    return res;
}

template <typename Tin, typename Tout>
__global__ __launch_bounds__(SCAN_T) void k_scan_reduce(const Tin* in, int64_t n, Tout* bsum) {
    __shared__ Tout sh[SCAN_T / 64 + 1];
    int64_t base = (int64_t)blockIdx.x * SCAN_B;
    Tout s = 0;
    for (int k = 0; k < SCAN_I; k++) {
        int64_t i = base + (int64_t)k * SCAN_T + threadIdx.x;
        if (i < n) s += (Tout)in[i];
    }
    Tout tot;
    block_exclusive_scan<Tout>(s, sh, tot);
    if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

template <typename Tout>
__global__ __launch_bounds__(SCAN_T) void k_scan_bsums(Tout* bsum, int64_t nb) {
    __shared__ Tout sh[SCAN_T / 64 + 1];
    Tout carry = 0;
    for (int64_t b0 = 0; b0 < nb; b0 += SCAN_T) {
        int64_t i = b0 + threadIdx.x;
        Tout v = i < nb ? bsum[i] : (Tout)0;
        Tout tot;
        Tout ex = block_exclusive_scan<Tout>(v, sh, tot);
        if (i < nb) bsum[i] = ex + carry;
        carry += tot;
    }
}

// out2 (may be NULL): a second copy of out[0 .. n)
template <typename Tin, typename Tout>
__global__ __launch_bounds__(SCAN_T) void k_scan_final(const Tin* in, int64_t n, const Tout* bsum,
                                                       Tout* out, Tout* out2) {
    __shared__ Tout vals[SCAN_B];
    __shared__ Tout sh[SCAN_T / 64 + 1];
    int64_t base = (int64_t)blockIdx.x * SCAN_B;
    for (int k = 0; k < SCAN_I; k++) {
        int64_t i = base + (int64_t)k * SCAN_T + threadIdx.x;
        vals[k * SCAN_T + threadIdx.x] = i < n ? (Tout)in[i] : (Tout)0;
    }
    __syncthreads();
    Tout s = 0;
    for (int k = 0; k < SCAN_I; k++) s += vals[threadIdx.x * SCAN_I + k];
    Tout tot;
    Tout run = block_exclusive_scan<Tout>(s, sh, tot) + bsum[blockIdx.x];
    for (int k = 0; k < SCAN_I; k++) {
        Tout v = vals[threadIdx.x * SCAN_I + k];
        vals[threadIdx.x * SCAN_I + k] = run;
        run += v;
    }
    __syncthreads();
    for (int k = 0; k < SCAN_I; k++) {
        int64_t i = base + (int64_t)k * SCAN_T + threadIdx.x;
        if (i < n) {
            out[i] = vals[k * SCAN_T + threadIdx.x];
            if (out2) out2[i] = vals[k * SCAN_T + threadIdx.x];
        }
    }
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == SCAN_T - 1) out[n] = run;
}

// Short arrays in one workgroup: tiles of SCAN_B scanned in turn with a
// running carry (three launches of a few microseconds each otherwise; past
// two tiles the three launches are quicker than the serial tiles).
constexpr int64_t SCAN_ONE_MAX = 2 * SCAN_B;

template <typename Tin, typename Tout>
__device__ inline void scan_one(const Tin* in, int64_t n, Tout* out, Tout* out2) {
    __shared__ Tout vals[SCAN_B];
    __shared__ Tout sh[SCAN_T / 64 + 1];
    Tout carry = 0;
    for (int64_t base = 0; base < n || base == 0; base += SCAN_B) {
        for (int k = 0; k < SCAN_I; k++) {
            int64_t i = base + (int64_t)k * SCAN_T + threadIdx.x;
            vals[k * SCAN_T + threadIdx.x] = i < n ? (Tout)in[i] : (Tout)0;
        }
        __syncthreads();
        Tout sum = 0;
        for (int k = 0; k < SCAN_I; k++) sum += vals[threadIdx.x * SCAN_I + k];
        Tout tot;
        Tout run = block_exclusive_scan<Tout>(sum, sh, tot) + carry;
        for (int k = 0; k < SCAN_I; k++) {
            Tout v = vals[threadIdx.x * SCAN_I + k];
            vals[threadIdx.x * SCAN_I + k] = run;
            run += v;
        }
        __syncthreads();
        for (int k = 0; k < SCAN_I; k++) {
            int64_t i = base + (int64_t)k * SCAN_T + threadIdx.x;
            if (i < n) {
                out[i] = vals[k * SCAN_T + threadIdx.x];
                if (out2) out2[i] = vals[k * SCAN_T + threadIdx.x];
            }
        }
        carry += tot;
        __syncthreads();  // vals is refilled by the next tile
    }
    if (threadIdx.x == 0) out[n] = carry;
}

template <typename Tin, typename Tout>
__global__ __launch_bounds__(SCAN_T) void k_scan_one(const Tin* in, int64_t n, Tout* out,
                                                     Tout* out2) {
    scan_one<Tin, Tout>(in, n, out, out2);
}

// Up to SCAN_MANY short int64 arrays of one length, one workgroup each, in one
// launch (the planner's per-tile counts are scanned three at a time).
constexpr int SCAN_MANY = 3;
struct ScanJobs {
    const int64_t* in[SCAN_MANY];
    int64_t* out[SCAN_MANY];
};
__global__ __launch_bounds__(SCAN_T) void k_scan_many(ScanJobs j, int64_t n) {
    scan_one<int64_t, int64_t>(j.in[blockIdx.x], n, j.out[blockIdx.x], nullptr);
}

// scratch must hold ceil(n / SCAN_B) Tout
// out2 (may be NULL): a second copy of the n exclusive sums (not the total)
template <typename Tin, typename Tout>
hipError_t scan_exclusive(const Tin* in, int64_t n, Tout* out, Tout* scratch, hipStream_t s,
                          Tout* out2 = nullptr) {
    if (n <= SCAN_ONE_MAX) {
        hipLaunchKernelGGL((k_scan_one<Tin, Tout>), dim3(1), dim3(SCAN_T), 0, s, in, n, out, out2);
        return hipGetLastError();
    }
    int64_t nb = (n + SCAN_B - 1) / SCAN_B;
    if (nb < 1) nb = 1;
    hipLaunchKernelGGL((k_scan_reduce<Tin, Tout>), dim3((unsigned)nb), dim3(SCAN_T), 0, s, in, n,
                       scratch);
    hipLaunchKernelGGL((k_scan_bsums<Tout>), dim3(1), dim3(SCAN_T), 0, s, scratch, nb);
    hipLaunchKernelGGL((k_scan_final<Tin, Tout>), dim3((unsigned)nb), dim3(SCAN_T), 0, s, in, n,
                       scratch, out, out2);
    return hipGetLastError();
}

// scan_exclusive of k <= SCAN_MANY int64 arrays of length n: one launch when
// they are short, else one scan after another (sharing the scratch)
hipError_t scan_exclusive_many(const int64_t* const* in, int64_t* const* out, int k, int64_t n,
                               int64_t* scratch, hipStream_t s) {
    if (n <= SCAN_ONE_MAX) {
        ScanJobs j{};
        for (int i = 0; i < k; i++) {
            j.in[i] = in[i];
            j.out[i] = out[i];
        }
        hipLaunchKernelGGL(k_scan_many, dim3((unsigned)k), dim3(SCAN_T), 0, s, j, n);
        return hipGetLastError();
    }
    for (int i = 0; i < k; i++) {
        hipError_t e = scan_exclusive<int64_t, int64_t>(in[i], n, out[i], scratch, s);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// ---------------------------------------------------------------------------

struct RowInfo {
    int32_t ring_lo, nrings;
    double dalpha;  // RA half-width (radians) that can hold a neighbour; > pi = any
};

// 1. binning ------------------------------------------------------------------
// counter[k] += 1 for every lane with valid set: lanes in runs of equal keys
// over consecutive lanes (a scan's consecutive samples share cells) take one
// atomic per run, all runs in the same vector instruction, so a wave costs
// one atomic round trip whatever its keys.  Returns each valid lane the
// counter's old value plus its offset in its run: distinct values, as
// separate atomics would give, in another order.
__device__ inline uint32_t wave_atomic_inc(uint32_t* counter, uint32_t k, bool valid) {
    const int lane = threadIdx.x & 63;
    const uint32_t kprev = (uint32_t)__shfl_up((int)k, 1, 64);
    const uint64_t vmask = __ballot(valid);
    const bool prev_valid = lane > 0 && ((vmask >> (lane - 1)) & 1ull);
    const bool start = valid && (!prev_valid || kprev != k);
    const uint64_t starts = __ballot(start);
    // a run ends before the next start or the next invalid lane
    const uint64_t stops = starts | ~vmask;
    uint32_t base = 0;
    if (start) {
        const uint64_t after = lane == 63 ? 0ull : stops & ~((2ull << lane) - 1ull);
        const int next = after ? __ffsll((long long)after) - 1 : 64;
        base = atomicAdd(&counter[k], (uint32_t)(next - lane));
    }
    // the run's first lane: the highest start at or below this lane
    const uint64_t upto = lane == 63 ? starts : starts & ((2ull << lane) - 1ull);
    const int first = upto ? 63 - __clzll((long long)upto) : lane;
    const uint32_t b0 = (uint32_t)__shfl((int)base, first, 64);
    return valid ? b0 + (uint32_t)(lane - first) : 0u;
}

__global__ void k_bin(const double* __restrict__ ra_deg, const double* __restrict__ dec_deg,
                      int64_t n, int64_t nside, int64_t cell_base, int64_t n_cells,
                      uint32_t* __restrict__ key, uint32_t* __restrict__ cnt, int* flag) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    bool valid = false;
    uint32_t c32 = 0;
    if (i < n) {
        const double a = ra_deg[i], d = dec_deg[i];
        if (!isfinite(a) || !isfinite(d) || fabs(d) > 90.0) {
            atomicOr(flag, 1);
            key[i] = BAD_KEY;
        } else {
            const int64_t c = hp_ang2pix(nside, sin(d * kDeg), a * kDeg) - cell_base;
            if (c < 0 || c >= n_cells) {
                key[i] = BAD_KEY;
            } else {
                key[i] = c32 = (uint32_t)c;
                valid = true;
            }
        }
    }
    (void)wave_atomic_inc(cnt, c32, valid);
}

__global__ void k_ang2pix(const double* __restrict__ ra_deg, const double* __restrict__ dec_deg,
                          int64_t n, int64_t nside, int64_t* __restrict__ pix) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double a = ra_deg[i], d = dec_deg[i];
    pix[i] = hp_ang2pix(nside, sin(d * kDeg), a * kDeg);
}

// 2. sort ------------------------------------------------------------------------
__global__ void k_scatter(const uint32_t* __restrict__ key, int64_t n, uint32_t* __restrict__ cursor,
                          uint32_t* __restrict__ srt_idx) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t c = i < n ? key[i] : BAD_KEY;
    const bool valid = c != BAD_KEY;
    const uint32_t pos = wave_atomic_inc(cursor, valid ? c : 0u, valid);
    if (valid) srt_idx[pos] = (uint32_t)i;
}

__device__ inline void sift_down(uint32_t* v, uint32_t root, uint32_t end) {
    while (2 * root + 1 < end) {
        uint32_t child = 2 * root + 1;
        if (child + 1 < end && v[child] < v[child + 1]) child++;
        if (v[root] < v[child]) {
            uint32_t t = v[root];
            v[root] = v[child];
            v[child] = t;
            root = child;
        } else {
            return;
        }
    }
}

// The atomic scatter leaves each cell's samples in arbitrary order; ordering
// them by original index makes the key (cell, index) total and the layout
// deterministic.  Single samples are copied; a cell of 2 .. RANK_CELL
// samples is placed by rank, one wave per cell: the sample at position p of
// cell c goes to off[c] + #{q in c : idx[q] < idx[p]} (sample indices are
// distinct, so the ranks are a permutation of the cell), the cell held in
// the wave's registers and each sample broadcast in turn.  Larger cells are
// copied as they are and sorted by a workgroup each.
constexpr int RANK_PER_LANE = 8;
constexpr uint32_t RANK_CELL = 64 * RANK_PER_LANE;
constexpr int RANK_WAVES = 4096;  // persistent waves over the cell list
constexpr int BIG_SORT_T = 256;
constexpr uint32_t BIG_SORT_MAX = 4096;

// one thread per cell: copy single samples, list the others (one atomic a wave)
__global__ __launch_bounds__(256) void k_cell_list(const uint32_t* __restrict__ off,
                                                   int64_t n_cells, const uint32_t* __restrict__ idx,
                                                   uint32_t* __restrict__ idx2,
                                                   uint32_t* __restrict__ list,
                                                   uint32_t* __restrict__ list_count) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t len = 0, a = 0;
    if (c < n_cells) {
        a = off[c];
        len = off[c + 1] - a;
    }
    if (len == 1) idx2[a] = idx[a];
    const bool many = len > 1;
    const uint64_t m = __ballot(many);
    if (!m) return;  // uniform
    const int lane = threadIdx.x & 63;
    const int leader = __ffsll((long long)m) - 1;
    uint32_t base = 0;
    if (lane == leader) base = atomicAdd(list_count, (uint32_t)__popcll(m));
    base = (uint32_t)__shfl((int)base, leader, 64);
    if (many) list[base + (uint32_t)__popcll(m & ((1ull << lane) - 1ull))] = (uint32_t)c;
}

// rank placement of one cell of m samples, 64 (NK - 1) < m <= 64 NK
template <int NK>
__device__ inline void rank_cell(const uint32_t* __restrict__ idx, uint32_t* __restrict__ idx2,
                                 uint32_t a, uint32_t m, int lane) {
    uint32_t v[NK], r[NK];
#pragma unroll
    for (int k = 0; k < NK; k++) {
        const uint32_t q = (uint32_t)(k * 64 + lane);
        v[k] = q < m ? idx[a + q] : 0xFFFFFFFFu;
        r[k] = 0;
    }
#pragma unroll
    for (int k2 = 0; k2 < NK; k2++) {
        const int lanes = k2 < NK - 1 ? 64 : (int)(m - (uint32_t)(64 * (NK - 1)));
        for (int l2 = 0; l2 < lanes; l2++) {
            const uint32_t x = (uint32_t)__builtin_amdgcn_readlane((int)v[k2], l2);
#pragma unroll
            for (int k = 0; k < NK; k++) r[k] += x < v[k] ? 1u : 0u;
        }
    }
#pragma unroll
    for (int k = 0; k < NK; k++) {
        const uint32_t q = (uint32_t)(k * 64 + lane);
        if (q < m) idx2[a + r[k]] = v[k];
    }
}

__global__ __launch_bounds__(256) void k_cell_rank(
    const uint32_t* __restrict__ off, const uint32_t* __restrict__ idx,
    uint32_t* __restrict__ idx2, const uint32_t* __restrict__ list,
    const uint32_t* __restrict__ list_count, uint32_t* __restrict__ big,
    uint32_t* __restrict__ big_count) {
    const int lane = threadIdx.x & 63;
    const uint32_t nlist = *list_count;
    for (uint32_t w = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); w < nlist;
         w += gridDim.x * (blockDim.x >> 6)) {
        // w is the wave's: every value below is uniform over it
        const uint32_t c = (uint32_t)__builtin_amdgcn_readfirstlane((int)list[w]);
        const uint32_t a = (uint32_t)__builtin_amdgcn_readfirstlane((int)off[c]);
        const uint32_t m = (uint32_t)__builtin_amdgcn_readfirstlane((int)off[c + 1]) - a;
        switch ((m + 63) / 64) {
            case 1: rank_cell<1>(idx, idx2, a, m, lane); break;
            case 2: rank_cell<2>(idx, idx2, a, m, lane); break;
            case 3: rank_cell<3>(idx, idx2, a, m, lane); break;
            case 4: rank_cell<4>(idx, idx2, a, m, lane); break;
            case 5: rank_cell<5>(idx, idx2, a, m, lane); break;
            case 6: rank_cell<6>(idx, idx2, a, m, lane); break;
            case 7: rank_cell<7>(idx, idx2, a, m, lane); break;
            case 8: rank_cell<8>(idx, idx2, a, m, lane); break;
            default:
                for (uint32_t q = lane; q < m; q += 64) idx2[a + q] = idx[a + q];
                if (lane == 0) big[atomicAdd(big_count, 1u)] = c;
        }
    }
}
static_assert(RANK_CELL == 8 * 64, "k_cell_rank's cases cover cells up to RANK_CELL samples");

// One workgroup per listed cell: bitonic sort in LDS (padded to a power of
// two with UINT32_MAX); cells beyond BIG_SORT_MAX fall back to a heap sort.
__global__ __launch_bounds__(BIG_SORT_T) void k_cell_sort_big(
    const uint32_t* __restrict__ off, uint32_t* __restrict__ idx,
    const uint32_t* __restrict__ worklist, const uint32_t* __restrict__ wl_count) {
    __shared__ uint32_t sv[BIG_SORT_MAX];
    uint32_t nwork = *wl_count;
    for (uint32_t w = blockIdx.x; w < nwork; w += gridDim.x) {
        uint32_t c = worklist[w];
        uint32_t a = off[c], len = off[c + 1] - a;
        uint32_t* v = idx + a;
        if (len > BIG_SORT_MAX) {
            if (threadIdx.x == 0) {
                for (uint32_t st = len / 2; st-- > 0;) sift_down(v, st, len);
                for (uint32_t end = len - 1; end > 0; end--) {
                    uint32_t t = v[0];
                    v[0] = v[end];
                    v[end] = t;
                    sift_down(v, 0, end);
                }
            }
            __syncthreads();
            continue;
        }
        uint32_t P = 1;
        while (P < len) P <<= 1;
        for (uint32_t i = threadIdx.x; i < P; i += BIG_SORT_T) sv[i] = i < len ? v[i] : 0xFFFFFFFFu;
        __syncthreads();
        for (uint32_t k = 2; k <= P; k <<= 1) {
            for (uint32_t j = k >> 1; j > 0; j >>= 1) {
                for (uint32_t i = threadIdx.x; i < P; i += BIG_SORT_T) {
                    uint32_t pj = i ^ j;
                    if (pj > i) {
                        uint32_t x = sv[i], y = sv[pj];
                        bool up = (i & k) == 0;
                        if ((x > y) == up) {
                            sv[i] = y;
                            sv[pj] = x;
                        }
                    }
                }
                __syncthreads();
            }
        }
        for (uint32_t i = threadIdx.x; i < len; i += BIG_SORT_T) v[i] = sv[i];
        __syncthreads();
    }
}

// 4. planner --------------------------------------------------------------------
// Tile pieces: for ring k of the tile's band, up to two runs of cells (wrapped
// indices, ascending) -> (first sorted position, length, first slot, packed
// cell range a | b << 16).  Slots number the tile's candidates ring by ring.
__global__ void k_tile_plan(const RowInfo* __restrict__ rows, int32_t ntx, int64_t ntiles,
                            int32_t tile_rings, int64_t nside, int64_t cell_base, int64_t n_cells,
                            const uint32_t* __restrict__ cell_off, hg_map m, double eps,
                            int4* __restrict__ tile_piece, int* flag) {
    int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t tile = gid / tile_rings;
    int rk = (int)(gid % tile_rings);
    if (tile >= ntiles) return;
    int tx = (int)(tile % ntx), ty = (int)(tile / ntx);
    RowInfo ri = rows[ty];
    int4* out = tile_piece + (tile * tile_rings + rk) * 2;
    out[0] = make_int4(0, 0, 0, 0);
    out[1] = make_int4(0, 0, 0, 0);
    if (rk >= ri.nrings) return;
    Ring r = hp_ring(nside, ri.ring_lo + rk);
    int64_t i0 = (int64_t)tx * TILE_PGX * PG;
    int64_t i1 = i0 + TILE_PGX * PG - 1;
    if (i1 > m.nx - 1) i1 = m.nx - 1;
    double a0 = col_ra_lo(m, i0) - ri.dalpha - eps, a1 = col_ra_hi(m, i1) + ri.dalpha + eps;
    int64_t pa[2], pb[2];
    int np = hp_ring_pieces(r, a0, a1, &pa[0], &pb[0], &pa[1], &pb[1]);
    for (int q = 0; q < np; q++) {
        int64_t ka = r.first + pa[q] - cell_base, kb = r.first + pb[q] - cell_base;
        if (ka < 0 || kb >= n_cells) {
            atomicOr(flag, 4);
            continue;
        }
        uint32_t p0 = cell_off[ka], p1 = cell_off[kb + 1];
        out[q] = make_int4((int)p0, (int)(p1 - p0), 0, (int)(pa[q] | (pb[q] << 16)));
    }
}

__global__ void k_tile_prefix(int4* __restrict__ tile_piece, int64_t ntiles, int32_t tile_rings,
                              int32_t chunk, int64_t* __restrict__ tile_nslots,
                              int64_t* __restrict__ tile_ncp, int64_t* __restrict__ tile_nch,
                              int* flag, int* __restrict__ nch_max) {
    int64_t tile = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (tile >= ntiles) return;
    int4* tp = tile_piece + tile * tile_rings * 2;
    int64_t s = 0;
    for (int k = 0; k < 2 * tile_rings; k++) {
        int4 p = tp[k];
        p.z = (int)s;
        tp[k] = p;
        s += p.y;
    }
    if (s > (int64_t)SLOT_MASK) atomicOr(flag, 2);
    tile_nslots[tile] = s;
    const int64_t nch = (s + chunk - 1) / chunk;
    tile_ncp[tile] = (int64_t)TILE_PGS * (nch + 1);
    tile_nch[tile] = nch;
    // *nch_max (from 0) only grows, so a value read is never above the
    // current maximum and the read spares the atomics of smaller counts
    const int c = (int)(nch < INT32_MAX ? nch : INT32_MAX);
    if (c > *(volatile int*)nch_max) atomicMax(nch_max, c);
}

// Pixel-group pieces: the group's own ring / cell ranges, intersected with its
// tile's pieces, as (first sorted position, length, first tile slot).
__global__ void k_pg_plan(const RowInfo* __restrict__ pg_rows, const RowInfo* __restrict__ tile_rows,
                          int32_t npgx, int64_t npg, int32_t ntx, int32_t pg_rings,
                          int32_t tile_rings, int64_t nside, int64_t cell_base,
                          const uint32_t* __restrict__ cell_off, hg_map m, double eps,
                          const int4* __restrict__ tile_piece, int4* __restrict__ pg_piece,
                          int* flag) {
    int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t pg = gid / pg_rings;
    int rk = (int)(gid % pg_rings);
    if (pg >= npg) return;
    int gx = (int)(pg % npgx), gy = (int)(pg / npgx);
    int tx = gx / TILE_PGX, ty = gy / TILE_PGY;
    int64_t tile = (int64_t)ty * ntx + tx;
    RowInfo pr = pg_rows[gy];
    int4* out = pg_piece + (pg * pg_rings + rk) * 2;
    out[0] = make_int4(0, 0, 0, 0);
    out[1] = make_int4(0, 0, 0, 0);
    if (rk >= pr.nrings) return;
    int64_t ring = pr.ring_lo + rk;
    Ring r = hp_ring(nside, ring);
    int64_t i0 = (int64_t)gx * PG, i1 = i0 + PG - 1;
    if (i1 > m.nx - 1) i1 = m.nx - 1;
    double a0 = col_ra_lo(m, i0) - pr.dalpha - eps, a1 = col_ra_hi(m, i1) + pr.dalpha + eps;
    int64_t pa[2], pb[2];
    int np = hp_ring_pieces(r, a0, a1, &pa[0], &pb[0], &pa[1], &pb[1]);
    RowInfo tr = tile_rows[ty];
    int64_t tk = ring - tr.ring_lo;
    if (tk < 0 || tk >= tr.nrings) {
        atomicOr(flag, 8);
        return;
    }
    const int4* tp = tile_piece + (tile * tile_rings + tk) * 2;
    int nout = 0;
    for (int qt = 0; qt < 2; qt++) {
        int4 t = tp[qt];
        if (t.y == 0) continue;
        int64_t A = t.w & 0xFFFF, B = (t.w >> 16) & 0xFFFF;
        for (int qp = 0; qp < np; qp++) {
            int64_t lo = pa[qp] > A ? pa[qp] : A, hi = pb[qp] < B ? pb[qp] : B;
            if (lo > hi) continue;
            uint32_t p0 = cell_off[r.first + lo - cell_base];
            uint32_t p1 = cell_off[r.first + hi + 1 - cell_base];
            if (p1 == p0) continue;
            if (nout == 2) {
                atomicOr(flag, 16);
                continue;
            }
            out[nout++] = make_int4((int)p0, (int)(p1 - p0), t.z + (int)(p0 - (uint32_t)t.x), 0);
        }
    }
}

// A group's entries are numbered below 2^PERM_INDEX_BITS (the bucket
// permutation packs the number with the entry's position in its chunk).
constexpr int PERM_POS_BITS = 7;
constexpr uint32_t PERM_POS_MASK = (1u << PERM_POS_BITS) - 1u;
constexpr int PERM_INDEX_BITS = 32 - PERM_POS_BITS;
static_assert(MAX_CHUNK <= (1 << PERM_POS_BITS), "a chunk position fits the permutation's low bits");

__global__ void k_pg_capacity(const int4* __restrict__ pg_piece, int64_t npg, int32_t pg_rings,
                              int64_t* __restrict__ cap, int* __restrict__ flag) {
    int64_t pg = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (pg >= npg) return;
    const int4* p = pg_piece + pg * pg_rings * 2;
    int64_t s = 0;
    for (int k = 0; k < 2 * pg_rings; k++) s += p[k].y;
    cap[pg] = s;
    if (s >= ((int64_t)1 << PERM_INDEX_BITS)) atomicOr(flag, 32);
}

__global__ __launch_bounds__(256) void k_slot_fill(const int4* __restrict__ tile_piece,
                                                   int32_t tile_rings,
                                                   const int64_t* __restrict__ tile_base,
                                                   const uint32_t* __restrict__ srt_idx,
                                                   uint32_t* __restrict__ slot_idx) {
    // workgroup (tile, y) of gridDim.y copies every gridDim.y-th run of 256
    // of each piece: a map of few tiles with many slots each still fills
    // the device
    int64_t tile = blockIdx.x;
    const int4* tp = tile_piece + tile * tile_rings * 2;
    uint32_t* dst = slot_idx + tile_base[tile];
    const int step = blockDim.x * gridDim.y;
    for (int k = 0; k < 2 * tile_rings; k++) {
        int4 p = tp[k];
        for (int t = blockIdx.y * blockDim.x + threadIdx.x; t < p.y; t += step)
            dst[p.z + t] = srt_idx[p.x + t];
    }
}

// 5. neighbour gather -------------------------------------------------------------
// Weights are stored in FP32; the precision forms round them to the MFMA input
// type first (round to nearest even), so that W is the sum of exactly the
// weights the kernels multiply by.
__device__ inline float round_weight(float w, int32_t prec) {
    if (prec == HG_PREC_MFMA_BF16) {
        uint32_t u = __float_as_uint(w);
        u += 0x7FFFu + ((u >> 16) & 1u);  // finite weights (either sign)
        return __uint_as_float(u & 0xFFFF0000u);
    }
    if (prec == HG_PREC_MFMA_F16) return (float)(_Float16)w;
    return w;
}

// Squared angular distance d^2 = (2 asin(sqrt h))^2 from the haversine h.  For
// h < 1e-4 (d < 1.15 deg) the Maclaurin series of asin^2(x) in x^2 = h,
// h (1 + h/3 + 8 h^2/45 + 4 h^3/35 + ...), cut after the h^3 term, is exact to
// FP64 rounding (the next term is below 1e-17 relative); larger h takes asin.
// SMALL: the caller knows h < 1e-4 (supports below 1.15 deg), so the asin
// branch, which costs registers in every inlined copy, is left out.
template <bool SMALL>
__device__ inline double dist2(double h) {
    if (SMALL || h < 1e-4)
        return 4.0 * h * (1.0 + h * (1.0 / 3.0 + h * (8.0 / 45.0 + h * (4.0 / 35.0))));
    double d = 2.0 * asin(fmin(1.0, sqrt(h)));
    return d * d;
}

// sin x for the half-angle differences of the haversine.  Below 2^-7 rad the
// Maclaurin polynomial x - x^3/3! + x^5/5! - x^7/7! is within an ulp of sin x
// (the first dropped term, x^9/9!, is below 4e-23 |x|), at a few FMAs instead
// of a full range-reduced sin; larger arguments (wide supports, the RA wrap,
// fields near a pole) call sin.
__device__ inline double sin_poly(double x) {
    const double x2 = x * x;
    double p = fma(x2, -1.0 / 5040.0, 1.0 / 120.0);
    p = fma(p, x2, -1.0 / 6.0);
    return fma(x * x2, p, x);
}
constexpr double SIN_POLY_MAX = 0.0078125;  // 2^-7

// Out of line: sin's full range reduction would otherwise hold its registers
// across the whole candidate loop, though arguments past 2^-7 are rare.
__device__ __attribute__((noinline)) double sin_wide(double x) { return sin(x); }

// The four half-angle sines of a candidate against a pixel group: (dec - dec0,
// dec - dec1, ra - ra0, ra - ra1) / 2.  Arguments past the polynomial's range
// go through one shared call of sin, rotated into place, so that the kernel
// carries a single inlined copy of it.
__device__ inline void half_sines(double a0, double a1, double a2, double a3, double& s0,
                                  double& s1, double& s2, double& s3) {
    s0 = sin_poly(a0);
    s1 = sin_poly(a1);
    s2 = sin_poly(a2);
    s3 = sin_poly(a3);
    const bool big = fabs(a0) >= SIN_POLY_MAX || fabs(a1) >= SIN_POLY_MAX ||
                     fabs(a2) >= SIN_POLY_MAX || fabs(a3) >= SIN_POLY_MAX;
    if (big) {
#pragma unroll 1
        for (int k = 0; k < 4; k++) {
            const double r = fabs(a0) >= SIN_POLY_MAX ? sin_wide(a0) : s0;
            a0 = a1;
            a1 = a2;
            a2 = a3;
            s0 = s1;
            s1 = s2;
            s2 = s3;
            s3 = r;
        }
    }
}

// Kernel constants for the weight of Eq. 1 (w for the plan's hg_kernel type).
struct KernelArgs {
    double inv_two_s2;      // Gaussian: 1 / 2 sigma^2
    double inv_a2, pi_b;    // Gauss-sinc: 1 / a^2, pi / b
    double inv_two_smaj2, inv_two_smin2, cos_pa, sin_pa;  // elliptical
};

KernelArgs kernel_args(const Plan& P) {
    KernelArgs ka{};
    const double f2s = 1.0 / sqrt(8.0 * log(2.0));
    if (P.kern.type == HG_KERNEL_GAUSS) {
        ka.inv_two_s2 = 1.0 / (2.0 * P.sigma * P.sigma);
    } else if (P.kern.type == HG_KERNEL_GAUSS_SINC) {
        const double a = P.kern.p1 * kDeg, b = P.kern.p2 * kDeg;
        ka.inv_a2 = 1.0 / (a * a);
        ka.pi_b = 3.14159265358979323846 / b;
    } else {
        const double smaj = P.kern.fwhm_deg * kDeg * f2s, smin = P.kern.p1 * kDeg * f2s;
        ka.inv_two_smaj2 = 1.0 / (2.0 * smaj * smaj);
        ka.inv_two_smin2 = 1.0 / (2.0 * smin * smin);
        ka.cos_pa = cos(P.kern.p2 * kDeg);
        ka.sin_pa = sin(P.kern.p2 * kDeg);
    }
    return ka;
}

// e^x for x <= 0, to within 3e-13 relative: ample for a weight that is then
// rounded to FP32 (it changes about one rounding in a million, by an ulp).
// x = n ln 2 + r with |r| <= ln 2 / 2, r from one fused multiply-add (for the
// n that matter, |n| <= 160, the error of ln 2 in a double shifts r by under
// 4e-15), e^r by its Taylor series to r^10 (remainder below 2.4e-13), scaled
// by 2^n.  x is clamped at -800, where e^x is already 0 in FP64.
__device__ inline double exp_w(double x) {
    x = fmax(x, -800.0);
    const double n = rint(x * 1.4426950408889634);  // x / ln 2
    const double r = fma(-n, 0.6931471805599453, x);
    double p = 1.0 / 3628800.0;  // 1/10!
    p = fma(p, r, 1.0 / 362880.0);
    p = fma(p, r, 1.0 / 40320.0);
    p = fma(p, r, 1.0 / 5040.0);
    p = fma(p, r, 1.0 / 720.0);
    p = fma(p, r, 1.0 / 120.0);
    p = fma(p, r, 1.0 / 24.0);
    p = fma(p, r, 1.0 / 6.0);
    p = fma(p, r, 0.5);
    p = fma(p, r, 1.0);
    p = fma(p, r, 1.0);
    return ldexp(p, (int)n);
}

// What the elliptical kernel needs of a pair beyond d^2: sin(dRA/2) as the
// haversine took it, dRA = RA_n - RA_p itself (for its whole turns), and the
// cosines and sines of the two declinations.
struct PairGeom {
    double sa, dra, cos_n, sin_n, cos_p, sin_p;
};

// The weight of a pair in support, from its squared distance d2 and (for the
// elliptical kernel) the pair's geometry: the bearing theta of the sample seen
// from the cell has sin theta : cos theta = E : N with E = cos dec_n sin dRA,
// N = cos dec_p sin dec_n - sin dec_p cos dec_n cos dRA (both sin d times the
// unit components), so the offsets along the axes at position angle pa are
// u = d cos(theta - pa), v = d sin(theta - pa).  sin dRA and cos dRA come from
// the haversine's half-angle sine: with dRA = 2 pi k + r, |r| <= pi,
// sin(r/2) = (-1)^k sin(dRA/2) and cos(r/2) = sqrt(1 - sin^2(r/2)) >= 0, so
// sin dRA = 2 sin(r/2) cos(r/2) and cos dRA = 1 - 2 sin^2(r/2).
template <int KT>
__device__ inline double kernel_weight(const KernelArgs& ka, double d2, const PairGeom& g) {
    if (KT == HG_KERNEL_GAUSS) return exp_w(-d2 * ka.inv_two_s2);
    if (KT == HG_KERNEL_GAUSS_SINC) {
        const double x = sqrt(d2) * ka.pi_b;
        const double sinc = x > 0.0 ? sin(x) / x : 1.0;
        return sinc * exp_w(-d2 * ka.inv_a2);
    }
    const double turns = rint(g.dra * (0.5 / kPi));
    const double sh = ((int64_t)turns & 1) ? -g.sa : g.sa;  // sin(r/2)
    const double ch = sqrt(fmax(0.0, 1.0 - sh * sh));       // cos(r/2)
    const double e = g.cos_n * (2.0 * sh * ch);
    const double nn = g.cos_p * g.sin_n - g.sin_p * g.cos_n * (1.0 - 2.0 * sh * sh);
    const double r2 = e * e + nn * nn;
    if (!(r2 > 0.0)) return 1.0;  // d = 0
    const double ct = nn / sqrt(r2), st = e / sqrt(r2);
    const double cu = ct * ka.cos_pa + st * ka.sin_pa;  // cos(theta - pa)
    const double sv = st * ka.cos_pa - ct * ka.sin_pa;  // sin(theta - pa)
    return exp_w(-d2 * (cu * cu * ka.inv_two_smaj2 + sv * sv * ka.inv_two_smin2));
}

// One wave per pixel group.  Lanes walk the group's candidates in slot order;
// each lane tests its candidate against the group's (up to) four pixels with
// the exact FP64 haversine test, and surviving candidates are compacted in
// order into the group's entry list with their four FP32 weights.  HPX: the
// map is a HEALPix patch, whose two rows have their own pixel RAs.
constexpr int GATHER_WAVES = 4;
// Candidates that pass the support test wait in a per-wave LDS queue (their
// entry word and four haversines) until a whole wave of them is there, so
// that the weights, most of the gather's arithmetic, are computed on full
// waves of real pairs instead of on every candidate lane; GATHER_QCAP holds
// one wave's worth left over plus one pass.  The elliptical kernel, whose
// weight needs more of each pair's geometry, computes in place.
constexpr int GATHER_QCAP = 128;
constexpr size_t GATHER_QUEUE_BYTES = GATHER_QCAP * (4 * sizeof(double) + sizeof(uint32_t));
inline size_t gather_lds_bytes(int64_t npc) {
    const size_t lists = (size_t)GATHER_WAVES * 3 * (npc + 1) * sizeof(int);
    return (lists + 15) / 16 * 16 + (size_t)GATHER_WAVES * GATHER_QUEUE_BYTES;
}
__device__ inline void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}
constexpr int BUCKET_WAVES = 4;
constexpr int BUCKET_REGS = 16;  // slot words a lane holds per round of the bucketing
// tiles whose chunks' presence words (one 64-bit word per 64 positions of a
// chunk) number at most this many are dealt (chunk = compacted slot mod the
// chunk count); denser tiles keep consecutive slots per chunk
constexpr int SCRAMBLE_MAX_WORDS = 1024;
__host__ __device__ inline int chunk_words(int32_t chunk) { return (chunk + 63) / 64; }

template <bool SMALL, int KT, bool HPX>
__global__ __launch_bounds__(64 * GATHER_WAVES) void k_gather(
    const int4* __restrict__ pg_piece, int32_t pg_rings, const int64_t* __restrict__ pg_base,
    const double4* __restrict__ srt_coord, int32_t npgx, int64_t npg, hg_map m, double h_r,
    KernelArgs ka, int32_t prec, uint32_t* __restrict__ ent_slot, float4* __restrict__ ent_w,
    uint32_t* __restrict__ pg_cnt, int32_t* __restrict__ pix_count, double* __restrict__ pix_W,
    float* __restrict__ pix_Wf) {
    extern __shared__ int sh_gather[];
    // the wave index through a scalar register, so that the group's scalars
    // (its entry base among them) come by scalar loads, outside the vector
    // memory counter that the candidate loads are waited on by
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    int64_t pg = (int64_t)blockIdx.x * GATHER_WAVES + wave;
    if (pg >= npg) return;  // uniform per wave; no block barrier below
    int npc = 2 * pg_rings;
    int* pref = sh_gather + wave * 3 * (npc + 1);
    int* ppos = pref + (npc + 1);
    int* pslot = ppos + (npc + 1);
    const int4* pp = pg_piece + pg * npc;
    constexpr bool QUEUE = KT != HG_KERNEL_ELLIPTICAL;
    const size_t lists = ((size_t)GATHER_WAVES * 3 * (npc + 1) * sizeof(int) + 15) / 16 * 16;
    double* qh = (double*)((char*)sh_gather + lists + (size_t)wave * GATHER_QUEUE_BYTES);
    uint32_t* qkey = (uint32_t*)(qh + 4 * GATHER_QCAP);
    int qn = 0;  // queued candidates (wave-uniform)
    if (lane == 0) {
        int s = 0;
        for (int k = 0; k < npc; k++) {
            int4 p = pp[k];
            pref[k] = s;
            ppos[k] = p.x;
            pslot[k] = p.z;
            s += p.y;
        }
        pref[npc] = s;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    int total = pref[npc];
    int gx = (int)(pg % npgx), gy = (int)(pg / npgx);
    int64_t ix = (int64_t)gx * PG, iy = (int64_t)gy * PG;
    bool vx1 = ix + 1 < m.nx, vy1 = iy + 1 < m.ny;
    // pra[k]: pixel k = (column k & 1, row k >> 1); the rows share RAs unless HPX
    double pra[4];
    pra[0] = pix_ra(m, ix, iy);
    pra[1] = pix_ra(m, ix + 1, iy);
    pra[2] = HPX ? pix_ra(m, ix, iy + 1) : pra[0];
    pra[3] = HPX ? pix_ra(m, ix + 1, iy + 1) : pra[1];
    double pdec0 = pix_dec(m, iy), pdec1 = pix_dec(m, iy + 1);
    double pcos0 = cos(pdec0), pcos1 = cos(pdec1);
    const double psin0 = KT == HG_KERNEL_ELLIPTICAL ? sin(pdec0) : 0.0;
    const double psin1 = KT == HG_KERNEL_ELLIPTICAL ? sin(pdec1) : 0.0;
    int cnt[4] = {0, 0, 0, 0};
    double wsum[4] = {0.0, 0.0, 0.0, 0.0};
    int64_t base_out = pg_base[pg];
    int written = 0;
    // Candidate v's coordinates and slot are loaded one pass ahead of their
    // use, so that the load's latency overlaps the previous pass's arithmetic.
    // lo: the piece holding the candidate loaded last; v only grows, so lo
    // only advances (each search stops by pref[npc] = total > v).
    int lo = 0;
    double4 cn = make_double4(0.0, 0.0, 0.0, 0.0);
    uint32_t sn = 0;
    if (lane < total) {
        while (pref[lo + 1] <= lane) lo++;
        const int off = lane - pref[lo];
        cn = srt_coord[ppos[lo] + off];
        sn = (uint32_t)(pslot[lo] + off);
    }
    // Weights of the first n queued candidates, one a lane, written to the
    // entry list after those written before (QUEUE only).
    auto drain = [&](int n) {
        if (lane < n) {
            const uint32_t key = qkey[lane];
            const uint32_t mk = key >> SLOT_SHIFT;
            const PairGeom g{0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
            float wq[4];
#pragma unroll
            for (int k = 0; k < 4; k++) {
                const double h = qh[k * GATHER_QCAP + lane];
                float wf = 0.f;
                if ((mk >> k) & 1u)
                    wf = round_weight((float)kernel_weight<KT>(ka, dist2<SMALL>(h), g), prec);
                wq[k] = wf;
                cnt[k] += (mk >> k) & 1u;
                wsum[k] += (double)wf;
            }
            ent_slot[base_out + written + lane] = key;
            ent_w[base_out + written + lane] = make_float4(wq[0], wq[1], wq[2], wq[3]);
        }
        written += n;
    };
    for (int v0 = 0; v0 < total; v0 += 64) {
        int v = v0 + lane;
        bool active = v < total;
        uint32_t mask = 0;
        float w[4] = {0.f, 0.f, 0.f, 0.f};
        const double4 c = cn;
        const uint32_t slot = sn;
        if (v + 64 < total) {
            while (pref[lo + 1] <= v + 64) lo++;
            const int off = v + 64 - pref[lo];
            cn = srt_coord[ppos[lo] + off];
            sn = (uint32_t)(pslot[lo] + off);
        }
        double hk[4] = {0.0, 0.0, 0.0, 0.0};
        if (active) {
            double sd0, sd1, sa[4];
            half_sines(0.5 * (c.y - pdec0), 0.5 * (c.y - pdec1), 0.5 * (c.x - pra[0]),
                       0.5 * (c.x - pra[1]), sd0, sd1, sa[0], sa[1]);
            if (HPX) {
                double u0, u1;
                half_sines(0.5 * (c.x - pra[2]), 0.5 * (c.x - pra[3]), 0.0, 0.0, sa[2], sa[3],
                           u0, u1);
            } else {
                sa[2] = sa[0];
                sa[3] = sa[1];
            }
#pragma unroll
            for (int k = 0; k < 4; k++) {
                bool ok = ((k & 1) == 0 || vx1) && ((k >> 1) == 0 || vy1);
                double sd = (k >> 1) ? sd1 : sd0;
                double sa_k = sa[k];
                double pc = (k >> 1) ? pcos1 : pcos0;
                hk[k] = sd * sd + pc * c.z * sa_k * sa_k;
                if (ok && hk[k] <= h_r) mask |= 1u << k;
            }
            if constexpr (!QUEUE) {
                // The four pixels' weights in turn, each pixel and its pair
                // geometry rotated through the first place; the loop is
                // unrolled, so the rotations are only renamings (four inlined
                // copies of the weight hold fewer live registers than one copy
                // in a loop did).
                double h0 = hk[0], h1 = hk[1], h2 = hk[2], h3 = hk[3];
                double s0 = sa[0], s1 = sa[1], s2 = sa[2], s3 = sa[3];
                double r0 = c.x - pra[0], r1 = c.x - pra[1], r2 = c.x - pra[2], r3 = c.x - pra[3];
                uint32_t mk = mask;
#pragma unroll
                for (int k = 0; k < 4; k++) {
                    float wf = 0.f;
                    if (mk & 1u) {
                        const PairGeom g{s0, r0, c.z, c.w, (k >> 1) ? pcos1 : pcos0,
                                         (k >> 1) ? psin1 : psin0};
                        wf = round_weight((float)kernel_weight<KT>(ka, dist2<SMALL>(h0), g), prec);
                    }
                    h0 = h1;
                    h1 = h2;
                    h2 = h3;
                    s0 = s1;
                    s1 = s2;
                    s2 = s3;
                    r0 = r1;
                    r1 = r2;
                    r2 = r3;
                    w[0] = w[1];
                    w[1] = w[2];
                    w[2] = w[3];
                    w[3] = wf;
                    mk >>= 1;
                }
#pragma unroll
                for (int k = 0; k < 4; k++) {
                    cnt[k] += (mask >> k) & 1u;
                    wsum[k] += (double)w[k];
                }
            }
        }
        bool keep = active && mask != 0;
        uint64_t bal = __ballot(keep);
        if constexpr (QUEUE) {
            // append in candidate order (the entry list stays in slot order)
            if (keep) {
                int o = qn + __popcll(bal & ((1ull << lane) - 1ull));
                qkey[o] = slot | (mask << SLOT_SHIFT);
#pragma unroll
                for (int k = 0; k < 4; k++) qh[k * GATHER_QCAP + o] = hk[k];
            }
            qn += __popcll(bal);
            if (qn >= 64) {
                wave_lds_sync();
                drain(64);
                // move the rest (fewer than 64) to the front; each lane moves
                // its own entry, reading and writing one place apart by 64
                const int rest = qn - 64;
                if (lane < rest) {
                    qkey[lane] = qkey[64 + lane];
#pragma unroll
                    for (int k = 0; k < 4; k++)
                        qh[k * GATHER_QCAP + lane] = qh[k * GATHER_QCAP + 64 + lane];
                }
                wave_lds_sync();
                qn = rest;
            }
        } else {
            if (keep) {
                int o = written + __popcll(bal & ((1ull << lane) - 1ull));
                ent_slot[base_out + o] = slot | (mask << SLOT_SHIFT);
                ent_w[base_out + o] = make_float4(w[0], w[1], w[2], w[3]);
            }
            written += __popcll(bal);
        }
    }
    if constexpr (QUEUE) {
        if (qn > 0) {
            wave_lds_sync();
            drain(qn);
        }
    }
#pragma unroll
    for (int k = 0; k < 4; k++) {
        int c = cnt[k];
        double s = wsum[k];
        for (int o = 32; o > 0; o >>= 1) {
            c += __shfl_xor(c, o, 64);
            s += __shfl_xor(s, o, 64);
        }
        cnt[k] = c;
        wsum[k] = s;
    }
    if (lane == 0) {
        pg_cnt[pg] = (uint32_t)written;
#pragma unroll
        for (int k = 0; k < 4; k++) {
            int64_t i = ix + (k & 1), j = iy + (k >> 1);
            if (i < m.nx && j < m.ny) {
                int64_t p = j * m.nx + i;
                pix_count[p] = cnt[k];
                pix_W[p] = wsum[k];
                pix_Wf[p] = (float)wsum[k];
            }
        }
    }
}

// sum of a[0..n) into *out, which starts at 0: a grid-stride pass, a
// workgroup reduction, one atomic per workgroup (the total of the pixels'
// neighbour counts, kept out of the gather, where one atomic per pixel group
// on a single address serialised)
__global__ __launch_bounds__(256) void k_sum_counts(const int32_t* __restrict__ a, int64_t n,
                                                    unsigned long long* __restrict__ out) {
    __shared__ unsigned long long red[4];
    unsigned long long t = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        t += (unsigned long long)a[i];
    for (int o = 32; o > 0; o >>= 1) t += __shfl_xor(t, o, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = t;
    __syncthreads();
    if (threadIdx.x == 0) atomicAdd(out, red[0] + red[1] + red[2] + red[3]);
}

// the gather instance for a kernel shape, support size and map kind
template <bool HPX>
auto gather_kernel(int32_t type, bool small) {
    if (type == HG_KERNEL_GAUSS)
        return small ? k_gather<true, HG_KERNEL_GAUSS, HPX> : k_gather<false, HG_KERNEL_GAUSS, HPX>;
    if (type == HG_KERNEL_GAUSS_SINC)
        return small ? k_gather<true, HG_KERNEL_GAUSS_SINC, HPX>
                     : k_gather<false, HG_KERNEL_GAUSS_SINC, HPX>;
    return small ? k_gather<true, HG_KERNEL_ELLIPTICAL, HPX>
                 : k_gather<false, HG_KERNEL_ELLIPTICAL, HPX>;
}

// Per (pixel group, chunk): first entry whose slot is in the chunk, relative to
// the group's entry base; entries are in ascending slot order.
__global__ __launch_bounds__(256) void k_chunk_ptr(
    int32_t npgx, int64_t npg, int32_t ntx, int32_t chunk, const int64_t* __restrict__ tile_base,
    const int64_t* __restrict__ cp_base, const int64_t* __restrict__ pg_base,
    const uint32_t* __restrict__ pg_cnt, const uint32_t* __restrict__ ent_slot,
    uint32_t* __restrict__ chunk_ptr) {
    int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    int64_t pg = (int64_t)blockIdx.x * 4 + wave;
    if (pg >= npg) return;
    int gx = (int)(pg % npgx), gy = (int)(pg / npgx);
    int64_t tile = (int64_t)(gy / TILE_PGY) * ntx + gx / TILE_PGX;
    int lp = (gy % TILE_PGY) * TILE_PGX + gx % TILE_PGX;
    int64_t nslots = tile_base[tile + 1] - tile_base[tile];
    int64_t nch = (nslots + chunk - 1) / chunk;
    uint32_t* cp = chunk_ptr + cp_base[tile] + (int64_t)lp * (nch + 1);
    const uint32_t* es = ent_slot + pg_base[pg];
    uint32_t ne = pg_cnt[pg];
    for (int64_t c = lane; c <= nch; c += 64) {
        uint32_t target = (uint32_t)(c * chunk);
        uint32_t lo = 0, hi = ne;
        while (lo < hi) {
            uint32_t mid = (lo + hi) >> 1;
            if ((es[mid] & SLOT_MASK) < target)
                lo = mid + 1;
            else
                hi = mid;
        }
        cp[c] = lo;
    }
}

inline unsigned blocks_for(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

// Several device buffers (whole dwords each) set to zero by one launch
// instead of one runtime call apiece.
struct ZeroList {
    uint32_t* p[8];
    int64_t dwords[8];
    int32_t n;
};
__global__ __launch_bounds__(256) void k_zero(ZeroList z) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int k = 0; k < z.n; k++)
        for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < z.dwords[k]; i += stride)
            z.p[k][i] = 0u;
}

// Slot compaction.  A tile's slots are every sample of its candidate cell runs;
// those no pixel of the tile has in its support are dropped, so that the
// channel kernel stages only samples it uses.  Slot order (ring, cell,
// index) is kept, so each group's entries stay in ascending slot order.
__device__ inline int64_t pg_tile(int64_t pg, int32_t npgx, int32_t ntx) {
    int gx = (int)(pg % npgx), gy = (int)(pg / npgx);
    return (int64_t)(gy / TILE_PGY) * ntx + gx / TILE_PGX;
}

// entries a lane keeps in flight in the slot marking and remapping (16 kept
// the marking as it was and slowed the remapping, 0.039 -> 0.050 ms on a
// million samples, at six waves a SIMD instead of eight)
constexpr int ENTRY_REGS = 4;

__global__ __launch_bounds__(256) void k_mark_used(
    int32_t npgx, int64_t npg, int32_t ntx, const int64_t* __restrict__ tile_base,
    const int64_t* __restrict__ pg_base, const uint32_t* __restrict__ pg_cnt,
    const uint32_t* __restrict__ ent_slot, uint32_t* __restrict__ used) {
    int64_t pg = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (pg >= npg) return;
    const int lane = threadIdx.x & 63;
    const int64_t tb = tile_base[pg_tile(pg, npgx, ntx)];
    const uint32_t* es = ent_slot + pg_base[pg];
    const uint32_t n = pg_cnt[pg];
    // ENTRY_REGS entries a lane per pass, their loads in flight together (a
    // group of a wide support holds thousands of entries); workgroup row y
    // of gridDim.y takes every gridDim.y-th pass
    for (uint32_t t0 = 64 * ENTRY_REGS * blockIdx.y; t0 < n; t0 += 64 * ENTRY_REGS * gridDim.y) {
        uint32_t w[ENTRY_REGS];
#pragma unroll
        for (int k = 0; k < ENTRY_REGS; k++) {
            const uint32_t t = t0 + lane + 64 * k;
            w[k] = t < n ? es[t] : 0u;
        }
#pragma unroll
        for (int k = 0; k < ENTRY_REGS; k++)
            if (t0 + lane + 64 * k < n) used[tb + (w[k] & SLOT_MASK)] = 1u;
    }
}

__global__ void k_tile_rebase(const int64_t* __restrict__ tile_base, int64_t ntiles,
                              const int64_t* __restrict__ newpos, int32_t chunk,
                              int64_t* __restrict__ tile_base2, int64_t* __restrict__ tile_ncp,
                              int64_t* __restrict__ tile_nch, int64_t* __restrict__ tile_pad,
                              int32_t* __restrict__ tile_scr) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t > ntiles) return;
    tile_base2[t] = newpos[tile_base[t]];
    if (t == ntiles) return;
    int64_t ns = newpos[tile_base[t + 1]] - newpos[tile_base[t]];
    const int64_t nch = (ns + chunk - 1) / chunk;
    tile_ncp[t] = (int64_t)TILE_PGS * (nch + 1);
    tile_nch[t] = nch;
    // Dealt tiles: slot p of the compacted list goes to chunk p mod nch, so
    // that every chunk samples the whole tile (a run of consecutive slots
    // lies in one or two sky cells, i.e. in a few pixel groups only); the
    // chunks' unused tail slots are padding.
    const bool scr = nch >= 2 && nch * chunk_words(chunk) <= SCRAMBLE_MAX_WORDS &&
                     nch * chunk <= (int64_t)SLOT_MASK;
    tile_scr[t] = scr ? 1 : 0;
    tile_pad[t] = scr ? nch * chunk : ns;
}

// Tile-local slot of compacted slot p in a dealt tile: chunk p mod nch,
// position p / nch in it.
__device__ inline uint32_t dealt_slot(int64_t p, int64_t nch, int32_t chunk) {
    return (uint32_t)((p % nch) * chunk + p / nch);
}

__global__ __launch_bounds__(256) void k_remap_entries(
    int32_t npgx, int64_t npg, int32_t ntx, int32_t chunk, const int64_t* __restrict__ tile_base,
    const int64_t* __restrict__ tile_base2, const int64_t* __restrict__ tile_nch,
    const int32_t* __restrict__ tile_scr, const int64_t* __restrict__ pg_base,
    const uint32_t* __restrict__ pg_cnt, const int64_t* __restrict__ newpos,
    uint32_t* __restrict__ ent_slot) {
    int64_t pg = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (pg >= npg) return;
    const int lane = threadIdx.x & 63;
    const int64_t tile = pg_tile(pg, npgx, ntx);
    const int64_t tb = tile_base[tile], tb2 = tile_base2[tile];
    const bool scr = tile_scr[tile] != 0;
    const int64_t nch = tile_nch[tile];
    uint32_t* es = ent_slot + pg_base[pg];
    const uint32_t n = pg_cnt[pg];
    // ENTRY_REGS entries a lane per pass: their loads, then their position
    // lookups, each in flight together; workgroup row y of gridDim.y takes
    // every gridDim.y-th pass
    for (uint32_t t0 = 64 * ENTRY_REGS * blockIdx.y; t0 < n; t0 += 64 * ENTRY_REGS * gridDim.y) {
        uint32_t w[ENTRY_REGS];
        int64_t np[ENTRY_REGS];
#pragma unroll
        for (int k = 0; k < ENTRY_REGS; k++) {
            const uint32_t t = t0 + lane + 64 * k;
            w[k] = t < n ? es[t] : 0u;
        }
#pragma unroll
        for (int k = 0; k < ENTRY_REGS; k++)
            np[k] = t0 + lane + 64 * k < n ? newpos[tb + (w[k] & SLOT_MASK)] : tb2;
#pragma unroll
        for (int k = 0; k < ENTRY_REGS; k++) {
            const uint32_t t = t0 + lane + 64 * k;
            const int64_t p = np[k] - tb2;
            const uint32_t loc = scr ? dealt_slot(p, nch, chunk) : (uint32_t)p;
            if (t < n) es[t] = loc | (w[k] & ~SLOT_MASK);
        }
    }
}

__global__ void k_compact_slots(const uint32_t* __restrict__ used,
                                const int64_t* __restrict__ newpos, int64_t n,
                                const uint32_t* __restrict__ src, uint32_t* __restrict__ dst) {
    int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g < n && used[g]) dst[newpos[g]] = src[g];
}



// The tile slot lists in their final layout (base tile_base3): a dealt tile's
// slot c * chunk + j holds compacted slot j * nch + c, or, past the chunk's
// real slots, the tile's first sample (staged and never used); other tiles
// are copied as they are.  One workgroup per tile.
__global__ __launch_bounds__(256) void k_deal_slots(
    const int64_t* __restrict__ tile_base2, const int64_t* __restrict__ tile_base3,
    const int64_t* __restrict__ tile_nch, const int32_t* __restrict__ tile_scr, int32_t chunk,
    const uint32_t* __restrict__ src, uint32_t* __restrict__ dst) {
    const int64_t t = blockIdx.x;
    const int64_t b2 = tile_base2[t], ns = tile_base2[t + 1] - b2;
    const int64_t b3 = tile_base3[t], np = tile_base3[t + 1] - b3;
    const bool scr = tile_scr[t] != 0;
    const int64_t nch = tile_nch[t];
    for (int64_t q = threadIdx.x; q < np; q += blockDim.x) {
        int64_t p = q;
        if (scr) {
            p = (q % chunk) * nch + q / chunk;
            if (p >= ns) p = 0;
        }
        dst[b3 + q] = src[b2 + p];
    }
}

// Entries bucketed by chunk, one wave per pixel group.  A dealt tile's
// entries leave the remap in ascending compacted slot, i.e. with chunks
// interleaved; each entry's tile-local slot is (chunk c, position j < chunk).
// The group's entries are marked in one 64-bit word per 64 positions of a
// chunk (LDS: bit j mod 64 of word j / 64 of chunk c), the chunks' popcounts
// scanned into the group's chunk pointers, and every entry's bucketed place
// is pointer c plus the number of its chunk's entries at lower positions --
// a function of the set alone, so every entry
// is placed at once, each bucket is in ascending slot order, and the layout
// does not depend on the order of the atomics.  The entries themselves stay
// where they are: perm[place] holds the entry's index in the group's list
// (the block fills read its weights through it) above PERM_POS_BITS bits of
// its position in its chunk (the slot the fills store, so that they need not
// read the entry's slot word).  Other tiles keep their (already sorted)
// order, take their pointers by binary search and an identity perm.
template <bool WIDE>
__global__ __launch_bounds__(64 * BUCKET_WAVES) void k_bucket_entries(
    int32_t npgx, int64_t npg, int32_t ntx, int32_t chunk, const int64_t* __restrict__ tile_blk,
    const int32_t* __restrict__ tile_scr, const int64_t* __restrict__ cp_base,
    const int64_t* __restrict__ pg_base, const uint32_t* __restrict__ pg_cnt,
    const uint32_t* __restrict__ ent_slot, uint32_t* __restrict__ chunk_ptr,
    uint32_t* __restrict__ perm, int32_t words) {
    static_assert(MAX_CHUNK <= 128, "a chunk's positions fit two 64-bit words");
    // per group: `words` presence words and as many chunk pointers; words
    // bounds nch * chunk_words(chunk) of every dealt tile (the host sizes it
    // from the largest chunk count before compaction, which only drops slots).
    // A wave a group, or (WIDE, for groups of many entries) the whole
    // workgroup a group, its T threads sharing the group's passes.
    constexpr int T = WIDE ? 64 * BUCKET_WAVES : 64;
    extern __shared__ unsigned long long sh_bucket[];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int tid = WIDE ? (int)threadIdx.x : lane;
    const int64_t pg = WIDE ? (int64_t)blockIdx.x : (int64_t)blockIdx.x * BUCKET_WAVES + wave;
    // uniform per wave (per workgroup if WIDE): no barrier is skipped
    if (pg >= npg) return;
    unsigned long long* bits = sh_bucket + (WIDE ? 0 : (int64_t)wave * words);
    uint32_t* ptr = (uint32_t*)(sh_bucket + (int64_t)(WIDE ? 1 : BUCKET_WAVES) * words) +
                    (WIDE ? 0 : (int64_t)wave * words);
    auto sync = [&]() {
        if constexpr (WIDE)
            __syncthreads();
        else
            __builtin_amdgcn_wave_barrier();
    };
    const int gx = (int)(pg % npgx), gy = (int)(pg / npgx);
    const int64_t tile = (int64_t)(gy / TILE_PGY) * ntx + gx / TILE_PGX;
    const int lp = (gy % TILE_PGY) * TILE_PGX + gx % TILE_PGX;
    const int64_t nch = tile_blk[tile + 1] - tile_blk[tile];
    uint32_t* cp = chunk_ptr + cp_base[tile] + (int64_t)lp * (nch + 1);
    const int64_t base = pg_base[pg];
    const uint32_t* es = ent_slot + base;
    uint32_t* pm = perm + base;
    const uint32_t ne = pg_cnt[pg];
    if (!tile_scr[tile]) {
        for (int64_t c = tid; c <= nch; c += T) {
            const uint32_t target = (uint32_t)(c * chunk);
            uint32_t lo = 0, hi = ne;
            while (lo < hi) {
                const uint32_t mid = (lo + hi) >> 1;
                if ((es[mid] & SLOT_MASK) < target)
                    lo = mid + 1;
                else
                    hi = mid;
            }
            cp[c] = lo;
        }
        for (uint32_t t = tid; t < ne; t += T)
            pm[t] = (t << PERM_POS_BITS) | ((es[t] & SLOT_MASK) % (uint32_t)chunk);
        return;
    }
    // dealt tiles: nch * nw <= SCRAMBLE_MAX_WORDS
    const int nw = chunk_words(chunk);
    for (int64_t i = tid; i < nch * nw; i += T) bits[i] = 0ull;
    sync();
    // the group's slot words come BUCKET_REGS a lane at a time, all loads of
    // a round issued before any is used, so that a wave waits for memory once
    // a round rather than once an entry
    for (uint32_t t0 = 0; t0 < ne; t0 += T * BUCKET_REGS) {
        uint32_t loc[BUCKET_REGS];
#pragma unroll
        for (int k = 0; k < BUCKET_REGS; k++) {
            const uint32_t t = t0 + tid + T * k;
            loc[k] = t < ne ? es[t] & SLOT_MASK : 0u;
        }
#pragma unroll
        for (int k = 0; k < BUCKET_REGS; k++) {
            if (t0 + tid + T * k < ne) {
                const uint32_t c = loc[k] / chunk, j = loc[k] % chunk;
                atomicOr(&bits[c * nw + j / 64], 1ull << (j % 64));
            }
        }
    }
    sync();
    // exclusive scan of the chunks' entry counts: the chunk pointers (one wave)
    if (!WIDE || wave == 0) {
        uint32_t carry = 0;
        for (int64_t c0 = 0; c0 < nch; c0 += 64) {
            const int64_t c = c0 + lane;
            uint32_t v = 0;
            if (c < nch)
                for (int w = 0; w < nw; w++) v += (uint32_t)__builtin_popcountll(bits[c * nw + w]);
            uint32_t x = v;
            for (int o = 1; o < 64; o <<= 1) {
                const uint32_t y = __shfl_up(x, o, 64);
                if (lane >= o) x += y;
            }
            const uint32_t excl = carry + x - v;
            if (c < nch) {
                cp[c] = excl;
                ptr[c] = excl;
            }
            carry += __shfl(x, 63, 64);
        }
        if (lane == 0) cp[nch] = carry;
    }
    sync();
    for (uint32_t t0 = 0; t0 < ne; t0 += T * BUCKET_REGS) {
        uint32_t loc[BUCKET_REGS];
#pragma unroll
        for (int k = 0; k < BUCKET_REGS; k++) {
            const uint32_t t = t0 + tid + T * k;
            loc[k] = t < ne ? es[t] & SLOT_MASK : 0u;
        }
#pragma unroll
        for (int k = 0; k < BUCKET_REGS; k++) {
            const uint32_t t = t0 + tid + T * k;
            if (t < ne) {
                const uint32_t c = loc[k] / chunk, j = loc[k] % chunk;
                const unsigned long long* cw = bits + c * nw;
                uint32_t at = ptr[c];
                for (uint32_t w = 0; w < j / 64; w++) at += (uint32_t)__builtin_popcountll(cw[w]);
                const unsigned long long below = (1ull << (j % 64)) - 1ull;
                pm[at + (uint32_t)__builtin_popcountll(cw[j / 64] & below)] =
                    (t << PERM_POS_BITS) | j;
            }
        }
    }
}

// host-side ring band of a declination range [d0, d1] (radians) widened by r
void ring_range(int64_t nside, double d0, double d1, double r, double eps, int32_t* lo,
                int32_t* cnt) {
    double za = sin(fmax(-0.5 * kPi, d0 - r - eps));
    double zb = sin(fmin(0.5 * kPi, d1 + r + eps));
    double t_lo = hp_ring_coord(nside, zb), t_hi = hp_ring_coord(nside, za);
    int64_t a = (int64_t)floor(t_lo) - 1, b = (int64_t)ceil(t_hi) + 1;
    if (a < 1) a = 1;
    if (b > 4 * nside - 1) b = 4 * nside - 1;
    *lo = (int32_t)a;
    *cnt = (int32_t)(b - a + 1);
}

double ra_halfwidth(double d0, double d1, double r, double eps) {
    double far = fmax(fabs(d0), fabs(d1));
    if (far + r + eps >= 0.5 * kPi - 1e-12) return 4.0 * kPi;  // support reaches a pole
    double x = sin(r) / cos(far);
    if (x >= 1.0) return 4.0 * kPi;
    return asin(x);
}

}  // namespace

hipError_t launch_ang2pix(int64_t nside, const double* ra_deg, const double* dec_deg, int64_t n,
                          int64_t* pix, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_ang2pix, dim3(blocks_for(n, 256)), dim3(256), 0, s, ra_deg, dec_deg, n,
                       nside, pix);
    return hipGetLastError();
}

// Plan geometry that needs no sample data (row a1 of the path): ring bands per
// tile row and per pixel-group row.
static void plan_rows(Plan& P, std::vector<RowInfo>& trows, std::vector<RowInfo>& prows,
                      double eps) {
    const hg_map& m = P.map;
    trows.resize(P.nty);
    prows.resize(P.npgy);
    int32_t tmax = 1, pmax = 1;
    for (int ty = 0; ty < P.nty; ty++) {
        int64_t j0 = (int64_t)ty * TILE_PGY * PG, j1 = j0 + TILE_PGY * PG - 1;
        if (j1 > m.ny - 1) j1 = m.ny - 1;
        double d0 = pix_dec(m, j0), d1 = pix_dec(m, j1);
        RowInfo ri;
        ring_range(P.nside, d0, d1, P.r_rad, eps, &ri.ring_lo, &ri.nrings);
        ri.dalpha = ra_halfwidth(d0, d1, P.r_rad, eps);
        trows[ty] = ri;
        if (ri.nrings > tmax) tmax = ri.nrings;
    }
    for (int gy = 0; gy < P.npgy; gy++) {
        int64_t j0 = (int64_t)gy * PG, j1 = j0 + PG - 1;
        if (j1 > m.ny - 1) j1 = m.ny - 1;
        double d0 = pix_dec(m, j0), d1 = pix_dec(m, j1);
        RowInfo ri;
        ring_range(P.nside, d0, d1, P.r_rad, eps, &ri.ring_lo, &ri.nrings);
        ri.dalpha = ra_halfwidth(d0, d1, P.r_rad, eps);
        prows[gy] = ri;
        if (ri.nrings > pmax) pmax = ri.nrings;
    }
    P.tile_rings = tmax;
    P.pg_rings = pmax;
}

void plan_band(Plan& P, double eps) {
    const hg_map& m = P.map;
    double d0 = pix_dec(m, 0), d1 = pix_dec(m, m.ny - 1);
    int32_t lo, cnt;
    ring_range(P.nside, d0, d1, P.r_rad, eps, &lo, &cnt);
    P.ring_lo = lo;
    P.ring_hi = lo + cnt - 1;
    Ring a = hp_ring(P.nside, P.ring_lo), b = hp_ring(P.nside, P.ring_hi);
    P.cell_base = a.first;
    P.n_cells = b.first + b.n - a.first;
}

// Chunk-major entry blocks.  For tile t and chunk c, block b = tile_blk[t] + c
// holds the entries of all 64 pixel groups whose slots fall in the chunk,
// group after group (local order), each group's entries in slot order.  One
// wave per block: lane k is pixel group k of the tile.
__device__ inline int64_t tile_of_block(const int64_t* tile_blk, int64_t ntiles, int64_t b) {
    int64_t lo = 0, hi = ntiles - 1;  // last tile with tile_blk[t] <= b
    while (lo < hi) {
        int64_t mid = (lo + hi + 1) >> 1;
        if (tile_blk[mid] <= b)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

struct BlockLane {
    int64_t tile, c, src, pgb;  // src: run's first bucketed place; pgb: group's first entry
    int n;
};

// lane l of block b (of tile `tile`): group l's run of entries in the block's chunk
__device__ inline BlockLane block_lane_at(int64_t b, int64_t tile, int lane, int32_t npgx,
                                          int32_t npgy, int32_t ntx, const int64_t* tile_blk,
                                          const int64_t* cp_base, const uint32_t* chunk_ptr,
                                          const int64_t* pg_base) {
    BlockLane r;
    r.tile = tile;
    r.c = b - tile_blk[r.tile];
    int64_t nch = tile_blk[r.tile + 1] - tile_blk[r.tile];
    int tx = (int)(r.tile % ntx), ty = (int)(r.tile / ntx);
    int gx = tx * TILE_PGX + lane % TILE_PGX, gy = ty * TILE_PGY + lane / TILE_PGX;
    bool valid = gx < npgx && gy < npgy;
    const uint32_t* cp = chunk_ptr + cp_base[r.tile] + (int64_t)lane * (nch + 1);
    r.n = valid ? (int)(cp[r.c + 1] - cp[r.c]) : 0;
    r.pgb = valid ? pg_base[(int64_t)gy * npgx + gx] : 0;
    r.src = valid ? r.pgb + cp[r.c] : 0;
    return r;
}

__device__ inline BlockLane block_lane(int64_t b, int lane, int32_t npgx, int32_t npgy, int32_t ntx,
                                       int64_t ntiles, const int64_t* tile_blk,
                                       const int64_t* cp_base, const uint32_t* chunk_ptr,
                                       const int64_t* pg_base) {
    return block_lane_at(b, tile_of_block(tile_blk, ntiles, b), lane, npgx, npgy, ntx, tile_blk,
                         cp_base, chunk_ptr, pg_base);
}

// A block's units are its groups' runs cut in fours, group after group; lane l
// holds group l's first unit, run start and length.  For unit i: the group
// holding it (the last l whose first unit is <= i; an empty group shares its
// first unit with the next group), found by a binary search over the wave's
// registers, with that group's run and the unit's place in it.
struct UnitRef {
    int64_t src, pgb;
    int n, t;
};
// src: the run's first place in the bucketed order (pg_base + chunk pointer);
// pgb: the group's first entry
__device__ inline int64_t shfl64(int64_t v, int lane) {
    const uint32_t lo = (uint32_t)v, hi = (uint32_t)((uint64_t)v >> 32);
    return (int64_t)(((uint64_t)(uint32_t)__shfl((int)hi, lane, 64) << 32) |
                     (uint32_t)__shfl((int)lo, lane, 64));
}
__device__ inline UnitRef unit_ref(int i, int first, int64_t src, int64_t pgb, int n) {
    int lo = 0;
#pragma unroll
    for (int step = 32; step > 0; step >>= 1)
        if (__shfl(first, lo + step, 64) <= i) lo += step;  // lo + step <= 63
    UnitRef u;
    u.src = shfl64(src, lo);
    u.pgb = shfl64(pgb, lo);
    u.n = __shfl(n, lo, 64);
    u.t = i - __shfl(first, lo, 64);
    return u;
}

// The four entries of a unit (a run's last unit padded with zero weights and
// its last real slot): slots relative to the chunk's first slot and the
// weights, both through the bucket permutation (its value carries the
// entry's index in the group's list and its position in the chunk; pg_base
// is the group's first entry: a run never spans groups).
__device__ inline void load_unit(const UnitRef& u, const float4* ent_w, const uint32_t* perm,
                                 uint32_t sl[4], float4 w[4]) {
#pragma unroll
    for (int k = 0; k < 4; k++) {
        const int e = 4 * u.t + k;
        const bool real = e < u.n;
        const uint32_t pv = perm[u.src + (real ? e : u.n - 1)];
        sl[k] = pv & PERM_POS_MASK;
        const float4 v = ent_w[u.pgb + (pv >> PERM_POS_BITS)];
        w[k] = real ? v : make_float4(0.f, 0.f, 0.f, 0.f);
    }
}

__global__ __launch_bounds__(256) void k_block_meta(
    int32_t npgx, int32_t npgy, int32_t ntx, int64_t ntiles, int64_t n_blocks,
    const int64_t* __restrict__ tile_blk, const int64_t* __restrict__ cp_base,
    const uint32_t* __restrict__ chunk_ptr, const int64_t* __restrict__ pg_base,
    int64_t* __restrict__ blk_cnt, uint16_t* __restrict__ blk_pgoff, int32_t* __restrict__ blk_tile,
    int* __restrict__ run_max) {
    int64_t b = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    int lane = threadIdx.x & 63;
    if (b >= n_blocks) return;  // uniform per wave
    // launched over a bound on the block count: blocks past the real count
    // (the last tile's end) hold nothing
    if (b >= tile_blk[ntiles]) {
        if (lane == 0) blk_cnt[b] = 0;
        return;
    }
    BlockLane r = block_lane(b, lane, npgx, npgy, ntx, ntiles, tile_blk, cp_base, chunk_ptr,
                             pg_base);
    if (lane == 0) blk_tile[b] = (int32_t)r.tile;
    // the longest (group, chunk) run: the channel kernel holds a run's slots
    // one a lane, so chunks past 64 slots need every run within 64 entries
    int rm = r.n;
    for (int o = 32; o > 0; o >>= 1) rm = max(rm, __shfl_xor(rm, o, 64));
    if (lane == 0 && rm > 64) atomicMax(run_max, rm);
    // units are groups of four entries; a group's run starts on a unit and
    // its last unit is padded: po[l] = 4 x (first unit) + (padding entries)
    const int ng = (r.n + 3) >> 2;
    int x = ng;  // inclusive scan over the 64 groups
    for (int o = 1; o < 64; o <<= 1) {
        int y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    uint16_t* po = blk_pgoff + b * PGOFF_STRIDE;
    po[lane] = (uint16_t)(4 * (x - ng) + (4 * ng - r.n));
    if (lane == 63) {
        po[64] = (uint16_t)(4 * x);
        po[65] = po[66] = po[67] = 0;
        blk_cnt[b] = x;
    }
}

// The group layout of a block as its meta pass wrote it, rebuilt in the
// wave's registers: lane l's first unit (exclusive scan of the groups' unit
// counts) and the block's unit count.
__device__ inline int block_units(int n, int& first) {
    const int ng = (n + 3) >> 2;
    int x = ng;
    for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl_up(x, o, 64);
        if ((threadIdx.x & 63) >= o) x += y;
    }
    first = x - ng;
    return __shfl(x, 63, 64);
}

// Entry-block fills read each group's entries through the bucket permutation,
// so one tile's blocks (its chunks) read the same groups' lists scattered
// over them.  The dispatcher deals workgroups round-robin over the 8 XCDs,
// each with its own L2: the fills launch a multiple of 8 workgroups and
// workgroup w takes run (w mod 8) x (grid / 8) + w / 8, so that runs of
// consecutive blocks, one tile's chunks, read those lists through one L2.
constexpr int FILL_XCDS = 8;
__device__ inline int64_t fill_block(int lane_wave) {
    const int64_t per = gridDim.x / FILL_XCDS;
    const int64_t w = (int64_t)(blockIdx.x % FILL_XCDS) * per + blockIdx.x / FILL_XCDS;
    return w * 4 + lane_wave;
}
inline unsigned fill_grid(int64_t n_blocks) {
    return (unsigned)(((n_blocks + 4 * FILL_XCDS - 1) / (4 * FILL_XCDS)) * FILL_XCDS);
}

// A unit's weight record is NV 16-byte rows, one unit a lane.  Stored from
// registers, each store instruction would write one row a lane, 16 NV bytes
// apart, touching every cache line of the wave's records NV times; through
// LDS (this wave's own NV KB), each store instruction writes 1 KB contiguous.
// Records of units at or past nvalid (relative to the first) are not stored.
template <int NV>
__device__ inline void store_records(uint4* __restrict__ dst, const uint4 (&rec)[NV], int nvalid,
                                     uint4* tw, int lane) {
#pragma unroll
    for (int v = 0; v < NV; v++) tw[lane * NV + v] = rec[v];
    wave_lds_sync();
#pragma unroll
    for (int j = 0; j < NV; j++) {
        const int idx = j * 64 + lane;
        if (idx < nvalid * NV) dst[idx] = tw[idx];
    }
    wave_lds_sync();
}

// One wave per block: lane l knows group l's run (first entry, count); the
// block's units are then written flat, lane i taking units i and i + 64 of
// each pass of 128 (coalesced writes; both units' loads in flight together).
__global__ __launch_bounds__(256) void k_block_fill(
    int32_t npgx, int32_t npgy, int32_t ntx, int64_t n_blocks,
    const int32_t* __restrict__ blk_tile, const int64_t* __restrict__ tile_blk,
    const int64_t* __restrict__ cp_base, const uint32_t* __restrict__ chunk_ptr,
    const int64_t* __restrict__ pg_base, const float4* __restrict__ ent_w,
    const uint32_t* __restrict__ perm,
    const int64_t* __restrict__ blk_base,
    float4* __restrict__ e2_w, uint4* __restrict__ e2_s) {
    __shared__ uint4 sh_rec[4][64 * 4];
    uint4* tw = sh_rec[threadIdx.x >> 6];
    const int64_t b = fill_block(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (b >= n_blocks) return;  // uniform per wave; only wave-level syncs below
    const int64_t base = blk_base[b];
    BlockLane r = block_lane_at(b, blk_tile[b], lane, npgx, npgy, ntx, tile_blk, cp_base,
                                chunk_ptr, pg_base);
    int first;
    const int nu = block_units(r.n, first);
    for (int i0 = 0; i0 < nu; i0 += 128) {  // same trip count on every lane
        const int ia = i0 + lane, ib = ia + 64;
        const UnitRef ua = unit_ref(ia, first, r.src, r.pgb, r.n);
        const UnitRef ub = unit_ref(ib, first, r.src, r.pgb, r.n);
        uint32_t sa[4], sb[4];
        float4 wa[4] = {}, wb[4] = {};
        if (ia < nu) load_unit(ua, ent_w, perm, sa, wa);
        if (ib < nu) load_unit(ub, ent_w, perm, sb, wb);
        if (ia < nu) e2_s[base + ia] = make_uint4(sa[0], sa[1], sa[2], sa[3]);
        if (ib < nu) e2_s[base + ib] = make_uint4(sb[0], sb[1], sb[2], sb[3]);
        // [pixel q][entry k]: pixel q's weights for the unit's four entries
        auto rows = [](const float4 w[4], uint4 (&r)[4]) {
            r[0] = make_uint4(__float_as_uint(w[0].x), __float_as_uint(w[1].x),
                              __float_as_uint(w[2].x), __float_as_uint(w[3].x));
            r[1] = make_uint4(__float_as_uint(w[0].y), __float_as_uint(w[1].y),
                              __float_as_uint(w[2].y), __float_as_uint(w[3].y));
            r[2] = make_uint4(__float_as_uint(w[0].z), __float_as_uint(w[1].z),
                              __float_as_uint(w[2].z), __float_as_uint(w[3].z));
            r[3] = make_uint4(__float_as_uint(w[0].w), __float_as_uint(w[1].w),
                              __float_as_uint(w[2].w), __float_as_uint(w[3].w));
        };
        uint4 r[4];
        rows(wa, r);
        store_records<4>((uint4*)e2_w + (base + i0) * 4, r, nu - i0, tw, lane);
        rows(wb, r);
        store_records<4>((uint4*)e2_w + (base + i0 + 64) * 4, r, nu - i0 - 64, tw, lane);
    }
}

// max over a[0..n) (values below 2^31) into *out, which starts at 0: a
// grid-stride pass, a workgroup reduction, one atomic per workgroup
__global__ __launch_bounds__(256) void k_max_count(const int64_t* __restrict__ a, int64_t n,
                                                   int* __restrict__ out) {
    __shared__ int red[4];
    int m = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        m = max(m, (int)a[i]);
    for (int o = 32; o > 0; o >>= 1) m = max(m, __shfl_xor(m, o, 64));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) atomicMax(out, max(max(red[0], red[1]), max(red[2], red[3])));
}

// Precision forms: the same blocks, counted in groups of four entries (the K
// of the 4x4x4 MFMA).  A group holds four chunk-local slots and the 4 x 4 weights
// [pixel][entry] as BF16 / FP16 bits; a run whose length is not a multiple of
// four is padded with zero weights on its last slot.
__global__ __launch_bounds__(256) void k_block_meta_g(
    int32_t npgx, int32_t npgy, int32_t ntx, int64_t ntiles, int64_t n_blocks,
    const int64_t* __restrict__ tile_blk, const int64_t* __restrict__ cp_base,
    const uint32_t* __restrict__ chunk_ptr, const int64_t* __restrict__ pg_base,
    int64_t* __restrict__ blk_cnt, uint16_t* __restrict__ blk_pgoff, int32_t* __restrict__ blk_tile,
    int* __restrict__ run_max) {
    int64_t b = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    int lane = threadIdx.x & 63;
    if (b >= n_blocks) return;  // uniform per wave
    // launched over a bound on the block count: blocks past the real count
    // (the last tile's end) hold nothing
    if (b >= tile_blk[ntiles]) {
        if (lane == 0) blk_cnt[b] = 0;
        return;
    }
    BlockLane r = block_lane(b, lane, npgx, npgy, ntx, ntiles, tile_blk, cp_base, chunk_ptr,
                             pg_base);
    if (lane == 0) blk_tile[b] = (int32_t)r.tile;
    // the longest (group, chunk) run: the channel kernel holds a run's slots
    // one a lane, so chunks past 64 slots need every run within 64 entries
    int rm = r.n;
    for (int o = 32; o > 0; o >>= 1) rm = max(rm, __shfl_xor(rm, o, 64));
    if (lane == 0 && rm > 64) atomicMax(run_max, rm);
    int ng = (r.n + 3) >> 2;
    int x = ng;
    for (int o = 1; o < 64; o <<= 1) {
        int y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    uint16_t* po = blk_pgoff + b * PGOFF_STRIDE;
    po[lane] = (uint16_t)(x - ng);
    if (lane == 63) {
        po[64] = (uint16_t)x;
        po[65] = po[66] = po[67] = 0;
        blk_cnt[b] = x;
    }
}

__device__ inline uint16_t weight_bits(float w, int32_t prec) {
    if (prec == HG_PREC_MFMA_BF16) return (uint16_t)(__float_as_uint(w) >> 16);  // already rounded
    _Float16 h = (_Float16)w;
    uint16_t u;
    __builtin_memcpy(&u, &h, 2);
    return u;
}

// A unit's weights in the MFMA input type, [pixel q][entry k] halves packed
// in pairs: two 16-byte rows.
__device__ inline void unit_rows_g(const float4 w[4], int32_t prec, uint4 (&r)[2]) {
    const float wk[4][4] = {{w[0].x, w[0].y, w[0].z, w[0].w},
                            {w[1].x, w[1].y, w[1].z, w[1].w},
                            {w[2].x, w[2].y, w[2].z, w[2].w},
                            {w[3].x, w[3].y, w[3].z, w[3].w}};  // [entry][pixel]
    uint32_t wb[8];
#pragma unroll
    for (int j = 0; j < 8; j++) {
        const int q = j >> 1, k = 2 * (j & 1);
        wb[j] = (uint32_t)weight_bits(wk[k][q], prec) |
                ((uint32_t)weight_bits(wk[k + 1][q], prec) << 16);
    }
    r[0] = make_uint4(wb[0], wb[1], wb[2], wb[3]);
    r[1] = make_uint4(wb[4], wb[5], wb[6], wb[7]);
}

// k_block_fill for the 16-bit forms: the same walk over a block's units (groups
// of four entries), weights stored in the MFMA input type.
__global__ __launch_bounds__(256) void k_block_fill_g(
    int32_t npgx, int32_t npgy, int32_t ntx, int64_t n_blocks, int32_t prec,
    const int32_t* __restrict__ blk_tile, const int64_t* __restrict__ tile_blk,
    const int64_t* __restrict__ cp_base, const uint32_t* __restrict__ chunk_ptr,
    const int64_t* __restrict__ pg_base, const float4* __restrict__ ent_w,
    const uint32_t* __restrict__ perm,
    const int64_t* __restrict__ blk_base,
    uint16_t* __restrict__ e3_w, uint4* __restrict__ e3_s) {
    __shared__ uint4 sh_rec[4][64 * 2];
    uint4* tw = sh_rec[threadIdx.x >> 6];
    const int64_t b = fill_block(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (b >= n_blocks) return;  // uniform per wave; only wave-level syncs below
    const int64_t base = blk_base[b];
    BlockLane r = block_lane_at(b, blk_tile[b], lane, npgx, npgy, ntx, tile_blk, cp_base,
                                chunk_ptr, pg_base);
    int first;
    const int nu = block_units(r.n, first);
    for (int i0 = 0; i0 < nu; i0 += 128) {  // same trip count on every lane
        const int ia = i0 + lane, ib = ia + 64;
        const UnitRef ua = unit_ref(ia, first, r.src, r.pgb, r.n);
        const UnitRef ub = unit_ref(ib, first, r.src, r.pgb, r.n);
        uint32_t sa[4], sb[4];
        float4 wa[4] = {}, wb[4] = {};
        if (ia < nu) load_unit(ua, ent_w, perm, sa, wa);
        if (ib < nu) load_unit(ub, ent_w, perm, sb, wb);
        if (ia < nu) e3_s[base + ia] = make_uint4(sa[0], sa[1], sa[2], sa[3]);
        if (ib < nu) e3_s[base + ib] = make_uint4(sb[0], sb[1], sb[2], sb[3]);
        uint4 r[2];
        unit_rows_g(wa, prec, r);
        store_records<2>((uint4*)e3_w + (base + i0) * 2, r, nu - i0, tw, lane);
        unit_rows_g(wb, prec, r);
        store_records<2>((uint4*)e3_w + (base + i0 + 64) * 2, r, nu - i0 - 64, tw, lane);
    }
}

// The sizes the host reads once the entry blocks are laid out, gathered for
// one copy: [0] neighbour pairs, [1] entry units, [2] units in the largest
// block, [3] slots after compaction, [4] chunk pointers, [5] the longest
// (group, chunk) run if over 64 entries (else 0), then the per-tile block
// offsets tile_blk[0 .. ntiles].
constexpr int64_t PACK_HEAD = 6;
__global__ __launch_bounds__(256) void k_pack_sizes(
    const unsigned long long* __restrict__ nnz, const int64_t* __restrict__ units,
    const int* __restrict__ blk_max, const int64_t* __restrict__ slots,
    const int64_t* __restrict__ cps, const int* __restrict__ run_max,
    const int64_t* __restrict__ tile_blk, int64_t ntiles, int64_t* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i <= ntiles) out[PACK_HEAD + i] = tile_blk[i];
    if (i == 0) {
        out[0] = (int64_t)*nnz;
        out[1] = *units;
        out[2] = *blk_max;
        out[3] = *slots;
        out[4] = *cps;
        out[5] = *run_max;
    }
}

// small kernel: gather the totals the host needs to size the second stage
__global__ void k_totals(const uint32_t* cell_off, int64_t n_cells, const int64_t* tile_base,
                         int64_t ntiles, const int64_t* pg_base, int64_t npg,
                         const int64_t* cp_base, const int64_t* tile_blk, const int* flag,
                         int64_t* out) {
    out[0] = cell_off[n_cells];
    out[1] = tile_base[ntiles];
    out[2] = pg_base[npg];
    out[3] = cp_base[ntiles];
    out[4] = *flag;
    out[5] = tile_blk[ntiles];
}

__global__ void k_sorted_coords_dev(const double* __restrict__ ra_deg,
                                    const double* __restrict__ dec_deg,
                                    const uint32_t* __restrict__ srt_idx,
                                    const uint32_t* __restrict__ n_used_dev, int64_t n,
                                    int32_t with_sin, double4* __restrict__ out) {
    int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n || q >= (int64_t)*n_used_dev) return;
    uint32_t k = srt_idx[q];
    double ra = ra_deg[k] * kDeg, dec = dec_deg[k] * kDeg;
    // (RA, Dec, cos Dec, sin Dec or 0): the sine only for the elliptical kernel
    out[q] = make_double4(ra, dec, cos(dec), with_sin ? sin(dec) : 0.0);
}

// Runs the whole setup.  Allocation sizes that depend on the data are read
// back as they are needed (the candidate arrays', the compacted slots' and
// blocks', the entry blocks'), each with one stream synchronisation, and the
// launch order's chunk counts with the one at the end.
hipError_t launch_setup(Plan& P, const double* ra_deg, const double* dec_deg, hipStream_t s,
                        std::string& err, int& status) {
    const double eps = 1e-9;
    status = HG_OK;
    std::vector<RowInfo> trows, prows;
    plan_rows(P, trows, prows, eps);
    if (gather_lds_bytes(2 * (int64_t)P.pg_rings) > (size_t)LDS_BYTES) {
        status = HG_ERR_UNSUPPORTED;
        err = "support spans too many HEALPix rings; use a coarser nside";
        return hipSuccess;
    }
    const int64_t n = P.n;
    const int64_t npc_t = (int64_t)P.tile_rings * 2, npc_p = (int64_t)P.pg_rings * 2;
    int64_t big = std::max<int64_t>(std::max<int64_t>(n, P.n_cells + 1),
                                    std::max<int64_t>(P.npg + 1, P.ntiles + 1));
    int64_t scan_nb = (big + SCAN_B - 1) / SCAN_B + 1;

    DevBuf key, srt2, cnt, cursor, rows_t, sizes, tslots, tcp, tnch, pcap, totals, bcnt, btile, wl;
    HostBuf hbuf;  // page-locked: row tables in, sizes out
    DevBuf used, newpos, ctmp, tbase2, slot2, tpad, tscr, tbase3, slot3, perm;
    // Buffers go back to the allocation cache, where a setup on another
    // stream may take them at once: the stream's work is drained first.
    auto cleanup = [&]() {
        (void)hipStreamSynchronize(s);
        dev_free(used);
        dev_free(newpos);
        dev_free(ctmp);
        dev_free(tbase2);
        dev_free(slot2);
        dev_free(tpad);
        dev_free(tscr);
        dev_free(tbase3);
        dev_free(slot3);
        dev_free(perm);
        dev_free(wl);
        dev_free(tnch);
        dev_free(bcnt);
        dev_free(btile);
        dev_free(key);
        dev_free(srt2);
        dev_free(sizes);
        host_free(hbuf);
        dev_free(cnt);
        dev_free(cursor);
        dev_free(rows_t);
        dev_free(tslots);
        dev_free(tcp);
        dev_free(pcap);
        dev_free(totals);
    };
#define HG_STEP(x)              \
    do {                        \
        hipError_t e_ = (x);    \
        if (e_ != hipSuccess) { \
            cleanup();          \
            return e_;          \
        }                       \
    } while (0)
    const int64_t n1 = n ? n : 1;
    if (P.opts.device_mem_cap > 0) {
        // first-stage footprint, checked before anything is allocated
        size_t need = 64 + (size_t)scan_nb * 8 + 64 + (size_t)n1 * (4 + 4 + 4 + sizeof(double4)) +
                      (size_t)(P.n_cells + 1) * 20 + sizeof(RowInfo) * (trows.size() + prows.size()) +
                      sizeof(int4) * (size_t)(P.ntiles * npc_t + P.npg * npc_p) +
                      sizeof(int64_t) * (size_t)(4 * (P.ntiles + 1) + 2 * (P.npg + 1)) +
                      4 * (size_t)P.npg + 16 * (size_t)P.npix;
        if ((int64_t)need > P.opts.device_mem_cap) {
            status = HG_ERR_NOMEM;
            err = "setup needs at least " + std::to_string(need) + " device bytes, over the cap";
            return hipSuccess;
        }
    }
    HG_STEP(dev_alloc(P.scratch, 64 + (size_t)scan_nb * 8));
    HG_STEP(dev_alloc(totals, 64));
    HG_STEP(dev_alloc(key, (size_t)n1 * 4));
    HG_STEP(dev_alloc(srt2, (size_t)n1 * 4));
    HG_STEP(dev_alloc(cnt, (size_t)(P.n_cells + 1) * 4));
    HG_STEP(dev_alloc(cursor, (size_t)(P.n_cells + 1) * 4));
    HG_STEP(dev_alloc(wl, (size_t)(2 * P.n_cells + 2) * 4));  // two counts, two cell lists
    HG_STEP(dev_alloc(P.cell_off, (size_t)(P.n_cells + 1) * 4));
    HG_STEP(dev_alloc(P.srt_idx, (size_t)n1 * 4));
    HG_STEP(dev_alloc(P.srt_coord, (size_t)n1 * sizeof(double4)));
    HG_STEP(dev_alloc(rows_t, sizeof(RowInfo) * (trows.size() + prows.size())));
    HG_STEP(dev_alloc(P.tile_piece, sizeof(int4) * (size_t)(P.ntiles * npc_t)));
    HG_STEP(dev_alloc(tslots, sizeof(int64_t) * (size_t)(P.ntiles + 1)));
    HG_STEP(dev_alloc(tcp, sizeof(int64_t) * (size_t)(P.ntiles + 1)));
    HG_STEP(dev_alloc(tnch, sizeof(int64_t) * (size_t)(P.ntiles + 1)));
    HG_STEP(dev_alloc(P.tile_blk, sizeof(int64_t) * (size_t)(P.ntiles + 1)));
    HG_STEP(dev_alloc(P.tile_nslots, sizeof(int64_t) * (size_t)(P.ntiles + 1)));
    HG_STEP(dev_alloc(P.cp_base, sizeof(int64_t) * (size_t)(P.ntiles + 1)));
    HG_STEP(dev_alloc(P.pg_piece, sizeof(int4) * (size_t)(P.npg * npc_p)));
    HG_STEP(dev_alloc(pcap, sizeof(int64_t) * (size_t)(P.npg + 1)));
    HG_STEP(dev_alloc(P.pg_base, sizeof(int64_t) * (size_t)(P.npg + 1)));
    HG_STEP(dev_alloc(P.pg_cnt, sizeof(uint32_t) * (size_t)P.npg));
    HG_STEP(dev_alloc(P.pix_count, sizeof(int32_t) * (size_t)P.npix));
    HG_STEP(dev_alloc(P.pix_W, sizeof(double) * (size_t)P.npix));
    HG_STEP(dev_alloc(P.pix_Wf, sizeof(float) * (size_t)P.npix));

    int* flag = (int*)P.scratch.p;
    unsigned long long* nnz_total = (unsigned long long*)((char*)P.scratch.p + 8);
    int* blk_max = (int*)((char*)P.scratch.p + 16);  // most units in one block
    int* run_max = (int*)((char*)P.scratch.p + 32);  // longest run past 64 entries, else 0
    void* scan_tmp = (char*)P.scratch.p + 64;

    {
        ZeroList z{};
        const std::pair<void*, int64_t> bufs[] = {
            {P.scratch.p, 16},
            {cnt.p, P.n_cells + 1},
            {P.pix_count.p, P.npix},
            {P.pix_W.p, 2 * P.npix},
            {P.pix_Wf.p, P.npix},
            {P.pg_cnt.p, P.npg},
            {wl.p, 2},
            {totals.p, 16}};
        int64_t most = 0;
        for (const auto& b : bufs) {
            z.p[z.n] = (uint32_t*)b.first;
            z.dwords[z.n++] = b.second;
            most = std::max(most, b.second);
        }
        hipLaunchKernelGGL(k_zero, dim3(std::max<unsigned>(1, std::min<unsigned>(2048, blocks_for(most, 256)))),
                           dim3(256), 0, s, z);
        HG_STEP(hipGetLastError());
    }
    // the planner's row tables, one copy for both (tile rows, then group
    // rows) from page-locked memory, which also receives the sizes read
    // back below (stream order puts those copies after this one)
    const size_t rows_bytes = sizeof(RowInfo) * (trows.size() + prows.size());
    const size_t back_off = (rows_bytes + 63) / 64 * 64;
    HG_STEP(host_alloc(hbuf, back_off + sizeof(int64_t) * (size_t)(PACK_HEAD + P.ntiles + 1)));
    int64_t* back = (int64_t*)((char*)hbuf.p + back_off);
    std::copy(trows.begin(), trows.end(), (RowInfo*)hbuf.p);
    std::copy(prows.begin(), prows.end(), (RowInfo*)hbuf.p + trows.size());
    HG_STEP(hipMemcpyAsync(rows_t.p, hbuf.p, rows_bytes, hipMemcpyHostToDevice, s));
    const RowInfo* rows_p = (const RowInfo*)rows_t.p + trows.size();

    // 1-3: bin, count, look-up table, scatter, per-cell order, sorted coordinates
    if (n > 0) {
        hipLaunchKernelGGL(k_bin, dim3(blocks_for(n, 256)), dim3(256), 0, s, ra_deg, dec_deg, n,
                           P.nside, P.cell_base, P.n_cells, (uint32_t*)key.p, (uint32_t*)cnt.p,
                           flag);
        HG_STEP(hipGetLastError());
    }
    // the scatter's cursors start as a copy of the cell offsets
    HG_STEP((scan_exclusive<uint32_t, uint32_t>((const uint32_t*)cnt.p, P.n_cells,
                                                (uint32_t*)P.cell_off.p, (uint32_t*)scan_tmp, s,
                                                n > 0 ? (uint32_t*)cursor.p : nullptr)));
    if (n > 0) {
        hipLaunchKernelGGL(k_scatter, dim3(blocks_for(n, 256)), dim3(256), 0, s,
                           (const uint32_t*)key.p, n, (uint32_t*)cursor.p, (uint32_t*)P.srt_idx.p);
        HG_STEP(hipGetLastError());
        // wl: [0] listed cells, [1] big cells, then the two lists
        uint32_t* list = (uint32_t*)wl.p + 2;
        uint32_t* big = list + P.n_cells;
        hipLaunchKernelGGL(k_cell_list, dim3(blocks_for(P.n_cells, 256)), dim3(256), 0, s,
                           (const uint32_t*)P.cell_off.p, P.n_cells, (const uint32_t*)P.srt_idx.p,
                           (uint32_t*)srt2.p, list, (uint32_t*)wl.p);
        HG_STEP(hipGetLastError());
        hipLaunchKernelGGL(k_cell_rank, dim3(RANK_WAVES / 4), dim3(256), 0, s,
                           (const uint32_t*)P.cell_off.p, (const uint32_t*)P.srt_idx.p,
                           (uint32_t*)srt2.p, (const uint32_t*)list, (const uint32_t*)wl.p, big,
                           (uint32_t*)wl.p + 1);
        HG_STEP(hipGetLastError());
        std::swap(P.srt_idx, srt2);
        hipLaunchKernelGGL(k_cell_sort_big, dim3(1024), dim3(BIG_SORT_T), 0, s,
                           (const uint32_t*)P.cell_off.p, (uint32_t*)P.srt_idx.p,
                           (const uint32_t*)big, (const uint32_t*)wl.p + 1);
        HG_STEP(hipGetLastError());
        hipLaunchKernelGGL(k_sorted_coords_dev, dim3(blocks_for(n, 256)), dim3(256), 0, s, ra_deg,
                           dec_deg, (const uint32_t*)P.srt_idx.p,
                           (const uint32_t*)P.cell_off.p + P.n_cells, n,
                           (int32_t)(P.kern.type == HG_KERNEL_ELLIPTICAL),
                           (double4*)P.srt_coord.p);
        HG_STEP(hipGetLastError());
    }
    // 4: planner (geometry and look-up table only)
    {
        int64_t nt = P.ntiles * P.tile_rings;
        hipLaunchKernelGGL(k_tile_plan, dim3(blocks_for(nt, 256)), dim3(256), 0, s,
                           (const RowInfo*)rows_t.p, P.ntx, P.ntiles, P.tile_rings, P.nside,
                           P.cell_base, P.n_cells, (const uint32_t*)P.cell_off.p, P.map, eps,
                           (int4*)P.tile_piece.p, flag);
        HG_STEP(hipGetLastError());
        // totals[6]: the most chunks a tile has before compaction (sizes the
        // bucketing's LDS)
        hipLaunchKernelGGL(k_tile_prefix, dim3(blocks_for(P.ntiles, 256)), dim3(256), 0, s,
                           (int4*)P.tile_piece.p, P.ntiles, P.tile_rings, P.chunk,
                           (int64_t*)tslots.p, (int64_t*)tcp.p, (int64_t*)tnch.p, flag,
                           (int*)((int64_t*)totals.p + 6));
        HG_STEP(hipGetLastError());
        {
            const int64_t* in[] = {(const int64_t*)tnch.p, (const int64_t*)tslots.p,
                                   (const int64_t*)tcp.p};
            int64_t* out[] = {(int64_t*)P.tile_blk.p, (int64_t*)P.tile_nslots.p,
                              (int64_t*)P.cp_base.p};
            HG_STEP(scan_exclusive_many(in, out, 3, P.ntiles, (int64_t*)scan_tmp, s));
        }
        int64_t np = P.npg * P.pg_rings;
        hipLaunchKernelGGL(k_pg_plan, dim3(blocks_for(np, 256)), dim3(256), 0, s,
                           rows_p, (const RowInfo*)rows_t.p, P.npgx, P.npg,
                           P.ntx, P.pg_rings, P.tile_rings, P.nside, P.cell_base,
                           (const uint32_t*)P.cell_off.p, P.map, eps,
                           (const int4*)P.tile_piece.p, (int4*)P.pg_piece.p, flag);
        HG_STEP(hipGetLastError());
        hipLaunchKernelGGL(k_pg_capacity, dim3(blocks_for(P.npg, 256)), dim3(256), 0, s,
                           (const int4*)P.pg_piece.p, P.npg, P.pg_rings, (int64_t*)pcap.p, flag);
        HG_STEP(hipGetLastError());
        HG_STEP((scan_exclusive<int64_t, int64_t>((const int64_t*)pcap.p, P.npg,
                                                  (int64_t*)P.pg_base.p, (int64_t*)scan_tmp, s)));
    }
    hipLaunchKernelGGL(k_totals, dim3(1), dim3(1), 0, s, (const uint32_t*)P.cell_off.p, P.n_cells,
                       (const int64_t*)P.tile_nslots.p, P.ntiles, (const int64_t*)P.pg_base.p,
                       P.npg, (const int64_t*)P.cp_base.p, (const int64_t*)P.tile_blk.p,
                       (const int*)flag, (int64_t*)totals.p);
    HG_STEP(hipGetLastError());
    HG_STEP(hipMemcpyAsync(back, totals.p, 7 * sizeof(int64_t), hipMemcpyDeviceToHost, s));
    HG_STEP(hipStreamSynchronize(s));
    int64_t tot[7];
    std::copy(back, back + 7, tot);
    const int64_t nch_pre_max = tot[6];
    P.n_used = tot[0];
    P.total_slots = tot[1];
    P.ent_cap = tot[2];
    P.chunk_ptrs = tot[3];
    P.n_blocks = tot[5];
    if (tot[4] & 1) {
        status = HG_ERR_ARG;
        err = "sample coordinates must be finite with |dec| <= 90 degrees";
        cleanup();
        return hipSuccess;
    }
    if (tot[4] & 2) {
        status = HG_ERR_UNSUPPORTED;
        err = "a tile holds more than 2^28 candidate samples";
        cleanup();
        return hipSuccess;
    }
    if (tot[4] & 32) {
        status = HG_ERR_UNSUPPORTED;
        err = "a pixel group has 2^25 or more candidate samples";
        cleanup();
        return hipSuccess;
    }
    if (tot[4] & ~(3 | 32)) {
        status = HG_ERR_INTERNAL;
        err = "planner consistency check failed (flag " + std::to_string(tot[4]) + ")";
        cleanup();
        return hipSuccess;
    }
    if (P.opts.device_mem_cap > 0) {
        // slot list, entries, chunk pointers, and the slot compaction's
        // transient arrays (flag, new position, compacted list: 16 B a slot);
        // the entry blocks take 20 B an entry in the FP32 form (12 B in the
        // 16-bit forms) and pad each (group, chunk) run to four entries
        const size_t blk_entry = P.opts.precision == HG_PREC_FP32 ? 20 : 12;
        // (the dealing's padded slot list and the entries' bucketed order add
        // 4 B a slot plus 4 B per tile and chunk slot, and 4 B an entry)
        size_t need = (size_t)P.total_slots * (4 + 16 + 4) + (size_t)P.ntiles * P.chunk * 4 +
                      (size_t)P.ent_cap * (20 + 4 + blk_entry) + (size_t)P.chunk_ptrs * (4 + 60);
        size_t have = 0;
        for (DevBuf* b : {&P.srt_idx, &P.srt_coord, &P.cell_off, &P.tile_piece, &P.tile_nslots,
                          &P.pg_piece, &P.pg_base, &P.pg_cnt, &P.cp_base, &P.pix_count, &P.pix_W,
                          &P.pix_Wf, &P.scratch})
            have += b->bytes;
        if ((int64_t)(need + have) > P.opts.device_mem_cap) {
            status = HG_ERR_NOMEM;
            err = "plan needs " + std::to_string(need + have) + " device bytes, over the cap";
            cleanup();
            return hipSuccess;
        }
    }
    HG_STEP(dev_alloc(P.slot_idx, (size_t)(P.total_slots ? P.total_slots : 1) * 4));
    HG_STEP(dev_alloc(P.ent_slot, (size_t)(P.ent_cap ? P.ent_cap : 1) * 4));
    HG_STEP(dev_alloc(P.ent_w, (size_t)(P.ent_cap ? P.ent_cap : 1) * 16));
    HG_STEP(dev_alloc(P.chunk_ptr, (size_t)(P.chunk_ptrs ? P.chunk_ptrs : 1) * 4));
    // block sizes, then the partial sums of their scan (the block count is
    // not bounded by the scans' shared partial-sum area)
    const int64_t bscan_nb = (P.n_blocks + SCAN_B - 1) / SCAN_B + 1;
    HG_STEP(dev_alloc(bcnt, sizeof(int64_t) * (size_t)(P.n_blocks + 1 + bscan_nb)));
    HG_STEP(dev_alloc(btile, sizeof(int32_t) * (size_t)(P.n_blocks + 1)));
    HG_STEP(dev_alloc(P.blk_base, sizeof(int64_t) * (size_t)(P.n_blocks + 1)));
    HG_STEP(dev_alloc(P.blk_pgoff, sizeof(uint16_t) * PGOFF_STRIDE * (size_t)(P.n_blocks + 1)));

    // 5: candidate slots, neighbour gather, chunk pointers
    // Fields of few pixels and many samples have few tiles and groups, each
    // with long lists: the per-tile and per-group passes over them split each
    // list over more workgroups (a tile's slots are at most its chunk count
    // before compaction times the chunk; a group's candidates average
    // ent_cap / npg).
    const unsigned fill_y = (unsigned)std::min<int64_t>(
        64, std::max<int64_t>(1, nch_pre_max * P.chunk / 4096));
    const unsigned ent_y = (unsigned)std::min<int64_t>(
        16, std::max<int64_t>(1, P.ent_cap / std::max<int64_t>(1, P.npg) / 2048));
    hipLaunchKernelGGL(k_slot_fill, dim3((unsigned)P.ntiles, fill_y), dim3(256), 0, s,
                       (const int4*)P.tile_piece.p, P.tile_rings, (const int64_t*)P.tile_nslots.p,
                       (const uint32_t*)P.srt_idx.p, (uint32_t*)P.slot_idx.p);
    HG_STEP(hipGetLastError());
    {
        const size_t shm = gather_lds_bytes(npc_p);
        const KernelArgs ka = kernel_args(P);
        // every in-support h is at most h_r; below 1e-4 no asin is needed
        const bool small = P.h_r < 1e-4;
        const bool hpx = P.map.proj == HG_PROJ_HEALPIX;
        auto kern = hpx ? gather_kernel<true>(P.kern.type, small)
                        : gather_kernel<false>(P.kern.type, small);
        hipLaunchKernelGGL(kern, dim3(blocks_for(P.npg, GATHER_WAVES)), dim3(64 * GATHER_WAVES),
                           shm, s, (const int4*)P.pg_piece.p, P.pg_rings,
                           (const int64_t*)P.pg_base.p, (const double4*)P.srt_coord.p, P.npgx,
                           P.npg, P.map, P.h_r, ka, P.opts.precision, (uint32_t*)P.ent_slot.p,
                           (float4*)P.ent_w.p, (uint32_t*)P.pg_cnt.p, (int32_t*)P.pix_count.p,
                           (double*)P.pix_W.p, (float*)P.pix_Wf.p);
        HG_STEP(hipGetLastError());
        hipLaunchKernelGGL(k_sum_counts, dim3(256), dim3(256), 0, s,
                           (const int32_t*)P.pix_count.p, P.npix, nnz_total);
        HG_STEP(hipGetLastError());
    }
    // 5b: drop the slots no pixel of their tile uses, recount chunks, deal the
    // slots of each tile over its chunks, and bucket every group's entries by
    // chunk (with the chunk pointers)
    if (P.total_slots > 0) {
        const int64_t ts = P.total_slots;
        const int64_t ts_pad = ts + P.ntiles * (int64_t)P.chunk;  // padding: < chunk a tile
        HG_STEP(dev_alloc(used, (size_t)ts * 4));
        HG_STEP(dev_alloc(newpos, (size_t)(ts + 1) * 8));
        HG_STEP(dev_alloc(ctmp, (size_t)((ts + SCAN_B - 1) / SCAN_B + 1) * 8));
        HG_STEP(dev_alloc(tbase2, sizeof(int64_t) * (size_t)(P.ntiles + 1)));
        HG_STEP(dev_alloc(slot2, (size_t)ts * 4));
        HG_STEP(dev_alloc(tpad, sizeof(int64_t) * (size_t)(P.ntiles + 1)));
        HG_STEP(dev_alloc(tscr, sizeof(int32_t) * (size_t)(P.ntiles + 1)));
        HG_STEP(dev_alloc(tbase3, sizeof(int64_t) * (size_t)(P.ntiles + 1)));
        HG_STEP(dev_alloc(slot3, (size_t)ts_pad * 4));
        HG_STEP(dev_alloc(perm, (size_t)(P.ent_cap ? P.ent_cap : 1) * 4));
        {
            ZeroList z{};
            z.p[0] = (uint32_t*)used.p;
            z.dwords[0] = ts;
            z.n = 1;
            hipLaunchKernelGGL(k_zero, dim3(std::max<unsigned>(1, std::min<unsigned>(2048, blocks_for(ts, 256)))),
                               dim3(256), 0, s, z);
            HG_STEP(hipGetLastError());
        }
        hipLaunchKernelGGL(k_mark_used, dim3(blocks_for(P.npg, 4), ent_y), dim3(256), 0, s, P.npgx, P.npg,
                           P.ntx, (const int64_t*)P.tile_nslots.p, (const int64_t*)P.pg_base.p,
                           (const uint32_t*)P.pg_cnt.p, (const uint32_t*)P.ent_slot.p,
                           (uint32_t*)used.p);
        HG_STEP(hipGetLastError());
        HG_STEP((scan_exclusive<uint32_t, int64_t>((const uint32_t*)used.p, ts,
                                                   (int64_t*)newpos.p, (int64_t*)ctmp.p, s)));
        hipLaunchKernelGGL(k_tile_rebase, dim3(blocks_for(P.ntiles + 1, 256)), dim3(256), 0, s,
                           (const int64_t*)P.tile_nslots.p, P.ntiles, (const int64_t*)newpos.p,
                           P.chunk, (int64_t*)tbase2.p, (int64_t*)tcp.p, (int64_t*)tnch.p,
                           (int64_t*)tpad.p, (int32_t*)tscr.p);
        HG_STEP(hipGetLastError());
        HG_STEP((scan_exclusive<int64_t, int64_t>((const int64_t*)tpad.p, P.ntiles,
                                                  (int64_t*)tbase3.p, (int64_t*)scan_tmp, s)));
        hipLaunchKernelGGL(k_remap_entries, dim3(blocks_for(P.npg, 4), ent_y), dim3(256), 0, s, P.npgx,
                           P.npg, P.ntx, P.chunk, (const int64_t*)P.tile_nslots.p,
                           (const int64_t*)tbase2.p, (const int64_t*)tnch.p,
                           (const int32_t*)tscr.p, (const int64_t*)P.pg_base.p,
                           (const uint32_t*)P.pg_cnt.p, (const int64_t*)newpos.p,
                           (uint32_t*)P.ent_slot.p);
        HG_STEP(hipGetLastError());
        hipLaunchKernelGGL(k_compact_slots, dim3(blocks_for(ts, 256)), dim3(256), 0, s,
                           (const uint32_t*)used.p, (const int64_t*)newpos.p, ts,
                           (const uint32_t*)P.slot_idx.p, (uint32_t*)slot2.p);
        HG_STEP(hipGetLastError());
        hipLaunchKernelGGL(k_deal_slots, dim3((unsigned)P.ntiles), dim3(256), 0, s,
                           (const int64_t*)tbase2.p, (const int64_t*)tbase3.p,
                           (const int64_t*)tnch.p, (const int32_t*)tscr.p, P.chunk,
                           (const uint32_t*)slot2.p, (uint32_t*)slot3.p);
        HG_STEP(hipGetLastError());
        // the dealt slot lists and their tile offsets replace the plan's (the
        // old buffers go back to the cache with the transients)
        std::swap(P.slot_idx, slot3);
        std::swap(P.tile_nslots, tbase3);
        {
            const int64_t* in[] = {(const int64_t*)tnch.p, (const int64_t*)tcp.p};
            int64_t* out[] = {(int64_t*)P.tile_blk.p, (int64_t*)P.cp_base.p};
            HG_STEP(scan_exclusive_many(in, out, 2, P.ntiles, (int64_t*)scan_tmp, s));
        }
        // LDS for the largest dealt tile only (not the dealt limit), so that
        // more groups' waves are resident on the usual workloads
        const int32_t words = (int32_t)std::max<int64_t>(
            1, std::min<int64_t>(SCRAMBLE_MAX_WORDS, nch_pre_max * chunk_words(P.chunk)));
        // groups of many candidates (dense fields) take a workgroup each
        const bool wide = P.ent_cap / std::max<int64_t>(1, P.npg) >= 4096;
        const size_t bshm =
            (size_t)(wide ? 1 : BUCKET_WAVES) * words * (sizeof(unsigned long long) + 4);
        hipLaunchKernelGGL(wide ? k_bucket_entries<true> : k_bucket_entries<false>,
                           dim3(wide ? (unsigned)P.npg : blocks_for(P.npg, BUCKET_WAVES)),
                           dim3(64 * BUCKET_WAVES), bshm, s, P.npgx, P.npg, P.ntx, P.chunk,
                           (const int64_t*)P.tile_blk.p, (const int32_t*)tscr.p,
                           (const int64_t*)P.cp_base.p, (const int64_t*)P.pg_base.p,
                           (const uint32_t*)P.pg_cnt.p, (const uint32_t*)P.ent_slot.p,
                           (uint32_t*)P.chunk_ptr.p, (uint32_t*)perm.p, words);
        HG_STEP(hipGetLastError());
    } else {
        hipLaunchKernelGGL(k_chunk_ptr, dim3(blocks_for(P.npg, 4)), dim3(256), 0, s, P.npgx,
                           P.npg, P.ntx, P.chunk, (const int64_t*)P.tile_nslots.p,
                           (const int64_t*)P.cp_base.p, (const int64_t*)P.pg_base.p,
                           (const uint32_t*)P.pg_cnt.p, (const uint32_t*)P.ent_slot.p,
                           (uint32_t*)P.chunk_ptr.p);
        HG_STEP(hipGetLastError());
        // no slots, no entries: the block fills read no entry
        HG_STEP(dev_alloc(perm, 4));
    }
    // chunk-major blocks for the channel kernels.  P.n_blocks still holds the
    // count before compaction, a bound on the real one: the meta pass and
    // the scan run over the bound (blocks past the real count hold nothing),
    // so every size is read back with one synchronisation.
    const bool grouped = P.opts.precision != HG_PREC_FP32;
    const bool compacted = P.total_slots > 0;
    if (P.n_blocks > 0) {
        hipLaunchKernelGGL(grouped ? k_block_meta_g : k_block_meta, dim3(blocks_for(P.n_blocks, 4)),
                           dim3(256), 0, s, P.npgx, P.npgy, P.ntx, P.ntiles, P.n_blocks,
                           (const int64_t*)P.tile_blk.p, (const int64_t*)P.cp_base.p,
                           (const uint32_t*)P.chunk_ptr.p, (const int64_t*)P.pg_base.p,
                           (int64_t*)bcnt.p, (uint16_t*)P.blk_pgoff.p, (int32_t*)btile.p,
                           run_max);
        HG_STEP(hipGetLastError());
        // the largest block sizes the channel kernel's LDS entry area (an
        // atomic per block in the meta pass, read first to skip smaller
        // counts, made that pass three times slower)
        hipLaunchKernelGGL(k_max_count, dim3(256), dim3(256), 0, s, (const int64_t*)bcnt.p,
                           P.n_blocks, blk_max);
        HG_STEP(hipGetLastError());
    }
    HG_STEP((scan_exclusive<int64_t, int64_t>((const int64_t*)bcnt.p, P.n_blocks,
                                              (int64_t*)P.blk_base.p,
                                              (int64_t*)bcnt.p + P.n_blocks + 1, s)));
    HG_STEP(dev_alloc(sizes, sizeof(int64_t) * (size_t)(PACK_HEAD + P.ntiles + 1)));
    hipLaunchKernelGGL(k_pack_sizes, dim3(blocks_for(P.ntiles + 1, 256)), dim3(256), 0, s,
                       (const unsigned long long*)nnz_total, (const int64_t*)P.blk_base.p + P.n_blocks,
                       (const int*)blk_max, (const int64_t*)P.tile_nslots.p + P.ntiles,
                       (const int64_t*)P.cp_base.p + P.ntiles, (const int*)run_max,
                       (const int64_t*)P.tile_blk.p, P.ntiles, (int64_t*)sizes.p);
    HG_STEP(hipGetLastError());
    HG_STEP(hipMemcpyAsync(back, sizes.p, sizeof(int64_t) * (size_t)(PACK_HEAD + P.ntiles + 1),
                           hipMemcpyDeviceToHost, s));
    HG_STEP(hipStreamSynchronize(s));
    // The compaction's transient arrays go back to the allocation cache only
    // now that the stream has drained: a setup on another stream (a batch
    // sets fields up in parallel) may take them at once.
    for (DevBuf* b : {&slot2, &slot3, &used, &newpos, &ctmp, &tbase2, &tpad, &tscr, &tbase3})
        dev_free(*b);
    // per-tile block offsets: the channel kernel's launch order
    P.tile_blk_host.assign(back + PACK_HEAD, back + PACK_HEAD + P.ntiles + 1);
    if (compacted) {
        // the buffers were sized for the counts before compaction, which bound these
        P.total_slots = back[3];
        P.n_blocks = P.tile_blk_host[(size_t)P.ntiles];
        P.chunk_ptrs = back[4];
    }
    P.nnz = back[0];
    P.nnz_entries = back[1];
    P.blk_max = (int)back[2];
    P.run_max = (int)back[5];
    const int64_t n_ent = P.nnz_entries;
    // a chunk length the channel kernel cannot stage is rebuilt shorter by
    // the caller: the entry blocks are not filled
    if (!channel_lds_fits(grouped, P.chunk, P.blk_max) || !channel_runs_fit(P.chunk, P.run_max)) {
        cleanup();
        return hipSuccess;
    }
    if (grouped) {
        HG_STEP(dev_alloc(P.e3_w, (size_t)(n_ent ? n_ent : 1) * 32));
        HG_STEP(dev_alloc(P.e3_s, (size_t)(n_ent ? n_ent : 1) * 16));
        if (P.n_blocks > 0) {
            hipLaunchKernelGGL(k_block_fill_g, dim3(fill_grid(P.n_blocks)), dim3(256), 0, s,
                               P.npgx, P.npgy, P.ntx, P.n_blocks, P.opts.precision,
                               (const int32_t*)btile.p, (const int64_t*)P.tile_blk.p,
                               (const int64_t*)P.cp_base.p, (const uint32_t*)P.chunk_ptr.p,
                               (const int64_t*)P.pg_base.p, (const float4*)P.ent_w.p,
                               (const uint32_t*)perm.p,
                               (const int64_t*)P.blk_base.p,
                               (uint16_t*)P.e3_w.p, (uint4*)P.e3_s.p);
            HG_STEP(hipGetLastError());
        }
    } else {
        HG_STEP(dev_alloc(P.e2_w, (size_t)(n_ent ? n_ent : 1) * 64));
        HG_STEP(dev_alloc(P.e2_s, (size_t)(n_ent ? n_ent : 1) * 16));
        if (P.n_blocks > 0) {
            hipLaunchKernelGGL(k_block_fill, dim3(fill_grid(P.n_blocks)), dim3(256), 0, s,
                               P.npgx, P.npgy, P.ntx, P.n_blocks,
                               (const int32_t*)btile.p, (const int64_t*)P.tile_blk.p,
                               (const int64_t*)P.cp_base.p, (const uint32_t*)P.chunk_ptr.p,
                               (const int64_t*)P.pg_base.p, (const float4*)P.ent_w.p,
                               (const uint32_t*)perm.p,
                               (const int64_t*)P.blk_base.p,
                               (float4*)P.e2_w.p, (uint4*)P.e2_s.p);
            HG_STEP(hipGetLastError());
        }
    }
    cleanup();
    return hipSuccess;
#undef HG_STEP
}

}  // namespace hg
