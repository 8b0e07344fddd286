// Channel phase of libhegrid: the weighted sums of Eq. (1) for many channels
// against a plan built once by setup (channels are independent, Sec. 4.2; the
// neighbour structure is shared by all of them, Sec. 4.3.1).
//
// For each pixel p and channel c:  S[c,p] = sum_{n in N(p)} w[p,n] v[n,c],
// V[c,p] = S[c,p] / W_p.  This is a sparse (pixels x samples) by dense
// (samples x channels) product.  Layout of the work:
//
//   * a workgroup of WAVES waves (8 or 16) owns one tile (16 x 16 pixels =
//     8 x 8 pixel groups of 2 x 2) and one block of 64 G channels (G = 1, 2
//     or 4); WAVES and G are the kernel's shape, chosen per launch (the
//     plan's entry blocks do not depend on them);
//   * the tile's candidate samples (its slots) are processed in chunks of
//     `chunk` slots.  For each chunk the workgroup stages, in LDS, the block's
//     channels of every slot (one row per sample, read from the
//     channel-contiguous values in HBM) and the chunk's entry block (the
//     entries of all 64 groups, prepared by setup);
//   * staging is pipelined: the copies of later chunks go straight from
//     global memory to LDS (global_load_lds) while the waves compute the
//     current one;
//   * each wave owns 64 / WAVES pixel groups spread over the tile.  The MFMA
//     rows are a group's four pixels (A = their weights) and the columns are
//     the block's channels, G l + g for the g-th instruction (B = values);
//       - FP32 form: v_mfma_f32_4x4x1_16b_f32, one sample per instruction;
//       - BF16 / FP16 forms: v_mfma_f32_4x4x4_16b_{bf16,f16}, four samples
//         (one group of four entries) per instruction, FP32 accumulation;
//   * summation is two-level: each chunk's entries accumulate into a fresh
//     MFMA tile that is then added to the group's FP32 total, so no serial
//     FP32 chain is longer than one chunk;
//   * the epilogue divides by the FP32 weight sum and writes [c][j][i] as
//     rows of 16 pixels after a transpose through LDS.
#include "hg_common.h"

namespace hg {
namespace {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef short v4s __attribute__((ext_vector_type(4)));
typedef _Float16 v4h __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) void lds_void;
#define CONST_AS __attribute__((address_space(4)))

static_assert(TILE_PGX == 8 && TILE_PGY == 8, "wave/group mapping assumes 8 x 8 groups");
constexpr int TILE_PX = TILE_PGX * PG;  // 16 pixels per tile side

constexpr int FORM_F32 = 0;  // FP32 values in LDS, one entry per MFMA
constexpr int FORM_M16 = 1;  // 16-bit values in LDS, groups of four entries per MFMA

// Longest chunk a form stages: the FP32 form's 1 KB rows fill LDS with two
// chunks of 64; the 16-bit forms' rows are half as long.
template <int FORM>
constexpr int max_chunk() {
    return FORM == FORM_F32 ? 64 : MAX_CHUNK;
}

template <int FORM, int G>
struct Form {
    static constexpr int VB = FORM == FORM_F32 ? 4 : 2;   // bytes per staged value
    static constexpr int CW = 64 * G;                      // channels per workgroup
    static constexpr int RB = CW * VB;                     // bytes per staged row
    static constexpr int RPI = 1024 / RB;                  // rows per copy (16 B a lane)
    static constexpr int LPR = 64 / RPI;                   // lanes per row of a copy
    // a unit is a group of four entries of one pixel group: weights [pixel][entry]
    static constexpr int WB = FORM == FORM_F32 ? 64 : 32;  // weight bytes per unit
    static constexpr int SB = 16;                          // slot bytes per unit
    static constexpr int OCW = CW < 128 ? CW : 128;        // channels per epilogue pass
    static constexpr int OUT_STRIDE = OCW + 4;             // LDS floats per pixel there
};

// Per wave: the staged rows of a chunk come in row groups of RPI adjacent
// slots (one copy instruction each); wave w takes row groups w, w + WAVES, ...
template <int FORM, int G, int WAVES>
struct Rows {
    static constexpr int RPI = Form<FORM, G>::RPI;
    static constexpr int GPW = (max_chunk<FORM>() / RPI + WAVES - 1) / WAVES;  // row groups per wave
    static constexpr int NRW = GPW * RPI;                              // rows per wave
};

// One staged chunk in LDS: `chunk` value rows, then the entry block (weights,
// slots) for up to `ucap` units, then the 65 per-group offsets.  ucap is the
// plan's largest block (a multiple of 4), so a chunk takes what the plan needs
// rather than the 64 x chunk worst case, and more chunks fit in flight.
constexpr int MAX_NBUF = 4;
// Chunk metadata ring: two halves of 16 chunks, each chunk's staged-row sample
// indices (up to the form's longest chunk, uint32) and the 17 entry-block
// offsets of a half.
constexpr int META_RUN = 16;
template <int FORM>
constexpr int meta_rows() {
    return 2 * META_RUN * max_chunk<FORM>() * 4;
}
template <int FORM>
constexpr int meta_lds() {
    return meta_rows<FORM>() + 2 * (META_RUN + 1) * 8 + TILE_PGS;  // + the group map
}
inline int meta_lds(bool m16) { return m16 ? meta_lds<FORM_M16>() : meta_lds<FORM_F32>(); }

struct LdsLayout {
    int vals, ew, es, po, stride;
    __device__ __host__ static LdsLayout make(int rb, int wb, int chunk, int ucap) {
        LdsLayout L;
        L.vals = 0;
        L.ew = L.vals + chunk * rb;
        L.es = L.ew + ucap * wb;
        L.po = L.es + ucap * 16;
        L.stride = L.po + 144;
        return L;
    }
};

// Direct global -> LDS copies (lane i writes bytes [i*size, (i+1)*size) after
// the wave-uniform LDS address).  They are issued through inline assembly so
// that the compiler does not order every later LDS read behind them: the
// kernel itself waits for them (s_waitcnt vmcnt) before the barrier that hands
// a staged chunk to the compute loop.  No output register is involved: the
// data goes to LDS only.
__device__ inline uint32_t lds_addr(const char* l) {
    return __builtin_amdgcn_readfirstlane((uint32_t)(uintptr_t)(lds_void*)l);
}
// The global address is a wave-uniform 64-bit base in scalar registers plus a
// 32-bit per-lane byte offset, so the lane part of the address costs one VGPR.
__device__ inline const void* uniform_ptr(const void* p) {
    uint64_t u = (uint64_t)(uintptr_t)p;
    uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)u);
    uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(u >> 32));
    return (const void*)(uintptr_t)(((uint64_t)hi << 32) | lo);
}
__device__ inline void dma16s(const void* base, uint32_t voff, const char* l) {
    asm volatile("s_mov_b32 m0, %2\n\ts_nop 1\n\tglobal_load_lds_dwordx4 %0, %1"
                 :
                 : "v"(voff), "s"(uniform_ptr(base)), "s"(lds_addr(l))
                 : "memory", "m0");
}
// The same with a per-lane 64-bit address: one copy serves several rows.
__device__ inline void dma16v(const void* addr, const char* l) {
    asm volatile("s_mov_b32 m0, %1\n\ts_nop 1\n\tglobal_load_lds_dwordx4 %0, off"
                 :
                 : "v"(addr), "s"(lds_addr(l))
                 : "memory", "m0");
}
__device__ inline void dma4s(const void* base, uint32_t voff, const char* l) {
    asm volatile("s_mov_b32 m0, %2\n\ts_nop 1\n\tglobal_load_lds_dword %0, %1"
                 :
                 : "v"(voff), "s"(uniform_ptr(base)), "s"(lds_addr(l))
                 : "memory", "m0");
}

__device__ inline float bf16_bits_to_f32(uint32_t b) { return __uint_as_float(b << 16); }

__device__ inline float f16_bits_to_f32(uint32_t b) {
    _Float16 h;
    uint16_t u = (uint16_t)b;
    __builtin_memcpy(&h, &u, 2);
    return (float)h;
}

// One row group: RPI adjacent staged rows of RB bytes, lane l covering 16
// bytes of row l / LPR at byte offset 16 (l % LPR).  row: this lane's sample
// index (read from the chunk's metadata in LDS); r, the rows present (the
// group's last rows may be beyond the chunk).  DMA: one copy straight to LDS.
// Otherwise (values that need a conversion, are misaligned or end inside the
// block) through registers, channels past nchan read as 0.
template <int FORM, int G, int DT, bool VEC>
__device__ inline void stage_group(char* dst, const void* values, int64_t ld, int32_t nchan,
                                   int c_lo, uint32_t row, int r, int lane, bool dma) {
    typedef Form<FORM, G> F;
    const int rl = lane / F::LPR, pc = lane % F::LPR;
    if (rl >= r) return;
    if (dma) {
        // the element size equals the staged size here (FP32 from FP32, or 16-bit)
        const char* src = (const char*)values + ((int64_t)row * ld + c_lo) * F::VB + 16 * pc;
        dma16v(src, dst);
        return;
    }
    char* d = dst + lane * 16;
    if (FORM == FORM_F32) {
        const int c = c_lo + 4 * pc;  // this lane's four channels
        float f[4] = {0.f, 0.f, 0.f, 0.f};
        if (DT == HG_F32) {
            const float* src = (const float*)values + (int64_t)row * ld;
            if (VEC && c + 3 < nchan) {
                const float4 v = *(const float4*)(src + c);
                f[0] = v.x;
                f[1] = v.y;
                f[2] = v.z;
                f[3] = v.w;
            } else {
                for (int k = 0; k < 4; k++)
                    if (c + k < nchan) f[k] = src[c + k];
            }
        } else {
            const uint16_t* src = (const uint16_t*)values + (int64_t)row * ld;
            uint32_t u[4] = {0, 0, 0, 0};
            if (VEC && c + 3 < nchan) {
                const uint2 raw = *(const uint2*)(src + c);
                u[0] = raw.x & 0xFFFF;
                u[1] = raw.x >> 16;
                u[2] = raw.y & 0xFFFF;
                u[3] = raw.y >> 16;
            } else {
                for (int k = 0; k < 4; k++)
                    if (c + k < nchan) u[k] = src[c + k];
            }
#pragma unroll
            for (int k = 0; k < 4; k++)
                f[k] = (DT == HG_BF16) ? bf16_bits_to_f32(u[k]) : f16_bits_to_f32(u[k]);
        }
        *(float4*)d = make_float4(f[0], f[1], f[2], f[3]);
    } else {
        const int c = c_lo + 8 * pc;  // eight 16-bit channels
        const uint16_t* src = (const uint16_t*)values + (int64_t)row * ld + c;
        uint32_t u[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        if (VEC && c + 7 < nchan) {
            const uint4 raw = *(const uint4*)src;
            u[0] = raw.x & 0xFFFF;
            u[1] = raw.x >> 16;
            u[2] = raw.y & 0xFFFF;
            u[3] = raw.y >> 16;
            u[4] = raw.z & 0xFFFF;
            u[5] = raw.z >> 16;
            u[6] = raw.w & 0xFFFF;
            u[7] = raw.w >> 16;
        } else {
            for (int k = 0; k < 8; k++)
                if (c + k < nchan) u[k] = src[k];
        }
        *(uint4*)d = make_uint4(u[0] | (u[1] << 16), u[2] | (u[3] << 16), u[4] | (u[5] << 16),
                                u[6] | (u[7] << 16));
    }
}

// FP32 form: this lane's G values of one staged row, and the G MFMAs of one
// entry (A = this lane's pixel's weight, column block g = channel G l + g).
template <int G>
struct VF;
template <>
struct VF<4> {
    typedef float4 T;
    __device__ static float at(const T& v, int g) { return g == 0 ? v.x : g == 1 ? v.y : g == 2 ? v.z : v.w; }
};
template <>
struct VF<2> {
    typedef float2 T;
    __device__ static float at(const T& v, int g) { return g == 0 ? v.x : v.y; }
};
template <>
struct VF<1> {
    typedef float T;
    __device__ static float at(const T& v, int) { return v; }
};

template <int G>
__device__ inline void mfma_f32(v4f* part, float a, const typename VF<G>::T& v) {
#pragma unroll
    for (int g = 0; g < G; g++)
        part[g] = __builtin_amdgcn_mfma_f32_4x4x1f32(a, VF<G>::at(v, g), part[g], 0, 0, 0);
}

// 16-bit forms: this lane's G values of one staged row as raw bits.
template <int G>
struct VH;
template <>
struct VH<4> {
    typedef uint2 T;
};
template <>
struct VH<2> {
    typedef uint32_t T;
};
template <>
struct VH<1> {
    typedef uint16_t T;
};

// One group of four entries on the 16-bit MFMA.  a: this lane's pixel's four
// weights (entries 0..3); v0..v3: this lane's G channels of the four entries'
// samples.  Column block g takes channel G l + g of each entry:
// B_g = {v0[g], v1[g], v2[g], v3[g]}.
template <int DT, int G>
__device__ inline void mfma_16(v4f* part, uint2 a, const typename VH<G>::T& v0,
                               const typename VH<G>::T& v1, const typename VH<G>::T& v2,
                               const typename VH<G>::T& v3) {
    uint2 b[G];
    if constexpr (G == 4) {
        b[0] = make_uint2(__builtin_amdgcn_perm(v1.x, v0.x, 0x05040100u),
                          __builtin_amdgcn_perm(v3.x, v2.x, 0x05040100u));
        b[1] = make_uint2(__builtin_amdgcn_perm(v1.x, v0.x, 0x07060302u),
                          __builtin_amdgcn_perm(v3.x, v2.x, 0x07060302u));
        b[2] = make_uint2(__builtin_amdgcn_perm(v1.y, v0.y, 0x05040100u),
                          __builtin_amdgcn_perm(v3.y, v2.y, 0x05040100u));
        b[3] = make_uint2(__builtin_amdgcn_perm(v1.y, v0.y, 0x07060302u),
                          __builtin_amdgcn_perm(v3.y, v2.y, 0x07060302u));
    } else if constexpr (G == 2) {
        b[0] = make_uint2(__builtin_amdgcn_perm(v1, v0, 0x05040100u),
                          __builtin_amdgcn_perm(v3, v2, 0x05040100u));
        b[1] = make_uint2(__builtin_amdgcn_perm(v1, v0, 0x07060302u),
                          __builtin_amdgcn_perm(v3, v2, 0x07060302u));
    } else {
        b[0] = make_uint2((uint32_t)v0 | ((uint32_t)v1 << 16), (uint32_t)v2 | ((uint32_t)v3 << 16));
    }
#pragma unroll
    for (int g = 0; g < G; g++) {
        if (DT == HG_BF16) {
            v4s A, B;
            __builtin_memcpy(&A, &a, 8);
            __builtin_memcpy(&B, &b[g], 8);
            part[g] = __builtin_amdgcn_mfma_f32_4x4x4bf16_1k(A, B, part[g], 0, 0, 0);
        } else {
            v4h A, B;
            __builtin_memcpy(&A, &a, 8);
            __builtin_memcpy(&B, &b[g], 8);
            part[g] = __builtin_amdgcn_mfma_f32_4x4x4f16(A, B, part[g], 0, 0, 0);
        }
    }
}

// Wait until at most k of this wave's copies are outstanding, for a
// wave-uniform k.  The counter field of s_waitcnt is an immediate, so k is
// rounded down to 0, 1, 2, 4, 8, 16 or 32 (waiting for a little more than
// needed).  vmcnt is 6 bits: [3:0] and [15:14]; expcnt and lgkmcnt left open.
__device__ inline void wait_copies(int k) {
    if (k >= 32)
        __builtin_amdgcn_s_waitcnt(0x8F70);  // vmcnt(32)
    else if (k >= 16)
        __builtin_amdgcn_s_waitcnt(0x4F70);  // vmcnt(16)
    else if (k >= 8)
        __builtin_amdgcn_s_waitcnt(0x0F78);  // vmcnt(8)
    else if (k >= 4)
        __builtin_amdgcn_s_waitcnt(0x0F74);  // vmcnt(4)
    else if (k >= 2)
        __builtin_amdgcn_s_waitcnt(0x0F72);  // vmcnt(2)
    else if (k >= 1)
        __builtin_amdgcn_s_waitcnt(0x0F71);  // vmcnt(1)
    else
        __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0)
}

// Wave w's class of pixel groups: with 16 waves, four groups of one
// (x mod 4, y mod 4) class; with 8 waves, eight of one (x mod 4, y mod 2)
// class.  A chunk's samples are spatially compact, so classes spread each
// chunk's entries over the waves.  The waves that share a SIMD (w mod 4
// equal) take different x classes, so the chunk's matrix work also splits
// evenly over the SIMDs.
template <int WAVES>
__device__ inline void wave_group(int wave, int k, int& lx, int& ly) {
    if (WAVES == 16) {
        lx = ((wave - (wave >> 2)) & 3) + 4 * (k & 1);
        ly = (wave >> 2) + 4 * (k >> 1);
    } else {
        lx = ((wave + (wave >> 2)) & 3) + 4 * (k & 1);
        ly = (wave >> 2) + 2 * (k >> 1);
    }
}

template <int FORM, int DT, bool VEC, int WAVES, int G>
__device__ __attribute__((always_inline)) inline void grid_item(
    const void* __restrict__ values, int64_t ld, int32_t nchan, int32_t npgx, int32_t npgy,
    int32_t ntx, int32_t nx, int32_t ny, int32_t chunk, const int64_t* __restrict__ tile_base,
    const uint32_t* __restrict__ slot_idx, const int64_t* __restrict__ tile_blk,
    const int64_t* __restrict__ blk_base, const uint16_t* __restrict__ blk_pgoff,
    const void* __restrict__ ent_w, const void* __restrict__ ent_s,
    const float* __restrict__ pix_Wf, float* __restrict__ out, int32_t out_vec, int32_t ucap,
    int32_t nbuf, const uint32_t* __restrict__ pg_cnt, int32_t balance, int64_t tile, int64_t cb,
    char* smem) {
    typedef Form<FORM, G> F;
    typedef Rows<FORM, G, WAVES> RW;
    constexpr int THREADS = 64 * WAVES;
    constexpr int PGW = TILE_PGS / WAVES;  // pixel groups per wave
    // the FP32 form reads the next unit ahead of this unit's MFMAs where the
    // registers allow it (16 waves of 256 channels have 128 registers a lane,
    // which the accumulators and one unit's operands already take)
    constexpr bool PIPE = !(FORM == FORM_F32 && WAVES == 16 && G == 4);
    const LdsLayout L = LdsLayout::make(F::RB, F::WB, chunk, ucap);
    int tx = (int)(tile % ntx), ty = (int)(tile / ntx);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int c_lo = (int)cb * F::CW;
    // value rows go straight to LDS when they need no conversion, are aligned
    // and are complete
    const bool dma_rows = (FORM == FORM_F32 ? DT == HG_F32 : true) && VEC && c_lo + F::CW <= nchan;

    const int64_t s_base = tile_base[tile];
    const int64_t nslots = tile_base[tile + 1] - s_base;
    const int64_t blk0 = tile_blk[tile];
    const int64_t nch = tile_blk[tile + 1] - blk0;
    const uint32_t* sidx = slot_idx + s_base;

    char* ring_rows = smem + nbuf * L.stride;
    constexpr int MAXC = max_chunk<FORM>();
    char* ring_blk = ring_rows + meta_rows<FORM>();
    uint8_t* gmap = (uint8_t*)(ring_blk + 2 * (META_RUN + 1) * 8);
    // Which pixel groups each wave owns.  Balanced: within each quadrant of
    // 4 x 4 groups, the groups are ranked by their entry count (all chunks)
    // and dealt to the waves in snake order, the direction alternating from
    // quadrant to quadrant, so every wave keeps one group (16 waves) or two
    // (8 waves) of every quadrant -- the spread over the tile that shares a
    // chunk's work out -- while the waves' totals even out (drift scans put
    // stripes of dense rows across a tile).  Otherwise (the default) the
    // fixed classes of wave_group: dealt chunks already spread each group's
    // entries evenly over the tile's chunks.
    if (balance) {
        if (wave == 0) {
            const int gx = tx * TILE_PGX + (lane & 7), gy = ty * TILE_PGY + (lane >> 3);
            const int c = gx < npgx && gy < npgy ? (int)pg_cnt[(int64_t)gy * npgx + gx] : -1;
            const int q = ((lane >> 5) << 1) | ((lane >> 2) & 1);  // quadrant of group `lane`
            int rank = 0;
#pragma unroll
            for (int j = 0; j < TILE_PGS; j++) {
                const int cj = __builtin_amdgcn_readlane(c, j);
                const int qj = ((j >> 5) << 1) | ((j >> 2) & 1);
                rank += qj == q && (cj > c || (cj == c && j < lane));
            }
            constexpr int PER_Q = 16 / WAVES;  // groups of a quadrant per wave
            const int jj = rank / WAVES, ii = rank % WAVES;
            const int w = ((q + jj) & 1) ? WAVES - 1 - ii : ii;
            gmap[w * PGW + q * PER_Q + jj] = (uint8_t)lane;
        }
        __syncthreads();
    }
    bool pv[PGW];
    int lxs[PGW], lys[PGW];
#pragma unroll
    for (int k = 0; k < PGW; k++) {
        if (balance) {
            const int g = gmap[wave * PGW + k];
            lxs[k] = g & 7;
            lys[k] = g >> 3;
        } else {
            wave_group<WAVES>(wave, k, lxs[k], lys[k]);
        }
        pv[k] = tx * TILE_PGX + lxs[k] < npgx && ty * TILE_PGY + lys[k] < npgy;
    }

    // The chunk metadata (the staged rows' sample indices and the entry
    // block's extent) reaches LDS through the same asynchronous copies as the
    // data, sixteen chunks at a time into one half of a two-half ring, long
    // before it is read; the loop issues no scalar loads, whose latency the
    // LDS waits of the compute phase would otherwise absorb.  The vector
    // memory counter thus only counts copies, which the pipeline waits for
    // explicitly.
    struct Meta {
        const uint32_t* rr;  // the chunk's staged-row sample indices in the ring (LDS)
        int nrows, ne;       // rows of this wave's groups present in the chunk; units
        int64_t blk, eb;
    };
    // staged slot of this wave's t-th row
    auto row_slot = [&](int t) { return F::RPI * (wave + WAVES * (t / F::RPI)) + t % F::RPI; };
    auto rd64 = [&](const char* p) {
        uint32_t lo = __builtin_amdgcn_readfirstlane(*(const uint32_t*)p);
        uint32_t hi = __builtin_amdgcn_readfirstlane(*(const uint32_t*)(p + 4));
        return (int64_t)(((uint64_t)hi << 32) | lo);
    };
    auto meta_of = [&](int64_t ch) {
        Meta m;
        const int h = (int)((ch / META_RUN) & 1), j = (int)(ch % META_RUN);
        const uint32_t* rr = (const uint32_t*)(ring_rows) + (h * META_RUN + j) * MAXC;
        const char* bb = ring_blk + (h * (META_RUN + 1) + j) * 8;
        int64_t s0 = ch * chunk;
        int ns = (int)((nslots - s0) < chunk ? (nslots - s0) : chunk);
        m.rr = rr;
        m.nrows = 0;
#pragma unroll
        for (int t = 0; t < RW::NRW; t++) m.nrows += row_slot(t) < ns;
        m.blk = blk0 + ch;
        m.eb = rd64(bb);
        m.ne = (int)(rd64(bb + 8) - m.eb);
        return m;
    };
    // Copy the metadata of chunks [c0, c0 + 16) into ring half h: wave w the
    // row indices of chunks c0 + w, c0 + w + WAVES, ... (64 a copy), wave 0
    // also the 17 block offsets.  Returns the copies this wave issued (each
    // has at least one active lane).
    auto refill = [&](int64_t c0, int h) {
        int k = 0;
#pragma unroll
        for (int q = 0; q < META_RUN / WAVES; q++) {
            const int j = wave + WAVES * q;
            const int64_t c = c0 + j;
            if (c < nch) {
                const int64_t s0 = c * chunk;
                const int ns = (int)((nslots - s0) < chunk ? (nslots - s0) : chunk);
#pragma unroll
                for (int part = 0; part < MAXC; part += 64) {
                    if (part < ns) {
                        if (lane < ns - part)
                            dma4s(sidx + s0 + part, 4u * lane,
                                  ring_rows + ((h * META_RUN + j) * MAXC + part) * 4);
                        k++;
                    }
                }
            }
        }
        if (wave == 0) {
            // blk_base[blk0 + c0 + t] for t <= 16 while c0 + t <= nch
            if (c0 + (lane >> 1) <= nch && lane < 2 * (META_RUN + 1))
                dma4s(blk_base + blk0 + c0, 4u * lane, ring_blk + h * (META_RUN + 1) * 8);
            k++;
        }
        return k;
    };
    // row groups of this wave present in a chunk, and its copy count
    auto groups_of = [&](const Meta& m) { return (m.nrows + F::RPI - 1) / F::RPI; };
    auto issue = [&](const Meta& m, int buf) {
        char* base = smem + buf * L.stride;
#pragma unroll
        for (int q = 0; q < RW::GPW; q++) {
            const int t0 = q * F::RPI;
            if (t0 < m.nrows) {
                const int rl = lane / F::LPR;
                const uint32_t row = rl < m.nrows - t0 ? m.rr[row_slot(t0) + rl] : 0u;
                stage_group<FORM, G, DT, VEC>(base + L.vals + row_slot(t0) * F::RB, values, ld,
                                              nchan, c_lo, row, m.nrows - t0, lane, dma_rows);
            }
        }
        // a unit's weights are WB bytes, its slots 16 bytes (one lane)
        constexpr int UPC = 1024 / F::WB;  // units per weight copy
        const char* w = (const char*)ent_w + m.eb * F::WB;
        for (int i = wave * UPC; i < m.ne; i += WAVES * UPC)
            if (i + lane / (64 / UPC) < m.ne)
                dma16s(w + (int64_t)i * F::WB, 16u * lane, base + L.ew + i * F::WB);
        const uint4* sl = (const uint4*)ent_s + m.eb;
        for (int i = wave * 64; i < m.ne; i += THREADS)
            if (i + lane < m.ne) dma16s(sl + i, 16u * lane, base + L.es + i * 16);
        if (wave == WAVES - 1 && lane < PGOFF_STRIDE / 2)
            dma4s(blk_pgoff + m.blk * PGOFF_STRIDE, 4u * lane, base + L.po);
    };
    // Copy instructions issue() is certain to start for this wave (each
    // counted one has at least one active lane).  Copies whose lanes may all
    // be off are left out, which only makes the waits below stricter.
    auto copies = [&](const Meta& m) {
        constexpr int UPC = 1024 / F::WB;
        int k = dma_rows ? groups_of(m) : 0;
        if (m.ne > wave * UPC) k += (m.ne - wave * UPC + WAVES * UPC - 1) / (WAVES * UPC);
        if (m.ne > wave * 64) k += (m.ne - wave * 64 + THREADS - 1) / THREADS;
        if (wave == WAVES - 1) k += 1;
        return k;
    };
    v4f acc[PGW][G];
#pragma unroll
    for (int k = 0; k < PGW; k++)
#pragma unroll
        for (int g = 0; g < G; g++) acc[k][g] = (v4f){0.f, 0.f, 0.f, 0.f};

    // nbuf chunks are resident: while chunk ch is computed, chunks up to
    // ch + nbuf - 2 are in flight and chunk ch + nbuf - 1 is issued into the
    // buffer chunk ch - 1 used.  Metadata half h holds chunks [16 t, 16 t + 16)
    // for t = h mod 2; the half of chunks [i + 16, i + 32) is refilled at
    // iteration i (i a multiple of 16), before that iteration's data copies,
    // and first read nbuf - 1 iterations before chunk i + 16, by which time
    // the data copies issued after it have been waited for.
    // k1, k2: this wave's copies for chunks ch + 1 and ch + 2 (those may
    // still be outstanding when chunk ch is waited for), a refill counted
    // with the chunk issued right after it.
    if (nch > 0) {
        refill(0, 0);
        if (nch > META_RUN) refill(META_RUN, 1);
        __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0)
        __syncthreads();
    }
    int k1 = 0, k2 = 0;
    for (int i = 0; i < nbuf - 1 && i < nch; i++) {
        Meta m = meta_of(i);
        issue(m, i);
        if (i == 1) k1 = copies(m);
        if (i == 2) k2 = copies(m);
    }
    int cur = 0;  // ch mod nbuf
    for (int64_t ch = 0; ch < nch; ch++) {
        // Wait for this wave's copies of chunk ch (later chunks may stay in
        // flight); the barrier then makes every wave's copies visible and
        // retires all reads of chunk ch - 1's buffer.
        wait_copies(k1 + k2);
        __syncthreads();
        int kn = 0;
        if (ch % META_RUN == 0 && ch >= META_RUN && ch + META_RUN < nch)
            kn += refill(ch + META_RUN, (int)(((ch / META_RUN) + 1) & 1));
        if (ch + nbuf - 1 < nch) {
            Meta mn = meta_of(ch + nbuf - 1);
            kn += copies(mn);
            issue(mn, cur == 0 ? nbuf - 1 : cur - 1);
        }
        if (nbuf == 4) {
            k1 = k2;
            k2 = kn;
        } else if (nbuf == 3) {
            k1 = kn;
        } else {
            k1 = 0;
        }
        const char* base = smem + cur * L.stride;
        cur = cur + 1 == nbuf ? 0 : cur + 1;
        const char* vals = base + L.vals;
        const char* ew = base + L.ew;
        const uint32_t* es = (const uint32_t*)(base + L.es);
        const uint16_t* po = (const uint16_t*)(base + L.po);
        // The wave's groups: their unit ranges (all 65 offsets come in with
        // one read, lane l holding offset l) and their slot runs (at most
        // `chunk` slots each, lane i holding the run's i-th), all read before
        // any is used so that the LDS latency is paid once per chunk.  Ranges
        // and slots are wave-uniform and go to scalar registers by v_readlane.
        // FP32 form: offsets count entries, 4 x (first unit) + (entries of
        // padding in the run's last unit); 16-bit forms: offsets count units,
        // and whole units are multiplied.  eK: first unit, nK: entries to do.
        const uint32_t po_lane = po[lane];
        const int po_end = __builtin_amdgcn_readfirstlane((int)po[TILE_PGS]);
        int eK[PGW], nK[PGW];
        uint32_t slK[PGW];
#pragma unroll
        for (int k = 0; k < PGW; k++) {
            const int lp = lys[k] * TILE_PGX + lxs[k];
            const int a = (int)__builtin_amdgcn_readlane(po_lane, lp);
            const int b = lp + 1 < TILE_PGS ? (int)__builtin_amdgcn_readlane(po_lane, lp + 1) : po_end;
            if (FORM == FORM_F32) {
                eK[k] = a >> 2;
                nK[k] = (b & ~3) - (a & ~3) - (a & 3);
            } else {
                eK[k] = a;
                nK[k] = 4 * (b - a);
            }
            slK[k] = es[4 * eK[k] + (lane < nK[k] ? lane : 0)];
        }
        // A wave holding more than its share of this chunk's entries gets a
        // higher issue priority: the chunk ends with its longest wave, which
        // otherwise shares its SIMD evenly with lighter waves until they are
        // done and then runs alone.
        {
            int mine = 0;
#pragma unroll
            for (int k = 0; k < PGW; k++) mine += pv[k] ? nK[k] : 0;
            // against the chunk's total entries (padding included)
            const int share = mine * WAVES / (FORM == FORM_F32 ? 1 : 4);
            if (share >= 2 * po_end)
                __builtin_amdgcn_s_setprio(3);
            else if (2 * share >= 3 * po_end)
                __builtin_amdgcn_s_setprio(2);
            else if (share >= po_end)
                __builtin_amdgcn_s_setprio(1);
            else
                __builtin_amdgcn_s_setprio(0);
        }
#pragma unroll
        for (int k = 0; k < PGW; k++) {
            if (!pv[k]) continue;
            const int e = eK[k], n = nK[k];
            if (n == 0) continue;
            v4f part[G];
#pragma unroll
            for (int g = 0; g < G; g++) part[g] = (v4f){0.f, 0.f, 0.f, 0.f};
            const int q = lane & 3;
            const uint32_t slot_lane = slK[k];
            if constexpr (FORM == FORM_F32) {
                static_assert(max_chunk<FORM_F32>() <= 64, "a run's slots fit the wave's lanes");
                // Each entry's slot comes from v_readlane into a scalar
                // register, so the value read needs no second LDS round trip.
                // Entries go a unit (four) at a time: one 16-byte read brings
                // this lane's pixel's four weights.  The next unit's five LDS
                // reads are issued before this unit's 4 G MFMAs, so their
                // latency overlaps the matrix work.  A run's last unit
                // multiplies only its real entries.
                typedef typename VF<G>::T VT;
                const char* wq = ew + e * F::WB + q * 16;
                const char* vl = vals + lane * (G * 4);
                auto ldv = [&](int j) {
                    return *(const VT*)(vl + __builtin_amdgcn_readlane(slot_lane, j) * F::RB);
                };
                int j = 0;
                if (!PIPE) {
                    for (; j + 4 <= n; j += 4) {
                        const float4 a = *(const float4*)(wq + j * 16);
                        const VT v0 = ldv(j), v1 = ldv(j + 1), v2 = ldv(j + 2), v3 = ldv(j + 3);
                        mfma_f32<G>(part, a.x, v0);
                        mfma_f32<G>(part, a.y, v1);
                        mfma_f32<G>(part, a.z, v2);
                        mfma_f32<G>(part, a.w, v3);
                        // schedule: all LDS reads of the step, then its MFMAs
                        __builtin_amdgcn_sched_group_barrier(0x100, 5, 0);
                        __builtin_amdgcn_sched_group_barrier(0x008, 4 * G, 0);
                    }
                } else if (n >= 4) {
                    float4 a = *(const float4*)wq;
                    VT v0 = ldv(0), v1 = ldv(1), v2 = ldv(2), v3 = ldv(3);
                    for (; j + 8 <= n; j += 4) {
                        const float4 an = *(const float4*)(wq + (j + 4) * 16);
                        const VT u0 = ldv(j + 4), u1 = ldv(j + 5), u2 = ldv(j + 6), u3 = ldv(j + 7);
                        mfma_f32<G>(part, a.x, v0);
                        mfma_f32<G>(part, a.y, v1);
                        mfma_f32<G>(part, a.z, v2);
                        mfma_f32<G>(part, a.w, v3);
                        __builtin_amdgcn_sched_group_barrier(0x100, 5, 0);
                        __builtin_amdgcn_sched_group_barrier(0x008, 4 * G, 0);
                        a = an;
                        v0 = u0;
                        v1 = u1;
                        v2 = u2;
                        v3 = u3;
                    }
                    mfma_f32<G>(part, a.x, v0);
                    mfma_f32<G>(part, a.y, v1);
                    mfma_f32<G>(part, a.z, v2);
                    mfma_f32<G>(part, a.w, v3);
                    j += 4;
                }
                if (j < n) {
                    const int r = n - j;  // 1..3 entries left
                    const float4 a = *(const float4*)(wq + j * 16);
                    mfma_f32<G>(part, a.x, ldv(j));
                    if (r > 1) mfma_f32<G>(part, a.y, ldv(j + 1));
                    if (r > 2) mfma_f32<G>(part, a.z, ldv(j + 2));
                }
            } else {
                // groups of four entries, slots picked by v_readlane, the
                // next group's reads issued ahead of this group's MFMAs.  A
                // lane holds one entry's slot: setup builds chunks past 64
                // slots only where no group's run in a chunk exceeds 64
                // entries.
                typedef typename VH<G>::T VT;
                const char* vl = vals + lane * (G * 2);
                auto ldv = [&](int j) {
                    return *(const VT*)(vl + __builtin_amdgcn_readlane(slot_lane, j) * F::RB);
                };
                const char* wq = ew + e * 32 + q * 8;
                const int nt = n / 4;
                uint2 a = *(const uint2*)wq;
                VT v0 = ldv(0), v1 = ldv(1), v2 = ldv(2), v3 = ldv(3);
                for (int t = 0; t + 1 < nt; t++) {
                    const uint2 an = *(const uint2*)(wq + (t + 1) * 32);
                    const VT u0 = ldv(4 * t + 4), u1 = ldv(4 * t + 5), u2 = ldv(4 * t + 6),
                             u3 = ldv(4 * t + 7);
                    mfma_16<DT, G>(part, a, v0, v1, v2, v3);
                    a = an;
                    v0 = u0;
                    v1 = u1;
                    v2 = u2;
                    v3 = u3;
                }
                mfma_16<DT, G>(part, a, v0, v1, v2, v3);
            }
#pragma unroll
            for (int g = 0; g < G; g++) acc[k][g] += part[g];
        }
    }

    // Epilogue.  acc[k][g] register i, lane l = pixel i of group k, channel
    // c_lo + G l + g.  Normalised values go through LDS ([pixel][channel],
    // OCW channels per pass) so that the [c][j][i] output is written as rows
    // of 16 contiguous pixels instead of one scattered float per lane.
    __syncthreads();
    float* ol = (float*)smem;
    const int64_t P = (int64_t)nx * ny;
    const int x0 = tx * TILE_PX, y0 = ty * TILE_PX;
    constexpr int PASSES = F::CW / F::OCW;
    constexpr int LPP = F::OCW / G;  // lanes per pass
#pragma unroll
    for (int h = 0; h < PASSES; h++) {
        if (lane / LPP == h) {
            const int cl0 = G * (lane % LPP);
#pragma unroll
            for (int k = 0; k < PGW; k++) {
                if (!pv[k]) continue;
#pragma unroll
                for (int i = 0; i < 4; i++) {
                    int pxl = lxs[k] * PG + (i & 1), pyl = lys[k] * PG + (i >> 1);
                    if (x0 + pxl >= nx || y0 + pyl >= ny) continue;
                    float W = pix_Wf[(int64_t)(y0 + pyl) * nx + x0 + pxl];
                    float* d = ol + (pyl * TILE_PX + pxl) * F::OUT_STRIDE + cl0;
#pragma unroll
                    for (int g = 0; g < G; g++) d[g] = acc[k][g][i] / W;
                }
            }
        }
        __syncthreads();
        for (int t = threadIdx.x; t < F::OCW * TILE_PX * (TILE_PX / 4); t += THREADS) {
            int qd = t % (TILE_PX / 4), row = t / (TILE_PX / 4);
            int pyl = row % TILE_PX, cl = row / TILE_PX;
            int c = c_lo + h * F::OCW + cl, y = y0 + pyl, x = x0 + 4 * qd;
            if (c >= nchan || y >= ny || x >= nx) continue;
            const float* src = ol + (pyl * TILE_PX + 4 * qd) * F::OUT_STRIDE + cl;
            float* dst = out + (int64_t)c * P + (int64_t)y * nx + x;
            if (out_vec && x + 3 < nx) {
                *(float4*)dst = make_float4(src[0], src[F::OUT_STRIDE], src[2 * F::OUT_STRIDE],
                                            src[3 * F::OUT_STRIDE]);
            } else {
                for (int j = 0; j < 4 && x + j < nx; j++) dst[j] = src[j * F::OUT_STRIDE];
            }
        }
        __syncthreads();
    }
}

template <int FORM, int DT, bool VEC, int WAVES, int G>
__global__ __launch_bounds__(64 * WAVES) void k_channels(
    const void* __restrict__ values, int64_t ld, int32_t nchan, int32_t ncb, int32_t npgx,
    int32_t npgy, int32_t ntx, int32_t nx, int32_t ny, int32_t chunk,
    const int64_t* __restrict__ tile_base, const uint32_t* __restrict__ slot_idx,
    const int64_t* __restrict__ tile_blk, const int64_t* __restrict__ blk_base,
    const uint16_t* __restrict__ blk_pgoff, const void* __restrict__ ent_w,
    const void* __restrict__ ent_s, const float* __restrict__ pix_Wf, float* __restrict__ out,
    int32_t out_vec, int32_t ucap, int32_t nbuf, const uint32_t* __restrict__ pg_cnt,
    int32_t balance, const int64_t* __restrict__ order) {
    extern __shared__ __attribute__((aligned(16))) char smem[];
    // Workgroup b takes the plan's item order[b] (tile * ncb + channel block),
    // laid out as for the batched form: a tile's channel blocks on one XCD,
    // tiles placed longest first over the XCDs, each XCD's items by decreasing
    // cost; -1 marks an idle workgroup.  Without an order (NULL), workgroup b
    // takes item b.
    const int64_t item = order ? order[blockIdx.x] : (int64_t)blockIdx.x;
    if (item < 0) return;
    grid_item<FORM, DT, VEC, WAVES, G>(values, ld, nchan, npgx, npgy, ntx, nx, ny, chunk,
                                       tile_base, slot_idx, tile_blk, blk_base, blk_pgoff, ent_w,
                                       ent_s, pix_Wf, out, out_vec, ucap, nbuf, pg_cnt, balance,
                                       item / ncb, item % ncb, smem);
}

// Batched form: one launch over the (field, tile, channel block) items of many
// fields.  Workgroup b takes item b.  The host lays the items out so that the
// hardware's in-order, round-robin dispatch does the scheduling: position b
// runs on XCD b mod 8, each XCD's items were assigned by longest-processing-
// time-first over the 8 XCDs with a tile's channel blocks kept together (one
// L2), and within an XCD they are ordered by decreasing cost, so a CU that
// frees up always takes the largest item left.  Padding items (field < 0)
// return at once.
template <int FORM, int DT, bool VEC, int WAVES, int G>
__global__ __launch_bounds__(64 * WAVES) void k_channels_batch(
    const FieldDesc* __restrict__ fields, const BatchItem* __restrict__ items) {
    extern __shared__ __attribute__((aligned(16))) char smem[];
    // descriptors and items are never written by the kernel: reading them
    // through the constant address space keeps them in scalar registers
    const CONST_AS BatchItem* it = (const CONST_AS BatchItem*)items + blockIdx.x;
    const int32_t f = it->field;
    if (f < 0) return;
    const CONST_AS FieldDesc& d = ((const CONST_AS FieldDesc*)fields)[f];
    grid_item<FORM, DT, VEC, WAVES, G>(d.values, d.ld, d.nchan, d.npgx, d.npgy, d.ntx, d.nx, d.ny,
                                       d.chunk, d.tile_base, d.slot_idx, d.tile_blk, d.blk_base,
                                       d.blk_pgoff, d.ent_w, d.ent_s, d.pix_Wf, d.out, d.out_vec,
                                       d.ucap, d.nbuf, d.pg_cnt, d.balance, it->tile, it->cb, smem);
}

// LDS plan of a field: entry capacity, resident chunks and dynamic LDS bytes
// (the output transpose of the epilogue reuses the same space).
size_t lds_stride(bool m16, int chunk, int ucap, int g) {
    const int rb = 64 * g * (m16 ? 2 : 4);
    return LdsLayout::make(rb, m16 ? 32 : 64, chunk, ucap).stride;
}

void lds_plan(bool m16, int chunk, int blk_max, int g, int32_t& ucap, int32_t& nbuf) {
    ucap = (blk_max < 4 ? 4 : (blk_max + 3) / 4 * 4);
    nbuf = (int32_t)((LDS_BYTES - meta_lds(m16)) / lds_stride(m16, chunk, ucap, g));
    if (nbuf > MAX_NBUF) nbuf = MAX_NBUF;
    if (nbuf < 2) nbuf = 2;  // not reached: setup checks the fit for the widest block
}

size_t out_lds(int g) {
    const int ocw = g >= 2 ? 128 : 64;
    return (size_t)TILE_PX * TILE_PX * (ocw + 4) * 4;
}

size_t lds_shm(bool m16, int chunk, int ucap, int nbuf, int g) {
    size_t shm = (size_t)nbuf * lds_stride(m16, chunk, ucap, g) + meta_lds(m16);
    return shm < out_lds(g) ? out_lds(g) : shm;
}

// Kernel instances: every dtype and vector path at the default shape (16
// waves, 256 channels); the tuned shapes for the aligned paths the workloads
// use (FP32 values in the FP32 form, BF16 / FP16 values in the 16-bit forms).
template <int FORM, int DT, bool VEC>
constexpr bool shape_instances() {
    return VEC && ((FORM == FORM_F32 && DT == HG_F32) || FORM == FORM_M16);
}

template <template <int, int, bool, int, int> class K, int FORM, int DT, bool VEC>
const void* pick_shape(int waves, int g) {
    if constexpr (shape_instances<FORM, DT, VEC>()) {
        if (waves == 8) {
            if (g == 4) return K<FORM, DT, VEC, 8, 4>::f();
            if (g == 2) return K<FORM, DT, VEC, 8, 2>::f();
            return K<FORM, DT, VEC, 8, 1>::f();
        }
        if (g == 2) return K<FORM, DT, VEC, 16, 2>::f();
        if (g == 1) return K<FORM, DT, VEC, 16, 1>::f();
    }
    return K<FORM, DT, VEC, 16, 4>::f();
}

template <template <int, int, bool, int, int> class K>
const void* pick(bool m16, int32_t dtype, bool vec, int waves, int g) {
    if (m16) {
        if (dtype == HG_BF16)
            return vec ? pick_shape<K, FORM_M16, HG_BF16, true>(waves, g)
                       : pick_shape<K, FORM_M16, HG_BF16, false>(waves, g);
        return vec ? pick_shape<K, FORM_M16, HG_F16, true>(waves, g)
                   : pick_shape<K, FORM_M16, HG_F16, false>(waves, g);
    }
    if (dtype == HG_F32)
        return vec ? pick_shape<K, FORM_F32, HG_F32, true>(waves, g)
                   : pick_shape<K, FORM_F32, HG_F32, false>(waves, g);
    if (dtype == HG_BF16)
        return vec ? pick_shape<K, FORM_F32, HG_BF16, true>(waves, g)
                   : pick_shape<K, FORM_F32, HG_BF16, false>(waves, g);
    return vec ? pick_shape<K, FORM_F32, HG_F16, true>(waves, g)
               : pick_shape<K, FORM_F32, HG_F16, false>(waves, g);
}
template <int FORM, int DT, bool VEC, int WAVES, int G>
struct SingleKernel {
    static const void* f() { return (const void*)k_channels<FORM, DT, VEC, WAVES, G>; }
};
template <int FORM, int DT, bool VEC, int WAVES, int G>
struct BatchKernel {
    static const void* f() { return (const void*)k_channels_batch<FORM, DT, VEC, WAVES, G>; }
};

}  // namespace

bool values_vec(const Plan& P, const void* values, int64_t ld, int32_t dtype) {
    uintptr_t a = (uintptr_t)values;
    if (P.opts.precision != HG_PREC_FP32) return a % 16 == 0 && ld % 8 == 0;
    if (dtype == HG_F32) return a % 16 == 0 && ld % 4 == 0;
    return a % 8 == 0 && ld % 4 == 0;
}

Shape effective_shape(bool m16, int32_t dtype, bool vec, Shape s) {
    const bool tuned = vec && (m16 || dtype == HG_F32);
    if (!tuned || (s.waves != 8 && s.waves != 16) || (s.g != 1 && s.g != 2 && s.g != 4))
        return Shape{};
    return s;
}

FieldDesc field_desc(const Plan& P, const void* values, int64_t ld, int32_t nchan, float* out,
                     Shape shape) {
    FieldDesc d{};
    bool m16 = P.opts.precision != HG_PREC_FP32;
    const int cw = 64 * shape.g;
    d.values = values;
    d.ld = ld;
    d.nchan = nchan;
    d.ncb = (nchan + cw - 1) / cw;
    d.npgx = P.npgx;
    d.npgy = P.npgy;
    d.ntx = P.ntx;
    d.nx = P.map.nx;
    d.ny = P.map.ny;
    d.chunk = P.chunk;
    lds_plan(m16, P.chunk, P.blk_max, shape.g, d.ucap, d.nbuf);
    d.out_vec = ((uintptr_t)out % 16 == 0) && (P.map.nx % 4 == 0);
    d.tile_base = (const int64_t*)P.tile_nslots.p;
    d.slot_idx = (const uint32_t*)P.slot_idx.p;
    d.tile_blk = (const int64_t*)P.tile_blk.p;
    d.blk_base = (const int64_t*)P.blk_base.p;
    d.blk_pgoff = (const uint16_t*)P.blk_pgoff.p;
    d.ent_w = m16 ? P.e3_w.p : P.e2_w.p;
    d.ent_s = m16 ? P.e3_s.p : P.e2_s.p;
    d.pix_Wf = (const float*)P.pix_Wf.p;
    d.pg_cnt = (const uint32_t*)P.pg_cnt.p;
    {
        // the fixed wave classes by default: with dealt chunks they measured
        // faster than the count-balanced assignment (drift field FP32 kernel
        // 3.535 -> 3.512 ms, 64-field batched launch 104.5 -> 101.9 ms);
        // HEGRID_BALANCE=1 selects the balanced one
        const char* b = getenv("HEGRID_BALANCE");
        d.balance = b ? atoi(b) : 0;
    }
    d.out = out;
    return d;
}

hipError_t launch_channels(Plan& P, const void* values, int64_t ld, int32_t nchan, int32_t dtype,
                           float* out, hipStream_t s, Shape shape, int32_t row0, int32_t row1) {
    const bool vec = values_vec(P, values, ld, dtype);
    const bool m16 = P.opts.precision != HG_PREC_FP32;
    shape = effective_shape(m16, dtype, vec, shape);
    const int32_t ncb = (nchan + 64 * shape.g - 1) / (64 * shape.g);
    const int64_t* order = nullptr;
    int64_t nwg = 0;
    hipError_t e = launch_order(P, ncb, s, &order, &nwg, row0, row1);
    if (e != hipSuccess) return e;
    return launch_channels_on(P, values, ld, nchan, dtype, out, s, shape, order, nwg);
}

// 1 + the largest sample index tile t stages (its slots' sample indices), 0
// when it stages none: one workgroup per tile.
__global__ __launch_bounds__(256) void k_tile_max_index(const int64_t* __restrict__ tile_base,
                                                        const uint32_t* __restrict__ slot_idx,
                                                        int64_t* __restrict__ tile_need) {
    __shared__ int64_t red[4];
    const int64_t t = blockIdx.x;
    const int64_t a = tile_base[t], b = tile_base[t + 1];
    int64_t m = 0;
    for (int64_t i = a + threadIdx.x; i < b; i += blockDim.x) {
        const int64_t v = (int64_t)slot_idx[i] + 1;
        m = v > m ? v : m;
    }
    for (int o = 32; o > 0; o >>= 1) {
        const int64_t y = __shfl_xor(m, o, 64);
        m = y > m ? y : m;
    }
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t r = red[0];
        for (int k = 1; k < 4; k++) r = red[k] > r ? red[k] : r;
        tile_need[t] = r;
    }
}

hipError_t launch_tile_max_index(const Plan& P, int64_t* tile_need, hipStream_t s) {
    if (P.ntiles == 0) return hipSuccess;
    hipLaunchKernelGGL(k_tile_max_index, dim3((unsigned)P.ntiles), dim3(256), 0, s,
                       (const int64_t*)P.tile_nslots.p, (const uint32_t*)P.slot_idx.p, tile_need);
    return hipGetLastError();
}

hipError_t launch_channels_on(Plan& P, const void* values, int64_t ld, int32_t nchan,
                              int32_t dtype, float* out, hipStream_t s, Shape shape,
                              const int64_t* order, int64_t nwg) {
    const bool vec = values_vec(P, values, ld, dtype);
    const bool m16 = P.opts.precision != HG_PREC_FP32;
    shape = effective_shape(m16, dtype, vec, shape);
    FieldDesc d = field_desc(P, values, ld, nchan, out, shape);
    hipError_t e = hipSuccess;
    if (nwg == 0) return hipSuccess;
    const void* kern = pick<SingleKernel>(m16, dtype, vec, shape.waves, shape.g);
    const size_t shm = lds_shm(m16, d.chunk, d.ucap, d.nbuf, shape.g);
    if (shm > 65536) {
        e = hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
        if (e != hipSuccess) return e;
    }
    void* args[] = {&d.values, &d.ld,      &d.nchan,     &d.ncb,     &d.npgx,  &d.npgy,
                    &d.ntx,    &d.nx,      &d.ny,        &d.chunk,   &d.tile_base, &d.slot_idx,
                    &d.tile_blk, &d.blk_base, &d.blk_pgoff, &d.ent_w, &d.ent_s, &d.pix_Wf,
                    &d.out,    &d.out_vec, &d.ucap,      &d.nbuf,    &d.pg_cnt, &d.balance,
                    &order};
    e = hipLaunchKernel(kern, dim3((unsigned)nwg), dim3((unsigned)(64 * shape.waves)), args, shm,
                        s);
    if (e != hipSuccess) return e;
    return hipGetLastError();
}

hipError_t launch_channels_plain_order(Plan& P, const void* values, int64_t ld, int32_t nchan,
                                      int32_t dtype, float* out, hipStream_t s, Shape shape) {
    const bool vec = values_vec(P, values, ld, dtype);
    const bool m16 = P.opts.precision != HG_PREC_FP32;
    const Shape eff = effective_shape(m16, dtype, vec, shape);
    const int64_t ncb = (nchan + 64 * eff.g - 1) / (64 * eff.g);
    return launch_channels_on(P, values, ld, nchan, dtype, out, s, shape, nullptr,
                              P.ntiles * ncb);
}

bool channel_lds_fits(bool m16, int chunk, int blk_max) {
    int32_t ucap, nbuf;
    lds_plan(m16, chunk, blk_max, 4, ucap, nbuf);
    if (!m16 && chunk > max_chunk<FORM_F32>()) return false;
    return (size_t)2 * lds_stride(m16, chunk, ucap, 4) + meta_lds(m16) <= (size_t)LDS_BYTES;
}

size_t field_lds_bytes(const FieldDesc& d, bool m16, Shape shape) {
    return lds_shm(m16, d.chunk, d.ucap, d.nbuf, shape.g);
}

BatchKernelInfo batch_kernel(bool m16, int32_t dtype, bool vec, size_t shm, Shape shape) {
    BatchKernelInfo k;
    shape = effective_shape(m16, dtype, vec, shape);
    k.main = pick<BatchKernel>(m16, dtype, vec, shape.waves, shape.g);
    k.shm = shm;
    k.threads = 64 * shape.waves;
    k.channels_per_block = 64 * shape.g;
    return k;
}

}  // namespace hg
