// Channel phase of libhegrid: the weighted sums of Eq. (1) for many channels
// against a plan built once by setup (channels are independent, Sec. 4.2; the
// neighbour structure is shared by all of them, Sec. 4.3.1).
//
// For each pixel p and channel c:  S[c,p] = sum_{n in N(p)} w[p,n] v[n,c],
// V[c,p] = S[c,p] / W_p.  This is a sparse (pixels x samples) by dense
// (samples x channels) product.  Layout of the work:
//
//   * a workgroup (16 waves) owns one tile (16 x 16 pixels = 8 x 8 pixel
//     groups of 2 x 2) and one block of 256 channels;
//   * the tile's candidate samples (its slots) are processed in chunks of
//     `chunk` slots.  For each chunk the workgroup stages, in LDS, the 256
//     channels of every slot (one row per sample, read from the
//     channel-contiguous values in HBM) and the chunk's entry block (the
//     entries of all 64 groups, prepared by setup);
//   * staging is double-buffered: the loads for chunk c+1 go straight from
//     global memory to LDS (global_load_lds) while the waves compute chunk c;
//   * each wave owns 4 pixel groups spread over the tile.  The MFMA rows are
//     the group's four pixels (A = their weights) and the columns are the
//     workgroup's channels, 4*lane + g for the g-th instruction (B = values);
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

constexpr int CH_WAVES = 16;
constexpr int CH_THREADS = 64 * CH_WAVES;
constexpr int G = 4;        // MFMA column blocks of 64 channels per workgroup
constexpr int CW = 64 * G;  // channels per workgroup (256)
constexpr int PGW = TILE_PGS / CH_WAVES;
static_assert(TILE_PGX == 8 && TILE_PGY == 8 && CH_WAVES == 16,
              "wave/group mapping assumes 8x8 groups, 16 waves");
constexpr int TILE_PX = TILE_PGX * PG;  // 16 pixels per tile side
constexpr int OUT_STRIDE = CW / 2 + 4;  // LDS floats per pixel in the output transpose
constexpr int OUT_LDS = TILE_PX * TILE_PX * OUT_STRIDE * 4;

constexpr int FORM_F32 = 0;  // FP32 values in LDS, one entry per MFMA
constexpr int FORM_M16 = 1;  // 16-bit values in LDS, groups of four entries per MFMA

template <int FORM>
struct Form {
    static constexpr int VB = FORM == FORM_F32 ? 4 : 2;   // bytes per staged value
    static constexpr int RB = CW * VB;                     // bytes per staged row
    // a unit is a group of four entries of one pixel group: weights [pixel][entry]
    static constexpr int WB = FORM == FORM_F32 ? 64 : 32;  // weight bytes per unit
    static constexpr int SB = 16;                          // slot bytes per unit
    static constexpr int UPS = 4;                          // entries per unit
};

// One staged chunk in LDS: `chunk` value rows, then the entry block (weights,
// slots) for up to `ucap` units, then the 65 per-group offsets.  ucap is the
// plan's largest block (a multiple of 4), so a chunk takes what the plan needs
// rather than the 64 x chunk worst case, and more chunks fit in flight.
constexpr int LDS_BYTES = 160 * 1024;
constexpr int MAX_NBUF = 4;
// Chunk metadata ring: two halves of 16 chunks, each chunk's staged-row sample
// indices (MAX_CHUNK x uint32) and the 17 entry-block offsets of a half.
constexpr int META_RUN = 16;
constexpr int META_ROWS = 2 * META_RUN * MAX_CHUNK * 4;
constexpr int META_LDS = META_ROWS + 2 * (META_RUN + 1) * 8;

struct LdsLayout {
    int vals, ew, es, po, stride;
    template <int FORM>
    __device__ __host__ static LdsLayout make(int chunk, int ucap) {
        typedef Form<FORM> F;
        LdsLayout L;
        L.vals = 0;
        L.ew = L.vals + chunk * F::RB;
        L.es = L.ew + ucap * F::WB;
        L.po = L.es + ucap * F::SB;
        L.stride = L.po + 144;
        return L;
    }
};

// Direct global -> LDS copies (lane i writes bytes [i*size, (i+1)*size) after
// the wave-uniform LDS address).  They are issued through inline assembly so
// that the compiler does not order every later LDS read behind them: the
// kernel itself waits for them (s_waitcnt vmcnt) before the barrier that hands
// a staged chunk to the compute loop.
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

// FP32 form, one staged row (1 KB): channels [c_lo, c_lo + 256) of `row` as
// FP32; lane l writes channels 4l .. 4l+3.
template <int DT, bool VEC>
__device__ inline void stage_row_f32(char* dst, const void* values, int64_t ld, int32_t nchan,
                                     int c_lo, uint32_t row, int lane, bool dma) {
    int c = c_lo + 4 * lane;
    if (DT == HG_F32) {
        const float* src = (const float*)values + (int64_t)row * ld;
        if (dma) {
            dma16s(src + c_lo, 16u * lane, dst);
            return;
        }
        float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
        if (VEC && c + 3 < nchan) {
            v = *(const float4*)(src + c);
        } else {
            if (c + 0 < nchan) v.x = src[c + 0];
            if (c + 1 < nchan) v.y = src[c + 1];
            if (c + 2 < nchan) v.z = src[c + 2];
            if (c + 3 < nchan) v.w = src[c + 3];
        }
        ((float4*)dst)[lane] = v;
    } else {
        const uint16_t* src = (const uint16_t*)values + (int64_t)row * ld;
        uint32_t u[4] = {0, 0, 0, 0};
        if (VEC && c + 3 < nchan) {
            uint2 raw = *(const uint2*)(src + c);
            u[0] = raw.x & 0xFFFF;
            u[1] = raw.x >> 16;
            u[2] = raw.y & 0xFFFF;
            u[3] = raw.y >> 16;
        } else {
            for (int k = 0; k < 4; k++)
                if (c + k < nchan) u[k] = src[c + k];
        }
        float f[4];
#pragma unroll
        for (int k = 0; k < 4; k++)
            f[k] = (DT == HG_BF16) ? bf16_bits_to_f32(u[k]) : f16_bits_to_f32(u[k]);
        ((float4*)dst)[lane] = make_float4(f[0], f[1], f[2], f[3]);
    }
}

// 16-bit forms, two staged rows (512 B each, adjacent in LDS): lanes 0-31
// copy row a, lanes 32-63 row b, 8 channels per lane.
template <bool VEC>
__device__ inline void stage_rows_16(char* dst, const void* values, int64_t ld, int32_t nchan,
                                     int c_lo, uint32_t row_a, uint32_t row_b, int nrows,
                                     int lane, bool dma) {
    int half = lane >> 5;
    uint32_t row = half ? row_b : row_a;
    int c = c_lo + 8 * (lane & 31);
    const uint16_t* src = (const uint16_t*)values + (int64_t)row * ld + c;
    if (dma) {
        // one copy per row: lanes 0-31 fetch row a, lanes 32-63 row b, each
        // lane landing at its own 16-byte slot of the adjacent LDS rows
        const uint32_t voff = 16u * (lane & 31);
        const uint16_t* base = (const uint16_t*)values + c_lo;
        if (half == 0) dma16s(base + (int64_t)row_a * ld, voff, dst);
        else if (nrows > 1) dma16s(base + (int64_t)row_b * ld, voff, dst);
        return;
    }
    if (half >= nrows) return;
    uint32_t u[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    if (VEC && c + 7 < nchan) {
        uint4 raw = *(const uint4*)src;
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
    ((uint4*)dst)[lane] = make_uint4(u[0] | (u[1] << 16), u[2] | (u[3] << 16),
                                     u[4] | (u[5] << 16), u[6] | (u[7] << 16));
}

__device__ inline void mfma4_f32(v4f* part, float a, float4 v) {
    part[0] = __builtin_amdgcn_mfma_f32_4x4x1f32(a, v.x, part[0], 0, 0, 0);
    part[1] = __builtin_amdgcn_mfma_f32_4x4x1f32(a, v.y, part[1], 0, 0, 0);
    part[2] = __builtin_amdgcn_mfma_f32_4x4x1f32(a, v.z, part[2], 0, 0, 0);
    part[3] = __builtin_amdgcn_mfma_f32_4x4x1f32(a, v.w, part[3], 0, 0, 0);
}

// One group of four entries on the 16-bit MFMA.  a: this lane's pixel's four
// weights (entries 0..3); v0..v3: this lane's channels 4l..4l+3 of the four
// entries' samples.  Column block g takes channel 4l+g of each entry.
template <int DT>
__device__ inline void mfma4_16(v4f* part, uint2 a, uint2 v0, uint2 v1, uint2 v2, uint2 v3) {
    // B_g = {v0[g], v1[g], v2[g], v3[g]}: gather 16-bit halves
    uint2 b[4];
    b[0] = make_uint2(__builtin_amdgcn_perm(v1.x, v0.x, 0x05040100u),
                      __builtin_amdgcn_perm(v3.x, v2.x, 0x05040100u));
    b[1] = make_uint2(__builtin_amdgcn_perm(v1.x, v0.x, 0x07060302u),
                      __builtin_amdgcn_perm(v3.x, v2.x, 0x07060302u));
    b[2] = make_uint2(__builtin_amdgcn_perm(v1.y, v0.y, 0x05040100u),
                      __builtin_amdgcn_perm(v3.y, v2.y, 0x05040100u));
    b[3] = make_uint2(__builtin_amdgcn_perm(v1.y, v0.y, 0x07060302u),
                      __builtin_amdgcn_perm(v3.y, v2.y, 0x07060302u));
#pragma unroll
    for (int g = 0; g < 4; g++) {
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
// rounded down to 0, 2, 4 or 8 (waiting for a little more than needed) to
// keep the choice to three scalar branches.
__device__ inline void wait_copies(int k) {
    if (k >= 8)
        __builtin_amdgcn_s_waitcnt(0x0F78);  // vmcnt(8), expcnt and lgkmcnt open
    else if (k >= 4)
        __builtin_amdgcn_s_waitcnt(0x0F74);  // vmcnt(4)
    else if (k >= 2)
        __builtin_amdgcn_s_waitcnt(0x0F72);  // vmcnt(2)
    else
        __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0)
}

template <int FORM, int DT, bool VEC>
__device__ __attribute__((always_inline)) inline void grid_item(
    const void* __restrict__ values, int64_t ld, int32_t nchan, int32_t npgx, int32_t npgy,
    int32_t ntx, int32_t nx, int32_t ny, int32_t chunk, const int64_t* __restrict__ tile_base,
    const uint32_t* __restrict__ slot_idx, const int64_t* __restrict__ tile_blk,
    const int64_t* __restrict__ blk_base, const uint16_t* __restrict__ blk_pgoff,
    const void* __restrict__ ent_w, const void* __restrict__ ent_s,
    const float* __restrict__ pix_Wf, float* __restrict__ out, int32_t out_vec, int32_t ucap,
    int32_t nbuf, int64_t tile, int64_t cb, char* smem) {
    typedef Form<FORM> F;
    const LdsLayout L = LdsLayout::make<FORM>(chunk, ucap);
    int tx = (int)(tile % ntx), ty = (int)(tile / ntx);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int c_lo = (int)cb * CW;
    // value rows go straight to LDS when they need no conversion, are aligned
    // and are complete
    const bool dma_rows = (FORM == FORM_F32 ? DT == HG_F32 : true) && VEC && c_lo + CW <= nchan;

    const int64_t s_base = tile_base[tile];
    const int64_t nslots = tile_base[tile + 1] - s_base;
    const int64_t blk0 = tile_blk[tile];
    const int64_t nch = tile_blk[tile + 1] - blk0;
    const uint32_t* sidx = slot_idx + s_base;

    // Wave w owns the four groups of one (x mod 4, y mod 4) class: a chunk's
    // samples are spatially compact, so this spreads each chunk's entries
    // over the 16 waves.  The class of wave w is y mod 4 = w / 4, x mod 4 =
    // (w - w / 4) mod 4, so the four waves that share a SIMD (w mod 4 equal)
    // own a diagonal of classes, one in every row and column: the chunk's
    // matrix work then splits more evenly over the SIMDs than with the
    // classes of one column per SIMD.
    bool pv[PGW];
    int lxs[PGW], lys[PGW];
#pragma unroll
    for (int k = 0; k < PGW; k++) {
        lxs[k] = ((wave - (wave >> 2)) & 3) + 4 * (k & 1);
        lys[k] = (wave >> 2) + 4 * (k >> 1);
        pv[k] = tx * TILE_PGX + lxs[k] < npgx && ty * TILE_PGY + lys[k] < npgy;
    }

    // Per chunk each wave stages up to four rows: w + 16 t in the FP32 form,
    // the adjacent pairs (2w, 2w+1) and (2w+32, 2w+33) in the 16-bit forms
    // (the rows that exist are always the first nrows of these).  The chunk metadata (the
    // rows' sample indices and the entry block's extent) reaches LDS through
    // the same asynchronous copies as the data, sixteen chunks at a time into
    // one half of a two-half ring, long before it is read; the loop issues no
    // scalar loads, whose latency the LDS waits of the compute phase would
    // otherwise absorb.  The vector memory counter thus only counts copies,
    // which the pipeline waits for explicitly.
    char* ring_rows = smem + nbuf * L.stride;
    char* ring_blk = ring_rows + META_ROWS;
    struct Meta {
        uint32_t row0, row1, row2, row3;
        int nrows, ne;
        int64_t blk, eb;
    };
    auto row_slot = [&](int t) {
        return FORM == FORM_F32 ? wave + CH_WAVES * t : 2 * wave + 32 * (t >> 1) + (t & 1);
    };
    auto rd64 = [&](const char* p) {
        uint32_t lo = __builtin_amdgcn_readfirstlane(*(const uint32_t*)p);
        uint32_t hi = __builtin_amdgcn_readfirstlane(*(const uint32_t*)(p + 4));
        return (int64_t)(((uint64_t)hi << 32) | lo);
    };
    auto meta_of = [&](int64_t ch) {
        Meta m;
        const int h = (int)((ch / META_RUN) & 1), j = (int)(ch % META_RUN);
        const uint32_t* rr = (const uint32_t*)(ring_rows) + (h * META_RUN + j) * MAX_CHUNK;
        const char* bb = ring_blk + (h * (META_RUN + 1) + j) * 8;
        int64_t s0 = ch * chunk;
        int ns = (int)((nslots - s0) < chunk ? (nslots - s0) : chunk);
        const int r0 = row_slot(0), r1 = row_slot(1), r2 = row_slot(2), r3 = row_slot(3);
        m.nrows = (r0 < ns) + (r1 < ns) + (r2 < ns) + (r3 < ns);  // chunk <= 64
        m.row0 = r0 < ns ? __builtin_amdgcn_readfirstlane(rr[r0]) : 0u;
        m.row1 = r1 < ns ? __builtin_amdgcn_readfirstlane(rr[r1]) : 0u;
        m.row2 = r2 < ns ? __builtin_amdgcn_readfirstlane(rr[r2]) : 0u;
        m.row3 = r3 < ns ? __builtin_amdgcn_readfirstlane(rr[r3]) : 0u;
        m.blk = blk0 + ch;
        m.eb = rd64(bb);
        m.ne = (int)(rd64(bb + 8) - m.eb);
        return m;
    };
    // Copy the metadata of chunks [c0, c0 + 16) into ring half h: wave w the
    // row indices of chunk c0 + w, wave 0 also the 17 block offsets.  Returns
    // the copies this wave issued (each has at least one active lane).
    auto refill = [&](int64_t c0, int h) {
        int k = 0;
        const int64_t c = c0 + wave;
        if (c < nch) {
            const int64_t s0 = c * chunk;
            const int ns = (int)((nslots - s0) < chunk ? (nslots - s0) : chunk);
            if (lane < ns)
                dma4s(sidx + s0, 4u * lane,
                      ring_rows + (h * META_RUN + wave) * MAX_CHUNK * 4);
            k++;
        }
        if (wave == 0) {
            // blk_base[blk0 + c0 + t] for t <= 16 while c0 + t <= nch
            if (c0 + (lane >> 1) <= nch && lane < 2 * (META_RUN + 1))
                dma4s(blk_base + blk0 + c0, 4u * lane, ring_blk + h * (META_RUN + 1) * 8);
            k++;
        }
        return k;
    };
    auto issue = [&](const Meta& m, int buf) {
        char* base = smem + buf * L.stride;
        if (FORM == FORM_F32) {
            if (m.nrows > 0)
                stage_row_f32<DT, VEC>(base + L.vals + row_slot(0) * F::RB, values, ld, nchan,
                                       c_lo, m.row0, lane, dma_rows);
            if (m.nrows > 1)
                stage_row_f32<DT, VEC>(base + L.vals + row_slot(1) * F::RB, values, ld, nchan,
                                       c_lo, m.row1, lane, dma_rows);
            if (m.nrows > 2)
                stage_row_f32<DT, VEC>(base + L.vals + row_slot(2) * F::RB, values, ld, nchan,
                                       c_lo, m.row2, lane, dma_rows);
            if (m.nrows > 3)
                stage_row_f32<DT, VEC>(base + L.vals + row_slot(3) * F::RB, values, ld, nchan,
                                       c_lo, m.row3, lane, dma_rows);
            // a unit's weights are 64 bytes (four lanes), its slots 16 bytes (one lane)
            const char* w = (const char*)ent_w + m.eb * 64;
            for (int i = wave * 16; i < m.ne; i += CH_WAVES * 16)
                if (i + (lane >> 2) < m.ne)
                    dma16s(w + (int64_t)i * 64, 16u * lane, base + L.ew + i * 64);
            const uint4* sl = (const uint4*)ent_s + m.eb;
            for (int i = wave * 64; i < m.ne; i += CH_THREADS)
                if (i + lane < m.ne) dma16s(sl + i, 16u * lane, base + L.es + i * 16);
        } else {
            if (m.nrows > 0)
                stage_rows_16<VEC>(base + L.vals + row_slot(0) * F::RB, values, ld, nchan, c_lo,
                                   m.row0, m.row1, m.nrows < 2 ? m.nrows : 2, lane, dma_rows);
            if (m.nrows > 2)
                stage_rows_16<VEC>(base + L.vals + row_slot(2) * F::RB, values, ld, nchan, c_lo,
                                   m.row2, m.row3, m.nrows - 2, lane, dma_rows);
            // a group's weights are 32 bytes (two lanes), its slots 16 bytes (one lane)
            const char* w = (const char*)ent_w + m.eb * 32;
            for (int i = wave * 32; i < m.ne; i += CH_WAVES * 32)
                if (i + (lane >> 1) < m.ne)
                    dma16s(w + (int64_t)i * 32, 16u * lane, base + L.ew + i * 32);
            const uint4* sl = (const uint4*)ent_s + m.eb;
            for (int i = wave * 64; i < m.ne; i += CH_THREADS)
                if (i + lane < m.ne) dma16s(sl + i, 16u * lane, base + L.es + i * 16);
        }
        if (wave == CH_WAVES - 1 && lane < PGOFF_STRIDE / 2)
            dma4s(blk_pgoff + m.blk * PGOFF_STRIDE, 4u * lane, base + L.po);
    };
    // Copy instructions issue() is certain to start for this wave (each
    // counted one has at least one active lane).  Copies whose lanes may all
    // be off are left out, which only makes the waits below stricter.
    auto copies = [&](const Meta& m) {
        int k = 0;
        if (FORM == FORM_F32) {
            if (dma_rows) k += m.nrows;
            if (m.ne > wave * 16) k += (m.ne - wave * 16 + CH_WAVES * 16 - 1) / (CH_WAVES * 16);
            if (m.ne > wave * 64) k += (m.ne - wave * 64 + CH_THREADS - 1) / CH_THREADS;
        } else {
            if (dma_rows && m.nrows > 0) k += m.nrows;
            if (m.ne > wave * 32) k += (m.ne - wave * 32 + CH_WAVES * 32 - 1) / (CH_WAVES * 32);
            if (m.ne > wave * 64) k += (m.ne - wave * 64 + CH_THREADS - 1) / CH_THREADS;
        }
        if (wave == CH_WAVES - 1) k += 1;
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
        // The wave's four groups: their unit ranges (all 65 offsets come in
        // with one read, lane l holding offset l) and their slot runs (at most
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
            const int share = mine * CH_WAVES / (FORM == FORM_F32 ? 1 : 4);
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
            if (FORM == FORM_F32) {
                // Each entry's slot comes from v_readlane into a scalar
                // register, so the value read needs no second LDS round trip.
                // Entries go a unit (four) at a time: one 16-byte read brings
                // this lane's pixel's four weights, and the step's five LDS
                // reads are in flight together ahead of its sixteen MFMAs.  A
                // run's last unit multiplies only its real entries.
                const uint32_t slot_lane = slK[k];
                const char* wq = ew + e * F::WB + q * 16;
                const char* vl = vals + lane * 16;
                int j = 0;
                for (; j + 4 <= n; j += 4) {
                    uint32_t s0 = __builtin_amdgcn_readlane(slot_lane, j);
                    uint32_t s1 = __builtin_amdgcn_readlane(slot_lane, j + 1);
                    uint32_t s2 = __builtin_amdgcn_readlane(slot_lane, j + 2);
                    uint32_t s3 = __builtin_amdgcn_readlane(slot_lane, j + 3);
                    const float4 a = *(const float4*)(wq + j * 16);
                    float4 v0 = *(const float4*)(vl + s0 * F::RB);
                    float4 v1 = *(const float4*)(vl + s1 * F::RB);
                    float4 v2 = *(const float4*)(vl + s2 * F::RB);
                    float4 v3 = *(const float4*)(vl + s3 * F::RB);
                    mfma4_f32(part, a.x, v0);
                    mfma4_f32(part, a.y, v1);
                    mfma4_f32(part, a.z, v2);
                    mfma4_f32(part, a.w, v3);
                    // schedule: all LDS reads of the step, then its MFMAs
                    __builtin_amdgcn_sched_group_barrier(0x100, 5, 0);
                    __builtin_amdgcn_sched_group_barrier(0x008, 16, 0);
                }
                if (j < n) {
                    const int r = n - j;  // 1..3 entries left
                    const float4 a = *(const float4*)(wq + j * 16);
                    mfma4_f32(part, a.x,
                              *(const float4*)(vl + __builtin_amdgcn_readlane(slot_lane, j) * F::RB));
                    if (r > 1)
                        mfma4_f32(part, a.y, *(const float4*)(vl + __builtin_amdgcn_readlane(
                                                                       slot_lane, j + 1) * F::RB));
                    if (r > 2)
                        mfma4_f32(part, a.z, *(const float4*)(vl + __builtin_amdgcn_readlane(
                                                                       slot_lane, j + 2) * F::RB));
                }
            } else {
                // groups of four entries, slots picked by v_readlane
                const uint32_t slot_lane = slK[k];
                for (int t = 0; t < n / 4; t++) {
                    uint32_t s0 = __builtin_amdgcn_readlane(slot_lane, 4 * t + 0);
                    uint32_t s1 = __builtin_amdgcn_readlane(slot_lane, 4 * t + 1);
                    uint32_t s2 = __builtin_amdgcn_readlane(slot_lane, 4 * t + 2);
                    uint32_t s3 = __builtin_amdgcn_readlane(slot_lane, 4 * t + 3);
                    uint2 a = *(const uint2*)(ew + (e + t) * 32 + q * 8);
                    uint2 v0 = *(const uint2*)(vals + s0 * F::RB + lane * 8);
                    uint2 v1 = *(const uint2*)(vals + s1 * F::RB + lane * 8);
                    uint2 v2 = *(const uint2*)(vals + s2 * F::RB + lane * 8);
                    uint2 v3 = *(const uint2*)(vals + s3 * F::RB + lane * 8);
                    mfma4_16<DT>(part, a, v0, v1, v2, v3);
                }
            }
#pragma unroll
            for (int g = 0; g < G; g++) acc[k][g] += part[g];
        }
    }

    // Epilogue.  acc[k][g] register i, lane l = pixel i of group k, channel
    // c_lo + 4l + g.  Normalised values go through LDS ([pixel][channel],
    // 128 channels per pass) so that the [c][j][i] output is written as rows
    // of 16 contiguous pixels instead of one scattered float per lane.
    __syncthreads();
    float* ol = (float*)smem;
    const int64_t P = (int64_t)nx * ny;
    const int x0 = tx * TILE_PX, y0 = ty * TILE_PX;
#pragma unroll
    for (int h = 0; h < 2; h++) {
        if ((lane >> 5) == h) {
#pragma unroll
            for (int k = 0; k < PGW; k++) {
                if (!pv[k]) continue;
#pragma unroll
                for (int i = 0; i < 4; i++) {
                    int pxl = lxs[k] * PG + (i & 1), pyl = lys[k] * PG + (i >> 1);
                    if (x0 + pxl >= nx || y0 + pyl >= ny) continue;
                    float W = pix_Wf[(int64_t)(y0 + pyl) * nx + x0 + pxl];
                    float4 v = make_float4(acc[k][0][i] / W, acc[k][1][i] / W, acc[k][2][i] / W,
                                           acc[k][3][i] / W);
                    *(float4*)(ol + (pyl * TILE_PX + pxl) * OUT_STRIDE + 4 * (lane & 31)) = v;
                }
            }
        }
        __syncthreads();
        for (int t = threadIdx.x; t < (CW / 2) * TILE_PX * (TILE_PX / 4); t += CH_THREADS) {
            int qd = t % (TILE_PX / 4), row = t / (TILE_PX / 4);
            int pyl = row % TILE_PX, cl = row / TILE_PX;
            int c = c_lo + h * (CW / 2) + cl, y = y0 + pyl, x = x0 + 4 * qd;
            if (c >= nchan || y >= ny || x >= nx) continue;
            const float* src = ol + (pyl * TILE_PX + 4 * qd) * OUT_STRIDE + cl;
            float* dst = out + (int64_t)c * P + (int64_t)y * nx + x;
            if (out_vec && x + 3 < nx) {
                *(float4*)dst = make_float4(src[0], src[OUT_STRIDE], src[2 * OUT_STRIDE],
                                            src[3 * OUT_STRIDE]);
            } else {
                for (int j = 0; j < 4 && x + j < nx; j++) dst[j] = src[j * OUT_STRIDE];
            }
        }
        __syncthreads();
    }
}

template <int FORM, int DT, bool VEC>
__global__ __launch_bounds__(CH_THREADS) void k_channels(
    const void* __restrict__ values, int64_t ld, int32_t nchan, int32_t ncb, int32_t npgx,
    int32_t npgy, int32_t ntx, int32_t nx, int32_t ny, int32_t chunk,
    const int64_t* __restrict__ tile_base, const uint32_t* __restrict__ slot_idx,
    const int64_t* __restrict__ tile_blk, const int64_t* __restrict__ blk_base,
    const uint16_t* __restrict__ blk_pgoff, const void* __restrict__ ent_w,
    const void* __restrict__ ent_s, const float* __restrict__ pix_Wf, float* __restrict__ out,
    int32_t out_vec, int32_t ucap, int32_t nbuf, const int64_t* __restrict__ order) {
    extern __shared__ __attribute__((aligned(16))) char smem[];
    // Workgroup b takes the plan's item order[b] (tile * ncb + channel block),
    // laid out as for the batched form: a tile's channel blocks on one XCD,
    // tiles placed longest first over the XCDs, each XCD's items by decreasing
    // cost; -1 marks an idle workgroup.
    const int64_t item = order[blockIdx.x];
    if (item < 0) return;
    grid_item<FORM, DT, VEC>(values, ld, nchan, npgx, npgy, ntx, nx, ny, chunk, tile_base,
                             slot_idx, tile_blk, blk_base, blk_pgoff, ent_w, ent_s, pix_Wf, out,
                             out_vec, ucap, nbuf, item / ncb, item % ncb, smem);
}

// Batched form: one launch over the (field, tile, channel block) items of many
// fields.  Workgroup b takes item b.  The host lays the items out so that the
// hardware's in-order, round-robin dispatch does the scheduling: position b
// runs on XCD b mod 8, each XCD's items were assigned by longest-processing-
// time-first over the 8 XCDs with a tile's channel blocks kept together (one
// L2), and within an XCD they are ordered by decreasing cost, so a CU that
// frees up always takes the largest item left.  Padding items (field < 0)
// return at once.
template <int FORM, int DT, bool VEC>
__global__ __launch_bounds__(CH_THREADS) void k_channels_batch(
    const FieldDesc* __restrict__ fields, const BatchItem* __restrict__ items) {
    extern __shared__ __attribute__((aligned(16))) char smem[];
    // descriptors and items are never written by the kernel: reading them
    // through the constant address space keeps them in scalar registers
    const CONST_AS BatchItem* it = (const CONST_AS BatchItem*)items + blockIdx.x;
    const int32_t f = it->field;
    if (f < 0) return;
    const CONST_AS FieldDesc& d = ((const CONST_AS FieldDesc*)fields)[f];
    grid_item<FORM, DT, VEC>(d.values, d.ld, d.nchan, d.npgx, d.npgy, d.ntx, d.nx, d.ny, d.chunk,
                             d.tile_base, d.slot_idx, d.tile_blk, d.blk_base, d.blk_pgoff,
                             d.ent_w, d.ent_s, d.pix_Wf, d.out, d.out_vec, d.ucap, d.nbuf,
                             it->tile, it->cb, smem);
}

// LDS plan of a field: entry capacity, resident chunks and dynamic LDS bytes
// (the output transpose of the epilogue reuses the same space).
size_t lds_stride(bool m16, int chunk, int ucap) {
    return m16 ? LdsLayout::make<FORM_M16>(chunk, ucap).stride
               : LdsLayout::make<FORM_F32>(chunk, ucap).stride;
}

void lds_plan(bool m16, int chunk, int blk_max, int32_t& ucap, int32_t& nbuf) {
    ucap = (blk_max < 4 ? 4 : (blk_max + 3) / 4 * 4);
    nbuf = (int32_t)((LDS_BYTES - META_LDS) / lds_stride(m16, chunk, ucap));
    if (nbuf > MAX_NBUF) nbuf = MAX_NBUF;
    if (nbuf < 2) nbuf = 2;  // not reached: a block holds at most 64 x chunk entries
}

size_t lds_shm(bool m16, int chunk, int ucap, int nbuf) {
    size_t shm = (size_t)nbuf * lds_stride(m16, chunk, ucap) + META_LDS;
    return shm < (size_t)OUT_LDS ? (size_t)OUT_LDS : shm;
}

template <int FORM, int DT, bool VEC>
hipError_t launch_typed(const FieldDesc& d, const int64_t* order, int64_t nwg, hipStream_t s) {
    size_t shm = lds_shm(FORM == FORM_M16, d.chunk, d.ucap, d.nbuf);
    auto kern = k_channels<FORM, DT, VEC>;
    if (shm > 65536) {
        hipError_t e = hipFuncSetAttribute((const void*)kern,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(kern, dim3((unsigned)nwg), dim3(CH_THREADS), shm, s, d.values, d.ld,
                       d.nchan, d.ncb, d.npgx, d.npgy, d.ntx, d.nx, d.ny, d.chunk, d.tile_base,
                       d.slot_idx, d.tile_blk, d.blk_base, d.blk_pgoff, d.ent_w, d.ent_s,
                       d.pix_Wf, d.out, d.out_vec, d.ucap, d.nbuf, order);
    return hipGetLastError();
}

// One function pointer per (form, dtype, vec) for the two launch forms.
template <template <int, int, bool> class K>
const void* pick(bool m16, int32_t dtype, bool vec) {
    if (m16) {
        if (dtype == HG_BF16)
            return vec ? K<FORM_M16, HG_BF16, true>::f() : K<FORM_M16, HG_BF16, false>::f();
        return vec ? K<FORM_M16, HG_F16, true>::f() : K<FORM_M16, HG_F16, false>::f();
    }
    if (dtype == HG_F32)
        return vec ? K<FORM_F32, HG_F32, true>::f() : K<FORM_F32, HG_F32, false>::f();
    if (dtype == HG_BF16)
        return vec ? K<FORM_F32, HG_BF16, true>::f() : K<FORM_F32, HG_BF16, false>::f();
    return vec ? K<FORM_F32, HG_F16, true>::f() : K<FORM_F32, HG_F16, false>::f();
}
template <int FORM, int DT, bool VEC>
struct BatchKernel {
    static const void* f() { return (const void*)k_channels_batch<FORM, DT, VEC>; }
};

}  // namespace

bool values_vec(const Plan& P, const void* values, int64_t ld, int32_t dtype) {
    uintptr_t a = (uintptr_t)values;
    if (P.opts.precision != HG_PREC_FP32) return a % 16 == 0 && ld % 8 == 0;
    if (dtype == HG_F32) return a % 16 == 0 && ld % 4 == 0;
    return a % 8 == 0 && ld % 4 == 0;
}

FieldDesc field_desc(const Plan& P, const void* values, int64_t ld, int32_t nchan, float* out) {
    FieldDesc d{};
    bool m16 = P.opts.precision != HG_PREC_FP32;
    d.values = values;
    d.ld = ld;
    d.nchan = nchan;
    d.ncb = (nchan + CW - 1) / CW;
    d.npgx = P.npgx;
    d.npgy = P.npgy;
    d.ntx = P.ntx;
    d.nx = P.map.nx;
    d.ny = P.map.ny;
    d.chunk = P.chunk;
    lds_plan(m16, P.chunk, P.blk_max, d.ucap, d.nbuf);
    d.out_vec = ((uintptr_t)out % 16 == 0) && (P.map.nx % 4 == 0);
    d.tile_base = (const int64_t*)P.tile_nslots.p;
    d.slot_idx = (const uint32_t*)P.slot_idx.p;
    d.tile_blk = (const int64_t*)P.tile_blk.p;
    d.blk_base = (const int64_t*)P.blk_base.p;
    d.blk_pgoff = (const uint16_t*)P.blk_pgoff.p;
    d.ent_w = m16 ? P.e3_w.p : P.e2_w.p;
    d.ent_s = m16 ? P.e3_s.p : P.e2_s.p;
    d.pix_Wf = (const float*)P.pix_Wf.p;
    d.out = out;
    return d;
}

hipError_t launch_channels(Plan& P, const void* values, int64_t ld, int32_t nchan, int32_t dtype,
                           float* out, hipStream_t s) {
    bool vec = values_vec(P, values, ld, dtype);
    FieldDesc d = field_desc(P, values, ld, nchan, out);
    const int64_t* order = nullptr;
    int64_t nwg = 0;
    hipError_t e = launch_order(P, d.ncb, s, &order, &nwg);
    if (e != hipSuccess) return e;
    if (P.opts.precision != HG_PREC_FP32) {
        if (dtype == HG_BF16)
            return vec ? launch_typed<FORM_M16, HG_BF16, true>(d, order, nwg, s)
                       : launch_typed<FORM_M16, HG_BF16, false>(d, order, nwg, s);
        return vec ? launch_typed<FORM_M16, HG_F16, true>(d, order, nwg, s)
                   : launch_typed<FORM_M16, HG_F16, false>(d, order, nwg, s);
    }
    if (dtype == HG_F32)
        return vec ? launch_typed<FORM_F32, HG_F32, true>(d, order, nwg, s)
                   : launch_typed<FORM_F32, HG_F32, false>(d, order, nwg, s);
    if (dtype == HG_BF16)
        return vec ? launch_typed<FORM_F32, HG_BF16, true>(d, order, nwg, s)
                   : launch_typed<FORM_F32, HG_BF16, false>(d, order, nwg, s);
    return vec ? launch_typed<FORM_F32, HG_F16, true>(d, order, nwg, s)
               : launch_typed<FORM_F32, HG_F16, false>(d, order, nwg, s);
}

bool channel_lds_fits(bool m16, int chunk, int blk_max) {
    int32_t ucap, nbuf;
    lds_plan(m16, chunk, blk_max, ucap, nbuf);
    return (size_t)2 * lds_stride(m16, chunk, ucap) + META_LDS <= (size_t)LDS_BYTES;
}

size_t field_lds_bytes(const FieldDesc& d, bool m16) {
    return lds_shm(m16, d.chunk, d.ucap, d.nbuf);
}

BatchKernelInfo batch_kernel(bool m16, int32_t dtype, bool vec, size_t shm) {
    BatchKernelInfo k;
    k.main = pick<BatchKernel>(m16, dtype, vec);
    k.shm = shm;
    k.threads = CH_THREADS;
    k.channels_per_block = CW;
    return k;
}

}  // namespace hg
