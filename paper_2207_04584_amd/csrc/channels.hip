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
//     channels of every slot (one 1 KB row per sample, read from the
//     channel-contiguous values in HBM) and the chunk's entry block (the
//     (group, slot, four weights) entries of all 64 groups, prepared by setup);
//   * staging is double-buffered: the loads for chunk c+1 go straight from
//     global memory to LDS (global_load_lds) while the waves compute chunk c;
//   * each wave owns 4 pixel groups spread over the tile; per entry it reads one 16-byte value
//     vector per lane and issues four FP32 MFMA 4x4x1 (16 blocks)
//     instructions: A = the group's four weights (rows = pixels), B = one
//     value per lane (columns = channels 4*lane + g), so one entry updates
//     4 pixels x 256 channels with FP32 multiply-adds;
//   * FP32 summation is two-level: each chunk's entries accumulate into a
//     fresh MFMA tile that is then added to the group's total, so no serial
//     FP32 chain is longer than one chunk;
//   * while chunk c is computed, chunk c+1 is being copied and chunk c+2's
//     rows are prefetched into L2, so the copy that follows hits in L2;
//   * the epilogue divides by the FP32 weight sum and writes [c][j][i] as
//     rows of 16 pixels after a transpose through LDS.
#include "hg_common.h"

namespace hg {
namespace {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) void lds_void;

constexpr int CH_WAVES = 16;
constexpr int CH_THREADS = 64 * CH_WAVES;
constexpr int G = 4;        // 64-channel groups per workgroup
constexpr int CW = 64 * G;  // channels per workgroup (256)
constexpr int PGW = TILE_PGS / CH_WAVES;
constexpr int TILE_PX = TILE_PGX * PG;  // 16 pixels per tile side
constexpr int OUT_STRIDE = CW / 2 + 4;  // LDS floats per pixel in the output transpose
constexpr int OUT_LDS = TILE_PX * TILE_PX * OUT_STRIDE * 4;
constexpr int TRASH_LDS = 256;
static_assert(TILE_PGX == 8 && TILE_PGY == 8 && CH_WAVES == 16, "wave/group mapping assumes 8x8 groups, 16 waves");

__device__ inline float bf16_bits_to_f32(uint32_t b) { return __uint_as_float(b << 16); }

__device__ inline float f16_bits_to_f32(uint32_t b) {
    _Float16 h;
    uint16_t u = (uint16_t)b;
    __builtin_memcpy(&h, &u, 2);
    return (float)h;
}

struct LdsLayout {
    int vals, ew, es, po, stride;
    __device__ __host__ static LdsLayout make(int chunk) {
        LdsLayout L;
        L.vals = 0;
        L.ew = L.vals + chunk * CW * 4;
        L.es = L.ew + TILE_PGS * chunk * 16;
        L.po = L.es + TILE_PGS * chunk * 4;
        L.stride = L.po + 144;
        return L;
    }
};

// Direct global -> LDS copies (lane i writes bytes [i*size, (i+1)*size) after
// the wave-uniform LDS address).  They are issued through inline assembly so
// that the compiler does not order every later LDS read behind them: the
// kernel itself waits for them (s_waitcnt vmcnt(0)) before the barrier that
// hands a staged chunk to the compute loop.
__device__ inline uint32_t lds_addr(const char* l) {
    return __builtin_amdgcn_readfirstlane((uint32_t)(uintptr_t)(lds_void*)l);
}
__device__ inline void dma16(const void* g, const char* l) {
    asm volatile("s_mov_b32 m0, %1\n\ts_nop 1\n\tglobal_load_lds_dwordx4 %0, off"
                 :
                 : "v"(g), "s"(lds_addr(l))
                 : "memory", "m0");
}
__device__ inline void dma4(const void* g, const char* l) {
    asm volatile("s_mov_b32 m0, %1\n\ts_nop 1\n\tglobal_load_lds_dword %0, off"
                 :
                 : "v"(g), "s"(lds_addr(l))
                 : "memory", "m0");
}

// One staged row: channels [c_lo, c_lo + 256) of sample `row`, as FP32.
template <int DT, bool VEC>
__device__ inline void stage_row(char* dst, const void* values, int64_t ld, int32_t nchan, int c_lo,
                                 uint32_t row, int lane) {
    int c = c_lo + 4 * lane;
    if (DT == HG_F32) {
        const float* src = (const float*)values + (int64_t)row * ld;
        if (VEC && c_lo + CW <= nchan) {
            // wave-uniform: whole row in range, 16-byte aligned -> direct to LDS
            dma16(src + c, dst);
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

__device__ inline void mfma4(v4f* part, float a, float4 v) {
    part[0] = __builtin_amdgcn_mfma_f32_4x4x1f32(a, v.x, part[0], 0, 0, 0);
    part[1] = __builtin_amdgcn_mfma_f32_4x4x1f32(a, v.y, part[1], 0, 0, 0);
    part[2] = __builtin_amdgcn_mfma_f32_4x4x1f32(a, v.z, part[2], 0, 0, 0);
    part[3] = __builtin_amdgcn_mfma_f32_4x4x1f32(a, v.w, part[3], 0, 0, 0);
}

template <int DT, bool VEC>
__global__ __launch_bounds__(CH_THREADS) void k_channels_fp32(
    const void* __restrict__ values, int64_t ld, int32_t nchan, int32_t ncb, int32_t npgx,
    int32_t npgy, int32_t ntx, int64_t ntiles, int32_t nx, int32_t ny, int32_t chunk,
    const int64_t* __restrict__ tile_base, const uint32_t* __restrict__ slot_idx,
    const int64_t* __restrict__ tile_blk, const int64_t* __restrict__ blk_base,
    const uint16_t* __restrict__ blk_pgoff, const float4* __restrict__ e2_w,
    const uint32_t* __restrict__ e2_s, const float* __restrict__ pix_Wf, float* __restrict__ out,
    int32_t out_vec) {
    extern __shared__ __attribute__((aligned(16))) char smem[];
    const LdsLayout L = LdsLayout::make(chunk);
    char* trash = smem + 2 * L.stride;

    // Workgroups are dispatched round-robin over the 8 XCDs; give each XCD a
    // contiguous run of (tile, channel block) so that a tile's channel blocks
    // (which share its entry blocks) and neighbouring tiles (which share halo
    // samples) meet in the same L2.
    int64_t nwg = gridDim.x, b = blockIdx.x;
    int64_t q8 = nwg / 8, r8 = nwg % 8, xcd = b % 8, idx = b / 8;
    int64_t logical = xcd * q8 + (xcd < r8 ? xcd : r8) + idx;
    int64_t tile = logical / ncb, cb = logical % ncb;
    int tx = (int)(tile % ntx), ty = (int)(tile / ntx);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int c_lo = (int)cb * CW;
    // value rows go straight to LDS when they are FP32, aligned and complete
    const bool dma_rows = DT == HG_F32 && VEC && c_lo + CW <= nchan;

    const int64_t s_base = tile_base[tile];
    const int64_t nslots = tile_base[tile + 1] - s_base;
    const int64_t blk0 = tile_blk[tile];
    const int64_t nch = tile_blk[tile + 1] - blk0;
    const uint32_t* sidx = slot_idx + s_base;

    // Wave w owns the groups whose (x mod 4, y mod 4) is (w mod 4, w / 4): a
    // chunk's samples are spatially compact, so this spreads each chunk's
    // entries evenly over the 16 waves.
    bool pv[PGW];
    int lxs[PGW], lys[PGW];
#pragma unroll
    for (int k = 0; k < PGW; k++) {
        lxs[k] = (wave & 3) + 4 * (k & 1);
        lys[k] = (wave >> 2) + 4 * (k >> 1);
        pv[k] = tx * TILE_PGX + lxs[k] < npgx && ty * TILE_PGY + lys[k] < npgy;
    }

    // Per chunk each wave needs its staged rows' sample indices and the entry
    // block's range.  All indices are wave-uniform, so these are scalar loads:
    // the vector-memory counter then only counts the asynchronous copies,
    // which the pipeline below waits for explicitly.
    struct Meta {
        uint32_t row0, row1, first;
        int nrows;
        int64_t blk, eb;
        int ne;
    };
    auto load_meta = [&](int64_t ch) {
        Meta m;
        int64_t s0 = ch * chunk;
        int ns = (int)((nslots - s0) < chunk ? (nslots - s0) : chunk);
        m.first = sidx[s0];
        m.nrows = (wave < ns) + (wave + CH_WAVES < ns);  // chunk <= 32: at most two rows
        m.row0 = wave < ns ? sidx[s0 + wave] : m.first;
        m.row1 = wave + CH_WAVES < ns ? sidx[s0 + wave + CH_WAVES] : m.first;
        m.blk = blk0 + ch;
        m.eb = blk_base[m.blk];
        m.ne = (int)(blk_base[m.blk + 1] - m.eb);
        return m;
    };
    auto issue = [&](const Meta& m, int buf) {
        char* base = smem + buf * L.stride;
        if (m.nrows > 0)
            stage_row<DT, VEC>(base + L.vals + wave * CW * 4, values, ld, nchan, c_lo, m.row0,
                               lane);
        if (m.nrows > 1)
            stage_row<DT, VEC>(base + L.vals + (wave + CH_WAVES) * CW * 4, values, ld, nchan,
                               c_lo, m.row1, lane);
        for (int i = wave * 64; i < m.ne; i += CH_THREADS) {
            if (i + lane < m.ne) {
                dma16(e2_w + m.eb + i + lane, base + L.ew + i * 16);
                dma4(e2_s + m.eb + i + lane, base + L.es + i * 4);
            }
        }
        if (wave == CH_WAVES - 1 && lane < PGOFF_STRIDE / 2)
            dma4((const uint32_t*)(blk_pgoff + m.blk * PGOFF_STRIDE) + lane, base + L.po);
    };
    // L2 prefetch of a later chunk's rows: exactly one copy instruction per
    // wave (lanes touch both halves of every 128-byte line of the wave's rows;
    // the data lands in a scratch area of LDS and is never read).
    auto prefetch = [&](const Meta& m) {
        int q = lane >> 4, part = lane & 15;
        uint32_t row = q == 0 ? m.row0 : m.row1;
        const float* src = (const float*)values + (int64_t)row * ld + c_lo + part * 16;
        if (lane < 32 && (q < m.nrows || lane == 0)) dma4(src, trash);
    };

    v4f acc[PGW][G];
#pragma unroll
    for (int k = 0; k < PGW; k++)
#pragma unroll
        for (int g = 0; g < G; g++) acc[k][g] = (v4f){0.f, 0.f, 0.f, 0.f};

    Meta m1{}, m2{};
    bool pf = false;  // a prefetch is the youngest outstanding copy
    if (nch > 0) {
        Meta m0 = load_meta(0);
        if (nch > 1) m1 = load_meta(1);
        if (nch > 2) m2 = load_meta(2);
        issue(m0, 0);
        if (dma_rows && nch > 1) {
            prefetch(m1);
            pf = true;
        }
    }
    for (int64_t ch = 0; ch < nch; ch++) {
        // Chunk ch's copies are complete (only the prefetch, if any, may still
        // be in flight); the barrier makes every wave's copies visible and
        // retires all reads of the other buffer.
        if (pf)
            __builtin_amdgcn_s_waitcnt(0x3F71);  // vmcnt(1) expcnt(7) lgkmcnt(15)
        else
            __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        pf = false;
        if (ch + 1 < nch) {
            Meta m3 = (ch + 3 < nch) ? load_meta(ch + 3) : m2;
            issue(m1, (int)((ch + 1) & 1));
            if (dma_rows && ch + 2 < nch) {
                prefetch(m2);
                pf = true;
            }
            m1 = m2;
            m2 = m3;
        }
        const char* base = smem + (ch & 1) * L.stride;
        const float* vals = (const float*)(base + L.vals);
        const float* ew = (const float*)(base + L.ew);
        const uint32_t* es = (const uint32_t*)(base + L.es);
        const uint16_t* po = (const uint16_t*)(base + L.po);
#pragma unroll
        for (int k = 0; k < PGW; k++) {
            if (!pv[k]) continue;
            int lp = lys[k] * TILE_PGX + lxs[k];
            // the group's entry range is wave-uniform: keep it in scalar registers
            int e = __builtin_amdgcn_readfirstlane((int)po[lp]);
            int e1 = __builtin_amdgcn_readfirstlane((int)po[lp + 1]);
            if (e == e1) continue;
            v4f part[G];
#pragma unroll
            for (int g = 0; g < G; g++) part[g] = (v4f){0.f, 0.f, 0.f, 0.f};
            // The group's run of at most `chunk` (<= 64) slots is read with one
            // coalesced LDS load, lane i holding entry e+i; each entry's slot
            // then comes from v_readlane into a scalar register, so the value
            // read needs no second LDS round trip.
            const int q = lane & 3;
            const int n = e1 - e;
            uint32_t slot_lane = es[e + (lane < n ? lane : 0)];
            const float* ewq = ew + e * 4 + q;
            for (int j = 0; j < n; j++) {
                uint32_t sj = __builtin_amdgcn_readlane(slot_lane, j);
                float a0 = ewq[j * 4];
                float4 v0 = ((const float4*)(vals + sj * CW))[lane];
                mfma4(part, a0, v0);
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
    const int x0 = tx * TILE_PGX * PG, y0 = ty * TILE_PGY * PG;
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

template <int DT, bool VEC>
hipError_t launch_typed(Plan& P, const void* values, int64_t ld, int32_t nchan, float* out,
                        hipStream_t s) {
    int64_t ncb = (nchan + CW - 1) / CW;
    int64_t nwg = ncb * P.ntiles;
    size_t shm = (size_t)2 * LdsLayout::make(P.chunk).stride + TRASH_LDS;
    if (shm < (size_t)OUT_LDS) shm = OUT_LDS;
    auto kern = k_channels_fp32<DT, VEC>;
    if (shm > 65536) {
        hipError_t e = hipFuncSetAttribute((const void*)kern,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(kern, dim3((unsigned)nwg), dim3(CH_THREADS), shm, s, values, ld, nchan,
                       (int32_t)ncb, P.npgx, P.npgy, P.ntx, P.ntiles, P.map.nx, P.map.ny, P.chunk,
                       (const int64_t*)P.tile_nslots.p, (const uint32_t*)P.slot_idx.p,
                       (const int64_t*)P.tile_blk.p, (const int64_t*)P.blk_base.p,
                       (const uint16_t*)P.blk_pgoff.p, (const float4*)P.e2_w.p,
                       (const uint32_t*)P.e2_s.p, (const float*)P.pix_Wf.p, out,
                       (int32_t)(((uintptr_t)out % 16 == 0) && (P.map.nx % 4 == 0)));
    return hipGetLastError();
}

}  // namespace

hipError_t launch_channels(Plan& P, const void* values, int64_t ld, int32_t nchan, int32_t dtype,
                           float* out, hipStream_t s) {
    uintptr_t a = (uintptr_t)values;
    if (dtype == HG_F32) {
        bool vec = (a % 16 == 0) && (ld % 4 == 0);
        return vec ? launch_typed<HG_F32, true>(P, values, ld, nchan, out, s)
                   : launch_typed<HG_F32, false>(P, values, ld, nchan, out, s);
    }
    bool vec = (a % 8 == 0) && (ld % 4 == 0);
    if (dtype == HG_BF16)
        return vec ? launch_typed<HG_BF16, true>(P, values, ld, nchan, out, s)
                   : launch_typed<HG_BF16, false>(P, values, ld, nchan, out, s);
    return vec ? launch_typed<HG_F16, true>(P, values, ld, nchan, out, s)
               : launch_typed<HG_F16, false>(P, values, ld, nchan, out, s);
}

}  // namespace hg
