// Channel phase of libhegrid: the weighted sums of Eq. (1) for many channels
// against a plan built once by setup (channels are independent, Sec. 4.2; the
// neighbour structure is shared by all of them, Sec. 4.3.1).
//
// For each pixel p and channel c:  S[c,p] = sum_{n in N(p)} w[p,n] v[n,c],
// V[c,p] = S[c,p] / W_p.  This is a sparse (pixels x samples) by dense
// (samples x channels) product.  Layout of the work:
//
//   * a workgroup owns one tile (16 x 16 pixels = 8 x 8 pixel groups of 2 x 2)
//     and one block of 64*G channels;
//   * the tile's candidate samples (its "slots") are staged chunk by chunk in
//     LDS as rows of 64*G channels (channel-contiguous, as the values sit in
//     HBM, so every row is one coalesced read);
//   * each wave owns PGW pixel groups; for every (group, sample) entry of the
//     chunk it issues G FP32 MFMA 4x4x1 (16 blocks) instructions: the A operand
//     is the group's four weights (rows = the four pixels), the B operand is one
//     staged value per lane (columns = 64 consecutive channels), so one entry
//     updates 4 pixels x 64 channels per instruction with FP32 multiply-adds;
//   * the epilogue divides by the FP32 weight sum and writes [c][j][i].
#include "hg_common.h"

namespace hg {
namespace {

typedef float v4f __attribute__((ext_vector_type(4)));

constexpr int CH_WAVES = 16;
constexpr int CH_THREADS = 64 * CH_WAVES;

__device__ inline float bf16_bits_to_f32(uint32_t b) { return __uint_as_float(b << 16); }

__device__ inline float f16_bits_to_f32(uint32_t b) {
    _Float16 h;
    uint16_t u = (uint16_t)b;
    __builtin_memcpy(&h, &u, 2);
    return (float)h;
}

// Stage rows [s0, s0 + ns) of the tile's slots, channels [c_lo, c_lo + 64G),
// into lds[r][0 .. 64G) as FP32 (zero beyond nchan and beyond ns).
template <int DT, int G, bool VEC>
__device__ inline void stage_chunk(float* lds, const void* values, int64_t ld, int32_t nchan,
                                   int c_lo, const uint32_t* sidx, int64_t s0, int ns, int chunk) {
    constexpr int CW = 64 * G;
    if (DT == HG_F32) {
        constexpr int F4 = CW / 4;
        const float* vals = (const float*)values;
        for (int t = threadIdx.x; t < chunk * F4; t += CH_THREADS) {
            int r = t / F4, q = t % F4;
            float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
            if (r < ns) {
                const float* src = vals + (int64_t)sidx[s0 + r] * ld;
                int c = c_lo + 4 * q;
                if (VEC && c + 3 < nchan) {
                    v = *(const float4*)(src + c);
                } else {
                    if (c + 0 < nchan) v.x = src[c + 0];
                    if (c + 1 < nchan) v.y = src[c + 1];
                    if (c + 2 < nchan) v.z = src[c + 2];
                    if (c + 3 < nchan) v.w = src[c + 3];
                }
            }
            ((float4*)lds)[t] = v;
        }
    } else {
        constexpr int F8 = CW / 8;
        const uint16_t* vals = (const uint16_t*)values;
        for (int t = threadIdx.x; t < chunk * F8; t += CH_THREADS) {
            int r = t / F8, q = t % F8;
            uint32_t u[8] = {0, 0, 0, 0, 0, 0, 0, 0};
            bool any = false;
            if (r < ns) {
                const uint16_t* src = vals + (int64_t)sidx[s0 + r] * ld;
                int c = c_lo + 8 * q;
                if (VEC && c + 7 < nchan) {
                    uint4 raw = *(const uint4*)(src + c);
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
                        if (c + k < nchan) u[k] = src[c + k];
                }
                any = true;
            }
            float f[8];
#pragma unroll
            for (int k = 0; k < 8; k++)
                f[k] = any ? (DT == HG_BF16 ? bf16_bits_to_f32(u[k]) : f16_bits_to_f32(u[k])) : 0.f;
            float4* dst = (float4*)(lds + r * CW + 8 * q);
            dst[0] = make_float4(f[0], f[1], f[2], f[3]);
            dst[1] = make_float4(f[4], f[5], f[6], f[7]);
        }
    }
}

template <int DT, int G, int PGW, bool VEC>
__global__ __launch_bounds__(CH_THREADS) void k_channels_fp32(
    const void* __restrict__ values, int64_t ld, int32_t nchan, int32_t npgx, int32_t npgy,
    int32_t ntx, int64_t ntiles, int32_t nx, int32_t ny, int32_t chunk,
    const int64_t* __restrict__ tile_base, const uint32_t* __restrict__ slot_idx,
    const int64_t* __restrict__ cp_base, const uint32_t* __restrict__ chunk_ptr,
    const int64_t* __restrict__ pg_base, const uint32_t* __restrict__ ent_slot,
    const float* __restrict__ ent_w, const float* __restrict__ pix_Wf, float* __restrict__ out) {
    static_assert(PGW * CH_WAVES == TILE_PGS, "waves x groups per wave must cover a tile");
    extern __shared__ float lds[];
    constexpr int CW = 64 * G;

    // Workgroups are dispatched round-robin over the 8 XCDs; give each XCD a
    // contiguous run of (channel block, tile) so that neighbouring tiles, which
    // share halo samples, meet in the same L2.
    int64_t nwg = gridDim.x, b = blockIdx.x;
    int64_t q8 = nwg / 8, r8 = nwg % 8, xcd = b % 8, idx = b / 8;
    int64_t logical = xcd * q8 + (xcd < r8 ? xcd : r8) + idx;
    int64_t cb = logical / ntiles, tile = logical % ntiles;
    int tx = (int)(tile % ntx), ty = (int)(tile / ntx);
    int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    int c_lo = (int)cb * CW;

    int64_t s_base = tile_base[tile];
    int64_t nslots = tile_base[tile + 1] - s_base;
    int64_t nch = (nslots + chunk - 1) / chunk;
    const uint32_t* sidx = slot_idx + s_base;
    const uint32_t* cpt = chunk_ptr + cp_base[tile];

    bool pv[PGW];
    int64_t eb[PGW];
    const uint32_t* cp[PGW];
    int gxs[PGW], gys[PGW];
#pragma unroll
    for (int k = 0; k < PGW; k++) {
        int lp = wave + CH_WAVES * k;
        int gx = tx * TILE_PGX + lp % TILE_PGX, gy = ty * TILE_PGY + lp / TILE_PGX;
        gxs[k] = gx;
        gys[k] = gy;
        pv[k] = gx < npgx && gy < npgy;
        eb[k] = pv[k] ? pg_base[(int64_t)gy * npgx + gx] : 0;
        cp[k] = cpt + (int64_t)lp * (nch + 1);
    }
    v4f acc[PGW][G];
#pragma unroll
    for (int k = 0; k < PGW; k++)
#pragma unroll
        for (int g = 0; g < G; g++) acc[k][g] = (v4f){0.f, 0.f, 0.f, 0.f};

    for (int64_t ch = 0; ch < nch; ch++) {
        int64_t s0 = ch * chunk;
        int ns = (int)((nslots - s0) < chunk ? (nslots - s0) : chunk);
        __syncthreads();
        stage_chunk<DT, G, VEC>(lds, values, ld, nchan, c_lo, sidx, s0, ns, chunk);
        __syncthreads();
#pragma unroll
        for (int k = 0; k < PGW; k++) {
            if (!pv[k]) continue;
            uint32_t e = cp[k][ch], e1 = cp[k][ch + 1];
            if (e == e1) continue;
            const uint32_t* es = ent_slot + eb[k];
            const float* ew = ent_w + eb[k] * 4 + (lane & 3);
            // Two-level FP32 summation: the chunk's entries go into a fresh
            // MFMA accumulator, which is then added to the group's total, so no
            // serial FP32 chain is longer than one chunk.
            v4f part[G];
#pragma unroll
            for (int g = 0; g < G; g++) part[g] = (v4f){0.f, 0.f, 0.f, 0.f};
            for (; e < e1; e++) {
                uint32_t sl = (es[e] & SLOT_MASK) - (uint32_t)s0;
                float a = ew[(int64_t)e * 4];
                const float* row = lds + sl * CW + lane;
#pragma unroll
                for (int g = 0; g < G; g++)
                    part[g] = __builtin_amdgcn_mfma_f32_4x4x1f32(a, row[g * 64], part[g], 0, 0, 0);
            }
#pragma unroll
            for (int g = 0; g < G; g++) acc[k][g] += part[g];
        }
    }

    const int64_t P = (int64_t)nx * ny;
#pragma unroll
    for (int k = 0; k < PGW; k++) {
        if (!pv[k]) continue;
#pragma unroll
        for (int i = 0; i < 4; i++) {
            int px = gxs[k] * PG + (i & 1), py = gys[k] * PG + (i >> 1);
            if (px >= nx || py >= ny) continue;
            int64_t p = (int64_t)py * nx + px;
            float W = pix_Wf[p];
#pragma unroll
            for (int g = 0; g < G; g++) {
                int c = c_lo + g * 64 + lane;
                if (c < nchan) out[(int64_t)c * P + p] = acc[k][g][i] / W;
            }
        }
    }
}

template <int DT, int G, bool VEC>
hipError_t launch_typed(Plan& P, const void* values, int64_t ld, int32_t nchan, float* out,
                        hipStream_t s) {
    constexpr int CW = 64 * G;
    int64_t ncb = (nchan + CW - 1) / CW;
    int64_t nwg = ncb * P.ntiles;
    size_t shm = (size_t)P.chunk * CW * sizeof(float);
    auto kern = k_channels_fp32<DT, G, TILE_PGS / CH_WAVES, VEC>;
    if (shm > 65536) {
        hipError_t e = hipFuncSetAttribute((const void*)kern,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(kern, dim3((unsigned)nwg), dim3(CH_THREADS), shm, s, values, ld, nchan,
                       P.npgx, P.npgy, P.ntx, P.ntiles, P.map.nx, P.map.ny, P.chunk,
                       (const int64_t*)P.tile_nslots.p, (const uint32_t*)P.slot_idx.p,
                       (const int64_t*)P.cp_base.p, (const uint32_t*)P.chunk_ptr.p,
                       (const int64_t*)P.pg_base.p, (const uint32_t*)P.ent_slot.p,
                       (const float*)P.ent_w.p, (const float*)P.pix_Wf.p, out);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_channels(Plan& P, const void* values, int64_t ld, int32_t nchan, int32_t dtype,
                           float* out, hipStream_t s) {
    constexpr int G = 4;
    uintptr_t a = (uintptr_t)values;
    if (dtype == HG_F32) {
        bool vec = (a % 16 == 0) && (ld % 4 == 0);
        return vec ? launch_typed<HG_F32, G, true>(P, values, ld, nchan, out, s)
                   : launch_typed<HG_F32, G, false>(P, values, ld, nchan, out, s);
    }
    bool vec = (a % 16 == 0) && (ld % 8 == 0);
    if (dtype == HG_BF16)
        return vec ? launch_typed<HG_BF16, G, true>(P, values, ld, nchan, out, s)
                   : launch_typed<HG_BF16, G, false>(P, values, ld, nchan, out, s);
    return vec ? launch_typed<HG_F16, G, true>(P, values, ld, nchan, out, s)
               : launch_typed<HG_F16, G, false>(P, values, ld, nchan, out, s);
}

}  // namespace hg
