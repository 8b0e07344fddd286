// Algorithm 1 as the paper states it, kept beside the tiled matrix-core path
// to measure what that path's design buys on the same plan and inputs.
//
// Per channel, one launch; per thread, gamma output cells (Sec. 4.3.3's cells
// per thread; here 1, 2 or 4 cells of one 2x2 pixel group, which share one
// candidate list).  A thread walks the HEALPix cell runs of every ring that
// can hold a neighbour of its cells (Alg. 1's ring and pixel ranges, the
// plan's per-group ring pieces), tests each sample in them with the FP64
// haversine, and for those within the support adds w v and w for the
// launch's channel (Eq. 1).  Distances and weights are recomputed for every
// channel and the values are read with the channel's stride, as the
// per-channel kernel of Sec. 4.1.2 does; sums are FP64.
#include "hg_common.h"

namespace hg {
namespace {

template <int GAMMA>
__global__ void k_literal(const int4* __restrict__ pg_piece, int32_t pg_rings,
                          const double4* __restrict__ srt_coord,
                          const uint32_t* __restrict__ srt_idx, int32_t npgx, int32_t npgy,
                          hg_map m, double h_r, double two_s2, const float* __restrict__ values,
                          int64_t ld, int32_t chan, float* __restrict__ out) {
    // thread -> (pixel group, first cell): GAMMA 4 = the whole group, 2 = one
    // row of it, 1 = one cell
    constexpr int PER_PG = 4 / GAMMA;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t npg = (int64_t)npgx * npgy;
    if (t >= npg * PER_PG) return;
    const int64_t pg = t / PER_PG;
    const int sub = (int)(t % PER_PG);
    const int64_t ix = (pg % npgx) * PG, iy = (pg / npgx) * PG;
    int64_t ci[GAMMA], cj[GAMMA];
    bool valid[GAMMA];
    double pra[GAMMA], pdec[GAMMA], pcos[GAMMA];
#pragma unroll
    for (int g = 0; g < GAMMA; g++) {
        const int k = GAMMA == 4 ? g : GAMMA == 2 ? 2 * sub + g : sub;  // cell k of the group
        ci[g] = ix + (k & 1);
        cj[g] = iy + (k >> 1);
        valid[g] = ci[g] < m.nx && cj[g] < m.ny;
        pra[g] = pix_ra(m, ci[g], cj[g]);
        pdec[g] = pix_dec(m, cj[g]);
        pcos[g] = cos(pdec[g]);
    }
    double S[GAMMA], W[GAMMA];
    int cnt[GAMMA];
#pragma unroll
    for (int g = 0; g < GAMMA; g++) {
        S[g] = 0.0;
        W[g] = 0.0;
        cnt[g] = 0;
    }
    const int4* pp = pg_piece + pg * (2 * pg_rings);
    for (int r = 0; r < 2 * pg_rings; r++) {
        const int4 piece = pp[r];  // (first sorted position, length, -, -)
        for (int q = 0; q < piece.y; q++) {
            const double4 c = srt_coord[piece.x + q];
            const uint32_t orig = srt_idx[piece.x + q];
            const float v = values[(int64_t)orig * ld + chan];
#pragma unroll
            for (int g = 0; g < GAMMA; g++) {
                const double sd = sin(0.5 * (c.y - pdec[g]));
                const double sa = sin(0.5 * (c.x - pra[g]));
                const double h = sd * sd + pcos[g] * c.z * sa * sa;
                if (valid[g] && h <= h_r) {
                    const double d = 2.0 * asin(fmin(1.0, sqrt(h)));
                    const double w = exp(-(d * d) / two_s2);
                    S[g] += w * (double)v;
                    W[g] += w;
                    cnt[g]++;
                }
            }
        }
    }
    const int64_t P = (int64_t)m.nx * m.ny;
#pragma unroll
    for (int g = 0; g < GAMMA; g++)
        if (valid[g])
            out[(int64_t)chan * P + cj[g] * m.nx + ci[g]] =
                cnt[g] > 0 ? (float)(S[g] / W[g]) : __builtin_nanf("");
}

}  // namespace

hipError_t launch_literal(const Plan& P, const float* values, int64_t ld, int32_t nchan,
                          float* out, int32_t gamma, int32_t block, hipStream_t s) {
    const int64_t threads = P.npg * (4 / gamma);
    const unsigned grid = (unsigned)((threads + block - 1) / block);
    const double two_s2 = 2.0 * P.sigma * P.sigma;
    for (int32_t c = 0; c < nchan; c++) {
        auto kern = gamma == 4 ? k_literal<4> : gamma == 2 ? k_literal<2> : k_literal<1>;
        hipLaunchKernelGGL(kern, dim3(grid), dim3(block), 0, s, (const int4*)P.pg_piece.p,
                           P.pg_rings, (const double4*)P.srt_coord.p,
                           (const uint32_t*)P.srt_idx.p, P.npgx, P.npgy, P.map, P.h_r, two_s2,
                           values, ld, c, out);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace hg
