// Host runtime of libhegrid: the C ABI declared in include/hegrid.h, argument
// validation, plan construction (geometry and kernel constants), a caching
// device allocator, channel-kernel timing and the parity exports.
#include <chrono>
#include <cstring>
#include <exception>
#include <map>
#include <mutex>
#include <new>

#include "hg_common.h"

struct hg_plan {
    hg::Plan P;
};

namespace hg {
namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
    g_err = msg;
    return code;
}

int fail_hip(hipError_t e, const char* what) {
    if (e == hipErrorOutOfMemory)
        return fail(HG_ERR_NOMEM, std::string(what) + ": out of device memory");
    return fail(HG_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

// ---------------------------------------------------------------------------
// caching allocator: freed blocks are kept per device and reused by size
// (best fit within 2x), so repeated setups of the same field do not return to
// hipMalloc.  On an allocation failure the cache is released and the
// allocation retried once.
std::mutex g_mu;
std::map<int, std::multimap<size_t, void*>> g_cache;

size_t round_bytes(size_t b) {
    const size_t g = 1 << 16;
    return (b + g - 1) / g * g;
}

void release_cache_locked(int dev) {
    auto& c = g_cache[dev];
    for (auto& kv : c) (void)hipFree(kv.second);
    c.clear();
}

int cur_device() {
    int d = 0;
    (void)hipGetDevice(&d);
    return d;
}

bool g_inited = false;

int ensure_device() {
    if (g_inited) return HG_OK;
    int n = 0;
    hipError_t e = hipGetDeviceCount(&n);
    if (e != hipSuccess || n <= 0) return fail(HG_ERR_DEVICE, "no HIP device available");
    g_inited = true;
    return HG_OK;
}

int64_t choose_nside(Plan& P) {
    if (P.opts.nside > 0) return P.opts.nside;
    const hg_map& m = P.map;
    double cosd = cos(m.dec0_deg * kDeg);
    double w = m.nx * m.dra_deg * kDeg * (cosd > 0.05 ? cosd : 0.05) + 2 * P.r_rad;
    double h = m.ny * m.ddec_deg * kDeg + 2 * P.r_rad;
    double rho = (double)P.n / (w * h);  // samples per steradian near the map
    double target = 0.5 * P.r_rad;
    if (rho > 0) target = fmin(target, sqrt(64.0 / rho));
    if (target < 1e-6) target = 1e-6;
    int64_t N = 1;
    while (N < 8192 && sqrt(kPi / 3.0) / (double)N > target) N *= 2;
    for (;;) {
        P.nside = N;
        plan_band(P, 1e-9);
        if (P.n_cells <= ((int64_t)1 << 25) || N == 1) break;
        N /= 2;
    }
    return N;
}

}  // namespace

hipError_t dev_alloc(DevBuf& b, size_t bytes) {
    if (b.p) dev_free(b);
    size_t want = round_bytes(bytes ? bytes : 1);
    int dev = cur_device();
    {
        std::lock_guard<std::mutex> lk(g_mu);
        auto& c = g_cache[dev];
        auto it = c.lower_bound(want);
        if (it != c.end() && it->first <= 2 * want) {
            b.p = it->second;
            b.bytes = it->first;
            c.erase(it);
            return hipSuccess;
        }
    }
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, want);
    if (e == hipErrorOutOfMemory) {
        (void)hipGetLastError();
        {
            std::lock_guard<std::mutex> lk(g_mu);
            release_cache_locked(dev);
        }
        e = hipMalloc(&p, want);
    }
    if (e != hipSuccess) return e;
    b.p = p;
    b.bytes = want;
    return hipSuccess;
}

void dev_free(DevBuf& b) {
    if (!b.p) return;
    std::lock_guard<std::mutex> lk(g_mu);
    g_cache[cur_device()].emplace(b.bytes, b.p);
    b.p = nullptr;
    b.bytes = 0;
}

namespace {

void plan_free(Plan& P) {
    for (DevBuf* b : {&P.srt_idx, &P.srt_coord, &P.cell_off, &P.tile_piece, &P.tile_nslots,
                      &P.pg_piece, &P.pg_base, &P.pg_cnt, &P.slot_idx, &P.ent_slot, &P.ent_w,
                      &P.cp_base, &P.chunk_ptr, &P.pix_count, &P.pix_W, &P.pix_Wf, &P.scratch,
                      &P.tile_blk, &P.blk_base, &P.blk_pgoff, &P.e2_w, &P.e2_s, &P.e3_w, &P.e3_s})
        dev_free(*b);
    for (auto& e : P.ev_pending) {
        (void)hipEventDestroy(e.first);
        (void)hipEventDestroy(e.second);
    }
    for (auto& e : P.ev_free) {
        (void)hipEventDestroy(e.first);
        (void)hipEventDestroy(e.second);
    }
    P.ev_pending.clear();
    P.ev_free.clear();
}

int64_t plan_bytes(const Plan& P) {
    int64_t s = 0;
    for (const DevBuf* b : {&P.srt_idx, &P.srt_coord, &P.cell_off, &P.tile_piece, &P.tile_nslots,
                            &P.pg_piece, &P.pg_base, &P.pg_cnt, &P.slot_idx, &P.ent_slot, &P.ent_w,
                            &P.cp_base, &P.chunk_ptr, &P.pix_count, &P.pix_W, &P.pix_Wf,
                            &P.scratch, &P.tile_blk, &P.blk_base, &P.blk_pgoff, &P.e2_w, &P.e2_s,
                            &P.e3_w, &P.e3_s})
        s += (int64_t)b->bytes;
    return s;
}

hipError_t resolve_timing(Plan& P) {
    for (auto& e : P.ev_pending) {
        hipError_t r = hipEventSynchronize(e.second);
        if (r != hipSuccess) return r;
        float ms = 0.f;
        r = hipEventElapsedTime(&ms, e.first, e.second);
        if (r != hipSuccess) return r;
        P.ch_ms_total += ms;
        P.ch_ms_last = ms;
        P.ch_timed_calls++;
        P.ev_free.push_back(e);
    }
    P.ev_pending.clear();
    return hipSuccess;
}

bool finite(double x) { return std::isfinite(x); }

int validate_setup(const double* ra, const double* dec, int64_t n, const hg_kernel* k,
                   const hg_map* m, const hg_opts* o) {
    if (!k || !m || (n > 0 && (!ra || !dec)))
        return fail(HG_ERR_ARG, "NULL argument (kernel, map or coordinates)");
    if (n < 0 || n >= ((int64_t)1 << 31)) return fail(HG_ERR_ARG, "n must be in [0, 2^31)");
    if (!finite(k->fwhm_deg) || !(k->fwhm_deg > 0)) return fail(HG_ERR_ARG, "fwhm_deg must be > 0");
    if (!finite(k->support_deg) || !(k->support_deg >= 0) || k->support_deg > 10.0)
        return fail(HG_ERR_ARG, "support_deg must be in [0, 10]");
    if (m->nx <= 0 || m->ny <= 0) return fail(HG_ERR_ARG, "map nx and ny must be > 0");
    if ((int64_t)m->nx * m->ny >= ((int64_t)1 << 31)) return fail(HG_ERR_ARG, "map too large");
    if (!finite(m->ra0_deg) || !finite(m->dec0_deg) || !finite(m->dra_deg) ||
        !finite(m->ddec_deg) || !(m->dra_deg > 0) || !(m->ddec_deg > 0))
        return fail(HG_ERR_ARG, "map centre must be finite and spacings > 0");
    double d0 = m->dec0_deg - (m->ny - 1) / 2.0 * m->ddec_deg;
    double d1 = m->dec0_deg + (m->ny - 1) / 2.0 * m->ddec_deg;
    if (!(d0 > -90.0) || !(d1 < 90.0))
        return fail(HG_ERR_ARG, "pixel centres must lie strictly between the poles");
    if (o) {
        if (o->precision != HG_PREC_FP32 && o->precision != HG_PREC_MFMA_BF16 &&
            o->precision != HG_PREC_MFMA_F16)
            return fail(HG_ERR_UNSUPPORTED, "unknown or unsupported precision form");
        if (o->nside < 0 || o->nside > 16384 || (o->nside & (o->nside - 1)))
            return fail(HG_ERR_ARG, "nside must be 0 or a power of two <= 16384");
        if (o->chunk != 0 && (o->chunk < 8 || o->chunk > MAX_CHUNK || o->chunk % 8))
            return fail(HG_ERR_ARG, "chunk must be 0 or a multiple of 8 in [8, 32]");
        if (o->device_mem_cap < 0) return fail(HG_ERR_ARG, "device_mem_cap must be >= 0");
        if (o->reserved || o->reserved2) return fail(HG_ERR_ARG, "reserved fields must be 0");
    }
    return HG_OK;
}

template <typename F>
int guarded(F&& f) {
    try {
        return f();
    } catch (const std::bad_alloc&) {
        return fail(HG_ERR_NOMEM, "host allocation failed");
    } catch (const std::exception& e) {
        return fail(HG_ERR_INTERNAL, std::string("internal error: ") + e.what());
    } catch (...) {
        return fail(HG_ERR_INTERNAL, "internal error");
    }
}

}  // namespace
}  // namespace hg

using namespace hg;

extern "C" {

const char* hg_last_error(void) { return g_err.c_str(); }

int hg_grid_setup(const double* ra_deg, const double* dec_deg, int64_t n, const hg_kernel* k,
                  const hg_map* m, const hg_opts* o, void* hip_stream, hg_plan** out) {
    return guarded([&]() -> int {
        g_err.clear();
        if (!out) return fail(HG_ERR_ARG, "out must not be NULL");
        *out = nullptr;
        int rc = validate_setup(ra_deg, dec_deg, n, k, m, o);
        if (rc) return rc;
        rc = ensure_device();
        if (rc) return rc;
        auto t0 = std::chrono::steady_clock::now();
        hg_plan* h = new hg_plan();
        Plan& P = h->P;
        P.device = cur_device();
        P.map = *m;
        P.kern = *k;
        if (o) P.opts = *o;
        P.n = n;
        P.sigma = k->fwhm_deg * kDeg / sqrt(8.0 * log(2.0));
        P.r_rad = k->support_deg * kDeg;
        double sh = sin(0.5 * P.r_rad);
        P.h_r = sh * sh;
        P.chunk = (o && o->chunk) ? o->chunk : MAX_CHUNK;
        P.npix = (int64_t)m->nx * m->ny;
        P.npgx = (m->nx + PG - 1) / PG;
        P.npgy = (m->ny + PG - 1) / PG;
        P.npg = (int64_t)P.npgx * P.npgy;
        P.ntx = (P.npgx + TILE_PGX - 1) / TILE_PGX;
        P.nty = (P.npgy + TILE_PGY - 1) / TILE_PGY;
        P.ntiles = (int64_t)P.ntx * P.nty;
        P.nside = choose_nside(P);
        plan_band(P, 1e-9);
        if (P.n_cells > ((int64_t)1 << 28)) {
            delete h;
            return fail(HG_ERR_UNSUPPORTED, "nside too fine for this field (over 2^28 cells)");
        }
        hipStream_t s = (hipStream_t)hip_stream;
        std::string err;
        int status = HG_OK;
        hipError_t e = launch_setup(P, ra_deg, dec_deg, s, err, status);
        if (e != hipSuccess) {
            plan_free(P);
            delete h;
            return fail_hip(e, "grid_setup");
        }
        if (status != HG_OK) {
            plan_free(P);
            delete h;
            return fail(status, err);
        }
        P.setup_ms =
            std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        *out = h;
        return HG_OK;
    });
}

int hg_grid_channels(hg_plan* h, const void* values, int64_t ld, int32_t nchan, int32_t dtype,
                     float* out, void* hip_stream) {
    return guarded([&]() -> int {
        g_err.clear();
        if (!h) return fail(HG_ERR_ARG, "plan must not be NULL");
        Plan& P = h->P;
        if (P.finished) return fail(HG_ERR_STATE, "plan already finished");
        if (nchan < 0) return fail(HG_ERR_ARG, "nchan must be >= 0");
        if (dtype != HG_F32 && dtype != HG_BF16 && dtype != HG_F16)
            return fail(HG_ERR_ARG, "unknown dtype");
        if (nchan == 0) return HG_OK;
        if (!out || (!values && P.n > 0)) return fail(HG_ERR_ARG, "values and out must not be NULL");
        if (ld < nchan) return fail(HG_ERR_ARG, "ld must be >= nchan");
        if (P.opts.precision == HG_PREC_MFMA_BF16 && dtype != HG_BF16)
            return fail(HG_ERR_UNSUPPORTED, "a BF16-MFMA plan grids BF16 values");
        if (P.opts.precision == HG_PREC_MFMA_F16 && dtype != HG_F16)
            return fail(HG_ERR_UNSUPPORTED, "an FP16-MFMA plan grids FP16 values");
        hipError_t e = hipSetDevice(P.device);
        if (e != hipSuccess) return fail_hip(e, "grid_channels");
        hipStream_t s = (hipStream_t)hip_stream;
        bool timed = (P.opts.flags & HG_FLAG_TIME_CHANNELS) != 0;
        std::pair<hipEvent_t, hipEvent_t> ev{nullptr, nullptr};
        if (timed) {
            if (!P.ev_free.empty()) {
                ev = P.ev_free.back();
                P.ev_free.pop_back();
            } else {
                e = hipEventCreate(&ev.first);
                if (e == hipSuccess) e = hipEventCreate(&ev.second);
                if (e != hipSuccess) return fail_hip(e, "grid_channels (events)");
            }
            e = hipEventRecord(ev.first, s);
            if (e != hipSuccess) return fail_hip(e, "grid_channels (events)");
        }
        e = launch_channels(P, values, ld, nchan, dtype, out, s);
        if (e != hipSuccess) return fail_hip(e, "grid_channels");
        if (timed) {
            e = hipEventRecord(ev.second, s);
            if (e != hipSuccess) return fail_hip(e, "grid_channels (events)");
            P.ev_pending.push_back(ev);
        }
        P.ch_calls++;
        return HG_OK;
    });
}

int hg_grid_finish(hg_plan* h) {
    return guarded([&]() -> int {
        g_err.clear();
        if (!h) return HG_OK;
        Plan& P = h->P;
        (void)hipSetDevice(P.device);
        hipError_t e = hipDeviceSynchronize();
        plan_free(P);
        delete h;
        if (e != hipSuccess) return fail_hip(e, "grid_finish");
        return HG_OK;
    });
}

int hg_plan_stats(hg_plan* h, hg_stats* st) {
    return guarded([&]() -> int {
        g_err.clear();
        if (!h || !st) return fail(HG_ERR_ARG, "NULL argument");
        Plan& P = h->P;
        hipError_t e = resolve_timing(P);
        if (e != hipSuccess) return fail_hip(e, "plan_stats");
        std::memset(st, 0, sizeof *st);
        st->n_samples = P.n;
        st->n_used = P.n_used;
        st->nnz = P.nnz;
        st->n_entries = P.nnz_entries;
        st->n_cells = P.n_cells;
        st->total_slots = P.total_slots;
        st->device_bytes = plan_bytes(P);
        st->nside = (int32_t)P.nside;
        st->chunk = P.chunk;
        st->setup_ms = P.setup_ms;
        st->last_channels_ms = P.ch_ms_last;
        st->total_channels_ms = P.ch_ms_total;
        st->channels_calls = P.ch_calls;
        return HG_OK;
    });
}

int hg_plan_counts(const hg_plan* h, int32_t* host_counts) {
    return guarded([&]() -> int {
        g_err.clear();
        if (!h || !host_counts) return fail(HG_ERR_ARG, "NULL argument");
        const Plan& P = h->P;
        hipError_t e = hipMemcpy(host_counts, P.pix_count.p, 4 * (size_t)P.npix,
                                 hipMemcpyDeviceToHost);
        if (e != hipSuccess) return fail_hip(e, "plan_counts");
        return HG_OK;
    });
}

int hg_plan_weight_sums(const hg_plan* h, double* host_W) {
    return guarded([&]() -> int {
        g_err.clear();
        if (!h || !host_W) return fail(HG_ERR_ARG, "NULL argument");
        const Plan& P = h->P;
        hipError_t e = hipMemcpy(host_W, P.pix_W.p, 8 * (size_t)P.npix, hipMemcpyDeviceToHost);
        if (e != hipSuccess) return fail_hip(e, "plan_weight_sums");
        return HG_OK;
    });
}

int hg_plan_neighbours(const hg_plan* h, int64_t* row_ptr, int64_t* idx, float* w, int64_t cap,
                       int64_t* nnz) {
    return guarded([&]() -> int {
        g_err.clear();
        if (!h || !row_ptr || !nnz) return fail(HG_ERR_ARG, "NULL argument");
        const Plan& P = h->P;
        std::vector<int32_t> cnt(P.npix);
        std::vector<int64_t> pgb(P.npg + 1), tb(P.ntiles + 1);
        std::vector<uint32_t> pgc(P.npg), es(P.ent_cap ? P.ent_cap : 1),
            sl(P.total_slots ? P.total_slots : 1);
        std::vector<float> ew(4 * (P.ent_cap ? P.ent_cap : 1));
        hipError_t e = hipMemcpy(cnt.data(), P.pix_count.p, 4 * (size_t)P.npix, hipMemcpyDeviceToHost);
        if (e == hipSuccess)
            e = hipMemcpy(pgb.data(), P.pg_base.p, 8 * (size_t)(P.npg + 1), hipMemcpyDeviceToHost);
        if (e == hipSuccess)
            e = hipMemcpy(tb.data(), P.tile_nslots.p, 8 * (size_t)(P.ntiles + 1),
                          hipMemcpyDeviceToHost);
        if (e == hipSuccess)
            e = hipMemcpy(pgc.data(), P.pg_cnt.p, 4 * (size_t)P.npg, hipMemcpyDeviceToHost);
        if (e == hipSuccess && P.ent_cap)
            e = hipMemcpy(es.data(), P.ent_slot.p, 4 * (size_t)P.ent_cap, hipMemcpyDeviceToHost);
        if (e == hipSuccess && P.ent_cap)
            e = hipMemcpy(ew.data(), P.ent_w.p, 16 * (size_t)P.ent_cap, hipMemcpyDeviceToHost);
        if (e == hipSuccess && P.total_slots)
            e = hipMemcpy(sl.data(), P.slot_idx.p, 4 * (size_t)P.total_slots,
                          hipMemcpyDeviceToHost);
        if (e != hipSuccess) return fail_hip(e, "plan_neighbours");
        row_ptr[0] = 0;
        for (int64_t p = 0; p < P.npix; p++) row_ptr[p + 1] = row_ptr[p] + cnt[p];
        *nnz = row_ptr[P.npix];
        if (cap < *nnz || (!idx && !w)) return HG_OK;
        std::vector<int64_t> fill(row_ptr, row_ptr + P.npix);
        std::vector<std::pair<int64_t, float>> tmp((size_t)*nnz);
        for (int64_t pg = 0; pg < P.npg; pg++) {
            int gx = (int)(pg % P.npgx), gy = (int)(pg / P.npgx);
            int64_t tile = (int64_t)(gy / TILE_PGY) * P.ntx + gx / TILE_PGX;
            for (uint32_t t = 0; t < pgc[pg]; t++) {
                int64_t ei = pgb[pg] + t;
                uint32_t word = es[ei];
                uint32_t slot = word & SLOT_MASK, mask = word >> SLOT_SHIFT;
                int64_t orig = sl[tb[tile] + slot];
                for (int k = 0; k < 4; k++) {
                    if (!(mask & (1u << k))) continue;
                    int64_t i = (int64_t)gx * PG + (k & 1), j = (int64_t)gy * PG + (k >> 1);
                    int64_t p = j * P.map.nx + i;
                    int64_t at = fill[p]++;
                    if (at >= row_ptr[p + 1]) return fail(HG_ERR_INTERNAL, "neighbour export overflow");
                    tmp[at] = {orig, ew[4 * ei + k]};
                }
            }
        }
        for (int64_t p = 0; p < P.npix; p++) {
            if (fill[p] != row_ptr[p + 1]) return fail(HG_ERR_INTERNAL, "neighbour export count");
            std::sort(tmp.begin() + row_ptr[p], tmp.begin() + row_ptr[p + 1]);
        }
        for (int64_t t = 0; t < *nnz; t++) {
            if (idx) idx[t] = tmp[t].first;
            if (w) w[t] = tmp[t].second;
        }
        return HG_OK;
    });
}

int hg_ang2pix_ring(int32_t nside, const double* ra_deg, const double* dec_deg, int64_t n,
                    int64_t* pix, void* hip_stream) {
    return guarded([&]() -> int {
        g_err.clear();
        if (nside < 1 || nside > 16384) return fail(HG_ERR_ARG, "nside must be in [1, 16384]");
        if (n < 0) return fail(HG_ERR_ARG, "n must be >= 0");
        if (n > 0 && (!ra_deg || !dec_deg || !pix)) return fail(HG_ERR_ARG, "NULL argument");
        if (n == 0) return HG_OK;
        int rc = ensure_device();
        if (rc) return rc;
        hipError_t e = launch_ang2pix(nside, ra_deg, dec_deg, n, pix, (hipStream_t)hip_stream);
        if (e != hipSuccess) return fail_hip(e, "ang2pix_ring");
        return HG_OK;
    });
}

}  // extern "C"
