// Host runtime of libhegrid: the C ABI declared in include/hegrid.h, argument
// validation, plan construction (geometry and kernel constants), a caching
// device allocator, channel-kernel timing and the parity exports.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cstring>
#include <exception>
#include <map>
#include <mutex>
#include <new>
#include <thread>

#include "hg_common.h"

struct hg_plan {
    hg::Plan P;
    bool owned_by_batch = false;  // plans of a batch are freed by hg_batch_destroy
};

struct hg_batch {
    std::vector<hg_plan*> plans;
    int device = 0;
    int32_t dtype = 0;
    hg_opts opts{};
    hg::DevBuf descs, items;
    int64_t n_items = 0, n_positions = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_pending, ev_free;
    int64_t runs = 0, timed_runs = 0;
    double run_ms_last = 0, run_ms_total = 0, setup_ms = 0;
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
    double w, h;  // extent of the map plus the support on each side (radians)
    if (m.proj == HG_PROJ_HEALPIX) {
        double cosd = cos(0.5 * (pix_dec(m, 0) + pix_dec(m, m.ny - 1)));
        w = m.nx * (kPi / (2.0 * m.nside)) * (cosd > 0.05 ? cosd : 0.05) + 2 * P.r_rad;
        h = pix_dec(m, m.ny - 1) - pix_dec(m, 0) + 2 * P.r_rad;
    } else {
        double cosd = cos(m.dec0_deg * kDeg);
        w = m.nx * m.dra_deg * kDeg * (cosd > 0.05 ? cosd : 0.05) + 2 * P.r_rad;
        h = m.ny * m.ddec_deg * kDeg + 2 * P.r_rad;
    }
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

// First chunk length of a batch field: the longest of the form's lengths
// (112, 88 for the 16-bit forms; 56, 48 for FP32) whose predicted densest
// block fits two staged chunks in LDS and keeps a group's run in a chunk
// within a lane each, else the next (64; 32).  A dealt chunk samples its
// whole tile, so a group's mean run in a chunk is the chunk times the
// group's share of the tile's slot region: (R + 1)^2 pi over (16 + 2R)^2 for
// a support of R pixels, whatever the density.  The margins over the mean
// stand for the spread between groups and tiles (measured on 64 fields of
// 2-5 arcmin beams: 2 for the 16-bit forms; 1.2 and 1.5 for the FP32 form,
// whose 56-slot blocks of a 3 arcmin beam already fit within 1.39 of the
// mean); a miss costs the field a second setup at the next length.
int32_t batch_first_chunk(const Plan& P, bool m16) {
    const hg_map& m = P.map;
    const double pix = m.proj == HG_PROJ_HEALPIX ? sqrt(kPi / 3.0) / (double)m.nside
                                                 : m.ddec_deg * kDeg;
    const double R = P.r_rad / pix;
    const double tile = 16.0 + 2.0 * R;
    const double share = kPi * (R + 1.0) * (R + 1.0) / (tile * tile);
    const int32_t c16[2] = {112, 88}, c32[2] = {56, 48};
    const double g16[2] = {2.0, 2.0}, g32[2] = {1.2, 1.5};
    for (int k = 0; k < 2; k++) {
        const int32_t c = m16 ? c16[k] : c32[k];
        const double g = m16 ? g16[k] : g32[k];
        const double run = c * share;
        const double units = 64.0 * (run / 4.0 + 1.0);
        if ((c <= 64 || g * run <= 64.0) && channel_lds_fits(m16, c, (int)(g * units))) return c;
    }
    return m16 ? 64 : 32;
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

// Page-locked host buffers for set-up's small transfers (row tables in,
// sizes out), pooled by size for the life of the process: page-locking
// costs more per call than the copies it speeds up, and copies to or from
// pageable memory are staged by the runtime.  Portable: any device may copy
// through them.
namespace {
std::multimap<size_t, void*> g_host_pool;
}

hipError_t host_alloc(HostBuf& b, size_t bytes) {
    if (b.p) host_free(b);
    const size_t g = 4096;
    const size_t want = ((bytes ? bytes : 1) + g - 1) / g * g;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        auto it = g_host_pool.lower_bound(want);
        if (it != g_host_pool.end() && it->first <= 4 * want) {
            b.p = it->second;
            b.bytes = it->first;
            g_host_pool.erase(it);
            return hipSuccess;
        }
    }
    void* p = nullptr;
    hipError_t e = hipHostMalloc(&p, want, hipHostMallocPortable);
    if (e != hipSuccess) return e;
    b.p = p;
    b.bytes = want;
    return hipSuccess;
}

void host_free(HostBuf& b) {
    if (!b.p) return;
    std::lock_guard<std::mutex> lk(g_mu);
    g_host_pool.emplace(b.bytes, b.p);
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
    ring_free(P.ring);
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
    for (auto& kv : P.orders) {
        dev_free(kv.second.items);
        if (kv.second.ready) {
            (void)hipEventSynchronize(kv.second.ready);  // the upload has read its source
            (void)hipEventDestroy(kv.second.ready);
        }
        host_free(kv.second.host);
    }
    P.orders.clear();
}

int64_t plan_bytes(const Plan& P) {
    int64_t s = 0;
    for (const DevBuf* b : {&P.srt_idx, &P.srt_coord, &P.cell_off, &P.tile_piece, &P.tile_nslots,
                            &P.pg_piece, &P.pg_base, &P.pg_cnt, &P.slot_idx, &P.ent_slot, &P.ent_w,
                            &P.cp_base, &P.chunk_ptr, &P.pix_count, &P.pix_W, &P.pix_Wf,
                            &P.scratch, &P.tile_blk, &P.blk_base, &P.blk_pgoff, &P.e2_w, &P.e2_s,
                            &P.e3_w, &P.e3_s})
        s += (int64_t)b->bytes;
    for (int k = 0; k < RING_SLOTS; k++) s += (int64_t)(P.ring.vals[k].bytes + P.ring.out[k].bytes);
    for (const auto& kv : P.orders) s += (int64_t)kv.second.items.bytes;
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

Shape shape_of(const hg_opts& o) {
    Shape s;
    if (o.waves) s.waves = o.waves;
    if (o.chan_block) s.g = o.chan_block / 64;
    return s;
}

// A buffer the kernels read or write must be device memory of the device they
// run on (hipMalloc, or managed).  Host memory is refused before anything is
// enqueued: pageable memory would fault the GPU (no XNACK here), and
// page-locked memory would be read over the host link.
int require_device(const void* p, int dev, const char* what) {
    hipPointerAttribute_t a;
    hipError_t e = hipPointerGetAttributes(&a, p);
    if (e != hipSuccess) {
        (void)hipGetLastError();  // pageable host memory is reported as an error
        return fail(HG_ERR_ARG, std::string(what) + " is not device memory");
    }
    if (a.type != hipMemoryTypeDevice && a.type != hipMemoryTypeManaged)
        return fail(HG_ERR_ARG, std::string(what) + " is host memory; a device pointer is required");
    if (a.type == hipMemoryTypeDevice && a.device != dev)
        return fail(HG_ERR_ARG, std::string(what) + " is on device " + std::to_string(a.device) +
                                    ", the plan on device " + std::to_string(dev));
    return HG_OK;
}

int validate_map(const hg_map* m) {
    if (!m) return fail(HG_ERR_ARG, "NULL map");
    if (m->nx <= 0 || m->ny <= 0) return fail(HG_ERR_ARG, "map nx and ny must be > 0");
    if ((int64_t)m->nx * m->ny >= ((int64_t)1 << 31)) return fail(HG_ERR_ARG, "map too large");
    if (m->proj == HG_PROJ_HEALPIX) {
        const int64_t ns = m->nside, top = (int64_t)m->ring0 - (m->ny - 1);
        if (m->ra0_deg != 0.0 || m->dec0_deg != 0.0 || m->dra_deg != 0.0 || m->ddec_deg != 0.0)
            return fail(HG_ERR_ARG, "a HEALPix map leaves ra0, dec0, dra and ddec at 0");
        if (ns < 1 || ns > ((int64_t)1 << 20) || (ns & (ns - 1)))
            return fail(HG_ERR_ARG, "HEALPix map nside must be a power of two <= 2^20");
        if (m->pix0 < 0 || m->pix0 >= 4 * ns || m->nx > 4 * ns)
            return fail(HG_ERR_ARG, "HEALPix map needs 0 <= pix0 < 4 nside and nx <= 4 nside");
        if (top < 1 || m->ring0 > 4 * ns - 1)
            return fail(HG_ERR_ARG, "HEALPix map rows ring0 - ny + 1 .. ring0 must be rings "
                                    "1 .. 4 nside - 1");
        if (top < ns || m->ring0 > 3 * ns)
            return fail(HG_ERR_UNSUPPORTED, "HEALPix map rows must lie in the equatorial belt "
                                            "(nside <= ring <= 3 nside)");
        return HG_OK;
    }
    if (m->proj != HG_PROJ_CAR) return fail(HG_ERR_UNSUPPORTED, "unknown map projection");
    if (m->nside || m->ring0 || m->pix0)
        return fail(HG_ERR_ARG, "a plate-carree map leaves nside, ring0 and pix0 at 0");
    if (!finite(m->ra0_deg) || !finite(m->dec0_deg) || !finite(m->dra_deg) ||
        !finite(m->ddec_deg) || !(m->dra_deg > 0) || !(m->ddec_deg > 0))
        return fail(HG_ERR_ARG, "map centre must be finite and spacings > 0");
    double d0 = m->dec0_deg - (m->ny - 1) / 2.0 * m->ddec_deg;
    double d1 = m->dec0_deg + (m->ny - 1) / 2.0 * m->ddec_deg;
    if (!(d0 > -90.0) || !(d1 < 90.0))
        return fail(HG_ERR_ARG, "pixel centres must lie strictly between the poles");
    return HG_OK;
}

int validate_setup(const double* ra, const double* dec, int64_t n, const hg_kernel* k,
                   const hg_map* m, const hg_opts* o) {
    if (!k || !m || (n > 0 && (!ra || !dec)))
        return fail(HG_ERR_ARG, "NULL argument (kernel, map or coordinates)");
    if (n < 0 || n >= ((int64_t)1 << 31)) return fail(HG_ERR_ARG, "n must be in [0, 2^31)");
    if (k->type != HG_KERNEL_GAUSS && k->type != HG_KERNEL_GAUSS_SINC &&
        k->type != HG_KERNEL_ELLIPTICAL)
        return fail(HG_ERR_UNSUPPORTED, "unknown kernel type");
    if (k->reserved) return fail(HG_ERR_ARG, "kernel reserved field must be 0");
    if (k->type != HG_KERNEL_GAUSS_SINC && (!finite(k->fwhm_deg) || !(k->fwhm_deg > 0)))
        return fail(HG_ERR_ARG, "fwhm_deg must be > 0");
    if (k->type == HG_KERNEL_GAUSS_SINC &&
        (!finite(k->p1) || !(k->p1 > 0) || !finite(k->p2) || !(k->p2 > 0)))
        return fail(HG_ERR_ARG, "the Gauss-sinc kernel needs a = p1 > 0 and b = p2 > 0");
    if (k->type == HG_KERNEL_ELLIPTICAL && (!finite(k->p1) || !(k->p1 > 0) || !finite(k->p2)))
        return fail(HG_ERR_ARG, "the elliptical kernel needs a minor FWHM p1 > 0 and a finite "
                                "position angle p2");
    if (!finite(k->support_deg) || !(k->support_deg >= 0) || k->support_deg > 10.0)
        return fail(HG_ERR_ARG, "support_deg must be in [0, 10]");
    int rc = validate_map(m);
    if (rc != HG_OK) return rc;
    if (o) {
        if (o->precision != HG_PREC_FP32 && o->precision != HG_PREC_MFMA_BF16 &&
            o->precision != HG_PREC_MFMA_F16)
            return fail(HG_ERR_UNSUPPORTED, "unknown or unsupported precision form");
        if (o->nside < 0 || o->nside > 16384 || (o->nside & (o->nside - 1)))
            return fail(HG_ERR_ARG, "nside must be 0 or a power of two <= 16384");
        if (o->chunk != 0 && (o->chunk < 8 || o->chunk > MAX_CHUNK || o->chunk % 8))
            return fail(HG_ERR_ARG, "chunk must be 0 or a multiple of 8 in [8, 112]");
        if (o->chunk > 64 && o->precision == HG_PREC_FP32)
            return fail(HG_ERR_ARG, "the FP32 form stages at most 64 slots a chunk");
        if (o->device_mem_cap < 0) return fail(HG_ERR_ARG, "device_mem_cap must be >= 0");
        if (o->waves != 0 && o->waves != 8 && o->waves != 16)
            return fail(HG_ERR_ARG, "waves must be 0, 8 or 16");
        if (o->chan_block != 0 && o->chan_block != 64 && o->chan_block != 128 &&
            o->chan_block != 256)
            return fail(HG_ERR_ARG, "chan_block must be 0, 64, 128 or 256");
    }
    return HG_OK;
}

std::vector<BatchItem> plan_batch_items(const std::vector<std::vector<int64_t>>& tile_blk,
                                        const std::vector<int32_t>& ncb, int64_t& n_items);

// Setup proper, after validation (shared by hg_grid_setup and hg_batch_create).
int make_plan(const double* ra_deg, const double* dec_deg, int64_t n, const hg_kernel* k,
              const hg_map* m, const hg_opts* o, hipStream_t s, hg_plan** out,
              bool batch_field = false) {
    auto t0 = std::chrono::steady_clock::now();
    hg_plan* h = new hg_plan();
    Plan& P = h->P;
    P.device = cur_device();
    P.map = *m;
    P.kern = *k;
    if (o) P.opts = *o;
    P.shape = shape_of(P.opts);
    P.n = n;
    P.sigma = k->type == HG_KERNEL_GAUSS_SINC ? 0.0 : k->fwhm_deg * kDeg / sqrt(8.0 * log(2.0));
    P.r_rad = k->support_deg * kDeg;
    double sh = sin(0.5 * P.r_rad);
    P.h_r = sh * sh;
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
    // Chunk length: the caller's, or the longest of a list that still fits two
    // staged chunks of the plan's densest entry block in LDS (longer chunks
    // mean fewer synchronisations per tile; the fit is known only once the
    // blocks are built, so a plan that does not fit is rebuilt shorter).  A
    // batch's fields start at the longest length predicted to fit (at most
    // 64 slots where the prediction sees no room for more).
    const bool m16 = P.opts.precision != HG_PREC_FP32;
    std::vector<int32_t> chunks;
    if (o && o->chunk)
        chunks = {o->chunk};
    else if (m16)
        chunks = {112, 88, 64, 48, 32, 16, 8};
    else
        chunks = {56, 48, 32, 16, 8};
    if ((batch_field || (P.opts.flags & HG_FLAG_PREDICT_CHUNK)) && !(o && o->chunk)) {
        // set up side by side, a field rebuilt at a shorter chunk delays the
        // batch: start at the longest chunk predicted to fit
        const int32_t first = batch_first_chunk(P, m16);
        while (chunks.size() > 1 && chunks.front() != first) chunks.erase(chunks.begin());
    }
    for (size_t ci = 0; ci < chunks.size(); ci++) {
        P.chunk = chunks[ci];
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
        const bool lds_ok = channel_lds_fits(m16, P.chunk, P.blk_max);
        const bool runs_ok = channel_runs_fit(P.chunk, P.run_max);
        if (lds_ok && runs_ok) break;
        plan_free(P);
        if (ci + 1 == chunks.size()) {
            delete h;
            return fail(HG_ERR_UNSUPPORTED,
                        !lds_ok ? "the densest entry block does not fit two staged chunks in "
                                  "LDS; use a smaller chunk"
                                : "a pixel group takes more than 64 entries of one chunk; use a "
                                  "chunk of at most 64 slots");
        }
    }
    P.setup_ms =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    *out = h;
    return HG_OK;
}

// Runs f, turning exceptions into error codes.
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

void batch_free(hg_batch* b) {
    (void)hipSetDevice(b->device);
    (void)hipDeviceSynchronize();
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    for (auto& e : b->ev_pending) {
        (void)hipEventDestroy(e.first);
        (void)hipEventDestroy(e.second);
    }
    for (auto& e : b->ev_free) {
        (void)hipEventDestroy(e.first);
        (void)hipEventDestroy(e.second);
    }
    dev_free(b->descs);
    dev_free(b->items);
    for (hg_plan* h : b->plans) {
        if (!h) continue;  // a field whose setup failed
        plan_free(h->P);
        delete h;
    }
    delete b;
}

// Every field's setup, on SETUP_THREADS host threads with a stream each, so
// that one field's short kernels and read-backs overlap another's work; the
// largest fields go first.  The streams start after the work already queued
// on the caller's stream s (which may be writing the coordinates).  On
// success b->plans holds the plans in field order and tile_blk[i] each
// field's first-block table; on failure b is freed and the lowest failing
// field's error is set.
// eight threads (on four hardware queues) measured 29.6-31.0 ms against 32.0-32.2
// ms with four for the 64-field workload's setup
constexpr int SETUP_THREADS = 8;

int setup_fields(hg_batch* b, const hg_field* fields, int32_t nfields, const hg_opts& po,
                 hipStream_t s, std::vector<std::vector<int64_t>>& tile_blk) {
    std::vector<hg_plan*> plans((size_t)nfields, nullptr);
    std::vector<int> rcs((size_t)nfields, HG_OK);
    std::vector<std::string> errs((size_t)nfields);
    std::vector<int32_t> order((size_t)nfields);
    for (int32_t i = 0; i < nfields; i++) order[i] = i;
    std::stable_sort(order.begin(), order.end(),
                     [&](int32_t a, int32_t c) { return fields[a].n > fields[c].n; });
    hipEvent_t ready = nullptr;
    hipError_t e = hipEventCreateWithFlags(&ready, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventRecord(ready, s);
    if (e != hipSuccess) {
        if (ready) (void)hipEventDestroy(ready);
        batch_free(b);
        return fail_hip(e, "batch_create");
    }
    const int dev = b->device;
    std::atomic<int32_t> next{0};
    auto work = [&]() {
        hipStream_t ws = nullptr;
        const bool ok = hipSetDevice(dev) == hipSuccess &&
                        hipStreamCreateWithFlags(&ws, hipStreamNonBlocking) == hipSuccess &&
                        hipStreamWaitEvent(ws, ready, 0) == hipSuccess;
        for (;;) {
            const int32_t j = next.fetch_add(1);
            if (j >= nfields) break;
            const int32_t i = order[j];
            if (!ok) {
                rcs[i] = HG_ERR_DEVICE;
                errs[i] = "could not create a setup stream";
                continue;
            }
            const hg_field& f = fields[i];
            const int r = guarded([&]() -> int {
                hg_plan* h = nullptr;
                int r2 = make_plan(f.ra_deg, f.dec_deg, f.n, &f.kernel, &f.map, &po, ws, &h,
                                   true);
                if (r2) return r2;
                plans[i] = h;
                h->owned_by_batch = true;
                // read back by setup with its other sizes
                tile_blk[i] = h->P.tile_blk_host;
                return HG_OK;
            });
            if (r) {
                rcs[i] = r;
                errs[i] = g_err;
            }
        }
        if (ws) {
            (void)hipStreamSynchronize(ws);
            (void)hipStreamDestroy(ws);
        }
    };
    std::vector<std::thread> pool;
    try {
        for (int t = 1; t < std::min<int32_t>(nfields, SETUP_THREADS); t++) pool.emplace_back(work);
    } catch (...) {
        // fewer threads than asked for: the ones running (and this one) share the fields
    }
    work();
    for (auto& t : pool) t.join();
    (void)hipEventDestroy(ready);
    for (int32_t i = 0; i < nfields; i++) b->plans.push_back(plans[i]);
    for (int32_t i = 0; i < nfields; i++) {
        if (rcs[i] != HG_OK) {
            std::string msg = "field " + std::to_string(i) + ": " + errs[i];
            batch_free(b);
            return fail(rcs[i], msg);
        }
    }
    return HG_OK;
}

hipError_t resolve_batch_timing(hg_batch* b) {
    for (auto& e : b->ev_pending) {
        hipError_t r = hipEventSynchronize(e.second);
        if (r != hipSuccess) return r;
        float ms = 0.f;
        r = hipEventElapsedTime(&ms, e.first, e.second);
        if (r != hipSuccess) return r;
        b->run_ms_total += ms;
        b->run_ms_last = ms;
        b->timed_runs++;
        b->ev_free.push_back(e);
    }
    b->ev_pending.clear();
    return hipSuccess;
}

// Work layout of the batched launch.  The unit of placement is a tile with all
// of its channel blocks (they read the same entry blocks and sample rows, so
// they should share one XCD's L2); its cost is (channel blocks) x (staged
// chunks + 2), the 2 standing for the fixed per-item work of the epilogue.
// Units go, largest first, to the XCD with the least work so far (longest
// processing time first); each XCD's items keep that order, and position
// 8 i + x of the launch holds the i-th item of XCD x (the dispatcher sends
// workgroup b to XCD b mod 8 and starts an XCD's workgroups in order).
std::vector<BatchItem> plan_batch_items(const std::vector<std::vector<int64_t>>& tile_blk,
                                        const std::vector<int32_t>& ncb, int64_t& n_items) {
    constexpr int NX = 8;
    struct Unit {
        int64_t cost, tile;
        int32_t field;
    };
    std::vector<Unit> units;
    for (size_t f = 0; f < tile_blk.size(); f++) {
        if (ncb[f] == 0) continue;
        for (size_t t = 0; t + 1 < tile_blk[f].size(); t++) {
            int64_t nch = tile_blk[f][t + 1] - tile_blk[f][t];
            units.push_back({ncb[f] * (nch + 2), (int64_t)t, (int32_t)f});
        }
    }
    std::stable_sort(units.begin(), units.end(),
                     [](const Unit& a, const Unit& b) { return a.cost > b.cost; });
    std::vector<std::vector<BatchItem>> lists(NX);
    std::vector<int64_t> load(NX, 0);
    n_items = 0;
    for (const Unit& u : units) {
        int x = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        load[x] += u.cost;
        for (int32_t cb = 0; cb < ncb[u.field]; cb++) lists[x].push_back({u.field, cb, u.tile});
        n_items += ncb[u.field];
    }
    size_t depth = 0;
    for (auto& l : lists) depth = std::max(depth, l.size());
    std::vector<BatchItem> pos(depth * NX, BatchItem{-1, 0, 0});
    for (int x = 0; x < NX; x++)
        for (size_t i = 0; i < lists[x].size(); i++) pos[i * NX + x] = lists[x][i];
    return pos;
}

}  // namespace

// The single-field launch uses the batched form's layout (plan_batch_items
// with one field): idle workgroups pad the XCDs' lists to equal length.  The
// order is built and uploaded on the first launch with a given channel-block
// count and kept with the plan; a later launch on another stream waits for
// the upload's event.
hipError_t launch_order(Plan& P, int32_t ncb, hipStream_t s, const int64_t** items, int64_t* n,
                        int32_t row0, int32_t row1) {
    if (P.tile_blk_host.size() != (size_t)P.ntiles + 1) return hipErrorNotInitialized;
    if (row1 < 0) {
        row0 = 0;
        row1 = P.nty;
    }
    const auto key = std::make_tuple(ncb, row0, row1);
    auto it = P.orders.find(key);
    if (it == P.orders.end()) {
        LaunchOrder o;
        int64_t n_items = 0;
        // the rows' tiles are contiguous: their chunk offsets, rebased
        const int64_t t0 = (int64_t)row0 * P.ntx, t1 = (int64_t)row1 * P.ntx;
        std::vector<int64_t> tb(P.tile_blk_host.begin() + t0, P.tile_blk_host.begin() + t1 + 1);
        for (auto& v : tb) v -= P.tile_blk_host[(size_t)t0];
        const std::vector<BatchItem> pos = plan_batch_items({tb}, {ncb}, n_items);
        o.n = (int64_t)pos.size();
        // page-locked source: an upload from pageable memory is staged by the
        // runtime, tens of microseconds before the first launch can start
        const size_t bytes = sizeof(int64_t) * (size_t)(o.n ? o.n : 1);
        hipError_t e = host_alloc(o.host, bytes);
        if (e == hipSuccess) {
            int64_t* h = (int64_t*)o.host.p;
            for (size_t i = 0; i < pos.size(); i++)
                h[i] = pos[i].field < 0 ? -1 : (t0 + pos[i].tile) * ncb + pos[i].cb;
            e = dev_alloc(o.items, bytes);
        }
        if (e == hipSuccess) e = hipEventCreateWithFlags(&o.ready, hipEventDisableTiming);
        if (e == hipSuccess && o.n > 0)
            e = hipMemcpyAsync(o.items.p, o.host.p, sizeof(int64_t) * (size_t)o.n,
                               hipMemcpyHostToDevice, s);
        if (e == hipSuccess) e = hipEventRecord(o.ready, s);
        if (e != hipSuccess) {
            if (o.ready) {
                (void)hipEventSynchronize(o.ready);
                (void)hipEventDestroy(o.ready);
            }
            (void)hipStreamSynchronize(s);  // a copy may have started from the source
            dev_free(o.items);
            host_free(o.host);
            return e;
        }
        it = P.orders.emplace(key, std::move(o)).first;
    } else {
        hipError_t e = hipStreamWaitEvent(s, it->second.ready, 0);
        if (e != hipSuccess) return e;
    }
    *items = (const int64_t*)it->second.items.p;
    *n = it->second.n;
    return hipSuccess;
}

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
        if (n > 0) {
            if ((rc = require_device(ra_deg, cur_device(), "ra_deg"))) return rc;
            if ((rc = require_device(dec_deg, cur_device(), "dec_deg"))) return rc;
        }
        return make_plan(ra_deg, dec_deg, n, k, m, o, (hipStream_t)hip_stream, out);
    });
}

}  // extern "C"

namespace {
// hg_grid_channels over tile rows [row0, row1) (row1 < 0: every row)
int grid_channels_rows(hg_plan* h, const void* values, int64_t ld, int32_t nchan, int32_t dtype,
                       float* out, void* hip_stream, int32_t row0, int32_t row1) {
    return guarded([&]() -> int {
        g_err.clear();
        if (!h) return fail(HG_ERR_ARG, "plan must not be NULL");
        Plan& P = h->P;
        if (P.finished) return fail(HG_ERR_STATE, "plan already finished");
        if (nchan < 0) return fail(HG_ERR_ARG, "nchan must be >= 0");
        if (dtype != HG_F32 && dtype != HG_BF16 && dtype != HG_F16)
            return fail(HG_ERR_ARG, "unknown dtype");
        if (row1 >= 0 && (row0 < 0 || row1 > P.nty || row0 > row1))
            return fail(HG_ERR_ARG, "tile rows must satisfy 0 <= row0 <= row1 <= the map's tile rows");
        if (nchan == 0 || row0 == row1) return HG_OK;
        if (!out || (!values && P.n > 0)) return fail(HG_ERR_ARG, "values and out must not be NULL");
        if (ld < nchan) return fail(HG_ERR_ARG, "ld must be >= nchan");
        if (P.opts.precision == HG_PREC_MFMA_BF16 && dtype != HG_BF16)
            return fail(HG_ERR_UNSUPPORTED, "a BF16-MFMA plan grids BF16 values");
        if (P.opts.precision == HG_PREC_MFMA_F16 && dtype != HG_F16)
            return fail(HG_ERR_UNSUPPORTED, "an FP16-MFMA plan grids FP16 values");
        int rc = require_device(out, P.device, "out");
        if (!rc && P.n > 0) rc = require_device(values, P.device, "values");
        if (rc) return rc;
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
        e = launch_channels(P, values, ld, nchan, dtype, out, s, P.shape, row0, row1);
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
}  // namespace

extern "C" {

int hg_grid_channels(hg_plan* h, const void* values, int64_t ld, int32_t nchan, int32_t dtype,
                     float* out, void* hip_stream) {
    return grid_channels_rows(h, values, ld, nchan, dtype, out, hip_stream, 0, -1);
}

int hg_grid_channels_rows(hg_plan* h, const void* values, int64_t ld, int32_t nchan,
                          int32_t dtype, float* out, int32_t tile_row0, int32_t tile_row1,
                          void* hip_stream) {
    if (tile_row1 < 0) {
        g_err = "tile_row1 must be >= 0";
        return HG_ERR_ARG;
    }
    return grid_channels_rows(h, values, ld, nchan, dtype, out, hip_stream, tile_row0, tile_row1);
}

int hg_plan_row_needs(const hg_plan* h, int32_t rows_per_band, int64_t* host_need,
                      int32_t nbands, void* hip_stream) {
    return guarded([&]() -> int {
        g_err.clear();
        if (!h) return fail(HG_ERR_ARG, "plan must not be NULL");
        const Plan& P = h->P;
        if (P.finished) return fail(HG_ERR_STATE, "plan already finished");
        if (rows_per_band < 1) return fail(HG_ERR_ARG, "rows_per_band must be >= 1");
        const int64_t want = ((int64_t)P.nty + rows_per_band - 1) / rows_per_band;
        if (nbands != want || !host_need)
            return fail(HG_ERR_ARG, "host_need must hold ceil(tile rows / rows_per_band) values");
        hipError_t e = hipSetDevice(P.device);
        if (e != hipSuccess) return fail_hip(e, "plan_row_needs");
        hipStream_t s = (hipStream_t)hip_stream;
        std::vector<int64_t> tn((size_t)P.ntiles);
        DevBuf d;
        e = dev_alloc(d, sizeof(int64_t) * (size_t)(P.ntiles ? P.ntiles : 1));
        if (e == hipSuccess) e = launch_tile_max_index(P, (int64_t*)d.p, s);
        if (e == hipSuccess && P.ntiles)
            e = hipMemcpyAsync(tn.data(), d.p, sizeof(int64_t) * tn.size(), hipMemcpyDeviceToHost,
                               s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        dev_free(d);
        if (e != hipSuccess) return fail_hip(e, "plan_row_needs");
        for (int32_t b = 0; b < nbands; b++) {
            int64_t m = 0;
            const int64_t r0 = (int64_t)b * rows_per_band;
            const int64_t r1 = std::min<int64_t>(r0 + rows_per_band, P.nty);
            for (int64_t t = r0 * P.ntx; t < r1 * P.ntx; t++) m = std::max(m, tn[(size_t)t]);
            host_need[b] = m;
        }
        return HG_OK;
    });
}

int hg_grid_channels_literal(hg_plan* h, const float* values, int64_t ld, int32_t nchan,
                             float* out, int32_t gamma, int32_t block_threads, void* hip_stream) {
    return guarded([&]() -> int {
        g_err.clear();
        if (!h) return fail(HG_ERR_ARG, "plan must not be NULL");
        Plan& P = h->P;
        if (P.finished) return fail(HG_ERR_STATE, "plan already finished");
        if (nchan < 0) return fail(HG_ERR_ARG, "nchan must be >= 0");
        if (gamma != 1 && gamma != 2 && gamma != 4)
            return fail(HG_ERR_ARG, "gamma must be 1, 2 or 4");
        if (P.kern.type != HG_KERNEL_GAUSS)
            return fail(HG_ERR_UNSUPPORTED, "the Algorithm 1 path has the Gaussian kernel only");
        if (block_threads < 64 || block_threads > 1024 || block_threads % 64)
            return fail(HG_ERR_ARG, "block_threads must be a multiple of 64 in [64, 1024]");
        if (nchan == 0) return HG_OK;
        if (!out || (!values && P.n > 0)) return fail(HG_ERR_ARG, "values and out must not be NULL");
        if (ld < nchan) return fail(HG_ERR_ARG, "ld must be >= nchan");
        int rc = require_device(out, P.device, "out");
        if (!rc && P.n > 0) rc = require_device(values, P.device, "values");
        if (rc) return rc;
        hipError_t e = hipSetDevice(P.device);
        if (e == hipSuccess)
            e = launch_literal(P, values, ld, nchan, out, gamma, block_threads,
                               (hipStream_t)hip_stream);
        if (e != hipSuccess) return fail_hip(e, "grid_channels_literal");
        return HG_OK;
    });
}

int hg_grid_channels_host(hg_plan* h, const void* host_values, int64_t ld, int32_t nchan,
                          int32_t dtype, float* host_out, int32_t block, void* hip_stream,
                          hg_stream_info* info) {
    return guarded([&]() -> int {
        g_err.clear();
        if (!h) return fail(HG_ERR_ARG, "plan must not be NULL");
        Plan& P = h->P;
        if (P.finished) return fail(HG_ERR_STATE, "plan already finished");
        if (nchan < 0) return fail(HG_ERR_ARG, "nchan must be >= 0");
        if (dtype != HG_F32 && dtype != HG_BF16 && dtype != HG_F16)
            return fail(HG_ERR_ARG, "unknown dtype");
        if (block < 0) return fail(HG_ERR_ARG, "block must be >= 0");
        if (info) std::memset(info, 0, sizeof *info);
        if (nchan == 0) return HG_OK;
        if (!host_out || (!host_values && P.n > 0))
            return fail(HG_ERR_ARG, "values and out must not be NULL");
        if (ld < nchan) return fail(HG_ERR_ARG, "ld must be >= nchan");
        if (P.opts.precision == HG_PREC_MFMA_BF16 && dtype != HG_BF16)
            return fail(HG_ERR_UNSUPPORTED, "a BF16-MFMA plan grids BF16 values");
        if (P.opts.precision == HG_PREC_MFMA_F16 && dtype != HG_F16)
            return fail(HG_ERR_UNSUPPORTED, "an FP16-MFMA plan grids FP16 values");
        hipError_t e = hipSetDevice(P.device);
        if (e != hipSuccess) return fail_hip(e, "grid_channels_host");
        std::string err;
        int rc = grid_channels_host(P, host_values, ld, nchan, dtype, host_out,
                                    block ? block : 4096, (hipStream_t)hip_stream, info, err);
        if (rc) return fail(rc, err);
        return HG_OK;
    });
}

int hg_grid_channels_host_noalloc(hg_plan* h, const void* host_values, int64_t ld,
                                  int32_t nchan, int32_t dtype, float* host_out, int32_t block,
                                  void* hip_stream, hg_stream_info* info) {
    return guarded([&]() -> int {
        g_err.clear();
        if (!h) return fail(HG_ERR_ARG, "plan must not be NULL");
        Plan& P = h->P;
        if (P.finished) return fail(HG_ERR_STATE, "plan already finished");
        if (nchan < 0) return fail(HG_ERR_ARG, "nchan must be >= 0");
        if (dtype != HG_F32 && dtype != HG_BF16 && dtype != HG_F16)
            return fail(HG_ERR_ARG, "unknown dtype");
        if (block < 0) return fail(HG_ERR_ARG, "block must be >= 0");
        if (info) std::memset(info, 0, sizeof *info);
        if (nchan == 0) return HG_OK;
        if (!host_out || (!host_values && P.n > 0))
            return fail(HG_ERR_ARG, "values and out must not be NULL");
        if (ld < nchan) return fail(HG_ERR_ARG, "ld must be >= nchan");
        if (P.opts.precision == HG_PREC_MFMA_BF16 && dtype != HG_BF16)
            return fail(HG_ERR_UNSUPPORTED, "a BF16-MFMA plan grids BF16 values");
        if (P.opts.precision == HG_PREC_MFMA_F16 && dtype != HG_F16)
            return fail(HG_ERR_UNSUPPORTED, "an FP16-MFMA plan grids FP16 values");
        hipError_t e = hipSetDevice(P.device);
        if (e != hipSuccess) return fail_hip(e, "grid_channels_host_noalloc");
        std::string err;
        int rc = grid_channels_host_noalloc(P, host_values, ld, nchan, dtype, host_out, block,
                                            (hipStream_t)hip_stream, info, err);
        if (rc) return fail(rc, err);
        return HG_OK;
    });
}

int hg_grid_finish(hg_plan* h) {
    return guarded([&]() -> int {
        g_err.clear();
        if (!h) return HG_OK;
        if (h->owned_by_batch)
            return fail(HG_ERR_STATE, "plan belongs to a batch; hg_batch_destroy frees it");
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
        st->waves = P.shape.waves;
        st->chan_block = 64 * P.shape.g;
        st->setup_ms = P.setup_ms;
        st->last_channels_ms = P.ch_ms_last;
        st->total_channels_ms = P.ch_ms_total;
        st->channels_calls = P.ch_calls;
        return HG_OK;
    });
}

int hg_plan_set_shape(hg_plan* h, int32_t waves, int32_t chan_block) {
    return guarded([&]() -> int {
        g_err.clear();
        if (!h) return fail(HG_ERR_ARG, "plan must not be NULL");
        if (waves != 0 && waves != 8 && waves != 16)
            return fail(HG_ERR_ARG, "waves must be 0, 8 or 16");
        if (chan_block != 0 && chan_block != 64 && chan_block != 128 && chan_block != 256)
            return fail(HG_ERR_ARG, "chan_block must be 0, 64, 128 or 256");
        Plan& P = h->P;
        if (P.finished) return fail(HG_ERR_STATE, "plan already finished");
        P.opts.waves = waves;
        P.opts.chan_block = chan_block;
        P.shape = shape_of(P.opts);
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

int hg_map_pixel_ids(const hg_map* m, int64_t* host_ids) {
    return guarded([&]() -> int {
        g_err.clear();
        if (!m || !host_ids) return fail(HG_ERR_ARG, "NULL argument");
        int rc = validate_map(m);
        if (rc != HG_OK) return rc;
        if (m->proj != HG_PROJ_HEALPIX) return fail(HG_ERR_ARG, "not a HEALPix map");
        const int64_t ns = m->nside, per_ring = 4 * ns, cap = 2 * ns * (ns - 1);
        for (int64_t j = 0; j < m->ny; j++) {
            const int64_t first = cap + per_ring * (m->ring0 - j - ns);  // first pixel of the ring
            for (int64_t i = 0; i < m->nx; i++)
                host_ids[j * m->nx + i] = first + (m->pix0 + i) % per_ring;
        }
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

int hg_batch_create(const hg_field* fields, int32_t nfields, int32_t dtype, const hg_opts* o,
                    void* hip_stream, hg_batch** out) {
    return guarded([&]() -> int {
        g_err.clear();
        if (!out) return fail(HG_ERR_ARG, "out must not be NULL");
        *out = nullptr;
        if (!fields || nfields <= 0) return fail(HG_ERR_ARG, "need at least one field");
        if (dtype != HG_F32 && dtype != HG_BF16 && dtype != HG_F16)
            return fail(HG_ERR_ARG, "unknown dtype");
        int32_t prec = o ? o->precision : HG_PREC_FP32;
        if (prec == HG_PREC_MFMA_BF16 && dtype != HG_BF16)
            return fail(HG_ERR_UNSUPPORTED, "a BF16-MFMA batch grids BF16 values");
        if (prec == HG_PREC_MFMA_F16 && dtype != HG_F16)
            return fail(HG_ERR_UNSUPPORTED, "an FP16-MFMA batch grids FP16 values");
        for (int32_t i = 0; i < nfields; i++) {
            const hg_field& f = fields[i];
            int rc = validate_setup(f.ra_deg, f.dec_deg, f.n, &f.kernel, &f.map, o);
            if (!rc && (f.nchan < 0 || f.reserved)) rc = fail(HG_ERR_ARG, "nchan must be >= 0 and reserved 0");
            if (!rc && f.nchan > 0 && (!f.out || (!f.values && f.n > 0)))
                rc = fail(HG_ERR_ARG, "values and out must not be NULL");
            if (!rc && f.nchan > 0 && f.ld < f.nchan) rc = fail(HG_ERR_ARG, "ld must be >= nchan");
            if (rc) return fail(rc, "field " + std::to_string(i) + ": " + g_err);
        }
        int rc = ensure_device();
        if (rc) return rc;
        for (int32_t i = 0; i < nfields && !rc; i++) {
            const hg_field& f = fields[i];
            const int dev = cur_device();
            if (f.n > 0) {
                rc = require_device(f.ra_deg, dev, "ra_deg");
                if (!rc) rc = require_device(f.dec_deg, dev, "dec_deg");
            }
            if (!rc && f.nchan > 0) rc = require_device(f.out, dev, "out");
            if (!rc && f.nchan > 0 && f.n > 0) rc = require_device(f.values, dev, "values");
            if (rc) return fail(rc, "field " + std::to_string(i) + ": " + g_err);
        }
        auto t0 = std::chrono::steady_clock::now();
        hg_batch* b = new hg_batch();
        b->device = cur_device();
        b->dtype = dtype;
        if (o) b->opts = *o;
        hg_opts po = b->opts;
        po.flags &= ~HG_FLAG_TIME_CHANNELS;
        hipStream_t s = (hipStream_t)hip_stream;
        std::vector<std::vector<int64_t>> tile_blk(nfields);
        rc = setup_fields(b, fields, nfields, po, s, tile_blk);
        if (rc) return rc;  // b freed, error set
        std::vector<FieldDesc> descs;
        std::vector<int32_t> ncb;
        bool vec = true;
        for (int32_t i = 0; i < nfields; i++) {
            const hg_field& f = fields[i];
            if (f.nchan > 0 && f.n > 0) vec = vec && values_vec(b->plans[i]->P, f.values, f.ld, dtype);
        }
        // one kernel for every field: its shape holds for all of them
        const Shape shape = effective_shape(b->opts.precision != HG_PREC_FP32, dtype, vec,
                                            shape_of(b->opts));
        for (int32_t i = 0; i < nfields; i++) {
            const hg_field& f = fields[i];
            const Plan& P = b->plans[i]->P;
            descs.push_back(field_desc(P, f.values, f.ld, f.nchan, f.out, shape));
            ncb.push_back(descs.back().ncb);
        }
        std::vector<BatchItem> pos = plan_batch_items(tile_blk, ncb, b->n_items);
        b->n_positions = (int64_t)pos.size();
        if (b->n_items > 0) {
            if (b->n_positions >= ((int64_t)1 << 31)) {
                batch_free(b);
                return fail(HG_ERR_UNSUPPORTED, "batch has too many work items");
            }
            hipError_t e = dev_alloc(b->descs, sizeof(FieldDesc) * descs.size());
            if (e == hipSuccess) e = dev_alloc(b->items, sizeof(BatchItem) * pos.size());
            if (e == hipSuccess)
                e = hipMemcpy(b->descs.p, descs.data(), sizeof(FieldDesc) * descs.size(),
                              hipMemcpyHostToDevice);
            if (e == hipSuccess)
                e = hipMemcpy(b->items.p, pos.data(), sizeof(BatchItem) * pos.size(),
                              hipMemcpyHostToDevice);
            const bool m16 = b->opts.precision != HG_PREC_FP32;
            size_t shm = 0;
            for (const FieldDesc& d : descs) shm = std::max(shm, field_lds_bytes(d, m16, shape));
            BatchKernelInfo ki = batch_kernel(m16, dtype, vec, shm, shape);
            if (e == hipSuccess && ki.shm > 65536)
                e = hipFuncSetAttribute(ki.main, hipFuncAttributeMaxDynamicSharedMemorySize,
                                        (int)ki.shm);
            // the whole batch is one kernel node of a graph, replayed by hg_batch_run
            if (e == hipSuccess) e = hipGraphCreate(&b->graph, 0);
            if (e == hipSuccess) {
                void* d_descs = b->descs.p;
                void* d_items = b->items.p;
                void* args[] = {&d_descs, &d_items};
                hipKernelNodeParams kp{};
                kp.func = const_cast<void*>(ki.main);
                kp.gridDim = dim3((unsigned)b->n_positions);
                kp.blockDim = dim3((unsigned)ki.threads);
                kp.sharedMemBytes = (unsigned)ki.shm;
                kp.kernelParams = args;
                kp.extra = nullptr;
                hipGraphNode_t node;
                e = hipGraphAddKernelNode(&node, b->graph, nullptr, 0, &kp);
            }
            if (e == hipSuccess) e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
            if (e != hipSuccess) {
                batch_free(b);
                return fail_hip(e, "batch_create");
            }
        }
        b->setup_ms =
            std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        *out = b;
        return HG_OK;
    });
}

int hg_batch_run(hg_batch* b, void* hip_stream) {
    return guarded([&]() -> int {
        g_err.clear();
        if (!b) return fail(HG_ERR_ARG, "batch must not be NULL");
        if (!b->exec) return HG_OK;  // no channels to grid
        hipError_t e = hipSetDevice(b->device);
        if (e != hipSuccess) return fail_hip(e, "batch_run");
        hipStream_t s = (hipStream_t)hip_stream;
        bool timed = (b->opts.flags & HG_FLAG_TIME_CHANNELS) != 0;
        std::pair<hipEvent_t, hipEvent_t> ev{nullptr, nullptr};
        if (timed) {
            if (!b->ev_free.empty()) {
                ev = b->ev_free.back();
                b->ev_free.pop_back();
            } else {
                e = hipEventCreate(&ev.first);
                if (e == hipSuccess) e = hipEventCreate(&ev.second);
                if (e != hipSuccess) return fail_hip(e, "batch_run (events)");
            }
            e = hipEventRecord(ev.first, s);
            if (e != hipSuccess) return fail_hip(e, "batch_run (events)");
        }
        e = hipGraphLaunch(b->exec, s);
        if (e != hipSuccess) return fail_hip(e, "batch_run");
        if (timed) {
            e = hipEventRecord(ev.second, s);
            if (e != hipSuccess) return fail_hip(e, "batch_run (events)");
            b->ev_pending.push_back(ev);
        }
        b->runs++;
        return HG_OK;
    });
}

int hg_batch_destroy(hg_batch* b) {
    return guarded([&]() -> int {
        g_err.clear();
        if (!b) return HG_OK;
        batch_free(b);
        return HG_OK;
    });
}

int hg_batch_stats(hg_batch* b, hg_batch_info* st) {
    return guarded([&]() -> int {
        g_err.clear();
        if (!b || !st) return fail(HG_ERR_ARG, "NULL argument");
        hipError_t e = resolve_batch_timing(b);
        if (e != hipSuccess) return fail_hip(e, "batch_stats");
        std::memset(st, 0, sizeof *st);
        st->n_fields = (int32_t)b->plans.size();
        st->n_items = b->n_items;
        st->n_workgroups = b->n_positions;
        for (hg_plan* h : b->plans) {
            st->n_samples += h->P.n;
            st->nnz += h->P.nnz;
            st->n_entries += h->P.nnz_entries;
            st->device_bytes += plan_bytes(h->P);
        }
        st->device_bytes += (int64_t)(b->descs.bytes + b->items.bytes);
        st->setup_ms = b->setup_ms;
        st->last_run_ms = b->run_ms_last;
        st->total_run_ms = b->run_ms_total;
        st->runs = b->runs;
        return HG_OK;
    });
}

int hg_batch_plan(hg_batch* b, int32_t i, hg_plan** out) {
    return guarded([&]() -> int {
        g_err.clear();
        if (!b || !out) return fail(HG_ERR_ARG, "NULL argument");
        *out = nullptr;
        if (i < 0 || i >= (int32_t)b->plans.size()) return fail(HG_ERR_ARG, "field index out of range");
        *out = b->plans[i];
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
        for (const void* q : {(const void*)ra_deg, (const void*)dec_deg, (const void*)pix})
            if ((rc = require_device(q, cur_device(), "ra_deg, dec_deg and pix"))) return rc;
        hipError_t e = launch_ang2pix(nside, ra_deg, dec_deg, n, pix, (hipStream_t)hip_stream);
        if (e != hipSuccess) return fail_hip(e, "ang2pix_ring");
        return HG_OK;
    });
}

}  // extern "C"
