// Host-streamed channel phase of libhegrid: a cube whose values and maps live
// in host memory is gridded block by block of channels (channels are
// independent, Sec. 4.2), with the host-to-device copy of block b+1, the
// channel kernel of block b and the device-to-host copy of block b-1 in flight
// together on three streams.  This takes the place of the paper's pinned
// buffers, per-stream device pool and transfer/compute overlap (Sec. 4.3.2).
//
// Two device slots hold a block's values [n][ldd] and its maps [w][ny][nx].
// Per slot s the events h2d[s], ker[s] and d2h[s] order the streams:
//   copy-in stream : wait ker[s] (slot's values free)  -> copy values -> h2d[s]
//   compute stream : wait h2d[s], wait d2h[s] (maps free) -> kernel    -> ker[s]
//   copy-out stream: wait ker[s]                        -> copy maps   -> d2h[s]
// If the caller's buffers are pinned (page-locked, e.g. from hipHostMalloc)
// the copies go straight between them and the device (a 2-D copy picks the
// block's columns out of the [n][ld] rows).  Otherwise blocks pass through two
// pinned slots of the library: host threads gather block b's columns into a
// free slot while the device works on earlier blocks, and scatter finished
// maps back into the caller's cube.
#include <algorithm>
#include <chrono>
#include <cstring>
#include <mutex>
#include <thread>

#include "hg_common.h"

namespace hg {
namespace {

bool is_pinned(const void* p) {
    if (!p) return false;
    hipPointerAttribute_t a;
    hipError_t e = hipPointerGetAttributes(&a, p);
    if (e != hipSuccess) {
        (void)hipGetLastError();  // pageable memory is reported as an error here
        return false;
    }
    return a.type == hipMemoryTypeHost;
}

// Run f(lo, hi) over [0, n) on up to `threads` host threads.
template <typename F>
void parallel_rows(int64_t n, int threads, F&& f) {
    if (n <= 0) return;
    int t = (int)std::min<int64_t>(threads, (n + 1023) / 1024);
    if (t <= 1) {
        f((int64_t)0, n);
        return;
    }
    std::vector<std::thread> pool;
    int64_t per = (n + t - 1) / t;
    for (int i = 0; i < t; i++) {
        int64_t lo = i * per, hi = std::min(n, lo + per);
        if (lo < hi) pool.emplace_back([&f, lo, hi] { f(lo, hi); });
    }
    for (auto& th : pool) th.join();
}

hipError_t ensure_ring(Plan& P, size_t val_bytes, size_t out_bytes, bool staged) {
    HostRing& R = P.ring;
    hipError_t e = hipSuccess;
    if (!R.h2d) e = hipStreamCreateWithFlags(&R.h2d, hipStreamNonBlocking);
    if (e == hipSuccess && !R.d2h) e = hipStreamCreateWithFlags(&R.d2h, hipStreamNonBlocking);
    for (int s = 0; s < RING_SLOTS && e == hipSuccess; s++) {
        if (!R.ev_h2d[s]) e = hipEventCreateWithFlags(&R.ev_h2d[s], hipEventDisableTiming);
        if (e == hipSuccess && !R.ev_ker[s])
            e = hipEventCreateWithFlags(&R.ev_ker[s], hipEventDisableTiming);
        if (e == hipSuccess && !R.ev_d2h[s])
            e = hipEventCreateWithFlags(&R.ev_d2h[s], hipEventDisableTiming);
        if (e == hipSuccess && R.vals[s].bytes < val_bytes) e = dev_alloc(R.vals[s], val_bytes);
        if (e == hipSuccess && R.out[s].bytes < out_bytes) e = dev_alloc(R.out[s], out_bytes);
    }
    if (e != hipSuccess || !staged) return e;
    if (R.pin_in_bytes < val_bytes) {
        for (int s = 0; s < RING_SLOTS; s++) {
            if (R.pin_in[s]) (void)hipHostFree(R.pin_in[s]);
            R.pin_in[s] = nullptr;
        }
        R.pin_in_bytes = 0;
        for (int s = 0; s < RING_SLOTS && e == hipSuccess; s++)
            e = hipHostMalloc(&R.pin_in[s], val_bytes, hipHostMallocDefault);
        if (e == hipSuccess) R.pin_in_bytes = val_bytes;
    }
    if (e == hipSuccess && R.pin_out_bytes < out_bytes) {
        for (int s = 0; s < RING_SLOTS; s++) {
            if (R.pin_out[s]) (void)hipHostFree(R.pin_out[s]);
            R.pin_out[s] = nullptr;
        }
        R.pin_out_bytes = 0;
        for (int s = 0; s < RING_SLOTS && e == hipSuccess; s++)
            e = hipHostMalloc(&R.pin_out[s], out_bytes, hipHostMallocDefault);
        if (e == hipSuccess) R.pin_out_bytes = out_bytes;
    }
    return e;
}

struct Timed {
    std::vector<hipEvent_t> ev;  // pairs (start, end)
    bool on = false;
    hipError_t mark(hipStream_t s, size_t& idx) {
        if (!on) return hipSuccess;
        hipEvent_t x;
        hipError_t e = hipEventCreate(&x);
        if (e != hipSuccess) return e;
        ev.push_back(x);
        idx = ev.size() - 1;
        return hipEventRecord(x, s);
    }
    double sum(const std::vector<std::pair<size_t, size_t>>& pairs) {
        double t = 0;
        for (auto& pr : pairs) {
            float ms = 0;
            if (hipEventElapsedTime(&ms, ev[pr.first], ev[pr.second]) == hipSuccess) t += ms;
        }
        return t;
    }
    ~Timed() {
        for (hipEvent_t x : ev) (void)hipEventDestroy(x);
    }
};

}  // namespace

void ring_free(HostRing& R) {
    for (int s = 0; s < RING_SLOTS; s++) {
        dev_free(R.vals[s]);
        dev_free(R.out[s]);
        if (R.pin_in[s]) (void)hipHostFree(R.pin_in[s]);
        if (R.pin_out[s]) (void)hipHostFree(R.pin_out[s]);
        R.pin_in[s] = R.pin_out[s] = nullptr;
        for (hipEvent_t* ev : {&R.ev_h2d[s], &R.ev_ker[s], &R.ev_d2h[s]})
            if (*ev) {
                (void)hipEventDestroy(*ev);
                *ev = nullptr;
            }
    }
    R.pin_in_bytes = R.pin_out_bytes = 0;
    if (R.h2d) (void)hipStreamDestroy(R.h2d);
    if (R.d2h) (void)hipStreamDestroy(R.d2h);
    R.h2d = R.d2h = nullptr;
}

int grid_channels_host(Plan& P, const void* host_values, int64_t ld, int32_t nchan, int32_t dtype,
                       float* host_out, int32_t block, hipStream_t cs, hg_stream_info* info,
                       std::string& err) {
    auto t0 = std::chrono::steady_clock::now();
    const size_t es = dtype == HG_F32 ? 4 : 2;
    const int64_t n = P.n, npix = P.npix;
    const int32_t blk = std::min(block, nchan);
    const int nb = (nchan + blk - 1) / blk;
    const bool direct = is_pinned(host_values) && is_pinned(host_out);
    const bool staged = !direct;
    // Device row stride: 16-byte aligned rows for the kernel's vector
    // loads, except when one block takes whole page-locked rows: then the
    // rows keep the host's stride and go over in one linear copy (a 2-D copy
    // of short rows runs far below the link's rate; unaligned rows take the
    // kernel's scalar staging instead).
    const bool linear = direct && nb == 1 && blk == ld;
    const int64_t ldd = linear ? ld : (blk + 7) / 8 * 8;
    const size_t val_bytes = (size_t)std::max<int64_t>(n, 1) * ldd * es;
    const size_t out_bytes = (size_t)blk * npix * 4;
    if (P.opts.device_mem_cap > 0) {
        int64_t have = 0;
        for (int s = 0; s < RING_SLOTS; s++)
            have += (int64_t)(P.ring.vals[s].bytes + P.ring.out[s].bytes);
        int64_t need = (int64_t)RING_SLOTS * (int64_t)(val_bytes + out_bytes);
        if (need > have) {
            int64_t used = 0;
            for (const DevBuf* b : {&P.srt_idx, &P.srt_coord, &P.cell_off, &P.tile_piece,
                                    &P.tile_nslots, &P.pg_piece, &P.pg_base, &P.pg_cnt,
                                    &P.slot_idx, &P.ent_slot, &P.ent_w, &P.cp_base, &P.chunk_ptr,
                                    &P.pix_count, &P.pix_W, &P.pix_Wf, &P.scratch, &P.tile_blk,
                                    &P.blk_base, &P.blk_pgoff, &P.e2_w, &P.e2_s, &P.e3_w, &P.e3_s})
                used += (int64_t)b->bytes;
            if (used + need > P.opts.device_mem_cap) {
                err = "streaming ring needs " + std::to_string(need) +
                      " device bytes beyond the cap; use a smaller block";
                return HG_ERR_NOMEM;
            }
        }
    }
    hipError_t e = ensure_ring(P, val_bytes, out_bytes, staged);
    if (e != hipSuccess) {
        err = std::string("streaming ring: ") + hipGetErrorString(e);
        return e == hipErrorOutOfMemory ? HG_ERR_NOMEM : HG_ERR_DEVICE;
    }
    HostRing& R = P.ring;
    const int threads = (int)std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    Timed tm;
    tm.on = info != nullptr;
    std::vector<std::pair<size_t, size_t>> t_h2d, t_ker, t_d2h;
    const char* vin = (const char*)host_values;
    char* vout = (char*)host_out;

    // host side of the staged path
    auto gather = [&](int b) {  // block b's columns -> pinned slot, rows of ldd
        const int64_t c0 = (int64_t)b * blk;
        const int64_t w = std::min<int64_t>(blk, nchan - c0);
        char* dst = (char*)R.pin_in[b % RING_SLOTS];
        parallel_rows(n, threads, [&](int64_t lo, int64_t hi) {
            for (int64_t r = lo; r < hi; r++)
                std::memcpy(dst + (size_t)(r * ldd) * es, vin + (size_t)(r * ld + c0) * es,
                            (size_t)w * es);
        });
    };
    auto scatter = [&](int b) {  // pinned maps of block b -> caller's cube
        const int64_t c0 = (int64_t)b * blk;
        const int64_t w = std::min<int64_t>(blk, nchan - c0);
        const char* src = (const char*)R.pin_out[b % RING_SLOTS];
        char* dst = vout + (size_t)c0 * npix * 4;
        const int64_t total = w * npix * 4;
        parallel_rows((total + 65535) / 65536, threads, [&](int64_t lo, int64_t hi) {
            int64_t a = lo * 65536, z = std::min(total, hi * 65536);
            std::memcpy(dst + a, src + a, (size_t)(z - a));
        });
    };

    for (int b = 0; b < nb && e == hipSuccess; b++) {
        const int s = b % RING_SLOTS;
        const int64_t c0 = (int64_t)b * blk;
        const int64_t w = std::min<int64_t>(blk, nchan - c0);
        size_t i0 = 0, i1 = 0;
        // copy-in
        if (b >= RING_SLOTS) e = hipStreamWaitEvent(R.h2d, R.ev_ker[s], 0);
        if (n > 0 && e == hipSuccess) {
            if (staged) {
                // the slot's previous copy-in must have left the pinned buffer
                if (b >= RING_SLOTS) e = hipEventSynchronize(R.ev_h2d[s]);
                if (e == hipSuccess) gather(b);
            }
            if (e == hipSuccess) e = tm.mark(R.h2d, i0);
            if (e == hipSuccess) {
                if (staged)
                    e = hipMemcpyAsync(R.vals[s].p, R.pin_in[s], (size_t)n * ldd * es,
                                       hipMemcpyHostToDevice, R.h2d);
                else if (linear)
                    e = hipMemcpyAsync(R.vals[s].p, vin, (size_t)n * ld * es,
                                       hipMemcpyHostToDevice, R.h2d);
                else
                    e = hipMemcpy2DAsync(R.vals[s].p, (size_t)ldd * es, vin + (size_t)c0 * es,
                                         (size_t)ld * es, (size_t)w * es, (size_t)n,
                                         hipMemcpyHostToDevice, R.h2d);
            }
            if (e == hipSuccess) e = tm.mark(R.h2d, i1);
            if (tm.on) t_h2d.push_back({i0, i1});
        }
        if (e == hipSuccess) e = hipEventRecord(R.ev_h2d[s], R.h2d);
        // kernel
        if (e == hipSuccess) e = hipStreamWaitEvent(cs, R.ev_h2d[s], 0);
        if (e == hipSuccess && b >= RING_SLOTS) e = hipStreamWaitEvent(cs, R.ev_d2h[s], 0);
        if (e == hipSuccess) e = tm.mark(cs, i0);
        if (e == hipSuccess)
            e = launch_channels(P, n > 0 ? R.vals[s].p : nullptr, ldd, (int32_t)w, dtype,
                                (float*)R.out[s].p, cs, P.shape);
        if (e == hipSuccess) e = tm.mark(cs, i1);
        if (tm.on) t_ker.push_back({i0, i1});
        if (e == hipSuccess) e = hipEventRecord(R.ev_ker[s], cs);
        // copy-out
        if (e == hipSuccess) e = hipStreamWaitEvent(R.d2h, R.ev_ker[s], 0);
        if (e == hipSuccess) e = tm.mark(R.d2h, i0);
        if (e == hipSuccess)
            e = hipMemcpyAsync(staged ? R.pin_out[s] : vout + (size_t)c0 * npix * 4, R.out[s].p,
                               (size_t)w * npix * 4, hipMemcpyDeviceToHost, R.d2h);
        if (e == hipSuccess) e = tm.mark(R.d2h, i1);
        if (tm.on) t_d2h.push_back({i0, i1});
        if (e == hipSuccess) e = hipEventRecord(R.ev_d2h[s], R.d2h);
        // staged: hand the previous block's maps back while this one runs
        if (staged && b >= 1 && e == hipSuccess) {
            e = hipEventSynchronize(R.ev_d2h[(b - 1) % RING_SLOTS]);
            if (e == hipSuccess) scatter(b - 1);
        }
    }
    if (e == hipSuccess && staged && nb > 0) {
        e = hipEventSynchronize(R.ev_d2h[(nb - 1) % RING_SLOTS]);
        if (e == hipSuccess) scatter(nb - 1);
    }
    hipError_t e2 = hipStreamSynchronize(R.d2h);
    if (e == hipSuccess) e = e2;
    e2 = hipStreamSynchronize(R.h2d);
    if (e == hipSuccess) e = e2;
    e2 = hipStreamSynchronize(cs);
    if (e == hipSuccess) e = e2;
    if (e != hipSuccess) {
        err = std::string("grid_channels_host: ") + hipGetErrorString(e);
        return e == hipErrorOutOfMemory ? HG_ERR_NOMEM : HG_ERR_DEVICE;
    }
    P.ch_calls += nb;
    if (info) {
        std::memset(info, 0, sizeof *info);
        info->blocks = nb;
        info->pinned = direct ? 1 : 0;
        info->h2d_bytes = (int64_t)n * nchan * (int64_t)es;
        info->d2h_bytes = (int64_t)nchan * npix * 4;
        info->kernel_ms = tm.sum(t_ker);
        info->h2d_ms = tm.sum(t_h2d);
        info->d2h_ms = tm.sum(t_d2h);
        info->wall_ms = std::chrono::duration<double, std::milli>(
                            std::chrono::steady_clock::now() - t0)
                            .count();
    }
    return HG_OK;
}

}  // namespace hg

// ---------------------------------------------------------------------------
// The same streamed channel phase for callers that cannot allocate
// (hg_grid_channels_host_noalloc): the two device slots live in one fixed
// staging array of HG_NOALLOC_STAGING_BYTES per device instead of plan-owned
// buffers, the copy streams and their events are made once per device, the
// caller's buffers must be page-locked (no pinned staging of the library's
// own), and the kernel takes its work items in plain order (no launch-order
// buffer).  The kernels and the per-cell arithmetic are those of
// hg_grid_channels_host, so the maps are identical.  Calls that overlap on
// one device race on the array and the streams.
namespace hg {
namespace {

static __device__ __align__(256) unsigned char scratch[HG_NOALLOC_STAGING_BYTES];

struct NoAllocDevice {
    bool ready = false;
    char* ptr = nullptr;  // this device's copy of `scratch` (never the host-side name)
    hipStream_t h2d = nullptr, d2h = nullptr;
    hipEvent_t ev_h2d[RING_SLOTS] = {nullptr, nullptr};
    hipEvent_t ev_ker[RING_SLOTS] = {nullptr, nullptr};
    hipEvent_t ev_d2h[RING_SLOTS] = {nullptr, nullptr};
};
constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex g_noalloc_mu;
NoAllocDevice g_noalloc[NOALLOC_MAX_DEVICES];

// Once per device, with that device current: the staging array's device
// address, two copy streams and the slot events.
int noalloc_device(int dev, NoAllocDevice** out, std::string& err) {
    if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) {
        err = "device index beyond the staging table";
        return HG_ERR_UNSUPPORTED;
    }
    std::lock_guard<std::mutex> lk(g_noalloc_mu);
    NoAllocDevice& D = g_noalloc[dev];
    if (!D.ready) {
        void* p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            err = std::string("staging array address: ") + hipGetErrorString(e);
            return HG_ERR_DEVICE;
        }
        if (!D.h2d) e = hipStreamCreateWithFlags(&D.h2d, hipStreamNonBlocking);
        if (e == hipSuccess && !D.d2h) e = hipStreamCreateWithFlags(&D.d2h, hipStreamNonBlocking);
        for (int s = 0; s < RING_SLOTS && e == hipSuccess; s++)
            for (hipEvent_t* ev : {&D.ev_h2d[s], &D.ev_ker[s], &D.ev_d2h[s]})
                if (e == hipSuccess && !*ev) e = hipEventCreateWithFlags(ev, hipEventDisableTiming);
        if (e != hipSuccess) {
            err = std::string("staging streams: ") + hipGetErrorString(e);
            return HG_ERR_DEVICE;
        }
        D.ptr = (char*)p;
        D.ready = true;
    }
    *out = &D;
    return HG_OK;
}

size_t round256(size_t b) { return (b + 255) / 256 * 256; }

}  // namespace

int grid_channels_host_noalloc(Plan& P, const void* host_values, int64_t ld, int32_t nchan,
                               int32_t dtype, float* host_out, int32_t block, hipStream_t cs,
                               hg_stream_info* info, std::string& err) {
    auto t0 = std::chrono::steady_clock::now();
    if ((P.n > 0 && !is_pinned(host_values)) || !is_pinned(host_out)) {
        err = "host_values and host_out must be page-locked (hipHostMalloc or pinned tensors)";
        return HG_ERR_ARG;
    }
    const size_t es = dtype == HG_F32 ? 4 : 2;
    const int64_t n = P.n, npix = P.npix;
    // staging bytes of a block of b channels: two slots of values and of maps
    auto need = [&](int64_t b, int64_t ldd) {
        return 2 * round256((size_t)std::max<int64_t>(n, 1) * ldd * es) +
               2 * round256((size_t)b * npix * 4);
    };
    int64_t blk = block;
    if (blk == 0) {
        // the widest block that fits the staging array
        blk = std::min<int64_t>(nchan, 4096);
        while (blk > 1 && need(blk, (blk + 7) / 8 * 8) > (size_t)HG_NOALLOC_STAGING_BYTES) blk--;
    }
    blk = std::min<int64_t>(blk, nchan);
    const int nb = (int)((nchan + blk - 1) / blk);
    const bool linear = nb == 1 && blk == ld;
    const int64_t ldd = linear ? ld : (blk + 7) / 8 * 8;
    if (need(blk, ldd) > (size_t)HG_NOALLOC_STAGING_BYTES) {
        err = "a block of " + std::to_string(blk) + " channels needs " +
              std::to_string(need(blk, ldd)) + " bytes of staging, over the fixed " +
              std::to_string((size_t)HG_NOALLOC_STAGING_BYTES) + "; use a smaller block";
        return HG_ERR_ARG;
    }
    NoAllocDevice* D = nullptr;
    int rc = noalloc_device(P.device, &D, err);
    if (rc) return rc;
    char* vals[RING_SLOTS];
    float* outs[RING_SLOTS];
    const size_t val_al = round256((size_t)std::max<int64_t>(n, 1) * ldd * es);
    const size_t out_al = round256((size_t)blk * npix * 4);
    for (int s = 0; s < RING_SLOTS; s++) {
        vals[s] = D->ptr + s * val_al;
        outs[s] = (float*)(D->ptr + RING_SLOTS * val_al + s * out_al);
    }
    const char* vin = (const char*)host_values;
    char* vout = (char*)host_out;
    hipError_t e = hipSuccess;
    for (int b = 0; b < nb && e == hipSuccess; b++) {
        const int s = b % RING_SLOTS;
        const int64_t c0 = (int64_t)b * blk;
        const int64_t w = std::min<int64_t>(blk, nchan - c0);
        if (b >= RING_SLOTS) e = hipStreamWaitEvent(D->h2d, D->ev_ker[s], 0);
        if (n > 0 && e == hipSuccess) {
            if (linear)
                e = hipMemcpyAsync(vals[s], vin, (size_t)n * ld * es, hipMemcpyHostToDevice, D->h2d);
            else
                e = hipMemcpy2DAsync(vals[s], (size_t)ldd * es, vin + (size_t)c0 * es,
                                     (size_t)ld * es, (size_t)w * es, (size_t)n,
                                     hipMemcpyHostToDevice, D->h2d);
        }
        if (e == hipSuccess) e = hipEventRecord(D->ev_h2d[s], D->h2d);
        if (e == hipSuccess) e = hipStreamWaitEvent(cs, D->ev_h2d[s], 0);
        if (e == hipSuccess && b >= RING_SLOTS) e = hipStreamWaitEvent(cs, D->ev_d2h[s], 0);
        if (e == hipSuccess)
            e = launch_channels_plain_order(P, n > 0 ? vals[s] : nullptr, ldd, (int32_t)w, dtype,
                                            outs[s], cs, P.shape);
        if (e == hipSuccess) e = hipEventRecord(D->ev_ker[s], cs);
        if (e == hipSuccess) e = hipStreamWaitEvent(D->d2h, D->ev_ker[s], 0);
        if (e == hipSuccess)
            e = hipMemcpyAsync(vout + (size_t)c0 * npix * 4, outs[s], (size_t)w * npix * 4,
                               hipMemcpyDeviceToHost, D->d2h);
        if (e == hipSuccess) e = hipEventRecord(D->ev_d2h[s], D->d2h);
    }
    hipError_t e2 = hipStreamSynchronize(D->d2h);
    if (e == hipSuccess) e = e2;
    e2 = hipStreamSynchronize(D->h2d);
    if (e == hipSuccess) e = e2;
    e2 = hipStreamSynchronize(cs);
    if (e == hipSuccess) e = e2;
    if (e != hipSuccess) {
        err = std::string("grid_channels_host_noalloc: ") + hipGetErrorString(e);
        return HG_ERR_DEVICE;
    }
    P.ch_calls += nb;
    if (info) {
        std::memset(info, 0, sizeof *info);
        info->blocks = nb;
        info->pinned = 1;
        info->h2d_bytes = (int64_t)n * nchan * (int64_t)es;
        info->d2h_bytes = (int64_t)nchan * npix * 4;
        info->wall_ms = std::chrono::duration<double, std::milli>(
                            std::chrono::steady_clock::now() - t0)
                            .count();
    }
    return HG_OK;
}

}  // namespace hg
