#!/usr/bin/env python3
"""Throughput of the whole gridding path on one MI355X.

Default workload (drift): 1,000,000 samples on 40 drift-scan tracks over a
5 x 5 degree field, a 300 x 300 map at 1 arcmin, Gaussian FWHM 3 arcmin with
3 sigma support, 1024 FP32 channels (synthetic, seeded).  One step = the whole
path on that batch: grid_setup (FP64 binning, sort, look-up table, planner,
neighbour gather) + grid_channels (all 1024 channels) + finish, with
coordinates and values already resident in HBM.

--map healpix / --kernel sinc|elliptical (drift workload): the same samples
gridded onto a HEALPix target patch over the same 5 x 5 degrees (nside 4096,
0.86 arcmin pixels, 228 x 465 cells) and/or with a Gauss-tapered sinc or an
elliptical Gaussian kernel.

--workload batch: 64 independent fields (sample counts log-uniform in
1e4..2e6, square maps of side 32..512 at 1 arcmin, 256 / 1024 / 4096 FP16
channels, FWHM U(2, 5) arcmin).  One step = hg_batch_create (every field's
setup) + one batched channel launch + destroy.  --precision picks the FP16
MFMA form (default) or the FP32 form reading the same FP16 values.

--workload paper: the paper-scale stand-in for its simulated set (1.9e7
samples of 19-beam drift scans over 60 x 20 degrees, a 3600 x 1200 map, 50
FP32 channels), end to end from page-locked host memory: one step =
coordinates to the GPU + setup + channels streamed in and the cube streamed
back + finish.

--workload literal: the drift workload through Algorithm 1 as the paper
states it (one launch per channel, gamma cells per thread, FP64), the
comparison path.

--workload fifo: the 64 fields of the batch workload through a FIFO of host
threads with a stream each (setup, then channel kernel, per field), the
paper's style of pipeline, to set the batched form against.

    python bench.py [--workload drift|batch|paper|literal|fifo] [--steps K] [--warmup W]
                    [--gpus 1] [--streams S] [--map car|healpix]
                    [--kernel gauss|sinc|elliptical]
                    [--precision mfma|fp32] [--no-cpu-baseline]

Prints one JSON line.  value = sum(N * C) / (seconds per step) in G
sample*channel updates per second.  The line also carries the roofline of
the dominant kernel (the channel kernel; its duration from HIP events
recorded around each launch on the stream it runs on) and the FP64 reference
gridder timed on a bounded sample of the same workload on the host.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
PEAK_FP32_MFMA_TFLOPS = 157.3
PEAK_F16_MFMA_TFLOPS = 2500.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def _host_facts():
    """CPU model and logical core count of the host the bench runs on."""
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    model = ln.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return model, os.cpu_count() or 1


def cpu_baseline(f, vals_host, n_pix, seed=7, gpu_out=None, code="f32", threads=None):
    """The reference gridder as it stands, on a random subset of the map's
    pixels with all channels, split over `threads` host threads (each a
    separate single-threaded call on its own pixels; the calls run in C with
    the interpreter lock released); scaled to the full map.  value is the
    all-thread rate, value_1core the mean rate of one thread while all run.
    With gpu_out (the timed path's last map, host [C][P]) the same pixels
    also give the path's error against the reference: per channel max
    |V - V_ref| over max |V_ref|, and the same with RMS norms, worst channel."""
    from concurrent.futures import ThreadPoolExecutor

    import numpy as np

    import oracle
    m = f["map"]
    P = m["nx"] * m["ny"]
    model, ncpu = _host_facts()
    threads = max(1, min(threads or ncpu, n_pix))
    pix = np.sort(np.random.default_rng(seed).choice(P, n_pix, replace=False))
    parts = np.array_split(pix, threads)

    def one(part):
        t0 = time.perf_counter()
        r = oracle.grid(f["ra"], f["dec"], vals_host, code, m, f["kernel"]["fwhm_deg"],
                        f["kernel"]["support_deg"], pix=part, kernel=f["kernel"])
        return r, time.perf_counter() - t0

    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=threads) as ex:
        done = list(ex.map(one, parts))
    dt = time.perf_counter() - t0
    Vr = np.concatenate([d[0][0] for d in done], axis=1)
    cnt = np.concatenate([d[0][1] for d in done])
    busy = sum(d[1] for d in done)
    n, C = vals_host.shape
    res = {"value": n * C / (dt * P / n_pix) / 1e9, "unit": "G sample*channel updates/s",
           "cores": threads, "kind": "oracle",
           "sample": f"{n_pix} of {P} pixels x all {C} channels on {threads} threads "
                     f"({dt:.1f} s wall, {busy:.1f} s of thread time), scaled by "
                     f"{P / n_pix:.1f} to the full map",
           "value_1core": n * C / (busy * P / n_pix) / 1e9,
           "cpu_model": model, "nproc": ncpu}
    if gpu_out is not None:
        res["parity"] = parity(gpu_out[:, pix], Vr, cnt)
    return res


def parity(V, Vr, cnt):
    """Per channel max |V - V_ref| / max |V_ref| and the RMS analogue over
    cells with neighbours (worst channel), and whether the empty cells
    match."""
    import numpy as np
    ok = cnt > 0
    Vk = V[:, ok].astype(np.float64)
    R = Vr[:, ok]
    d = np.abs(Vk - R)
    e_max = float((d.max(1) / np.maximum(np.abs(R).max(1), 1e-300)).max()) if d.size else 0.0
    e_rms = float((np.sqrt((d ** 2).mean(1)) /
                   np.maximum(np.sqrt((R ** 2).mean(1)), 1e-300)).max()) if d.size else 0.0
    return {"e_max": e_max, "e_rms": e_rms, "nan_match": bool((np.isnan(V) == np.isnan(Vr)).all()),
            "pixels": int(ok.sum())}


def measured_traffic(workload, form=None):
    """HBM bytes per launch of the dominant kernel from the committed PMC
    record in profiles/ (form: None for the record's own kernel, else a key
    of the record such as "bf16_form"), or None when there is none or the
    sources it was taken on (the kernel, and the setup that lays out its
    work) have changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"k_channels_{workload}_traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    for src, digest in rec["sources_sha256"].items():
        if hashlib.sha256(open(os.path.join(ROOT, src), "rb").read()).hexdigest() != digest:
            return None
    if form is not None:
        rec = rec.get(form)
        if rec is None:
            return None
    return rec["fetch_bytes_per_launch"] + rec["write_bytes_per_launch"]


def host_values(v):
    """A device tensor as the reference gridder reads it: (array, dtype code)."""
    import numpy as np
    import torch
    if v.dtype == torch.float32:
        return v.cpu().numpy(), "f32"
    code = "bf16" if v.dtype == torch.bfloat16 else "f16"
    return v.cpu().view(torch.int16).numpy().view(np.uint16), code


def roofline(flops, bytes_alg, ms, peak_tflops, kernel):
    t_mfma = flops / (peak_tflops * 1e12)
    t_hbm = bytes_alg / (PEAK_HBM_GBS * 1e9)
    if t_mfma >= t_hbm:
        ach = flops / (ms * 1e-3) / 1e12
        roof = {"bound": "mfma", "achieved": ach, "peak": peak_tflops, "unit": "TFLOP/s",
                "frac": ach / peak_tflops, "traffic": None}
    else:
        ach = bytes_alg / (ms * 1e-3) / 1e9
        roof = {"bound": "hbm", "achieved": ach, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": ach / PEAK_HBM_GBS, "traffic": None}
    roof["kernel"] = kernel
    roof["hbm_frac"] = bytes_alg / (ms * 1e-3) / 1e9 / PEAK_HBM_GBS
    roof["mfma_frac"] = flops / (ms * 1e-3) / 1e12 / peak_tflops
    return roof


def cpu_baseline_batch(fields, vals_dev, nnz_per_field, n_pix, seed=7):
    """The reference gridder, single-threaded, on a random subset of pixels of
    one mid-sized field with all its channels; its rate in (neighbour pair x
    channel) per second, applied to the whole batch's sum of nnz * C."""
    import numpy as np

    import oracle
    order = sorted(range(len(fields)), key=lambda i: nnz_per_field[i] * fields[i]["nchan"])
    i = order[len(order) // 2]
    f = fields[i]
    m = f["map"]
    P = m["nx"] * m["ny"]
    pix = np.sort(np.random.default_rng(seed).choice(P, min(n_pix, P), replace=False))
    hv, code = host_values(vals_dev[i])
    t0 = time.perf_counter()
    _, cnt, _, _ = oracle.grid(f["ra"], f["dec"], hv, code, m, f["kernel"]["fwhm_deg"],
                               f["kernel"]["support_deg"], pix=pix)
    dt = time.perf_counter() - t0
    rate = max(int(cnt.sum()), 1) * f["nchan"] / dt
    total = sum(nnz_per_field[j] * fields[j]["nchan"] for j in range(len(fields)))
    full_s = total / rate
    nc = sum(len(g["ra"]) * g["nchan"] for g in fields)
    return {"value": nc / full_s / 1e9, "unit": "G sample*channel updates/s", "cores": 1,
            "kind": "oracle",
            "sample": f"field {i} ({len(f['ra'])} samples, {m['nx']}x{m['ny']}, {f['nchan']} ch): "
                      f"{len(pix)} pixels x all channels in {dt:.1f} s; rate per (pair x "
                      f"channel) scaled to the batch's sum of nnz x C"}


def time_steps(step, args, label):
    """W untimed steps, then K timed steps bracketed by synchronisations;
    returns ms per step."""
    import torch
    for i in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / args.steps
    log(f"{label}: {args.steps} timed steps, {ms:.3f} ms/step")
    return ms


def drift_leg(args, f, ra, dec, vals, precision, label):
    """Setup + channels per step on the drift workload in one form, in the
    autotuned shape; returns (record, plan stats, last map)."""
    import numpy as np
    import torch

    from paper_2207_04584_amd import api, tune
    m, k = f["map"], f["kernel"]
    C = vals.shape[1]
    out = torch.empty((C, m["ny"], m["nx"]), dtype=torch.float32, device=vals.device)
    if args.no_tune:
        best = {"chunk": 0, "waves": 0, "chan_block": 0, "cached": False, "table": {}}
    else:
        t0 = time.perf_counter()
        best = tune.tune_plan(ra, dec, m, k, vals, precision=precision, use_cache=False)
        log(f"{label}: tuned in {time.perf_counter() - t0:.1f} s -> chunk {best['chunk']}, "
            f"{best['waves']} waves x {best['chan_block']} channels ({best['ms']:.3f} ms)")
    ch_ms, setup_ms, st = [], [], {}

    def step():
        nonlocal st
        plan = api.Plan(ra, dec, m, k, precision=precision, chunk=best["chunk"],
                        waves=best["waves"], chan_block=best["chan_block"], time_channels=True)
        plan.grid(vals, out)
        st = plan.stats()
        plan.close()
        ch_ms.append(st["last_channels_ms"])
        setup_ms.append(st["setup_ms"])

    for _ in range(args.warmup):
        step()
    ch_ms.clear()
    setup_ms.clear()
    ms_step = time_steps(step, argparse.Namespace(warmup=0, steps=args.steps), label)
    rec = {"ms_per_step": ms_step, "channels_ms": float(np.mean(ch_ms)),
           "setup_ms": float(np.mean(setup_ms)),
           "shape": {"chunk": st["chunk"], "waves": st["waves"], "chan_block": st["chan_block"],
                     "tuned": not args.no_tune, "candidates_timed": len(best.get("table", {}))}}
    return rec, st, out


def run_drift(args):
    import numpy as np
    import torch

    from paper_2207_04584_amd import api, synth

    dev = torch.device("cuda:0")
    f = synth.config("cfg2")
    variant = []
    if args.map == "healpix":
        # the same 5 x 5 deg of sky as a HEALPix patch at nside 4096 (0.86' pixels)
        f["map"] = synth.healpix_patch(180.0, 30.0, 5.0, 5.0, 4096)
        variant.append("HEALPix nside-4096 target patch")
    if args.kernel == "sinc":
        f["kernel"] = dict(f["kernel"], type=api.HG_KERNEL_GAUSS_SINC, p1=2.5 * synth.ARCMIN,
                           p2=3.0 * synth.ARCMIN)
        variant.append("Gauss-tapered sinc a=2.5' b=3'")
    elif args.kernel == "elliptical":
        f["kernel"] = dict(f["kernel"], type=api.HG_KERNEL_ELLIPTICAL, p1=2.0 * synth.ARCMIN,
                           p2=30.0)
        variant.append("elliptical Gaussian 3'x2' at PA 30 deg")
    C = f["nchan"]
    n = f["ra"].shape[0]
    m, k = f["map"], f["kernel"]
    P = m["nx"] * m["ny"]
    log(f"generating {n} samples x {C} channels on {torch.cuda.get_device_name(0)}")
    ra = torch.from_numpy(f["ra"]).to(dev)
    dec = torch.from_numpy(f["dec"]).to(dev)
    vals = synth.sky_values(f, C, device=dev)
    torch.cuda.synchronize()

    rec, st, out = drift_leg(args, f, ra, dec, vals, api.HG_PREC_FP32, "plain FP32 form")
    ms_step, ch_avg = rec["ms_per_step"], rec["channels_ms"]
    nnz = st["nnz"]
    value = n * C / (ms_step * 1e-3) / 1e9
    log(f"plain FP32: {ms_step:.3f} ms/step; channel kernel {ch_avg:.3f} ms; setup "
        f"{rec['setup_ms']:.2f} ms")
    roof = roofline(2.0 * nnz * C, 4.0 * n * C + 4.0 * P * C, ch_avg, PEAK_FP32_MFMA_TFLOPS,
                    "k_channels (FP32 form, FP32 values)")
    roof["traffic"] = None if variant else measured_traffic("drift")
    workload = ("drift-scan field: 1e6 samples on 40 tracks, 5x5 deg, "
                "300x300 map at 1 arcmin, FWHM 3 arcmin, support 3 sigma, "
                "1024 FP32 channels; step = setup + channels")
    if variant:
        workload += "; variant: " + ", ".join(variant) + f" ({m['nx']}x{m['ny']} cells)"
    res = {
        "metric": "G sample*channel updates/s (plain FP32 form)",
        "value": value, "unit": "G sample*channel updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": workload, "n_samples": n, "channels": C, "map": [m["ny"], m["nx"]],
                   "nnz": nnz, "entry_units": st["n_entries"], "form": "fp32",
                   "shape": rec["shape"]},
        "channels_ms": ch_avg, "setup_ms": rec["setup_ms"],
        "channels_only_value": n * C / (ch_avg * 1e-3) / 1e9,
        "roofline": roof,
    }
    if not args.no_cpu_baseline:
        log(f"cpu baseline: reference gridder on {args.cpu_pixels} pixels")
        vals_host = vals.cpu().numpy()
        res["cpu_baseline"] = cpu_baseline(f, vals_host, args.cpu_pixels,
                                           gpu_out=out.reshape(C, -1).cpu().numpy())
        log(f"cpu baseline: {res['cpu_baseline']['sample']}; parity "
            f"{res['cpu_baseline'].get('parity')}")
        del vals_host
    if not args.no_mfma_leg and not variant:
        # the precision form on the same workload: the same cube stored as
        # BF16, BF16 weights x values on MFMA with FP32 accumulation
        vb = vals.to(torch.bfloat16)
        del out
        rb, sb, outb = drift_leg(args, f, ra, dec, vb, api.HG_PREC_MFMA_BF16, "BF16-MFMA form")
        rb["value"] = n * C / (rb["ms_per_step"] * 1e-3) / 1e9
        rb["channels_only_value"] = n * C / (rb["channels_ms"] * 1e-3) / 1e9
        rb["roofline"] = roofline(2.0 * sb["nnz"] * C, 2.0 * n * C + 4.0 * P * C,
                                  rb["channels_ms"], PEAK_F16_MFMA_TFLOPS,
                                  "k_channels (BF16 MFMA form)")
        rb["roofline"]["traffic"] = measured_traffic("drift", "bf16_form")
        rb["speedup_vs_plain"] = {"step": ms_step / rb["ms_per_step"],
                                  "channels": ch_avg / rb["channels_ms"]}
        if not args.no_cpu_baseline:
            hv, code = host_values(vb)
            cb = cpu_baseline(f, hv, args.cpu_pixels // 2, seed=8,
                              gpu_out=outb.reshape(C, -1).cpu().numpy(), code=code)
            rb["parity"] = cb["parity"]
            rb["parity"]["reference"] = "FP64 reference gridder on the stored BF16 values"
            del hv
        log(f"BF16-MFMA: {rb['ms_per_step']:.3f} ms/step; channel kernel "
            f"{rb['channels_ms']:.3f} ms; parity {rb.get('parity')}")
        res["mfma_form"] = dict({"dtype": "bf16", "workload": "the same drift-scan cube stored as "
                                 "BF16; step = setup + channels"}, **rb)
        del vb, outb
    if not args.no_batch_leg and not variant:
        del vals
        torch.cuda.empty_cache()
        res["batched_form"] = batch_legs(args)
    return res


def batch_inputs(args):
    """The 64-field workload's fields with their coordinates and FP16 values
    resident on the GPU."""
    import torch

    from paper_2207_04584_amd import synth

    dev = torch.device("cuda:0")
    fs = synth.batch_fields(args.fields, scale=args.scale)
    log(f"generating {len(fs)} fields on {torch.cuda.get_device_name(0)}")
    fields, vals_dev = [], []
    for f in fs:
        v = synth.sky_values(f, f["nchan"], device=dev, dtype="f16")
        vals_dev.append(v)
        fields.append({"ra": torch.from_numpy(f["ra"]).to(dev),
                       "dec": torch.from_numpy(f["dec"]).to(dev), "map": f["map"],
                       "kernel": f["kernel"], "values": v})
    torch.cuda.synchronize()
    nc = sum(f["ra"].shape[0] * f["nchan"] for f in fs)
    pc = sum(f["map"]["nx"] * f["map"]["ny"] * f["nchan"] for f in fs)
    log(f"sum N*C = {nc:.3e}, values {2 * nc / 1e9:.1f} GB, out {4 * pc / 1e9:.1f} GB")
    return fs, fields, vals_dev, nc, pc


def run_fifo(args):
    """The 64 fields through the paper's style of pipeline
    (pipeline.grid_fields_fifo: a FIFO of fields served by host threads with
    a stream each, setup then channel kernel per field), to set the batched
    form against on the same fields and form."""
    import torch

    from paper_2207_04584_amd import api, pipeline

    fs, fields, _, nc, _ = batch_inputs(args)
    mfma = args.precision == "mfma"
    prec = api.HG_PREC_MFMA_F16 if mfma else api.HG_PREC_FP32

    def step():
        pipeline.grid_fields_fifo(fields, n_streams=args.streams, precision=prec)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    ms_step = (time.perf_counter() - t0) * 1e3 / args.steps
    log(f"timed {args.steps} steps: {ms_step:.1f} ms/step, {args.streams} streams")
    return {
        "metric": "G sample*channel updates/s (FIFO multi-stream pipeline, " +
                  ("FP16-MFMA form)" if mfma else "plain FP32 form)"),
        "value": nc / (ms_step * 1e-3) / 1e9, "unit": "G sample*channel updates/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f16" if mfma else "f32", "data": "synthetic",
        "config": {"workload": f"the {len(fs)}-field batching workload; step = every field's "
                               "setup and channel kernel, fields taken in turn by host threads "
                               "with a stream each",
                   "fields": len(fs), "streams": args.streams, "sum_NC": nc,
                   "form": args.precision},
    }


def batch_leg(args, fs, fields, vals_dev, nc, pc, precision, steps, warmup):
    """One form of the batched workload: hg_batch_create (every field's
    setup) + one batched launch + destroy per step, in the autotuned shape."""
    import numpy as np

    from paper_2207_04584_amd import api, tune
    mfma = precision != api.HG_PREC_FP32
    if args.no_tune:
        best = {"waves": 0, "chan_block": 0, "table": {}}
    else:
        t0 = time.perf_counter()
        best = tune.tune_batch(fields, precision=precision, use_cache=False)
        log(f"batch {'fp16-mfma' if mfma else 'fp32'}: tuned in {time.perf_counter() - t0:.1f} s "
            f"-> {best['waves']} waves x {best['chan_block']} channels ({best['ms']:.1f} ms)")
    run_ms, setup_ms, info, nnz_f = [], [], {}, []

    def step():
        nonlocal info
        b = api.Batch(fields, precision=precision, time_runs=True, waves=best["waves"],
                      chan_block=best["chan_block"])
        b.run()
        info = b.stats()
        if not nnz_f:  # per-field nnz, for the flop count and the reference's scaling
            nnz_f.extend(int(b.plan(i).stats()["nnz"]) for i in range(len(fields)))
        b.close()
        run_ms.append(info["last_run_ms"])
        setup_ms.append(info["setup_ms"])

    for _ in range(warmup):
        step()
    run_ms.clear()
    setup_ms.clear()
    ms_step = time_steps(step, argparse.Namespace(warmup=0, steps=steps),
                         "batch " + ("fp16-mfma" if mfma else "fp32"))
    run_avg = float(np.mean(run_ms))
    flops = 2.0 * sum(nnz_f[i] * fs[i]["nchan"] for i in range(len(fs)))
    bytes_alg = 2.0 * nc + 4.0 * pc
    kname = ("k_channels_batch (FP16 MFMA form)" if mfma else
             "k_channels_batch (FP32 form, FP16 values)")
    rec = {"form": "fp16-mfma" if mfma else "fp32", "ms_per_step": ms_step,
           "value": nc / (ms_step * 1e-3) / 1e9, "channels_ms": run_avg,
           "setup_ms": float(np.mean(setup_ms)), "channels_only_value": nc / (run_avg * 1e-3) / 1e9,
           "nnz": info["nnz"], "items": info["n_items"],
           "shape": {"waves": best["waves"] or 16, "chan_block": best["chan_block"] or 256,
                     "tuned": not args.no_tune, "candidates_timed": len(best.get("table", {}))},
           "roofline": roofline(flops, bytes_alg, run_avg,
                                PEAK_F16_MFMA_TFLOPS if mfma else PEAK_FP32_MFMA_TFLOPS, kname)}
    return rec, nnz_f


def batch_legs(args):
    """The 64-field batching workload in the FP16-MFMA form and in the FP32
    form on the same FP16 values (a few steps each), with the error of one
    field's sampled pixels against the reference for each form."""
    import numpy as np
    import torch

    from paper_2207_04584_amd import api
    fs, fields, vals_dev, nc, pc = batch_inputs(args)
    steps, warmup = min(args.steps, 5), min(args.warmup, 2)
    out = {}
    for prec in (api.HG_PREC_MFMA_F16, api.HG_PREC_FP32):
        rec, nnz_f = batch_leg(args, fs, fields, vals_dev, nc, pc, prec, steps, warmup)
        if not args.no_cpu_baseline:
            # one mid-cost field, sampled pixels and channels, against the reference
            order = sorted(range(len(fs)), key=lambda i: nnz_f[i] * fs[i]["nchan"])
            i = order[len(order) // 2]
            with api.Batch(fields[i:i + 1], precision=prec) as b:
                o = b.run()[0]
                torch.cuda.synchronize()
                cnt_all = b.plan(0).counts()
            fi = fs[i]
            P = fi["map"]["nx"] * fi["map"]["ny"]
            rng = np.random.default_rng(9)
            pix = np.sort(rng.choice(P, min(600, P), replace=False))
            chans = np.sort(rng.choice(fi["nchan"], min(16, fi["nchan"]), replace=False))
            hv, code = host_values(vals_dev[i][:, torch.from_numpy(chans).to(vals_dev[i].device)]
                                   .contiguous())
            import oracle
            Vr, cr, _, _ = oracle.grid(fi["ra"], fi["dec"], hv, code, fi["map"],
                                       fi["kernel"]["fwhm_deg"], fi["kernel"]["support_deg"],
                                       pix=pix)
            V = o.reshape(fi["nchan"], -1)[torch.from_numpy(chans).to(o.device)].cpu().numpy()
            rec["parity"] = dict(parity(V[:, pix], Vr, cr), field=i,
                                 counts_match=bool(np.array_equal(cnt_all[pix], cr)))
        log(f"batch {rec['form']}: {rec['ms_per_step']:.1f} ms/step, launch {rec['channels_ms']:.1f} "
            f"ms; parity {rec.get('parity')}")
        out[rec["form"]] = rec
    out["speedup_mfma_vs_fp32"] = {
        "step": out["fp32"]["ms_per_step"] / out["fp16-mfma"]["ms_per_step"],
        "launch": out["fp32"]["channels_ms"] / out["fp16-mfma"]["channels_ms"]}
    out["workload"] = (f"{len(fs)} fields, samples log-uniform 1e4..2e6, maps 32..512 at "
                       "1 arcmin, 256/1024/4096 FP16 channels, FWHM U(2,5) arcmin; step = batch "
                       "setup + one batched launch")
    out["sum_NC"] = nc
    return out


def run_batch(args):
    from paper_2207_04584_amd import api

    fs, fields, vals_dev, nc, pc = batch_inputs(args)
    mfma = args.precision == "mfma"
    prec = api.HG_PREC_MFMA_F16 if mfma else api.HG_PREC_FP32
    rec, nnz_f = batch_leg(args, fs, fields, vals_dev, nc, pc, prec, args.steps, args.warmup)
    log(f"timed {args.steps} steps: {rec['ms_per_step']:.3f} ms/step; batched launch "
        f"{rec['channels_ms']:.3f} ms; setup {rec['setup_ms']:.1f} ms; items {rec['items']}")
    res = {
        "metric": "G sample*channel updates/s (" + ("FP16-MFMA batched form)" if mfma else
                                                    "plain FP32 form, batched)"),
        "value": rec["value"], "unit": "G sample*channel updates/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": rec["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f16" if mfma else "f32", "data": "synthetic",
        "config": {"workload": f"{len(fs)} fields, samples log-uniform 1e4..2e6, maps 32..512 "
                               "at 1 arcmin, 256/1024/4096 FP16 channels, FWHM U(2,5) arcmin; "
                               "step = batch setup + one batched launch",
                   "fields": len(fs), "scale": args.scale, "sum_NC": nc, "nnz": rec["nnz"],
                   "items": rec["items"], "form": args.precision, "shape": rec["shape"]},
        "channels_ms": rec["channels_ms"], "setup_ms": rec["setup_ms"],
        "channels_only_value": rec["channels_only_value"],
        "roofline": rec["roofline"],
    }
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline_batch(fs, vals_dev, nnz_f, 2 * args.cpu_pixels)
        log(f"cpu baseline: {res['cpu_baseline']['sample']}")
    return res


def run_literal(args):
    """The drift workload through Algorithm 1 as the paper
    states it (hg_grid_channels_literal: one launch per channel, gamma cells
    per thread), to set the tiled matrix-core path against.  A sweep over
    gamma and workgroup size on 16 channels picks the configuration the
    timed steps (setup + all 1024 channels + finish) use."""
    import numpy as np
    import torch

    from paper_2207_04584_amd import api, synth

    dev = torch.device("cuda:0")
    f = synth.config("cfg2")
    C = f["nchan"]
    n = f["ra"].shape[0]
    m, k = f["map"], f["kernel"]
    ra = torch.from_numpy(f["ra"]).to(dev)
    dec = torch.from_numpy(f["dec"]).to(dev)
    vals = synth.sky_values(f, C, device=dev)
    out = torch.empty((C, m["ny"], m["nx"]), dtype=torch.float32, device=dev)
    torch.cuda.synchronize()
    sweep = {}
    with api.Plan(ra, dec, m, k) as p:
        sub = vals[:, :16]
        for gamma in (1, 2, 4):
            for block in (64, 128, 256, 512):
                p.grid_literal(sub, out=out[:16], gamma=gamma, block=block)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                p.grid_literal(sub, out=out[:16], gamma=gamma, block=block)
                torch.cuda.synchronize()
                sweep[f"gamma{gamma}_block{block}"] = (time.perf_counter() - t0) * 1e3 / 16
                log(f"literal sweep: gamma {gamma}, block {block}: "
                    f"{sweep[f'gamma{gamma}_block{block}']:.3f} ms per channel")
    best = min(sweep, key=sweep.get)
    gamma, block = (int(x) for x in best.replace("gamma", "").split("_block"))
    setup_ms = []

    def step():
        plan = api.Plan(ra, dec, m, k)
        plan.grid_literal(vals, out=out, gamma=gamma, block=block)
        torch.cuda.synchronize()
        setup_ms.append(plan.stats()["setup_ms"])
        plan.close()

    for _ in range(args.warmup):
        step()
    setup_ms.clear()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    ms_step = (time.perf_counter() - t0) * 1e3 / args.steps
    log(f"timed {args.steps} steps: {ms_step:.1f} ms/step with gamma {gamma}, block {block}")
    return {
        "metric": "G sample*channel updates/s (Algorithm 1 as stated, FP64)",
        "value": n * C / (ms_step * 1e-3) / 1e9, "unit": "G sample*channel updates/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "drift-scan field as the default workload (1e6 samples, 300x300, "
                               "1024 FP32 channels); step = setup + Algorithm 1 per channel",
                   "gamma": gamma, "block": block},
        "setup_ms": float(np.mean(setup_ms)), "sweep_ms_per_channel": sweep,
    }


def run_paper(args):
    """End to end from host memory on the paper-scale stand-in (its simulated
    set, Table 2 of Sec. 5.1.2): coordinates and values start in page-locked
    host memory and the cube ends there.  One step = coordinates to the GPU +
    setup, with the values' copy to the GPU on a second stream behind it
    (api.grid_from_host) + channels + the cube back + finish; with
    --paper-bands B (default 8) the channels run in B bands of tile rows, each
    started once the values of its samples have arrived and its rows copied
    back while later bands run (0: one launch after the whole copy); with
    --paper-streamed, setup and then the channels streamed in blocks
    (hg_grid_channels_host), the copies overlapped with the kernel only."""
    import numpy as np
    import torch

    from paper_2207_04584_amd import api, synth

    dev = torch.device("cuda:0")
    f = synth.paper_field(n=args.paper_samples)
    n, C = f["ra"].shape[0], f["nchan"]
    m, k = f["map"], f["kernel"]
    P = m["nx"] * m["ny"]
    log(f"paper-scale field: {n} samples x {C} channels, {m['nx']}x{m['ny']} map, "
        f"{torch.cuda.get_device_name(0)}")
    ra_h = torch.from_numpy(f["ra"]).pin_memory()
    dec_h = torch.from_numpy(f["dec"]).pin_memory()
    vals = synth.sky_values(f, C, device=dev).cpu().pin_memory()
    out = torch.empty((C, m["ny"], m["nx"]), dtype=torch.float32, pin_memory=True)
    overlap = not args.paper_streamed
    if overlap:
        dev_vals = torch.empty((n, C), dtype=torch.float32, device=dev)
        dev_out = torch.empty((C, m["ny"], m["nx"]), dtype=torch.float32, device=dev)
    torch.cuda.synchronize()
    rec = {"setup": [], "kernel": [], "h2d": [], "d2h": [], "wall": []}
    st = {}

    def step():
        nonlocal st
        t0 = time.perf_counter()
        if overlap:
            _, info = api.grid_from_host(ra_h, dec_h, m, k, vals, out=out, dev_values=dev_vals,
                                         dev_out=dev_out, bands=args.paper_bands, pieces=16)
            st = {"nnz": info["nnz"], "setup_ms": info["setup_ms"]}
            info["wall_ms"] = (time.perf_counter() - t0) * 1e3
        else:
            ra = ra_h.to(dev, non_blocking=True)
            dec = dec_h.to(dev, non_blocking=True)
            plan = api.Plan(ra, dec, m, k)
            _, info = plan.grid_host(vals, out=out)
            st = plan.stats()
            plan.close()
        rec["setup"].append(st["setup_ms"])
        rec["kernel"].append(info["kernel_ms"])
        rec["h2d"].append(info["h2d_ms"])
        rec["d2h"].append(info["d2h_ms"])
        rec["wall"].append(info["wall_ms"])

    for i in range(args.warmup):
        step()
        log(f"warmup {i + 1}/{args.warmup}: setup {rec['setup'][-1]:.1f} ms, H2D "
            f"{rec['h2d'][-1]:.1f} ms, kernel {rec['kernel'][-1]:.1f} ms, wall "
            f"{rec['wall'][-1]:.1f} ms")
    for v in rec.values():
        v.clear()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_step = (t1 - t0) * 1e3 / args.steps
    mean = {key: float(np.mean(v)) for key, v in rec.items()}
    log(f"timed {args.steps} steps: {ms_step:.1f} ms/step; setup {mean['setup']:.1f} ms; "
        f"H2D {mean['h2d']:.1f}, kernel {mean['kernel']:.1f}, D2H {mean['d2h']:.1f} ms")
    nnz = st["nnz"]
    roof = roofline(2.0 * nnz * C, 4.0 * n * C + 4.0 * P * C, mean["kernel"],
                    PEAK_FP32_MFMA_TFLOPS, "k_channels (FP32 form, FP32 values)")
    res = {
        "metric": "G sample*channel updates/s (end to end from host memory, plain FP32 form)",
        "value": n * C / (ms_step * 1e-3) / 1e9, "unit": "G sample*channel updates/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"paper-scale stand-in: {n} samples from 19-beam drift scans over "
                               "60x20 deg at (30, 41) deg, 3600x1200 map at 1 arcmin, FWHM 3 "
                               "arcmin, 50 FP32 channels in page-locked host memory; step = "
                               + (("coordinates H2D + setup (values H2D on a second stream, in 16 "
                                   f"index pieces) + channels in {args.paper_bands} bands of tile "
                                   "rows, each started once its samples' piece has arrived, its "
                                   "rows D2H while later bands run") if overlap and args.paper_bands
                                  else "coordinates H2D + setup (values H2D on a second stream) + "
                                  "channels + cube D2H" if overlap else
                                  "coordinates H2D + setup + streamed channels + cube D2H"),
                   "n_samples": n, "channels": C, "map": [m["ny"], m["nx"]], "nnz": nnz},
        "setup_ms": mean["setup"], "phases_wall_ms": mean["wall"], "h2d_ms": mean["h2d"],
        "channels_ms": mean["kernel"], "d2h_ms": mean["d2h"],
        "bands": args.paper_bands if overlap else 0,
        "roofline": roof,
        "paper_context": {"hegrid_s": 40.94, "hardware": "V100 + Xeon Gold 6151",
                          "samples": 1.9e7, "channels": 50,
                          "note": "the paper's end-to-end time includes reading HDF5 files; "
                                  "this step starts from arrays in host memory"},
    }
    if not args.no_cpu_baseline:
        log(f"cpu baseline: reference gridder on {args.cpu_pixels} pixels")
        res["cpu_baseline"] = cpu_baseline(f, vals.numpy(), args.cpu_pixels,
                                           gpu_out=out.reshape(C, -1).numpy())
        log(f"cpu baseline: {res['cpu_baseline']['sample']}")
    return res


def run_cube(args):
    """The large-cube workload at its real size: 1e6 samples of 19 interleaved
    drift-scan beams, 600 x 600 map, 65,536 BF16 channels in page-locked host
    memory, streamed through the device in blocks of 4096 channels with the
    copies in and out overlapped with the BF16-MFMA kernel
    (hg_grid_channels_host).  The host holds the cube a slab of several blocks
    at a time (the whole cube is 131 GB of values and 94 GB of maps); each
    slab is generated on the GPU and copied to page-locked memory before its
    call, outside the timing.  One step = setup + every slab's streamed call."""
    import numpy as np
    import torch

    from paper_2207_04584_amd import api, synth
    dev = torch.device("cuda:0")
    f = synth.config("cfg5")
    C, block, slab = 65536, 4096, args.cube_slab
    nslabs = args.cube_slabs or C // slab
    n = f["ra"].shape[0]
    m, k = f["map"], f["kernel"]
    P = m["nx"] * m["ny"]
    log(f"cube: {n} samples, {nslabs} slabs of {slab} channels (blocks of {block}), "
        f"{m['nx']}x{m['ny']} map, {torch.cuda.get_device_name(0)}")
    ra = torch.from_numpy(f["ra"]).to(dev)
    dec = torch.from_numpy(f["dec"]).to(dev)
    vals_h = synth.pinned_empty((n, slab), torch.bfloat16)
    out_h = synth.pinned_empty((slab, m["ny"], m["nx"]), torch.float32)
    dev_slab = torch.empty((n, slab), dtype=torch.bfloat16, device=dev)

    def fill(s0):
        for b0 in range(s0, s0 + slab, block):
            v = synth.sky_values(f, C, device=dev, dtype="bf16", chan_lo=b0, chan_hi=b0 + block)
            dev_slab[:, b0 - s0:b0 - s0 + block].copy_(v)
            del v
        vals_h.copy_(dev_slab)
        torch.cuda.synchronize()

    t0 = time.perf_counter()
    plan = api.Plan(ra, dec, m, k, precision=api.HG_PREC_MFMA_BF16, time_channels=True)
    torch.cuda.synchronize()
    setup_ms = (time.perf_counter() - t0) * 1e3
    st = plan.stats()
    fill(0)
    plan.grid_host(vals_h, out=out_h, block=block)  # warm-up: the device ring is allocated
    infos = []
    for i in range(nslabs):
        fill(i * slab)
        _, info = plan.grid_host(vals_h, out=out_h, block=block)
        infos.append(info)
        log(f"slab {i}: wall {info['wall_ms']:.0f} ms, copies in {info['h2d_ms']:.0f} ms, "
            f"kernels {info['kernel_ms']:.0f} ms, copies out {info['d2h_ms']:.0f} ms")
    plan.close()
    wall = sum(i["wall_ms"] for i in infos)
    ker = sum(i["kernel_ms"] for i in infos)
    h2d = sum(i["h2d_ms"] for i in infos)
    d2h = sum(i["d2h_ms"] for i in infos)
    nblocks = sum(i["blocks"] for i in infos)
    hb = sum(i["h2d_bytes"] for i in infos)
    db = sum(i["d2h_bytes"] for i in infos)
    Cd = nblocks * block
    e2e = setup_ms + wall
    per_block = ker / max(nblocks, 1)
    roof = roofline(2.0 * st["nnz"] * block, 2.0 * n * block + 4.0 * P * block, per_block,
                    PEAK_F16_MFMA_TFLOPS, "k_channels (BF16 MFMA form), one 4096-channel block")
    return {
        "metric": "G sample*channel updates/s (BF16-MFMA form, streamed from host memory)",
        "value": n * Cd / (e2e * 1e-3) / 1e9, "unit": "G sample*channel updates/s", "n_gpus": 1,
        "steps": 1, "warmup": 1, "ms_per_step": e2e, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "bf16", "data": "synthetic",
        "config": {"workload": f"large drift-scan cube: 1e6 samples of 19 interleaved beams over "
                               f"10x10 deg, 600x600 map at 1 arcmin, {Cd} BF16 channels streamed "
                               f"from page-locked host memory in blocks of {block}; step = setup "
                               "+ every block's copy in, kernel and copy out",
                   "n_samples": n, "channels": Cd, "blocks": nblocks, "slab_channels": slab,
                   "nnz": st["nnz"]},
        "setup_ms": setup_ms, "stream_wall_ms": wall, "kernel_ms_sum": ker, "h2d_ms_sum": h2d,
        "d2h_ms_sum": d2h, "h2d_GBps": hb / (h2d * 1e-3) / 1e9, "d2h_GBps": db / (d2h * 1e-3) / 1e9,
        "overlap": (h2d + ker + d2h) / wall,
        "host_link_bound_ms": max(h2d, d2h), "kernel_ms_per_block": per_block,
        "roofline": roof,
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", choices=["drift", "batch", "paper", "literal", "fifo", "cube"],
                    default="drift")
    ap.add_argument("--cube-slab", type=int, default=8192,
                    help="cube workload: channels per host slab (a multiple of 4096)")
    ap.add_argument("--cube-slabs", type=int, default=0,
                    help="cube workload: slabs to stream (0 = the whole cube)")
    ap.add_argument("--streams", type=int, default=4)
    ap.add_argument("--map", choices=["car", "healpix"], default="car",
                    help="drift workload: plate-carree map or a HEALPix target patch")
    ap.add_argument("--kernel", choices=["gauss", "sinc", "elliptical"], default="gauss",
                    help="drift workload: kernel shape")
    ap.add_argument("--paper-samples", type=int, default=19_000_000)
    ap.add_argument("--paper-bands", type=int, default=8,
                    help="paper workload: bands of tile rows (0: the whole map at once)")
    ap.add_argument("--paper-streamed", action="store_true",
                    help="paper workload: stream the channels after setup (hg_grid_channels_host) "
                         "instead of copying the values during setup")
    ap.add_argument("--precision", choices=["mfma", "fp32"], default="mfma")
    ap.add_argument("--fields", type=int, default=64)
    ap.add_argument("--scale", type=float, default=1.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-tune", action="store_true",
                    help="use the default kernel shape instead of the autotuned one")
    ap.add_argument("--no-mfma-leg", action="store_true",
                    help="drift workload: skip the BF16-MFMA form on the same cube")
    ap.add_argument("--no-batch-leg", action="store_true",
                    help="drift workload: skip the 64-field batched workload in both forms")
    ap.add_argument("--cpu-pixels", type=int, default=9600)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first run one plain elementwise pass over 1 GiB (read 1 GiB, write "
                         "1 GiB) so that hardware byte counters can be scaled against it")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (the path "
              "would shard by channel block or by field, with no exchange)", file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        import torch
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda:0")
        dst = torch.mul(src, 2.0)
        torch.cuda.synchronize()
        log(f"copy calibration: {src.numel() * 4} bytes read, {dst.numel() * 4} bytes written")
        del src, dst
    run = {"drift": run_drift, "batch": run_batch, "paper": run_paper,
           "literal": run_literal, "fifo": run_fifo, "cube": run_cube}[args.workload]
    res = run(args)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
