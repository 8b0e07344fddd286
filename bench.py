#!/usr/bin/env python3
"""Throughput of the whole gridding path on one MI355X.

Workload: 1,000,000 samples on 40 drift-scan tracks over a 5 x 5 degree field,
a 300 x 300 map at 1 arcmin, Gaussian FWHM 3 arcmin with 3 sigma support, 1024
FP32 channels (synthetic, seeded).  One step = the whole path on that batch:
grid_setup (FP64 binning, sort, look-up table, planner, neighbour gather) +
grid_channels (all 1024 channels) + finish, with coordinates and values
already resident in HBM.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu-baseline]

Prints one JSON line.  value = N * C / (seconds per step) in G sample*channel
updates per second.  The line also carries the roofline of the dominant
kernel (the channel kernel; its duration from HIP events recorded around each
launch on the stream it runs on) and the FP64 reference gridder timed on a
bounded sample of the same workload on the host.
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


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_baseline(f, vals_host, n_pix, seed=7):
    """The reference gridder as it stands, single-threaded, on a random subset
    of the map's pixels with all channels; scaled to the full map."""
    import numpy as np

    import oracle
    m = f["map"]
    P = m["nx"] * m["ny"]
    pix = np.sort(np.random.default_rng(seed).choice(P, n_pix, replace=False))
    t0 = time.perf_counter()
    oracle.grid(f["ra"], f["dec"], vals_host, "f32", m, f["kernel"]["fwhm_deg"],
                f["kernel"]["support_deg"], pix=pix)
    dt = time.perf_counter() - t0
    full_s = dt * P / n_pix
    n, C = vals_host.shape
    return {"value": n * C / full_s / 1e9, "unit": "G sample*channel updates/s", "cores": 1,
            "kind": "oracle",
            "sample": f"{n_pix} of {P} pixels x all {C} channels ({dt:.1f} s), scaled by "
                      f"{P / n_pix:.1f} to the full map"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-pixels", type=int, default=3000)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (the path "
              "shards by channel block or field with no exchange; see DESIGN.md)",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2207_04584_amd import api, synth

    dev = torch.device("cuda:0")
    f = synth.config("cfg2")
    C = f["nchan"]
    n = f["ra"].shape[0]
    m, k = f["map"], f["kernel"]
    P = m["nx"] * m["ny"]
    log(f"generating {n} samples x {C} channels on {torch.cuda.get_device_name(0)}")
    ra = torch.from_numpy(f["ra"]).to(dev)
    dec = torch.from_numpy(f["dec"]).to(dev)
    vals = synth.sky_values(f, C, device=dev)
    out = torch.empty((C, m["ny"], m["nx"]), dtype=torch.float32, device=dev)
    torch.cuda.synchronize()

    ch_ms, setup_ms, nnz, entries = [], [], 0, 0

    def step():
        nonlocal nnz, entries
        plan = api.Plan(ra, dec, m, k, time_channels=True)
        plan.grid(vals, out)
        st = plan.stats()
        plan.close()
        ch_ms.append(st["last_channels_ms"])
        setup_ms.append(st["setup_ms"])
        nnz, entries = st["nnz"], st["n_entries"]

    for i in range(args.warmup):
        step()
        log(f"warmup {i + 1}/{args.warmup}: channels {ch_ms[-1]:.3f} ms, setup {setup_ms[-1]:.2f} ms")
    ch_ms.clear()
    setup_ms.clear()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_step = (t1 - t0) * 1e3 / args.steps
    value = n * C / (ms_step * 1e-3) / 1e9
    ch_avg = float(np.mean(ch_ms))
    log(f"timed {args.steps} steps: {ms_step:.3f} ms/step; channel kernel {ch_avg:.3f} ms; "
        f"setup {np.mean(setup_ms):.2f} ms")

    flops = 2.0 * nnz * C
    bytes_alg = 4.0 * n * C + 4.0 * P * C
    t_mfma = flops / (PEAK_FP32_MFMA_TFLOPS * 1e12)
    t_hbm = bytes_alg / (PEAK_HBM_GBS * 1e9)
    if t_mfma >= t_hbm:
        ach = flops / (ch_avg * 1e-3) / 1e12
        roof = {"bound": "mfma", "achieved": ach, "peak": PEAK_FP32_MFMA_TFLOPS,
                "unit": "TFLOP/s", "frac": ach / PEAK_FP32_MFMA_TFLOPS, "traffic": None}
    else:
        ach = bytes_alg / (ch_avg * 1e-3) / 1e9
        roof = {"bound": "hbm", "achieved": ach, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": ach / PEAK_HBM_GBS, "traffic": None}
    roof["kernel"] = "k_channels_fp32"
    roof["hbm_frac"] = bytes_alg / (ch_avg * 1e-3) / 1e9 / PEAK_HBM_GBS

    res = {
        "metric": "G sample*channel updates/s (plain FP32 form)",
        "value": value, "unit": "G sample*channel updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "drift-scan field: 1e6 samples on 40 tracks, 5x5 deg, "
                               "300x300 map at 1 arcmin, FWHM 3 arcmin, support 3 sigma, "
                               "1024 FP32 channels; step = setup + channels",
                   "n_samples": n, "channels": C, "map": [m["ny"], m["nx"]], "nnz": nnz,
                   "entries": entries, "form": "fp32"},
        "channels_ms": ch_avg, "setup_ms": float(np.mean(setup_ms)),
        "channels_only_value": n * C / (ch_avg * 1e-3) / 1e9,
        "roofline": roof,
    }
    if not args.no_cpu_baseline:
        log(f"cpu baseline: reference gridder on {args.cpu_pixels} pixels")
        vals_host = vals.cpu().numpy()
        res["cpu_baseline"] = cpu_baseline(f, vals_host, args.cpu_pixels)
        log(f"cpu baseline: {res['cpu_baseline']['sample']}")
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
