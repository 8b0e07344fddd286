"""Autotuner of the channel kernel's shapes.

The paper tunes its cell-update kernel's block size by hand: a sweep of
threads per block on the V100 (Sec. 5.3.2) and a hand-picked size on the
MI50 (Sec. 5.4).  Here the shapes of the tiled kernel are swept per workload
and the fastest is kept:

  * chunk      -- tile slots staged in LDS per step (setup lays the entry
                  blocks out per chunk, so each chunk length is a new plan);
  * waves      -- waves per workgroup, 8 or 16 (4 or 8 pixel groups a wave);
  * chan_block -- channels per workgroup, 64, 128 or 256.

waves and chan_block leave the maps unchanged bit for bit (every cell's sums
are the same operations in the same order), so they are set on one plan
(hg_plan_set_shape) and timed there; chunk changes the two-level summation
and is checked against the reference like any other plan.  Each candidate is
timed with HIP events recorded around the channel launch by the library
(HG_FLAG_TIME_CHANNELS), the fastest of a few launches (interference only
ever adds time, and medians of three let it pick a shape 4 % off the best).

Results go to a JSON cache (``$HEGRID_TUNE_CACHE``, else
``~/.cache/hegrid/tune.json``) keyed by the device name, the form, the value
dtype, the channel count and the workload's density (neighbours per pixel
and tiles, rounded on a log scale), so a later run of the same kind of
workload reuses the choice without timing anything.  This module only
orders library calls and reads their timings; every step of the gridding
runs in the library's kernels.
"""
import json
import math
import os

from . import api

SHAPES = ((16, 256), (16, 128), (16, 64), (8, 256), (8, 128), (8, 64))
# chunk lengths to try: the FP32 form stages at most 64 slots (1 KB rows),
# the 16-bit forms up to 112 (512 B rows); a length whose densest entry
# block does not fit LDS is skipped
CHUNKS = {api.HG_PREC_FP32: (56, 48, 32), api.HG_PREC_MFMA_BF16: (112, 96, 80, 64, 48, 32),
          api.HG_PREC_MFMA_F16: (112, 96, 80, 64, 48, 32)}


def cache_path():
    return os.environ.get("HEGRID_TUNE_CACHE") or os.path.join(
        os.path.expanduser("~"), ".cache", "hegrid", "tune.json")


def _load():
    try:
        with open(cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(key, rec):
    data = _load()
    data[key] = rec
    path = cache_path()
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + f".{os.getpid()}.tmp"
        with open(tmp, "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)
        os.replace(tmp, path)
    except OSError:
        pass  # an unwritable cache only costs a new sweep next time


def _device_name():
    import torch
    return torch.cuda.get_device_name(torch.cuda.current_device())


def signature(stats, map, precision, dtype, nchan):
    """Cache key of a workload: device, form, dtype, channels, and the
    plan's neighbours per pixel and tile count (each to a factor of about
    1.4 and 2)."""
    npix = int(map["nx"]) * int(map["ny"])
    dens = max(stats["nnz"], 1) / npix
    ntiles = math.ceil(map["nx"] / 16) * math.ceil(map["ny"] / 16)
    return (f"{_device_name()}|prec{int(precision)}|{dtype}|C{int(nchan)}|"
            f"nbr{round(2 * math.log2(dens)) / 2:g}|tiles{round(math.log2(max(ntiles, 1)))}")


def _dtype_name(values):
    return str(values.dtype).replace("torch.", "")


def time_shapes(plan, values, out, shapes=SHAPES, reps=5):
    """Fastest device time (ms) of reps launches of the plan's channel kernel
    in each shape, after one untimed launch.
    The plan must have been made with time_channels=True."""
    res = {}
    for waves, cb in shapes:
        plan.set_shape(waves, cb)
        plan.grid(values, out)  # first launch of a shape loads its code object
        ms = []
        for _ in range(reps):
            plan.grid(values, out)
            ms.append(plan.stats()["last_channels_ms"])
        res[(waves, cb)] = float(min(ms))
    plan.set_shape(0, 0)
    return res


def tune_plan(ra_deg, dec_deg, map, kernel, values, precision=api.HG_PREC_FP32, chunks=None,
              shapes=SHAPES, reps=5, use_cache=True):
    """Sweep chunk x shape on this workload; returns the best
    {"chunk", "waves", "chan_block", "ms", "table", "key", "cached"}.
    With use_cache a stored choice for the same kind of workload is returned
    without timing (the plan is still built once, for its density)."""
    import torch
    chunks = CHUNKS[int(precision)] if chunks is None else tuple(chunks)
    nchan = values.shape[1]
    ny, nx = int(map["ny"]), int(map["nx"])
    out = torch.empty((nchan, ny, nx), dtype=torch.float32, device=values.device)
    key, table, best = None, {}, None
    for chunk in chunks:
        try:
            plan = api.Plan(ra_deg, dec_deg, map, kernel, precision=precision, chunk=chunk,
                            time_channels=True)
        except api.HegridError as e:
            if e.status == api.HG_ERR_UNSUPPORTED:  # the densest block does not fit this chunk
                continue
            raise
        try:
            if key is None:
                key = signature(plan.stats(), map, precision, _dtype_name(values), nchan)
                if use_cache:
                    rec = _load().get(key)
                    if rec is not None:
                        return dict(rec, key=key, cached=True)
            for (waves, cb), ms in time_shapes(plan, values, out, shapes, reps).items():
                table[f"chunk{chunk}_w{waves}_c{cb}"] = ms
                if best is None or ms < best["ms"]:
                    best = {"chunk": chunk, "waves": waves, "chan_block": cb, "ms": ms}
        finally:
            plan.close()
    if best is None:
        raise api.HegridError(api.HG_ERR_UNSUPPORTED, "no chunk length fits this workload")
    rec = dict(best, table=table)
    if key is not None:
        _store(key, rec)
    return dict(rec, key=key, cached=False)


def tuned_plan(ra_deg, dec_deg, map, kernel, values, precision=api.HG_PREC_FP32, **plan_kw):
    """A Plan in the tuned shape for this workload (cached, or swept now)."""
    best = tune_plan(ra_deg, dec_deg, map, kernel, values, precision=precision)
    return api.Plan(ra_deg, dec_deg, map, kernel, precision=precision, chunk=best["chunk"],
                    waves=best["waves"], chan_block=best["chan_block"], **plan_kw), best


def tune_batch(fields, precision=api.HG_PREC_MFMA_F16, shapes=SHAPES, reps=3, use_cache=True):
    """Shape of the batched launch (one kernel for every field, so one
    waves x chan_block for all; each field keeps the longest chunk that fits
    it).  fields as for api.Batch.  Returns {"waves", "chan_block", "ms",
    "table", "key", "cached"}."""
    dt = _dtype_name(next(f["values"] for f in fields if f.get("values") is not None))
    nc = sum(len(f["ra"]) * (0 if f.get("values") is None else f["values"].shape[1])
             for f in fields)
    key = (f"{_device_name()}|batch|prec{int(precision)}|{dt}|fields{len(fields)}|"
           f"nc{round(math.log2(max(nc, 1)))}")
    if use_cache:
        rec = _load().get(key)
        if rec is not None:
            return dict(rec, key=key, cached=True)
    table, best = {}, None
    for waves, cb in shapes:
        with api.Batch(fields, precision=precision, waves=waves, chan_block=cb,
                       time_runs=True) as b:
            b.run()  # first launch of a shape loads its code object
            ms = []
            for _ in range(reps):
                b.run()
                ms.append(b.stats()["last_run_ms"])
        t = float(min(ms))
        table[f"w{waves}_c{cb}"] = t
        if best is None or t < best["ms"]:
            best = {"waves": waves, "chan_block": cb, "ms": t}
    rec = dict(best, table=table)
    _store(key, rec)
    return dict(rec, key=key, cached=False)
