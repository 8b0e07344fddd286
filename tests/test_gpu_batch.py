"""GPU tests of the batched form (hg_batch_*): many fields in one graph-held
launch.

  * The batched launch runs the same per-item arithmetic as hg_grid_channels,
    so its maps must equal the single-field maps bit for bit (NaN included).
  * Against the FP64 reference, on the batching workload's geometry scaled
    down (log-uniform sample counts, square maps 32..512, FWHM U(2, 5)
    arcmin, FP16 values): counts bit-exact on every pixel, maps within 1e-6
    (FP32 form) or 2e-3 (FP16 MFMA form) on sampled channels.
  * Graph replays, with eager work on the same buffers in between, reproduce
    the first run.
"""
import math

import numpy as np
import pytest

import oracle
from paper_2207_04584_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2207_04584_amd import api  # noqa: E402
from parity_util import abs_values, assert_fp32_bound, norm_err, to_host_values  # noqa: E402

ARC = 1.0 / 60.0
DEV = "cuda:0"


def mixed_fields(dtype=torch.float32):
    """Fields of uneven shapes: ragged maps, a channel count that spills one
    sample past a 256-channel block, no samples, no channels, samples mostly
    outside the map, a map across RA = 0."""
    specs = [  # (seed, n, nx, ny, ra0, dec0, fwhm, C, spread)
        (1, 3000, 40, 37, 150.0, 20.0, 3.0, 300, 1.3),
        (2, 0, 16, 16, 10.0, -5.0, 3.0, 5, 1.0),
        (3, 500, 70, 20, 200.0, 45.0, 2.5, 0, 1.3),
        (4, 2000, 33, 65, 0.2, -30.0, 4.0, 7, 1.3),
        (5, 1500, 16, 16, 80.0, 60.0, 3.0, 256, 3.0),
        (6, 4000, 100, 8, 300.0, 10.0, 2.0, 513, 1.2),
        (7, 800, 5, 3, 45.0, 0.0, 5.0, 33, 1.5),
    ]
    fields = []
    for seed, n, nx, ny, ra0, dec0, fwhm, C, spread in specs:
        rng = np.random.default_rng(1000 + seed)
        ra = np.mod(ra0 + (rng.random(n) - 0.5) * nx * ARC * spread, 360.0)
        dec = dec0 + (rng.random(n) - 0.5) * ny * ARC * spread
        vals = None
        if C > 0:
            vals = torch.from_numpy(rng.normal(2.0, 1.0, size=(n, C)).astype(np.float32))
            vals = vals.to(dtype).to(DEV)
        fields.append({"ra": ra, "dec": dec, "map": synth.make_map(ra0, dec0, nx, ny),
                       "kernel": synth.make_kernel(fwhm), "values": vals})
    return fields


def expected_items(fields):
    total = 0
    for f in fields:
        if f["values"] is None:
            continue
        ntx = math.ceil(math.ceil(f["map"]["nx"] / 2) / 8)
        nty = math.ceil(math.ceil(f["map"]["ny"] / 2) / 8)
        total += ntx * nty * math.ceil(f["values"].shape[1] / 256)
    return total


@pytest.mark.parametrize("chunk", [0, 16])
def test_batch_equals_single_plans_bitwise(chunk):
    fields = mixed_fields()
    print(f"\n  {len(fields)} mixed fields, chunk={chunk}", flush=True)
    with api.Batch(fields, chunk=chunk, time_runs=True) as b:
        outs = [o.clone() if o is not None else None for o in b.run()]
        st = b.stats()
        assert st["n_fields"] == len(fields)
        assert st["n_items"] == expected_items(fields)
        assert st["n_workgroups"] % 8 == 0 and st["n_workgroups"] >= st["n_items"]
        assert st["runs"] == 1 and st["last_run_ms"] > 0
        for i, f in enumerate(fields):
            p = b.plan(i)
            cnt_b = p.counts()
            # a batch field may start at another chunk length than a single
            # plan (the chunk sets the summation's grouping): compare at the
            # field's own
            with api.Plan(f["ra"], f["dec"], f["map"], f["kernel"],
                          chunk=chunk or p.stats()["chunk"]) as q:
                np.testing.assert_array_equal(cnt_b, q.counts())
                if f["values"] is None:
                    continue
                ref = q.grid(f["values"]).cpu().numpy()
            got = outs[i].cpu().numpy()
            assert np.array_equal(got, ref, equal_nan=True), f"field {i} differs"
        nnz = sum(int(b.plan(i).counts().sum()) for i in range(len(fields)))
        assert st["nnz"] == nnz


def test_batch_graph_replays_with_eager_work_between():
    fields = mixed_fields()
    with api.Batch(fields) as b:
        first = [o.clone() for o in b.run() if o is not None]
        for rep in range(3):
            for o in b.outs:
                if o is not None:
                    o.fill_(-7.0)  # eager kernels on the bound buffers
            torch.cuda.synchronize()
            again = [o.clone() for o in b.run() if o is not None]
            torch.cuda.synchronize()
            for a, c in zip(first, again):
                assert torch.equal(torch.nan_to_num(a, nan=1e30), torch.nan_to_num(c, nan=1e30)), rep
        assert b.stats()["runs"] == 4


def test_batch_plan_is_borrowed():
    fields = mixed_fields()[:2]
    b = api.Batch(fields)
    p = b.plan(0)
    L = api.lib()
    assert L.hg_grid_finish(p._h) == api.HG_ERR_STATE
    assert "batch" in api.last_error()
    out = p.grid(fields[0]["values"])  # a borrowed plan still grids
    assert out.shape == (fields[0]["values"].shape[1], 37, 40)
    p.close()  # releases the borrow only
    b.run()
    b.close()
    with pytest.raises(api.HegridError):
        b.plan(0)


def test_batch_mixed_dtypes_rejected():
    fields = mixed_fields()[:2]
    fields[1]["values"] = torch.zeros((0, 5), dtype=torch.float16, device=DEV)
    with pytest.raises(api.HegridError):
        api.Batch(fields)


def scaled_workload(scale, n_fields):
    fs = synth.batch_fields(n_fields, scale=scale)
    out = []
    for f in fs:
        vals = synth.sky_values(f, f["nchan"], device=DEV, dtype="f16")
        out.append({"ra": f["ra"], "dec": f["dec"], "map": f["map"], "kernel": f["kernel"],
                    "values": vals})
    return out


@pytest.mark.parametrize("precision,tol", [(api.HG_PREC_FP32, 1e-6), (2, 2e-3)])
def test_batch_workload_against_reference(precision, tol):
    fields = scaled_workload(0.02, 64)
    print(f"\n  64 fields, n {min(len(f['ra']) for f in fields)}..{max(len(f['ra']) for f in fields)}"
          f", precision {precision}", flush=True)
    worst = 0.0
    with api.Batch(fields, precision=precision, time_runs=True) as b:
        outs = b.run()
        torch.cuda.synchronize()
        st = b.stats()
        print(f"  items {st['n_items']} nnz {st['nnz']} run {st['last_run_ms']:.3f} ms "
              f"setup {st['setup_ms']:.1f} ms", flush=True)
        for i, f in enumerate(fields):
            C = f["values"].shape[1]
            chans = np.array(sorted({0, C // 2, C - 1}))
            hv, code = to_host_values(f["values"])
            Vr, cr, Wr, margin = oracle.grid(f["ra"], f["dec"], hv, code, f["map"],
                                             f["kernel"]["fwhm_deg"],
                                             f["kernel"]["support_deg"], chans=chans)
            assert margin > 1e-12, f"field {i}: closest call {margin:g}"
            p = b.plan(i)
            np.testing.assert_array_equal(p.counts(), cr, err_msg=f"field {i}")
            V = outs[i].cpu().numpy().reshape(C, -1)[chans]
            ok = cr > 0
            np.testing.assert_array_equal(np.isnan(V), np.isnan(Vr), err_msg=f"field {i}")
            e_max, _ = norm_err(V, Vr, ok)
            worst = max(worst, e_max)
            assert e_max <= tol, f"field {i}: e_max {e_max:g} > {tol:g}"
    print(f"  worst e_max {worst:.3g}", flush=True)


def test_batch_workload_full_size_against_reference():
    """The 64-field batching workload at full size (sample counts 1e4..2e6,
    maps 32..512, 256/1024/4096 FP16 channels, FWHM U(2, 5) arcmin; about
    3e10 sample x channels) in the FP16 MFMA form, one graph-held launch.
    Reference: two channels of every field on 80 sampled pixels and the map
    corners (counts bit-exact there), plus the smallest field's every pixel.
    (Its densest field, about 7e4 neighbours per pixel, still fits 64-slot
    chunks; test_dense_fields_take_shorter_chunks reaches that fallback.)"""
    fs = synth.batch_fields(64)
    fields = []
    for f in fs:
        fields.append({"ra": f["ra"], "dec": f["dec"], "map": f["map"], "kernel": f["kernel"],
                       "values": synth.sky_values(f, f["nchan"], device=DEV, dtype="f16")})
    torch.cuda.synchronize()
    nc = sum(len(f["ra"]) * f["nchan"] for f in fs)
    print(f"\n  64 fields, sum N*C = {nc:.3e}", flush=True)
    rng = np.random.default_rng(44)
    small = min(range(64), key=lambda i: len(fs[i]["ra"]) * fs[i]["map"]["nx"] ** 2)
    worst = 0.0
    with api.Batch(fields, precision=2, time_runs=True) as b:
        outs = b.run()
        torch.cuda.synchronize()
        st = b.stats()
        print(f"  items {st['n_items']} nnz {st['nnz']} run {st['last_run_ms']:.1f} ms "
              f"setup {st['setup_ms']:.1f} ms", flush=True)
        dens = [b.plan(i).stats() for i in range(64)]
        densest = max(range(64), key=lambda i: dens[i]["nnz"] / (fs[i]["map"]["nx"] ** 2))
        print(f"  densest field {densest}: {dens[densest]['nnz'] / fs[densest]['map']['nx'] ** 2:.0f}"
              f" neighbours per pixel, chunk {dens[densest]['chunk']}", flush=True)
        for i, f in enumerate(fs):
            C = f["nchan"]
            P = f["map"]["nx"] * f["map"]["ny"]
            chans = np.array([int(rng.integers(C)), C - 1])
            nx = f["map"]["nx"]
            pix = None if i == small else np.unique(np.concatenate(
                [rng.choice(P, 80, replace=False), [0, nx - 1, P - nx, P - 1]]))
            hv, code = to_host_values(fields[i]["values"][:, chans].contiguous())
            Vr, cr, _, margin = oracle.grid(f["ra"], f["dec"], hv, code, f["map"],
                                            f["kernel"]["fwhm_deg"], f["kernel"]["support_deg"],
                                            pix=pix)
            assert margin > 1e-12, f"field {i}: closest call {margin:g}"
            cnt = b.plan(i).counts()
            sel = np.arange(P) if pix is None else pix
            np.testing.assert_array_equal(cnt[sel], cr, err_msg=f"field {i}")
            V = outs[i].reshape(C, -1)[torch.from_numpy(chans).to(DEV)].cpu().numpy()[:, sel]
            np.testing.assert_array_equal(np.isnan(V), np.isnan(Vr), err_msg=f"field {i}")
            e_max, _ = norm_err(V, Vr, cr > 0)
            worst = max(worst, e_max)
            assert e_max <= 2e-3, f"field {i}: e_max {e_max:g}"
    print(f"  worst e_max {worst:.3g} over 64 fields", flush=True)


@pytest.mark.parametrize("precision,first,tol", [(2, 64, 2e-3), (api.HG_PREC_FP32, 48, None)])
def test_dense_fields_take_shorter_chunks(precision, first, tol):
    """A field so dense for its tiles (a 12 arcmin beam, R = 15 px, over
    16 x 16-pixel tiles: most samples reach most of a tile's pixel groups)
    that its densest entry block does not fit two staged chunks of the first
    length in LDS: setup must build it at a shorter chunk (the length a batch
    field starts at is predicted from its support, and a miss is rebuilt
    shorter), inside a batch beside a light field, and the maps must still
    match the reference.
    With about 86,000 neighbours per pixel, FP32 summation in any order errs
    by up to gamma_K (K = 86,000: 5e-3) of the summed terms, so the FP32
    form is held to that rounding bound cell by cell (the 1e-6 gate applies
    to the workloads with a few hundred neighbours per pixel); the 16-bit
    form keeps its 2e-3 gate."""
    rng = np.random.default_rng(77)
    # 400,000 samples over the 1 x 1 deg field: a tile holds over 1024 chunks of
    # slots, so its slots stay in consecutive runs per chunk (dealing is for
    # lighter tiles), and a chunk near a tile's centre reaches all 64 groups
    n = 400_000
    ra = 150.0 + (rng.random(n) - 0.5) * 1.0
    dec = 20.0 + (rng.random(n) - 0.5) * 1.0
    dt = torch.float16 if precision == 2 else torch.float32
    C = 6
    vals = torch.from_numpy(rng.normal(3.0, 1.0, size=(n, C)).astype(np.float32)).to(dt).to(DEV)
    dense = {"ra": ra, "dec": dec, "map": synth.make_map(150.0, 20.0, 32, 32),
             "kernel": synth.make_kernel(12.0), "values": vals}
    light = mixed_fields(dt)[0]
    light["values"] = light["values"][:, :C].contiguous()
    with api.Batch([dense, light], precision=precision) as b:
        outs = b.run()
        torch.cuda.synchronize()
        st = b.plan(0).stats()
        print(f"\n  dense field: {st['nnz'] / 1024:.0f} neighbours per pixel, chunk {st['chunk']}",
              flush=True)
        assert st["chunk"] < first, "the dense field should need a shorter chunk"
        cnt = b.plan(0).counts()
        pix = np.unique(np.concatenate([rng.choice(1024, 120, replace=False), [0, 31, 992, 1023]]))
        hv, code = to_host_values(vals)
        Vr, cr, _, margin = oracle.grid(ra, dec, hv, code, dense["map"], dense["kernel"]["fwhm_deg"],
                                        dense["kernel"]["support_deg"], pix=pix)
        assert margin > 1e-12
        np.testing.assert_array_equal(cnt[pix], cr)
        V = outs[0].reshape(C, -1).cpu().numpy()[:, pix]
        np.testing.assert_array_equal(np.isnan(V), np.isnan(Vr))
        e_max, _ = norm_err(V, Vr, cr > 0)
        print(f"  e_max {e_max:.3g}", flush=True)
        if tol is None:
            Vabs = oracle.grid(ra, dec, abs_values(hv, code), code, dense["map"],
                               dense["kernel"]["fwhm_deg"], dense["kernel"]["support_deg"],
                               pix=pix)[0]
            assert_fp32_bound(V, Vr, Vabs, cr)
        else:
            assert e_max <= tol
