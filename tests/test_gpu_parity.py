"""GPU parity: the HIP path through the C ABI against the FP64 reference.

Bars (the neighbour decision is a comparison of FP64 values, both sides in FP64):
  * counts and neighbour lists: bit-exact, provided the reference's closest
    call min |h - h_R| / h_R exceeds 1e-12 (then no pair is near enough to the
    support edge for the two FP64 evaluations to disagree);
  * W: within 1e-6 relative (the library sums the FP32-rounded weights);
  * maps, FP32 form: per channel, max |V - V_ref| / max |V_ref| <= 1e-6 over
    pixels with neighbours on the workloads' sky data; on zero-mean random
    fields the same bound against the weighted mean of |v| (see norm_err);
    NaN exactly where the reference has no neighbour.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import healpix_ref as hpr
from paper_2207_04584_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2207_04584_amd import api  # noqa: E402
from parity_util import abs_values, assert_fp32_bound, norm_err, to_host_values  # noqa: E402

ARC = 1.0 / 60.0
DEV = "cuda:0"
FP32_TOL = 1e-6


def check_field(ra, dec, vals, m, k, pix=None, chans=None, check_lists=True, tol=FP32_TOL,
                term_scale=True, w_rtol=1e-6, **opts):
    """Run setup + channels on the GPU and compare with the reference."""
    print(f"\n  field n={len(ra)} map={m['nx']}x{m['ny']} C={vals.shape[1]} opts={opts}", flush=True)
    plan = api.Plan(ra, dec, m, k, **opts)
    try:
        out = plan.grid(vals).cpu().numpy().reshape(vals.shape[1], -1)
        cnt = plan.counts()
        W = plan.weight_sums()
        lists = plan.neighbours() if check_lists else None
        st = plan.stats()
    finally:
        plan.close()
    hv, code = to_host_values(vals)
    Vr, cr, Wr, margin = oracle.grid(ra, dec, hv, code, m, k["fwhm_deg"], k["support_deg"],
                                     chans=chans, pix=pix)
    sel = np.arange(cnt.shape[0]) if pix is None else np.asarray(pix)
    ch = np.arange(vals.shape[1]) if chans is None else np.asarray(chans)
    assert margin > 1e-12, f"closest call {margin:g}: decisions not provably identical"
    np.testing.assert_array_equal(cnt[sel], cr)
    ok = cr > 0
    np.testing.assert_allclose(W[sel][ok], Wr[ok], rtol=w_rtol)
    assert np.all(W[sel][~ok] == 0)
    V = out[np.ix_(ch, sel)]
    np.testing.assert_array_equal(np.isnan(V), np.isnan(Vr))
    Vabs = None
    if term_scale:
        Vabs = oracle.grid(ra, dec, abs_values(hv, code), code, m, k["fwhm_deg"],
                           k["support_deg"], chans=chans, pix=pix)[0]
    e_max, e_rms = norm_err(V, Vr, ok, Vabs)
    print(f"  e_max={e_max:.3g} e_rms={e_rms:.3g} (plain normwise e_max="
          f"{norm_err(V, Vr, ok)[0]:.3g})", flush=True)
    assert e_max <= tol, f"e_max {e_max:g} > {tol:g}"
    if Vabs is not None and opts.get("precision", 0) == 0:
        assert_fp32_bound(V, Vr, Vabs, cr)
    if check_lists:
        rp, idx, w = lists
        orp, oidx, ow = oracle.neighbours(ra, dec, m, k["fwhm_deg"], k["support_deg"], pix=pix)
        for q, p in enumerate(sel):
            np.testing.assert_array_equal(idx[rp[p]:rp[p + 1]], oidx[orp[q]:orp[q + 1]])
            np.testing.assert_allclose(w[rp[p]:rp[p + 1]], ow[orp[q]:orp[q + 1]],
                                       rtol=max(2e-7, w_rtol))
    assert st["nnz"] == int(cnt.sum())
    return e_max, e_rms, st


def rand_field(seed, n, nx, ny, ra0, dec0, fwhm=3.0, C=5, spread=1.3, dtype=torch.float32):
    rng = np.random.default_rng(seed)
    cosd = max(math.cos(math.radians(dec0)), 0.05)
    ra = np.mod(ra0 + (rng.random(n) - 0.5) * nx * ARC * spread, 360.0)
    dec = dec0 + (rng.random(n) - 0.5) * ny * ARC * spread
    dec = np.clip(dec, -89.999, 89.999)
    vals = torch.from_numpy(rng.normal(size=(n, C)).astype(np.float32)).to(dtype).to(DEV)
    del cosd
    return ra, dec, vals, synth.make_map(ra0, dec0, nx, ny), synth.make_kernel(fwhm)


@pytest.mark.parametrize("nside", [1, 2, 64, 1024, 8192, 16384])
def test_ang2pix_matches_reference(nside):
    rng = np.random.default_rng(nside)
    z = np.concatenate([rng.uniform(-1, 1, 20000), rng.uniform(0.6, 0.7, 5000),
                        rng.uniform(-0.7, -0.6, 5000), rng.uniform(0.999, 1.0, 2000),
                        rng.uniform(-1.0, -0.999, 2000)])
    ra = rng.uniform(0, 360, z.shape[0])
    ra[:100] = rng.uniform(359.999, 360.0, 100)
    dec = np.rad2deg(np.arcsin(z))
    got = api.ang2pix_ring(nside, ra, dec).cpu().numpy()
    want = hpr.ang2pix_radec(nside, ra, dec)
    assert np.count_nonzero(got != want) == 0


CASES = {
    "basic": dict(seed=1, n=3000, nx=37, ny=29, ra0=33.0, dec0=-12.0, C=5),
    "wrap_ra0": dict(seed=2, n=3000, nx=40, ny=30, ra0=0.1, dec0=20.0, C=3),
    "wrap_ra360": dict(seed=3, n=2500, nx=31, ny=33, ra0=359.9, dec0=-35.0, C=3),
    "high_dec": dict(seed=4, n=3000, nx=30, ny=20, ra0=120.0, dec0=86.0, C=3),
    "cap_belt_edge": dict(seed=5, n=3000, nx=33, ny=35, ra0=250.0, dec0=41.81, C=3),
    "equator": dict(seed=6, n=2000, nx=17, ny=19, ra0=75.0, dec0=0.0, C=3),
    "south": dict(seed=7, n=2000, nx=18, ny=21, ra0=300.0, dec0=-62.0, C=3),
    "one_pixel": dict(seed=8, n=500, nx=1, ny=1, ra0=10.0, dec0=10.0, C=2, spread=8.0),
    "one_row": dict(seed=9, n=800, nx=41, ny=1, ra0=10.0, dec0=10.0, C=2, spread=1.5),
    "one_col": dict(seed=10, n=800, nx=1, ny=43, ra0=10.0, dec0=10.0, C=2, spread=1.5),
    "wide_kernel": dict(seed=11, n=6000, nx=20, ny=22, ra0=200.0, dec0=15.0, fwhm=10.0, C=4),
    "pole_support": dict(seed=12, n=4000, nx=24, ny=30, ra0=45.0, dec0=89.4, fwhm=30.0, C=2),
    "many_channels": dict(seed=13, n=1500, nx=19, ny=18, ra0=150.0, dec0=5.0, C=300),
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_small_field_parity(name):
    c = dict(CASES[name])
    ra, dec, vals, m, k = rand_field(**c)
    check_field(ra, dec, vals, m, k)


@pytest.mark.parametrize("form", ["fp32", "bf16"])
def test_dense_groups_on_dealt_tiles(form):
    """Pixel groups of over 4,096 entries on tiles still light enough to deal
    (about 22 samples a square arcminute, 50,000 in all, under a 6.3 arcmin
    beam): the bucketing then takes a workgroup a group, and the slot fill,
    marking and remapping split each list over several workgroups.  Lists,
    counts, W and maps against the reference on every pixel.  With about
    4,400 neighbours a pixel the FP32 form is held to its rounding bound cell
    by cell (check_field's assert_fp32_bound; its normwise figure only to
    1e-3), the BF16 form to 2e-3 and its weights to their rounding unit."""
    if form == "fp32":
        prec, dt, u, tol = api.HG_PREC_FP32, torch.float32, 1e-6, 1e-3
    else:
        prec, dt, u = MFMA[form]
        tol = MFMA_TOL
    ra, dec, vals, m, k = rand_field(31, 50000, 32, 32, 60.0, 10.0, fwhm=6.3, C=3, spread=1.5,
                                     dtype=dt)
    _, _, st = check_field(ra, dec, vals, m, k, tol=tol, w_rtol=u, precision=prec)
    # a group's entries are at least the largest of its four pixels' counts,
    # so the groups average at least nnz / npix entries (and more candidates)
    npix = m["nx"] * m["ny"]
    print(f"  neighbours per pixel {st['nnz'] / npix:.0f}, chunk {st['chunk']}", flush=True)
    assert st["nnz"] / npix > 4096


@pytest.mark.parametrize("nside,chunk", [(64, 8), (512, 32), (16384, 24), (4096, 16)])
def test_nside_and_chunk_overrides(nside, chunk):
    ra, dec, vals, m, k = rand_field(21, 2500, 26, 23, 95.0, -20.0, C=7)
    check_field(ra, dec, vals, m, k, nside=nside, chunk=chunk)


def test_duplicate_positions():
    ra, dec, vals, m, k = rand_field(22, 600, 15, 15, 60.0, 30.0, C=3)
    ra = np.repeat(ra[:150], 4)
    dec = np.repeat(dec[:150], 4)
    check_field(ra, dec, vals, m, k)


def test_empty_and_outside_fields():
    m = synth.make_map(30.0, 10.0, 9, 7)
    k = synth.make_kernel(3.0)
    vals = torch.zeros((0, 4), device=DEV)
    with api.Plan(np.zeros(0), np.zeros(0), m, k) as p:
        out = p.grid(vals).cpu().numpy()
        assert np.all(np.isnan(out)) and np.all(p.counts() == 0)
    ra = np.array([31.0, 29.0, 30.0])
    dec = np.array([10.0, 10.0, 11.0])
    v = torch.ones((3, 2), device=DEV)
    with api.Plan(ra, dec, m, k) as p:
        assert np.all(np.isnan(p.grid(v).cpu().numpy()))


def test_single_sample_profile_on_gpu():
    m = synth.make_map(210.0, 40.0, 21, 17)
    k = synth.make_kernel(3.0)
    ra, dec = np.array([210.0 + 2.3 * ARC]), np.array([40.0 - 1.7 * ARC])
    with api.Plan(ra, dec, m, k) as p:
        out = p.grid(torch.full((1, 1), 3.5, device=DEV)).cpu().numpy()[0].ravel()
        W = p.weight_sums()
    _, cr, Wr, _ = oracle.grid(ra, dec, np.ones((1, 1)), "f64", m, k["fwhm_deg"],
                               k["support_deg"])
    ok = cr > 0
    np.testing.assert_allclose(W[ok], Wr[ok], rtol=1e-7)
    np.testing.assert_allclose(out[ok], 3.5, rtol=2.5e-7)  # (w * 3.5) / w in FP32
    assert np.all(np.isnan(out[~ok]))


def test_cfg1_parity():
    f = synth.config("cfg1")
    vals = synth.sky_values(f, 1, device=DEV)
    e_max, e_rms, st = check_field(f["ra"], f["dec"], vals, f["map"], f["kernel"],
                                   term_scale=False)
    print(f"  cfg1 e_max={e_max:.3g} e_rms={e_rms:.3g} nnz={st['nnz']}")


def test_cfg3_geometry_bf16_values_fp32_form():
    f = synth.config("cfg3")
    vals = synth.sky_values(f, 8192, device=DEV, dtype="bf16")
    chans = np.random.default_rng(31).choice(8192, 48, replace=False)
    e_max, e_rms, _ = check_field(f["ra"], f["dec"], vals, f["map"], f["kernel"], chans=chans,
                                  check_lists=False, term_scale=False)
    print(f"  cfg3 (fp32 form) e_max={e_max:.3g} e_rms={e_rms:.3g}")


def test_f16_values():
    ra, dec, vals, m, k = rand_field(23, 2000, 20, 20, 10.0, -5.0, C=33, dtype=torch.float16)
    check_field(ra, dec, vals, m, k, check_lists=False)


def test_strided_and_unaligned_values_agree_bitwise():
    ra, dec, vals, m, k = rand_field(24, 2500, 24, 22, 80.0, 12.0, C=70)
    big = torch.zeros((vals.shape[0], 75), device=DEV)
    big[:, 1:71] = vals
    with api.Plan(ra, dec, m, k) as p:
        a = p.grid(vals)
        b = p.grid(big[:, 1:71])  # ld = 75, base misaligned by one float
        torch.cuda.synchronize()
        assert torch.equal(torch.nan_to_num(a, 7.0), torch.nan_to_num(b, 7.0))


def test_runs_are_deterministic():
    f = synth.config("cfg1")
    vals = synth.sky_values(f, 300, device=DEV)
    outs = []
    for _ in range(3):
        with api.Plan(f["ra"], f["dec"], f["map"], f["kernel"]) as p:
            outs.append(torch.nan_to_num(p.grid(vals), 7.0).cpu())
    assert torch.equal(outs[0], outs[1]) and torch.equal(outs[0], outs[2])


def test_launch_orders_per_channel_block_count_and_stream():
    """A plan keeps one launch order per channel-block count: calls that
    alternate between counts, and a call on a second stream (which waits for
    the order's upload), give the same maps as a fresh plan."""
    f = synth.config("cfg1")
    vals = synth.sky_values(f, 600, device=DEV)
    with api.Plan(f["ra"], f["dec"], f["map"], f["kernel"]) as p:
        ref600 = torch.nan_to_num(p.grid(vals), 7.0)
    with api.Plan(f["ra"], f["dec"], f["map"], f["kernel"]) as p:
        a = p.grid(vals[:, :5])  # one channel block
        b = p.grid(vals)  # three
        c = p.grid(vals[:, :300])  # two
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            d = p.grid(vals, stream=side)  # the three-block order again, on another stream
        torch.cuda.synchronize()
    assert torch.equal(torch.nan_to_num(b, 7.0), ref600)
    assert torch.equal(torch.nan_to_num(d, 7.0), ref600)
    assert torch.equal(torch.nan_to_num(a, 7.0), ref600[:5])
    assert torch.equal(torch.nan_to_num(c, 7.0), ref600[:300])


def test_cfg2_full_size_sampled_parity():
    """1e6 drift-scan samples, 300 x 300 map, 1024 FP32 channels: the bench
    workload and launch configuration; reference on sampled pixels."""
    f = synth.config("cfg2")
    vals = synth.sky_values(f, 1024, device=DEV)
    rng = np.random.default_rng(41)
    # 2000 random pixels, the corners and edges (ragged tiles: 300 = 18 x 16 + 12),
    # and a full row and column; counts and neighbour lists bit-exact on all of them
    edge = np.concatenate([np.arange(0, 300, 7), 299 * 300 + np.arange(0, 300, 7),
                           300 * np.arange(0, 300, 7), 300 * np.arange(0, 300, 7) + 299])
    pix = np.unique(np.concatenate([rng.choice(90000, 2000, replace=False), edge,
                                    [0, 299, 89700, 89999, 150 * 300 + 150]]))
    e_max, e_rms, st = check_field(f["ra"], f["dec"], vals, f["map"], f["kernel"], pix=pix,
                                   check_lists=True, term_scale=False, time_channels=True)
    print(f"  cfg2 e_max={e_max:.3g} e_rms={e_rms:.3g} nnz={st['nnz']} "
          f"channels_ms={st['last_channels_ms']:.3f} setup_ms={st['setup_ms']:.2f}")


def test_memory_cap_and_bad_coordinates():
    ra, dec, vals, m, k = rand_field(25, 1000, 12, 12, 10.0, 10.0, C=2)
    with pytest.raises(api.HegridError) as e:
        api.Plan(ra, dec, m, k, device_mem_cap=1024)
    assert e.value.status == api.HG_ERR_NOMEM
    dec2 = dec.copy()
    dec2[17] = np.nan
    with pytest.raises(api.HegridError) as e:
        api.Plan(ra, dec2, m, k)
    assert e.value.status == api.HG_ERR_ARG
    p = api.Plan(ra, dec, m, k)
    p.close()
    with pytest.raises(api.HegridError) as e:
        p.grid(vals)
    assert e.value.status == api.HG_ERR_STATE


# ---------------------------------------------------------------------------
# Precision forms: BF16 / FP16 weights x values on MFMA, FP32 accumulation, W from
# the same rounded weights.  Bound: <= 2e-3 relative.  The weights
# carry the format's rounding (2^-9 for BF16, 2^-12 for FP16 at most, relative).
MFMA = {"bf16": (1, torch.bfloat16, 2.0 ** -8), "f16": (2, torch.float16, 2.0 ** -11)}
MFMA_TOL = 2e-3


@pytest.mark.parametrize("form", sorted(MFMA))
@pytest.mark.parametrize("name", ["basic", "wrap_ra0", "pole_support", "many_channels",
                                  "one_row"])
def test_precision_form_parity(form, name):
    prec, dt, u = MFMA[form]
    c = dict(CASES[name])
    c["dtype"] = dt
    ra, dec, vals, m, k = rand_field(**c)
    e_max, e_rms, _ = check_field(ra, dec, vals, m, k, tol=MFMA_TOL, w_rtol=u, precision=prec)
    print(f"  {form} {name}: e_max={e_max:.3g} e_rms={e_rms:.3g}")


@pytest.mark.parametrize("form", sorted(MFMA))
@pytest.mark.parametrize("chunk", [72, 96, 112])
def test_long_chunks_in_16bit_forms(form, chunk):
    """The 16-bit forms stage up to 112 slots a chunk (512 B rows): past 64
    the bucketing marks two presence words per chunk and the metadata ring
    takes two index copies per chunk.  About 2,000 slots a tile, so tens of
    dealt chunks per tile with ragged last chunks, against the reference (a
    2 arcmin beam keeps the densest entry block within LDS at 112)."""
    prec, dt, u = MFMA[form]
    ra, dec, vals, m, k = rand_field(41, 2500, 26, 23, 95.0, -20.0, fwhm=2.0, C=300, dtype=dt)
    check_field(ra, dec, vals, m, k, tol=MFMA_TOL, w_rtol=u, precision=prec, chunk=chunk)


def _dense_tile_field():
    # 200,000 samples under one 12 x 12-pixel tile with a 1 arcmin beam: past
    # the dealing limit at chunks over 64 slots (two presence words a chunk,
    # 1024 words a wave)
    return rand_field(42, 200_000, 12, 12, 40.0, 10.0, fwhm=1.0, C=9, dtype=torch.bfloat16)


def test_long_chunk_refused_where_a_group_takes_most_of_it():
    """A tile too dense to deal at chunks past 64 slots keeps consecutive
    slots per chunk; those lie in one sky cell (or the sliver of a cell that
    reaches the map), so single pixel groups take runs of up to 72 entries,
    past what the channel kernel holds (one slot a lane).  An explicit chunk
    of 72 is refused with a message; the default chunk builds."""
    ra, dec, vals, m, k = _dense_tile_field()
    with pytest.raises(api.HegridError) as e:
        api.Plan(ra, dec, m, k, precision=1, chunk=72)
    assert e.value.status == api.HG_ERR_UNSUPPORTED
    assert "64 entries" in str(e.value)
    with api.Plan(ra, dec, m, k, precision=1) as p:
        assert p.stats()["chunk"] <= 64


def test_cfg3_bf16_mfma_form():
    """8192 BF16 channels on the cfg1 geometry; reference on sampled channels."""
    f = synth.config("cfg3")
    vals = synth.sky_values(f, 8192, device=DEV, dtype="bf16")
    chans = np.random.default_rng(32).choice(8192, 48, replace=False)
    e_max, e_rms, st = check_field(f["ra"], f["dec"], vals, f["map"], f["kernel"], chans=chans,
                                   check_lists=False, term_scale=False, tol=MFMA_TOL,
                                   w_rtol=2.0 ** -8, precision=1, time_channels=True)
    print(f"  cfg3 bf16-mfma e_max={e_max:.3g} e_rms={e_rms:.3g} "
          f"channels_ms={st['last_channels_ms']:.3f}")


def test_precision_form_dtype_rules_and_unaligned_values():
    ra, dec, vals, m, k = rand_field(26, 2500, 24, 22, 80.0, 12.0, C=70, dtype=torch.bfloat16)
    with api.Plan(ra, dec, m, k, precision=1) as p:
        with pytest.raises(api.HegridError) as e:
            p.grid(vals.float())
        assert e.value.status == api.HG_ERR_UNSUPPORTED
        big = torch.zeros((vals.shape[0], 75), device=DEV, dtype=torch.bfloat16)
        big[:, 1:71] = vals
        a = p.grid(vals)
        b = p.grid(big[:, 1:71])  # ld = 75, misaligned: staged through registers
        torch.cuda.synchronize()
        assert torch.equal(torch.nan_to_num(a, 7.0), torch.nan_to_num(b, 7.0))
