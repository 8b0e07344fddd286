"""GPU tests of the paper-scale stand-in (the simulated set of Table 2 in
Sec. 5.1.2: 19-beam drift scans over 60 x 20 deg at (30, 41) deg, 3 arcmin
beam, 50 FP32 channels), run end to end from host memory as bench.py's
paper workload does: coordinates copied to the GPU, setup, channels streamed
in from page-locked (or pageable) host memory and the cube streamed back.

  * A 6 x 2 deg sub-field of the same recipe (2e5 samples, 360 x 120 map):
    counts on every pixel bit-exact, five channels within 1e-6 of the FP64
    reference on every pixel.
  * The full 1.9e7-sample field: counts and all 50 channels on pixels
    sampled over the map (corners, edges, interior) against the reference.
  * The overlapped form bench.py times (api.grid_from_host: the values'
    copy on a second stream behind the setup, then the device kernel) gives
    the streamed form's cube bit for bit, on the sub-field and at full size.
"""
import numpy as np
import pytest

import oracle
from paper_2207_04584_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2207_04584_amd import api  # noqa: E402
from parity_util import norm_err  # noqa: E402

DEV = "cuda:0"
FP32_TOL = 1e-6


def run_end_to_end(f, pinned):
    n, C = f["ra"].shape[0], f["nchan"]
    vals = synth.sky_values(f, C, device=DEV).cpu()
    if pinned:
        vals = vals.pin_memory()
    ra = torch.from_numpy(f["ra"]).to(DEV)
    dec = torch.from_numpy(f["dec"]).to(DEV)
    with api.Plan(ra, dec, f["map"], f["kernel"]) as p:
        out, info = p.grid_host(vals)
        cnt = p.counts()
        st = p.stats()
    print(f"\n  n={n} C={C} map={f['map']['nx']}x{f['map']['ny']} pinned={pinned} "
          f"nnz={st['nnz']} chunk={st['chunk']} {info}", flush=True)
    assert info["pinned"] == int(pinned) and info["blocks"] == 1
    return vals, out, cnt


@pytest.mark.parametrize("pinned", [False, True])
def test_paper_subfield_against_reference(pinned):
    f = synth.paper_field(n=200_000, width=6.0, height=2.0)
    assert f["map"]["nx"] == 360 and f["map"]["ny"] == 120
    vals, out, cnt = run_end_to_end(f, pinned)
    chans = np.array([0, 7, 24, 41, 49])
    Vr, cr, _, margin = oracle.grid(f["ra"], f["dec"], vals.numpy(), "f32", f["map"],
                                    f["kernel"]["fwhm_deg"], f["kernel"]["support_deg"],
                                    chans=chans)
    assert margin > 1e-12
    np.testing.assert_array_equal(cnt, cr)
    V = out.numpy().reshape(f["nchan"], -1)[chans]
    np.testing.assert_array_equal(np.isnan(V), np.isnan(Vr))
    e_max, e_rms = norm_err(V, Vr, cr > 0)
    print(f"  e_max={e_max:.3g} e_rms={e_rms:.3g}", flush=True)
    assert e_max <= FP32_TOL


def overlapped_equals(f, vals, out):
    ra = torch.from_numpy(f["ra"]).pin_memory()
    dec = torch.from_numpy(f["dec"]).pin_memory()
    out2, info = api.grid_from_host(ra, dec, f["map"], f["kernel"], vals)
    print(f"  overlapped: {info}", flush=True)
    assert torch.equal(torch.isnan(out2), torch.isnan(out))
    assert torch.equal(torch.nan_to_num(out2), torch.nan_to_num(out))


def test_paper_subfield_overlapped_form():
    f = synth.paper_field(n=200_000, width=6.0, height=2.0)
    vals, out, _ = run_end_to_end(f, pinned=True)
    overlapped_equals(f, vals, out)


def test_paper_full_size_sampled_pixels():
    f = synth.paper_field()
    assert f["ra"].shape[0] == 19_000_000
    nx, ny = f["map"]["nx"], f["map"]["ny"]
    vals, out, cnt = run_end_to_end(f, pinned=True)
    overlapped_equals(f, vals, out)
    rng = np.random.default_rng(6)
    xs = np.concatenate([[0, nx - 1, 0, nx - 1, nx // 2, 0, nx - 1], rng.integers(0, nx, 33)])
    ys = np.concatenate([[0, 0, ny - 1, ny - 1, ny // 2, ny // 2, ny // 2], rng.integers(0, ny, 33)])
    pix = np.unique(ys * nx + xs)
    Vr, cr, _, margin = oracle.grid(f["ra"], f["dec"], vals.numpy(), "f32", f["map"],
                                    f["kernel"]["fwhm_deg"], f["kernel"]["support_deg"], pix=pix)
    assert margin > 1e-12
    np.testing.assert_array_equal(cnt[pix], cr)
    assert cr.min() > 0  # the drift scans cover the whole map
    V = out.numpy().reshape(f["nchan"], -1)[:, pix]
    e_max, e_rms = norm_err(V, Vr, cr > 0)
    print(f"  {pix.shape[0]} pixels: counts {cr.min()}..{cr.max()}, e_max={e_max:.3g} "
          f"e_rms={e_rms:.3g}", flush=True)
    assert e_max <= FP32_TOL
