"""GPU tests of the channel phase by bands of tile rows (hg_grid_channels_rows,
hg_plan_row_needs) and of the banded end-to-end path (api.grid_from_host with
bands > 0).

A band runs the same per-tile work as the whole-map launch, so bands that
cover the map give its cube bit for bit and leave other rows alone.  A band's
need is a bound, checked against the neighbour lists the plan exports (every
neighbour of a band's pixels has a smaller index than the band's need; those
lists are themselves checked against the FP64 reference in test_gpu_parity).
"""
import numpy as np
import pytest

from paper_2207_04584_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2207_04584_amd import api  # noqa: E402

DEV = "cuda:0"
ARC = 1.0 / 60.0


def field(n=7000, nx=41, ny=53, C=40, seed=5, dtype=torch.float32, sort_dec=False):
    rng = np.random.default_rng(seed)
    ra = 150.0 + (rng.random(n) - 0.5) * nx * ARC * 1.2
    dec = 20.0 + (rng.random(n) - 0.5) * ny * ARC * 1.2
    if sort_dec:  # samples in scan order: declination grows with the index
        o = np.argsort(dec, kind="stable")
        ra, dec = ra[o], dec[o]
    vals = torch.from_numpy(rng.normal(1.0, 1.0, size=(n, C)).astype(np.float32)).to(dtype)
    return ra, dec, vals, synth.make_map(150.0, 20.0, nx, ny), synth.make_kernel(3.0)


def same(a, b):
    return torch.equal(torch.nan_to_num(a, nan=1e30), torch.nan_to_num(b, nan=1e30))


FORMS = {"fp32": (api.HG_PREC_FP32, torch.float32), "bf16": (api.HG_PREC_MFMA_BF16, torch.bfloat16)}


@pytest.mark.parametrize("form", sorted(FORMS))
def test_row_bands_cover_the_map_bitwise(form):
    prec, dt = FORMS[form]
    ra, dec, vals, m, k = field(dtype=dt)
    vals = vals.to(DEV)
    with api.Plan(ra, dec, m, k, precision=prec) as p:
        rows = p.tile_rows
        assert rows == 4  # 53 pixel rows: a ragged last tile row
        ref = p.grid(vals)
        got = torch.full_like(ref, 1234.5)
        for r0, r1 in [(0, 1), (1, 3), (3, 4), (2, 2)]:
            p.grid_rows(vals, got, r0, r1)
        torch.cuda.synchronize()
        assert same(got, ref)
        # one band writes its rows only
        part = torch.full_like(ref, 1234.5)
        p.grid_rows(vals, part, 1, 2)
        torch.cuda.synchronize()
        assert same(part[:, 16:32], ref[:, 16:32])
        assert torch.all(part[:, :16] == 1234.5) and torch.all(part[:, 32:] == 1234.5)


def test_row_needs_bound_every_neighbour():
    ra, dec, vals, m, k = field(sort_dec=True)
    with api.Plan(ra, dec, m, k) as p:
        need = p.row_needs(1)
        row_ptr, idx, _ = p.neighbours()
        ny, nx = p.shape
        assert need.shape == (p.tile_rows,)
        assert np.all(need <= len(ra)) and np.all(need >= 0)
        for b in range(p.tile_rows):
            y0, y1 = 16 * b, min(16 * b + 16, ny)
            lo, hi = row_ptr[y0 * nx], row_ptr[y1 * nx]
            if hi > lo:
                assert idx[lo:hi].max() < need[b], f"band {b}"
        # samples in scan order: bands further along the scan need later
        # samples, and the first band far fewer than all of them
        d = np.diff(need)
        assert np.all(d >= 0) or np.all(d <= 0)
        assert min(need[0], need[-1]) < 0.6 * len(ra)
        # two rows a band: the larger of the pair's needs
        need2 = p.row_needs(2)
        assert need2.shape == (2,)
        assert need2[0] == max(need[0], need[1]) and need2[1] == max(need[2], need[3])


def test_row_arguments_are_checked():
    ra, dec, vals, m, k = field(n=800, C=3)
    vals = vals.to(DEV)
    with api.Plan(ra, dec, m, k) as p:
        out = torch.empty((3,) + p.shape, device=DEV)
        for r0, r1 in [(-1, 2), (2, 1), (0, 5)]:
            with pytest.raises(api.HegridError) as e:
                p.grid_rows(vals, out, r0, r1)
            assert e.value.status == api.HG_ERR_ARG
        need = np.zeros(8, dtype=np.int64)
        buf = need.ctypes.data_as(api.ctypes.c_void_p)
        L = api.lib()
        assert L.hg_plan_row_needs(p._handle(), 0, buf, 8, None) == api.HG_ERR_ARG
        assert L.hg_plan_row_needs(p._handle(), 1, buf, 2, None) == api.HG_ERR_ARG  # 4 bands
        assert L.hg_plan_row_needs(p._handle(), 1, None, 4, None) == api.HG_ERR_ARG
        assert L.hg_plan_row_needs(p._handle(), 1, buf, 4, None) == api.HG_OK


@pytest.mark.parametrize("sort_dec", [True, False])
@pytest.mark.parametrize("bands,pieces,C", [(3, 5, 33), (4, 1, 33), (9, 16, 33), (3, 5, 600)])
def test_banded_from_host_equals_unbanded(sort_dec, bands, pieces, C):
    """The banded path (values in pieces, bands gated on the pieces they
    need, rows back while later bands run: channel by channel, or in one 2-D
    copy past 512 channels) against the plain call, bit for bit; samples in
    scan order and in random order (then every band waits for nearly every
    piece)."""
    ra, dec, vals, m, k = field(n=9000, C=C, sort_dec=sort_dec)
    host = vals.pin_memory()
    ref, _ = api.grid_from_host(ra, dec, m, k, host)
    ref = ref.clone()
    got, info = api.grid_from_host(ra, dec, m, k, host, bands=bands, pieces=pieces)
    per = -(-4 // bands)  # tile rows a band (the map has 4)
    assert info["bands"] == -(-4 // per)
    assert torch.equal(torch.isnan(got), torch.isnan(ref))
    assert torch.equal(torch.nan_to_num(got), torch.nan_to_num(ref))
    assert info["kernel_ms"] > 0 and info["d2h_ms"] >= 0
