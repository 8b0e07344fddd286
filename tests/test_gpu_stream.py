"""GPU tests of the host-streamed channel phase (hg_grid_channels_host).

The streamed call runs the channel kernel of hg_grid_channels on blocks of
channels copied in from host memory, so its cube must equal the device-path
cube bit for bit, for pageable and page-locked buffers, ragged last blocks,
strided rows and the 16-bit MFMA form; on the large-cube geometry (19-beam
drift scan, BF16 channels) scaled down, sampled channels of every block are
also checked against the FP64 reference.
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
from parity_util import norm_err, to_host_values  # noqa: E402

DEV = "cuda:0"
ARC = 1.0 / 60.0


def field(n=6000, nx=45, ny=38, C=700, seed=3, dtype=torch.float32, ld=None):
    rng = np.random.default_rng(seed)
    ra = 120.0 + (rng.random(n) - 0.5) * nx * ARC * 1.2
    dec = -10.0 + (rng.random(n) - 0.5) * ny * ARC * 1.2
    ld = C if ld is None else ld
    full = torch.from_numpy(rng.normal(1.0, 1.0, size=(n, ld)).astype(np.float32)).to(dtype)
    return ra, dec, full[:, :C], synth.make_map(120.0, -10.0, nx, ny), synth.make_kernel(3.0)


@pytest.mark.parametrize("pinned", [False, True])
@pytest.mark.parametrize("block", [256, 300, 0])
def test_streamed_equals_device_path(pinned, block):
    ra, dec, vals, m, k = field()
    if pinned:
        vals = vals.contiguous().pin_memory()
    out = torch.empty((vals.shape[1], m["ny"], m["nx"]), dtype=torch.float32,
                      pin_memory=pinned)
    with api.Plan(ra, dec, m, k) as p:
        got, info = p.grid_host(vals, out=out, block=block)
        ref = p.grid(vals.to(DEV)).cpu()
    nb = -(-vals.shape[1] // (block or 4096))
    print(f"\n  pinned={pinned} block={block}: {info}", flush=True)
    assert info["blocks"] == nb and info["pinned"] == int(pinned)
    assert info["h2d_bytes"] == vals.numel() * 4 and info["d2h_bytes"] == out.numel() * 4
    assert info["kernel_ms"] > 0
    assert torch.equal(torch.nan_to_num(got, nan=1e30), torch.nan_to_num(ref, nan=1e30))


def test_streamed_strided_rows_and_repeat_calls():
    ra, dec, vals, m, k = field(C=333, ld=520)  # rows of 520 channels, 333 used
    assert vals.stride(0) == 520
    with api.Plan(ra, dec, m, k) as p:
        ref = p.grid(vals.contiguous().to(DEV)).cpu()
        for block in (128, 100):  # the ring grows or is reused between calls
            got, info = p.grid_host(vals, block=block)
            assert info["pinned"] == 0  # the view of pageable rows is staged
            assert torch.equal(torch.nan_to_num(got, nan=1e30), torch.nan_to_num(ref, nan=1e30))


@pytest.mark.parametrize("dtype,prec", [(torch.bfloat16, api.HG_PREC_MFMA_BF16),
                                        (torch.float16, api.HG_PREC_MFMA_F16),
                                        (torch.bfloat16, api.HG_PREC_FP32)])
def test_streamed_16bit_forms(dtype, prec):
    ra, dec, vals, m, k = field(C=520, dtype=dtype)
    with api.Plan(ra, dec, m, k, precision=prec) as p:
        got, _ = p.grid_host(vals, block=256)
        ref = p.grid(vals.to(DEV)).cpu()
    assert torch.equal(torch.nan_to_num(got, nan=1e30), torch.nan_to_num(ref, nan=1e30))


def test_streamed_empty_field_and_no_channels():
    m, k = synth.make_map(10.0, 0.0, 20, 20), synth.make_kernel(3.0)
    with api.Plan(np.zeros(0), np.zeros(0), m, k) as p:
        out, info = p.grid_host(torch.zeros((0, 9)), block=4)
        assert info["blocks"] == 3 and torch.isnan(out).all()
    ra, dec, vals, m, k = field(C=1)
    with api.Plan(ra, dec, m, k) as p:
        out, info = p.grid_host(vals[:, :0])
        assert info["blocks"] == 0 and out.numel() == 0


def test_streamed_ring_respects_memory_cap():
    # the ring for 2000-channel blocks (two slots of 6000 x 2000 values and
    # 2000 maps, about 120 MB) cannot fit a cap of three times the plan (setup
    # itself needs some transient room beyond the plan)
    ra, dec, vals, m, k = field(C=2000)
    with api.Plan(ra, dec, m, k) as p:
        plan_bytes = p.stats()["device_bytes"]
    assert 3 * plan_bytes < 100e6
    with api.Plan(ra, dec, m, k, device_mem_cap=3 * plan_bytes) as p:
        with pytest.raises(api.HegridError) as ei:
            p.grid_host(vals, block=2000)
        assert ei.value.status == api.HG_ERR_NOMEM
        out, info = p.grid_host(vals[:, :8], block=8)  # a small ring still fits
        assert info["blocks"] == 1


def test_streamed_cube_against_reference():
    """Large-cube geometry (19 interleaved drift-scan beams, BF16 values,
    continuum + line sources), scaled to 40,000 samples on a 60 x 60 map and
    4 blocks of 512 channels; 4 channels of every block checked."""
    f = synth.config("cfg5")
    keep = np.random.default_rng(5).choice(f["ra"].shape[0], 40000, replace=False)
    keep.sort()
    ra, dec = f["ra"][keep], f["dec"][keep]
    sub = dict(f, ra=ra, dec=dec, map=synth.make_map(180.0, 30.0, 60, 60))
    C, block = 2048, 512
    vals = synth.sky_values(sub, C, device=DEV, dtype="bf16").cpu()
    with api.Plan(ra, dec, sub["map"], f["kernel"], precision=api.HG_PREC_MFMA_BF16) as p:
        out, info = p.grid_host(vals, block=block)
        cnt = p.counts()
    print(f"\n  cube: {info}", flush=True)
    chans = np.array([b * block + o for b in range(C // block) for o in (0, 77, 300, 511)])
    hv, code = to_host_values(vals)
    Vr, cr, _, margin = oracle.grid(ra, dec, hv, code, sub["map"], f["kernel"]["fwhm_deg"],
                                    f["kernel"]["support_deg"], chans=chans)
    assert margin > 1e-12
    np.testing.assert_array_equal(cnt, cr)
    V = out.numpy().reshape(C, -1)[chans]
    np.testing.assert_array_equal(np.isnan(V), np.isnan(Vr))
    e_max, e_rms = norm_err(V, Vr, cr > 0)
    print(f"  e_max={e_max:.3g} e_rms={e_rms:.3g}", flush=True)
    assert e_max <= 2e-3


def cube_slab(f, C, lo, hi, dev_slab, block=4096):
    """Channels [lo, hi) of the cube as one contiguous BF16 [n][hi - lo]
    device array, generated block by block (each block's FP32 intermediate
    is 16 GB at 1e6 samples)."""
    for b0 in range(lo, hi, block):
        b1 = min(hi, b0 + block)
        v = synth.sky_values(f, C, device=DEV, dtype="bf16", chan_lo=b0, chan_hi=b1)
        dev_slab[:, b0 - lo:b1 - lo].copy_(v)
        del v
    return dev_slab


def test_cfg5_full_size_streamed():
    """The large-cube workload at its real size: 1e6 samples of 19 interleaved
    drift-scan beams, a 600 x 600 map, 65,536 BF16 channels streamed from
    page-locked host memory in 16 blocks of 4096, the copies in and out
    overlapped with the kernel (hg_grid_channels_host, BF16 MFMA form).  The
    host cannot hold the whole cube (131 GB of values and 94 GB of maps), so
    it goes through in slabs of several blocks, each one call.  Reference:
    16 channels of blocks 0, 7 and 15 on 400 sampled pixels and the corners."""
    import psutil
    avail = psutil.virtual_memory().available
    # page-locked slabs of 8192 channels: 16.4 GB of values and 11.8 GB of maps
    if avail < 60e9:
        pytest.skip(f"needs about 60 GB of free host memory, {avail / 1e9:.0f} GB available")
    f = synth.config("cfg5")
    C, block = 65536, 4096
    slab = 8192
    n = f["ra"].shape[0]
    m = f["map"]
    P = m["nx"] * m["ny"]
    print(f"\n  {n} samples, {C} channels, slabs of {slab} ({avail / 1e9:.0f} GB host free)",
          flush=True)
    rng = np.random.default_rng(55)
    offs = np.sort(rng.choice(block, 16, replace=False))
    check = {b: b * block + offs for b in (0, 7, 15)}
    pix = np.unique(np.concatenate([rng.choice(P, 400, replace=False),
                                    [0, m["nx"] - 1, P - m["nx"], P - 1]]))
    vals_h = synth.pinned_empty((n, slab), torch.bfloat16)
    out_h = synth.pinned_empty((slab, m["ny"], m["nx"]), torch.float32)
    dev_slab = torch.empty((n, slab), dtype=torch.bfloat16, device=DEV)
    got, ref_vals, infos = {}, {}, []
    with api.Plan(f["ra"], f["dec"], m, f["kernel"], precision=api.HG_PREC_MFMA_BF16) as p:
        cnt = p.counts()
        for s0 in range(0, C, slab):
            cube_slab(f, C, s0, s0 + slab, dev_slab)
            vals_h.copy_(dev_slab)
            torch.cuda.synchronize()
            _, info = p.grid_host(vals_h, out=out_h, block=block)
            infos.append(info)
            print(f"  slab {s0 // slab}: {info['blocks']} blocks, wall {info['wall_ms']:.0f} ms, "
                  f"h2d {info['h2d_ms']:.0f} ms, kernels {info['kernel_ms']:.0f} ms, "
                  f"d2h {info['d2h_ms']:.0f} ms", flush=True)
            assert info["pinned"] == 1 and info["blocks"] == slab // block
            for b, ch in check.items():
                if s0 <= ch[0] < s0 + slab:
                    loc = torch.from_numpy(ch - s0)
                    got[b] = out_h.reshape(slab, -1)[loc][:, pix].numpy().copy()
                    ref_vals[b] = to_host_values(vals_h[:, loc].contiguous())
    del vals_h, out_h, dev_slab
    torch.cuda.synchronize()
    assert sum(i["blocks"] for i in infos) == C // block
    worst = 0.0
    for b, ch in check.items():
        hv, code = ref_vals[b]
        Vr, cr, _, margin = oracle.grid(f["ra"], f["dec"], hv, code, m, f["kernel"]["fwhm_deg"],
                                        f["kernel"]["support_deg"], pix=pix)
        assert margin > 1e-12
        np.testing.assert_array_equal(cnt[pix], cr)
        np.testing.assert_array_equal(np.isnan(got[b]), np.isnan(Vr))
        e_max, e_rms = norm_err(got[b], Vr, cr > 0)
        worst = max(worst, e_max)
        print(f"  block {b}: e_max={e_max:.3g} e_rms={e_rms:.3g}", flush=True)
        assert e_max <= 2e-3
    print(f"  worst e_max {worst:.3g}", flush=True)
