"""GPU test of hg_grid_channels_host_noalloc, the streamed channel phase
through the library's fixed per-device staging array (no allocation): its
cubes must equal hg_grid_channels_host's bit for bit on two calls in a row,
the second with a smaller input, in the FP32 and the BF16-MFMA forms; blocks
beyond the staging array and pageable buffers are refused before any work."""
import numpy as np
import pytest

from paper_2207_04584_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2207_04584_amd import api  # noqa: E402

ARC = 1.0 / 60.0


def field(n, nx, ny, C, seed, dtype=torch.float32):
    rng = np.random.default_rng(seed)
    ra = 120.0 + (rng.random(n) - 0.5) * nx * ARC * 1.2
    dec = -10.0 + (rng.random(n) - 0.5) * ny * ARC * 1.2
    vals = torch.from_numpy(rng.normal(1.0, 1.0, size=(n, C)).astype(np.float32)).to(dtype)
    return ra, dec, vals.pin_memory(), synth.make_map(120.0, -10.0, nx, ny), synth.make_kernel(3.0)


def same(a, b):
    return torch.equal(torch.nan_to_num(a, nan=1e30), torch.nan_to_num(b, nan=1e30))


@pytest.mark.parametrize("precision,dtype", [(api.HG_PREC_FP32, torch.float32),
                                             (api.HG_PREC_MFMA_BF16, torch.bfloat16)])
def test_noalloc_equals_streamed_path_on_two_calls(precision, dtype):
    cases = [(6000, 45, 38, 700, 11, 256), (2500, 30, 25, 150, 12, 0)]  # second call smaller
    for n, nx, ny, C, seed, block in cases:
        ra, dec, vals, m, k = field(n, nx, ny, C, seed, dtype)
        print(f"\n  n={n} map={nx}x{ny} C={C} block={block} precision={precision}", flush=True)
        with api.Plan(ra, dec, m, k, precision=precision) as p:
            ref = torch.empty((C, ny, nx), dtype=torch.float32, pin_memory=True)
            got = torch.full((C, ny, nx), -7.0, dtype=torch.float32, pin_memory=True)
            p.grid_host(vals, out=ref, block=block)
            _, info = p.grid_host_noalloc(vals, got, block=block)
        print(f"  {info}", flush=True)
        assert info["blocks"] == (-(-C // block) if block else 1) and info["pinned"] == 1
        assert same(got, ref), "the no-allocation path differs from hg_grid_channels_host"
        assert torch.isfinite(got).any()


def test_noalloc_refuses_oversized_blocks_and_pageable_buffers():
    rng = np.random.default_rng(13)
    n, nx, ny, C = 3000, 600, 600, 200
    ra = 120.0 + (rng.random(n) - 0.5) * 0.5
    dec = -10.0 + (rng.random(n) - 0.5) * 0.5
    m, k = synth.make_map(120.0, -10.0, nx, ny), synth.make_kernel(3.0)
    vals = torch.ones((n, C), dtype=torch.float32).pin_memory()
    out = torch.full((C, ny, nx), -7.0, dtype=torch.float32, pin_memory=True)
    with api.Plan(ra, dec, m, k) as p:
        # two map slots of 200 x 600 x 600 FP32 exceed the 256 MiB array
        with pytest.raises(api.HegridError) as ei:
            p.grid_host_noalloc(vals, out, block=200)
        assert ei.value.status == api.HG_ERR_ARG
        assert bool((out == -7.0).all()), "a refused call must not write the output"
        # pageable values
        with pytest.raises(api.HegridError) as ei:
            p.grid_host_noalloc(vals.clone(), out, block=8)
        assert ei.value.status == api.HG_ERR_ARG
        # block 0 picks a block that fits
        _, info = p.grid_host_noalloc(vals, out, block=0)
        assert info["blocks"] >= 2  # 200 channels of 600 x 600 maps do not fit one block
        got = out.clone()
        ref, _ = p.grid_host(vals, out=out, block=0)
        assert same(got, ref)
