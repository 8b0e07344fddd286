"""GPU tests of the FIFO multi-stream pipeline (pipeline.grid_fields_fifo):
fields set up and gridded one at a time by host threads with a stream each.
It runs the library's own per-field kernels, so its maps must equal the
batched form's and the single-plan maps bit for bit (NaN included), for
several stream counts and both forms; and a failing field is reported by
index after the other workers stop.
"""
import numpy as np
import pytest

from paper_2207_04584_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2207_04584_amd import api, pipeline  # noqa: E402

DEV = "cuda:0"
ARC = 1.0 / 60.0


def fields(dtype=torch.float32, count=9):
    out = []
    for i in range(count):
        rng = np.random.default_rng(500 + i)
        n = int(rng.integers(0, 4000)) if i != 3 else 0
        nx, ny = int(rng.integers(3, 60)), int(rng.integers(3, 60))
        ra0, dec0 = float(rng.uniform(0, 360)), float(rng.uniform(-60, 60))
        C = int(rng.choice([0, 1, 7, 256, 300])) if i != 2 else 0
        ra = np.mod(ra0 + (rng.random(n) - 0.5) * nx * ARC * 1.3, 360.0)
        dec = dec0 + (rng.random(n) - 0.5) * ny * ARC * 1.3
        vals = None
        if C:
            vals = torch.from_numpy(rng.normal(1.0, 1.0, (n, C)).astype(np.float32))
            vals = vals.to(dtype).to(DEV)
        out.append({"ra": ra, "dec": dec, "map": synth.make_map(ra0, dec0, nx, ny),
                    "kernel": synth.make_kernel(float(rng.uniform(2, 5))), "values": vals})
    return out


def same(a, b):
    return torch.equal(torch.nan_to_num(a, nan=1e30), torch.nan_to_num(b, nan=1e30))


@pytest.mark.parametrize("streams,chunk", [(1, 0), (3, 0), (8, 0), (3, 48)])
def test_fifo_equals_batch_bitwise(streams, chunk):
    """The FIFO's plans take their chunk lengths as a batch's fields do
    (predicted from the support, or the one given)."""
    fs = fields()
    got = pipeline.grid_fields_fifo(fs, n_streams=streams, chunk=chunk)
    with api.Batch(fs, chunk=chunk) as b:
        ref = [o.clone() if o is not None else None for o in b.run()]
    for i, (g, r) in enumerate(zip(got, ref)):
        assert (g is None) == (r is None), i
        if g is not None:
            assert same(g, r), f"field {i}"


def test_fifo_f16_mfma_equals_single_plans():
    fs = fields(dtype=torch.float16, count=5)
    got = pipeline.grid_fields_fifo(fs, n_streams=2, precision=api.HG_PREC_MFMA_F16)
    for i, f in enumerate(fs):
        if f["values"] is None:
            assert got[i] is None
            continue
        with api.Plan(f["ra"], f["dec"], f["map"], f["kernel"],
                      precision=api.HG_PREC_MFMA_F16, predict_chunk=True) as p:
            assert same(got[i], p.grid(f["values"])), f"field {i}"


def test_fifo_reports_failing_field():
    fs = fields(count=4)
    fs[2] = dict(fs[2], map=dict(fs[2]["map"], nx=0))  # rejected by setup
    with pytest.raises(api.HegridError) as ei:
        pipeline.grid_fields_fifo(fs, n_streams=2)
    assert "field 2" in str(ei.value) and ei.value.status == api.HG_ERR_ARG
