"""The autotuner (tune.py): it times every (chunk, waves, chan_block)
candidate, keeps the fastest, caches it under the workload's key and returns
the cached choice next time; a plan in the tuned shape grids identically to
the default shape at the same chunk (the shape does not change any cell's
arithmetic) and matches the reference."""
import numpy as np
import pytest

import oracle
from paper_2207_04584_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2207_04584_amd import api, tune  # noqa: E402
from parity_util import norm_err, to_host_values  # noqa: E402

DEV = "cuda:0"


@pytest.mark.parametrize("precision,dt,tol", [(api.HG_PREC_FP32, "f32", 1e-6),
                                              (api.HG_PREC_MFMA_BF16, "bf16", 2e-3)])
def test_tuned_plan_grids_like_the_default_and_the_reference(tmp_path, monkeypatch, precision,
                                                             dt, tol):
    monkeypatch.setenv("HEGRID_TUNE_CACHE", str(tmp_path / "tune.json"))
    f = synth.uniform_field((131,), 40000, 100.0, -10.0, 1.0, 0.8, 56, 44, nchan=300)
    vals = synth.sky_values(f, 300, device=DEV, dtype=dt)
    best = tune.tune_plan(f["ra"], f["dec"], f["map"], f["kernel"], vals, precision=precision,
                          reps=2)
    print(f"\n  best {best['chunk']} / {best['waves']} waves / {best['chan_block']} channels: "
          f"{best['ms']:.3f} ms of {len(best['table'])} candidates", flush=True)
    assert not best["cached"]
    assert len(best["table"]) >= len(tune.SHAPES)  # at least one chunk fully swept
    assert best["ms"] == min(best["table"].values())
    again = tune.tune_plan(f["ra"], f["dec"], f["map"], f["kernel"], vals, precision=precision)
    assert again["cached"] and again["key"] == best["key"]
    assert (again["chunk"], again["waves"], again["chan_block"]) == \
        (best["chunk"], best["waves"], best["chan_block"])
    plan, _ = tune.tuned_plan(f["ra"], f["dec"], f["map"], f["kernel"], vals, precision=precision)
    with plan:
        st = plan.stats()
        assert (st["chunk"], st["waves"], st["chan_block"]) == \
            (best["chunk"], best["waves"], best["chan_block"])
        got = plan.grid(vals)
    with api.Plan(f["ra"], f["dec"], f["map"], f["kernel"], precision=precision,
                  chunk=best["chunk"]) as p:
        ref = p.grid(vals)
    torch.cuda.synchronize()
    assert torch.equal(torch.nan_to_num(got, nan=1e30), torch.nan_to_num(ref, nan=1e30))
    chans = np.array([0, 151, 299])
    hv, code = to_host_values(vals[:, torch.from_numpy(chans).to(DEV)].contiguous())
    Vr, cr, _, margin = oracle.grid(f["ra"], f["dec"], hv, code, f["map"], f["kernel"]["fwhm_deg"],
                                    f["kernel"]["support_deg"])
    assert margin > 1e-12
    V = got.reshape(300, -1)[torch.from_numpy(chans).to(DEV)].cpu().numpy()
    np.testing.assert_array_equal(np.isnan(V), np.isnan(Vr))
    e_max, _ = norm_err(V, Vr, cr > 0)
    assert e_max <= tol


def test_tuned_batch_shape(tmp_path, monkeypatch):
    monkeypatch.setenv("HEGRID_TUNE_CACHE", str(tmp_path / "tune.json"))
    fs = synth.batch_fields(5, scale=0.05)
    fields = [{"ra": f["ra"], "dec": f["dec"], "map": f["map"], "kernel": f["kernel"],
               "values": synth.sky_values(f, f["nchan"], device=DEV, dtype="f16")} for f in fs]
    best = tune.tune_batch(fields, precision=api.HG_PREC_MFMA_F16, reps=1)
    assert not best["cached"] and len(best["table"]) == len(tune.SHAPES)
    assert tune.tune_batch(fields, precision=api.HG_PREC_MFMA_F16)["cached"]
    with api.Batch(fields, precision=api.HG_PREC_MFMA_F16, waves=best["waves"],
                   chan_block=best["chan_block"]) as b:
        outs = [o.clone() for o in b.run()]
    with api.Batch(fields, precision=api.HG_PREC_MFMA_F16) as b:
        refs = b.run()
        for o, r in zip(outs, refs):
            assert torch.equal(torch.nan_to_num(o, nan=1e30), torch.nan_to_num(r, nan=1e30))
