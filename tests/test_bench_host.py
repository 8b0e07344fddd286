"""Host logic of bench.py without a GPU: the CPU-baseline leg's parity report
(the timed path's error on the sampled pixels against the reference gridder)
is zero-ish for the reference's own map rounded to FP32, finds a planted
error, and flags a cell whose emptiness disagrees; --gpus above 1 is refused."""
import os
import subprocess
import sys

import numpy as np

import oracle
from paper_2207_04584_amd import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def small_field():
    f = synth.config("cfg1")
    vals = np.random.default_rng(0).normal(5.0, 1.0, size=(f["ra"].shape[0], 3))
    vals = vals.astype(np.float32)
    V, _, _, _ = oracle.grid(f["ra"], f["dec"], vals, "f32", f["map"], f["kernel"]["fwhm_deg"],
                             f["kernel"]["support_deg"])
    return f, vals, V.astype(np.float32)


def test_parity_report_of_the_reference_itself():
    f, vals, gpu = small_field()
    par = bench.cpu_baseline(f, vals, 300, gpu_out=gpu)["parity"]
    assert par["e_max"] < 1e-7 and par["e_rms"] < 1e-7 and par["nan_match"]
    assert par["pixels"] > 0


def test_parity_report_finds_planted_errors():
    f, vals, gpu = small_field()
    P = gpu.shape[1]
    bad = gpu.copy()
    bad[2, :] *= 1.0 + 3e-6  # every sampled pixel of channel 2
    par = bench.cpu_baseline(f, vals, P, gpu_out=bad)["parity"]
    assert 2e-6 < par["e_max"] < 4e-6
    hole = gpu.copy()
    filled = np.nonzero(~np.isnan(gpu[0]))[0][0]
    hole[:, filled] = np.nan
    assert not bench.cpu_baseline(f, vals, P, gpu_out=hole)["parity"]["nan_match"]


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True)
    assert r.returncode != 0 and "one GPU" in r.stderr
