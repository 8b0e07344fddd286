"""Helpers shared by the GPU parity tests (host-side comparison only)."""
import numpy as np


def to_host_values(v):
    """Stored values as the reference reads them: (array, dtype code)."""
    import torch
    if v.dtype == torch.float32:
        return v.cpu().numpy(), "f32"
    if v.dtype == torch.bfloat16:
        return v.cpu().view(torch.int16).numpy().view(np.uint16), "bf16"
    return v.cpu().view(torch.int16).numpy().view(np.uint16), "f16"


def norm_err(V, Vr, ok, Vabs=None):
    """Per channel: max |V - V_ref| / max |S| and rms |V - V_ref| / rms |S| over
    pixels with neighbours, worst channel.  S is V_ref itself (the plain
    normwise error) or, when given, the weighted mean of |v|: FP32 summation
    of K terms errs by up to ~K u sum|w v|, so on zero-mean data, where the
    map is much smaller than its terms, the error is measured against the size
    of the terms."""
    if not ok.any():
        return 0.0, 0.0
    S = np.abs(Vr if Vabs is None else Vabs)[:, ok]
    d = np.abs(V[:, ok] - Vr[:, ok])
    scale = S.max(1)
    scale[scale == 0] = 1.0
    e_max = (d.max(1) / scale).max()
    e_rms = (np.sqrt((d ** 2).mean(1)) / np.maximum(np.sqrt((S ** 2).mean(1)), 1e-300)).max()
    return float(e_max), float(e_rms)


def abs_values(hv, code):
    if code == "f32":
        return np.abs(hv)
    return hv & np.uint16(0x7FFF)  # clear the sign bit of bf16 / f16


U32 = 2.0 ** -24


def assert_fp32_bound(V, Vr, Vabs, cnt):
    """The FP32 form's rounding bound, cell by cell, whatever the summation
    order.  With FP32 weights w' = w (1 + e), |e| <= u, the exact weighted
    mean with w' is within u (A + |V_ref|) of V_ref, A = sum w |v| / W; any
    order of K FP32 multiply-adds errs by at most gamma_K sum |w' v|; the
    division by the FP32-rounded W adds 2u |V|.  So
        |V - V_ref| <= (gamma_K + 2u) A + 3u |V_ref|,  gamma_K = K u / (1 - K u).
    On zero-mean random values A can be far larger than max |V_ref|, which is
    why these fields are not held to 1e-6 of max |V_ref| itself."""
    ok = cnt > 0
    K = cnt[ok].astype(np.float64)
    gam = K * U32 / (1 - K * U32)
    bound = (gam + 2 * U32) * np.abs(Vabs[:, ok]) + 3 * U32 * np.abs(Vr[:, ok])
    err = np.abs(V[:, ok] - Vr[:, ok])
    worst = float((err / np.maximum(bound, 1e-300)).max()) if err.size else 0.0
    print(f"  worst error / FP32 rounding bound = {worst:.3g}", flush=True)
    assert np.all(err <= bound * (1 + 1e-9)), f"error exceeds the FP32 bound by {worst:g}x"
