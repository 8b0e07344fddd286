"""Argument checks of the C boundary that need a device: buffers the kernels
read or write must be device memory of the plan's device.  Host buffers are
refused with HG_ERR_ARG before anything is enqueued.  Only page-locked host
memory is passed here, so even a check that let it through would have the
kernel write over the host link rather than fault."""
import ctypes

import numpy as np
import pytest

from paper_2207_04584_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2207_04584_amd import api  # noqa: E402

DEV = "cuda:0"


def _plan():
    f = synth.uniform_field((77,), 600, 40.0, 10.0, 0.2, 0.2, 8, 8, nchan=4)
    return f, api.Plan(f["ra"], f["dec"], f["map"], f["kernel"])


def test_channels_refuse_host_buffers():
    f, plan = _plan()
    L = api.lib()
    vals = synth.sky_values(f, 4, device=DEV)
    out_dev = torch.empty((4, 8, 8), dtype=torch.float32, device=DEV)
    out_pin = torch.empty((4, 8, 8), dtype=torch.float32, pin_memory=True)
    vals_pin = vals.cpu().pin_memory()
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    try:
        rc = L.hg_grid_channels(plan._handle(), ctypes.c_void_p(vals.data_ptr()), 4, 4, api.HG_F32,
                                ctypes.c_void_p(out_pin.data_ptr()), s)
        assert rc == api.HG_ERR_ARG and "out" in api.last_error()
        rc = L.hg_grid_channels(plan._handle(), ctypes.c_void_p(vals_pin.data_ptr()), 4, 4,
                                api.HG_F32, ctypes.c_void_p(out_dev.data_ptr()), s)
        assert rc == api.HG_ERR_ARG and "values" in api.last_error()
        # the binding refuses a host output before the library is called
        with pytest.raises(api.HegridError) as e:
            plan.grid(vals, out=torch.empty((4, 8, 8), dtype=torch.float32))
        assert e.value.status == api.HG_ERR_ARG
        # and the plan still grids device buffers afterwards
        assert torch.isfinite(plan.grid(vals, out=out_dev)).any()
    finally:
        plan.close()
    torch.cuda.synchronize()


def test_setup_refuses_host_coordinates():
    f = synth.uniform_field((78,), 300, 40.0, 10.0, 0.2, 0.2, 8, 8, nchan=1)
    L = api.lib()
    ra = torch.from_numpy(np.ascontiguousarray(f["ra"])).pin_memory()
    dec = torch.from_numpy(np.ascontiguousarray(f["dec"])).pin_memory()
    k, m, o = api.make_kernel(f["kernel"]), api.make_map(f["map"]), api.hg_opts()
    h = ctypes.c_void_p()
    rc = L.hg_grid_setup(ctypes.c_void_p(ra.data_ptr()), ctypes.c_void_p(dec.data_ptr()),
                         ra.shape[0], ctypes.byref(k), ctypes.byref(m), ctypes.byref(o), None,
                         ctypes.byref(h))
    assert rc == api.HG_ERR_ARG and "ra_deg" in api.last_error()
    assert not h


def test_support_over_too_many_rings_is_refused():
    """A support that spans more HEALPix rings than the gather's LDS holds
    (a pixel group's ring pieces plus its queue of in-support candidates,
    against the 160 KB a workgroup can have) is refused with
    HG_ERR_UNSUPPORTED before any launch: 4 deg on nside 8192 is about 1,700
    rings, past the 1,514 that fit.  A tenth of that support sets up."""
    rng = np.random.default_rng(3)
    ra = 30.0 + (rng.random(200) - 0.5) * 0.2
    dec = (rng.random(200) - 0.5) * 0.2
    m = synth.make_map(30.0, 0.0, 4, 4)
    with pytest.raises(api.HegridError) as e:
        api.Plan(ra, dec, m, {"fwhm_deg": 3.0, "support_deg": 4.0}, nside=8192)
    assert e.value.status == api.HG_ERR_UNSUPPORTED and "rings" in str(e.value)
    with api.Plan(ra, dec, m, {"fwhm_deg": 0.3, "support_deg": 0.4}, nside=8192) as p:
        assert p.stats()["nnz"] > 0
