"""The C ABI without a GPU: the library loads, exports every declared entry
point, the ctypes structs match the header's layout, and argument errors are
reported before any device work."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

import oracle
from paper_2207_04584_amd import api

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hegrid.h")


def declared_functions():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"\b(hg_[a-z0-9_]+)\s*\(", text)))


def test_header_and_binding_agree_on_entry_points():
    assert declared_functions() == sorted(api.ABI_FUNCTIONS)


def test_library_exports_every_declared_symbol():
    L = api.lib()
    for name in declared_functions():
        assert hasattr(L, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", api.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r" T (hg_\w+)", out))
    assert set(declared_functions()) <= exported


PROBE = r"""
#include <stddef.h>
#include <stdio.h>
#include "hegrid.h"
#define F(T, m) printf(#T " " #m " %zu %zu\n", offsetof(T, m), sizeof(((T*)0)->m));
int main(void) {
  printf("hg_map size %zu\nhg_kernel size %zu\nhg_opts size %zu\nhg_stats size %zu\n",
         sizeof(hg_map), sizeof(hg_kernel), sizeof(hg_opts), sizeof(hg_stats));
  printf("hg_field size %zu\nhg_batch_info size %zu\nhg_stream_info size %zu\n",
         sizeof(hg_field), sizeof(hg_batch_info), sizeof(hg_stream_info));
  %FIELDS%
  return 0;
}
"""


def test_struct_layouts_match_header(tmp_path):
    lines = []
    structs = {"hg_map": api.hg_map, "hg_kernel": api.hg_kernel, "hg_opts": api.hg_opts,
               "hg_stats": api.hg_stats, "hg_field": api.hg_field,
               "hg_batch_info": api.hg_batch_info, "hg_stream_info": api.hg_stream_info}
    for cname, cls in structs.items():
        for f, _ in cls._fields_:
            lines.append(f"F({cname}, {f})")
    src = tmp_path / "probe.c"
    src.write_text(PROBE.replace("%FIELDS%", "\n  ".join(lines)))
    exe = tmp_path / "probe"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o",
                    str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout
    for ln in out.splitlines():
        parts = ln.split()
        if parts[1] == "size":
            assert int(parts[2]) == ctypes.sizeof(structs[parts[0]]), ln
        else:
            desc = getattr(structs[parts[0]], parts[1])
            assert (desc.offset, desc.size) == (int(parts[2]), int(parts[3])), ln


def _setup(ra=None, dec=None, n=0, k=None, m=None, o=None, out=True):
    L = api.lib()
    h = ctypes.c_void_p(123)
    rc = L.hg_grid_setup(ra, dec, n, ctypes.byref(k) if k else None,
                         ctypes.byref(m) if m else None, ctypes.byref(o) if o else None, None,
                         ctypes.byref(h) if out else None)
    return rc, h


def good():
    return (api.hg_kernel(0.05, 0.064), api.hg_map(180.0, 30.0, 1 / 60, 1 / 60, 16, 16))


@pytest.mark.parametrize("case", ["null_out", "null_kernel", "neg_n", "null_coords", "fwhm",
                                  "support", "nx", "spacing", "pole", "nside", "chunk",
                                  "chunk_long", "chunk_long_f32", "waves", "chan_block",
                                  "memcap"])
def test_setup_rejects_bad_arguments_without_a_device(case):
    k, m = good()
    o = api.hg_opts()
    kw = dict(k=k, m=m, o=o)
    if case == "null_out":
        kw["out"] = False
    elif case == "null_kernel":
        kw["k"] = None
    elif case == "neg_n":
        kw["n"] = -1
    elif case == "null_coords":
        kw["n"] = 5
    elif case == "fwhm":
        k.fwhm_deg = 0.0
    elif case == "support":
        k.support_deg = float("nan")
    elif case == "nx":
        m.nx = 0
    elif case == "spacing":
        m.ddec_deg = -1.0
    elif case == "pole":
        m.dec0_deg = 89.9
    elif case == "nside":
        o.nside = 3
    elif case == "chunk":
        o.chunk = 7
    elif case == "chunk_long":  # past the 16-bit forms' 112 slots
        o.precision = api.HG_PREC_MFMA_BF16
        o.chunk = 120
    elif case == "chunk_long_f32":  # the FP32 form's 1 KB rows: 64 slots at most
        o.chunk = 72
    elif case == "waves":
        o.waves = 12
    elif case == "chan_block":
        o.chan_block = 96
    elif case == "memcap":
        o.device_mem_cap = -5
    rc, h = _setup(**kw)
    assert rc == api.HG_ERR_ARG, api.last_error()
    assert api.last_error()
    if case != "null_out":
        assert not h.value  # *out is cleared on failure


def hpx_map(nside=64, ring0=100, pix0=10, nx=12, ny=9):
    return api.make_map(dict(proj=api.HG_PROJ_HEALPIX, nside=nside, ring0=ring0, pix0=pix0,
                             nx=nx, ny=ny))


@pytest.mark.parametrize("case", ["hpx_radec", "hpx_nside", "hpx_nx", "hpx_pix0", "hpx_ring",
                                  "car_nside"])
def test_setup_rejects_bad_maps_without_a_device(case):
    k, m = good()
    if case == "car_nside":
        m.nside = 4
    else:
        m = hpx_map()
        if case == "hpx_radec":
            m.ra0_deg = 10.0
        elif case == "hpx_nside":
            m.nside = 48
        elif case == "hpx_nx":
            m.nx = 4 * 64 + 1
        elif case == "hpx_pix0":
            m.pix0 = 4 * 64
        elif case == "hpx_ring":
            m.ring0 = 4 * 64  # past the last ring, 4 nside - 1
    rc, h = _setup(k=k, m=m, o=api.hg_opts())
    assert rc == api.HG_ERR_ARG, api.last_error()
    assert not h.value


@pytest.mark.parametrize("case", ["polar_north", "polar_south", "unknown_proj"])
def test_polar_cap_rows_and_unknown_projections_are_unsupported(case):
    k, _ = good()
    if case == "polar_north":
        m = hpx_map(ring0=70, ny=8)  # rows reach ring 63 < nside
    elif case == "polar_south":
        m = hpx_map(ring0=3 * 64 + 1, ny=4)  # row 0 is ring 193 > 3 nside
    else:
        m = hpx_map()
        m.proj = 7
    rc, h = _setup(k=k, m=m, o=api.hg_opts())
    assert rc == api.HG_ERR_UNSUPPORTED, api.last_error()


@pytest.mark.parametrize("nside,ring0,pix0,nx,ny", [(1, 3, 0, 4, 3), (64, 100, 10, 12, 9),
                                                    (64, 192, 250, 9, 129), (2048, 5000, 8190, 7, 5)])
def test_map_pixel_ids_match_the_reference(nside, ring0, pix0, nx, ny):
    """hg_map_pixel_ids (host arithmetic, no device) against the reference's
    own RING numbering of the same patch; the last two patches wrap past the
    end of their rings, and (64, 192, ...) spans the whole belt."""
    m = dict(proj=api.HG_PROJ_HEALPIX, nside=nside, ring0=ring0, pix0=pix0, nx=nx, ny=ny)
    ids = api.map_pixel_ids(m)
    _, _, ref = oracle.cell_centres(m)
    np.testing.assert_array_equal(ids.ravel(), ref)
    assert len(np.unique(ids)) == nx * ny


def test_map_pixel_ids_refuses_plate_carree():
    _, m = good()
    ids = np.empty(m.nx * m.ny, dtype=np.int64)
    assert api.lib().hg_map_pixel_ids(ctypes.byref(m), ids.ctypes.data) == api.HG_ERR_ARG
    assert api.lib().hg_map_pixel_ids(None, None) == api.HG_ERR_ARG


def test_unknown_precision_is_unsupported():
    k, m = good()
    o = api.hg_opts(precision=99)
    rc, h = _setup(k=k, m=m, o=o)
    assert rc == api.HG_ERR_UNSUPPORTED


def test_channels_and_finish_state_rules():
    L = api.lib()
    assert L.hg_grid_finish(None) == api.HG_OK
    assert L.hg_grid_channels(None, None, 1, 1, 0, None, None) == api.HG_ERR_ARG
    st = api.hg_stats()
    assert L.hg_plan_stats(None, ctypes.byref(st)) == api.HG_ERR_ARG
    assert L.hg_plan_counts(None, None) == api.HG_ERR_ARG
    assert L.hg_ang2pix_ring(0, None, None, 1, None, None) == api.HG_ERR_ARG
    assert L.hg_grid_channels_host(None, None, 1, 1, 0, None, 0, None, None) == api.HG_ERR_ARG
    assert L.hg_grid_channels_literal(None, None, 1, 1, None, 4, 256, None) == api.HG_ERR_ARG
    assert L.hg_ang2pix_ring(8, None, None, 0, None, None) == api.HG_OK  # nothing to do


def _gpu_present():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


@pytest.mark.skipif(_gpu_present(), reason="checks the no-device path")
def test_valid_setup_without_device_reports_device_error():
    k, m = good()
    rc, h = _setup(k=k, m=m, o=api.hg_opts())
    assert rc == api.HG_ERR_DEVICE
    assert "device" in api.last_error()


def _field(n=0, nchan=0):
    k, m = good()
    return api.hg_field(None, None, n, k, m, None, nchan, nchan, 0, None)


def _batch(fields, nfields=None, dtype=api.HG_F32, o=None, out=True):
    L = api.lib()
    h = ctypes.c_void_p(123)
    arr = None
    if fields is not None:
        arr = (api.hg_field * max(len(fields), 1))(*fields)
    rc = L.hg_batch_create(arr, len(fields) if nfields is None else nfields, dtype,
                           ctypes.byref(o) if o else None, None,
                           ctypes.byref(h) if out else None)
    return rc, h


@pytest.mark.parametrize("case", ["null_out", "null_fields", "zero_fields", "dtype", "map",
                                  "nchan", "reserved", "null_out_buf", "ld", "null_values",
                                  "chunk"])
def test_batch_create_rejects_bad_arguments_without_a_device(case):
    fields, kw = [_field()], {}
    f = fields[0]
    if case == "null_out":
        kw["out"] = False
    elif case == "null_fields":
        fields, kw["nfields"] = None, 1
    elif case == "zero_fields":
        kw["nfields"] = 0
    elif case == "dtype":
        kw["dtype"] = 7
    elif case == "map":
        f.map.nx = 0
    elif case == "nchan":
        f.nchan = -1
    elif case == "reserved":
        f.reserved = 2
    elif case == "null_out_buf":
        f.nchan, f.ld, f.values = 4, 4, 1
    elif case == "ld":
        f.nchan, f.ld, f.values, f.out = 4, 3, 1, 1
    elif case == "null_values":
        f.n, f.ra_deg, f.dec_deg, f.nchan, f.ld, f.out = 5, 1, 1, 4, 4, 1
    elif case == "chunk":
        kw["o"] = api.hg_opts(chunk=12)
    if fields is None:
        L = api.lib()
        h = ctypes.c_void_p(123)
        rc = L.hg_batch_create(None, 1, 0, None, None, ctypes.byref(h))
    else:
        rc, h = _batch(fields, **kw)
    assert rc == api.HG_ERR_ARG, api.last_error()
    if case in ("map", "nchan", "reserved", "null_out_buf", "ld", "null_values", "chunk"):
        assert api.last_error().startswith("field 0: "), api.last_error()
    if case != "null_out":
        assert not h.value


def test_batch_precision_must_match_dtype():
    for prec, dtype in ((1, api.HG_F32), (1, api.HG_F16), (2, api.HG_BF16)):
        rc, h = _batch([_field()], dtype=dtype, o=api.hg_opts(precision=prec))
        assert rc == api.HG_ERR_UNSUPPORTED, (prec, dtype)


def test_batch_null_handles():
    L = api.lib()
    assert L.hg_batch_destroy(None) == api.HG_OK
    assert L.hg_batch_run(None, None) == api.HG_ERR_ARG
    info = api.hg_batch_info()
    assert L.hg_batch_stats(None, ctypes.byref(info)) == api.HG_ERR_ARG
    h = ctypes.c_void_p()
    assert L.hg_batch_plan(None, 0, ctypes.byref(h)) == api.HG_ERR_ARG


@pytest.mark.skipif(_gpu_present(), reason="checks the no-device path")
def test_valid_batch_without_device_reports_device_error():
    rc, h = _batch([_field(), _field()])
    assert rc == api.HG_ERR_DEVICE
    assert not h.value


def test_binding_refuses_a_host_output_tensor():
    """The kernels write through `out`'s address, so a host tensor must be
    refused by the binding (HG_ERR_ARG) before any library call; so must one
    on another device or of the wrong shape."""
    import torch
    dev = torch.device("cuda", 0)  # a device object needs no GPU
    with pytest.raises(api.HegridError) as e:
        api._out_arg(torch.empty(3, 2, 2, dtype=torch.float32), 3, 2, 2, dev)
    assert e.value.status == api.HG_ERR_ARG and "device" in str(e.value)
    with pytest.raises(api.HegridError):
        api._out_arg(torch.empty(3, 2, 2, dtype=torch.float64), 3, 2, 2, dev)
    with pytest.raises(api.HegridError):
        api._out_arg(torch.empty(2, 2, 2, dtype=torch.float32), 3, 2, 2, dev)


def test_binding_constants_match_the_header():
    """Every integer #define and kernel enum value of include/hegrid.h that
    the binding also names has the same value there (status codes, dtypes,
    forms, projections, flags, kernel shapes)."""
    hdr = open(os.path.join(os.path.dirname(api.LIB_PATH), "..", "include", "hegrid.h")).read()
    pairs = re.findall(r"^#define (HG_\w+) (\d+)u?\b", hdr, flags=re.M)
    pairs += re.findall(r"^\s+(HG_KERNEL_\w+) = (\d+)", hdr, flags=re.M)  # the kernel enum
    found = 0
    for name, val in pairs:
        if hasattr(api, name):
            assert getattr(api, name) == int(val), name
            found += 1
    assert found == 20
