"""Thin ctypes binding of libhegrid (include/hegrid.h).

Argument marshalling only: torch supplies device memory (``data_ptr()``) and
the current HIP stream; every step of the gridding runs in the library's
kernels.  There is no fallback: if ``libhegrid.so`` is missing or cannot be
loaded, every call raises.
"""
import ctypes
import os

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libhegrid.so")

HG_OK, HG_ERR_ARG, HG_ERR_STATE, HG_ERR_NOMEM, HG_ERR_DEVICE, HG_ERR_UNSUPPORTED, \
    HG_ERR_INTERNAL = range(7)
HG_F32, HG_BF16, HG_F16 = 0, 1, 2
HG_PREC_FP32, HG_PREC_MFMA_BF16, HG_PREC_MFMA_F16 = 0, 1, 2
HG_FLAG_TIME_CHANNELS = 1
HG_FLAG_PREDICT_CHUNK = 2

ABI_FUNCTIONS = ("hg_grid_setup", "hg_grid_channels", "hg_grid_finish", "hg_plan_stats",
                 "hg_plan_counts", "hg_plan_weight_sums", "hg_plan_neighbours",
                 "hg_ang2pix_ring", "hg_grid_channels_host", "hg_grid_channels_literal",
                 "hg_batch_create", "hg_batch_run", "hg_batch_destroy", "hg_batch_stats",
                 "hg_batch_plan", "hg_map_pixel_ids", "hg_plan_set_shape", "hg_last_error",
                 "hg_grid_channels_host_noalloc", "hg_grid_channels_rows", "hg_plan_row_needs")


class HegridError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"[status {status}] {msg}")
        self.status = status


class hg_map(ctypes.Structure):
    _fields_ = [("ra0_deg", ctypes.c_double), ("dec0_deg", ctypes.c_double),
                ("dra_deg", ctypes.c_double), ("ddec_deg", ctypes.c_double),
                ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
                ("proj", ctypes.c_int32), ("nside", ctypes.c_int32),
                ("ring0", ctypes.c_int32), ("pix0", ctypes.c_int32)]


HG_PROJ_CAR, HG_PROJ_HEALPIX = 0, 1


class hg_kernel(ctypes.Structure):
    _fields_ = [("fwhm_deg", ctypes.c_double), ("support_deg", ctypes.c_double),
                ("type", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("p1", ctypes.c_double), ("p2", ctypes.c_double)]


HG_KERNEL_GAUSS, HG_KERNEL_GAUSS_SINC, HG_KERNEL_ELLIPTICAL = 0, 1, 2


class hg_opts(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("nside", ctypes.c_int32),
                ("chunk", ctypes.c_int32), ("waves", ctypes.c_int32),
                ("device_mem_cap", ctypes.c_int64), ("flags", ctypes.c_uint32),
                ("chan_block", ctypes.c_int32)]


class hg_stats(ctypes.Structure):
    _fields_ = [("n_samples", ctypes.c_int64), ("n_used", ctypes.c_int64),
                ("nnz", ctypes.c_int64), ("n_entries", ctypes.c_int64),
                ("n_cells", ctypes.c_int64), ("total_slots", ctypes.c_int64),
                ("device_bytes", ctypes.c_int64), ("nside", ctypes.c_int32),
                ("chunk", ctypes.c_int32), ("waves", ctypes.c_int32),
                ("chan_block", ctypes.c_int32), ("setup_ms", ctypes.c_double),
                ("last_channels_ms", ctypes.c_double), ("total_channels_ms", ctypes.c_double),
                ("channels_calls", ctypes.c_int64)]


class hg_stream_info(ctypes.Structure):
    _fields_ = [("blocks", ctypes.c_int32), ("pinned", ctypes.c_int32),
                ("h2d_bytes", ctypes.c_int64), ("d2h_bytes", ctypes.c_int64),
                ("wall_ms", ctypes.c_double), ("kernel_ms", ctypes.c_double),
                ("h2d_ms", ctypes.c_double), ("d2h_ms", ctypes.c_double)]


class hg_field(ctypes.Structure):
    _fields_ = [("ra_deg", ctypes.c_void_p), ("dec_deg", ctypes.c_void_p), ("n", ctypes.c_int64),
                ("kernel", hg_kernel), ("map", hg_map), ("values", ctypes.c_void_p),
                ("ld", ctypes.c_int64), ("nchan", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("out", ctypes.c_void_p)]


class hg_batch_info(ctypes.Structure):
    _fields_ = [("n_fields", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("n_items", ctypes.c_int64), ("n_workgroups", ctypes.c_int64),
                ("n_samples", ctypes.c_int64), ("nnz", ctypes.c_int64),
                ("n_entries", ctypes.c_int64), ("device_bytes", ctypes.c_int64),
                ("setup_ms", ctypes.c_double), ("last_run_ms", ctypes.c_double),
                ("total_run_ms", ctypes.c_double), ("runs", ctypes.c_int64)]


_lib = None


def lib():
    """Load libhegrid.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise HegridError(HG_ERR_DEVICE, f"{LIB_PATH} is not built "
                          "(python -m paper_2207_04584_amd.build)")
    L = ctypes.CDLL(LIB_PATH)
    P, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    L.hg_grid_setup.argtypes = [P, P, i64, ctypes.POINTER(hg_kernel), ctypes.POINTER(hg_map),
                                ctypes.POINTER(hg_opts), P, ctypes.POINTER(ctypes.c_void_p)]
    L.hg_grid_channels.argtypes = [P, P, i64, i32, i32, P, P]
    L.hg_grid_channels_rows.argtypes = [P, P, i64, i32, i32, P, i32, i32, P]
    L.hg_plan_row_needs.argtypes = [P, i32, P, i32, P]
    L.hg_grid_channels_literal.argtypes = [P, P, i64, i32, P, i32, i32, P]
    L.hg_grid_finish.argtypes = [P]
    L.hg_plan_stats.argtypes = [P, ctypes.POINTER(hg_stats)]
    L.hg_plan_counts.argtypes = [P, P]
    L.hg_plan_set_shape.argtypes = [P, i32, i32]
    L.hg_plan_weight_sums.argtypes = [P, P]
    L.hg_plan_neighbours.argtypes = [P, P, P, P, i64, ctypes.POINTER(ctypes.c_int64)]
    L.hg_ang2pix_ring.argtypes = [i32, P, P, i64, P, P]
    L.hg_map_pixel_ids.argtypes = [ctypes.POINTER(hg_map), P]
    L.hg_grid_channels_host.argtypes = [P, P, i64, i32, i32, P, i32, P,
                                        ctypes.POINTER(hg_stream_info)]
    L.hg_grid_channels_host_noalloc.argtypes = [P, P, i64, i32, i32, P, i32, P,
                                                ctypes.POINTER(hg_stream_info)]
    L.hg_batch_create.argtypes = [ctypes.POINTER(hg_field), i32, i32, ctypes.POINTER(hg_opts), P,
                                  ctypes.POINTER(ctypes.c_void_p)]
    L.hg_batch_run.argtypes = [P, P]
    L.hg_batch_destroy.argtypes = [P]
    L.hg_batch_stats.argtypes = [P, ctypes.POINTER(hg_batch_info)]
    L.hg_batch_plan.argtypes = [P, i32, ctypes.POINTER(ctypes.c_void_p)]
    for f in ABI_FUNCTIONS:
        if f != "hg_last_error":
            getattr(L, f).restype = ctypes.c_int
    L.hg_last_error.argtypes = []
    L.hg_last_error.restype = ctypes.c_char_p
    _lib = L
    return L


def last_error():
    return lib().hg_last_error().decode()


def _check(rc, what):
    if rc != HG_OK:
        raise HegridError(rc, f"{what}: {last_error()}")


def _torch():
    import torch
    return torch


def _stream_ptr(stream):
    torch = _torch()
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _dev_f64(x):
    torch = _torch()
    t = torch.as_tensor(x, dtype=torch.float64)
    if t.device.type != "cuda":
        t = t.to("cuda")
    return t.contiguous()


def make_map(m):
    """A map dict as the C struct: plate carree {"ra0_deg", "dec0_deg",
    "dra_deg", "ddec_deg", "nx", "ny"}, or a HEALPix patch {"proj":
    HG_PROJ_HEALPIX, "nside", "ring0", "pix0", "nx", "ny"} (row j = ring
    ring0 - j, column i = pixel (pix0 + i) mod 4 nside of the ring)."""
    proj = int(m.get("proj", HG_PROJ_CAR))
    if proj == HG_PROJ_HEALPIX:
        return hg_map(0.0, 0.0, 0.0, 0.0, int(m["nx"]), int(m["ny"]), proj, int(m["nside"]),
                      int(m["ring0"]), int(m["pix0"]))
    return hg_map(float(m["ra0_deg"]), float(m["dec0_deg"]), float(m["dra_deg"]),
                  float(m["ddec_deg"]), int(m["nx"]), int(m["ny"]), proj,
                  int(m.get("nside", 0)), int(m.get("ring0", 0)), int(m.get("pix0", 0)))


def map_pixel_ids(m):
    """HEALPix RING pixel numbers of a HEALPix map's cells, int64 [ny][nx]
    (host arithmetic in the library; no device needed)."""
    hm = make_map(m)
    ids = np.empty((hm.ny, hm.nx), dtype=np.int64)
    _check(lib().hg_map_pixel_ids(ctypes.byref(hm), ids.ctypes.data_as(ctypes.c_void_p)),
           "hg_map_pixel_ids")
    return ids


def make_kernel(k):
    return hg_kernel(float(k["fwhm_deg"]), float(k["support_deg"]), int(k.get("type", 0)), 0,
                     float(k.get("p1", 0.0)), float(k.get("p2", 0.0)))


_DTYPES = None


def _dtype_code(t):
    torch = _torch()
    codes = {torch.float32: HG_F32, torch.bfloat16: HG_BF16, torch.float16: HG_F16}
    if t.dtype not in codes:
        raise HegridError(HG_ERR_ARG, f"unsupported value dtype {t.dtype}")
    return codes[t.dtype]


class Plan:
    """A gridding plan: grid_setup on construction, grid_channels per call,
    grid_finish on close().  predict_chunk (with chunk 0): start at the chunk
    length predicted from the support, as a batch's fields do
    (HG_FLAG_PREDICT_CHUNK), rather than at the longest."""

    def __init__(self, ra_deg, dec_deg, map, kernel, precision=HG_PREC_FP32, nside=0, chunk=0,
                 device_mem_cap=0, time_channels=False, stream=None, waves=0, chan_block=0,
                 predict_chunk=False):
        L = lib()
        ra, dec = _dev_f64(ra_deg), _dev_f64(dec_deg)
        if ra.shape != dec.shape or ra.dim() != 1:
            raise HegridError(HG_ERR_ARG, "ra and dec must be 1-D and of equal length")
        self.map = dict(map)
        self.kernel = dict(kernel)
        self.n = ra.shape[0]
        self._m, self._k = make_map(map), make_kernel(kernel)
        self._o = hg_opts(int(precision), int(nside), int(chunk), int(waves), int(device_mem_cap),
                          (HG_FLAG_TIME_CHANNELS if time_channels else 0)
                          | (HG_FLAG_PREDICT_CHUNK if predict_chunk else 0), int(chan_block))
        self._h = ctypes.c_void_p()
        rc = L.hg_grid_setup(ctypes.c_void_p(ra.data_ptr() if self.n else 0),
                             ctypes.c_void_p(dec.data_ptr() if self.n else 0), self.n,
                             ctypes.byref(self._k), ctypes.byref(self._m), ctypes.byref(self._o),
                             _stream_ptr(stream), ctypes.byref(self._h))
        _check(rc, "hg_grid_setup")

    @property
    def shape(self):
        return int(self.map["ny"]), int(self.map["nx"])

    def _handle(self):
        if not self._h:
            raise HegridError(HG_ERR_STATE, "plan is closed")
        return self._h

    def grid(self, values, out=None, stream=None):
        """values: cuda tensor [n][C] (float32 / bfloat16 / float16, unit
        channel stride); returns float32 [C][ny][nx] on the same device."""
        torch = _torch()
        values, ld = _values_arg(values, self.n)
        nchan = values.shape[1]
        ny, nx = self.shape
        if out is None:
            out = torch.empty((nchan, ny, nx), dtype=torch.float32, device=values.device)
        _out_arg(out, nchan, ny, nx, values.device)
        rc = lib().hg_grid_channels(self._handle(), ctypes.c_void_p(values.data_ptr()), ld, nchan,
                                    _dtype_code(values), ctypes.c_void_p(out.data_ptr()),
                                    _stream_ptr(stream))
        _check(rc, "hg_grid_channels")
        return out

    def grid_rows(self, values, out, row0, row1, stream=None):
        """The channel phase for tile rows [row0, row1) (map rows [16 row0,
        min(16 row1, ny))) into out, the whole cube's float32 [C][ny][nx]
        device buffer; other rows of out are left as they are."""
        values, ld = _values_arg(values, self.n)
        nchan = values.shape[1]
        ny, nx = self.shape
        _out_arg(out, nchan, ny, nx, values.device)
        rc = lib().hg_grid_channels_rows(self._handle(), ctypes.c_void_p(values.data_ptr()), ld,
                                         nchan, _dtype_code(values),
                                         ctypes.c_void_p(out.data_ptr()), int(row0), int(row1),
                                         _stream_ptr(stream))
        _check(rc, "hg_grid_channels_rows")
        return out

    @property
    def tile_rows(self):
        return (self.shape[0] + 15) // 16

    def row_needs(self, rows_per_band, stream=None):
        """Per band of rows_per_band tile rows: 1 + the largest sample index
        the band's tiles stage (0 if none), as an int64 numpy array."""
        nb = (self.tile_rows + rows_per_band - 1) // rows_per_band
        need = np.zeros(nb, dtype=np.int64)
        _check(lib().hg_plan_row_needs(self._handle(), int(rows_per_band),
                                       need.ctypes.data_as(ctypes.c_void_p), nb,
                                       _stream_ptr(stream)), "hg_plan_row_needs")
        return need

    def grid_host(self, values, out=None, block=0, stream=None):
        """values: host (CPU) tensor [n][C] of float32 / bfloat16 / float16
        with unit channel stride, pageable or pinned; streamed to the GPU in
        blocks of `block` channels (0 = 4096).  Returns (out, info): out a
        float32 host tensor [C][ny][nx] (allocated pinned if not given), info
        the call's hg_stream_info as a dict."""
        torch = _torch()
        if values.dim() == 1:
            values = values.reshape(-1, 1)
        if values.device.type != "cpu" or values.shape[0] != self.n or (
                self.n > 0 and values.stride(1) != 1):
            raise HegridError(HG_ERR_ARG, "values must be a host tensor [n][C] with unit "
                              "channel stride")
        nchan = values.shape[1]
        ld = values.stride(0) if values.shape[0] > 1 else nchan
        ny, nx = self.shape
        if out is None:
            out = torch.empty((nchan, ny, nx), dtype=torch.float32, pin_memory=True)
        if (out.dtype != torch.float32 or out.device.type != "cpu" or not out.is_contiguous()
                or out.numel() != nchan * ny * nx):
            raise HegridError(HG_ERR_ARG, "out must be a contiguous float32 host tensor "
                              "[C][ny][nx]")
        info = hg_stream_info()
        rc = lib().hg_grid_channels_host(self._handle(),
                                         ctypes.c_void_p(values.data_ptr() if self.n else 0),
                                         ld, nchan, _dtype_code(values),
                                         ctypes.c_void_p(out.data_ptr()), int(block),
                                         _stream_ptr(stream), ctypes.byref(info))
        _check(rc, "hg_grid_channels_host")
        return out, {f: getattr(info, f) for f, _ in hg_stream_info._fields_}

    def grid_host_noalloc(self, values, out, block=0, stream=None):
        """hg_grid_channels_host_noalloc: as grid_host, through the library's
        fixed per-device staging array (no device allocation).  values and
        out must be page-locked host tensors (out float32 [C][ny][nx]);
        returns (out, info)."""
        torch = _torch()
        if values.dim() == 1:
            values = values.reshape(-1, 1)
        if values.device.type != "cpu" or values.shape[0] != self.n or (
                self.n > 0 and values.stride(1) != 1):
            raise HegridError(HG_ERR_ARG, "values must be a host tensor [n][C] with unit "
                              "channel stride")
        nchan = values.shape[1]
        ld = values.stride(0) if values.shape[0] > 1 else nchan
        ny, nx = self.shape
        if (out.dtype != torch.float32 or out.device.type != "cpu" or not out.is_contiguous()
                or out.numel() != nchan * ny * nx):
            raise HegridError(HG_ERR_ARG, "out must be a contiguous float32 host tensor "
                              "[C][ny][nx]")
        info = hg_stream_info()
        rc = lib().hg_grid_channels_host_noalloc(
            self._handle(), ctypes.c_void_p(values.data_ptr() if self.n else 0), ld, nchan,
            _dtype_code(values), ctypes.c_void_p(out.data_ptr()), int(block),
            _stream_ptr(stream), ctypes.byref(info))
        _check(rc, "hg_grid_channels_host_noalloc")
        return out, {f: getattr(info, f) for f, _ in hg_stream_info._fields_}

    def grid_literal(self, values, out=None, gamma=4, block=256, stream=None):
        """Algorithm 1 as the paper states it (one launch per channel, one
        thread per `gamma` cells, FP64 distances, weights and sums), the
        comparison path: values a float32 device tensor [n][C] with unit
        channel stride; returns out float32 [C][ny][nx] on the device."""
        torch = _torch()
        if values.dim() == 1:
            values = values.reshape(-1, 1)
        if (values.dtype != torch.float32 or values.device.type != "cuda"
                or values.shape[0] != self.n or (self.n > 0 and values.stride(1) != 1)):
            raise HegridError(HG_ERR_ARG, "values must be a float32 device tensor [n][C] with "
                              "unit channel stride")
        nchan = values.shape[1]
        ld = values.stride(0) if values.shape[0] > 1 else nchan
        ny, nx = self.shape
        if out is None:
            out = torch.empty((nchan, ny, nx), dtype=torch.float32, device=values.device)
        _out_arg(out, nchan, ny, nx, values.device)
        rc = lib().hg_grid_channels_literal(self._handle(),
                                            ctypes.c_void_p(values.data_ptr() if self.n else 0),
                                            ld, nchan, ctypes.c_void_p(out.data_ptr()), int(gamma),
                                            int(block), _stream_ptr(stream))
        _check(rc, "hg_grid_channels_literal")
        return out

    def stats(self):
        st = hg_stats()
        _check(lib().hg_plan_stats(self._handle(), ctypes.byref(st)), "hg_plan_stats")
        return {f: getattr(st, f) for f, _ in hg_stats._fields_}

    def set_shape(self, waves=0, chan_block=0):
        """The channel kernel's shape for later grid calls (waves per
        workgroup 8 / 16, channels per workgroup 64 / 128 / 256; 0 = default);
        the maps do not depend on it."""
        _check(lib().hg_plan_set_shape(self._handle(), int(waves), int(chan_block)),
               "hg_plan_set_shape")

    def counts(self):
        ny, nx = self.shape
        c = np.empty(ny * nx, dtype=np.int32)
        _check(lib().hg_plan_counts(self._handle(), c.ctypes.data_as(ctypes.c_void_p)),
               "hg_plan_counts")
        return c

    def weight_sums(self):
        ny, nx = self.shape
        w = np.empty(ny * nx, dtype=np.float64)
        _check(lib().hg_plan_weight_sums(self._handle(), w.ctypes.data_as(ctypes.c_void_p)),
               "hg_plan_weight_sums")
        return w

    def neighbours(self):
        """(row_ptr, idx, w): per pixel, ascending original sample index."""
        ny, nx = self.shape
        row_ptr = np.zeros(ny * nx + 1, dtype=np.int64)
        nnz = ctypes.c_int64(0)
        L = lib()
        _check(L.hg_plan_neighbours(self._handle(), row_ptr.ctypes.data_as(ctypes.c_void_p), None,
                                    None, 0, ctypes.byref(nnz)), "hg_plan_neighbours")
        idx = np.empty(max(nnz.value, 1), dtype=np.int64)
        w = np.empty(max(nnz.value, 1), dtype=np.float32)
        _check(L.hg_plan_neighbours(self._handle(), row_ptr.ctypes.data_as(ctypes.c_void_p),
                                    idx.ctypes.data_as(ctypes.c_void_p),
                                    w.ctypes.data_as(ctypes.c_void_p), nnz.value,
                                    ctypes.byref(nnz)), "hg_plan_neighbours")
        return row_ptr, idx[:nnz.value], w[:nnz.value]

    @classmethod
    def _borrowed(cls, handle, map, kernel, n, owner):
        p = cls.__new__(cls)
        p.map, p.kernel, p.n = dict(map), dict(kernel), int(n)
        p._h = handle
        p._owner = owner  # keeps the batch (which frees the plan) alive
        return p

    def close(self):
        if getattr(self, "_owner", None) is not None:
            self._h, self._owner = ctypes.c_void_p(), None
            return
        if self._h:
            h, self._h = self._h, ctypes.c_void_p()
            _check(lib().hg_grid_finish(h), "hg_grid_finish")

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _values_arg(values, n):
    if values.dim() == 1:
        values = values.reshape(-1, 1)
    if values.dim() == 2 and values.shape[0] == n == 0 and values.device.type == "cuda":
        return values, values.shape[1]  # nothing is read
    if values.shape[0] != n or values.stride(1) != 1 or values.device.type != "cuda":
        raise HegridError(HG_ERR_ARG, "values must be a cuda tensor [n][C] with unit channel "
                          "stride")
    return values, (values.stride(0) if values.shape[0] > 1 else values.shape[1])


def _out_arg(out, nchan, ny, nx, device):
    """out must be a contiguous float32 [C][ny][nx] tensor on the values'
    device: the kernel writes through its address, which for host memory
    would be a GPU memory fault rather than an error."""
    torch = _torch()
    if out.dtype != torch.float32 or not out.is_contiguous() or out.numel() != nchan * ny * nx:
        raise HegridError(HG_ERR_ARG, "out must be a contiguous float32 [C][ny][nx] tensor")
    if out.device.type != "cuda" or out.device != device:
        raise HegridError(HG_ERR_ARG, f"out must be on the values' device ({device}), not "
                          f"{out.device}")


_side_streams = {}


def _side_stream(dev):
    """One copy stream per device, made once: a stream made per call lands on
    a different hardware queue each time, sometimes the current stream's."""
    torch = _torch()
    key = dev.index
    if key not in _side_streams:
        _side_streams[key] = torch.cuda.Stream(device=dev)
    return _side_streams[key]


_out_streams = {}


def _out_stream(dev):
    """A second copy stream per device (the cube's way back), made once."""
    torch = _torch()
    key = dev.index
    if key not in _out_streams:
        _out_streams[key] = torch.cuda.Stream(device=dev)
    return _out_streams[key]


_hip = None
BAND_LINEAR_MAX = 512  # channels up to which a band's rows go back channel by channel


def _hip_lib():
    """The HIP runtime, for the device-to-host copies of a band of map rows
    (strided over the channels); copies are plumbing, not the path."""
    global _hip
    if _hip is None:
        H = ctypes.CDLL("libamdhip64.so")
        sz = ctypes.c_size_t
        H.hipMemcpy2DAsync.argtypes = [ctypes.c_void_p, sz, ctypes.c_void_p, sz, sz, sz,
                                       ctypes.c_int, ctypes.c_void_p]
        H.hipMemcpy2DAsync.restype = ctypes.c_int
        H.hipMemcpyAsync.argtypes = [ctypes.c_void_p, ctypes.c_void_p, sz, ctypes.c_int,
                                     ctypes.c_void_p]
        H.hipMemcpyAsync.restype = ctypes.c_int
        _hip = H
    return _hip


def grid_from_host(ra_deg, dec_deg, map, kernel, values, out=None, precision=HG_PREC_FP32,
                   chunk=0, dev_values=None, dev_out=None, bands=0, pieces=16):
    """Eq. 1 end to end from host memory, with the values' copy to the device
    hidden behind the setup: setup reads only the coordinates, so the values
    go over on a stream of their own while the plan is built on the current
    stream; then the channel kernel runs on the device copy and the cube comes
    back.  ra_deg, dec_deg: host FP64 [n]; values: host tensor [n][C] (pinned,
    for the copy to be asynchronous); out: pinned float32 [C][ny][nx] or None.
    dev_values, dev_out: device buffers to reuse (allocated when None).

    bands > 0 pipelines the rest as well: the values go over in `pieces`
    index ranges, each with an event; the map is gridded in `bands` bands of
    tile rows (hg_grid_channels_rows), each band started once the values of
    every sample it stages have arrived (hg_plan_row_needs; for samples in
    scan order a band needs a narrow index range), and each finished band's
    rows go back on a third stream while later bands compute.  The maps equal
    the unbanded call's bit for bit.

    Returns (out, info): info holds the phases' times in ms (h2d of the
    values, setup, kernel -- summed over the bands --, d2h of the cube, and
    with bands the span from the first band's start to the last band's end)."""
    torch = _torch()
    dev = torch.device("cuda", torch.cuda.current_device())
    if values.dim() == 1:
        values = values.reshape(-1, 1)
    n, nchan = values.shape
    ny, nx = int(map["ny"]), int(map["nx"])
    if dev_values is None:
        dev_values = torch.empty((n, nchan), dtype=values.dtype, device=dev)
    if dev_out is None:
        dev_out = torch.empty((nchan, ny, nx), dtype=torch.float32, device=dev)
    if out is None:
        out = torch.empty((nchan, ny, nx), dtype=torch.float32, pin_memory=True)
    cur = torch.cuda.current_stream()
    side = _side_stream(dev)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    ra = torch.as_tensor(ra_deg, dtype=torch.float64).to(dev, non_blocking=True)
    dec = torch.as_tensor(dec_deg, dtype=torch.float64).to(dev, non_blocking=True)
    # the values follow the coordinates over the bus (setup waits only for
    # those), and their buffer is free once the current stream's earlier work
    # is done
    side.wait_stream(cur)
    npieces = max(1, min(int(pieces), n)) if bands > 0 else 1
    cuts = [k * n // npieces for k in range(npieces + 1)]
    piece_ev = []
    with torch.cuda.stream(side):
        ev[0].record()
        for k in range(npieces):
            a, b = cuts[k], cuts[k + 1]
            if b > a:
                dev_values[a:b].copy_(values[a:b], non_blocking=True)
            piece_ev.append(torch.cuda.Event())
            piece_ev[-1].record()
        ev[1].record()
    try:
        plan = Plan(ra, dec, map, kernel, precision=precision, chunk=chunk, time_channels=True)
    except Exception:
        side.synchronize()  # the copy still writes dev_values, which may be freed on return
        raise
    info = {}
    try:
        if bands <= 0:
            cur.wait_stream(side)
            plan.grid(dev_values, dev_out)
            ev[2].record(cur)
            out.copy_(dev_out, non_blocking=True)
            ev[3].record(cur)
            cur.synchronize()
            st = plan.stats()
            info["d2h_ms"] = ev[2].elapsed_time(ev[3])
            info["kernel_ms"] = st["last_channels_ms"]
        else:
            rows = plan.tile_rows
            per = (rows + bands - 1) // bands
            need = plan.row_needs(per)
            outs = _out_stream(dev)
            hip = _hip_lib()
            row_bytes = nx * 4
            band_ev = [torch.cuda.Event() for _ in need]
            d2h = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
            ev[2].record(cur)
            for i, bnd in enumerate(sorted(range(len(need)), key=lambda b: need[b])):
                if need[bnd] > 0:
                    k = next(k for k in range(npieces) if cuts[k + 1] >= need[bnd])
                    cur.wait_event(piece_ev[k])
                r0, r1 = bnd * per, min((bnd + 1) * per, rows)
                plan.grid_rows(dev_values, dev_out, r0, r1)
                band_ev[bnd].record(cur)
                outs.wait_event(band_ev[bnd])
                y0, y1 = 16 * r0, min(16 * r1, ny)
                if i == 0:
                    d2h[0].record(outs)
                # a band's rows are one contiguous piece per channel: linear
                # copies of those overlap the values' copies in the other
                # direction, where one 2-D copy of the band waited for them
                # (87.8 against 77.6 ms per step on the paper-scale field);
                # past BAND_LINEAR_MAX channels, one 2-D copy per band
                if nchan <= BAND_LINEAR_MAX:
                    for c in range(nchan):
                        off = (c * ny + y0) * row_bytes
                        rc = hip.hipMemcpyAsync(ctypes.c_void_p(out.data_ptr() + off),
                                                ctypes.c_void_p(dev_out.data_ptr() + off),
                                                (y1 - y0) * row_bytes, 2,
                                                ctypes.c_void_p(outs.cuda_stream))
                        if rc != 0:
                            raise HegridError(HG_ERR_DEVICE, f"hipMemcpyAsync failed ({rc})")
                else:
                    rc = hip.hipMemcpy2DAsync(ctypes.c_void_p(out.data_ptr() + y0 * row_bytes),
                                              ny * row_bytes,
                                              ctypes.c_void_p(dev_out.data_ptr() + y0 * row_bytes),
                                              ny * row_bytes, (y1 - y0) * row_bytes, nchan, 2,
                                              ctypes.c_void_p(outs.cuda_stream))
                    if rc != 0:
                        raise HegridError(HG_ERR_DEVICE, f"hipMemcpy2DAsync failed ({rc})")
            ev[3].record(cur)
            d2h[1].record(outs)
            outs.synchronize()
            cur.synchronize()
            st = plan.stats()
            info["d2h_ms"] = d2h[0].elapsed_time(d2h[1])
            info["kernel_ms"] = st["total_channels_ms"]
            info["bands_ms"] = ev[2].elapsed_time(ev[3])
            info["bands"] = len(need)
    finally:
        side.synchronize()
        plan.close()
    info.update({"h2d_ms": ev[0].elapsed_time(ev[1]), "setup_ms": st["setup_ms"],
                 "nnz": st["nnz"]})
    return out, info


class Batch:
    """Many fields gridded by one graph-held launch (hg_batch_create /
    hg_batch_run / hg_batch_destroy).

    fields: list of dicts with 'ra', 'dec' (degrees), 'map', 'kernel',
    'values' (cuda tensor [n][C], all of one dtype, or None for C = 0) and an
    optional 'out' (float32 cuda [C][ny][nx]; allocated if absent).  The
    tensors are bound at creation and kept alive by the batch; run() grids all
    of them and returns the list of outputs."""

    def __init__(self, fields, precision=HG_PREC_FP32, nside=0, chunk=0, device_mem_cap=0,
                 time_runs=False, stream=None, waves=0, chan_block=0):
        torch = _torch()
        L = lib()
        self._keep = []
        self.outs = []
        self.fields = []
        arr = (hg_field * len(fields))()
        dtype = None
        for i, f in enumerate(fields):
            ra, dec = _dev_f64(f["ra"]), _dev_f64(f["dec"])
            n = ra.shape[0]
            m, k = f["map"], f["kernel"]
            vals, out, ld, nchan = f.get("values"), f.get("out"), 0, 0
            if vals is not None:
                vals, ld = _values_arg(vals, n)
                nchan = vals.shape[1]
                code = _dtype_code(vals)
                if dtype is None:
                    dtype = code
                elif code != dtype:
                    raise HegridError(HG_ERR_ARG, "all fields of a batch share one dtype")
                if out is None:
                    out = torch.empty((nchan, m["ny"], m["nx"]), dtype=torch.float32,
                                      device=vals.device)
                _out_arg(out, nchan, m["ny"], m["nx"], vals.device)
            self._keep += [ra, dec, vals, out]
            self.outs.append(out)
            self.fields.append({"map": dict(m), "kernel": dict(k), "n": n, "nchan": nchan})
            arr[i] = hg_field(ra.data_ptr() if n else None, dec.data_ptr() if n else None, n,
                              make_kernel(k), make_map(m),
                              vals.data_ptr() if vals is not None and n else None, ld, nchan, 0,
                              out.data_ptr() if out is not None else None)
        if dtype is None:
            dtype = {1: HG_BF16, 2: HG_F16}.get(int(precision), HG_F32)
        self.dtype = dtype
        self._o = hg_opts(int(precision), int(nside), int(chunk), int(waves), int(device_mem_cap),
                          HG_FLAG_TIME_CHANNELS if time_runs else 0, int(chan_block))
        self._h = ctypes.c_void_p()
        _check(L.hg_batch_create(arr, len(fields), dtype, ctypes.byref(self._o),
                                 _stream_ptr(stream), ctypes.byref(self._h)), "hg_batch_create")

    def _handle(self):
        if not self._h:
            raise HegridError(HG_ERR_STATE, "batch is closed")
        return self._h

    def run(self, stream=None):
        _check(lib().hg_batch_run(self._handle(), _stream_ptr(stream)), "hg_batch_run")
        return self.outs

    def stats(self):
        st = hg_batch_info()
        _check(lib().hg_batch_stats(self._handle(), ctypes.byref(st)), "hg_batch_stats")
        return {f: getattr(st, f) for f, _ in hg_batch_info._fields_}

    def plan(self, i):
        """Field i's plan, borrowed (counts, weight sums, neighbours, grid)."""
        h = ctypes.c_void_p()
        _check(lib().hg_batch_plan(self._handle(), int(i), ctypes.byref(h)), "hg_batch_plan")
        f = self.fields[i]
        return Plan._borrowed(h, f["map"], f["kernel"], f["n"], self)

    def close(self):
        if self._h:
            h, self._h = self._h, ctypes.c_void_p()
            _check(lib().hg_batch_destroy(h), "hg_batch_destroy")
            self._keep = []

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def ang2pix_ring(nside, ra_deg, dec_deg, stream=None):
    """HEALPix RING pixel of each direction, computed by the library on the GPU."""
    torch = _torch()
    ra, dec = _dev_f64(ra_deg), _dev_f64(dec_deg)
    pix = torch.empty(ra.shape[0], dtype=torch.int64, device=ra.device)
    rc = lib().hg_ang2pix_ring(int(nside), ctypes.c_void_p(ra.data_ptr()),
                               ctypes.c_void_p(dec.data_ptr()), ra.shape[0],
                               ctypes.c_void_p(pix.data_ptr()), _stream_ptr(stream))
    _check(rc, "hg_ang2pix_ring")
    return pix
