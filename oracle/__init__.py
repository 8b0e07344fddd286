"""FP64 reference gridder and HEALPix reference -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product path never does, and the
two share no code: this package holds a plain C gridder (``oracle.c``, built
with gcc into ``liboracle.so``) and a numpy HEALPix reference used only to
check the library's sky-cell binning.

The gridder follows the gather form of Eq. (1) (Sec. 2.2) with the inclusive
support test of Algorithm 1; see ``oracle.c`` for the readings taken where the
paper is silent.
"""
import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

F64, F32, BF16, F16 = 0, 1, 2, 3
_DTYPE_CODE = {"f64": F64, "f32": F32, "bf16": BF16, "f16": F16}


class _Map(ctypes.Structure):
    _fields_ = [
        ("ra0_deg", ctypes.c_double),
        ("dec0_deg", ctypes.c_double),
        ("dra_deg", ctypes.c_double),
        ("ddec_deg", ctypes.c_double),
        ("nx", ctypes.c_int32),
        ("ny", ctypes.c_int32),
        ("proj", ctypes.c_int32),
        ("nside", ctypes.c_int32),
        ("ring0", ctypes.c_int32),
        ("pix0", ctypes.c_int32),
    ]


def build(force=True):
    """Compile oracle.c with gcc (plain -O2, no contraction, no fast-math)."""
    if not force and os.path.exists(LIB):
        return LIB
    tmp = LIB + ".tmp"
    subprocess.check_call(
        ["gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
         SRC, "-o", tmp, "-lm"])
    os.replace(tmp, LIB)
    return LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        lib = ctypes.CDLL(LIB)
        P = ctypes.c_void_p
        i64, i32, f64 = ctypes.c_int64, ctypes.c_int32, ctypes.c_double
        lib.oracle_grid.argtypes = [i64, P, P, P, i32, i64, P, i64, ctypes.POINTER(_Map), f64, f64,
                                    i32, P, i64, P, P, P, P]
        lib.oracle_grid.restype = ctypes.c_int
        lib.oracle_neighbours.argtypes = [i64, P, P, ctypes.POINTER(_Map), f64, f64, i32, P, i64,
                                          P, P, P, i64, P]
        lib.oracle_neighbours.restype = ctypes.c_int
        lib.oracle_grid_k.argtypes = [i64, P, P, P, i32, i64, P, i64, ctypes.POINTER(_Map), f64,
                                      f64, i32, f64, f64, i32, P, i64, P, P, P, P]
        lib.oracle_grid_k.restype = ctypes.c_int
        lib.oracle_neighbours_k.argtypes = [i64, P, P, ctypes.POINTER(_Map), f64, f64, i32, f64,
                                            f64, i32, P, i64, P, P, P, i64, P]
        lib.oracle_neighbours_k.restype = ctypes.c_int
        lib.oracle_cell_centres.argtypes = [ctypes.POINTER(_Map), P, P, P]
        lib.oracle_cell_centres.restype = ctypes.c_int
        _lib = lib
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _mk_map(m):
    """A map dict: plate carree (ra0_deg, dec0_deg, dra_deg, ddec_deg, nx, ny)
    or, with proj = 1, a HEALPix patch (nside, ring0, pix0, nx, ny)."""
    if int(m.get("proj", 0)) == 1:
        return _Map(0.0, 0.0, 0.0, 0.0, int(m["nx"]), int(m["ny"]), 1, int(m["nside"]),
                    int(m["ring0"]), int(m["pix0"]))
    return _Map(float(m["ra0_deg"]), float(m["dec0_deg"]), float(m["dra_deg"]),
                float(m["ddec_deg"]), int(m["nx"]), int(m["ny"]), 0, 0, 0, 0)


def cell_centres(m):
    """(ra, dec) radians [ny*nx] of the map's cell centres and, for a HEALPix
    patch, the cells' RING numbers (else -1)."""
    lib = _load()
    mm = _mk_map(m)
    n = mm.nx * mm.ny
    ra, dec = np.empty(n), np.empty(n)
    ids = np.empty(n, dtype=np.int64)
    rc = lib.oracle_cell_centres(ctypes.byref(mm), _ptr(ra), _ptr(dec), _ptr(ids))
    if rc:
        raise ValueError(f"oracle_cell_centres failed ({rc})")
    return ra, dec, ids


def _coords(ra_deg, dec_deg):
    ra = np.ascontiguousarray(ra_deg, dtype=np.float64)
    dec = np.ascontiguousarray(dec_deg, dtype=np.float64)
    assert ra.shape == dec.shape and ra.ndim == 1
    return ra, dec


def _shape(kernel):
    """(type, p1, p2) of a kernel dict; the Gaussian when None or untyped."""
    if kernel is None:
        return 0, 0.0, 0.0
    return int(kernel.get("type", 0)), float(kernel.get("p1", 0.0)), float(kernel.get("p2", 0.0))


def grid(ra_deg, dec_deg, values, dtype, m, fwhm_deg, support_deg, chans=None, pix=None,
         brute=False, kernel=None):
    """Reference maps for the selected channels and cells.

    kernel: optional dict with "type" (0 Gaussian, 1 Gauss-tapered sinc, 2
    elliptical Gaussian) and its "p1", "p2" (see oracle.c); fwhm_deg and
    support_deg are passed separately as for the Gaussian.

    values: array [n][ld]; float64 / float32, or uint16 bit patterns for
    ``dtype`` 'bf16' / 'f16' (decoded exactly to FP64 inside the oracle).
    Returns (V [nchan][npix] float64, count [npix] int32, W [npix] float64,
    margin) where margin = min |h - h_R| / h_R over the pairs tested.
    """
    lib = _load()
    ra, dec = _coords(ra_deg, dec_deg)
    code = _DTYPE_CODE[dtype]
    vals = np.ascontiguousarray(values)
    want = {F64: np.float64, F32: np.float32, BF16: np.uint16, F16: np.uint16}[code]
    if vals.dtype != want:
        if code == F16 and vals.dtype == np.float16:
            vals = vals.view(np.uint16)
        else:
            raise TypeError(f"values dtype {vals.dtype} does not match '{dtype}'")
    if vals.ndim == 1:
        vals = vals.reshape(-1, 1)
    assert vals.shape[0] == ra.shape[0]
    ld = vals.shape[1]
    chans = np.arange(ld, dtype=np.int64) if chans is None else np.ascontiguousarray(
        chans, dtype=np.int64)
    npix_all = int(m["nx"]) * int(m["ny"])
    if pix is not None:
        pix = np.ascontiguousarray(pix, dtype=np.int64)
    npix = npix_all if pix is None else pix.shape[0]
    out = np.empty((chans.shape[0], npix), dtype=np.float64)
    count = np.empty(npix, dtype=np.int32)
    W = np.empty(npix, dtype=np.float64)
    margin = ctypes.c_double(0.0)
    mp = _mk_map(m)
    kt, p1, p2 = _shape(kernel)
    rc = lib.oracle_grid_k(ra.shape[0], _ptr(ra), _ptr(dec), _ptr(vals), code, ld, _ptr(chans),
                           chans.shape[0], ctypes.byref(mp), float(fwhm_deg), float(support_deg),
                           kt, p1, p2, int(bool(brute)), _ptr(pix), npix, _ptr(out),
                           _ptr(count), _ptr(W), ctypes.byref(margin))
    if rc != 0:
        raise ValueError(f"oracle_grid failed with status {rc}")
    return out, count, W, margin.value


def neighbours(ra_deg, dec_deg, m, fwhm_deg, support_deg, pix=None, brute=False, kernel=None):
    """CSR neighbour lists (ascending original index) and FP64 weights."""
    lib = _load()
    ra, dec = _coords(ra_deg, dec_deg)
    if pix is not None:
        pix = np.ascontiguousarray(pix, dtype=np.int64)
    npix = int(m["nx"]) * int(m["ny"]) if pix is None else pix.shape[0]
    row_ptr = np.zeros(npix + 1, dtype=np.int64)
    nnz = ctypes.c_int64(0)
    mp = _mk_map(m)
    kt, p1, p2 = _shape(kernel)
    args = (ra.shape[0], _ptr(ra), _ptr(dec), ctypes.byref(mp), float(fwhm_deg),
            float(support_deg), kt, p1, p2, int(bool(brute)), _ptr(pix), npix, _ptr(row_ptr))
    rc = lib.oracle_neighbours_k(*args, None, None, 0, ctypes.byref(nnz))
    if rc != 0:
        raise ValueError(f"oracle_neighbours failed with status {rc}")
    idx = np.empty(max(nnz.value, 1), dtype=np.int64)
    w = np.empty(max(nnz.value, 1), dtype=np.float64)
    rc = lib.oracle_neighbours_k(*args, _ptr(idx), _ptr(w), nnz.value, ctypes.byref(nnz))
    if rc != 0:
        raise ValueError(f"oracle_neighbours failed with status {rc}")
    return row_ptr, idx[:nnz.value], w[:nnz.value]
