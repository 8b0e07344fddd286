"""Seeded synthetic single-dish observations (inputs only).

This module draws sample positions and sky values; it holds none of the
gridding arithmetic, and both the library's tests and the reference gridder's
tests take their inputs from it.  The paper's own data (a simulated HDF5 set
and FAST drift scans, Table 2 of Sec. 5.1.2) are not available; these
generators stand in for them with the shapes the paper describes: a 3 arcmin
(180 arcsec) beam, drift scans along RA (Sec. 2.1), many independent channels
(Sec. 1) and hundreds of neighbours per cell.

Coordinates are drawn with numpy (PCG64 from SeedSequence([220704584, k]),
k = workload number) and are identical everywhere.  Values are drawn with
torch on the requested device from a generator seeded from the same
sequence; CPU and GPU draws differ, so a test hands the same tensor to both
sides.
"""
import math

import numpy as np

ROOT_SEED = 220704584
ARCMIN = 1.0 / 60.0
FWHM_TO_SIGMA = 1.0 / math.sqrt(8.0 * math.log(2.0))


def _rng(*key):
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([ROOT_SEED, *key])))


def _torch_seed(*key):
    return int(np.random.SeedSequence([ROOT_SEED, *key]).generate_state(1, np.uint64)[0] >> 1)


def make_map(ra0, dec0, nx, ny, pix_arcmin=1.0):
    return {"ra0_deg": float(ra0), "dec0_deg": float(dec0), "dra_deg": pix_arcmin * ARCMIN,
            "ddec_deg": pix_arcmin * ARCMIN, "nx": int(nx), "ny": int(ny)}


def healpix_patch(ra0, dec0, width_deg, height_deg, nside):
    """A HEALPix target map over a width x height box around (ra0, dec0), in
    the equatorial belt: the rings whose centres' z = 4/3 - 2r/(3 nside) fall
    in the box's Dec range (rows run south to north, so ring0 is the southern
    one) and, in each ring, the pixels over its RA range (spacing 360/(4 nside)
    deg).  The map dict the library and the reference gridder take."""
    z_lo = math.sin(math.radians(dec0 - 0.5 * height_deg))
    z_hi = math.sin(math.radians(dec0 + 0.5 * height_deg))
    r_north = math.ceil((4.0 / 3.0 - z_hi) * 1.5 * nside)
    r_south = math.floor((4.0 / 3.0 - z_lo) * 1.5 * nside)
    dphi = 360.0 / (4 * nside)
    return {"proj": 1, "nside": int(nside), "ring0": int(r_south),
            "pix0": int(math.floor((ra0 - 0.5 * width_deg) / dphi)) % (4 * nside),
            "nx": int(round(width_deg / dphi)), "ny": int(r_south - r_north + 1)}


def make_kernel(fwhm_arcmin, support_sigmas=3.0):
    fwhm = fwhm_arcmin * ARCMIN
    return {"fwhm_deg": fwhm, "support_deg": support_sigmas * fwhm * FWHM_TO_SIGMA}


def uniform_coords(rng, n, ra0, dec0, width_deg, height_deg):
    """Samples uniform in coordinates over a width x height box."""
    ra = ra0 + (rng.random(n) - 0.5) * width_deg
    dec = dec0 + (rng.random(n) - 0.5) * height_deg
    return ra, dec


def drift_scan_coords(rng, n_lines, per_line, ra0, dec0, width_deg, height_deg,
                      spacing_arcmin=0.5, jitter_arcmin=0.2, line_decs=None):
    """Constant-Dec drift-scan tracks (Sec. 2.1), repeated passes across the
    field, each pass with a random phase, plus on-sky Gaussian jitter."""
    if line_decs is None:
        step = height_deg / n_lines
        line_decs = dec0 - 0.5 * height_deg + (np.arange(n_lines) + 0.5) * step
    ras, decs = [], []
    for dl in line_decs:
        dra = spacing_arcmin * ARCMIN / math.cos(math.radians(dl))
        per_pass = max(1, int(width_deg / dra))
        got = 0
        while got < per_line:
            m = min(per_pass, per_line - got)
            phase = rng.random() * dra
            ras.append(ra0 - 0.5 * width_deg + phase + np.arange(m) * dra)
            decs.append(np.full(m, dl))
            got += m
    ra = np.concatenate(ras)
    dec = np.concatenate(decs)
    jit = jitter_arcmin * ARCMIN
    dec = dec + rng.normal(0.0, jit, dec.shape[0])
    ra = ra + rng.normal(0.0, jit, ra.shape[0]) / np.cos(np.deg2rad(dec))
    return ra, dec


def hex19_track_decs(rng, dec0, height_deg, mean_spacing_arcmin=0.72, rot_deg=23.4):
    """Track declinations of repeated drifts of a 19-beam hexagonal receiver
    rotated by 23.4 degrees (Sec. 2.1): the beams' Dec offsets per drift, with
    successive drifts offset in Dec so the tracks interleave over the field."""
    q, r = np.meshgrid(np.arange(-2, 3), np.arange(-2, 3))
    keep = np.maximum(np.maximum(np.abs(q), np.abs(r)), np.abs(q + r)) <= 2
    q, r = q[keep].astype(float), r[keep].astype(float)
    y = r * math.sqrt(3.0) / 2.0  # axial hex coordinates -> unit-spacing plane
    x = q + r / 2.0
    a = math.radians(rot_deg)
    offs = np.sort(x * math.sin(a) + y * math.cos(a))  # Dec offsets, beam units
    span = offs[-1] - offs[0]
    beam = mean_spacing_arcmin * 19.0 / span  # beam spacing (arcmin) for the mean
    drift = span * beam * ARCMIN  # Dec advance per drift
    n_drift = int(math.ceil(height_deg / drift)) + 1
    start = dec0 - 0.5 * height_deg + rng.random() * drift - drift
    decs = (start + np.arange(n_drift)[:, None] * drift + offs[None, :] * beam * ARCMIN).ravel()
    lo, hi = dec0 - 0.5 * height_deg, dec0 + 0.5 * height_deg
    return np.sort(decs[(decs >= lo) & (decs <= hi)])


def _unit(ra_deg, dec_deg, xp):
    a = xp.deg2rad(ra_deg)
    d = xp.deg2rad(dec_deg)
    return xp.stack([xp.cos(d) * xp.cos(a), xp.cos(d) * xp.sin(a), xp.sin(d)], -1)


def _torch():
    import torch
    return torch


def sky_values(field, nchan, device="cpu", dtype="f32", chan_lo=0, chan_hi=None, block_key=0):
    """Values [n][chan_hi - chan_lo] of the sky model of ``field``.

    recipe 'points': sum of point sources (amplitude U(1,10), spatial FWHM
      3 arcmin) plus N(0, noise) -- one continuum channel per source draw;
    recipe 'spectral': smooth continuum 5 (1 + 0.5 sin(2 pi x / 2deg)
      cos(2 pi y / 2deg)) (1 + 0.2 (c/C - 1/2)) plus line sources (A ~ U(1,10),
      spatial FWHM 3 arcmin, centre channel U(0, C), spectral sigma U(2, 20)
      channels) plus N(0, noise).
    Channels [chan_lo, chan_hi) of a C = nchan cube are produced, so a cube
    can be generated block by block.  Returns a torch tensor of dtype
    float32 / bfloat16 / float16 on ``device``.
    """
    torch = _torch()
    chan_hi = nchan if chan_hi is None else chan_hi
    nb = chan_hi - chan_lo
    key = field["key"]
    rng = _rng(*key, 1)  # sources: fixed per field, independent of the block
    ra = torch.as_tensor(field["ra"], dtype=torch.float64, device=device)
    dec = torch.as_tensor(field["dec"], dtype=torch.float64, device=device)
    n = ra.shape[0]
    recipe = field["recipe"]
    box = field["box"]  # (ra0, dec0, width, height) of the source region
    sig_src = 3.0 * ARCMIN * FWHM_TO_SIGMA
    n_src = field["n_sources"]
    s_ra, s_dec = uniform_coords(rng, n_src, *box)
    amp = rng.uniform(1.0, 10.0, n_src)
    c0 = rng.uniform(0.0, nchan, n_src)
    sc = rng.uniform(2.0, 20.0, n_src)
    u = _unit(ra, dec, torch)
    us = _unit(torch.as_tensor(s_ra, device=device), torch.as_tensor(s_dec, device=device), torch)
    # chord -> angle, degrees; [n][n_src]
    chord = torch.cdist(u, us)
    dist = torch.rad2deg(2.0 * torch.asin(torch.clamp(chord * 0.5, max=1.0)))
    spatial = torch.exp(-0.5 * (dist / sig_src) ** 2).to(torch.float32)
    del chord, dist
    chans = torch.arange(chan_lo, chan_hi, dtype=torch.float64, device=device)
    if recipe == "points":
        vals = (spatial * torch.as_tensor(amp, dtype=torch.float32, device=device)).sum(
            1, keepdim=True).expand(n, nb).contiguous()
    elif recipe == "spectral":
        line = torch.exp(-0.5 * ((chans[None, :] - torch.as_tensor(c0, device=device)[:, None]) /
                                 torch.as_tensor(sc, device=device)[:, None]) ** 2)
        line = (line * torch.as_tensor(amp, device=device)[:, None]).to(torch.float32)
        vals = spatial @ line  # [n][nb]
        x = (ra - box[0]) * math.cos(math.radians(box[1]))
        y = dec - box[1]
        cont = 5.0 * (1.0 + 0.5 * torch.sin(2 * math.pi * x / 2.0) * torch.cos(2 * math.pi * y / 2.0))
        tilt = 1.0 + 0.2 * (chans / nchan - 0.5)
        vals += cont.to(torch.float32)[:, None] * tilt.to(torch.float32)[None, :]
    else:
        raise ValueError(recipe)
    del spatial
    g = torch.Generator(device=device)
    g.manual_seed(_torch_seed(*key, 2, block_key, chan_lo))
    vals += field["noise"] * torch.randn(vals.shape, generator=g, device=device,
                                         dtype=torch.float32)
    tdt = {"f32": torch.float32, "bf16": torch.bfloat16, "f16": torch.float16}[dtype]
    return vals.to(tdt)


def _field(key, ra, dec, m, k, recipe, n_sources, noise, box, nchan, dtype):
    return {"key": tuple(key), "ra": ra, "dec": dec, "map": m, "kernel": k, "recipe": recipe,
            "n_sources": n_sources, "noise": noise, "box": box, "nchan": nchan, "dtype": dtype}


def uniform_field(key, n, ra0, dec0, width, height, nx, ny, fwhm_arcmin=3.0, nchan=1,
                  dtype="f32", recipe="spectral", n_sources=5, noise=1.0, pix_arcmin=1.0):
    rng = _rng(*key, 0)
    ra, dec = uniform_coords(rng, n, ra0, dec0, width, height)
    return _field(key, ra, dec, make_map(ra0, dec0, nx, ny, pix_arcmin), make_kernel(fwhm_arcmin),
                  recipe, n_sources, noise, (ra0, dec0, width, height), nchan, dtype)


def config(name):
    """The five seeded workloads (geometry and value recipe; values are drawn
    separately with sky_values)."""
    if name == "cfg1":  # plain method, 1 channel
        return uniform_field((1,), 20000, 180.0, 30.0, 1.0, 1.0, 64, 64, nchan=1,
                             recipe="points", n_sources=5, noise=0.1)
    if name == "cfg2":  # plain FP32, 1024 channels, 40-line drift scan
        rng = _rng(2, 0)
        ra, dec = drift_scan_coords(rng, 40, 25000, 180.0, 30.0, 5.0, 5.0)
        return _field((2,), ra, dec, make_map(180.0, 30.0, 300, 300), make_kernel(3.0),
                      "spectral", 20, 1.0, (180.0, 30.0, 5.0, 5.0), 1024, "f32")
    if name == "cfg3":  # precision form: cfg1 geometry, 8192 BF16 channels
        f = uniform_field((1,), 20000, 180.0, 30.0, 1.0, 1.0, 64, 64, nchan=8192, dtype="bf16",
                          recipe="spectral", n_sources=20, noise=1.0)
        f["key"] = (3,)
        return f
    if name == "cfg5":  # 19-beam drift scan, 65,536 BF16 channels
        rng = _rng(5, 0)
        decs = hex19_track_decs(rng, 30.0, 10.0)
        per = int(math.ceil(1_000_000 / decs.shape[0]))
        ra, dec = drift_scan_coords(rng, decs.shape[0], per, 180.0, 30.0, 10.0, 10.0,
                                    line_decs=decs)
        ra, dec = ra[:1_000_000], dec[:1_000_000]
        return _field((5,), ra, dec, make_map(180.0, 30.0, 600, 600), make_kernel(3.0),
                      "spectral", 200, 1.0, (180.0, 30.0, 10.0, 10.0), 65536, "bf16")
    if name == "paper":
        return paper_field()
    raise KeyError(name)


def paper_field(n=19_000_000, width=60.0, height=20.0, ra0=30.0, dec0=41.0, nchan=50):
    """Stand-in for the paper's simulated set (Table 2 of Sec. 5.1.2): a
    60 x 20 deg map centred on (30, 41) deg, a 180 arcsec beam, 1.5e7 to
    1.9e7 samples and 50 channels, here from repeated drifts of a 19-beam
    receiver (as cfg5) at 1 arcmin pixels (a third of the beam).  Smaller
    ``width``/``height``/``n`` give the same recipe on a sub-field: the
    samples per track and the track spacing follow from n and height."""
    rng = _rng(6, 0)
    decs = hex19_track_decs(rng, dec0, height)
    per = int(math.ceil(n / decs.shape[0]))
    ra, dec = drift_scan_coords(rng, decs.shape[0], per, ra0, dec0, width, height,
                                line_decs=decs)
    ra, dec = np.mod(ra[:n], 360.0), dec[:n]
    nx, ny = int(round(width * 60.0)), int(round(height * 60.0))
    return _field((6,), ra, dec, make_map(ra0, dec0, nx, ny), make_kernel(3.0), "spectral", 20,
                  1.0, (ra0, dec0, width, height), nchan, "f32")


def batch_fields(n_fields=64, scale=1.0):
    """The batching workload: fields of log-uniform sample counts (1e4..2e6),
    square maps of side {32..512} at 1 arcmin, channels {256, 1024, 4096},
    FWHM U(2, 5) arcmin, FP16 values.  ``scale`` < 1 shrinks sample counts and
    channels for quick tests."""
    rng = _rng(4, 0)
    fields = []
    for f in range(n_fields):
        n = int(round(math.exp(rng.uniform(math.log(1e4), math.log(2e6))) * scale))
        side = int(rng.choice([32, 64, 128, 256, 512]))
        nchan = int(rng.choice([256, 1024, 4096]))
        fwhm = float(rng.uniform(2.0, 5.0))
        ra0 = float(rng.uniform(30.0, 330.0))
        dec0 = float(rng.uniform(-60.0, 60.0))
        width = side * ARCMIN
        if scale < 1.0:
            nchan = max(8, int(nchan * scale))
            n = max(100, n)
        fl = uniform_field((4, f), n, ra0, dec0, width, width, side, side, fwhm_arcmin=fwhm,
                           nchan=nchan, dtype="f16", recipe="spectral", n_sources=20, noise=1.0)
        fields.append(fl)
    return fields


_HIP = None


def pinned_empty(shape, dtype):
    """An uninitialised page-locked host tensor of exactly the requested size,
    for the host-memory cubes of the streamed workloads.  torch's pinned
    allocator rounds every request up to a power of two (a 33 GB slab takes
    64 GB), so the buffer comes from hipHostMalloc instead and is released
    with hipHostFree when the tensor's storage goes."""
    import ctypes
    import weakref
    torch = _torch()
    global _HIP
    if _HIP is None:
        _HIP = ctypes.CDLL("libamdhip64.so")
        _HIP.hipHostMalloc.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_size_t,
                                       ctypes.c_uint]
        _HIP.hipHostFree.argtypes = [ctypes.c_void_p]
    nbytes = int(np.prod(shape)) * torch.empty((), dtype=dtype).element_size()
    ptr = ctypes.c_void_p()
    rc = _HIP.hipHostMalloc(ctypes.byref(ptr), max(nbytes, 1), 0)
    if rc != 0 or not ptr.value:
        raise MemoryError(f"hipHostMalloc of {nbytes} bytes failed (status {rc})")
    buf = (ctypes.c_uint8 * max(nbytes, 1)).from_address(ptr.value)
    weakref.finalize(buf, _HIP.hipHostFree, ptr.value)
    t = torch.frombuffer(buf, dtype=torch.uint8)[:nbytes]
    return t.view(dtype).reshape(shape)
