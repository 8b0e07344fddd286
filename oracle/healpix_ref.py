"""HEALPix RING-scheme reference in numpy -- TEST INFRASTRUCTURE ONLY.

Used only by the tests, to check the library's FP64 sky-cell binning (the
HEALPix partition of Sec. 4.1.1, step 1 of the pre-processing of Fig. 3).  It
is written from the geometry of the HEALPix paper (Gorski et al. 2005, cited
by the HEGrid paper in Sec. 4.1.1):

  * 12 * nside^2 equal-area pixels on 4*nside - 1 iso-latitude rings;
  * north cap, ring i < nside: 4i pixels at z = 1 - i^2 / (3 nside^2),
    azimuths (pi / 2i)(j - 1/2), j = 1..4i;
  * equatorial belt, nside <= i <= 3 nside: 4 nside pixels at
    z = 4/3 - 2i / (3 nside), azimuths (pi / 2 nside)(j - 1 + s/2) with
    s = (i - nside + 1) mod 2 (rings with s = 1 are offset by half a pixel,
    so that at nside = 1 the base pixels 4..7 sit at azimuths 0, pi/2, pi,
    3 pi/2 and pixels 0..3 at pi/4, 3 pi/4, ...);
  * south cap mirrors the north cap;
  * pixels are numbered ring by ring from the north pole, by increasing
    azimuth within a ring.

ang2pix inverts that layout by search, not by a closed formula: in the HEALPix
projection (Calabretta & Roukema 2007, "Mapping on the HEALPix grid") every
pixel is the same diamond about its projected centre, so the pixel holding a
point is its nearest centre in the L1 metric of that plane, found among a few
candidates from pix2ang.  The library's binning inverts the same layout by the
closed formula of its edge lines; the two share no steps.
"""
import numpy as np


def npix(nside):
    return 12 * nside * nside


def ring_info(nside, i):
    """(first pixel, pixel count, z of centres, shifted?) of ring i (1-based)."""
    n = nside
    if i < n:
        return 2 * i * (i - 1), 4 * i, 1.0 - i * i / (3.0 * n * n), True
    if i <= 3 * n:
        return (2 * n * (n - 1) + (i - n) * 4 * n, 4 * n, 4.0 / 3.0 - 2.0 * i / (3.0 * n),
                ((i - n + 1) % 2) == 1)
    k = 4 * n - i
    return npix(n) - 2 * k * (k + 1), 4 * k, -(1.0 - k * k / (3.0 * n * n)), True


def pix2ang(nside, pix):
    """Pixel centres (z = cos theta, phi in [0, 2 pi)) of RING pixels."""
    pix = np.asarray(pix, dtype=np.int64)
    n = nside
    ncap = 2 * n * (n - 1)
    z = np.empty(pix.shape, dtype=np.float64)
    phi = np.empty(pix.shape, dtype=np.float64)
    north = pix < ncap
    south = pix >= npix(n) - ncap
    belt = ~north & ~south
    if north.any():
        p = pix[north]
        i = np.floor(0.5 * (1.0 + np.sqrt(1.0 + 2.0 * p))).astype(np.int64)
        i = np.where(2 * i * (i - 1) > p, i - 1, i)  # guard the sqrt rounding
        i = np.where(2 * i * (i + 1) <= p, i + 1, i)
        j = p - 2 * i * (i - 1) + 1
        z[north] = 1.0 - i * i / (3.0 * n * n)
        phi[north] = (j - 0.5) * np.pi / (2.0 * i)
    if belt.any():
        p = pix[belt] - ncap
        i = p // (4 * n) + n
        j = p % (4 * n) + 1
        s = (i - n + 1) % 2
        z[belt] = 4.0 / 3.0 - 2.0 * i / (3.0 * n)
        phi[belt] = (j - 1 + 0.5 * s) * np.pi / (2.0 * n)
    if south.any():
        ps = npix(n) - 1 - pix[south]
        k = np.floor(0.5 * (1.0 + np.sqrt(1.0 + 2.0 * ps))).astype(np.int64)
        k = np.where(2 * k * (k - 1) > ps, k - 1, k)
        k = np.where(2 * k * (k + 1) <= ps, k + 1, k)
        first = npix(n) - 2 * k * (k + 1)
        j = pix[south] - first + 1
        z[south] = -(1.0 - k * k / (3.0 * n * n))
        phi[south] = (j - 0.5) * np.pi / (2.0 * k)
    return z, phi


def _project(nside, z, phi, quad):
    """HEALPix projection (Calabretta & Roukema 2007) in units where every
    pixel is the diamond |X - Xc| + |Y - Yc| <= 1/2: X = 2 nside x / pi,
    Y = 2 nside y / pi.  Belt (|z| <= 2/3): x = phi, y = (3 pi / 8) z.  Caps:
    sigma = sqrt(3 (1 - |z|)), x = phi_c + (phi - phi_c) sigma,
    y = +-(pi / 4)(2 - sigma), phi_c the centre of azimuth quadrant `quad`."""
    n = float(nside)
    za = np.abs(z)
    sig = np.sqrt(np.maximum(3.0 * (1.0 - za), 0.0))
    phic = (quad + 0.5) * (0.5 * np.pi)
    cap = za > 2.0 / 3.0
    x = np.where(cap, phic + (phi - phic) * sig, phi)
    y = np.where(cap, np.sign(z) * (0.25 * np.pi) * (2.0 - sig), (3.0 * np.pi / 8.0) * z)
    return x * (2.0 * n / np.pi), y * (2.0 * n / np.pi)


def ang2pix(nside, z, phi):
    """RING pixel containing the direction (z = cos theta, phi).

    Inverted by search rather than by a closed formula: in the HEALPix
    projection plane every pixel is a diamond of half-diagonal 1/2 about its
    projected centre, so the diamond lattice is the Voronoi partition of the
    centres in the L1 metric and the containing pixel is the L1-nearest
    centre.  Candidates are three rings about the point's projected Y (ring i
    sits at Y = nside - i/2) times three pixels about its azimuth in each
    ring, their centres taken from pix2ang (the layout).  A polar-cap chart
    holds only its own azimuth quadrant, so cap pixels of another quadrant
    than the point's are not candidates; a point's X distance wraps with
    period 4 nside."""
    n = nside
    z = np.asarray(z, dtype=np.float64).ravel()
    phi = np.mod(np.asarray(phi, dtype=np.float64).ravel(), 2.0 * np.pi)
    quad = np.minimum(np.floor(phi / (0.5 * np.pi)), 3.0)
    X, Y = _project(n, z, phi, quad)
    i0 = np.rint(2.0 * (n - Y)).astype(np.int64)
    best = np.full(z.shape, np.inf)
    out = np.full(z.shape, -1, dtype=np.int64)
    ncap = 2 * n * (n - 1)
    for di in (-1, 0, 1):
        i = np.clip(i0 + di, 1, 4 * n - 1)
        kk = np.minimum(np.minimum(i, 4 * n - i), n)  # pixels per ring / 4
        nr = 4 * kk
        first = np.where(i < n, 2 * i * (i - 1),
                         np.where(i <= 3 * n, ncap + (i - n) * 4 * n, npix(n) - 2 * kk * (kk + 1)))
        shift = np.where((i >= n) & (i <= 3 * n), (i - n + 1) % 2, 1)
        # pixel whose centre azimuth (k + shift/2) 2 pi / nr is nearest phi
        k0 = np.rint(phi * nr / (2.0 * np.pi) - 0.5 * shift).astype(np.int64)
        for dk in (-1, 0, 1):
            p = first + np.mod(k0 + dk, nr)
            zc, pc = pix2ang(n, p)
            qc = np.minimum(np.floor(pc / (0.5 * np.pi)), 3.0)
            cap_c = np.abs(zc) > 2.0 / 3.0 + 1e-15
            Xc, Yc = _project(n, zc, pc, quad)
            dX = np.mod(X - Xc + 2.0 * n, 4.0 * n) - 2.0 * n
            d = np.abs(dX) + np.abs(Y - Yc)
            d = np.where(cap_c & (qc != quad), np.inf, d)
            take = d < best
            best = np.where(take, d, best)
            out = np.where(take, p, out)
    return out


def ang2pix_radec(nside, ra_deg, dec_deg):
    dec = np.deg2rad(np.asarray(dec_deg, dtype=np.float64))
    ra = np.deg2rad(np.asarray(ra_deg, dtype=np.float64))
    return ang2pix(nside, np.sin(dec), ra)
