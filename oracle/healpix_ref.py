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

ang2pix inverts that layout: in the belt the pixel edges are the lines
nside (phi / (pi/2) + 1/2) -+ (3/4) nside z = const, in the caps the edges are
the curves of constant  nside sqrt(3 (1 - |z|)) * t  and
nside sqrt(3 (1 - |z|)) * (1 - t), t the azimuth fraction inside a base pixel.
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


def ang2pix(nside, z, phi):
    """RING pixel containing the direction (z = cos theta, phi)."""
    n = nside
    z = np.asarray(z, dtype=np.float64)
    phi = np.mod(np.asarray(phi, dtype=np.float64), 2.0 * np.pi)
    tt = phi / (0.5 * np.pi)  # in [0, 4)
    tt = np.where(tt >= 4.0, 0.0, tt)
    za = np.abs(z)
    out = np.empty(z.shape, dtype=np.int64)

    belt = za <= 2.0 / 3.0
    if belt.any():
        t1 = n * (0.5 + tt[belt])
        t2 = n * z[belt] * 0.75
        jp = np.floor(t1 - t2).astype(np.int64)  # ascending edge index
        jm = np.floor(t1 + t2).astype(np.int64)  # descending edge index
        ir = n + 1 + jp - jm  # 1 .. 2n+1, counted from the z = 2/3 ring
        kshift = 1 - (ir & 1)
        ip = (jp + jm - n + kshift + 1) // 2
        ip = np.mod(ip, 4 * n)
        out[belt] = 2 * n * (n - 1) + (ir - 1) * 4 * n + ip

    cap = ~belt
    if cap.any():
        tc = tt[cap]
        tp = tc - np.floor(tc)
        tmp = n * np.sqrt(3.0 * (1.0 - za[cap]))
        jp = np.floor(tp * tmp).astype(np.int64)
        jm = np.floor((1.0 - tp) * tmp).astype(np.int64)
        ir = jp + jm + 1  # ring counted from the nearer pole
        ip = np.floor(tc * ir).astype(np.int64)
        ip = np.mod(ip, 4 * ir)
        out[cap] = np.where(z[cap] > 0, 2 * ir * (ir - 1) + ip, npix(n) - 2 * ir * (ir + 1) + ip)
    return out


def ang2pix_radec(nside, ra_deg, dec_deg):
    dec = np.deg2rad(np.asarray(dec_deg, dtype=np.float64))
    ra = np.deg2rad(np.asarray(ra_deg, dtype=np.float64))
    return ang2pix(nside, np.sin(dec), ra)
