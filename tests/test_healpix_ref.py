"""Pins of the numpy HEALPix reference (used to check the library's binning).

HEALPix facts from Gorski et al. (2005), the partition cited in Sec. 4.1.1:
12 nside^2 equal-area pixels on 4 nside - 1 iso-latitude rings, 4i pixels on
polar-cap ring i and 4 nside on each belt ring, and at nside = 1 the twelve
base pixels sit in three rings at z = 2/3, 0, -2/3.
"""
import numpy as np
import pytest

from oracle import healpix_ref as hp


@pytest.mark.parametrize("nside", [1, 2, 4, 16, 256])
def test_round_trip_all_pixels(nside):
    p = np.arange(hp.npix(nside))
    z, phi = hp.pix2ang(nside, p)
    np.testing.assert_array_equal(hp.ang2pix(nside, z, phi), p)


@pytest.mark.parametrize("nside", [1, 2, 8, 64])
def test_ring_sizes_and_latitudes(nside):
    p = np.arange(hp.npix(nside))
    z, _ = hp.pix2ang(nside, p)
    zs, counts = np.unique(np.round(z, 12), return_counts=True)
    zs, counts = zs[::-1], counts[::-1]  # north to south
    assert zs.shape[0] == 4 * nside - 1
    want = [4 * min(i, nside, 4 * nside - i) for i in range(1, 4 * nside)]
    np.testing.assert_array_equal(counts, want)
    for i in range(1, 4 * nside):
        first, n, zc, _ = hp.ring_info(nside, i)
        assert n == want[i - 1]
        assert zc == pytest.approx(zs[i - 1], abs=1e-12)
        zz, _ = hp.pix2ang(nside, np.arange(first, first + n))
        assert np.allclose(zz, zc)


def test_base_pixels():
    z, phi = hp.pix2ang(1, np.arange(12))
    np.testing.assert_allclose(z, [2 / 3] * 4 + [0] * 4 + [-2 / 3] * 4, atol=1e-15)
    q = np.pi / 4
    np.testing.assert_allclose(phi, [q, 3 * q, 5 * q, 7 * q, 0, 2 * q, 4 * q, 6 * q,
                                     q, 3 * q, 5 * q, 7 * q], atol=1e-15)


@pytest.mark.parametrize("nside", [4, 32])
def test_equal_area(nside):
    rng = np.random.default_rng(nside)
    n = 600 * hp.npix(nside) if nside == 4 else 60 * hp.npix(nside)
    z = rng.uniform(-1, 1, n)  # uniform on the sphere
    phi = rng.uniform(0, 2 * np.pi, n)
    counts = np.bincount(hp.ang2pix(nside, z, phi), minlength=hp.npix(nside))
    e = n / hp.npix(nside)
    chi2 = np.sum((counts - e) ** 2 / e)
    dof = hp.npix(nside) - 1
    assert abs(chi2 - dof) < 5 * np.sqrt(2 * dof)


@pytest.mark.parametrize("nside", [8, 1024])
def test_points_land_in_the_nearest_pixel_region(nside):
    rng = np.random.default_rng(3)
    z = rng.uniform(-1, 1, 20000)
    phi = rng.uniform(0, 2 * np.pi, 20000)
    pix = hp.ang2pix(nside, z, phi)
    zc, pc = hp.pix2ang(nside, pix)
    # angular distance to the assigned centre stays within the largest pixel radius
    cosd = z * zc + np.sqrt(1 - z * z) * np.sqrt(1 - zc * zc) * np.cos(phi - pc)
    d = np.arccos(np.clip(cosd, -1, 1))
    assert d.max() < 1.5 * np.sqrt(4 * np.pi / hp.npix(nside))
