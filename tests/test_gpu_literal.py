"""GPU tests of the Algorithm 1 comparison path (hg_grid_channels_literal):
one launch per channel, one thread per gamma cells of a 2x2 pixel group,
FP64 distances, weights and sums.  Its maps must match the FP64 reference
to FP32 rounding (the sums are FP64; only the store rounds), for every
gamma and several workgroup sizes, with NaN exactly where a cell has no
neighbour; and match the tiled FP32 path within that path's 1e-6.
"""
import numpy as np
import pytest

import oracle
from paper_2207_04584_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2207_04584_amd import api  # noqa: E402
from parity_util import norm_err  # noqa: E402

DEV = "cuda:0"
ARC = 1.0 / 60.0


def field(seed=11, n=4000, nx=37, ny=29, ra0=150.0, dec0=-20.0, C=6, spread=1.4):
    """Samples over the map except its left third, which is left empty."""
    rng = np.random.default_rng(seed)
    ra = ra0 + (rng.random(n) - 0.5) * nx * ARC * spread
    dec = dec0 + (rng.random(n) - 0.5) * ny * ARC * spread
    keep = ra > ra0 - nx * ARC / 6.0
    ra, dec = ra[keep], dec[keep]
    n = ra.shape[0]
    vals = torch.from_numpy(rng.normal(1.0, 1.0, size=(n, C)).astype(np.float32)).to(DEV)
    return ra, dec, vals, synth.make_map(ra0, dec0, nx, ny), synth.make_kernel(3.0)


@pytest.mark.parametrize("gamma,block", [(1, 64), (1, 256), (2, 128), (2, 1024), (4, 256),
                                         (4, 64)])
def test_literal_matches_reference(gamma, block):
    ra, dec, vals, m, k = field()
    with api.Plan(ra, dec, m, k) as p:
        lit = p.grid_literal(vals, gamma=gamma, block=block).cpu().numpy()
        tiled = p.grid(vals).cpu().numpy()
    C = vals.shape[1]
    Vr, cr, _, margin = oracle.grid(ra, dec, vals.cpu().numpy(), "f32", m, k["fwhm_deg"],
                                    k["support_deg"])
    assert margin > 1e-12
    V = lit.reshape(C, -1)
    np.testing.assert_array_equal(np.isnan(V), np.isnan(Vr))
    assert np.isnan(V).any() and not np.isnan(V).all()  # the field leaves some cells empty
    ok = cr > 0
    # FP64 sums: the only rounding is the store to FP32
    np.testing.assert_allclose(V[:, ok], Vr[:, ok], rtol=1.2e-7, atol=1e-12)
    e_max, _ = norm_err(tiled.reshape(C, -1), V, ok)
    assert e_max <= 1e-6


def test_literal_ragged_and_strided_channels():
    ra, dec, vals, m, k = field(seed=12, n=1500, nx=9, ny=5, C=9)
    view = vals[:, 2:7]  # five channels, rows of nine
    with api.Plan(ra, dec, m, k) as p:
        lit = p.grid_literal(view, gamma=4, block=64).cpu().numpy()
    Vr, cr, _, _ = oracle.grid(ra, dec, vals.cpu().numpy(), "f32", m, k["fwhm_deg"],
                               k["support_deg"], chans=np.arange(2, 7))
    V = lit.reshape(5, -1)
    np.testing.assert_array_equal(np.isnan(V), np.isnan(Vr))
    ok = cr > 0
    np.testing.assert_allclose(V[:, ok], Vr[:, ok], rtol=1.2e-7, atol=1e-12)
