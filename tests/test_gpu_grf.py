"""GPU parity of the random field of SaltSDT (Alg. 4, sg_grf): the
hand-written FP32 FFTs against the FP64 oracle (NumPy FFTs) on the same
white noise, relative L2 <= 1e-4, on ragged, 2D, single-axis and
power-of-two volumes, isotropic, anisotropic and zero correlation lengths;
and the salt stage fed with GPU fields equals the oracle's on those fields."""
import os

import numpy as np
import pytest

from oracle import builder as OB
from paper_2605_30541_amd import sgwave

pytestmark = pytest.mark.gpu
TOL = 1e-4


def rel_l2(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / np.linalg.norm(b))


def _noise(shape, seed):
    grid, _ = sgwave.grf_grid(*shape)
    return np.random.default_rng(seed).standard_normal(grid).astype(np.float32)


@pytest.mark.parametrize("shape,ell,p", [((37, 50, 27), (3.0, 5.0, 2.5), 2.0), ((20, 33, 12), (0.0, 0.0, 0.0), 1.0),
                                         ((64, 64, 64), (9.0, 4.0, 12.0), 1.5), ((1, 300, 517), (0.0, 20.0, 35.0), 2.5),
                                         ((1, 1, 1000), (0.0, 0.0, 7.0), 3.0), ((129, 7, 65), (5.0, 5.0, 5.0), 1.2),
                                         ((200, 300, 250), (15.0, 25.0, 40.0), 2.0)])
def test_grf_matches_the_oracle(shape, ell, p):
    import torch
    noise = _noise(shape, sum(shape))
    got = sgwave.grf(torch.from_numpy(noise).cuda(), shape, ell, p).cpu().numpy()
    ref = OB.grf(noise.astype(np.float64), shape, ell, p)
    e = rel_l2(got, ref)
    print("%s ell %s p %.1f: rel-L2 %.2e, mean %.1e, std %.6f" % (shape, ell, p, e, got.mean(), got.std()), flush=True)
    assert e <= TOL
    assert abs(float(got.astype(np.float64).mean())) < 1e-5 and abs(float(got.astype(np.float64).std()) - 1.0) < 1e-5


def test_grf_of_one_cell_is_zero():
    import torch
    got = sgwave.grf(torch.from_numpy(_noise((1, 1, 1), 3)).cuda(), (1, 1, 1), (5.0, 5.0, 5.0), 2.0)
    assert float(got.abs().max()) == 0.0


def test_salt_bodies_with_sampled_fields_equal_the_oracle():
    """Two bodies whose fields come from sg_grf (l_k = max(r_k f, 5) cells):
    the salted volume and mask equal the oracle's SaltSDT run on the same
    fields bit for bit, and each field is within 1e-4 of the oracle's."""
    import torch
    nz, ny, nx, h = 48, 40, 56, 10.0
    V = (1500.0 + 25.0 * np.arange(nz)[:, None, None] + np.zeros((1, ny, nx))).astype(np.float32)
    centres = np.array([[220.0, 200.0, 250.0], [300.0, 120.0, 400.0]])
    radii = np.array([[120.0, 90.0, 150.0], [80.0, 70.0, 60.0]])
    rots = np.stack([np.eye(3), np.array([[0.8, -0.6, 0.0], [0.6, 0.8, 0.0], [0.0, 0.0, 1.0]])])
    fields, refs = [], []
    for i in range(2):
        ell = tuple(max(r / h * 0.25, 5.0) for r in radii[i])
        noise = _noise((nz, ny, nx), 100 + i)
        fields.append(sgwave.grf(torch.from_numpy(noise).cuda(), (nz, ny, nx), ell, 2.0))
        refs.append(OB.grf(noise.astype(np.float64), (nz, ny, nx), ell, 2.0))
    grf = torch.stack(fields).contiguous()
    for i in range(2):
        assert rel_l2(grf[i].cpu().numpy(), refs[i]) <= TOL
    out, mask = sgwave.salt_sdt(torch.from_numpy(V).cuda(), h, h, h, centres, radii, rots, grf, 0.3, 4500.0, 1500.0, 50)
    ref_v, ref_k = OB.salt_sdt(V.astype(np.float64), h, h, h, centres, radii, rots,
                               grf.cpu().numpy().astype(np.float64), 0.3, 4500.0, 1500.0, 50)
    assert np.array_equal(mask.cpu().numpy().astype(bool), ref_k)
    assert np.array_equal(out.cpu().numpy(), ref_v.astype(np.float32))
    assert ref_k.sum() > 1000
