"""GPU parity of SaltSDT (Alg. 4) with the FP64 oracle on the same float32
inputs: the salt mask K and the output volume must match exactly (every
decision is an FP64 comparison on both sides).  Cases: rotated ellipsoids
under a smooth random field on an anisotropic grid, a water layer and a
small-component cut, a noisy field that leaves many components, empty and
covering bodies, no bodies, 2D slices, tiny ragged volumes and rows wider
than one workgroup."""
import numpy as np
import pytest

from oracle import builder as OB
from paper_2605_30541_amd import sgwave

pytestmark = pytest.mark.gpu


def _dev(a, dtype=np.float32):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype)).cuda()


def _rot(a, b, c):
    """Rotation from three angles (radians) about z, y and x."""
    ca, sa, cb, sb, cc, sc = np.cos(a), np.sin(a), np.cos(b), np.sin(b), np.cos(c), np.sin(c)
    Rz = np.array([[1, 0, 0], [0, ca, -sa], [0, sa, ca]])
    Ry = np.array([[cb, 0, sb], [0, 1, 0], [-sb, 0, cb]])
    Rx = np.array([[cc, -sc, 0], [sc, cc, 0], [0, 0, 1]])
    return Rz @ Ry @ Rx


def _field(nb, shape, sigma, seed):
    from scipy.ndimage import gaussian_filter
    rng = np.random.default_rng(seed)
    out = np.empty((nb,) + shape, np.float32)
    for i in range(nb):
        g = gaussian_filter(rng.standard_normal(shape), sigma, mode="wrap")
        out[i] = g / g.std()
    return out


def _model(shape, seed):
    nz, ny, nx = shape
    rng = np.random.default_rng(seed)
    z = np.arange(nz)[:, None, None]
    V = 1500.0 + 40.0 * z + rng.normal(0, 20.0, shape)
    V[:3] = 1500.0
    return np.broadcast_to(V, shape).astype(np.float32)


def _run(V, h, centres, radii, rots, grf, amp, v_salt, v_water, minv):
    got, mask = sgwave.salt_sdt(_dev(V), *h, centres, radii, rots, _dev(grf) if len(centres) else None,
                                        amp, v_salt, v_water, minv)
    import torch
    torch.cuda.synchronize()
    ref, K = OB.salt_sdt(V.astype(np.float64), *h, centres, radii, rots, grf.astype(np.float64), amp, v_salt,
                         v_water, minv)
    return got.cpu().numpy(), mask.cpu().numpy().astype(bool), ref, K


def _report(name, mask, K):
    print("%s: %d salt voxels, %d mismatched" % (name, K.sum(), (mask != K).sum()), flush=True)


@pytest.mark.parametrize("shape,h", [((40, 36, 44), (10.0, 12.5, 8.0)), ((33, 50, 27), (8.0, 8.0, 8.0))])
def test_salt_bodies_under_a_random_field_match_the_oracle(shape, h):
    nz, ny, nx = shape
    ext = np.array(shape) * np.array(h)
    centres = [ext * (0.45, 0.4, 0.5), ext * (0.7, 0.75, 0.3), ext * (0.2, 0.2, 0.8)]
    radii = [ext * (0.25, 0.3, 0.2), ext * (0.15, 0.1, 0.2), ext * (0.06, 0.07, 0.06)]
    rots = [_rot(0.3, -0.5, 1.1), _rot(-1.2, 0.2, 0.4), np.eye(3)]
    grf = _field(3, shape, 3.0, nz)
    V = _model(shape, ny)
    minv = 150
    got, mask, ref, K = _run(V, h, centres, radii, rots, grf, 0.15, 4500.0, 1600.0, minv)
    _report("bodies %s" % (shape,), mask, K)
    assert 0 < K.sum() < K.size
    assert np.array_equal(mask, K)
    assert np.array_equal(got, ref.astype(np.float32))
    # the small-component cut and the water limit both act on this case
    _, K1 = OB.salt_sdt(V.astype(np.float64), *h, centres, radii, rots, grf.astype(np.float64), 0.15, 4500.0,
                        0.0, 1)
    assert K1.sum() > K.sum()


def test_noisy_field_with_many_components_matches_the_oracle():
    shape, h = (30, 34, 38), (10.0, 10.0, 10.0)
    grf = _field(1, shape, 1.2, 5)
    V = _model(shape, 6)
    c, r = [(150.0, 170.0, 190.0)], [(120.0, 140.0, 150.0)]
    for minv in (1, 40):
        got, mask, ref, K = _run(V, h, c, r, [_rot(0.2, 0.1, -0.3)], grf, 0.9, 4400.0, 0.0, minv)
        from scipy.ndimage import label, generate_binary_structure
        ncomp = label(K, structure=generate_binary_structure(3, 1))[1]
        _report("noisy, min %d (%d components)" % (minv, ncomp), mask, K)
        assert ncomp >= (5 if minv == 1 else 1)
        assert np.array_equal(mask, K)
        assert np.array_equal(got, ref.astype(np.float32))


def test_empty_covering_and_no_bodies():
    shape, h = (20, 18, 22), (10.0, 10.0, 10.0)
    V = _model(shape, 1)
    grf = _field(2, shape, 2.0, 2)
    # a body outside the model adds nothing; one covering it salts all below the water
    got, mask, ref, K = _run(V, h, [(5000.0, 5000.0, 5000.0), (100.0, 90.0, 110.0)],
                                [(100.0, 100.0, 100.0), (60.0, 50.0, 70.0)], [np.eye(3)] * 2, grf, 0.2, 4500.0,
                                1600.0, 10)
    assert np.array_equal(mask, K) and np.array_equal(got, ref.astype(np.float32))
    got, mask, ref, K = _run(V, h, [(100.0, 90.0, 110.0)], [(1e5, 1e5, 1e5)], [np.eye(3)], grf[:1], 0.2,
                                4500.0, 1600.0, 10)
    inner = np.zeros(shape, bool)
    inner[1:-1, 1:-1, 1:-1] = True    # closing counts the outside as empty: the outer shell goes
    assert np.array_equal(K, inner & (V >= 1600.0)) and np.array_equal(mask, K)
    assert np.array_equal(got, ref.astype(np.float32))
    got, mask, _, _ = _run(V, h, [], np.zeros((0, 3)), np.zeros((0, 3, 3)), np.zeros((0,) + shape), 0.2,
                                   4500.0, 1600.0, 10)
    assert not mask.any() and np.array_equal(got, V)


@pytest.mark.parametrize("shape", [(1, 1, 1), (2, 1, 3), (25, 1, 61), (7, 5, 1), (6, 7, 5), (12, 10, 300),
                                   (9, 6, 517)])
def test_tiny_slice_and_wide_volumes(shape):
    """A dimension under 3 voxels leaves no salt (the opening's erosion sees
    the empty outside on both sides); rows of 300 and 517 voxels span several
    64-voxel blocks of the row pass and several workgroups per row."""
    h = (10.0, 10.0, 10.0)
    nz, ny, nx = shape
    V = _model(shape, 3)
    ext = np.array(shape) * 10.0
    grf = _field(1, shape, 1.0, 4) if min(shape) > 1 else np.random.default_rng(4).standard_normal(
        (1,) + shape).astype(np.float32)
    got, mask, ref, K = _run(V, h, [ext / 2], [ext / 2.5 + 5.0], [_rot(0.4, 0.0, 0.0)], grf, 0.1, 4500.0, 0.0,
                                1)
    _report("slice %s" % (shape,), mask, K)
    if min(shape) >= 5:
        assert K.sum() > 0
    assert np.array_equal(mask, K)
    assert np.array_equal(got, ref.astype(np.float32))


@pytest.mark.parametrize("sign", [1.0, -1.0])
def test_field_reaching_far_from_the_body(sign):
    """Each body's distances are computed on its ellipsoid's box widened by
    the largest a rbar xi; a field spike far from the body (a 6-voxel cube
    where a rbar xi exceeds the distance to the body) must still salt that
    cube's core, for either sign of the amplitude."""
    shape, h = (30, 40, 90), (10.0, 10.0, 10.0)
    V = _model(shape, 8)
    grf = (0.3 * _field(1, shape, 2.0, 9)).astype(np.float32)
    grf[0, 20:26, 30:36, 75:81] = 200.0 * sign
    c, r = [(120.0, 100.0, 150.0)], [(60.0, 50.0, 70.0)]
    got, mask, ref, K = _run(V, h, c, r, [_rot(0.3, 0.2, 0.1)], grf, 0.2 * sign, 4500.0, 0.0, 20)
    _report("far field, sign %+d" % sign, mask, K)
    assert K[21:25, 31:35, 76:80].all()     # the cube's core (opening trims its edges)
    assert np.array_equal(mask, K)
    assert np.array_equal(got, ref.astype(np.float32))


def test_many_bodies_and_the_size_cut_boundary():
    """Twelve small bodies leave many components; the size cut is set to one
    component's exact size, which must be kept (components of fewer voxels go)."""
    from scipy.ndimage import label, generate_binary_structure
    shape, h = (40, 48, 56), (10.0, 10.0, 10.0)
    rng = np.random.default_rng(77)
    ext = np.array(shape) * 10.0
    centres = rng.uniform(0.15, 0.85, (12, 3)) * ext
    radii = rng.uniform(25.0, 70.0, (12, 3))
    rots = [_rot(*rng.uniform(-1, 1, 3)) for _ in range(12)]
    grf = _field(12, shape, 2.0, 78)
    V = _model(shape, 79)
    _, K1 = OB.salt_sdt(V.astype(np.float64), *h, centres, radii, rots, grf.astype(np.float64), 0.1, 4500.0, 0.0, 1)
    lab, nc = label(K1, structure=generate_binary_structure(3, 1))
    sizes = np.sort(np.bincount(lab.ravel())[1:])
    assert nc >= 6
    cut = int(sizes[len(sizes) // 2])
    got, mask, ref, K = _run(V, h, centres, radii, rots, grf, 0.1, 4500.0, 0.0, cut)
    _report("12 bodies, %d components, cut %d" % (nc, cut), mask, K)
    kept = np.bincount(label(K, structure=generate_binary_structure(3, 1))[0].ravel())[1:]
    assert cut in kept and kept.min() >= cut and len(kept) < nc
    assert np.array_equal(mask, K)
    assert np.array_equal(got, ref.astype(np.float32))


def test_salt_without_a_mask_output_through_the_c_abi():
    """mask_out may be NULL: the volume is the same as with a mask."""
    import ctypes
    import torch
    shape, h = (24, 20, 28), (10.0, 10.0, 10.0)
    V = _model(shape, 31)
    c, r, R = np.array([[120.0, 100.0, 140.0]]), np.array([[70.0, 60.0, 80.0]]), _rot(0.2, 0.3, 0.1).reshape(1, 9)
    grf = _field(1, shape, 2.0, 32)
    Vd, gd = _dev(V), _dev(grf)
    ref, _ = sgwave.salt_sdt(Vd, *h, c, r, R.reshape(1, 3, 3), gd, 0.2, 4500.0, 1600.0, 10)
    out = torch.empty_like(Vd)
    ws = torch.empty(sgwave.sg_salt_workspace_size(*shape), dtype=torch.uint8, device="cuda")
    c64, r64, R64 = (np.ascontiguousarray(a, np.float64) for a in (c, r, R))
    st = sgwave.lib().sg_salt_sdt(ctypes.c_void_p(Vd.data_ptr()), *shape, *h, 1, c64.ctypes.data, r64.ctypes.data,
                                  R64.ctypes.data, ctypes.c_void_p(gd.data_ptr()), 0.2, 4500.0, 1600.0, 10,
                                  ctypes.c_void_p(out.data_ptr()), None, ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                                  None)
    torch.cuda.synchronize()
    assert st == sgwave.SG_OK
    assert torch.equal(out, ref)
    assert (ref == 4500.0).any()
