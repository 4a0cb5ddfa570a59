"""GPU fault sequences (a primary and its Riedel-shear subsidiaries, App. B
Fault prose): sg_fault_sequence / sg_fault_labels_sequence against the
oracle's sequence and against the same faults applied by single calls."""
import numpy as np
import pytest

from oracle import builder as OB
from paper_2605_30541_amd import sgwave

pytestmark = pytest.mark.gpu
TOL = 1e-5
H = 10.0


def _dev(a, dtype=np.float32):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype)).cuda()


def _host(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy()


def rel_l2(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / np.linalg.norm(b))


def _model(nz, ny, nx, seed):
    rng = np.random.default_rng(seed)
    z = np.arange(nz)[:, None, None]
    x = np.arange(nx)[None, None, :]
    y = np.arange(ny)[None, :, None]
    V = 1700.0 + 30.0 * z + 80.0 * np.sin(x / 7.0 + y / 5.0) + 150.0 * (np.floor((z + 2 * np.sin(x / 9.0)) / 5) % 3)
    L = (np.floor((z + 2 * np.sin(x / 9.0)) / 5)).astype(np.int32)
    return (V + rng.normal(0, 4.0, V.shape)).astype(np.float32), np.broadcast_to(L, V.shape).copy()


PRIMARY = dict(cz=200.0, cy=180.0, cx=240.0, azimuth_deg=20.0, dip_deg=60.0, radius=900.0, slip=40.0, direction=1,
               die_r=120.0, die_strike=250.0, die_theta_deg=25.0)
CFG = dict(OB.RIEDEL_DEFAULTS, along_strike=150.0, across_min=20.0, across_max=120.0, size_scale=0.3,
           slip_min=0.3, slip_max=0.6, min_distance=40.0)


def _faults(case, ny):
    subs = sgwave.riedel_subsidiaries(PRIMARY if ny > 1 else dict(PRIMARY, cy=0.0, azimuth_deg=0.0), CFG,
                                      np.random.default_rng(80).random((8, 5)))
    prim = PRIMARY if ny > 1 else dict(PRIMARY, cy=0.0, azimuth_deg=0.0)
    if case == "empty":
        return []
    if case == "one":
        return [prim]
    if case == "two":
        return [prim, subs[0]]
    if case == "2d-slice":
        return [prim] + subs[:3]
    miss = dict(prim, cz=5000.0, cy=9000.0, cx=9000.0)
    whole = dict(prim, radius=5000.0, slip=25.0, die_r=4000.0, die_strike=8000.0, die_theta_deg=80.0,
                 direction=-1)
    return [prim, subs[0], subs[1], miss, subs[2], whole, subs[3], miss, miss] + subs[4:]


@pytest.mark.parametrize("case", ["empty", "one", "two", "primary-subsidiaries-miss-whole", "2d-slice"])
def test_fault_sequence_matches_oracle_and_single_calls(case):
    import torch
    nz, ny, nx = 40, (1 if case == "2d-slice" else 36), 48
    V, L = _model(nz, ny, nx, 5)
    faults = _faults(case, ny)
    print("case %s: %d faults" % (case, len(faults)), flush=True)
    v, lab = _dev(V), _dev(L, np.int32)
    got = sgwave.fault_sequence(v, H, H, H, faults, 1480.0)
    glab = sgwave.fault_labels_sequence(lab, H, H, H, faults, -1)
    one, onel = v.clone(), lab.clone()
    for f in faults:
        one = sgwave.fault(one, H, H, H, f, 1480.0)
        onel = sgwave.fault_labels(onel, H, H, H, f, -1)
    got, glab, one, onel = _host(got), _host(glab), _host(one), _host(onel)
    assert np.array_equal(got, one) and np.array_equal(glab, onel)
    ref = OB.fault_sequence(V.astype(np.float64), H, H, H, faults, 1480.0)
    rl = OB.fault_labels_sequence(L, H, H, H, faults, -1)
    e = rel_l2(got, ref)
    same = float(np.mean(glab == rl))
    print("  rel-L2 %.2e, labels equal on %.6f of voxels, moved %.3f" % (e, same, float(np.mean(got != V))),
          flush=True)
    assert e <= TOL
    assert same >= 0.9999
    if case == "empty":
        assert np.array_equal(got, V) and np.array_equal(glab, L)
