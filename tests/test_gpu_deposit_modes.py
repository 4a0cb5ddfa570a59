"""GPU parity of Deposit's simplex-noise form and sinusoidal bedform mode
(App. B, the Deposit prose) and of the 3D simplex noise they use, against
the FP64 oracle on the same float32 inputs."""
import numpy as np
import pytest

from oracle import builder as OB
from paper_2605_30541_amd import sgwave

pytestmark = pytest.mark.gpu
TOL = 1e-5


def _dev(a, dtype=np.float32):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype)).cuda()


def _host(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy().astype(np.float64)


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("shape,origin,step", [((37, 41, 53), (-3.7, 2.2, -11.9), (0.13, 0.21, 0.17)),
                                               ((1, 300, 517), (5.5, -40.0, 0.0), (1.0, 0.05, 0.031)),
                                               ((64, 1, 64), (300.0, 7.0, -300.0), (0.5, 0.0, 0.77)),
                                               ((9, 11, 13), (0.0, 0.0, 0.0), (1.0, 1.0, 1.0))])
def test_simplex_noise_matches_the_oracle(shape, origin, step):
    rng = np.random.default_rng(sum(shape))
    perm = rng.permutation(256)
    got = _host(sgwave.simplex_noise3d(_dev(perm, np.int32), shape, origin, step, 1.7))
    Z, Y, X = np.meshgrid(*[o + np.arange(n) * s for o, n, s in zip(origin, shape, step)], indexing="ij")
    ref = 1.7 * OB.simplex_noise3d(perm, Z, Y, X)
    err = np.abs(got - ref).max()
    print("%s: max |diff| %.2e, range %.3f..%.3f" % (shape, err, ref.min(), ref.max()), flush=True)
    assert err <= 1e-6 * 1.7


@pytest.mark.parametrize("case", ["beds-only", "noisy", "crossing-contacts", "one-bed", "2d-slice"])
def test_deposit_simplex_matches_the_oracle(case):
    rng = np.random.default_rng({"beds-only": 11, "noisy": 12, "crossing-contacts": 13, "one-bed": 14,
                                 "2d-slice": 15}[case])
    t, ny, nx = 70, (1 if case == "2d-slice" else 7), 45
    nb = 1 if case == "one-bed" else 9
    thick = np.clip(rng.normal(t / nb, 2.0, nb), 0.5, None).astype(np.float32)
    vbed = rng.normal(2600.0, 150.0, nb).astype(np.float32)
    off = rng.uniform(0, 300, nb).astype(np.float32)
    pb, pt = rng.permutation(256), rng.permutation(256)
    a_B, a_eta = {"beds-only": (0.0, 0.0), "noisy": (3.0, 60.0), "crossing-contacts": (25.0, 40.0),
                  "one-bed": (0.0, 80.0), "2d-slice": (4.0, 50.0)}[case]
    args = (t, ny, nx, 5.0, 10.0, 12.5)
    lam_b, lam_t = (80.0, 300.0, 240.0), (35.0, 200.0, 260.0)
    got = _host(sgwave.deposit_simplex(*args, _dev(thick), _dev(vbed), 0.4, _dev(pb, np.int32), lam_b, a_B,
                                       _dev(pt, np.int32), lam_t, _dev(off), a_eta, 0.15, 0.2))
    ref = OB.deposit_simplex(*args, thick.astype(np.float64), vbed.astype(np.float64), 0.4, pb, lam_b, a_B, pt,
                             lam_t, off.astype(np.float64), a_eta, 0.15, 0.2)
    e = rel_l2(got, ref)
    print("%s: deposit_simplex rel-L2 %.2e, max |diff| %.2e m/s" % (case, e, np.abs(got - ref).max()), flush=True)
    assert e <= TOL


@pytest.mark.parametrize("case", ["plain", "rough-textured", "no-smoothing", "wide-smoothing", "tall-band",
                                  "one-cell-band"])
def test_deposit_sinusoidal_matches_the_oracle(case):
    rng = np.random.default_rng({"plain": 21, "rough-textured": 22, "no-smoothing": 23, "wide-smoothing": 24,
                                 "tall-band": 25, "one-cell-band": 26}[case])
    t, ny, nx = {"tall-band": (4096, 2, 3), "one-cell-band": (1, 5, 6)}.get(case, (80, 6, 40))
    sigma = {"no-smoothing": 0.0, "wide-smoothing": 60.0}.get(case, 3.0)
    freq = rng.uniform(0.02, 0.12, t).astype(np.float32)
    rug = rng.uniform(-1, 1, (ny, nx)).astype(np.float32)
    pt = rng.permutation(256)
    a_r, a_eta = (0.35, 45.0) if case in ("rough-textured", "tall-band") else (0.0, 0.0)
    args = (t, ny, nx, 2.5, 10.0, 12.5, 3100.0, 0.3)
    got = _host(sgwave.deposit_sinusoidal(*args, _dev(freq), sigma, 150.0, 60.0, 0.9,
                                          _dev(rug) if a_r else None, a_r, _dev(pt, np.int32),
                                          (40.0, 150.0, 200.0), a_eta, 0.1, 0.1))
    ref = OB.deposit_sinusoidal(*args, freq.astype(np.float64), sigma, 150.0, 60.0, 0.9, rug.astype(np.float64),
                                a_r, pt, (40.0, 150.0, 200.0), a_eta, 0.1, 0.1)
    e = rel_l2(got, ref)
    print("%s: deposit_sinusoidal rel-L2 %.2e, max |diff| %.2e m/s" % (case, e, np.abs(got - ref).max()),
          flush=True)
    assert e <= TOL
