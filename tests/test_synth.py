"""The seeded input generators (no GPU): deterministic, in range, and shaped
like the workloads they stand in for."""
import numpy as np

from paper_2605_30541_amd import synth


def test_field_slice_is_seeded_and_in_range():
    a = synth.field_slice(42, 620, 1001)
    b = synth.field_slice(42, 620, 1001)
    c = synth.field_slice(43, 620, 1001)
    assert a.dtype == np.float32 and a.shape == (620, 1001)
    assert np.array_equal(a, b) and not np.array_equal(a, c)
    assert a.min() >= 1500.0 and a.max() <= 4500.0
    # increasing with depth on average; a salt body at 4500 m/s exists
    assert a[:100].mean() < a[-100:].mean()
    assert (a == 4500.0).sum() > 1000


def test_field_slice_small_and_shallow_models_terminate():
    for (nz, nx, dz, dx) in ((37, 53, 8.0, 11.0), (30, 70, 10.0, 10.0), (6, 7, 10.0, 10.0), (2, 2, 1.0, 1.0)):
        v = synth.field_slice(3, nz, nx, dz, dx)
        assert v.shape == (nz, nx) and np.isfinite(v).all()


def test_uneven_sizes_and_geometry_helpers():
    sizes = synth.uneven_sizes(42, 8)
    assert len(sizes) == 8
    assert all(400 <= nz <= 620 and 601 <= nx <= 1001 for nz, nx in sizes)
    assert sizes == synth.uneven_sizes(42, 8)
    rec = synth.surface_receivers(1001, 10.0)
    assert rec.shape == (1001, 2) and rec[-1, 1] == 10000.0 and np.all(rec[:, 0] == 10.0)
    sl = synth.shot_line(64, 1100.0, 8900.0)
    assert sl.shape == (64, 2) and sl[0, 1] == 1100.0 and sl[-1, 1] == 8900.0
    v = synth.field_slice(1, 100, 80)
    s = synth.smoothed_1d(v, 500.0, 10.0)
    assert s.shape == v.shape and np.allclose(s, s[:, :1])
    assert np.all(np.diff(s[:, 0]) > -1.0)             # smooth, mostly increasing trend
    f = synth.flat_layers(64, 128, 10.0, [0.0, 200.0, 400.0], [1500.0, 2500.0, 3500.0])
    assert f[19, 0] == 1500.0 and f[20, 0] == 2500.0 and f[40, 5] == 3500.0
