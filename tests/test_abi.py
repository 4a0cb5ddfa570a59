"""Host-side tests of the C ABI (no GPU): the library loads, exports every
function the header declares, and its host-only calls validate and compute
what they document."""
import ctypes
import math

import numpy as np
import pytest

import oracle
from paper_2605_30541_amd import sgwave
from paper_2605_30541_amd.sgwave import Geometry, Plan, SGError


def test_library_exports_every_header_function():
    names = sgwave.header_functions()
    assert "sg_forward" in names and "sg_adjoint_gradient" in names and "sg_batch_forward" in names
    L = sgwave.lib()
    for n in names:
        assert hasattr(L, n), n
    assert sgwave.sg_abi_version() == 2
    assert set(names) == set(sgwave._SIGS)


def test_status_strings():
    assert sgwave.sg_status_string(0) == "SG_OK"
    assert sgwave.sg_status_string(2) == "SG_ECFL"
    assert sgwave.sg_status_string(99) == "SG_UNKNOWN"


def test_ricker_matches_oracle():
    for f0, dt, nt in ((15.0, 1e-3, 500), (12.0, 8e-4, 10000), (4.5, 1e-3, 8001)):
        a = sgwave.sg_ricker(f0, dt, nt)
        b = oracle.ricker(f0, dt, nt)
        assert np.abs(a - b).max() <= 6e-8 * np.abs(b).max()


def test_bandpass_ricker_matches_oracle():
    """The band-limited sources of App. E.4 for the paper's five bands (Table
    "bands", peak frequencies of App. E.4) at the paper's and the field
    workload's sampling: equal to the oracle's (SciPy zero-phase
    second-order-section filtering) to float rounding."""
    import json
    import os
    golden = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_params.json")))
    for f0, b in zip(golden["peak_frequencies_hz"]["value"], golden["bands"]):
        for dt, nt in ((1e-3, 8001), (8e-4, 10000)):
            a = sgwave.sg_bandpass_ricker(f0, b["fmin"], b["fmax"], dt, nt)
            r = oracle.bandpass_ricker(f0, (b["fmin"], b["fmax"]), dt, nt)
            assert np.abs(a - r).max() <= 2e-7 * np.abs(r).max(), (f0, dt)
    for bad in ((10.0, 5.0, 5.0, 1e-3, 500), (10.0, 0.0, 5.0, 1e-3, 500), (10.0, 3.0, 600.0, 1e-3, 500),
                (10.0, 3.0, 25.0, 1e-3, 27)):
        with pytest.raises(SGError) as e:
            sgwave.sg_bandpass_ricker(*bad)
        assert e.value.status == sgwave.SG_EINVAL


def test_cfl_limit_matches_paper_constant():
    assert sgwave.sg_cfl_dt_max(10.0, 10.0, 5000.0) == pytest.approx(oracle.cfl_dt_max(10.0, 5000.0), rel=1e-14)


def _geom(**kw):
    base = dict(nz=64, nx=128, dz=10.0, dx=10.0, dt=1e-3, nt=500, nbl=20, vmax_hint=3500.0)
    base.update(kw)
    return Geometry(**base)


def test_plan_validation_errors():
    Plan(_geom())
    bad = [dict(nz=0), dict(nx=-1), dict(dt=0.0), dict(dz=float("nan")), dict(nt=1), dict(nbl=-1),
           dict(top=7), dict(damp_R=0.0), dict(damp_R=1.5), dict(vmax_hint=0.0), dict(rec_every=0),
           dict(snap_count=3, snap_every=0), dict(snap_count=6, snap_every=100)]
    for kw in bad:
        with pytest.raises(SGError) as e:
            Plan(_geom(**kw))
        assert e.value.status == sgwave.SG_EINVAL, kw
        assert e.value.message
    Plan(_geom(snap_count=5, snap_every=100, nt=401))
    with pytest.raises(SGError):
        Plan(_geom(snap_count=5, snap_every=100, nt=400))


def test_largest_grid():
    """A stored field (padded grid + 4-cell guard ring, rows padded to 32
    floats) may hold 2^29 cells, no more: 32-bit byte offsets reach every cell
    of the FP64 imaging accumulator."""
    # free top, no sponge: stored field (nz + 8) x pitch, pitch = nx + 8 rounded up to 32
    nx = 16384 - 8                                   # pitch 16384
    nz_max = (1 << 29) // 16384 - 8                  # 32760 rows: exactly 2^29 cells
    g = _geom(nz=nz_max, nx=nx, nbl=0, nt=10)
    p = Plan(g)
    assert p.padded_shape == (nz_max, nx)
    with pytest.raises(SGError) as e:
        Plan(_geom(nz=nz_max + 1, nx=nx, nbl=0, nt=10))
    assert e.value.status == sgwave.SG_EINVAL and "2^29" in e.value.message


def test_plan_cfl_rejection_and_override():
    dtmax = oracle.cfl_dt_max(10.0, 5000.0)
    Plan(_geom(dt=dtmax * 0.999, vmax_hint=5000.0))
    with pytest.raises(SGError) as e:
        Plan(_geom(dt=dtmax * 1.001, vmax_hint=5000.0))
    assert e.value.status == sgwave.SG_ECFL
    Plan(_geom(dt=dtmax * 1.001, vmax_hint=5000.0), flags=sgwave.SG_ALLOW_UNSTABLE)


def test_dispersion_warning():
    # h <= vmin / (4 fmax): 10 m passes at 1500 m/s, 25 Hz (15 m) and fails at 50 Hz (7.5 m)
    assert Plan(_geom(vmin_hint=1500.0, fmax_hint=25.0)).warnings == 0
    assert Plan(_geom(vmin_hint=1500.0, fmax_hint=50.0)).warnings & sgwave.SG_WARN_DISPERSION


def test_padded_shape_and_workspace_size():
    p = Plan(_geom())
    assert p.padded_shape == (84, 168)                     # 64+20 x 128+40
    p2 = Plan(_geom(top=sgwave.SG_TOP_ABSORBING))
    assert p2.padded_shape == (104, 168)
    w1 = sgwave.sg_forward_workspace_size(p, 1, 128)
    w4 = sgwave.sg_forward_workspace_size(p, 4, 128)
    assert w4 > w1 > 2 * 84 * 168 * 4
    # fields dominate: 3 more shots add at least 3 x 2 padded fields
    assert w4 - w1 >= 3 * 2 * 84 * 168 * 4


def test_tuning_validation():
    p = Plan(_geom())
    assert p.get_tuning(1) == dict(variant=2, tile_x=128, tile_z=64, time_block=4, rows_per_thread=8)
    p.set_tuning(variant=2, tile_x=128, tile_z=64, time_block=4)
    assert p.get_tuning(1) == dict(variant=2, tile_x=128, tile_z=64, time_block=4, rows_per_thread=8)
    p.set_tuning(variant=2, tile_x=128, tile_z=64, time_block=3, rows_per_thread=16)
    assert p.get_tuning(1)["rows_per_thread"] == 16
    with pytest.raises(SGError) as e:
        p.set_tuning(variant=2, tile_x=64, tile_z=32, time_block=4)
    assert e.value.status == sgwave.SG_EUNSUPPORTED
    with pytest.raises(SGError):
        p.set_tuning(variant=2, tile_x=64, tile_z=64, rows_per_thread=16)
    p.set_tuning(variant=1)
    assert p.get_tuning(1) == dict(variant=1, tile_x=0, tile_z=0, time_block=1, rows_per_thread=0)
    with pytest.raises(SGError):
        p.set_tuning(variant=5)
    with pytest.raises(SGError):
        p.set_tuning(variant=2, time_block=9)
    # column sweep: strips of 128 or 256 columns, time blocks up to 6
    p.set_tuning(variant=3)
    assert p.get_tuning(1) == dict(variant=3, tile_x=256, tile_z=0, time_block=4, rows_per_thread=0)
    p.set_tuning(variant=3, tile_x=128, time_block=6)
    assert p.get_tuning(1) == dict(variant=3, tile_x=128, tile_z=0, time_block=6, rows_per_thread=0)
    p.set_tuning(variant=3, tile_x=256, tile_z=160, time_block=4)
    assert p.get_tuning(1)["tile_z"] == 160
    for bad in (dict(tile_x=192), dict(time_block=7), dict(tile_z=4), dict(rows_per_thread=8)):
        with pytest.raises(SGError):
            p.set_tuning(variant=3, **bad)
    p.clear_tuning()


def test_forward_argument_errors_touch_nothing():
    """Validation happens before any device work: these calls fail on the
    host with null device pointers and never reach the GPU."""
    p = Plan(_geom())
    L = sgwave.lib()
    src = np.array([[20.0, 640.0]])
    rec = np.stack([np.full(128, 10.0), np.arange(128) * 10.0], 1)
    dp = ctypes.POINTER(ctypes.c_double)

    def shots(src_, rec_, wavelet=1):
        return sgwave.sg_shots(len(src_), src_.ctypes.data_as(dp), len(rec_), rec_.ctypes.data_as(dp),
                               ctypes.c_void_p(wavelet), 0)
    fake = ctypes.c_void_p(0x1000)
    cases = [
        (None, shots(src, rec), fake, 1 << 30, sgwave.SG_EINVAL),          # vp NULL
        (fake, shots(src, rec), None, 1 << 30, sgwave.SG_EINVAL),          # ws NULL
        (fake, shots(np.array([[20.0, 1280.0]]), rec), fake, 1 << 30, sgwave.SG_EINVAL),  # src outside
        (fake, shots(src, np.array([[-1.0, 5.0]])), fake, 1 << 30, sgwave.SG_EINVAL),    # rec outside
        (fake, shots(src, rec, wavelet=0), fake, 1 << 30, sgwave.SG_EINVAL),            # no wavelet
        (fake, shots(src, rec), fake, 16, sgwave.SG_ENOSPACE),                          # small ws
    ]
    for vp, sh, ws, nbytes, want in cases:
        st = L.sg_forward(p.handle, vp, ctypes.byref(sh), None, None, ws, nbytes, None)
        assert st == want, (st, want, sgwave.sg_last_error())
        assert sgwave.sg_last_error()


def test_destroy_null_is_ok():
    assert sgwave.lib().sg_plan_destroy(None) == 0


def test_wave_residual_workspace_and_argument_errors():
    """Workspace of the residual pass (FP64 partial sums per workgroup and
    frame) and its argument checks, which return before any device work."""
    def blocks(nz, nx, z0):   # 4 partial sums per tile of 64 columns x 32 rows
        if nx <= 8 or nz - 4 - z0 <= 0:
            return 0
        return 4 * (-(-(nx - 8) // 64)) * (-(-(nz - 4 - z0) // 32))
    for T, nz, nx, top, z0 in ((10, 619, 1000, sgwave.SG_TOP_FREE, 1), (10, 619, 1000, sgwave.SG_TOP_ABSORBING, 4),
                               (3, 9, 9, sgwave.SG_TOP_FREE, 1)):
        need = (T - 2) * blocks(nz, nx, z0) * 16
        assert sgwave.sg_wave_residual_workspace_size(T, nz, nx, top) == max(-(-need // 256) * 256, 256)
    assert sgwave.sg_wave_residual_workspace_size(2, 50, 50) == 256
    assert sgwave.sg_wave_residual_workspace_size(10, 5, 5) == 256
    for bad in ((0, 10, 10, 0), (5, 0, 10, 0), (5, 10, 10, 2), (70000, 10, 10, 0)):
        with pytest.raises(SGError) as e:
            sgwave.sg_wave_residual_workspace_size(*bad)
        assert e.value.status == sgwave.SG_EINVAL
    L = sgwave.lib()
    fake = ctypes.c_void_p(4096)
    ws = sgwave.sg_wave_residual_workspace_size(10, 40, 50)
    # (pointers, sizes, spacings, top, workspace bytes) -> expected status
    cases = [((None, 10, 40, 50, fake, 10.0, 10.0, 1e-3, 0, fake, fake, fake, ws), sgwave.SG_EINVAL),
             ((fake, 10, 40, 50, fake, 0.0, 10.0, 1e-3, 0, fake, fake, fake, ws), sgwave.SG_EINVAL),
             ((fake, 10, 40, 50, fake, 10.0, 10.0, float("nan"), 0, fake, fake, fake, ws), sgwave.SG_EINVAL),
             ((fake, 10, 40, 50, fake, 10.0, 10.0, 1e-3, 3, fake, fake, fake, ws), sgwave.SG_EINVAL),
             ((fake, 10, 40, 50, fake, 10.0, 10.0, 1e-3, 0, fake, fake, fake, ws - 1), sgwave.SG_ENOSPACE)]
    for args, status in cases:
        assert L.sg_wave_residual(*args, None) == status


def test_builder_argument_errors_touch_nothing():
    """The builder calls validate before any device work (fake pointers)."""
    L = sgwave.lib()
    a, b = ctypes.c_void_p(4096), ctypes.c_void_p(8192)
    E = sgwave.SG_EINVAL
    assert L.sg_squish(a, 10, 2, 3, 10.0, b, a, None) == E                # output aliases the input
    assert L.sg_squish(a, 0, 2, 3, 10.0, b, b, None) == E
    assert L.sg_squish(a, 10, 2, 3, 0.0, a, b, None) == E
    assert L.sg_squish(a, 10, 2, 3, 10.0, None, b, None) == E
    good = dict(cz=1.0, cy=1.0, cx=1.0, azimuth_deg=0.0, dip_deg=60.0, radius=100.0, slip=5.0, direction=1,
                die_r=10.0, die_strike=10.0, die_theta_deg=10.0)
    for bad in (dict(direction=0), dict(radius=0.0), dict(die_r=-1.0), dict(slip=float("inf")),
                dict(die_theta_deg=float("nan"))):
        p = sgwave.sg_fault_params(**dict(good, **bad))
        assert L.sg_fault(a, 10, 2, 3, 10.0, 10.0, 10.0, ctypes.byref(p), 0.0, b, None) == E, bad
    p = sgwave.sg_fault_params(**good)
    assert L.sg_fault(a, 10, 2, 3, 10.0, -1.0, 10.0, ctypes.byref(p), 0.0, b, None) == E
    assert L.sg_fault(a, 10, 2, 3, 10.0, 10.0, 10.0, None, 0.0, b, None) == E
    assert L.sg_fault_labels(a, 10, 2, 3, 10.0, 10.0, 10.0, ctypes.byref(p), 0, a, None) == E   # aliasing
    assert L.sg_fault_labels(a, 10, 2, 3, 10.0, 10.0, 0.0, ctypes.byref(p), 0, b, None) == E
    assert L.sg_fault_labels(a, 10, 2, 3, 10.0, 10.0, 10.0, None, 0, b, None) == E
    bad = sgwave.sg_fault_params(**dict(good, direction=2))
    assert L.sg_fault_labels(a, 10, 2, 3, 10.0, 10.0, 10.0, ctypes.byref(bad), 0, b, None) == E
    for field, val in (("rough_noct", 0), ("rough_noct", 25), ("rough_gd", 0), ("rough_amplitude", float("nan")),
                       ("rough_lam_dip", 0.0)):
        rp = sgwave.sg_fault_params(**good)
        rp.rough_lattice, rp.rough_noct, rp.rough_gd, rp.rough_gs = 4096, 2, 3, 3
        rp.rough_amplitude, rp.rough_lam_strike, rp.rough_lam_dip = 10.0, 100.0, 100.0
        setattr(rp, field, val)
        assert L.sg_fault(a, 10, 2, 3, 10.0, 10.0, 10.0, ctypes.byref(rp), 0.0, b, None) == E, field
    assert L.sg_fractal_noise2d(a, 0, 4, 4, 10, 10, 10.0, 10.0, 100.0, 100.0, 0.0, 5.0, b, None) == E
    assert L.sg_fractal_noise2d(a, 2, 4, 4, 10, 10, 10.0, 10.0, 0.0, 100.0, 0.0, 5.0, b, None) == E
    assert L.sg_fractal_noise2d(a, 2, 0, 4, 10, 10, 10.0, 10.0, 100.0, 100.0, 0.0, 5.0, b, None) == E


def test_deposit_argument_errors_touch_nothing():
    L = sgwave.lib()
    a, b = ctypes.c_void_p(4096), ctypes.c_void_p(8192)
    E = sgwave.SG_EINVAL
    ok = [40, 3, 5, 5.0, 10.0, 10.0, 4, a, a, 0.5, a, 2.0, a, 2, 2, 2, 30.0, 100.0, 100.0, a, 10.0, 0.2, 0.2, b, None]
    for i, bad in ((0, 0), (6, 0), (6, 130), (3, 0.0), (16, -1.0), (21, 0.0), (9, float("nan")), (7, None),
                   (23, None), (10, None)):
        args = list(ok)
        args[i] = bad
        assert L.sg_deposit(*args) == E, (i, bad)


def test_simplex_deposit_argument_errors_touch_nothing():
    """The simplex noise, the simplex Deposit and the sinusoidal mode reject
    NULL pointers, sizes, spacings, lengths and parameters out of range
    before any device work (fake device pointers)."""
    L = sgwave.lib()
    a, b = ctypes.c_void_p(4096), ctypes.c_void_p(8192)
    E = sgwave.SG_EINVAL
    ok = [a, 4, 5, 6, 0.0, 0.0, 0.0, 0.1, 0.1, 0.1, 1.0, b, None]
    for i, bad in ((0, None), (11, None), (1, 0), (3, -2), (4, float("nan")), (8, float("inf")), (10, float("nan")),
                   (5, 2.0 ** 41), (9, 2.0 ** 40)):
        args = list(ok)
        args[i] = bad
        assert L.sg_simplex_noise3d(*args) == E, (i, bad)
    ok = [40, 3, 5, 5.0, 10.0, 10.0, 4, a, a, 0.5, a, 60.0, 200.0, 200.0, 2.0, a, 30.0, 100.0, 100.0, a, 10.0, 0.2,
          0.2, b, None]
    for i, bad in ((0, 0), (6, 0), (6, 130), (3, 0.0), (7, None), (10, None), (15, None), (19, None), (23, None),
                   (11, 0.0), (13, -5.0), (16, float("inf")), (18, 0.0), (14, float("nan")), (20, float("nan")),
                   (21, 0.0), (9, float("inf"))):
        args = list(ok)
        args[i] = bad
        assert L.sg_deposit_simplex(*args) == E, (i, bad)
    ok = [40, 3, 5, 5.0, 10.0, 10.0, 3000.0, 0.2, a, 2.0, 100.0, 30.0, 0.5, a, 0.1, a, 30.0, 100.0, 100.0, 10.0, 0.2,
          0.2, b, None]
    for i, bad in ((0, 0), (0, 4097), (2, 0), (8, None), (15, None), (22, None), (13, None), (9, -1.0), (9, 256.0),
                   (9, float("nan")), (3, 0.0), (16, 0.0), (20, float("inf")), (6, float("nan")), (12, float("inf")),
                   (14, float("nan"))):
        args = list(ok)
        args[i] = bad
        assert L.sg_deposit_sinusoidal(*args) == E, (i, bad)


def test_salt_argument_errors_touch_nothing():
    """SaltSDT validates sizes, body parameters and the workspace before any
    device work (fake device pointers; host body arrays are real)."""
    L = sgwave.lib()
    a, b, ws = ctypes.c_void_p(4096), ctypes.c_void_p(8192), ctypes.c_void_p(1 << 20)
    need = sgwave.sg_salt_workspace_size(10, 4, 6)
    assert need >= 38 * 240
    c = np.array([50.0, 20.0, 30.0])
    r = np.array([20.0, 20.0, 20.0])
    R = np.eye(3).ravel()
    P = lambda x: x.ctypes.data
    ok = [a, 10, 4, 6, 10.0, 10.0, 10.0, 1, P(c), P(r), P(R), a, 0.2, 4500.0, 1500.0, 10, b, None, ws, need, None]
    r_bad, R_bad = np.array([20.0, 0.0, 20.0]), np.array([1.0, 0, 0, 0, float("nan"), 0, 0, 0, 1])
    R_skew = np.array([1.0, 0, 0, 0, 1.001, 0, 0, 0, 1])
    for i, bad in ((0, None), (16, None), (16, a), (1, 0), (7, -1), (7, 4097), (4, 0.0), (6, float("inf")),
                   (12, float("nan")), (15, -1), (15, 1 << 33), (9, P(r_bad)), (10, P(R_bad)), (10, P(R_skew)),
                   (11, None),
                   (18, ctypes.c_void_p((1 << 20) + 8))):
        args = list(ok)
        args[i] = bad
        assert L.sg_salt_sdt(*args) == sgwave.SG_EINVAL, (i, bad)
    args = list(ok)
    args[19] = need - 1
    assert L.sg_salt_sdt(*args) == sgwave.SG_ENOSPACE
    n = ctypes.c_size_t(0)
    assert L.sg_salt_workspace_size(1 << 12, 1 << 12, 1 << 8, ctypes.byref(n)) == sgwave.SG_EINVAL


def test_binding_fails_loudly_without_the_library(monkeypatch, tmp_path):
    """No CPU fallback exists behind the binding: with the library missing,
    the first call raises instead of computing anything."""
    monkeypatch.setattr(sgwave, "LIB_PATH", str(tmp_path / "libsgwave.so"))
    monkeypatch.setattr(sgwave, "_lib", None)
    with pytest.raises(RuntimeError, match="not built"):
        sgwave.lib()
    with pytest.raises(RuntimeError, match="not built"):
        sgwave.sg_salt_workspace_size(4, 4, 4)


def test_binding_rejects_host_tensors_before_the_library():
    """The binding checks every tensor before marshalling: host (CPU) tensors
    are refused with ValueError, so the kernels never see a host address."""
    import torch
    p = Plan(_geom())
    g = p.geom
    src = np.array([[20.0, 640.0]])
    rec = np.stack([np.full(128, 10.0), np.arange(128) * 10.0], 1)
    w = torch.zeros((1, g.nt), dtype=torch.float32)
    vp = torch.full((g.nz, g.nx), 2000.0)
    ws = torch.empty(16, dtype=torch.uint8)
    with pytest.raises(ValueError, match="CUDA"):
        sgwave.sg_forward(p, vp, sgwave.Shots(src, rec, w), None, None, ws)
    with pytest.raises(ValueError, match="required"):
        sgwave.sg_forward(p, None, sgwave.Shots(src, rec, w), None, None, ws)
    with pytest.raises(ValueError, match="CUDA"):
        sgwave.squish(torch.zeros((4, 2, 3)), 10.0, torch.zeros((2, 3)))
    with pytest.raises(ValueError, match="CUDA"):
        sgwave.wave_residual(torch.zeros((5, 9, 9)), torch.zeros((9, 9)), 10.0, 10.0, 1e-3)


def test_grf_grid_and_argument_errors():
    """The random field's periodic grid is the next power of two per axis;
    extents past 1024, negative lengths or exponent, NULL or aliased buffers
    and a short workspace are refused before any device work."""
    assert sgwave.grf_grid(37, 50, 27)[0] == (64, 64, 32)
    assert sgwave.grf_grid(619, 1000, 1000)[0] == (1024, 1024, 1024)
    assert sgwave.grf_grid(1, 1, 1)[0] == (1, 1, 1)
    L = sgwave.lib()
    with pytest.raises(SGError):
        sgwave.grf_grid(1025, 2, 2)
    fake = ctypes.c_void_p(0x1000)
    other = ctypes.c_void_p(0x2000)
    need = sgwave.grf_grid(8, 8, 8)[1]
    cases = [(fake, -1.0, 2.0, other, need, sgwave.SG_EINVAL), (fake, 3.0, -0.5, other, need, sgwave.SG_EINVAL),
             (None, 3.0, 2.0, other, need, sgwave.SG_EINVAL), (fake, 3.0, 2.0, fake, need, sgwave.SG_EINVAL),
             (fake, 3.0, 2.0, other, need - 1, sgwave.SG_ENOSPACE)]
    for noise, ell, p, out, nbytes, want in cases:
        st = L.sg_grf(noise, 8, 8, 8, ell, ell, ell, p, out, ctypes.c_void_p(0x3000), nbytes, None)
        assert st == want, (st, want, sgwave.sg_last_error())


def test_riedel_subsidiaries_match_the_oracle():
    """The host recipe equals the oracle's on the same draws (FP64, same
    operation order), with and without the spacing filter; bad arguments
    are rejected."""
    from oracle import builder as OB
    primary = dict(cz=1200.0, cy=2500.0, cx=3000.0, azimuth_deg=25.0, dip_deg=60.0, radius=3000.0, slip=120.0,
                   direction=1, die_r=400.0, die_strike=2000.0, die_theta_deg=30.0)
    cfg = dict(OB.RIEDEL_DEFAULTS, along_strike=1500.0, across_min=100.0, across_max=700.0, size_scale=0.3,
               slip_min=0.2, slip_max=0.5, min_distance=250.0)
    u = np.random.default_rng(70).random((30, 5))
    for c in (cfg, dict(cfg, min_distance=0.0)):
        got = sgwave.riedel_subsidiaries(primary, c, u)
        ref = OB.riedel_subsidiaries(primary, c, u)
        assert len(got) == len(ref) > 0
        for g, r in zip(got, ref):
            for k in ("cz", "cy", "cx", "azimuth_deg", "dip_deg", "radius", "slip", "direction", "die_r",
                      "die_strike", "die_theta_deg"):
                assert g[k] == pytest.approx(r[k], rel=1e-13, abs=1e-9), k
    assert sgwave.riedel_subsidiaries(primary, cfg, np.zeros((0, 5))) == []
    for bad_cfg in (dict(cfg, synthetic_fraction=1.5), dict(cfg, across_min=800.0), dict(cfg, size_scale=0.0),
                    dict(cfg, min_distance=-1.0), dict(cfg, slip_max=0.1)):
        with pytest.raises(SGError) as e:
            sgwave.riedel_subsidiaries(primary, bad_cfg, u)
        assert e.value.status == sgwave.SG_EINVAL
    with pytest.raises(SGError):
        sgwave.riedel_subsidiaries(primary, cfg, u + 1.0)
    with pytest.raises(SGError):
        sgwave.riedel_subsidiaries(dict(primary, radius=0.0), cfg, u)


def test_fault_sequence_argument_errors_touch_nothing():
    """Sequences reject NULL and overlapping buffers, a missing second volume
    and bad fault parameters before any device work (fake pointers)."""
    L = sgwave.lib()
    f = sgwave._fault_params(dict(cz=100.0, cy=50.0, cx=60.0, azimuth_deg=0.0, dip_deg=60.0, radius=300.0,
                                  slip=30.0, direction=1, die_r=60.0, die_strike=200.0, die_theta_deg=30.0))
    arr = (sgwave.sg_fault_params * 3)(f, f, f)
    bad = (sgwave.sg_fault_params * 3)(f, f, f)
    bad[2].direction = 0
    n = 10 * 12 * 14 * 4
    v, out, ws = ctypes.c_void_p(1 << 20), ctypes.c_void_p(2 << 20), ctypes.c_void_p(3 << 20)
    ok = [v, 10, 12, 14, 10.0, 10.0, 10.0, arr, 3, 1500.0, out, ws, None]
    E = sgwave.SG_EINVAL
    for i, badv in ((0, None), (10, None), (11, None), (8, -1), (1, 0), (4, 0.0), (7, None), (7, bad),
                    (10, ctypes.c_void_p((1 << 20) + n - 4)), (11, ctypes.c_void_p((2 << 20) + 64))):
        args = list(ok)
        args[i] = badv
        assert L.sg_fault_sequence(*args) == E, (i, badv)
        assert L.sg_fault_labels_sequence(*args[:9], 0, *args[10:]) == E, (i, badv)
