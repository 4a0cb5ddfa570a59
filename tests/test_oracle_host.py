"""Pins of the oracle's host-side formulas against numbers the paper prints and
against closed forms (no GPU)."""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_params.json")))


def _taylor_weights(M):
    """Independent derivation: solve sum_m c_m (m^(2k)) * 2 = [k==1] * 2 for
    k = 1..M exactly (even moments of the symmetric stencil), c_0 from k = 0."""
    A = [[Fraction(2 * m ** (2 * k)) for m in range(1, M + 1)] for k in range(1, M + 1)]
    rhs = [Fraction(2 if k == 1 else 0) for k in range(1, M + 1)]
    # moment k=1 of u=x^2: sum c_m 2 m^2 h^2 / h^2 = 2 -> exact second derivative of x^2
    n = M
    aug = [row[:] + [r] for row, r in zip(A, rhs)]
    for i in range(n):
        piv = next(r for r in range(i, n) if aug[r][i] != 0)
        aug[i], aug[piv] = aug[piv], aug[i]
        for r in range(n):
            if r != i and aug[r][i] != 0:
                f = aug[r][i] / aug[i][i]
                aug[r] = [x - f * y for x, y in zip(aug[r], aug[i])]
    c = [aug[i][n] / aug[i][i] for i in range(n)]
    return [-2 * sum(c)] + c


def test_fd_coefficients_match_taylor_and_fornberg():
    c = oracle.fd_coefficients(4)
    assert c == _taylor_weights(4)
    assert [str(x) for x in c] == GOLDEN["fornberg_c8"]["value"]


def test_fd_coefficients_exact_on_polynomials():
    # sum_m c_m (u(j+m) + u(j-m)) == u''(j) exactly for u = x^p, p <= 9
    c = oracle.fd_coefficients(4)
    for p in range(0, 10):
        for j in (-3, 0, 2, 7):
            approx = c[0] * Fraction(j) ** p + sum(
                c[m] * (Fraction(j + m) ** p + Fraction(j - m) ** p) for m in range(1, 5))
            exact = Fraction(p * (p - 1)) * Fraction(j) ** (p - 2) if p >= 2 else Fraction(0)
            assert approx == exact, (p, j)
    # and not exact at degree 10 (the stencil is 8th order, not higher)
    p, j = 10, 0
    approx = sum(c[m] * 2 * Fraction(m) ** p for m in range(1, 5))
    assert approx != 0


def test_cfl_constants():
    # s_max = (sqrt(d sum|a_m|))^-1, App. E.3.2; 8th order in 2D
    assert oracle.cfl_smax(4, 2) == pytest.approx(0.52311, abs=5e-6)
    # exact von Neumann limit of the same leapfrog scheme
    assert oracle.von_neumann_courant(4, 2) == pytest.approx(0.55463, abs=5e-6)
    assert oracle.von_neumann_courant() > oracle.cfl_smax()
    # 2nd-order stencil in 1D: the classic Courant limit 1 (both formulas agree)
    assert oracle.cfl_smax(1, 1) == pytest.approx(1.0)
    assert oracle.von_neumann_courant(1, 1) == pytest.approx(1.0)


def test_cfl_forces_paper_dt():
    g = GOLDEN["grid"]
    dtmax = oracle.cfl_dt_max(g["h_m"], g["vmax"])
    # the paper says the bound forces dt = 1 ms: 1 ms is admissible, 1.1 ms is not
    assert dtmax >= GOLDEN["cfl_forces_dt_ms"]["value"] * 1e-3
    assert dtmax < 1.1e-3


def test_dispersion_rule_holds_for_paper_grid():
    g = GOLDEN["grid"]
    fmax_top = max(b["fmax"] for b in GOLDEN["bands"])
    hmax = oracle.dispersion_h_max(g["vmin"], fmax_top, GOLDEN["dispersion_G"]["value"])
    assert hmax == pytest.approx(15.0)
    assert g["h_m"] <= hmax


def test_saved_counts_match_table():
    for row in GOLDEN["saved_samples"]:
        assert oracle.n_saved(row["N"], row["k"]) == row["n_saved"], row["cite"]


def test_nyquist_margins_match_table():
    dts = GOLDEN["saved_interval_s"]["value"]
    lim = 1.0 / (2.0 * dts)
    assert round(lim, GOLDEN["nyquist_limit_hz"]["decimals"]) == GOLDEN["nyquist_limit_hz"]["value"]
    for b in GOLDEN["bands"]:
        assert round(oracle.nyquist_margin(b["fmax"], dts), 2) == pytest.approx(b["margin"], abs=1e-9), b


def test_subsample_rule_is_conservative_for_k14():
    # k = floor(N/(2 fmax T)) is the largest admissible factor; the paper's uniform k = 14
    # must not exceed it for any band (App. E.3.3)
    for N, T in ((5001, 5.0), (8001, 8.0)):
        for b in GOLDEN["bands"]:
            assert oracle.subsample_factor(N, b["fmax"], T) >= 14


def test_c_damp_and_sponge_thickness():
    s = GOLDEN["sponge"]
    assert oracle.c_damp(s["nbl"], s["R"]) == pytest.approx(1.5 * math.log(1000.0) / 60.0, rel=1e-15)
    assert oracle.c_damp(60) == pytest.approx(0.172694, abs=5e-7)
    assert s["nbl"] * GOLDEN["grid"]["h_m"] / 1000.0 == pytest.approx(s["thickness_km"])


def test_ricker_closed_form_properties():
    f0, dt, nt = 12.5, 1e-4, 4000
    w = oracle.ricker(f0, dt, nt)
    t = np.arange(nt) * dt
    i0 = int(round(1.0 / f0 / dt))
    # peak of 1 at t0 = 1/f0
    assert w[i0] == pytest.approx(1.0, abs=1e-12)
    assert np.argmax(w) == i0
    # zero crossings at tau = +-1/(sqrt(2) pi f0)
    tz = 1.0 / f0 + np.array([-1, 1]) / (math.sqrt(2) * math.pi * f0)
    for z in tz:
        j = int(z / dt)
        assert w[j] * w[j + 1] <= 0
    # minima value -2 exp(-3/2) at tau = +-sqrt(3/2)/(pi f0)
    assert w.min() == pytest.approx(-2 * math.exp(-1.5), rel=1e-5)
    # zero mean over the whole line (its spectrum vanishes at 0 Hz); amplitude
    # spectrum peaks at f0.  Use a late centre so the pulse is not truncated.
    wl = oracle.ricker(f0, dt, nt, t0=0.2)
    assert abs(np.sum(wl) * dt) < 1e-12
    W = np.abs(np.fft.rfft(wl, n=1 << 18))
    f = np.fft.rfftfreq(1 << 18, dt)
    assert f[np.argmax(W)] == pytest.approx(f0, abs=0.05)


def test_bandpass_wavelet_energy_scaling():
    dt, nt = 1e-3, 8001
    for f0, b in zip(GOLDEN["peak_frequencies_hz"]["value"], GOLDEN["bands"]):
        w = oracle.bandpass_ricker(f0, (b["fmin"], b["fmax"]), dt, nt)
        B = b["fmax"] - b["fmin"]
        # l2 normalised, then scaled by sqrt(B / 24 Hz) (App. E.4)
        assert np.linalg.norm(w) == pytest.approx(math.sqrt(B / 24.0), rel=1e-12)
        # pass band: most energy between the corners
        W = np.abs(np.fft.rfft(w)) ** 2
        f = np.fft.rfftfreq(nt, dt)
        inside = W[(f >= b["fmin"]) & (f <= b["fmax"])].sum()
        assert inside / W.sum() > 0.8


def _butterworth_bandpass_power(f, band, fs, order):
    """Squared gain of a band-pass Butterworth filter whose low-pass prototype
    has `order` poles, designed through the bilinear map with the corners
    pre-warped: with t = tan(pi f / fs) and t1, t2 the warped corners,
    |H|^2 = 1 / (1 + x^(2 order)), x = (t^2 - t1 t2) / (t (t2 - t1)).
    Forward-backward filtering multiplies by H(z) H(1/z) = |H|^2 on the unit
    circle, so this is the whole gain of the zero-phase filter, real and
    non-negative (-6 dB in amplitude at each corner)."""
    t = np.tan(np.pi * f / fs)
    t1, t2 = np.tan(np.pi * band[0] / fs), np.tan(np.pi * band[1] / fs)
    x = (t * t - t1 * t2) / (t * (t2 - t1))
    return 1.0 / (1.0 + x ** (2 * order))


@pytest.mark.parametrize("ib", range(5))
def test_bandpass_wavelet_is_the_zero_phase_4th_order_butterworth(ib):
    """App. E.4: 4th-order zero-phase Butterworth.  A Ricker centred in a long
    trace (zero at both ends, so the filter acts as on an infinite sequence)
    gives an output whose spectrum over the Ricker's is real, non-negative and
    proportional to the closed-form squared Butterworth gain of order 4.
    Order 2 or 8, or a single causal pass (complex ratio, |H| not |H|^2),
    fails it; so does a filter that is not symmetric in time."""
    dt, nt = 1e-3, 1 << 15
    f0 = GOLDEN["peak_frequencies_hz"]["value"][ib]
    b = GOLDEN["bands"][ib]
    band = (b["fmin"], b["fmax"])
    c = nt // 2
    y = oracle.bandpass_ricker(f0, band, dt, nt, t0=c * dt)
    r = oracle.ricker(f0, dt, nt, t0=c * dt)
    # zero phase: the output is as symmetric about the centre as the input
    assert np.abs(y[c + 1:c + 4000] - y[c - 1:c - 4000:-1]).max() < 1e-10 * np.abs(y).max()
    Y, R = np.fft.rfft(y), np.fft.rfft(r)
    f = np.fft.rfftfreq(nt, dt)
    ok = (np.abs(R) > 1e-6 * np.abs(R).max()) & (f > 0)
    ratio = Y[ok] / R[ok]
    G = _butterworth_bandpass_power(f[ok], band, 1.0 / dt, 4)
    scale = np.sum(ratio.real * G) / np.sum(G * G)
    assert scale > 0
    assert np.abs(ratio.imag).max() < 1e-7 * scale
    assert np.abs(ratio.real - scale * G).max() < 1e-7 * scale
    # the -6 dB points sit at the band corners
    for fc in band:
        assert _butterworth_bandpass_power(np.array([fc]), band, 1.0 / dt, 4)[0] == pytest.approx(0.5, rel=1e-12)
