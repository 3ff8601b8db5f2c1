"""Pins of the oracle's tabulated field (a field map, the position-dependent
field information of Sect. 4.1 stored as a grid) and of the fit in it.

References, none of them the oracle's code:
  * scipy's RegularGridInterpolator (linear) for the interpolated values;
  * central differences of that interpolator for the gradient inside a cell;
  * the analytic solenoid the map was sampled from: the interpolation error
    falls as the square of the spacing (trilinear interpolation is second
    order), and so does the difference of a transport in the map to the
    transport in the analytic field; its Jacobian, which uses the map's
    gradient (first order in the spacing), converges linearly;
  * a map of a uniform field gives the uniform-field transport;
  * the RKN step's Jacobian in the map against central differences at fixed
    step size (exact); the whole transport's Jacobian against central
    differences only to 5e-3: those also see the adaptive step sizes move
    with the input, and where a step crosses a cell face the field's
    gradient jumps, so the step's truncation error is no longer of fifth
    order and that motion shows;
  * a fit in the map agrees with the fit in the analytic field, and the gap
    falls as the square of the spacing.
"""
import numpy as np
import pytest
from scipy.interpolate import RegularGridInterpolator

from paper_2105_01796_amd import synth

SOL = synth.Field(1, (0.0, 0.0, 2.0), 1e-7)
DIAG = [0, 6, 11, 15, 18, 20]


def _grid_axes(m):
    nz, ny, nx, _ = m.map_values.shape
    return [m.map_origin[a] + m.map_spacing[a] * np.arange(n) for a, n in enumerate((nx, ny, nz))]


def test_map_interpolation_is_trilinear(oracle_lib):
    rng = np.random.default_rng(3)
    vals = rng.standard_normal((7, 6, 5, 3))            # [z][y][x][3], an arbitrary table
    m = synth.Field(2, (0.0, 0.0, 0.0), 0.0, vals, (-10.0, 5.0, -30.0), (4.0, 2.5, 10.0))
    ax = _grid_axes(m)
    interp = [RegularGridInterpolator(ax, vals[..., c].transpose(2, 1, 0), method="linear") for c in range(3)]
    lo = np.array([a[0] for a in ax])
    hi = np.array([a[-1] for a in ax])
    for _ in range(200):
        r = lo + (hi - lo) * rng.random(3)
        B, dB = oracle_lib.field_at(m, r)
        ref = np.array([f(r)[0] for f in interp])
        assert np.abs(B - ref).max() < 1e-13
        for b in range(3):
            e = 1e-6 * m.map_spacing[b]
            # stay inside the cell for the difference quotient
            u = (r[b] - lo[b]) / m.map_spacing[b]
            if min(u - np.floor(u), np.ceil(u) - u) < 1e-3:
                continue
            rp, rm = r.copy(), r.copy()
            rp[b] += e
            rm[b] -= e
            fd = np.array([(f(rp)[0] - f(rm)[0]) / (2 * e) for f in interp])
            assert np.abs(dB[:, b] - fd).max() < 1e-7
    # outside the grid the point is clamped to the boundary; no derivative along clamped axes
    r = np.array([hi[0] + 50.0, 0.5 * (lo[1] + hi[1]) + 0.3, lo[2] - 7.0])
    B, dB = oracle_lib.field_at(m, r)
    rc = np.array([hi[0], r[1], lo[2]])
    assert np.abs(B - np.array([f(rc)[0] for f in interp])).max() < 1e-13
    assert np.all(dB[:, 0] == 0.0) and np.all(dB[:, 2] == 0.0) and np.any(dB[:, 1] != 0.0)


def test_sampled_solenoid_converges_quadratically(oracle_lib):
    rng = np.random.default_rng(4)
    pts = np.stack([rng.uniform(0, 900, 100), rng.uniform(-300, 300, 100), rng.uniform(-4000, 4000, 100)], 1)
    err = {}
    for h in (40.0, 20.0):
        m = synth.sample_field_map(SOL, (-50.0, -350.0, -4200.0), (950.0, 350.0, 4200.0), (h, h, h))
        e = 0.0
        for r in pts:
            B, _ = oracle_lib.field_at(m, r)
            Ba, _ = oracle_lib.field_at(SOL, r)
            e = max(e, np.abs(B - Ba).max())
        err[h] = e
    # |d2 Bz/dz2| = 2 a B0 = 4e-7 T/mm^2: the error is at most h^2/8 of that
    assert err[40.0] <= 40.0 ** 2 / 8 * 4e-7 * 1.01
    assert 3.0 < err[40.0] / err[20.0] < 5.0


def test_transport_in_maps(oracle_lib):
    det = synth.telescope(30)
    x = np.array([0.0, 150.0, 0.05, 0.9, 0.7, 0.0])
    # a map of a uniform field is that field
    uni = synth.Field(0, (0.3, -0.5, 1.7), 0.0)
    mu = synth.sample_field_map(uni, (-50.0, -300.0, -300.0), (950.0, 300.0, 1000.0), (50.0, 50.0, 50.0))
    st, xu, Fu, tu = oracle_lib.transport(det, uni, 0, 20, x)
    st2, xm, Fm, tm = oracle_lib.transport(det, mu, 0, 20, x)
    assert st == st2 == 0 and tu == tm
    assert np.abs(xm - xu).max() < 1e-12 and np.abs(Fm - Fu).max() < 1e-11
    # a map of the solenoid: the transport converges to the analytic one as h^2,
    # its Jacobian as h
    st, xa, Fa, _ = oracle_lib.transport(det, SOL, 0, 20, x)
    scale = np.maximum(np.abs(Fa), np.abs(Fa).max(axis=0, keepdims=True) * 1e-3)
    d, dF = {}, {}
    for h in (40.0, 20.0, 10.0):
        m = synth.sample_field_map(SOL, (-50.0, -400.0, -200.0), (950.0, 400.0, 1200.0), (h, h, h))
        st, xm, Fm, _ = oracle_lib.transport(det, m, 0, 20, x)
        assert st == 0
        d[h] = np.abs(xm[:2] - xa[:2]).max()
        dF[h] = np.max(np.abs(Fm - Fa) / scale)
    assert d[40.0] < 5e-3 and 3.0 < d[40.0] / d[20.0] < 5.0 and 3.0 < d[20.0] / d[10.0] < 5.0
    assert dF[20.0] < 5e-3 and 1.5 < dF[20.0] / dF[10.0] < 2.5
    # the whole transport's Jacobian against central differences (see above)
    m = synth.sample_field_map(SOL, (-50.0, -400.0, -200.0), (950.0, 400.0, 1200.0), (40.0, 40.0, 40.0))
    J = np.zeros((6, 6))
    for j in range(6):
        e = 1e-6
        a, b = x.copy(), x.copy()
        a[j] += e
        b[j] -= e
        J[:, j] = (oracle_lib.transport(det, m, 0, 20, a)[1] - oracle_lib.transport(det, m, 0, 20, b)[1]) / (2 * e)
    Fm = oracle_lib.transport(det, m, 0, 20, x)[2]
    scale = np.maximum(np.abs(Fm), np.abs(Fm).max(axis=0, keepdims=True) * 1e-3)
    assert np.max(np.abs(J - Fm) / scale) < 5e-3


def test_rkn_step_jacobian_in_a_map(oracle_lib):
    m = synth.sample_field_map(SOL, (-50.0, -400.0, -200.0), (950.0, 400.0, 1200.0), (40.0, 40.0, 40.0))
    F = np.array([13.0, 5.0, 151.0, 0.1, 0.6, 0.05, np.sqrt(1 - 0.6 ** 2 - 0.05 ** 2), 0.7])
    for h in (5.0, 30.0, 60.0):           # within one cell, and across cell faces
        Fn, D, _ = oracle_lib.rkn_step(m, F, h)
        J = np.zeros((8, 8))
        for j in range(8):
            a, b = F.copy(), F.copy()
            a[j] += 1e-6
            b[j] -= 1e-6
            J[:, j] = (oracle_lib.rkn_step(m, a, h)[0] - oracle_lib.rkn_step(m, b, h)[0]) / 2e-6
        assert np.abs(J - D).max() < 1e-7


def test_fit_in_the_map_matches_the_analytic_field(oracle_lib):
    ev5 = synth.make_config(5, 300)
    ev6 = synth.make_config(6, 300)
    assert np.array_equal(ev5.loc, ev6.loc) and ev6.field.kind == 2
    r5 = oracle_lib.fit(ev5)
    sd = np.sqrt(r5.tgt_cov[DIAG])
    gap = {}
    for h in (50.0, 25.0):
        ev6.field = synth.sample_field_map(ev5.field, (-50.0, -1000.0, -6000.0), (950.0, 1000.0, 6000.0), (h, h, h))
        r6 = oracle_lib.fit(ev6)
        ok = (r5.status == 0) & (r6.status == 0)
        assert ok.mean() > 0.99
        gap[h] = np.max(np.abs(r6.tgt_par[:, ok] - r5.tgt_par[:, ok]) / sd[:, ok])
    # worst track (0.6 GeV, the longest path): 0.11 sigma in q/p at 25 mm; median 1e-3 sigma
    assert gap[25.0] < 0.2 and 3.0 < gap[50.0] / gap[25.0] < 5.0
