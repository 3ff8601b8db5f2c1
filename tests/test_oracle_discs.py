"""Pins of the oracle's disc surfaces: measuring surfaces whose local
coordinates are polar, (r, phi) about the surface centre in its (u, v) plane
(the surface-type dispatch the survey ranks next; Sect. 4.1 names the local
<-> global transforms and their Jacobians).

References, none of them the oracle's code:
  * B = 0: the straight line's crossing of the plane in closed form, turned
    into polar coordinates with numpy;
  * the transport Jacobians into and out of a disc: central differences;
  * noise-free disc hits with the seed at the truth give back the truth;
  * fitted tracks on a disc telescope whose phi straddles +-pi: pulls are
    standard normal at the target and at every disc (phi residuals wrapped);
  * the two-filter smoother agrees with RTS there as on planes;
  * a disc as the seed surface is refused.
"""
import numpy as np
import pytest

from paper_2105_01796_amd import synth

DIAG = [0, 6, 11, 15, 18, 20]
MU = 0.1056583755
C = 299.792458


def _disc_det(n=10):
    det = synth.telescope(n)
    det.center[:, 1:] += np.array([0.0, 100.0, 0.0])[:, None]
    det.stype = np.ones(det.n, np.int32)
    det.stype[0] = 0
    return det


def _wrap(a):
    return np.angle(np.exp(1j * a))


def test_straight_line_onto_a_disc(oracle_lib):
    det = _disc_det()
    fld = synth.Field(0, (0.0, 0.0, 0.0), 0.0)
    for x, sb in [([0.3, -1.2, 0.09, 1.38, -0.2, 0.7], 4), ([-2.0, 5.0, -0.05, 1.7, 1.5, -3.0], 10)]:
        x = np.array(x)
        st, xo, F, tr = oracle_lib.transport(det, fld, 0, sb, x)
        assert st == 0
        phi, th = x[2], x[3]
        T = np.array([np.cos(phi) * np.sin(th), np.sin(phi) * np.sin(th), np.cos(th)])
        r0 = np.array([0.0, x[0], x[1]])                  # seed plane x = 0: u = y, v = z
        s = (det.center[0, sb] - r0[0]) / T[0]
        r = r0 + s * T
        a, b = r[1] - det.center[1, sb], r[2] - det.center[2, sb]
        ref = np.array([np.hypot(a, b), np.arctan2(b, a), phi, th, x[4],
                        x[5] + s * np.sqrt(1 + MU * MU * x[4] ** 2) / C])
        assert np.allclose(xo, ref, rtol=1e-13, atol=1e-12)


@pytest.mark.parametrize("field", [synth.Field(0, (0.0, 0.0, 0.0), 0.0), synth.Field(0, (0.0, 0.0, 2.0), 0.0),
                                   synth.Field(1, (0.0, 0.0, 2.0), 1e-7)])
def test_disc_transport_jacobians(oracle_lib, field):
    det = _disc_det()
    # plane -> disc, disc -> disc (forwards and backwards)
    x0 = np.array([0.3, 10.0, 0.06, 1.5, 0.5, 0.2])
    st, xd, _, _ = oracle_lib.transport(det, field, 0, 3, x0)
    assert st == 0 and abs(abs(xd[1]) - np.pi) < 0.5           # phi near +-pi
    for sa, sb, x in ((0, 3, x0), (3, 7, xd), (3, 1, xd)):
        st, xo, F, _ = oracle_lib.transport(det, field, sa, sb, x)
        assert st == 0
        J = np.zeros((6, 6))
        for j in range(6):
            e = 1e-6
            a, b = x.copy(), x.copy()
            a[j] += e
            b[j] -= e
            ya, yb = oracle_lib.transport(det, field, sa, sb, a)[1], oracle_lib.transport(det, field, sa, sb, b)[1]
            d = ya - yb
            d[1] = _wrap(d[1])
            J[:, j] = d / (2 * e)
        scale = np.maximum(np.abs(F), np.abs(F).max(axis=0, keepdims=True) * 1e-3)
        assert np.max(np.abs(J - F) / scale) < 3e-5, (sa, sb)


def test_noise_free_disc_fit_returns_truth(oracle_lib):
    ev = synth.telescope_event(50, 11, bz=2.0, center_offset=(0.0, 100.0, 0.0), discs=True)
    ev.loc = np.ascontiguousarray(ev.truth_hit[:2])
    ev.seed_par = ev.truth_par0.copy()
    r = oracle_lib.fit(ev)
    assert np.all(r.status == 0)
    d = r.tgt_par - ev.truth_par0
    assert np.abs(d[:2]).max() < 1e-6 and np.abs(d[2:4]).max() < 1e-8
    dh = r.par - ev.truth_hit
    dh[1] = _wrap(dh[1])
    assert np.abs(dh[0]).max() < 1e-6 and np.abs(dh[1]).max() < 1e-8
    assert r.chi2.max() < 1e-8


@pytest.mark.parametrize("smoother", ["rts", "two_filter"])
def test_disc_pulls_are_standard_normal(oracle_lib, smoother):
    ev = synth.make_config(7, 10000, seed=2005)
    assert np.any(ev.loc[1] > 3.0) and np.any(ev.loc[1] < -3.0)     # phi straddles +-pi
    r = oracle_lib.fit(ev, smoother=smoother)
    assert np.all(r.status == 0)
    N = ev.n_tracks
    p = (r.tgt_par - ev.truth_par0) / np.sqrt(r.tgt_cov[DIAG])
    assert np.all(np.abs(p.mean(axis=1)) < 4 / np.sqrt(N)), p.mean(axis=1)
    assert np.all(np.abs(p.std(axis=1) - 1) < 4 / np.sqrt(2 * N)), p.std(axis=1)
    dh = r.par - ev.truth_hit
    dh[1] = _wrap(dh[1])
    ph = dh / np.sqrt(r.cov[DIAG])
    for s in np.unique(ev.surface_id):
        q = ph[:, ev.surface_id == s]
        M = q.shape[1]
        assert np.all(np.abs(q.mean(axis=1)) < 4.5 / np.sqrt(M)), (s, q.mean(axis=1))
        assert np.all(np.abs(q.std(axis=1) - 1) < 4.5 / np.sqrt(2 * M)), (s, q.std(axis=1))
    nmeas = 2 * np.diff(ev.hit_offsets)
    assert abs((r.chi2 - nmeas).sum() / np.sqrt(2 * nmeas.sum())) < 4
    assert np.all(np.abs(r.par[1]) <= np.pi)


def test_disc_seed_surface_is_refused(oracle_lib):
    ev = synth.make_config(7, 20, seed=2006)
    ev.detector.stype = ev.detector.stype.copy()
    ev.detector.stype[0] = 1
    r = oracle_lib.fit(ev)
    assert np.all(r.status == oracle_lib.ST_BAD_INPUT)
