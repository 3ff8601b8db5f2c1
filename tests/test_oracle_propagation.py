"""Pins of the oracle's propagation (adaptive RKN, Sect. 4.1) and Jacobians.

References used, none of them the oracle's own code:
  * B = 0: straight line to a plane normal to x, closed form for the bound
    parameters and for their derivatives;
  * uniform B along z: the exact helix, with its crossing of a plane found by
    Newton iteration on the closed-form trajectory;
  * solenoid-like field: scipy's DOP853 at 1e-12 tolerance with an event at
    the plane;
  * every Jacobian: central finite differences of the map it differentiates.
"""
import numpy as np
import pytest
from scipy.integrate import solve_ivp

from paper_2105_01796_amd import synth

C = 299.792458
KB = 0.299792458e-3
MU = 0.1056583755


def _straight(x, dx):
    l0, l1, phi, th, lam, t = x
    s = dx / (np.sin(th) * np.cos(phi))
    out = np.array([l0 + dx * np.tan(phi), l1 + dx / (np.tan(th) * np.cos(phi)), phi, th, lam,
                    t + s * np.sqrt(1 + MU * MU * lam * lam) / C])
    J = np.eye(6)
    J[0, 2] = dx / np.cos(phi) ** 2
    J[1, 2] = dx * np.sin(phi) / (np.tan(th) * np.cos(phi) ** 2)
    J[1, 3] = -dx / (np.sin(th) ** 2 * np.cos(phi))
    g = np.sqrt(1 + MU * MU * lam * lam) / C
    J[5, 2] = g * dx * np.sin(phi) / (np.sin(th) * np.cos(phi) ** 2)
    J[5, 3] = -g * dx * np.cos(th) / (np.sin(th) ** 2 * np.cos(phi))
    J[5, 4] = s * MU * MU * lam / (C * np.sqrt(1 + MU * MU * lam * lam))
    return out, J


@pytest.mark.parametrize("x", [[0.0, 0.0, 0.0, np.pi / 2, 0.5, 0.0],
                               [0.3, -1.2, 0.09, 1.38, -0.2, 0.7],
                               [-2.0, 5.0, -0.3, 1.9, 1.5, -3.0]])
def test_field_free_transport_is_straight_line(oracle_lib, x):
    det = synth.telescope(10)
    fld = synth.Field(0, (0.0, 0.0, 0.0), 0.0)
    x = np.array(x)
    for sa, sb in [(0, 1), (0, 10), (3, 7)]:
        st, xo, F, tr = oracle_lib.transport(det, fld, sa, sb, x)
        assert st == 0 and tr == 1          # one step lands exactly
        ref, J = _straight(x, det.center[0, sb] - det.center[0, sa])
        assert np.allclose(xo, ref, rtol=1e-14, atol=1e-12)
        assert np.allclose(F, J, rtol=1e-12, atol=1e-13)


def _helix_state(x0, lam, bz, xplane):
    phi0, th = x0[2], x0[3]
    rho = np.array([-lam * KB * bz])
    r0 = np.array([[0.0], [x0[0]], [x0[1]]])
    n = np.array([1.0, 0.0, 0.0])
    c = np.array([xplane, 0.0, 0.0])
    # Newton on the closed-form helix (independent of the RKN integrator)
    s = np.array([xplane / (np.sin(th) * np.cos(phi0))])
    for _ in range(50):
        half = 0.5 * rho * s
        ch = np.sin(th) * s * np.sinc(half / np.pi)
        xx = ch * np.cos(phi0 + half)
        g = xx - xplane
        dg = np.sin(th) * np.cos(phi0 + rho * s)
        s = s - g / dg
    half = 0.5 * rho * s
    ch = np.sin(th) * s * np.sinc(half / np.pi)
    y = x0[0] + ch * np.sin(phi0 + half)
    z = x0[1] + s * np.cos(th)
    t = x0[5] + s * np.sqrt(1 + MU * MU * lam * lam) / C
    return np.array([y[0], z[0], phi0 + rho[0] * s[0], th, lam, t[0]])


@pytest.mark.parametrize("p,phi,th,q", [(1.0, 0.1, 1.4, 1), (1.0, -0.1, 1.7, -1), (10.0, 0.05, 1.5, 1),
                                         (0.7, 0.0, 1.57, -1), (3.0, 0.2, 1.2, 1)])
def test_uniform_field_transport_follows_exact_helix(oracle_lib, p, phi, th, q):
    det = synth.telescope(30)
    fld = synth.Field(0, (0.0, 0.0, 2.0), 0.0)
    x = np.array([0.1, -0.2, phi, th, q / p, 0.0])
    errs = {}
    for tol in (1e-4, 1e-6):
        st, xo, F, tr = oracle_lib.transport(det, fld, 0, 30, x, tol=tol)
        assert st == 0
        ref = _helix_state(x, q / p, 2.0, 900.0)
        e = np.abs(xo - ref)
        errs[tol] = e[:2].max()
        assert e[:2].max() < 1e-6          # mm, over 900 mm of flight
        assert e[2:4].max() < 1e-8
        assert e[5] < 1e-8                  # ns (path-length truncation / beta c)
        assert e[4] == 0.0
    # truncation error falls with the tolerance (order-of-magnitude check)
    assert errs[1e-6] < errs[1e-4] / 20 + 1e-12


def test_solenoid_transport_matches_dop853(oracle_lib):
    det = synth.telescope(30)
    a, b0z = 1e-7, 2.0
    fld = synth.Field(1, (0.0, 0.0, b0z), a)
    for (p, phi, th, q, z0) in [(0.8, 0.05, 0.6, 1, 300.0), (5.0, -0.08, 2.6, -1, -500.0), (1.5, 0.0, 1.2, 1, 0.0)]:
        x = np.array([0.0, z0, phi, th, q / p, 0.0])
        lam = q / p

        def rhs(s, y):
            r, T = y[:3], y[3:6]
            B = np.array([a * b0z * r[0] * r[2], a * b0z * r[1] * r[2], b0z * (1 - a * r[2] ** 2)])
            return np.concatenate([T, lam * KB * np.cross(T, B), [np.sqrt(1 + MU * MU * lam * lam) / C]])

        T0 = [np.sin(th) * np.cos(phi), np.sin(th) * np.sin(phi), np.cos(th)]
        y0 = np.concatenate([[0.0, 0.0, z0], T0, [0.0]])
        for sb in (5, 12):
            xp = det.center[0, sb]
            ev = lambda s, y: y[0] - xp
            ev.terminal = True
            ev.direction = 1
            sol = solve_ivp(rhs, (0, 1e5), y0, method="DOP853", rtol=1e-12, atol=1e-12, events=ev)
            ye = sol.y_events[0][0]
            ref = np.array([ye[1], ye[2], np.arctan2(ye[4], ye[3]),
                            np.arctan2(np.hypot(ye[3], ye[4]), ye[5]), lam, ye[6]])
            st, xo, F, tr = oracle_lib.transport(det, fld, 0, sb, x)
            assert st == 0
            assert np.abs(xo[:2] - ref[:2]).max() < 2e-6
            assert np.abs(xo[2:4] - ref[2:4]).max() < 1e-8
            assert abs(xo[5] - ref[5]) < 1e-8


@pytest.mark.parametrize("field", [synth.Field(0, (0.0, 0.0, 2.0), 0.0), synth.Field(0, (0.3, -0.5, 1.7), 0.0),
                                   synth.Field(1, (0.0, 0.0, 2.0), 1e-7)])
def test_rkn_step_jacobian_matches_finite_differences(oracle_lib, field):
    F0 = np.array([120.0, 40.0, 700.0, 0.3, 0.7, 0.1, 0.7, 0.8])
    F0[4:7] /= np.linalg.norm(F0[4:7])
    for h in (5.0, 60.0):
        Fn, D, err = oracle_lib.rkn_step(field, F0, h)
        J = np.zeros((8, 8))
        for j in range(8):
            e = 1e-6
            a, b = F0.copy(), F0.copy()
            a[j] += e
            b[j] -= e
            J[:, j] = (oracle_lib.rkn_step(field, a, h)[0] - oracle_lib.rkn_step(field, b, h)[0]) / (2 * e)
        assert np.abs(J - D).max() < 1e-7 * max(1.0, np.abs(D).max())


@pytest.mark.parametrize("field,x,sb", [
    (synth.Field(0, (0.0, 0.0, 2.0), 0.0), [0.3, -0.2, 0.08, 1.45, 0.5, 0.1], 5),
    (synth.Field(0, (0.0, 0.0, 2.0), 0.0), [-1.0, 2.0, -0.12, 1.7, -1.0, 0.0], 10),
    (synth.Field(1, (0.0, 0.0, 2.0), 1e-7), [0.0, 150.0, 0.05, 0.9, 0.7, 0.0], 20),
])
def test_transport_jacobian_matches_finite_differences(oracle_lib, field, x, sb):
    """F = J_fb P_corr D J_bf against central differences of the whole adaptive
    transport (landing included).  The finite differences also see the step
    sizes move with the input, a truncation-level effect (~1e-6 relative)."""
    det = synth.telescope(30)
    x = np.array(x)
    st, xo, F, tr = oracle_lib.transport(det, field, 0, sb, x)
    assert st == 0
    J = np.zeros((6, 6))
    for j in range(6):
        e = 1e-6 if j != 4 else 1e-7
        a, b = x.copy(), x.copy()
        a[j] += e
        b[j] -= e
        J[:, j] = (oracle_lib.transport(det, field, 0, sb, a)[1] - oracle_lib.transport(det, field, 0, sb, b)[1]) / (2 * e)
    scale = np.maximum(np.abs(F), np.abs(F).max(axis=0, keepdims=True) * 1e-3)
    assert np.max(np.abs(J - F) / scale) < 3e-5


@pytest.mark.parametrize("field,x", [
    (synth.Field(0, (0.0, 0.0, 2.0), 0.0), [0.1, -0.2, 0.1, 1.4, 1.0, 0.0]),
    (synth.Field(0, (0.3, -0.5, 1.7), 0.0), [-1.0, 2.0, -0.12, 1.7, -0.8, 0.3]),
    (synth.Field(1, (0.0, 0.0, 2.0), 1e-7), [0.0, 150.0, 0.05, 0.9, 0.7, 0.0]),
])
def test_backward_transport_retraces_the_trajectory(oracle_lib, field, x):
    """Transport against the direction of flight (the two-filter smoother's
    backward filter, Sect. 2 / Fig. 2): from the state reached on plane 30
    back to plane 0 returns the starting state (the forward leg is pinned to
    the exact helix and to DOP853 above, so this ties the backward leg to the
    true trajectory), time runs backwards, and the backward Jacobian is the
    inverse of the forward one; it also matches central differences."""
    det = synth.telescope(30)
    x = np.array(x)
    st, xo, F, _ = oracle_lib.transport(det, field, 0, 30, x, tol=1e-7)
    assert st == 0
    st, xb, G, tr = oracle_lib.transport(det, field, 30, 0, xo, tol=1e-7)
    assert st == 0 and tr > 1
    assert np.abs(xb[:2] - x[:2]).max() < 1e-6
    assert np.abs(xb[2:4] - x[2:4]).max() < 1e-9
    assert xb[4] == x[4] and abs(xb[5] - x[5]) < 1e-9 and xo[5] > x[5]
    assert np.abs(G @ F - np.eye(6)).max() < 1e-6
    J = np.zeros((6, 6))
    for j in range(6):
        e = 1e-6 if j != 4 else 1e-7
        a, b = xo.copy(), xo.copy()
        a[j] += e
        b[j] -= e
        J[:, j] = (oracle_lib.transport(det, field, 30, 0, a)[1] - oracle_lib.transport(det, field, 30, 0, b)[1]) / (2 * e)
    st, _, G4, _ = oracle_lib.transport(det, field, 30, 0, xo)
    scale = np.maximum(np.abs(G4), np.abs(G4).max(axis=0, keepdims=True) * 1e-3)
    assert np.max(np.abs(J - G4) / scale) < 3e-5


def test_misaligned_plane_transport_lands_on_plane(oracle_lib):
    det = synth.misalign(synth.telescope(10), np.array([[0, 0.1, -0.2, 0.05, 0.0, 0.3, 0, 0, 0, 0, 0]] * 3 +
                                                        [[0, 0.01, 0.02, -0.03, 0.01, 0, 0, 0, 0, 0, 0]] * 3))
    fld = synth.Field(0, (0.0, 0.0, 2.0), 0.0)
    x = np.array([0.1, 0.2, 0.05, 1.5, 0.4, 0.0])
    for sb in (1, 2, 3, 4):
        st, xo, F, tr = oracle_lib.transport(det, fld, 0, sb, x)
        assert st == 0
        # independent check: the state lies on the helix through the start point and on the plane
        R = det.rot[:, sb].reshape(3, 3)
        c = det.center[:, sb]
        r = c + xo[0] * R[:, 0] + xo[1] * R[:, 1]
        rho = -x[4] * KB * 2.0
        s = (xo[2] - x[2]) / rho
        half = 0.5 * rho * s
        ch = np.sin(x[3]) * s * np.sinc(half / np.pi)
        r_h = np.array([ch * np.cos(x[2] + half), x[0] + ch * np.sin(x[2] + half), x[1] + s * np.cos(x[3])])
        assert np.abs(r - r_h).max() < 1e-6
        assert abs(xo[3] - x[3]) < 1e-9


def test_highland_noise_value(oracle_lib):
    """Thin scatterer on a plane normal to x, x/X0 = 0.005.
    Hand value for p = 2 GeV, beta = 2/sqrt(4 + m^2) = 0.99860745265,
    normal incidence: theta0 = 13.6 MeV/(beta p) sqrt(0.005) (1 + 0.038 ln(0.005/beta^2))
                             = 3.84610179e-4 rad."""
    det = synth.telescope(3, x_over_X0=0.005)
    Q = oracle_lib.ms_noise(det, 1, np.array([0.0, 0.0, 0.0, np.pi / 2, 0.5, 0.0]))
    th0 = 3.84610179e-4
    assert abs(np.sqrt(Q[3, 3]) - th0) < 1e-12
    assert abs(np.sqrt(Q[2, 2]) - th0) < 1e-12          # sin(theta) = 1
    assert np.count_nonzero(Q) == 2
    # oblique incidence: the path in X0 grows by 1/|n.T|, phi term by 1/sin^2(theta)
    th, ph = 1.2, 0.3
    Q2 = oracle_lib.ms_noise(det, 1, np.array([0.0, 0.0, ph, th, 0.5, 0.0]))
    beta = 2 / np.sqrt(4 + MU * MU)
    L = 0.005 / (np.sin(th) * np.cos(ph))
    t0 = 0.0136 / (beta * 2) * np.sqrt(L) * (1 + 0.038 * np.log(L / beta ** 2))
    assert abs(Q2[3, 3] - t0 ** 2) < 1e-15 and abs(Q2[2, 2] - t0 ** 2 / np.sin(th) ** 2) < 1e-15
    # no material -> no noise
    assert not np.any(oracle_lib.ms_noise(det, 0, np.array([0.0, 0.0, 0.0, 1.5, 0.5, 0.0])))
