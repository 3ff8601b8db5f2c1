"""Pins of the oracle's curved measuring surfaces: cylinders (local position
along the axis and azimuth about it) and lines -- straws, whose hit is the
signed distance of closest approach to the wire, a one-dimensional
measurement (the survey's "more surface types"; Sect. 4.1 names the local
<-> global transforms and their Jacobians).

References, none of them the oracle's code:
  * B = 0: the straight line's crossing of a cylinder (a quadratic) and its
    closest approach to a wire (two skew lines) in closed form with numpy;
  * uniform B: the generator's exact helix, Newton on its closed form, onto
    the cylinder and to the wire's closest approach;
  * solenoid: scipy's DOP853 at 1e-12 with an event on the surface's
    constraint;
  * transport Jacobians into, between and out of cylinders and lines:
    central differences, in three fields;
  * the one-dimensional update: joint-Gaussian conditioning of the state on
    one linear observation (numpy);
  * noise-free hits with the seed at the truth give back the truth; pulls of
    fitted tracks through the barrel (workload C8) are standard normal at the
    target, at every cylinder and for the straws' drift distance; the chi2
    follows its degrees of freedom (one per straw hit).
"""
import numpy as np
import pytest

from paper_2105_01796_amd import synth

DIAG = [0, 6, 11, 15, 18, 20]
MU = 0.1056583755
C = 299.792458
KB = 0.299792458e-3


def _wrap(a):
    return np.angle(np.exp(1j * a))


def _T(phi, th):
    return np.array([np.cos(phi) * np.sin(th), np.sin(phi) * np.sin(th), np.cos(th)])


def _det():
    return synth.barrel_detector()


def _line_frame(w, T):
    m = np.cross(w, T)
    return m / np.linalg.norm(m)


def test_straight_line_onto_a_cylinder_and_a_wire(oracle_lib):
    det = _det()
    fld = synth.Field(0, (0.0, 0.0, 0.0), 0.0)
    for x in ([0.3, -1.2, 0.09, 1.38, -0.2, 0.7], [-2.0, 5.0, -0.05, 1.7, 1.5, -3.0]):
        x = np.array(x)
        T = _T(x[2], x[3])
        r0 = np.array([0.0, x[0], x[1]])                  # seed plane x = 0: u = y, v = z
        g = np.sqrt(1 + MU * MU * x[4] ** 2) / C
        # cylinder 3 (radius 90 about z): |r0_xy + s T_xy| = R
        R = det.radius[3]
        a, b, c = T[0] ** 2 + T[1] ** 2, r0[0] * T[0] + r0[1] * T[1], r0[0] ** 2 + r0[1] ** 2 - R * R
        s = (-b + np.sqrt(b * b - a * c)) / a
        r = r0 + s * T
        ref = np.array([r[2], np.arctan2(r[1], r[0]), x[2], x[3], x[4], x[5] + s * g])
        st, xo, F, tr = oracle_lib.transport(det, fld, 0, 3, x)
        assert st == 0
        assert np.allclose(xo, ref, rtol=1e-13, atol=1e-12), (xo, ref)
        # a wire of the second straw layer (x = 210 mm, y = 0 or the nearest)
        sb = 1 + 5 + 1 * 9 + 4
        c = det.center[:, sb]
        w = np.array([0.0, 0.0, 1.0])
        d0 = c - r0
        tw = T @ w
        s = (d0 @ T - tw * (d0 @ w)) / (1.0 - tw * tw)
        d = r0 + s * T - c
        e = _line_frame(w, T)
        ref = np.array([d @ e, d @ w, x[2], x[3], x[4], x[5] + s * g])
        st, xo, F, tr = oracle_lib.transport(det, fld, 0, sb, x)
        assert st == 0
        assert np.allclose(xo, ref, rtol=1e-12, atol=1e-11), (xo, ref)
        # the closest approach: d's part across the wire is orthogonal to the
        # track, and |loc0| is its length
        dp = d - (d @ w) * w
        assert abs(dp @ T) < 1e-9 and abs(abs(xo[0]) - np.linalg.norm(dp)) < 1e-10


def _helix_start(x):
    """Seed-plane state -> (r0 (3,1), phi, theta) for synth's helix functions."""
    return np.array([[0.0], [x[0]], [x[1]]]), np.array([x[2]]), np.array([x[3]])


def test_uniform_field_onto_a_cylinder_and_a_wire(oracle_lib):
    det = _det()
    bz = 2.0
    fld = synth.Field(0, (0.0, 0.0, bz), 0.0)
    for x in ([0.1, 2.0, 0.05, 1.45, 1 / 1.5, 0.0], [-0.4, -3.0, -0.08, 1.68, -1 / 2.5, 0.0]):
        x = np.array(x)
        r0, ph, th = _helix_start(x)
        rho = -x[4] * KB * bz
        # cylinder 5 (radius 150)
        s = synth.helix_to_cylinder(r0, ph, th, rho, det.radius[5])
        r = synth.helix_point(r0, ph, th, rho, s)[:, 0]
        st, xo, F, tr = oracle_lib.transport(det, fld, 0, 5, x)
        assert st == 0
        assert abs(xo[0] - r[2]) < 1e-6 and abs(_wrap(xo[1] - np.arctan2(r[1], r[0]))) * 150 < 1e-6
        assert abs(_wrap(xo[2] - (ph[0] + rho * s[0]))) < 1e-8
        # straw: the wire nearest to where the helix crosses x = 240 mm
        sx = synth.helix_to_plane(r0, ph, th, rho, np.array([240.0, 0.0, 0.0]), np.array([1.0, 0.0, 0.0]))
        yc = synth.helix_point(r0, ph, th, rho, sx)[1, 0]
        i = int(np.clip(np.rint((yc + 40.0) / 10.0), 0, 8))
        sb = 1 + 5 + 2 * 9 + i
        c = det.center[:, sb]
        s = synth.helix_to_wire(r0, ph, th, rho, c[0], np.array([c[1]]))
        r = synth.helix_point(r0, ph, th, rho, s)[:, 0]
        T = synth.helix_dir(ph, th, rho, s)[:, 0]
        d = r - c
        e = _line_frame(np.array([0.0, 0.0, 1.0]), T)
        st, xo, F, tr = oracle_lib.transport(det, fld, 0, sb, x)
        assert st == 0
        assert abs(xo[0] - d @ e) < 1e-6 and abs(xo[1] - d[2]) < 1e-6, (xo[:2], d @ e, d[2])


def test_solenoid_onto_a_cylinder_and_a_wire(oracle_lib):
    from scipy.integrate import solve_ivp
    det = _det()
    a_sol, b0 = 1e-7, 2.0
    fld = synth.Field(1, (0.0, 0.0, b0), a_sol)
    x = np.array([0.2, 40.0, 0.06, 1.2, 1 / 0.9, 0.0])
    lam = x[4]

    def rhs(s, y):
        r, T = y[:3], y[3:]
        B = np.array([a_sol * b0 * r[0] * r[2], a_sol * b0 * r[1] * r[2], b0 * (1 - a_sol * r[2] ** 2)])
        return np.concatenate([T, lam * KB * np.cross(T, B)])

    y0 = np.concatenate([[0.0, x[0], x[1]], _T(x[2], x[3])])
    R = det.radius[4]
    ev_cyl = lambda s, y: y[0] ** 2 + y[1] ** 2 - R * R
    ev_cyl.terminal = True
    sol = solve_ivp(rhs, (0, 2000), y0, method="DOP853", rtol=1e-12, atol=1e-12, events=ev_cyl)
    r = sol.y_events[0][0][:3]
    st, xo, F, tr = oracle_lib.transport(det, fld, 0, 4, x)
    assert st == 0
    assert abs(xo[0] - r[2]) < 1e-7 and abs(_wrap(xo[1] - np.arctan2(r[1], r[0]))) * R < 1e-7
    sb = 1 + 5 + 4 * 9 + 5                 # wire at (300, 10, 0)
    c = det.center[:, sb]
    ev_pca = lambda s, y: (y[0] - c[0]) * y[3] + (y[1] - c[1]) * y[4]
    ev_pca.terminal = True
    ev_pca.direction = 1
    sol = solve_ivp(rhs, (0, 2000), y0, method="DOP853", rtol=1e-12, atol=1e-12, events=ev_pca)
    y = sol.y_events[0][0]
    d = y[:3] - c
    e = _line_frame(np.array([0.0, 0.0, 1.0]), y[3:])
    # RKN truncation at the default tolerance (1e-4 mm per step) over the
    # ~0.35 m path, and shrinking with the tolerance
    for tol, bound in ((1e-4, 5e-7), (1e-7, 5e-9)):
        st, xo, F, tr = oracle_lib.transport(det, fld, 0, sb, x, tol=tol)
        assert st == 0
        assert abs(xo[0] - d @ e) < bound and abs(xo[1] - d[2]) < bound, (tol, xo[:2], d @ e, d[2])


@pytest.mark.parametrize("field", [synth.Field(0, (0.0, 0.0, 0.0), 0.0), synth.Field(0, (0.0, 0.0, 2.0), 0.0),
                                   synth.Field(1, (0.0, 0.0, 2.0), 1e-7)])
def test_curved_surface_transport_jacobians(oracle_lib, field):
    det = _det()
    x0 = np.array([0.3, 10.0, 0.03, 1.5, 0.5, 0.2])
    st, xc, _, _ = oracle_lib.transport(det, field, 0, 2, x0)          # onto cylinder 2
    assert st == 0
    sw = 1 + 5 + 0 * 9 + 4                                              # wire (180, 0, 0)
    st, xw, _, _ = oracle_lib.transport(det, field, 2, sw, xc)
    assert st == 0
    sw2 = 1 + 5 + 3 * 9 + 4                                             # wire (270, 0, 0)
    cases = ((0, 2, x0), (2, 4, xc), (2, sw, xc), (sw, sw2, xw), (sw, 0, xw), (4, 2, oracle_lib.transport(det, field, 2, 4, xc)[1]))
    for sa, sb, x in cases:
        st, xo, F, _ = oracle_lib.transport(det, field, sa, sb, x)
        assert st == 0, (sa, sb)
        J = np.zeros((6, 6))
        for j in range(6):
            e = 1e-6
            a, b = x.copy(), x.copy()
            a[j] += e
            b[j] -= e
            ya, yb = oracle_lib.transport(det, field, sa, sb, a)[1], oracle_lib.transport(det, field, sa, sb, b)[1]
            d = ya - yb
            d[1:3] = _wrap(d[1:3])
            J[:, j] = d / (2 * e)
        scale = np.maximum(np.abs(F), np.abs(F).max(axis=0, keepdims=True) * 1e-3)
        assert np.max(np.abs(J - F) / scale) < 3e-5, (sa, sb, np.max(np.abs(J - F) / scale))


def test_one_dimensional_update_is_gaussian_conditioning(oracle_lib):
    """A fit whose only measurements are straws: the oracle's update on a line
    equals conditioning on the linear observation loc0.  Checked through a
    field-free two-surface track whose Jacobians are linear: the filtered
    state at the first straw against numpy's conditioning of the predicted
    Gaussian (prediction = the oracle's own transport)."""
    det = _det()
    fld = synth.Field(0, (0.0, 0.0, 0.0), 0.0)
    rng = np.random.default_rng(3)
    x = np.array([0.2, 1.0, 0.02, 1.5, 0.3, 0.0])
    A = rng.standard_normal((6, 6)) * 0.01
    C0 = A @ A.T + np.diag([1e-2, 1e-2, 4e-6, 4e-6, 1e-4, 1.0])
    sw = 1 + 5 + 0 * 9 + 4
    st, xp, F, _ = oracle_lib.transport(det, fld, 0, sw, x)
    Cp = F @ C0 @ F.T
    m, v = xp[0] + 0.05, 0.01
    # conditioning on y = e0 . x + noise(v)
    S = Cp[0, 0] + v
    K = Cp[:, 0] / S
    xf_ref = xp + K * (m - xp[0])
    Cf_ref = Cp - np.outer(K, Cp[0])
    chi2_ref = (m - xp[0]) ** 2 / S
    # the same through the oracle's linear smoother with H = e0: emulate with V11 huge
    # is not what the fit does; use the fit itself on a one-hit line track instead
    ev = synth.barrel_event(1, 5)
    ev.hit_offsets = np.array([0, 3], np.int32)
    ev.surface_id = np.array([sw, sw + 9, sw + 18], np.int32)
    ev.loc = np.array([[m, 0.0, 0.0], [0.0, 0.0, 0.0]])
    ev.cov = np.array([[v, v, v], [0.0, 0.0, 0.0], [0.0, 0.0, 0.0]])
    ev.seed_par = x[:, None].copy()
    ev.seed_cov = np.array([C0[i, j] for i in range(6) for j in range(i, 6)])[:, None]
    ev.field = fld
    ev.multiple_scattering = False
    r = oracle_lib.fit(ev, extras=True)
    assert r.status[0] == 0
    PK = [(i, j) for i in range(6) for j in range(i, 6)]
    Cf = np.zeros((6, 6))
    for q, (i, j) in enumerate(PK):
        Cf[i, j] = Cf[j, i] = r.filt_cov[q, 0]
    assert np.allclose(r.filt_par[:, 0], xf_ref, rtol=1e-12, atol=1e-12)
    assert np.allclose(Cf, Cf_ref, rtol=1e-9, atol=1e-15)
    assert r.ndf[0] == 3 - 4                                  # three 1-D hits, no field: 3 - 4
    assert chi2_ref >= 0


def test_noise_free_barrel_fit_returns_truth(oracle_lib):
    ev = synth.barrel_event(50, 12, bz=2.0)
    ev.loc = np.ascontiguousarray(ev.truth_hit[:2])
    straw = np.isin(ev.surface_id, np.nonzero(ev.detector.stype == 3)[0])
    ev.loc[1, straw] = 0.0
    ev.seed_par = ev.truth_par0.copy()
    r = oracle_lib.fit(ev)
    assert np.all(r.status == 0)
    d = r.tgt_par - ev.truth_par0
    assert np.abs(d[:2]).max() < 1e-6 and np.abs(d[2:4]).max() < 1e-8
    dh = r.par - ev.truth_hit
    dh[1] = _wrap(dh[1])
    assert np.abs(dh[0]).max() < 1e-6
    assert np.abs(dh[1, ~straw]).max() < 1e-8
    assert r.chi2.max() < 1e-8
    assert np.all(r.ndf == 5 * 2 + 5 - 5)


@pytest.mark.parametrize("smoother", ["rts", "two_filter"])
def test_barrel_pulls_are_standard_normal(oracle_lib, smoother):
    ev = synth.make_config(8, 10000, seed=2008)
    r = oracle_lib.fit(ev, smoother=smoother)
    assert np.all(r.status == 0)
    N = ev.n_tracks
    p = (r.tgt_par - ev.truth_par0) / np.sqrt(r.tgt_cov[DIAG])
    assert np.all(np.abs(p.mean(axis=1)) < 4 / np.sqrt(N)), p.mean(axis=1)
    assert np.all(np.abs(p.std(axis=1) - 1) < 4 / np.sqrt(2 * N)), p.std(axis=1)
    dh = r.par - ev.truth_hit
    dh[1] = _wrap(dh[1])
    ph = dh / np.sqrt(r.cov[DIAG])
    stype = ev.detector.stype
    for s in np.unique(ev.surface_id):
        sel = ev.surface_id == s
        M = sel.sum()
        if M < 200:
            continue
        rows = [0, 1] if stype[s] == 2 else [0]
        q = ph[rows][:, sel]
        assert np.all(np.abs(q.mean(axis=1)) < 4.5 / np.sqrt(M)), (s, q.mean(axis=1))
        assert np.all(np.abs(q.std(axis=1) - 1) < 4.5 / np.sqrt(2 * M)), (s, q.std(axis=1))
    nmeas = np.array([sum(2 if stype[s] == 2 else 1 for s in ev.surface_id[a:b])
                      for a, b in zip(ev.hit_offsets[:-1], ev.hit_offsets[1:])])
    assert abs((r.chi2 - nmeas).sum() / np.sqrt(2 * nmeas.sum())) < 4
    assert np.all(r.ndf == nmeas - 5)


def test_curved_surface_inputs_are_checked(oracle_lib):
    ev = synth.make_config(8, 20, seed=2009)
    ev.detector.radius = ev.detector.radius.copy()
    ev.detector.radius[2] = 0.0                      # a cylinder without a radius
    r = oracle_lib.fit(ev)
    assert np.all(r.status == oracle_lib.ST_BAD_INPUT)
    ev = synth.make_config(8, 20, seed=2009)
    straw = np.nonzero(np.isin(ev.surface_id, np.nonzero(ev.detector.stype == 3)[0]))[0]
    ev.cov[0, straw[0]] = -1.0                       # straw variance not positive
    ev.loc[1, straw[1:]] = np.nan                    # unread on a straw: no effect
    r = oracle_lib.fit(ev)
    t_bad = np.searchsorted(ev.hit_offsets, straw[0], side="right") - 1
    assert r.status[t_bad] == oracle_lib.ST_BAD_INPUT
    assert np.sum(r.status == 0) == ev.n_tracks - 1
