"""Pins of the oracle's gradients (forward-mode dual numbers through the fit).

  * central finite differences (h = 1e-6 in mm / rad / GeV^-1 / ns) of the
    scalar L = sum g_chi2 chi2 + sum g_par . smoothed + sum g_tgt . target,
    with respect to the hits, the alignment of every surface and the seed;
  * the envelope theorem for the chi2 gradient with respect to a hit: for the
    least-squares objective d(min chi2)/dm_k = 2 V_k^-1 (m_k - H x_{k|n}); the
    extended filter satisfies it to linearisation level.
"""
import numpy as np
import pytest

from paper_2105_01796_amd import synth


def _L(oracle_lib, ev, g_chi2, g_par, g_tgt, **kw):
    r = oracle_lib.fit(ev, **kw)
    assert np.all(r.status == 0)
    return (g_chi2 * r.chi2).sum() + (g_par * r.par).sum() + (g_tgt * r.tgt_par).sum()


def _fd(oracle_lib, ev, g, setter, h=1e-6, **kw):
    setter(ev, +h); lp = _L(oracle_lib, ev, *g, **kw)
    setter(ev, -2 * h); lm = _L(oracle_lib, ev, *g, **kw)
    setter(ev, +h)
    return (lp - lm) / (2 * h)


@pytest.mark.parametrize("cfg", [1, 2, 4])
def test_vjp_matches_central_differences(oracle_lib, cfg):
    ev = synth.make_config(cfg, 3, seed=4004)
    rng = np.random.default_rng(5)
    g = (np.ones(ev.n_tracks), rng.standard_normal((6, ev.n_hits)), rng.standard_normal((6, ev.n_tracks)))
    g_meas, g_align, g_seed = oracle_lib.fit_vjp(ev, *g)
    scale_m = np.abs(g_meas).max()
    for hidx in [0, 4, 9, 13, 22, 29]:
        for a in range(2):
            def set_m(e, d, hidx=hidx, a=a):
                e.loc[a, hidx] += d
            fd = _fd(oracle_lib, ev, g, set_m)
            assert abs(fd - g_meas[a, hidx]) < 1e-5 * max(abs(g_meas[a, hidx]), 1e-2 * scale_m), (hidx, a)
    for t in range(ev.n_tracks):
        for c in range(6):
            h = 1e-6 if c != 4 else 1e-8
            def set_s(e, d, t=t, c=c):
                e.seed_par[c, t] += d
            fd = _fd(oracle_lib, ev, g, set_s, h=h)
            assert abs(fd - g_seed[c, t]) < 1e-5 * max(abs(g_seed[c, t]), 1e-2 * np.abs(g_seed[:, t]).max())
    base = ev.detector
    scale_a = np.abs(g_align).max(axis=1)
    for s in [1, 5, 10]:
        for c in range(6):
            def set_a(e, d, s=s, c=c):
                al = np.zeros((6, base.n))
                set_a.off = getattr(set_a, "off", 0.0) + d
                al[c, s] = set_a.off
                e.detector = synth.misalign(base, al)
            fd = _fd(oracle_lib, ev, g, set_a)
            ev.detector = base
            assert abs(fd - g_align[c, s]) < 1e-5 * max(abs(g_align[c, s]), 1e-2 * scale_a[c]), (s, c, fd, g_align[c, s])


def test_chi2_gradient_envelope_theorem(oracle_lib):
    ev = synth.make_config(1, 20, seed=4005)
    r = oracle_lib.fit(ev)
    g_meas, _, _ = oracle_lib.fit_vjp(ev, np.ones(ev.n_tracks))
    V = ev.cov
    res = ev.loc - r.par[:2]
    det = V[0] * V[2] - V[1] ** 2
    env = 2 * np.stack([(V[2] * res[0] - V[1] * res[1]) / det, (-V[1] * res[0] + V[0] * res[1]) / det])
    rel = np.abs(g_meas - env).max() / np.abs(env).max()
    assert rel < 1e-3
