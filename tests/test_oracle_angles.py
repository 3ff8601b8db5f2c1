"""Absurd hit values end the fit (reading r28): an angle of 64 rad or more is
no angle a fit at the detector's scale produces, so the angle wrap turns it
into NaN instead of turning it back by 2 pi without end; the track fails and
every other track is fitted exactly as without it (tracks are independent).
"""
import numpy as np
import pytest

import oracle
from paper_2105_01796_amd import synth


@pytest.mark.parametrize("cfg,comp", [(7, 1), (2, 0), (2, 1)])
def test_absurd_hit_value_fails_only_its_track(cfg, comp):
    ev = synth.make_config(cfg, 40)
    good = oracle.fit(ev)
    off = ev.hit_offsets
    bad = [3, 17]
    ev.loc = ev.loc.copy()
    for t in bad:
        ev.loc[comp, off[t] + 4] = 1e200            # finite, passes the input checks
    out = oracle.fit(ev)
    st = out.status
    assert np.all(st[bad] != 0) and np.all(np.isnan(out.tgt_par[:, bad]))
    keep = np.setdiff1d(np.arange(ev.n_tracks), bad)
    assert np.array_equal(st[keep], good.status[keep])
    assert np.array_equal(out.tgt_par[:, keep], good.tgt_par[:, keep])
    assert np.array_equal(out.chi2[keep], good.chi2[keep])
