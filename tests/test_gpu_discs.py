"""HIP fit on disc measuring surfaces (polar local coordinates, azimuth
straddling +-pi) vs the CPU oracle, through the C ABI.  Workload C7: the C2
telescope measured on discs.  FP64 relative 1e-9, identical status and ndf;
mixed precision within 1e-3 sigma.
"""
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
from parity import attach_offsets, compare, par_err  # noqa: E402
from test_gpu_parity import _announce, _fit, _sampled, kf  # noqa: E402,F401

import oracle  # noqa: E402
from paper_2105_01796_amd import synth  # noqa: E402

pytestmark = pytest.mark.gpu


def _ref(ev, **kw):
    return attach_offsets(oracle.fit(ev, extras=True, **kw), ev)


def test_discs_fp64_launch_shapes(kf):
    _announce("C7 (discs) fp64 n=3000")
    ev = synth.make_config(7, 3000)
    ref = _ref(ev)
    for sched, block, occ, split, jac in ((1, 256, 1, 0, 0), (2, 64, 1, 0, 0), (2, 128, 2, 1, 0), (1, 64, 1, 0, 1)):
        out = _fit(kf, ev, schedule=sched, block=block, occupancy=occ, split_smoother=split, jacobians=jac)
        compare(out, ref, label=f"C7 sched {sched} block {block} occ {occ} split {split} jac {jac}")


def test_discs_other_options(kf):
    _announce("C7 discs: two-filter, perigee, solenoid, mixed, bad seed surface")
    ev = synth.make_config(7, 2000)
    compare(_fit(kf, ev, smoother=1), _ref(ev, smoother="two_filter"), label="C7 two-filter")
    compare(_fit(kf, ev, target=1, perigee=(0.0, 0.0, 0.0)), _ref(ev, perigee=np.zeros(3)), label="C7 perigee")
    out = _fit(kf, ev, precision=kf.KF_PREC_MIXED)
    ref = _ref(ev)
    assert np.array_equal(out.status.cpu().numpy(), ref.status)
    _, sp = par_err(out.par, ref.par, ref.cov)
    _, st = par_err(out.tgt_par, ref.tgt_par, ref.tgt_cov)
    print(f"  discs mixed C7: max |d|/sigma hits {sp.max():.2e} target {st.max():.2e}", flush=True)
    assert sp.max() < 1e-3 and st.max() < 1e-3
    # discs in a solenoid-like field
    evs = synth.make_config(7, 1000)
    evs.field = synth.Field(1, (0.0, 0.0, 2.0), 1e-7)
    compare(_fit(kf, evs), _ref(evs), tol=1e-8, label="C7 solenoid")
    # a disc as seed surface is refused per track
    bad = synth.make_config(7, 200)
    bad.detector.stype = bad.detector.stype.copy()
    bad.detector.stype[0] = 1
    out = _fit(kf, bad)
    assert np.all(out.status.cpu().numpy() == kf.KF_ST_BAD_INPUT)
    # an unknown type on a hit surface fails the tracks that cross it, as in the oracle
    odd = synth.telescope_event(300, 71, ragged=(4, 8), center_offset=(0.0, 100.0, 0.0), discs=True)
    odd.detector.stype = odd.detector.stype.copy()
    odd.detector.stype[4] = 2
    out = _fit(kf, odd)
    ref = _ref(odd)
    st = out.status.cpu().numpy()
    assert np.array_equal(st, ref.status) and np.any(st == kf.KF_ST_BAD_INPUT) and np.any(st == 0)
    compare(out, ref, label="C7 unknown type on surface 4")


def test_discs_full_size_sampled(kf):
    _announce("C7 discs 1e5 tracks, sampled parity")
    ev = synth.make_config(7)
    out = _fit(kf, ev)
    rng = np.random.default_rng(7)
    idx = np.unique(np.concatenate([[0, ev.n_tracks - 1], rng.choice(ev.n_tracks, 500, replace=False)]))
    compare(_sampled(out, ev, idx), _ref(ev.subset(idx)), label="C7 sampled")
