"""HIP fit in a tabulated field (KF_FIELD_MAP, trilinear) vs the CPU oracle,
through the C ABI.  Workload C6: the solenoid tracks of C5 with the field
given as the solenoid sampled every 25 mm.  Bars as for the solenoid (the
tracks are the same): FP64 relative 1e-9 per element, with the fitted loc1
and theta variance on the seed plane held to the FP64 floor of 1e-8
(parity.py); the two-filter and perigee variants keep 1e-8 for the whole
result; identical status and ndf; mixed precision within 1e-3 sigma.
"""
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
from parity import attach_offsets, compare, par_err  # noqa: E402
from test_gpu_parity import FLOOR, TOL, _announce, _fit, _sampled, kf  # noqa: E402,F401

import oracle  # noqa: E402
from paper_2105_01796_amd import synth  # noqa: E402

pytestmark = pytest.mark.gpu


def _ref(ev, **kw):
    return attach_offsets(oracle.fit(ev, extras=True, **kw), ev)


def test_map_fp64_launch_shapes(kf):
    _announce("C6 (solenoid map) fp64 n=2000")
    ev = synth.make_config(6, 2000)
    ref = _ref(ev)
    for sched, block, occ, split in ((1, 256, 1, 0), (2, 64, 1, 0), (2, 128, 2, 0), (2, 64, 1, 1), (1, 256, 2, 1)):
        out = _fit(kf, ev, schedule=sched, block=block, occupancy=occ, split_smoother=split)
        compare(out, ref, floor_rows=FLOOR[5], label=f"C6 sched {sched} block {block} occ {occ} split {split}")


def test_map_with_other_options(kf):
    _announce("C6 map: recomputed Jacobians, two-filter, perigee, mixed")
    ev = synth.make_config(6, 1500)
    compare(_fit(kf, ev, jacobians=kf.KF_JAC_RECOMPUTE), _ref(ev), floor_rows=FLOOR[5], label="C6 recompute")
    compare(_fit(kf, ev, smoother=1), _ref(ev, smoother="two_filter"), tol=TOL[5], label="C6 two-filter")
    c = (0.0, 0.0, 0.0)
    compare(_fit(kf, ev, target=1, perigee=c), _ref(ev, perigee=np.array(c)), tol=TOL[5], label="C6 perigee")
    out = _fit(kf, ev, precision=kf.KF_PREC_MIXED)
    ref = _ref(ev)
    assert np.array_equal(out.status.cpu().numpy(), ref.status)
    _, sp = par_err(out.par, ref.par, ref.cov)
    _, st = par_err(out.tgt_par, ref.tgt_par, ref.tgt_cov)
    print(f"  map mixed C6: max |d|/sigma hits {sp.max():.2e} target {st.max():.2e}", flush=True)
    assert sp.max() < 1e-3 and st.max() < 1e-3


def test_map_full_size_sampled(kf):
    _announce("C6 map 1e5 tracks, sampled parity")
    ev = synth.make_config(6, 100_000)
    out = _fit(kf, ev)
    rng = np.random.default_rng(6)
    idx = np.unique(np.concatenate([[0, ev.n_tracks - 1], rng.choice(ev.n_tracks, 400, replace=False)]))
    compare(_sampled(out, ev, idx), _ref(ev.subset(idx)), floor_rows=FLOOR[5], label="C6 sampled")
