"""HIP fit with the perigee target (Sect. 2; Sect. 5.2) vs the CPU oracle's,
through the C ABI.  Same bars as the seed-surface target (parity.py): FP64
relative 1e-9 (1e-8 on the solenoid workload), identical status and ndf;
mixed precision within 1e-3 sigma.
"""
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
from parity import attach_offsets, compare, par_err  # noqa: E402
from test_gpu_parity import TOL, _announce, _fit, _sampled, kf  # noqa: E402,F401

import oracle  # noqa: E402
from paper_2105_01796_amd import synth  # noqa: E402

pytestmark = pytest.mark.gpu

PERIGEE = 1   # KF_TARGET_PERIGEE
REFS = [(0.0, 0.0, 0.0), (-30.0, 4.0, 2.0)]   # on the seed plane's track origin; 30 mm behind it


def _ref(ev, c, **kw):
    return attach_offsets(oracle.fit(ev, extras=True, perigee=np.array(c), **kw), ev)


@pytest.mark.parametrize("cfg,n", [(1, 100), (2, 3000), (3, 3000), (5, 2000)])
def test_perigee_fp64(kf, cfg, n):
    _announce(f"C{cfg} perigee fp64 n={n}")
    ev = synth.make_config(cfg, n)
    for c in REFS:
        ref = _ref(ev, c)
        for sched in (1, 2):
            out = _fit(kf, ev, schedule=sched, target=PERIGEE, perigee=c)
            compare(out, ref, tol=TOL[cfg], label=f"C{cfg} perigee {c} sched {sched}")


def test_perigee_with_two_filter_and_mixed(kf):
    _announce("C2 perigee with the two-filter smoother; mixed precision")
    ev = synth.make_config(2, 3000)
    c = REFS[1]
    out = _fit(kf, ev, target=PERIGEE, perigee=c, smoother=1)
    compare(out, _ref(ev, c, smoother="two_filter"), label="C2 perigee two-filter")
    out = _fit(kf, ev, target=PERIGEE, perigee=c, precision=kf.KF_PREC_MIXED)
    ref = _ref(ev, c)
    assert np.array_equal(out.status.cpu().numpy(), ref.status)
    _, st = par_err(out.tgt_par, ref.tgt_par, ref.tgt_cov)
    print(f"  perigee mixed C2: max |d|/sigma {st.max():.2e}", flush=True)
    assert st.max() < 1e-3


def test_perigee_failures(kf):
    """A perigee the step cap does not reach fails the track (status, NaN
    outputs) while its neighbours keep theirs."""
    _announce("C1 perigee failures (step cap)")
    ev = synth.make_config(1, 100)
    for c, ms in (((-2000.0, 0.0, 0.0), 2), ((-500.0, 30.0, 0.0), 6)):
        out = _fit(kf, ev, target=PERIGEE, perigee=c, max_steps=ms)
        ref = _ref(ev, c, max_steps=ms)
        compare(out, ref, label=f"C1 perigee {c} max_steps {ms}")
        st = out.status.cpu().numpy()
        assert (st == kf.KF_ST_STEP_CAP).sum() > 0


def test_perigee_full_size_sampled_and_staged(kf):
    _announce("C2 perigee 1e5 tracks sampled; staged equals device")
    import torch
    ev = synth.make_config(2)
    c = REFS[1]
    out = _fit(kf, ev, target=PERIGEE, perigee=c)
    rng = np.random.default_rng(21)
    idx = np.unique(np.concatenate([[0, ev.n_tracks - 1], rng.choice(ev.n_tracks, 500, replace=False)]))
    compare(_sampled(out, ev, idx), _ref(ev.subset(idx), c), label="C2 perigee full/sampled")
    small = ev.subset(np.arange(4000))
    dev = _fit(kf, small, extras=False, schedule=2, target=PERIGEE, perigee=c)
    bh = kf.Batch.staged_from_event(small)
    sp = kf.StagedPlan(bh, kf.Options(schedule=2, target=PERIGEE, perigee=c), n_chunks=3, n_streams=2)
    host = sp.run()
    torch.cuda.synchronize()
    for name in ("par", "cov", "tgt_par", "tgt_cov", "chi2", "status"):
        assert np.array_equal(getattr(host, name).numpy(), getattr(dev, name).cpu().numpy(), equal_nan=True), name


def test_staged_and_captured_variants_equal_device_fit(kf):
    """The host-staged path and a captured graph give the device fit bit for
    bit with the perigee target, the two-filter smoother and a field map."""
    _announce("staged / graph equal device fit: two-filter, perigee, field map")
    import torch
    cases = [(synth.make_config(2, 3000), dict(smoother=1)),
             (synth.make_config(3, 3000), dict(target=PERIGEE, perigee=REFS[1], smoother=1)),
             (synth.make_config(6, 1500), dict(target=PERIGEE, perigee=REFS[0]))]
    for ev, opt in cases:
        dev = _fit(kf, ev, extras=False, schedule=2, **opt)
        bh = kf.Batch.staged_from_event(ev)
        host = kf.StagedPlan(bh, kf.Options(schedule=2, **opt), n_chunks=3, n_streams=2).run()
        torch.cuda.synchronize()
        g = kf.Plan(kf.Batch.from_event(ev), kf.Options(schedule=2, **opt), extras=False).capture()
        for rep in range(3):
            g.out.par.fill_(-1.0)
            torch.cuda.synchronize()
            g.run()
            torch.cuda.synchronize()
            for name in ("par", "cov", "tgt_par", "tgt_cov", "chi2", "status"):
                want = getattr(dev, name).cpu().numpy()
                assert np.array_equal(getattr(g.out, name).cpu().numpy(), want, equal_nan=True), (ev.name, rep, name)
                if rep == 0:
                    assert np.array_equal(getattr(host, name).numpy(), want, equal_nan=True), (ev.name, name)
        g.release()
