"""HIP two-filter smoother (Sect. 2, Fig. 2) vs the CPU oracle's, through the C ABI.

The same bars as the RTS path (parity.py): FP64 relative 1e-9 per element
(1e-8 on the solenoid workload), identical status, ndf and RKN trial counts
(>= 99.9 % of hits); mixed precision within 1e-3 sigma of the FP64 oracle.
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

TWO = 1   # KF_SMOOTHER_TWO_FILTER


def _ref(ev, scale=oracle.DEFAULT_BWD_SCALE, **kw):
    return attach_offsets(oracle.fit(ev, extras=True, smoother="two_filter", bwd_scale=scale, **kw), ev)


@pytest.mark.parametrize("cfg,n", [(1, 100), (2, 3000), (3, 3000), (4, 2000), (5, 2000)])
def test_two_filter_fp64_launch_shapes(kf, cfg, n):
    _announce(f"C{cfg} two-filter fp64 n={n}")
    ev = synth.make_config(cfg, n)
    ref = _ref(ev)
    for sched, block, occ in ((1, 256, 1), (2, 64, 1), (2, 128, 2), (1, 64, 3)):
        out = _fit(kf, ev, schedule=sched, block=block, occupancy=occ, smoother=TWO)
        compare(out, ref, tol=TOL[cfg], label=f"C{cfg} two-filter sched {sched} block {block} occ {occ}")


def test_two_filter_backward_scale(kf):
    """bwd_scale reaches the kernel (0 selects the default 1e3)."""
    _announce("C2 two-filter bwd_scale 1e2 / 1e5 / default")
    ev = synth.make_config(2, 2000)
    for scale in (1e2, 1e5):
        out = _fit(kf, ev, smoother=TWO, bwd_scale=scale)
        compare(out, _ref(ev, scale), label=f"C2 two-filter scale {scale:g}")
    out = _fit(kf, ev, smoother=TWO, bwd_scale=0.0)
    compare(out, _ref(ev, 1e3), label="C2 two-filter default scale")


@pytest.mark.parametrize("cfg,n", [(2, 3000), (5, 2000)])
def test_two_filter_mixed_within_1e3_sigma(kf, cfg, n):
    _announce(f"C{cfg} two-filter mixed n={n}")
    ev = synth.make_config(cfg, n)
    out = _fit(kf, ev, precision=kf.KF_PREC_MIXED, smoother=TWO)
    ref = _ref(ev)
    assert np.array_equal(out.status.cpu().numpy(), ref.status)
    _, sp = par_err(out.par, ref.par, ref.cov)
    _, st = par_err(out.tgt_par, ref.tgt_par, ref.tgt_cov)
    print(f"  two-filter mixed C{cfg}: max |d|/sigma hits {sp.max():.2e} target {st.max():.2e}", flush=True)
    assert sp.max() < 1e-3 and st.max() < 1e-3


def test_two_filter_failure_modes(kf):
    """Every failure status next to good tracks, as the RTS edge-case batch."""
    _announce("two-filter edge cases")
    ev = synth.make_config(3, 300)
    off = ev.hit_offsets
    ev.loc[0, off[3] + 1] = np.nan
    ev.cov[2, off[5]] = -1.0
    ev.surface_id[off[7] + 2] = 500
    ev.seed_cov[0, 9] = 0.0
    ev.seed_par[2, 11] = np.pi / 2
    for sched in (1, 2):
        out = _fit(kf, ev, schedule=sched, smoother=TWO)
        compare(out, _ref(ev), label=f"two-filter edge sched {sched}")
    out = _fit(kf, synth.make_config(1, 64), max_steps=1, smoother=TWO)
    assert np.all(out.status.cpu().numpy() == kf.KF_ST_STEP_CAP)


def test_two_filter_full_size_sampled(kf):
    _announce("C2 two-filter full size (1e5 tracks), sampled parity")
    ev = synth.make_config(2)
    out = _fit(kf, ev, smoother=TWO)
    rng = np.random.default_rng(12)
    idx = np.unique(np.concatenate([[0, ev.n_tracks - 1], rng.choice(ev.n_tracks, 600, replace=False)]))
    compare(_sampled(out, ev, idx), _ref(ev.subset(idx)), label="C2 two-filter full/sampled")
    assert np.all(out.status.cpu().numpy() == 0)


def test_two_filter_autotuner_and_graph(kf):
    """The autotuner keeps the smoother (fused shapes only) and a captured plan
    replays the same result."""
    _announce("two-filter autotune + graph plan")
    import torch
    ev = synth.make_config(3, 4000)
    b = kf.Batch.from_event(ev)
    p = kf.Plan(b, kf.Options(smoother=TWO), extras=True)
    opt, ms = p.autotune()
    assert opt.smoother == TWO and opt.split_smoother == 0 and ms > 0
    eager = p.run()
    torch.cuda.synchronize()
    ref = _ref(ev)
    compare(eager, ref, label="two-filter autotuned")
    ref_t = {n: getattr(eager, n).clone() for n in ("par", "cov", "tgt_par", "tgt_cov", "chi2")}
    g = kf.Plan(b, opt, extras=False).capture()
    for rep in range(3):
        g.out.par.fill_(-1.0)                      # eager work between replays
        torch.cuda.synchronize()
        g.run()
        torch.cuda.synchronize()
        for n, v in ref_t.items():
            assert torch.equal(getattr(g.out, n), v), (rep, n)
    g.release()


def test_two_filter_and_perigee_solenoid_sampled(kf):
    """The solenoid workload at 2e5 tracks with the two-filter smoother and
    the perigee target together, checked on sampled tracks."""
    _announce("C5 2e5 tracks, two-filter + perigee, sampled parity")
    ev = synth.make_config(5, 200_000)
    out = _fit(kf, ev, smoother=TWO, target=1, perigee=(0.0, 0.0, 0.0))
    rng = np.random.default_rng(55)
    idx = np.unique(np.concatenate([[0, ev.n_tracks - 1], rng.choice(ev.n_tracks, 400, replace=False)]))
    ref = attach_offsets(oracle.fit(ev.subset(idx), extras=True, smoother="two_filter", perigee=np.zeros(3)),
                         ev.subset(idx))
    compare(_sampled(out, ev, idx), ref, tol=TOL[5], label="C5 two-filter perigee sampled")
