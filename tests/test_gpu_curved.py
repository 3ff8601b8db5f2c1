"""HIP fit on cylinders and straws (lines) vs the CPU oracle, through the C
ABI.  Workload C8: five cylinders about the z axis (hits: z and the
azimuth) and five layers of straws (1-D hits: the signed drift distance) in
a 2 T field, with material.  FP64 relative 1e-9 per element, identical
status and ndf (one measured coordinate per straw hit); mixed precision
within 1e-3 sigma.  Also: the solenoid field and a field map, the two-filter
smoother, the perigee target, the launch shapes these kernels are built for
(one wave per SIMD), the failure cases of the new types, and the entry points
that refuse them.
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


def test_barrel_fp64_launch_shapes(kf):
    _announce("C8 (cylinders, straws) fp64 n=3000")
    ev = synth.make_config(8, 3000)
    ref = _ref(ev)
    assert np.all(ref.ndf == 5 * 2 + 5 * 1 - 5)
    for sched, block, split, jac, wpc in ((1, 256, 0, 0, 0), (2, 64, 0, 0, 0), (2, 128, 1, 0, 0), (1, 64, 0, 1, 0),
                                          (2, 64, 0, 1, 4), (1, 128, 1, 0, 0)):
        label = f"C8 sched {sched} block {block} split {split} jac {jac} wpc {wpc}"
        _announce("  " + label)
        out = _fit(kf, ev, schedule=sched, block=block, occupancy=1, split_smoother=split, jacobians=jac,
                   waves_per_cu=wpc)
        compare(out, ref, label=label)


def test_barrel_other_options(kf):
    _announce("C8: two-filter, perigee, mixed precision")
    ev = synth.make_config(8, 2000)
    compare(_fit(kf, ev, smoother=1), _ref(ev, smoother="two_filter"), label="C8 two-filter")
    compare(_fit(kf, ev, target=1, perigee=(0.0, 0.0, 0.0)), _ref(ev, perigee=np.zeros(3)), label="C8 perigee")
    out = _fit(kf, ev, precision=kf.KF_PREC_MIXED)
    ref = _ref(ev)
    assert np.array_equal(out.status.cpu().numpy(), ref.status)
    _, sp = par_err(out.par, ref.par, ref.cov)
    _, st = par_err(out.tgt_par, ref.tgt_par, ref.tgt_cov)
    print(f"  barrel mixed C8: max |d|/sigma hits {sp.max():.2e} target {st.max():.2e}", flush=True)
    assert sp.max() < 1e-3 and st.max() < 1e-3


def test_barrel_nonuniform_fields(kf):
    _announce("C8 in the solenoid field and in a field map")
    ev = synth.make_config(8, 1000)
    ev.field = synth.Field(1, (0.0, 0.0, 2.0), 1e-7)
    compare(_fit(kf, ev), _ref(ev), label="C8 solenoid")
    compare(_fit(kf, ev, schedule=1, jacobians=1), _ref(ev), label="C8 solenoid recomputed Jacobians")
    evm = synth.make_config(8, 1000)
    evm.field = synth.sample_field_map(synth.Field(1, (0.0, 0.0, 2.0), 1e-7), (-50.0, -200.0, -200.0),
                                       (350.0, 200.0, 200.0), (25.0, 25.0, 25.0))
    compare(_fit(kf, evm), _ref(evm), label="C8 field map")


def test_barrel_failures(kf):
    """Bad inputs of the new types fail exactly the tracks that meet them, as
    in the oracle: a cylinder without a positive radius, a straw hit with a
    non-positive or non-finite variance; a straw hit's unread second
    coordinate may hold anything."""
    _announce("C8 failure cases")
    ev = synth.make_config(8, 400)
    det = ev.detector
    det.radius = det.radius.copy()
    det.radius[3] = 0.0                                  # cylinder 3 (the third layer) has no radius
    off = ev.hit_offsets
    ev.cov = ev.cov.copy()
    ev.loc = ev.loc.copy()
    ev.cov[0, off[5] + 7] = -1.0                         # straw hit with a negative variance
    ev.cov[0, off[9] + 6] = np.nan                       # ... and a NaN one
    ev.loc[1, off[11] + 8] = np.nan                      # unread coordinate of a straw hit
    ev.cov[2, off[11] + 8] = -5.0                        # unread variance of a straw hit
    ref = _ref(ev)
    out = _fit(kf, ev)
    st = out.status.cpu().numpy()
    assert np.all(st == kf.KF_ST_BAD_INPUT), "every track crosses cylinder 3"
    assert np.array_equal(st, ref.status)
    det.radius[3] = synth.BARREL_RADII[2]
    ref = _ref(ev)
    out = _fit(kf, ev)
    st = out.status.cpu().numpy()
    assert st[5] == kf.KF_ST_BAD_INPUT and st[9] == kf.KF_ST_BAD_INPUT and st[11] == 0
    compare(out, ref, label="C8 bad straw hits")
    # an unknown type fails the tracks that cross it
    det.stype = det.stype.copy()
    det.stype[7] = 9
    out = _fit(kf, ev)
    ref = _ref(ev)
    st = out.status.cpu().numpy()
    assert np.array_equal(st, ref.status) and np.any(st == kf.KF_ST_BAD_INPUT) and np.any(st == 0)
    compare(out, ref, label="C8 unknown type on surface 7")


def test_barrel_entry_points(kf):
    """Staged and graph-captured fits equal the device fit bit for bit; the
    autotuner stays at one wave per SIMD; an occupancy above one and the
    adjoint are refused before any launch."""
    import torch
    _announce("C8 staged, graph plan, autotuner, refusals")
    ev = synth.make_config(8, 5000)
    dev_fit = _fit(kf, ev, extras=False, schedule=2, block=64)
    bh = kf.Batch.staged_from_event(ev)
    st = kf.StagedPlan(bh, kf.Options(schedule=2, block=64), n_chunks=4, n_streams=2).run()
    plan = kf.Plan(kf.Batch.from_event(ev), kf.Options(schedule=2, block=64)).capture()
    gr = plan.run()
    torch.cuda.synchronize()
    for name in ("par", "cov", "tgt_par", "tgt_cov", "chi2", "ndf", "status"):
        for other, lab in ((st, "staged"), (gr, "graph")):
            x, y = getattr(dev_fit, name).cpu().numpy(), getattr(other, name).cpu().numpy()
            assert np.array_equal(x, y, equal_nan=True), f"{lab} {name}"
    tp = kf.Plan(kf.Batch.from_event(ev), kf.Options())
    opt, ms = tp.autotune()
    assert opt.occupancy == 1 and ms > 0
    out = tp.run()
    torch.cuda.synchronize()
    compare(out, _ref(ev), label="C8 autotuned")
    b = kf.Batch.from_event(ev)
    with pytest.raises(kf.KFError) as e:
        kf.Plan(b, kf.Options(occupancy=2)).run()
    assert e.value.code == kf.KF_E_VALUE
    g = torch.ones(ev.n_tracks, dtype=torch.float64, device=b.loc.device)
    with pytest.raises(kf.KFError) as e:
        kf.kf_fit_tracks_vjp(b, g)
    assert e.value.code == kf.KF_E_VALUE


def test_barrel_full_size_sampled(kf):
    _announce("C8 1e5 tracks, sampled parity")
    ev = synth.make_config(8)
    out = _fit(kf, ev)
    rng = np.random.default_rng(8)
    idx = np.unique(np.concatenate([[0, ev.n_tracks - 1], rng.choice(ev.n_tracks, 500, replace=False)]))
    compare(_sampled(out, ev, idx), _ref(ev.subset(idx)), label="C8 sampled")
