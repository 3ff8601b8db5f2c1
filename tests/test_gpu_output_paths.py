"""The two output paths of the RTS smoother (kf_config.output): KF_OUT_STAGED
(the wave's smoothed states staged in LDS and written out every two smoother
steps) and KF_OUT_SLOTS (each state through its workspace slot, then the
tile flush) compute the same smoother and only route its results, so every
output must be equal bit for bit, on every workload and launch shape, with
failed tracks among good ones, and meet the oracle's bar.  Also: the one-step
stage (taken when the two-step stage does not fit the LDS, here 512 surfaces
with 256-thread workgroups) and the autotuner with the output axis.
"""
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
from parity import SOLENOID_FLOOR_ROWS, attach_offsets, compare  # noqa: E402
from test_gpu_parity import _announce, kf  # noqa: E402,F401

import oracle  # noqa: E402
from paper_2105_01796_amd import synth  # noqa: E402

pytestmark = pytest.mark.gpu

FIELDS = ("par", "cov", "tgt_par", "tgt_cov", "chi2", "ndf", "status")


def _fit(kf, ev, **opt):
    import torch
    out = kf.Plan(kf.Batch.from_event(ev), kf.Options(**opt), extras=True).run()
    torch.cuda.synchronize()
    return out


def _same(a, b, label):
    for name in FIELDS:
        x, y = getattr(a, name).cpu().numpy(), getattr(b, name).cpu().numpy()
        ok = np.array_equal(x, y, equal_nan=True) if x.dtype.kind == "f" else np.array_equal(x, y)
        assert ok, f"{label}: {name} differs between the staged and slot output paths"


SHAPES = [dict(schedule=1, block=256), dict(schedule=2, block=64), dict(schedule=2, block=64, jacobians=1),
          dict(schedule=1, block=64, split_smoother=1), dict(schedule=2, block=128, occupancy=2),
          dict(schedule=2, block=64, precision=1)]


@pytest.mark.parametrize("cfg,n", [(1, 100), (2, 3000), (3, 3000), (5, 2000), (7, 2000), (8, 2000)])
def test_output_paths_bitwise(kf, cfg, n):
    _announce(f"output paths C{cfg} n={n}")
    ev = synth.make_config(cfg, n)
    staged_default = None
    for sh in SHAPES:
        if cfg == 8 and sh.get("occupancy", 1) != 1:
            continue                                   # cylinders and straws: one wave per SIMD
        print(f"  shape {sh}", flush=True)
        a = _fit(kf, ev, output=kf.KF_OUT_STAGED, **sh)
        b = _fit(kf, ev, output=kf.KF_OUT_SLOTS, **sh)
        _same(a, b, f"C{cfg} {sh}")
        if sh == SHAPES[1]:
            staged_default = a
    ref = attach_offsets(oracle.fit(ev, extras=True), ev)
    compare(staged_default, ref, floor_rows=SOLENOID_FLOOR_ROWS if cfg == 5 else None, label=f"C{cfg} staged")


def test_output_paths_failure_batch(kf):
    _announce("output paths: failure batch")
    ev = synth.make_config(3, 300)
    off = ev.hit_offsets
    ev.loc[0, off[3] + 1] = np.nan
    ev.cov[2, off[5]] = -1.0
    ev.surface_id[off[7] + 2] = 500
    ev.seed_cov[0, 9] = 0.0
    ev.seed_par[2, 11] = np.pi / 2
    cnt = np.diff(off).astype(np.int64)
    keep = np.ones(ev.n_hits, bool)
    for t, k in [(13, 2), (14, 1), (15, 0)]:
        keep[off[t] + k: off[t + 1]] = False
        cnt[t] = k
    ev.loc, ev.cov, ev.surface_id, ev.truth_hit = ev.loc[:, keep], ev.cov[:, keep], ev.surface_id[keep], ev.truth_hit[:, keep]
    ev.hit_offsets = np.concatenate([[0], np.cumsum(cnt)]).astype(np.int32)
    ref = attach_offsets(oracle.fit(ev, extras=True), ev)
    for sh in SHAPES[:4]:
        a = _fit(kf, ev, output=kf.KF_OUT_STAGED, **sh)
        b = _fit(kf, ev, output=kf.KF_OUT_SLOTS, **sh)
        _same(a, b, f"failure batch {sh}")
        compare(a, ref, label=f"failure batch staged {sh}")


def test_one_step_stage_and_autotuner(kf):
    """512 surfaces with 256-thread workgroups leave no LDS for the two-step
    stage: the one-step stage is taken, with the same results."""
    import torch
    _announce("output paths: one-step stage (512 surfaces), autotuner")
    ev = synth.telescope_event(400, 91, n_planes=511, pitch=1.0, bz=2.0, x_over_X0=0.001, ms=True, ragged=(8, 40))
    assert ev.detector.n == 512
    a = _fit(kf, ev, schedule=1, block=256, output=kf.KF_OUT_STAGED)
    b = _fit(kf, ev, schedule=1, block=256, output=kf.KF_OUT_SLOTS)
    _same(a, b, "512 surfaces")
    compare(a, attach_offsets(oracle.fit(ev, extras=True), ev), label="512 surfaces staged")
    ev = synth.make_config(3, 5000)
    plan = kf.Plan(kf.Batch.from_event(ev), kf.Options(), extras=True)
    opt, ms = plan.autotune()
    assert opt.output in (kf.KF_OUT_STAGED, kf.KF_OUT_SLOTS) and ms > 0
    out = plan.run()
    torch.cuda.synchronize()
    print(f"  autotuned: schedule {opt.schedule} block {opt.block} occupancy {opt.occupancy} output "
          f"{'staged' if opt.output == kf.KF_OUT_STAGED else 'slots'} {ms:.3f} ms", flush=True)
    compare(out, attach_offsets(oracle.fit(ev, extras=True), ev), label="autotuned with the output axis")
