"""The largest sizes the C ABI accepts: 512 surfaces (the whole table staged
in LDS next to the per-wave areas) and 64 hits per track, against the CPU
oracle through the C ABI -- fit (both smoothers, fused and separate
smoother kernels, stored and recomputed Jacobians) and adjoint (the
per-workgroup LDS stash then forces 64-thread groups, and the alignment
gradient of 512 surfaces takes the chunked reduction)."""
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
from parity import attach_offsets, compare  # noqa: E402
from test_gpu_parity import _announce, _fit, kf  # noqa: E402,F401
from test_gpu_adjoint import _close, _cotangents, _gpu_vjp  # noqa: E402

import oracle  # noqa: E402
from paper_2105_01796_amd import synth  # noqa: E402

pytestmark = pytest.mark.gpu


def _max_event(n):
    # 511 planes 1 mm apart plus the seed plane = 512 surfaces; 60-64 hits per track
    ev = synth.telescope_event(n, 77, n_planes=511, pitch=1.0, bz=2.0, x_over_X0=0.001, ms=True,
                               ragged=(60, 64), name="max")
    assert ev.detector.n == 512 and np.diff(ev.hit_offsets).max() == 64
    return ev


def test_fit_at_max_sizes(kf):
    _announce("512 surfaces, 64 hits: fit shapes")
    ev = _max_event(300)
    ref = attach_offsets(oracle.fit(ev, extras=True), ev)
    for sched, block, occ, split, jac in ((1, 256, 1, 0, 0), (2, 64, 1, 0, 0), (2, 256, 2, 1, 0), (1, 64, 1, 0, 1)):
        out = _fit(kf, ev, schedule=sched, block=block, occupancy=occ, split_smoother=split, jacobians=jac)
        compare(out, ref, label=f"max sched {sched} block {block} occ {occ} split {split} jac {jac}")
    reft = attach_offsets(oracle.fit(ev, extras=True, smoother="two_filter"), ev)
    compare(_fit(kf, ev, smoother=1), reft, label="max two-filter")


def test_vjp_at_max_sizes(kf):
    _announce("512 surfaces, 64 hits: adjoint")
    ev = _max_event(24)
    g = _cotangents(ev, 5)
    ref_m, ref_a, ref_s = oracle.fit_vjp(ev, *g)
    for sched in (1, 2):
        out = _gpu_vjp(kf, ev, g, schedule=sched)
        assert np.all(out.status.cpu().numpy() == 0)
        _close(out.meas.cpu().numpy(), ref_m, f"max sched {sched} meas")
        _close(out.align.cpu().numpy(), ref_a, f"max sched {sched} align")
        _close(out.seed.cpu().numpy(), ref_s, f"max sched {sched} seed")
