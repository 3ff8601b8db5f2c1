"""kf_fit_tracks_noalloc (the fit with the library's static scratch as its
workspace) against kf_fit_tracks, through the C ABI.

Three calls in a row on one device, each with a smaller input than the one
before (fewer tracks; the last also fewer hits per track), the middle one on
cylinders and straws, both schedules: the outputs equal those of
kf_fit_tracks with a caller workspace bit for bit, and both meet the oracle's
FP64 bar (relative 1e-9 per element).  A batch larger than the scratch is
refused with KF_E_SCRATCH.
"""
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
from parity import attach_offsets, compare  # noqa: E402

import oracle  # noqa: E402
from paper_2105_01796_amd import synth  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def kf():
    import torch
    from paper_2105_01796_amd import kfmi
    assert torch.cuda.is_available()
    kfmi.lib()
    return kfmi


def _new_out(kf, b):
    import torch
    N, H = b.n_tracks, b.n_hits
    f64 = dict(dtype=torch.float64, device=b.loc.device)
    fill = float("nan")
    return kf.Fit(torch.full((6, H), fill, **f64), torch.full((21, H), fill, **f64),
                  torch.full((6, N), fill, **f64), torch.full((21, N), fill, **f64), torch.full((N,), fill, **f64),
                  torch.full((N,), -1, dtype=torch.int32, device=b.loc.device),
                  torch.full((N,), 255, dtype=torch.uint8, device=b.loc.device))


def _same(a, b):
    for name in ("par", "cov", "tgt_par", "tgt_cov", "chi2", "ndf", "status"):
        x = getattr(a, name).cpu().numpy()
        y = getattr(b, name).cpu().numpy()
        assert np.array_equal(x, y, equal_nan=True) if x.dtype.kind == "f" else np.array_equal(x, y), name


@pytest.mark.parametrize("schedule", [1, 2])
def test_noalloc_equals_workspace_fit_on_calls_in_a_row(kf, schedule):
    import torch
    # first call: 3000 ragged tracks of up to 30 hits (the larger input), then
    # 1000 tracks through five cylinders and five layers of straws, then 100
    # tracks of 10 hits on planes in a uniform field with material
    for step, (cfg, n) in enumerate(((3, 3000), (8, 1000), (2, 100))):
        print(f"noalloc: call {step + 1}, C{cfg} n={n} schedule={schedule}", flush=True)
        ev = synth.make_config(cfg, n)
        b = kf.Batch.from_event(ev)
        opt = kf.Options(schedule=schedule, block=64, occupancy=1, waves_per_cu=4)
        ref_gpu = kf.Plan(b, opt).run()
        got = kf.kf_fit_tracks_noalloc(b, _new_out(kf, b), opt)
        torch.cuda.synchronize()
        _same(got, ref_gpu)
        ref = attach_offsets(oracle.fit(ev), ev)
        compare(got, ref, check_trials=False, label=f"noalloc C{cfg} n={n}")


def test_noalloc_refuses_batch_beyond_scratch(kf):
    ev = synth.make_config(2, 20000)      # 313 tiles x 10 hits x 52 doubles > 64 MiB
    b = kf.Batch.from_event(ev)
    with pytest.raises(kf.KFError) as e:
        kf.kf_fit_tracks_noalloc(b, _new_out(kf, b))
    assert e.value.code == kf.KF_E_SCRATCH
