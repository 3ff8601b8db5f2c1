"""HIP fit vs the CPU oracle, element by element, through the C ABI.

FP64 path: relative 1e-9 per element (in the solenoid field the fitted loc1
and theta variance on the seed plane are held to the FP64 floor, 1e-8; see
parity.py), identical status and ndf, RKN trial counts identical on >= 99.9 %
of hits.  Mixed path: parameters within 1e-3 sigma.
Full-size runs (1e5 tracks, the benchmark's launch configuration) are checked
on a sample of tracks that the oracle fits one by one (tracks are independent,
so a sub-batch has the same exact answer).
"""
import sys
import os
from types import SimpleNamespace

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
from parity import DIAG, SOLENOID_FLOOR_ROWS, attach_offsets, compare, par_err  # noqa: E402

import oracle  # noqa: E402
from paper_2105_01796_amd import synth  # noqa: E402

pytestmark = pytest.mark.gpu

# FP64 relative bar: 1e-9 per element; in the solenoid field the fitted loc1
# and theta variance on the seed plane are held to the FP64 floor instead
# (SOLENOID_FLOOR_ROWS, see parity.py).  TOL is the whole-result bar that the
# smoother-variant and perigee modules still use for the solenoid.
TOL = {1: 1e-9, 2: 1e-9, 3: 1e-9, 4: 1e-9, 5: 1e-8}
FLOOR = {5: SOLENOID_FLOOR_ROWS}


@pytest.fixture(scope="module")
def kf():
    import torch
    from paper_2105_01796_amd import kfmi
    assert torch.cuda.is_available()
    kfmi.lib()
    return kfmi


def _fit(kf, ev, extras=True, detector=None, **opt):
    import torch
    b = kf.Batch.from_event(ev, detector=detector)
    out = kf.Plan(b, kf.Options(**opt), extras=extras).run()
    torch.cuda.synchronize()
    return out


def _ref(ev, **kw):
    return attach_offsets(oracle.fit(ev, extras=True, **kw), ev)


def _announce(msg):
    print(msg, flush=True)


@pytest.mark.parametrize("schedule,block,occ,split", [(1, 64, 1, 0), (2, 64, 1, 0), (1, 256, 1, 1), (2, 128, 2, 1),
                                                      (1, 64, 3, 0), (2, 256, 3, 1)])
def test_c1_fp64_all_launch_shapes(kf, schedule, block, occ, split):
    _announce(f"C1 fp64 schedule={schedule} block={block} occ={occ} split={split}")
    ev = synth.make_config(1)
    out = _fit(kf, ev, schedule=schedule, block=block, occupancy=occ, split_smoother=split)
    compare(out, _ref(ev), label="C1")


@pytest.mark.parametrize("cfg,n", [(2, 3000), (3, 3000), (4, 2000), (5, 2000)])
def test_configs_fp64_small(kf, cfg, n):
    _announce(f"C{cfg} fp64 n={n}")
    ev = synth.make_config(cfg, n)
    for sched in (1, 2):
        out = _fit(kf, ev, schedule=sched)
        compare(out, _ref(ev), floor_rows=FLOOR.get(cfg), label=f"C{cfg} sched {sched}")


@pytest.mark.parametrize("cfg,n", [(2, 3000), (3, 3000), (5, 2000)])
def test_fused_one_wave_per_simd_shapes(kf, cfg, n):
    """The fused kernel at one wave per SIMD (the benchmarked shape family):
    direct and sorted schedules, 64- to 256-thread groups."""
    _announce(f"C{cfg} fp64 fused occ 1 shapes n={n}")
    ev = synth.make_config(cfg, n)
    ref = _ref(ev)
    for sched, block in ((1, 256), (2, 256), (2, 64), (1, 128)):
        for prec in (kf.KF_PREC_FP64,):
            out = _fit(kf, ev, schedule=sched, block=block, occupancy=1, split_smoother=0, precision=prec)
            compare(out, ref, floor_rows=FLOOR.get(cfg), label=f"C{cfg} fused occ1 sched {sched} block {block}")


@pytest.mark.parametrize("cfg,n", [(1, 100), (2, 3000), (3, 3000), (5, 2000)])
def test_recomputed_jacobians_fp64(kf, cfg, n):
    """KF_JAC_RECOMPUTE: the smoother propagates each filtered state again
    instead of reading a stored Jacobian; same bar as the stored variant."""
    _announce(f"C{cfg} fp64 recomputed Jacobians n={n}")
    ev = synth.make_config(cfg, n)
    ref = _ref(ev)
    for sched, block, occ in ((1, 256, 1), (2, 64, 1), (2, 128, 2)):
        out = _fit(kf, ev, schedule=sched, block=block, occupancy=occ, jacobians=kf.KF_JAC_RECOMPUTE)
        compare(out, ref, floor_rows=FLOOR.get(cfg), label=f"C{cfg} recompute sched {sched} occ {occ}")


@pytest.mark.parametrize("cfg,n,chunks,streams", [(3, 3000, 5, 2), (5, 2000, 3, 3), (2, 1000, 1, 1), (1, 100, 200, 2)])
def test_staged_fit_equals_device_fit(kf, cfg, n, chunks, streams):
    """kf_fit_tracks_staged (pinned host buffers, chunks pipelined over
    streams) gives the device-resident fit bit for bit."""
    _announce(f"C{cfg} staged n={n} chunks={chunks} streams={streams}")
    import torch
    ev = synth.make_config(cfg, n)
    ref = _fit(kf, ev, extras=False, schedule=2)
    b = kf.Batch.staged_from_event(ev)
    p = kf.StagedPlan(b, kf.Options(schedule=2), n_chunks=chunks, n_streams=streams)
    out = p.run()
    torch.cuda.synchronize()
    for name in ("par", "cov", "tgt_par", "tgt_cov", "chi2", "ndf", "status"):
        got, want = getattr(out, name).numpy(), getattr(ref, name).cpu().numpy()
        assert np.array_equal(got, want, equal_nan=True), name


def test_field_free_and_misaligned_geometry(kf):
    _announce("B=0 and misaligned planes, fp64")
    ev = synth.telescope_event(1000, 31, bz=0.0)
    compare(_fit(kf, ev), _ref(ev), label="B=0")
    ev = synth.make_config(4, 1000)
    # give the fitter the tilted/shifted planes the hits were simulated on
    out = _fit(kf, ev, detector=ev.detector_true)
    compare(out, _ref(ev, detector=ev.detector_true), label="misaligned")


@pytest.mark.parametrize("bz", [0.0, 2.0])
def test_zero_qop_seeds(kf, bz):
    """Seeds with q/p = 0 exactly.  Field off: q/p is unobservable and stays 0,
    so every gap is a straight line whose transport Jacobian has a zero q/p
    column (no 0 * inf).  2 T: the first gap is straight, q/p then moves off 0
    through the first update."""
    _announce(f"q/p = 0 seeds, Bz = {bz}")
    ev = synth.telescope_event(500, 41, bz=bz)
    ev.seed_par[4, :] = 0.0
    ref = _ref(ev)
    assert np.all(ref.status == 0)
    for sched in (1, 2):
        compare(_fit(kf, ev, schedule=sched), ref, label=f"q/p=0 Bz={bz} sched {sched}")
    out = _fit(kf, ev, precision=kf.KF_PREC_MIXED)
    _, sp = par_err(out.tgt_par, ref.tgt_par, ref.tgt_cov)
    assert np.array_equal(out.status.cpu().numpy(), ref.status) and sp.max() < 1e-3


def _sampled(out, ev, idx):
    """GPU outputs restricted to tracks idx (with their hits), as numpy."""
    off = ev.hit_offsets.astype(np.int64)
    hit_idx = np.concatenate([np.arange(off[i], off[i + 1]) for i in idx])
    g = lambda t: t.detach().cpu().numpy()
    return SimpleNamespace(par=g(out.par)[:, hit_idx], cov=g(out.cov)[:, hit_idx], tgt_par=g(out.tgt_par)[:, idx],
                           tgt_cov=g(out.tgt_cov)[:, idx], chi2=g(out.chi2)[idx], ndf=g(out.ndf)[idx],
                           status=g(out.status)[idx], trials=g(out.trials)[hit_idx])


@pytest.mark.parametrize("cfg", [2, 3])
def test_full_size_sampled_fp64(kf, cfg):
    _announce(f"C{cfg} fp64 full size (1e5 tracks), sampled parity")
    ev = synth.make_config(cfg)
    out = _fit(kf, ev)                      # default launch configuration (as benchmarked)
    rng = np.random.default_rng(cfg)
    idx = np.sort(np.concatenate([[0, ev.n_tracks - 1], rng.choice(ev.n_tracks, 600, replace=False)]))
    idx = np.unique(idx)
    sub = ev.subset(idx)
    compare(_sampled(out, ev, idx), _ref(sub), label=f"C{cfg} full/sampled")
    st = out.status.cpu().numpy()
    assert np.all(st == 0)


def test_full_size_solenoid_sampled_fp64(kf):
    _announce("C5 fp64 200k tracks, sampled parity")
    ev = synth.make_config(5, 200_000)
    out = _fit(kf, ev)
    rng = np.random.default_rng(5)
    idx = np.unique(np.concatenate([[0, ev.n_tracks - 1], rng.choice(ev.n_tracks, 400, replace=False)]))
    compare(_sampled(out, ev, idx), _ref(ev.subset(idx)), floor_rows=FLOOR[5], label="C5 sampled")


@pytest.mark.parametrize("cfg,n,jac", [(1, 100, 0), (2, 3000, 0), (3, 3000, 0), (5, 2000, 0), (2, 3000, 1),
                                       (5, 2000, 1)])
def test_mixed_precision_within_1e3_sigma(kf, cfg, n, jac):
    _announce(f"C{cfg} mixed n={n} jacobians={'recompute' if jac else 'store'}")
    ev = synth.make_config(cfg, n)
    out = _fit(kf, ev, precision=kf.KF_PREC_MIXED, jacobians=jac)
    ref = _ref(ev)
    assert np.array_equal(out.status.cpu().numpy(), ref.status)
    _, sp = par_err(out.par, ref.par, ref.cov)
    _, st = par_err(out.tgt_par, ref.tgt_par, ref.tgt_cov)
    worst_hit = sp.max(axis=1)
    worst_tgt = st.max(axis=1)
    print(f"  mixed C{cfg}: max |d|/sigma per param, hits {np.array2string(worst_hit, precision=2)}"
          f" target {np.array2string(worst_tgt, precision=2)}", flush=True)
    assert worst_hit.max() < 1e-3 and worst_tgt.max() < 1e-3
    chi = np.abs(out.chi2.cpu().numpy() - ref.chi2)
    assert chi.max() < 1e-3 * np.sqrt(2 * ref.ndf.max())


def test_edge_cases(kf):
    _announce("edge cases")
    import torch
    # no tracks at all
    ev = synth.make_config(1, 5)
    e0 = ev.subset(np.array([], dtype=np.int64))
    b = kf.Batch.from_event(e0)
    out = kf.kf_fit_tracks(b)
    torch.cuda.synchronize()
    assert out.chi2.numel() == 0
    # one batch with every failure mode next to good tracks
    ev = synth.make_config(3, 300)
    off = ev.hit_offsets
    ev.loc[0, off[3] + 1] = np.nan                     # non-finite hit
    ev.cov[2, off[5]] = -1.0                           # non-SPD hit covariance
    ev.surface_id[off[7] + 2] = 500                    # surface id out of range
    ev.seed_cov[0, 9] = 0.0                            # seed covariance not SPD
    ev.seed_par[2, 11] = np.pi / 2                     # moving parallel to the planes
    # a 2-hit track, a 1-hit track and a 0-hit track (too few)
    cnt = np.diff(off).astype(np.int64)
    keep = np.ones(ev.n_hits, bool)
    for t, k in [(13, 2), (14, 1), (15, 0)]:
        keep[off[t] + k: off[t + 1]] = False
        cnt[t] = k
    ev.loc, ev.cov, ev.surface_id, ev.truth_hit = ev.loc[:, keep], ev.cov[:, keep], ev.surface_id[keep], ev.truth_hit[:, keep]
    ev.hit_offsets = np.concatenate([[0], np.cumsum(cnt)]).astype(np.int32)
    for sched, jac in ((1, 0), (2, 0), (2, 1)):
        out = _fit(kf, ev, schedule=sched, jacobians=jac)
        ref = _ref(ev)
        compare(out, ref, label=f"edge sched {sched} jacobians {jac}")
        st = out.status.cpu().numpy()
        assert st[3] == kf.KF_ST_BAD_INPUT and st[5] == kf.KF_ST_BAD_INPUT and st[7] == kf.KF_ST_BAD_INPUT
        assert st[9] == kf.KF_ST_BAD_INPUT and st[11] == kf.KF_ST_NO_INTERSECT
        assert st[13] == st[14] == st[15] == kf.KF_ST_TOO_FEW
        assert (st == 0).sum() == ev.n_tracks - 8
    # tracks longer than the declared max_hits are rejected, others fitted
    ev = synth.make_config(3, 500)
    b = kf.Batch.from_event(ev)
    b.max_hits = 12
    out = kf.Plan(b, kf.Options(), extras=True).run()
    torch.cuda.synchronize()
    n = np.diff(ev.hit_offsets)
    st = out.status.cpu().numpy()
    assert np.all(st[n > 12] == kf.KF_ST_BAD_INPUT) and np.all(st[n <= 12] == 0)
    # step cap: one trial per gap is never enough in a field
    out = _fit(kf, synth.make_config(1, 64), max_steps=1)
    assert np.all(out.status.cpu().numpy() == kf.KF_ST_STEP_CAP)


def test_run_to_run_bitwise_determinism(kf):
    _announce("determinism")
    ev = synth.make_config(3, 20000)
    a = _fit(kf, ev)
    b = _fit(kf, ev)
    for name in ("par", "cov", "tgt_par", "tgt_cov", "chi2"):
        assert np.array_equal(getattr(a, name).cpu().numpy(), getattr(b, name).cpu().numpy(), equal_nan=True), name


def test_graph_plan_replays_match_eager(kf):
    """kf_plan_create records the whole fit (length sort + kernels) into a HIP
    graph.  Replay it several times with eager work and synchronisations in
    between; every replay must equal the eager fit bit for bit."""
    _announce("graph plan replays")
    import torch
    ev = synth.make_config(3, 5000)
    b = kf.Batch.from_event(ev)
    eager = kf.Plan(b, kf.Options(), extras=False).run()
    torch.cuda.synchronize()
    ref = {n: getattr(eager, n).clone() for n in ("par", "cov", "tgt_par", "tgt_cov", "chi2", "status")}
    p = kf.Plan(b, kf.Options(), extras=False).capture()
    for rep in range(4):
        for n in ("par", "tgt_par", "chi2"):
            getattr(p.out, n).fill_(-1.0)                   # eager work between replays
        torch.cuda.synchronize()
        p.run()
        torch.cuda.synchronize()
        for n, v in ref.items():
            assert torch.equal(getattr(p.out, n), v) or (n != "status" and torch.allclose(
                getattr(p.out, n), v, rtol=0, atol=0, equal_nan=True)), (rep, n)
    p.release()


def test_autotuner_picks_a_valid_shape(kf):
    _announce("autotune")
    import torch
    ev = synth.make_config(3, 20000)
    b = kf.Batch.from_event(ev)
    p = kf.Plan(b, kf.Options(), extras=True)
    opt, ms = p.autotune()
    print(f"  autotune C3 20k: {opt} {ms:.3f} ms", flush=True)
    assert ms > 0 and opt.schedule in (1, 2) and opt.block in (64, 256) and opt.occupancy in (1, 2, 3)
    out = p.run()
    torch.cuda.synchronize()
    rng = np.random.default_rng(7)
    idx = np.unique(rng.choice(ev.n_tracks, 300, replace=False))
    compare(_sampled(out, ev, idx), _ref(ev.subset(idx)), label="autotuned")


@pytest.mark.parametrize("cfg,comp", [(7, 1), (2, 0)])
def test_absurd_hit_value_ends(kf, cfg, comp):
    """A finite but absurd hit coordinate (1e200 mm or rad) passes the input
    checks; the angle wrap turns the resulting angle into NaN (reading r28)
    instead of looping, so the track fails (the propagation that follows
    reaches its step cap) exactly as in the oracle, and every other track is
    fitted as usual."""
    _announce(f"absurd hit value: C{cfg} loc{comp} = 1e200")
    ev = synth.make_config(cfg, 200)
    off = ev.hit_offsets
    ev.loc = ev.loc.copy()
    for t in (3, 17):
        ev.loc[comp, off[t] + 4] = 1e200
    ref = _ref(ev)
    assert ref.status[3] == ref.status[17] == kf.KF_ST_STEP_CAP
    for sched in (1, 2):
        out = _fit(kf, ev, schedule=sched)
        compare(out, ref, label=f"absurd hit C{cfg} sched {sched}")
