"""The solenoid workload at its declared size: 1e6 tracks over 30 planes in
the inhomogeneous solenoid field (ragged 8-30 hits), FP64 and mixed
precision, forward fit and adjoint, through the C ABI.

Every check is on sampled tracks that the oracle fits (or differentiates) as
a sub-batch: tracks are independent, so a track's fit and its rows of the
measurement and seed gradients do not depend on the rest of the batch.  The
alignment gradient sums over every track; it is checked by additivity over
two halves of the batch and bitwise run-to-run equality.

Bars: FP64 fit as everywhere (relative 1e-9 per element, the two solenoid
floor elements of the seed-plane state 1e-8); mixed fit 1e-3 sigma; FP64
adjoint relative 1e-5 against the oracle's dual-number gradient (per
element, floor 1e-3 of the gradient row's largest magnitude); mixed adjoint
1e-3 of the row's largest magnitude (the bar derived in test_gpu_adjoint).
"""
import os
import sys
from types import SimpleNamespace

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
from parity import SOLENOID_FLOOR_ROWS, attach_offsets, compare, par_err  # noqa: E402

import oracle  # noqa: E402
from paper_2105_01796_amd import synth  # noqa: E402

pytestmark = pytest.mark.gpu

N_FULL = 1_000_000


@pytest.fixture(scope="module")
def kf():
    import torch
    from paper_2105_01796_amd import kfmi
    assert torch.cuda.is_available()
    kfmi.lib()
    return kfmi


@pytest.fixture(scope="module")
def c5():
    print(f"C5: generating {N_FULL} tracks", flush=True)
    ev = synth.make_config(5, N_FULL)
    rng = np.random.default_rng(55)
    idx = np.unique(np.concatenate([[0, ev.n_tracks - 1], rng.choice(ev.n_tracks, 300, replace=False)]))
    off = ev.hit_offsets.astype(np.int64)
    hit_idx = np.concatenate([np.arange(off[i], off[i + 1]) for i in idx])
    return SimpleNamespace(ev=ev, idx=idx, hit_idx=hit_idx, sub=ev.subset(idx), off=off)


def _sampled(out, c):
    g = lambda t: t.detach().cpu().numpy()
    h, i = c.hit_idx, c.idx
    return SimpleNamespace(par=g(out.par)[:, h], cov=g(out.cov)[:, h], tgt_par=g(out.tgt_par)[:, i],
                           tgt_cov=g(out.tgt_cov)[:, i], chi2=g(out.chi2)[i], ndf=g(out.ndf)[i],
                           status=g(out.status)[i], trials=None)


def _fit(kf, ev, **opt):
    import torch
    b = kf.Batch.from_event(ev)
    out = kf.Plan(b, kf.Options(**opt)).run()
    torch.cuda.synchronize()
    return out


def test_c5_full_size_fit_fp64_and_mixed(kf, c5):
    print("C5 1e6 fp64 fit, sampled parity", flush=True)
    ref = attach_offsets(oracle.fit(c5.sub), c5.sub)
    out = _fit(kf, c5.ev)
    st = out.status.cpu().numpy()
    print(f"  tracks ok {int((st == 0).sum())} of {st.size}", flush=True)
    compare(_sampled(out, c5), ref, floor_rows=SOLENOID_FLOOR_ROWS, check_trials=False, label="C5 1e6 fp64")
    del out
    print("C5 1e6 mixed fit, sampled parity", flush=True)
    out = _fit(kf, c5.ev, precision=kf.KF_PREC_MIXED)
    s = _sampled(out, c5)
    assert np.array_equal(s.status, ref.status)
    _, sp = par_err(s.par, ref.par, ref.cov)
    _, stt = par_err(s.tgt_par, ref.tgt_par, ref.tgt_cov)
    print(f"  mixed C5 1e6: max |d|/sigma per param, hits {np.array2string(sp.max(axis=1), precision=2)}"
          f" target {np.array2string(stt.max(axis=1), precision=2)}", flush=True)
    assert sp.max() < 1e-3 and stt.max() < 1e-3


def _close(g, ref, label, rel, floor):
    g = np.atleast_2d(np.asarray(g, dtype=np.float64))
    ref = np.atleast_2d(np.asarray(ref, dtype=np.float64))
    fin = np.isfinite(ref)
    assert np.array_equal(np.isfinite(g), fin), f"{label}: NaN pattern differs"
    r = np.where(fin, ref, 0.0)
    scale = np.abs(r).max(axis=1, keepdims=True)
    den = np.maximum(np.abs(r), floor * scale)
    den = np.where(den > 0, den, 1.0)
    err = np.where(fin, np.abs(np.where(fin, g, 0.0) - r) / den, 0.0)
    worst = err.max() if err.size else 0.0
    print(f"  {label}: worst rel err {worst:.2e}", flush=True)
    assert worst < rel, (label, worst)
    return worst


def _vjp(kf, ev, g, **opt):
    import torch
    b = kf.Batch.from_event(ev)
    dev = b.loc.device
    t = [torch.as_tensor(x, dtype=torch.float64, device=dev) for x in g]
    out = kf.VjpPlan(b, kf.Options(**opt), want_align=True, want_seed=True).run(*t)
    torch.cuda.synchronize()
    return out


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_c5_full_size_adjoint(kf, c5, precision):
    import torch
    print(f"C5 1e6 adjoint ({precision}), sampled rows", flush=True)
    ev = c5.ev
    rng = np.random.default_rng(56)
    g = (rng.uniform(0.5, 1.5, ev.n_tracks), rng.standard_normal((6, ev.n_hits)),
         rng.standard_normal((6, ev.n_tracks)))
    prec = kf.KF_PREC_MIXED if precision == "mixed" else kf.KF_PREC_FP64
    full = _vjp(kf, ev, g, precision=prec)
    st = full.status.cpu().numpy()
    fit_st = _fit(kf, ev, precision=prec).status.cpu().numpy()
    assert np.array_equal(st, fit_st), "adjoint and fit statuses differ"
    i, h = c5.idx, c5.hit_idx
    ref_m, _, ref_s = oracle.fit_vjp(c5.sub, g[0][i], g[1][:, h], g[2][:, i])
    rel, floor = (1e-5, 1e-3) if precision == "fp64" else (1e-3, 1.0)
    _close(full.meas.cpu().numpy()[:, h], ref_m, f"C5 1e6 {precision} meas", rel, floor)
    _close(full.seed.cpu().numpy()[:, i], ref_s, f"C5 1e6 {precision} seed", rel, floor)
    # the alignment gradient: additive over two halves, bitwise reproducible
    half = ev.n_tracks // 2
    off = c5.off
    parts = []
    for lo, hi in ((0, half), (half, ev.n_tracks)):
        sel = np.arange(lo, hi)
        hs = np.arange(off[lo], off[hi])
        parts.append(_vjp(kf, ev.subset(sel), (g[0][sel], g[1][:, hs], g[2][:, sel]),
                          precision=prec).align.cpu().numpy())
    fa = full.align.cpu().numpy()
    assert np.allclose(fa, parts[0] + parts[1], rtol=1e-9, atol=1e-12 * np.abs(fa).max())
    again = _vjp(kf, ev, g, precision=prec)
    # failed tracks (a few dozen tracks that no longer reach a plane) have NaN rows
    assert torch.equal(again.align, full.align)
    assert np.array_equal(again.meas.cpu().numpy(), full.meas.cpu().numpy(), equal_nan=True)
    assert np.array_equal(again.seed.cpu().numpy(), full.seed.cpu().numpy(), equal_nan=True)
