"""Element-wise comparison of the HIP fit with the CPU oracle.

Tolerances (FP64 path, relative 1e-9 per element):
  parameters  |g - o| <= tol * max(|o|, sigma_o)
  covariance  |g - o| <= tol * sqrt(C_ii C_jj)
  chi2        |g - o| <= tol * max(chi2, 1)
In the solenoid field (C5, and C6 with the field as a map) two elements of the
fitted state on the seed plane sit at the FP64 rounding floor: loc1 (z on the
plane x = 0) and the theta variance C33.  On the most forward tracks
(|eta| 2.3-2.5) the fit extrapolates from hits metres out in z back to the seed
plane, so rounding of ~1e-16 relative on metre-scale positions is ~1e-9 of the
20 um target precision; the oracle compiled with and without FMA contraction
already differs by 2e-9 there (tests/test_oracle_noise_floor.py).  Those two
elements get SOLENOID_FLOOR = 1e-8 (observed worst 3.5e-9 and 2.3e-9 on 3000
tracks); every other element of those workloads (every per-hit state and
covariance, chi2, the other target elements, worst observed 4.1e-10) keeps
1e-9.
Status and ndf must be identical.  RKN trial counts must be identical on at
least 99.9 % of the hits: the landing test compares a distance computed from
positions of ~1e3 mm (rounding ~1e-13 mm) with land_tol, so a residual that
falls within rounding of the threshold may take one more landing iteration on
one side; the final second-order move onto the plane makes the result
independent of that iteration (the values are still held to the bar above).
Mixed path: |g - o| <= 1e-3 sigma_o for the parameters.
"""
import numpy as np

PK = [(i, j) for i in range(6) for j in range(i, 6)]
DIAG = [PK.index((i, i)) for i in range(6)]

SOLENOID_FLOOR = 1e-8
# target rows held to SOLENOID_FLOOR in the solenoid field: loc1 and C33
SOLENOID_FLOOR_ROWS = {"tgt_par": (1,), "tgt_cov": (PK.index((3, 3)),)}


def _np(t):
    return t.detach().cpu().numpy() if hasattr(t, "detach") else np.asarray(t)


def par_err(g, o, ocov):
    sig = np.sqrt(np.abs(ocov[DIAG]))
    d = np.abs(_np(g) - o)
    return d / np.maximum(np.abs(o), sig), d / sig


def cov_err(g, o):
    sig = np.sqrt(np.abs(o[DIAG]))
    scale = np.stack([sig[i] * sig[j] for (i, j) in PK])
    return np.abs(_np(g) - o) / scale


def compare(out, ref, tol=1e-9, sel_hits=None, sel_tracks=None, check_trials=True, label="", floor_rows=None,
            floor_tol=SOLENOID_FLOOR):
    """Return a dict of worst errors; assert the FP64 bar.  floor_rows: rows of
    tgt_par / tgt_cov held to floor_tol instead of tol (SOLENOID_FLOOR_ROWS in
    the solenoid field)."""
    ok = ref.status == 0
    st = _np(out.status)
    assert np.array_equal(st, ref.status), f"{label} status differs: {np.nonzero(st != ref.status)[0][:10]}"
    assert np.array_equal(_np(out.ndf), ref.ndf), f"{label} ndf differs"
    hits_ok = np.repeat(ok, np.diff(ref_offsets(ref)))
    rp, _ = par_err(out.par, ref.par, ref.cov)
    rc = cov_err(out.cov, ref.cov)
    tp, _ = par_err(out.tgt_par, ref.tgt_par, ref.tgt_cov)
    tc = cov_err(out.tgt_cov, ref.tgt_cov)
    chi = np.abs(_np(out.chi2) - ref.chi2) / np.maximum(ref.chi2, 1.0)
    floor_rows = floor_rows or {}
    fp = list(floor_rows.get("tgt_par", ()))
    fc = list(floor_rows.get("tgt_cov", ()))
    keep_p = [i for i in range(6) if i not in fp]
    keep_c = [q for q in range(21) if q not in fc]
    res = dict(par=rp[:, hits_ok].max(initial=0), cov=rc[:, hits_ok].max(initial=0),
               tgt_par=tp[keep_p][:, ok].max(initial=0), tgt_cov=tc[keep_c][:, ok].max(initial=0),
               chi2=chi[ok].max(initial=0))
    for k, v in res.items():
        assert v <= tol, f"{label} {k}: max rel err {v:.3e} > {tol:.0e}"
    if fp or fc:
        res["tgt_floor"] = max(tp[fp][:, ok].max(initial=0) if fp else 0.0, tc[fc][:, ok].max(initial=0) if fc else 0.0)
        assert res["tgt_floor"] <= floor_tol, f"{label} floor elements: max rel err {res['tgt_floor']:.3e}"
    print(f"  {label}: worst " + ", ".join(f"{k} {v:.2e}" for k, v in res.items()), flush=True)
    # failed tracks: NaN outputs
    bad = ~ok
    if bad.any():
        assert np.all(np.isnan(_np(out.tgt_par)[:, bad])) and np.all(np.isnan(_np(out.chi2)[bad]))
    if check_trials and out.trials is not None and ref.trials is not None:
        tr = _np(out.trials)
        same = (tr[hits_ok] == ref.trials[hits_ok]).mean() if hits_ok.any() else 1.0
        res["trials_same"] = same
        assert same >= 0.999, f"{label} RKN trial counts agree on only {same:.5f} of hits"
    return res


def ref_offsets(ref):
    return ref._offsets


def attach_offsets(ref, ev):
    ref._offsets = ev.hit_offsets
    return ref
