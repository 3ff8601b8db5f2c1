"""CPU oracle for the batched Kalman-filter track fit -- TEST INFRASTRUCTURE.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The product (the HIP library and its binding) never
does.  The arithmetic lives in kf_oracle.cpp (plain FP64 C++, one track at a
time, OpenMP over tracks); this module only marshals numpy arrays.

All arrays are component-major ([component][item]) float64 / int32, the same
layout the HIP library takes, so one generated event feeds both.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "kf_oracle.cpp")
LIB = os.path.join(HERE, "libkf_oracle.so")

# status codes (same meaning as the HIP library's per-track status byte)
ST_OK, ST_NO_INTERSECT, ST_STEP_CAP, ST_NOT_SPD, ST_BAD_INPUT, ST_TOO_FEW = range(6)

DEFAULT_TOL = 1e-4
DEFAULT_LAND_TOL = 1e-6
DEFAULT_MAX_STEPS = 1000


def build(force: bool = False) -> str:
    """Compile the oracle with g++ (portable x86-64 code, OpenMP)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        cmd = ["g++", "-O2", "-std=c++17", "-fopenmp", "-fPIC", "-shared", "-Wall", "-Wno-unused-function",
               SRC, "-o", LIB + ".tmp"]
        subprocess.check_call(cmd)
        os.replace(LIB + ".tmp", LIB)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(LIB)
        P = C.c_void_p
        i, d = C.c_int, C.c_double
        fit_args = [i, P, P, P, P, i, P, P, P, P, i, P, d, P, P, i, i, d, d, d, i]
        L.kfo_fit.argtypes = fit_args + [P] * 12 + [i, i, d, i, P, P]
        L.kfo_fit.restype = i
        L.kfo_fit_vjp.argtypes = fit_args + [P] * 6 + [i, P]
        L.kfo_fit_vjp.restype = i
        L.kfo_count_ops.argtypes = fit_args + [P, P]
        L.kfo_count_ops.restype = i
        L.kfo_transport.argtypes = [i, P, P, P, i, P, d, d, d, d, i, i, i, P, P, P, P, P]
        L.kfo_transport.restype = i
        L.kfo_transport_perigee.argtypes = [i, P, P, P, i, P, d, d, d, d, i, i, P, P, P, P, P]
        L.kfo_transport_perigee.restype = i
        L.kfo_rkn_step.argtypes = [i, P, d, d, P, d, P, P]
        L.kfo_rkn_step.restype = d
        L.kfo_linear_smoother.argtypes = [i] + [P] * 11
        L.kfo_linear_smoother.restype = i
        L.kfo_linear_two_filter.argtypes = [i] + [P] * 7 + [d, P, P]
        L.kfo_linear_two_filter.restype = i
        L.kfo_ms_noise.argtypes = [i, P, P, P, i, P, d, P]
        L.kfo_ms_noise.restype = i
        L.kfo_field_at.argtypes = [i, P, d, P, P, P]
        L.kfo_field_at.restype = None
        L.kfo_set_field_map.argtypes = [P, P, P, P]
        L.kfo_set_field_map.restype = i
        L.kfo_set_surface_radius.argtypes = [i, P]
        L.kfo_set_surface_radius.restype = i
        L.kfo_version.restype = C.c_char_p
        L.kfo_count_update.argtypes = [P] * 5
        L.kfo_count_update.restype = i
        L.kfo_count_rts_step.argtypes = [P] * 8
        L.kfo_count_rts_step.restype = i
        L.kfo_count_transport.argtypes = [i, P, P, P, i, P, d, d, d, d, i, i, i, P, P, P, P]
        L.kfo_count_transport.restype = i
        L.kfo_count_rkn_step.argtypes = [i, P, d, d, P, d, P]
        L.kfo_count_rkn_step.restype = i
        L.kfo_count_units.argtypes = fit_args + [P, i, P, P]
        L.kfo_count_units.restype = i
        L.kfo_count_ms_noise.argtypes = [i, P, P, P, i, P, d, P]
        L.kfo_count_ms_noise.restype = i
        L.kfo_count_cov_transport.argtypes = [P, P, P, P]
        L.kfo_count_cov_transport.restype = i
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


_map_keep = []


def _use_field(field):
    """Hand a tabulated field (kind 2) to the library before a call."""
    if int(field.kind) != 2:
        return
    vals = np.ascontiguousarray(field.map_values, dtype=np.float64)
    nz, ny, nx, three = vals.shape
    assert three == 3
    n = np.array([nx, ny, nz], dtype=np.int32)
    o = np.asarray(field.map_origin, dtype=np.float64)
    h = np.asarray(field.map_spacing, dtype=np.float64)
    _map_keep[:] = [vals, n, o, h]
    if lib().kfo_set_field_map(_p(n), _p(o), _p(h), _p(vals)):
        raise ValueError("bad field map")


_radius_keep = []


def _use_surfaces(det):
    """Hand the detector's cylinder radii (if any) to the library before a call."""
    rad = getattr(det, "radius", None)
    if rad is None:
        _radius_keep[:] = []
        lib().kfo_set_surface_radius(0, None)
        return
    r = np.ascontiguousarray(rad, dtype=np.float64)
    _radius_keep[:] = [r]
    lib().kfo_set_surface_radius(int(r.size), _p(r))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


@dataclass
class FitResult:
    par: np.ndarray        # (6, H) smoothed
    cov: np.ndarray        # (21, H)
    tgt_par: np.ndarray    # (6, N)
    tgt_cov: np.ndarray    # (21, N)
    chi2: np.ndarray       # (N,)
    ndf: np.ndarray        # (N,)
    status: np.ndarray     # (N,) u8
    filt_par: np.ndarray | None = None
    filt_cov: np.ndarray | None = None
    pred_par: np.ndarray | None = None
    pred_cov: np.ndarray | None = None
    trials: np.ndarray | None = None


class _Args:
    """Common input marshalling for kfo_fit / kfo_fit_vjp / kfo_count_ops."""

    def __init__(self, ev, detector=None, ms=None, mass=None, tol=DEFAULT_TOL, land_tol=DEFAULT_LAND_TOL,
                 max_steps=DEFAULT_MAX_STEPS, loc=None, seed_par=None, align=None):
        det = detector if detector is not None else ev.detector
        _use_field(ev.field)
        _use_surfaces(det)
        self.keep = dict(
            off=_i32(ev.hit_offsets), sid=_i32(ev.surface_id), loc=_f64(ev.loc if loc is None else loc),
            cov=_f64(ev.cov), center=_f64(det.center), rot=_f64(det.rot), x0=_f64(det.x_over_X0),
            b0=_f64(ev.field.b0), seed=_f64(ev.seed_par if seed_par is None else seed_par),
            seed_cov=_f64(ev.seed_cov), align=None if align is None else _f64(align),
            stype=None if getattr(det, "stype", None) is None else _i32(det.stype))
        k = self.keep
        self.N = ev.n_tracks
        self.H = ev.n_hits
        self.S = det.center.shape[1]
        if k["align"] is not None and k["align"].shape != (6, self.S):
            raise ValueError("align must have shape (6, S)")
        self.args = [self.N, _p(k["off"]), _p(k["sid"]), _p(k["loc"]), _p(k["cov"]), self.S, _p(k["center"]),
                     _p(k["rot"]), _p(k["x0"]), _p(k["align"]), int(ev.field.kind), _p(k["b0"]), float(ev.field.a),
                     _p(k["seed"]), _p(k["seed_cov"]), int(ev.seed_surface),
                     int(ev.multiple_scattering if ms is None else ms), float(ev.mass if mass is None else mass),
                     float(tol), float(land_tol), int(max_steps)]


SMOOTHERS = {"rts": 0, "two_filter": 1}
DEFAULT_BWD_SCALE = 1e3


def fit(ev, n_threads: int = 0, extras: bool = False, smoother: str = "rts", bwd_scale: float = DEFAULT_BWD_SCALE,
        perigee=None, **kw) -> FitResult:
    """Filter + smoother for every track of `ev` (FP64).

    smoother: "rts" (stored Jacobians) or "two_filter" (a backward filter
    started from the last filtered covariance times `bwd_scale`, combined with
    the forward filter).  perigee: None (target = the seed surface) or a
    reference point (3,): the target result is given at the perigee of the
    line through it parallel to z, (d0, z0, phi, theta, q/p, t)."""
    a = _Args(ev, **kw)
    N, H = a.N, a.H
    out = FitResult(np.empty((6, H)), np.empty((21, H)), np.empty((6, N)), np.empty((21, N)),
                    np.empty(N), np.empty(N, np.int32), np.empty(N, np.uint8))
    if extras:
        out.filt_par, out.filt_cov = np.empty((6, H)), np.empty((21, H))
        out.pred_par, out.pred_cov = np.empty((6, H)), np.empty((21, H))
        out.trials = np.empty(H, np.int32)
    lib().kfo_fit(*a.args, _p(out.par), _p(out.cov), _p(out.tgt_par), _p(out.tgt_cov), _p(out.chi2),
                  _p(out.ndf), _p(out.status), _p(out.filt_par), _p(out.filt_cov), _p(out.pred_par),
                  _p(out.pred_cov), _p(out.trials), int(n_threads), SMOOTHERS[smoother], float(bwd_scale),
                  0 if perigee is None else 1, _p(None if perigee is None else _f64(perigee)), _p(a.keep["stype"]))
    return out


def fit_vjp(ev, g_chi2, g_par=None, g_tgt=None, n_threads: int = 0, **kw):
    """Exact VJP (forward-mode duals) -> (g_meas (2,H), g_align (6,S), g_seed (6,N)).

    g_align is the derivative with respect to each surface's alignment
    correction (dx, dy, dz, alpha, beta, gamma) at its given value (`align`
    keyword, zero if absent)."""
    a = _Args(ev, **kw)
    g_chi2 = _f64(g_chi2)
    g_par = None if g_par is None else _f64(g_par)
    g_tgt = None if g_tgt is None else _f64(g_tgt)
    g_meas = np.zeros((2, a.H))
    g_align = np.zeros((6, a.S))
    g_seed = np.zeros((6, a.N))
    lib().kfo_fit_vjp(*a.args, _p(g_chi2), _p(g_par), _p(g_tgt), _p(g_meas), _p(g_align), _p(g_seed),
                      int(n_threads), _p(a.keep["stype"]))
    return g_meas, g_align, g_seed


def count_ops(ev, **kw) -> np.ndarray:
    """(N, 5) non-trivial op counts per track: add/sub, mul, div, sqrt, transcendental."""
    a = _Args(ev, **kw)
    out = np.zeros((a.N, 5), dtype=np.int64)
    lib().kfo_count_ops(*a.args, _p(out), _p(a.keep["stype"]))
    return out


UNITS = ("seed check", "scatterer noise", "transport", "F (C+Q) F^T", "update", "chi2 sum", "RTS smoother")


def count_units(ev, t, **kw):
    """(status, units (7, 5), total (5,)) for track t: the counts of each unit of
    its fit (UNITS order; columns as count_ops) on the fit's own states, and the
    count of the whole fit."""
    a = _Args(ev, **kw)
    units = np.zeros((7, 5), dtype=np.int64)
    total = np.zeros(5, dtype=np.int64)
    st = lib().kfo_count_units(*a.args, _p(a.keep["stype"]), int(t), _p(units), _p(total))
    return st, units, total


def count_update(xp, Cp, m, V3):
    """(status, counts (5,)) of one gain-matrix update: xp (6,), Cp (6,6), m (2,), V3 = (v00, v01, v11)."""
    out = np.zeros(5, dtype=np.int64)
    st = lib().kfo_count_update(_p(_f64(xp)), _p(_f64(Cp)), _p(_f64(m)), _p(_f64(V3)), _p(out))
    return st, out


def count_rts_step(xf, Cf, F, xp1, Cp1, xs1, Cs1):
    """(status, counts (5,)) of one RTS step (6-vectors and 6x6 matrices)."""
    out = np.zeros(5, dtype=np.int64)
    st = lib().kfo_count_rts_step(*[_p(_f64(a)) for a in (xf, Cf, F, xp1, Cp1, xs1, Cs1)], _p(out))
    return st, out


def count_transport(det, field, sa, sb, x, mass=0.1056583755, tol=DEFAULT_TOL, land_tol=DEFAULT_LAND_TOL,
                    max_steps=DEFAULT_MAX_STEPS):
    """(status, counts (5,), trials) of one bound-to-bound transport."""
    _use_field(field)
    _use_surfaces(det)
    center, rot, x0 = _f64(det.center), _f64(det.rot), _f64(det.x_over_X0)
    b0, xi = _f64(field.b0), _f64(x)
    out = np.zeros(5, dtype=np.int64)
    tr = np.zeros(1, np.int32)
    stype = None if getattr(det, "stype", None) is None else _i32(det.stype)
    st = lib().kfo_count_transport(center.shape[1], _p(center), _p(rot), _p(x0), int(field.kind), _p(b0),
                                   float(field.a), float(mass), float(tol), float(land_tol), int(max_steps),
                                   int(sa), int(sb), _p(xi), _p(tr), _p(stype), _p(out))
    return st, out, int(tr[0])


def count_ms_noise(det, s, x, mass=0.1056583755):
    """counts (5,) of the thin-scatterer noise of surface s at bound state x."""
    center, rot, x0 = _f64(det.center), _f64(det.rot), _f64(det.x_over_X0)
    out = np.zeros(5, dtype=np.int64)
    lib().kfo_count_ms_noise(center.shape[1], _p(center), _p(rot), _p(x0), int(s), _p(_f64(x)), float(mass),
                             _p(out))
    return out


def count_cov_transport(F, C, Q):
    """counts (5,) of F (C + Q) F^T as the track fit forms it (6x6 each)."""
    out = np.zeros(5, dtype=np.int64)
    lib().kfo_count_cov_transport(_p(_f64(F)), _p(_f64(C)), _p(_f64(Q)), _p(out))
    return out


def count_rkn_step(field, F, h, mass=0.1056583755):
    """counts (5,) of one RKN step of the free state at fixed h."""
    _use_field(field)
    out = np.zeros(5, dtype=np.int64)
    lib().kfo_count_rkn_step(int(field.kind), _p(_f64(field.b0)), float(field.a), float(mass), _p(_f64(F)),
                             float(h), _p(out))
    return out


def transport(det, field, sa, sb, x, mass=0.1056583755, tol=DEFAULT_TOL, land_tol=DEFAULT_LAND_TOL,
              max_steps=DEFAULT_MAX_STEPS):
    """Bound state x on surface sa -> (status, x' on sb, F = dx'/dx (6,6), trials)."""
    _use_field(field)
    _use_surfaces(det)
    center, rot, x0 = _f64(det.center), _f64(det.rot), _f64(det.x_over_X0)
    b0 = _f64(field.b0)
    xi = _f64(x)
    xo = np.empty(6)
    F = np.empty((6, 6))
    tr = np.zeros(1, np.int32)
    stype = None if getattr(det, "stype", None) is None else _i32(det.stype)
    st = lib().kfo_transport(center.shape[1], _p(center), _p(rot), _p(x0), int(field.kind), _p(b0),
                             float(field.a), float(mass), float(tol), float(land_tol), int(max_steps),
                             int(sa), int(sb), _p(xi), _p(xo), _p(F), _p(tr), _p(stype))
    return st, xo, F, int(tr[0])


def transport_perigee(det, field, sa, c, x, mass=0.1056583755, tol=DEFAULT_TOL, land_tol=DEFAULT_LAND_TOL,
                      max_steps=DEFAULT_MAX_STEPS):
    """Bound state x on plane sa -> (status, perigee parameters (d0, z0, phi,
    theta, q/p, t) w.r.t. the line through c parallel to z, F (6,6), trials)."""
    _use_field(field)
    center, rot, x0 = _f64(det.center), _f64(det.rot), _f64(det.x_over_X0)
    b0, cc, xi = _f64(field.b0), _f64(c), _f64(x)
    xo = np.empty(6)
    F = np.empty((6, 6))
    tr = np.zeros(1, np.int32)
    st = lib().kfo_transport_perigee(center.shape[1], _p(center), _p(rot), _p(x0), int(field.kind), _p(b0),
                                     float(field.a), float(mass), float(tol), float(land_tol), int(max_steps),
                                     int(sa), _p(cc), _p(xi), _p(xo), _p(F), _p(tr))
    return st, xo, F, int(tr[0])


def rkn_step(field, F, h, mass=0.1056583755):
    """One RKN step of the free state (x,y,z,t,Tx,Ty,Tz,q/p) -> (F', D (8,8), err)."""
    _use_field(field)
    b0 = _f64(field.b0)
    Fi = _f64(F)
    Fn = np.empty(8)
    D = np.empty((8, 8))
    e = lib().kfo_rkn_step(int(field.kind), _p(b0), float(field.a), float(mass), _p(Fi), float(h), _p(Fn), _p(D))
    return Fn, D, e


def field_at(field, r):
    """(B (3,), dB/dr (3,3)) of the oracle's field at r."""
    _use_field(field)
    b0, rr = _f64(field.b0), _f64(r)
    B, dB = np.empty(3), np.empty((3, 3))
    lib().kfo_field_at(int(field.kind), _p(b0), float(field.a), _p(rr), _p(B), _p(dB))
    return B, dB


def linear_smoother(F, Q, m, V, x0, C0):
    """Linear-Gaussian filter + RTS with the oracle's update/RTS routines.

    F, Q: (n,6,6); m: (n,2); V: (n,3); x0: (6,); C0: (6,6).
    Returns xs (n+1,6), Cs (n+1,6,6), xf (n,6), Cf (n,6,6), chi2 (n,)."""
    n = F.shape[0]
    F, Q, m, V, x0, C0 = map(_f64, (F, Q, m, V, x0, C0))
    xs = np.empty((n + 1, 6)); Cs = np.empty((n + 1, 6, 6))
    xf = np.empty((n, 6)); Cf = np.empty((n, 6, 6)); chi2 = np.empty(n)
    st = lib().kfo_linear_smoother(n, _p(F), _p(Q), _p(m), _p(V), _p(x0), _p(C0), _p(xs), _p(Cs), _p(xf),
                                   _p(Cf), _p(chi2))
    if st:
        raise RuntimeError(f"linear smoother status {st}")
    return xs, Cs, xf, Cf, chi2


def linear_two_filter(F, G, Q, m, V, x0, C0, scale):
    """Linear-Gaussian filter + two-filter smoother with the oracle's routines.

    G: (n,6,6) backward transports (the inverses of F); the backward filter
    starts from the last filtered state with its covariance times `scale`.
    Returns xs (n+1,6), Cs (n+1,6,6)."""
    n = F.shape[0]
    F, G, Q, m, V, x0, C0 = map(_f64, (F, G, Q, m, V, x0, C0))
    xs = np.empty((n + 1, 6)); Cs = np.empty((n + 1, 6, 6))
    st = lib().kfo_linear_two_filter(n, _p(F), _p(G), _p(Q), _p(m), _p(V), _p(x0), _p(C0), float(scale), _p(xs),
                                     _p(Cs))
    if st:
        raise RuntimeError(f"linear two-filter status {st}")
    return xs, Cs


def ms_noise(det, s, x, mass=0.1056583755):
    """Process noise Q (6,6) of the thin scatterer on surface s for bound state x."""
    center, rot, x0 = _f64(det.center), _f64(det.rot), _f64(det.x_over_X0)
    xi = _f64(x)
    Q = np.empty((6, 6))
    lib().kfo_ms_noise(center.shape[1], _p(center), _p(rot), _p(x0), int(s), _p(xi), float(mass), _p(Q))
    return Q
