"""Seeded synthetic detector data for batched track fitting.

This module only *generates inputs*: telescope geometry, field description,
truth trajectories, smeared hits and smeared seeds.  It holds none of the
fitting arithmetic (no Runge-Kutta-Nystrom stepping, no transport Jacobian,
no Kalman update, no smoothing); both the CPU oracle and the HIP path take
what it produces as plain arrays.

Workload shapes follow the paper's telescope study (Sect. 5, "Performance
Evaluation"): planar surfaces perpendicular to the global x axis, 30 mm
apart, a 2 T field along z, single muons with pT uniform in 1-10 GeV, hits
smeared by Gaussian noise of 50 um in both local directions, starting
parameters smeared truth.  The paper's Fatras samples are not available;
this generator stands in for them.  Extensions (material with Highland
kicks, ragged hit patterns, misalignment, a solenoid-like field) are
parameters of the same recipe.

Conventions (shared *by definition* with the fitters, not by code):
  units mm, GeV, T, ns, rad;
  bound parameters (loc0, loc1, phi, theta, q/p, t);
  plane frame columns R = [u v n]; a plane normal to x has u = y, v = z, n = x;
  surface 0 is the seed/target plane x = 0, surfaces 1..P are the telescope;
  covariance packing: upper triangle, row-major, 21 entries.
"""
from __future__ import annotations

import os
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field as dc_field
import numpy as np

# physical constants of the generator (truth simulation only)
C_LIGHT = 299.792458          # mm / ns
K_B = 0.299792458e-3          # GeV / (T mm): curvature = K_B * B * q / p
M_MU = 0.1056583755           # GeV

SIGMA_HIT = 0.05              # mm (50 um, Sect. 5)
SEED_SIGMA = (0.1, 0.1, 2e-3, 2e-3, 0.05, 1.0)   # l0, l1 [mm], phi, theta, rel q/p, t [ns]

FIELD_UNIFORM = 0
FIELD_SOLENOID = 1
FIELD_MAP = 2

PACK_IDX = [(i, j) for i in range(6) for j in range(i, 6)]   # 21 packed entries


# ----------------------------------------------------------------------------
# containers (all arrays are component-major, i.e. [component][item])
# ----------------------------------------------------------------------------
@dataclass
class Detector:
    center: np.ndarray      # (3, S) f64
    rot: np.ndarray         # (9, S) f64, row-major 3x3 with columns u, v, n
    x_over_X0: np.ndarray   # (S,) f64
    stype: np.ndarray | None = None   # (S,) int32 surface types: 0 plane, 1 disc, 2 cylinder, 3 line
                                      # (None: all planes)
    radius: np.ndarray | None = None  # (S,) f64 cylinder radii (type 2), or None

    @property
    def n(self) -> int:
        return self.center.shape[1]


@dataclass
class Field:
    kind: int = FIELD_UNIFORM
    b0: tuple = (0.0, 0.0, 2.0)   # T
    a: float = 0.0                # 1/mm^2, solenoid shape parameter
    # FIELD_MAP: values at origin + (i, j, k) * spacing, array [nz][ny][nx][3] (T)
    map_values: np.ndarray | None = None
    map_origin: tuple = (0.0, 0.0, 0.0)
    map_spacing: tuple = (1.0, 1.0, 1.0)

    def is_zero(self) -> bool:
        return self.kind == FIELD_UNIFORM and not any(self.b0)


def analytic_field(field: Field, x, y, z):
    """B of a uniform or solenoid-like field at arrays x, y, z -> (Bx, By, Bz)."""
    if field.kind == FIELD_UNIFORM:
        return tuple(np.full(np.shape(x), float(b)) for b in field.b0)
    g = field.a * field.b0[2]
    return g * x * z, g * y * z, field.b0[2] * (1.0 - field.a * z * z)


def sample_field_map(field: Field, lo, hi, spacing) -> Field:
    """A tabulated field (FIELD_MAP) holding `field` sampled on the grid from
    lo to (at least) hi with the given spacing per axis."""
    lo = np.asarray(lo, float)
    sp = np.asarray(spacing, float)
    n = np.ceil((np.asarray(hi, float) - lo) / sp).astype(int) + 1
    ax = [lo[a] + sp[a] * np.arange(n[a]) for a in range(3)]
    Z, Y, X = np.meshgrid(ax[2], ax[1], ax[0], indexing="ij")
    B = np.stack(analytic_field(field, X, Y, Z), axis=-1)
    return Field(FIELD_MAP, tuple(field.b0), float(field.a), np.ascontiguousarray(B), tuple(lo), tuple(sp))


@dataclass
class Event:
    name: str
    detector: Detector            # geometry handed to the fitter
    field: Field
    hit_offsets: np.ndarray       # (N+1,) i32, CSR over tracks
    surface_id: np.ndarray        # (H,) i32
    loc: np.ndarray               # (2, H) f64
    cov: np.ndarray               # (3, H) f64: v00, v01, v11
    seed_par: np.ndarray          # (6, N) f64
    seed_cov: np.ndarray          # (21, N) f64 packed upper
    seed_surface: int
    truth_par0: np.ndarray        # (6, N) truth at the seed/target plane
    truth_hit: np.ndarray         # (6, H) truth bound params at each hit (before any kick)
    multiple_scattering: bool = False
    mass: float = M_MU
    detector_true: Detector | None = None
    align_true: np.ndarray | None = None   # (6, S) generator misalignment (dx,dy,dz,a,b,g)
    meta: dict = dc_field(default_factory=dict)

    @property
    def n_tracks(self) -> int:
        return self.hit_offsets.shape[0] - 1

    @property
    def n_hits(self) -> int:
        return int(self.hit_offsets[-1])

    def subset(self, idx) -> "Event":
        """Tracks `idx` (sorted, unique) as a new event with its own CSR."""
        idx = np.asarray(idx, dtype=np.int64)
        off = self.hit_offsets.astype(np.int64)
        cnt = off[idx + 1] - off[idx]
        new_off = np.zeros(len(idx) + 1, dtype=np.int64)
        np.cumsum(cnt, out=new_off[1:])
        hit_idx = np.concatenate([np.arange(off[i], off[i + 1]) for i in idx]) if len(idx) else np.zeros(0, np.int64)
        return Event(
            name=self.name + "[subset]", detector=self.detector, field=self.field,
            hit_offsets=new_off.astype(np.int32), surface_id=self.surface_id[hit_idx].copy(),
            loc=self.loc[:, hit_idx].copy(), cov=self.cov[:, hit_idx].copy(),
            seed_par=self.seed_par[:, idx].copy(), seed_cov=self.seed_cov[:, idx].copy(),
            seed_surface=self.seed_surface, truth_par0=self.truth_par0[:, idx].copy(),
            truth_hit=self.truth_hit[:, hit_idx].copy(),
            multiple_scattering=self.multiple_scattering, mass=self.mass,
            detector_true=self.detector_true, align_true=self.align_true, meta=dict(self.meta))


# ----------------------------------------------------------------------------
# geometry
# ----------------------------------------------------------------------------
R_PERP_X = np.array([[0.0, 0.0, 1.0],     # columns: u = (0,1,0), v = (0,0,1), n = (1,0,0)
                     [1.0, 0.0, 0.0],
                     [0.0, 1.0, 0.0]])


def rot_xyz(alpha, beta, gamma) -> np.ndarray:
    """Rx(alpha) @ Ry(beta) @ Rz(gamma) (right-handed, active)."""
    ca, sa, cb, sb, cg, sg = np.cos(alpha), np.sin(alpha), np.cos(beta), np.sin(beta), np.cos(gamma), np.sin(gamma)
    rx = np.array([[1, 0, 0], [0, ca, -sa], [0, sa, ca]])
    ry = np.array([[cb, 0, sb], [0, 1, 0], [-sb, 0, cb]])
    rz = np.array([[cg, -sg, 0], [sg, cg, 0], [0, 0, 1]])
    return rx @ ry @ rz


def telescope(n_planes: int, pitch: float = 30.0, x_over_X0: float = 0.0) -> Detector:
    """Seed plane at x = 0 (surface 0, no material) plus planes at x = pitch*i."""
    S = n_planes + 1
    center = np.zeros((3, S))
    center[0] = pitch * np.arange(S)
    rot = np.repeat(R_PERP_X.reshape(9, 1), S, axis=1)
    x0 = np.full(S, float(x_over_X0))
    x0[0] = 0.0
    return Detector(center, rot, x0)


def misalign(det: Detector, align: np.ndarray) -> Detector:
    """c <- c + (dx,dy,dz); R <- R @ Rx(a) @ Ry(b) @ Rz(g)  (local axes u, v, n)."""
    center = det.center + align[:3]
    rot = det.rot.copy()
    for s in range(det.n):
        R = det.rot[:, s].reshape(3, 3) @ rot_xyz(*align[3:, s])
        rot[:, s] = R.reshape(9)
    return Detector(center, rot, det.x_over_X0.copy(), None if det.stype is None else det.stype.copy())


# ----------------------------------------------------------------------------
# truth trajectories
# ----------------------------------------------------------------------------
def _sinc(a):
    return np.sinc(a / np.pi)


def helix_point(r0, phi0, theta, rho, s):
    """Exact helix for B along z: phi(s) = phi0 + rho*s, dz/ds = cos(theta).

    rho = dphi/ds = -(q/p) K_B Bz.  Cancellation-free chord form.
    """
    half = 0.5 * rho * s
    ch = np.sin(theta) * s * _sinc(half)
    x = r0[0] + ch * np.cos(phi0 + half)
    y = r0[1] + ch * np.sin(phi0 + half)
    z = r0[2] + s * np.cos(theta)
    return np.stack([x, y, z])


def helix_dir(phi0, theta, rho, s):
    ph = phi0 + rho * s
    st = np.sin(theta)
    return np.stack([st * np.cos(ph), st * np.sin(ph), np.cos(theta) * np.ones_like(ph)])


def helix_to_plane(r0, phi0, theta, rho, c, n, iters=30):
    """Path length s > 0 where the helix meets the plane n.(r - c) = 0 (Newton)."""
    T0 = helix_dir(phi0, theta, rho, np.zeros_like(phi0))
    nT = n[0] * T0[0] + n[1] * T0[1] + n[2] * T0[2]
    s = ((c[0] - r0[0]) * n[0] + (c[1] - r0[1]) * n[1] + (c[2] - r0[2]) * n[2]) / nT
    for _ in range(iters):
        r = helix_point(r0, phi0, theta, rho, s)
        T = helix_dir(phi0, theta, rho, s)
        g = n[0] * (r[0] - c[0]) + n[1] * (r[1] - c[1]) + n[2] * (r[2] - c[2])
        dg = n[0] * T[0] + n[1] * T[1] + n[2] * T[2]
        ds = g / dg
        s = s - ds
        if np.all(np.abs(ds) < 1e-13 * np.maximum(1.0, np.abs(s))):
            break
    return s


def helix_to_cylinder(r0, phi0, theta, rho, radius, iters=40):
    """Path length s > 0 where the helix (B along z) first reaches the cylinder
    x^2 + y^2 = radius^2 about the z axis, from inside (Newton on
    g = |r_xy|^2 - radius^2 from the straight-line crossing)."""
    T0 = helix_dir(phi0, theta, rho, np.zeros_like(phi0))
    a = T0[0] ** 2 + T0[1] ** 2
    b = r0[0] * T0[0] + r0[1] * T0[1]
    c = r0[0] ** 2 + r0[1] ** 2 - radius ** 2
    s = (-b + np.sqrt(b * b - a * c)) / a
    for _ in range(iters):
        r = helix_point(r0, phi0, theta, rho, s)
        T = helix_dir(phi0, theta, rho, s)
        g = r[0] ** 2 + r[1] ** 2 - radius ** 2
        dg = 2.0 * (r[0] * T[0] + r[1] * T[1])
        ds = g / dg
        s = s - ds
        if np.all(np.abs(ds) < 1e-13 * np.maximum(1.0, np.abs(s))):
            break
    return s


def helix_to_wire(r0, phi0, theta, rho, wx, wy, iters=40):
    """Path length s of the helix's closest approach to the wire through
    (wx, wy) parallel to z: Newton on g = (r - w)_xy . T_xy, from the
    straight-line closest approach."""
    T0 = helix_dir(phi0, theta, rho, np.zeros_like(phi0))
    s = -((r0[0] - wx) * T0[0] + (r0[1] - wy) * T0[1]) / (T0[0] ** 2 + T0[1] ** 2)
    st = np.sin(theta)
    for _ in range(iters):
        r = helix_point(r0, phi0, theta, rho, s)
        T = helix_dir(phi0, theta, rho, s)
        dx, dy = r[0] - wx, r[1] - wy
        g = dx * T[0] + dy * T[1]
        # dT_xy/ds = rho (-T_y, T_x)
        dg = T[0] ** 2 + T[1] ** 2 + rho * (-dx * T[1] + dy * T[0])
        ds = g / dg
        s = s - ds
        if np.all(np.abs(ds) < 1e-13 * np.maximum(1.0, np.abs(s))):
            break
    return s


def highland_theta0(p, mass, path_x0):
    """PDG Highland width of the projected scattering angle, unit charge."""
    beta = p / np.sqrt(p * p + mass * mass)
    return 0.0136 / (beta * p) * np.sqrt(path_x0) * (1.0 + 0.038 * np.log(path_x0 / (beta * beta)))


def _solenoid_B(x, y, z, b0z, a):
    return a * b0z * x * z, a * b0z * y * z, b0z * (1.0 - a * z * z)


def _rk4_x(state, lam, x, dx, b0z, a, mass):
    """One classical RK4 step in the global x coordinate (truth simulation)."""
    g = np.sqrt(1.0 + mass * mass * lam * lam) / C_LIGHT

    def f(xx, st):
        y, z, t, tx, ty, tz = st
        bx, by, bz = _solenoid_B(xx, y, z, b0z, a)
        inv = 1.0 / tx
        k = lam * K_B * inv
        return np.stack([ty * inv, tz * inv, g * inv,
                         k * (ty * bz - tz * by), k * (tz * bx - tx * bz), k * (tx * by - ty * bx)])

    k1 = f(x, state)
    k2 = f(x + 0.5 * dx, state + 0.5 * dx * k1)
    k3 = f(x + 0.5 * dx, state + 0.5 * dx * k2)
    k4 = f(x + dx, state + dx * k3)
    return state + (dx / 6.0) * (k1 + 2 * k2 + 2 * k3 + k4)


# ----------------------------------------------------------------------------
# hit selection (holes)
# ----------------------------------------------------------------------------
def choose_planes(n_hits, n_avail, u_hole, p_hole):
    """Walk planes 1..n_avail in order; each is a hole with probability p_hole
    unless the planes left equal the hits still needed.  Returns a boolean
    mask (N, P) with exactly n_hits True per row."""
    N, P = u_hole.shape
    mask = np.zeros((N, P), dtype=bool)
    taken = np.zeros(N, dtype=np.int64)
    for j in range(P):
        left = n_avail - j                      # planes j..n_avail-1 remaining
        need = n_hits - taken
        avail = j < n_avail
        forced = left <= need
        take = avail & (need > 0) & (forced | (u_hole[:, j] >= p_hole))
        mask[:, j] = take
        taken += take
    assert np.all(taken == n_hits)
    return mask


# ----------------------------------------------------------------------------
# event assembly
# ----------------------------------------------------------------------------
def _pack_diag(var):
    out = np.zeros((21,) + var.shape[1:])
    for k, (i, j) in enumerate(PACK_IDX):
        if i == j:
            out[k] = var[i]
    return out


def _make_seeds(rng_smear, truth0, f_inf):
    sig = np.array(SEED_SIGMA)[:, None] * np.ones_like(truth0)
    sig[4] = SEED_SIGMA[4] * np.abs(truth0[4])
    seed = truth0 + sig * rng_smear.T
    sig_c = sig.copy()
    sig_c[4] = SEED_SIGMA[4] * np.abs(seed[4])
    return seed, _pack_diag(sig_c ** 2) * f_inf


def _assemble(name, det, fld, mask, hit_state, rng_hits, seed_rand, truth0, ms, f_inf,
              det_true=None, align=None, meta=None):
    """mask (N,P) selects planes 1..P; hit_state (6, N, P) truth bound params."""
    N, P = mask.shape
    counts = mask.sum(axis=1)
    off = np.zeros(N + 1, dtype=np.int64)
    np.cumsum(counts, out=off[1:])
    tr, pl = np.nonzero(mask)                       # row-major: track order, plane order
    sid = (pl + 1).astype(np.int32)
    truth_hit = hit_state[:, tr, pl]
    loc = truth_hit[:2] + SIGMA_HIT * rng_hits[tr, pl].T
    cov = np.zeros((3, len(tr)))
    cov[0] = SIGMA_HIT ** 2
    cov[2] = SIGMA_HIT ** 2
    seed, seed_cov = _make_seeds(seed_rand, truth0, f_inf)
    return Event(name=name, detector=det, field=fld, hit_offsets=off.astype(np.int32),
                 surface_id=sid, loc=np.ascontiguousarray(loc), cov=cov,
                 seed_par=seed, seed_cov=seed_cov, seed_surface=0, truth_par0=truth0,
                 truth_hit=np.ascontiguousarray(truth_hit), multiple_scattering=ms,
                 detector_true=det_true, align_true=align, meta=meta or {})


def _kinematics(rng, N, pt_range=(1.0, 10.0), pt_log=False, phi_max=0.1, eta_max=0.2):
    q = rng.integers(0, 2, N) * 2.0 - 1.0
    if pt_log:
        pt = np.exp(rng.uniform(np.log(pt_range[0]), np.log(pt_range[1]), N))
    else:
        pt = rng.uniform(pt_range[0], pt_range[1], N)
    phi = rng.uniform(-phi_max, phi_max, N)
    eta = rng.uniform(-eta_max, eta_max, N)
    theta = 2.0 * np.arctan(np.exp(-eta))
    p = pt / np.sin(theta)
    return q, p, phi, theta


def _to_discs(ev):
    """Measure every hit surface as a disc: local polar coordinates (r, phi)
    about the surface centre in its (u, v) plane; r smeared by the hit
    resolution, phi by resolution / r (the same unit normal draws)."""
    unit = (ev.loc - ev.truth_hit[:2]) / SIGMA_HIT
    a, b = ev.truth_hit[0], ev.truth_hit[1]
    r = np.hypot(a, b)
    ph = np.arctan2(b, a)
    s_ph = SIGMA_HIT / r
    ev.truth_hit[0], ev.truth_hit[1] = r, ph
    ev.loc = np.ascontiguousarray(np.stack([r + SIGMA_HIT * unit[0],
                                            np.angle(np.exp(1j * (ph + s_ph * unit[1])))]))
    ev.cov = np.stack([np.full_like(r, SIGMA_HIT ** 2), np.zeros_like(r), s_ph ** 2])
    st = np.ones(ev.detector.n, dtype=np.int32)
    st[ev.seed_surface] = 0
    ev.detector.stype = st
    return ev


def telescope_event(n_tracks, seed, n_planes=10, bz=2.0, x_over_X0=0.0, ms=False,
                    ragged=None, p_hole=0.1, f_inf=1.0, misalign_sigma=None,
                    pt_range=(1.0, 10.0), phi_max=0.1, eta_max=0.2, name="telescope", pitch=30.0,
                    center_offset=None, discs=False):
    """Uniform field along z (or no field), planes normal to x, exact helices.

    ragged=(nmin, nmax): hit count per track uniform in [nmin, nmax], hole
    pattern from `choose_planes`; otherwise every plane is hit.
    misalign_sigma=(pos_mm, ang_rad): hits are simulated in a misaligned
    copy of the telescope while the fitter gets the nominal one.
    center_offset: shift of every measuring surface's centre within its plane;
    discs: measure in polar coordinates about that centre (`_to_discs`).
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    N, P = n_tracks, n_planes
    det = telescope(P, pitch=pitch, x_over_X0=x_over_X0 if ms else 0.0)
    if center_offset is not None:
        det.center[:, 1:] += np.asarray(center_offset, float)[:, None]
    fld = Field(FIELD_UNIFORM, (0.0, 0.0, float(bz)), 0.0)
    q, p, phi, theta = _kinematics(rng, N, pt_range, False, phi_max, eta_max)
    lam = q / p
    kicks = rng.standard_normal((N, P, 2)) if ms else None
    hit_rand = rng.standard_normal((N, P, 2))
    seed_rand = rng.standard_normal((N, 6))
    if ragged is not None:
        n_hits = rng.integers(ragged[0], ragged[1] + 1, N)
        u_hole = rng.random((N, P))
        mask = choose_planes(n_hits, np.full(N, P), u_hole, p_hole)
    else:
        mask = np.ones((N, P), dtype=bool)
    det_true, align = det, None
    if misalign_sigma is not None:
        align = np.zeros((6, P + 1))
        align[:3, 1:] = misalign_sigma[0] * rng.standard_normal((3, P))
        align[3:, 1:] = misalign_sigma[1] * rng.standard_normal((3, P))
        det_true = misalign(det, align)

    rho = -lam * K_B * bz
    g_t = np.sqrt(1.0 + M_MU ** 2 * lam ** 2) / C_LIGHT
    r = np.zeros((3, N))
    t = np.zeros(N)
    ph = phi.copy()
    th = theta.copy()
    hit_state = np.zeros((6, N, P))
    truth0 = np.stack([np.zeros(N), np.zeros(N), phi, theta, lam, np.zeros(N)])
    for j in range(P):
        s_id = j + 1
        R = det_true.rot[:, s_id].reshape(3, 3)
        c = det_true.center[:, s_id]
        u, v, n = R[:, 0], R[:, 1], R[:, 2]
        s = helix_to_plane(r, ph, th, rho, c, n)
        r = helix_point(r, ph, th, rho, s)
        ph = ph + rho * s
        t = t + s * g_t
        d = r - c[:, None]
        hit_state[:, :, j] = np.stack([u @ d, v @ d, ph, th, lam, t])
        if ms and det.x_over_X0[s_id] > 0:
            T = helix_dir(ph, th, rho, np.zeros(N))
            path = det.x_over_X0[s_id] / np.abs(n @ T)
            th0 = highland_theta0(p, M_MU, path)
            ph = ph + th0 * kicks[:, j, 0] / np.sin(th)
            th = th + th0 * kicks[:, j, 1]
    ev = _assemble(name, det, fld, mask, hit_state, hit_rand, seed_rand, truth0, ms, f_inf,
                   det_true=det_true, align=align,
                   meta=dict(seed=seed, n_planes=P, bz=bz, ragged=ragged))
    return _to_discs(ev) if discs else ev


def _integrate_slice(st, lam, xs, pitch, substeps, b0z, a, min_nT):
    """Truth states at every plane for the rows of `st`: (reach, states (6, M, P))."""
    M, P = st.shape[1], len(xs)
    alive = np.ones(M, dtype=bool)
    reach = np.zeros(M, dtype=np.int64)
    hs = np.zeros((6, M, P))
    for j in range(P):
        x0 = xs[j]
        h = pitch / substeps
        for k in range(substeps):
            st = _rk4_x(st, lam, x0 + k * h, h, b0z, a, M_MU)
            alive &= st[3] >= min_nT
            st[3] = np.where(alive, st[3], 1.0)   # keep dead rows finite
        reach += alive
        tn = np.sqrt(st[3] ** 2 + st[4] ** 2 + st[5] ** 2)
        hs[:, :, j] = np.stack([st[0], st[1], np.arctan2(st[4], st[3]),
                                np.arccos(st[5] / tn), lam, st[2]])
    return reach, hs


def _integrate_rows(st, lam, xs, pitch, substeps, b0z, a, min_nT, rows_per_task=32768):
    """_integrate_slice over row blocks on a thread pool (numpy releases the
    GIL in its array loops).  Every operation is elementwise per row, so the
    result does not depend on the split."""
    M = st.shape[1]
    starts = list(range(0, M, rows_per_task))
    workers = max(1, min(16, os.cpu_count() or 1, len(starts)))
    with ThreadPoolExecutor(max_workers=workers) as ex:
        parts = list(ex.map(lambda r0: _integrate_slice(st[:, r0:r0 + rows_per_task], lam[r0:r0 + rows_per_task], xs,
                                                        pitch, substeps, b0z, a, min_nT), starts))
    return np.concatenate([p[0] for p in parts]), np.concatenate([p[1] for p in parts], axis=1)


def solenoid_event(n_tracks, seed, n_planes=30, b0z=2.0, a=1e-7, nmin=8, p_hole=0.1,
                   min_nT=0.05, substeps=6, f_inf=1.0, pt_range=(0.5, 100.0), eta_max=2.5,
                   phi_max=0.1, name="solenoid"):
    """Solenoid-like field Bz = B0 (1 - a z^2), B_rho = a B0 rho z, planes
    normal to x; truth integrated with RK4 in x; planes are reachable while
    the direction keeps Tx >= min_nT; tracks with fewer than nmin reachable
    planes are redrawn."""
    rng = np.random.Generator(np.random.PCG64(seed))
    N, P = n_tracks, n_planes
    det = telescope(P)
    fld = Field(FIELD_SOLENOID, (0.0, 0.0, float(b0z)), float(a))
    chunks, got, drawn = [], 0, 0
    while got < N:
        M = max(1024, int((N - got) * 1.3))
        q, p, phi, theta = _kinematics(rng, M, pt_range, True, phi_max, eta_max)
        lam = q / p
        drawn += M
        st = np.stack([np.zeros(M), np.zeros(M), np.zeros(M),
                       np.sin(theta) * np.cos(phi), np.sin(theta) * np.sin(phi), np.cos(theta)])
        pitch = det.center[0, 1] - det.center[0, 0]
        reach, hs = _integrate_rows(st, lam, det.center[0, :P], pitch, substeps, b0z, a, min_nT)
        ok = reach >= nmin
        take = np.nonzero(ok)[0][: N - got]
        chunks.append((q[take], p[take], phi[take], theta[take], reach[take], hs[:, take]))
        got += len(take)
    cat = [np.concatenate([c[i] for c in chunks], axis=-1) for i in range(5)]
    q, p, phi, theta, reach = cat
    hs = np.concatenate([c[5] for c in chunks], axis=1)
    lam = q / p
    n_hits = rng.integers(nmin, np.minimum(P, reach) + 1)
    u_hole = rng.random((N, P))
    mask = choose_planes(n_hits, reach, u_hole, p_hole)
    hit_rand = rng.standard_normal((N, P, 2))
    seed_rand = rng.standard_normal((N, 6))
    truth0 = np.stack([np.zeros(N), np.zeros(N), phi, theta, lam, np.zeros(N)])
    return _assemble(name, det, fld, mask, hs, hit_rand, seed_rand, truth0, False, f_inf,
                     meta=dict(seed=seed, n_planes=P, drawn=drawn, redrawn=drawn - N))


# ----------------------------------------------------------------------------
# named workloads
# ----------------------------------------------------------------------------
CONFIG_SEEDS = {1: 1001, 2: 1002, 3: 1003, 4: 1004, 5: 1005, 6: 1005, 7: 1007, 8: 1008}


# barrel workload: five cylinders about the z axis, then five layers of
# straws (wires parallel to z), seed plane x = 0 through the axis
BARREL_RADII = (30.0, 60.0, 90.0, 120.0, 150.0)
STRAW_LAYERS_X = (180.0, 210.0, 240.0, 270.0, 300.0)
STRAW_PITCH = 10.0
STRAW_WIRES = 9                 # per layer, y = -40 .. 40 mm
SIGMA_STRAW = 0.1               # mm, drift-distance resolution


def barrel_detector(x_over_X0=0.0) -> Detector:
    """Seed plane x = 0 (surface 0), cylinders 1..5 (axis z through the origin,
    u = x, v = y, so the azimuth about the axis is measured from x), then the
    straws of layer l, wire i as surface 6 + 9 l + i (wire through
    (x_l, y_i, 0) along z)."""
    nc, nl, nw = len(BARREL_RADII), len(STRAW_LAYERS_X), STRAW_WIRES
    S = 1 + nc + nl * nw
    center = np.zeros((3, S))
    rot = np.zeros((9, S))
    rot[:, 0] = np.array([[0.0, 0.0, 1.0], [1.0, 0.0, 0.0], [0.0, 1.0, 0.0]]).reshape(9)   # u = y, v = z, n = x
    rot[:, 1:] = np.eye(3).reshape(9, 1)
    stype = np.zeros(S, dtype=np.int32)
    radius = np.zeros(S)
    stype[1:1 + nc] = 2
    radius[1:1 + nc] = BARREL_RADII
    y0 = -0.5 * STRAW_PITCH * (nw - 1)
    for l, xl in enumerate(STRAW_LAYERS_X):
        for i in range(nw):
            s = 1 + nc + l * nw + i
            center[:, s] = (xl, y0 + i * STRAW_PITCH, 0.0)
            stype[s] = 3
    x0 = np.full(S, float(x_over_X0))
    x0[0] = 0.0
    return Detector(center=center, rot=rot, x_over_X0=x0, stype=stype, radius=radius)


def barrel_event(n_tracks, seed, bz=2.0, x_over_X0=0.0, ms=False, f_inf=1.0, pt_range=(1.0, 10.0),
                 phi_max=0.1, eta_max=0.2, name="barrel"):
    """Exact helices (uniform Bz) through five cylinders (hits: position
    along the axis and azimuth, 50 um and 50 um / radius) and five straw
    layers (hit: the signed distance of closest approach to the nearest
    wire, 100 um; the position along the wire is not measured)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    N = n_tracks
    nc, nl, nw = len(BARREL_RADII), len(STRAW_LAYERS_X), STRAW_WIRES
    P = nc + nl
    det = barrel_detector(x_over_X0 if ms else 0.0)
    fld = Field(FIELD_UNIFORM, (0.0, 0.0, float(bz)), 0.0)
    q, p, phi, theta = _kinematics(rng, N, pt_range, False, phi_max, eta_max)
    lam = q / p
    kicks = rng.standard_normal((N, P, 2)) if ms else None
    hit_rand = rng.standard_normal((N, P, 2))
    seed_rand = rng.standard_normal((N, 6))
    rho = -lam * K_B * bz
    g_t = np.sqrt(1.0 + M_MU ** 2 * lam ** 2) / C_LIGHT
    r = np.zeros((3, N))
    t = np.zeros(N)
    ph = phi.copy()
    th = theta.copy()
    hit_state = np.zeros((6, N, P))
    sid = np.zeros((N, P), dtype=np.int32)
    sig = np.zeros((2, N, P))
    for j in range(P):
        if j < nc:
            s = helix_to_cylinder(r, ph, th, rho, BARREL_RADII[j])
            r = helix_point(r, ph, th, rho, s)
            ph = ph + rho * s
            t = t + s * g_t
            az = np.arctan2(r[1], r[0])
            hit_state[:, :, j] = np.stack([r[2], az, ph, th, lam, t])
            sid[:, j] = 1 + j
            sig[0, :, j] = SIGMA_HIT
            sig[1, :, j] = SIGMA_HIT / BARREL_RADII[j]
            normal = np.stack([np.cos(az), np.sin(az), np.zeros(N)])
        else:
            l = j - nc
            xl = STRAW_LAYERS_X[l]
            cx = np.array([xl, 0.0, 0.0])
            sx = helix_to_plane(r, ph, th, rho, cx, np.array([1.0, 0.0, 0.0]))
            yc = helix_point(r, ph, th, rho, sx)[1]
            y0 = -0.5 * STRAW_PITCH * (nw - 1)
            wi = np.clip(np.rint((yc - y0) / STRAW_PITCH), 0, nw - 1).astype(np.int64)
            wy = y0 + wi * STRAW_PITCH
            s = helix_to_wire(r, ph, th, rho, xl, wy)
            r = helix_point(r, ph, th, rho, s)
            ph = ph + rho * s
            t = t + s * g_t
            T = helix_dir(ph, th, rho, np.zeros(N))
            txy = np.hypot(T[0], T[1])
            e = np.stack([-T[1] / txy, T[0] / txy, np.zeros(N)])        # (z x T)/|z x T|
            d = r - np.stack([np.full(N, xl), wy, np.zeros(N)])
            hit_state[:, :, j] = np.stack([(e * d).sum(axis=0), d[2], ph, th, lam, t])
            sid[:, j] = 1 + nc + l * nw + wi
            sig[0, :, j] = SIGMA_STRAW
            normal = None
        if ms and det.x_over_X0[sid[0, j]] > 0:
            T = helix_dir(ph, th, rho, np.zeros(N))
            if normal is not None:
                cosi = np.abs((normal * T).sum(axis=0))
            else:
                cosi = np.hypot(T[0], T[1])                       # |z x T|: across the wire
            path = det.x_over_X0[sid[0, j]] / cosi
            th0 = highland_theta0(p, M_MU, path)
            ph = ph + th0 * kicks[:, j, 0] / np.sin(th)
            th = th + th0 * kicks[:, j, 1]
    off = np.arange(N + 1, dtype=np.int64) * P
    truth_hit = hit_state.reshape(6, N * P)
    loc = truth_hit[:2] + sig.reshape(2, N * P) * hit_rand.reshape(N * P, 2).T
    straw = np.zeros((N, P), dtype=bool)
    straw[:, nc:] = True
    straw = straw.reshape(-1)
    loc[1, straw] = 0.0                                            # not measured on a straw
    loc[1, ~straw] = np.angle(np.exp(1j * loc[1, ~straw]))
    cov = np.zeros((3, N * P))
    cov[0] = sig[0].reshape(-1) ** 2
    cov[2] = sig[1].reshape(-1) ** 2                                # 0 on straws (unread)
    truth0 = np.stack([np.zeros(N), np.zeros(N), phi, theta, lam, np.zeros(N)])
    seed_par, seed_cov = _make_seeds(seed_rand, truth0, f_inf)
    return Event(name=name, detector=det, field=fld, hit_offsets=off.astype(np.int32),
                 surface_id=sid.reshape(-1), loc=np.ascontiguousarray(loc), cov=cov,
                 seed_par=seed_par, seed_cov=seed_cov, seed_surface=0, truth_par0=truth0,
                 truth_hit=np.ascontiguousarray(truth_hit), multiple_scattering=ms,
                 meta=dict(seed=seed, bz=bz))


def make_config(cfg: int, n_tracks: int | None = None, seed: int | None = None, **kw) -> Event:
    """The five workloads:
    1: 100 tracks, 10 planes, 2 T, no material.
    2: 1e5 tracks, 10 planes, 2 T, 0.5 % X0 per plane with Highland kicks.
    3: 1e5 tracks, 30 planes, 2 T, ragged 5-30 hits with holes (p = 0.1).
    4: 1e5 tracks, 10 planes, 2 T, misaligned truth (10 um, 0.1 mrad).
    5: 1e6 tracks, 30 planes, solenoid field, pT log-uniform 0.5-100 GeV,
       |eta| < 2.5, ragged 8-30 hits over reachable planes.
    6: the tracks of 5, fitted with the field given as a map: the solenoid
       sampled every 25 mm over x -50..950, y -1000..1000, z -6000..6000 mm
       (41 x 81 x 481 points, 38 MB).
    7: C2 measured on discs: every plane's centre moved to y = +100 mm and
       the hits given in polar coordinates (r, phi) about it (phi straddles
       +-pi), 50 um in r and 50 um / r in phi.
    8: 1e5 tracks (C1 kinematics) through a barrel: five cylinders about the
       z axis (radius 30..150 mm; hits: z and the azimuth) and five layers of
       straws (wires parallel to z at x = 180..300 mm, 10 mm apart; hit: the
       signed drift distance, 100 um), 2 T, 0.2 % X0 per layer with Highland
       kicks.
    """
    seed = CONFIG_SEEDS[cfg] if seed is None else seed
    if cfg == 1:
        return telescope_event(n_tracks or 100, seed, name="C1", **kw)
    if cfg == 2:
        return telescope_event(n_tracks or 100_000, seed, x_over_X0=0.005, ms=True, name="C2", **kw)
    if cfg == 3:
        return telescope_event(n_tracks or 100_000, seed, n_planes=30, ragged=(5, 30), name="C3", **kw)
    if cfg == 4:
        return telescope_event(n_tracks or 100_000, seed, misalign_sigma=(0.01, 1e-4), name="C4", **kw)
    if cfg == 5:
        return solenoid_event(n_tracks or 1_000_000, seed, name="C5", **kw)
    if cfg == 7:
        return telescope_event(n_tracks or 100_000, seed, x_over_X0=0.005, ms=True, center_offset=(0.0, 100.0, 0.0),
                               discs=True, name="C7", **kw)
    if cfg == 8:
        return barrel_event(n_tracks or 100_000, seed, x_over_X0=0.002, ms=True, name="C8", **kw)
    if cfg == 6:
        ev = solenoid_event(n_tracks or 1_000_000, seed, name="C6", **kw)
        ev.field = sample_field_map(ev.field, (-50.0, -1000.0, -6000.0), (950.0, 1000.0, 6000.0), (25.0, 25.0, 25.0))
        return ev
    raise ValueError(f"unknown config {cfg}")
