"""Python binding of libkfmi.so (argument marshalling only).

Every step of the fit runs in the HIP library.  PyTorch provides device
memory and the current stream.  If the library is not built or cannot be
loaded, every call raises: there is no CPU fallback.

Names mirror include/kf.h: kf_fit_tracks, kf_fit_tracks_vjp, kf_workspace_bytes,
kf_vjp_workspace_bytes, kf_status_string, kf_version.  TrackFit is the
torch.autograd.Function over the fit: its backward is kf_fit_tracks_vjp.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass, replace

import numpy as np
import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libkfmi.so")

# ---- constants (include/kf.h) ----
KF_OK, KF_E_NULL, KF_E_SIZE, KF_E_ENUM, KF_E_WS, KF_E_HIP, KF_E_VALUE = 0, -1, -2, -3, -4, -5, -6
KF_E_SCRATCH = -7
KF_NOALLOC_SCRATCH_BYTES = 64 << 20
KF_ST_OK, KF_ST_NO_INTERSECT, KF_ST_STEP_CAP, KF_ST_NOT_SPD, KF_ST_BAD_INPUT, KF_ST_TOO_FEW = range(6)
KF_FIELD_UNIFORM, KF_FIELD_SOLENOID, KF_FIELD_MAP = 0, 1, 2
KF_PREC_FP64, KF_PREC_MIXED = 0, 1
KF_SCHED_AUTO, KF_SCHED_DIRECT, KF_SCHED_SORTED = 0, 1, 2
KF_JAC_STORE, KF_JAC_RECOMPUTE = 0, 1
KF_OUT_AUTO, KF_OUT_STAGED, KF_OUT_SLOTS = 0, 1, 2
KF_SMOOTHER_RTS, KF_SMOOTHER_TWO_FILTER = 0, 1
KF_TARGET_SEED_SURFACE, KF_TARGET_PERIGEE = 0, 1
KF_SURF_PLANE, KF_SURF_DISC, KF_SURF_CYLINDER, KF_SURF_LINE = 0, 1, 2, 3
KF_MAX_SURFACES = 512
KF_MAX_HITS = 64


class kf_surfaces(C.Structure):
    _fields_ = [("n", C.c_int32), ("center", C.c_void_p), ("rot", C.c_void_p), ("x_over_X0", C.c_void_p),
                ("align", C.c_void_p), ("type", C.c_void_p), ("radius", C.c_void_p)]


class kf_field(C.Structure):
    _fields_ = [("kind", C.c_int32), ("b0", C.c_double * 3), ("a", C.c_double), ("map_n", C.c_int32 * 3),
                ("map_origin", C.c_double * 3), ("map_spacing", C.c_double * 3), ("map", C.c_void_p)]


class kf_measurements(C.Structure):
    _fields_ = [("n_tracks", C.c_int32), ("max_hits", C.c_int32), ("n_hits", C.c_int64),
                ("hit_offsets", C.c_void_p), ("surface_id", C.c_void_p), ("loc", C.c_void_p),
                ("cov", C.c_void_p)]


class kf_seeds(C.Structure):
    _fields_ = [("par", C.c_void_p), ("cov", C.c_void_p), ("surface_id", C.c_int32)]


class kf_config(C.Structure):
    _fields_ = [("precision", C.c_int32), ("multiple_scattering", C.c_int32), ("mass", C.c_double),
                ("rk_tol", C.c_double), ("land_tol", C.c_double), ("max_steps", C.c_int32),
                ("schedule", C.c_int32), ("block", C.c_int32), ("waves_per_cu", C.c_int32),
                ("occupancy", C.c_int32), ("split_smoother", C.c_int32), ("jacobians", C.c_int32),
                ("smoother", C.c_int32), ("bwd_scale", C.c_double), ("target", C.c_int32),
                ("perigee", C.c_double * 3), ("output", C.c_int32)]


class kf_outputs(C.Structure):
    _fields_ = [("par", C.c_void_p), ("cov", C.c_void_p), ("tgt_par", C.c_void_p), ("tgt_cov", C.c_void_p),
                ("chi2", C.c_void_p), ("ndf", C.c_void_p), ("status", C.c_void_p), ("trials", C.c_void_p),
                ("filt_par", C.c_void_p), ("filt_cov", C.c_void_p)]


class kf_cotangents(C.Structure):
    _fields_ = [("chi2", C.c_void_p), ("par", C.c_void_p), ("tgt_par", C.c_void_p)]


class kf_gradients(C.Structure):
    _fields_ = [("meas", C.c_void_p), ("align", C.c_void_p), ("seed", C.c_void_p), ("status", C.c_void_p)]


# every symbol include/kf.h declares
EXPORTS = ("kf_version", "kf_status_string", "kf_workspace_bytes", "kf_fit_tracks", "kf_plan_create",
           "kf_plan_launch", "kf_plan_destroy", "kf_autotune", "kf_vjp_workspace_bytes", "kf_fit_tracks_vjp",
           "kf_staged_workspace_bytes", "kf_fit_tracks_staged", "kf_fit_tracks_noalloc")

_lib = None


def lib():
    """Load libkfmi.so (after torch, so the HIP runtime torch loaded is reused)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built (run __graft_entry__.build() or "
                               "python -m paper_2105_01796_amd.build)")
        L = C.CDLL(LIB_PATH)
        P = C.c_void_p
        L.kf_version.restype = C.c_char_p
        L.kf_version.argtypes = []
        L.kf_status_string.restype = C.c_char_p
        L.kf_status_string.argtypes = [C.c_int]
        L.kf_workspace_bytes.restype = C.c_size_t
        L.kf_workspace_bytes.argtypes = [P, P, C.c_int32]
        L.kf_fit_tracks.restype = C.c_int
        L.kf_fit_tracks.argtypes = [P, P, P, P, P, P, P, C.c_size_t, P]
        L.kf_plan_create.restype = C.c_int
        L.kf_plan_create.argtypes = [P, P, P, P, P, P, P, C.c_size_t, C.POINTER(C.c_void_p)]
        L.kf_plan_launch.restype = C.c_int
        L.kf_plan_launch.argtypes = [P, P]
        L.kf_plan_destroy.restype = None
        L.kf_plan_destroy.argtypes = [P]
        L.kf_autotune.restype = C.c_int
        L.kf_autotune.argtypes = [P, P, P, P, P, P, P, C.c_size_t, P, P, C.POINTER(C.c_float)]
        L.kf_vjp_workspace_bytes.restype = C.c_size_t
        L.kf_vjp_workspace_bytes.argtypes = [P, P, C.c_int32]
        L.kf_fit_tracks_vjp.restype = C.c_int
        L.kf_fit_tracks_vjp.argtypes = [P, P, P, P, P, P, P, P, C.c_size_t, P]
        L.kf_staged_workspace_bytes.restype = C.c_size_t
        L.kf_staged_workspace_bytes.argtypes = [P, P, C.c_int32, C.c_int32, C.c_int32]
        L.kf_fit_tracks_staged.restype = C.c_int
        L.kf_fit_tracks_staged.argtypes = [P, P, P, P, P, P, P, C.c_size_t, C.c_int32, P, C.c_int32]
        L.kf_fit_tracks_noalloc.restype = C.c_int
        L.kf_fit_tracks_noalloc.argtypes = [P, P, P, P, P, P, P]
        _lib = L
    return _lib


def kf_version() -> str:
    return lib().kf_version().decode()


def kf_status_string(code: int) -> str:
    return lib().kf_status_string(int(code)).decode()


class KFError(RuntimeError):
    def __init__(self, code, what="kf_fit_tracks"):
        super().__init__(f"{what} failed: {code} ({kf_status_string(code)})")
        self.code = code


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _dev(t, dtype, device):
    return torch.as_tensor(t).to(device=device, dtype=dtype).contiguous()


@dataclass
class Batch:
    """Device-resident inputs of one fit (component-major, as in kf.h)."""
    hit_offsets: torch.Tensor     # (N+1,) i32
    surface_id: torch.Tensor      # (H,) i32
    loc: torch.Tensor             # (2, H) f64
    cov: torch.Tensor             # (3, H) f64
    seed_par: torch.Tensor        # (6, N) f64
    seed_cov: torch.Tensor        # (21, N) f64
    seed_surface: int
    center: torch.Tensor          # (3, S) f64
    rot: torch.Tensor             # (9, S) f64
    x_over_X0: torch.Tensor       # (S,) f64
    field_kind: int = KF_FIELD_UNIFORM
    b0: tuple = (0.0, 0.0, 2.0)
    field_a: float = 0.0
    multiple_scattering: bool = False
    mass: float = 0.1056583755
    max_hits: int = 0             # 0: computed from hit_offsets
    align: torch.Tensor | None = None   # (6, S) f64 alignment corrections, or None
    surface_type: torch.Tensor | None = None   # (S,) int32 KF_SURF_* per surface, or None (all planes)
    surface_radius: torch.Tensor | None = None   # (S,) f64 cylinder radii: set to fit cylinders and lines
    field_map: torch.Tensor | None = None   # KF_FIELD_MAP: (nz, ny, nx, 3) f64 on the device
    map_origin: tuple = (0.0, 0.0, 0.0)
    map_spacing: tuple = (1.0, 1.0, 1.0)

    @property
    def n_tracks(self) -> int:
        return self.hit_offsets.numel() - 1

    @property
    def n_hits(self) -> int:
        return self.surface_id.numel()

    @classmethod
    def staged_from_event(cls, ev, device="cuda", detector=None, align=None) -> "Batch":
        """Measurements and seeds in pinned host memory, the detector on the
        device: the input of kf_fit_tracks_staged."""
        b = cls.from_event(ev, device=device, detector=detector, align=align)
        for name in ("hit_offsets", "surface_id", "loc", "cov", "seed_par", "seed_cov"):
            setattr(b, name, getattr(b, name).cpu().pin_memory())
        return b

    @classmethod
    def from_event(cls, ev, device="cuda", detector=None, align=None) -> "Batch":
        det = detector if detector is not None else ev.detector
        f64, i32 = torch.float64, torch.int32
        counts = (ev.hit_offsets[1:] - ev.hit_offsets[:-1]) if ev.n_tracks else []
        return cls(hit_offsets=_dev(ev.hit_offsets, i32, device), surface_id=_dev(ev.surface_id, i32, device),
                   loc=_dev(ev.loc, f64, device), cov=_dev(ev.cov, f64, device),
                   seed_par=_dev(ev.seed_par, f64, device), seed_cov=_dev(ev.seed_cov, f64, device),
                   seed_surface=int(ev.seed_surface), center=_dev(det.center, f64, device),
                   rot=_dev(det.rot, f64, device), x_over_X0=_dev(det.x_over_X0, f64, device),
                   field_kind=int(ev.field.kind), b0=tuple(float(b) for b in ev.field.b0),
                   field_a=float(ev.field.a), multiple_scattering=bool(ev.multiple_scattering),
                   mass=float(ev.mass), max_hits=int(max(counts)) if len(counts) else 1,
                   align=None if align is None else _dev(align, f64, device),
                   surface_type=None if getattr(det, "stype", None) is None else _dev(det.stype, i32, device),
                   surface_radius=_radius(det, device),
                   field_map=None if int(ev.field.kind) != KF_FIELD_MAP else _dev(ev.field.map_values, f64, device),
                   map_origin=tuple(float(v) for v in getattr(ev.field, "map_origin", (0.0, 0.0, 0.0))),
                   map_spacing=tuple(float(v) for v in getattr(ev.field, "map_spacing", (1.0, 1.0, 1.0))))


def _radius(det, device):
    """The detector's cylinder radii on the device when it has cylinders or
    lines (zeros where it gives none), else None."""
    st = getattr(det, "stype", None)
    rad = getattr(det, "radius", None)
    if st is None or not (np.asarray(st) >= KF_SURF_CYLINDER).any():
        return None
    if rad is None:
        rad = np.zeros(len(st))
    return _dev(rad, torch.float64, device)


@dataclass
class Fit:
    par: torch.Tensor
    cov: torch.Tensor
    tgt_par: torch.Tensor
    tgt_cov: torch.Tensor
    chi2: torch.Tensor
    ndf: torch.Tensor
    status: torch.Tensor
    trials: torch.Tensor | None = None
    filt_par: torch.Tensor | None = None
    filt_cov: torch.Tensor | None = None


@dataclass
class Options:
    precision: int = KF_PREC_FP64
    rk_tol: float = 1e-4
    land_tol: float = 1e-6
    max_steps: int = 1000
    schedule: int = KF_SCHED_AUTO
    block: int = 0
    waves_per_cu: int = 0
    occupancy: int = 0
    split_smoother: int = 0
    jacobians: int = 0          # KF_JAC_STORE / KF_JAC_RECOMPUTE
    smoother: int = 0           # KF_SMOOTHER_RTS / KF_SMOOTHER_TWO_FILTER
    bwd_scale: float = 0.0      # two-filter: backward start covariance inflation (0 = 1e3)
    target: int = 0             # KF_TARGET_SEED_SURFACE / KF_TARGET_PERIGEE
    perigee: tuple = (0.0, 0.0, 0.0)   # perigee target: a point of the line parallel to z (mm)
    output: int = 0             # KF_OUT_AUTO / KF_OUT_STAGED / KF_OUT_SLOTS (RTS smoother's output path)


def _max_hits(b: Batch) -> int:
    max_hits = b.max_hits
    if max_hits <= 0:
        max_hits = int((b.hit_offsets[1:] - b.hit_offsets[:-1]).max().item()) if b.n_tracks else 1
    return max(1, min(max_hits, KF_MAX_HITS))


def _structs(b: Batch, opt: Options):
    """kf_config, kf_surfaces, kf_field, kf_measurements, kf_seeds for a batch."""
    cfg = kf_config(opt.precision, int(b.multiple_scattering), b.mass, opt.rk_tol, opt.land_tol, opt.max_steps,
                    opt.schedule, opt.block, opt.waves_per_cu, opt.occupancy, opt.split_smoother, opt.jacobians,
                    opt.smoother, opt.bwd_scale, opt.target, (C.c_double * 3)(*opt.perigee), opt.output)
    if b.align is not None and tuple(b.align.shape) != (6, b.center.shape[1]):
        raise ValueError("align must have shape (6, S)")
    surf = kf_surfaces(b.center.shape[1], _ptr(b.center), _ptr(b.rot), _ptr(b.x_over_X0), _ptr(b.align),
                       _ptr(b.surface_type), _ptr(b.surface_radius))
    if b.field_kind == KF_FIELD_MAP:
        if b.field_map is None or b.field_map.dim() != 4 or b.field_map.shape[3] != 3:
            raise ValueError("field_map must have shape (nz, ny, nx, 3)")
        nz, ny, nx, _ = b.field_map.shape
        field = kf_field(b.field_kind, (C.c_double * 3)(*b.b0), b.field_a, (C.c_int32 * 3)(nx, ny, nz),
                         (C.c_double * 3)(*b.map_origin), (C.c_double * 3)(*b.map_spacing), _ptr(b.field_map))
    else:
        field = kf_field(b.field_kind, (C.c_double * 3)(*b.b0), b.field_a)
    meas = kf_measurements(b.n_tracks, _max_hits(b), b.n_hits, _ptr(b.hit_offsets), _ptr(b.surface_id),
                           _ptr(b.loc), _ptr(b.cov))
    seeds = kf_seeds(_ptr(b.seed_par), _ptr(b.seed_cov), b.seed_surface)
    return cfg, surf, field, meas, seeds


class Plan:
    """Marshalled arguments + workspace for repeated fits of one batch shape.

    Holds the ctypes structs so a timed loop only pays the library call."""

    def __init__(self, b: Batch, opt: Options | None = None, extras: bool = False, out: Fit | None = None):
        opt = opt or Options()
        dev = b.loc.device
        N, H = b.n_tracks, b.n_hits
        self.batch, self.opt = b, opt
        self.cfg, self.surf, self.field, self.meas, self.seeds = _structs(b, opt)
        f64 = dict(dtype=torch.float64, device=dev)
        if out is None:
            out = Fit(torch.empty((6, H), **f64), torch.empty((21, H), **f64), torch.empty((6, N), **f64),
                      torch.empty((21, N), **f64), torch.empty(N, **f64),
                      torch.empty(N, dtype=torch.int32, device=dev), torch.empty(N, dtype=torch.uint8, device=dev))
            if extras:
                out.trials = torch.empty(H, dtype=torch.int32, device=dev)
                out.filt_par = torch.empty((6, H), **f64)
                out.filt_cov = torch.empty((21, H), **f64)
        self.out = out
        self.outs = kf_outputs(_ptr(out.par), _ptr(out.cov), _ptr(out.tgt_par), _ptr(out.tgt_cov), _ptr(out.chi2),
                               _ptr(out.ndf), _ptr(out.status), _ptr(out.trials), _ptr(out.filt_par),
                               _ptr(out.filt_cov))
        nbytes = lib().kf_workspace_bytes(C.byref(self.cfg), C.byref(self.meas), self.surf.n)
        if nbytes == 0:
            raise KFError(KF_E_SIZE)
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
        self.ws_bytes = nbytes

        self.graph = None

    def _args(self):
        return (C.byref(self.cfg), C.byref(self.surf), C.byref(self.field), C.byref(self.meas),
                C.byref(self.seeds), C.byref(self.outs), _ptr(self.ws), self.ws_bytes)

    def capture(self) -> "Plan":
        """Record the whole fit once into a HIP graph (kf_plan_create); run()
        then replays it with one launch."""
        if self.graph is None:
            h = C.c_void_p()
            rc = lib().kf_plan_create(*self._args(), C.byref(h))
            if rc != KF_OK:
                raise KFError(rc)
            self.graph = h
        return self

    def autotune(self, stream=None) -> tuple:
        """Time every launch shape on this batch (kf_autotune); the winner
        becomes this plan's configuration.  Returns (Options, ms per fit)."""
        if stream is None:
            stream = torch.cuda.current_stream(self.batch.loc.device)
        best = kf_config()
        ms = C.c_float()
        rc = lib().kf_autotune(*self._args(), C.c_void_p(stream.cuda_stream), C.byref(best), C.byref(ms))
        if rc != KF_OK:
            raise KFError(rc)
        self.cfg = best
        self.release()
        o = Options(best.precision, best.rk_tol, best.land_tol, best.max_steps, best.schedule, best.block,
                    best.waves_per_cu, best.occupancy, best.split_smoother, best.jacobians, best.smoother,
                    best.bwd_scale, best.target, tuple(best.perigee), best.output)
        return o, ms.value

    def release(self):
        if self.graph is not None:
            lib().kf_plan_destroy(self.graph)
            self.graph = None

    def __del__(self):
        try:
            self.release()
        except Exception:
            pass

    def run(self, stream=None) -> Fit:
        if stream is None:
            stream = torch.cuda.current_stream(self.batch.loc.device)
        s = C.c_void_p(stream.cuda_stream)
        if self.graph is not None:
            rc = lib().kf_plan_launch(self.graph, s)
        else:
            rc = lib().kf_fit_tracks(*self._args(), s)
        if rc != KF_OK:
            raise KFError(rc)
        return self.out


def kf_fit_tracks(batch: Batch, opt: Options | None = None, extras: bool = False) -> Fit:
    """Filter + RTS smoother of every track in `batch` on its device (async on
    the current stream)."""
    return Plan(batch, opt, extras).run()


def kf_fit_tracks_noalloc(batch: Batch, out: Fit, opt: Options | None = None, stream=None) -> Fit:
    """The fit of kf_fit_tracks with the library's static scratch as its
    workspace (no device allocation by the library; the caller provides the
    outputs `out`).  Raises KFError(KF_E_SCRATCH) for batches too large for
    KF_NOALLOC_SCRATCH_BYTES."""
    opt = opt or Options()
    cfg, surf, field, meas, seeds = _structs(batch, opt)
    outs = kf_outputs(_ptr(out.par), _ptr(out.cov), _ptr(out.tgt_par), _ptr(out.tgt_cov), _ptr(out.chi2),
                      _ptr(out.ndf), _ptr(out.status), _ptr(out.trials), _ptr(out.filt_par), _ptr(out.filt_cov))
    if stream is None:
        stream = torch.cuda.current_stream(batch.loc.device)
    rc = lib().kf_fit_tracks_noalloc(C.byref(cfg), C.byref(surf), C.byref(field), C.byref(meas), C.byref(seeds),
                                     C.byref(outs), C.c_void_p(stream.cuda_stream))
    if rc != KF_OK:
        raise KFError(rc, "kf_fit_tracks_noalloc")
    return out


# ---------------------------------------------------------------------------
# adjoint
# ---------------------------------------------------------------------------
@dataclass
class Grad:
    meas: torch.Tensor                # (2, H) dL/d(loc0, loc1)
    align: torch.Tensor | None        # (6, S) dL/d(alignment correction)
    seed: torch.Tensor | None         # (6, N) dL/d(starting parameters)
    status: torch.Tensor              # (N,) u8 status of the recomputed fit


class StagedPlan:
    """kf_fit_tracks_staged for a batch from Batch.staged_from_event: pinned
    host inputs and outputs, n_chunks chunks pipelined over n_streams streams
    (default priority) so that copies overlap the fit."""

    def __init__(self, b: Batch, opt: Options | None = None, n_chunks: int = 8, n_streams: int = 2):
        opt = opt or Options()
        dev = b.center.device
        N, H = b.n_tracks, b.n_hits
        self.batch, self.opt, self.device = b, opt, dev
        self.cfg, self.surf, self.field, self.meas, self.seeds = _structs(b, opt)
        pin = dict(pin_memory=True)
        out = Fit(torch.empty((6, H), dtype=torch.float64, **pin), torch.empty((21, H), dtype=torch.float64, **pin),
                  torch.empty((6, N), dtype=torch.float64, **pin), torch.empty((21, N), dtype=torch.float64, **pin),
                  torch.empty(N, dtype=torch.float64, **pin), torch.empty(N, dtype=torch.int32, **pin),
                  torch.empty(N, dtype=torch.uint8, **pin))
        self.out = out
        self.outs = kf_outputs(_ptr(out.par), _ptr(out.cov), _ptr(out.tgt_par), _ptr(out.tgt_cov), _ptr(out.chi2),
                               _ptr(out.ndf), _ptr(out.status), None, None, None)
        self.n_chunks, self.n_streams = int(n_chunks), int(n_streams)
        nbytes = lib().kf_staged_workspace_bytes(C.byref(self.cfg), C.byref(self.meas), self.surf.n, self.n_chunks,
                                                 self.n_streams)
        if nbytes == 0:
            raise KFError(KF_E_SIZE, "kf_staged_workspace_bytes")
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
        self.ws_bytes = nbytes
        self.streams = [torch.cuda.Stream(device=dev) for _ in range(self.n_streams)]
        self._handles = (C.c_void_p * self.n_streams)(*[s.cuda_stream for s in self.streams])

    def run(self, stream=None) -> Fit:
        """Enqueue behind `stream` (default: current); on return `stream`
        waits for every chunk, so work later on it sees the host outputs."""
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        for s in self.streams:
            s.wait_stream(stream)
        rc = lib().kf_fit_tracks_staged(C.byref(self.cfg), C.byref(self.surf), C.byref(self.field),
                                        C.byref(self.meas), C.byref(self.seeds), C.byref(self.outs), _ptr(self.ws),
                                        self.ws_bytes, self.n_chunks, self._handles, self.n_streams)
        if rc != KF_OK:
            raise KFError(rc, "kf_fit_tracks_staged")
        for s in self.streams:
            stream.wait_stream(s)
        return self.out


class VjpPlan:
    """Marshalled arguments + workspace of kf_fit_tracks_vjp for one batch."""

    def __init__(self, b: Batch, opt: Options | None = None, want_align: bool = True, want_seed: bool = False):
        opt = opt or Options()
        dev = b.loc.device
        N, H, S = b.n_tracks, b.n_hits, b.center.shape[1]
        self.batch, self.opt = b, opt
        self.cfg, self.surf, self.field, self.meas, self.seeds = _structs(b, opt)
        f64 = dict(dtype=torch.float64, device=dev)
        self.grad = Grad(torch.empty((2, H), **f64), torch.empty((6, S), **f64) if want_align else None,
                         torch.empty((6, N), **f64) if want_seed else None,
                         torch.empty(N, dtype=torch.uint8, device=dev))
        self.grads = kf_gradients(_ptr(self.grad.meas), _ptr(self.grad.align), _ptr(self.grad.seed),
                                  _ptr(self.grad.status))
        nbytes = lib().kf_vjp_workspace_bytes(C.byref(self.cfg), C.byref(self.meas), self.surf.n)
        if nbytes == 0:
            raise KFError(KF_E_SIZE, "kf_fit_tracks_vjp")
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
        self.ws_bytes = nbytes

    def run(self, g_chi2=None, g_par=None, g_tgt=None, stream=None) -> Grad:
        """Enqueue the VJP for cotangents (N,), (6, H), (6, N) (each may be None = 0)."""
        dev = self.batch.loc.device
        keep = [None if g is None else g.to(device=dev, dtype=torch.float64).contiguous()
                for g in (g_chi2, g_par, g_tgt)]
        cot = kf_cotangents(*(_ptr(g) for g in keep))
        if stream is None:
            stream = torch.cuda.current_stream(dev)
        rc = lib().kf_fit_tracks_vjp(C.byref(self.cfg), C.byref(self.surf), C.byref(self.field),
                                     C.byref(self.meas), C.byref(self.seeds), C.byref(cot), C.byref(self.grads),
                                     _ptr(self.ws), self.ws_bytes, C.c_void_p(stream.cuda_stream))
        if rc != KF_OK:
            raise KFError(rc, "kf_fit_tracks_vjp")
        self._keep = keep          # cotangents must outlive the enqueued work
        return self.grad


def kf_fit_tracks_vjp(batch: Batch, g_chi2=None, g_par=None, g_tgt=None, opt: Options | None = None,
                      want_align: bool = True, want_seed: bool = False) -> Grad:
    """dL/d(measurements, alignment, seeds) for L = g_chi2 . chi2 + g_par . par
    + g_tgt . tgt_par (async on the current stream)."""
    return VjpPlan(batch, opt, want_align, want_seed).run(g_chi2, g_par, g_tgt)


class TrackFit(torch.autograd.Function):
    """(loc (2, H), align (6, S) or None) -> (smoothed par (6, H), target par
    (6, N), chi2 (N,)) by kf_fit_tracks; backward by kf_fit_tracks_vjp in the
    same precision (opt.precision).  Every other input of the batch is a
    constant."""

    @staticmethod
    def forward(ctx, loc, align, batch: Batch, opt):
        b = replace(batch, loc=loc.detach().to(torch.float64).contiguous(),
                    align=None if align is None else align.detach().to(torch.float64).contiguous())
        out = Plan(b, opt).run()
        ctx.batch, ctx.opt = b, opt
        ctx.has_align = align is not None
        return out.par, out.tgt_par, out.chi2

    @staticmethod
    def backward(ctx, g_par, g_tgt, g_chi2):
        want_align = ctx.has_align and ctx.needs_input_grad[1]
        g = VjpPlan(ctx.batch, ctx.opt, want_align=want_align).run(g_chi2, g_par, g_tgt)
        return (g.meas if ctx.needs_input_grad[0] else None), (g.align if want_align else None), None, None


def fit_tracks(batch: Batch, loc: torch.Tensor | None = None, align: torch.Tensor | None = None,
               opt: Options | None = None):
    """Differentiable fit: returns (par, tgt_par, chi2) with gradients flowing
    to `loc` (defaults to batch.loc) and `align` (defaults to batch.align)."""
    return TrackFit.apply(batch.loc if loc is None else loc, batch.align if align is None else align, batch, opt)
