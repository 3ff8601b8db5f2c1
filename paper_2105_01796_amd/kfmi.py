"""Python binding of libkfmi.so (argument marshalling only).

Every step of the fit runs in the HIP library.  PyTorch provides device
memory and the current stream.  If the library is not built or cannot be
loaded, every call raises: there is no CPU fallback.

Names mirror include/kf.h: kf_fit_tracks, kf_workspace_bytes, kf_status_string,
kf_version.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libkfmi.so")

# ---- constants (include/kf.h) ----
KF_OK, KF_E_NULL, KF_E_SIZE, KF_E_ENUM, KF_E_WS, KF_E_HIP, KF_E_VALUE = 0, -1, -2, -3, -4, -5, -6
KF_ST_OK, KF_ST_NO_INTERSECT, KF_ST_STEP_CAP, KF_ST_NOT_SPD, KF_ST_BAD_INPUT, KF_ST_TOO_FEW = range(6)
KF_FIELD_UNIFORM, KF_FIELD_SOLENOID = 0, 1
KF_PREC_FP64, KF_PREC_MIXED = 0, 1
KF_SCHED_AUTO, KF_SCHED_DIRECT, KF_SCHED_SORTED = 0, 1, 2
KF_MAX_SURFACES = 512
KF_MAX_HITS = 64


class kf_surfaces(C.Structure):
    _fields_ = [("n", C.c_int32), ("center", C.c_void_p), ("rot", C.c_void_p), ("x_over_X0", C.c_void_p)]


class kf_field(C.Structure):
    _fields_ = [("kind", C.c_int32), ("b0", C.c_double * 3), ("a", C.c_double)]


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
                ("occupancy", C.c_int32), ("split_smoother", C.c_int32)]


class kf_outputs(C.Structure):
    _fields_ = [("par", C.c_void_p), ("cov", C.c_void_p), ("tgt_par", C.c_void_p), ("tgt_cov", C.c_void_p),
                ("chi2", C.c_void_p), ("ndf", C.c_void_p), ("status", C.c_void_p), ("trials", C.c_void_p),
                ("filt_par", C.c_void_p), ("filt_cov", C.c_void_p)]


# every symbol include/kf.h declares
EXPORTS = ("kf_version", "kf_status_string", "kf_workspace_bytes", "kf_fit_tracks", "kf_plan_create",
           "kf_plan_launch", "kf_plan_destroy", "kf_autotune")

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
        _lib = L
    return _lib


def kf_version() -> str:
    return lib().kf_version().decode()


def kf_status_string(code: int) -> str:
    return lib().kf_status_string(int(code)).decode()


class KFError(RuntimeError):
    def __init__(self, code):
        super().__init__(f"kf_fit_tracks failed: {code} ({kf_status_string(code)})")
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

    @property
    def n_tracks(self) -> int:
        return self.hit_offsets.numel() - 1

    @property
    def n_hits(self) -> int:
        return self.surface_id.numel()

    @classmethod
    def from_event(cls, ev, device="cuda", detector=None) -> "Batch":
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
                   mass=float(ev.mass), max_hits=int(max(counts)) if len(counts) else 1)


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


class Plan:
    """Marshalled arguments + workspace for repeated fits of one batch shape.

    Holds the ctypes structs so a timed loop only pays the library call."""

    def __init__(self, b: Batch, opt: Options | None = None, extras: bool = False, out: Fit | None = None):
        opt = opt or Options()
        dev = b.loc.device
        N, H = b.n_tracks, b.n_hits
        self.batch, self.opt = b, opt
        max_hits = b.max_hits
        if max_hits <= 0:
            max_hits = int((b.hit_offsets[1:] - b.hit_offsets[:-1]).max().item()) if N else 1
        max_hits = max(1, min(max_hits, KF_MAX_HITS))
        self.cfg = kf_config(opt.precision, int(b.multiple_scattering), b.mass, opt.rk_tol, opt.land_tol,
                             opt.max_steps, opt.schedule, opt.block, opt.waves_per_cu, opt.occupancy,
                             opt.split_smoother)
        self.surf = kf_surfaces(b.center.shape[1], _ptr(b.center), _ptr(b.rot), _ptr(b.x_over_X0))
        self.field = kf_field(b.field_kind, (C.c_double * 3)(*b.b0), b.field_a)
        self.meas = kf_measurements(N, max_hits, H, _ptr(b.hit_offsets), _ptr(b.surface_id), _ptr(b.loc),
                                    _ptr(b.cov))
        self.seeds = kf_seeds(_ptr(b.seed_par), _ptr(b.seed_cov), b.seed_surface)
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
                    best.waves_per_cu, best.occupancy, best.split_smoother)
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
