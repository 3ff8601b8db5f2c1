"""The C ABI of libkfmi.so on the CPU: the library loads, exports every symbol
include/kf.h declares, and rejects bad arguments on the host before any device
work (no GPU needed: validation precedes every HIP call)."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def kf():
    from paper_2105_01796_amd import kfmi
    kfmi.lib()
    return kfmi


def _declared():
    txt = open(os.path.join(ROOT, "include", "kf.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(kf_[a-z_]+)\s*\(", txt)))


def test_exports_every_declared_symbol(kf):
    decl = _declared()
    assert set(decl) == set(kf.EXPORTS), decl
    L = kf.lib()
    for name in decl:
        assert hasattr(L, name), name
    assert "gfx950" in kf.kf_version()


def test_status_strings(kf):
    for code in [0, -1, -2, -3, -4, -5, -6, -7, 1, 2, 3, 4, 5]:
        assert kf.kf_status_string(code) != "unknown code"
    assert kf.kf_status_string(99) == "unknown code"


def _args(kf, N=10, H=100, max_hits=10, S=11):
    fake = C.c_void_p(0x1000)     # never dereferenced on the host
    cfg = kf.kf_config(0, 0, 0.1056583755, 1e-4, 1e-6, 1000, 0, 0, 0, 0, 0, 0)
    surf = kf.kf_surfaces(S, fake, fake, fake)
    fld = kf.kf_field(0, (C.c_double * 3)(0, 0, 2), 0.0)
    meas = kf.kf_measurements(N, max_hits, H, fake, fake, fake, fake)
    seeds = kf.kf_seeds(fake, fake, 0)
    out = kf.kf_outputs(fake, fake, fake, fake, fake, fake, fake, None, None, None)
    return cfg, surf, fld, meas, seeds, out


def _call(kf, cfg, surf, fld, meas, seeds, out, ws=C.c_void_p(0x2000), nbytes=None):
    L = kf.lib()
    if nbytes is None:
        nbytes = L.kf_workspace_bytes(C.byref(cfg), C.byref(meas), surf.n)
    return L.kf_fit_tracks(C.byref(cfg), C.byref(surf), C.byref(fld), C.byref(meas), C.byref(seeds),
                           C.byref(out), ws, nbytes, None)


def test_null_struct_pointers(kf):
    L = kf.lib()
    assert L.kf_fit_tracks(None, None, None, None, None, None, None, 0, None) == kf.KF_E_NULL


def test_argument_validation(kf):
    a = _args(kf)
    cfg, surf, fld, meas, seeds, out = a
    # bad enums
    cfg.precision = 7
    assert _call(kf, *a) == kf.KF_E_ENUM
    cfg.precision = 0
    cfg.schedule = 9
    assert _call(kf, *a) == kf.KF_E_ENUM
    cfg.schedule = 0
    fld.kind = 5
    assert _call(kf, *a) == kf.KF_E_ENUM
    fld.kind = 0
    # bad values
    cfg.rk_tol = 0.0
    assert _call(kf, *a) == kf.KF_E_VALUE
    cfg.rk_tol = 1e-4
    cfg.block = 100
    assert _call(kf, *a) == kf.KF_E_VALUE
    cfg.block = 0
    cfg.occupancy = 9
    assert _call(kf, *a) == kf.KF_E_VALUE
    cfg.occupancy = 0
    cfg.split_smoother = 2
    assert _call(kf, *a) == kf.KF_E_VALUE
    cfg.split_smoother = 0
    cfg.jacobians = 2
    assert _call(kf, *a) == kf.KF_E_VALUE
    cfg.jacobians = kf.KF_JAC_RECOMPUTE
    cfg.split_smoother = 1                     # the split smoother needs stored Jacobians
    assert _call(kf, *a) == kf.KF_E_VALUE
    cfg.split_smoother = 0
    cfg.jacobians = kf.KF_JAC_STORE
    cfg.smoother = 2
    assert _call(kf, *a) == kf.KF_E_VALUE
    cfg.smoother = kf.KF_SMOOTHER_TWO_FILTER
    cfg.split_smoother = 1                     # the two-filter smoother is fused only
    assert _call(kf, *a) == kf.KF_E_VALUE
    cfg.split_smoother = 0
    for bad in (0.5, 1.0, -3.0, float("nan"), float("inf")):
        cfg.bwd_scale = bad
        assert _call(kf, *a) == kf.KF_E_VALUE, bad
    cfg.bwd_scale = 0.0
    cfg.smoother = kf.KF_SMOOTHER_RTS
    cfg.target = 2
    assert _call(kf, *a) == kf.KF_E_VALUE
    cfg.target = kf.KF_TARGET_PERIGEE
    cfg.perigee[1] = float("nan")
    assert _call(kf, *a) == kf.KF_E_VALUE
    cfg.perigee[1] = 0.0
    cfg.target = kf.KF_TARGET_SEED_SURFACE
    cfg.output = 3                               # KF_OUT_* out of range
    assert _call(kf, *a) == kf.KF_E_VALUE
    cfg.output = kf.KF_OUT_SLOTS
    # cylinders and lines (surface types with radii) run one wave per SIMD only
    surf.type = C.c_void_p(0x1000)
    surf.radius = C.c_void_p(0x1000)
    cfg.occupancy = 2
    assert _call(kf, *a) == kf.KF_E_VALUE
    cfg.occupancy = 0
    surf.type = None
    surf.radius = None
    # tabulated field: pointer, grid size and spacing are checked
    fld.kind = kf.KF_FIELD_MAP
    assert _call(kf, *a) == kf.KF_E_NULL
    fld.map = C.c_void_p(0x3000)
    assert _call(kf, *a) == kf.KF_E_VALUE           # map_n = 0
    fld.map_n[0], fld.map_n[1], fld.map_n[2] = 4, 4, 1
    fld.map_spacing[0] = fld.map_spacing[1] = fld.map_spacing[2] = 10.0
    assert _call(kf, *a) == kf.KF_E_VALUE           # fewer than 2 points along z
    fld.map_n[2] = 4
    fld.map_spacing[1] = -1.0
    assert _call(kf, *a) == kf.KF_E_VALUE
    fld.map_spacing[1] = 10.0
    fld.kind = 0
    fld.b0[2] = float("nan")
    assert _call(kf, *a) == kf.KF_E_VALUE
    fld.b0[2] = 2.0
    # bad sizes
    meas.max_hits = kf.KF_MAX_HITS + 1
    assert _call(kf, *a, nbytes=1 << 30) == kf.KF_E_SIZE
    meas.max_hits = 10
    meas.n_tracks = -1
    assert _call(kf, *a, nbytes=1 << 30) == kf.KF_E_SIZE
    meas.n_tracks = 10
    surf.n = 0
    assert _call(kf, *a, nbytes=1 << 30) == kf.KF_E_SIZE
    surf.n = 11
    seeds.surface_id = 11
    assert _call(kf, *a) == kf.KF_E_SIZE
    seeds.surface_id = 0
    # null inner pointers
    surf.center = None
    assert _call(kf, *a) == kf.KF_E_NULL
    surf.center = C.c_void_p(0x1000)
    out.chi2 = None
    assert _call(kf, *a) == kf.KF_E_NULL
    out.chi2 = C.c_void_p(0x1000)
    out.filt_par = C.c_void_p(0x1000)      # filt_par without filt_cov
    assert _call(kf, *a) == kf.KF_E_NULL
    out.filt_par = None
    # workspace
    assert _call(kf, *a, ws=None) == kf.KF_E_WS
    need = kf.lib().kf_workspace_bytes(C.byref(cfg), C.byref(meas), surf.n)
    assert need >= 64 * 10 * 52 * 8          # one 64-track tile x 10 hits x 52 doubles
    assert _call(kf, *a, nbytes=need - 1) == kf.KF_E_WS
    # nothing to do: no tracks is OK without touching the device
    meas.n_tracks = 0
    assert _call(kf, *a) == kf.KF_OK


def test_noalloc_checks_arguments_and_scratch_size_on_the_host(kf):
    """kf_fit_tracks_noalloc validates like kf_fit_tracks and refuses a batch
    whose workspace exceeds its static scratch before touching the device."""
    L = kf.lib()

    def call(cfg, surf, fld, meas, seeds, out):
        return L.kf_fit_tracks_noalloc(C.byref(cfg), C.byref(surf), C.byref(fld), C.byref(meas),
                                       C.byref(seeds), C.byref(out), None)

    assert L.kf_fit_tracks_noalloc(None, None, None, None, None, None, None) == kf.KF_E_NULL
    a = _args(kf, N=20000, H=200000, max_hits=10)
    cfg, surf, fld, meas, seeds, out = a
    assert L.kf_workspace_bytes(C.byref(cfg), C.byref(meas), surf.n) > kf.KF_NOALLOC_SCRATCH_BYTES
    assert call(*a) == kf.KF_E_SCRATCH
    cfg.precision = 7
    assert call(*a) == kf.KF_E_ENUM
    cfg.precision = 0
    meas.max_hits = kf.KF_MAX_HITS + 1
    assert call(*a) == kf.KF_E_SIZE
    meas.max_hits = 10
    meas.n_tracks = 0
    assert call(*a) == kf.KF_OK


def test_workspace_size_grows_with_tracks_and_hits(kf):
    L = kf.lib()
    cfg = kf.kf_config(0, 0, 0.1, 1e-4, 1e-6, 1000, 0, 0, 0, 0, 0)
    sizes = []
    for N, mh in [(1, 10), (64, 10), (65, 10), (1000, 30)]:
        m = kf.kf_measurements(N, mh, N * mh, None, None, None, None)
        sizes.append(L.kf_workspace_bytes(C.byref(cfg), C.byref(m), 31))
    assert sizes[0] == sizes[1] < sizes[2] < sizes[3]
    m = kf.kf_measurements(10, 0, 0, None, None, None, None)
    assert L.kf_workspace_bytes(C.byref(cfg), C.byref(m), 31) == 0


def _vjp_call(kf, cfg, surf, fld, meas, seeds, cot, grad, ws=C.c_void_p(0x2000), nbytes=None):
    L = kf.lib()
    if nbytes is None:
        nbytes = L.kf_vjp_workspace_bytes(C.byref(cfg), C.byref(meas), surf.n)
    return L.kf_fit_tracks_vjp(C.byref(cfg), C.byref(surf), C.byref(fld), C.byref(meas), C.byref(seeds),
                               C.byref(cot) if cot is not None else None,
                               C.byref(grad) if grad is not None else None, ws, nbytes, None)


def test_vjp_argument_validation(kf):
    cfg, surf, fld, meas, seeds, _ = _args(kf)
    fake = C.c_void_p(0x1000)
    cot = kf.kf_cotangents(fake, None, None)
    grad = kf.kf_gradients(fake, fake, None, None)
    L = kf.lib()
    assert L.kf_fit_tracks_vjp(None, None, None, None, None, None, None, None, 0, None) == kf.KF_E_NULL
    assert _vjp_call(kf, cfg, surf, fld, meas, seeds, None, grad) == kf.KF_E_NULL
    assert _vjp_call(kf, cfg, surf, fld, meas, seeds, cot, None) == kf.KF_E_NULL
    cfg.precision = 7
    assert _vjp_call(kf, cfg, surf, fld, meas, seeds, cot, grad) == kf.KF_E_ENUM
    cfg.precision = 0
    fld.kind = 3
    assert _vjp_call(kf, cfg, surf, fld, meas, seeds, cot, grad) == kf.KF_E_ENUM
    fld.kind = 0
    cfg.land_tol = -1.0
    assert _vjp_call(kf, cfg, surf, fld, meas, seeds, cot, grad) == kf.KF_E_VALUE
    cfg.land_tol = 1e-6
    cfg.smoother = kf.KF_SMOOTHER_TWO_FILTER    # the adjoint is that of the RTS fit
    assert _vjp_call(kf, cfg, surf, fld, meas, seeds, cot, grad) == kf.KF_E_VALUE
    cfg.smoother = kf.KF_SMOOTHER_RTS
    cfg.target = kf.KF_TARGET_PERIGEE           # ... ending on the seed surface
    assert _vjp_call(kf, cfg, surf, fld, meas, seeds, cot, grad) == kf.KF_E_VALUE
    cfg.target = kf.KF_TARGET_SEED_SURFACE
    surf.type = C.c_void_p(0x4000)              # ... on planes
    assert _vjp_call(kf, cfg, surf, fld, meas, seeds, cot, grad) == kf.KF_E_VALUE
    surf.type = None
    surf.radius = C.c_void_p(0x4000)            # (no cylinders)
    assert _vjp_call(kf, cfg, surf, fld, meas, seeds, cot, grad) == kf.KF_E_VALUE
    surf.radius = None
    fld.kind = kf.KF_FIELD_MAP                  # ... in an analytic field
    fld.map = C.c_void_p(0x3000)
    fld.map_n[0] = fld.map_n[1] = fld.map_n[2] = 4
    fld.map_spacing[0] = fld.map_spacing[1] = fld.map_spacing[2] = 10.0
    assert _vjp_call(kf, cfg, surf, fld, meas, seeds, cot, grad) == kf.KF_E_VALUE
    fld.kind = 0
    surf.n = kf.KF_MAX_SURFACES + 1
    assert _vjp_call(kf, cfg, surf, fld, meas, seeds, cot, grad, nbytes=1 << 40) == kf.KF_E_SIZE
    surf.n = 11
    grad.meas = None                       # required when there are hits
    assert _vjp_call(kf, cfg, surf, fld, meas, seeds, cot, grad) == kf.KF_E_NULL
    grad.meas = fake
    assert _vjp_call(kf, cfg, surf, fld, meas, seeds, cot, grad, ws=None) == kf.KF_E_WS
    need = L.kf_vjp_workspace_bytes(C.byref(cfg), C.byref(meas), surf.n)
    # per-hit state (87 doubles x max_hits per track slot) + alignment contributions (6 per hit and track)
    assert need >= 64 * 10 * 87 * 8 + 6 * (100 + 10) * 8
    assert _vjp_call(kf, cfg, surf, fld, meas, seeds, cot, grad, nbytes=need - 1) == kf.KF_E_WS
    m = kf.kf_measurements(10, 0, 0, None, None, None, None)
    assert L.kf_vjp_workspace_bytes(C.byref(cfg), C.byref(m), 11) == 0


def test_staged_argument_validation(kf):
    """kf_fit_tracks_staged: host-side checks, and a workspace of one chunk
    slot per stream sized for the largest chunk."""
    import numpy as np
    L = kf.lib()
    cfg, surf, fld, _, seeds, out = _args(kf)
    off = np.array([0, 10, 25, 25, 40], dtype=np.int32)          # host CSR, chunk sizes 10+15 | 0+15 hits
    meas = kf.kf_measurements(4, 15, 40, C.c_void_p(off.ctypes.data), C.c_void_p(0x1000), C.c_void_p(0x1000),
                              C.c_void_p(0x1000))
    one = L.kf_staged_workspace_bytes(C.byref(cfg), C.byref(meas), surf.n, 2, 1)
    assert one > 0 and L.kf_staged_workspace_bytes(C.byref(cfg), C.byref(meas), surf.n, 2, 3) == 3 * one
    assert L.kf_staged_workspace_bytes(C.byref(cfg), C.byref(meas), surf.n, 0, 1) == 0
    assert L.kf_staged_workspace_bytes(C.byref(cfg), C.byref(meas), surf.n, 2, 0) == 0
    # more chunks than tracks are clamped to one track per chunk
    assert L.kf_staged_workspace_bytes(C.byref(cfg), C.byref(meas), surf.n, 99, 1) > 0
    streams = (C.c_void_p * 2)(0x3000, 0x3000)

    def call(n_chunks=2, n_streams=2, ws=C.c_void_p(0x2000), nbytes=1 << 40, st=streams):
        return L.kf_fit_tracks_staged(C.byref(cfg), C.byref(surf), C.byref(fld), C.byref(meas), C.byref(seeds),
                                      C.byref(out), ws, nbytes, n_chunks, st, n_streams)
    assert call(n_chunks=0) == kf.KF_E_VALUE
    assert call(n_streams=0) == kf.KF_E_VALUE
    assert call(st=None) == kf.KF_E_NULL
    out.trials = C.c_void_p(0x1000)                              # optional outputs are not staged
    assert call() == kf.KF_E_VALUE
    out.trials = None
    assert call(ws=None) == kf.KF_E_WS
    assert call(nbytes=2 * one - 1) == kf.KF_E_WS
    off[4] = 41                                                  # offsets disagree with n_hits
    assert call() == kf.KF_E_SIZE
    off[4] = 40
    meas.n_tracks = 0
    assert call() == kf.KF_OK
