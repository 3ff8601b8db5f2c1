#!/usr/bin/env python3
"""Throughput of the batched Kalman-filter track fit on one MI355X.

Workload (default): 1e5 muon tracks, 10 planes normal to x at x = 30..300 mm,
uniform Bz = 2 T, 0.5 % X0 per plane with Highland multiple scattering,
pT 1-10 GeV, |phi| < 0.1, |eta| < 0.2, 50 um hits; seeded synthetic data.
One step = one filter + RTS-smoother pass over all tracks (inputs resident
in HBM), launched as the product runs it: the launch shape is picked by the
library's autotuner (kf_autotune, untimed) and the whole launch sequence is
captured once in a HIP graph (kf_plan_create) that every step replays.
Prints one JSON line.  Besides the FP64 headline it times the
mixed-precision fit, the same fit with the two-filter smoother (a backward
Kalman filter, i.e. a second propagation, instead of RTS), the fit with the
fitted parameters given at the perigee, a fit + adjoint
step (kf_fit_tracks then kf_fit_tracks_vjp with chi2, smoothed-parameter and
target cotangents) in FP64 and in mixed precision, the fit from pinned host
buffers (PCIe included), and, as an extra key, 1e6 tracks of the solenoid
workload (FP64 and mixed fit, fit + adjoint).  Per-step times come with their
mean, RMS spread and median (the paper reports mean +- RMS over repeated
runs).

The roofline entry uses the oracle's count of non-trivial floating-point
operations per track (add/sub, mul, div, sqrt) times the tracks in a launch,
divided by the fit launch's average duration measured with HIP events on the
launch stream; the peak is MI355X's FP64 vector rate.  `traffic` is the HBM
traffic of one fit launch from the committed counter summary
profiles/k_fwd_c2_1e5_traffic.txt (FETCH_SIZE + WRITE_SIZE, each scaled by
the same counter's reading for a plain copy of known size), reported only
while the fit sources still hash to the value recorded there.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "tracks fitted/s (filter+smoother; +adjoint) at 1e5 tracks, FP64 vs mixed"
PEAK_FP64_TFLOPS = 78.6
PEAK_HBM_GBS = 8000.0

WORKLOADS = {
    1: "100 tracks, 10 planes x=30..300 mm, Bz=2 T, pT 1-10 GeV, no material",
    2: "1e5 tracks, 10 planes x=30..300 mm, Bz=2 T, 0.5% X0/plane Highland MS, pT 1-10 GeV, |phi|<0.1, |eta|<0.2",
    3: "1e5 tracks, 30 planes x=30..900 mm, Bz=2 T, ragged 5-30 hits (holes p=0.1)",
    4: "1e5 tracks, 10 planes, Bz=2 T, misaligned truth",
    5: "solenoid B=2T(1-0.1(z/1m)^2), 30 planes, pT log-uniform 0.5-100 GeV, |eta|<2.5, ragged 8-30 hits",
    6: "the tracks of C5 with the field as a map: the solenoid sampled every 25 mm (41x81x481 points, "
       "38 MB), trilinear",
    7: "C2 measured on discs: polar hits (r, phi) about centres 100 mm off the tracks, phi straddling +-pi",
    8: "1e5 tracks through a barrel: 5 cylinders about z (r=30..150 mm; hits z, azimuth) and 5 layers of "
       "straws (wires along z at x=180..300 mm; 1-D drift-distance hits), Bz=2 T, 0.2% X0/layer Highland MS",
}


FIT_SOURCES = ("kf_fit.hip", "kf_fit_kernels.hpp", "kf_curved.hpp", "kf_common.hpp", "kf_device.hpp",
               *(f"kf_fit_{fk}_{p}.hip" for fk in ("uniform", "solenoid", "map") for p in ("fp64", "mixed")))
VJP_SOURCES = ("kf_vjp.hip", "kf_adjoint.hpp", "kf_gap_reverse.hpp", "kf_common.hpp", "kf_device.hpp")
PROFILES = os.path.join(ROOT, "profiles")
TRAFFIC_FILE = os.path.join(PROFILES, "k_fwd_c2_1e5_traffic.txt")
FIT_COUNTER_FILE = os.path.join(PROFILES, "k_fwd_c2_1e5_fp64_counters.txt")
VJP_COUNTER_FILE = os.path.join(PROFILES, "k_vjp_c2_1e5_fp64_counters.txt")


def source_hash(names) -> str:
    h = hashlib.sha256()
    for name in names:
        with open(os.path.join(ROOT, "paper_2105_01796_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def fit_source_hash() -> str:
    return source_hash(FIT_SOURCES)


def recorded(path: str, key: str, config: int, n_tracks: int, sources):
    """A figure per launch from a counter summary under profiles/, or None when
    the summary is missing, for another workload, or older than the kernel's
    sources."""
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    try:
        if kv.get("source_hash") != source_hash(sources):
            return None
        if int(kv["config"]) != config or int(kv["tracks"]) != n_tracks:
            return None
        return float(kv[key])
    except (KeyError, ValueError):
        return None


def recorded_traffic(config: int, n_tracks: int):
    """HBM bytes per FP64 fit launch (FETCH_SIZE + WRITE_SIZE, copy-calibrated)."""
    return recorded(TRAFFIC_FILE, "hbm_bytes_per_launch", config, n_tracks, FIT_SOURCES)


def log(msg: str) -> None:
    """Progress on stderr (stdout carries only the JSON line)."""
    print(f"bench: {msg}", file=sys.stderr, flush=True)


def host_threads() -> int:
    n = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    env = os.environ.get("OMP_NUM_THREADS")
    if env and env.isdigit():
        n = min(n, int(env))
    return max(1, n)


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def step_stats(per):
    """Mean, RMS spread (the paper's mean +- RMS over repeated runs), median,
    min and max of the per-step times (ms)."""
    import numpy as np
    a = np.asarray(per, dtype=float)
    return {"mean": float(a.mean()), "rms": float(a.std()), "median": float(np.median(a)),
            "min": float(a.min()), "max": float(a.max()), "n": int(a.size)}


def time_plan(plan, steps, warmup):
    import torch
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        plan.run(stream)
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0.record(stream)
    for a, b in ev:
        a.record(stream)
        plan.run(stream)
        b.record(stream)
    t1.record(stream)
    torch.cuda.synchronize()
    total_ms = t0.elapsed_time(t1)
    per = [a.elapsed_time(b) for a, b in ev]
    return total_ms / steps, sum(per) / len(per), per


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", type=int, default=2, choices=sorted(WORKLOADS))
    ap.add_argument("--tracks", type=int, default=None)
    ap.add_argument("--schedule", type=int, default=0)
    ap.add_argument("--block", type=int, default=0)
    ap.add_argument("--occupancy", type=int, default=0)
    ap.add_argument("--waves-per-cu", type=int, default=0)
    ap.add_argument("--jacobians", choices=("store", "recompute"), default="store",
                    help="without --autotune: transport Jacobians stored for the smoother or recomputed by it")
    ap.add_argument("--output", choices=("auto", "staged", "slots"), default="auto",
                    help="RTS smoother output path (auto: the autotuner's, else staged)")
    ap.add_argument("--no-mixed", action="store_true", help="skip the mixed-precision leg")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the fit + adjoint leg")
    ap.add_argument("--no-two-filter", action="store_true", help="skip the two-filter smoother leg")
    ap.add_argument("--no-perigee", action="store_true", help="skip the perigee-target leg")
    ap.add_argument("--no-solenoid", action="store_true",
                    help="skip the extra leg on 1e6 solenoid tracks (FP64 and mixed fit, fit + adjoint)")
    ap.add_argument("--no-staged", action="store_true",
                    help="skip the host-buffer leg (copies in, fit, copies out, chunked over streams)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run one plain 512 MiB device copy first (reference for HBM counters)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="use the given (or default) launch settings instead of the autotuner's")
    ap.add_argument("--no-graph", action="store_true", help="launch eagerly instead of replaying a HIP graph")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: this build measures one GPU only (tracks are independent; the multi-GPU "
              "sharding is described in DESIGN.md and not built). Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2105_01796_amd import kfmi, synth

    t_gen = time.time()
    ev = synth.make_config(args.config, args.tracks)
    t_gen = time.time() - t_gen
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    batch = kfmi.Batch.from_event(ev, device=dev)
    N = ev.n_tracks
    base_opt = dict(schedule=args.schedule, block=args.block, occupancy=args.occupancy,
                    waves_per_cu=args.waves_per_cu,
                    jacobians=kfmi.KF_JAC_RECOMPUTE if args.jacobians == "recompute" else kfmi.KF_JAC_STORE,
                    output={"auto": kfmi.KF_OUT_AUTO, "staged": kfmi.KF_OUT_STAGED,
                            "slots": kfmi.KF_OUT_SLOTS}[args.output])

    if args.copy_calibration:
        src = torch.empty(1 << 26, dtype=torch.float64, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    def prepared_plan(precision, **extra):
        """Plan with autotuned launch settings, captured in a HIP graph."""
        plan = kfmi.Plan(batch, kfmi.Options(precision=precision, **base_opt, **extra))
        tuned = None
        if not args.no_autotune:
            opt, tune_ms = plan.autotune()
            tuned = {"schedule": opt.schedule, "block": opt.block, "occupancy": opt.occupancy,
                     "waves_per_cu": opt.waves_per_cu, "split_smoother": opt.split_smoother,
                     "jacobians": "recompute" if opt.jacobians == kfmi.KF_JAC_RECOMPUTE else "store",
                     "output": "slots" if opt.output == kfmi.KF_OUT_SLOTS else "staged",
                     "tuner_ms": round(tune_ms, 4)}
        if not args.no_graph:
            plan.capture()
        return plan, tuned

    # FP64 leg (the headline value)
    log(f"workload C{args.config}, {N} tracks, {ev.n_hits} hits: FP64 fit (autotune, graph)")
    plan64, tuned64 = prepared_plan(kfmi.KF_PREC_FP64)
    ms64, kms64, per64 = time_plan(plan64, args.steps, args.warmup)
    st = plan64.out.status.cpu().numpy()
    n_ok = int((st == 0).sum())

    mixed = None
    if not args.no_mixed:
        log("mixed-precision fit")
        planm, tunedm = prepared_plan(kfmi.KF_PREC_MIXED)
        msm, kmsm, perm = time_plan(planm, args.steps, args.warmup)
        mixed = {"value": N / (msm * 1e-3), "ms_per_step": msm, "launch_ms": kmsm,
                 "launch_ms_stats": step_stats(perm),
                 "speedup_vs_fp64": ms64 / msm, "launch": tunedm}

    two_filter = None
    if not args.no_two_filter:
        # the other smoother of Sect. 2: a backward Kalman filter (second
        # propagation) combined with the forward filter, same workload
        log("two-filter smoother")
        plant, tunedt = prepared_plan(kfmi.KF_PREC_FP64, smoother=kfmi.KF_SMOOTHER_TWO_FILTER)
        mst, kmst, _ = time_plan(plant, args.steps, args.warmup)
        two_filter = {"value": N / (mst * 1e-3), "unit": "tracks/s", "ms_per_step": mst, "launch_ms": kmst,
                      "rts_speedup": mst / ms64, "launch": tunedt,
                      "tracks_ok": int((plant.out.status.cpu().numpy() == 0).sum()),
                      "what": "filter + two-filter smoother (backward filter from the last hit, "
                              "combined with the forward filter), FP64"}
        del plant

    perigee = None
    if not args.no_perigee:
        # fitted parameters at the perigee of the z axis instead of the seed
        # plane: one more FP64 propagation per track after the smoother
        log("perigee target")
        planp, _ = prepared_plan(kfmi.KF_PREC_FP64, target=kfmi.KF_TARGET_PERIGEE, perigee=(0.0, 0.0, 0.0))
        msp, kmsp, _ = time_plan(planp, args.steps, args.warmup)
        perigee = {"value": N / (msp * 1e-3), "unit": "tracks/s", "ms_per_step": msp, "launch_ms": kmsp,
                   "extra_ms": msp - ms64,
                   "tracks_ok": int((planp.out.status.cpu().numpy() == 0).sum()),
                   "what": "filter + RTS smoother + propagation of the fitted state to the perigee of the "
                           "z axis, FP64"}
        del planp

    staged = None
    if not args.no_staged:
        # the same fit from pinned host buffers: transfers included (PCIe), chunks
        # pipelined over streams so that copies overlap the fit
        log("host-staged fit")
        bh = kfmi.Batch.staged_from_event(ev, device=dev)
        opt_st = dict(base_opt)
        if tuned64:
            opt_st.update({k: tuned64[k] for k in ("schedule", "block", "occupancy", "waves_per_cu", "split_smoother")})
            opt_st["jacobians"] = kfmi.KF_JAC_RECOMPUTE if tuned64["jacobians"] == "recompute" else kfmi.KF_JAC_STORE
            opt_st["output"] = kfmi.KF_OUT_SLOTS if tuned64["output"] == "slots" else kfmi.KF_OUT_STAGED
        runs = {}
        for chunks, streams in ((1, 1), (4, 2), (8, 2), (8, 3)):
            sp = kfmi.StagedPlan(bh, kfmi.Options(**opt_st), n_chunks=chunks, n_streams=streams)
            ms_s, _, _ = time_plan(sp, min(args.steps, 5), 1)
            runs[f"{chunks}x{streams}"] = ms_s
            del sp
        best = min(runs, key=runs.get)
        in_bytes = ev.n_hits * (4 + 5 * 8) + (N + 1) * 4 + N * 27 * 8
        out_bytes = ev.n_hits * 27 * 8 + N * (27 * 8 + 8 + 4 + 1)
        staged = {"value": N / (runs[best] * 1e-3), "unit": "tracks/s", "ms_per_step": runs[best],
                  "chunks_x_streams": best, "ms_by_chunks_x_streams": runs,
                  "h2d_bytes": in_bytes, "d2h_bytes": out_bytes,
                  "what": "pinned host inputs -> kf_fit_tracks_staged -> pinned host outputs, FP64 "
                          "(PCIe-inclusive; not the headline value)"}

    adjoint = None
    if (not args.no_adjoint and int(ev.field.kind) != kfmi.KF_FIELD_MAP    # the adjoint needs an analytic
            and getattr(ev.detector, "stype", None) is None):              # field and planes
        log("fit + adjoint")
        rng_g = np.random.default_rng(1)
        g_chi2 = torch.ones(N, dtype=torch.float64, device=dev)
        g_par = torch.as_tensor(rng_g.standard_normal((6, ev.n_hits)), device=dev)
        g_tgt = torch.as_tensor(rng_g.standard_normal((6, N)), device=dev)
        vjp = kfmi.VjpPlan(batch, kfmi.Options(), want_align=True, want_seed=True)

        class FitAndAdjoint:
            def run(self, stream):
                plan64.run(stream)
                vjp.run(g_chi2, g_par, g_tgt, stream=stream)

        class AdjointOnly:
            def __init__(self, v):
                self.v = v

            def run(self, stream):
                self.v.run(g_chi2, g_par, g_tgt, stream=stream)

        adj_steps = max(1, min(args.steps, 5))
        msa, kmsa, _ = time_plan(FitAndAdjoint(), adj_steps, min(args.warmup, 1))
        msv, _, perv = time_plan(AdjointOnly(vjp), adj_steps, 1)
        st_a = vjp.grad.status.cpu().numpy()
        adjoint = {"value": N / (msa * 1e-3), "unit": "tracks/s", "ms_per_step": msa, "steps": adj_steps,
                   "vjp_ms": msv, "vjp_ms_stats": step_stats(perv), "tracks_ok": int((st_a == 0).sum()),
                   "what": "kf_fit_tracks + kf_fit_tracks_vjp (d chi2, d smoothed params, d target params "
                           "-> d measurements, d alignment of every plane, d seeds), FP64"}
        if mixed is not None:
            vjpm = kfmi.VjpPlan(batch, kfmi.Options(precision=kfmi.KF_PREC_MIXED), want_align=True, want_seed=True)

            class MixedFitAndAdjoint:
                def run(self, stream):
                    planm.run(stream)
                    vjpm.run(g_chi2, g_par, g_tgt, stream=stream)

            msam, _, _ = time_plan(MixedFitAndAdjoint(), adj_steps, 1)
            msvm, _, _ = time_plan(AdjointOnly(vjpm), adj_steps, 1)
            adjoint["mixed"] = {"value": N / (msam * 1e-3), "unit": "tracks/s", "ms_per_step": msam,
                                "vjp_ms": msvm, "speedup_vs_fp64": msa / msam,
                                "what": "the same step with the mixed fit and the mixed adjoint (FP32 "
                                        "recompute and replay of the propagation, FP64 reverse sweep)"}
            del vjpm
        del vjp

    solenoid = None
    if not args.no_solenoid and args.config == 2:
        # 1e6 tracks of the solenoid workload (30 planes, ragged 8-30 hits, pT
        # 0.5-100 GeV, |eta| < 2.5): FP64 and mixed fits, and fit + adjoint in
        # both precisions; an extra key, the headline stays the workload above
        log("solenoid workload, 1e6 tracks: generating")
        t5 = time.time()
        ev5 = synth.make_config(5, 1_000_000)
        t5 = time.time() - t5
        b5 = kfmi.Batch.from_event(ev5, device=dev)
        N5 = ev5.n_tracks
        rng5 = np.random.default_rng(5)
        g5 = (torch.ones(N5, dtype=torch.float64, device=dev),
              torch.as_tensor(rng5.standard_normal((6, ev5.n_hits)), device=dev),
              torch.as_tensor(rng5.standard_normal((6, N5)), device=dev))
        solenoid = {"workload": "C5: " + WORKLOADS[5], "tracks": N5, "hits": ev5.n_hits,
                    "gen_seconds": round(t5, 2)}
        for name, prec in (("fp64", kfmi.KF_PREC_FP64), ("mixed", kfmi.KF_PREC_MIXED)):
            log(f"solenoid workload, 1e6 tracks: {name} fit and fit + adjoint")
            p5 = kfmi.Plan(b5, kfmi.Options(precision=prec, **base_opt))
            if not args.no_autotune:
                p5.autotune()
            if not args.no_graph:
                p5.capture()
            ms5, _, per5 = time_plan(p5, 5, 1)
            v5 = kfmi.VjpPlan(b5, kfmi.Options(precision=prec), want_align=True, want_seed=True)

            class Fit5AndAdjoint:
                def run(self, stream):
                    p5.run(stream)
                    v5.run(*g5, stream=stream)

            ms5a, _, _ = time_plan(Fit5AndAdjoint(), 3, 1)
            solenoid[name] = {"fit": {"value": N5 / (ms5 * 1e-3), "unit": "tracks/s", "ms_per_step": ms5,
                                      "ms_stats": step_stats(per5),
                                      "tracks_ok": int((p5.out.status.cpu().numpy() == 0).sum())},
                              "fit_adjoint": {"value": N5 / (ms5a * 1e-3), "unit": "tracks/s", "ms_per_step": ms5a,
                                              "tracks_ok": int((v5.grad.status.cpu().numpy() == 0).sum())}}
            p5.release()
            del p5, v5
            torch.cuda.empty_cache()
        del b5, g5, ev5

    # algorithmic work per track (oracle operation count on a sample)
    import oracle
    rng = np.random.default_rng(0)
    idx = np.sort(rng.choice(N, min(N, 400), replace=False))
    cnt = oracle.count_ops(ev.subset(idx))
    flops_per_track = float(cnt[:, :4].sum(axis=1).mean())
    hits_per_track = ev.n_hits / N
    flops = flops_per_track * N
    achieved = flops / (kms64 * 1e-3) / 1e12
    io_bytes = ev.n_hits * (2 + 3) * 8 + ev.n_hits * 4 + (N + 1) * 4 + N * 27 * 8 \
        + ev.n_hits * 27 * 8 + N * 27 * 8 + N * (8 + 4 + 1)
    traffic = recorded_traffic(args.config, N)
    roofline = {"bound": "alu", "achieved": achieved, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                "frac": achieved / PEAK_FP64_TFLOPS, "traffic": traffic,
                "flops_per_track": flops_per_track, "hits_per_track": hits_per_track,
                "io_bytes_per_launch": io_bytes, "io_GBs": io_bytes / (kms64 * 1e-3) / 1e9}
    # the FP64 instructions the fit kernel executes (hardware counters of the
    # same launch shape, recorded under profiles/): the executed rate beside the
    # algorithmic one (the kernel recomputes each filtered state in the smoother)
    ex = recorded(FIT_COUNTER_FILE, "fp64_flops_per_launch", args.config, N, FIT_SOURCES)
    roofline["executed"] = None if ex is None else {
        "flops_per_launch": ex, "achieved": ex / (kms64 * 1e-3) / 1e12, "frac": ex / (kms64 * 1e-3) / 1e12 /
        PEAK_FP64_TFLOPS, "source": os.path.relpath(FIT_COUNTER_FILE, ROOT),
        "what": "64 x (ADD + MUL + 2 FMA + TRANS) F64 wave instructions per launch (every lane counted)"}
    if adjoint is not None:
        exa = recorded(VJP_COUNTER_FILE, "fp64_flops_per_launch", args.config, N, VJP_SOURCES)
        adjoint["roofline"] = None if exa is None else {
            "bound": "alu", "achieved": exa / (adjoint["vjp_ms"] * 1e-3) / 1e12, "peak": PEAK_FP64_TFLOPS,
            "unit": "TFLOP/s", "frac": exa / (adjoint["vjp_ms"] * 1e-3) / 1e12 / PEAK_FP64_TFLOPS,
            "flops_per_launch": exa, "source": os.path.relpath(VJP_COUNTER_FILE, ROOT),
            "what": "executed FP64 work of the adjoint kernel (64 x (ADD + MUL + 2 FMA + TRANS) F64 wave "
                    "instructions, hardware counters recorded) over the adjoint call's event time"}

    cpu = None
    if not args.no_cpu_baseline:
        log("CPU baseline (oracle)")
        nth = host_threads()
        m = min(N, 20000)
        sub = ev.subset(np.arange(m))
        oracle.fit(sub, n_threads=nth)        # warm
        t0 = time.time()
        done = 0
        while True:
            oracle.fit(sub, n_threads=nth)
            done += m
            if time.time() - t0 >= args.cpu_seconds:
                break
        dt = time.time() - t0
        # one thread on a smaller sample (about a quarter of the all-core time)
        m1 = min(N, 2000)
        sub1 = ev.subset(np.arange(m1))
        t1 = time.time()
        done1 = 0
        while True:
            oracle.fit(sub1, n_threads=1)
            done1 += m1
            if time.time() - t1 >= args.cpu_seconds / 4:
                break
        dt1 = time.time() - t1
        cpu = {"value": done / dt, "unit": "tracks/s", "cores": nth, "kind": "oracle",
               "sample": f"first {m} tracks of the same workload, fitted {done // m}x in {dt:.1f} s "
                         f"(FP64 filter+smoother, OpenMP over tracks)",
               "cpu_model": cpu_model(), "nproc": os.cpu_count(),
               "one_thread": {"value": done1 / dt1, "unit": "tracks/s",
                              "sample": f"first {m1} tracks, fitted {done1 // m1}x in {dt1:.1f} s on 1 thread"}}

    out = {
        "metric": METRIC,
        "value": N / (ms64 * 1e-3),
        "unit": "tracks/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms64,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"C{args.config}: " + WORKLOADS[args.config], "tracks": N,
                   "hits": ev.n_hits, "precision": "fp64", "launch_ms": kms64,
                   "launch_ms_min": min(per64), "launch_ms_stats": step_stats(per64), "tracks_ok": n_ok,
                   "options": base_opt,
                   "launch": tuned64, "graph": not args.no_graph,
                   "gen_seconds": round(t_gen, 2)},
        "mixed": mixed,
        "adjoint": adjoint,
        "two_filter": two_filter,
        "perigee": perigee,
        "staged": staged,
        "solenoid_1e6": solenoid,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
