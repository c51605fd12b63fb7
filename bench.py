#!/usr/bin/env python3
"""Throughput of per-pixel TDM-MIMO beat-cube synthesis on one MI355X.

One step = one rs_beat_synthesize call (every stage of the path: pixel
geometry, binary64 phase arguments, phasors, the complex contraction on the
matrix cores, the split-K reduction) on the 256x256 room-plus-pedestrian
frame: 65,536 pixels, 3 Tx x 4 Rx, Ns = 256, L = 128, complex64 output, split
fp16 matrix-core form.  Inputs are resident in HBM before timing starts.

Printed as one JSON line: terms/s (P*M*N*Ns*L per second), the roofline of
the contraction kernel (HIP-event durations of that kernel during the timed
steps), p50/p99 step latency, parity vs the CPU oracle on sampled entries,
the plain binary64 form on the same frame, the 64-frame batched launch, the
serving loop at a fixed request rate, and the oracle timed on the host cores.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "scatterer-sample terms/s (P*M*N*Ns*L/s) MFMA vs FP64-direct at stated err; p50/p99"
PEAK_FP16 = 2.5e15     # dense fp16 matrix flop/s, MI355X
PEAK_FP64 = 78.6e12    # fp64 vector flop/s, MI355X
FLOP_MFMA = 24         # 3 split products x complex MAC (4 real MACs) x 2
FLOP_PLAIN = 8         # one binary64 complex MAC

# HBM bytes per launch of k_mfma_split16 on the headline frame: rocprofv3 --pmc
# FETCH_SIZE and WRITE_SIZE (KiB per dispatch) scaled by what the same counters
# read for a 1 GiB device copy (fetch x 2.0, write x 1.0).  They hold only for
# the kernel sources they were taken on; any change to those sources turns
# the figure into null until the counters are taken again.
TRAFFIC = {"sources": ("rs_mfma.hip", "rs_device.h", "rs_internal.h", "rs_split16.h"),
           "sources_sha256": "44849d3c15d1a5854c90d8e613516197a2a84f380176b3013655c7f83f33458a",
           "fetch_bytes": 2.0 * 5289 * 1024, "write_bytes": 65362 * 1024}
# The same for one rs_range_doppler_ws call on the 100-frame walk (k_rd_fused,
# k_rd_merge, k_rd_peak summed).
RD_TRAFFIC = {"sources": ("rs_rd.hip", "rs_fft.h"),
              "sources_sha256": "95099bdcdb4bfc8754d0a938c3fa665fedb0f6060603a9d34e880fcf3a09d309",
              "fetch_bytes": 2.0 * (158861 + 20530 + 52) * 1024, "write_bytes": (42880 + 12825 + 55) * 1024}


# VALU wave-instructions per launch of k_render on the 100-frame walk
# (rocprofv3 --pmc SQ_INSTS_VALU); like the records above, null once its
# source changes.  The kernel is bound by vector issue (binary64 geometry):
# 256 CUs x 4 SIMDs x 2.4 GHz / 4 cycles per wave64 instruction.
RENDER_VALU = {"sources": ("rs_scene.hip",),
               "sources_sha256": "d633d719d222e4f30f07c373dc0120ef798efeae22df77f242c89bcfeabb7333",
               "valu_instr": 25334220}
PEAK_VALU_ISSUE = 256 * 4 * 2.4e9 / 4

# Offered load of the serving leg, frozen so that latencies stay comparable
# between runs: 0.6 x the capacity measured with the whole 48-request pool
# queued at once (4.44e13 terms/s) / the pool's mean request (1.94e11 terms).
SERVING_RATE = 137.5


def sources_sha256(sources):
    import hashlib
    h = hashlib.sha256()
    for f in sources:
        with open(os.path.join(ROOT, "paper_2307_09226_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(rec=None):
    """HBM bytes of a counter record, or None once its sources changed."""
    rec = TRAFFIC if rec is None else rec
    if sources_sha256(rec["sources"]) != rec["sources_sha256"]:
        return None
    return rec["fetch_bytes"] + rec["write_bytes"]


def tile_of(desc):
    """Tile configuration string of a matrix-core plan description."""
    pipe = desc["waves"] == 8 and desc.get("schedule") == "pipelined"
    return f"{desc['wave_rows']}x{desc['tile_l']}x{desc['waves']}" + ("i" if pipe else "")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=100,
                    help="untimed steps first; the clock takes ~50 steps (~25 ms) of load to settle")
    ap.add_argument("--no-extras", action="store_true",
                    help="only the headline single-frame measurement")
    ap.add_argument("--legs", default="plain,variants,nufft,batch,doppler_time,serving,cpu",
                    help="extra legs after the headline (comma-separated subset)")
    ap.add_argument("--serving-requests", type=int, default=2000)
    ap.add_argument("--serving-rate", type=float, default=SERVING_RATE,
                    help="requests/s; 0 = 0.6 x the capacity measured in this run")
    ap.add_argument("--serving-policy", choices=("shortest", "equal"), default="shortest")
    ap.add_argument("--serving-slice-terms", type=float, default=0.0,
                    help="terms per slice of the serving loop (0 = the library's default)")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="only run 5 device-to-device copies of this many MiB (the "
                         "calibration kernel for the HBM byte counters) and exit")
    return ap.parse_args()


def pct(a, q):
    return float(np.percentile(np.asarray(a), q)) if len(a) else None


def timed_steps(fn, steps, warmup, events=True):
    """warmup untimed, then exactly `steps` timed calls bracketed by
    synchronisation; with `events`, per-step durations from events on the
    current stream (each pair of event records costs a few microseconds of
    device time, so throughput passes run without them)."""
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(steps if events else 0)]
    t0 = time.perf_counter()
    if events:
        for a, b in evs:
            a.record()
            fn()
            b.record()
    else:
        for _ in range(steps):
            fn()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    per = [a.elapsed_time(b) for a, b in evs]
    return wall, per


def parity_sampled(radar, px, cube_np, k=512, seed=11):
    import oracle
    rng = np.random.default_rng(seed)
    C, L, Ns = radar.cube_shape()
    c = rng.integers(0, C, k).astype(np.int32)
    l = rng.integers(0, L, k).astype(np.int32)
    n = rng.integers(0, Ns, k).astype(np.int32)
    ref = oracle.entries(radar, px, c, l, n)
    got = cube_np[c, l, n].astype(np.complex128)
    d = got - ref
    return {"relL2": float(np.linalg.norm(d) / np.linalg.norm(ref)),
            "maxabs": float(np.max(np.abs(d)) / np.max(np.abs(ref))),
            "entries": int(k)}


def cpu_baseline(radar, px, seconds):
    """The oracle's direct sum on a bounded sample of the same frame: a
    number of seeded output entries, each a full sum over all pixels."""
    import oracle
    o = oracle.default()
    cores = o.max_threads()
    rng = np.random.default_rng(5)
    C, L, Ns = radar.cube_shape()

    def run(k):
        c = rng.integers(0, C, k).astype(np.int32)
        l = rng.integers(0, L, k).astype(np.int32)
        n = rng.integers(0, Ns, k).astype(np.int32)
        t = time.perf_counter()
        o.entries(radar, px, c, l, n)
        return time.perf_counter() - t

    k0 = max(64, cores * 8)
    dt = run(k0)
    rate = k0 * px.P / dt
    k = int(max(k0, min(200000, rate * seconds / px.P)))
    dt = run(k)
    # one thread, on a sample of about three seconds
    o1 = o
    k1 = max(16, int(rate / max(cores, 1) * 3.0 / px.P))
    c = rng.integers(0, C, k1).astype(np.int32)
    l = rng.integers(0, L, k1).astype(np.int32)
    n = rng.integers(0, Ns, k1).astype(np.int32)
    t = time.perf_counter()
    o1.entries(radar, px, c, l, n, threads=1)
    dt1 = time.perf_counter() - t
    o.max_threads(cores)   # the thread count is process-wide: restore it
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            model = next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")), "")
    except OSError:
        pass
    return {"value": k * px.P / dt, "unit": "terms/s", "cores": cores, "kind": "oracle",
            "sample": f"{k} seeded output entries of the headline frame, each summed over "
                      f"all {px.P} pixels ({k * px.P:.3e} terms, {dt:.1f} s)",
            "cpu_model": model, "value_one_thread": k1 * px.P / dt1,
            "sample_one_thread": f"{k1} entries ({k1 * px.P:.3e} terms, {dt1:.1f} s)"}


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print(f"bench.py runs on exactly one GPU (asked for {args.gpus}); multi-GPU runs are "
              "not part of this build", file=sys.stderr)
        sys.exit(2)
    import torch
    if args.copy_probe_mib > 0:
        copy_probe(args.copy_probe_mib)
        return
    from paper_2307_09226_amd import rs, scenes

    dev = "cuda:0"
    radar, px = scenes.workload_frame()
    terms = px.P * radar.C * radar.Ns * radar.L
    dpx = rs.DevicePixels.from_host(px, dev)

    # ---- headline: split-fp16 matrix-core form ---------------------------------
    plan = rs.rs_cube_plan(radar, rs.RS_FORM_MFMA_SPLIT16, rs.RS_C64, max_pixels=px.P)
    cube = rs.new_cube(plan, dev)
    # the plan's tile configuration is tuned on the frame itself (every built
    # configuration, 1 + 3 syntheses each), as a user tuning a plan would
    rule_tile = tile_of(json.loads(plan.describe(px.P)))
    tuned_tile = rs.rs_plan_tune(plan, dpx, cube, reps=3)
    # the caller keeps the workspace (the allocating call adds a stream-ordered
    # allocation and release per step, ~6 us)
    wsp = torch.empty(max(plan.workspace_bytes(px.P), 1), dtype=torch.uint8, device=dev)
    step = lambda: rs.rs_beat_synthesize_ws(plan, dpx, cube, wsp)
    timer = rs.KernelTimer(capacity=args.steps + args.warmup + 8)
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    timer.read()
    # throughput: the K timed steps, every TIMER_STRIDE-th with the library's
    # HIP events around its contraction kernel (the kernel duration for the
    # roofline; each event record costs the stream ~5.6 us, so timing every
    # step would slow the steps it measures); then K more steps with an event
    # pair around each for the step-latency percentiles
    TIMER_STRIDE = 4
    ctr = {"i": 0}

    def sampled_step():
        if ctr["i"] % TIMER_STRIDE == 0:
            with timer:
                step()
        else:
            step()
        ctr["i"] += 1
    wall, _ = timed_steps(sampled_step, args.steps, 0, events=False)
    kms = timer.read()
    _, per = timed_steps(step, args.steps, 0)
    ms_step = wall * 1e3 / args.steps
    value = terms / (wall / args.steps)
    kavg = float(np.mean(kms)) if kms else float("nan")
    achieved = FLOP_MFMA * terms / (kavg * 1e-3)
    out = {
        "metric": METRIC, "value": value, "unit": "terms/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f16 hi/lo split, f32 accumulate (f64 phase arguments)", "data": "synthetic",
        "config": {"workload": "room+pedestrian frame 256x256 px (65,536), 3 Tx x 4 Rx, "
                               "Ns=256, L=128, Fs=10 MHz, Tb=3x40 us, complex64 cube",
                   "form": "mfma_split16", "P": px.P, "M": radar.M, "N": radar.N,
                   "Ns": radar.Ns, "L": radar.L, "terms_per_step": terms,
                   "plan": json.loads(plan.describe(px.P)), "tile_tuned": tuned_tile,
                   "tile_rule": rule_tile},
        "p50_ms": pct(per, 50), "p99_ms": pct(per, 99),
        "latency_pass": "p50/p99 from a second pass of the same K steps with an event pair around each",
        "kernel_timing": "HIP events around the contraction kernel of every 4th timed step",
        "roofline": {"bound": "mfma", "achieved": achieved / 1e12, "peak": PEAK_FP16 / 1e12,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP16, "traffic": measured_traffic(),
                     "kernel": "k_mfma_split16", "kernel_ms": kavg,
                     "flop_per_term": FLOP_MFMA, "terms_per_launch": terms,
                     "traffic_unit": "HBM bytes per launch",
                     "algorithmic_bytes": 20 * px.P + 8 * radar.C * radar.L * radar.Ns},
    }
    torch.cuda.synchronize()
    out["parity"] = parity_sampled(radar, px, cube.cpu().numpy())

    legs = set() if args.no_extras else set(args.legs.split(","))
    if "plain" in legs:
        P_STEPS, P_WARM = 10, 5  # the binary64 load settles its clock over a few launches
        # ---- plain binary64 form on the same frame -------------------------------
        pplan = rs.rs_cube_plan(radar, rs.RS_FORM_FP64_DIRECT, rs.RS_C64, max_pixels=px.P)
        pcube = rs.new_cube(pplan, dev)
        pstep = lambda: rs.rs_beat_synthesize(pplan, dpx, pcube)
        with timer:
            pwall, pper = timed_steps(pstep, P_STEPS, P_WARM)
        pk = timer.read()
        pk_avg = float(np.mean(pk[P_WARM:])) if len(pk) > P_WARM else float("nan")
        torch.cuda.synchronize()
        out["plain_fp64"] = {
            "terms_per_s": terms / (pwall / P_STEPS), "ms_per_step": pwall * 1e3 / P_STEPS,
            "p50_ms": pct(pper, 50), "p99_ms": pct(pper, 99), "kernel_ms": pk_avg,
            "roofline": {"bound": "fp64 vector", "achieved": FLOP_PLAIN * terms / (pk_avg * 1e-3) / 1e12,
                         "peak": PEAK_FP64 / 1e12, "unit": "TFLOP/s",
                         "frac": FLOP_PLAIN * terms / (pk_avg * 1e-3) / PEAK_FP64},
            "parity": parity_sampled(radar, px, pcube.cpu().numpy()),
        }
        out["mfma_speedup_vs_plain"] = out["value"] / out["plain_fp64"]["terms_per_s"]
        pplan.close()

    if "variants" in legs:
        # ---- signal-model variants on the same frame (matrix-core form) -----------
        import dataclasses
        out["variants"] = {"workload": "the headline frame with model flags", "models": {}}
        for model, name in ((15, "far field + Tx slot + intra-chirp Doppler + RVP"),
                            (16, "strength per block (L x P strengths, 1 +- 0.5 swing)")):
            vr = dataclasses.replace(radar, model=model)
            vpx = scenes.block_strengths(px, radar.L, seed=7) if model & 16 else px
            vplan = rs.rs_cube_plan(vr, rs.RS_FORM_MFMA_SPLIT16, rs.RS_C64, max_pixels=px.P)
            vcube = rs.new_cube(vplan, dev)
            vdpx = rs.DevicePixels.from_host(vpx, dev) if model & 16 else dpx
            with timer:
                vwall, vper = timed_steps(lambda: rs.rs_beat_synthesize(vplan, vdpx, vcube), 20, 20)
            vk = timer.read()
            torch.cuda.synchronize()
            vk_avg = float(np.mean(vk[20:]))
            out["variants"]["models"][str(model)] = {
                "name": name, "ms_per_step": vwall * 1e3 / 20, "terms_per_s": terms / (vwall / 20),
                "kernel_ms": vk_avg, "mfma_frac": FLOP_MFMA * terms / (vk_avg * 1e-3) / PEAK_FP16,
                "parity": parity_sampled(vr, vpx, vcube.cpu().numpy(), k=128),
            }
            del vcube, vdpx
            vplan.close()

    if "nufft" in legs:
        # ---- NUFFT form on the same frame (an approximation sized by a tolerance) --
        out["nufft"] = {"workload": "the headline frame", "tolerances": {}}
        for tol in (1e-4, 1e-6):
            nplan = rs.rs_cube_plan_nufft(radar, rs.RS_C64, max_pixels=px.P, tolerance=tol)
            ncube = rs.new_cube(nplan, dev)
            nwall, nper = timed_steps(lambda: rs.rs_beat_synthesize(nplan, dpx, ncube), 50, 20)
            torch.cuda.synchronize()
            out["nufft"]["tolerances"][f"{tol:g}"] = {
                "plan": json.loads(nplan.describe(px.P)),
                "ms_per_step": nwall * 1e3 / 50, "p50_ms": pct(nper, 50), "p99_ms": pct(nper, 99),
                "direct_sum_terms_per_s": terms / (nwall / 50),
                "speedup_vs_mfma": (terms / (nwall / 50)) / value,
                "parity_vs_exact": parity_sampled(radar, px, ncube.cpu().numpy(), k=256),
            }
            del ncube
            nplan.close()
        # the largest serving-size request (12 x 16 array, 192 channels): the
        # NUFFT's work grows with P C w^2, the direct sum's with P C Ns L
        big = max((q for q in scenes.serving_requests(48) if q.radar.C == 192),
                  key=lambda q: q.pixels.P * q.radar.Ns * q.radar.L)
        bterms = big.pixels.P * big.radar.C * big.radar.Ns * big.radar.L
        bd = rs.DevicePixels.from_host(big.pixels, dev)
        bn = rs.rs_cube_plan_nufft(big.radar, rs.RS_C64, max_pixels=big.pixels.P, tolerance=1e-6)
        bm = rs.rs_cube_plan(big.radar, rs.RS_FORM_MFMA_SPLIT16, rs.RS_C64, max_pixels=big.pixels.P)
        bcn, bcm = rs.new_cube(bn, dev), rs.new_cube(bm, dev)
        nw, _ = timed_steps(lambda: rs.rs_beat_synthesize(bn, bd, bcn), 5, 2)
        mw, _ = timed_steps(lambda: rs.rs_beat_synthesize(bm, bd, bcm), 3, 1)
        torch.cuda.synchronize()
        out["nufft"]["largest_request"] = {
            "workload": f"{big.radar.M} Tx x {big.radar.N} Rx, Ns={big.radar.Ns}, L={big.radar.L}, "
                        f"{big.pixels.P} pixels (terms {bterms:.3e})",
            "nufft_ms": nw * 1e3 / 5, "mfma_ms": mw * 1e3 / 3, "speedup_vs_mfma": (mw / 3) / (nw / 5),
            "parity_vs_exact": parity_sampled(big.radar, big.pixels, bcn.cpu().numpy(), k=128),
        }
        del bcn, bcm, bd
        bn.close()
        bm.close()

    if "batch" in legs:
        # ---- 64 animation frames in one persistent launch -------------------------
        frames = scenes.animation_frames(seed=3, nframes=64)
        brad = scenes.radar_batch()
        bplan = rs.rs_cube_plan(brad, rs.RS_FORM_MFMA_SPLIT16, rs.RS_C64,
                                max_pixels=max(f.P for f in frames))
        dfr = [rs.DevicePixels.from_host(f, dev) for f in frames]
        cubes = rs.new_cube(bplan, dev, count=len(frames))
        bterms = sum(f.P for f in frames) * brad.C * brad.Ns * brad.L
        big = int(np.argmax([f.P for f in frames]))

        # two warm-up launches: the first touches of the cubes and of the
        # launch's workspace are slow
        def batch_run():
            with timer:
                bwall, _ = timed_steps(lambda: rs.rs_beat_synthesize_batch(bplan, dfr, cubes), 3, 2)
            bk = timer.read()
            torch.cuda.synchronize()
            return bwall * 1e3 / 3, float(np.mean(bk[2:])) if len(bk) > 2 else None

        # the rule's tile, then the tile tuned on the largest frame through a
        # tile cache (a fresh file: every run tunes)
        b_rule_tile = tile_of(json.loads(bplan.describe(frames[big].P)))
        b_rule_ms, b_rule_k = batch_run()
        import tempfile
        with tempfile.TemporaryDirectory() as td:
            b_tile = rs.rs_plan_tune_cached(bplan, dfr[big], cubes[big], os.path.join(td, "tiles.txt"), reps=2)
        bms, bkms = batch_run()
        out["batch"] = {
            "workload": "64 animation frames, 3 Tx x 4 Rx, Ns=256, L=64, one persistent launch",
            "pixels_min": min(f.P for f in frames), "pixels_max": max(f.P for f in frames),
            "pixels_total": sum(f.P for f in frames), "terms": bterms,
            "tile": b_tile, "tile_tuned_on": f"largest frame ({frames[big].P} pixels), rs_plan_tune_cached",
            "ms": bms, "terms_per_s": bterms / (bms * 1e-3), "kernel_ms": bkms,
            "mfma_frac": (FLOP_MFMA * bterms / (bkms * 1e-3)) / PEAK_FP16 if bkms else None,
            "rule_tile": b_rule_tile, "rule_ms": b_rule_ms, "rule_kernel_ms": b_rule_k,
            "parity_frame0": parity_sampled(brad, frames[0], cubes[0].cpu().numpy(), k=128),
            "parity_largest": parity_sampled(brad, frames[big], cubes[big].cpu().numpy(), k=128),
        }
        del cubes, dfr
        bplan.close()

    if "doppler_time" in legs:
        # ---- walking circle: 100 CPIs, range-Doppler maps, Doppler-time ------------
        out["doppler_time"] = doppler_time_leg(rs, scenes, dev, timer)

    if "serving" in legs and args.serving_requests > 0:
        # ---- serving loop at a fixed request rate -----------------------------------
        out["serving"] = serving(rs, scenes, dev, args)

    if "cpu" in legs:
        # ---- CPU oracle on the host cores -------------------------------------------
        out["cpu_baseline"] = cpu_baseline(radar, px, args.cpu_seconds)
    timer.close()
    plan.close()
    print(json.dumps(out), flush=True)


def doppler_time_leg(rs, scenes, dev, timer):
    """The walking-circle scenario (3 m radius, 100 frames at 24 Hz): the
    100 cubes in one batched launch, then range-Doppler maps of all of them
    and the max-power velocity per CPI against the pedestrian's radial
    velocity (E_velo)."""
    import torch
    radar = scenes.radar_frame()
    cw = scenes.circle_walk()
    F = len(cw.frames)
    plan = rs.rs_cube_plan(radar, rs.RS_FORM_MFMA_SPLIT16, rs.RS_C64,
                           max_pixels=max(f.P for f in cw.frames))
    dfr = [rs.DevicePixels.from_host(f, dev) for f in cw.frames]
    cubes = rs.new_cube(plan, dev, count=F)
    terms = sum(f.P for f in cw.frames) * radar.C * radar.Ns * radar.L
    with timer:
        swall, _ = timed_steps(lambda: rs.rs_beat_synthesize_batch(plan, dfr, cubes), 3, 1)
    sk = timer.read()
    power = torch.empty((F, radar.Ns, radar.L), dtype=torch.float32, device=dev)
    dtime = torch.empty((F, radar.L), dtype=torch.float32, device=dev)
    peaks = torch.empty(F * rs.RD_PEAK_DTYPE.itemsize, dtype=torch.uint8, device=dev)
    rd_ws = torch.empty(rs.rs_range_doppler_workspace_bytes(plan, F, True), dtype=torch.uint8, device=dev)
    rd_call = lambda: rs.rs_range_doppler_ws(plan, cubes, True, power, dtime, peaks, rd_ws)  # noqa: E731
    rd_steps = 50
    rwall, _ = timed_steps(rd_call, rd_steps, 5, events=False)
    _, rper = timed_steps(rd_call, 20, 0)   # latency pass: an event pair around each call
    torch.cuda.synchronize()
    pk = np.frombuffer(peaks.cpu().numpy().tobytes(), dtype=rs.RD_PEAK_DTYPE)
    v_est = pk["velocity_mps"].astype(np.float64)
    err = np.abs(v_est - cw.v_radial)
    rd_ms = rwall * 1e3 / rd_steps
    # algorithmic bytes: every cube entry read once (complex64), the power
    # map written once (float32)
    rd_bytes = F * radar.C * radar.L * radar.Ns * 8 + F * radar.Ns * radar.L * 4

    # the same walk with the frames ray-cast on the device (strength factors
    # drawn on the device): no pixel passes through host memory
    g = 256
    room = scenes.Room(W=12.0, D=10.0)
    structs = rs.scene_array([rs.scene_struct(room, scenes.Pedestrian(centre=c, velocity=v))
                              for c, v in zip(cw.centres, cw.velocities)])
    pix = [torch.empty(F * g * g, dtype=torch.float32, device=dev) for _ in range(5)]
    gen = torch.Generator(device=dev)
    gen.manual_seed(5)
    noise = torch.empty(F * g * g, dtype=torch.float32, device=dev).log_normal_(0.0, 0.5, generator=gen)
    holder = {}

    def render():
        holder["frames"] = rs.rs_render_scenes(structs, g, g, noise, dev, out=pix)
    rtimer = rs.KernelTimer(capacity=16)
    with rtimer:
        rnd_wall, _ = timed_steps(render, 10, 2)
    render_ms = rnd_wall * 1e3 / 10
    rk = rtimer.read()[2:]  # the ray-cast kernel of the 10 timed calls
    rtimer.close()
    render_kernel_ms = float(np.mean(rk)) if rk else None

    def pipeline():
        fr = rs.rs_render_scenes(structs, g, g, noise, dev, out=pix)
        rs.rs_beat_synthesize_batch(plan, fr, cubes)
        rd_call()
    pwall, _ = timed_steps(pipeline, 3, 1)
    torch.cuda.synchronize()
    pk2 = np.frombuffer(peaks.cpu().numpy().tobytes(), dtype=rs.RD_PEAK_DTYPE)
    err2 = np.abs(pk2["velocity_mps"].astype(np.float64) - cw.v_radial)
    render_bytes = F * g * g * (20 + 4)
    plan.close()
    return {"workload": f"walking circle, radius 3 m, {F} frames at 24 Hz (4.52 m/s), room 12 x 10 m, "
                        "256x256 px, 3 Tx x 4 Rx, Ns=256, L=128",
            "pixels_total": sum(f.P for f in cw.frames), "terms": terms,
            "synth_ms": swall * 1e3 / 3, "synth_terms_per_s": terms / (swall / 3),
            "synth_kernel_ms": float(np.mean(sk[1:])) if len(sk) > 1 else None,
            "rd_ms": rd_ms, "rd_p50_ms": pct(rper, 50),
            "rd_algorithmic_bytes": rd_bytes,
            "rd_roofline": {"bound": "hbm", "achieved": rd_bytes / (rd_ms * 1e-3) / 1e9, "peak": 8000.0,
                            "unit": "GB/s", "frac": rd_bytes / (rd_ms * 1e-3) / 8e12,
                            "time": "whole rs_range_doppler_ws call (3 launches, workspace allocated once), "
                                    "throughput pass without events",
                            "traffic": measured_traffic(RD_TRAFFIC),
                            "traffic_unit": "HBM bytes per call (all launches)"},
            "E_velo_mps": float(np.mean(err)), "max_abs_error_mps": float(err.max()),
            "doppler_bin_mps": float(radar.c0 / (2 * radar.fc * radar.Tb * radar.L)),
            "corr_v_est_v_true": float(np.corrcoef(v_est, cw.v_radial)[0, 1]),
            "paper_E_velo_mps": 1.3,
            "device_rendered": {
                "render_ms": render_ms,
                "render_kernel_ms": render_kernel_ms,
                "render_roofline": render_roofline(render_bytes, render_kernel_ms),
                "render_synth_rd_ms": pwall * 1e3 / 3,
                "E_velo_mps": float(np.mean(err2)), "max_abs_error_mps": float(err2.max())},
            "v_est": [round(float(v), 3) for v in v_est],
            "v_true": [round(float(v), 3) for v in cw.v_radial]}


def render_roofline(nbytes, kernel_ms):
    """k_render against the vector issue rate (measured instruction count),
    with its HBM fraction beside it."""
    if not kernel_ms:
        return None
    instr = RENDER_VALU["valu_instr"] if sources_sha256(RENDER_VALU["sources"]) == RENDER_VALU["sources_sha256"]         else None
    rate = instr / (kernel_ms * 1e-3) if instr else None
    return {"bound": "alu", "achieved": rate / 1e9 if rate else None, "peak": PEAK_VALU_ISSUE / 1e9,
            "unit": "G wave64 VALU instructions/s", "frac": rate / PEAK_VALU_ISSUE if rate else None,
            "hbm_gbps": nbytes / (kernel_ms * 1e-3) / 1e9, "hbm_frac": nbytes / (kernel_ms * 1e-3) / 8e12,
            "time": "k_render alone (HIP events around the launch); render_ms is the whole call from "
                    "Python, host work included"}


def copy_probe(mib):
    """A plain copy of known size: reads and writes mib MiB once per launch."""
    import torch
    n = mib << 20
    src = torch.ones(n, dtype=torch.uint8, device="cuda:0")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(5):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes": n, "launches": 5}), flush=True)


def serving(rs, scenes, dev, args):
    """Poisson arrivals of mixed cube requests at a fixed rate; latency is
    completion minus submission per request.  Capacity (terms/s with every
    pool request queued at once, measured twice; the first pass is the
    warm-up) is reported beside the offered load."""
    import torch
    pool_n = 48
    pool = scenes.serving_requests(pool_n)
    plans = {}
    items = []
    for q in pool:
        key = (q.radar.M, q.radar.N, q.radar.Ns, q.radar.L)
        if key not in plans:
            plans[key] = rs.rs_cube_plan(q.radar, rs.RS_FORM_MFMA_SPLIT16, rs.RS_C64,
                                         max_pixels=262144)
        items.append((plans[key], rs.DevicePixels.from_host(q.pixels, dev), q.terms))
    mean_terms = float(np.mean([t for _, _, t in items]))
    max_slots = 16
    policy = {"shortest": rs.RS_SCHED_SHORTEST, "equal": rs.RS_SCHED_EQUAL}[args.serving_policy]
    sess = rs.Session(hbm_budget=16 << 30, max_slots=max_slots, queue_cap=100000, policy=policy,
                      slice_terms=args.serving_slice_terms)
    # one output buffer per pool entry; a request writes its entry's buffer
    bufs = [rs.new_cube(p, dev) for p, _, _ in items]
    torch.cuda.synchronize()
    # each pool request alone (rs_beat_synthesize, median of 3 after a warm-up):
    # the service time a request's latency is compared with (its slowdown)
    alone_ms = []
    for k, (p, d, _) in enumerate(items):
        _, per = timed_steps(lambda: rs.rs_beat_synthesize(p, d, bufs[k]), 3, 1)
        alone_ms.append(float(np.median(per)))

    def run(order, arrivals):
        tickets = []
        terms = 0.0
        t0 = time.perf_counter()
        for i, k in enumerate(order):
            while time.perf_counter() - t0 < arrivals[i]:
                time.sleep(0.0002)
            p, d, tm = items[k]
            tickets.append(sess.submit(p, d, bufs[k]))
            terms += tm
        sess.drain()
        wall = time.perf_counter() - t0
        lat, big = [], []
        for t, k in zip(tickets, order):
            st, (ts, ta, td) = sess.poll(t)
            assert st == rs.RS_REQ_DONE, st
            lat.append((td - ts) * 1e-6)
        return wall, terms, lat

    # capacity: every pool request queued at once (twice; the second is timed)
    allk = np.arange(len(items))
    run(allk, np.zeros(len(items)))
    wall, terms, _ = run(allk, np.zeros(len(items)))
    cap_terms = terms / wall
    rate = args.serving_rate if args.serving_rate > 0 else 0.6 * cap_terms / mean_terms
    n = args.serving_requests
    order = np.random.default_rng(7).integers(0, len(items), n)
    arrivals = scenes.poisson_arrivals(n, rate, seed=7)
    wall, terms, lat = run(order, arrivals)
    st = sess.stats()
    sess.close()
    for p in plans.values():
        p.close()
    lat = np.asarray(lat)
    sizes = np.array([items[k][2] for k in order])
    small = sizes <= np.median(sizes)
    slow = lat / np.array([alone_ms[k] for k in order])
    return {"workload": "Poisson arrivals of mixed requests (1x4, 3x4, 12x16 arrays; Ns 128/256/512; "
                        "L 64/128/256; 4k-262k pixels), drawn from a pool of 48 seeded requests",
            "policy": args.serving_policy, "slice_terms": args.serving_slice_terms or 1.2e11,
            "pool_mean_terms": mean_terms, "capacity_terms_per_s": cap_terms,
            "rate_req_per_s": rate, "offered_terms_per_s": rate * mean_terms, "requests": n,
            "throughput_req_per_s": n / wall, "terms_per_s": terms / wall,
            "latency_p50_ms": pct(lat, 50), "latency_p99_ms": pct(lat, 99), "latency_mean_ms": float(lat.mean()),
            "latency_p50_ms_small_half": pct(lat[small], 50), "latency_p99_ms_small_half": pct(lat[small], 99),
            "slowdown_p50": pct(slow, 50), "slowdown_p99": pct(slow, 99),
            "slowdown_note": "latency / the request's own rs_beat_synthesize time alone (median of 3)",
            "alone_ms_p50": pct(alone_ms, 50), "alone_ms_max": float(np.max(alone_ms)),
            "launches": int(st["launches"]), "footprint_peak_bytes": int(st["footprint_peak"]),
            "request_bytes_peak": int(st["request_bytes_peak"]), "max_slots": max_slots}


if __name__ == "__main__":
    main()
