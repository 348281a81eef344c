#!/usr/bin/env python
"""Benchmark of the whole hot path on one MI355X.

A step is one pass of the path over the slab workload (512x512x128 uint16, ~2,000 ellipsoid
nuclei, anisotropic spacing (1, 1, 2), D 642 directions, M 64 rays x L 16 radial points per
contour-iteration, 500 iterations): reset contour state from the seeds, pre-pass, evolve, exact
energy + selection, readback. Inputs (raw volume, direction table) are resident in HBM before the
timed region; the seeds are re-sent each step (48 KB).

Prints ONE JSON line: vertex-updates/s (one vertex-update = one sampled ray of one active contour
in one iteration); the evolve kernel's roofline (algorithmic FP32 FLOPs over its HIP-event time
against the vector ALU's rate, with the VALU issue rate and HBM traffic from the committed counters
and the logical-gather bandwidth beside it); the FP64 oracle timed on a bounded sample on the host
cores; and, under "workloads", the 2D image (8192^2, 40,000 cells), the batched subvolumes (256,
engine against the plain loop) and the served tile stream (tiles cut from a 2048x2048x512 volume,
Poisson arrivals, p50/p99 latency), each with its parity check and oracle figure (--quick skips them).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# Algorithmic FP32 FLOPs per vertex-update (one ray of L = 16 radial points): per sample point the
# position c + s u (3 FMA), voxel coordinates (3 mul), fractions (3 sub), the 7 (3D) / 3 (2D) lerps
# of the interpolation (sub + FMA each), and the sums S I, dS/dR I, dS/dr I u (2 + 2 + 1 + 3 FMA):
# 44 (3D) / 26 (2D) FLOPs, plus half of the radius, cube (square) root and weights that the two
# antithetic points at one radius share: 47 / 29 per point.
FLOP_PER_VU = {3: 16 * 47, 2: 16 * 29}
# Unpacked FP32 FMA rate: 256 CUs x 64 lanes x 2 FLOPs x 2.4 GHz (the packed FP32 instructions that
# double it to the published 157.3 TFLOP/s are switched off in this build's compile flags).
VALU_PEAK_TFLOPS = 256 * 64 * 2 * 2.4e9 / 1e12
# VALU lane-instruction issue rate: 256 CUs x 64 lanes x 2.4 GHz.
LANE_ISSUE_PEAK = 256 * 64 * 2.4e9
COUNTERS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles", "evolve_slab_counters.json")


def measured_counters(workload, launch_auto, launches):
    """The committed counters of the evolve kernel: HBM bytes per evolve call (FETCH_SIZE and
    WRITE_SIZE summed over its launches, scaled by the copy-kernel calibration) and VALU busy; None
    when they were taken on other evolve sources, shapes or launch counts."""
    try:
        with open(COUNTERS) as f:
            c = json.load(f)
        h = hashlib.sha256()
        root = os.path.dirname(os.path.abspath(__file__))
        for name in c["source_files"]:
            with open(os.path.join(root, name), "rb") as f:
                h.update(f.read())
    except (OSError, KeyError, ValueError):
        return None
    if (h.hexdigest() != c["source_sha256"] or c["workload"] != workload or not launch_auto
            or c.get("launches_per_evolve") != launches):
        return None
    return c
METRIC = "contour vertex-updates/s at fixed accuracy"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def host_cpu():
    """CPU model and logical CPU count of the host the oracle runs on."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"cpu_model": model, "logical_cpus": os.cpu_count()}


def cpu_baseline(wl, gpu_out, n_sample):
    """The FP64 oracle on the first n_sample contours of the same workload (all iterations), with
    the pre-pass prorated by n_sample / n_contours. Also checks those contours against the GPU."""
    import numpy as np

    import oracle
    oracle.build(force=False)
    p = wl.params
    n = len(wl.seeds)
    S = n if n_sample <= 0 else min(n_sample, n)
    t0 = time.perf_counter()
    J = oracle.prepass(wl.raw, p)
    t_pre = time.perf_counter() - t0
    t0 = time.perf_counter()
    st = oracle.init_state(p, wl.seeds[:S], ids=wl.ids[:S], shape_zyx=wl.raw.shape)
    _, done = oracle.evolve(J, p, wl.dirs, st, wl.n_iter)
    oracle.finalize_status(st)
    e_vox, _ = oracle.energy_vox(J, p, st.c, st.R)
    oracle.cull(p, st.c, st.R, e_vox, st.status, st.ids)
    t_evo = time.perf_counter() - t0
    secs = t_evo + t_pre * S / n
    vu = done * p.n_rays
    dR = float(np.max(np.abs(gpu_out["radii"][:S] - st.R)))
    dc = float(np.max(np.linalg.norm(gpu_out["centers"][:S] - st.c, axis=1)))
    same_iters = float(np.mean(gpu_out["iters"][:S] == st.iters))
    parity = {"contours": S, "max_abs_dR": dR, "max_abs_dc": dc, "same_iters_frac": same_iters,
              "ok": bool(dR <= 0.05 and dc <= 0.5 and same_iters >= 0.99)}
    base = {"value": vu / secs, "unit": "vertex-updates/s", "cores": oracle.num_threads(), "kind": "oracle",
            "sample": (f"first {S} of {n} contours, all {wl.n_iter} iterations, FP64 oracle "
                       f"(gcc -O2, OpenMP over contours); pre-pass over the full volume prorated by {S}/{n}; "
                       f"{secs:.1f} s of CPU work")}
    # one thread on a bounded subset: the first 40 contours' evolution (pre-pass excluded)
    threads = oracle.num_threads()
    S1 = min(40, n)
    oracle.set_num_threads(1)
    try:
        t0 = time.perf_counter()
        st1 = oracle.init_state(p, wl.seeds[:S1], ids=wl.ids[:S1], shape_zyx=wl.raw.shape)
        _, done1 = oracle.evolve(J, p, wl.dirs, st1, wl.n_iter)
        t1 = time.perf_counter() - t0
    finally:
        oracle.set_num_threads(threads)
    # and the tiny workload (64^3, 8 contours, 100 iterations) whole, on one thread
    import synth
    tw = synth.tiny_config()
    oracle.set_num_threads(1)
    try:
        t0 = time.perf_counter()
        Jt = oracle.prepass(tw.raw, tw.params)
        stt = oracle.init_state(tw.params, tw.seeds, ids=tw.ids, shape_zyx=tw.raw.shape)
        _, done_t = oracle.evolve(Jt, tw.params, tw.dirs, stt, tw.n_iter)
        tt = time.perf_counter() - t0
    finally:
        oracle.set_num_threads(threads)
    base["single_thread_tiny"] = {"value": done_t * tw.params.n_rays / tt, "unit": "vertex-updates/s", "cores": 1,
                                  "sample": f"{tw.name}: pre-pass and all {tw.n_iter} iterations, {tt:.2f} s"}
    base["host"] = host_cpu()
    base["single_thread"] = {"value": done1 * p.n_rays / t1, "unit": "vertex-updates/s", "cores": 1,
                             "sample": f"first {S1} contours, all {wl.n_iter} iterations, evolution only, "
                                       f"{t1:.1f} s"}
    return base, parity


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--lanes", type=int, default=0, help="lanes per contour: 16..256 (0: automatic)")
    ap.add_argument("--unroll", type=int, default=0, help="pair-points in flight per lane (0: automatic)")
    ap.add_argument("--layout", type=int, default=0, help="volume layout: 0 auto, 1 plain, 2 quad, 3 plain with 64-bit addressing, 4 column pairs")
    ap.add_argument("--tile", type=int, default=-1,
                    help="LDS box per contour in voxels (-1: automatic, 0: off)")
    ap.add_argument("--exact", action="store_true",
                    help="exact lattice sums instead of Monte-Carlo samples (params flags bit 1); reports "
                         "contour-iterations/s next to the Monte-Carlo path's")
    ap.add_argument("--cpu-sample", type=int, default=0, help="contours in the oracle baseline (0: all)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--sweep", action="store_true",
                    help="only time the evolve kernel for every (lanes, pair-points in flight, layout) shape")
    ap.add_argument("--sweep-prepass", action="store_true",
                    help="sweeps: re-run the pre-pass before every timed evolve, as a bench step does")
    ap.add_argument("--sweep-tile", action="store_true",
                    help="only time the evolve kernel for whole-wave shapes x LDS box capacities, checking "
                         "that every capacity reproduces the box-free result bit for bit")
    ap.add_argument("--smooth", type=float, default=0.3, help="star: smoothing weight of the star contours")
    ap.add_argument("--workload", default="slab",
                    choices=["slab", "plane", "batched", "served", "lattice", "gradient", "star", "repel"],
                    help="slab: the plain path on the slab volume (default); plane: the plain path on the "
                         "8192^2 2D image; batched: 256 uneven subvolumes through the engine vs the plain "
                         "per-volume loop; served: Poisson tile requests; lattice: the slab volume seeded with "
                         "the initial contour lattice, evolved with and without culling passes; "
                         "gradient: the slab with the centre force in its weight form and its image-gradient "
                         "form (flags bit 2): variance of one iteration's force at fixed states, and "
                         "accuracy and time of free runs with 64, 32 and 16 rays; star: the slab with "
                         "star-shaped contours (per-direction radii) against the sphere: time and fit to the "
                         "generator's ellipsoids; repel: the slab with two seeds per nucleus and the slab "
                         "lattice, evolved with soft repulsion between neighbours at several strengths: time, "
                         "separation of the seed pairs, recall and precision")
    ap.add_argument("--serve-seconds", type=float, default=20.0, help="served: arrival window (s)")
    ap.add_argument("--rate", type=float, default=200.0, help="served: mean arrivals per second")
    ap.add_argument("--rate-hi", type=float, default=2000.0,
                    help="served: mean arrivals per second of the second, saturating stream")
    ap.add_argument("--serve-seconds-hi", type=float, default=5.0, help="served: window of the saturating stream (s)")
    ap.add_argument("--chunk", type=int, default=25, help="served: iterations per engine step")
    ap.add_argument("--chunk-idle", type=int, default=200,
                    help="served: iterations per step while one job runs and none waits (0: always --chunk)")
    ap.add_argument("--served-check", type=int, default=48,
                    help="served: requests checked against the plain path (bitwise) and the FP64 oracle")
    ap.add_argument("--quick", action="store_true",
                    help="the slab line only (default: also the 2D, batched and served workloads as extra keys)")
    ap.add_argument("--extra-steps", type=int, default=3, help="timed steps of the 2D and batched extras")
    ap.add_argument("--cull-every", type=int, default=25, help="lattice: iterations between culling passes")
    ap.add_argument("--grace", type=int, default=50,
                    help="lattice: iterations before the culling threshold retires a contour")
    ap.add_argument("--e-cull-factor", type=float, default=0.25,
                    help="lattice: culling threshold of the lax rules as a multiple of E0")
    ap.add_argument("--repel-every", type=int, default=5,
                    help="repel: iterations between refreshes of the neighbours' snapshot")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a plain 1 GiB device-to-device copy 4 times (calibrates HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: --gpus {args.gpus} is not supported: the path runs on one GPU (a large volume "
              "would shard into slabs with halos, one per GPU, exchanging only border contours before the "
              "selection).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import synth
    from paper_1804_06304_amd import snk

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.copy_probe:
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(4):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_read_per_copy": src.numel() * 4, "copies": 4}), flush=True)
        return
    if args.workload == "batched":
        return bench_batched(args)
    if args.workload == "served":
        return bench_served(args)
    if args.workload == "lattice":
        return bench_lattice(args)
    if args.workload == "gradient":
        return bench_gradient(args)
    if args.workload == "star":
        return bench_star(args)
    if args.workload == "repel":
        return bench_repel(args)
    t0 = time.perf_counter()
    wl = synth.slab_config() if args.workload == "slab" else synth.plane_config()
    if args.exact:
        wl.params = wl.params.replace(flags=wl.params.flags | 2)
    log(f"workload {wl.name}: generated in {time.perf_counter() - t0:.1f} s")
    p = wl.params
    stream = torch.cuda.current_stream()
    raw = torch.from_numpy(wl.raw).to("cuda:0")
    ctx = snk.Context(0, stream)
    ctx.set_params(p)
    ctx.set_launch(args.lanes, args.unroll, args.layout)
    ctx.set_tile(args.tile)
    ctx.set_directions(wl.dirs)
    ctx.load_volume(raw)
    torch.cuda.synchronize()

    if args.sweep_tile:
        layout = 2 if p.dim == 3 else 1
        for g in (64, 128, 256):
            for u in (1, 2):
                ref = None
                for cap in (0, -1, 2048, 3072, 3584, 4096, 4224, 6144):
                    ctx.set_launch(g, u, layout)
                    ctx.set_tile(cap)
                    ms = []
                    for _ in range(3):
                        ctx.load_seeds(wl.seeds, ids=wl.ids)
                        if args.sweep_prepass:
                            ctx.prepass()
                        ctx.evolve(wl.n_iter)
                        ms.append(ctx.get_timing()["evolve_ms"])
                    st = ctx.get_state()
                    if ref is None:
                        ref = st
                    same = all(np.array_equal(st[k], ref[k]) for k in ref)
                    cap = ctx.get_timing()["tile_voxels"] if cap < 0 else cap
                    log(f"sweep-tile lanes={g} pairs_in_flight={u} tile={cap}: evolve {min(ms):.3f} ms "
                        f"(min of 3; {[round(v, 3) for v in ms]}) bitwise={'yes' if same else 'NO'}")
        ctx.close()
        return

    if args.sweep:
        for layout in ((2, 1) if p.dim == 3 else (4, 1, 2)):
            for g in (16, 32, 64, 128, 256):
                for u in ((1, 2, 4) if g in (32, 64, 128) else (1, 2)):
                    ctx.set_launch(g, u, layout)
                    ms = []
                    for _ in range(3):
                        ctx.load_seeds(wl.seeds, ids=wl.ids)
                        if args.sweep_prepass:
                            ctx.prepass()
                        ctx.evolve(wl.n_iter)
                        ms.append(ctx.get_timing()["evolve_ms"])
                    log(f"sweep layout={layout} lanes={g} pairs_in_flight={u}: evolve {min(ms):.3f} ms "
                        f"(min of 3; {[round(v, 3) for v in ms]})")
        ctx.close()
        return

    def step():
        ctx.load_seeds(wl.seeds, ids=wl.ids)
        ctx.prepass()
        ctx.evolve(wl.n_iter)
        ctx.finalize()
        out = ctx.read()
        return out, ctx.get_timing()

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    evolve_ms, prepass_ms, finalize_ms, evolved = [], [], [], 0
    launches0 = ctx.get_timing()["evolve_launches"]
    t0 = time.perf_counter()
    for _ in range(args.steps):
        out, tm = step()
        evolve_ms.append(tm["evolve_ms"])
        prepass_ms.append(tm["prepass_ms"])
        finalize_ms.append(tm["finalize_ms"])
        evolved += tm["evolved"]
    torch.cuda.synchronize()
    secs = time.perf_counter() - t0
    launches_per_evolve = (tm["evolve_launches"] - launches0) // args.steps
    ctx.close()

    M, L, d = p.n_rays, p.n_radial, p.dim
    vu = evolved * M
    per_launch_vu = vu / args.steps
    bytes_per_vu = L * (2 ** d) * 4
    ev_ms = float(np.mean(evolve_ms))
    achieved = per_launch_vu * bytes_per_vu / (ev_ms * 1e-3) / 1e9
    log(f"per step: prepass {np.mean(prepass_ms):.3f} ms, evolve {ev_ms:.3f} ms, finalize {np.mean(finalize_ms):.3f} ms,"
        f" wall {secs / args.steps * 1e3:.3f} ms; vertex-updates/step {per_launch_vu:.4g};"
        f" kept {int(out['keep'].sum())}/{len(out['keep'])}; launch lanes {tm['lanes_per_contour']}"
        f" pairs {tm['pairs_in_flight']} layout {tm['layout']} tile {tm['tile_voxels']}")
    ctr = measured_counters(wl.name, args.lanes == 0 and args.unroll == 0 and args.layout == 0 and args.tile < 0,
                            launches_per_evolve)
    traffic = float(ctr["hbm_bytes_per_evolve"]) if ctr else None
    line = {
        "metric": METRIC, "value": vu / secs, "unit": "vertex-updates/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": secs / args.steps * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": wl.name,
                   "volume": "512x512x128 u16, h=(1,1,2)" if d == 3 else "8192x8192 u8 (2D)",
                   "contours": len(wl.seeds),
                   "n_iter": wl.n_iter, "n_dirs": p.n_dirs, "n_rays": M, "n_radial": L,
                   "lanes_per_contour": args.lanes or "auto", "pairs_in_flight": args.unroll or "auto",
                   "layout": {0: "auto", 1: "plain", 2: "quad", 3: "plain64", 4: "pairs"}[args.layout],
                   "tile_voxels": "auto" if args.tile < 0 else args.tile,
                   "resolved_launch": {"lanes_per_contour": tm["lanes_per_contour"],
                                       "pairs_in_flight": tm["pairs_in_flight"],
                                       "layout": {0: "plain64", 1: "plain", 2: "quad", 3: "pairs"}[tm["layout"]],
                                       "tile_voxels": tm["tile_voxels"]}},
        "kernels_ms": {"prepass": float(np.mean(prepass_ms)), "evolve": ev_ms,
                       "finalize": float(np.mean(finalize_ms))},
        "roofline": roofline_of(per_launch_vu, d, ev_ms, achieved, ctr, launches_per_evolve),
    }
    # the evolve kernel alone (HIP events around its launches) and its rates in other units
    ci_step = evolved / args.steps
    line["evolve_only"] = {"vertex_updates_per_s": per_launch_vu / (ev_ms * 1e-3),
                           "contour_iterations_per_s": ci_step / (ev_ms * 1e-3),
                           "sample_points_per_s": per_launch_vu * L / (ev_ms * 1e-3),
                           "note": f"a sample point is one {2 ** d}-tap interpolated gather; "
                                   f"{L} per vertex-update"}
    if args.exact:
        # no rays are sampled: report contour-iterations/s (and its time per contour-iteration) to
        # set beside the Monte-Carlo path's on the same workload
        ci = evolved / args.steps
        line.update({"metric": "contour-iterations/s, exact lattice sums", "value": ci * args.steps / secs,
                     "unit": "contour-iterations/s",
                     "evolve_ns_per_contour_iteration": ev_ms * 1e6 / ci, "roofline": None})
        line["config"]["sums"] = "exact lattice (flags bit 1)"
    if not args.no_cpu_baseline:
        log("cpu baseline: FP64 oracle on the same workload ...")
        base, parity = cpu_baseline(wl, out, args.cpu_sample)
        line["cpu_baseline"] = base
        line["parity_sample"] = parity
    if not args.quick and args.workload == "slab" and not args.exact:
        # the other workloads, as extra keys beside the slab line (a failure in one is recorded, not fatal)
        extras = {}
        for name, fn in (("plane", lambda: run_plane(args)),
                         ("batched", lambda: run_batched(args, args.extra_steps, 1)),
                         ("served", lambda: run_served(args))):
            try:
                extras[name] = fn()
            except Exception as exc:   # keep the headline line
                log(f"{name}: failed: {exc!r}")
                extras[name] = {"error": repr(exc)}
            torch.cuda.synchronize()
            torch.cuda.empty_cache()
        line["workloads"] = extras
    print(json.dumps(line), flush=True)


def roofline_of(vu_per_call, d, ev_ms, logical_gbs, ctr, launches):
    """Roofline of the evolve kernel per evolve call. The kernel issues vector instructions faster
    than it moves bytes (the committed counters: VALU busy, lane-instructions per sample point, HBM
    bytes well below the logical gathers), so its bound is the vector ALU: achieved = algorithmic
    FP32 FLOPs per call over the call's HIP-event time, against the unpacked FP32 rate. Beside it:
    the VALU issue rate from the committed counters (hash-gated to the evolve sources) and the
    logical-gather bandwidth against the HBM peak."""
    secs = ev_ms * 1e-3
    tf = vu_per_call * FLOP_PER_VU[d] / secs / 1e12
    traffic = float(ctr["hbm_bytes_per_evolve"]) if ctr else None
    valu = float(ctr["sq_insts_valu_per_evolve"]) if ctr and "sq_insts_valu_per_evolve" in ctr else None
    return {"bound": "alu", "achieved": tf, "peak": VALU_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": tf / VALU_PEAK_TFLOPS,
            "traffic": traffic,
            "kernel": f"evolve_kernel<{d},*,false>", "launches_per_evolve": launches,
            "per": "one evolve call: its launches back to back on one stream, HIP events around them",
            "algorithmic_flops": f"{FLOP_PER_VU[d]} FP32 FLOPs per vertex-update (L = 16 points x "
                                 f"{FLOP_PER_VU[d] // 16} per point)",
            "peak_basis": "256 CUs x 64 lanes x 2 FLOPs (FMA) x 2.4 GHz, unpacked FP32 (published 157.3 "
                          "counts packed FP32, which this build does not emit)",
            "frac_of_published_fp32": tf / 157.3,
            "counters_source": ("profiles/evolve_slab_counters.json: rocprofv3 --pmc counters of the same "
                                "evolve sources and launch shape, committed with their source hash; null when "
                                "the sources have changed since") ,
            "traffic_gbs": traffic / secs / 1e9 if traffic else None,
            "hbm_frac": traffic / secs / 1e9 / HBM_PEAK_GBS if traffic else None,
            "valu_busy_pct": ctr.get("valu_busy_pct") if ctr else None,
            "valu_issue_frac": valu * 64 / secs / LANE_ISSUE_PEAK if valu else None,
            "logical_gather": {"achieved": logical_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                               "frac": logical_gbs / HBM_PEAK_GBS,
                               "bytes": f"{16 * 2 ** d * 4} B per vertex-update (L x 2^d taps x 4 B); above 1 "
                                        "means LDS and caches serve the gathers, not HBM"}}


def match_truth(kept, truth, dmax):
    """Greedy one-to-one matching of kept centres to true centres closer than dmax (physical)."""
    import numpy as np
    from scipy.spatial import cKDTree
    if len(kept) == 0 or len(truth) == 0:
        return 0
    d, j = cKDTree(truth).query(kept, k=4, distance_upper_bound=dmax)
    pairs = sorted((d[i, k], i, j[i, k]) for i in range(len(kept)) for k in range(4) if np.isfinite(d[i, k]))
    used_k, used_t, m = set(), set(), 0
    for _, i, t in pairs:
        if i not in used_k and t not in used_t:
            used_k.add(i)
            used_t.add(t)
            m += 1
    return m


def bench_star(args):
    """Star-shaped contours (one radius per table direction, snk_set_star) against the sphere on the
    slab workload (500 iterations, selection), both from the same seeds and R0: evolve time and
    vertex-updates/s, and the fit to the generator's ellipsoids. For each contour kept and matched
    to its own nucleus, the cell-radius estimate rho R_k along every table direction T_k (rho R for
    the sphere) is compared with the nucleus' radial extent a(T_k) from its centre: the relative
    error sum_k |rho R_k - a(T_k)| / sum_k a(T_k), median over contours; also the centre error."""
    import numpy as np
    import torch

    import synth
    from paper_1804_06304_amd import snk

    wl = synth.slab_config()
    p = wl.params
    raw = torch.from_numpy(wl.raw).to("cuda:0")
    stream = torch.cuda.current_stream()
    truth = wl.truth
    rho = 2.0 ** (-1.0 / 3.0)
    T = wl.dirs.astype(np.float64)

    def extent(i):
        local = T @ truth["rots"][i]          # direction components along the principal axes
        return 1.0 / np.sqrt(((local / truth["axes"][i]) ** 2).sum(axis=1))

    rows = []
    for smooth in (-1.0, args.smooth, 0.0):
        ctx = snk.Context(0, stream)
        ctx.set_params(p)
        ctx.set_star(smooth)
        if smooth >= 0.0:
            ctx.set_launch(args.lanes, 0, 0)   # star contours: 64 or 128 lanes (0: automatic)
        ctx.set_directions(wl.dirs)
        ctx.load_volume(raw)
        ms = []
        for _ in range(1 + max(1, args.steps)):
            ctx.load_seeds(wl.seeds, ids=wl.ids)
            ctx.prepass()
            ctx.evolve(wl.n_iter)
            ms.append(ctx.get_timing()["evolve_ms"])
        evolved = ctx.get_timing()["evolved"]
        ctx.finalize()
        out = ctx.read()
        Rk = ctx.get_star_radii() if smooth >= 0 else np.repeat(out["radii"][:, None], p.n_dirs, axis=1)
        ctx.close()
        kept = np.where(out["keep"].astype(bool))[0]
        cerr = np.linalg.norm(out["centers"][kept] - truth["centers"][kept], axis=1)
        own = kept[cerr < 4.0]
        fit = np.array([np.abs(rho * Rk[i] - extent(i)).sum() / extent(i).sum() for i in own])
        ev = float(np.mean(ms[1:]))
        row = {"contour": "sphere" if smooth < 0 else "star", "smooth": None if smooth < 0 else smooth,
               "evolve_ms": ev, "vertex_updates_per_s": evolved * p.n_rays / (ev * 1e-3),
               "kept": int(len(kept)), "matched": int(len(own)),
               "median_fit_error": float(np.median(fit)), "p90_fit_error": float(np.percentile(fit, 90)),
               "median_centre_error": float(np.median(cerr[cerr < 4.0]))}
        rows.append(row)
        log(f"{row['contour']:6s} smooth {smooth:5.2f}: evolve {ev:.3f} ms ({row['vertex_updates_per_s']:.3g} "
            f"vertex-updates/s), kept {row['kept']}, fit error median {row['median_fit_error']:.3f} "
            f"(p90 {row['p90_fit_error']:.3f}), centre error {row['median_centre_error']:.3f}")
    line = {"metric": "star-shaped vs spherical contours on the slab: time and fit to the nuclei",
            "unit": "relative radial error", "value": rows[1]["median_fit_error"], "n_gpus": 1,
            "data": "synthetic", "config": {"workload": wl.name, "n_dirs": p.n_dirs, "n_rays": p.n_rays,
                                            "n_iter": wl.n_iter},
            "runs": rows}
    print(json.dumps(line), flush=True)


def bench_repel(args):
    """Soft repulsion between neighbouring contours (snk_set_repulsion) on the slab volume, 500
    iterations, exact energy and selection, at kappa = 0 (the paper's contour) and two strengths.
    Two seed sets: every nucleus seeded twice (the slab's seeds and a copy displaced by up to 1.5
    voxels along each axis, distinct ids), and the initial lattice (pitch sqrt(1.5) R0, whose
    neighbours' inner spheres overlap from the start). Reports evolve time and contour-iterations/s,
    the median final distance between the two copies of a seed, detections, and recall / precision
    against the generator's nuclei (a kept centre within 4 voxels of a nucleus centre, one to one)."""
    import numpy as np
    import torch

    import synth
    from paper_1804_06304_amd import snk

    wl = synth.slab_config()
    p = wl.params
    raw = torch.from_numpy(wl.raw).to("cuda:0")
    truth = wl.truth["centers"]
    rng = np.random.default_rng(synth.CONFIG_SEED_BASE + 7)
    n0 = len(wl.seeds)
    shift = rng.uniform(-1.5, 1.5, size=wl.seeds.shape) * np.asarray(p.spacing)[None, :]
    doubled = np.concatenate([wl.seeds, wl.seeds + shift])
    ids = np.concatenate([wl.ids, wl.ids + np.uint32(1 << 20)]).astype(np.uint32)
    ctx = snk.Context(0, torch.cuda.current_stream())
    ctx.set_params(p)
    ctx.set_directions(wl.dirs)
    ctx.load_volume(raw)
    rows = []
    for seeding in ("doubled", "lattice"):
        for kappa in (0.0, 0.02, 0.1):
            ctx.set_repulsion(kappa, args.repel_every)
            ms = []
            try:
                for _ in range(args.warmup + max(1, args.steps)):
                    if seeding == "doubled":
                        ctx.load_seeds(doubled, ids=ids)
                        n = len(doubled)
                    else:
                        n = ctx.seed_lattice()
                    ctx.evolve(wl.n_iter)
                    ms.append(ctx.get_timing()["evolve_ms"])
            except snk.SnkError as e:
                # a neighbour list over its cap (SNK_ERANGE) ends this run, not the bench
                rows.append({"seeding": seeding, "kappa": kappa, "error": str(e)})
                log(f"repel {seeding} kappa {kappa}: {e}")
                continue
            evolved = ctx.get_timing()["evolved"]
            ctx.finalize()
            out = ctx.read()
            kept = out["centers"][out["keep"] == 1]
            m = match_truth(kept, truth, 4.0)
            ev = float(np.mean(ms[args.warmup:]))
            row = {"seeding": seeding, "kappa": kappa, "every": args.repel_every if kappa > 0 else None,
                   "contours": int(n), "evolve_ms": ev, "contour_iterations_per_s": evolved / (ev * 1e-3),
                   "kept": int(len(kept)), "recall": m / len(truth), "precision": m / max(1, len(kept))}
            if seeding == "doubled":
                c = out["centers"]
                row["median_pair_distance"] = float(np.median(np.linalg.norm(c[:n0] - c[n0:], axis=1)))
            rows.append(row)
            log(f"repel {row}")
    ctx.close()
    base = next(r for r in rows if r["seeding"] == "doubled" and r["kappa"] == 0.0)
    strong = next(r for r in rows if r["seeding"] == "doubled" and r["kappa"] == 0.1)
    line = {"metric": "soft repulsion on the slab: time, seed-pair separation, recall and precision",
            "unit": "evolve time ratio (kappa 0.1 / kappa 0, doubled seeds)",
            "value": strong["evolve_ms"] / base["evolve_ms"] if "evolve_ms" in strong else None, "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "dtype": "f32", "data": "synthetic",
            "config": {"workload": wl.name, "n_iter": wl.n_iter, "every": args.repel_every,
                       "nuclei": int(len(truth))},
            "runs": rows}
    print(json.dumps(line), flush=True)


def bench_gradient(args):
    """Centre force in its weight form (Eqs. (7)-(10)) against its image-gradient form (flags bit 2)
    on the slab workload. (1) Variance: from the states after 100 iterations, one iteration's
    centre force is drawn 64 times (iteration numbers 101..164, i.e. independent draws) in both
    forms; per contour the ratio of the variances is the factor by which the gradient form needs
    fewer samples for the same noise. (2) Free runs (500 iterations, selection) with 64, 32 and 16
    rays per iteration and two Philox seeds: median centre error against the generator's nuclei,
    median distance between the two seeds' final centres (the Monte-Carlo spread), recall, time."""
    import numpy as np
    import torch

    import synth
    from paper_1804_06304_amd import snk

    wl = synth.slab_config()
    raw = torch.from_numpy(wl.raw).to("cuda:0")
    truth = wl.truth["centers"]
    stream = torch.cuda.current_stream()

    def context(params):
        ctx = snk.Context(0, stream)
        ctx.set_params(params)
        ctx.set_directions(wl.dirs)
        ctx.load_volume(raw)
        return ctx

    # (1) variance of one iteration's centre force at fixed states
    base = context(wl.params)
    base.load_seeds(wl.seeds, ids=wl.ids)
    base.evolve(100)
    s = base.get_state()
    base.close()
    live = (s["status"] & 0x0F) == 0
    draws = {}
    for flags in (0, 4):
        ctx = context(wl.params.replace(flags=flags))
        ctx.load_seeds(wl.seeds, ids=wl.ids)
        rows = []
        for k in range(64):
            ctx.set_state(s["centers"], s["radii"], s["iters"] * 0 + 100 + k, s["status"], s["streak"])
            rows.append(ctx.trace_step()[:, 7:10].copy())
        ctx.close()
        draws[flags] = np.stack(rows)  # (64, n, 3): centre steps
    v_w = draws[0].var(0).sum(1)[live]
    v_g = draws[4].var(0).sum(1)[live]
    ok = v_g > 0
    ratio = v_w[ok] / v_g[ok]
    mean_gap = np.linalg.norm(draws[0].mean(0) - draws[4].mean(0), axis=1)[live]
    sd_w = np.sqrt(v_w / 64.0)
    log(f"variance: {int(live.sum())} live contours after 100 iterations; var(weight)/var(gradient) median "
        f"{np.median(ratio):.2f}, quartiles {np.percentile(ratio, 25):.2f} / {np.percentile(ratio, 75):.2f}; "
        f"|mean difference| / sd of the weight-form mean: median {np.median(mean_gap / np.maximum(sd_w, 1e-12)):.2f}")

    # (2) free runs
    runs = []
    for flags, M in ((0, 64), (4, 64), (0, 32), (4, 32), (4, 16)):
        finals = []
        ms = []
        for seed in (wl.params.seed, wl.params.seed + 1):
            ctx = context(wl.params.replace(flags=flags, n_rays=M, seed=seed))
            ctx.load_seeds(wl.seeds, ids=wl.ids)
            ctx.evolve(wl.n_iter)
            ms.append(ctx.get_timing()["evolve_ms"])
            ctx.finalize()
            finals.append(ctx.read())
            ctx.close()
        a, b = finals
        err = np.linalg.norm(a["centers"] - truth, axis=1)
        spread = np.linalg.norm(a["centers"] - b["centers"], axis=1)
        rspread = np.abs(a["radii"] - b["radii"])
        kept = a["keep"].astype(bool)
        m = match_truth(a["centers"][kept], truth, 4.0)
        row = {"form": "gradient" if flags else "weight", "n_rays": M, "evolve_ms": float(np.mean(ms)),
               "median_centre_error": float(np.median(err)), "median_seed_spread_centre": float(np.median(spread)),
               "p90_seed_spread_centre": float(np.percentile(spread, 90)),
               "median_seed_spread_radius": float(np.median(rspread)), "kept": int(kept.sum()),
               "recall": m / len(truth), "mean_iterations": float(np.mean(a["iters"]))}
        runs.append(row)
        log(f"{row['form']:8s} M {M:2d}: evolve {row['evolve_ms']:.3f} ms, centre error {row['median_centre_error']:.3f}, "
            f"seed spread centre {row['median_seed_spread_centre']:.3f} (p90 {row['p90_seed_spread_centre']:.3f}), "
            f"radius {row['median_seed_spread_radius']:.3f}, kept {row['kept']}, recall {row['recall']:.3f}, "
            f"iterations {row['mean_iterations']:.0f}")
    line = {"metric": "centre-force variance ratio and fixed-accuracy runs, weight vs image-gradient form",
            "unit": "ratio", "value": float(np.median(ratio)), "n_gpus": 1, "data": "synthetic",
            "config": {"workload": wl.name, "state": "after 100 iterations", "draws": 64},
            "variance_ratio_quartiles": [float(np.percentile(ratio, q)) for q in (25, 50, 75)],
            "runs": runs}
    print(json.dumps(line), flush=True)


def bench_lattice(args):
    """The paper's unattended workflow on the slab volume: contours on the initial lattice (pitch
    sqrt(1.5) R0), evolved to the iteration limit with culling passes every --cull-every iterations,
    against the same lattice evolved without culling; every run ends with the exact energy and the
    selection. Culling rules: the final threshold E0 with the competition (the default rule), and
    the laxer culling threshold --e-cull-factor x E0 with and without the competition. Reports time,
    contour-iterations, detections and recall / precision against the generator's nuclei (a kept
    centre within 4 voxels of a nucleus centre, one to one)."""
    import numpy as np
    import torch

    import synth
    from paper_1804_06304_amd import snk

    wl = synth.slab_config()
    p = wl.params
    raw = torch.from_numpy(wl.raw).to("cuda:0")
    ctx = snk.Context(0, torch.cuda.current_stream())
    ctx.set_params(p)
    ctx.set_directions(wl.dirs)
    ctx.load_volume(raw)
    truth = wl.truth["centers"]
    lax = args.e_cull_factor * p.e0
    forms = {"plain": None, "e0_compete": (None, True), "lax_compete": (lax, True), "lax_no_compete": (lax, False)}
    res = {}
    for form, rule in forms.items():
        runs = []
        for rep_ in range(args.warmup + args.steps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            n = ctx.seed_lattice()
            if rule is None:
                ctx.evolve(wl.n_iter)
            else:
                ctx.set_cull(*rule)
                ctx.evolve_cull(wl.n_iter, args.cull_every, args.grace)
            tm_e = ctx.get_timing()
            ctx.finalize()
            out = ctx.read()
            secs = time.perf_counter() - t0
            tm = ctx.get_timing()
            if rep_ >= args.warmup:
                runs.append((secs, tm_e["evolve_ms"], tm["finalize_ms"], tm_e["evolved"], out))
        out = runs[-1][4]
        kept = out["centers"][out["keep"] == 1]
        m = match_truth(kept, truth, 4.0)
        res[form] = {"wall_ms": float(np.mean([r[0] for r in runs])) * 1e3,
                     "evolve_ms": float(np.mean([r[1] for r in runs])),
                     "finalize_ms": float(np.mean([r[2] for r in runs])),
                     "contour_iterations": int(runs[-1][3]), "contours": int(n),
                     "culled": int(np.sum((out["status"] & 0x0F) == snk.CULLED)), "kept": int(len(kept)),
                     "recall": m / len(truth), "precision": m / max(1, len(kept))}
        log(f"lattice {form}: {res[form]}")
    ctx.close()
    c = res["lax_no_compete"]
    line = {
        "metric": "lattice workflow: contour-iterations/s with culling passes", "value":
            c["contour_iterations"] / (c["wall_ms"] * 1e-3), "unit": "contour-iterations/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": c["wall_ms"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "slab-lattice-seeded", "volume": "512x512x128 u16, h=(1,1,2)",
                   "nuclei": int(len(truth)), "n_iter": wl.n_iter, "cull_every": args.cull_every,
                   "grace": args.grace, "e_cull": lax, "pitch": float(np.sqrt(1.5) * p.r_init)},
        "runs": res,
        "speedup_wall_lax_no_compete": res["plain"]["wall_ms"] / c["wall_ms"],
    }
    print(json.dumps(line), flush=True)


def plain_pass(snk, ctx, wl, raw_dev):
    """One volume through the plain per-volume path (a context reused across volumes)."""
    ctx.set_params(wl.params)
    ctx.set_directions(wl.dirs)
    ctx.load_volume(raw_dev)
    ctx.load_seeds(wl.seeds, ids=wl.ids)
    ctx.prepass()
    ctx.evolve(wl.n_iter)
    ctx.finalize()
    return ctx.read()


KEYS = ("radii", "centers", "e_mc", "e_vox", "iters", "status", "keep")


def oracle_run(wl, raw_np):
    """The FP64 oracle's whole run of one workload (pre-pass, evolution, exact energy, selection);
    returns its state, kept flags, vertex-updates and seconds."""
    import oracle
    p = wl.params
    t0 = time.perf_counter()
    J = oracle.prepass(raw_np, p)
    st = oracle.init_state(p, wl.seeds, ids=wl.ids, shape_zyx=raw_np.shape)
    _, done = oracle.evolve(J, p, wl.dirs, st, wl.n_iter)
    oracle.finalize_status(st)
    e_vox, _ = oracle.energy_vox(J, p, st.c, st.R)
    keep = oracle.cull(p, st.c, st.R, e_vox, st.status, st.ids)
    return st, keep, done * p.n_rays, time.perf_counter() - t0


def compare_with_oracle(outs, refs):
    """Free-run agreement of GPU results with the oracle's runs of the same contours: the worst radius
    and centre differences over every contour, the fraction with identical iteration counts and of
    identical keep flags."""
    import numpy as np
    dR, dc, same, n, kept_same = 0.0, 0.0, 0, 0, 0
    for got, (st, keep) in zip(outs, refs):
        if len(st.R) == 0:
            continue
        dR = max(dR, float(np.max(np.abs(got["radii"] - st.R))))
        dc = max(dc, float(np.max(np.linalg.norm(got["centers"] - st.c, axis=1))))
        same += int(np.sum(got["iters"] == st.iters))
        kept_same += int(np.sum(got["keep"] == keep))
        n += len(st.R)
    return {"contours": n, "max_abs_dR": dR, "max_abs_dc": dc, "same_iters_frac": same / max(n, 1),
            "same_keep_frac": kept_same / max(n, 1),
            "ok": bool(dR <= 0.05 and dc <= 0.5 and same >= 0.99 * n)}


def run_plane(args):
    """The 2D workload (8192^2 u8, 40,000 touching cells, 300 iterations) through the plain path:
    vertex-updates/s per step and the evolve kernel's rates, the FP64 oracle over the whole workload
    (the CPU figure) and its agreement with the GPU's run."""
    import numpy as np
    import torch

    import oracle
    import synth
    from paper_1804_06304_amd import snk

    t0 = time.perf_counter()
    wl = synth.plane_config()
    log(f"plane: {wl.name} generated in {time.perf_counter() - t0:.1f} s")
    p = wl.params
    raw = torch.from_numpy(wl.raw).to("cuda:0")
    ctx = snk.Context(0, torch.cuda.current_stream())
    ctx.set_params(p)
    ctx.set_directions(wl.dirs)
    ctx.load_volume(raw)
    ev, evolved, wall = [], 0, 0.0
    for k in range(1 + args.extra_steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.load_seeds(wl.seeds, ids=wl.ids)
        ctx.prepass()
        ctx.evolve(wl.n_iter)
        ctx.finalize()
        out = ctx.read()
        tm = ctx.get_timing()
        if k > 0:
            wall += time.perf_counter() - t0
            ev.append(tm["evolve_ms"])
            evolved += tm["evolved"]
    ctx.close()
    steps = args.extra_steps
    vu = evolved * p.n_rays
    ev_ms = float(np.mean(ev))
    res = {"workload": wl.name, "value": vu / wall, "unit": "vertex-updates/s", "steps": steps,
           "ms_per_step": wall / steps * 1e3, "evolve_ms": ev_ms,
           "evolve_vertex_updates_per_s": vu / steps / (ev_ms * 1e-3),
           "evolve_tflops": vu / steps * FLOP_PER_VU[2] / (ev_ms * 1e-3) / 1e12,
           "launch": {"lanes_per_contour": tm["lanes_per_contour"], "pairs_in_flight": tm["pairs_in_flight"],
                      "layout": tm["layout"], "tile_voxels": tm["tile_voxels"]}}
    log(f"plane: {res['ms_per_step']:.2f} ms per step, evolve {ev_ms:.3f} ms, {res['value']:.4g} vu/s")
    if not args.no_cpu_baseline:
        log("plane: FP64 oracle over the whole workload ...")
        st, keep, ovu, secs = oracle_run(wl, wl.raw)
        res["cpu_baseline"] = {"value": ovu / secs, "unit": "vertex-updates/s", "cores": oracle.num_threads(),
                               "kind": "oracle", "sample": f"the whole workload ({len(wl.seeds)} contours, "
                                                           f"{wl.n_iter} iterations, pre-pass, energy, selection), "
                                                           f"{secs:.1f} s"}
        res["parity_vs_oracle"] = compare_with_oracle([out], [(st, keep)])
        log(f"plane: oracle {secs:.1f} s; parity {res['parity_vs_oracle']}")
    return res


def run_batched(args, steps, warmup):
    """256 cubic u16 subvolumes (edge 32..160, 10..800 nuclei, D 162 or 642, 200 iterations): the
    engine's captured batched run against the plain per-volume loop on the same resident inputs,
    with the engine's result checked against the plain path and, on every 8th subvolume, against
    the FP64 oracle (whose time on that 1/8 subset gives the CPU figure, extrapolated)."""
    import numpy as np
    import torch

    import oracle
    import synth
    from synth.volumes import subvolume_workloads
    from paper_1804_06304_amd import snk

    t0 = time.perf_counter()
    jobs = subvolume_workloads(synth.CONFIG_SEED_BASE + 4, device="cuda:0")
    torch.cuda.synchronize()
    n_contours = sum(len(w.seeds) for w in jobs)
    log(f"batched: {len(jobs)} subvolumes, {n_contours} contours, "
        f"{sum(w.raw.numel() for w in jobs) / 1e6:.0f} M voxels, generated in {time.perf_counter() - t0:.1f} s")
    stream = torch.cuda.current_stream()
    vu_of = lambda outs: sum(int(o["iters"].sum()) * w.params.n_rays for w, o in zip(jobs, outs))

    ctx = snk.Context(0, stream)
    ctx.set_tile(args.tile)
    for w in jobs[:8]:
        plain_pass(snk, ctx, w, w.raw)   # warm up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plain_outs = [plain_pass(snk, ctx, w, w.raw) for w in jobs]
    torch.cuda.synchronize()
    plain_s = time.perf_counter() - t0
    ctx.close()
    plain_vu = vu_of(plain_outs)
    log(f"batched: plain per-volume loop {plain_s * 1e3:.1f} ms, {plain_vu / plain_s:.4g} vertex-updates/s")

    eng = snk.Engine(0, stream, 64 << 30)
    ids = [eng.submit(w.params, w.dirs, w.raw, w.seeds, ids=w.ids, n_iter=w.n_iter) for w in jobs]
    t0 = time.perf_counter()
    eng.run()   # autotune per launch class + capture
    tune_ms = (time.perf_counter() - t0) * 1e3
    log(f"batched: engine first run (autotune + capture) {tune_ms:.1f} ms")
    for _ in range(warmup):
        eng.run()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        eng.run()
    torch.cuda.synchronize()
    secs = time.perf_counter() - t0
    outs = [eng.read(j) for j in ids]
    st = eng.get_stats()
    classes = eng.tuned_shapes()
    eng.close()
    # the tuned lanes and pair-points forced with and without the persistent work queue (no LDS box)
    forced = {}
    for pers in (0, 1):
        e2 = snk.Engine(0, stream, 64 << 30)
        e2.set_launch(st["lanes_per_contour"], st["pairs_in_flight"], pers, 0)
        for w in jobs:
            e2.submit(w.params, w.dirs, w.raw, w.seeds, ids=w.ids, n_iter=w.n_iter)
        e2.run()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            e2.run()
        torch.cuda.synchronize()
        forced["persistent" if pers else "one_workgroup_per_contour"] = (time.perf_counter() - t0) / steps * 1e3
        e2.close()
    log(f"batched: forced shapes (ms per pass): {forced}")
    vu = vu_of(outs) * steps
    same = all(np.array_equal(a["iters"], b["iters"]) for a, b in zip(outs, plain_outs))
    drift = max(float(np.max(np.abs(a["radii"] - b["radii"]), initial=0.0)) for a, b in zip(outs, plain_outs))
    res = {"workload": "batched-256-subvolumes-u16", "value": vu / secs, "unit": "vertex-updates/s",
           "steps": steps, "ms_per_step": secs / steps * 1e3, "volumes": len(jobs), "contours": n_contours,
           "n_iter": jobs[0].n_iter, "graph_ms": st["last_ms"], "autotune_and_capture_ms": tune_ms,
           "launch_last_class": {"lanes_per_contour": st["lanes_per_contour"],
                                 "pairs_in_flight": st["pairs_in_flight"], "persistent": st["persistent"],
                                 "layout": st["layout"]},
           "plain_loop": {"value": plain_vu / plain_s, "ms": plain_s * 1e3},
           "speedup_vs_plain_loop": (vu / secs) / (plain_vu / plain_s),
           "parity_vs_plain": {"same_iters": bool(same), "max_abs_dR": drift}}
    res["tuned_classes"] = classes
    res["forced_shapes_ms"] = {"lanes_per_contour": st["lanes_per_contour"], "pairs_in_flight": st["pairs_in_flight"],
                               "tile_voxels": 0, **forced}
    log(f"batched: engine {secs / steps * 1e3:.1f} ms per pass, {res['value']:.4g} vu/s, "
        f"{res['speedup_vs_plain_loop']:.2f}x the plain loop")
    if not args.no_cpu_baseline:
        sub = jobs[::8]
        log(f"batched: FP64 oracle on every 8th subvolume ({len(sub)}) ...")
        refs, ovu, osecs = [], 0, 0.0
        for w in sub:
            o_st, o_keep, v, sec = oracle_run(w, w.raw.cpu().numpy())
            refs.append((o_st, o_keep))
            ovu += v
            osecs += sec
        res["cpu_baseline"] = {"value": ovu / osecs, "unit": "vertex-updates/s", "cores": oracle.num_threads(),
                               "kind": "oracle",
                               "sample": f"every 8th subvolume ({len(sub)} of {len(jobs)}, "
                                         f"{sum(len(w.seeds) for w in sub)} contours), whole runs, {osecs:.1f} s; "
                                         f"the whole batch extrapolates to {osecs * len(jobs) / len(sub):.0f} s"}
        res["parity_vs_oracle"] = compare_with_oracle(outs[::8], refs)
        log(f"batched: oracle {osecs:.1f} s; parity {res['parity_vs_oracle']}")
    return res


def bench_batched(args):
    res = run_batched(args, args.steps, args.warmup)
    line = {"metric": METRIC, "value": res["value"], "unit": "vertex-updates/s", "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": res["ms_per_step"], "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f32", "data": "synthetic",
            "config": {"workload": res["workload"], "volumes": res["volumes"], "contours": res["contours"],
                       "n_iter": res["n_iter"]}}
    line.update({k: v for k, v in res.items() if k not in line and k not in ("workload", "volumes", "contours")})
    print(json.dumps(line), flush=True)


def serve_stream(snk, eng, vol_dev, V, arrivals, reqs, chunk, keep_outputs=(), chunk_idle=0):
    """Serve `arrivals` (times in seconds, request indices into `reqs`) through the engine: each
    request's tile is cut from the resident volume when it arrives, submitted, and stepped with the
    others until done (continuous batching). A step advances every running contour by `chunk`
    iterations, or by `chunk_idle` when a single job runs and none waits (fewer round trips at low
    load; a request arriving meanwhile joins at the next step). Returns latencies (s),
    vertex-updates, the wall time and the outputs of the requests listed in keep_outputs."""
    import numpy as np
    import torch
    job_req, held, lat, vu, kept = {}, {}, [], 0, {}
    nxt = 0
    t0 = time.perf_counter()
    while nxt < len(arrivals) or job_req:
        now = time.perf_counter() - t0
        while nxt < len(arrivals) and arrivals[nxt] <= now:
            wl, lo, hi = reqs[nxt]
            tile = vol_dev[lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]].contiguous()
            j = eng.submit(wl.params, wl.dirs, tile, wl.seeds, ids=wl.ids, n_iter=wl.n_iter)
            job_req[j] = nxt
            held[j] = tile          # borrowed by the engine until the job completes
            nxt += 1
        st = eng.get_stats()
        if st["running"] or st["pending"]:
            alone = st["pending"] + st["running"] <= 1
            eng.step(chunk_idle if (chunk_idle > 0 and alone) else chunk)
        elif nxt < len(arrivals):
            time.sleep(max(0.0, arrivals[nxt] - (time.perf_counter() - t0)))
        for j in eng.poll():
            r = job_req.pop(j)
            lat.append(time.perf_counter() - t0 - arrivals[r])
            out = eng.read(j)
            if r in keep_outputs:
                kept[r] = out
            vu += int(out["iters"].sum()) * reqs[r][0].params.n_rays
            eng.release(j)
            held.pop(j, None)
    return np.asarray(lat), vu, time.perf_counter() - t0, kept


def poisson_arrivals(rng, rate, window):
    import numpy as np
    t, out = 0.0, []
    while True:
        t += rng.exponential(1.0 / rate)
        if t > window:
            return np.asarray(out)
        out.append(t)


def run_served(args):
    """Tile-segmentation requests cut from a 2048 x 2048 x 512 uint16 volume (about 215,000 nuclei,
    20-400 per 128^3 block, gain 0.7-1, Poisson counts) resident on the device: tile cores of edge
    U{64..256} plus a 16-voxel halo, seeds at the true centres in the core, D 162, M 32, 200
    iterations. Poisson arrivals at `rate` per second over `serve_seconds`, and at `rate_hi` (a load
    the engine cannot keep up with), through the engine's continuous batching; the plain path serving
    the first stream one request at a time; a sample of requests checked bit for bit against the plain
    path and against the FP64 oracle, whose time on those tiles gives the CPU figure."""
    import numpy as np
    import torch

    import oracle
    import synth
    from synth.volumes import served_volume, tile_workload
    from paper_1804_06304_amd import snk

    t0 = time.perf_counter()
    V = served_volume(synth.CONFIG_SEED_BASE + 5)
    n_obj = len(V.objects().centers)
    t1 = time.perf_counter()
    vol = V.whole("cuda:0")
    torch.cuda.synchronize()
    log(f"served: volume {V.shape} with {n_obj} nuclei: objects {t1 - t0:.1f} s, voxels on the device "
        f"{time.perf_counter() - t1:.1f} s")
    stream = torch.cuda.current_stream()
    rng = np.random.default_rng(0x5E7)

    def requests(n):
        out = []
        for _ in range(n):
            lo, hi, clo, chi, idx = V.tile(rng)
            out.append((tile_workload(V, lo, hi, idx, None, seed=synth.CONFIG_SEED_BASE + 5), lo, hi))
        return out

    free_b, total_b = torch.cuda.mem_get_info(0)
    budget = min(64 << 30, free_b // 2)
    eng = snk.Engine(0, stream, budget)
    warm = requests(4)
    _, _, _, _ = serve_stream(snk, eng, vol, V, np.zeros(len(warm)), warm, args.chunk)
    res = {"workload": "served-tiles-of-2048x2048x512-u16", "hbm_budget_gib": round(budget / 2**30, 1),
           "nuclei": n_obj, "n_iter": 200, "chunk": args.chunk, "chunk_idle": args.chunk_idle, "streams": {}}
    sample = tuple(range(args.served_check))
    outs1, reqs1 = None, None
    for rate, window in ((args.rate, args.serve_seconds), (args.rate_hi, args.serve_seconds_hi)):
        arr = poisson_arrivals(rng, rate, window)
        reqs = requests(len(arr))
        log(f"served: {len(arr)} requests at {rate:g}/s over {window:g} s ...")
        lat, vu, secs, kept = serve_stream(snk, eng, vol, V, arr, reqs, args.chunk, keep_outputs=sample,
                                           chunk_idle=args.chunk_idle)
        lat_ms = lat * 1e3
        res["streams"][f"{rate:g}_per_s"] = {
            "rate_per_s": rate, "window_s": window, "requests": len(arr), "wall_s": secs,
            "vertex_updates_per_s": vu / secs,
            "latency_ms": {"p50": float(np.percentile(lat_ms, 50)), "p99": float(np.percentile(lat_ms, 99)),
                           "max": float(lat_ms.max())},
            "tile_voxels_mean": float(np.mean([np.prod(h - l) for _, l, h in reqs]))}
        log(f"served: {rate:g}/s -> {vu / secs:.4g} vu/s, p50 {np.percentile(lat_ms, 50):.2f} ms, "
            f"p99 {np.percentile(lat_ms, 99):.2f} ms")
        if outs1 is None:
            outs1, reqs1, arr1 = kept, reqs, arr
    st = eng.get_stats()
    res["engine_launch"] = {"lanes_per_contour": st["lanes_per_contour"], "pairs_in_flight": st["pairs_in_flight"],
                            "persistent": st["persistent"], "layout": st["layout"]}
    eng.close()

    # the plain path serving the first stream's requests one at a time, in arrival order
    ctx = snk.Context(0, stream)
    n_plain = int(np.searchsorted(arr1, min(10.0, args.serve_seconds)))   # the stream's first 10 s
    plat, pvu = [], 0
    t0 = time.perf_counter()
    for r in range(n_plain):
        now = time.perf_counter() - t0
        if arr1[r] > now:
            time.sleep(arr1[r] - now)
        wl, lo, hi = reqs1[r]
        tile = vol[lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]].contiguous()
        o = plain_pass(snk, ctx, wl, tile)
        plat.append(time.perf_counter() - t0 - arr1[r])
        pvu += int(o["iters"].sum()) * wl.params.n_rays
    psecs = time.perf_counter() - t0
    plat = np.asarray(plat) * 1e3
    res["plain_same_stream"] = {"requests": n_plain, "window_s": float(arr1[n_plain - 1]) if n_plain else 0.0,
                                "vertex_updates_per_s": pvu / psecs,
                                "latency_ms": {"p50": float(np.percentile(plat, 50)),
                                               "p99": float(np.percentile(plat, 99))}}
    log(f"served: plain path on the same stream {pvu / psecs:.4g} vu/s, p50 {np.percentile(plat, 50):.2f} ms")

    # the plain path back to back (no arrival gaps) on the saturating stream's first requests: the
    # per-volume launch at full load, to set beside the engine's delivered rate at that load
    n_sat = min(len(reqs), 500)
    svu = 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for r in range(n_sat):
        wl, lo, hi = reqs[r]
        tile = vol[lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]].contiguous()
        o = plain_pass(snk, ctx, wl, tile)
        svu += int(o["iters"].sum()) * wl.params.n_rays
    ssecs = time.perf_counter() - t0
    res["plain_back_to_back"] = {"requests": n_sat, "vertex_updates_per_s": svu / ssecs,
                                 "ms_per_request": ssecs / n_sat * 1e3}
    sat = res["streams"][f"{args.rate_hi:g}_per_s"]["vertex_updates_per_s"]
    res["engine_vs_plain_at_saturation"] = sat / (svu / ssecs)
    log(f"served: plain path back to back {svu / ssecs:.4g} vu/s; engine at {args.rate_hi:g}/s delivers "
        f"{res['engine_vs_plain_at_saturation']:.2f}x that")

    # bit-for-bit against the plain path in the engine's launch shape (no LDS boxes in the engine)
    el = res["engine_launch"]
    ctx.set_launch(el["lanes_per_contour"], el["pairs_in_flight"], 0)
    ctx.set_tile(0)
    bitwise, refs, outs, ovu, osecs = True, [], [], 0, 0.0
    for r in sorted(outs1):
        wl, lo, hi = reqs1[r]
        tile = vol[lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]].contiguous()
        o = plain_pass(snk, ctx, wl, tile)
        bitwise &= all(np.array_equal(o[k], outs1[r][k]) for k in KEYS)
        if not args.no_cpu_baseline:
            o_st, o_keep, v, sec = oracle_run(wl, tile.cpu().numpy())
            refs.append((o_st, o_keep))
            outs.append(outs1[r])
            ovu += v
            osecs += sec
    ctx.close()
    res["parity_vs_plain"] = {"requests": len(outs1), "bitwise": bool(bitwise)}
    if not args.no_cpu_baseline and refs:
        res["parity_vs_oracle"] = compare_with_oracle(outs, refs)
        res["cpu_baseline"] = {"value": ovu / osecs, "unit": "vertex-updates/s", "cores": oracle.num_threads(),
                               "kind": "oracle", "sample": f"{len(refs)} served tiles, whole runs, {osecs:.1f} s "
                                                           "(throughput only)"}
        log(f"served: oracle on {len(refs)} tiles {osecs:.1f} s; parity {res['parity_vs_oracle']}")
    del vol
    torch.cuda.empty_cache()
    return res


def bench_served(args):
    res = run_served(args)
    s0 = res["streams"][f"{args.rate:g}_per_s"]
    line = {"metric": "contour vertex-updates/s at fixed accuracy; p50/p99 tile latency when served",
            "value": s0["vertex_updates_per_s"], "unit": "vertex-updates/s", "n_gpus": 1, "steps": s0["requests"],
            "warmup": 4, "ms_per_step": s0["wall_s"] / max(s0["requests"], 1) * 1e3, "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
            "config": {"workload": res["workload"], "rate_per_s": args.rate, "window_s": args.serve_seconds}}
    line.update({k: v for k, v in res.items() if k != "workload"})
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
