#!/usr/bin/env python
"""Benchmark of the whole hot path on one MI355X.

A step is one pass of the path over the slab workload (512x512x128 uint16, ~2,000 ellipsoid
nuclei, anisotropic spacing (1, 1, 2), D 642 directions, M 64 rays x L 16 radial points per
contour-iteration, 500 iterations): reset contour state from the seeds, pre-pass, evolve, exact
energy + selection, readback. Inputs (raw volume, direction table) are resident in HBM before the
timed region; the seeds are re-sent each step (48 KB).

Prints ONE JSON line: vertex-updates/s (one vertex-update = one sampled ray of one active contour
in one iteration), the evolve kernel's achieved logical-gather bandwidth against the 8 TB/s HBM
peak (from HIP events recorded around each launch on the launch stream), and the FP64 oracle
timed on a bounded sample on the host cores.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "contour vertex-updates/s at fixed accuracy"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


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
    return base, parity


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--waves", type=int, default=0, help="wave64s per contour (0: automatic)")
    ap.add_argument("--unroll", type=int, default=0, help="gathers in flight per thread (0: automatic)")
    ap.add_argument("--box", type=int, default=0, help="LDS footprint floats per contour (0: automatic, -1: off)")
    ap.add_argument("--cpu-sample", type=int, default=0, help="contours in the oracle baseline (0: all)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--sweep", action="store_true",
                    help="only time the evolve kernel for every (waves, gathers-in-flight) launch shape")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a plain 1 GiB device-to-device copy 4 times (calibrates HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: --gpus {args.gpus} is not supported: this build runs the path on one GPU "
              "(DESIGN.md describes how it would shard over slabs).", file=sys.stderr)
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
    t0 = time.perf_counter()
    wl = synth.slab_config()
    log(f"workload {wl.name}: generated in {time.perf_counter() - t0:.1f} s")
    p = wl.params
    stream = torch.cuda.current_stream()
    raw = torch.from_numpy(wl.raw).to("cuda:0")
    ctx = snk.Context(0, stream)
    ctx.set_params(p)
    ctx.set_launch(args.waves, args.unroll, args.box)
    ctx.set_directions(wl.dirs)
    ctx.load_volume(raw)
    torch.cuda.synchronize()

    if args.sweep:
        for box in (0, -1):
            for w in (1, 2, 4, 8):
                for u in (1, 2, 4):
                    ctx.set_launch(w, u, box)
                    ms = []
                    for _ in range(3):
                        ctx.load_seeds(wl.seeds, ids=wl.ids)
                        ctx.evolve(wl.n_iter)
                        ms.append(ctx.get_timing()["evolve_ms"])
                    log(f"sweep box={box} waves={w} gathers_in_flight={u}: evolve {min(ms):.3f} ms "
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
    t0 = time.perf_counter()
    for _ in range(args.steps):
        out, tm = step()
        evolve_ms.append(tm["evolve_ms"])
        prepass_ms.append(tm["prepass_ms"])
        finalize_ms.append(tm["finalize_ms"])
        evolved += tm["evolved"]
    torch.cuda.synchronize()
    secs = time.perf_counter() - t0
    ctx.close()

    M, L, d = p.n_rays, p.n_radial, p.dim
    vu = evolved * M
    per_launch_vu = vu / args.steps
    bytes_per_vu = L * (2 ** d) * 4
    ev_ms = float(np.mean(evolve_ms))
    achieved = per_launch_vu * bytes_per_vu / (ev_ms * 1e-3) / 1e9
    log(f"per step: prepass {np.mean(prepass_ms):.3f} ms, evolve {ev_ms:.3f} ms, finalize {np.mean(finalize_ms):.3f} ms,"
        f" wall {secs / args.steps * 1e3:.3f} ms; vertex-updates/step {per_launch_vu:.4g};"
        f" kept {int(out['keep'].sum())}/{len(out['keep'])}")
    line = {
        "metric": METRIC, "value": vu / secs, "unit": "vertex-updates/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": secs / args.steps * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": wl.name, "volume": "512x512x128 u16, h=(1,1,2)", "contours": len(wl.seeds),
                   "n_iter": wl.n_iter, "n_dirs": p.n_dirs, "n_rays": M, "n_radial": L,
                   "waves_per_contour": args.waves or "auto", "gathers_in_flight": args.unroll or "auto",
                   "lds_box_floats": args.box or "auto"},
        "kernels_ms": {"prepass": float(np.mean(prepass_ms)), "evolve": ev_ms,
                       "finalize": float(np.mean(finalize_ms))},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "evolve_kernel<3,*,false>",
                     "algorithmic_bytes": f"{bytes_per_vu} B per vertex-update (L x 2^d taps x 4 B, logical gathers)"},
    }
    if not args.no_cpu_baseline:
        log("cpu baseline: FP64 oracle on the same workload ...")
        base, parity = cpu_baseline(wl, out, args.cpu_sample)
        line["cpu_baseline"] = base
        line["parity_sample"] = parity
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
