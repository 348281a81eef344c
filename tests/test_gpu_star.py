"""Star-shaped contours (per-direction radii, snk_set_star) on the GPU against the FP64 oracle.

The model is not in the paper (a builder-defined extension of its sphere); the oracle's star
functions are pinned on the CPU (tied radii reproduce the sphere, frozen-point derivatives, the
smoothing step, the direction tables). Here the HIP kernel is checked against that oracle: one
teacher-forced iteration (every direction's radius, the centre, the energy), a free run, and the
error paths.
"""
import sys

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def snk():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1804_06304_amd import snk as mod
    mod.load()
    return mod


@pytest.fixture(scope="module")
def stream():
    import torch
    return torch.cuda.current_stream()


def make_ctx(snk, stream, wl, smooth, lanes=0):
    import torch
    ctx = snk.Context(0, stream)
    ctx.set_params(wl.params)
    ctx.set_launch(lanes, 0, 0)
    ctx.set_star(smooth)
    ctx.set_directions(wl.dirs)
    raw = torch.from_numpy(np.ascontiguousarray(wl.raw)).to("cuda:0")
    ctx.load_volume(raw)
    ctx._raw = raw
    return ctx


def workload(which):
    if which == "tiny":
        wl = synth.tiny_config()
    elif which == "tiny96":
        # more rays than one wave holds: the duplicate-direction pass scans every ray
        wl = synth.tiny_config()
        wl.params = wl.params.replace(n_rays=96)
    elif which == "aniso":
        wl = synth.slab_config(n_target=40, shape_xyz=(96, 80, 40), n_iter=50)
    else:
        wl = synth.plane_config(n_target=120, size=256, n_iter=50)
    return wl


def inner_seeds(wl, n, rng):
    """Seeds away from the faces (plus the workload's own)."""
    nx, ny, nz = wl.shape_xyz
    h = np.array(wl.params.spacing)
    ext = (np.array([nx, ny, nz]) - 1) * h
    s = rng.uniform(0.15, 0.85, size=(n, 3)) * ext
    if wl.params.dim == 2:
        s[:, 2] = 0.0
    return np.concatenate([wl.seeds, s])


@pytest.mark.parametrize("which,smooth,lanes", [("tiny", 0.0, 0), ("tiny", 0.6, 64), ("aniso", 0.3, 0),
                                                ("aniso", 0.3, 64), ("plane", 0.3, 0), ("plane", 0.3, 64),
                                                ("tiny96", 0.3, 0), ("tiny96", 0.3, 64)])
def test_star_one_step_parity(snk, stream, which, smooth, lanes):
    """Teacher forced: both sides start from the oracle's state after a few star iterations (and,
    for the first check, from untied random radii), rounded to FP32; one GPU iteration must give
    every direction's radius step, the centre step and the energy of the oracle's iteration; one
    wave (64 lanes) or two (the automatic 128) per contour; up to 64 rays (one wave's duplicate-
    direction pass) or 96 (every lane scanning all rays)."""
    wl = workload(which)
    p = wl.params
    rng = np.random.default_rng(2)
    seeds = inner_seeds(wl, 24, rng)
    ids = np.arange(len(seeds), dtype=np.uint32) * 5 + 1
    J = oracle.prepass(wl.raw, p)
    tables = oracle.star_tables(wl.dirs, p.dim)
    st = oracle.star_init(p, seeds, ids=ids, shape_zyx=wl.raw.shape)
    D = p.n_dirs
    lo = oracle.r_geom_min(p.dim, p.dR)
    st.Rk[:] = rng.uniform(max(lo, 0.7 * p.r_init), 1.3 * p.r_init, size=st.Rk.shape)
    ctx = make_ctx(snk, stream, wl, smooth, lanes)
    ctx.load_seeds(seeds, ids=ids)
    worst = {}
    for pre in (0, 4):
        if pre:
            oracle.star_evolve(J, p, wl.dirs, tables, smooth, st, pre)
        c32 = st.c.astype(np.float32).astype(np.float64)
        R32 = st.Rk.astype(np.float32)
        live = (st.status & 0x0F) == oracle.ACTIVE
        ctx.set_state(c32, R32.mean(axis=1), st.iters, st.status, st.streak)
        ctx.set_star_radii(R32)
        ctx.evolve(1)
        got = ctx.read()
        Rg = ctx.get_star_radii()
        for i in np.where(live)[0]:
            t = oracle.star_step_terms(J, p, wl.dirs, tables, smooth, c32[i], R32[i].astype(np.float64),
                                       st.iters[i] + 1, ids[i])
            Rn = R32[i] + t["dR"]
            inside = (Rn > lo + 1e-3) & (Rn < p.r_max - 1e-3)
            dR_g = Rg[i].astype(np.float64) - R32[i]
            err = np.abs(dR_g - t["dR"])[inside]
            tol = (1e-5 * np.maximum(np.abs(t["dR"]), t["dR_abs"]) + t["dR_slack"] + 2e-6 * np.abs(R32[i]))[inside]
            assert np.all(err <= tol), (which, pre, i, err.max(), np.argmax(err / tol))
            worst["dR"] = max(worst.get("dR", 0.0), float(np.max(err / tol)) if len(err) else 0.0)
            e_err = abs(got["e_mc"][i] - t["E"])
            e_tol = 1e-5 * max(abs(t["E"]), t["E_abs"]) + 1e-7
            assert e_err <= e_tol, (which, pre, i, got["e_mc"][i], t["E"])
            worst["E"] = max(worst.get("E", 0.0), e_err / e_tol)
            dc_g = got["centers"][i] - c32[i]
            dc_tol = 1e-5 * np.maximum(np.abs(t["dc"]), t["dc_abs"]) + t["dc_slack"] + 2e-6 * np.abs(c32[i]) + 1e-7
            assert np.all(np.abs(dc_g - t["dc"])[: p.dim] <= dc_tol[: p.dim]), (which, pre, i, dc_g, t["dc"])
            worst["dc"] = max(worst.get("dc", 0.0), float(np.max((np.abs(dc_g - t["dc"]) / dc_tol)[: p.dim])))
        say(f"  star one-step {which} smooth {smooth} after {pre}: {int(live.sum())} live, worst err/tol "
            + ", ".join(f"{k} {v:.3f}" for k, v in worst.items()))
    ctx.close()


@pytest.mark.parametrize("lanes", [0, 64])
def test_star_free_run(snk, stream, lanes):
    """Tiny workload, star contours with smoothing: after 100 iterations the GPU's per-direction
    radii (each within 0.05 voxel, the free-run radius bar), centres, iteration counts and states
    follow the oracle's (FP32 against FP64: the Monte-Carlo trajectories drift apart only by
    rounding; measured drift below 1e-4)."""
    wl = synth.tiny_config()
    p = wl.params
    smooth = 0.3
    J = oracle.prepass(wl.raw, p)
    tables = oracle.star_tables(wl.dirs, p.dim)
    st = oracle.star_init(p, wl.seeds, ids=wl.ids, shape_zyx=wl.raw.shape)
    oracle.star_evolve(J, p, wl.dirs, tables, smooth, st, wl.n_iter)
    ctx = make_ctx(snk, stream, wl, smooth, lanes)
    ctx.load_seeds(wl.seeds, ids=wl.ids)
    ctx.evolve(wl.n_iter)
    assert ctx.get_timing()["lanes_per_contour"] == (lanes or 128)
    ctx.finalize()
    got = ctx.read()
    Rg = ctx.get_star_radii()
    ctx.close()
    assert np.array_equal(got["iters"], st.iters)
    # the oracle's contours stop alike; finalize turns the ones still active into MAXITER
    ref_status = np.where((st.status & 0x0F) == oracle.ACTIVE, (st.status & 0x10) | oracle.MAXITER, st.status)
    assert np.array_equal(got["status"], ref_status)
    assert np.max(np.abs(got["radii"] - st.R)) <= 0.05
    assert np.max(np.abs(Rg - st.Rk)) <= 0.05
    assert np.max(np.linalg.norm(got["centers"] - st.c, axis=1)) <= 0.5
    assert np.array_equal(got["e_vox"], got["e_mc"])
    # selection on the last Monte-Carlo energy and the mean radius, as the oracle's greedy does it
    e = got["e_mc"].astype(np.float64)
    amb = oracle.cull_ambiguity(p, got["centers"], got["radii"], e)
    keep_ref = oracle.cull(p, got["centers"], got["radii"], e, got["status"], wl.ids)
    ok = amb == 0
    assert np.array_equal(got["keep"][ok], keep_ref[ok])
    assert got["keep"].sum() > 0
    say(f"  star free run: max |dR_k| {np.max(np.abs(Rg - st.Rk)):.4f}, max |dR mean| "
        f"{np.max(np.abs(got['radii'] - st.R)):.4f}, kept {int(got['keep'].sum())}/{len(got['keep'])}")


def test_star_error_paths(snk, stream):
    """n_radial other than 16, exact sums and the gradient-form centre force are refused at the next
    evolve; so is a direction table without antipodes; snk_trace_step is refused; the sphere is back
    after snk_set_star(-1); lanes per contour other than 64 or 128 are refused."""
    wl = synth.tiny_config()
    for bad in (wl.params.replace(n_radial=8), wl.params.replace(flags=2), wl.params.replace(flags=4)):
        w = synth.tiny_config()
        w.params = bad
        ctx = make_ctx(snk, stream, w, 0.2)
        ctx.load_seeds(w.seeds)
        with pytest.raises(snk.SnkError):
            ctx.evolve(1)
        ctx.close()
    rng = np.random.default_rng(0)
    dirs = rng.normal(size=(40, 3))
    dirs /= np.linalg.norm(dirs, axis=1)[:, None]
    w = synth.tiny_config()
    w.params = w.params.replace(n_dirs=40)
    w.dirs = dirs
    ctx = make_ctx(snk, stream, w, 0.2)
    ctx.load_seeds(w.seeds)
    with pytest.raises(snk.SnkError):
        ctx.evolve(1)
    ctx.close()
    ctx = make_ctx(snk, stream, wl, 0.2)
    ctx.load_seeds(wl.seeds)
    with pytest.raises(snk.SnkError):
        ctx.trace_step()
    ctx.set_star(-1.0)
    assert ctx.trace_step().shape[0] == len(wl.seeds)
    ctx.close()
    # star contours run one or two waves per contour
    ctx = make_ctx(snk, stream, wl, 0.2, lanes=256)
    ctx.load_seeds(wl.seeds)
    with pytest.raises(snk.SnkError):
        ctx.evolve(1)
    ctx.close()
