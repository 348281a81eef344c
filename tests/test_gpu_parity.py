"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle on the same seeded inputs.

Bars (stated per test):
  * pre-pass: |J_gpu - J_ref| <= 2e-6 * max|I| (FP32 sums of positive weights);
  * one step (teacher forced from the oracle's state rounded to FP32): for every term X in
    {A, B_R, B_c, E_mc, dR, dc}, |X_gpu - X_ref| <= 1e-5 * max(|X_ref|, X_abs) + slack, where X_abs
    is X with every summand replaced by its magnitude and slack is the oracle's bound on what a
    sample lying within 4e-6 s_max of a kink of S can change when FP32 places it on the other side;
  * free run (parity_util.check_free_run): every contour within |R_gpu - R_ref| <= 0.05 and
    |c_gpu - c_ref| <= 0.5 voxel of the oracle's own run; iteration counts identical, or within the
    range the oracle's stop rule allows when each decision within 1% of the convergence tolerance
    may go either way; the kept set equal to the oracle run's own, apart from decisions whose
    margins are smaller than the two runs' disagreement in the quantities compared;
  * exact energy: |E_gpu - E_ref| <= 1e-5 * max(|E_ref|, E_abs) at the GPU's final state;
    selection on given states: identical keep sets apart from decisions the oracle flags as within
    1e-4 (energy) or 1e-3 voxel (overlap) of a threshold.
"""
import sys

import copy

import numpy as np
import pytest

import oracle
import synth
from parity_util import check_free_run, expected_kinked_steps, oracle_reference, tol_check

pytestmark = pytest.mark.gpu

_FULL = {}


def full_workload(which):
    """The full-size slab or plane workload, generated once per session (a shallow copy, so a test
    may replace its parameter record)."""
    if which not in _FULL:
        _FULL[which] = synth.slab_config() if which == "slab" else synth.plane_config()
    return copy.copy(_FULL[which])


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


def make_ctx(snk, stream, wl, lanes=0, on_device=True, unroll=0, layout=0, tile=-1):
    import torch
    ctx = snk.Context(0, stream)
    ctx.set_params(wl.params)
    ctx.set_launch(lanes, unroll, layout)
    ctx.set_tile(tile)
    ctx.set_directions(wl.dirs)
    if on_device:
        raw = torch.from_numpy(np.ascontiguousarray(wl.raw)).to("cuda:0")
        ctx.load_volume(raw)
        ctx._raw = raw  # keep the borrowed buffer alive
    else:
        ctx.load_volume(wl.raw)
    return ctx


def extra_seeds(wl, n, rng):
    """Seeds spread over the whole volume (background, blob edges, near and on the faces)."""
    nx, ny, nz = wl.shape_xyz
    h = np.array(wl.params.spacing)
    ext = (np.array([nx, ny, nz]) - 1) * h
    s = rng.uniform(0.0, 1.0, size=(n, 3)) * ext
    s[: n // 8, 0] = rng.uniform(0.0, 1.5, size=n // 8)            # near the x = 0 face
    s[n // 8: n // 4, 1] = ext[1] - rng.uniform(0.0, 1.5, size=n // 4 - n // 8)
    if wl.params.dim == 2:
        s[:, 2] = 0.0
    return s


def one_step_parity(snk, stream, wl, prerun_iters, n_extra=56, seed=0, lanes=0, unroll=0, layout=0,
                    max_kinked=None, tile=-1):
    """Teacher-forced one-step parity of every active contour at each prerun count. Contour-steps
    whose slack is in use (a sample within the oracle's band around a kink of S, or for the
    image-gradient force around a voxel face) are counted: for Monte-Carlo sums at most the
    analytic expectation plus four Poisson deviations; for the exact and image-gradient forms at
    most `max_kinked` of the steps."""
    p = wl.params
    rng = np.random.default_rng(seed)
    seeds = np.concatenate([wl.seeds, extra_seeds(wl, n_extra, rng)]) if n_extra else wl.seeds
    ids = np.arange(len(seeds), dtype=np.uint32) * 7 + 3
    r0 = rng.uniform(oracle.r_geom_min(p.dim, p.dR), p.r_max, size=len(seeds))
    r0[: len(wl.seeds)] = p.r_init
    J = oracle.prepass(wl.raw, p)
    st = oracle.init_state(p, seeds, r0=r0, ids=ids, shape_zyx=wl.raw.shape)
    ctx = make_ctx(snk, stream, wl, lanes=lanes, unroll=unroll, layout=layout, tile=tile)
    ctx.load_seeds(seeds, r0=r0.astype(np.float32), ids=ids)
    worst = {}
    kinked = 0
    steps = 0
    done = 0
    expect = 0.0
    for target in prerun_iters:
        if target > done:
            oracle.evolve(J, p, wl.dirs, st, target - done)
            done = target
        # teacher forcing: both sides start from the oracle state rounded to FP32
        c32 = st.c.astype(np.float32).astype(np.float64)
        R32 = st.R.astype(np.float32)
        ref = st.copy()
        ref.c[:] = c32
        ref.R[:] = R32.astype(np.float64)
        active = (ref.status & 0x0F) == oracle.ACTIVE
        tr, _ = oracle.evolve(J, p, wl.dirs, ref, 1, trace=True)
        ctx.set_state(c32, R32, st.iters, st.status, st.streak)
        say(f"  one-step parity {wl.name}: after {target} iterations, {int(active.sum())} active")
        g = ctx.trace_step()
        a = np.where(active)[0]
        assert np.all(g[a, 10] == tr[a, 29])  # same iteration number n
        d = p.dim
        checks = [("A", g[a, 0], tr[a, 0], tr[a, 5], 0.0), ("B_R", g[a, 1], tr[a, 1], tr[a, 6], tr[a, 20]),
                  ("E_mc", g[a, 5], tr[a, 10], tr[a, 11], 0.0), ("dR", g[a, 6], tr[a, 12], tr[a, 13], tr[a, 24])]
        for k in range(d):
            checks.append((f"B_c{k}", g[a, 2 + k], tr[a, 2 + k], tr[a, 7 + k], tr[a, 21 + k]))
            checks.append((f"dc{k}", g[a, 7 + k], tr[a, 14 + k], tr[a, 17 + k], tr[a, 25 + k]))
        for name, gv, rv, ra, sl in checks:
            worst[name] = max(worst.get(name, 0.0), tol_check(f"{name} at n={target}", gv, rv, ra, sl))
        kinked += int((tr[a, 28] > 0).sum())
        steps += len(a)
        expect += expected_kinked_steps(p, tr[a, 30])
        # the state after the step matches too
        gs = ctx.get_state()
        assert np.all(gs["iters"][a] == ref.iters[a])
        # a sample on the other side of a kink moves the state by up to the step's slack
        assert np.all(np.abs(gs["radii"][a] - ref.R[a]) < 1e-4 + tr[a, 24])
        slack_c = np.linalg.norm(tr[a, 25:25 + d], axis=1)
        assert np.all(np.linalg.norm(gs["centers"][a] - ref.c[a], axis=1) < 1e-4 + slack_c)
    ctx.close()
    say(f"  worst err/tol: " + ", ".join(f"{k} {v:.3f}" for k, v in worst.items()) +
        f"; contour-steps with a near-kink sample: {kinked}/{steps} (Monte-Carlo expectation {expect:.2f})")
    if p.flags & 6:
        assert kinked <= (0.3 if max_kinked is None else max_kinked) * steps
    else:
        assert kinked <= expect + 4.0 * np.sqrt(expect) + 1.0
    return worst


# ------------------------------------------------------------------------------------------------

@pytest.mark.parametrize("which", ["tiny-u8", "aniso-u16", "plane-u8", "f32"])
def test_prepass_parity(snk, stream, which):
    rng = np.random.default_rng(1)
    if which == "tiny-u8":
        wl = synth.tiny_config()
    elif which == "aniso-u16":
        wl = synth.slab_config(n_target=60, shape_xyz=(100, 77, 23), n_iter=10)
    elif which == "plane-u8":
        wl = synth.plane_config(n_target=300, size=300, n_iter=10)
    else:
        wl = synth.tiny_config()
        wl.raw = rng.normal(50.0, 20.0, size=(19, 70, 131)).astype(np.float32)
        wl.params = wl.params.replace(sigma_pre=1.7, spacing=(1.0, 1.3, 0.8))
    say(f"prepass parity: {which} {wl.raw.shape} {wl.raw.dtype}")
    for on_device in (True, False):
        ctx = make_ctx(snk, stream, wl, on_device=on_device)
        ctx.prepass()
        got = ctx.read_volume(wl.raw.shape)
        ctx.close()
        ref = oracle.prepass(wl.raw, wl.params)
        I = (wl.raw.astype(np.float64) - wl.params.i_offset) * wl.params.i_scale
        err = np.max(np.abs(got - ref))
        assert err <= 2e-6 * np.max(np.abs(I)), (which, err)


def test_one_step_parity_tiny(snk, stream):
    say("one-step parity tiny (64^3 u8, D 162, M 32)")
    one_step_parity(snk, stream, synth.tiny_config(), [0, 1, 7, 40, 99])


def test_one_step_parity_aniso_u16(snk, stream):
    wl = synth.slab_config(n_target=40, shape_xyz=(96, 80, 40), n_iter=50)
    say("one-step parity anisotropic u16 (h = 1,1,2; D 642, M 64)")
    one_step_parity(snk, stream, wl, [0, 3, 30])


@pytest.mark.parametrize("lanes,layout", [(0, 0), (64, 2), (16, 1), (32, 2), (64, 4), (32, 4)])
def test_one_step_parity_2d(snk, stream, lanes, layout):
    wl = synth.plane_config(n_target=120, size=256, n_iter=50)
    say(f"one-step parity 2D (256^2 u8, D 64, M 16), lanes {lanes}, layout {layout}")
    one_step_parity(snk, stream, wl, [0, 2, 25], n_extra=40, lanes=lanes, layout=layout)


@pytest.mark.parametrize("lanes,unroll,layout", [(16, 1, 0), (16, 2, 1), (32, 1, 2), (32, 2, 3), (64, 1, 1),
                                                 (64, 2, 2), (64, 4, 3), (128, 1, 3), (128, 2, 1), (128, 4, 2),
                                                 (256, 1, 2), (256, 2, 0), (16, 2, 4), (64, 2, 4), (128, 4, 4)])
def test_one_step_parity_launch_shapes(snk, stream, lanes, unroll, layout):
    """Every contour group size (several contours per wave, one wave, 2 and 4 waves per contour),
    one, two or four pair-points in flight, and every volume layout."""
    say(f"one-step parity tiny, {lanes} lanes per contour, {unroll} pair-points in flight, layout {layout}")
    one_step_parity(snk, stream, synth.tiny_config(), [0, 12], n_extra=24, lanes=lanes, unroll=unroll,
                    layout=layout)


def test_layouts_bitwise(snk, stream):
    """The quad records and column pairs hold exact copies of the volume and the arithmetic is the
    same, so a free run reads identical results from every layout (same launch shape otherwise)."""
    wl = synth.tiny_config()
    say("free run tiny: plain vs quad vs 64-bit-addressed plain vs column-pair layout")
    outs = []
    for layout in (1, 2, 3, 4):
        ctx = make_ctx(snk, stream, wl, lanes=128, unroll=1, layout=layout)
        ctx.load_seeds(wl.seeds, ids=wl.ids)
        ctx.evolve(wl.n_iter)
        ctx.finalize()
        outs.append(ctx.read())
        ctx.close()
    for o in outs[1:]:
        for k in ("radii", "centers", "e_mc", "e_vox", "iters", "status", "keep"):
            assert np.array_equal(outs[0][k], o[k]), k


@pytest.mark.parametrize("size", [256, 203])
def test_layouts_bitwise_2d(snk, stream, size):
    """2D: the column pairs and the quad records hold exact copies of the image, so a free run reads
    identical results from the plain, quad, 64-bit-addressed and column-pair layouts; the automatic
    layout of a 2D image is the column pairs, and with an LDS box the iterations whose ball does not fit
    read the plain copy. A ragged size puts cells on the last row and column."""
    wl = synth.plane_config(n_target=120, size=size, n_iter=60)
    say(f"free run 2D {size}^2: plain vs quad vs 64-bit plain vs column pairs, with and without LDS boxes")
    outs = []
    runs = [(layout, lanes, unroll, -1) for layout in (1, 2, 3, 4, 0) for lanes, unroll in ((64, 2), (32, 4), (16, 1))]
    # an LDS box with the automatic layout: the iterations whose ball does not fit read the plain copy
    runs += [(0, 64, 2, 1024), (4, 64, 2, 2048)]
    for layout, lanes, unroll, tile in runs:
        ctx = make_ctx(snk, stream, wl, lanes=lanes, unroll=unroll, layout=layout, tile=tile)
        ctx.load_seeds(wl.seeds, ids=wl.ids)
        ctx.evolve(wl.n_iter)
        tm = ctx.get_timing()
        if layout == 0 and tile < 0:
            assert tm["layout"] == 3, tm["layout"]   # column pairs
        if tile > 0:
            assert tm["layout"] == 1 and tm["tile_voxels"] == tile, tm
        ctx.finalize()
        outs.append(((lanes, unroll), ctx.read()))
        ctx.close()
    for shape, o in outs:
        ref = next(r for sh, r in outs if sh == shape)
        for k in ("radii", "centers", "e_mc", "e_vox", "iters", "status", "keep"):
            assert np.array_equal(ref[k], o[k]), (shape, k)


@pytest.mark.parametrize("which", ["tiny", "aniso", "plane"])
def test_pair_points_in_flight_bitwise(snk, stream, which):
    """A lane consumes its pair-points in the same order whatever number it keeps in flight (past
    the last one, masked slots add exact zeros), so free runs with 1, 2 and 4 in flight are
    identical for the same lanes per contour, with and without LDS boxes."""
    if which == "tiny":
        wl = synth.tiny_config()
    elif which == "aniso":
        wl = synth.slab_config(n_target=40, shape_xyz=(96, 80, 40), n_iter=80)
    else:
        wl = synth.plane_config(n_target=120, size=256, n_iter=80)
    layout = 2 if wl.params.dim == 3 else 1
    for lanes, tile in ((64, 0), (128, 0), (128, 3000)):
        ref = None
        for unroll in (1, 2, 4):
            say(f"pair-points in flight {which}: lanes {lanes} pairs {unroll} tile {tile}")
            ctx = make_ctx(snk, stream, wl, lanes=lanes, unroll=unroll, layout=layout, tile=tile)
            ctx.load_seeds(wl.seeds, ids=wl.ids)
            ctx.evolve(wl.n_iter)
            out = ctx.read()
            assert ctx.get_timing()["pairs_in_flight"] == unroll
            ctx.close()
            if ref is None:
                ref = out
                continue
            for k in ("radii", "centers", "e_mc", "iters", "status"):
                assert np.array_equal(out[k], ref[k]), (k, lanes, unroll, tile)


@pytest.mark.parametrize("which", ["tiny", "aniso", "plane"])
def test_lds_box_bitwise(snk, stream, which):
    """LDS boxes hold exact copies of the volume and the corner arithmetic is unchanged, so a free
    run gives identical results with boxes of any capacity (tiny ones: most iterations read the
    volume; mid-sized ones: iterations switch between box and volume as R changes) and without
    them, for every whole-wave launch shape, from quad records and column pairs alike in 3D; seeds
    near and on the faces take the clamped path."""
    rng = np.random.default_rng(11)
    if which == "tiny":
        wl = synth.tiny_config()
    elif which == "aniso":
        wl = synth.slab_config(n_target=40, shape_xyz=(96, 80, 40), n_iter=60)
    else:
        wl = synth.plane_config(n_target=120, size=256, n_iter=60)
    seeds = np.concatenate([wl.seeds, extra_seeds(wl, 24, rng)])
    ids = np.arange(len(seeds), dtype=np.uint32)
    n_iter = min(wl.n_iter, 60)
    layouts = (2, 4) if wl.params.dim == 3 else (1,)
    for lanes, unroll in ((64, 2), (128, 1), (128, 4), (256, 2)):
        ref = None
        for tile, layout in [(t, lay) for t in (0, 512, 3000, 12000, -1) for lay in layouts]:
            say(f"lds box {which}: lanes {lanes} pairs {unroll} tile {tile} layout {layout}")
            ctx = make_ctx(snk, stream, wl, lanes=lanes, unroll=unroll, layout=layout, tile=tile)
            ctx.load_seeds(seeds, ids=ids)
            ctx.evolve(n_iter)
            got = ctx.get_state()
            e_mc = ctx.read()["e_mc"]
            used = ctx.get_timing()["tile_voxels"]
            ctx.close()
            if tile == -1:
                # a few contours per CU fit the L2: the automatic shape stages no boxes
                assert used == 0
            if ref is None:
                ref = (got, e_mc)
                continue
            for k in got:
                assert np.array_equal(got[k], ref[0][k]), (k, lanes, unroll, tile)
            assert np.array_equal(e_mc, ref[1]), (lanes, unroll, tile)


def test_one_step_parity_many_rays(snk, stream):
    """More antithetic pairs than lanes (M = 128 on one wave): a block of draws takes two passes."""
    wl = synth.tiny_config()
    wl.params = wl.params.replace(n_rays=128, n_radial=8)
    say("one-step parity tiny, M = 128, L = 8, 1 wave")
    one_step_parity(snk, stream, wl, [0, 5], n_extra=16, lanes=64, unroll=2)


def test_one_step_parity_unrotated_and_odd_sizes(snk, stream):
    wl = synth.tiny_config()
    wl.params = wl.params.replace(flags=1, n_rays=6, n_radial=5)
    say("one-step parity: rotation off, M = 6, L = 5 (ragged thread mapping)")
    one_step_parity(snk, stream, wl, [0, 4], n_extra=16)


@pytest.mark.parametrize("which,lanes,layout", [("tiny", 0, 0), ("tiny", 64, 3), ("tiny", 16, 1),
                                                 ("aniso", 0, 0), ("plane", 0, 0), ("plane", 32, 3)])
def test_one_step_parity_exact(snk, stream, which, lanes, layout):
    """Exact lattice sums (flags bit 1) against the oracle's exact mode, teacher forced; contours
    near the faces take the clamp-to-edge path."""
    if which == "tiny":
        wl = synth.tiny_config()
    elif which == "aniso":
        wl = synth.slab_config(n_target=60, shape_xyz=(100, 77, 23), n_iter=10)
    else:
        wl = synth.plane_config(n_target=120, size=256, n_iter=50)
    wl.params = wl.params.replace(flags=2)
    say(f"one-step parity, exact sums: {which}, lanes {lanes}, layout {layout}")
    # lattice points share radii by symmetry, so more contour-steps have a point within the kink
    # tolerance than with random samples (their effect is in the slack either way)
    one_step_parity(snk, stream, wl, [0, 6], n_extra=32, lanes=lanes, layout=layout, max_kinked=0.3)


def test_free_run_exact(snk, stream):
    wl = synth.tiny_config()
    wl.params = wl.params.replace(flags=2)
    say("free run tiny, exact sums: 100 iterations")
    got = free_run(snk, stream, wl)
    ref = oracle_reference(wl.raw, wl.params, wl.dirs, wl.seeds, wl.n_iter, ids=wl.ids)
    check_free_run(got, ref, wl.params, "tiny exact sums")


@pytest.mark.parametrize("which,lanes,layout,tile", [("tiny", 0, 0, -1), ("tiny", 64, 1, 0), ("tiny", 256, 2, 0),
                                                      ("aniso", 0, 0, -1), ("aniso", 128, 1, 2048),
                                                      ("plane", 0, 0, -1), ("plane", 128, 1, 0)])
def test_one_step_parity_gradient_form(snk, stream, which, lanes, layout, tile):
    """Centre force in its image-gradient form (flags bit 2) against the oracle's, teacher forced,
    with and without LDS boxes; contours near and beyond the faces take the clamped path, where
    the gradient along a clamped axis is zero."""
    if which == "tiny":
        wl = synth.tiny_config()
    elif which == "aniso":
        wl = synth.slab_config(n_target=60, shape_xyz=(100, 77, 23), n_iter=10)
    else:
        wl = synth.plane_config(n_target=120, size=256, n_iter=50)
    wl.params = wl.params.replace(flags=4)
    say(f"one-step parity, gradient-form centre force: {which}, lanes {lanes}, layout {layout}, tile {tile}")
    # samples next to a voxel face also count as near a kink (the normal derivative jumps there)
    one_step_parity(snk, stream, wl, [0, 6], n_extra=48, lanes=lanes, layout=layout, tile=tile, max_kinked=0.3)


def test_gradient_form_leaves_energy_and_radius_terms(snk, stream):
    """Flags bit 2 changes only the centre sums: A, B_R, E_mc and the radius step of one iteration
    are bit-identical to the weight form's at the same state and launch shape."""
    wl = synth.tiny_config()
    rng = np.random.default_rng(4)
    seeds = np.concatenate([wl.seeds, extra_seeds(wl, 24, rng)])
    ctx = make_ctx(snk, stream, wl, lanes=128, unroll=2, layout=2)
    ctx.load_seeds(seeds)
    ctx.evolve(3)
    s = ctx.get_state()
    ctx.close()
    rows = []
    for flags in (0, 4):
        w = copy.copy(wl)
        w.params = wl.params.replace(flags=flags)
        ctx = make_ctx(snk, stream, w, lanes=128, unroll=2, layout=2)
        ctx.load_seeds(seeds)
        ctx.set_state(s["centers"], s["radii"], s["iters"], s["status"], s["streak"])
        rows.append(ctx.trace_step())
        ctx.close()
    assert np.any(rows[0][:, 2:5] != rows[1][:, 2:5])
    for col in (0, 1, 5, 6):
        assert np.array_equal(rows[0][:, col], rows[1][:, col]), col


def test_free_run_gradient_form(snk, stream):
    wl = synth.tiny_config()
    wl.params = wl.params.replace(flags=4)
    say("free run tiny, gradient-form centre force: 100 iterations")
    got = free_run(snk, stream, wl)
    ref = oracle_reference(wl.raw, wl.params, wl.dirs, wl.seeds, wl.n_iter, ids=wl.ids)
    check_free_run(got, ref, wl.params, "tiny gradient form")


def free_run(snk, stream, wl, seeds=None, ids=None, lanes=0, chunks=None):
    seeds = wl.seeds if seeds is None else seeds
    ctx = make_ctx(snk, stream, wl, lanes=lanes)
    ctx.load_seeds(seeds, ids=ids)
    for k in (chunks or [wl.n_iter]):
        ctx.evolve(k)
    ctx.finalize()
    out = ctx.read()
    out["timing"] = ctx.get_timing()
    ctx.close()
    return out


def test_free_run_tiny(snk, stream):
    wl = synth.tiny_config()
    say("free run tiny: 100 iterations, then exact energy and selection")
    got = free_run(snk, stream, wl)
    ref = oracle_reference(wl.raw, wl.params, wl.dirs, wl.seeds, wl.n_iter, ids=wl.ids)
    r = check_free_run(got, ref, wl.params, "tiny")
    assert r["differing_iters"] == 0
    assert got["timing"]["evolved"] == ref["evolved"]
    # the selection on the GPU's own final state equals the oracle's greedy there too
    e_ref, _ = oracle.energy_vox(ref["J"], wl.params, got["centers"], got["radii"].astype(np.float64))
    amb = oracle.cull_ambiguity(wl.params, got["centers"], got["radii"], e_ref)
    keep_ref = oracle.cull(wl.params, got["centers"], got["radii"], got["e_vox"].astype(np.float64),
                           got["status"], wl.ids)
    ok = amb == 0
    assert np.array_equal(got["keep"][ok], keep_ref[ok])


def test_free_run_2d(snk, stream):
    wl = synth.plane_config(n_target=200, size=320, n_iter=60)
    say("free run 2D: 320^2, 60 iterations")
    got = free_run(snk, stream, wl)
    ref = oracle_reference(wl.raw, wl.params, wl.dirs, wl.seeds, wl.n_iter, ids=wl.ids)
    check_free_run(got, ref, wl.params, "2D 320^2")


@pytest.mark.parametrize("n", [1500, 9000])
def test_selection_matches_greedy_dense(snk, stream, n):
    """Dense random contours (many overlapping chains): the GPU's parallel rounds (one workgroup
    at 1,500 contours; grid-wide rounds then the one-workgroup finish at 9,000) equal the
    oracle's sequential greedy on the GPU's own energies."""
    wl = synth.tiny_config()
    p = wl.params.replace(e0=-0.002)
    wl.params = p
    rng = np.random.default_rng(5)
    seeds = rng.uniform(2.0, 61.0, size=(n, 3))
    R = rng.uniform(5.0, 9.0, size=n).astype(np.float32)
    ctx = make_ctx(snk, stream, wl)
    ctx.load_seeds(seeds, r0=R)
    st = np.full(n, oracle.MAXITER, np.uint8)
    st[::17] = oracle.OUT
    st[::23] = oracle.CONVERGED | oracle.CLAMPED
    ctx.set_state(seeds, R, np.full(n, 5, np.int32), st)
    say(f"selection parity: {n} dense contours")
    ctx.finalize()
    got = ctx.read()
    ctx.close()
    keep_ref = oracle.cull(p, got["centers"], got["radii"], got["e_vox"].astype(np.float64), st,
                           np.arange(n, dtype=np.uint32))
    amb = oracle.cull_ambiguity(p, got["centers"], got["radii"], got["e_vox"].astype(np.float64))
    ok = amb == 0
    assert got["keep"].sum() >= 10
    assert np.array_equal(got["keep"][ok], keep_ref[ok]), (np.where(got["keep"] != keep_ref)[0][:10])
    J = oracle.prepass(wl.raw, p)
    e_ref, e_abs = oracle.energy_vox(J, p, got["centers"], got["radii"].astype(np.float64))
    tol_check("E_vox dense", got["e_vox"], e_ref, e_abs, 0.0, rel=1e-5)


def test_determinism_split_and_order(snk, stream):
    """Bit-identical reruns; evolve(30)+evolve(70) == evolve(100); per-id results do not depend
    on the seed order."""
    wl = synth.tiny_config()
    say("determinism / split / order")
    a = free_run(snk, stream, wl)
    b = free_run(snk, stream, wl)
    c = free_run(snk, stream, wl, chunks=[30, 70])
    for k in ("radii", "centers", "e_mc", "e_vox", "iters", "status", "keep"):
        assert np.array_equal(a[k], b[k]), k
        assert np.array_equal(a[k], c[k]), k
    perm = np.random.default_rng(3).permutation(len(wl.seeds))
    d = free_run(snk, stream, wl, seeds=wl.seeds[perm], ids=wl.ids[perm])
    for k in ("radii", "centers", "e_mc", "e_vox", "iters", "status", "keep"):
        assert np.array_equal(a[k][perm], d[k]), k


def test_edge_cases(snk, stream):
    wl = synth.tiny_config()
    p = wl.params
    say("edge cases: empty seed set, seeds outside, radius clamps, 1 iteration")
    ctx = make_ctx(snk, stream, wl)
    ctx.load_seeds(np.zeros((0, 3)))
    ctx.evolve(5)
    ctx.finalize()
    assert len(ctx.read()["radii"]) == 0
    seeds = np.array([[-3.0, 10.0, 10.0], [70.0, 5.0, 5.0], [0.0, 0.0, 0.0], [63.0, 63.0, 63.0], [30.0, 31.0, 29.0]])
    r0 = np.array([5.0, 5.0, 0.1, 1e3, 7.0], np.float32)
    ctx.load_seeds(seeds, r0=r0)
    s = ctx.get_state()
    assert list(s["status"][:2]) == [oracle.OUT, oracle.OUT]
    lo = oracle.r_geom_min(3, p.dR)
    assert abs(s["radii"][2] - lo) < 1e-5 and abs(s["radii"][3] - p.r_max) < 1e-4
    ctx.evolve(1)
    g = ctx.get_state()
    assert list(g["iters"]) == [0, 0, 1, 1, 1]
    J = oracle.prepass(wl.raw, p)
    st = oracle.init_state(p, seeds, r0=r0, shape_zyx=wl.raw.shape)
    oracle.evolve(J, p, wl.dirs, st, 1)
    assert np.max(np.abs(g["radii"] - st.R)) < 1e-4
    with pytest.raises(snk.SnkError):
        ctx.set_state(seeds[:2], r0[:2], np.zeros(2, np.int32), np.zeros(2, np.uint8))
    bad = p.replace(n_rays=7)
    with pytest.raises(snk.SnkError):
        ctx.set_params(bad)
    ctx.close()
    # seeds go up from one pinned staging buffer without a host wait: back-to-back loads (each
    # reusing the buffer while the previous upload may still be in flight) leave the last one
    ctx = make_ctx(snk, stream, wl)
    many = np.random.default_rng(5).uniform(8.0, 56.0, size=(4000, 3))
    ctx.load_seeds(many)
    ctx.load_seeds(wl.seeds, ids=wl.ids)
    ctx.evolve(3)
    a = ctx.get_state()
    ctx.load_seeds(wl.seeds, ids=wl.ids)
    ctx.evolve(3)
    b = ctx.get_state()
    for k in a:
        assert np.array_equal(a[k], b[k]), k
    ctx.close()


def test_full_size_slab_sampled(snk, stream):
    """The benchmark workload at full size (512x512x128 u16, ~2,000 nuclei, D 642, M 64) in the
    benchmark's launch configuration: one-step parity of every contour from the seeds and after
    20 iterations, and a 20-iteration free run of all contours."""
    wl = full_workload("slab")
    say(f"full-size slab: {wl.name}")
    worst = one_step_parity(snk, stream, wl, [0, 20], n_extra=0)
    assert worst
    got = free_run(snk, stream, wl, chunks=[20])
    J = oracle.prepass(wl.raw, wl.params)
    st = oracle.init_state(wl.params, wl.seeds, ids=wl.ids)
    oracle.evolve(J, wl.params, wl.dirs, st, 20)
    assert np.array_equal(got["iters"], st.iters)
    assert np.max(np.abs(got["radii"] - st.R)) <= 0.05
    assert np.max(np.linalg.norm(got["centers"] - st.c, axis=1)) <= 0.5


def test_full_size_slab_free_run(snk, stream):
    """The benchmark workload end to end as the benchmark runs it (automatic launch shape, all 500
    iterations as one evolve call, then exact energy and selection) against the oracle's own
    500-iteration run of the same contours: every contour's iteration count within the oracle's
    stop range, radii and centres of all contours, E_vox at 1e-5, and the kept set against the
    oracle run's kept set (check_free_run)."""
    wl = full_workload("slab")
    p = wl.params
    say(f"full-size slab free run: {wl.name}, {wl.n_iter} iterations")
    ctx = make_ctx(snk, stream, wl)
    ctx.load_seeds(wl.seeds, ids=wl.ids)
    l0 = ctx.get_timing()["evolve_launches"]
    ctx.evolve(wl.n_iter)
    ctx.finalize()
    got = ctx.read()
    tm = ctx.get_timing()
    ctx.close()
    say(f"  launch lanes {tm['lanes_per_contour']} pairs {tm['pairs_in_flight']} layout {tm['layout']} "
        f"tile {tm['tile_voxels']}, {tm['evolve_launches'] - l0} launches")
    assert tm["evolve_launches"] - l0 == 2
    ref = oracle_reference(wl.raw, p, wl.dirs, wl.seeds, wl.n_iter, ids=wl.ids)
    r = check_free_run(got, ref, p, "slab 500 iterations")
    assert r["differing_iters"] <= 0.01 * r["contours"]


def test_full_size_plane_free_run(snk, stream):
    """The 2D workload at full size (8192^2 u8, 40,000 cells, D 64, M 16, L 16) for all 300
    iterations in the benchmark's launch configuration, then exact energy and selection, against
    the oracle's own 300-iteration run (check_free_run)."""
    wl = full_workload("plane")
    p = wl.params
    say(f"full-size plane free run: {wl.name}, {wl.n_iter} iterations")
    got = free_run(snk, stream, wl)
    ref = oracle_reference(wl.raw, p, wl.dirs, wl.seeds, wl.n_iter, ids=wl.ids)
    r = check_free_run(got, ref, p, "plane 300 iterations")
    assert r["differing_iters"] <= 0.01 * r["contours"]


def test_full_size_split_calls_identical(snk, stream):
    """The benchmark workload in its automatic shape (LDS boxes, each call of 64 or more iterations
    as two launches): the same 500 iterations split into calls of different lengths give
    bit-identical contours."""
    wl = full_workload("slab")
    say(f"split calls: {wl.name}")
    ref, tm_ref = None, None
    for chunks in ([500], [200, 300], [256, 244], [300, 200], [100, 100, 100, 200]):
        ctx = make_ctx(snk, stream, wl)
        ctx.load_seeds(wl.seeds, ids=wl.ids)
        for k in chunks:
            ctx.evolve(k)
        out = ctx.read()
        tm = ctx.get_timing()
        ctx.close()
        if ref is None:
            ref, tm_ref = out, tm
            continue
        for k in ("radii", "centers", "e_mc", "iters", "status"):
            assert np.array_equal(out[k], ref[k]), (chunks, k)
    assert tm_ref["lanes_per_contour"] == 128 and tm_ref["tile_voxels"] > 0


def test_full_size_plane_sampled(snk, stream):
    """The 2D workload at full size (8192^2 u8, 40,000 cells, D 64, M 16) in the benchmark's launch
    configuration: one-step parity of every contour from the seeds and after 20 iterations, and a
    20-iteration free run of all contours."""
    wl = full_workload("plane")
    say(f"full-size plane: {wl.name}")
    worst = one_step_parity(snk, stream, wl, [0, 20], n_extra=0)
    assert worst
    got = free_run(snk, stream, wl, chunks=[20])
    J = oracle.prepass(wl.raw, wl.params)
    st = oracle.init_state(wl.params, wl.seeds, ids=wl.ids, shape_zyx=wl.raw.shape)
    oracle.evolve(J, wl.params, wl.dirs, st, 20)
    same = got["iters"] == st.iters
    assert same.mean() >= 0.999
    assert np.max(np.abs(got["radii"] - st.R)[same]) <= 0.05
    assert np.max(np.linalg.norm(got["centers"] - st.c, axis=1)[same]) <= 0.5
