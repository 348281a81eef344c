"""GPU tests of the batch / serving engine through the C ABI.

Bars: with the same launch shape the engine's batched and served paths reproduce the plain
per-volume path bit for bit (same kernels, same per-contour reduction order); against the FP64
oracle each job meets the free-run bar (|dR| <= 0.05, |dc| <= 0.5 voxel, same iteration counts);
a job's result is identical alone and in a mix; admission respects the HBM budget.
"""
import sys

import numpy as np
import pytest

import oracle
import synth
from parity_util import check_free_run, oracle_reference

pytestmark = pytest.mark.gpu

KEYS = ("radii", "centers", "e_mc", "e_vox", "iters", "status", "keep")


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
def jobs():
    """Small uneven batch: cubic u16 subvolumes of different edge, nucleus count and table size."""
    return synth.subvolume_batch(n_vol=6, edge_lo=32, edge_hi=72, n_iter=40)


def plain(snk, wl, lanes, unroll):
    import torch
    ctx = snk.Context(0, torch.cuda.current_stream())
    ctx.set_params(wl.params)
    ctx.set_launch(lanes, unroll, 0)
    ctx.set_directions(wl.dirs)
    ctx.load_volume(wl.raw)
    ctx.load_seeds(wl.seeds, ids=wl.ids)
    ctx.evolve(wl.n_iter)
    ctx.finalize()
    out = ctx.read()
    ctx.close()
    return out


def test_batched_equals_plain_and_oracle(snk, jobs):
    say("engine batched: " + ", ".join(w.name for w in jobs))
    eng = snk.Engine(0, None, 8 << 30)
    eng.set_launch(256, 2, 1)
    ids = [eng.submit(w.params, w.dirs, w.raw, w.seeds, ids=w.ids, n_iter=w.n_iter) for w in jobs]
    eng.run()
    stats = eng.get_stats()
    assert stats["completed"] == len(jobs) and stats["graph_replays"] == 1
    for w, j in zip(jobs, ids):
        got = eng.read(j)
        ref = plain(snk, w, 256, 2)
        for k in KEYS:
            assert np.array_equal(got[k], ref[k]), (w.name, k)
        ref = oracle_reference(w.raw, w.params, w.dirs, w.seeds, w.n_iter, ids=w.ids)
        check_free_run(got, ref, w.params, f"batched {w.name}")
    # replay of the captured graph gives the same results
    first = {j: eng.read(j) for j in ids}
    eng.run()
    assert eng.get_stats()["graph_replays"] == 2
    for j in ids:
        again = eng.read(j)
        for k in KEYS:
            assert np.array_equal(again[k], first[j][k])
    eng.close()


def test_autotuned_batched_within_tolerance(snk, jobs):
    say("engine batched with per-class autotuning")
    eng = snk.Engine(0, None, 8 << 30)
    ids = [eng.submit(w.params, w.dirs, w.raw, w.seeds, ids=w.ids, n_iter=w.n_iter) for w in jobs]
    eng.run()
    s = eng.get_stats()
    say(f"  tuned shape of the last class: lanes {s['lanes_per_contour']}, pair-points in flight "
        f"{s['pairs_in_flight']}, persistent {s['persistent']}, layout {s['layout']}")
    for w, j in zip(jobs, ids):
        got = eng.read(j)
        ref = plain(snk, w, 256, 2)
        assert np.array_equal(got["iters"], ref["iters"])
        assert np.max(np.abs(got["radii"] - ref["radii"]), initial=0.0) <= 0.05
    # one tuned shape per launch class (dim, D, M, L), each picked among lanes, pair-points, LDS box
    # capacities and work-queue residencies
    classes = {(3, w.params.n_dirs, w.params.n_rays, 16) for w in jobs}
    shapes = eng.tuned_shapes()
    say(f"  tuned classes: {shapes}")
    assert {(r["dim"], r["n_dirs"], r["n_rays"], r["n_radial"]) for r in shapes} == classes
    for r in shapes:
        assert r["lanes_per_contour"] in (64, 128, 256) and r["pairs_in_flight"] in (1, 2)
        assert r["persistent"] in (0, 1) and r["tile_voxels"] in (0, 2048, 4224, 8192)
        assert r["workgroups_per_cu"] >= 0 and r["trials"] >= 18 and r["trial_us"] > 0
    eng.close()


@pytest.mark.parametrize("shape", [(128, 2, 1, 4224, 2), (256, 1, 0, 2048, 0), (64, 2, 1, 8192, 0)])
def test_batched_lds_box_and_queue_equal_plain(snk, jobs, shape):
    """Forced gather tile (LDS box per workgroup) and work-queue residency: the batched run equals the
    plain path with the same lanes and pair-points bit for bit (a box changes where corners are
    read, never the arithmetic)."""
    lanes, unroll, pers, tile, per_cu = shape
    say(f"engine batched with an LDS box: lanes {lanes}, pair-points {unroll}, persistent {pers}, "
        f"box {tile}, workgroups per CU {per_cu}")
    eng = snk.Engine(0, None, 8 << 30)
    eng.set_launch(lanes, unroll, pers)
    eng.set_tile(tile, per_cu)
    ids = [eng.submit(w.params, w.dirs, w.raw, w.seeds, ids=w.ids, n_iter=w.n_iter) for w in jobs]
    eng.run()
    for w, j in zip(jobs, ids):
        got = eng.read(j)
        ref = plain(snk, w, lanes, unroll)
        for k in KEYS:
            assert np.array_equal(got[k], ref[k]), (w.name, k)
    eng.close()


def test_engine_set_tile_errors(snk, jobs):
    eng = snk.Engine(0, None, 1 << 30)
    with pytest.raises(snk.SnkError) as ex:
        eng.set_tile(2048, 0)                    # no forced shape
    assert ex.value.code == snk.SNK_ESTATE
    eng.set_launch(128, 1, 1)
    with pytest.raises(snk.SnkError) as ex:
        eng.set_tile(20000, 0)
    assert ex.value.code == snk.SNK_EINVAL
    eng.close()


def test_served_alone_equals_mix(snk, jobs):
    """Continuous batching: a job gives the same result alone and when other jobs arrive while it
    runs (and it joins a running mix)."""
    say("engine served: alone vs mix")
    eng = snk.Engine(0, None, 8 << 30)
    eng.set_launch(128, 1, 1)
    target = jobs[2]
    j0 = eng.submit(target.params, target.dirs, target.raw, target.seeds, ids=target.ids, n_iter=target.n_iter)
    done = []
    while j0 not in done:
        eng.step(7)
        done += eng.poll()
    alone = eng.read(j0)
    # mix: others first, the target arrives after two steps, more arrive later
    others = [eng.submit(w.params, w.dirs, w.raw, w.seeds, ids=w.ids, n_iter=w.n_iter) for w in jobs[:2]]
    eng.step(7)
    eng.step(7)
    j1 = eng.submit(target.params, target.dirs, target.raw, target.seeds, ids=target.ids, n_iter=target.n_iter)
    eng.step(7)
    late = [eng.submit(w.params, w.dirs, w.raw, w.seeds, ids=w.ids, n_iter=w.n_iter) for w in jobs[3:]]
    pending = set(others + late + [j1])
    guard = 0
    while pending and guard < 200:
        eng.step(7)
        pending -= set(eng.poll())
        guard += 1
    assert not pending
    mixed = eng.read(j1)
    for k in KEYS:
        assert np.array_equal(alone[k], mixed[k]), k
    ref = plain(snk, target, 128, 1)
    for k in KEYS:
        assert np.array_equal(alone[k], ref[k]), k
    # every served job against the oracle's own run of it
    for w, j in zip(jobs[:2] + [target] + jobs[3:], others + [j1] + late):
        oref = oracle_reference(w.raw, w.params, w.dirs, w.seeds, w.n_iter, ids=w.ids)
        check_free_run(eng.read(j), oref, w.params, f"served {w.name}")
    s = eng.get_stats()
    assert s["bytes_in_use"] == 0 and s["running"] == 0
    eng.close()


def test_admission_by_budget(snk, jobs):
    say("engine admission by HBM budget")
    big = max(jobs, key=lambda w: w.raw.size)
    eng = snk.Engine(0, None, 1 << 20)
    with pytest.raises(snk.SnkError) as ex:
        eng.submit(big.params, big.dirs, big.raw, big.seeds, n_iter=5)
    assert ex.value.code == snk.SNK_EBUSY
    eng.close()
    # budget for about one job: the second waits until the first completes
    small = min(jobs, key=lambda w: w.raw.size)
    probe = snk.Engine(0, None, 8 << 30)
    probe.submit(small.params, small.dirs, small.raw, small.seeds, n_iter=1000)
    probe.step(1)
    one = probe.get_stats()["bytes_in_use"]
    probe.close()
    assert one > 0
    eng = snk.Engine(0, None, int(one * 1.5))
    a = eng.submit(small.params, small.dirs, small.raw, small.seeds, n_iter=10)
    b = eng.submit(small.params, small.dirs, small.raw, small.seeds, n_iter=10)
    eng.step(20)
    s = eng.get_stats()
    assert s["completed"] == 1 and s["pending"] == 1, s
    eng.step(20)
    assert eng.get_stats()["completed"] == 2
    ra, rb = eng.read(a), eng.read(b)
    for k in KEYS:
        assert np.array_equal(ra[k], rb[k])
    eng.close()
    # releasing a finished job while another runs must not credit the budget a second time
    eng = snk.Engine(0, None, int(one * 1.5))
    a = eng.submit(small.params, small.dirs, small.raw, small.seeds, n_iter=10)
    b = eng.submit(small.params, small.dirs, small.raw, small.seeds, n_iter=1000)
    c = eng.submit(small.params, small.dirs, small.raw, small.seeds, n_iter=10)
    eng.step(20)
    assert eng.poll() == [a]
    eng.step(20)                       # b admitted and running, c waits
    eng.release(a)
    assert eng.get_stats()["bytes_in_use"] == one
    eng.step(20)
    s = eng.get_stats()
    assert s["running"] == 1 and s["pending"] == 1, s
    eng.close()


def test_submit_rejects_non_unit_directions(snk, jobs):
    """The evolve kernels decide that a sample ball lies inside the volume assuming |u| <= 1, so a
    direction table with a row that is not a unit vector is refused at submission (SNK_EINVAL), as
    snk_set_directions refuses it."""
    w = jobs[0]
    eng = snk.Engine(0, None, 1 << 30)
    bad = np.array(w.dirs, dtype=np.float64)
    bad[3] *= 1.5
    with pytest.raises(snk.SnkError) as ex:
        eng.submit(w.params, bad, w.raw, w.seeds, ids=w.ids, n_iter=5)
    assert ex.value.code == snk.SNK_EINVAL
    assert eng.get_stats()["submitted"] == 0
    eng.close()


def test_served_cut_tiles_alone_mix_and_oracle(snk):
    """The served workload's requests: tiles (cores of 40..64 voxels plus a 16-voxel halo, clamped at
    the faces) cut from a volume of the served recipe held on the device. Each cut equals the same box
    generated on its own; each request's result is identical alone and in a mix where requests arrive
    while others run; and each meets the free-run bar against the FP64 oracle's run of its tile."""
    import torch

    from synth.volumes import LargeVolume, tile_workload
    V = LargeVolume(synth.CONFIG_SEED_BASE + 5, shape_xyz=(320, 320, 160))
    vol = V.whole("cuda:0")
    rng = np.random.default_rng(11)
    reqs = []
    while len(reqs) < 5:
        lo, hi, clo, chi, idx = V.tile(rng, 40, 64, 16)
        if len(idx) == 0:
            continue
        tile = vol[lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]].contiguous()
        assert torch.equal(tile, V.box(lo, hi, "cuda:0"))
        reqs.append(tile_workload(V, lo, hi, idx, tile, n_iter=200, seed=synth.CONFIG_SEED_BASE + 5))
    say("served cut tiles: " + ", ".join(w.name for w in reqs))
    eng = snk.Engine(0, None, 8 << 30)
    eng.set_launch(128, 2, 1)
    alone = []
    for w in reqs:
        j = eng.submit(w.params, w.dirs, w.raw, w.seeds, ids=w.ids, n_iter=w.n_iter)
        done = []
        while j not in done:
            eng.step(25)
            done += eng.poll()
        alone.append(eng.read(j))
        eng.release(j)
    # mix: two at once, the others arriving one per step while those run
    jobs = [eng.submit(w.params, w.dirs, w.raw, w.seeds, ids=w.ids, n_iter=w.n_iter) for w in reqs[:2]]
    for w in reqs[2:]:
        eng.step(25)
        jobs.append(eng.submit(w.params, w.dirs, w.raw, w.seeds, ids=w.ids, n_iter=w.n_iter))
    pending, guard = set(jobs), 0
    while pending and guard < 100:
        eng.step(25)
        pending -= set(eng.poll())
        guard += 1
    assert not pending
    for w, j, a in zip(reqs, jobs, alone):
        mixed = eng.read(j)
        for k in KEYS:
            assert np.array_equal(a[k], mixed[k]), (w.name, k)
        ref = oracle_reference(w.raw.cpu().numpy(), w.params, w.dirs, w.seeds, w.n_iter, ids=w.ids)
        check_free_run(mixed, ref, w.params, f"served tile {w.name}")
    eng.close()
