"""GPU parity of the soft repulsion between neighbouring contours (snk_set_repulsion; not in the
paper) against the oracle's orc_evolve_repel on the same seeded inputs.

Bars: kappa = 0 is bit-identical to the plain evolution; one teacher-forced step (every contour set
to the oracle's state rounded to FP32, neighbours at that same snapshot) gives dR and dc within
1e-5 * max(|X_ref|, X_abs) + kink slack, X_abs including the magnitudes of the repulsion terms; free
runs with the snapshot refreshed every iteration and every 5 iterations agree with the oracle's run
(statuses and counts for >= 90% of the contours, and where they agree, radii within 0.05 and centres
within 0.5 voxel).
"""
import sys

import numpy as np
import pytest

import oracle
import synth
from parity_util import tol_check

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


def crowded():
    """The tiny workload with three seeds per blob (offsets of about a voxel) plus a dense cluster,
    so that inner spheres overlap."""
    wl = synth.tiny_config()
    rng = np.random.default_rng(4)
    seeds = np.concatenate([wl.seeds, wl.seeds + rng.uniform(-1.5, 1.5, wl.seeds.shape),
                            wl.seeds + rng.uniform(-1.5, 1.5, wl.seeds.shape),
                            rng.uniform(20.0, 44.0, size=(12, 3))])
    return wl, seeds, np.arange(len(seeds), dtype=np.uint32) * 3 + 1


def make_ctx(snk, wl, kappa, every, lanes=0):
    import torch
    ctx = snk.Context(0, torch.cuda.current_stream())
    ctx.set_params(wl.params)
    ctx.set_launch(lanes, 0, 0)
    ctx.set_directions(wl.dirs)
    ctx.load_volume(wl.raw)
    ctx.set_repulsion(kappa, every)
    return ctx


def test_zero_kappa_equals_plain(snk):
    wl, seeds, ids = crowded()
    out = []
    for kappa in (None, 0.0):
        ctx = make_ctx(snk, wl, 0.0, 3)
        if kappa is None:
            ctx.set_repulsion(0.0, 1)
        ctx.load_seeds(seeds, ids=ids)
        ctx.evolve(40)
        out.append(ctx.get_state())
        ctx.close()
    for k in out[0]:
        assert np.array_equal(out[0][k], out[1][k]), k


def test_one_step_parity(snk):
    wl, seeds, ids = crowded()
    p = wl.params
    kappa = 0.3
    J = oracle.prepass(wl.raw, p)
    st = oracle.init_state(p, seeds, ids=ids, shape_zyx=wl.raw.shape)
    ctx = make_ctx(snk, wl, kappa, 1)
    ctx.load_seeds(seeds, ids=ids)
    done = 0
    with_rep = 0
    for target in (0, 3, 12, 30):
        if target > done:
            oracle.evolve_repel(J, p, wl.dirs, st, target - done, 1, kappa)
            done = target
        c32 = st.c.astype(np.float32).astype(np.float64)
        R32 = st.R.astype(np.float32)
        ref = st.copy()
        ref.c[:] = c32
        ref.R[:] = R32.astype(np.float64)
        active = (ref.status & 0x0F) == oracle.ACTIVE
        # the plain step's terms, to see which contours feel a repulsion
        plain = ref.copy()
        tp, _ = oracle.evolve(J, p, wl.dirs, plain, 1, trace=True)
        tr, _ = oracle.evolve_repel(J, p, wl.dirs, ref, 1, 1, kappa, trace=True)
        ctx.set_state(c32, R32, st.iters, st.status, st.streak)
        g = ctx.trace_step()
        a = np.where(active)[0]
        say(f"repulsion one-step parity after {target}: {len(a)} active")
        tol_check(f"dR n={target}", g[a, 6], tr[a, 12], tr[a, 13], tr[a, 24])
        for k in range(p.dim):
            tol_check(f"dc{k} n={target}", g[a, 7 + k], tr[a, 14 + k], tr[a, 17 + k], tr[a, 25 + k])
        with_rep += int(np.sum(np.abs(tr[a, 12] - tp[a, 12]) > 1e-6))
    ctx.close()
    assert with_rep >= 20, with_rep


@pytest.mark.parametrize("every", [1, 5])
def test_free_run(snk, every):
    wl, seeds, ids = crowded()
    p = wl.params
    kappa = 0.3
    ctx = make_ctx(snk, wl, kappa, every)
    ctx.load_seeds(seeds, ids=ids)
    ctx.evolve(wl.n_iter)
    got = ctx.get_state()
    ctx.close()
    J = oracle.prepass(wl.raw, p)
    st = oracle.init_state(p, seeds, ids=ids, shape_zyx=wl.raw.shape)
    oracle.evolve_repel(J, p, wl.dirs, st, wl.n_iter, every, kappa)
    same = (got["status"] == st.status) & (got["iters"] == st.iters)
    dR = np.abs(got["radii"] - st.R)
    dc = np.linalg.norm(got["centers"] - st.c, axis=1)
    say(f"repulsion free run every {every}: {len(st.R)} contours, agreement {same.mean():.3f}, "
        f"max dR {dR[same].max():.2e}, max dc {dc[same].max():.2e}")
    assert same.mean() >= 0.9
    assert dR[same].max() <= 0.05 and dc[same].max() <= 0.5
    # the repulsion changes the result (against the plain run)
    plain = oracle.init_state(p, seeds, ids=ids, shape_zyx=wl.raw.shape)
    oracle.evolve(J, p, wl.dirs, plain, wl.n_iter)
    assert np.max(np.linalg.norm(plain.c - st.c, axis=1)) > 0.5


def test_errors(snk):
    wl, seeds, ids = crowded()
    ctx = make_ctx(snk, wl, 0.0, 1)
    for kappa, every in ((-0.1, 1), (float("nan"), 1), (0.2, 0)):
        with pytest.raises(snk.SnkError) as ex:
            ctx.set_repulsion(kappa, every)
        assert ex.value.code == snk.SNK_EINVAL
    ctx.close()
    # sub-wave groups do not carry the repulsion
    ctx = make_ctx(snk, wl, 0.2, 1, lanes=32)
    ctx.load_seeds(seeds, ids=ids)
    with pytest.raises(snk.SnkError) as ex:
        ctx.evolve(2)
    assert ex.value.code == snk.SNK_EINVAL
    ctx.close()
    # more than 64 overlapping neighbours
    ctx = make_ctx(snk, wl, 0.2, 1)
    ctx.load_seeds(np.full((70, 3), 32.0) + np.linspace(0, 0.5, 70)[:, None])
    with pytest.raises(snk.SnkError) as ex:
        ctx.evolve(1)
    assert ex.value.code == snk.SNK_ERANGE
    ctx.close()
