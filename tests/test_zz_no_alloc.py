"""snk_finalize_noalloc (selection scratch in the library's static device array) against snk_finalize.

Both run the same exact-energy and selection kernels on the same contour states, so their outputs
must be identical bit for bit: the exact energies (FP64 sums rounded to FP32 for the readback), the
keep flags and the statuses. Two calls in a row, the second on a smaller input, show that what the
first call leaves in the shared array does not leak into the second; the dense case runs the
grid-wide selection rounds (above 1,024 contours), the small one the single-workgroup path.
"""
import sys

import numpy as np
import pytest

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


def dense_state(n, seed):
    rng = np.random.default_rng(seed)
    centers = rng.uniform(2.0, 61.0, size=(n, 3))
    radii = rng.uniform(5.0, 9.0, size=n).astype(np.float32)
    status = np.full(n, 2, np.uint8)           # MAXITER
    status[::17] = 3                            # OUT
    status[::23] = 1 | 0x10                     # CONVERGED, clamped
    return centers, radii, np.full(n, 5, np.int32), status


def finalize_both(snk, ctx, state):
    """snk_finalize, then the same state again through snk_finalize_noalloc; both readbacks."""
    out = []
    for fn in (ctx.finalize, ctx.finalize_noalloc):
        ctx.set_state(*state)
        fn()
        out.append(ctx.read())
    return out


def assert_identical(a, b, what):
    for k in ("e_vox", "keep", "status", "radii", "iters"):
        assert np.array_equal(a[k], b[k]), (what, k, np.where(a[k] != b[k])[0][:10])
    assert np.array_equal(a["centers"], b["centers"]), what


def make_ctx(snk, wl, p):
    import torch
    ctx = snk.Context(0, torch.cuda.current_stream())
    ctx.set_params(p)
    ctx.set_directions(wl.dirs)
    raw = torch.from_numpy(np.ascontiguousarray(wl.raw)).to("cuda:0")
    ctx.load_volume(raw)
    ctx._raw = raw
    return ctx


def test_noalloc_finalize_equals_finalize_twice(snk):
    wl = synth.tiny_config()
    p = wl.params.replace(e0=-0.002)
    ctx = make_ctx(snk, wl, p)
    try:
        # first call: 9,000 dense contours (grid-wide rounds)
        n1 = 9000
        st1 = dense_state(n1, 5)
        ctx.load_seeds(st1[0], r0=st1[1])
        ctx.prepass()
        say(f"no-alloc finalize: call 1, {n1} dense contours")
        a, b = finalize_both(snk, ctx, st1)
        assert a["keep"].sum() >= 10
        assert_identical(a, b, "dense 9000")
        # second call, smaller: the tiny workload's 8 contours after 40 evolved iterations
        ctx.load_seeds(wl.seeds, ids=wl.ids)
        ctx.evolve(40)
        g = ctx.get_state()
        st2 = (g["centers"], g["radii"], g["iters"], g["status"], g["streak"])
        say("no-alloc finalize: call 2, 8 evolved contours")
        a, b = finalize_both(snk, ctx, st2)
        assert a["keep"].sum() >= 1
        assert_identical(a, b, "tiny 8")
        # a third, mid-sized one on the single-workgroup path
        n3 = 700
        st3 = dense_state(n3, 6)
        ctx.load_seeds(st3[0], r0=st3[1])
        say(f"no-alloc finalize: call 3, {n3} dense contours")
        a, b = finalize_both(snk, ctx, st3)
        assert_identical(a, b, "dense 700")
    finally:
        ctx.close()


def test_noalloc_finalize_rejects_beyond_its_limits(snk):
    wl = synth.tiny_config()
    ctx = make_ctx(snk, wl, wl.params)
    try:
        n = (1 << 17) + 1
        rng = np.random.default_rng(7)
        ctx.load_seeds(rng.uniform(2.0, 61.0, size=(n, 3)))
        ctx.prepass()
        say(f"no-alloc finalize: {n} contours must be refused")
        with pytest.raises(snk.SnkError) as e:
            ctx.finalize_noalloc()
        assert e.value.code == snk.SNK_EINVAL
        # a fresh volume whose pre-pass has not run is refused too (the pre-pass allocates)
        ctx.load_volume(wl.raw)
        ctx.load_seeds(wl.seeds, ids=wl.ids)
        with pytest.raises(snk.SnkError) as e:
            ctx.finalize_noalloc()
        assert e.value.code == snk.SNK_ESTATE
        # the context stays usable: the allocating path still works
        ctx.finalize()
        assert len(ctx.read()["keep"]) == len(wl.seeds)
    finally:
        ctx.close()
