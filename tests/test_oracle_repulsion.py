"""Oracle pins of the soft repulsion between neighbouring contours (not in the paper; the block
before orc_evolve_repel in oracle/snk_oracle.c).

What fixes it without another implementation: the gradient the evolution uses equals central
finite differences of the penalty itself (centre and radius, 3D and 2D, anisotropic spacing); the
penalty and its gradient vanish for neighbours whose inner spheres do not overlap and for contours
that are not live; on an all-zero image, where every Monte-Carlo sum is exactly zero, one step moves
two overlapping contours by -(eps/2) times that finite-difference gradient, symmetrically apart;
and with kappa = 0 the chunked evolution is the paper's, bit for bit.
"""
import numpy as np
import pytest

import oracle
import synth


def _config(rng, n, dim, box):
    c = rng.uniform(0.0, box, size=(n, 3))
    if dim == 2:
        c[:, 2] = 0.0
    R = rng.uniform(4.5, 9.0, size=n)
    live = (rng.random(n) < 0.85).astype(np.uint8)
    return c, R, live


@pytest.mark.parametrize("dim,seed", [(3, 0), (3, 1), (2, 2)])
def test_repulsion_gradient_equals_finite_differences(dim, seed):
    p = synth.Params(dim=dim, dR=1.0)
    rng = np.random.default_rng(seed)
    c_s, R_s, live = _config(rng, 40, dim, 30.0)
    kappa = 0.37
    checked = 0
    for self in range(40):
        c = c_s[self] + rng.uniform(-0.5, 0.5, 3) * (np.arange(3) < dim)
        R = R_s[self] * rng.uniform(0.9, 1.1)
        # stay away from the kinks of the penalty: t near 1 (contact) and coincident centres
        rho = 2.0 ** (-1.0 / dim)
        d = np.linalg.norm((c - c_s)[:, :dim], axis=1)
        t = d / (rho * (R + R_s))
        mask = (np.arange(40) != self) & (live == 1)
        if np.any(mask & (np.abs(t - 1.0) < 1e-3)) or np.any(mask & (d < 1e-3)):
            continue
        gc, gR = oracle.repel_grad(p, c_s, R_s, live, self, c, R, kappa)
        h = 1e-6
        for a in range(dim):
            e = np.zeros(3)
            e[a] = h
            fd = (oracle.repel_energy(p, c_s, R_s, live, self, c + e, R, kappa)
                  - oracle.repel_energy(p, c_s, R_s, live, self, c - e, R, kappa)) / (2 * h)
            assert abs(gc[a] - fd) <= 1e-6 * max(1.0, abs(fd)), (self, a, gc[a], fd)
        fdR = (oracle.repel_energy(p, c_s, R_s, live, self, c, R + h, kappa)
               - oracle.repel_energy(p, c_s, R_s, live, self, c, R - h, kappa)) / (2 * h)
        assert abs(gR - fdR) <= 1e-6 * max(1.0, abs(fdR)), (self, gR, fdR)
        if np.any(mask & (t < 1.0)):
            checked += 1
    assert checked >= 10


def test_repulsion_only_between_overlapping_live_contours():
    p = synth.Params(dim=3, dR=1.0)
    rho = 2.0 ** (-1.0 / 3)
    c_s = np.array([[10.0, 10.0, 10.0], [10.0, 10.0, 10.0], [40.0, 10.0, 10.0]])
    R_s = np.array([6.0, 6.0, 6.0])
    c = np.array([10.0 + rho * 12.0 * 1.0001, 10.0, 10.0])       # just beyond contact with 0
    for live in ([1, 1, 1], [1, 0, 1]):
        assert oracle.repel_energy(p, c_s, R_s, live, 1, c, 6.0, 1.0) == 0.0
        gc, gR = oracle.repel_grad(p, c_s, R_s, live, 1, c, 6.0, 1.0)
        assert np.all(gc == 0.0) and gR == 0.0
    c_in = np.array([10.0 + rho * 12.0 * 0.5, 10.0, 10.0])       # overlapping contour 0 (t = 0.5)
    assert oracle.repel_energy(p, c_s, R_s, [1, 1, 1], 1, c_in, 6.0, 1.0) == pytest.approx(0.25)
    # a non-live neighbour does not repel; the contour's own snapshot never does
    assert oracle.repel_energy(p, c_s, R_s, [0, 1, 1], 1, c_in, 6.0, 1.0) == 0.0
    assert oracle.repel_energy(p, c_s, R_s, [1, 1, 1], 0, c_s[0], 6.0, 1.0) == pytest.approx(1.0)  # from 1 only


@pytest.mark.parametrize("dim", [3, 2])
def test_zero_image_step_is_the_repulsion_descent(dim):
    """All-zero image: A, B_R and B_c are exactly zero, so the only force is the repulsion; one step
    of two overlapping contours equals -(eps/2) times the finite-difference gradient of the
    penalty, and the two move symmetrically apart and shrink alike."""
    shape = (40, 40, 40) if dim == 3 else (1, 80, 80)
    h = (1.0, 1.0, 2.0) if dim == 3 else (1.0, 1.0, 1.0)
    p = synth.Params(dim=dim, spacing=h, sigma_pre=0.0, dR=1.0, eps0=8.0, r_max=20.0, n_dirs=162 if dim == 3 else 64,
                     n_rays=32, n_radial=16, conv_window=0)
    J = np.zeros(shape)
    dirs = synth.directions_for(dim, p.n_dirs)
    mid = np.array([20.0, 20.0, 38.0 if dim == 3 else 0.0]) if dim == 3 else np.array([40.0, 40.0, 0.0])
    off = np.array([3.0, 1.0, 0.5 if dim == 3 else 0.0])
    seeds = np.stack([mid - off, mid + off])
    st = oracle.init_state(p, seeds, r0=np.array([6.0, 6.0]), shape_zyx=shape)
    kappa = 0.5
    before = st.copy()
    live = np.ones(2, np.uint8)
    oracle.evolve_repel(J, p, dirs, st, 1, 1, kappa)
    eps = p.eps0
    for i in range(2):
        hh = 1e-6
        fd = np.zeros(3)
        for a in range(dim):
            e = np.zeros(3)
            e[a] = hh
            fd[a] = (oracle.repel_energy(p, before.c, before.R, live, i, before.c[i] + e, before.R[i], kappa)
                     - oracle.repel_energy(p, before.c, before.R, live, i, before.c[i] - e, before.R[i], kappa)) / (2 * hh)
        fdR = (oracle.repel_energy(p, before.c, before.R, live, i, before.c[i], before.R[i] + hh, kappa)
               - oracle.repel_energy(p, before.c, before.R, live, i, before.c[i], before.R[i] - hh, kappa)) / (2 * hh)
        assert np.allclose(st.c[i] - before.c[i], -0.5 * eps * fd, rtol=1e-6, atol=1e-12)
        assert st.R[i] - before.R[i] == pytest.approx(-0.5 * eps * fdR, rel=1e-6)
    assert np.allclose(st.c[0] - before.c[0], -(st.c[1] - before.c[1]), atol=1e-12)
    assert np.linalg.norm(st.c[0] - st.c[1]) > np.linalg.norm(before.c[0] - before.c[1])
    assert st.R[0] < before.R[0] and st.R[0] == pytest.approx(st.R[1], rel=1e-12)


def test_zero_kappa_is_the_papers_contour():
    wl = synth.tiny_config()
    p = wl.params
    J = oracle.prepass(wl.raw, p)
    a = oracle.init_state(p, wl.seeds, ids=wl.ids, shape_zyx=wl.raw.shape)
    b = a.copy()
    ta, na = oracle.evolve(J, p, wl.dirs, a, 25, trace=True)
    tb, nb = oracle.evolve_repel(J, p, wl.dirs, b, 25, 3, 0.0, trace=True)
    assert na == nb
    for f in ("c", "R", "iters", "status", "streak", "e_mc"):
        assert np.array_equal(getattr(a, f), getattr(b, f)), f
    assert np.array_equal(ta, tb)


def test_repulsion_separates_doubled_seeds():
    """Behaviour: two seeds per blob of the tiny workload; with repulsion the two contours of a blob
    end farther apart than without (their inner spheres push each other off)."""
    wl = synth.tiny_config()
    p = wl.params.replace(conv_window=0)
    J = oracle.prepass(wl.raw, p)
    seeds = np.concatenate([wl.seeds - 0.8, wl.seeds + 0.8])
    runs = {}
    for kappa in (0.0, 0.3):
        st = oracle.init_state(p, seeds, shape_zyx=wl.raw.shape)
        oracle.evolve_repel(J, p, wl.dirs, st, 60, 1, kappa)
        runs[kappa] = np.linalg.norm(st.c[:8] - st.c[8:], axis=1)
    assert np.median(runs[0.3]) > np.median(runs[0.0]) + 1.0
