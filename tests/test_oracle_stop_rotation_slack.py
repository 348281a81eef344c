"""Oracle pins for the stop rule's OUT transition, the sampler's rotation invariance and the kink
slack (CPU only).

  * OUT (Results: contours that leave the image stop): stepping one iteration at a time, a contour
    is OUT exactly when its centre lies outside [0, (n_a - 1) h_a] on some axis, and it never moves
    again; contours are driven through every face of an anisotropic volume, several landing within
    one voxel beyond the face.
  * Rotation invariance (Sec. II-E: samples uniform in the ball): an analytic ellipsoid in several
    orientations, evolved from 32 Philox streams each, settles at the same radius within the
    streams' Monte-Carlo spread, with the icosphere table and with a deliberately lopsided table
    (a 45-degree cap) that only the random rotations make uniform. Without the rotation the cap
    table's radius depends on the orientation far beyond that spread, so the pin has power.
  * Kink slack (a reading: FP32 may put a sample on the other side of a kink of S, or of a voxel
    face for the image-gradient centre force): for samples placed exactly on a kink (or a face),
    the slack the oracle reports equals the change of B_R and B_c found by moving the contour a
    hair either way, so that the samples really cross.
  * Stop ranges: the earliest and latest stop the rule allows when near decisions may flip equal a
    brute force over every combination of those decisions.
"""
import itertools
import math

import numpy as np
import pytest

import synth


# ------------------------------------------------------------------------------------------
# OUT transition
# ------------------------------------------------------------------------------------------

def test_out_transition_every_face(orc):
    """A bright band along one face (clamp-to-edge makes the image beyond it bright as well) pulls
    contours seeded close to that face through it. After every single step each contour that was
    active has advanced its counter by one and is OUT exactly when its centre is outside the box
    [0, (n_a - 1) h_a]; contours already stopped do not change; a single 40-step call ends in the
    same state. Each face sees several OUT contours, some within one voxel beyond the face (where
    an n_a h_a bound or a bound without the spacing would keep them active)."""
    dirs = synth.icosphere(2)
    h = np.array([1.0, 1.0, 2.0])
    shape = (12, 20, 22)                        # z, y, x
    ext = (np.array([22, 20, 12]) - 1) * h
    rng = np.random.default_rng(0)
    for axis in range(3):
        for side in (0, 1):
            J = np.zeros(shape)
            sl = [slice(None)] * 3
            thick = 3 if axis < 2 else 2
            sl[2 - axis] = slice(0, thick) if side == 0 else slice(shape[2 - axis] - thick, None)
            J[tuple(sl)] = 1.0
            n_out, n_band = 0, 0
            for eps0 in (200.0, 400.0):
                p = synth.Params(dim=3, spacing=tuple(h), dR=1.0, r_init=4.5, conv_tol=1e-3, conv_window=0,
                                 eps0=eps0, sigma_pre=0.0)
                n = 16
                seeds = rng.uniform(0.3, 0.7, size=(n, 3)) * ext
                lo, hi = (0.5, 4.0) if axis < 2 else (0.2, 1.5)
                d = rng.uniform(lo, hi, size=n) * h[axis]
                seeds[:, axis] = d if side == 0 else ext[axis] - d
                ids = np.arange(n, dtype=np.uint32)
                st = orc.init_state(p, seeds, ids=ids, shape_zyx=shape)
                assert np.all(st.status == orc.ACTIVE)
                for _ in range(40):
                    before = st.copy()
                    orc.evolve(J, p, dirs, st, 1)
                    was = (before.status & 0x0F) == orc.ACTIVE
                    assert np.array_equal(st.iters[was], before.iters[was] + 1)
                    for f in ("c", "R", "iters", "status", "streak"):
                        assert np.array_equal(getattr(st, f)[~was], getattr(before, f)[~was]), f
                    outside = np.any((st.c < 0.0) | (st.c > ext), axis=1)
                    is_out = (st.status & 0x0F) == orc.OUT
                    assert np.array_equal(is_out[was], outside[was]), (axis, side, eps0)
                    assert np.all((st.status[was & ~outside] & 0x0F) == orc.ACTIVE)
                one = orc.init_state(p, seeds, ids=ids, shape_zyx=shape)
                orc.evolve(J, p, dirs, one, 40)
                for f in ("c", "R", "iters", "status"):
                    assert np.array_equal(getattr(one, f), getattr(st, f)), f
                out = (st.status & 0x0F) == orc.OUT
                beyond = -st.c[:, axis] if side == 0 else st.c[:, axis] - ext[axis]
                n_out += int(out.sum())
                n_band += int(np.sum(out & (beyond > 0.0) & (beyond < h[axis])))
            assert n_out >= 8 and n_band >= 2, (axis, side, n_out, n_band)


# ------------------------------------------------------------------------------------------
# statistical rotation invariance
# ------------------------------------------------------------------------------------------

def _analytic_ellipsoid(Q, a=(7.0, 5.0, 4.0), c0=(24.3, 23.7, 24.1), sigma=1.0, n=49):
    """An ellipsoid with semi-axes a along the columns of Q, centre c0 (off the lattice), and an
    erfc edge of width sigma, sampled at the voxel centres of an n^3 grid (h = 1)."""
    from scipy.special import erfc
    z, y, x = np.meshgrid(*[np.arange(n, dtype=np.float64)] * 3, indexing="ij")
    P = np.stack([x - c0[0], y - c0[1], z - c0[2]], -1) @ Q
    g = np.sqrt(((P / np.asarray(a)) ** 2).sum(-1))
    return 0.5 * erfc((g - 1.0) * float(np.mean(a)) / (math.sqrt(2.0) * sigma))


def test_rotation_invariance_statistical(orc):
    ico = synth.icosphere(3)
    cap = np.ascontiguousarray(ico[ico[:, 2] > math.cos(math.radians(45.0))])
    c0 = np.array([24.3, 23.7, 24.1])
    rng = np.random.default_rng(11)
    rots = [synth._random_rotation(rng) for _ in range(5)]
    vols = [_analytic_ellipsoid(Q) for Q in rots]
    K = 32

    def settle(tab, flags):
        means, ses = [], []
        for J in vols:
            p = synth.Params(dim=3, spacing=(1.0, 1.0, 1.0), dR=1.0, n_dirs=len(tab), n_rays=32, n_radial=16,
                             sigma_pre=0.0, i_offset=0.0, i_scale=1.0, eps0=8.0, r_min=0.0, r_max=20.0,
                             conv_window=0, flags=flags)
            seeds = c0[None] + rng.uniform(-1.0, 1.0, size=(K, 3))
            st = orc.init_state(p, seeds, r0=8.0, ids=np.arange(K, dtype=np.uint32) * 5 + 1, shape_zyx=J.shape)
            orc.evolve(J, p, tab, st, 1000)
            assert np.all(st.iters == 1000)
            if flags == 0:
                assert np.linalg.norm(st.c.mean(0) - c0) < 0.05
            means.append(st.R.mean())
            ses.append(st.R.std(ddof=1) / math.sqrt(K))
        return np.array(means), np.array(ses)

    m_ico, s_ico = settle(ico, 0)
    m_cap, s_cap = settle(cap, 0)
    allm, alls = np.concatenate([m_ico, m_cap]), np.concatenate([s_ico, s_cap])
    w = 1.0 / alls ** 2
    grand = float((allm * w).sum() / w.sum())
    se_grand = float(1.0 / math.sqrt(w.sum()))
    z = np.abs(allm - grand) / np.sqrt(alls ** 2 + se_grand ** 2)
    assert np.all(z < 4.0), (allm, alls, grand)
    # power: the same cap table without the random rotation is far from invariant
    m_fix, s_fix = settle(cap, 1)
    assert np.ptp(m_fix) > 20.0 * np.sqrt(np.max(s_fix) ** 2 + np.max(s_cap) ** 2), (m_fix, s_fix)


# ------------------------------------------------------------------------------------------
# kink slack
# ------------------------------------------------------------------------------------------

def _half_bright(shape, axis_zyx, cut):
    """Smooth positive values above index `cut` along one axis, zero at and below it."""
    from scipy.ndimage import gaussian_filter
    rng = np.random.default_rng(4)
    J = 1.0 + np.abs(gaussian_filter(rng.normal(size=shape), 2.0, mode="nearest")) * 3.0
    idx = np.arange(shape[axis_zyx])
    keep = (idx > cut).reshape([-1 if a == axis_zyx else 1 for a in range(3)])
    return np.where(keep, J, 0.0)


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("kink", ["outer", "inner"])
def test_kink_slack_equals_jump(orc, dim, kink):
    """A contour whose radius is chosen so that one antithetic pair's radial point lies exactly on
    a kink of S (outer: R - dR/2; inner: rho R - rho dR/2; the other two kinks sit at fixed
    fractions of R + dR/2, rho and 1, which no radius can place a sample on). The image is zero on
    the side the pair's second ray points to, so only the first sample carries weight there. The
    oracle flags exactly that pair, and its slack on B_R and on each B_c component equals the jump
    of B_R and B_c between the contour at R(1 + eta) and R(1 - eta), where the sample sits on either
    side of the kink."""
    if dim == 3:
        shape, dirs = (32, 32, 40), synth.icosphere(2)
        p = synth.Params(dim=3, dR=1.0, n_dirs=162, n_rays=8, n_radial=16, sigma_pre=0.0)
        c = np.array([20.0, 15.7, 15.4])
    else:
        shape, dirs = (1, 36, 40), synth.circle_directions(64)
        p = synth.Params(dim=2, dR=1.0, n_dirs=64, n_rays=8, n_radial=16, sigma_pre=0.0)
        c = np.array([20.0, 17.6, 0.0])
    J = _half_bright(shape, 2, 20)          # zero for x <= 20, i.e. left of the centre
    rho = 2.0 ** (-1.0 / dim)
    lo = orc.r_geom_min(dim, p.dR) + 0.3
    checked = 0
    for n, cid in itertools.product((1, 3, 9, 27), (2, 5)):
        R0 = 8.0
        t0 = orc.mc_terms(J, p, dirs, c, R0, n, cid, want_samples=True)
        off = t0["pts"][:, :dim] - c[:dim]
        s = np.linalg.norm(off, axis=1)
        t = s / (R0 + 0.5 * p.dR)
        ux = off[:, 0] / s
        for j in np.argsort(-np.abs(ux)):
            if ux[j] <= 0:
                continue          # the bright sample of its pair is the one with u_x > 0
            if kink == "outer":   # (R + dR/2) t = R - dR/2
                R = 0.5 * p.dR * (1.0 + t[j]) / (1.0 - t[j]) if t[j] < 1 else -1
            else:                 # (R + dR/2) t = rho (R - dR/2)
                R = 0.5 * p.dR * (rho + t[j]) / (rho - t[j]) if t[j] < rho else -1
            if not (lo < R < 14.0) or s[j] * R / R0 * ux[j] < 2.5:
                continue
            st = orc.init_state(p, c[None], r0=R, ids=np.array([cid], np.uint32))
            st.iters[:] = n - 1
            tr, _ = orc.evolve(J, p, dirs, st, 1, trace=True)
            if int(tr[0, 28]) != 2:
                continue          # another sample happens to lie near a kink too
            eta = 1e-10
            hi_t = orc.mc_terms(J, p, dirs, c, R * (1 + eta), n, cid)
            lo_t = orc.mc_terms(J, p, dirs, c, R * (1 - eta), n, cid)
            jump_BR = abs(hi_t["B_R"] - lo_t["B_R"])
            jump_Bc = np.abs(hi_t["B_c"] - lo_t["B_c"])[:dim]
            assert jump_BR > 0.1 * abs(tr[0, 20])
            assert abs(tr[0, 20] - jump_BR) <= 1e-6 * jump_BR, (tr[0, 20], jump_BR)
            assert np.allclose(tr[0, 21:21 + dim], jump_Bc, rtol=1e-6, atol=1e-9 * jump_BR), (tr[0, 21:24], jump_Bc)
            # the step slack is the same jump carried through the update
            twoRd = (2.0 * R) ** dim
            eps = p.eps0 / math.sqrt(n)
            assert abs(tr[0, 24] - 0.5 * eps * jump_BR / twoRd) <= 1e-6 * tr[0, 24]
            checked += 1
            break
    assert checked >= 4, checked


@pytest.mark.parametrize("dim", [2, 3])
def test_face_slack_equals_jump(orc, dim):
    """Image-gradient centre force (flags bit 2): a contour placed so that one sample lies exactly
    on a voxel face (along z on a grid with h_z = 2 in 3D, along y in 2D). The oracle's slack on
    that component equals the jump of B_c when the whole contour (all its samples) moves a hair
    along that axis either way, so that the sample changes cells and the interpolant's slope with
    it."""
    from scipy.ndimage import gaussian_filter
    rng = np.random.default_rng(8)
    if dim == 3:
        J = gaussian_filter(rng.normal(size=(20, 30, 34)), 1.0, mode="nearest") * 4.0
        dirs = synth.icosphere(2)
        h = (1.0, 1.0, 2.0)
        p = synth.Params(dim=3, dR=1.0, n_dirs=162, n_rays=8, n_radial=16, sigma_pre=0.0, flags=4, spacing=h)
        c = np.array([16.3, 14.6, 19.2])
        ax = 2
    else:
        J = gaussian_filter(rng.normal(size=(36, 40)), 1.0, mode="nearest")[None] * 4.0
        dirs = synth.circle_directions(64)
        h = (1.0, 1.0, 1.0)
        p = synth.Params(dim=2, dR=1.0, n_dirs=64, n_rays=8, n_radial=16, sigma_pre=0.0, flags=4)
        c = np.array([19.3, 17.6, 0.0])
        ax = 1
    R = 6.3
    checked = 0
    for n in (1, 2, 5, 11, 23):
        t0 = orc.mc_terms(J, p, dirs, c, R, n, 3, want_samples=True)
        v = t0["pts"][:, ax] / h[ax]
        for j in np.argsort(np.abs(v - np.round(v)))[::7][:6]:
            cc = c.copy()
            cc[ax] += (np.round(v[j]) - v[j]) * h[ax]   # sample j now on the face v = round(v_j)
            st = orc.init_state(p, cc[None], r0=R, ids=np.array([3], np.uint32))
            st.iters[:] = n - 1
            tr, _ = orc.evolve(J, p, dirs, st, 1, trace=True)
            if int(tr[0, 28]) != 1:
                continue
            eta = 1e-9
            e = np.zeros(3)
            e[ax] = eta
            jump = abs(orc.mc_terms(J, p, dirs, cc + e, R, n, 3)["B_c"][ax] -
                       orc.mc_terms(J, p, dirs, cc - e, R, n, 3)["B_c"][ax])
            if jump == 0.0:
                continue                               # S = 0 at that sample
            assert abs(tr[0, 21 + ax] - jump) <= 1e-5 * jump, (tr[0, 21 + ax], jump)
            assert np.all(np.delete(tr[0, 21:21 + dim], ax) == 0.0)
            checked += 1
    assert checked >= 4, checked


# ------------------------------------------------------------------------------------------
# stop ranges
# ------------------------------------------------------------------------------------------

def test_stop_ranges_brute_force(orc):
    """stop_ranges against a brute force: every combination of the near decisions of short random
    move sequences, the stop rule replayed literally (streak of consecutive small moves, freeze at
    conv_window), must stop within [n_lo, n_hi], and both ends must be reached; the exact decisions
    give n_stop. Runs that stop early for another reason (NaN tail) end there."""
    rng = np.random.default_rng(2)
    p = synth.Params(conv_tol=1.0, conv_window=3)
    n, N = 400, 14
    moves = np.exp(rng.normal(0.0, 0.6, size=(n, N)))
    near_pick = rng.random((n, N)) < 0.25
    moves[near_pick] = 1.0 + rng.uniform(-0.045, 0.045, size=int(near_pick.sum()))
    stop_early = rng.random(n) < 0.1
    for i in np.where(stop_early)[0]:
        moves[i, rng.integers(3, N):] = np.nan
    delta = 0.05
    n_stop, n_lo, n_hi, conv = orc.stop_ranges(moves, p, delta)

    def rule(small, ran):
        streak = 0
        for k in range(ran):
            streak = streak + 1 if small[k] else 0
            if streak >= p.conv_window:
                return k + 1, True
        return ran, False

    for i in range(n):
        ran = int(np.sum(~np.isnan(moves[i])))
        m = moves[i, :ran]
        small = m < p.conv_tol
        ex, cv = rule(small, ran)
        assert ex == n_stop[i] and cv == conv[i]
        near = np.where(np.abs(m - p.conv_tol) <= delta * p.conv_tol)[0]
        ends = set()
        for bits in itertools.product((False, True), repeat=len(near)):
            sm = small.copy()
            sm[near] = bits
            ends.add(rule(sm, ran)[0])
        assert min(ends) == n_lo[i] and max(ends) == n_hi[i], (i, ends, n_lo[i], n_hi[i])
