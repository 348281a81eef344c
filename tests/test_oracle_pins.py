"""Pins of the FP64 oracle against facts the paper and mathematics fix (CPU only).

Each test checks one piece of the oracle against something other than the oracle itself:
published known-answer vectors, an independent library routine, a closed form from the paper
(Eq. (3), the alpha = d normalisation of Eq. (4), the zero-mean weight of Sec. II-B), finite
differences, exact symmetries, or an independent i.i.d. Monte-Carlo estimate.
"""
import math
import os
import shutil
import subprocess

import numpy as np
import pytest

import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
RHO3 = 2.0 ** (-1.0 / 3.0)
RHO2 = 2.0 ** (-0.5)


def _kat_rows():
    rows = []
    with open(os.path.join(ROOT, "tests", "golden", "philox4x32_10_kat.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            v = [int(t, 16) for t in line.split()]
            rows.append((v[0:4], v[4:6], v[6:10]))
    return rows


# ------------------------------------------------------------------------------------------
# random numbers
# ------------------------------------------------------------------------------------------

def test_philox_known_answers(orc):
    rows = _kat_rows()
    assert len(rows) == 3
    for ctr, key, want in rows:
        assert orc.philox(ctr, key) == want


ROCRAND_SRC = r"""
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>
#include <cstdlib>
int main(int argc, char **argv) {
  unsigned long long seed = strtoull(argv[1], 0, 0) | (strtoull(argv[2], 0, 0) << 32);
  unsigned long long c0 = strtoull(argv[3], 0, 0), c1 = strtoull(argv[4], 0, 0);
  unsigned long long c2 = strtoull(argv[5], 0, 0), c3 = strtoull(argv[6], 0, 0);
  rocrand_device::philox4x32_10_engine e(seed, c2 | (c3 << 32), 0);
  unsigned long long total = c0 | (c1 << 32), chunk = total / 8, done = 0;
  for (int i = 0; i < 7; ++i) { e.discard(4ull * chunk); done += chunk; }
  e.discard(4ull * (total - done));
  uint4 v = e.next4();
  printf("%u %u %u %u\n", v.x, v.y, v.z, v.w);
  return 0;
}
"""


def test_philox_matches_rocrand(orc, tmp_path):
    """Cross-check against rocRAND's open-source Philox4x32-10 engine, run as a host program."""
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    src = tmp_path / "rr.cpp"
    src.write_text(ROCRAND_SRC)
    exe = tmp_path / "rr"
    subprocess.check_call([hipcc, "-O1", "-x", "hip", "--offload-arch=gfx950", str(src), "-o", str(exe)],
                          stdout=subprocess.DEVNULL, stderr=subprocess.DEVNULL)
    rng = np.random.default_rng(7)
    cases = [([0, 0, 0, 0], [0, 0])] + [
        (list(rng.integers(0, 2 ** 32, 4)), list(rng.integers(0, 2 ** 32, 2))) for _ in range(12)]
    cases += [([5, 17, 3, 1], [0x40000002, 0x18040630])]  # a contour-iteration counter shape
    for ctr, key in cases:
        out = subprocess.check_output([str(exe), str(key[0]), str(key[1])] + [str(c) for c in ctr])
        assert [int(t) for t in out.split()] == orc.philox(ctr, key)


def test_uniform_mapping_exact(orc):
    assert orc.uniform(0) == 2.0 ** -24
    assert orc.uniform(0xFFFFFFFF) == 1.0 - 2.0 ** -24
    for x in np.random.default_rng(1).integers(0, 2 ** 32, 2000):
        u = orc.uniform(int(x))
        assert 0.0 < u < 1.0
        assert float(np.float32(u)) == u  # exactly representable in FP32


def test_rotation_is_uniform_proper_rotation(orc):
    p = synth.Params()
    cols = []
    for n in range(1, 1201):
        Q = orc.rotation(p, n, 3)
        assert np.allclose(Q @ Q.T, np.eye(3), atol=1e-12)
        assert abs(np.linalg.det(Q) - 1.0) < 1e-12
        cols.append(Q[:, 0])
    cols = np.array(cols)
    # a uniform rotation maps e_x to a uniform point on the sphere: mean 0, E[v_i^2] = 1/3
    assert np.all(np.abs(cols.mean(0)) < 4.0 / math.sqrt(3 * len(cols)))
    assert np.all(np.abs((cols ** 2).mean(0) - 1.0 / 3.0) < 0.04)
    p2 = synth.Params(dim=2)
    Q2 = orc.rotation(p2, 4, 9)
    assert np.allclose(Q2[:2, :2] @ Q2[:2, :2].T, np.eye(2), atol=1e-12)
    assert np.allclose(orc.rotation(synth.Params(flags=1), 4, 9), np.eye(3))


# ------------------------------------------------------------------------------------------
# weight function and energy (Sec. II-B, Eqs. (3)-(5))
# ------------------------------------------------------------------------------------------

def _gl_integral(f, breaks, order=8):
    """Gauss-Legendre on each interval between sorted breakpoints (exact for piecewise
    polynomials of degree < 2*order)."""
    x, w = np.polynomial.legendre.leggauss(order)
    total = 0.0
    b = np.unique(np.asarray(breaks, dtype=np.float64))
    for lo, hi in zip(b[:-1], b[1:]):
        t = 0.5 * (hi - lo) * x + 0.5 * (hi + lo)
        total += 0.5 * (hi - lo) * float(np.dot(w, f(t)))
    return total


def _kinks(dim, R, dR):
    rho = RHO3 if dim == 3 else RHO2
    a, dr = rho * R, rho * dR
    return [0.0, a - dr / 2, a + dr / 2, R - dR / 2, R + dR / 2]


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("dR", [0.75, 1.0])
@pytest.mark.parametrize("R", [4.5, 6.0, 9.3, 15.0])
def test_weight_zero_mean(orc, dim, dR, R):
    """int_0^inf S(r) r^(d-1) dr = 0 (Sec. II-B): fixes rho = 2^(-1/d) and dr = rho*dR."""
    f = lambda r: orc.weight_vec(dim, r, R, dR)[..., 0] * r ** (dim - 1)
    g = lambda r: np.abs(orc.weight_vec(dim, r, R, dR)[..., 0]) * r ** (dim - 1)
    ks = _kinks(dim, R, dR)
    val = _gl_integral(f, ks)
    scale = _gl_integral(g, ks)
    assert abs(val) < 1e-12 * scale


@pytest.mark.parametrize("dim", [2, 3])
def test_weight_shape_and_derivatives(orc, dim):
    R, dR = 7.3, 0.9
    rho = RHO3 if dim == 3 else RHO2
    ks = _kinks(dim, R, dR)
    # four regions: -1 core, +1 shell, zero outside, continuous at every kink
    assert orc.weight(dim, 0.1, R, dR)[0] == -1.0
    assert orc.weight(dim, 0.5 * (ks[2] + ks[3]), R, dR)[0] == 1.0
    assert orc.weight(dim, ks[4] + 0.01, R, dR)[0] == 0.0
    for k in ks[1:]:
        lo, hi = orc.weight(dim, k - 1e-9, R, dR)[0], orc.weight(dim, k + 1e-9, R, dR)[0]
        assert abs(lo - hi) < 1e-8
    # ramp widths: inner dr = rho*dR, outer dR (Sec. II-B: dr = dR / cbrt(2) in 3D)
    assert abs((ks[2] - ks[1]) - rho * dR) < 1e-12 and abs((ks[4] - ks[3]) - dR) < 1e-12
    # dS/dr and dS/dR agree with finite differences away from kinks
    rng = np.random.default_rng(3)
    for r in rng.uniform(0.0, ks[4] + 1.0, 400):
        if min(abs(r - k) for k in ks) < 1e-4:
            continue
        h = 1e-6
        S, Sr, SR = orc.weight(dim, r, R, dR)
        fr = (orc.weight(dim, r + h, R, dR)[0] - orc.weight(dim, r - h, R, dR)[0]) / (2 * h)
        fR = (orc.weight(dim, r, R + h, dR)[0] - orc.weight(dim, r, R - h, dR)[0]) / (2 * h)
        assert abs(fr - Sr) < 1e-6 and abs(fR - SR) < 1e-6


def _hat_energy_ideal_blob(orc, dim, R, r0, dR):
    """E-hat of the ideal blob I = 1 + sgn(r0 - r) centred on the contour (the oracle's S)."""
    meas = 4.0 * math.pi if dim == 3 else 2.0 * math.pi
    f = lambda r: orc.weight_vec(dim, r, R, dR)[..., 0] * np.where(r < r0, 2.0, 0.0) * meas * r ** (dim - 1)
    return _gl_integral(f, _kinks(dim, R, dR) + [r0])


@pytest.mark.parametrize("r0", [4.0, 6.5, 11.0])
def test_ideal_blob_energy_eq3(orc, r0):
    """Eq. (3): 0 for R < r0; -(8/3) pi (R^3 - r0^3) for R/cbrt(2) < r0 < R; -(8/3) pi r0^3 beyond."""
    dR = 1e-4
    for R in np.linspace(0.5 * r0, 2.0 * r0, 31):
        if R < orc.r_geom_min(3, dR):
            continue
        if R < r0:
            want = 0.0
        elif R * RHO3 < r0:
            want = -(8.0 / 3.0) * math.pi * (R ** 3 - r0 ** 3)
        else:
            want = -(8.0 / 3.0) * math.pi * r0 ** 3
        got = _hat_energy_ideal_blob(orc, 3, R, r0, dR)
        assert abs(got - want) < 1e-3 * (8.0 / 3.0) * math.pi * r0 ** 3, (R, got, want)


@pytest.mark.parametrize("r0", [4.0, 9.0])
def test_ideal_disk_energy_2d(orc, r0):
    """2D analogue of Eq. (3) with rho = 1/sqrt(2) (Sec. II-A): 0; -2 pi (R^2 - r0^2); -2 pi r0^2."""
    dR = 1e-4
    for R in np.linspace(0.5 * r0, 2.0 * r0, 25):
        if R < r0:
            want = 0.0
        elif R * RHO2 < r0:
            want = -2.0 * math.pi * (R ** 2 - r0 ** 2)
        else:
            want = -2.0 * math.pi * r0 ** 2
        got = _hat_energy_ideal_blob(orc, 2, R, r0, dR)
        assert abs(got - want) < 1e-3 * 2.0 * math.pi * r0 ** 2


@pytest.mark.parametrize("dim", [2, 3])
def test_normalisation_alpha_gives_symmetric_slopes(orc, dim):
    """Eq. (4): with E = E-hat / ||p - q||^d the slopes on both sides of R* = 2^(1/d) r0 have equal
    magnitude and opposite sign, E(R*) = -pi/6 (3D) / -pi/4 (2D) for the contrast-2 blob, and R*
    is the unique minimum. Evaluated through the oracle's estimator with a deterministic radial
    quadrature (sample points held fixed)."""
    r0, dR = 5.0, 2e-3
    rstar = 2.0 ** (1.0 / dim) * r0
    big = 2.5 * r0
    N = 400000
    u = (np.arange(N) + 0.5) / N
    r = big * u ** (1.0 / dim)            # equal-measure radial nodes in the ball of radius `big`
    pts = np.zeros((N, 3))
    pts[:, 0] = r
    vals = np.where(r < r0, 2.0, 0.0)
    vol = (4.0 / 3.0 * math.pi if dim == 3 else math.pi) * big ** dim
    E = lambda R: orc.energy_fixed(dim, dR, pts, vals, vol / N, [0.0, 0.0, 0.0], R)
    h = 0.02
    left = (E(rstar - h) - E(rstar - 3 * h)) / (2 * h)
    right = (E(rstar + 3 * h) - E(rstar + h)) / (2 * h)
    assert left < 0 < right
    # on both sides |dE/dR| = pi r0^d / R^(d+1): the one-sided limits at R* are equal
    lim_l = -left * (rstar - 2 * h) ** (dim + 1)
    lim_r = right * (rstar + 2 * h) ** (dim + 1)
    assert abs(lim_l / lim_r - 1.0) < 0.01
    assert abs(lim_r / (math.pi * r0 ** dim) - 1.0) < 0.01
    want = -math.pi / 6.0 if dim == 3 else -math.pi / 4.0
    assert abs(E(rstar) - want) < 2e-3
    Rs = np.linspace(0.8 * r0, 2.2 * r0, 57)
    Es = np.array([E(v) for v in Rs])
    assert abs(Rs[np.argmin(Es)] - rstar) <= (Rs[1] - Rs[0]) * 1.01


# ------------------------------------------------------------------------------------------
# gradient (Eqs. (7)-(11)) and the p,q <-> c,R identity
# ------------------------------------------------------------------------------------------

def _smooth_volume(shape, seed=11, sigma=2.0, scale=3.0):
    from scipy.ndimage import gaussian_filter
    rng = np.random.default_rng(seed)
    return gaussian_filter(rng.normal(size=shape), sigma, mode="nearest") * scale + 0.5


@pytest.mark.parametrize("dim,spacing", [(3, (1.0, 1.0, 1.0)), (3, (1.0, 1.0, 2.0)), (2, (1.0, 1.0, 1.0))])
def test_exact_sums_are_gradient_of_exact_energy(orc, dim, spacing):
    """Exact mode (flags bit 1): the lattice sums give E equal to the exact Eq. (5) energy, and
    g_R, g_c equal its central differences in R and c (the lattice held fixed); p,q form too. Points
    crossing a kink of S within the difference step are detected by one-sided differences and
    skipped (at most a few of the cases)."""
    if dim == 3:
        J = _smooth_volume((24, 26, 28))
        dirs = synth.icosphere(2)
        p = synth.Params(dim=3, dR=1.0, n_dirs=162, n_rays=32, n_radial=16, spacing=spacing, flags=2)
    else:
        J = _smooth_volume((1, 40, 44))
        dirs = synth.circle_directions(64)
        p = synth.Params(dim=2, dR=1.0, n_dirs=64, n_rays=16, n_radial=16, flags=2)
    rng = np.random.default_rng(11)
    h = 1e-6
    smooth = 0
    for trial in range(12):
        c = np.array([rng.uniform(9, 15), rng.uniform(9, 15), rng.uniform(9, 13) if dim == 3 else 0.0])
        R = rng.uniform(4.5, 7.5)
        t = orc.mc_terms(J, p, dirs, c, R, 1 + trial, 3)
        t2 = orc.mc_terms(J, p, dirs, c, R, 99, 77)   # no random numbers: n and id do not matter
        assert t["g_R"] == t2["g_R"] and np.array_equal(t["g_c"], t2["g_c"])
        E = lambda cc, RR: orc.energy_vox(J, p, np.array([cc]), np.array([RR]))[0][0]
        assert abs(E(c, R) - t["E"]) < 1e-12 * max(1.0, abs(t["E"]))
        e0 = E(c, R)
        cases = [((c, R + h), (c, R - h), t["g_R"])]
        for a in range(dim):
            e = np.zeros(3)
            e[a] = h
            cases.append(((c + e, R), (c - e, R), t["g_c"][a]))
        ex = np.array([h / 2, 0.0, 0.0])
        cases.append(((c + ex, R - h / 2), (c - ex, R + h / 2), t["dEdp"][0]))   # p_x alone
        cases.append(((c + ex, R + h / 2), (c - ex, R - h / 2), t["dEdq"][0]))   # q_x alone
        for plus, minus, g in cases:
            ep, em = E(*plus), E(*minus)
            fwd, bwd = (ep - e0) / h, (e0 - em) / h
            if abs(fwd - bwd) > 1e-4 * (abs(g) + 1e-3):
                continue   # a lattice point crossed a kink of S within +-h
            smooth += 1
            assert abs((ep - em) / (2 * h) - g) < 1e-5 * (abs(g) + 1e-3), (trial, g, (ep - em) / (2 * h))
    assert smooth >= 0.9 * 12 * (3 + dim)


@pytest.mark.parametrize("dim", [2, 3])
def test_gradient_matches_finite_differences(orc, dim):
    if dim == 3:
        J = _smooth_volume((24, 26, 28))
        p = synth.Params(dim=3, dR=1.0, n_dirs=162, n_rays=32, n_radial=16)
        dirs = synth.icosphere(2)
        c = np.array([13.3, 12.1, 11.7])
    else:
        J = _smooth_volume((1, 40, 44))
        p = synth.Params(dim=2, dR=1.0, n_dirs=64, n_rays=16, n_radial=16)
        dirs = synth.circle_directions(64)
        c = np.array([21.3, 19.6, 0.0])
    R = 6.4
    checked = 0
    for n in (1, 2, 7, 33):
        t = orc.mc_terms(J, p, dirs, c, R, n, 5, want_samples=True)
        pts, vals, sc = t["pts"], t["vals"], t["scale"]
        E = lambda cc, RR: orc.energy_fixed(dim, p.dR, pts, vals, sc, cc, RR)
        assert abs(E(c, R) - t["E"]) < 1e-12 * max(1.0, abs(t["E"]))
        h = 1e-6
        gR = (E(c, R + h) - E(c, R - h)) / (2 * h)
        scale = np.abs(t["g_R"]) + 1e-3
        assert abs(gR - t["g_R"]) < 1e-5 * scale, (n, gR, t["g_R"])
        for a in range(dim):
            e = np.zeros(3); e[a] = h
            gc = (E(c + e, R) - E(c - e, R)) / (2 * h)
            assert abs(gc - t["g_c"][a]) < 1e-5 * (np.abs(t["g_c"]).max() + 1e-3)
        # Eqs. (7)-(8): move p_x alone (c_x by h/2, R by -h/2) or q_x alone
        ex = np.array([h / 2, 0.0, 0.0])
        dpx = (E(c + ex, R - h / 2) - E(c - ex, R + h / 2)) / (2 * h)
        dqx = (E(c + ex, R + h / 2) - E(c - ex, R - h / 2)) / (2 * h)
        tol = 1e-5 * (np.abs(t["dEdp"]).max() + np.abs(t["dEdq"]).max() + 1e-3)
        assert abs(dpx - t["dEdp"][0]) < tol and abs(dqx - t["dEdq"][0]) < tol
        # Eqs. (9)-(10): dE/dp_y = dE/dq_y (p, q stay aligned, Eq. (6))
        for a in range(1, dim):
            assert t["dEdp"][a] == t["dEdq"][a]
            ey = np.zeros(3); ey[a] = h / 2
            dpy = (E(c + ey, R) - E(c - ey, R)) / (2 * h)
            assert abs(dpy - t["dEdp"][a]) < tol
        # p,q <-> c,R identity: dE/dc = dE/dp + dE/dq, dE/dR = dE/dq_x - dE/dp_x
        assert np.allclose(t["dEdp"][:dim] + t["dEdq"][:dim], t["g_c"][:dim], rtol=1e-10, atol=1e-14)
        assert abs((t["dEdq"][0] - t["dEdp"][0]) - t["g_R"]) < 1e-10 * (abs(t["g_R"]) + 1e-12)
        checked += 1
    assert checked == 4


def test_evolve_pq_and_cr_forms_agree(orc):
    """The oracle updates in p,q form (Eqs. (12)-(15)) and checks the c,R form every iteration;
    evolve raises on any disagreement."""
    wl = synth.tiny_config()
    J = orc.prepass(wl.raw, wl.params)
    st = orc.init_state(wl.params, wl.seeds)
    orc.evolve(J, wl.params, wl.dirs, st, 30)
    assert np.all(st.iters == 30)


# ------------------------------------------------------------------------------------------
# Monte-Carlo estimator (Sec. II-E)
# ------------------------------------------------------------------------------------------

def _iid_reference(orc, J, dim, h, c, R, dR, n_pts, seed):
    """Independent i.i.d. estimate of (A, B_R, B_c) by rejection sampling in the ball, with
    scipy's order-1 map_coordinates (mode 'nearest') as the interpolant."""
    from scipy.ndimage import map_coordinates
    rng = np.random.default_rng(seed)
    smax = R + 0.5 * dR
    pts = []
    need = n_pts
    while need > 0:
        x = rng.uniform(-smax, smax, size=(2 * need, dim))
        x = x[(x ** 2).sum(1) < smax ** 2][:need]
        pts.append(x)
        need -= len(x)
    x = np.concatenate(pts)
    r = np.sqrt((x ** 2).sum(1))
    u = x / r[:, None]
    pos = x + c[:dim]
    if dim == 3:
        coords = np.stack([pos[:, 2] / h[2], pos[:, 1] / h[1], pos[:, 0] / h[0]])
        I = map_coordinates(J, coords, order=1, mode="nearest")
    else:
        coords = np.stack([pos[:, 1] / h[1], pos[:, 0] / h[0]])
        I = map_coordinates(J[0], coords, order=1, mode="nearest")
    w = orc.weight_vec(dim, r, R, dR)
    V = (4.0 / 3.0 * math.pi if dim == 3 else math.pi) * smax ** dim
    terms = np.concatenate([(w[:, 0] * I)[:, None], (w[:, 2] * I)[:, None], -(w[:, 1] * I)[:, None] * u], axis=1)
    return V * terms.mean(0), V * terms.std(0) / math.sqrt(len(terms))


@pytest.mark.parametrize("dim", [2, 3])
def test_mc_estimator_unbiased(orc, dim):
    if dim == 3:
        J = _smooth_volume((18, 20, 22), seed=5)
        p = synth.Params(dim=3, dR=1.0, n_dirs=162, n_rays=32, n_radial=16, spacing=(1.0, 1.0, 1.0))
        dirs = synth.icosphere(2)
        c = np.array([10.2, 9.6, 8.9])
    else:
        J = _smooth_volume((1, 30, 34), seed=5)
        p = synth.Params(dim=2, dR=1.0, n_dirs=64, n_rays=16, n_radial=16)
        dirs = synth.circle_directions(64)
        c = np.array([16.2, 14.4, 0.0])
    R = 5.5
    K = 1500
    samples = np.array([np.concatenate([[t["A"], t["B_R"]], t["B_c"][:dim]]) for t in
                        (orc.mc_terms(J, p, dirs, c, R, n, 2) for n in range(1, K + 1))])
    mean, se = samples.mean(0), samples.std(0) / math.sqrt(K)
    ref, ref_se = _iid_reference(orc, J, dim, p.spacing, c, R, p.dR, 1_500_000, seed=9)
    z = np.abs(mean - ref) / np.sqrt(se ** 2 + ref_se ** 2)
    assert np.all(z < 4.5), (mean, ref, z)


# ------------------------------------------------------------------------------------------
# centre force in its image-gradient form (flags bit 2)
# ------------------------------------------------------------------------------------------

@pytest.mark.parametrize("dim,spacing,near_face", [(3, (1.0, 1.0, 1.0), False), (3, (1.0, 1.0, 2.0), False),
                                                   (3, (1.0, 1.0, 1.0), True), (2, (1.0, 1.0, 1.0), False),
                                                   (2, (1.0, 1.0, 1.0), True)])
def test_gradient_form_is_derivative_with_offsets_fixed(orc, dim, spacing, near_face):
    """Flags bit 2: the centre force equals the central difference of the same-sample energy
    estimator when the sample offsets (not the sample points) are held fixed, i.e. the whole sample
    cloud moves with c, samples clamped beyond a face included. The trilinear interpolant is
    linear along each axis inside a cell, so the difference is exact unless a sample crosses a
    voxel face within the step (such cases are detected and skipped)."""
    if dim == 3:
        J = _smooth_volume((20, 26, 28))
        p = synth.Params(dim=3, dR=1.0, n_dirs=162, n_rays=32, n_radial=16, spacing=spacing, flags=4)
        dirs = synth.icosphere(2)
        c = np.array([1.5, 12.1, 2.3 * spacing[2]]) if near_face else np.array([13.3, 12.1, 9.7 * spacing[2]])
    else:
        J = _smooth_volume((1, 40, 44))
        p = synth.Params(dim=2, dR=1.0, n_dirs=64, n_rays=16, n_radial=16, flags=4)
        dirs = synth.circle_directions(64)
        c = np.array([2.1, 19.6, 0.0]) if near_face else np.array([21.3, 19.6, 0.0])
    h = np.array(spacing[:dim] if dim == 3 else spacing[:2])
    R = 6.4
    checked = 0
    for n in (1, 2, 7, 33):
        t = orc.mc_terms(J, p, dirs, c, R, n, 5, want_samples=True)
        pts, sc = t["pts"], t["scale"]

        def E(shift):
            moved = pts.copy()
            moved[:, :dim] += shift[:dim]
            vals = np.array([orc.interp(J, dim, moved[j, :dim] / h) for j in range(len(moved))])
            return orc.energy_fixed(dim, p.dR, moved, vals, sc, c + shift, R)

        d = 1e-7
        g = t["g_c"]
        for a in range(dim):
            e = np.zeros(3); e[a] = d
            vox = pts[:, a] / h[a]
            nmax = J.shape[2 - a] - 1 if dim == 3 else J.shape[2 - a] - 1
            inside = (vox > 0) & (vox < nmax)
            crosses = np.floor((pts[:, a] + d) / h[a]) != np.floor((pts[:, a] - d) / h[a])
            if np.any(crosses & inside):
                continue
            fd = (E(e) - E(-e)) / (2 * d)
            assert abs(fd - g[a]) < 1e-6 * (np.abs(g).max() + 1e-3), (n, a, fd, g[a])
            checked += 1
    assert checked >= 3 * dim


@pytest.mark.parametrize("dim", [2, 3])
def test_gradient_form_linear_field(orc, dim):
    """Flags bit 2 on an affine image I = b + a . v (v in voxel coordinates): the trilinear
    interpolant reproduces it exactly, so every interior sample sees grad I = a / h and the centre
    force is sum_j S_j * (a / h) times the same scale, where sum_j S_j times the scale is the A term
    of the same samples on the constant image I = 1."""
    a = np.array([0.37, -0.21, 0.13])
    if dim == 3:
        shape, spacing = (30, 32, 34), (1.0, 1.0, 2.0)
        p = synth.Params(dim=3, dR=1.0, n_dirs=162, n_rays=32, n_radial=16, spacing=spacing, flags=4)
        dirs = synth.icosphere(2)
        c = np.array([16.3, 15.2, 14.1 * 2.0])
    else:
        shape, spacing = (1, 40, 44), (1.0, 1.0, 1.0)
        p = synth.Params(dim=2, dR=1.0, n_dirs=64, n_rays=16, n_radial=16, flags=4)
        dirs = synth.circle_directions(64)
        c = np.array([21.3, 19.6, 0.0])
    z, y, x = np.meshgrid(*[np.arange(k, dtype=np.float64) for k in shape], indexing="ij")
    J = 2.0 + a[0] * x + a[1] * y + (a[2] * z if dim == 3 else 0.0)
    ones = np.ones(shape)
    R = 6.4
    for n in (1, 5, 40):
        t = orc.mc_terms(J, p, dirs, c, R, n, 3)
        t1 = orc.mc_terms(ones, p, dirs, c, R, n, 3)
        expect = t1["A"] * a[:dim] / np.array(spacing[:dim])
        assert np.allclose(t["B_c"][:dim], expect, rtol=1e-9, atol=1e-12), (t["B_c"], expect)


@pytest.mark.parametrize("dim", [2, 3])
def test_gradient_form_unbiased(orc, dim):
    """Flags bit 2 estimates the same centre force as the weight form: its mean over many
    iterations' draws agrees with an independent i.i.d. estimate of -integral dS/dr u I over the
    ball (the expectation of the weight form), while A and B_R are unchanged."""
    if dim == 3:
        J = _smooth_volume((18, 20, 22), seed=5)
        p = synth.Params(dim=3, dR=1.0, n_dirs=162, n_rays=32, n_radial=16, spacing=(1.0, 1.0, 1.0), flags=4)
        dirs = synth.icosphere(2)
        c = np.array([10.2, 9.6, 8.9])
    else:
        J = _smooth_volume((1, 30, 34), seed=5)
        p = synth.Params(dim=2, dR=1.0, n_dirs=64, n_rays=16, n_radial=16, flags=4)
        dirs = synth.circle_directions(64)
        c = np.array([16.2, 14.4, 0.0])
    R = 5.5
    K = 1500
    samples = np.array([np.concatenate([[t["A"], t["B_R"]], t["B_c"][:dim]]) for t in
                        (orc.mc_terms(J, p, dirs, c, R, n, 2) for n in range(1, K + 1))])
    mean, se = samples.mean(0), samples.std(0) / math.sqrt(K)
    ref, ref_se = _iid_reference(orc, J, dim, p.spacing, c, R, p.dR, 1_500_000, seed=9)
    z = np.abs(mean - ref) / np.sqrt(se ** 2 + ref_se ** 2)
    assert np.all(z < 4.5), (mean, ref, z)


# ------------------------------------------------------------------------------------------
# star-shaped contours (per-direction radii; not in the paper)
# ------------------------------------------------------------------------------------------

def test_star_tables_geometry(orc):
    """Antipodes are the opposite directions; the 2D ring's graph links each angle to its two
    neighbours only; the icosphere graph is symmetric, contains every vertex's nearest neighbour
    and has degrees 5..8 (6-nearest made symmetric)."""
    ring = synth.circle_directions(64)
    anti, off, idx = orc.star_tables(ring, 2)
    assert np.allclose(ring[anti], -ring, atol=1e-12)
    for k in range(64):
        assert sorted(idx[off[k]:off[k + 1]]) == sorted([(k - 1) % 64, (k + 1) % 64])
    for sub in (2, 3):
        ico = synth.icosphere(sub)
        anti, off, idx = orc.star_tables(ico, 3)
        assert np.allclose(ico[anti], -ico, atol=1e-6)
        D = len(ico)
        nb = [set(idx[off[k]:off[k + 1]].tolist()) for k in range(D)]
        dots = ico @ ico.T
        np.fill_diagonal(dots, -2.0)
        for k in range(D):
            assert 5 <= len(nb[k]) <= 8
            assert int(np.argmax(dots[k])) in nb[k]
            for j in nb[k]:
                assert k in nb[j]


def _star_case(orc, dim):
    if dim == 3:
        J = _smooth_volume((24, 26, 28))
        p = synth.Params(dim=3, dR=1.0, n_dirs=162, n_rays=32, n_radial=16, flags=1)
        dirs = synth.icosphere(2)
        c = np.array([13.3, 12.1, 11.7])
    else:
        J = _smooth_volume((1, 40, 44))
        p = synth.Params(dim=2, dR=1.0, n_dirs=64, n_rays=16, n_radial=16, flags=1)
        dirs = synth.circle_directions(64)
        c = np.array([21.3, 19.6, 0.0])
    return J, p, dirs, c


@pytest.mark.parametrize("dim", [2, 3])
def test_star_with_tied_radii_is_the_sphere(orc, dim):
    """With every R_k equal to R, one star iteration reproduces the sphere's estimator with the
    rotation off (same Philox draws and points): the energy, the centre force, and the mean over
    directions of the radius steps (the smoothing terms cancel in it), whatever lambda is."""
    J, p, dirs, c = _star_case(orc, dim)
    tables = orc.star_tables(dirs, dim)
    R = 6.4
    for n in (1, 2, 9):
        sph = orc.mc_terms(J, p, dirs, c, R, n, 5)
        for lam in (0.0, 0.7):
            st = orc.star_step_terms(J, p, dirs, tables, lam, c, np.full(p.n_dirs, R), n, 5)
            assert abs(st["E"] - sph["E"]) < 1e-12 * max(1.0, abs(sph["E"]))
            assert np.allclose(st["g_c"][:dim], sph["g_c"][:dim], rtol=1e-11, atol=1e-14)
            eps = p.eps0 / math.sqrt(n)
            assert abs(st["dR"].mean() - (-0.5 * eps * sph["g_R"])) < 1e-11 * (abs(sph["g_R"]) * eps + 1e-12)


@pytest.mark.parametrize("dim", [2, 3])
def test_star_radius_force_is_frozen_point_derivative(orc, dim):
    """Untied radii: for each direction sampled in the iteration, D g_k (from the radius step with
    lambda = 0) equals D times the central difference in R_k of the estimator with its sample points
    and volume factors held fixed, E = sum over rays of (V_ray / (M L)) (2 R_ray)^-d sum_l S I
    (the minus ray takes the radius of the antipodal direction)."""
    J, p, dirs, c = _star_case(orc, dim)
    tables = orc.star_tables(dirs, dim)
    rng = np.random.default_rng(3)
    Rk = rng.uniform(5.5, 7.5, size=p.n_dirs)
    D, M, L = p.n_dirs, p.n_rays, p.n_radial
    V = (4.0 / 3.0 * math.pi if dim == 3 else math.pi)
    for n in (1, 4):
        t = orc.star_step_terms(J, p, dirs, tables, 0.0, c, Rk, n, 7, want_samples=True)
        pts, vals, rdir = t["pts"], t["vals"], t["ray_dir"]
        r = np.linalg.norm(pts[:, :dim] - c[:dim], axis=1)
        vol = V * (Rk[rdir] + 0.5 * p.dR) ** dim

        def E(R):
            w = np.array([orc.weight(dim, r[j], R[rdir[j]], p.dR)[0] for j in range(len(r))])
            return float(np.sum(vol / (M * L) * (2.0 * R[rdir]) ** (-dim) * w * vals))

        # pair m's rays are samples [2m L, (2m + 1) L) along +T_k and [(2m + 1) L, (2m + 2) L) along
        # -T_k: the minus ray uses the antipodal direction's radius, and at each radial index the
        # two distances are in the ratio of the rays' R + dR/2
        anti = tables[0]
        plus = (np.arange(M // 2)[:, None] * 2 * L + np.arange(L)[None, :]).ravel()
        minus = plus + L
        assert np.all(rdir[minus] == anti[rdir[plus]])
        ratio = r[minus] / r[plus]
        expect = (Rk[rdir[minus]] + 0.5 * p.dR) / (Rk[rdir[plus]] + 0.5 * p.dR)
        assert np.allclose(ratio, expect, rtol=1e-12)
        u = (pts[plus, :dim] - c[:dim]) / r[plus, None]
        assert np.allclose(u, dirs[rdir[plus]][:, :dim], atol=1e-12)
        eps = p.eps0 / math.sqrt(n)
        gk = -2.0 * t["dR"] / (eps * D)
        assert abs(E(Rk) - t["E"]) < 1e-12 * max(1.0, abs(t["E"]))
        sampled = np.unique(rdir)
        assert np.all(gk[np.setdiff1d(np.arange(D), sampled)] == 0.0)
        h = 1e-6
        for k in sampled[:12]:
            Rp, Rm = Rk.copy(), Rk.copy()
            Rp[k] += h
            Rm[k] -= h
            fd = (E(Rp) - E(Rm)) / (2 * h)
            assert abs(fd - gk[k]) < 1e-6 * (np.abs(gk).max() + 1e-9), (n, k, fd, gk[k])


def test_star_smoothing_step_on_empty_image(orc):
    """On a zero image the radius steps are the smoothing alone: each radius moves toward the mean
    of its graph neighbours by min(1, eps lambda / 2) of the gap (the neighbour means taken from the
    graph's symmetric edge list), and tied radii do not move."""
    J = np.zeros((20, 22, 24))
    p = synth.Params(dim=3, dR=1.0, n_dirs=162, n_rays=32, n_radial=16, flags=1)
    dirs = synth.icosphere(2)
    tables = orc.star_tables(dirs, 3)
    anti, off, idx = tables
    nb = {k: set() for k in range(p.n_dirs)}
    for k in range(p.n_dirs):
        for j in idx[off[k]:off[k + 1]]:
            nb[k].add(int(j)); nb[int(j)].add(k)
    rng = np.random.default_rng(5)
    Rk = rng.uniform(5.0, 8.0, size=p.n_dirs)
    c = np.array([10.0, 11.0, 9.5])
    for lam, n in ((0.35, 3), (0.35, 100), (5.0, 2)):
        t = orc.star_step_terms(J, p, dirs, tables, lam, c, Rk, n, 1)
        f = min(1.0, 0.5 * p.eps0 / math.sqrt(n) * lam)
        for k in range(p.n_dirs):
            mk = np.mean([Rk[j] for j in nb[k]])
            assert abs(t["dR"][k] - (-f * (Rk[k] - mk))) < 1e-12
        assert t["E"] == 0.0 and np.all(t["g_c"] == 0.0)
    t = orc.star_step_terms(J, p, dirs, tables, 2.0, c, np.full(p.n_dirs, 6.0), 4, 1)
    assert np.all(t["dR"] == 0.0)


def test_star_fits_an_ellipsoid(orc):
    """Behaviour (not a pin): radii started tied at 8 on a blurred axis-aligned ellipsoid (semi-axes
    9, 6, 5) spread along its axes without smoothing: along the long axis they end above, along the
    short axis below, the tied start, apart by most of the cube root of 2 times the axes'
    difference (the per-direction optimum of the energy is that multiple of the blob's radial
    extent); strong smoothing keeps them nearly tied; the centre stays on the blob's."""
    shape = (48, 48, 48)
    z, y, x = np.meshgrid(*[np.arange(k, dtype=np.float64) for k in shape], indexing="ij")
    ax = np.array([9.0, 6.0, 5.0])
    cen = np.array([23.7, 24.2, 23.9])
    ind = (((x - cen[0]) / ax[0]) ** 2 + ((y - cen[1]) / ax[1]) ** 2 + ((z - cen[2]) / ax[2]) ** 2 < 1.0)
    from scipy.ndimage import gaussian_filter
    J = gaussian_filter(ind.astype(float), 1.0)
    dirs = synth.icosphere(2)
    p = synth.Params(dim=3, dR=1.0, n_dirs=162, n_rays=64, n_radial=16, flags=1, eps0=8.0, r_max=20.0,
                     conv_window=0, r_init=8.0)
    tables = orc.star_tables(dirs, 3)
    spread = {}
    for lam in (0.0, 5.0):
        st = orc.star_init(p, cen[None, :])
        orc.star_evolve(J, p, dirs, tables, lam, st, 300)
        along = lambda a: st.Rk[0][np.abs(dirs[:, a]) > 0.9].mean()
        spread[lam] = along(0) - along(2)
        if lam == 0.0:
            assert along(0) > 8.0 > along(2)
        assert np.linalg.norm(st.c[0] - cen) < 0.5
    assert spread[0.0] > 0.6 * 2 ** (1 / 3) * (ax[0] - ax[2]), spread
    assert abs(spread[5.0]) < 0.25 * spread[0.0], spread


def test_constant_image_has_no_force(orc):
    """Constant image: the c-force vanishes exactly for antithetic pairs, and A, B_R are zero in
    expectation (Sec. II-B: the energy does not move contours in uniform regions)."""
    J = np.full((20, 20, 20), 3.0)
    p = synth.Params(dim=3, dR=1.0, n_dirs=162, n_rays=32, n_radial=16)
    dirs = synth.icosphere(2)
    c = np.array([9.5, 10.1, 9.8])
    R = 5.0
    A, BR = [], []
    for n in range(1, 801):
        t = orc.mc_terms(J, p, dirs, c, R, n, 1)
        assert np.all(np.abs(t["B_c"]) < 1e-10)
        A.append(t["A"]); BR.append(t["B_R"])
    for x in (np.array(A), np.array(BR)):
        assert abs(x.mean()) < 4.5 * x.std() / math.sqrt(len(x))


# ------------------------------------------------------------------------------------------
# pre-pass and interpolation against scipy
# ------------------------------------------------------------------------------------------

@pytest.mark.parametrize("dtype", [np.uint8, np.uint16, np.float32])
def test_prepass_matches_scipy_gaussian(orc, dtype):
    from scipy.ndimage import gaussian_filter1d
    rng = np.random.default_rng(2)
    raw = rng.integers(0, 250, size=(11, 17, 23)).astype(dtype)
    p = synth.Params(dim=3, spacing=(1.0, 1.0, 2.0), sigma_pre=1.3, i_offset=17.0, i_scale=0.01)
    J = orc.prepass(raw, p)
    ref = (raw.astype(np.float64) - 17.0) * 0.01
    for axis, h in ((2, 1.0), (1, 1.0), (0, 2.0)):
        s = 1.3 / h
        ref = gaussian_filter1d(ref, s, axis=axis, mode="nearest", radius=int(math.ceil(3 * s)))
    assert np.max(np.abs(J - ref)) < 1e-12


def test_prepass_2d_and_disabled(orc):
    from scipy.ndimage import gaussian_filter1d
    rng = np.random.default_rng(4)
    raw = rng.integers(0, 250, size=(1, 19, 21)).astype(np.uint8)
    p = synth.Params(dim=2, sigma_pre=1.1)
    J = orc.prepass(raw, p)
    ref = raw.astype(np.float64)[0]
    for axis in (1, 0):
        ref = gaussian_filter1d(ref, 1.1, axis=axis, mode="nearest", radius=4)
    assert np.max(np.abs(J[0] - ref)) < 1e-12
    J0 = orc.prepass(raw, p.replace(sigma_pre=0.0, i_offset=3.0, i_scale=2.0))
    assert np.array_equal(J0, (raw.astype(np.float64) - 3.0) * 2.0)


def test_interp_matches_scipy_map_coordinates(orc):
    from scipy.ndimage import map_coordinates
    rng = np.random.default_rng(6)
    J = rng.normal(size=(7, 9, 11))
    pts = rng.uniform(-2.5, 13.0, size=(3000, 3))
    got = np.array([orc.interp(J, 3, v) for v in pts])
    ref = map_coordinates(J, pts[:, ::-1].T, order=1, mode="nearest")
    assert np.max(np.abs(got - ref)) < 1e-12
    J2 = rng.normal(size=(1, 9, 11))
    got2 = np.array([orc.interp(J2, 2, v) for v in pts[:, :2]])
    ref2 = map_coordinates(J2[0], pts[:, 1::-1].T, order=1, mode="nearest")
    assert np.max(np.abs(got2 - ref2)) < 1e-12


# ------------------------------------------------------------------------------------------
# exact energy (Eq. (5))
# ------------------------------------------------------------------------------------------

@pytest.mark.parametrize("dim", [2, 3])
def test_energy_vox_bruteforce(orc, dim):
    rng = np.random.default_rng(8)
    if dim == 3:
        J = rng.normal(size=(10, 12, 14))
        p = synth.Params(dim=3, spacing=(1.0, 1.0, 2.0), dR=0.75)
    else:
        J = rng.normal(size=(1, 15, 13))
        p = synth.Params(dim=2, dR=1.0)
    nz, ny, nx = J.shape
    h = np.array(p.spacing)
    cs = rng.uniform(-1.0, 14.0, size=(6, 3))
    if dim == 2:
        cs[:, 2] = 0.0
    Rs = rng.uniform(4.0, 7.0, size=6)
    e, _ = orc.energy_vox(J, p, cs, Rs)
    kz, ky, kx = np.meshgrid(np.arange(-20, 40) if dim == 3 else np.array([0]), np.arange(-20, 40),
                             np.arange(-20, 40), indexing="ij")
    vals = J[np.clip(kz, 0, nz - 1), np.clip(ky, 0, ny - 1), np.clip(kx, 0, nx - 1)]
    for i in range(6):
        d = np.sqrt((kx * h[0] - cs[i, 0]) ** 2 + (ky * h[1] - cs[i, 1]) ** 2 +
                    ((kz * h[2] - cs[i, 2]) ** 2 if dim == 3 else 0.0))
        m = d < Rs[i] + 0.5 * p.dR
        S = orc.weight_vec(dim, d[m], Rs[i], p.dR)[:, 0]
        meas = h[0] * h[1] * (h[2] if dim == 3 else 1.0)
        want = meas * float((S * vals[m]).sum()) / (2 * Rs[i]) ** dim
        assert abs(e[i] - want) < 1e-12 * max(1.0, abs(want))


# ------------------------------------------------------------------------------------------
# symmetry of the whole iteration
# ------------------------------------------------------------------------------------------

def test_cube_symmetry_exact(orc):
    """Swapping the x and y axes, or mirroring x, of the volume, the direction table and the
    seeds (rotation disabled so the sampling frame moves with them) gives the same contours."""
    wl = synth.tiny_config()
    p = wl.params.replace(flags=1)
    J = orc.prepass(wl.raw, p)
    base = orc.init_state(p, wl.seeds)
    orc.evolve(J, p, wl.dirs, base, 12)

    Jt = np.ascontiguousarray(J.transpose(0, 2, 1))
    st = orc.init_state(p, wl.seeds[:, [1, 0, 2]])
    orc.evolve(Jt, p, wl.dirs[:, [1, 0, 2]], st, 12)
    assert np.allclose(st.c[:, [1, 0, 2]], base.c, atol=1e-9)
    assert np.allclose(st.R, base.R, atol=1e-9)

    Jf = np.ascontiguousarray(J[:, :, ::-1])
    seeds = wl.seeds.copy(); seeds[:, 0] = 63.0 - seeds[:, 0]
    dirs = wl.dirs.copy(); dirs[:, 0] = -dirs[:, 0]
    st = orc.init_state(p, seeds)
    orc.evolve(Jf, p, dirs, st, 12)
    cf = st.c.copy(); cf[:, 0] = 63.0 - cf[:, 0]
    assert np.allclose(cf, base.c, atol=1e-9)
    assert np.allclose(st.R, base.R, atol=1e-9)


# ------------------------------------------------------------------------------------------
# the whole iteration settles at the minimiser of the continuous energy
# ------------------------------------------------------------------------------------------

def _fibonacci_sphere(n):
    k = np.arange(n) + 0.5
    z = 1.0 - 2.0 * k / n
    phi = k * math.pi * (3.0 - math.sqrt(5.0))
    s = np.sqrt(1.0 - z * z)
    return np.stack([s * np.cos(phi), s * np.sin(phi), z], 1)


def _quadrature_energy(orc, J, h, dim, dR, c, R, dirs, ngl):
    """(2R)^-d times the integral of S(|x - c|; R) I(x) over the ball |x - c| < R + dR/2 (Eq. (5)
    with the lattice sum replaced by the integral the sampler estimates), I the trilinear
    (bilinear) interpolant of J by scipy: Gauss-Legendre in r on each interval where S is linear,
    times an equal-weight angular rule."""
    from scipy.ndimage import map_coordinates
    from scipy.special import roots_legendre
    rho = 2.0 ** (-1.0 / dim)
    a, dr = rho * R, rho * dR
    br = [0.0, a - dr / 2, a + dr / 2, R - dR / 2, R + dR / 2]
    x, w = roots_legendre(ngl)
    r = np.concatenate([lo + (hi - lo) * (x + 1) / 2 for lo, hi in zip(br[:-1], br[1:])])
    wr = np.concatenate([w * (hi - lo) / 2 for lo, hi in zip(br[:-1], br[1:])])
    S = orc.weight_vec(dim, r, R, dR)[:, 0]
    P = c[None, None, :dim] + r[None, :, None] * dirs[:, None, :]
    v = P / np.asarray(h[:dim])
    Jd = J if dim == 3 else J[0]
    I = map_coordinates(Jd, [v[..., ax].ravel() for ax in range(dim)][::-1], order=1,
                        mode="nearest").reshape(P.shape[:2])
    sphere = 4.0 * math.pi if dim == 3 else 2.0 * math.pi
    return sphere * float((I * (S * wr * r ** (dim - 1))[None, :]).mean(0).sum()) / (2.0 * R) ** dim


def _quadrature_minimiser(orc, J, h, dim, dR, c, lo, hi):
    """argmin over R of the quadrature energy at the fixed centre c: coarse scan, then a parabola
    through a fine scan around the best coarse point."""
    if dim == 3:
        coarse, fine = _fibonacci_sphere(2000), _fibonacci_sphere(20000)
    else:
        t = (np.arange(4096) + 0.5) * 2.0 * math.pi / 4096
        coarse = fine = np.stack([np.cos(t), np.sin(t)], 1)
    Rs = np.arange(lo, hi, 0.1)
    Es = [_quadrature_energy(orc, J, h, dim, dR, c, R, coarse, 8) for R in Rs]
    Rf = np.linspace(-0.1, 0.1, 11) + Rs[int(np.argmin(Es))]
    Ef = [_quadrature_energy(orc, J, h, dim, dR, c, R, fine, 24) for R in Rf]
    cf = np.polyfit(Rf, Ef, 2)
    assert cf[0] > 0
    return -cf[1] / (2.0 * cf[0])


def _symmetric_blob(which):
    """A blob point-symmetric about a lattice point c0 (so that c0 is a stationary centre of the
    interpolated image too), with its volume J, parameters and direction table."""
    if which == "ball":
        h, shape, c0 = (1.0, 1.0, 1.0), (49, 49, 49), np.array([24.0, 24.0, 24.0])
        z, y, x = np.meshgrid(*[np.arange(n) for n in shape], indexing="ij")
        J = synth.blurred_ball(np.sqrt((x - 24.0) ** 2 + (y - 24.0) ** 2 + (z - 24.0) ** 2), 6.0, 1.0, 3)
        p = synth.Params(dim=3, spacing=h, dR=1.0, n_dirs=642, n_rays=64)
        dirs = synth.icosphere(3)
    elif which == "ellipsoid":
        # semi-axes 7, 5, 4 in a random orientation on the anisotropic grid h = (1, 1, 2)
        h, shape, c0 = (1.0, 1.0, 2.0), (25, 49, 49), np.array([24.0, 24.0, 24.0])
        rot = synth._random_rotation(np.random.default_rng(7))
        cov = synth.render_ellipsoids(shape, h, c0[None], np.array([[7.0, 5.0, 4.0]]), rot[None], ss=4)
        J = synth._blur(cov, 1.0)
        p = synth.Params(dim=3, spacing=h, dR=0.75, n_dirs=642, n_rays=64)
        dirs = synth.icosphere(3)
    else:
        h, shape, c0 = (1.0, 1.0, 1.0), (1, 65, 65), np.array([32.0, 32.0, 0.0])
        y, x = np.meshgrid(np.arange(65), np.arange(65), indexing="ij")
        J = synth.blurred_ball(np.sqrt((x - 32.0) ** 2 + (y - 32.0) ** 2), 8.0, 1.0, 2)[None]
        p = synth.Params(dim=2, spacing=h, dR=1.0, n_dirs=64, n_rays=16)
        dirs = synth.circle_directions(64)
    p = p.replace(sigma_pre=0.0, i_offset=0.0, i_scale=1.0, eps0=8.0, r_min=0.0, r_max=20.0,
                  n_radial=16, conv_window=0)
    return np.ascontiguousarray(J, dtype=np.float64), h, c0, p, dirs


@pytest.mark.parametrize("which,starts,n_iter,tol", [
    ("ball", (6.2, 9.5), 1500, 0.01),
    ("disk", (9.0, 14.0), 1500, 0.01),
    ("ellipsoid", (6.2, 8.0), 4000, 0.015),
])
def test_iteration_settles_at_the_continuous_minimiser(orc, which, starts, n_iter, tol):
    """The sampler's forces are unbiased estimates of the exact derivatives of the continuous energy
    (S vanishes on the ball's outer edge, so moving that edge contributes nothing), hence the
    descent with steps eps0 / sqrt(n) (Sec. II-D) settles where an independent quadrature of that
    energy (scipy interpolation, Gauss-Legendre and angular rules) has its minimum over R at the
    blob's centre. Contours started below and above the optimum, 32 Philox streams each, must end
    with mean radius within tol of that minimiser and mean centre at the blob's centre. A dropped
    normalisation term, a wrong sign, or a sampler that is not uniform in the ball moves the
    settling point far beyond tol."""
    J, h, c0, p, dirs = _symmetric_blob(which)
    dim = p.dim
    rstar = _quadrature_minimiser(orc, J, h, dim, p.dR, c0, 5.0, 16.0)
    K = 32
    rng = np.random.default_rng(3)
    seeds = c0[None] + rng.uniform(-1.0, 1.0, size=(K, 3)) * (np.arange(3) < dim)
    for r0 in starts:
        st = orc.init_state(p, seeds, r0=r0, ids=np.arange(K, dtype=np.uint32) * 7 + 3, shape_zyx=J.shape)
        orc.evolve(J, p, dirs, st, n_iter)
        assert np.all(st.status == orc.ACTIVE) and np.all(st.iters == n_iter)
        assert abs(st.R.mean() - rstar) < tol, (which, r0, st.R.mean(), rstar)
        assert st.R.std() < 0.05, (which, r0, st.R.std())
        assert np.max(np.abs(st.c.mean(0) - c0)[:dim]) < 0.05, (which, r0, st.c.mean(0))


# ------------------------------------------------------------------------------------------
# stop rule and selection (Results)
# ------------------------------------------------------------------------------------------

def test_status_rules(orc):
    J = np.zeros((20, 20, 20))
    p = synth.Params(dim=3, dR=1.0, r_init=5.0, conv_tol=1e-3, conv_window=3)
    dirs = synth.icosphere(2)
    st = orc.init_state(p, np.array([[10.0, 10.0, 10.0], [0.0, 19.0, 5.0]]))
    orc.evolve(J, p, dirs, st, 10)
    # zero image: no force at all -> converged after exactly conv_window steps
    assert list(st.status) == [orc.CONVERGED, orc.CONVERGED] and list(st.iters) == [3, 3]
    # radius clamping to the geometric minimum
    p2 = p.replace(r_init=1.0)
    assert abs(orc.initial_radius(p2, 1.0) - orc.r_geom_min(3, 1.0)) < 1e-15
    assert abs(orc.r_geom_min(3, 1.0) - (1 + RHO3) / (2 * (1 - RHO3))) < 1e-15
    # a contour pushed out of the volume is marked OUT
    Jr = np.zeros((20, 20, 20)); Jr[:, :, :4] = 1.0
    p3 = p.replace(eps0=400.0, conv_window=0)
    st3 = orc.init_state(p3, np.array([[3.0, 10.0, 10.0]]))
    orc.evolve(Jr, p3, dirs, st3, 50)
    assert (st3.status[0] & 0x0F) == orc.OUT and st3.c[0, 0] < 0.0 and st3.iters[0] < 50


def test_cull_hand_cases(orc):
    p = synth.Params(dim=3, e0=-0.05)
    thr = lambda R: RHO3 * R
    R = np.array([6.0, 6.0, 6.0, 6.0, 5.0])
    d = 0.9 * thr(6.0)
    # chain 0-1-2 along x with neighbours overlapping but 0, 2 apart; 3 isolated above E0; 4 OUT
    c = np.array([[0.0, 0, 0], [d, 0, 0], [2 * d, 0, 0], [100.0, 0, 0], [0.5, 0, 0]])
    e = np.array([-0.3, -0.2, -0.25, -0.01, -0.9])
    status = np.array([orc.MAXITER, orc.CONVERGED, orc.MAXITER | orc.CLAMPED, orc.MAXITER, orc.OUT], np.uint8)
    ids = np.arange(5, dtype=np.uint32)
    keep = orc.cull(p, c, R, e, status, ids)
    assert list(keep) == [1, 0, 1, 0, 0]
    # middle one lowest: it suppresses both neighbours
    e2 = np.array([-0.3, -0.4, -0.25, -0.06, -0.9])
    assert list(orc.cull(p, c, R, e2, status, ids)) == [0, 1, 0, 1, 0]
    # tie in energy: lower id wins
    c3 = np.array([[0.0, 0, 0], [1.0, 0, 0]])
    keep3 = orc.cull(p, c3, np.array([6.0, 6.0]), np.array([-0.2, -0.2]),
                     np.array([2, 2], np.uint8), np.array([7, 3], np.uint32))
    assert list(keep3) == [0, 1]
    # overlap uses rho * max(R', R''): distance just inside / outside
    c4 = np.array([[0.0, 0, 0], [thr(8.0) - 1e-6, 0, 0], [50.0, 0, 0], [50.0 + thr(8.0) + 1e-6, 0, 0]])
    keep4 = orc.cull(p, c4, np.array([4.0, 8.0, 4.0, 8.0]), np.array([-0.2, -0.3, -0.2, -0.3]),
                     np.full(4, 2, np.uint8), np.arange(4, dtype=np.uint32))
    assert list(keep4) == [0, 1, 1, 1]


def test_cull_threshold_order_irrelevant(orc):
    """Thresholding before or after the competition selects the same set (greedy in ascending
    energy): compare against a brute-force greedy over all contours followed by the threshold."""
    rng = np.random.default_rng(12)
    p = synth.Params(dim=3, e0=-0.1)
    for trial in range(20):
        n = 60
        c = rng.uniform(0, 30, size=(n, 3))
        R = rng.uniform(3, 8, size=n)
        e = rng.uniform(-0.3, 0.05, size=n)
        status = np.full(n, orc.MAXITER, np.uint8)
        ids = rng.permutation(n).astype(np.uint32)
        keep = orc.cull(p, c, R, e, status, ids)
        order = sorted(range(n), key=lambda i: (e[i], ids[i]))
        acc = []
        for i in order:
            if all(np.linalg.norm(c[i] - c[j]) >= RHO3 * max(R[i], R[j]) for j in acc):
                acc.append(i)
        want = np.zeros(n, np.uint8)
        for i in acc:
            if e[i] <= p.e0:
                want[i] = 1
        assert np.array_equal(keep, want)


def test_lattice_seeds(orc):
    """Initial lattice (figures of Sec. II-A / II-B): neighbours sqrt(1.5) R0 apart along each axis,
    centred in the volume, every centre inside."""
    p = synth.Params(dim=3, spacing=(1.0, 1.0, 2.0), r_init=6.0)
    shape = (23, 61, 50)   # z, y, x
    pts = orc.lattice_seeds(p, shape)
    pitch = np.sqrt(1.5) * 6.0
    ext = (np.array([50, 61, 23]) - 1) * np.array([1.0, 1.0, 2.0])
    k = np.maximum(1, np.floor(ext / pitch)).astype(int)
    assert len(pts) == k.prod()
    for a in range(3):
        u = np.unique(np.round(pts[:, a], 9))
        assert len(u) == k[a]
        assert np.allclose(np.diff(u), pitch)
        assert abs((u[0] + u[-1]) / 2 - ext[a] / 2) < 1e-9     # centred
        assert u[0] >= 0 and u[-1] <= ext[a]
    p2 = synth.Params(dim=2, r_init=5.0)
    pts2 = orc.lattice_seeds(p2, (1, 30, 40))
    assert np.all(pts2[:, 2] == 0.0) and len(pts2) == int(29 // np.sqrt(37.5)) * int(39 // np.sqrt(37.5))


def _greedy_cull(c, R, e, live, ids, young, e0, dim, compete=True):
    """Brute-force reference of one culling pass: which live contours survive."""
    rho = 2.0 ** (-1.0 / dim)
    cand = [i for i in range(len(R)) if live[i] and np.isfinite(e[i]) and (young or e[i] <= e0)]
    cand.sort(key=lambda i: (e[i], ids[i]))
    acc = []
    for i in cand:
        if not compete or all(np.linalg.norm(c[i, :dim] - c[j, :dim]) >= rho * max(R[i], R[j]) for j in acc):
            acc.append(i)
    return set(acc)


@pytest.mark.parametrize("seed,young,e_cull,compete", [(4, False, -0.0025, True), (5, False, -0.0025, False),
                                                      (6, True, -0.0025, False), (7, False, 0.01, False)])
def test_cull_pass_threshold_and_competition_options(orc, seed, young, e_cull, compete):
    """The pass's own threshold e_cull replaces E0 for its candidates (a laxer one keeps contours
    that are not yet cells), and with the competition switched off every candidate survives: the
    pass retires exactly the live contours the brute force retires, and nothing else."""
    rng = np.random.default_rng(seed)
    p = synth.Params(dim=3, dR=1.0, e0=-0.01)
    n = 150
    c = np.column_stack([rng.uniform(2, 31, n), rng.uniform(2, 29, n), rng.uniform(2, 17, n)])
    R = rng.uniform(4.4, 8.0, n)
    status = rng.choice([orc.ACTIVE, orc.CONVERGED, orc.MAXITER, orc.OUT], size=n, p=[0.5, 0.3, 0.1, 0.1])
    status = status.astype(np.uint8) | np.where(rng.random(n) < 0.2, orc.CLAMPED, 0).astype(np.uint8)
    ids = rng.permutation(n).astype(np.uint32)
    e_mc = rng.uniform(-0.03, 0.02, n)
    e_mc[::31] = np.nan
    st = orc.State(c=c.copy(), R=R.copy(), iters=np.zeros(n, np.int32), status=status.copy(),
                   streak=np.zeros(n, np.uint8), e_mc=e_mc.copy(), ids=ids)
    k = orc.cull_pass(p, st, young, e_cull=e_cull, compete=compete)
    live = np.isin(status & 0x0F, [orc.ACTIVE, orc.CONVERGED])
    keep = _greedy_cull(c, R, e_mc, live, ids, young, e_cull, 3, compete)
    for i in range(n):
        if not live[i] or i in keep:
            assert st.status[i] == status[i]
        else:
            assert st.status[i] == (status[i] & orc.CLAMPED) | orc.CULLED
    assert k == int(live.sum()) - len(keep)
    # the laxer threshold keeps every live contour between E0 and e_cull that the E0 pass retires
    if not young and not compete and e_cull > p.e0:
        between = live & np.isfinite(e_mc) & (e_mc > p.e0) & (e_mc <= e_cull)
        assert between.sum() > 0 and all(i in keep for i in np.where(between)[0])
    # without competition and outside the grace period the pass is a pure threshold
    if not compete and not young:
        assert keep == set(np.where(live & np.isfinite(e_mc) & (e_mc <= e_cull))[0].tolist())


@pytest.mark.parametrize("seed,young", [(0, False), (1, False), (2, True), (3, True)])
def test_cull_pass_matches_brute_force(orc, seed, young):
    """A culling pass retires exactly the live contours that lose the greedy competition (ranked by
    E_mc), and after the run's grace period also those above E0; other statuses are untouched and
    keep their clamp flag."""
    rng = np.random.default_rng(seed)
    p = synth.Params(dim=3, dR=1.0, e0=-0.01)
    n = 120
    c = np.column_stack([rng.uniform(2, 31, n), rng.uniform(2, 29, n), rng.uniform(2, 17, n)])
    R = rng.uniform(4.4, 8.0, n)
    status = rng.choice([orc.ACTIVE, orc.CONVERGED, orc.MAXITER, orc.OUT], size=n, p=[0.5, 0.3, 0.1, 0.1])
    status = status.astype(np.uint8) | np.where(rng.random(n) < 0.2, orc.CLAMPED, 0).astype(np.uint8)
    iters = rng.integers(0, 60, n).astype(np.int32)
    ids = rng.permutation(n).astype(np.uint32)
    e_mc = rng.uniform(-0.08, 0.02, n)
    e_mc[::29] = np.nan
    st = orc.State(c=c.copy(), R=R.copy(), iters=iters.copy(), status=status.copy(),
                   streak=np.zeros(n, np.uint8), e_mc=e_mc.copy(), ids=ids)
    k = orc.cull_pass(p, st, young)
    live = np.isin(status & 0x0F, [orc.ACTIVE, orc.CONVERGED])
    keep = _greedy_cull(c, R, e_mc, live, ids, young, p.e0, 3)
    for i in range(n):
        if not live[i]:
            assert st.status[i] == status[i]
        elif i in keep:
            assert st.status[i] == status[i]
        else:
            assert st.status[i] == (status[i] & orc.CLAMPED) | orc.CULLED
    assert k == int(live.sum()) - len(keep)
    assert 0 < k < int(live.sum())
