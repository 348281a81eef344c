"""Free-run comparison of a GPU result with the FP64 oracle's own run of the same contours.

The bar (the parity contract of the free run):
  * iteration counts: each GPU count lies in the range the oracle's stop rule allows when every
    convergence decision whose move lies within STOP_DELTA * conv_tol of conv_tol may go either way
    (`oracle.stop_ranges` on the oracle's per-step moves of the same run with the freeze switched
    off); a contour whose count differs from the oracle's must therefore be one with such a near
    decision; statuses agree where the counts agree;
  * every contour (not only those with equal counts): |R_gpu - R_ref| <= 0.05 voxel and
    |c_gpu - c_ref| <= 0.5 voxel;
  * exact energy: |E_gpu - E_ref| <= 1e-5 * max(|E_ref|, E_abs) with E_ref the oracle's Eq. (5) sum at
    the GPU's own final state;
  * selection: the kept set equals the oracle run's own kept set, apart from decisions
    `oracle.cull_ambiguity_tol` flags when each contour's tolerances are the two runs' own
    disagreement in its energy and in its centre plus radius (and contours whose status differs).
"""
import sys

import numpy as np

import oracle

# relative band around conv_tol within which a convergence decision may go either way between
# an FP32 and an FP64 trajectory of the same contour
STOP_DELTA = 1e-2


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def tol_check(name, got, ref, ref_abs, slack, rel=1e-5):
    got, ref = np.asarray(got, np.float64), np.asarray(ref, np.float64)
    tol = rel * np.maximum(np.abs(ref), ref_abs) + slack + 1e-30
    err = np.abs(got - ref)
    bad = np.where(err > tol)[0]
    assert len(bad) == 0, (f"{name}: {len(bad)} of {len(ref)} outside tolerance; worst "
                           f"idx {bad[:5]} got {got[bad[:5]]} ref {ref[bad[:5]]} tol {tol[bad[:5]]}")
    return float(np.max(err / tol)) if len(ref) else 0.0


# the oracle's band around a kink of S, in units of s_max = R + dR/2 (its ORC_KINK_REL)
KINK_REL = 1.5e-6


def expected_kinked_steps(p, radii):
    """Expected number of Monte-Carlo contour-steps with at least one radial point within
    KINK_REL * s_max of a kink of S, for steps at the given radii R: a point sits at s_max * e with
    e^d uniform on (0, 1), so it falls in the band of a kink at e_k with probability about
    2 KINK_REL d e_k^(d-1) (half that at e_k = 1), and a step has (M/2) * L independent radii."""
    d = p.dim
    rho = 2.0 ** (-1.0 / d)
    R = np.asarray(radii, np.float64)
    smax = R + 0.5 * p.dR
    ek = [(rho * R - 0.5 * rho * p.dR) / smax, np.full_like(R, rho), (R - 0.5 * p.dR) / smax]
    q = sum(2.0 * KINK_REL * d * np.clip(e, 0.0, 1.0) ** (d - 1) for e in ek) + KINK_REL * d
    n_r = (p.n_rays // 2) * p.n_radial
    return float(np.sum(1.0 - (1.0 - q) ** n_r))


def oracle_reference(raw, p, dirs, seeds, n_iter, ids=None, r0=None, delta=STOP_DELTA):
    """The oracle's whole run (pre-pass, evolution with the stop rule, exact energy, selection) and
    the stop ranges of each contour from a second run with the freeze switched off."""
    ref = oracle.run(raw, p, dirs, seeds, n_iter, r0=r0, ids=ids)
    n = len(ref["state"].R)
    free = oracle.init_state(p.replace(conv_window=0), seeds, r0=r0, ids=ids, shape_zyx=raw.shape)
    moves = np.full((n, n_iter), np.nan)
    oracle.evolve(ref["J"], p.replace(conv_window=0), dirs, free, n_iter, moves=moves)
    n_stop, n_lo, n_hi, _ = oracle.stop_ranges(moves, p, delta)
    # the frozen run follows the unfrozen trajectory up to its stop
    assert np.array_equal(n_stop, ref["state"].iters), "stop rule replay disagrees with the oracle run"
    ref["stop"] = (n_stop, n_lo, n_hi)
    ref["moves"] = moves
    return ref


def check_free_run(got, ref, p, label, r_tol=0.05, c_tol=0.5):
    """Asserts the free-run bar (module docstring) and returns a summary dict."""
    st = ref["state"]
    n = len(st.R)
    n_stop, n_lo, n_hi = ref["stop"]
    it = np.asarray(got["iters"])
    same = it == st.iters
    in_range = (it >= n_lo) & (it <= n_hi)
    near = n_lo < n_hi
    bad = np.where(~in_range)[0]
    assert len(bad) == 0, (f"{label}: {len(bad)} contours stop outside the oracle's range; first "
                           f"{[(int(i), int(it[i]), int(n_lo[i]), int(n_hi[i])) for i in bad[:5]]}")
    assert np.all(same | near)
    assert np.array_equal(got["status"][same], st.status[same]), label
    dR = np.abs(got["radii"] - st.R)
    dc = np.linalg.norm(got["centers"] - st.c, axis=1)
    assert np.max(dR, initial=0.0) <= r_tol, (label, float(np.max(dR)), int(np.argmax(dR)))
    assert np.max(dc, initial=0.0) <= c_tol, (label, float(np.max(dc)), int(np.argmax(dc)))
    # exact energy at the GPU's own final state
    e_ref, e_abs = oracle.energy_vox(ref["J"], p, got["centers"], got["radii"].astype(np.float64))
    fin = np.isfinite(e_ref)
    worst_e = tol_check(f"{label} E_vox", got["e_vox"][fin], e_ref[fin], e_abs[fin], 0.0, rel=1e-5)
    # kept set against the oracle run's own kept set
    e_gpu = got["e_vox"].astype(np.float64)
    tol_e = np.abs(e_gpu - ref["e_vox"]) + 1e-5 * np.maximum(np.abs(ref["e_vox"]), ref["e_abs"])
    tol_d = dc + dR + 1e-6
    cand = lambda s: np.isin(s & 0x0F, (oracle.CONVERGED, oracle.MAXITER))
    tol_e[cand(got["status"]) != cand(st.status)] = np.inf
    tol_e[~np.isfinite(tol_e)] = np.inf
    amb = oracle.cull_ambiguity_tol(p, st.c, st.R, ref["e_vox"], tol_e, tol_d)
    ok = amb == 0
    mism = np.where((got["keep"] != ref["keep"]) & ok)[0]
    assert len(mism) == 0, (f"{label}: kept sets differ on {len(mism)} unflagged contours, e.g. "
                            f"{[(int(i), int(got['keep'][i]), int(ref['keep'][i])) for i in mism[:5]]}")
    out = {"contours": n, "same_iters": int(same.sum()), "near_tau": int(near.sum()),
           "differing_iters": int((~same).sum()), "max_dR": float(np.max(dR, initial=0.0)),
           "max_dc": float(np.max(dc, initial=0.0)), "max_dR_same": float(np.max(dR[same], initial=0.0)),
           "worst_E_vox_err_over_tol": worst_e, "kept_gpu": int(got["keep"].sum()),
           "kept_oracle": int(ref["keep"].sum()), "selection_flagged": int(amb.sum()),
           "kept_differing_flagged": int(np.sum(got["keep"] != ref["keep"]))}
    say(f"  {label}: " + ", ".join(f"{k} {v:.4g}" if isinstance(v, float) else f"{k} {v}" for k, v in out.items()))
    return out
