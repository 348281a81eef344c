"""FP64 CPU oracle of snakuscule evolution -- TEST INFRASTRUCTURE ONLY.

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py`` may
import this package. The product path (the HIP library and its Python binding) never imports,
links or calls it, and shares no code with it: the C source ``snk_oracle.c`` carries its own
Philox, Gaussian pre-pass, interpolation, weight function, estimator, update and selection.

This module is argument marshalling around ``libsnk_oracle.so`` (built with plain gcc, OpenMP
over contours, no fast-math).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "snk_oracle.c")
_LIB = os.path.join(_HERE, "libsnk_oracle.so")

TRACE_W = 32
ACTIVE, CONVERGED, MAXITER, OUT, NONFINITE, CULLED, CLAMPED = 0, 1, 2, 3, 4, 5, 0x10


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, no fast-math, OpenMP)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-Wall",
                               "-Wno-unknown-pragmas", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Params(C.Structure):
    _fields_ = [("dim", C.c_int32), ("spacing", C.c_double * 3), ("sigma_pre", C.c_double),
                ("i_offset", C.c_double), ("i_scale", C.c_double), ("dR", C.c_double),
                ("eps0", C.c_double), ("r_min", C.c_double), ("r_max", C.c_double),
                ("r_init", C.c_double), ("n_dirs", C.c_int32), ("n_rays", C.c_int32),
                ("n_radial", C.c_int32), ("seed", C.c_uint64), ("conv_tol", C.c_double),
                ("conv_window", C.c_int32), ("e0", C.c_double), ("flags", C.c_int32)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = C.CDLL(_LIB)
        P = C.POINTER
        d, i64, i32, u32 = C.c_double, C.c_int64, C.c_int32, C.c_uint32
        vp = C.c_void_p
        L.orc_philox4x32_10.argtypes = [P(C.c_uint32), P(C.c_uint32), P(C.c_uint32)]
        L.orc_uniform.argtypes = [u32]; L.orc_uniform.restype = d
        L.orc_r_geom_min.argtypes = [C.c_int, d]; L.orc_r_geom_min.restype = d
        L.orc_weight.argtypes = [C.c_int, d, d, d, P(d)]
        L.orc_weight_many.argtypes = [C.c_int, vp, i64, d, d, vp]
        L.orc_prepass.argtypes = [vp, C.c_int, i64, i64, i64, P(_Params), vp]
        L.orc_interp.argtypes = [vp, i64, i64, i64, C.c_int, d, d, d]; L.orc_interp.restype = d
        L.orc_interp_grad.argtypes = [vp, i64, i64, i64, C.c_int, d, d, d, P(d)]
        L.orc_interp_grad.restype = d
        L.orc_star_tables.argtypes = [C.c_int, vp, i32, vp, vp, vp, i32]
        L.orc_star_tables.restype = i32
        L.orc_star_step_terms.argtypes = [vp, i64, i64, i64, P(_Params), vp, vp, vp, vp, d, P(d), vp, u32, u32,
                                          P(d), vp, vp, vp, vp, vp, vp]
        L.orc_star_evolve.argtypes = [vp, i64, i64, i64, P(_Params), vp, vp, vp, vp, d, i64, vp, vp, vp, vp,
                                      vp, vp, vp, vp, i32]
        L.orc_star_evolve.restype = i64
        L.orc_rotation.argtypes = [P(_Params), u32, u32, P(d)]
        L.orc_initial_radius.argtypes = [P(_Params), d]; L.orc_initial_radius.restype = d
        L.orc_evolve.argtypes = [vp, i64, i64, i64, P(_Params), vp, i64, vp, vp, vp, vp, vp, vp, vp,
                                 i32, vp, P(i64)]
        L.orc_evolve.restype = i64
        L.orc_evolve_log.argtypes = [vp, i64, i64, i64, P(_Params), vp, i64, vp, vp, vp, vp, vp, vp, vp,
                                     i32, vp, vp, P(i64)]
        L.orc_evolve_log.restype = i64
        L.orc_mc_terms.argtypes = [vp, i64, i64, i64, P(_Params), vp, P(d), d, u32, u32, P(d), vp, vp]
        L.orc_energy_fixed.argtypes = [C.c_int, d, vp, vp, i64, d, P(d), d]
        L.orc_energy_fixed.restype = d
        L.orc_energy_vox.argtypes = [vp, i64, i64, i64, P(_Params), i64, vp, vp, vp, vp]
        L.orc_cull.argtypes = [P(_Params), i64, vp, vp, vp, vp, vp, vp]; L.orc_cull.restype = i64
        L.orc_cull_ambiguity.argtypes = [P(_Params), i64, vp, vp, vp, d, d, vp]
        L.orc_cull_ambiguity.restype = i64
        L.orc_cull_ambiguity_tol.argtypes = [P(_Params), i64, vp, vp, vp, vp, vp, vp]
        L.orc_cull_ambiguity_tol.restype = i64
        L.orc_num_threads.restype = C.c_int
        L.orc_set_num_threads.argtypes = [C.c_int]
        L.orc_set_num_threads.restype = None
        L.orc_lattice_seeds.argtypes = [P(_Params), i64, i64, i64, d, vp, i64]
        L.orc_lattice_seeds.restype = i64
        L.orc_cull_pass.argtypes = [P(_Params), i64, vp, vp, vp, vp, vp, i32]
        L.orc_cull_pass.restype = i64
        L.orc_cull_pass_t.argtypes = [P(_Params), i64, vp, vp, vp, vp, vp, i32, C.c_double, i32]
        L.orc_cull_pass_t.restype = i64
        L.orc_evolve_repel.argtypes = [vp, i64, i64, i64, P(_Params), vp, i64, vp, vp, vp, vp, vp, vp, vp, i32, i32,
                                       C.c_double, vp, P(i64)]
        L.orc_evolve_repel.restype = i64
        L.orc_repel_energy.argtypes = [P(_Params), i64, vp, vp, vp, i64, vp, C.c_double, C.c_double]
        L.orc_repel_energy.restype = C.c_double
        L.orc_repel_grad.argtypes = [P(_Params), i64, vp, vp, vp, i64, vp, C.c_double, C.c_double, vp]
        L.orc_repel_grad.restype = None
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def params_struct(p, r_init: float | None = None) -> _Params:
    s = _Params()
    s.dim = int(p.dim)
    for i in range(3):
        s.spacing[i] = float(p.spacing[i])
    s.sigma_pre, s.i_offset, s.i_scale = float(p.sigma_pre), float(p.i_offset), float(p.i_scale)
    s.dR, s.eps0 = float(p.dR), float(p.eps0)
    s.r_min, s.r_max = float(p.r_min), float(p.r_max)
    s.r_init = float(r_init if r_init is not None else getattr(p, "r_init", 0.0))
    s.n_dirs, s.n_rays, s.n_radial = int(p.n_dirs), int(p.n_rays), int(p.n_radial)
    s.seed = int(p.seed) & 0xFFFFFFFFFFFFFFFF
    s.conv_tol, s.conv_window, s.e0, s.flags = float(p.conv_tol), int(p.conv_window), float(p.e0), int(p.flags)
    return s


_DT = {np.dtype(np.uint8): 0, np.dtype(np.uint16): 1, np.dtype(np.float32): 2}


# ---------------------------------------------------------------------------------------------
# elementary pieces
# ---------------------------------------------------------------------------------------------

def philox(ctr, key):
    c = (C.c_uint32 * 4)(*[int(v) & 0xFFFFFFFF for v in ctr])
    k = (C.c_uint32 * 2)(*[int(v) & 0xFFFFFFFF for v in key])
    o = (C.c_uint32 * 4)()
    lib().orc_philox4x32_10(c, k, o)
    return [int(v) for v in o]


def uniform(x: int) -> float:
    return lib().orc_uniform(int(x) & 0xFFFFFFFF)


def r_geom_min(dim: int, dR: float) -> float:
    return lib().orc_r_geom_min(int(dim), float(dR))


def weight(dim: int, r: float, R: float, dR: float):
    o = (C.c_double * 3)()
    lib().orc_weight(int(dim), float(r), float(R), float(dR), o)
    return o[0], o[1], o[2]


def weight_vec(dim: int, r, R: float, dR: float) -> np.ndarray:
    """S, dS/dr, dS/dR at every radius in r (array of shape r.shape + (3,))."""
    r = np.ascontiguousarray(r, dtype=np.float64)
    out = np.empty(r.shape + (3,))
    lib().orc_weight_many(int(dim), _ptr(r), r.size, float(R), float(dR), _ptr(out))
    return out


def rotation(p, n: int, cid: int) -> np.ndarray:
    q = (C.c_double * 9)()
    ps = params_struct(p)
    lib().orc_rotation(C.byref(ps), int(n), int(cid), q)
    return np.array(q[:]).reshape(3, 3)


def prepass(raw: np.ndarray, p) -> np.ndarray:
    raw = np.ascontiguousarray(raw)
    nz, ny, nx = raw.shape
    J = np.empty(raw.shape, dtype=np.float64)
    ps = params_struct(p)
    lib().orc_prepass(_ptr(raw), _DT[raw.dtype], nx, ny, nz, C.byref(ps), _ptr(J))
    return J


def interp(J: np.ndarray, dim: int, v) -> float:
    nz, ny, nx = J.shape
    return lib().orc_interp(_ptr(J), nx, ny, nz, int(dim), float(v[0]), float(v[1]),
                            float(v[2]) if len(v) > 2 else 0.0)


def interp_grad(J: np.ndarray, dim: int, v):
    """Trilinear (bilinear) value at voxel coordinates v and its gradient with respect to them
    (zero along axes outside [0, n - 1])."""
    nz, ny, nx = J.shape
    g = (C.c_double * 3)()
    val = lib().orc_interp_grad(_ptr(J), nx, ny, nz, int(dim), float(v[0]), float(v[1]),
                                float(v[2]) if len(v) > 2 else 0.0, g)
    return val, np.array(g[:dim])


def star_tables(dirs, dim: int):
    """Direction tables of the star contour: (anti, nb_off, nb_idx); raises if the table has no
    antipodes."""
    d = np.ascontiguousarray(dirs, dtype=np.float64)
    D = len(d)
    anti = np.zeros(D, np.int32)
    off = np.zeros(D + 1, np.int32)
    cap = 16 * D
    idx = np.zeros(cap, np.int32)
    r = lib().orc_star_tables(int(dim), _ptr(d), D, _ptr(anti), _ptr(off), _ptr(idx), cap)
    if r < 0:
        raise ValueError("direction table without antipodes" if r == -1 else "direction graph too large")
    return anti, off, idx[:r].copy()


def star_step_terms(J, p, dirs, tables, lam, c, Rk, n, cid, want_samples=False):
    """One star iteration's terms at (c, R_k) without updating: E, g_c, dc (+ magnitudes, slack)
    and the radius steps before clamping (+ magnitudes, slack)."""
    J = np.ascontiguousarray(J, dtype=np.float64)
    nz, ny, nx = J.shape
    d = np.ascontiguousarray(dirs, dtype=np.float64)
    anti, off, idx = tables
    ps = params_struct(p)
    D = p.n_dirs
    out = (C.c_double * 18)()
    cc = (C.c_double * 3)(*[float(v) for v in list(c) + [0.0] * (3 - len(c))])
    R = np.ascontiguousarray(Rk, dtype=np.float64)
    dR, dRa, dRs = np.zeros(D), np.zeros(D), np.zeros(D)
    N = p.n_rays * p.n_radial
    pts = np.zeros((N, 3)) if want_samples else None
    vals = np.zeros(N) if want_samples else None
    rdir = np.zeros(N, np.int32) if want_samples else None
    lib().orc_star_step_terms(_ptr(J), nx, ny, nz, C.byref(ps), _ptr(d), _ptr(anti), _ptr(off), _ptr(idx),
                              float(lam), cc, _ptr(R), int(n), int(cid), out, _ptr(dR), _ptr(dRa), _ptr(dRs),
                              _ptr(pts) if want_samples else None, _ptr(vals) if want_samples else None,
                              _ptr(rdir) if want_samples else None)
    o = np.array(out[:])
    res = {"E": o[0], "E_abs": o[1], "g_c": o[2:5], "g_c_abs": o[5:8], "dc": o[8:11], "dc_abs": o[11:14],
           "dc_slack": o[14:17], "n_kink": int(o[17]), "dR": dR, "dR_abs": dRa, "dR_slack": dRs}
    if want_samples:
        res["pts"], res["vals"], res["ray_dir"] = pts, vals, rdir
    return res


class StarState:
    """Star contours: centres (n x 3 physical), radii per direction (n x D), mean radii, counters."""

    def __init__(self, c, Rk, ids):
        n = len(c)
        self.c = np.ascontiguousarray(c, dtype=np.float64).copy()
        self.Rk = np.ascontiguousarray(Rk, dtype=np.float64).copy()
        self.R = self.Rk.mean(axis=1)
        self.ids = np.ascontiguousarray(ids, dtype=np.uint32)
        self.iters = np.zeros(n, np.int32)
        self.status = np.zeros(n, np.uint8)
        self.streak = np.zeros(n, np.uint8)
        self.e_mc = np.zeros(n)


def star_init(p, seeds, r0=None, ids=None, shape_zyx=None):
    """Initial star state: every direction's radius at the clamped R0 (as init_state), centres at
    the seeds (OUT when a seed lies outside the volume)."""
    st = init_state(p, seeds, r0=r0, ids=ids, shape_zyx=shape_zyx)
    s = StarState(st.c, np.repeat(st.R[:, None], p.n_dirs, axis=1), st.ids)
    s.status[:] = st.status
    return s


def star_evolve(J, p, dirs, tables, lam, st: StarState, n_iter: int) -> int:
    J = np.ascontiguousarray(J, dtype=np.float64)
    nz, ny, nx = J.shape
    d = np.ascontiguousarray(dirs, dtype=np.float64)
    anti, off, idx = tables
    ps = params_struct(p)
    n = len(st.c)
    return lib().orc_star_evolve(_ptr(J), nx, ny, nz, C.byref(ps), _ptr(d), _ptr(anti), _ptr(off), _ptr(idx),
                                 float(lam), n, _ptr(st.ids), _ptr(st.c), _ptr(st.Rk), _ptr(st.R),
                                 _ptr(st.iters), _ptr(st.status), _ptr(st.streak), _ptr(st.e_mc), int(n_iter))


def initial_radius(p, r0: float) -> float:
    ps = params_struct(p)
    return lib().orc_initial_radius(C.byref(ps), float(r0))


def mc_terms(J, p, dirs, c, R, n, cid, want_samples=False):
    """Monte-Carlo terms of one contour at state (c, R) and iteration n (no update)."""
    J = np.ascontiguousarray(J, dtype=np.float64)
    nz, ny, nx = J.shape
    d = np.ascontiguousarray(dirs, dtype=np.float64)
    ps = params_struct(p)
    out = (C.c_double * 17)()
    cc = (C.c_double * 3)(*[float(v) for v in list(c) + [0.0] * (3 - len(c))])
    N = p.n_rays * p.n_radial
    pts = np.zeros((N, 3)) if want_samples else None
    vals = np.zeros(N) if want_samples else None
    lib().orc_mc_terms(_ptr(J), nx, ny, nz, C.byref(ps), _ptr(d), cc, float(R), int(n), int(cid), out,
                       _ptr(pts) if want_samples else None, _ptr(vals) if want_samples else None)
    o = np.array(out[:])
    res = {"A": o[0], "B_R": o[1], "B_c": o[2:5], "scale": o[5], "dEdp": o[6:9], "dEdq": o[9:12],
           "E": o[12], "g_R": o[13], "g_c": o[14:17]}
    if want_samples:
        res["pts"], res["vals"] = pts, vals
    return res


def energy_fixed(dim, dR, pts, vals, scale, c, R) -> float:
    cc = (C.c_double * 3)(*[float(v) for v in list(c) + [0.0] * (3 - len(c))])
    return lib().orc_energy_fixed(int(dim), float(dR), _ptr(np.ascontiguousarray(pts)),
                                  _ptr(np.ascontiguousarray(vals)), len(vals), float(scale), cc, float(R))


# ---------------------------------------------------------------------------------------------
# whole-run driver
# ---------------------------------------------------------------------------------------------

@dataclass
class State:
    c: np.ndarray          # (n, 3) float64 physical
    R: np.ndarray          # (n,) float64
    iters: np.ndarray      # (n,) int32
    status: np.ndarray     # (n,) uint8
    streak: np.ndarray     # (n,) uint8
    e_mc: np.ndarray       # (n,) float64
    ids: np.ndarray        # (n,) uint32

    def copy(self) -> "State":
        return State(*(np.array(getattr(self, f)) for f in
                       ("c", "R", "iters", "status", "streak", "e_mc", "ids")))


def init_state(p, seeds, r0=None, ids=None, shape_zyx=None) -> State:
    """Contours at the seeds with R = clamp(R0); with the volume shape given, seeds outside the
    volume start OUT."""
    seeds = np.asarray(seeds, dtype=np.float64)
    n = len(seeds)
    c = np.zeros((n, 3))
    c[:, : seeds.shape[1]] = seeds
    if p.dim == 2:
        c[:, 2] = 0.0
    if r0 is None:
        r0 = np.full(n, float(p.r_init))
    R = np.array([initial_radius(p, float(v)) for v in np.broadcast_to(r0, (n,))])
    ids = np.arange(n, dtype=np.uint32) if ids is None else np.ascontiguousarray(ids, dtype=np.uint32)
    status = np.zeros(n, np.uint8)
    if shape_zyx is not None:
        nz, ny, nx = shape_zyx
        ext = (np.array([nx, ny, nz]) - 1) * np.asarray(p.spacing, dtype=np.float64)
        for a in range(p.dim):
            status[(c[:, a] < 0.0) | (c[:, a] > ext[a])] = OUT
    return State(c, R, np.zeros(n, np.int32), status, np.zeros(n, np.uint8), np.zeros(n), ids)


def evolve(J, p, dirs, st: State, n_iter: int, trace: bool = False, moves: np.ndarray | None = None):
    """Run up to n_iter further iterations on every ACTIVE contour (in place). Returns
    (trace array or None, number of contour-iterations run). With `moves` (an (n, n_iter) float64
    array, NaN-filled by the caller) each step's move max(|R change|, |c change|) is written at
    [contour, step of this call]. Raises if the p,q and c,R forms of the gradient ever disagree."""
    J = np.ascontiguousarray(J, dtype=np.float64)
    nz, ny, nx = J.shape
    d = np.ascontiguousarray(dirs, dtype=np.float64)
    ps = params_struct(p)
    n = len(st.R)
    tr = np.zeros((n, TRACE_W)) if trace else None
    if moves is not None:
        assert moves.shape == (n, n_iter) and moves.dtype == np.float64 and moves.flags.c_contiguous
    done = C.c_int64(0)
    mism = lib().orc_evolve_log(_ptr(J), nx, ny, nz, C.byref(ps), _ptr(d), n, _ptr(st.ids), _ptr(st.c),
                                _ptr(st.R), _ptr(st.iters), _ptr(st.status), _ptr(st.streak), _ptr(st.e_mc),
                                int(n_iter), _ptr(tr) if trace else None,
                                _ptr(moves) if moves is not None else None, C.byref(done))
    if mism:
        raise AssertionError(f"p,q and c,R gradient forms disagree on {mism} contour-iterations")
    return tr, int(done.value)


def evolve_repel(J, p, dirs, st: State, n_iter: int, every: int, kappa: float, trace: bool = False):
    """evolve() with soft repulsion of strength kappa between neighbouring contours, the neighbours
    held at a snapshot taken every `every` iterations (not in the paper). Returns (trace or None,
    contour-iterations run)."""
    J = np.ascontiguousarray(J, dtype=np.float64)
    nz, ny, nx = J.shape
    d = np.ascontiguousarray(dirs, dtype=np.float64)
    ps = params_struct(p)
    n = len(st.R)
    tr = np.zeros((n, TRACE_W)) if trace else None
    done = C.c_int64(0)
    mism = lib().orc_evolve_repel(_ptr(J), nx, ny, nz, C.byref(ps), _ptr(d), n, _ptr(st.ids), _ptr(st.c),
                                  _ptr(st.R), _ptr(st.iters), _ptr(st.status), _ptr(st.streak), _ptr(st.e_mc),
                                  int(n_iter), int(every), float(kappa), _ptr(tr) if trace else None,
                                  C.byref(done))
    if mism:
        raise AssertionError(f"p,q and c,R gradient forms disagree on {mism} contour-iterations")
    return tr, int(done.value)


def repel_energy(p, c_s, R_s, live_s, self: int, c, R: float, kappa: float) -> float:
    """The repulsion penalty of contour `self` at (c, R) against snapshot contours (c_s, R_s, live_s)."""
    ps = params_struct(p)
    cs = np.ascontiguousarray(c_s, np.float64)
    rs = np.ascontiguousarray(R_s, np.float64)
    ls = np.ascontiguousarray(live_s, np.uint8)
    cc = np.zeros(3)
    cc[: len(c)] = c
    return float(lib().orc_repel_energy(C.byref(ps), len(rs), _ptr(cs), _ptr(rs), _ptr(ls), int(self), _ptr(cc),
                                        float(R), float(kappa)))


def repel_grad(p, c_s, R_s, live_s, self: int, c, R: float, kappa: float):
    """(dP/dc (3), dP/dR) of that penalty, as the evolution forms it."""
    ps = params_struct(p)
    cs = np.ascontiguousarray(c_s, np.float64)
    rs = np.ascontiguousarray(R_s, np.float64)
    ls = np.ascontiguousarray(live_s, np.uint8)
    cc = np.zeros(3)
    cc[: len(c)] = c
    out = np.zeros(4)
    lib().orc_repel_grad(C.byref(ps), len(rs), _ptr(cs), _ptr(rs), _ptr(ls), int(self), _ptr(cc), float(R),
                         float(kappa), _ptr(out))
    return out[:3], float(out[3])


def stop_ranges(moves: np.ndarray, p, delta: float):
    """Where the stop rule (freeze after conv_window consecutive moves below conv_tol) ends a run
    whose every step's move is known, and how far that end can move when each decision whose move
    lies within delta * conv_tol of conv_tol may go either way.

    moves: (n, n_iter) moves of runs from the seeds (streak 0) with the freeze switched off
    (conv_window = 0), NaN after a run stopped for another reason (OUT, NONFINITE). Returns
    (n_stop, n_lo, n_hi, converged): the iteration count at which the rule stops each contour (the
    run's own end when it never converges), the earliest end when every near decision counts as
    small and the latest when none does (the rule is monotone in its decisions), and whether the
    exact decisions converge."""
    n, N = moves.shape
    W, tau = int(p.conv_window), float(p.conv_tol)
    ran = np.sum(~np.isnan(moves), axis=1)          # steps each unfrozen run made
    m = np.where(np.isnan(moves), np.inf, moves)
    near = np.abs(m - tau) <= delta * tau

    def first_stop(small):
        # first step index (1-based) ending W consecutive small moves; 0 if none
        out = np.zeros(n, np.int64)
        if W <= 0:
            return out
        run = np.zeros(n, np.int64)
        for k in range(N):
            run = np.where(small[:, k], run + 1, 0)
            hit = (run >= W) & (out == 0)
            out[hit] = k + 1
        return out

    def end(conv):
        return np.where((conv > 0) & (conv <= ran), conv, ran)

    exact = first_stop(m < tau)
    early = first_stop((m < tau) | near)
    late = first_stop((m < tau) & ~near)
    return end(exact), end(early), np.where(late > 0, end(late), ran), (exact > 0) & (exact <= ran)


def finalize_status(st: State) -> None:
    """Contours still ACTIVE when evolution ends stopped on the iteration limit."""
    base = st.status & 0x0F
    st.status[base == ACTIVE] = (st.status[base == ACTIVE] & CLAMPED) | MAXITER


def energy_vox(J, p, c, R):
    J = np.ascontiguousarray(J, dtype=np.float64)
    nz, ny, nx = J.shape
    c = np.ascontiguousarray(c, dtype=np.float64)
    R = np.ascontiguousarray(R, dtype=np.float64)
    n = len(R)
    e = np.zeros(n)
    ea = np.zeros(n)
    ps = params_struct(p)
    lib().orc_energy_vox(_ptr(J), nx, ny, nz, C.byref(ps), n, _ptr(c), _ptr(R), _ptr(e), _ptr(ea))
    return e, ea


def cull(p, c, R, e_vox, status, ids):
    c = np.ascontiguousarray(c, dtype=np.float64)
    R = np.ascontiguousarray(R, dtype=np.float64)
    e_vox = np.ascontiguousarray(e_vox, dtype=np.float64)
    status = np.ascontiguousarray(status, dtype=np.uint8)
    ids = np.ascontiguousarray(ids, dtype=np.uint32)
    keep = np.zeros(len(R), np.uint8)
    ps = params_struct(p)
    lib().orc_cull(C.byref(ps), len(R), _ptr(c), _ptr(R), _ptr(e_vox), _ptr(status), _ptr(ids), _ptr(keep))
    return keep


def cull_ambiguity(p, c, R, e_vox, rel_e=1e-4, tol_d=1e-3):
    amb = np.zeros(len(R), np.uint8)
    ps = params_struct(p)
    lib().orc_cull_ambiguity(C.byref(ps), len(R), _ptr(np.ascontiguousarray(c, dtype=np.float64)),
                             _ptr(np.ascontiguousarray(R, dtype=np.float64)),
                             _ptr(np.ascontiguousarray(e_vox, dtype=np.float64)), float(rel_e), float(tol_d),
                             _ptr(amb))
    return amb


def cull_ambiguity_tol(p, c, R, e_vox, tol_e, tol_d):
    """Selection decisions within per-contour tolerances of a threshold (energy vs E0 or vs an
    overlapping rival's energy; pair distance vs the overlap radius); see orc_cull_ambiguity_tol."""
    n = len(R)
    amb = np.zeros(n, np.uint8)
    ps = params_struct(p)
    f = lambda a: np.ascontiguousarray(np.broadcast_to(np.asarray(a, np.float64), (n,) + np.shape(a)[1:]))
    cc = np.ascontiguousarray(c, dtype=np.float64)
    lib().orc_cull_ambiguity_tol(C.byref(ps), n, _ptr(cc), _ptr(f(R)), _ptr(f(e_vox)), _ptr(f(tol_e)),
                                 _ptr(f(tol_d)), _ptr(amb))
    return amb


def lattice_seeds(p, shape_zyx, pitch=None):
    """Centres (n x 3, physical) of the initial lattice: pitch sqrt(1.5) * r_init unless given."""
    nz, ny, nx = shape_zyx
    pitch = float(np.sqrt(1.5) * p.r_init if pitch is None else pitch)
    ps = params_struct(p)
    n = lib().orc_lattice_seeds(C.byref(ps), nx, ny, nz, pitch, None, 0)
    out = np.zeros((n, 3))
    lib().orc_lattice_seeds(C.byref(ps), nx, ny, nz, pitch, _ptr(out), n)
    return out


def cull_pass(p, st: State, young: bool, e_cull=None, compete: bool = True) -> int:
    """One culling pass at the current state (in place, ranking by E_mc); young: the run is still in
    its grace period, so every live contour with a finite energy is a candidate, otherwise those with
    E_mc <= e_cull (default E0); compete: overlapping candidates compete. Returns the number
    retired."""
    ps = params_struct(p)
    thr = float(p.e0 if e_cull is None else e_cull)
    return int(lib().orc_cull_pass_t(C.byref(ps), len(st.R), _ptr(st.c), _ptr(st.R), _ptr(st.e_mc),
                                     _ptr(st.status), _ptr(st.ids), int(bool(young)), thr, int(bool(compete))))


def evolve_cull(J, p, dirs, st: State, n_iter: int, every: int, grace: int, e_cull=None, compete: bool = True):
    """Evolution in chunks of `every` iterations with a culling pass after each chunk (the pass after
    `done` iterations of the run is young while done < grace); returns the number of
    contour-iterations run."""
    done, total = 0, 0
    while True:
        k = min(every, n_iter - done)
        if k > 0:
            _, ran = evolve(J, p, dirs, st, k)
            total += ran
            done += k
        cull_pass(p, st, done < grace, e_cull, compete)
        if done >= n_iter:
            return total


def run(raw, p, dirs, seeds, n_iter, r0=None, ids=None):
    """Whole path: pre-pass, init, evolve n_iter, stop status, exact energy, selection."""
    J = prepass(raw, p)
    st = init_state(p, seeds, r0, ids, shape_zyx=raw.shape)
    _, done = evolve(J, p, dirs, st, n_iter)
    finalize_status(st)
    e_vox, e_abs = energy_vox(J, p, st.c, st.R)
    keep = cull(p, st.c, st.R, e_vox, st.status, st.ids)
    return {"J": J, "state": st, "e_vox": e_vox, "e_abs": e_abs, "keep": keep, "evolved": done}


def num_threads() -> int:
    return int(lib().orc_num_threads())


def set_num_threads(n: int) -> None:
    """Threads of the oracle's loops over contours (timing only)."""
    lib().orc_set_num_threads(int(n))
