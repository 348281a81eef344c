"""Python binding of libsnk.so (the C ABI in include/snk.h): argument marshalling only.

Every function here has the name of the C entry point it calls and does no computation of its
own: all work runs in the HIP kernels of the library. If the library has not been built, loading
it raises immediately -- there is no fallback path.

Device buffers may be passed as torch tensors (their ``data_ptr()`` is borrowed) and a HIP stream
as ``torch.cuda.Stream`` / raw handle; torch is used only for device memory and streams.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsnk.so")

SNK_OK, SNK_EINVAL, SNK_ENOMEM, SNK_EDEVICE, SNK_ESTATE, SNK_EBUSY, SNK_ERANGE = 0, -1, -2, -3, -4, -5, -6
SNK_U8, SNK_U16, SNK_F32 = 0, 1, 2
ACTIVE, CONVERGED, MAXITER, OUT, NONFINITE, CULLED, CLAMPED = 0, 1, 2, 3, 4, 5, 0x10
TRACE_W = 16

EXPORTS = [
    "snk_create", "snk_destroy", "snk_set_params", "snk_set_launch", "snk_set_tile", "snk_set_star",
    "snk_get_star_radii", "snk_set_star_radii", "snk_set_directions",
    "snk_load_volume", "snk_prepass", "snk_load_seeds", "snk_evolve", "snk_finalize", "snk_finalize_noalloc",
    "snk_read",
    "snk_get_state", "snk_set_state", "snk_trace_step", "snk_read_volume", "snk_get_timing",
    "snk_sync", "snk_last_error", "snk_version", "snk_seed_lattice", "snk_evolve_cull", "snk_set_cull", "snk_set_repulsion",
    "snk_engine_create", "snk_engine_destroy", "snk_engine_last_error", "snk_engine_set_launch", "snk_engine_set_tile",
    "snk_engine_submit", "snk_engine_run", "snk_engine_step", "snk_engine_poll", "snk_engine_read",
    "snk_engine_job_times", "snk_engine_release", "snk_engine_get_stats", "snk_engine_tuned_shapes",
]


class SnkError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"snk error {code}: {msg}")
        self.code = code


class snk_params(C.Structure):
    _fields_ = [("dim", C.c_int32), ("spacing", C.c_double * 3), ("sigma_pre", C.c_double),
                ("i_offset", C.c_double), ("i_scale", C.c_double), ("dR", C.c_double),
                ("eps0", C.c_double), ("r_min", C.c_double), ("r_max", C.c_double), ("r_init", C.c_double),
                ("n_dirs", C.c_int32), ("n_rays", C.c_int32), ("n_radial", C.c_int32),
                ("seed", C.c_uint64), ("conv_tol", C.c_double), ("conv_window", C.c_int32),
                ("e0", C.c_double), ("flags", C.c_int32)]


class snk_timing(C.Structure):
    _fields_ = [("prepass_ms", C.c_double), ("evolve_ms", C.c_double), ("finalize_ms", C.c_double),
                ("evolved", C.c_int64), ("evolve_launches", C.c_int64), ("lanes_per_contour", C.c_int32),
                ("pairs_in_flight", C.c_int32), ("layout", C.c_int32), ("tile_voxels", C.c_int32)]


class snk_engine_stats(C.Structure):
    _fields_ = [("submitted", C.c_int64), ("admitted", C.c_int64), ("completed", C.c_int64),
                ("pending", C.c_int64), ("running", C.c_int64), ("bytes_in_use", C.c_uint64),
                ("budget", C.c_uint64), ("last_ms", C.c_double), ("last_evolve_ms", C.c_double),
                ("last_evolved", C.c_int64), ("lanes_per_contour", C.c_int32), ("pairs_in_flight", C.c_int32),
                ("persistent", C.c_int32), ("layout", C.c_int32), ("graph_replays", C.c_int32)]


_lib = None


def load(path: str = LIB_PATH):
    """Load libsnk.so (raises if it is missing: build it with __graft_entry__.build())."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"HIP library not built: {path} is missing (run __graft_entry__.build())")
    L = C.CDLL(path)
    vp, i32, i64, u8p = C.c_void_p, C.c_int32, C.c_int64, C.c_void_p
    sig = {
        "snk_create": [C.POINTER(C.c_void_p), C.c_int, vp],
        "snk_destroy": [vp],
        "snk_set_params": [vp, C.POINTER(snk_params)],
        "snk_set_launch": [vp, i32, i32, i32],
        "snk_set_tile": [vp, i32],
        "snk_set_star": [vp, C.c_double],
        "snk_get_star_radii": [vp, vp, C.c_int64, C.POINTER(C.c_int64)],
        "snk_set_star_radii": [vp, vp, C.c_int64],
        "snk_set_directions": [vp, vp, i32],
        "snk_load_volume": [vp, vp, C.c_int, i64, i64, i64, C.c_int],
        "snk_prepass": [vp],
        "snk_load_seeds": [vp, vp, vp, vp, i64],
        "snk_evolve": [vp, i32],
        "snk_seed_lattice": [vp, C.c_double, C.POINTER(i64)],
        "snk_evolve_cull": [vp, i32, i32, i32],
        "snk_set_cull": [vp, C.c_double, i32],
        "snk_set_repulsion": [vp, C.c_double, i32],
        "snk_finalize": [vp],
        "snk_finalize_noalloc": [vp],
        "snk_read": [vp, vp, vp, vp, vp, vp, vp, vp, i64, C.POINTER(i64)],
        "snk_get_state": [vp, vp, vp, vp, vp, vp, i64, C.POINTER(i64)],
        "snk_set_state": [vp, vp, vp, vp, vp, vp, i64],
        "snk_trace_step": [vp, vp],
        "snk_read_volume": [vp, vp, C.c_int],
        "snk_get_timing": [vp, C.POINTER(snk_timing)],
        "snk_sync": [vp],
        "snk_last_error": [vp],
        "snk_version": [],
        "snk_engine_create": [C.POINTER(C.c_void_p), C.c_int, vp, C.c_uint64],
        "snk_engine_destroy": [vp],
        "snk_engine_last_error": [vp],
        "snk_engine_set_launch": [vp, i32, i32, i32, i32],
        "snk_engine_submit": [vp, C.POINTER(snk_params), vp, i32, vp, C.c_int, i64, i64, i64, C.c_int, vp, vp, vp,
                              i64, i32, C.POINTER(C.c_uint64)],
        "snk_engine_run": [vp],
        "snk_engine_step": [vp, i32, C.POINTER(i32)],
        "snk_engine_poll": [vp, vp, i64, C.POINTER(i64)],
        "snk_engine_read": [vp, C.c_uint64, vp, vp, vp, vp, vp, vp, vp, i64, C.POINTER(i64)],
        "snk_engine_job_times": [vp, C.c_uint64, C.POINTER(C.c_double), C.POINTER(C.c_double)],
        "snk_engine_release": [vp, C.c_uint64],
        "snk_engine_get_stats": [vp, C.POINTER(snk_engine_stats)],
        "snk_engine_set_tile": [vp, i32, i32],
        "snk_engine_tuned_shapes": [vp, vp, i64, C.POINTER(i64)],
    }
    for name, args in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = C.c_char_p if name in ("snk_last_error", "snk_version", "snk_engine_last_error") else C.c_int32
    _lib = L
    return L


def _ptr(a):
    if a is None:
        return None
    if hasattr(a, "data_ptr"):
        return C.c_void_p(int(a.data_ptr()))
    return a.ctypes.data_as(C.c_void_p)


def _stream_handle(stream):
    if stream is None:
        return None
    if hasattr(stream, "cuda_stream"):
        return C.c_void_p(int(stream.cuda_stream))
    return C.c_void_p(int(stream))


def _check(h, code):
    if code != SNK_OK:
        raise SnkError(code, load().snk_last_error(h).decode())


def to_params(p) -> snk_params:
    """Marshal any object with the snk_params field names into the C struct."""
    s = snk_params()
    s.dim = int(p.dim)
    for i in range(3):
        s.spacing[i] = float(p.spacing[i])
    for f in ("sigma_pre", "i_offset", "i_scale", "dR", "eps0", "r_min", "r_max", "r_init", "conv_tol", "e0"):
        setattr(s, f, float(getattr(p, f)))
    for f in ("n_dirs", "n_rays", "n_radial", "conv_window", "flags"):
        setattr(s, f, int(getattr(p, f)))
    s.seed = int(p.seed) & 0xFFFFFFFFFFFFFFFF
    return s


# ------------------------------------------------------------------------------------------------
# entry points (same names as the C ABI)
# ------------------------------------------------------------------------------------------------

def snk_version() -> str:
    return load().snk_version().decode()


def snk_create(device: int = 0, stream=None):
    h = C.c_void_p()
    code = load().snk_create(C.byref(h), int(device), _stream_handle(stream))
    if code != SNK_OK:
        raise SnkError(code, load().snk_last_error(None).decode())
    return h


def snk_destroy(h) -> None:
    _check(h, load().snk_destroy(h))


def snk_set_params(h, params) -> None:
    s = params if isinstance(params, snk_params) else to_params(params)
    _check(h, load().snk_set_params(h, C.byref(s)))


def snk_set_launch(h, lanes_per_contour: int = 0, pairs_in_flight: int = 0, layout: int = 0) -> None:
    _check(h, load().snk_set_launch(h, int(lanes_per_contour), int(pairs_in_flight), int(layout)))


def snk_set_tile(h, tile_voxels: int = -1) -> None:
    _check(h, load().snk_set_tile(h, int(tile_voxels)))


def snk_set_star(h, smooth: float = -1.0) -> None:
    _check(h, load().snk_set_star(h, float(smooth)))


def snk_get_star_radii(h) -> np.ndarray:
    n = _count(h)
    got = C.c_int64(0)
    probe = np.zeros(1, np.float32)
    load().snk_get_star_radii(h, _ptr(probe), 0, C.byref(got))
    out = np.zeros(max(int(got.value), 1), np.float32)
    _check(h, load().snk_get_star_radii(h, _ptr(out), len(out), C.byref(got)))
    return out[: int(got.value)].reshape(n, -1) if n else out[:0].reshape(0, 0)


def snk_set_star_radii(h, radii) -> None:
    r = np.ascontiguousarray(radii, dtype=np.float32)
    _check(h, load().snk_set_star_radii(h, _ptr(r), r.shape[0]))


def snk_set_directions(h, dirs) -> None:
    d = np.ascontiguousarray(dirs, dtype=np.float32)
    _check(h, load().snk_set_directions(h, _ptr(d), int(d.shape[0])))


_DT = {np.dtype(np.uint8): SNK_U8, np.dtype(np.uint16): SNK_U16, np.dtype(np.float32): SNK_F32}


def _dtype_code(a) -> int:
    if hasattr(a, "data_ptr"):
        import torch
        return {torch.uint8: SNK_U8, torch.uint16: SNK_U16, torch.float32: SNK_F32}[a.dtype]
    return _DT[np.dtype(a.dtype)]


def snk_load_volume(h, data, on_device: bool | None = None) -> None:
    """data: numpy array [z][y][x] (copied) or a contiguous device tensor (borrowed)."""
    if on_device is None:
        on_device = hasattr(data, "data_ptr") and getattr(data, "is_cuda", False)
    if not hasattr(data, "data_ptr"):
        data = np.ascontiguousarray(data)
    nz, ny, nx = data.shape
    _check(h, load().snk_load_volume(h, _ptr(data), _dtype_code(data), nx, ny, nz, int(bool(on_device))))


def snk_prepass(h) -> None:
    _check(h, load().snk_prepass(h))


def snk_load_seeds(h, centers, r0=None, ids=None) -> None:
    c = np.zeros((len(centers), 3), dtype=np.float64)
    cc = np.asarray(centers, dtype=np.float64)
    c[:, : cc.shape[1]] = cc
    r = None if r0 is None else np.ascontiguousarray(r0, dtype=np.float32)
    i = None if ids is None else np.ascontiguousarray(ids, dtype=np.uint32)
    _check(h, load().snk_load_seeds(h, _ptr(c), _ptr(r), _ptr(i), len(c)))


def snk_evolve(h, n_iter: int) -> None:
    _check(h, load().snk_evolve(h, int(n_iter)))


def snk_seed_lattice(h, pitch: float = 0.0) -> int:
    """Seeds on the initial lattice (pitch <= 0: sqrt(1.5) * r_init); returns the contour count."""
    n = C.c_int64(0)
    _check(h, load().snk_seed_lattice(h, float(pitch), C.byref(n)))
    return int(n.value)


def snk_evolve_cull(h, n_iter: int, cull_every: int, grace_iters: int) -> None:
    _check(h, load().snk_evolve_cull(h, int(n_iter), int(cull_every), int(grace_iters)))


def snk_set_cull(h, e_cull=None, compete: bool = True) -> None:
    """Culling passes' threshold (None: params.e0) and competition."""
    _check(h, load().snk_set_cull(h, float("nan") if e_cull is None else float(e_cull), int(bool(compete))))


def snk_set_repulsion(h, kappa: float = 0.0, every: int = 1) -> None:
    """Soft repulsion between neighbouring contours (0: off), neighbours refreshed every `every` iterations."""
    _check(h, load().snk_set_repulsion(h, float(kappa), int(every)))


def snk_finalize(h) -> None:
    _check(h, load().snk_finalize(h))


def snk_finalize_noalloc(h) -> None:
    _check(h, load().snk_finalize_noalloc(h))


def _count(h) -> int:
    n = C.c_int64(0)
    load().snk_get_state(h, None, None, None, None, None, 0, C.byref(n))
    return int(n.value)


def snk_read(h) -> dict:
    n = _count(h)
    out = {"radii": np.zeros(n, np.float32), "centers": np.zeros((n, 3), np.float64),
           "e_mc": np.zeros(n, np.float32), "e_vox": np.zeros(n, np.float32),
           "iters": np.zeros(n, np.int32), "status": np.zeros(n, np.uint8), "keep": np.zeros(n, np.uint8)}
    got = C.c_int64(0)
    _check(h, load().snk_read(h, _ptr(out["radii"]), _ptr(out["centers"]), _ptr(out["e_mc"]), _ptr(out["e_vox"]),
                              _ptr(out["iters"]), _ptr(out["status"]), _ptr(out["keep"]), n, C.byref(got)))
    return out


def snk_get_state(h) -> dict:
    n = _count(h)
    out = {"centers": np.zeros((n, 3), np.float64), "radii": np.zeros(n, np.float32),
           "iters": np.zeros(n, np.int32), "status": np.zeros(n, np.uint8), "streak": np.zeros(n, np.uint8)}
    got = C.c_int64(0)
    _check(h, load().snk_get_state(h, _ptr(out["centers"]), _ptr(out["radii"]), _ptr(out["iters"]),
                                   _ptr(out["status"]), _ptr(out["streak"]), n, C.byref(got)))
    return out


def snk_set_state(h, centers, radii, iters, status, streak=None) -> None:
    c = np.zeros((len(radii), 3), dtype=np.float64)
    cc = np.asarray(centers, dtype=np.float64)
    c[:, : cc.shape[1]] = cc
    r = np.ascontiguousarray(radii, dtype=np.float32)
    it = np.ascontiguousarray(iters, dtype=np.int32)
    st = np.ascontiguousarray(status, dtype=np.uint8)
    sk = None if streak is None else np.ascontiguousarray(streak, dtype=np.uint8)
    _check(h, load().snk_set_state(h, _ptr(c), _ptr(r), _ptr(it), _ptr(st), _ptr(sk), len(r)))


def snk_trace_step(h) -> np.ndarray:
    n = _count(h)
    terms = np.zeros((n, TRACE_W), np.float32)
    _check(h, load().snk_trace_step(h, _ptr(terms)))
    return terms


def snk_read_volume(h, shape_zyx) -> np.ndarray:
    out = np.zeros(shape_zyx, np.float32)
    _check(h, load().snk_read_volume(h, _ptr(out), 0))
    return out


def snk_get_timing(h) -> dict:
    t = snk_timing()
    _check(h, load().snk_get_timing(h, C.byref(t)))
    return {"prepass_ms": t.prepass_ms, "evolve_ms": t.evolve_ms, "finalize_ms": t.finalize_ms,
            "evolved": int(t.evolved), "evolve_launches": int(t.evolve_launches),
            "lanes_per_contour": int(t.lanes_per_contour), "pairs_in_flight": int(t.pairs_in_flight),
            "layout": int(t.layout), "tile_voxels": int(t.tile_voxels)}


def snk_sync(h) -> None:
    _check(h, load().snk_sync(h))


def snk_last_error(h) -> str:
    return load().snk_last_error(h).decode()


# ------------------------------------------------------------------------------------------------
# engine (batched + served)
# ------------------------------------------------------------------------------------------------

def _echeck(e, code):
    if code != SNK_OK:
        raise SnkError(code, load().snk_engine_last_error(e).decode())


def snk_engine_create(device: int = 0, stream=None, hbm_budget_bytes: int = 64 << 30):
    e = C.c_void_p()
    code = load().snk_engine_create(C.byref(e), int(device), _stream_handle(stream), int(hbm_budget_bytes))
    if code != SNK_OK:
        raise SnkError(code, "snk_engine_create failed")
    return e


def snk_engine_destroy(e) -> None:
    _echeck(e, load().snk_engine_destroy(e))


def snk_engine_last_error(e) -> str:
    return load().snk_engine_last_error(e).decode()


def snk_engine_set_launch(e, lanes_per_contour: int = 0, pairs_in_flight: int = 1, persistent: int = 1,
                          layout: int = 0) -> None:
    _echeck(e, load().snk_engine_set_launch(e, int(lanes_per_contour), int(pairs_in_flight), int(persistent),
                                            int(layout)))


def snk_engine_set_tile(e, tile_voxels: int = 0, workgroups_per_cu: int = 0) -> None:
    _echeck(e, load().snk_engine_set_tile(e, int(tile_voxels), int(workgroups_per_cu)))


def snk_engine_submit(e, params, dirs, vol, centers, r0=None, ids=None, n_iter: int = 100,
                      on_device: bool | None = None) -> int:
    s = params if isinstance(params, snk_params) else to_params(params)
    d = np.ascontiguousarray(dirs, dtype=np.float32)
    if on_device is None:
        on_device = hasattr(vol, "data_ptr") and getattr(vol, "is_cuda", False)
    if not hasattr(vol, "data_ptr"):
        vol = np.ascontiguousarray(vol)
    nz, ny, nx = vol.shape
    c = np.zeros((len(centers), 3), dtype=np.float64)
    cc = np.asarray(centers, dtype=np.float64)
    if len(cc):
        c[:, : cc.shape[1]] = cc
    r = None if r0 is None else np.ascontiguousarray(r0, dtype=np.float32)
    i = None if ids is None else np.ascontiguousarray(ids, dtype=np.uint32)
    job = C.c_uint64(0)
    _echeck(e, load().snk_engine_submit(e, C.byref(s), _ptr(d), int(d.shape[0]), _ptr(vol), _dtype_code(vol), nx, ny,
                                        nz, int(bool(on_device)), _ptr(c), _ptr(r), _ptr(i), len(c), int(n_iter),
                                        C.byref(job)))
    return int(job.value)


def snk_engine_run(e) -> None:
    _echeck(e, load().snk_engine_run(e))


def snk_engine_step(e, chunk: int) -> int:
    k = C.c_int32(0)
    _echeck(e, load().snk_engine_step(e, int(chunk), C.byref(k)))
    return int(k.value)


def snk_engine_poll(e, cap: int = 1 << 16) -> list:
    buf = np.zeros(cap, np.uint64)
    n = C.c_int64(0)
    _echeck(e, load().snk_engine_poll(e, _ptr(buf), cap, C.byref(n)))
    return [int(v) for v in buf[: n.value]]


def snk_engine_read(e, job: int) -> dict:
    n = C.c_int64(0)
    load().snk_engine_read(e, int(job), None, None, None, None, None, None, None, 0, C.byref(n))
    n = int(n.value)
    out = {"radii": np.zeros(n, np.float32), "centers": np.zeros((n, 3), np.float64),
           "e_mc": np.zeros(n, np.float32), "e_vox": np.zeros(n, np.float32),
           "iters": np.zeros(n, np.int32), "status": np.zeros(n, np.uint8), "keep": np.zeros(n, np.uint8)}
    got = C.c_int64(0)
    _echeck(e, load().snk_engine_read(e, int(job), _ptr(out["radii"]), _ptr(out["centers"]), _ptr(out["e_mc"]),
                                      _ptr(out["e_vox"]), _ptr(out["iters"]), _ptr(out["status"]),
                                      _ptr(out["keep"]), n, C.byref(got)))
    return out


def snk_engine_job_times(e, job: int):
    a, b = C.c_double(0), C.c_double(0)
    _echeck(e, load().snk_engine_job_times(e, int(job), C.byref(a), C.byref(b)))
    return a.value, b.value


def snk_engine_release(e, job: int) -> None:
    _echeck(e, load().snk_engine_release(e, int(job)))


TUNED_W = 11
TUNED_FIELDS = ("dim", "n_dirs", "n_rays", "n_radial", "lanes_per_contour", "pairs_in_flight", "persistent",
                "workgroups_per_cu", "tile_voxels", "trial_us", "trials")


def snk_engine_tuned_shapes(e) -> list:
    """The autotuned launch shape of every class so far, one dict per class."""
    n = C.c_int64(0)
    _echeck(e, load().snk_engine_tuned_shapes(e, None, 0, C.byref(n)))
    rows = np.zeros((max(n.value, 1), TUNED_W), np.int32)
    _echeck(e, load().snk_engine_tuned_shapes(e, _ptr(rows), n.value, C.byref(n)))
    return [dict(zip(TUNED_FIELDS, (int(v) for v in r))) for r in rows[: n.value]]


def snk_engine_get_stats(e) -> dict:
    s = snk_engine_stats()
    _echeck(e, load().snk_engine_get_stats(e, C.byref(s)))
    return {f: getattr(s, f) for f, _ in snk_engine_stats._fields_}


class Engine:
    """Owns one snk_engine handle; methods forward to the snk_engine_* entry points."""

    def __init__(self, device: int = 0, stream=None, hbm_budget_bytes: int = 64 << 30):
        self.e = snk_engine_create(device, stream, hbm_budget_bytes)

    def close(self):
        if self.e is not None:
            snk_engine_destroy(self.e)
            self.e = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __getattr__(self, name):
        f = globals().get("snk_engine_" + name)
        if f is None:
            raise AttributeError(name)
        return lambda *a, **k: f(self.e, *a, **k)


class Context:
    """Owns one snk_ctx handle; methods forward to the entry points above."""

    def __init__(self, device: int = 0, stream=None):
        self.h = snk_create(device, stream)

    def close(self):
        if self.h is not None:
            snk_destroy(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __getattr__(self, name):
        f = globals().get("snk_" + name)
        if f is None:
            raise AttributeError(name)
        return lambda *a, **k: f(self.h, *a, **k)
