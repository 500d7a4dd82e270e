"""Thin Python binding of the C ABI in ``include/rt3d.h`` (librt3d.so, HIP kernels for gfx950).

Argument marshalling only: every step of the hot path runs in the library's kernels.  Host arrays
are numpy float64; device arrays are torch float64 CUDA tensors (passed by ``data_ptr()``, with
``torch.cuda.current_stream()`` as the context stream).  Every non-zero status raises
:class:`Rt3dError` carrying the status and the library's message.

The library must have been built (``python -m paper_1107_5719_amd.build``); importing this module
raises if ``librt3d.so`` is missing.  There is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import json
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librt3d.so")

RT3D_OK = 0
RT3D_ERR_ARG = -1
RT3D_ERR_OOM = -2
RT3D_ERR_HIP = -3
RT3D_ERR_NOT_CONVERGED = -4
RT3D_ERR_NONFINITE = -5
RT3D_ERR_STATE = -6
RT3D_HOST = 0
RT3D_DEVICE = 1
RT3D_FP64 = 0
RT3D_FP32_SWEEP = 1
RT3D_MEMBER_RUNNING = 0
RT3D_MEMBER_CONVERGED = 1
RT3D_MEMBER_MAX_ITER = 2
RT3D_MEMBER_NONFINITE = 3
RT3D_OS_JACOBI = 0
RT3D_OS_GAUSS_SEIDEL = 1
RT3D_COEF_FP64 = 0
RT3D_COEF_FP32 = 1

EXPORTED = [
    "rt3d_create", "rt3d_destroy", "rt3d_set_medium", "rt3d_set_J", "rt3d_get_J",
    "rt3d_formal_solution", "rt3d_build_lstar", "rt3d_get_lstar", "rt3d_os_step",
    "rt3d_solve_to_convergence", "rt3d_set_acceleration", "rt3d_set_anderson", "rt3d_set_os_method", "rt3d_set_coef_storage", "rt3d_get_emergent_top", "rt3d_set_timing", "rt3d_get_stats",
    "rt3d_status_str", "rt3d_last_error", "rt3d_quadrature", "rt3d_segment_table", "rt3d_validate",
    "rt3d_adjoint_emergent", "rt3d_get_history", "rt3d_sweep_shapes", "rt3d_set_sweep_shape", "rt3d_autotune",
    "rt3d_batch_create", "rt3d_batch_destroy", "rt3d_batch_size", "rt3d_batch_last_error",
    "rt3d_batch_set_medium", "rt3d_batch_set_J", "rt3d_batch_get_J", "rt3d_batch_get_Jfs",
    "rt3d_batch_set_acceleration", "rt3d_batch_set_anderson", "rt3d_batch_set_sweep_shape",
    "rt3d_batch_formal_solution",
    "rt3d_batch_solve", "rt3d_batch_autotune", "rt3d_batch_get_stats", "rt3d_formal_solution_noalloc",
]


class Rt3dError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"rt3d status {status}: {message}")
        self.status = status


class GridDesc(C.Structure):
    _fields_ = [("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int), ("n_theta", C.c_int),
                ("n_phi", C.c_int), ("I_top", C.c_double), ("bottom_bc", C.c_int)]


if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1107_5719_amd.build`")

_lib = C.CDLL(LIB_PATH)
_vp, _i, _d = C.c_void_p, C.c_int, C.c_double
_sig = {
    "rt3d_create": (_i, [C.POINTER(_vp), C.POINTER(GridDesc), _i, _vp]),
    "rt3d_destroy": (None, [_vp]),
    "rt3d_set_medium": (_i, [_vp, _vp, _vp, _vp, _i]),
    "rt3d_set_J": (_i, [_vp, _vp, _i]),
    "rt3d_get_J": (_i, [_vp, _vp, _i]),
    "rt3d_formal_solution": (_i, [_vp, _vp, _vp, _i]),
    "rt3d_build_lstar": (_i, [_vp]),
    "rt3d_get_lstar": (_i, [_vp, _vp, _i]),
    "rt3d_os_step": (_i, [_vp, _i, C.POINTER(_d)]),
    "rt3d_solve_to_convergence": (_i, [_vp, _d, _i, _i, C.POINTER(_i), C.POINTER(_d)]),
    "rt3d_set_acceleration": (_i, [_vp, _i, _i]),
    "rt3d_set_anderson": (_i, [_vp, _i]),
    "rt3d_set_os_method": (_i, [_vp, _i]),
    "rt3d_set_coef_storage": (_i, [_vp, _i]),
    "rt3d_get_emergent_top": (_i, [_vp, _vp, _i]),
    "rt3d_set_timing": (_i, [_vp, _i]),
    "rt3d_get_stats": (_i, [_vp, C.c_char_p, _i]),
    "rt3d_status_str": (C.c_char_p, [_i]),
    "rt3d_last_error": (C.c_char_p, [_vp]),
    "rt3d_quadrature": (_i, [_i, _i, _vp, _vp, _vp, _vp]),
    "rt3d_segment_table": (_i, [C.POINTER(GridDesc), _i, _i, _vp, _vp, _vp, _i]),
    "rt3d_validate": (_i, [C.POINTER(GridDesc), _vp, _vp, _vp]),
    "rt3d_get_history": (_i, [_vp, _vp, _vp, _vp, _i]),
    "rt3d_adjoint_emergent": (_i, [_vp, _vp, _d, _i, _i, _vp, _vp, _i, C.POINTER(_i), C.POINTER(_d)]),
    "rt3d_sweep_shapes": (_i, [_vp, _vp, _i]),
    "rt3d_set_sweep_shape": (_i, [_vp, _i]),
    "rt3d_autotune": (_i, [_vp, C.c_char_p, _i, C.POINTER(_i), _vp]),
    "rt3d_batch_create": (_i, [C.POINTER(_vp), _i, _vp, _i, _i, _vp]),
    "rt3d_batch_destroy": (None, [_vp]),
    "rt3d_batch_size": (_i, [_vp]),
    "rt3d_batch_last_error": (C.c_char_p, [_vp]),
    "rt3d_batch_set_medium": (_i, [_vp, _i, _vp, _vp, _vp, _i]),
    "rt3d_batch_set_J": (_i, [_vp, _i, _vp, _i]),
    "rt3d_batch_get_J": (_i, [_vp, _i, _vp, _i]),
    "rt3d_batch_get_Jfs": (_i, [_vp, _i, _vp, _i]),
    "rt3d_batch_set_acceleration": (_i, [_vp, _i, _i]),
    "rt3d_batch_set_anderson": (_i, [_vp, _i]),
    "rt3d_batch_set_sweep_shape": (_i, [_vp, _i]),
    "rt3d_batch_formal_solution": (_i, [_vp]),
    "rt3d_batch_solve": (_i, [_vp, _d, _i, _i, _i, _vp, _vp, _vp]),
    "rt3d_batch_autotune": (_i, [_vp, C.c_char_p, _i, C.POINTER(_i), _vp]),
    "rt3d_batch_get_stats": (_i, [_vp, C.c_char_p, _i]),
    "rt3d_formal_solution_noalloc": (_i, [C.POINTER(GridDesc), _vp, _vp, _vp, _vp, _vp]),
}
for _name, (_res, _args) in _sig.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args


def library():
    """The loaded ctypes library (for tests that check the exported symbols)."""
    return _lib


def _raise(ctx, status: int, what: str, last_error=None, creation=False):
    if status == RT3D_OK:
        return status
    m = None
    if ctx:
        m = (last_error or _lib.rt3d_last_error)(ctx)
    elif creation:
        # with a NULL handle the library reports the calling thread's last failed creation
        m = _lib.rt3d_last_error(None)
    msg = m.decode() if m else ""
    if not msg:
        msg = _lib.rt3d_status_str(status).decode()
    raise Rt3dError(status, f"{what}: {msg}")


def _is_torch(x):
    return type(x).__module__.startswith("torch")


def _arg(x, n=None, writable=False):
    """Return (pointer, ptr_kind, keepalive) for a numpy array or a torch CUDA tensor."""
    if x is None:
        return None, RT3D_HOST, None
    if _is_torch(x):
        import torch

        if not x.is_cuda or x.dtype != torch.float64 or not x.is_contiguous():
            raise ValueError("device arrays must be contiguous float64 CUDA tensors")
        if n is not None and x.numel() != n:
            raise ValueError(f"expected {n} elements, got {x.numel()}")
        return C.c_void_p(x.data_ptr()), RT3D_DEVICE, x
    if writable:
        if not (isinstance(x, np.ndarray) and x.dtype == np.float64 and x.flags.c_contiguous):
            raise ValueError("host outputs must be C-contiguous float64 numpy arrays")
        a = x
    else:
        a = np.ascontiguousarray(x, dtype=np.float64)
    if n is not None and a.size != n:
        raise ValueError(f"expected {n} elements, got {a.size}")
    return a.ctypes.data_as(C.c_void_p), RT3D_HOST, a


def _desc(nx, ny, nz, n_theta, n_phi, I_top=0.0, bottom_bc=0):
    return GridDesc(int(nx), int(ny), int(nz), int(n_theta), int(n_phi), float(I_top), int(bottom_bc))


# ---- functions with the C names -------------------------------------------------------------------

def rt3d_create(desc: GridDesc, precision: int = RT3D_FP64, stream=None):
    """Returns an opaque context handle (c_void_p).  stream: a hipStream_t as int, or None for the
    current torch stream when torch is initialised on a GPU, else the default stream."""
    if stream is None:
        stream = 0
        try:
            import torch

            if torch.cuda.is_available():
                stream = torch.cuda.current_stream().cuda_stream
        except ImportError:
            pass
    ctx = C.c_void_p()
    st = _lib.rt3d_create(C.byref(ctx), C.byref(desc), int(precision), C.c_void_p(stream))
    _raise(None, st, "rt3d_create", creation=True)
    return ctx


def rt3d_destroy(ctx):
    _lib.rt3d_destroy(ctx)


def rt3d_set_medium(ctx, chi, eps, B):
    kinds = []
    ptrs = []
    keep = []
    for a in (chi, eps, B):
        p, k, h = _arg(a)
        ptrs.append(p)
        kinds.append(k)
        keep.append(h)
    if len(set(kinds)) != 1:
        raise ValueError("chi, eps and B must all be host arrays or all device tensors")
    return _raise(ctx, _lib.rt3d_set_medium(ctx, *ptrs, kinds[0]), "rt3d_set_medium")


def rt3d_set_J(ctx, J):
    p, k, h = _arg(J)
    return _raise(ctx, _lib.rt3d_set_J(ctx, p, k), "rt3d_set_J")


def rt3d_get_J(ctx, out):
    p, k, h = _arg(out, writable=True)
    return _raise(ctx, _lib.rt3d_get_J(ctx, p, k), "rt3d_get_J")


def rt3d_formal_solution_noalloc(nx, ny, nz, n_theta, n_phi, chi, S, I_bot, J_fs, I_top=0.0, bottom_bc=0,
                                 stream=None):
    """The context-free, allocation-free formal solution: chi, S, J_fs (and I_bot, or None) are
    contiguous float64 CUDA tensors; stream a raw hipStream_t handle (int) or None."""
    d = _desc(nx, ny, nz, n_theta, n_phi, I_top, bottom_bc)
    V = nx * ny * nz
    pc, kc, _ = _arg(chi, V)
    ps, ks, _ = _arg(S, V)
    pj, kj, _ = _arg(J_fs, V, writable=True)
    pb, kb, _ = _arg(I_bot, nx * ny)
    if RT3D_HOST in (kc, ks, kj) or (I_bot is not None and kb != RT3D_DEVICE):
        raise ValueError("rt3d_formal_solution_noalloc takes device tensors only")
    rc = _lib.rt3d_formal_solution_noalloc(C.byref(d), pc, ps, pb, pj, _vp(stream) if stream else None)
    return _raise(None, rc, "rt3d_formal_solution_noalloc", creation=True)


def rt3d_formal_solution(ctx, S, out):
    """S: None (S from the current J) or an array of the same kind as out."""
    po, ko, ho = _arg(out, writable=True)
    ps, ks, hs = _arg(S)
    if S is not None and ks != ko:
        raise ValueError("S and out must live in the same memory")
    return _raise(ctx, _lib.rt3d_formal_solution(ctx, ps, po, ko), "rt3d_formal_solution")


def rt3d_build_lstar(ctx):
    return _raise(ctx, _lib.rt3d_build_lstar(ctx), "rt3d_build_lstar")


def rt3d_get_lstar(ctx, out):
    p, k, h = _arg(out, writable=True)
    return _raise(ctx, _lib.rt3d_get_lstar(ctx, p, k), "rt3d_get_lstar")


def rt3d_os_step(ctx, inner_sweeps: int):
    """Returns max |dJ|/|J| of the step."""
    c = C.c_double(0.0)
    _raise(ctx, _lib.rt3d_os_step(ctx, int(inner_sweeps), C.byref(c)), "rt3d_os_step")
    return c.value


def rt3d_solve_to_convergence(ctx, tol: float, max_iter: int, inner_sweeps: int, check=True):
    """Returns (status, iterations, last max |dJ|/|J|); raises on any error except
    RT3D_ERR_NOT_CONVERGED unless check is False."""
    it = C.c_int(0)
    c = C.c_double(0.0)
    st = _lib.rt3d_solve_to_convergence(ctx, float(tol), int(max_iter), int(inner_sweeps),
                                        C.byref(it), C.byref(c))
    if check and st not in (RT3D_OK, RT3D_ERR_NOT_CONVERGED):
        _raise(ctx, st, "rt3d_solve_to_convergence")
    return st, it.value, c.value


def rt3d_set_acceleration(ctx, ng_order: int, ng_every: int):
    return _raise(ctx, _lib.rt3d_set_acceleration(ctx, int(ng_order), int(ng_every)),
                  "rt3d_set_acceleration")


def rt3d_set_anderson(ctx, depth: int):
    return _raise(ctx, _lib.rt3d_set_anderson(ctx, int(depth)), "rt3d_set_anderson")


def rt3d_set_os_method(ctx, method: int):
    return _raise(ctx, _lib.rt3d_set_os_method(ctx, int(method)), "rt3d_set_os_method")


def rt3d_set_coef_storage(ctx, storage: int):
    return _raise(ctx, _lib.rt3d_set_coef_storage(ctx, int(storage)), "rt3d_set_coef_storage")


def rt3d_get_emergent_top(ctx, out):
    p, k, h = _arg(out, writable=True)
    return _raise(ctx, _lib.rt3d_get_emergent_top(ctx, p, k), "rt3d_get_emergent_top")


def rt3d_set_timing(ctx, enable):
    """0 / False: off; 1 / True: every launch timed; 2: sampled (see include/rt3d.h)."""
    mode = int(enable) if not isinstance(enable, bool) else (1 if enable else 0)
    return _raise(ctx, _lib.rt3d_set_timing(ctx, mode), "rt3d_set_timing")


def rt3d_get_stats(ctx) -> dict:
    buf = C.create_string_buffer(8192)
    _raise(ctx, _lib.rt3d_get_stats(ctx, buf, len(buf)), "rt3d_get_stats")
    return json.loads(buf.value.decode())


def rt3d_get_history(ctx) -> dict:
    """The per-step record (see include/rt3d.h): arrays max_rel_dJ, ms, float64_fs, ng, anderson."""
    n = _lib.rt3d_get_history(ctx, None, None, None, 0)
    _raise(ctx, min(n, 0), "rt3d_get_history")
    c = np.zeros(n)
    ms = np.zeros(n)
    fl = np.zeros(n, dtype=np.int32)
    _lib.rt3d_get_history(ctx, c.ctypes.data_as(_vp), ms.ctypes.data_as(_vp), fl.ctypes.data_as(_vp), n)
    return {"max_rel_dJ": c, "ms": ms, "float64_fs": (fl & 1) != 0, "ng": (fl & 2) != 0,
            "anderson": (fl & 4) != 0}


def write_history_jsonl(path, history: dict, **extra):
    """One JSON object per step ({"step", "max_rel_dJ", "ms", "float64_fs", "ng", "anderson", **extra}),
    appended."""
    with open(path, "a") as f:
        for q in range(len(history["max_rel_dJ"])):
            rec = {"step": q + 1, "max_rel_dJ": float(history["max_rel_dJ"][q]), "ms": float(history["ms"][q]),
                   "float64_fs": bool(history["float64_fs"][q]), "ng": bool(history["ng"][q]),
                   "anderson": bool(history["anderson"][q])}
            rec.update(extra)
            f.write(json.dumps(rec) + "\n")


def rt3d_status_str(status: int) -> str:
    return _lib.rt3d_status_str(int(status)).decode()


def rt3d_last_error(ctx) -> str:
    m = _lib.rt3d_last_error(ctx)
    return m.decode() if m else ""


def rt3d_quadrature(n_theta: int, n_phi: int):
    nd = n_theta * n_phi
    mu, ox, oy, w = (np.zeros(nd) for _ in range(4))
    st = _lib.rt3d_quadrature(int(n_theta), int(n_phi), *(a.ctypes.data_as(_vp) for a in (mu, ox, oy, w)))
    _raise(None, st, "rt3d_quadrature")
    return mu, ox, oy, w


def rt3d_segment_table(desc: GridDesc, d: int, k: int, max_seg: int = 128):
    di = np.zeros(max_seg, dtype=np.int32)
    dj = np.zeros(max_seg, dtype=np.int32)
    ln = np.zeros(max_seg)
    n = _lib.rt3d_segment_table(C.byref(desc), int(d), int(k), di.ctypes.data_as(_vp),
                                dj.ctypes.data_as(_vp), ln.ctypes.data_as(_vp), int(max_seg))
    if n < 0:
        _raise(None, n, "rt3d_segment_table")
    return di[:n].copy(), dj[:n].copy(), ln[:n].copy()


def rt3d_validate(desc: GridDesc, chi=None, eps=None, B=None) -> int:
    args = [None if a is None else np.ascontiguousarray(a, dtype=np.float64) for a in (chi, eps, B)]
    ptrs = [None if a is None else a.ctypes.data_as(_vp) for a in args]
    return _lib.rt3d_validate(C.byref(desc), *ptrs)


def rt3d_adjoint_emergent(ctx, g_em, dchi_out, deps_out, tol: float = 1e-12, max_iter: int = 2000,
                          inner_sweeps: int = 30, check=True):
    """dL/dchi and dL/deps (written into dchi_out, deps_out) for g_em = dL/dI_em; all arrays host
    numpy or all device tensors.  Returns (status, adjoint steps, last max|d nu|/max|nu|)."""
    pg, kg, hg = _arg(g_em)
    pc, kc, hc = _arg(dchi_out, writable=True)
    pe, ke, he = _arg(deps_out, writable=True)
    if len({kg, kc, ke}) != 1:
        raise ValueError("g_em and the outputs must all be host arrays or all device tensors")
    it = C.c_int(0)
    rel = C.c_double(0.0)
    st = _lib.rt3d_adjoint_emergent(ctx, pg, float(tol), int(max_iter), int(inner_sweeps), pc, pe, kg,
                                    C.byref(it), C.byref(rel))
    if check and st not in (RT3D_OK, RT3D_ERR_NOT_CONVERGED):
        _raise(ctx, st, "rt3d_adjoint_emergent")
    return st, it.value, rel.value


def rt3d_sweep_shapes():
    """[(threads, lines per thread), ...] of the sweep workgroup shapes."""
    n = _lib.rt3d_sweep_shapes(None, None, 0)
    t = np.zeros(n, dtype=np.int32)
    l = np.zeros(n, dtype=np.int32)
    _lib.rt3d_sweep_shapes(t.ctypes.data_as(_vp), l.ctypes.data_as(_vp), n)
    return list(zip(t.tolist(), l.tolist()))


def rt3d_set_sweep_shape(ctx, shape: int):
    return _raise(ctx, _lib.rt3d_set_sweep_shape(ctx, int(shape)), "rt3d_set_sweep_shape")


def _autotune(fn, errfn, handle, cache_path, repeats, what):
    n = _lib.rt3d_sweep_shapes(None, None, 0)
    shape = C.c_int(-1)
    ms = np.zeros(n)
    path = None if cache_path is None else os.fsencode(cache_path)
    _raise(handle, fn(handle, path, int(repeats), C.byref(shape), ms.ctypes.data_as(_vp)), what, errfn)
    return shape.value, ms


def rt3d_autotune(ctx, cache_path=None, repeats: int = 3):
    """Returns (shape, ms per formal solution for every shape, -1 where not measured)."""
    return _autotune(_lib.rt3d_autotune, None, ctx, cache_path, repeats, "rt3d_autotune")


def rt3d_batch_create(descs, precision: int = RT3D_FP64, sweep_shape: int = 0, stream=None):
    """descs: a sequence of GridDesc.  stream: a hipStream_t as int other than the legacy default
    stream, or None for a stream the batch creates."""
    arr = (GridDesc * len(descs))(*descs)
    b = C.c_void_p()
    st = _lib.rt3d_batch_create(C.byref(b), len(descs), C.cast(arr, _vp), int(precision), int(sweep_shape),
                                C.c_void_p(stream or 0))
    _raise(None, st, "rt3d_batch_create", creation=True)
    return b


def rt3d_batch_destroy(b):
    _lib.rt3d_batch_destroy(b)


def rt3d_batch_size(b) -> int:
    return _lib.rt3d_batch_size(b)


def rt3d_batch_last_error(b) -> str:
    m = _lib.rt3d_batch_last_error(b)
    return m.decode() if m else ""


def _braise(b, status, what):
    return _raise(b, status, what, _lib.rt3d_batch_last_error)


def rt3d_batch_set_medium(b, member: int, chi, eps, B):
    ptrs, kinds, keep = [], [], []
    for a in (chi, eps, B):
        p, k, h = _arg(a)
        ptrs.append(p)
        kinds.append(k)
        keep.append(h)
    if len(set(kinds)) != 1:
        raise ValueError("chi, eps and B must all be host arrays or all device tensors")
    return _braise(b, _lib.rt3d_batch_set_medium(b, int(member), *ptrs, kinds[0]), "rt3d_batch_set_medium")


def rt3d_batch_set_J(b, member: int, J):
    p, k, h = _arg(J)
    return _braise(b, _lib.rt3d_batch_set_J(b, int(member), p, k), "rt3d_batch_set_J")


def rt3d_batch_get_J(b, member: int, out):
    p, k, h = _arg(out, writable=True)
    return _braise(b, _lib.rt3d_batch_get_J(b, int(member), p, k), "rt3d_batch_get_J")


def rt3d_batch_get_Jfs(b, member: int, out):
    p, k, h = _arg(out, writable=True)
    return _braise(b, _lib.rt3d_batch_get_Jfs(b, int(member), p, k), "rt3d_batch_get_Jfs")


def rt3d_batch_set_acceleration(b, ng_order: int, ng_every: int):
    return _braise(b, _lib.rt3d_batch_set_acceleration(b, int(ng_order), int(ng_every)),
                   "rt3d_batch_set_acceleration")


def rt3d_batch_set_anderson(b, depth: int):
    return _braise(b, _lib.rt3d_batch_set_anderson(b, int(depth)), "rt3d_batch_set_anderson")


def rt3d_batch_set_sweep_shape(b, shape: int):
    return _braise(b, _lib.rt3d_batch_set_sweep_shape(b, int(shape)), "rt3d_batch_set_sweep_shape")


def rt3d_batch_formal_solution(b):
    return _braise(b, _lib.rt3d_batch_formal_solution(b), "rt3d_batch_formal_solution")


def rt3d_batch_solve(b, tol: float, max_iter: int, inner_sweeps: int, poll_every: int = 4, check=True):
    """Returns (status, iterations[n], last c[n], member states[n]); raises on any error except
    RT3D_ERR_NOT_CONVERGED unless check is False."""
    n = _lib.rt3d_batch_size(b)
    it = np.zeros(n, dtype=np.int32)
    c = np.zeros(n)
    ms = np.zeros(n, dtype=np.int32)
    st = _lib.rt3d_batch_solve(b, float(tol), int(max_iter), int(inner_sweeps), int(poll_every),
                               it.ctypes.data_as(_vp), c.ctypes.data_as(_vp), ms.ctypes.data_as(_vp))
    if check and st not in (RT3D_OK, RT3D_ERR_NOT_CONVERGED):
        _braise(b, st, "rt3d_batch_solve")
    return st, it, c, ms


def rt3d_batch_autotune(b, cache_path=None, repeats: int = 3):
    return _autotune(_lib.rt3d_batch_autotune, _lib.rt3d_batch_last_error, b, cache_path, repeats,
                     "rt3d_batch_autotune")


def rt3d_batch_get_stats(b) -> dict:
    buf = C.create_string_buffer(4096)
    _braise(b, _lib.rt3d_batch_get_stats(b, buf, len(buf)), "rt3d_batch_get_stats")
    return json.loads(buf.value.decode())


# ---- convenience wrapper ----------------------------------------------------------------------------

class Solver:
    """Owns one context; methods map one-to-one onto the C calls."""

    def __init__(self, nx, ny, nz, n_theta, n_phi, I_top=0.0, bottom_bc=0, precision=RT3D_FP64,
                 stream=None):
        self.desc = _desc(nx, ny, nz, n_theta, n_phi, I_top, bottom_bc)
        self.shape = (nz, ny, nx)
        self.n_dir = n_theta * n_phi
        self._token = 0             # changes with every new medium (used by the autograd wrapper)
        self.ctx = rt3d_create(self.desc, precision, stream)

    def close(self):
        if self.ctx:
            rt3d_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def set_medium(self, chi, eps, B):
        rt3d_set_medium(self.ctx, chi, eps, B)
        self._token += 1

    def set_J(self, J):
        rt3d_set_J(self.ctx, J)

    def get_J(self, out=None):
        out = np.zeros(self.shape) if out is None else out
        rt3d_get_J(self.ctx, out)
        return out

    def formal_solution(self, S=None, out=None):
        out = np.zeros(self.shape) if out is None else out
        rt3d_formal_solution(self.ctx, S, out)
        return out

    def build_lstar(self):
        rt3d_build_lstar(self.ctx)

    def get_lstar(self, out=None):
        out = np.zeros((27,) + self.shape) if out is None else out
        rt3d_get_lstar(self.ctx, out)
        return out

    def os_step(self, inner_sweeps):
        return rt3d_os_step(self.ctx, inner_sweeps)

    def solve(self, tol, max_iter, inner_sweeps, log_path=None):
        """rt3d_solve_to_convergence; with log_path the per-step record is appended there as JSONL."""
        out = rt3d_solve_to_convergence(self.ctx, tol, max_iter, inner_sweeps)
        if log_path is not None:
            write_history_jsonl(log_path, self.history(), inner_sweeps=int(inner_sweeps))
        return out

    def history(self):
        return rt3d_get_history(self.ctx)

    def set_acceleration(self, ng_order, ng_every):
        rt3d_set_acceleration(self.ctx, ng_order, ng_every)

    def set_anderson(self, depth):
        """Anderson mixing of the outer iteration with a window of depth (1..8) differences; 0 off."""
        rt3d_set_anderson(self.ctx, depth)

    def set_os_method(self, method):
        """RT3D_OS_JACOBI or RT3D_OS_GAUSS_SEIDEL (multicolour) for the inner solve of the OS step."""
        rt3d_set_os_method(self.ctx, method)

    def set_coef_storage(self, storage):
        """RT3D_COEF_FP64 or RT3D_COEF_FP32: storage precision of the OS step's Jacobi coefficients."""
        rt3d_set_coef_storage(self.ctx, storage)

    def emergent_top(self, out=None):
        out = np.zeros((self.n_dir // 2, self.shape[1], self.shape[2])) if out is None else out
        rt3d_get_emergent_top(self.ctx, out)
        return out

    def set_timing(self, enable=True):
        rt3d_set_timing(self.ctx, enable)

    def stats(self):
        return rt3d_get_stats(self.ctx)

    def set_sweep_shape(self, shape):
        rt3d_set_sweep_shape(self.ctx, shape)

    def autotune(self, cache_path=None, repeats=3):
        return rt3d_autotune(self.ctx, cache_path, repeats)

    def adjoint(self, g_em, tol=1e-12, max_iter=2000, inner_sweeps=30, dchi=None, deps=None):
        """(dL/dchi, dL/deps, status, steps, last rel) for g_em = dL/dI_em (host numpy unless the
        outputs given are device tensors)."""
        dchi = np.zeros(self.shape) if dchi is None else dchi
        deps = np.zeros(self.shape) if deps is None else deps
        st, it, rel = rt3d_adjoint_emergent(self.ctx, g_em, dchi, deps, tol, max_iter, inner_sweeps)
        return dchi, deps, st, it, rel


class Batch:
    """Owns one batch of problems; methods map one-to-one onto the rt3d_batch_* calls.

    grids: a sequence of dicts with keys nx, ny, nz, n_theta, n_phi (and optionally I_top,
    bottom_bc)."""

    def __init__(self, grids, precision=RT3D_FP64, sweep_shape=0, stream=None):
        self.descs = [_desc(g["nx"], g["ny"], g["nz"], g["n_theta"], g["n_phi"], g.get("I_top", 0.0),
                            g.get("bottom_bc", 0)) for g in grids]
        self.shapes = [(d.nz, d.ny, d.nx) for d in self.descs]
        self.b = rt3d_batch_create(self.descs, precision, sweep_shape, stream)

    def close(self):
        if self.b:
            rt3d_batch_destroy(self.b)
            self.b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __len__(self):
        return len(self.descs)

    def set_medium(self, member, chi, eps, B):
        rt3d_batch_set_medium(self.b, member, chi, eps, B)

    def set_J(self, member, J):
        rt3d_batch_set_J(self.b, member, J)

    def get_J(self, member, out=None):
        out = np.zeros(self.shapes[member]) if out is None else out
        rt3d_batch_get_J(self.b, member, out)
        return out

    def get_Jfs(self, member, out=None):
        out = np.zeros(self.shapes[member]) if out is None else out
        rt3d_batch_get_Jfs(self.b, member, out)
        return out

    def set_acceleration(self, ng_order, ng_every):
        rt3d_batch_set_acceleration(self.b, ng_order, ng_every)

    def set_anderson(self, depth):
        """Anderson mixing of depth 0..8 for every member (0: off); switches Ng off."""
        rt3d_batch_set_anderson(self.b, depth)

    def set_sweep_shape(self, shape):
        rt3d_batch_set_sweep_shape(self.b, shape)

    def formal_solution(self):
        rt3d_batch_formal_solution(self.b)

    def solve(self, tol, max_iter, inner_sweeps, poll_every=4, check=True):
        return rt3d_batch_solve(self.b, tol, max_iter, inner_sweeps, poll_every, check)

    def autotune(self, cache_path=None, repeats=3):
        return rt3d_batch_autotune(self.b, cache_path, repeats)

    def stats(self):
        return rt3d_batch_get_stats(self.b)
