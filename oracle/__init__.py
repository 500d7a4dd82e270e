"""FP64 CPU oracle for the 3D scattering solve -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may import
this package.  The product path (the HIP library and its Python binding) never imports, calls or
links anything here, and nothing here imports the product path.

The arithmetic lives in ``oracle.c`` (plain C, FP64, built with gcc); this module only builds and
loads it and marshals numpy arrays.  ``dense_os_solution`` adds the plain definition of the converged
result for tiny grids: the linear system (I - Lambda diag(1-eps)) J = Lambda (eps B) + J_bc.
``loss_gradient_cs`` differentiates a loss on the emergent intensities of that converged result
with respect to every voxel's chi and eps by complex step (tiny grids).

Pins (closed forms, invariants, brute force) live in ``tests/test_oracle_*.py``.  Parity unpinned:
the *number* of outer iterations to convergence (it depends on the readings of the Jacobi depth and
the initial guess, which the paper does not state).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

_dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_ip = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so (gcc, -O2, OpenMP over directions)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        cmd = ["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-Wall", _SRC, "-o", _LIB + ".tmp", "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


_lib = None
_lib_path = None


def build_native(directory: str) -> str:
    """Compile oracle.c with the flags of the timed CPU baseline (gcc -O3 -march=native, OpenMP over
    directions) into `directory` -- on the host that will run it, since the instruction set follows
    that host -- and return the library's path.  The checker library (``build``) stays portable."""
    path = os.path.join(directory, "liboracle_native.so")
    cmd = ["gcc", "-O3", "-march=native", "-fopenmp", "-shared", "-fPIC", _SRC, "-o", path, "-lm"]
    subprocess.run(cmd, check=True, capture_output=True)
    return path


def use_library(path=None):
    """Load the oracle from another build of oracle.c (None: the in-tree checker library)."""
    global _lib, _lib_path
    _lib, _lib_path = None, path
    return lib()


def lib():
    global _lib
    if _lib is None:
        if _lib_path is None and (not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC)):
            build()
        L = C.CDLL(_lib_path or _LIB)
        i, d = C.c_int, C.c_double
        L.orc_gauss_legendre.argtypes = [i, _dp, _dp]
        L.orc_quadrature.argtypes = [i, i, _dp, _dp, _dp, _dp]
        L.orc_trace_layer.argtypes = [i, i, i, i, i, i, i, i, i, _ip, _dp, i]
        L.orc_formal_solution.argtypes = [i, i, i, i, i, _dp, _dp, d, C.c_void_p, _dp, C.c_void_p,
                                          C.c_void_p, i]
        L.orc_formal_solution_dirs.argtypes = [i, i, i, i, i, _dp, _dp, d, C.c_void_p, _dp,
                                               C.c_void_p, C.c_void_p, i, _ip, i]
        L.orc_lstar.argtypes = [i, i, i, i, i, _dp, _dp, i]
        L.orc_lambda_bruteforce.argtypes = [i, i, i, i, i, _dp, _dp, i]
        L.orc_os_step.argtypes = [i, i, i, i, i, _dp, _dp, _dp, d, i, _dp, _dp, i,
                                  C.POINTER(C.c_double), C.c_void_p, i]
        L.orc_os_step_method.argtypes = [i, i, i, i, i, _dp, _dp, _dp, d, i, _dp, _dp, i, i,
                                         C.POINTER(C.c_double), C.c_void_p, i]
        L.orc_os_inner.argtypes = [i, i, i, _dp, _dp, _dp, i, i, _dp]
        L.orc_gs_colour.argtypes = [i, i, i, C.POINTER(C.c_int)]
        L.orc_solve.argtypes = [i, i, i, i, i, _dp, _dp, _dp, d, i, C.c_void_p, _dp, d, i, i,
                                C.POINTER(C.c_int), C.POINTER(C.c_double), i]
        L.orc_solve_ng.argtypes = [i, i, i, i, i, _dp, _dp, _dp, d, i, C.c_void_p, _dp, d, i, i, i, i,
                                   C.POINTER(C.c_int), C.POINTER(C.c_double), i]
        L.orc_ng_extrapolate.argtypes = [C.c_long, i, _dp, i, _dp]
        L.orc_anderson_mix.argtypes = [C.c_long, i, _dp, _dp, _dp]
        L.orc_solve_anderson.argtypes = [i, i, i, i, i, _dp, _dp, _dp, d, i, C.c_void_p, _dp, d, i, i, i,
                                         C.POINTER(C.c_int), C.POINTER(C.c_double), i]
        L.orc_pp1d.argtypes = [i, i, _dp, _dp, d, d, d, _dp]
        L.orc_fs_complex.argtypes = [i, i, i, i, i, _dp, C.c_void_p, _dp, C.c_void_p, d, C.c_void_p,
                                     C.c_void_p, C.c_void_p, _dp, _dp, C.c_void_p, C.c_void_p]
        L.orc_formal_solution_slope.argtypes = [i, i, i, i, i, _dp, _dp, d, C.c_void_p, _dp, _dp,
                                                C.c_void_p, C.c_void_p, i]
        L.orc_diffusion_slope.argtypes = [i, i, _dp, _dp, _dp]
        _lib = L
    return _lib


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _check(rc, what):
    if rc < 0:
        raise RuntimeError(f"oracle {what} failed with code {rc}")
    return rc


def gauss_legendre(n: int):
    x = np.zeros(n)
    w = np.zeros(n)
    _check(lib().orc_gauss_legendre(n, x, w), "gauss_legendre")
    return x, w


def quadrature(n_theta: int, n_phi: int):
    """Returns (mu, ox, oy, W) over directions d = a * n_phi + b."""
    nd = n_theta * n_phi
    mu, ox, oy, wt = (np.zeros(nd) for _ in range(4))
    _check(lib().orc_quadrature(n_theta, n_phi, mu, ox, oy, wt), "quadrature")
    return mu, ox, oy, wt


def trace_layer(nx, ny, nz, n_theta, n_phi, d, i, j, k, max_seg=64):
    """Segments (voxel index, length) of line (i,j), direction d, inside layer k, in travel order."""
    v = np.zeros(max_seg, dtype=np.int32)
    ln = np.zeros(max_seg)
    n = _check(lib().orc_trace_layer(nx, ny, nz, n_theta, n_phi, d, i, j, k, v, ln, max_seg),
               "trace_layer")
    return v[:n].copy(), ln[:n].copy()


def _bottom_mode(bottom_from_B):
    """True / 1: B of the entry voxel; False / 0: zero; "diffusion" / 2: LTE diffusion."""
    if bottom_from_B == "diffusion":
        return 2
    return int(bottom_from_B)


def diffusion_slope(chi, B):
    """dB/dtau at the inner boundary per column: (B_0 - B_1) / ((chi_0 + chi_1) / 2) (works for
    complex chi too)."""
    return (B[0] - B[1]) / (0.5 * (chi[0] + chi[1]))


def formal_solution(chi, S, n_theta, n_phi, I_top=0.0, I_bot=None, want_emergent=False,
                    want_ibar=False, n_threads=0, I_slope=None):
    """J = FS(S).  chi, S: (nz, ny, nx).  I_bot: (ny, nx) or None (zero); I_slope: (ny, nx) or None,
    the LTE-diffusion gradient (an upward line of direction cosine mu enters with I_bot + mu I_slope).

    Returns J (and the top-plane emergent intensities [n_up, ny, nx] and the per-direction voxel
    intensities [n_dir, nz, ny, nx] when asked for)."""
    chi = _f64(chi)
    S = _f64(S)
    nz, ny, nx = chi.shape
    J = np.zeros_like(chi)
    nd = n_theta * n_phi
    Iem = np.zeros((nd // 2, ny, nx)) if want_emergent else None
    Ibar = np.zeros((nd,) + chi.shape) if want_ibar else None
    ib = None if I_bot is None else _f64(np.broadcast_to(I_bot, (ny, nx)))
    if I_slope is None:
        _check(lib().orc_formal_solution(nx, ny, nz, n_theta, n_phi, chi, S, float(I_top), _ptr(ib), J,
                                         _ptr(Iem), _ptr(Ibar), n_threads), "formal_solution")
    else:
        sl = _f64(np.broadcast_to(I_slope, (ny, nx)))
        ib = np.zeros((ny, nx)) if ib is None else ib
        _check(lib().orc_formal_solution_slope(nx, ny, nz, n_theta, n_phi, chi, S, float(I_top), _ptr(ib),
                                               sl, J, _ptr(Iem), _ptr(Ibar), n_threads), "formal_solution")
    out = [J]
    if want_emergent:
        out.append(Iem)
    if want_ibar:
        out.append(Ibar)
    return out[0] if len(out) == 1 else tuple(out)


def formal_solution_dirs(chi, S, n_theta, n_phi, dirs, I_top=0.0, I_bot=None, n_threads=0):
    """The share of J from the listed directions only (used to time a bounded sample)."""
    chi = _f64(chi)
    S = _f64(S)
    nz, ny, nx = chi.shape
    J = np.zeros_like(chi)
    dl = np.ascontiguousarray(dirs, dtype=np.int32)
    ib = None if I_bot is None else _f64(np.broadcast_to(I_bot, (ny, nx)))
    _check(lib().orc_formal_solution_dirs(nx, ny, nz, n_theta, n_phi, chi, S, float(I_top), _ptr(ib),
                                          J, None, None, n_threads, dl, dl.size), "formal_solution_dirs")
    return J


def lstar(chi, n_theta, n_phi, n_threads=0):
    """Lambda* as [27, nz, ny, nx], neighbour index o = 9(dk+1) + 3(dj+1) + (di+1)."""
    chi = _f64(chi)
    nz, ny, nx = chi.shape
    L = np.zeros((27,) + chi.shape)
    _check(lib().orc_lstar(nx, ny, nz, n_theta, n_phi, chi, L, n_threads), "lstar")
    return L


def lambda_bruteforce(chi, n_theta, n_phi, n_threads=0):
    """Dense Lambda [V, V] from unit-source formal solutions (tiny grids only)."""
    chi = _f64(chi)
    nz, ny, nx = chi.shape
    V = chi.size
    Lam = np.zeros((V, V))
    _check(lib().orc_lambda_bruteforce(nx, ny, nz, n_theta, n_phi, chi, Lam, n_threads), "bruteforce")
    return Lam


OS_JACOBI, OS_GAUSS_SEIDEL = 0, 1


def os_step(chi, eps, B, Lstar, J, n_theta, n_phi, M, I_top=0.0, bottom_from_B=True, n_threads=0,
            want_jfs=False, method=OS_JACOBI):
    """One operator-splitting step (M Jacobi or multicolour Gauss-Seidel sweeps).  Returns (J_new, c)
    (and J_fs when asked for)."""
    chi, eps, B, Lstar = _f64(chi), _f64(eps), _f64(B), _f64(Lstar)
    nz, ny, nx = chi.shape
    Jn = _f64(J).copy()
    c = C.c_double(0.0)
    Jfs = np.zeros_like(chi) if want_jfs else None
    _check(lib().orc_os_step_method(nx, ny, nz, n_theta, n_phi, chi, eps, B, float(I_top),
                                    _bottom_mode(bottom_from_B), Lstar, Jn, int(M), int(method), C.byref(c),
                                    _ptr(Jfs), n_threads), "os_step")
    return (Jn, c.value, Jfs) if want_jfs else (Jn, c.value)


def os_inner(eps, Lstar, r, M, method):
    """The inner solve alone: M sweeps (Jacobi or multicolour Gauss-Seidel) of the OS equations
    (1 - Lstar (1 - eps)) dJ = r from dJ = 0.  Returns dJ."""
    eps, Lstar, r = _f64(eps), _f64(Lstar), _f64(r)
    nz, ny, nx = eps.shape
    dJ = np.zeros_like(eps)
    _check(lib().orc_os_inner(nx, ny, nz, eps, Lstar, r, int(M), int(method), dJ), "os_inner")
    return dJ


def gs_colour(n, periodic, i):
    """(colour of index i, colours on the axis) in the Gauss-Seidel ordering."""
    nc = C.c_int(0)
    col = lib().orc_gs_colour(int(n), int(periodic), int(i), C.byref(nc))
    return col, nc.value


def solve(chi, eps, B, n_theta, n_phi, tol, max_iter, M, J0=None, Lstar=None, I_top=0.0,
          bottom_from_B=True, n_threads=0):
    """Outer OS iteration from J0 (default B) until c < tol.  Returns (J, iters, c, converged)."""
    chi, eps, B = _f64(chi), _f64(eps), _f64(B)
    nz, ny, nx = chi.shape
    J = (B if J0 is None else _f64(J0)).copy()
    Ls = None if Lstar is None else _f64(Lstar)
    it = C.c_int(0)
    c = C.c_double(0.0)
    rc = _check(lib().orc_solve(nx, ny, nz, n_theta, n_phi, chi, eps, B, float(I_top),
                                _bottom_mode(bottom_from_B), _ptr(Ls), J, float(tol), int(max_iter), int(M),
                                C.byref(it), C.byref(c), n_threads), "solve")
    return J, it.value, c.value, rc == 0


def solve_ng(chi, eps, B, n_theta, n_phi, tol, max_iter, M, ng_order, ng_every, J0=None, Lstar=None,
             I_top=0.0, bottom_from_B=True, n_threads=0):
    """Outer OS iteration with Ng acceleration (order 1..3 every ng_every steps; 0 = plain).
    Returns (J, iters, c, converged)."""
    chi, eps, B = _f64(chi), _f64(eps), _f64(B)
    nz, ny, nx = chi.shape
    J = (B if J0 is None else _f64(J0)).copy()
    Ls = None if Lstar is None else _f64(Lstar)
    it = C.c_int(0)
    c = C.c_double(0.0)
    rc = _check(lib().orc_solve_ng(nx, ny, nz, n_theta, n_phi, chi, eps, B, float(I_top),
                                   _bottom_mode(bottom_from_B), _ptr(Ls), J, float(tol), int(max_iter), int(M),
                                   int(ng_order), int(ng_every), C.byref(it), C.byref(c), n_threads),
                "solve_ng")
    return J, it.value, c.value, rc == 0


def solve_anderson(chi, eps, B, n_theta, n_phi, tol, max_iter, M, depth, J0=None, Lstar=None, I_top=0.0,
                   bottom_from_B=True, n_threads=0):
    """Outer OS iteration with Anderson mixing of depth 1..8.  Returns (J, iters, c, converged)."""
    chi, eps, B = _f64(chi), _f64(eps), _f64(B)
    nz, ny, nx = chi.shape
    J = (B if J0 is None else _f64(J0)).copy()
    Ls = None if Lstar is None else _f64(Lstar)
    it = C.c_int(0)
    c = C.c_double(0.0)
    rc = _check(lib().orc_solve_anderson(nx, ny, nz, n_theta, n_phi, chi, eps, B, float(I_top),
                                         _bottom_mode(bottom_from_B), _ptr(Ls), J, float(tol), int(max_iter),
                                         int(M), int(depth), C.byref(it), C.byref(c), n_threads),
                "solve_anderson")
    return J, it.value, c.value, rc == 0


def anderson_mix(X, G):
    """One Anderson mixing step from the window of inputs X[0..k] and outputs G[0..k] (oldest first).
    Returns (next input, ok)."""
    xs = _f64(np.stack([np.ravel(x) for x in X]))
    gs = _f64(np.stack([np.ravel(g) for g in G]))
    out = np.zeros(xs.shape[1])
    rc = _check(lib().orc_anderson_mix(xs.shape[1], xs.shape[0] - 1, xs, gs, out), "anderson_mix")
    return out.reshape(np.shape(X[0])), rc == 0


def ng_extrapolate(hist, order):
    """Ng extrapolation of the iterates hist[0..m] (oldest first).  Returns (x, ok)."""
    h = _f64(np.stack([np.ravel(x) for x in hist]))
    out = np.zeros(h.shape[1])
    rc = _check(lib().orc_ng_extrapolate(h.shape[1], int(order), h, h.shape[0] - 1, out), "ng")
    return out.reshape(np.shape(hist[0])), rc == 0


def pp1d(dtau, S, n_theta, I_top=0.0, I_bot=0.0, I_slope=0.0):
    """Plane-parallel J_k for layer thicknesses dtau[k] (k = 0 bottom) and sources S[k]; upward light
    enters the bottom with I_bot + mu I_slope."""
    dtau, S = _f64(dtau), _f64(S)
    J = np.zeros_like(dtau)
    _check(lib().orc_pp1d(dtau.size, n_theta, dtau, S, float(I_top), float(I_bot), float(I_slope), J),
           "pp1d")
    return J


def dense_os_solution(chi, eps, B, n_theta, n_phi, I_top=0.0, bottom_from_B=True, n_threads=0):
    """Converged J by its plain definition (tiny grids): solve (I - Lambda diag(1-eps)) J = rhs,
    rhs = Lambda (eps B) + J_bc, where J_bc is the mean intensity of the boundary light alone."""
    chi, eps, B = _f64(chi), _f64(eps), _f64(B)
    Lam = lambda_bruteforce(chi, n_theta, n_phi, n_threads)
    V = chi.size
    mode = _bottom_mode(bottom_from_B)
    J_bc = formal_solution(chi, np.zeros_like(chi), n_theta, n_phi, I_top=I_top,
                           I_bot=(B[0] if mode else None), n_threads=n_threads,
                           I_slope=(diffusion_slope(chi, B) if mode == 2 else None)).ravel()
    A = np.eye(V) - Lam * (1.0 - eps.ravel())[None, :]
    rhs = Lam @ (eps * B).ravel() + J_bc
    return np.linalg.solve(A, rhs).reshape(chi.shape)


# ---- derivatives through the converged solution (complex step) ------------------------------------

def fs_complex(chi, S, n_theta, n_phi, I_top=0.0, I_bot=None, want_emergent=False, I_slope=None):
    """The formal solution in complex arithmetic: chi and S may be complex (nz, ny, nx) arrays, and
    the LTE-diffusion gradient I_slope (ny, nx) too.  Returns J (complex) and, when asked for, the
    emergent top intensities [n_up, ny, nx] (complex)."""
    chi = np.asarray(chi)
    S = np.asarray(S)
    nz, ny, nx = chi.shape
    cr, ci = _f64(chi.real), _f64(chi.imag) if np.iscomplexobj(chi) else None
    sr, si = _f64(S.real), _f64(S.imag) if np.iscomplexobj(S) else None
    Jr, Ji = np.zeros(chi.shape), np.zeros(chi.shape)
    nup = n_theta * n_phi // 2
    Er = Ei = None
    if want_emergent:
        Er, Ei = np.zeros((nup, ny, nx)), np.zeros((nup, ny, nx))
    Ib = None if I_bot is None else _f64(I_bot)
    slr = sli = None
    if I_slope is not None:
        sl = np.asarray(I_slope)
        slr = _f64(sl.real)
        sli = _f64(sl.imag) if np.iscomplexobj(sl) else None
    _check(lib().orc_fs_complex(nx, ny, nz, n_theta, n_phi, cr, _ptr(ci), sr, _ptr(si), float(I_top),
                                _ptr(Ib), _ptr(slr), _ptr(sli), Jr, Ji, _ptr(Er), _ptr(Ei)), "fs_complex")
    J = Jr + 1j * Ji
    return (J, Er + 1j * Ei) if want_emergent else J


def _converged_emergent(chi, eps, B, n_theta, n_phi, I_top, bottom_from_B, Lam=None):
    """Converged J and emergent intensities by the plain definition, in complex arithmetic:
    J = (I - Lambda diag(1-eps))^{-1} FS(eps B; boundary light), then I_em = FS_em(eps B + (1-eps) J)."""
    V = chi.size
    mode = _bottom_mode(bottom_from_B)
    I_bot = B[0].real.copy() if mode else None
    I_slope = diffusion_slope(chi, B) if mode == 2 else None
    if Lam is None:
        Lam = np.zeros((V, V), dtype=complex)
        for u in range(V):
            e = np.zeros(V)
            e[u] = 1.0
            Lam[:, u] = fs_complex(chi, e.reshape(chi.shape), n_theta, n_phi).ravel()
    rhs = fs_complex(chi, eps * B, n_theta, n_phi, I_top=I_top, I_bot=I_bot, I_slope=I_slope).ravel()
    A = np.eye(V) - Lam * (1.0 - eps.ravel())[None, :]
    J = np.linalg.solve(A, rhs).reshape(chi.shape)
    S = eps * B + (1.0 - eps) * J
    _, Iem = fs_complex(chi, S, n_theta, n_phi, I_top=I_top, I_bot=I_bot, want_emergent=True,
                        I_slope=I_slope)
    return J, Iem


def emergent_loss(chi, eps, B, T, n_theta, n_phi, I_top=0.0, bottom_from_B=True):
    """L = sum over the upward directions and top-plane lines of (I_em - T)^2 at the converged
    solution (dense definition).  bottom_from_B as for solve (True, False or "diffusion").
    Returns (L, I_em, J)."""
    chi, eps, B = _f64(chi), _f64(eps), _f64(B)
    J, Iem = _converged_emergent(chi.astype(complex), eps.astype(complex), B.astype(complex), n_theta,
                                 n_phi, I_top, bottom_from_B)
    Iem = Iem.real
    return float(np.sum((Iem - T) ** 2)), Iem, J.real


def loss_gradient_cs(chi, eps, B, T, n_theta, n_phi, I_top=0.0, bottom_from_B=True, h=1e-30):
    """dL/dchi_v and dL/deps_v of emergent_loss for every voxel, by complex step: one complex
    evaluation of the converged solution per parameter with that parameter moved by i h; the
    derivative is Im L / h.  Tiny grids only (a dense Lambda per chi parameter)."""
    chi, eps, B = _f64(chi), _f64(eps), _f64(B)
    T = _f64(T)
    shape = chi.shape
    V = chi.size
    gchi = np.zeros(V)
    geps = np.zeros(V)
    chi_c, eps_c, B_c = chi.astype(complex), eps.astype(complex), B.astype(complex)
    for v in range(V):
        c = chi_c.copy().ravel()
        c[v] += 1j * h
        _, Iem = _converged_emergent(c.reshape(shape), eps_c, B_c, n_theta, n_phi, I_top, bottom_from_B)
        gchi[v] = np.sum((Iem - T) ** 2).imag / h
    Lam = np.zeros((V, V), dtype=complex)
    for u in range(V):
        e = np.zeros(V)
        e[u] = 1.0
        Lam[:, u] = fs_complex(chi_c, e.reshape(shape), n_theta, n_phi).ravel()
    for v in range(V):
        e_c = eps_c.copy().ravel()
        e_c[v] += 1j * h
        _, Iem = _converged_emergent(chi_c, e_c.reshape(shape), B_c, n_theta, n_phi, I_top, bottom_from_B,
                                     Lam=Lam)
        geps[v] = np.sum((Iem - T) ** 2).imag / h
    return gchi.reshape(shape), geps.reshape(shape)
