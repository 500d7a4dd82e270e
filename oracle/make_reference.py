"""Tightly converged FP64 oracle solutions of the benchmark workloads -- TEST INFRASTRUCTURE ONLY.

Runs on the CPU and calls nothing but the oracle (``oracle/``) and the seeded input generators
(``paper_1107_5719_amd/inputs.py``, which hold none of the method's arithmetic).  For each named
workload it solves the scattering problem with the oracle's own operator-splitting iteration (M
Jacobi sweeps per step, Ng or Anderson acceleration) until max |dJ|/|J| < tol (or until c stops
falling: the rounding floor of the iteration), and writes

    oracle/reference/<name>.npz    J (float64, [nz][ny][nx])
    oracle/reference/<name>.json   tol, M, acceleration, iterations, last and smallest c, why it
                                   stopped, wall seconds, and the
                                   SHA-256 of the inputs (chi, eps, B and the grid), of oracle.c and
                                   of J itself

The converged J does not depend on M or on the acceleration (the fixed point is that of the linear
system (I - Lambda diag(1-eps)) J = Lambda (eps B) + J_bc); they only set how fast it is reached.
The benchmark reads these files to state the error of each GPU form against the oracle; a file whose
input or oracle hash no longer matches is ignored there.  The directory is not under version control.

    python -m oracle.make_reference strat17 grf65 strat129 [--threads N] [--tol 1e-12] [--anderson DEPTH]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
REF_DIR = os.path.join(HERE, "reference")


def input_sha256(w, med) -> str:
    """SHA-256 of the grid, angle set, boundary light and the medium arrays."""
    h = hashlib.sha256()
    h.update(f"{w.nx}x{w.ny}x{w.nz}|{w.n_theta}x{w.n_phi}|I_top={w.I_top!r}".encode())
    for k in ("chi", "eps", "B"):
        h.update(np.ascontiguousarray(med[k], dtype=np.float64).tobytes())
    return h.hexdigest()


def oracle_sha256() -> str:
    with open(os.path.join(HERE, "oracle.c"), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def array_sha256(a) -> str:
    return hashlib.sha256(np.ascontiguousarray(a, dtype=np.float64).tobytes()).hexdigest()


def load(name: str, w, med):
    """(J, meta) of a stored reference whose input and oracle hashes match, else (None, reason)."""
    npz = os.path.join(REF_DIR, f"{name}.npz")
    meta_path = os.path.join(REF_DIR, f"{name}.json")
    if not (os.path.exists(npz) and os.path.exists(meta_path)):
        return None, "no stored oracle solution (python -m oracle.make_reference " + name + ")"
    with open(meta_path) as f:
        meta = json.load(f)
    if meta.get("input_sha256") != input_sha256(w, med):
        return None, "stored oracle solution belongs to other inputs"
    if meta.get("oracle_sha256") != oracle_sha256():
        return None, "stored oracle solution was made by another oracle.c"
    J = np.load(npz, allow_pickle=False)["J"]
    if array_sha256(J) != meta.get("J_sha256"):
        return None, "stored oracle solution does not match its recorded hash"
    return J, meta


def make(name: str, tol: float, M: int, ng_order: int, ng_every: int, threads: int, max_iter: int,
         stall: int, anderson: int = 0) -> dict:
    """The oracle's operator-splitting iteration, one oracle step at a time, with Ng acceleration (the
    schedule of the oracle's own solve_ng: the iterate joins a history restarted at each
    extrapolation, and the newest ng_order + 2 iterates are extrapolated once it holds ng_every
    steps) or, when `anderson` > 0, with the oracle's Anderson mixing of that depth over the newest
    (input, output) pairs of the step (the schedule of the oracle's own solve_anderson).  Stops at
    c < tol, after max_iter steps, or when c has not reached a new minimum for `stall` steps (the
    rounding floor of the iteration lies above tol)."""
    sys.path.insert(0, ROOT)
    import oracle
    from paper_1107_5719_amd.inputs import WORKLOADS, make_medium

    w = WORKLOADS[name]
    med = make_medium(w)
    src_sha = oracle_sha256()          # the source the loaded library was built from
    t0 = time.perf_counter()
    L = oracle.lstar(med["chi"], w.n_theta, w.n_phi, n_threads=threads)
    print(f"{name}: Lambda* built in {time.perf_counter() - t0:.1f} s", flush=True)
    J = med["B"].copy()
    if anderson:
        ng_order = 0
    hist = [J.copy()] if ng_order else []
    win_x, win_g = [], []
    c, c_min, n_min, n, reason = float("inf"), float("inf"), 0, 0, "max_iter"
    while n < max_iter:
        x_in = J
        J, c = oracle.os_step(med["chi"], med["eps"], med["B"], L, J, w.n_theta, w.n_phi, M, I_top=w.I_top,
                              n_threads=threads)
        n += 1
        print(f"{name}: step {n} c={c:.3e} ({time.perf_counter() - t0:.0f} s)", flush=True)
        if c < tol:
            reason = "tol"
            break
        if c < c_min:
            c_min, n_min = c, n
        elif n - n_min >= stall:
            reason = "stalled"
            break
        if anderson:
            win_x.append(x_in)
            win_g.append(J.copy())
            win_x, win_g = win_x[-(anderson + 1):], win_g[-(anderson + 1):]
            if len(win_x) >= 2:
                x, ok = oracle.anderson_mix(win_x, win_g)
                if ok:
                    J = x
        if ng_order:
            hist.append(J.copy())
            if len(hist) - 1 >= ng_every:
                x, ok = oracle.ng_extrapolate(hist, ng_order)
                if ok:
                    J = x
                hist = [J.copy()]
    secs = time.perf_counter() - t0
    os.makedirs(REF_DIR, exist_ok=True)
    np.savez(os.path.join(REF_DIR, f"{name}.npz"), J=J)
    meta = {"workload": name, "grid": [w.nx, w.ny, w.nz], "angles": [w.n_theta, w.n_phi], "tol": tol,
            "inner_sweeps": M, "ng_order": ng_order, "ng_every": ng_every if ng_order else 0,
            "anderson_depth": anderson, "iterations": n,
            "final_max_rel_dJ": c, "min_max_rel_dJ": min(c, c_min), "stop": reason,
            "seconds": round(secs, 1), "threads": threads,
            "input_sha256": input_sha256(w, med), "oracle_sha256": src_sha,
            "J_sha256": array_sha256(J)}
    with open(os.path.join(REF_DIR, f"{name}.json"), "w") as f:
        json.dump(meta, f, indent=1)
    return meta


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("names", nargs="+")
    ap.add_argument("--tol", type=float, default=1e-12)
    ap.add_argument("--inner-sweeps", type=int, default=30)
    ap.add_argument("--ng-order", type=int, default=3)
    ap.add_argument("--ng-every", type=int, default=6)
    ap.add_argument("--threads", type=int, default=0, help="OpenMP threads (0: the OpenMP default)")
    ap.add_argument("--max-iter", type=int, default=3000)
    ap.add_argument("--anderson", type=int, default=0,
                    help="Anderson mixing of this depth (1..8) instead of Ng")
    ap.add_argument("--stall", type=int, default=60,
                    help="stop when c has not reached a new minimum for this many steps")
    args = ap.parse_args()
    for name in args.names:
        meta = make(name, args.tol, args.inner_sweeps, args.ng_order, args.ng_every, args.threads, args.max_iter,
                    args.stall, args.anderson)
        print(json.dumps(meta), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
