#!/usr/bin/env python3
"""Benchmark of the 3D scattering hot path on one MI355X.

One step = one operator-splitting iteration over the whole grid: S update, formal solution (FS)
sweeps for every direction, angle reduction to J_fs with the residual, M Jacobi sweeps of the
27-point OS equations, J update and the max |dJ|/|J| convergence measure.  Lambda* is built once
before the timed region (it depends only on chi) and is part of the separately reported
time-to-converged J.  Inputs (chi, eps, B) are resident in HBM before timing starts.

value = voxel-angle FS updates per second of whole steps = V * n_dir * steps / elapsed.

Prints one JSON line.  Multi-GPU runs are not part of this build: --gpus > 1 exits with a message.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "voxel·angle FS updates/s + time-to-converged J, 129³×256 angles, FP32 vs FP64"
HBM_PEAK_GBS = 8000.0


def sweep_bytes_per_update(precision: str) -> int:
    """Algorithmic HBM bytes of the sweep kernel per voxel-angle update: chi and S of the voxel read
    once per direction, and one partial-plane value written once per direction."""
    s_r = 8 if precision == "fp64" else 4
    return 2 * s_r + s_r


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="strat129")
    ap.add_argument("--precision", choices=["fp64", "fp32"], default="fp64")
    ap.add_argument("--inner-sweeps", type=int, default=20, help="Jacobi sweeps per OS step (M)")
    ap.add_argument("--converge-max-iter", type=int, default=400,
                    help="outer-iteration cap of the time-to-converged-J run (0 skips it)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-every", type=int, default=8,
                    help="the CPU oracle times every n-th direction of the full grid")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (asked for --gpus {args.gpus}); the path "
              "would shard over directions with one all-reduce of J_fs per iteration, which is not "
              "part of this build.", file=sys.stderr)
        return 2
    if int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: launched with WORLD_SIZE > 1; one GPU only", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        return 1
    dev = torch.device("cuda:0")
    torch.zeros(1, device=dev)

    from paper_1107_5719_amd import rt3d
    from paper_1107_5719_amd.inputs import WORKLOADS, make_medium

    w = WORKLOADS[args.workload]
    med = make_medium(w)
    d_med = {k: torch.from_numpy(v).to(dev) for k, v in med.items()}
    torch.cuda.synchronize()
    V = w.n_vox
    n_dir = w.n_dir
    prec = rt3d.RT3D_FP64 if args.precision == "fp64" else rt3d.RT3D_FP32_SWEEP
    stream = torch.cuda.current_stream().cuda_stream

    # ---- timed steps -------------------------------------------------------------------------
    s = rt3d.Solver(w.nx, w.ny, w.nz, w.n_theta, w.n_phi, I_top=w.I_top, precision=prec, stream=stream)
    s.set_medium(d_med["chi"], d_med["eps"], d_med["B"])
    t0 = time.perf_counter()
    s.build_lstar()
    lstar_s = time.perf_counter() - t0
    for _ in range(args.warmup):
        s.os_step(args.inner_sweeps)
    s.set_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    last_c = None
    for _ in range(args.steps):
        last_c = s.os_step(args.inner_sweeps)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    st = s.stats()
    s.set_timing(False)
    ms_per_step = 1e3 * elapsed / args.steps
    value = V * n_dir * args.steps / elapsed
    kern = st["kernels"]
    per_launch = {k: (v["total_ms"] / v["launches"] if v["launches"] else None) for k, v in kern.items()}
    sweep_ms = per_launch["sweep"]
    fs_ms = sum(per_launch[k] for k in ("source", "sweep", "reduce"))
    b_unit = sweep_bytes_per_update(args.precision)
    achieved = b_unit * V * n_dir / (sweep_ms * 1e-3) / 1e9
    roofline = {"kernel": "sweep_kernel", "bound": "hbm", "achieved": round(achieved, 1),
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": None, "bytes_per_update": b_unit,
                "sweep_ms_per_launch": round(sweep_ms, 4)}
    s.close()

    # ---- time to converged J (Lambda* build included) -----------------------------------------
    conv = None
    if args.converge_max_iter > 0:
        s2 = rt3d.Solver(w.nx, w.ny, w.nz, w.n_theta, w.n_phi, I_top=w.I_top, precision=prec,
                         stream=stream)
        s2.set_medium(d_med["chi"], d_med["eps"], d_med["B"])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        status, iters, c = s2.solve(w.tol, args.converge_max_iter, args.inner_sweeps)
        torch.cuda.synchronize()
        tconv = time.perf_counter() - t0
        conv = {"seconds": round(tconv, 4), "outer_iterations": iters,
                "inner_sweeps_per_step": args.inner_sweeps, "final_max_rel_dJ": c,
                "tol": w.tol, "converged": status == rt3d.RT3D_OK}
        s2.close()

    # ---- CPU oracle on a bounded sample of the same workload -------------------------------------
    cpu = None
    if not args.no_cpu_baseline:
        import oracle

        threads = min(os.cpu_count() or 1, 16)
        dirs = list(range(0, n_dir, args.cpu_sample_every))
        S = med["eps"] * med["B"] + (1 - med["eps"]) * med["B"]
        t0 = time.perf_counter()
        oracle.formal_solution_dirs(med["chi"], S, w.n_theta, w.n_phi, dirs, I_top=w.I_top,
                                    I_bot=med["B"][0], n_threads=threads)
        tcpu = time.perf_counter() - t0
        cpu = {"value": V * len(dirs) / tcpu, "unit": "voxel-angle FS updates/s", "cores": min(threads, len(dirs)),
               "kind": "oracle",
               "sample": f"FP64 oracle formal solution of {len(dirs)} of the {n_dir} directions "
                         f"(every {args.cpu_sample_every}th) on the full {w.nx}x{w.ny}x{w.nz} grid, "
                         f"{tcpu:.2f} s wall"}

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "voxel-angle FS updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32",
        "data": "synthetic",
        "config": {"workload": f"{w.name}: {w.nx}x{w.ny}x{w.nz} voxels x {n_dir} angles "
                               f"({w.n_theta} mu x {w.n_phi} phi), eps={w.eps:g}, tau_total={w.tau_total:g}, "
                               f"chi log-normal sigma={w.sigma}, seed {w.seed}",
                   "precision": "fp64" if args.precision == "fp64" else "fp32 sweeps, fp64 J/OS/convergence",
                   "inner_sweeps": args.inner_sweeps,
                   "step": "one OS iteration: S update, FS over all angles, J reduction + residual, "
                           "M Jacobi sweeps, J update + max rel dJ"},
        "fs_updates_per_s_fs_kernels_only": V * n_dir / (fs_ms * 1e-3),
        "kernel_ms_per_launch": {k: (round(v, 4) if v is not None else None) for k, v in per_launch.items()},
        "lstar_build_s": round(lstar_s, 4),
        "last_step_max_rel_dJ": last_c,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "time_to_converged": conv,
    }
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
