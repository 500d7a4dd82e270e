#!/usr/bin/env python3
"""Benchmark of the 3D scattering hot path on one MI355X.

One step = one operator-splitting iteration over the whole grid: S update, formal solution (FS)
sweeps for every direction, angle reduction to J_fs with the residual, M Jacobi sweeps of the
27-point OS equations, J update and the max |dJ|/|J| convergence measure.  Lambda* is built once
before the timed region (it depends only on chi) and is part of the separately reported
time-to-converged J.  Inputs (chi, eps, B) are resident in HBM before timing starts.

value = voxel-angle FS updates per second of whole steps = V * n_dir * steps / elapsed.

Prints one JSON line.  The library runs on one GPU: --gpus > 1 exits with a message.
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
# MI355X vector issue: 256 CUs x 4 SIMDs x 2.4 GHz; float64 16 lanes per SIMD and cycle (78.6 TFLOP/s
# counting an FMA as 2 flops, i.e. 39.3e12 lane-instructions/s), float32 32 lanes (78.6e12)
VALU_ISSUE_PEAK = {"fp64": 39.3e12, "fp32": 78.6e12}
SWEEP_KERNEL = {"fp64": "sweep_kernel<double,512,2>", "fp32": "sweep_kernel<float,512,2>"}
JACOBI_KERNEL = {"fp64": "jacobi_kernel_column<double,4>", "fp32": "jacobi_kernel_column<float,4>"}
# the (M, Ng order, Ng every) schedules over which time to converged J is summarised (median, worst)
SCHEDULES = [(12, 3, 6), (20, 3, 6), (30, 3, 6), (40, 3, 6), (12, 3, 8), (20, 3, 8), (30, 3, 8), (40, 3, 8)]
# the (M, depth) schedules of Anderson mixing
AA_SCHEDULES = [(12, 5), (20, 5), (30, 5), (12, 8), (20, 8), (30, 8)]


SWEEP_G = 2   # directions that share one gather of a voxel's chi, S and one partial-plane deposit


def sweep_bytes_per_update(precision: str, G: int = SWEEP_G) -> int:
    """Algorithmic HBM bytes of the formal-solution sweep per voxel-angle update, (2 s_r + 16) / G: chi
    and S of the voxel (s_r bytes each: 8 in float64, 4 in float32 sweeps) and a float64 read-modify-
    write of the voxel's J partial, shared by the G directions that use one gather and one deposit
    (G = 2 here: the lines of an x-mirrored direction pair are paired so that both cross the same
    voxel at every segment, and the pair has one partial plane)."""
    s_r = 8 if precision == "fp64" else 4
    return (2 * s_r + 16) // G


def jacobi_bytes_per_voxel(coef: str) -> int:
    """Algorithmic HBM bytes of one intermediate Jacobi sweep per voxel: 13 stored coefficients (the
    other 13 are their mirrors), the right-hand side chi (J_fs - J), E = (1 - eps)/D, the previous
    (1 - eps) dJ and the new one (float64 but for float32-stored coefficients)."""
    return 13 * (8 if coef == "fp64" else 4) + 4 * 8


def _kernel_sha() -> str:
    import hashlib

    src = os.path.join(ROOT, "paper_1107_5719_amd", "csrc", "kernels.h")
    return hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]


def measured_traffic(kernel: str):
    """HBM bytes per dispatch (FETCH_SIZE + WRITE_SIZE, scaled by the copy calibration) from the
    committed rocprofv3 summary, or None if the kernel source changed since it was measured."""
    prof = os.path.join(ROOT, "profiles", "strat129_hbm_bytes.txt")
    if not os.path.exists(prof):
        return None
    sha = _kernel_sha()
    for line in open(prof):
        if line.startswith("TRAFFIC "):
            f = dict(kv.split("=", 1) for kv in line.split()[1:])
            if f["kernel"] == kernel and f["source_sha"] == sha:
                return int(f["fetch_bytes"]) + int(f["write_bytes"])
    return None


def measured_valu(kernel: str):
    """SQ_INSTS_VALU (wave instructions per dispatch) of a kernel from the committed rocprofv3
    counter summary, or None if the kernel source changed since it was measured."""
    prof = os.path.join(ROOT, "profiles", "strat129_sq_counters.txt")
    if not os.path.exists(prof):
        return None
    sha = None
    for line in open(prof):
        if line.startswith("# kernel source sha256[:16]:"):
            sha = line.rsplit(":", 1)[1].strip()
        elif line.startswith(kernel + " ") and sha == _kernel_sha():
            f = dict(kv.split("=", 1) for kv in line.split() if "=" in kv)
            return float(f["SQ_INSTS_VALU"])
    return None


def oracle_reference(w, med):
    """The oracle's tightly converged J of a workload, as written by the committed CPU-only script
    (python -m oracle.make_reference <name>) into oracle/reference/: (J, meta) when the stored file
    belongs to these inputs, else (None, reason).  The input hash follows the script's definition:
    SHA-256 of the grid, angle set, top light and the chi, eps, B arrays."""
    import hashlib

    import numpy as np

    base = os.path.join(ROOT, "oracle", "reference", w.name)
    if not (os.path.exists(base + ".npz") and os.path.exists(base + ".json")):
        return None, f"no stored oracle solution (python -m oracle.make_reference {w.name})"
    meta = json.load(open(base + ".json"))
    h = hashlib.sha256(f"{w.nx}x{w.ny}x{w.nz}|{w.n_theta}x{w.n_phi}|I_top={w.I_top!r}".encode())
    for k in ("chi", "eps", "B"):
        h.update(np.ascontiguousarray(med[k], dtype=np.float64).tobytes())
    if meta.get("input_sha256") != h.hexdigest():
        return None, "stored oracle solution belongs to other inputs"
    J = np.load(base + ".npz", allow_pickle=False)["J"]
    if hashlib.sha256(np.ascontiguousarray(J).tobytes()).hexdigest() != meta.get("J_sha256"):
        return None, "stored oracle solution does not match its recorded hash"
    src = hashlib.sha256(open(os.path.join(ROOT, "oracle", "oracle.c"), "rb").read()).hexdigest()
    meta = {k: meta[k] for k in ("tol", "iterations", "final_max_rel_dJ", "min_max_rel_dJ", "stop",
                                 "inner_sweeps", "ng_order", "ng_every", "anderson_depth") if k in meta}
    meta["oracle_source_unchanged"] = src == json.load(open(base + ".json")).get("oracle_sha256")
    return J, meta


def _rel_err(J, ref) -> float:
    import torch

    return float(torch.max(torch.abs(J / ref - 1)).item())


def _cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip() + f" ({os.cpu_count()} logical CPUs visible)"
    except OSError:
        pass
    return f"unknown ({os.cpu_count()} logical CPUs visible)"


def _timed_steps(rt3d, torch, w, d_med, prec, stream, steps, warmup, M, coef=None):
    """K timed OS steps after W warm-up steps; per-kernel HIP-event times from the library.  coef:
    storage of the Jacobi coefficients (None: the form's default)."""
    s = rt3d.Solver(w.nx, w.ny, w.nz, w.n_theta, w.n_phi, I_top=w.I_top, precision=prec, stream=stream)
    if coef is not None:
        s.set_coef_storage(coef)
    s.set_medium(d_med["chi"], d_med["eps"], d_med["B"])
    t0 = time.perf_counter()
    s.build_lstar()
    lstar_s = time.perf_counter() - t0
    for _ in range(warmup):
        s.os_step(M)
    # sampled timing: per OS step the source, sweep and reduction launches are bracketed by HIP events
    # and the intermediate Jacobi sweeps by one pair (bracketing all 33 launches costs ~4% of the step)
    s.set_timing(2)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        s.os_step(M)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    st = s.stats()
    s.close()
    per_launch = {k: (v["total_ms"] / v["timed"] if v.get("timed") else None)
                  for k, v in st["kernels"].items()}
    return elapsed, per_launch, lstar_s, st


def _converge(rt3d, torch, w, d_med, prec, stream, M, ng_order, ng_every, tol, max_iter, os_method=0,
              coef=None, anderson=0):
    """Time from resident inputs (Lambda* build included) to max rel dJ < tol (Ng or, with anderson > 0,
    Anderson mixing of that depth)."""
    s = rt3d.Solver(w.nx, w.ny, w.nz, w.n_theta, w.n_phi, I_top=w.I_top, precision=prec, stream=stream)
    if coef is not None:
        s.set_coef_storage(coef)
    s.set_medium(d_med["chi"], d_med["eps"], d_med["B"])
    s.set_os_method(os_method)
    if anderson:
        s.set_anderson(anderson)
    elif ng_order:
        s.set_acceleration(ng_order, ng_every)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    status, iters, c = s.solve(tol, max_iter, M)
    torch.cuda.synchronize()
    secs = time.perf_counter() - t0
    st = s.stats()
    J = torch.zeros((w.nz, w.ny, w.nx), dtype=torch.float64, device="cuda")
    s.get_J(J)
    s.close()
    return J, {"seconds": round(secs, 4), "outer_iterations": iters, "final_max_rel_dJ": c,
               "converged": status == rt3d.RT3D_OK, "fp64_sweeps": st["fp64_sweeps"],
               "fp32_sweeps": st["fp32_sweeps"]}


def _batched(rt3d, torch, n_wl, M, ng, tol, ref_tol, max_iter, cache, aa_depth=0, aa_sweeps=None):
    """The many-wavelength form: n_wl wavelengths, grids drawn from {33, 65, 97}^3, 64 angles each.

    Time to converged J of all of them (inputs resident, Lambda* builds included) for three forms:
    the plain float64 path one wavelength at a time (one context each, shape autotuned per grid),
    the batch in float64 and the batch with float32 sweeps; each against a float64 batch solved to
    ref_tol.  Also the batched formal-solution rate, and (aa_depth > 0) the three forms again with
    Anderson mixing of that depth instead of Ng, at aa_sweeps inner sweeps (default M)."""
    from paper_1107_5719_amd.inputs import wavelength_batch

    mem = wavelength_batch(n_wl)
    grids = [m["grid"] for m in mem]
    dm = [{k: torch.from_numpy(m[k]).cuda() for k in ("chi", "eps", "B")} for m in mem]
    torch.cuda.synchronize()
    vox = sum(g["nx"] * g["ny"] * g["nz"] for g in grids)
    vox_ang = sum(g["nx"] * g["ny"] * g["nz"] * g["n_theta"] * g["n_phi"] for g in grids)
    sizes = {}
    for g in grids:
        sizes[g["nx"]] = sizes.get(g["nx"], 0) + 1

    def fetch(getter, i):
        J = torch.zeros(dm[i]["B"].shape, dtype=torch.float64, device="cuda")
        getter(i, J)
        return J

    def run_batch(prec, tol_, fs_reps, aa=0, M=M):
        b = rt3d.Batch(grids, precision=prec)
        for i, d in enumerate(dm):
            b.set_medium(i, d["chi"], d["eps"], d["B"])
        shape, ms = b.autotune(cache, repeats=3)
        fs = None
        if fs_reps:
            b.formal_solution()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(fs_reps):
                b.formal_solution()
            dt = (time.perf_counter() - t0) / fs_reps
            fs = {"ms": round(1e3 * dt, 3), "voxel_angle_updates_per_s": vox_ang / dt}
        if aa:
            b.set_anderson(aa)
        elif ng[0]:
            b.set_acceleration(*ng)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st, iters, cs, states = b.solve(tol_, max_iter, M, poll_every=4, check=False)
        torch.cuda.synchronize()
        secs = time.perf_counter() - t0
        stats = b.stats()
        Js = [fetch(b.get_J, i) for i in range(len(grids))]
        b.close()
        return Js, {"seconds": round(secs, 4), "converged": int((states == rt3d.RT3D_MEMBER_CONVERGED).sum()),
                    "iters_max": int(iters.max()), "iters_sum": int(iters.sum()), "replays": stats["replays"],
                    "graph_ms": round(stats["solve_ms"], 2), "sweep_shape": shape,
                    "shape_ms": [round(x, 3) for x in ms.tolist()], "formal_solution": fs}

    out = {"wavelengths": n_wl, "grids": {f"{n}^3": c for n, c in sorted(sizes.items())},
           "angles": grids[0]["n_theta"] * grids[0]["n_phi"], "voxels": vox, "voxel_angles": vox_ang,
           "tol": tol, "inner_sweeps": M, "ng_order": ng[0], "ng_every": ng[1]}
    J_ref, ref = run_batch(rt3d.RT3D_FP64, ref_tol, 0)
    out["reference"] = {"tol": ref_tol, **ref}

    def err(Js):
        return max(float(torch.max(torch.abs(a / r - 1)).item()) for a, r in zip(Js, J_ref))

    for name, prec in (("batched_fp64", rt3d.RT3D_FP64), ("batched_fp32", rt3d.RT3D_FP32_SWEEP)):
        Js, res = run_batch(prec, tol, 5)
        res["max_rel_err_vs_batched_fp64_reference"] = err(Js)
        out[name] = res
    # plain float64 path, one wavelength after another
    def run_sequential(aa=0, M=M):
        singles = []
        for i, g in enumerate(grids):
            s = rt3d.Solver(g["nx"], g["ny"], g["nz"], g["n_theta"], g["n_phi"])
            s.set_medium(dm[i]["chi"], dm[i]["eps"], dm[i]["B"])
            s.autotune(cache, repeats=3)
            if aa:
                s.set_anderson(aa)
            elif ng[0]:
                s.set_acceleration(*ng)
            singles.append(s)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        its = []
        for s in singles:
            st, it, c = s.solve(tol, max_iter, M)
            its.append(it)
        torch.cuda.synchronize()
        secs = time.perf_counter() - t0
        Js = [fetch(lambda i_, J_: singles[i_].get_J(J_), i) for i in range(len(grids))]
        for s in singles:
            s.close()
        return {"seconds": round(secs, 4), "iters_max": max(its), "iters_sum": sum(its),
                "max_rel_err_vs_batched_fp64_reference": err(Js)}

    out["sequential_fp64"] = run_sequential()
    secs = out["sequential_fp64"]["seconds"]
    out["batched_fp64_speedup"] = round(secs / out["batched_fp64"]["seconds"], 3)
    out["batched_fp32_speedup"] = round(secs / out["batched_fp32"]["seconds"], 3)
    if aa_depth > 0:
        M_aa = aa_sweeps or M
        aa = {"depth": aa_depth, "inner_sweeps": M_aa}
        for name, prec in (("batched_fp64", rt3d.RT3D_FP64), ("batched_fp32", rt3d.RT3D_FP32_SWEEP)):
            Js, res = run_batch(prec, tol, 0, aa=aa_depth, M=M_aa)
            res["max_rel_err_vs_batched_fp64_reference"] = err(Js)
            res.pop("formal_solution", None)
            aa[name] = res
        aa["sequential_fp64"] = run_sequential(aa=aa_depth, M=M_aa)
        secs_aa = aa["sequential_fp64"]["seconds"]
        aa["batched_fp64_speedup"] = round(secs_aa / aa["batched_fp64"]["seconds"], 3)
        aa["batched_fp32_speedup"] = round(secs_aa / aa["batched_fp32"]["seconds"], 3)
        # against the plain float64 path with Ng (the form above)
        aa["batched_fp64_speedup_over_sequential_ng"] = round(secs / aa["batched_fp64"]["seconds"], 3)
        aa["batched_fp32_speedup_over_sequential_ng"] = round(secs / aa["batched_fp32"]["seconds"], 3)
        out["anderson"] = aa
    return out


def _adjoint(rt3d, torch, n_fd, M):
    """The differentiation form on the 65^3 x 64 workload: loss L = sum (I_em - T)^2 of the emergent
    top intensities against a seeded target.  Time of the forward solve (to 3e-13 with Ng), of the
    adjoint (rt3d_adjoint_emergent to 1e-12, Ng as for the forward solve), and agreement with central
    finite differences of the forward solve (h = 1e-6 relative on chi, absolute on eps; and 1e-4
    relative on chi, where the rounding of L matters less) on n_fd seeded voxels."""
    import numpy as np
    from paper_1107_5719_amd.inputs import WORKLOADS, emergent_target, make_medium

    w = WORKLOADS["strat65adj"]
    m = make_medium(w)
    T = emergent_target(w.n_dir // 2, w.ny, w.nx, w.seed)
    dm = {k: torch.from_numpy(v).cuda() for k, v in m.items()}
    s = rt3d.Solver(w.nx, w.ny, w.nz, w.n_theta, w.n_phi)
    s.set_acceleration(3, 6)
    s.set_medium(dm["chi"], dm["eps"], dm["B"])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st, it, c = s.solve(3e-13, 2000, M)
    torch.cuda.synchronize()
    t_fwd = time.perf_counter() - t0
    s.solve(1e-300, 100, M)             # on to the rounding floor of the iteration for the checks
    J = torch.empty_like(dm["chi"])
    s.get_J(J)
    s.formal_solution()
    I0 = s.emergent_top()
    L0 = float(np.sum((I0 - T) ** 2))
    g = 2.0 * (I0 - T)
    s.adjoint(g, tol=1e-12, max_iter=2000, inner_sweeps=M)       # warm-up (allocates)
    s.set_J(J)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    dchi, deps, st2, it2, rel = s.adjoint(g, tol=1e-12, max_iter=2000, inner_sweeps=M)
    torch.cuda.synchronize()
    t_adj = time.perf_counter() - t0
    out = {"workload": f"{w.name}: {w.nx}x{w.ny}x{w.nz} voxels x {w.n_dir} angles, eps={w.eps:g}, "
                       f"tau_total={w.tau_total:g}, target uniform [0.2, 0.8] seed {w.seed}",
           "loss": L0, "inner_sweeps": M,
           "forward_solve": {"seconds": round(t_fwd, 4), "iterations": it, "tol": 3e-13},
           "adjoint": {"seconds": round(t_adj, 4), "iterations": it2, "tol": 1e-12, "final_rel": rel},
           "adjoint_over_forward": round(t_adj / t_fwd, 3)}
    if n_fd > 0:
        rng = np.random.Generator(np.random.PCG64(55))
        vox = rng.choice(w.n_vox, n_fd, replace=False)
        ulp = float(np.spacing(L0))
        stats = {}
        for key, name, grad, hrel in (("chi", "chi", dchi, 1e-6), ("eps", "eps", deps, 1e-6),
                                      ("chi_h1e-4", "chi", dchi, 1e-4)):
            rels, informative = [], 0
            for v in vox:
                idx = np.unravel_index(v, (w.nz, w.ny, w.nx))
                h = hrel * float(dm[name][idx]) if name == "chi" else hrel
                L = []
                for sgn in (1.0, -1.0):
                    p = dm[name].clone()
                    p[idx] += sgn * h
                    if name == "chi":
                        s.set_medium(p, dm["eps"], dm["B"])
                    else:
                        s.set_medium(dm["chi"], p, dm["B"])
                    s.set_J(J)
                    s.solve(1e-300, 40, M)
                    s.formal_solution()
                    L.append(float(np.sum((s.emergent_top() - T) ** 2)))
                fd = (L[0] - L[1]) / (2 * h)
                if 32 * ulp / h < 0.1 * abs(fd):          # the difference stands above rounding of L
                    informative += 1
                    rels.append(abs(grad[idx] - fd) / abs(fd))
            stats[key] = {"voxels": int(n_fd), "informative": informative,
                           "median_rel_diff": float(np.median(rels)) if rels else None,
                           "max_rel_diff": float(np.max(rels)) if rels else None}
        out["finite_differences"] = {"h": "1e-6 relative on chi, 1e-6 absolute on eps; chi_h1e-4: 1e-4 relative",
                                     "note": "a check is informative when 32 ulp(L)/h < |fd|/10",
                                     **stats}
    s.close()
    return out


def _config_line(rt3d, torch, w, stream, steps, warmup, M, ng, max_iter):
    """One smaller workload: OS-step rate of both forms and their time to converged J (tol of the
    workload, Lambda* included), with the error against the oracle's stored solution."""
    from paper_1107_5719_amd.inputs import make_medium

    med = make_medium(w)
    d_med = {k: torch.from_numpy(v).cuda() for k, v in med.items()}
    J_orc, meta = oracle_reference(w, med)
    J_orc = None if J_orc is None else torch.from_numpy(J_orc).cuda()
    row = {"workload": f"{w.name}: {w.nx}x{w.ny}x{w.nz} voxels x {w.n_dir} angles, eps={w.eps:g}, "
                       f"tau_total={w.tau_total:g}, noise {w.noise} sigma={w.sigma}, seed {w.seed}",
           "tol": w.tol, "inner_sweeps": M, "ng_order": ng[0], "ng_every": ng[1], "oracle_reference": meta}
    for form, prec in (("fp64", rt3d.RT3D_FP64), ("fp32", rt3d.RT3D_FP32_SWEEP)):
        elapsed, per_launch, lstar_s, st = _timed_steps(rt3d, torch, w, d_med, prec, stream, steps, warmup, M)
        J, conv = _converge(rt3d, torch, w, d_med, prec, stream, M, ng[0], ng[1], w.tol, max_iter)
        if J_orc is not None:
            conv["max_rel_err_vs_oracle"] = _rel_err(J, J_orc)
        row[form] = {"ms_per_step": round(1e3 * elapsed / steps, 4),
                     "voxel_angle_updates_per_s": w.n_vox * w.n_dir * steps / elapsed,
                     "kernel_ms_per_launch": {k: (round(v, 4) if v is not None else None)
                                              for k, v in per_launch.items()},
                     "time_to_converged": conv}
    row["fp32_form_speedup"] = round(row["fp64"]["time_to_converged"]["seconds"] /
                                     row["fp32"]["time_to_converged"]["seconds"], 3)
    return row


def _paper_grids(rt3d, torch, stream, steps, M, ng, max_iter):
    """The paper's slab on its two timing grids (65^3 and 129^2 x 193, 256 angles): OS-step rate and
    time to converged J (tol 1e-8, Lambda* included), both forms, with the error against the oracle's
    tightly converged J when one is stored."""
    from paper_1107_5719_amd.inputs import WORKLOADS, make_medium

    out = {}
    for name in ("slab65", "slab193"):
        w = WORKLOADS[name]
        med = make_medium(w)
        d_med = {k: torch.from_numpy(v).cuda() for k, v in med.items()}
        row = {"grid": f"{w.nx}x{w.ny}x{w.nz} x {w.n_dir} angles"}
        J_orc, orc_meta = oracle_reference(w, med)
        row["oracle_reference"] = orc_meta
        J_orc = None if J_orc is None else torch.from_numpy(J_orc).cuda()
        for form, prec in (("fp64", rt3d.RT3D_FP64), ("fp32", rt3d.RT3D_FP32_SWEEP)):
            elapsed, per_launch, lstar_s, st = _timed_steps(rt3d, torch, w, d_med, prec, stream, steps, 1, M)
            conv = None
            if max_iter > 0:
                J, conv = _converge(rt3d, torch, w, d_med, prec, stream, M, ng[0], ng[1], w.tol, max_iter)
                if J_orc is not None:
                    conv["max_rel_err_vs_oracle"] = _rel_err(J, J_orc)
            row[form] = {"ms_per_step": round(1e3 * elapsed / steps, 3),
                         "voxel_angle_updates_per_s": w.n_vox * w.n_dir * steps / elapsed,
                         "sweep_ms": per_launch["sweep"], "time_to_converged": conv}
        out[name] = row
        del d_med
    return out


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="strat129")
    ap.add_argument("--precision", choices=["fp64", "fp32"], default="fp64",
                    help="form whose step rate is the headline value")
    ap.add_argument("--inner-sweeps", type=int, default=30, help="Jacobi sweeps per OS step (M)")
    ap.add_argument("--ng-order", type=int, default=3)
    ap.add_argument("--ng-every", type=int, default=6)
    ap.add_argument("--gs-inner-sweeps", type=int, default=15,
                    help="Gauss-Seidel sweeps per OS step for its time to converged J (0: skip)")
    ap.add_argument("--converge-max-iter", type=int, default=600,
                    help="outer-iteration cap of the time-to-converged-J runs (0 skips them)")
    ap.add_argument("--reference-tol", type=float, default=1e-12,
                    help="tolerance of the float64 reference solve the converged forms are measured against")
    ap.add_argument("--batch-wavelengths", type=int, default=64,
                    help="wavelengths of the batched-form measurement (0 skips it)")
    ap.add_argument("--batch-inner-sweeps", type=int, default=8)
    ap.add_argument("--batch-anderson-depth", type=int, default=8,
                    help="also time the batched and one-at-a-time forms with Anderson mixing of this depth (0 skips)")
    ap.add_argument("--batch-anderson-sweeps", type=int, default=4,
                    help="inner sweeps of the Anderson-mixing runs of the batched measurement")
    ap.add_argument("--adjoint-fd-voxels", type=int, default=50,
                    help="finite-difference checks of the adjoint at 65^3 x 64 (0 skips them; -1 skips "
                         "the adjoint measurement)")
    ap.add_argument("--configs", type=int, default=1,
                    help="also measure the 17^3 x 64 and 65^3 x 256 workloads (0 skips)")
    ap.add_argument("--paper-grids", type=int, default=1,
                    help="also measure the paper's slab on its 65^3 and 129^2 x 193 grids (0 skips)")
    ap.add_argument("--tune-cache", default=None,
                    help="JSON cache of the sweep-shape autotuner (default: a file in the temp directory)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-every", type=int, default=4,
                    help="the CPU oracle times every n-th direction of the full grid")
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="only run a plain elementwise copy of this many MiB (3 times) and exit: the "
                         "reference for scaling HBM byte counters")
    args = ap.parse_args()
    if args.calibrate_copy_mib > 0:
        import torch

        n = args.calibrate_copy_mib * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.mul(src, 1.0, out=dst)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n, "launches": 3}), flush=True)
        return 0

    if args.gpus != 1:
        print(f"bench.py: the library runs on one GPU only (asked for --gpus {args.gpus}); the path "
              "would shard over directions with one all-reduce of J_fs per iteration, which is not "
              "implemented.", file=sys.stderr)
        return 2
    if int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: launched with WORLD_SIZE > 1; one GPU only", file=sys.stderr)
        return 2

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
    stream = torch.cuda.current_stream().cuda_stream
    forms = {"fp64": rt3d.RT3D_FP64, "fp32": rt3d.RT3D_FP32_SWEEP}
    M = args.inner_sweeps

    # ---- timed steps, both forms ----------------------------------------------------------------
    step = {}
    for name, prec in forms.items():
        elapsed, per_launch, lstar_s, st = _timed_steps(rt3d, torch, w, d_med, prec, stream, args.steps,
                                                        args.warmup, M)
        fs_ms = sum(per_launch[k] for k in ("source", "sweep", "reduce"))
        step[name] = {"ms_per_step": 1e3 * elapsed / args.steps,
                      "value": V * n_dir * args.steps / elapsed,
                      "fs_updates_per_s_fs_kernels_only": V * n_dir / (fs_ms * 1e-3),
                      "kernel_ms_per_launch": {k: (round(v, 4) if v is not None else None)
                                               for k, v in per_launch.items()},
                      "lstar_build_s": round(lstar_s, 4),
                      "sweeps": {"fp64": st["fp64_sweeps"], "fp32": st["fp32_sweeps"]}}
    main_form = args.precision
    upd = V * n_dir

    def sweep_roofline(form):
        """The sweep against HBM with the algorithmic bytes (2 s_r + 16)/G per voxel-angle update at
        G = SWEEP_G, from its average launch time in the timed steps (HIP events on the context
        stream)."""
        sweep_ms = step[form]["kernel_ms_per_launch"]["sweep"]
        upd_per_s = upd / (sweep_ms * 1e-3)
        b_unit = sweep_bytes_per_update(form)
        gbs = b_unit * upd_per_s / 1e9
        traffic = measured_traffic(SWEEP_KERNEL[form])
        valu = measured_valu(SWEEP_KERNEL[form])
        r = {"kernel": SWEEP_KERNEL[form], "bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS,
             "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": traffic,
             "G": SWEEP_G, "bytes_per_update": b_unit, "updates_per_launch": upd, "ms_per_launch": sweep_ms}
        # beside it: the measured HBM traffic (rocprofv3 FETCH_SIZE + WRITE_SIZE per launch) over the same
        # duration, and the vector issue (rocprofv3 SQ_INSTS_VALU x 64 lanes per update) against the
        # chip's issue rate for the sweep's precision
        r["counter_view"] = None if traffic is None else {
            "achieved": round(traffic / (sweep_ms * 1e-3) / 1e9, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(traffic / (sweep_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "bytes_per_update": round(traffic / upd, 2)}
        r["alu_view"] = None if valu is None else {
            "achieved": round(64 * valu / (sweep_ms * 1e-3) / 1e12, 2), "peak": VALU_ISSUE_PEAK[form] / 1e12,
            "unit": "T lane-instructions/s", "frac": round(64 * valu / (sweep_ms * 1e-3) / VALU_ISSUE_PEAK[form], 4),
            "lane_instructions_per_update": round(64 * valu / upd, 1)}
        return r

    roofline = sweep_roofline(main_form)
    roofline_other = sweep_roofline("fp32" if main_form == "fp64" else "fp64")
    roofline_jacobi = {}
    for form, coef in (("fp64", "fp64"), ("fp32", "fp32")):
        jac_ms = step[form]["kernel_ms_per_launch"]["jacobi"]
        jac_gbs = jacobi_bytes_per_voxel(coef) * V / (jac_ms * 1e-3) / 1e9
        traffic = measured_traffic(JACOBI_KERNEL[form])
        roofline_jacobi[form] = {
            "kernel": JACOBI_KERNEL[form], "bound": "hbm", "achieved": round(jac_gbs, 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(jac_gbs / HBM_PEAK_GBS, 4), "traffic": traffic,
            "traffic_over_algorithmic": None if traffic is None else round(traffic / (jacobi_bytes_per_voxel(coef) * V), 3),
            "bytes_per_voxel": jacobi_bytes_per_voxel(coef), "coef_storage": coef, "ms_per_launch": jac_ms,
            "os_solve_ms": round(M * jac_ms, 3)}

    # ---- time to converged J, both forms, against the oracle's tightly converged J ---------------------
    J_orc, orc_meta = oracle_reference(w, med)
    J_orc = None if J_orc is None else torch.from_numpy(J_orc).to(dev)
    conv = None
    if args.converge_max_iter > 0:
        conv = {"tol": w.tol, "inner_sweeps": M, "ng_order": args.ng_order, "ng_every": args.ng_every,
                "oracle_reference": orc_meta}
        J_gref = None
        if J_orc is None:
            # no stored oracle solution: a float64 GPU solve to reference_tol (Anderson mixing, depth 8)
            # stands in as the reference
            J_gref, ref = _converge(rt3d, torch, w, d_med, rt3d.RT3D_FP64, stream, M, 0, 0,
                                    args.reference_tol, 20 * args.converge_max_iter, anderson=8)
            conv["gpu_fp64_reference"] = {"tol": args.reference_tol, **ref}

        def errs(J):
            if J_orc is not None:
                return {"max_rel_err_vs_oracle": _rel_err(J, J_orc)}
            return {"max_rel_err_vs_gpu_fp64_reference": _rel_err(J, J_gref)}

        for name, prec in forms.items():
            J, res = _converge(rt3d, torch, w, d_med, prec, stream, M, args.ng_order, args.ng_every, w.tol,
                               args.converge_max_iter)
            conv[name] = {**res, **errs(J)}
        conv["fp32_form_speedup"] = round(conv["fp64"]["seconds"] / conv["fp32"]["seconds"], 3)
        # sweep precision x coefficient storage, each at the schedule above: the float32-sweep effect
        # with equal coefficient storage
        grid = {}
        for sname, prec in forms.items():
            for cname, coef in (("fp64", rt3d.RT3D_COEF_FP64), ("fp32", rt3d.RT3D_COEF_FP32)):
                J, res = _converge(rt3d, torch, w, d_med, prec, stream, M, args.ng_order, args.ng_every, w.tol,
                                   args.converge_max_iter, coef=coef)
                grid[f"sweeps_{sname}_coef_{cname}"] = {**res, **errs(J)}
        for cname in ("fp64", "fp32"):
            grid[f"fp32_sweep_speedup_coef_{cname}"] = round(
                grid[f"sweeps_fp64_coef_{cname}"]["seconds"] / grid[f"sweeps_fp32_coef_{cname}"]["seconds"], 3)
        conv["precision_grid"] = grid
        # a fixed set of schedules (M x Ng every), so that the forms' comparison does not rest on one
        # sharp optimum of the outer step count
        import statistics

        sched = {"schedules": [list(x) for x in SCHEDULES]}
        for name, prec in forms.items():
            rows = []
            for (m_, o_, e_) in SCHEDULES:
                J, res = _converge(rt3d, torch, w, d_med, prec, stream, m_, o_, e_, w.tol, args.converge_max_iter)
                rows.append({"inner_sweeps": m_, "ng_order": o_, "ng_every": e_, "seconds": res["seconds"],
                             "outer_iterations": res["outer_iterations"], "converged": res["converged"],
                             **errs(J)})
            secs = [r["seconds"] for r in rows]
            sched[name] = {"runs": rows, "median_s": statistics.median(secs), "worst_s": max(secs),
                           "best_s": min(secs)}
        sched["fp32_form_speedup_median"] = round(sched["fp64"]["median_s"] / sched["fp32"]["median_s"], 3)
        sched["fp32_form_speedup_worst"] = round(sched["fp64"]["worst_s"] / sched["fp32"]["worst_s"], 3)
        conv["schedules"] = sched
        # Anderson mixing of the outer iteration instead of Ng (window depth x inner sweeps M)
        aa = {"schedules": [list(x) for x in AA_SCHEDULES]}
        for name, prec in forms.items():
            rows = []
            for (m_, dep) in AA_SCHEDULES:
                J, res = _converge(rt3d, torch, w, d_med, prec, stream, m_, 0, 0, w.tol, args.converge_max_iter,
                                   anderson=dep)
                rows.append({"inner_sweeps": m_, "depth": dep, "seconds": res["seconds"],
                             "outer_iterations": res["outer_iterations"], "converged": res["converged"],
                             **errs(J)})
            secs = [r["seconds"] for r in rows]
            aa[name] = {"runs": rows, "median_s": statistics.median(secs), "worst_s": max(secs),
                        "best_s": min(secs)}
        aa["fp32_form_speedup_median"] = round(aa["fp64"]["median_s"] / aa["fp32"]["median_s"], 3)
        for name in forms:
            aa[f"{name}_speedup_over_ng_median"] = round(sched[name]["median_s"] / aa[name]["median_s"], 3)
            aa[f"{name}_speedup_over_ng_worst"] = round(sched[name]["worst_s"] / aa[name]["worst_s"], 3)
        conv["anderson"] = aa
        # headline: the median over each acceleration's fixed schedule set (no single tuned schedule)
        conv["headline"] = {
            "method": "median time to converged J over the fixed schedule sets (Anderson mixing: depth 5 and 8 x "
                      "M = 12, 20, 30; Ng order 3 every 6 or 8 steps x M = 12, 20, 30, 40), Lambda* build included",
            "anderson_fp64_s": aa["fp64"]["median_s"], "anderson_fp32_s": aa["fp32"]["median_s"],
            "ng_fp64_s": sched["fp64"]["median_s"], "ng_fp32_s": sched["fp32"]["median_s"],
            "fp32_form_speedup_anderson": aa["fp32_form_speedup_median"],
            "fp32_form_speedup_ng": sched["fp32_form_speedup_median"]}
        # the Fortran code's other inner solve: multicolour Gauss-Seidel, float64, half the sweeps
        if args.gs_inner_sweeps > 0:
            J, res = _converge(rt3d, torch, w, d_med, rt3d.RT3D_FP64, stream, args.gs_inner_sweeps,
                               args.ng_order, args.ng_every, w.tol, args.converge_max_iter,
                               os_method=rt3d.RT3D_OS_GAUSS_SEIDEL)
            conv["gauss_seidel_fp64"] = {"inner_sweeps": args.gs_inner_sweeps, **res, **errs(J)}
        # equal accuracy: the time each form needs to come within 1e-5 and within 1e-8 of the oracle (of
        # the GPU reference when no oracle solution is stored), stopping at c < target / 100
        conv["accuracy_targets"] = {}
        for target in (1e-5, 1e-8):
            row = {"stop_tol": target / 100}
            for name, prec in forms.items():
                J, res = _converge(rt3d, torch, w, d_med, prec, stream, M, args.ng_order, args.ng_every,
                                   target / 100, 20 * args.converge_max_iter)
                e = errs(J)
                err = e.get("max_rel_err_vs_oracle", e.get("max_rel_err_vs_gpu_fp64_reference"))
                row[name] = {"seconds": res["seconds"], "outer_iterations": res["outer_iterations"], **e,
                             "within_target": err <= target}
            row["fp32_form_speedup"] = round(row["fp64"]["seconds"] / row["fp32"]["seconds"], 3)
            conv["accuracy_targets"][f"{target:g}"] = row

    # ---- the smaller benchmark configurations: 17^3 x 64 (eps 1e-2) and 65^3 x 256 (GRF, eps 1e-4) ------
    configs = None
    if args.configs:
        configs = {}
        for cname in ("strat17", "grf65"):
            configs[cname] = _config_line(rt3d, torch, WORKLOADS[cname], stream, args.steps, args.warmup, M,
                                          (args.ng_order, args.ng_every), args.converge_max_iter)

    # ---- many wavelengths on uneven grids: batched forms against one-at-a-time ------------------------
    batched = None
    if args.batch_wavelengths > 0:
        import tempfile

        cache = args.tune_cache or os.path.join(tempfile.gettempdir(), "rt3d_tune.json")
        batched = _batched(rt3d, torch, args.batch_wavelengths, args.batch_inner_sweeps,
                           (args.ng_order, args.ng_every), w.tol, args.reference_tol, 3000, cache,
                           aa_depth=args.batch_anderson_depth, aa_sweeps=args.batch_anderson_sweeps)

    # ---- the paper's slab on the paper's grids ------------------------------------------------------
    paper_grids = None
    if args.paper_grids:
        paper_grids = _paper_grids(rt3d, torch, stream, 3, M, (args.ng_order, args.ng_every),
                                   args.converge_max_iter)

    # ---- gradients through the converged solution (adjoint) ----------------------------------------
    adjoint = None
    if args.adjoint_fd_voxels >= 0:
        adjoint = _adjoint(rt3d, torch, args.adjoint_fd_voxels, 30)

    # ---- CPU oracle on a bounded sample of the same workload -------------------------------------
    cpu = None
    if not args.no_cpu_baseline:
        import tempfile

        import oracle

        # the oracle as it stands, compiled here with the baseline's flags (gcc -O3 -march=native)
        try:
            oracle.use_library(oracle.build_native(tempfile.mkdtemp(prefix="rt3d_oracle_")))
            build_flags = "gcc -O3 -march=native -fopenmp"
        except Exception as e:            # no compiler on this host: the in-tree build
            oracle.use_library(None)
            build_flags = f"gcc -O2 -fopenmp (in-tree build; native build failed: {e})"
        threads = min(os.cpu_count() or 1, 16)
        dirs = list(range(0, n_dir, args.cpu_sample_every))
        S = med["eps"] * med["B"] + (1 - med["eps"]) * med["B"]
        t0 = time.perf_counter()
        oracle.formal_solution_dirs(med["chi"], S, w.n_theta, w.n_phi, dirs, I_top=w.I_top,
                                    I_bot=med["B"][0], n_threads=threads)
        tcpu = time.perf_counter() - t0
        cpu = {"value": V * len(dirs) / tcpu, "unit": "voxel-angle FS updates/s",
               "cores": min(threads, len(dirs)), "kind": "oracle",
               "sample": f"FP64 oracle formal solution of {len(dirs)} of the {n_dir} directions "
                         f"(every {args.cpu_sample_every}th) on the full {w.nx}x{w.ny}x{w.nz} grid, "
                         f"{tcpu:.2f} s wall"}
        # one thread (the serial analogue), on a smaller share of the directions
        dirs1 = list(range(0, n_dir, 8 * args.cpu_sample_every))
        t0 = time.perf_counter()
        oracle.formal_solution_dirs(med["chi"], S, w.n_theta, w.n_phi, dirs1, I_top=w.I_top,
                                    I_bot=med["B"][0], n_threads=1)
        t1 = time.perf_counter() - t0
        cpu["single_thread"] = {"value": V * len(dirs1) / t1, "cores": 1,
                                "sample": f"{len(dirs1)} directions (every {8 * args.cpu_sample_every}th), "
                                          f"{t1:.2f} s wall"}
        cpu["host_cpu"] = _cpu_model()
        cpu["build"] = build_flags

    out = {
        "metric": METRIC,
        "value": step[main_form]["value"],
        "unit": "voxel-angle FS updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": step[main_form]["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if main_form == "fp64" else "f32",
        "data": "synthetic",
        "config": {"workload": f"{w.name}: {w.nx}x{w.ny}x{w.nz} voxels x {n_dir} angles "
                               f"({w.n_theta} mu x {w.n_phi} phi), eps={w.eps:g}, tau_total={w.tau_total:g}, "
                               f"chi log-normal sigma={w.sigma}, seed {w.seed}",
                   "precision": "fp64" if main_form == "fp64" else "fp32 sweeps, fp64 J/OS/convergence",
                   "inner_sweeps": M,
                   "step": "one OS iteration: S update, FS over all angles, J reduction + residual, "
                           "M Jacobi sweeps, J update + max rel dJ"},
        "forms": step,
        "roofline": roofline,
        "roofline_other_form": roofline_other,
        "roofline_jacobi": roofline_jacobi,
        "cpu_baseline": cpu,
        "time_to_converged": conv,
        "configs": configs,
        "batched": batched,
        "adjoint": adjoint,
        "paper_grids": paper_grids,
    }
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
