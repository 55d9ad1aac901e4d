"""Benchmark: P2 Taylor-Green vortex, 128^3 cells, one S2O4 step of the DG
gas-kinetic scheme per timed step, on one MI355X.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--no-fp64] [--no-adjoint]

Prints one JSON line.  `value` is the FP32-bulk path's throughput in
DOF-updates/s (5 variables x 10 modes x 128^3 cells per step / seconds per
step); the FP64 path, the FP32-vs-FP64 relative L2 difference, the
adjoint/forward time ratio, a roofline entry for the dominant kernel (from
HIP events recorded by the library on its stream) and the FP64 CPU oracle
timed on a bounded sample (cpu_baseline) are reported beside it.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

# Algorithmic work per unit, from paper_2202_13821_amd/csrc/flopcount (see
# the package's flops.json): floating-point operations per face point and per
# volume point of each stage, for the kernels' own formulas.
FLOPS_JSON = os.path.join(ROOT, "paper_2202_13821_amd", "flops.json")

# Published MI355X peaks.  The FP32 vector peak is 256 CUs x 4 SIMDs x 32 FMA
# lanes x 2 flop x 2.4 GHz; on gfx950 FP32 instructions with VGPR operands
# issue in under 3 cycles per wavefront without packed-FP32 instructions.
MI355X_PEAK = {"fp32_vector": 157.3, "fp64_vector": 78.6, "hbm_GBs": 8000.0}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=128, help="cells per axis")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-rules", action="store_true",
                    help="skip the other compiled (degree, Gauss points) rules: P2 with 2 points, P3 with 3 and 4")
    ap.add_argument("--no-parity", action="store_true",
                    help="skip the comparison with the stored oracle reference of the 128^3 workload")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--adjoint-only", action="store_true",
                    help="profiling aid: run only the adjoint/forward timing (32^3) and print it")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one plain 1 GiB device copy (reference kernel for HBM counters)")
    return ap.parse_args()


def load_flops():
    if os.path.exists(FLOPS_JSON):
        with open(FLOPS_JSON) as f:
            return json.load(f)
    return None


def time_path(precision, n, steps, warmup, timing=True, k=2, nq=0, mapped=False, reps=3):
    """Seconds per step of `precision` on the n^3 Taylor-Green workload: the
    median of `reps` wall-clock repetitions of `steps` steps (inputs resident
    in HBM, torch.cuda.synchronize() on both sides, no event recording), then
    one more repetition with the library's per-launch HIP events on its
    stream (kernel averages).  Returns (median s/step, all repetitions, kernel
    timing, final state, solver, initial state); the state has had
    warmup + (reps + 1) * steps steps."""
    import numpy as np
    import torch

    from paper_2202_13821_amd import Solver, problems

    widths = np.tile(problems.mapped_widths(n, -np.pi, np.pi), 3) if mapped else None
    q0, lo, hi = problems.tgv((n, n, n), k, widths=widths)
    # P3 runs at a smaller CFL number (the DG limit falls like 1 / (2k + 1));
    # the mapped mesh's smallest cell is 0.75 of the uniform width
    dt = problems.tgv_dt(n, cfl=0.15 if k < 3 else 0.08) * (0.75 if mapped else 1.0)
    s = Solver((n, n, n), lo, hi, k, nq=nq, mu=1.0 / 1600.0, prandtl=0.72, precision=precision,
               device="cuda:0", widths=widths)
    q = torch.as_tensor(q0, device="cuda:0")
    s.step(q, dt, warmup)
    s.check()
    walls = []
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.step(q, dt, steps)
        torch.cuda.synchronize()
        walls.append((time.perf_counter() - t0) / steps)
    kern = None
    if timing:
        s.set_timing(True)
        s.step(q, dt, steps)
        kern = s.get_timing()
        s.set_timing(False)
    s.check()
    return float(np.median(walls)), walls, kern, q, s, q0


def adjoint_ratio(precision, n=32, nsteps=200, stride=15, k=2, nq=0):
    """adj/fwd on a Taylor-Green run (default: the P2 32^3, 200-step adjoint
    configuration): wall time of the gradient call (segment recomputation +
    reverse sweep) over that of the checkpointing forward call."""
    import torch

    from paper_2202_13821_amd import Solver, kinetic_energy, problems

    q0, lo, hi = problems.tgv((n, n, n), k)
    dt = problems.tgv_dt(n, cfl=0.15 if k < 3 else 0.08)
    s = Solver((n, n, n), lo, hi, k, nq=nq, mu=1.0 / 1600.0, prandtl=0.72, precision=precision, device="cuda:0",
               max_stride=stride)
    ck = s.new_checkpoints(nsteps, stride)
    q = torch.as_tensor(q0, device="cuda:0")
    # warm-up of both paths
    s.step(q.clone(), dt, 2, ck, stride)
    qq = q.clone().requires_grad_(True)
    (g,) = torch.autograd.grad(kinetic_energy(qq, s), qq)
    s.adjoint(ck, stride, dt, 2, g.contiguous())
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    qN = q.clone()
    s.step(qN, dt, nsteps, ck, stride)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    qq = qN.clone().requires_grad_(True)
    (g,) = torch.autograd.grad(kinetic_energy(qq, s), qq)
    g = g.contiguous()
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    s.adjoint(ck, stride, dt, nsteps, g)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    out = {"fwd_s": t1 - t0, "adj_s": t3 - t2, "adj_over_fwd": (t3 - t2) / (t1 - t0),
           "workload": f"P{k} TGV {n}^3{'' if not nq else f', {nq} Gauss points'}, {nsteps} steps, "
                       f"checkpoint stride {stride}"}
    # per-launch averages of the adjoint kernels from a separate, event-timed
    # call (outside the timed pair above), against their algorithmic flops
    s.set_timing(True)
    s.adjoint(ck, stride, dt, nsteps, g)
    kern = s.get_timing()
    s.set_timing(False)
    flops = load_flops()
    nqq = nq or k + 1
    tag = "fp64" if precision == "fp64" else "fp32"
    fr = (flops or {}).get("rules", {}).get(f"p{k}_nq{nqq}", {}).get(f"adjoint_{tag}")
    if fr:
        peak = MI355X_PEAK["fp64_vector" if precision == "fp64" else "fp32_vector"]
        rl = {"bound": "alu", "unit": "TFLOP/s", "peak": peak}
        for kern_name, key, pts in (("adj_face", "face", 3 * nqq * nqq), ("adj_volume", "volume", nqq ** 3)):
            ms, cnt = kern[kern_name]
            if not cnt:
                continue
            # launches alternate adjoint stage 2 and stage 1: average work per launch
            w = 0.5 * (fr[f"{key}_stage1"] + fr[f"{key}_stage2"]) * pts * n ** 3
            ach = w / (ms / cnt * 1e-3) / 1e12
            rl[kern_name] = {"achieved": ach, "frac": ach / peak, "avg_launch_ms": ms / cnt,
                             "flops_per_point": 0.5 * (fr[f"{key}_stage1"] + fr[f"{key}_stage2"])}
        out["roofline"] = rl
    return out


def parity_vs_oracle():
    """Both GPU paths from the initial state through the checkpoints of the
    stored FP64 oracle reference of this workload (tests/golden/oracle_c4.json,
    written by tests/golden/make_golden.py): relative L2 over its 64 sampled
    cells of the state and of the change since t = 0, per (rho, momentum,
    rho E), at its last checkpoint."""
    import numpy as np
    import torch

    from paper_2202_13821_amd import Solver, problems

    path = os.path.join(ROOT, "tests", "golden", "oracle_c4.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        g = json.load(f)
    if not g.get("checkpoints"):
        return None
    cp = g["checkpoints"][-1]
    n = g["shape"][0]
    q0, lo, hi = problems.tgv((n, n, n), 2)
    cells = np.array(g["cells"])
    ref, ref0 = np.array(cp["coeffs"]), np.array(g["coeffs0"])
    out = {"steps": cp["steps"], "sampled_cells": len(cells), "reference": "tests/golden/oracle_c4.json"}
    for prec in ("fp64", "fp32_bulk"):
        s = Solver((n, n, n), lo, hi, 2, mu=g["mu"], prandtl=g["prandtl"], precision=prec, device="cuda:0")
        q = torch.as_tensor(q0, device="cuda:0")
        s.step(q, g["dt"], cp["steps"])
        s.check()
        qf = q.cpu().numpy().reshape(5, 10, -1)
        samp = np.transpose(qf[:, :, cells], (2, 0, 1))
        s0 = np.transpose(q0.reshape(5, 10, -1)[:, :, cells], (2, 0, 1))
        st, inc = {}, {}
        for name, idx in (("rho", [0]), ("momentum", [1, 2, 3]), ("rhoE", [4])):
            st[name] = float(np.linalg.norm(samp[:, idx] - ref[:, idx]) / np.linalg.norm(ref[:, idx]))
            di = (samp[:, idx] - s0[:, idx]) - (ref[:, idx] - ref0[:, idx])
            inc[name] = float(np.linalg.norm(di) / np.linalg.norm(ref[:, idx] - ref0[:, idx]))
        out[prec] = {"rel_l2_state": st, "rel_l2_increment": inc}
        del s, q
    return out


def kernel_source_hash():
    from paper_2202_13821_amd.profiling import kernel_source_hash as h

    return h()


def measured_traffic(kernel_key):
    """HBM bytes per launch of a kernel from the committed rocprofv3 counter
    summary, or None if there is none or the kernel sources changed since."""
    path = os.path.join(ROOT, "profiles", "hbm_traffic_tgv128.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    if d.get("source_hash") != kernel_source_hash():
        return None
    return d.get("kernels", {}).get(kernel_key, {}).get("bytes_per_launch")


def cpu_baseline(n, seconds):
    """FP64 oracle operator on whole z-slabs of the same 128^3 Taylor-Green
    state (each face of the slab computed once), two evaluations per step."""
    import oracle as O
    from paper_2202_13821_amd import problems

    q0, lo, hi = problems.tgv((n, n, n), 2)
    c = O.make_cfg((n, n, n), 2, lo=lo, hi=hi, mu=1 / 1600, prandtl=0.72)
    dt = problems.tgv_dt(n)
    k1 = 1
    t0 = time.perf_counter()
    O.residual_slab(c, q0, dt, 0, k1)
    el = time.perf_counter() - t0
    # grow the slab until the sample is long enough
    if el < seconds:
        k1 = max(1, min(n, int(k1 * seconds / max(el, 1e-3))))
        t0 = time.perf_counter()
        O.residual_slab(c, q0, dt, 0, k1)
        el = time.perf_counter() - t0
    cells = n * n * k1
    per_step = 2.0 * el / cells  # seconds per cell per step
    return {"value": 50.0 / per_step, "unit": "DOF-updates/s", "cores": O.num_threads(), "kind": "oracle",
            "sample": f"oracle L and L_t on z-slab of {k1} x {n}^2 cells of the {n}^3 P2 TGV state "
                      f"({el:.1f} s), x2 evaluations per step"}


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {a.gpus}); the multi-GPU path (a domain "
              "decomposition with one halo exchange per stage) is designed but not built", file=sys.stderr)
        sys.exit(2)
    import torch

    if a.adjoint_only:
        print(json.dumps({"adjoint": {"fp32_bulk": adjoint_ratio("fp32_bulk"), "fp64": adjoint_ratio("fp64"),
                                      "fp32_bulk_128": adjoint_ratio("fp32_bulk", n=a.n, nsteps=6, stride=3),
                                      "p3_fp32_bulk": adjoint_ratio("fp32_bulk", nsteps=50, stride=7, k=3),
                                      "p3_fp64": adjoint_ratio("fp64", nsteps=50, stride=7, k=3)}}),
              flush=True)
        return
    n = a.n
    dof = 5 * 10 * n ** 3
    out = {"metric": "P2 TGV 128^3 DOF-updates/s, FP32-bulk vs FP64 at stated L2 error; adj/fwd",
           "unit": "DOF-updates/s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
           "data": "synthetic (analytic Taylor-Green initial data, L2-projected)",
           "config": {"workload": f"DG-HGKS P2 Taylor-Green vortex {n}^3 cells, 3x3x3 volume / 3x3 face "
                                  "Gauss points, Re 1600, Ma 0.1, Pr 0.72, CFL 0.15, FP32-bulk flux and "
                                  "projection with FP64 stage accumulation",
                      "cells": n ** 3, "modes": 10, "dof_per_step": dof}}
    sec32, walls32, k32, q32, s32, q0 = time_path("fp32_bulk", n, a.steps, a.warmup)
    out["value"] = dof / sec32
    out["dof_updates_per_variable_per_s"] = dof / 5 / sec32
    out["ms_per_step"] = 1e3 * sec32
    out["timing"] = {"method": "median of 3 wall-clock repetitions of `steps` steps (synchronize on both sides, "
                               "no event recording); kernel averages from a 4th, event-timed repetition",
                     "ms_per_step_reps": [1e3 * w for w in walls32]}
    out["kernels_ms_per_launch"] = {k: (v[0] / v[1] if v[1] else None) for k, v in k32.items()}
    flops = load_flops()
    face_ms = k32["face"][0] / max(k32["face"][1], 1)
    vol_ms = k32["volume"][0] / max(k32["volume"][1], 1)
    out["kernels_ms_per_step"] = {"face": 2 * face_ms, "volume": 2 * vol_ms}
    if flops:
        # face launches alternate stage 1 (F and Ft) / stage 2 (Ft only): average work per launch
        npts_face = 3 * n ** 3 * 9
        w = 0.5 * (flops["fp32"]["face_stage1"] + flops["fp32"]["face_stage2"]) * npts_face
        achieved = w / (face_ms * 1e-3) / 1e12
        out["roofline"] = {"bound": "alu", "kernel": "face_kernel<float,2,3> (both stages, averaged per launch)",
                           "achieved": achieved, "peak": MI355X_PEAK["fp32_vector"], "unit": "TFLOP/s",
                           "frac": achieved / MI355X_PEAK["fp32_vector"],
                           "traffic": measured_traffic("face_kernel<float,2,3>"),
                           "flops_per_launch": w, "avg_launch_ms": face_ms,
                           "flops_per_point": 0.5 * (flops["fp32"]["face_stage1"] + flops["fp32"]["face_stage2"])}
        wv = 0.5 * (flops["fp32"]["volume_stage1"] + flops["fp32"]["volume_stage2"]) * 27 * n ** 3
        vt = measured_traffic("volume_kernel<float,2,3>")
        # the stage updates fused into the volume kernel stream Q^n, Q*, P and
        # Q^{n+1}: 40 B per DOF-update per step in FP32-bulk, 20 B per launch
        alg_bytes = 20.0 * dof
        # what the face/volume split moves per launch if every operand crosses
        # HBM once: the float coefficients, each of the cell's three face
        # records once (5 x 6 tangential modes; F and Ft in stage 1, Ft in
        # stage 2), and the FP64 stage update with the float copy it writes
        nm, nt = 10, 6
        cell1 = 5 * nm * 4 + 5 * nm * 8 + 3 * 5 * 2 * nt * 4 + 5 * nm * 4 + 5 * nm * 8
        cell2 = 5 * nm * 4 + 5 * nm * 8 + 3 * 5 * nt * 4 + 5 * nm * 8 + 5 * nm * 4
        design_bytes = 0.5 * (cell1 + cell2) * n ** 3
        out["roofline_volume"] = {"bound": "alu", "achieved": wv / (vol_ms * 1e-3) / 1e12,
                                  "peak": MI355X_PEAK["fp32_vector"], "unit": "TFLOP/s",
                                  "frac": wv / (vol_ms * 1e-3) / 1e12 / MI355X_PEAK["fp32_vector"],
                                  "traffic": vt,
                                  "hbm": {"algorithmic_bytes_per_launch": alg_bytes,
                                          "algorithmic_GBs": alg_bytes / (vol_ms * 1e-3) / 1e9,
                                          "design_bytes_per_launch": design_bytes,
                                          "design_GBs": design_bytes / (vol_ms * 1e-3) / 1e9,
                                          "measured_GBs": (vt / (vol_ms * 1e-3) / 1e9) if vt else None,
                                          "measured_over_design": (vt / design_bytes) if vt else None,
                                          "peak_GBs": MI355X_PEAK["hbm_GBs"]}}
        per_step = flops["per_step_per_cell"]["fp32"] * n ** 3
        out["step_flops"] = per_step
        out["step_tflops"] = per_step / sec32 / 1e12
    if not a.no_fp64:
        del s32
        sec64, walls64, k64, q64, s64, _ = time_path("fp64", n, a.steps, a.warmup)
        out["fp64"] = {"value": dof / sec64, "ms_per_step": 1e3 * sec64, "ms_per_step_reps": [1e3 * w for w in walls64],
                       "kernels_ms_per_launch": {k: (v[0] / v[1] if v[1] else None) for k, v in k64.items()}}
        if flops:
            f64_ms = k64["face"][0] / max(k64["face"][1], 1)
            w64 = 0.5 * (flops["fp64"]["face_stage1"] + flops["fp64"]["face_stage2"]) * 3 * n ** 3 * 9
            out["fp64"]["roofline"] = {"bound": "alu", "kernel": "face_kernel<double,2,3>",
                                       "achieved": w64 / (f64_ms * 1e-3) / 1e12, "peak": MI355X_PEAK["fp64_vector"],
                                       "unit": "TFLOP/s",
                                       "frac": w64 / (f64_ms * 1e-3) / 1e12 / MI355X_PEAK["fp64_vector"]}
        out["speedup_fp32_bulk_vs_fp64"] = sec64 / sec32
        d = (q32 - q64).reshape(5, -1)
        r = q64.reshape(5, -1)
        groups = ((0,), (1, 2, 3), (4,))
        out["rel_l2_fp32_bulk_vs_fp64"] = max(
            float(torch.linalg.norm(d[list(g)]) / torch.linalg.norm(r[list(g)])) for g in groups)
        # the same after subtracting the initial state: the error of what the
        # flow did over the warmup + 4 x steps steps, per (rho, momentum, rho E)
        z = torch.as_tensor(q0, device=q64.device).reshape(5, -1)
        i64 = q64.reshape(5, -1) - z
        i32 = q32.reshape(5, -1) - z
        out["rel_l2_increment_fp32_bulk_vs_fp64"] = {
            name: float(torch.linalg.norm(i32[list(g)] - i64[list(g)]) / torch.linalg.norm(i64[list(g)]))
            for name, g in zip(("rho", "momentum", "rhoE"), groups)}
        out["steps_compared"] = a.warmup + 4 * a.steps
        del s64
    if not a.no_parity and n == 128:
        out["parity_vs_oracle"] = parity_vs_oracle()
    if not a.no_rules:
        # the other compiled quadrature rules on the same Taylor-Green workload
        out["rules"] = {}
        for k, nq in ((2, 2), (3, 3), (3, 4)):
            leg = {"degree": k, "gauss_points_per_axis": nq, "modes": (k + 1) * (k + 2) * (k + 3) // 6}
            dof_k = 5 * leg["modes"] * n ** 3
            for prec in ("fp32_bulk", "fp64"):
                sec, _, kk, qk, sk, _ = time_path(prec, n, min(a.steps, 5), 1, k=k, nq=nq, reps=1)
                ms = {x: (v[0] / v[1] if v[1] else None) for x, v in kk.items() if x in ("face", "volume")}
                leg[prec] = {"value": dof_k / sec, "ms_per_step": 1e3 * sec, "kernels_ms_per_launch": ms}
                fr = (flops or {}).get("rules", {}).get(f"p{k}_nq{nq}", {}).get("fp32" if prec != "fp64" else "fp64")
                if fr and ms["face"] and ms["volume"]:
                    peak = MI355X_PEAK["fp64_vector"] if prec == "fp64" else MI355X_PEAK["fp32_vector"]
                    rl = {"unit": "TFLOP/s", "peak": peak}
                    nsteps_ev = min(a.steps, 5)
                    for kern, pts in (("face", 3 * nq * nq), ("volume", nq ** 3)):
                        # work of both stages over the time of all launches of the
                        # class per step (FP64 P3 runs its stage-1 volume pass as two)
                        w = (fr[f"{kern}_stage1"] + fr[f"{kern}_stage2"]) * pts * n ** 3
                        t_step = kk[kern][0] / nsteps_ev * 1e-3
                        ach = w / t_step / 1e12
                        rl[kern] = {"achieved": ach, "frac": ach / peak, "ms_per_step": t_step * 1e3,
                                    "launches_per_step": kk[kern][1] / nsteps_ev}
                    rl["step_tflops"] = fr["per_step_per_cell"] * n ** 3 / sec / 1e12
                    leg[prec]["roofline"] = rl
                del qk, sk
            out["rules"][f"p{k}_nq{nq}"] = leg
    if not a.no_rules:
        # the same workload on the Section 5.1 mapped (non-uniform) mesh
        leg = {"mesh": "x = xi + 0.05 (b - a) sin(2 pi (xi - a) / (b - a)) per axis", "degree": 2,
               "gauss_points_per_axis": 3}
        for prec in ("fp32_bulk", "fp64"):
            sec, _, kk, qk, sk, _ = time_path(prec, n, min(a.steps, 5), 1, mapped=True, reps=1)
            leg[prec] = {"value": dof / sec, "ms_per_step": 1e3 * sec,
                         "kernels_ms_per_launch": {x: (v[0] / v[1] if v[1] else None) for x, v in kk.items()
                                                   if x in ("face", "volume")}}
            del qk, sk
        out["mapped_mesh"] = leg
    if not a.no_adjoint:
        out["adjoint"] = {"fp32_bulk": adjoint_ratio("fp32_bulk"), "fp64": adjoint_ratio("fp64"),
                          "fp32_bulk_128": adjoint_ratio("fp32_bulk", n=n, nsteps=6, stride=3)}
        if not a.no_rules:
            # P3 (4 Gauss points), 32^3, 50 steps
            out["adjoint"]["p3_fp32_bulk"] = adjoint_ratio("fp32_bulk", nsteps=50, stride=7, k=3)
            out["adjoint"]["p3_fp64"] = adjoint_ratio("fp64", nsteps=50, stride=7, k=3)
        out["adj_over_fwd"] = out["adjoint"]["fp32_bulk"]["adj_over_fwd"]
    if a.copy_calibration:
        x = torch.empty(1 << 28, dtype=torch.float32, device="cuda:0").fill_(1.0)
        y = torch.empty_like(x)
        torch.cuda.synchronize()
        y.copy_(x)
        torch.cuda.synchronize()
        out["copy_calibration_bytes"] = {"read": x.numel() * 4, "write": y.numel() * 4}
        del x, y
    out["kernel_source_hash"] = kernel_source_hash()
    if not a.no_cpu:
        out["cpu_baseline"] = cpu_baseline(n, a.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
