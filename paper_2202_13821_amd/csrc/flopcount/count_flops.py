"""Count the floating-point operations of one face point and one volume
point of the kernels' formulas and write paper_2202_13821_amd/flops.json.

The point functions of gks_point.hpp are compiled for the host to optimised
LLVM IR (common subexpressions merged, loops unrolled; the code is straight
line) and their IR instructions are counted: fadd/fsub/fmul = 1 flop,
llvm.fmuladd/llvm.fma = 2, fdiv = 1, sqrt/exp/erfc = 1 each (also listed
apart); vectorisation is disabled, and a vector operation would count once
per element.  The modal evaluation at the point and the projection onto the modes
are contractions whose useful flops (non-zero basis entries only) are added
in closed form (P2, 3 Gauss points per direction, 10 modes, 6 tangential
modes, 4 modes with a non-zero derivative along each axis).
"""
import json
import os
import re
import subprocess
import sys
from collections import Counter

HERE = os.path.dirname(os.path.abspath(__file__))
PKG = os.path.dirname(os.path.dirname(HERE))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def ir():
    out = os.path.join("/tmp", "dg_flopcount.ll")
    subprocess.run([HIPCC, "--cuda-host-only", "-O2", "-std=c++17", "-ffp-contract=on", "-fno-vectorize",
                    "-fno-slp-vectorize", "-funroll-loops", "-mllvm", "-unroll-threshold=1000000",
                    "-mllvm", "-unroll-max-count=4096", "-S", "-emit-llvm",
                    "-I", os.path.dirname(HERE), "-o", out, os.path.join(HERE, "flopcount.hip")], check=True)
    return open(out).read()


def _bodies(text):
    out = {}
    for m in re.finditer(r"define [^@]*@([\w.$]+)\(.*?\n\}", text, re.S):
        out[m.group(1)] = m.group(0)
    return out


def count(text, fname, bodies=None):
    """Operation counts of fname, including functions it calls that are
    defined in the same module (the per-direction lambdas of volume_flux)."""
    bodies = bodies or _bodies(text)
    body = bodies[fname]
    c = Counter()
    for line in body.splitlines()[1:]:
        line = line.strip()
        # vector operations count once per element (<N x float>)
        vw = re.search(r"<(\d+) x (float|double)>", line)
        w = int(vw.group(1)) if vw else 1
        if re.search(r"= (fadd|fsub|fmul)\b", line):
            c["addmul"] += w
        elif re.search(r"= fdiv\b", line):
            c["div"] += w
        elif "@llvm.fmuladd" in line or "@llvm.fma." in line:
            c["fma"] += w
        elif re.search(r"@(llvm\.sqrt|sqrtf?\b)", line):
            c["sqrt"] += 1
        elif re.search(r"@(llvm\.exp\.|expf?\b)", line):
            c["exp"] += 1
        elif re.search(r"@erfcf?\b", line):
            c["erfc"] += 1
        else:
            m = re.search(r"call [^@]*@([\w.$]+)\(", line)
            if m and m.group(1) in bodies:
                sub = count(text, m.group(1), bodies)
                for k, v in sub.items():
                    if k != "flops":
                        c[k] += v
    c["flops"] = c["addmul"] + 2 * c["fma"] + c["div"] + c["sqrt"] + c["exp"] + c["erfc"]
    return dict(c)


def main():
    text = ir()
    NM, NT, NQ2, NQ3 = 10, 6, 9, 27
    nd = 4  # P2 modes with a nonzero exponent along a given axis
    # evaluation of Q and the three derivatives at a point: (NM + 3 nd) FMAs per variable
    eval_pt = 5 * (NM + 3 * nd) * 2 + 15
    res = {"k": 2, "nq": 3, "counted_from": "optimised host LLVM IR of gks_point.hpp"}
    for T, tag in (("f32", "fp32"), ("f64", "fp64")):
        d = {}
        for st in ("s1", "s2"):
            nf = 2 if st == "s1" else 1
            face = count(text, f"fc_face_{T}_{st}")
            vol = count(text, f"fc_vol_{T}_{st}")
            # face: two traces, flux, projection on NT tangential modes (per point share)
            face_total = 2 * eval_pt + face["flops"] + nf * 5 * NT * 2
            # volume: one evaluation, flux, projection sum_q w F_d dB_n/dx_d over the
            # 3 nd non-zero (d, n) entries
            vol_total = eval_pt + vol["flops"] + nf * 5 * 3 * nd * 2
            d[f"face_stage{st[1]}"] = face_total
            d[f"volume_stage{st[1]}"] = vol_total
            d[f"face_point_flux_stage{st[1]}_detail"] = face
            d[f"volume_point_flux_stage{st[1]}_detail"] = vol
        res[tag] = d
    res["per_step_per_cell"] = {tag: 27 * (res[tag]["face_stage1"] + res[tag]["face_stage2"]
                                           + res[tag]["volume_stage1"] + res[tag]["volume_stage2"])
                                for tag in ("fp32", "fp64")}
    path = os.path.join(PKG, "flops.json")
    with open(path, "w") as f:
        json.dump(res, f, indent=1)
    json.dump(res, sys.stdout, indent=1)


if __name__ == "__main__":
    main()
