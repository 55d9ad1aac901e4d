"""Count the floating-point operations of one face point and one volume
point of the kernels' formulas (forward and adjoint) and write
paper_2202_13821_amd/flops.json.

The point functions of gks_point.hpp are compiled for the host to optimised
LLVM IR (common subexpressions merged, loops unrolled; the code is straight
line) and their IR instructions are counted: fadd/fsub/fmul = 1 flop,
llvm.fmuladd/llvm.fma = 2, fdiv = 1, sqrt/exp/erfc = 1 each (also listed
apart); vectorisation is disabled, and a vector operation would count once
per element.  The modal evaluation at the point and the projection onto the modes
are contractions whose useful flops (non-zero basis entries only) are added
in closed form for each compiled (degree, Gauss points) rule (P2: 10 modes,
6 tangential modes, 4 modes with a non-zero derivative along each axis;
P3: 20, 10 and 10).
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
                    "-fno-slp-vectorize", "-DDGK_FLOPCOUNT", "-funroll-loops", "-mllvm", "-unroll-threshold=1000000",
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


def nmodes(k):
    return (k + 1) * (k + 2) * (k + 3) // 6


def totals(counts, k, nq):
    """Per-point totals of one (degree, Gauss points) rule from the point-flux
    counts: flux + evaluation of Q and its three derivatives from the modes
    (both traces at a face point) + projection onto the modes."""
    NM, NT = nmodes(k), (k + 1) * (k + 2) // 2
    nd = NM - NT  # modes with a non-zero exponent (non-zero derivative) along a given axis
    # evaluation of Q and the three derivatives at a point: (NM + 3 nd) FMAs per variable
    eval_pt = 5 * (NM + 3 * nd) * 2 + 15
    d = {}
    for st in ("s1", "s2"):
        nf = 2 if st == "s1" else 1
        face, vol = counts[("face", st)], counts[("vol", st)]
        # face: two traces, flux, projection on NT tangential modes (per point share)
        d[f"face_stage{st[1]}"] = 2 * eval_pt + face["flops"] + nf * 5 * NT * 2
        # volume: one evaluation, flux, projection sum_q w F_d dB_n/dx_d over the
        # 3 nd non-zero (d, n) entries
        d[f"volume_stage{st[1]}"] = eval_pt + vol["flops"] + nf * 5 * 3 * nd * 2
    # per cell and step: 3 faces of nq^2 points and nq^3 volume points, both stages
    d["per_step_per_cell"] = (3 * nq * nq * (d["face_stage1"] + d["face_stage2"])
                              + nq ** 3 * (d["volume_stage1"] + d["volume_stage2"]))
    return d


def adjoint_totals(c, k, nq):
    """Per-point algorithmic flops of the adjoint kernels of one rule.  Face
    point of adjoint stage s (the reverse of forward stage s): the two traces
    and the two sides recomputed, the reverse of the finish, the reverses of
    the two sides, the two transposed trace evaluations and the record
    cotangent at the point (F_bar = sum_m phi_m Phi_bar_m).  Volume point:
    the evaluation, the reverse of the volume flux, the transposed evaluation
    and the transposed projection.  (The lane pair of the adjoint face kernel
    also runs the finish's reverse twice; the repeat is not counted.)"""
    NM, NT = nmodes(k), (k + 1) * (k + 2) // 2
    nd = NM - NT
    eval_pt = 5 * (NM + 3 * nd) * 2 + 15
    d = {}
    for st in ("s1", "s2"):
        nf = 2 if st == "s1" else 1
        d[f"face_stage{st[1]}"] = (4 * eval_pt + 2 * c["side"]["flops"] + c[("finvjp", st)]["flops"]
                                   + 2 * c["sidevjp"]["flops"] + nf * 5 * NT * 2)
        d[f"volume_stage{st[1]}"] = 2 * eval_pt + c[("volvjp", st)]["flops"] + nf * 5 * 3 * nd * 2
    d["per_step_per_cell"] = (3 * nq * nq * (d["face_stage1"] + d["face_stage2"])
                              + nq ** 3 * (d["volume_stage1"] + d["volume_stage2"]))
    return d


RULES = ((1, 2), (2, 3), (2, 2), (3, 4), (3, 3))


def compute():
    """The counts as written to flops.json (compiles the host IR)."""
    text = ir()
    res = {"k": 2, "nq": 3, "counted_from": "optimised host LLVM IR of gks_point.hpp"}
    rules = {f"p{k}_nq{nq}": {} for k, nq in RULES}
    for T, tag in (("f32", "fp32"), ("f64", "fp64")):
        counts = {(kind, st): count(text, f"fc_{kind}_{T}_{st}") for kind in ("face", "vol") for st in ("s1", "s2")}
        d = totals(counts, 2, 3)
        for st in ("s1", "s2"):
            d[f"face_point_flux_stage{st[1]}_detail"] = counts[("face", st)]
            d[f"volume_point_flux_stage{st[1]}_detail"] = counts[("vol", st)]
        res[tag] = {x: v for x, v in d.items() if x != "per_step_per_cell"}
        res.setdefault("per_step_per_cell", {})[tag] = d["per_step_per_cell"]
        ac = {"side": count(text, f"fc_side_{T}"), "sidevjp": count(text, f"fc_sidevjp_{T}")}
        for st in ("s1", "s2"):
            ac[("finvjp", st)] = count(text, f"fc_finvjp_{T}_{st}")
            ac[("volvjp", st)] = count(text, f"fc_volvjp_{T}_{st}")
        ad = adjoint_totals(ac, 2, 3)
        ad["detail"] = {"side": ac["side"], "side_reverse": ac["sidevjp"],
                        **{f"finish_reverse_stage{st[1]}": ac[("finvjp", st)] for st in ("s1", "s2")},
                        **{f"volume_reverse_stage{st[1]}": ac[("volvjp", st)] for st in ("s1", "s2")}}
        res.setdefault("adjoint", {})[tag] = ad
        for k, nq in RULES:
            rules[f"p{k}_nq{nq}"][tag] = totals(counts, k, nq)
            rules[f"p{k}_nq{nq}"][f"adjoint_{tag}"] = adjoint_totals(ac, k, nq)
    res["rules"] = rules
    return res


def main():
    res = compute()
    path = os.path.join(PKG, "flops.json")
    with open(path, "w") as f:
        json.dump(res, f, indent=1)
    json.dump(res, sys.stdout, indent=1)


if __name__ == "__main__":
    main()
