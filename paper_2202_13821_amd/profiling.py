"""Summaries of rocprofv3 output (CSV) for the profiles/ folder.

python -m paper_2202_13821_amd.profiling stats  <kernel_stats.csv>  <out.md>  "<command>"
python -m paper_2202_13821_amd.profiling traffic <fetch counter_collection.csv> <write counter_collection.csv>
                                                  <out.json> "<command fetch>" "<command write>"
python -m paper_2202_13821_amd.profiling counters <out.md> "<command prefix>" <counter_collection.csv>...

`counters` summarises SQ/GRBM counter passes per kernel: VALU instructions
per wavefront, SIMD cycles per VALU instruction (4 SIMDs x 256 CUs x the
kernel's GRBM_GUI_ACTIVE cycles / 8 XCDs, over the VALU instructions of all
wavefronts; about 2.6 is the issue rate of FP32 instructions with VGPR
operands on gfx950, 4 that of instructions reading an SGPR), resident
wavefronts per SIMD, and the fraction of wave time spent waiting.

`traffic` reads FETCH_SIZE and WRITE_SIZE (KiB per dispatch) of every kernel,
takes the plain device copy launched by `bench.py --copy-calibration`
(1 GiB read + 1 GiB written) as the reference of known size, scales each
kernel's counters by (known bytes / counted bytes of the copy) and writes
bytes per launch, with the hash of the kernel sources the counters were taken
with.
"""
import csv
import hashlib
import json
import os
import re
import sys
from collections import defaultdict

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def kernel_source_hash():
    h = hashlib.sha256()
    src = os.path.join(ROOT, "paper_2202_13821_amd", "csrc")
    for name in sorted(os.listdir(src)):
        if name.endswith((".hpp", ".hip")):
            with open(os.path.join(src, name), "rb") as f:
                h.update(f.read())
    # the build options (code generation) belong to the kernels too
    with open(os.path.join(ROOT, "paper_2202_13821_amd", "build.py"), "rb") as f:
        h.update(f.read())
    return h.hexdigest()[:16]


def short_name(name):
    """'void dgk::face_kernel<float, 2, 3, true>(...)' -> 'face_kernel<float,2,3,true>'"""
    m = re.search(r"dgk::(\w+<[^>]*>)", name)
    if m:
        return m.group(1).replace(" ", "")
    return name.split("(")[0].replace("void ", "").strip()


def _rows(path):
    with open(path, newline="") as f:
        return list(csv.DictReader(f))


def _col(row, *names):
    for n in names:
        for k in row:
            if k.lower() == n.lower():
                return row[k]
    raise KeyError(f"none of {names} in {list(row)}")


def stats(csv_path, out_md, command):
    rows = _rows(csv_path)
    lines = [f"# rocprofv3 kernel statistics", "", f"Command: `{command}`", "",
             "| kernel | calls | total ms | average ms | min ms | max ms | % |", "|---|---|---|---|---|---|---|"]
    for r in rows:
        name = short_name(_col(r, "Name", "KernelName", "Kernel_Name"))
        calls = int(float(_col(r, "Calls")))
        tot = float(_col(r, "TotalDurationNs", "DURATION (nsec)", "Total_Duration_Ns")) / 1e6
        avg = float(_col(r, "AverageNs", "AVERAGE (nsec)", "Average_Ns")) / 1e6
        mn = float(_col(r, "MinNs", "MIN (nsec)", "Min_Ns")) / 1e6
        mx = float(_col(r, "MaxNs", "MAX (nsec)", "Max_Ns")) / 1e6
        pct = float(_col(r, "Percentage", "PERCENT (INC)"))
        lines.append(f"| `{name}` | {calls} | {tot:.3f} | {avg:.4f} | {mn:.4f} | {mx:.4f} | {pct:.2f} |")
    with open(out_md, "w") as f:
        f.write("\n".join(lines) + "\n")


def _per_kernel(path, counter):
    vals = defaultdict(list)
    for r in _rows(path):
        if _col(r, "Counter_Name", "Counter-Name").strip() != counter:
            continue
        vals[short_name(_col(r, "Kernel_Name", "Kernel-Name"))].append(float(_col(r, "Counter_Value", "Counter-Value")))
    return vals


def traffic(fetch_csv, write_csv, out_json, cmd_fetch, cmd_write, copy_bytes=1 << 30):
    fetch = _per_kernel(fetch_csv, "FETCH_SIZE")
    write = _per_kernel(write_csv, "WRITE_SIZE")
    # reference: the largest elementwise copy kernel of torch (1 GiB read, 1 GiB written)
    copy_keys = [k for k in fetch if "copy" in k.lower() or "elementwise" in k.lower()]
    ref_f = max((max(fetch[k]) for k in copy_keys), default=None)
    copy_keys_w = [k for k in write if "copy" in k.lower() or "elementwise" in k.lower()]
    ref_w = max((max(write[k]) for k in copy_keys_w), default=None)
    sf = copy_bytes / (ref_f * 1024.0) if ref_f else None
    sw = copy_bytes / (ref_w * 1024.0) if ref_w else None
    out = {"source_hash": kernel_source_hash(), "commands": [cmd_fetch, cmd_write],
           "copy_reference": {"bytes_read": copy_bytes, "bytes_written": copy_bytes,
                              "FETCH_SIZE_KiB": ref_f, "WRITE_SIZE_KiB": ref_w,
                              "scale_fetch": sf, "scale_write": sw},
           "kernels": {}}
    for k in sorted(set(fetch) | set(write)):
        if not k.startswith(("face_kernel", "volume_kernel", "adj_", "convert")):
            continue
        f = sum(fetch.get(k, [0])) / max(len(fetch.get(k, [])), 1)
        w = sum(write.get(k, [0])) / max(len(write.get(k, [])), 1)
        fb = f * 1024.0 * (sf or 1.0)
        wb = w * 1024.0 * (sw or 1.0)
        out["kernels"][k] = {"FETCH_SIZE_KiB": f, "WRITE_SIZE_KiB": w, "read_bytes": fb, "write_bytes": wb,
                             "bytes_per_launch": fb + wb}
    # per kernel family averaged over the two stages, as bench.py reports them
    for fam in ("face_kernel<float,2,3", "volume_kernel<float,2,3", "face_kernel<double,2,3",
                "volume_kernel<double,2,3"):
        ks = [v["bytes_per_launch"] for k, v in out["kernels"].items() if k.startswith(fam)]
        if ks:
            out["kernels"][fam + ">"] = {"bytes_per_launch": sum(ks) / len(ks), "averaged_over": len(ks)}
    with open(out_json, "w") as f:
        json.dump(out, f, indent=1)
    return out


def counters(out_md, command, *csvs):
    vals = defaultdict(lambda: defaultdict(list))
    for path in csvs:
        for r in _rows(path):
            vals[short_name(_col(r, "Kernel_Name", "Kernel-Name"))][_col(r, "Counter_Name", "Counter-Name").strip()].append(
                float(_col(r, "Counter_Value", "Counter-Value")))
    avg = {k: {c: sum(v) / len(v) for c, v in d.items()} for k, d in vals.items()}
    lines = ["# rocprofv3 counters per kernel", "", f"Command (one run per counter set): `{command}`", "",
             "| kernel | VALU instr / wave | SIMD cycles / VALU instr | waves / SIMD | wait fraction | FP32 flop / wave | FP64 flop / wave |",
             "|---|---|---|---|---|---|---|"]
    for k in sorted(avg):
        d = avg[k]
        if not k.startswith(("face_kernel", "volume_kernel", "adj_")) or "SQ_WAVES" not in d:
            continue
        w = d["SQ_WAVES"]
        cyc = d.get("GRBM_GUI_ACTIVE", 0.0) / 8.0  # summed over the 8 XCDs
        valu = d.get("SQ_INSTS_VALU", 0.0)
        cpi = 4 * 256 * cyc / valu if cyc and valu else float("nan")
        occ = 4.0 * d["SQ_WAVE_CYCLES"] / cyc / 1024.0 if cyc and "SQ_WAVE_CYCLES" in d else float("nan")
        wait = d["SQ_WAIT_ANY"] / d["SQ_WAVE_CYCLES"] if "SQ_WAIT_ANY" in d else float("nan")
        f32 = 64 * d.get("SQ_INSTS_VALU_FLOPS_FP32", 0.0) / w
        f64 = 64 * d.get("SQ_INSTS_VALU_FLOPS_FP64", 0.0) / w
        lines.append(f"| `{k}` | {valu / w:.0f} | {cpi:.2f} | {occ:.2f} | {wait:.2f} | {f32:.3g} | {f64:.3g} |")
    with open(out_md, "w") as f:
        f.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    if sys.argv[1] == "stats":
        stats(sys.argv[2], sys.argv[3], sys.argv[4])
    elif sys.argv[1] == "traffic":
        print(json.dumps(traffic(*sys.argv[2:7]), indent=1))
    elif sys.argv[1] == "counters":
        counters(*sys.argv[2:])
