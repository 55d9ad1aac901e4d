"""Build the HIP library libdg_hgks.so for gfx950 (in-tree, under lib/).

The C-ABI (csrc/dg_hgks.hip) and four objects per compiled configuration
(csrc/instantiate.hip with -DDGK_T/-DDGK_K/-DDGK_NQ and -DDGK_PART: the
forward launches with the face passes, the forward volume passes, the
adjoint with its face passes, the adjoint's volume passes) are compiled in
parallel, then linked.
"""
import os
import subprocess
import sys
import tempfile

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIBDIR = os.path.join(PKG, "lib")
LIB = os.path.join(LIBDIR, "libdg_hgks.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # no packed-FP32 instructions (v_pk_*_f32) in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
]

# (precision, degree, Gauss points per axis) compiled into the library
CONFIGS = [(t, k, nq) for t in ("float", "double") for (k, nq) in ((1, 2), (2, 3), (2, 2), (3, 4), (3, 3))]

# The backend's iterative ILP scheduling strategy, where it measured faster
# (alternated builds in one session; results bit-identical, or within the
# adjoint tests' tolerances):
# - the FP32 forward kernels (face and volume) up to P2, which run two
#   wavefronts per SIMD (three for the P2 stage-2 volume pass): the P2 face
#   kernel took 4% less time per launch;
# - the forward volume kernels in FP64 at P2 (1-3% less) and at P3 with 4
#   points (16% less; with 3 points it was 25% slower), and in FP32 at P3
#   (3-10% less);
# - the P3 adjoint volume kernels: 40% less in FP64, 24% less in FP32.
# Elsewhere it was slower: up to 80% for the FP64 forward face kernel, 70%
# for the FP32 P2 adjoint volume kernel, 18-40% for the P3 adjoint face
# kernels.  The FP32 P3 forward face kernel was 4-5% faster with it, but its
# non-uniform-mesh variant then returned NaN where the default build matches
# the oracle, so it keeps the default.
SCHED_ILP = ["-mllvm", "-amdgpu-sched-strategy=iterative-ilp"]
# The backend's max-ILP strategy for the FP64 adjoint face kernel at P2: 2.7%
# less time per launch (it made the adjoint volume kernel 22% slower).
SCHED_MAX_ILP = ["-mllvm", "-amdgpu-sched-strategy=max-ilp"]


def _sched(t, k, nq, part):
    if part == 1:  # forward launches and face passes
        return SCHED_ILP if t == "float" and k <= 2 else []
    if part == 4:  # forward volume passes
        return SCHED_ILP if t == "float" or k == 2 or (k == 3 and nq == 4) else []
    if part == 2:  # adjoint launch sequence and face passes
        return SCHED_MAX_ILP if t == "double" and k == 2 else []
    if part == 3:  # adjoint volume passes
        return SCHED_ILP if k == 3 else []
    return []


PARTS = ((1, "fwd"), (4, "fwdvol"), (2, "adj"), (3, "adjvol"))


def _units():
    yield "dg_hgks", os.path.join(CSRC, "dg_hgks.hip"), []
    for t, k, nq in CONFIGS:
        defs = [f"-DDGK_T={t}", f"-DDGK_K={k}", f"-DDGK_NQ={nq}"]
        for part, tag in PARTS:
            yield (f"inst_{t}_{k}{nq}_{tag}", os.path.join(CSRC, "instantiate.hip"),
                   defs + [f"-DDGK_PART={part}"] + _sched(t, k, nq, part))


def build(verbose: bool = False, extra=(), jobs: int = None) -> str:
    os.makedirs(LIBDIR, exist_ok=True)
    jobs = jobs or max(1, min(len(PARTS) * len(CONFIGS) + 1, os.cpu_count() or 1, 16))
    inc = ["-I", os.path.join(ROOT, "include"), "-I", CSRC]
    with tempfile.TemporaryDirectory(prefix="dg_hgks_build_") as tmp:
        objs, pending = [], []
        for name, src, defs in _units():
            obj = os.path.join(tmp, name + ".o")
            cmd = [HIPCC, *FLAGS, *extra, *defs, *inc, "-c", "-o", obj, src]
            if verbose:
                print(" ".join(cmd), flush=True)
            while len([p for p in pending if p[0].poll() is None]) >= jobs:
                pending[0][0].wait()
                pending.sort(key=lambda p: p[0].poll() is None)
            pending.append((subprocess.Popen(cmd), cmd))
            objs.append(obj)
        failed = [cmd for proc, cmd in pending if proc.wait() != 0]
        if failed:
            raise subprocess.CalledProcessError(1, failed[0])
        link = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", LIB + ".tmp", *objs]
        if verbose:
            print(" ".join(link), flush=True)
        subprocess.run(link, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True, extra=sys.argv[1:]))
