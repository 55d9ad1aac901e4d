"""Build the HIP library libdg_hgks.so for gfx950 (in-tree, under lib/).

The C-ABI (csrc/dg_hgks.hip) and three objects per compiled configuration
(csrc/instantiate.hip with -DDGK_T/-DDGK_K/-DDGK_NQ and -DDGK_PART: the
forward launches, the adjoint with its face passes, the adjoint's volume
passes) are compiled in parallel, then linked.
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
# (alternated builds in one session, bit-identical results):
# - the FP32 forward kernels (face and volume) up to P2, which run two
#   wavefronts per SIMD (three for the P2 stage-2 volume pass): the P2 face
#   kernel took 4% less time per launch;
# - the P3 adjoint volume kernels: 40% less in FP64, 24% less in FP32.
# Elsewhere it was slower: up to 80% for the FP64 forward face kernel, 70%
# for the FP32 P2 adjoint volume kernel, 18-40% for the P3 adjoint face
# kernels.  At P3 the FP32 forward step was 4-8% faster, but the
# non-uniform-mesh operator built this way returned NaN where the default
# build matches the oracle, so the P3 forward kernels keep the default.
SCHED_ILP = ["-mllvm", "-amdgpu-sched-strategy=iterative-ilp"]


def _sched(t, k, part):
    if part == 1:
        return SCHED_ILP if t == "float" and k <= 2 else []
    if part == 3:
        return SCHED_ILP if k == 3 else []
    return []


def _units():
    yield "dg_hgks", os.path.join(CSRC, "dg_hgks.hip"), []
    for t, k, nq in CONFIGS:
        defs = [f"-DDGK_T={t}", f"-DDGK_K={k}", f"-DDGK_NQ={nq}"]
        for part, tag in ((1, "fwd"), (2, "adj"), (3, "adjvol")):
            yield (f"inst_{t}_{k}{nq}_{tag}", os.path.join(CSRC, "instantiate.hip"),
                   defs + [f"-DDGK_PART={part}"] + _sched(t, k, part))


def build(verbose: bool = False, extra=(), jobs: int = None) -> str:
    os.makedirs(LIBDIR, exist_ok=True)
    jobs = jobs or max(1, min(3 * len(CONFIGS) + 1, os.cpu_count() or 1, 16))
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
