"""Build the VALU issue-rate probe (valu_rate.hip) next to its source."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

if __name__ == "__main__":
    out = os.path.join(HERE, "valu_rate")
    subprocess.run([HIPCC, "--offload-arch=gfx950", "-O3", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                    "-o", out, os.path.join(HERE, "valu_rate.hip")], check=True)
    print(out)
