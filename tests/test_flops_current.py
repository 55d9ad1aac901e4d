"""The committed algorithmic flop counts (paper_2202_13821_amd/flops.json, the
roofline numerator of bench.py) match the point functions as they are now:
csrc/flopcount/count_flops.py recounts them from the host IR of the current
gks_point.hpp / gks_point_adj.hpp and must reproduce the file exactly."""
import importlib.util
import json
import os

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SCRIPT = os.path.join(ROOT, "paper_2202_13821_amd", "csrc", "flopcount", "count_flops.py")
FLOPS = os.path.join(ROOT, "paper_2202_13821_amd", "flops.json")


def test_flops_json_matches_current_sources():
    if not os.path.exists(os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")):
        pytest.skip("hipcc not available")
    spec = importlib.util.spec_from_file_location("count_flops", SCRIPT)
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    fresh = json.loads(json.dumps(mod.compute()))
    with open(FLOPS) as f:
        stored = json.load(f)
    assert fresh == stored, "flops.json is stale: rerun paper_2202_13821_amd/csrc/flopcount/count_flops.py"
