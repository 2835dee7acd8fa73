"""The bounds-checked debug build on the GPU: over a geometry matrix (every stencil, storage,
boundary kind and schedule, ragged and degenerate grids, both layouts, a group, the 1088^2
benchmark grid) no kernel meets an index out of range, and the results are bitwise those of the
normal build."""
import json
import os
import subprocess
import sys

import pytest

from paper_2504_20169_amd import lbm

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)
import bounds_cases  # noqa: E402


@pytest.mark.gpu
def test_bounds_checked_build_finds_no_index_out_of_range(tmp_path):
    if not os.path.exists(lbm.BOUNDS_LIB_PATH):
        pytest.fail("the bounds-checked build is missing: run __graft_entry__.build()")
    out = tmp_path / "bounds.json"
    env = dict(os.environ, LBM_MI355X_LIB=lbm.BOUNDS_LIB_PATH)
    print("bounds-checked build: subprocess over", len(bounds_cases.CASES), "cases", flush=True)
    res = subprocess.run([sys.executable, "-u", os.path.join(HERE, "bounds_cases.py"), str(out)],
                         env=env, capture_output=True, text=True, timeout=240)
    sys.stdout.write(res.stdout[-2000:])
    assert res.returncode == 0, res.stderr[-4000:]
    checked = json.load(open(out))
    assert checked.pop("build_flags") == lbm.LBM_BUILD_BOUNDS
    normal = bounds_cases.run_all()
    assert normal.pop("build_flags") == 0
    assert checked.keys() == normal.keys()
    diff = [k for k in normal if normal[k] != checked[k]]
    assert not diff, diff
