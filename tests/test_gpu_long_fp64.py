"""Full-length runs of the benchmark workloads against stored oracle values (GPU).

The 1024^2 + 32-cell PML vortex + pulse workload with the characteristic boundary (the bench's
headline configuration) runs its full 10^4 steps through the C ABI in the launch configuration
the bench times; its moments are compared at the sampled nodes of the stored oracle fixture
(tests/golden/make_long_fp64.py, written by the double oracle).  The bar is the parity bar:
1e-12 relative (rho, T relative to their largest value, u to the largest velocity component), or
4x the double oracle's own accumulated rounding at those nodes where that is higher, measured
against the same oracle run in x87 extended precision (the extended fixture).  FP32 and FP16
storage run the same workload and report their error against the oracle; FP32 is held to 1e-6.
"""
import os
import sys

import numpy as np
import pytest

from paper_2504_20169_amd import lbm
from paper_2504_20169_amd import workloads as wl
from _helpers import TOL, say

sys.path.insert(0, os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden"))
from make_long_fp64 import fixture_path, read_fixture  # noqa: E402

pytestmark = pytest.mark.gpu


def _errors(m, fix):
    _, x, y, rho, ux, uy, T = fix
    us = max(np.abs(ux).max(), np.abs(uy).max())
    return dict(rho=float(np.abs(m[0][y, x] - rho).max() / np.abs(rho).max()),
                ux=float(np.abs(m[1][y, x] - ux).max() / us),
                uy=float(np.abs(m[2][y, x] - uy).max() / us),
                T=float(np.abs(m[3][y, x] - T).max() / np.abs(T).max()))


def _floor(dbl, ext):
    """The double fixture's distance from the extended one, in the normalisations of _errors."""
    _, x, y = dbl[:3]
    m = [np.full((int(y.max()) + 1, int(x.max()) + 1), np.nan) for _ in range(4)]
    for k in range(4):
        m[k][y, x] = dbl[3 + k]
    return _errors(m, ext)


@pytest.mark.skipif(not (os.path.exists(fixture_path("vortex_1088")) and
                         os.path.exists(fixture_path("vortex_1088", "extended"))),
                    reason="oracle fixtures not written")
def test_vortex_1088_full_length_matches_the_oracle():
    fix = read_fixture("vortex_1088")
    hdr = fix[0]
    assert int(hdr["steps"]) == 10000 and hdr["grid"].split() == ["1088", "1088"]
    spec = wl.vortex_pulse(L=1024, W=32, sigma_max=0.0015, mach=0.1, bc="nrbc", seed=2)
    floor = _floor(fix, read_fixture("vortex_1088", "extended"))
    say("double oracle vs extended at the fixture nodes", {k: "%.2e" % v for k, v in floor.items()})
    errs = _run_all(spec, "nrbc", 32, 0.0015, 10000, fix, "vortex_1088")
    for k, v in errs["f64"].items():
        bar = max(TOL, 4.0 * floor[k])
        assert v <= bar, (k, v, bar, errs["f64"], floor)
    assert all(v < 1e-6 for v in errs["f32"].values()), errs["f32"]


@pytest.mark.skipif(not (os.path.exists(fixture_path("pulses_4224_zg")) and
                         os.path.exists(fixture_path("pulses_4224_zg", "extended"))),
                    reason="oracle fixtures not written")
def test_pulses_4224_zg_full_length_matches_the_oracle():
    """The 4096^2 + 64-cell PML multi-pulse workload with ZG edges, its full 2000 steps.  The bar
    is 1e-12, or 4x the double oracle's own rounding where the extended-precision fixture of the
    same run shows it higher (the velocity, of max |u| = Mach 0.05, differs from the double
    oracle by about 2e-12 relative after the 2000 steps)."""
    fix = read_fixture("pulses_4224_zg")
    hdr = fix[0]
    assert int(hdr["steps"]) == 2000 and hdr["grid"].split() == ["4224", "4224"]
    spec = wl.multi_pulse(L=4096, W=64, sigma_max=0.01, mach=0.05, bc="zg")
    floor = _floor(fix, read_fixture("pulses_4224_zg", "extended"))
    say("double oracle vs extended at the fixture nodes", {k: "%.2e" % v for k, v in floor.items()})
    errs = _run_all(spec, "zg", 64, 0.01, 2000, fix, "pulses_4224_zg")
    for k, v in errs["f64"].items():
        bar = max(TOL, 4.0 * floor[k])
        assert v <= bar, (k, v, bar, errs["f64"], floor)
    assert all(v < 1e-6 for v in errs["f32"].values()), errs["f32"]


def _run_all(spec, bc, W, sigma, steps, fix, name):
    """Run the workload in every storage through the C ABI in the bench's launch configuration;
    errors against the fixture per storage."""
    errs = {}
    for storage in ("f64", "f32", "f16"):
        say("case %s %d steps" % (name, steps), storage)
        r = lbm.Run(spec.Lx, spec.Ly, 0.8, 1.0, spec.ux0, 0.0, 1.0, storage=storage)
        r.set_launch(bulk_tx=64, graph_steps=32, overlap=2)
        r.set_bc(lbm.LBM_ALL, bc)
        r.set_pml(lbm.LBM_ALL, W, sigma)
        r.init(*spec.fields.as_tuple())
        r.step(steps)
        assert r.check() == lbm.LBM_OK
        errs[storage] = _errors(r.moments(), fix)
        r.close()
        say(storage, "vs oracle", {k: "%.2e" % v for k, v in errs[storage].items()})
    return errs
