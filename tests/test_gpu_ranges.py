"""LBM_DEBUG_RANGES (roctx ranges around lbm_step and lbm_group_step) changes no launch and no
bit: single runs (graph replays and an eager remainder) and a group with one flagged member."""
import numpy as np
import pytest

from paper_2504_20169_amd import lbm
from paper_2504_20169_amd import workloads as wl


def _make(L, W, bc, seed, flags=0):
    r = lbm.Run(L, L + 5, 0.8, 1.0, 0.05, 0.0, 1.0)
    r.set_bc(lbm.LBM_ALL, bc)
    if W:
        r.set_pml(lbm.LBM_ALL, W, 0.05)
    r.set_debug(flags)
    Nx, Ny = r.grid()
    r.init(*wl.noisy_state(Nx, Ny, seed, 1.0, 0.05, 0.0, 1.0).as_tuple())
    return r


@pytest.mark.gpu
def test_trace_ranges_keep_bits():
    out = []
    for flags in (0, lbm.LBM_DEBUG_RANGES):
        r = _make(60, 8, "nrbc", 5, flags)
        r.step(70)          # two graph replays of 32 steps and an eager remainder
        out.append(r.populations())
        r.close()
    assert np.array_equal(out[0], out[1])
    res = []
    for flags in (0, lbm.LBM_DEBUG_RANGES):
        g = lbm.Group()
        runs = [_make(50, 6, "zg", 7, flags), _make(41, 0, "nrbc", 8)]
        for r in runs:
            g.add(r)
        g.step(steps=np.array([40, 23], dtype=np.int64))
        res.append([r.populations() for r in runs])
        for r in runs:
            g.remove(r)
            r.close()
        g.close()
    assert all(np.array_equal(a, b) for a, b in zip(*res))
