"""NaN canary (GPU): with lbm_set_debug(LBM_DEBUG_POISON) every buffer that a step writes in full
is filled with NaN before the step's kernels, so a node or component that a step leaves unwritten
and a later kernel reads turns into NaN.  Each case runs the same workload with and without the
canary and requires the same bits in the moments, the populations and the PML field Q, and a
finite state: every stencil and storage, every boundary kind with and without a PML, the
appendix's PML-moment terms, the three launch schedules, graph replays plus an eager
remainder, and a batch of uneven runs in which one member carries the canary."""
import numpy as np
import pytest

from paper_2504_20169_amd import lbm
from paper_2504_20169_amd import workloads as wl
from _helpers import say

pytestmark = pytest.mark.gpu

# (lattice, storage, bc, W, pml_terms, overlap, L)
CASES = [
    (37, "f64", "nrbc", 6, 0, 2, 40),
    (37, "f64", "zg", 6, 0, 0, 40),
    (37, "f64", "nrbc", 6, 7, 2, 36),
    (37, "f64", "nrbc", 0, 0, 1, 40),
    (37, "f32", "nrbc", 8, 0, 2, 70),
    (37, "f16", "zg", 5, 0, 2, 33),
    (17, "f64", "nrbc", 6, 0, 2, 40),
    (17, "f64", "nrbc_a", 4, 0, 2, 30),
    (9, "f64", "zg", 3, 0, 2, 29),
    (37, "f64", "periodic", 0, 0, 2, 130),
]


def _make(lattice, storage, bc, W, terms, overlap, L, seed, poison):
    spec = wl.vortex_pulse(L=L, W=W, sigma_max=0.01, mach=0.1, bc="zg" if bc == "periodic" else "nrbc",
                           seed=seed, radius=5.0)
    r = lbm.Run(L, L, 0.8, 1.0, 0.1, 0.0, 1.0, storage=storage, lattice=lattice)
    r.set_launch(bulk_tx=64, graph_steps=16, overlap=overlap)
    if bc == "nrbc_a":
        r.set_bc(lbm.LBM_ALL, "nrbc")
        r.set_bc(lbm.LBM_XMAX, "nrbc_a")
    else:
        r.set_bc(lbm.LBM_ALL, bc)
    if W:
        r.set_pml(lbm.LBM_ALL, W, 0.01)
    if terms:
        r.set_nrbc_pml_terms(terms)
    if poison:
        r.set_debug(lbm.LBM_DEBUG_POISON)
    r.init(*spec.fields.as_tuple())
    return r


def _state(r):
    return list(r.moments()) + [r.populations(), r.pml_q()]


def _same(a, b):
    return all(x.shape == y.shape and np.array_equal(x, y) for x, y in zip(a, b))


@pytest.mark.parametrize("case", CASES, ids=lambda c: "q%d-%s-%s-W%d-t%d-ov%d" % c[:6])
def test_canary_leaves_the_bits(case):
    say("canary case", case)
    out = []
    for poison in (False, True):
        r = _make(*case, seed=11, poison=poison)
        r.step(37)                       # two graphs of 16 steps and an eager remainder of 5
        assert r.check() == lbm.LBM_OK
        out.append(_state(r))
        r.close()
    for x in out[1]:
        assert np.isfinite(x).all()
    assert _same(out[0], out[1]), case


def test_canary_in_a_batch():
    cases = [(37, "f64", "nrbc", 6, 0, 2, 40), (37, "f64", "zg", 4, 0, 2, 52), (37, "f64", "nrbc", 0, 0, 2, 30)]
    steps = np.array([37, 20, 33])
    out = []
    for poison in (False, True):
        g = lbm.Group()
        runs = [_make(*c, seed=20 + k, poison=poison and k == 1) for k, c in enumerate(cases)]
        for r in runs:
            g.add(r)
        g.step(steps=steps)
        g.synchronize()
        assert all(f == 0 for f in g.check())
        out.append([_state(r) for r in runs])
        for r in runs:
            g.remove(r)
            r.close()
        g.close()
    for a, b in zip(out[0], out[1]):
        assert _same(a, b)


def test_canary_toggled_between_steps():
    case = (37, "f64", "nrbc", 6, 0, 2, 40)
    a = _make(*case, seed=3, poison=False)
    b = _make(*case, seed=3, poison=False)
    a.step(40)
    b.step(16)
    b.set_debug(lbm.LBM_DEBUG_POISON)   # the captured graph is recaptured with the canary
    b.step(16)
    b.set_debug(0)
    b.step(8)
    assert _same(_state(a), _state(b))
    a.close()
    b.close()
