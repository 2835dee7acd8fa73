"""Batched runs and the serving loop on the GPU: every run's result is bitwise the same alone,
in a batch of uneven runs, and in the served mix, and matches the FP64 oracle (FP64 members to
the 1e-12 bar, FP32 within 1e-6, FP16 within 3% of the field's perturbation); FP32/FP16 storage
errors against the oracle."""
import numpy as np
import pytest

from paper_2504_20169_amd import lbm
from paper_2504_20169_amd import workloads as wl
from paper_2504_20169_amd.serve import Engine, GpuBackend, Job
from _helpers import TOL, make_pair, say

pytestmark = pytest.mark.gpu

CASES = [  # (L, W, bc, steps)
    (48, 0, "zg", 37), (64, 8, "nrbc", 51), (40, 4, "zg", 20), (72, 16, "nrbc", 45), (33, 5, "nrbc", 1),
]


def _make(L, W, bc, storage, seed):
    spec = wl.vortex_pulse(L=L, W=W, sigma_max=0.01, mach=0.1, bc=bc, seed=seed, radius=6.0)
    r = lbm.Run(L, L, 0.8, 1.0, 0.1, 0.0, 1.0, storage=storage)
    r.set_bc(lbm.LBM_ALL, bc)
    if W:
        r.set_pml(lbm.LBM_ALL, W, 0.01)
    r.init(*spec.fields.as_tuple())
    return r


def _oracle_moments(oracle_mod, L, W, bc, seed, steps, sigma_max=0.01, radius=6.0, mean=(1.0, 0.1, 0.0, 1.0)):
    """The FP64 oracle's moments for the run that _make (or the serving backend) builds."""
    spec = wl.vortex_pulse(L=L, W=W, sigma_max=sigma_max, mach=mean[1], bc=bc, seed=seed, radius=radius)
    o = oracle_mod.OracleRun(L, L, 0.8, *mean)
    o.set_bc(15, {"zg": 1, "nrbc": 2}[bc])
    if W:
        o.set_pml(15, W, sigma_max)
    o.init(*spec.fields.as_tuple())
    o.step(steps)
    return o.moments()


# Bars against the oracle by storage: FP64 the parity bar (rho, T relative to max |Z|, u to
# max |u|); FP32 1e-6 on the same scales; FP16 (11-bit significand on the stored deviations)
# relative to each field's perturbation max |Z - Z_mean|, so a lost or zeroed signal fails.
ORACLE_BAR = {"f64": TOL, "f32": 1e-6, "f16": 3e-2}


def _oracle_errors(m, mo, storage, mean=(1.0, 0.1, 0.0, 1.0)):
    us = max(np.abs(mo[1]).max(), np.abs(mo[2]).max())
    if storage == "f16":
        sc = [np.abs(mo[0] - mean[0]).max(), np.abs(mo[1] - mean[1]).max(),
              np.abs(mo[2] - mean[2]).max(), np.abs(mo[3] - mean[3]).max()]
        su = max(sc[1], sc[2])
        sc = [sc[0], su, su, sc[3]]
    else:
        sc = [np.abs(mo[0]).max(), us, us, np.abs(mo[3]).max()]
    return {k: float(np.abs(a - b).max() / s) for k, a, b, s in zip(("rho", "ux", "uy", "T"), m, mo, sc)}


def _check_against_oracle(oracle_mod, r, L, W, bc, seed, steps, storage, **kw):
    mo = _oracle_moments(oracle_mod, L, W, bc, seed, steps, **kw)
    e = _oracle_errors(r.moments(), mo, storage)
    say("vs oracle", storage, (L, W, bc, steps), {k: "%.2e" % v for k, v in e.items()})
    assert all(v <= ORACLE_BAR[storage] for v in e.values()), (storage, L, W, bc, e)


@pytest.mark.parametrize("storage", ["f64", "f32", "f16"])
def test_batch_equals_alone(oracle_mod, storage):
    alone = []
    for k, (L, W, bc, n) in enumerate(CASES):
        r = _make(L, W, bc, storage, 40 + k)
        r.step(n)
        alone.append(r.populations())
        r.close()
    g = lbm.Group()
    runs = [_make(L, W, bc, storage, 40 + k) for k, (L, W, bc, n) in enumerate(CASES)]
    for r in runs:
        g.add(r)
    steps = np.array([c[3] for c in CASES])
    g.step(steps=steps // 2)
    g.step(steps=steps - steps // 2)
    g.synchronize()
    for k, (r, a, c) in enumerate(zip(runs, alone, CASES)):
        assert r.step_count == c[3]
        assert np.array_equal(r.populations(), a), c
        _check_against_oracle(oracle_mod, r, c[0], c[1], c[2], 40 + k, c[3], storage)
    # remove one member mid-way; the others continue identically
    g.remove(runs[1])
    g.step(nsteps=3)
    for k in (0, 2, 3, 4):
        assert runs[k].step_count == CASES[k][3] + 3
    g.close()


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_batch_of_degenerate_frames_equals_alone(storage):
    """Runs whose characteristic ring covers nearly the whole grid (7x7 and 8x8 with the LODI
    boundary on every side: the frame off the ring is one node, or none), with a PML one cell
    wide, and a plain ZG run, advanced in one group: bitwise the runs stepped alone."""
    cases = [(7, 0, "nrbc", 9), (8, 0, "nrbc", 6), (9, 1, "nrbc", 7), (7, 0, "zg", 5)]
    alone = []
    for k, (L, W, bc, n) in enumerate(cases):
        say("case degenerate frame alone", storage, (L, W, bc, n))
        r = _make(L, W, bc, storage, 70 + k)
        r.step(n)
        alone.append(r.populations())
        r.close()
    g = lbm.Group()
    runs = [_make(L, W, bc, storage, 70 + k) for k, (L, W, bc, n) in enumerate(cases)]
    for r in runs:
        g.add(r)
    g.step(steps=np.array([c[3] for c in cases]))
    g.synchronize()
    for r, a, c in zip(runs, alone, cases):
        assert r.step_count == c[3] and r.check() == lbm.LBM_OK, c
        assert np.array_equal(r.populations(), a), c
    g.close()


@pytest.mark.parametrize("gs", [0, 8])
def test_batch_fused_schedule_equals_alone(oracle_mod, gs):
    """Phase A fused with the bulk tiles in one grid per step (eager and in graphs), over a batch
    of uneven runs with and without rings and PMLs: bitwise the runs alone."""
    alone = []
    for k, (L, W, bc, n) in enumerate(CASES):
        r = _make(L, W, bc, "f64", 70 + k)
        r.step(n)
        alone.append(r.populations())
        r.close()
    g = lbm.Group()
    runs = [_make(L, W, bc, "f64", 70 + k) for k, (L, W, bc, n) in enumerate(CASES)]
    for r in runs:
        g.add(r)
    g.set_launch(bulk_tx=64, graph_steps=gs, overlap=2)
    assert g.get_launch()["overlap"] == 2
    g.step(steps=np.array([c[3] for c in CASES]))
    g.synchronize()
    for k, (r, a, c) in enumerate(zip(runs, alone, CASES)):
        assert np.array_equal(r.populations(), a), c
        _check_against_oracle(oracle_mod, r, c[0], c[1], c[2], 70 + k, c[3], "f64")
    g.close()


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_group_graphs_and_autotune_keep_bits(storage):
    """Graph replays of batched steps (uneven counts, membership change in between) and the
    group autotuner change launches, never results."""
    alone = []
    for k, (L, W, bc, n) in enumerate(CASES):
        r = _make(L, W, bc, storage, 60 + k)
        r.step(n + 9)
        alone.append(r.populations())
        r.close()
    g = lbm.Group()
    runs = [_make(L, W, bc, storage, 60 + k) for k, (L, W, bc, n) in enumerate(CASES)]
    for r in runs:
        g.add(r)
    with pytest.raises(lbm.LbmError):
        g.set_launch(bulk_tx=64, graph_steps=3)
    with pytest.raises(lbm.LbmError):
        g.set_launch(bulk_tx=64, graph_steps=4, overlap=1)   # one stream: no side stream
    g.set_launch(bulk_tx=128, graph_steps=4)
    assert g.get_launch() == dict(bulk_tx=128, bulk_ty=2, graph_steps=4, overlap=2, split=-1)
    with pytest.raises(lbm.LbmError):
        g.set_launch(bulk_tx=128, graph_steps=4, split=9)
    before = [r.populations() for r in runs]
    c = g.autotune(steps=3)
    assert c["bulk_tx"] in (64, 128, 256) and c["graph_steps"] == 4
    for r, b in zip(runs, before):          # scratch runs only: members untouched
        assert np.array_equal(r.populations(), b)
    steps = np.array([c[3] for c in CASES])
    g.step(steps=steps)                     # graphs of 4 batched steps, uneven counts
    extra = runs.pop(2)
    g.remove(extra)                         # membership change: graph recaptured
    extra.step(9)
    g.step(nsteps=9)
    g.synchronize()
    runs.insert(2, extra)
    for r, a, cs in zip(runs, alone, CASES):
        assert r.step_count == cs[3] + 9
        assert np.array_equal(r.populations(), a), cs
    g.close()
    for r in runs:
        r.close()


def test_served_results_equal_alone(oracle_mod):
    """Jobs arriving while others are on the GPU give bitwise the same moments as alone, and
    those moments match the FP64 oracle within the FP32 bar; a job forced unstable from the host
    is retired as failed without disturbing the rest."""
    jobs = [Job(jid=k, L=L, W=W, steps=n * 7, bc=bc, seed=100 + k, sigma_max=0.01, arrival=0.01 * k)
            for k, (L, W, bc, n) in enumerate(CASES)]
    bad = Job(jid=99, L=40, W=6, steps=300, bc="zg", seed=7, sigma_max=80.0, arrival=0.0)
    be = GpuBackend(storage="f32")
    eng = Engine(be, hbm_budget=int(1e9), tick_steps=16)
    rep = eng.run_trace(jobs + [bad], realtime=False)
    be.close()
    say(rep)
    st = {j.jid: j.status for j in eng.finished}
    assert st[99] == "failed"
    for j in eng.finished:
        if j.jid == 99:
            continue
        assert j.status == "done"
        ref = GpuBackend(storage="f32")
        r = ref.start(Job(jid=j.jid, L=j.L, W=j.W, steps=j.steps, bc=j.bc, seed=j.seed, sigma_max=0.01))
        ref.group.remove(r)
        r.step(j.steps)
        rho, ux, uy, T = r.moments()
        r.close()
        ref.close()
        assert np.array_equal(rho, j.result["rho"]) and np.array_equal(ux, j.result["ux"])
        assert np.array_equal(T, j.result["T"])
        mo = _oracle_moments(oracle_mod, j.L, j.W, j.bc, j.seed, j.steps, sigma_max=0.01,
                             radius=min(16.0, j.L / 8.0))
        e = _oracle_errors([j.result["rho"], j.result["ux"], j.result["uy"], j.result["T"]], mo, "f32")
        say("served job", j.jid, "vs oracle", {k: "%.2e" % v for k, v in e.items()})
        assert all(v <= ORACLE_BAR["f32"] for v in e.values()), (j.jid, e)


@pytest.mark.parametrize("storage", ["f32", "f16"])
def test_reduced_storage_error_vs_oracle(oracle_mod, storage):
    """FP32 / FP16 deviation storage against the FP64 oracle on the vortex + pulse workload
    (reduced bulk, Mach 0.1, NRBC + PML), 400 steps.  FP32: within 1e-6 relative as in the FP64
    parity.  FP16: within 3% of each field's perturbation (a zeroed signal gives 1)."""
    spec = wl.vortex_pulse(L=96, W=12, sigma_max=0.0015, mach=0.1, bc="nrbc", radius=8.0)
    g, o = make_pair(oracle_mod, 96, 96, bc="nrbc", pml=(15, 12, 0.0015), mean=(1.0, 0.1, 0.0, 1.0),
                     fields=spec.fields, storage=storage)
    g.step(400)
    o.step(400)
    e = _oracle_errors(g.moments(), o.moments(), storage)
    say(storage, {k: "%.2e" % v for k, v in e.items()})
    assert all(v <= ORACLE_BAR[storage] for v in e.values()), e


@pytest.mark.parametrize("lattice", [37, 17])
def test_full_length_vortex_workload_stays_stable(lattice):
    """The benchmark workload (1024^2 bulk + 32-cell PML, NRBC, Mach 0.1 vortex + pulse) over
    its full 10^4 steps in every storage: every run stays finite and positive, FP32 deviation
    storage stays within 1e-6 of FP64 and FP16 within 1e-4 (relative to max |Z|; u relative to
    max |u|; measured 8.2e-7 and 1.1e-5 at most, on D2Q17's velocity)."""
    spec = wl.vortex_pulse(L=1024, W=32, sigma_max=0.0015, mach=0.1, bc="nrbc")
    out = {}
    for storage in ("f64", "f32", "f16"):
        r = lbm.Run(1024, 1024, 0.8, 1.0, 0.1, 0.0, 1.0, storage=storage, lattice=lattice)
        r.set_bc(lbm.LBM_ALL, "nrbc")
        r.set_pml(lbm.LBM_ALL, 32, 0.0015)
        r.init(*spec.fields.as_tuple())
        r.step(10000)
        assert r.check() == lbm.LBM_OK, storage
        out[storage] = r.moments()
        r.close()
    ref = out["f64"]
    us = max(np.abs(ref[1]).max(), np.abs(ref[2]).max())
    for storage, tol in (("f32", 1e-6), ("f16", 1e-4)):
        m = out[storage]
        e = dict(rho=np.abs(m[0] - ref[0]).max() / np.abs(ref[0]).max(),
                 u=max(np.abs(m[1] - ref[1]).max(), np.abs(m[2] - ref[2]).max()) / us,
                 T=np.abs(m[3] - ref[3]).max() / np.abs(ref[3]).max())
        say(lattice, storage, {k: "%.2e" % v for k, v in e.items()})
        assert all(v < tol for v in e.values()), (storage, e)
