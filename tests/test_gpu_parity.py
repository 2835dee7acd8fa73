"""GPU parity: the HIP library (through the C ABI) against the FP64 oracle, element by element.

Bar: FP64 storage matches to 1e-12 relative (rho, T relative to max |Z|; u relative to max |u|;
populations relative to their weight), or to 4x the oracle's own measured conditioning floor for
the case where that floor is higher (a floor above 1e-9 fails).  Cases span several tiles with ragged tails, every
boundary kind, PML on all or some sides, corners, mean flow, tiny grids and the full-size grids
in the launch configuration the benchmark times.
"""
import numpy as np
import pytest

from paper_2504_20169_amd import lbm
from paper_2504_20169_amd import workloads as wl
from _helpers import (TOL, assert_parity, make_pair, noise, oracle_self_sensitivity,
                      perm_lib_to_oracle, rel_errors, say)

pytestmark = pytest.mark.gpu


def test_plain_method_config(oracle_mod, perm):
    """64^2 bulk + 8-cell PML (80^2), quadratic ramp sigma_max = 0.1, ZG, rest state, Gaussian
    pulse A = 1e-3, b = 4 at the centre, 200 steps: the full workload, every node compared."""
    spec = wl.pulse_box(64, 8, 0.1, 200, "zg")
    say("case plain 80x80 ZG+PML 200 steps")
    case = dict(Lx=64, Ly=64, bc="zg", pml=(15, 8, 0.1), fields=spec.fields)
    g, o = make_pair(oracle_mod, **case)
    g.step(200)
    o.step(200)
    err = rel_errors(g, o, perm)
    say(err)
    assert_parity(err, oracle_mod, dict(case, steps=200))


@pytest.mark.parametrize("case", [
    dict(name="nrbc_pml_flow", Lx=70, Ly=45, bc="nrbc", pml=(15, 6, 0.05), mean=(1.0, 0.1, 0.0, 1.0), steps=80),
    dict(name="zg_pml_flow_diag", Lx=50, Ly=66, bc="zg", pml=(15, 5, 0.08), mean=(1.0, 0.05, -0.04, 1.0), steps=60),
    dict(name="periodic_ragged", Lx=67, Ly=61, bc="periodic", pml=None, mean=(1.0, 0.02, 0.01, 1.0), steps=100),
    dict(name="step_geometry", Lx=60, Ly=20, bc={"xmin": "nrbc", "xmax": "nrbc", "ymin": "periodic", "ymax": "periodic"},
         pml=(3, 10, 0.1), mean=(1.0, 0.05, 0.0, 1.0), steps=90),
    dict(name="mixed_sides", Lx=41, Ly=37, bc={"xmin": "zg", "xmax": "nrbc", "ymin": "nrbc", "ymax": "zg"},
         pml=(2 | 4, 5, 0.1), mean=(1.0, 0.06, 0.03, 1.02), steps=50),
    dict(name="tiny_open", Lx=7, Ly=7, bc="nrbc", pml=None, mean=(1.0, 0.0, 0.0, 1.0), steps=20),
    dict(name="tiny_periodic", Lx=3, Ly=5, bc="periodic", pml=None, mean=(1.0, 0.0, 0.0, 1.0), steps=20),
    dict(name="thin_pml_w1", Lx=30, Ly=28, bc="zg", pml=(15, 1, 0.1), mean=(1.0, 0.0, 0.0, 1.0), steps=40),
    dict(name="thin_pml_w2_nrbc", Lx=30, Ly=28, bc="nrbc", pml=(15, 2, 0.1), mean=(1.0, 0.03, 0.0, 1.0), steps=40),
    dict(name="x_periodic_y_open", Lx=33, Ly=40, bc={"xmin": "periodic", "xmax": "periodic", "ymin": "zg", "ymax": "nrbc"},
         pml=(4 | 8, 7, 0.05), mean=(1.0, 0.0, 0.04, 0.98), steps=60),
])
def test_parity_cases(oracle_mod, perm, case):
    say("case", case["name"])
    kw = dict(Lx=case["Lx"], Ly=case["Ly"], bc=case["bc"], pml=case["pml"], mean=case["mean"],
              fields=noise(11, case["mean"]))
    g, o = make_pair(oracle_mod, **kw)
    g.step(case["steps"])
    o.step(case["steps"])
    err = rel_errors(g, o, perm)
    say(case["name"], err)
    assert_parity(err, oracle_mod, dict(kw, steps=case["steps"]))


def test_vortex_pulse_workload_small(oracle_mod, perm):
    """The vortex + pulse workload (Mach 0.1, NRBC, PML) at a reduced bulk, 300 steps."""
    spec = wl.vortex_pulse(L=96, W=12, sigma_max=0.0015, mach=0.1, steps=300, bc="nrbc",
                           radius=8.0)
    say("case vortex_pulse 120^2 NRBC 300 steps")
    case = dict(Lx=96, Ly=96, bc="nrbc", pml=(15, 12, 0.0015), mean=(1.0, 0.1, 0.0, 1.0),
                fields=spec.fields)
    g, o = make_pair(oracle_mod, **case)
    g.step(300)
    o.step(300)
    err = rel_errors(g, o, perm)
    say(err)
    assert_parity(err, oracle_mod, dict(case, steps=300))


def test_moments_at_step_zero(oracle_mod, perm):
    case = dict(Lx=20, Ly=18, bc="nrbc", pml=(15, 3, 0.1), fields=noise(4))
    g, o = make_pair(oracle_mod, **case)
    assert_parity(rel_errors(g, o, perm), oracle_mod, dict(case, steps=0))


def test_pml_q_matches_oracle(oracle_mod, perm):
    """Q (eq. PMLQ) node by node, relative to max |Q|, within 1e-12 or 4x the oracle's own
    conditioning floor for this case if that is higher."""
    kw = dict(Lx=24, Ly=20, bc="nrbc", pml=(15, 5, 0.1), mean=(1.0, 0.05, 0.0, 1.0),
              fields=noise(5, (1.0, 0.05, 0.0, 1.0)))
    g, o = make_pair(oracle_mod, **kw)
    g.step(30)
    o.step(30)
    qg = g.pml_q()[perm]
    qo = o.pml_q()
    err = np.abs(qg - qo).max() / np.abs(qo).max()
    _, dq = oracle_self_sensitivity(oracle_mod, steps=30, **kw)
    say("Q rel err %.2e, conditioning floor %.2e" % (err, dq))
    assert err <= max(TOL, 4.0 * dq)
    assert dq < 1e-10  # the floor itself stays near rounding


@pytest.mark.parametrize("bc", ["zg", "nrbc"])
@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_sigma_zero_pml_bitwise_equals_plain(bc, storage):
    """sigma_max = 0 with W > 0 reproduces W = 0 on the same grid bit for bit."""
    W, L = 6, 40
    F = wl.noisy_state(L + 2 * W, L + 2 * W, 9, 1.0, 0.04, 0.0, 1.0)
    a = lbm.Run(L, L, 0.8, 1.0, 0.04, 0.0, 1.0, storage=storage)
    a.set_bc(15, bc)
    a.set_pml(15, W, 0.0)
    b = lbm.Run(L + 2 * W, L + 2 * W, 0.8, 1.0, 0.04, 0.0, 1.0, storage=storage)
    b.set_bc(15, bc)
    a.init(*F.as_tuple())
    b.init(*F.as_tuple())
    a.step(37)
    b.step(37)
    assert np.array_equal(a.populations(), b.populations())


def test_tile_shapes_graphs_and_overlap_bitwise_identical():
    """Tile shape, graph replay, the overlapped schedules (side stream; phase A fused with the
    bulk tiles) and the phase-A placement in the fused grid change launches, never bits."""
    F = wl.noisy_state(150, 140, 3, 1.0, 0.05, 0.0, 1.0)
    outs = []
    for tx, gs, ov, sp in ((64, 0, 0, -1), (128, 8, 0, -1), (256, 32, 0, -1), (64, 32, 0, -1),
                           (64, 0, 1, -1), (256, 8, 1, -1), (64, 0, 2, -1), (128, 8, 2, -1),
                           (256, 32, 2, -1), (64, 8, 2, 0), (64, 0, 2, 3), (128, 32, 2, 8)):
        r = lbm.Run(134, 124, 0.8, 1.0, 0.05, 0.0, 1.0)
        r.set_bc(15, "nrbc")
        r.set_pml(15, 8, 0.05)
        r.set_launch(bulk_tx=tx, graph_steps=gs, overlap=ov, split=sp)
        r.init(*F.as_tuple())
        r.step(41)
        outs.append(r.populations())
    for o in outs[1:]:
        assert np.array_equal(outs[0], o)


def test_profile_modes_count_launches_and_keep_bits():
    """Event timing in any mode changes the launch schedule, never the result."""
    F = wl.noisy_state(150, 140, 3, 1.0, 0.05, 0.0, 1.0)
    outs = []
    for mode, ov in ((0, 0), (1, 0), (2, 0), (2, 1), (3, 0), (1, 2), (2, 2), (3, 2)):
        r = lbm.Run(134, 124, 0.8, 1.0, 0.05, 0.0, 1.0)
        r.set_bc(15, "nrbc")
        r.set_pml(15, 8, 0.05)
        r.set_launch(graph_steps=8, overlap=ov)
        r.init(*F.as_tuple())
        r.profile(mode)
        r.step(23)
        ms, n = r.profile_read(reset=True)
        # mode 2: the step grid and the frame kernel of every step; mode 3: of every fourth
        # step of each batch of 8 (batches of 8, 8 and 7 steps: sub-steps 0 and 4 of each)
        expect = {0: [0, 0, 0], 1: [23, 23, 23], 2: [23, 23, 0], 3: [6, 6, 0]}[mode]
        assert list(n) == expect, (mode, n)
        assert all(m > 0 for m, c in zip(ms, n) if c)
        with pytest.raises(lbm.LbmError):
            r.profile(4)
        outs.append(r.populations())
        r.close()
    for o in outs[1:]:
        assert np.array_equal(outs[0], o)


def test_autotune_choice_is_valid_cached_and_keeps_bits(tmp_path):
    F = wl.noisy_state(106, 96, 4, 1.0, 0.05, 0.0, 1.0)
    cache = str(tmp_path / "tune.txt")

    def make():
        r = lbm.Run(90, 80, 0.8, 1.0, 0.05, 0.0, 1.0)
        r.set_bc(15, "nrbc")
        r.set_pml(15, 8, 0.05)
        r.init(*F.as_tuple())
        return r

    ref = make()
    ref.step(19)
    a = make()
    c = a.autotune(steps=4, cache_path=cache)
    assert c["bulk_tx"] in (64, 128, 256) and c["overlap"] in (0, 1, 2)
    lines = open(cache).read().split("\n")
    assert lines[0].split() == ["106", "96", "0", "37", str(c["bulk_tx"]), str(c["overlap"]),
                                str(c["split"])]
    assert (c["split"] in (0, 2, 4, 6, 8)) == (c["overlap"] == 2)
    a.step(19)
    assert np.array_equal(a.populations(), ref.populations())
    b = make()
    assert b.autotune(steps=4, cache_path=cache) == c      # read back, no new line
    assert len([l for l in open(cache).read().split("\n") if l]) == 1
    for r in (ref, a, b):
        r.close()


def test_conservation_on_gpu():
    e, w, rr = lbm.lbm_velocities()
    xi = rr * e.astype(float)
    r = lbm.Run(130, 70, 0.8)
    r.init(*wl.noisy_state(130, 70, 8, 1.0, 0.03, -0.02, 1.0, amp=2e-3).as_tuple())

    def cons():
        f = r.populations().sum(axis=(1, 2))
        return np.array([f.sum(), (f * xi[:, 0]).sum(), (f * xi[:, 1]).sum(), (f * (xi ** 2).sum(1)).sum()])

    c0 = cons()
    r.step(500)
    c1 = cons()
    assert np.all(np.abs(c1 - c0) <= 1e-12 * np.abs(c0).max()), c1 - c0


def test_error_norms_match_oracle(oracle_mod, perm):
    mean = (1.0, 0.05, 0.0, 1.0)
    g, o = make_pair(oracle_mod, 30, 26, bc="nrbc", pml=(15, 4, 0.1), mean=mean, fields=noise(6, mean))
    g.step(25)
    o.step(25)
    ref = wl.noisy_state(30, 26, 99, *mean)
    eg = g.error_norms(ref.rho, ref.ux, ref.T)
    eo = o.error_norms(ref.rho, ref.ux, ref.T)
    assert np.allclose(eg, eo, rtol=1e-12, atol=0)


def test_check_flags_blow_up_and_passes_stable():
    r = lbm.Run(40, 40, 0.8)
    r.set_bc(15, "zg")
    r.set_pml(15, 8, 50.0)  # host-chosen absurd absorption: the state overflows to inf/nan
    r.init(*wl.noisy_state(56, 56, 1).as_tuple())
    assert r.check() == lbm.LBM_OK
    r.step(200)
    assert r.check() == lbm.LBM_ERR_UNSTABLE


def test_check_interval_stops_a_blow_up_and_keeps_stable_bits():
    """With a check interval lbm_step scans the state every K steps: the absurd-absorption run
    stops at the first failing chunk with LBM_ERR_UNSTABLE, and a stable run gives the bits of
    the run stepped without checks."""
    r = lbm.Run(40, 40, 0.8)
    r.set_bc(15, "zg")
    r.set_pml(15, 8, 50.0)
    r.init(*wl.noisy_state(56, 56, 1).as_tuple())
    r.set_check_interval(10)
    with pytest.raises(lbm.LbmError) as ei:
        r.step(200)
    assert ei.value.status == lbm.LBM_ERR_UNSTABLE
    n = r.step_count
    assert 0 < n < 200 and n % 10 == 0, n
    out = []
    for every in (0, 32, 7):
        s = lbm.Run(50, 44, 0.8, 1.0, 0.05, 0.0, 1.0)
        s.set_bc(15, "nrbc")
        s.set_pml(15, 6, 0.05)
        s.init(*wl.noisy_state(62, 56, 3, 1.0, 0.05, 0.0, 1.0).as_tuple())
        s.set_check_interval(every)
        s.step(75)
        assert s.step_count == 75
        out.append(s.populations())
        s.close()
    assert all(np.array_equal(out[0], o) for o in out[1:])


def test_checkpoint_roundtrip_bitwise(tmp_path):
    def make():
        r = lbm.Run(60, 50, 0.8, 1.0, 0.05, 0.0, 1.0)
        r.set_bc(15, "nrbc")
        r.set_pml(15, 6, 0.05)
        r.init(*wl.noisy_state(72, 62, 2, 1.0, 0.05, 0.0, 1.0).as_tuple())
        return r
    a = make()
    a.step(30)
    b = make()
    b.step(12)
    b.save(tmp_path / "ck.bin")
    c = make()
    c.load(tmp_path / "ck.bin")
    c.step(18)
    assert c.step_count == 30
    assert np.array_equal(a.populations(), c.populations())
    assert all(np.array_equal(x, y) for x, y in zip(a.moments(), c.moments()))


def test_checkpoint_refuses_foreign_files(tmp_path):
    """A checkpoint with a flipped payload byte, of another format version, cut short, or written
    by a differently configured run is refused with LBM_ERR_ARG, and the refused load leaves the
    handle's state as it was."""
    def make(W=6):
        r = lbm.Run(60, 50, 0.8, 1.0, 0.05, 0.0, 1.0)
        r.set_bc(15, "nrbc")
        r.set_pml(15, W, 0.05)
        r.init(*wl.noisy_state(60 + 2 * W, 50 + 2 * W, 2, 1.0, 0.05, 0.0, 1.0).as_tuple())
        return r
    a = make()
    a.step(7)
    good = tmp_path / "ck.bin"
    a.save(good)
    raw = good.read_bytes()
    c = make()
    c.step(3)
    before = c.populations()
    flipped = bytearray(raw)
    flipped[-1] ^= 0x01
    cases = {"checksum": bytes(flipped), "not a checkpoint": b"LBMPML04" + raw[8:],
             "truncated": raw[:-8]}
    for what, data in cases.items():
        say("case checkpoint refused:", what)
        path = tmp_path / ("bad_%s.bin" % what.replace(" ", "_"))
        path.write_bytes(data)
        with pytest.raises(lbm.LbmError) as ei:
            c.load(path)
        assert ei.value.status == lbm.LBM_ERR_ARG and what in str(ei.value), str(ei.value)
        assert c.step_count == 3 and np.array_equal(c.populations(), before)
    other = make(W=5)
    with pytest.raises(lbm.LbmError) as ei:
        other.load(good)
    assert ei.value.status == lbm.LBM_ERR_ARG and "differs" in str(ei.value)
    c.load(good)
    assert c.step_count == 7 and np.array_equal(c.populations(), a.populations())


@pytest.mark.parametrize("which", ["vortex_1088", "pulses_4224", "pulses_4224_nrbc"])
def test_full_size_grids_in_bench_launch(oracle_mod, perm, which):
    """The full grids of the benchmark workloads (1024^2 + 32 PML with NRBC; 4096^2 + 64 PML with
    ZG and with NRBC), default launch configuration, noisy state so every node and path is
    distinct; a few steps compared node by node (moments everywhere; populations on the smaller
    grid)."""
    if which == "vortex_1088":
        L, W, bc, sig, mean, steps = 1024, 32, "nrbc", 0.0015, (1.0, 0.1, 0.0, 1.0), 4
    elif which == "pulses_4224":
        L, W, bc, sig, mean, steps = 4096, 64, "zg", 0.01, (1.0, 0.05, 0.0, 1.0), 2
    else:
        L, W, bc, sig, mean, steps = 4096, 64, "nrbc", 0.01, (1.0, 0.05, 0.0, 1.0), 2
    say("case full", which)
    g, o = make_pair(oracle_mod, L, L, bc=bc, pml=(15, W, sig), mean=mean,
                     fields=noise(21, mean, 5e-4))
    g.step(steps)
    o.step(steps)
    err = rel_errors(g, o, perm, with_f=(which == "vortex_1088"))
    say(which, err)
    assert_parity(err)


def test_torch_stream_and_allocator_interop():
    """Device memory from PyTorch's caching allocator and work on a PyTorch stream: same bits
    as the library's own stream and hipMalloc; moments can land in torch tensors."""
    import torch

    if not torch.cuda.is_available():
        pytest.skip("PyTorch in this process sees no HIP device")
    F = wl.noisy_state(60, 56, 12, 1.0, 0.05, 0.0, 1.0)
    outs = []
    for use_torch in (False, True):
        ts = torch.cuda.Stream()
        kw = dict(stream=ts, allocator=lbm.torch_allocator(ts)) if use_torch else {}
        r = lbm.Run(48, 44, 0.8, 1.0, 0.05, 0.0, 1.0, **kw)
        r.set_bc(15, "nrbc")
        r.set_pml(15, 6, 0.05)
        r.init(*F.as_tuple())
        r.step(70)
        outs.append(r.populations())
        if use_torch:
            rho = torch.empty((56, 60), dtype=torch.float64, device="cuda")
            r.moments_device(rho=rho.data_ptr())
            r.synchronize()
            assert np.array_equal(rho.cpu().numpy(), r.moments()[0])
        r.close()
    assert np.array_equal(outs[0], outs[1])


@pytest.mark.parametrize("bind", [True, False])
def test_torch_allocator_blocks_freed_under_pending_work(bind):
    """Blocks the caching allocator hands to the library may have been freed by work still queued
    on the default stream: the run (on a side stream) must not race with that work.  Queue a long
    chain of kernels on the default stream over tensors, free them, then create and step a run on a
    side stream with the torch allocator (bound to that stream, or synchronising the current one):
    bitwise the result of the library's own allocations."""
    import torch

    if not torch.cuda.is_available():
        pytest.skip("PyTorch in this process sees no HIP device")
    F = wl.noisy_state(60, 56, 12, 1.0, 0.05, 0.0, 1.0)

    def run(**kw):
        r = lbm.Run(48, 44, 0.8, 1.0, 0.05, 0.0, 1.0, **kw)
        r.set_bc(15, "nrbc")
        r.set_pml(15, 6, 0.05)
        r.init(*F.as_tuple())
        r.step(40)
        out = r.populations()
        r.close()
        return out

    ref = run()
    torch.cuda.synchronize()
    bufs = [torch.ones(1 << 20, dtype=torch.float64, device="cuda") for _ in range(8)]
    for _ in range(200):                 # pending work on the default stream
        for b in bufs:
            b.mul_(1.0000001).add_(1e-9)
    del bufs                             # blocks back in the cache while that work is queued
    ts = torch.cuda.Stream()
    got = run(stream=ts, allocator=lbm.torch_allocator(ts if bind else None))
    torch.cuda.synchronize()
    assert np.array_equal(ref, got)


@pytest.mark.parametrize("storage", ["f64", "f16"])
def test_population_layouts_bitwise_identical(oracle_mod, perm, storage):
    """The row-interleaved layout (default, any row padding) and one plane per velocity give the
    same bits; the row layout also matches the oracle."""
    mean = (1.0, 0.05, 0.0, 1.0)
    F = wl.noisy_state(86, 74, 14, *mean)
    outs = []
    for layout, pad in ((0, 0), (1, 0), (0, -1), (0, 40)):
        r = lbm.Run(70, 58, 0.8, *mean, storage=storage, layout=layout, row_pad=pad)
        r.set_bc(15, "nrbc")
        r.set_pml(15, 8, 0.05)
        r.init(*F.as_tuple())
        r.step(45)
        outs.append((r.populations(), r.moments()))
    for o in outs[1:]:
        assert np.array_equal(outs[0][0], o[0])
    if storage == "f64":
        o = oracle_mod.OracleRun(70, 58, 0.8, *mean)
        o.set_bc(15, 2)
        o.set_pml(15, 8, 0.05)
        o.init(*F.as_tuple())
        o.step(45)
        mo = o.moments()
        assert max(np.abs(a - b).max() for a, b in zip(outs[0][1], mo)) < 1e-12


@pytest.mark.parametrize("flags", [1, 2, 4, 7])
def test_nrbc_pml_terms_match_oracle(oracle_mod, perm, flags):
    """Appendix terms in the characteristic target: FP64 library vs oracle on noisy data with an
    NRBC behind a PML on every side (sigma_max = 0.01, 30 steps)."""
    mean = (1.0, 0.05, 0.02, 1.0)
    case = dict(Lx=44, Ly=38, mean=mean, bc="nrbc", pml=(15, 7, 0.01), fields=noise(9, mean),
                pml_terms=flags)
    g, o = make_pair(oracle_mod, **case)
    g.step(30)
    o.step(30)
    e = rel_errors(g, o, perm)
    say(flags, e)
    assert_parity(e, oracle_mod, dict(case, steps=30))
    g.close()
