"""The C-ABI library loads, exports every symbol include/lbm.h declares, and validates its
arguments on the host (no device work in these tests)."""
import os
import re
import subprocess
import sys

import numpy as np
import pytest

from paper_2504_20169_amd import lbm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "lbm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(lbm_[a-z_]+)\s*\(", src)))


def test_header_symbols_exported():
    lib = lbm.load()
    names = _declared()
    assert len(names) >= 30
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(lbm.EXPORTED) == names
    assert lbm.lbm_build_flags() == 0


def test_bounds_checked_build_exports_the_same_abi():
    """The bounds-checked debug build (built beside the library) exports every declared symbol
    and says which build it is (a host-only call)."""
    import ctypes
    if not os.path.exists(lbm.BOUNDS_LIB_PATH):
        pytest.skip("bounds-checked build not built")
    lib = ctypes.CDLL(lbm.BOUNDS_LIB_PATH)
    for n in _declared():
        assert hasattr(lib, n), n
    lib.lbm_build_flags.restype = ctypes.c_int32
    assert lib.lbm_build_flags() == lbm.LBM_BUILD_BOUNDS


@pytest.mark.parametrize("q", [37, 17, 9])
def test_velocity_table_matches_oracle(oracle_mod, q):
    e, w, r = lbm.lbm_velocities(q)
    eo, wo, ro = oracle_mod.lattice(q)
    assert abs(r - ro) < 1e-15
    lib = {(int(a), int(b)): wi for (a, b), wi in zip(e, w)}
    orc = {(int(a), int(b)): wi for (a, b), wi in zip(eo, wo)}
    assert set(lib) == set(orc)
    for k in lib:
        assert abs(lib[k] - orc[k]) <= 1e-16 + 1e-14 * orc[k]
    # library order: rest first, then +e/-e pairs
    assert tuple(e[0]) == (0, 0)
    for p in range((q - 1) // 2):
        assert tuple(e[1 + 2 * p]) == tuple(-e[2 + 2 * p])


def test_velocity_table_rejects_other_stencils():
    for bad in (5, 19, -1):
        with pytest.raises(lbm.LbmError):
            lbm.lbm_velocities(bad)
        assert lbm.load().lbm_velocities(bad, None, None, None) == lbm.LBM_ERR_ARG
    for ok in (0, 37, 17, 9):
        assert lbm.load().lbm_velocities(ok, None, None, None) == lbm.LBM_OK


@pytest.mark.parametrize("kw", [dict(tau=0.5), dict(tau=0.3), dict(nx=0), dict(ny=-1),
                                dict(rho0=0.0), dict(T0=-1.0), dict(storage=7),
                                dict(rho0=float("nan")), dict(storage="f16", f16_scale=3.0),
                                dict(layout=2), dict(row_pad=-2), dict(row_pad=5000),
                                dict(lattice=5), dict(lattice=-1)])
def test_create_rejects_bad_descriptor(kw):
    args = dict(nx=16, ny=16, tau=0.8)
    args.update(kw)
    with pytest.raises(lbm.LbmError) as ei:
        lbm.Run(**args)
    assert ei.value.status == lbm.LBM_ERR_ARG


def test_setters_validate_and_grid():
    r = lbm.Run(20, 10, 0.8)
    with pytest.raises(lbm.LbmError):
        r.set_pml(lbm.LBM_ALL, -1, 0.1)
    with pytest.raises(lbm.LbmError):
        r.set_pml(lbm.LBM_ALL, 4, -0.1)
    with pytest.raises(lbm.LbmError):
        r.set_bc(16, "zg")
    r.set_bc(lbm.LBM_ALL, "zg")
    r.set_pml(lbm.LBM_XMIN | lbm.LBM_YMAX, 5, 0.1)
    assert r.grid() == (25, 15)
    assert r.footprint() > 2 * 37 * 25 * 15 * 8
    with pytest.raises(lbm.LbmError) as ei:
        r.step(1)
    assert ei.value.status == lbm.LBM_ERR_STATE


def test_debug_flags_validated_on_host():
    r = lbm.Run(20, 10, 0.8)
    r.set_debug(lbm.LBM_DEBUG_POISON | lbm.LBM_DEBUG_RANGES)
    r.set_debug(0)
    with pytest.raises(lbm.LbmError) as ei:
        r.set_debug(4)
    assert ei.value.status == lbm.LBM_ERR_ARG
    r.set_check_interval(64)
    r.set_check_interval(0)
    with pytest.raises(lbm.LbmError) as ei:
        r.set_check_interval(-1)
    assert ei.value.status == lbm.LBM_ERR_ARG
    r.close()


def test_grid_size_limits():
    """Grids of up to 2^30 nodes are accepted.  A larger grid, or a frame whose Q and U planes
    would pass the 32-bit byte offsets the kernels use (4 GiB per plane), is refused with
    LBM_ERR_ARG when the geometry is set up, before any device memory is touched."""
    r = lbm.Run(32768, 32768, 0.8)                     # exactly 2^30 nodes
    assert r.footprint() > 2 * 37 * 2 ** 30 * 8
    with pytest.raises(lbm.LbmError) as ei:
        lbm.Run(32768, 32769, 0.8).footprint()
    assert ei.value.status == lbm.LBM_ERR_ARG and "too large" in str(ei.value)
    r = lbm.Run(1, 1, 0.8)                             # 32001^2 nodes, all of them frame
    r.set_bc(lbm.LBM_ALL, "zg")
    r.set_pml(lbm.LBM_ALL, 16000, 0.1)
    assert r.grid() == (32001, 32001)
    with pytest.raises(lbm.LbmError) as ei:
        r.footprint()
    assert ei.value.status == lbm.LBM_ERR_ARG and "frame arrays" in str(ei.value)
    r.set_pml(lbm.LBM_ALL, 8000, 0.1)                  # 16001^2: the frame fits
    assert r.footprint() > 2 * 37 * 16001 ** 2 * 8


@pytest.mark.parametrize("q", [37, 17, 9])
def test_cbc_a_kind_and_footprint(q):
    """CBC (A) is boundary kind 3; another kind is refused.  Its targets are formed ahead of the
    fill, so a run with a CBC (A) side holds four float64 target planes of the ring more than the
    same run with the LODI boundary."""
    def run(kind):
        r = lbm.Run(40, 30, 0.8, lattice=q)
        r.set_bc(lbm.LBM_ALL, "nrbc")
        r.set_bc(lbm.LBM_XMAX, kind)
        return r
    with pytest.raises(lbm.LbmError) as ei:
        lbm.Run(40, 30, 0.8, lattice=q).set_bc(lbm.LBM_XMAX, 4)
    assert ei.value.status == lbm.LBM_ERR_ARG
    a, b = run("nrbc_a"), run("nrbc")
    assert a.grid() == b.grid() == (40, 30)
    ring = 2 * 3 * 40 + (30 - 6) * 2 * 3                  # 3 layers on every side
    rplane = (ring + 63) // 64 * 64
    assert a.footprint() - b.footprint() == 4 * rplane * 8
    # the stencil sets the population count of every buffer
    for other in (37, 17, 9):
        c = lbm.Run(40, 30, 0.8, lattice=other)
        c.set_bc(lbm.LBM_ALL, "nrbc")
        assert c.q == other
        assert (c.footprint() > b.footprint()) == (other > q)


def test_launch_configuration_validated_on_host():
    r = lbm.Run(20, 10, 0.8)
    assert r.get_launch() == dict(bulk_tx=64, bulk_ty=4, graph_steps=32, overlap=2, split=-1)
    for kw in (dict(bulk_tx=32), dict(graph_steps=3), dict(graph_steps=-2), dict(overlap=3),
               dict(overlap=-1), dict(split=-2), dict(split=9)):
        with pytest.raises(lbm.LbmError) as ei:
            r.set_launch(**kw)
        assert ei.value.status == lbm.LBM_ERR_ARG, kw
    r.set_launch(bulk_tx=128, graph_steps=8, overlap=2, split=3)
    assert r.get_launch() == dict(bulk_tx=128, bulk_ty=2, graph_steps=8, overlap=2, split=3)
    r.set_launch(bulk_tx=256, graph_steps=0, overlap=1)
    with pytest.raises(lbm.LbmError) as ei:
        r.set_nrbc_pml_terms(8)
    assert ei.value.status == lbm.LBM_ERR_ARG
    r.set_nrbc_pml_terms(5)
    assert r.get_launch() == dict(bulk_tx=256, bulk_ty=1, graph_steps=0, overlap=1, split=-1)
    with pytest.raises(lbm.LbmError):
        r.profile(4)
    r.profile(3)
    r.profile(2)
    r.profile(0)


def test_row_padding_in_footprint():
    """Population rows are padded by 64 elements by default for FP64/FP32 storage, not FP16."""
    def fp(**kw):
        r = lbm.Run(100, 50, 0.8, **kw)
        return r.footprint()
    rows = 2 * 37 * 50  # two buffers x 37 population rows per grid row x Ny
    assert fp(row_pad=0) - fp(row_pad=-1) == rows * 64 * 8
    assert fp(row_pad=10) - fp(row_pad=-1) == rows * 10 * 8
    assert fp(storage="f32") - fp(storage="f32", row_pad=-1) == rows * 64 * 4
    assert fp(storage="f16") == fp(storage="f16", row_pad=-1)
    assert fp(layout=1, row_pad=10) == fp(layout=1, row_pad=-1)


def test_init_rejects_inconsistent_configuration():
    # PML on a periodic side / one-sided periodic / too small open axis are caught before any
    # device allocation.
    cases = []
    r = lbm.Run(16, 16, 0.8)
    r.set_pml(lbm.LBM_ALL, 4, 0.1)           # sides still periodic
    cases.append(r)
    r = lbm.Run(16, 16, 0.8)
    r.set_bc(lbm.LBM_XMIN, "zg")             # x periodic on one side only
    cases.append(r)
    r = lbm.Run(5, 16, 0.8)
    r.set_bc(lbm.LBM_XMIN | lbm.LBM_XMAX, "nrbc")  # open x with 5 nodes
    cases.append(r)
    for r in cases:
        Nx, Ny = r.grid()
        with pytest.raises(lbm.LbmError) as ei:
            r.init(np.ones((Ny, Nx)), 0.0, 0.0, 1.0)
        assert ei.value.status == lbm.LBM_ERR_ARG


def test_init_rejects_bad_fields():
    r = lbm.Run(8, 8, 0.8)
    f = np.ones((8, 8))
    bad = f.copy()
    bad[3, 3] = np.nan
    with pytest.raises(lbm.LbmError):
        r.init(bad, 0.0, 0.0, 1.0)
    with pytest.raises(lbm.LbmError):
        r.init(f, 0.0, 0.0, -f)


def test_missing_library_fails_loudly(tmp_path):
    """Every step runs in the HIP library: without it the binding raises at the first call and
    offers no CPU path (a fresh process pointed at a library file that does not exist)."""
    code = ("from paper_2504_20169_amd import lbm\n"
            "try:\n"
            "    lbm.Run(16, 16, 0.8)\n"
            "except RuntimeError as e:\n"
            "    print('raised:', e)\n"
            "else:\n"
            "    print('no error')\n")
    env = dict(os.environ, LBM_MI355X_LIB=str(tmp_path / "absent.so"))
    res = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True,
                         timeout=120, env=env, cwd=ROOT)
    assert res.returncode == 0, res.stderr
    assert res.stdout.startswith("raised:") and "not built" in res.stdout, res.stdout
