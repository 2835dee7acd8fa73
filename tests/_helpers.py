"""Shared test helpers: build the same run on the HIP library and on the oracle, compare."""
import sys

import numpy as np

from paper_2504_20169_amd import lbm
from paper_2504_20169_amd import workloads as wl

SIDES = {"xmin": 1, "xmax": 2, "ymin": 4, "ymax": 8}


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def perm_lib_to_oracle(oracle_mod, q=37):
    """perm[k] = library index of the oracle's velocity k (stencil D2Q37, D2Q17 or D2Q9)."""
    e, _, _ = lbm.lbm_velocities(q)
    eo, _, _ = oracle_mod.lattice(q)
    where = {(int(a), int(b)): i for i, (a, b) in enumerate(e)}
    return np.array([where[(int(a), int(b))] for a, b in eo])


def make_pair(oracle_mod, Lx, Ly, tau=0.8, mean=(1.0, 0.0, 0.0, 1.0), bc=None, pml=None,
              fields=None, storage="f64", launch=None, stream=None, allocator=None, gpu=True,
              pml_terms=0, lattice=37, precision="double"):
    """bc: dict side->kind ('zg'|'nrbc'|'periodic') or a kind for all sides; pml: (mask, W,
    sigma); lattice: 37, 17 or 9; precision: the oracle build ('double', or 'extended' to measure
    the double build's rounding).  Returns (gpu_run or None, oracle_run)."""
    rho0, ux0, uy0, T0 = mean
    o = oracle_mod.OracleRun(Lx, Ly, tau, rho0, ux0, uy0, T0, lattice=lattice, precision=precision)
    g = lbm.Run(Lx, Ly, tau, rho0, ux0, uy0, T0, storage=storage, stream=stream,
                allocator=allocator, lattice=lattice) if gpu else None
    kinds = {"periodic": 0, "zg": 1, "nrbc": 2, "nrbc_a": 3}
    if bc is not None:
        items = bc.items() if isinstance(bc, dict) else [(s, bc) for s in SIDES]
        for side, kind in items:
            o.set_bc(SIDES[side], kinds[kind])
            if g:
                g.set_bc(SIDES[side], kind)
    if pml is not None:
        mask, W, sig = pml
        o.set_pml(mask, W, sig)
        if g:
            g.set_pml(mask, W, sig)
    if pml_terms:
        o.set_nrbc_pml_terms(pml_terms)
        if g:
            g.set_nrbc_pml_terms(pml_terms)
    if g and launch:
        g.set_launch(**launch)
    Nx, Ny = o.grid()
    if g:
        assert g.grid() == (Nx, Ny)
    F = fields(Nx, Ny) if callable(fields) else fields
    o.init(*F.as_tuple())
    if g:
        g.init(*F.as_tuple())
    return g, o


def rel_errors(g, o, perm, with_f=True):
    """Relative differences (the 1e-12 bar's definition): rho and T relative to max |Z| of the
    oracle, ux and uy relative to the oracle's largest velocity component, populations relative to
    their weight."""
    mg = g.moments()
    mo = o.moments()
    out = {}
    us = max(np.abs(mo[1]).max(), np.abs(mo[2]).max())
    for name, a, b in zip(("rho", "ux", "uy", "T"), mg, mo):
        scale = us if name in ("ux", "uy") else np.abs(b).max()
        out[name] = float(np.abs(a - b).max() / scale) if scale > 0 else float(np.abs(a - b).max())
    if with_f:
        _, w, _ = lbm.lbm_velocities(g.q)
        fg = g.populations()[perm]
        fo = o.populations()
        wo = w[perm]
        out["f"] = float((np.abs(fg - fo).max(axis=(1, 2)) / wo).max())
    return out


def noise(seed, mean=(1.0, 0.0, 0.0, 1.0), amp=1e-3):
    return lambda Nx, Ny: wl.noisy_state(Nx, Ny, seed, *mean, amp=amp)


def oracle_floors(oracle_mod, Lx, Ly, tau=0.8, mean=(1.0, 0.0, 0.0, 1.0), bc=None, pml=None,
                  fields=None, steps=0, lattice=37, pml_terms=0):
    """The oracle's own conditioning floor for a case, with the normalisations of rel_errors (and
    Q relative to max |Q|): the larger of
      - how far the double oracle's own accumulated rounding has carried it, measured against
        the same oracle run in x87 extended precision (the per-step rounding of any FP64
        implementation is of this size), and
      - how far its result moves when its input density is perturbed at the rounding level
        (random relative +-2e-16).
    Two FP64 implementations that round differently cannot be expected to agree more closely.
    Returns a dict with keys rho, ux, uy, T, f, Q."""
    outs = []
    for k, prec in ((0, "double"), (1, "double"), (0, "extended")):
        def fk(Nx, Ny, k=k):
            F = fields(Nx, Ny) if callable(fields) else fields
            if k:
                u = wl.uniform(77, Nx * Ny).reshape(Ny, Nx)
                F = wl.Fields(F.rho * (1.0 + (u - 0.5) * 4e-16), F.ux, F.uy, F.T)
            return F
        _, o = make_pair(oracle_mod, Lx, Ly, tau, mean, bc, pml, fk, gpu=False, lattice=lattice,
                         pml_terms=pml_terms, precision=prec)
        o.step(steps)
        outs.append((o.moments(), o.populations(), o.pml_q()))
    m0, f0, q0 = outs[0]
    _, w, _ = oracle_mod.lattice(lattice)
    us = max(np.abs(m0[1]).max(), np.abs(m0[2]).max())
    qmax = np.abs(q0).max()
    fl = dict(rho=0.0, ux=0.0, uy=0.0, T=0.0, f=0.0, Q=0.0)
    for m1, f1, q1 in outs[1:]:
        for name, a, b in zip(("rho", "ux", "uy", "T"), m1, m0):
            scale = us if name in ("ux", "uy") else np.abs(b).max()
            d = float(np.abs(a - b).max())
            fl[name] = max(fl[name], d / scale if scale > 0 else d)
        fl["f"] = max(fl["f"], float((np.abs(f1 - f0).max(axis=(1, 2)) / w).max()))
        if qmax > 0:
            fl["Q"] = max(fl["Q"], float(np.abs(q1 - q0).max() / qmax))
    return fl


def oracle_self_sensitivity(oracle_mod, **case):
    """(f floor relative to the weights, Q floor relative to max |Q|) of oracle_floors."""
    fl = oracle_floors(oracle_mod, **case)
    return fl["f"], fl["Q"]


TOL = 1e-12


def assert_parity(err, oracle_mod=None, case=None, tol=TOL):
    """Every quantity of rel_errors within `tol` (1e-12), or, for a quantity above it, within 4x
    the oracle's own conditioning floor for the case (oracle_floors; measured only when some
    quantity exceeds the bar, and only for grids small enough to run the oracle twice).  The
    floor itself must stay below 1e-8: a larger one would mean the case is ill-conditioned, not
    that the bar may widen."""
    over = {k: v for k, v in err.items() if not v <= tol}
    if not over:
        return
    assert oracle_mod is not None and case is not None, ("above the bar, no floor to compare", err)
    Nx, Ny = case["Lx"], case["Ly"]
    if case.get("pml"):
        Nx += 2 * case["pml"][1]
        Ny += 2 * case["pml"][1]
    assert Nx * Ny <= 250000, ("above the bar on a grid too large for a floor run", err)
    fl = oracle_floors(oracle_mod, **case)
    say("conditioning floors", {k: "%.2e" % v for k, v in fl.items()})
    bad = {k: (v, fl[k]) for k, v in over.items() if not (v <= 4.0 * fl[k] and fl[k] < 1e-8)}
    assert not bad, (err, fl)
