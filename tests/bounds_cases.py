"""Geometry matrix for the bounds-checked debug build: every stencil, storage, boundary kind and
schedule, ragged and degenerate grids, both population layouts, a group of uneven runs, and the
1088^2 benchmark grid.  run_all() steps each case with whichever library build is loaded, checks
every run (an index out of range raises in the bounds-checked build) and returns each case's
check status and a hash of its populations, moments and PML auxiliary field.

Run as a script (python tests/bounds_cases.py OUT.json) with LBM_MI355X_LIB naming the
bounds-checked build; tests/test_gpu_bounds.py compares its hashes with the normal build's."""
import hashlib
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

# (name, nx, ny, W, pml mask, bc, bc mask, storage, lattice, steps, launch, extra)
CASES = [
    ("q37_nrbc_pml_f64", 61, 47, 9, 15, "nrbc", 15, "f64", 37, 20, {}, {}),
    ("q37_nrbc_pml_f32_tx128", 130, 70, 12, 15, "nrbc", 15, "f32", 37, 20, {"bulk_tx": 128}, {}),
    ("q37_nrbc_pml_f16_tx256", 260, 33, 7, 15, "nrbc", 15, "f16", 37, 20, {"bulk_tx": 256}, {}),
    ("q37_zg_pml_inorder", 75, 64, 10, 15, "zg", 15, "f64", 37, 21, {"overlap": 0}, {}),
    ("q37_zg_pml_side_stream", 75, 64, 10, 15, "zg", 15, "f32", 37, 21, {"overlap": 1}, {}),
    ("q37_cbca_terms", 66, 66, 8, 15, "nrbc_a", 15, "f64", 37, 20, {}, {"terms": 7, "sigma": 0.001}),
    ("q37_nrbc_terms_eager", 66, 50, 8, 15, "nrbc", 15, "f32", 37, 20, {"graph_steps": 0},
     {"terms": 2, "sigma": 0.001}),
    ("q37_y_open_x_periodic", 96, 70, 9, 12, "nrbc", 12, "f64", 37, 20, {}, {}),
    ("q37_x_open_pml_one_side", 80, 40, 6, 1, "zg", 3, "f64", 37, 20, {}, {}),
    ("q37_plain_zg", 70, 52, 0, 0, "zg", 15, "f64", 37, 20, {}, {}),
    ("q37_periodic", 64, 48, 0, 0, "periodic", 15, "f32", 37, 20, {}, {}),
    ("q37_tiny_nrbc", 7, 7, 0, 0, "nrbc", 15, "f64", 37, 12, {}, {}),
    ("q37_tiny_pml1", 8, 9, 1, 15, "nrbc", 15, "f64", 37, 12, {}, {}),
    ("q37_plane_layout", 90, 61, 8, 15, "nrbc", 15, "f64", 37, 20, {}, {"layout": 1}),
    ("q37_split_first", 150, 140, 8, 15, "nrbc", 15, "f64", 37, 20, {"split": 0}, {}),
    ("q17_nrbc_pml_f64", 90, 77, 10, 15, "nrbc", 15, "f64", 17, 20, {}, {}),
    ("q17_cbca_pml_f16", 90, 64, 10, 15, "nrbc_a", 15, "f16", 17, 20, {}, {}),
    ("q9_nrbc_pml_f32", 100, 90, 12, 15, "nrbc", 15, "f32", 9, 20, {}, {}),
    ("q9_zg_pml_f64_inorder", 70, 70, 5, 15, "zg", 15, "f64", 9, 20, {"overlap": 0}, {}),
    ("q37_bench_grid_1088", 1024, 1024, 32, 15, "nrbc", 15, "f64", 37, 4, {}, {}),
]

GROUP = [(80, 87, 8, "nrbc", 17), (133, 140, 17, "zg", 23), (61, 68, 5, "nrbc", 9),
         (40, 47, 0, "zg", 30), (7, 7, 0, "nrbc", 11)]


def _digest(*arrays):
    h = hashlib.sha1()
    for a in arrays:
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()


def _make(lbm, wl, nx, ny, W, pml_mask, bc, bc_mask, storage, lattice, launch, extra, seed):
    r = lbm.Run(nx, ny, 0.8, 1.0, 0.05, 0.01, 1.0, storage=storage, lattice=lattice,
                layout=extra.get("layout", 0))
    if bc_mask:
        r.set_bc(bc_mask, bc)
    if W:
        r.set_pml(pml_mask, W, extra.get("sigma", 0.05))
    if extra.get("terms"):
        r.set_nrbc_pml_terms(extra["terms"])
    if launch:
        r.set_launch(**launch)
    Nx, Ny = r.grid()
    F = wl.noisy_state(Nx, Ny, seed, 1.0, 0.05, 0.01, 1.0, amp=3e-3)
    r.init(*F.as_tuple())
    return r


def run_all():
    from paper_2504_20169_amd import lbm
    from paper_2504_20169_amd import workloads as wl
    out = {"build_flags": lbm.lbm_build_flags()}
    for k, (name, nx, ny, W, pm, bc, bm, st, q, steps, launch, extra) in enumerate(CASES):
        print("bounds case", name, flush=True)
        r = _make(lbm, wl, nx, ny, W, pm, bc, bm, st, q, launch, extra, 100 + k)
        r.step(steps)
        status = r.check()   # raises on an index out of range (bounds-checked build)
        out[name] = "%d %s" % (status, _digest(r.populations(), *r.moments(), r.pml_q()))
        r.close()
    print("bounds case group", flush=True)
    g = lbm.Group()
    runs = []
    for k, (nx, ny, W, bc, _) in enumerate(GROUP):
        r = _make(lbm, wl, nx, ny, W, 15, bc, 15, "f32", 37, {}, {}, 200 + k)
        g.add(r)
        runs.append(r)
    g.step(steps=np.array([c[4] for c in GROUP], dtype=np.int64))
    flags = g.check()
    assert not (flags == 2).any(), flags   # 2: an index out of range (bounds-checked build)
    for k, r in enumerate(runs):
        out["group_%d" % k] = "%d %d %s" % (flags[k], r.check(), _digest(r.populations(), *r.moments()))
    for r in runs:
        g.remove(r)
        r.close()
    g.close()
    return out


if __name__ == "__main__":
    import torch  # noqa: F401  (PyTorch first, as the benchmark loads it)
    res = run_all()
    with open(sys.argv[1], "w") as fh:
        json.dump(res, fh, indent=1)
    print("bounds cases done", len(res) - 1, flush=True)
