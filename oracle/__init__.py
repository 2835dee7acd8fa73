"""FP64 CPU oracle for the D2Q37 thermal LBM + PML + open boundaries (arXiv 2504.20169).

TEST INFRASTRUCTURE ONLY: only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg
of ``bench.py`` may import this package.  It shares no code with the HIP library; see the header
of ``lbm_oracle.c`` for what each function follows and how it is pinned.

Layouts: fields are row-major ``[Ny][Nx]`` float64 arrays; populations are ``[37][Ny][Nx]`` in
this oracle's own velocity order (``lattice()[0]``), which differs from the library's order.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lbm_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

SIDE_XMIN, SIDE_XMAX, SIDE_YMIN, SIDE_YMAX, SIDE_ALL = 1, 2, 4, 8, 15
BC_PERIODIC, BC_ZG, BC_NRBC = 0, 1, 2

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, no FP contraction, no fast-math, OpenMP)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
                               "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build(force=True)
    lib = ctypes.CDLL(_LIB)
    P = ctypes.c_void_p
    dp = ctypes.POINTER(ctypes.c_double)
    ip = ctypes.POINTER(ctypes.c_int)
    lib.orc_create.restype = P
    lib.orc_create.argtypes = [ctypes.c_int, ctypes.c_int] + [ctypes.c_double] * 5
    lib.orc_destroy.argtypes = [P]
    lib.orc_set_pml.argtypes = [P, ctypes.c_uint, ctypes.c_int, ctypes.c_double]
    lib.orc_set_bc.argtypes = [P, ctypes.c_uint, ctypes.c_int]
    lib.orc_set_nrbc_pml_terms.argtypes = [P, ctypes.c_uint]
    lib.orc_grid.argtypes = [P, ip, ip]
    lib.orc_init.argtypes = [P, dp, dp, dp, dp]
    lib.orc_step.argtypes = [P, ctypes.c_long, ctypes.c_int]
    lib.orc_step_count.restype = ctypes.c_long
    lib.orc_step_count.argtypes = [P]
    lib.orc_moments.argtypes = [P, dp, dp, dp, dp]
    lib.orc_populations.argtypes = [P, dp]
    lib.orc_pml_q.argtypes = [P, dp]
    lib.orc_sigma.argtypes = [P, dp]
    lib.orc_error_norms.argtypes = [P, dp, dp, dp, dp]
    lib.orc_lattice.argtypes = [ip, dp, dp]
    lib.orc_feq.argtypes = [ctypes.c_double] * 4 + [dp]
    lib.orc_moments_of.argtypes = [dp, dp]
    lib.orc_last_error.restype = ctypes.c_char_p
    lib.orc_threads.restype = ctypes.c_int
    _lib = lib
    return lib


def _dp(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _check(rc: int):
    if rc != 0:
        raise RuntimeError("oracle: " + _load().orc_last_error().decode())


def lattice():
    """(e [37,2] int, w [37], r) derived by the oracle's own quadrature solve."""
    lib = _load()
    e = np.zeros((37, 2), dtype=np.int32)
    w = np.zeros(37)
    r = ctypes.c_double()
    _check(lib.orc_lattice(e.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), _dp(w), ctypes.byref(r)))
    return e.astype(np.int64), w, r.value


def feq(rho, ux, uy, T) -> np.ndarray:
    out = np.zeros(37)
    _check(_load().orc_feq(rho, ux, uy, T, _dp(out)))
    return out


def moments_of(f: np.ndarray) -> np.ndarray:
    f = np.ascontiguousarray(f, dtype=np.float64)
    U = np.zeros(4)
    _check(_load().orc_moments_of(_dp(f), _dp(U)))
    return U


def threads() -> int:
    return int(_load().orc_threads())


class OracleRun:
    """One oracle simulation.  Mirrors the library's configuration order:
    create -> set_pml / set_bc -> init -> step ..."""

    def __init__(self, Lx, Ly, tau, rho0=1.0, ux0=0.0, uy0=0.0, T0=1.0):
        lib = _load()
        self._lib = lib
        self._h = lib.orc_create(int(Lx), int(Ly), float(tau), float(rho0), float(ux0),
                                 float(uy0), float(T0))
        if not self._h:
            raise RuntimeError("oracle: " + lib.orc_last_error().decode())
        self.Lx, self.Ly = int(Lx), int(Ly)

    def close(self):
        if self._h:
            self._lib.orc_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_pml(self, mask, W, sigma_max):
        _check(self._lib.orc_set_pml(self._h, int(mask), int(W), float(sigma_max)))

    def set_bc(self, mask, kind):
        _check(self._lib.orc_set_bc(self._h, int(mask), int(kind)))

    def set_nrbc_pml_terms(self, flags):
        """Appendix: moments of the PML collision term in the characteristic target update
        (bit 0 term I, bit 1 term II, bit 2 term III)."""
        _check(self._lib.orc_set_nrbc_pml_terms(self._h, int(flags)))

    def grid(self):
        nx, ny = ctypes.c_int(), ctypes.c_int()
        _check(self._lib.orc_grid(self._h, ctypes.byref(nx), ctypes.byref(ny)))
        return nx.value, ny.value

    def init(self, rho, ux, uy, T):
        Nx, Ny = self.grid()
        arrs = [np.ascontiguousarray(np.broadcast_to(a, (Ny, Nx)), dtype=np.float64)
                for a in (rho, ux, uy, T)]
        _check(self._lib.orc_init(self._h, *[_dp(a) for a in arrs]))

    def step(self, n, threads=0):
        _check(self._lib.orc_step(self._h, int(n), int(threads)))

    @property
    def step_count(self):
        return int(self._lib.orc_step_count(self._h))

    def moments(self):
        Nx, Ny = self.grid()
        out = [np.zeros((Ny, Nx)) for _ in range(4)]
        _check(self._lib.orc_moments(self._h, *[_dp(a) for a in out]))
        return out

    def populations(self):
        Nx, Ny = self.grid()
        out = np.zeros((37, Ny, Nx))
        _check(self._lib.orc_populations(self._h, _dp(out)))
        return out

    def pml_q(self):
        Nx, Ny = self.grid()
        out = np.zeros((37, Ny, Nx))
        _check(self._lib.orc_pml_q(self._h, _dp(out)))
        return out

    def sigma(self):
        Nx, Ny = self.grid()
        out = np.zeros((Ny, Nx))
        _check(self._lib.orc_sigma(self._h, _dp(out)))
        return out

    def error_norms(self, ref_rho, ref_ux, ref_T):
        refs = [np.ascontiguousarray(a, dtype=np.float64) for a in (ref_rho, ref_ux, ref_T)]
        out = np.zeros(3)
        _check(self._lib.orc_error_norms(self._h, *[_dp(a) for a in refs], _dp(out)))
        return out
