"""FP64 CPU oracle for the D2Q37 / D2Q17 / D2Q9 LBM + PML + open boundaries (arXiv 2504.20169).

TEST INFRASTRUCTURE ONLY: only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg
of ``bench.py`` may import this package.  It shares no code with the HIP library; see the header
of ``lbm_oracle.c`` for what each function follows and how it is pinned.

Layouts: fields are row-major ``[Ny][Nx]`` float64 arrays; populations are ``[q][Ny][Nx]`` in
this oracle's own velocity order (``lattice(q)[0]``), which differs from the library's order.

The C source is compiled once per velocity stencil (``-DORC_Q=37``, ``17`` and ``9``); every
entry point takes the stencil as ``q`` (``lattice=`` for runs), 37 by default.  A second build per
stencil (``precision="extended"``) takes the same steps in x87 extended precision; the tests use
it only to measure how far the double build's own rounding has carried it (its conditioning
floor), never as a reference of its own.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lbm_oracle.c")
_LIBS = {37: os.path.join(_HERE, "liboracle.so"), 17: os.path.join(_HERE, "liboracle17.so"),
         9: os.path.join(_HERE, "liboracle9.so")}
LATTICES = (37, 17, 9)
PRECISIONS = ("double", "extended")

SIDE_XMIN, SIDE_XMAX, SIDE_YMIN, SIDE_YMAX, SIDE_ALL = 1, 2, 4, 8, 15
BC_PERIODIC, BC_ZG, BC_NRBC, BC_NRBC_A = 0, 1, 2, 3

_libs = {}


def _lib_path(q: int, precision: str = "double") -> str:
    if q not in _LIBS:
        raise ValueError("oracle: velocity stencil must be one of %s, got %r" % (LATTICES, q))
    if precision not in PRECISIONS:
        raise ValueError("oracle: precision must be one of %s, got %r" % (PRECISIONS, precision))
    return _LIBS[q] if precision == "double" else _LIBS[q][:-3] + "_ext.so"


def build(force: bool = True) -> list:
    """Compile the oracle with gcc (-O2, no FP contraction, no fast-math, OpenMP), once per
    velocity stencil and precision."""
    out = []
    for q in LATTICES:
        for prec in PRECISIONS:
            path = _lib_path(q, prec)
            if force or not os.path.exists(path):
                tmp = path + ".tmp"
                extra = ["-DORC_REAL=long double"] if prec == "extended" else []
                subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
                                       "-DORC_Q=%d" % q] + extra + ["-shared", "-fPIC", "-o", tmp, _SRC,
                                                                    "-lm"])
                os.replace(tmp, path)
            out.append(path)
    return out


def _load(q: int = 37, precision: str = "double"):
    if (q, precision) in _libs:
        return _libs[(q, precision)]
    path = _lib_path(q, precision)
    if not os.path.exists(path):
        build(force=True)
    lib = ctypes.CDLL(path)
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
    _libs[(q, precision)] = lib
    return lib


def _dp(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _check(rc: int, q: int = 37):
    if rc != 0:
        raise RuntimeError("oracle: " + _load(q).orc_last_error().decode())


def lattice(q: int = 37):
    """(e [q,2] int, w [q], r) derived by the oracle's own quadrature solve."""
    lib = _load(q)
    e = np.zeros((q, 2), dtype=np.int32)
    w = np.zeros(q)
    r = ctypes.c_double()
    _check(lib.orc_lattice(e.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), _dp(w), ctypes.byref(r)), q)
    return e.astype(np.int64), w, r.value


def feq(rho, ux, uy, T, q: int = 37) -> np.ndarray:
    """Equilibrium of the stencil: eq. feq-4 for D2Q37, eq. feq-3 for D2Q17, eq. feq-2 for D2Q9."""
    out = np.zeros(q)
    _check(_load(q).orc_feq(rho, ux, uy, T, _dp(out)), q)
    return out


def moments_of(f: np.ndarray, q: int = 37) -> np.ndarray:
    f = np.ascontiguousarray(f, dtype=np.float64)
    if f.shape[0] != q:
        raise ValueError("oracle: expected %d populations, got %d" % (q, f.shape[0]))
    U = np.zeros(4)
    _check(_load(q).orc_moments_of(_dp(f), _dp(U)), q)
    return U


def threads() -> int:
    return int(_load().orc_threads())


class OracleRun:
    """One oracle simulation.  Mirrors the library's configuration order:
    create -> set_pml / set_bc -> init -> step ..."""

    def __init__(self, Lx, Ly, tau, rho0=1.0, ux0=0.0, uy0=0.0, T0=1.0, lattice=37,
                 precision="double"):
        lib = _load(lattice, precision)
        self.q = int(lattice)
        self._lib = lib
        self._h = lib.orc_create(int(Lx), int(Ly), float(tau), float(rho0), float(ux0),
                                 float(uy0), float(T0))
        if not self._h:
            raise RuntimeError("oracle: " + lib.orc_last_error().decode())
        self.Lx, self.Ly = int(Lx), int(Ly)

    def _ck(self, rc):
        if rc != 0:
            raise RuntimeError("oracle: " + self._lib.orc_last_error().decode())

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
        self._ck(self._lib.orc_set_pml(self._h, int(mask), int(W), float(sigma_max)))

    def set_bc(self, mask, kind):
        self._ck(self._lib.orc_set_bc(self._h, int(mask), int(kind)))

    def set_nrbc_pml_terms(self, flags):
        """Appendix: moments of the PML collision term in the characteristic target update
        (bit 0 term I, bit 1 term II, bit 2 term III)."""
        self._ck(self._lib.orc_set_nrbc_pml_terms(self._h, int(flags)))

    def grid(self):
        nx, ny = ctypes.c_int(), ctypes.c_int()
        self._ck(self._lib.orc_grid(self._h, ctypes.byref(nx), ctypes.byref(ny)))
        return nx.value, ny.value

    def init(self, rho, ux, uy, T):
        Nx, Ny = self.grid()
        arrs = [np.ascontiguousarray(np.broadcast_to(a, (Ny, Nx)), dtype=np.float64)
                for a in (rho, ux, uy, T)]
        self._ck(self._lib.orc_init(self._h, *[_dp(a) for a in arrs]))

    def step(self, n, threads=0):
        self._ck(self._lib.orc_step(self._h, int(n), int(threads)))

    @property
    def step_count(self):
        return int(self._lib.orc_step_count(self._h))

    def moments(self):
        Nx, Ny = self.grid()
        out = [np.zeros((Ny, Nx)) for _ in range(4)]
        self._ck(self._lib.orc_moments(self._h, *[_dp(a) for a in out]))
        return out

    def populations(self):
        Nx, Ny = self.grid()
        out = np.zeros((self.q, Ny, Nx))
        self._ck(self._lib.orc_populations(self._h, _dp(out)))
        return out

    def pml_q(self):
        Nx, Ny = self.grid()
        out = np.zeros((self.q, Ny, Nx))
        self._ck(self._lib.orc_pml_q(self._h, _dp(out)))
        return out

    def sigma(self):
        Nx, Ny = self.grid()
        out = np.zeros((Ny, Nx))
        self._ck(self._lib.orc_sigma(self._h, _dp(out)))
        return out

    def error_norms(self, ref_rho, ref_ux, ref_T):
        refs = [np.ascontiguousarray(a, dtype=np.float64) for a in (ref_rho, ref_ux, ref_T)]
        out = np.zeros(3)
        self._ck(self._lib.orc_error_norms(self._h, *[_dp(a) for a in refs], _dp(out)))
        return out
