"""ctypes binding of the C ABI in ``include/lbm.h`` (argument marshalling only).

Functions keep the C names (``lbm_create``, ``lbm_set_pml``, ...); ``Run`` and ``Group`` wrap
a handle.  Every step runs in the HIP library: if ``liblbm_mi355x.so`` is missing, loading
raises instead of falling back to anything else.  PyTorch is optional and only supplies device
memory (``torch_allocator()``) and streams (``stream=`` any object with ``.cuda_stream``).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# LBM_MI355X_LIB may name another build of the same library (same ABI, e.g. other flags).
LIB_PATH = os.environ.get("LBM_MI355X_LIB") or os.path.join(HERE, "liblbm_mi355x.so")
# The bounds-checked debug build of the same sources and ABI (lbm_build_flags() == LBM_BUILD_BOUNDS).
BOUNDS_LIB_PATH = os.path.join(HERE, "liblbm_mi355x_bounds.so")
LBM_BUILD_BOUNDS = 1

LBM_OK, LBM_ERR_ARG, LBM_ERR_STATE, LBM_ERR_OOM, LBM_ERR_DEVICE, LBM_ERR_UNSTABLE, \
    LBM_ERR_UNSUPPORTED = range(7)
LBM_F64, LBM_F32_DEV, LBM_F16_DEV = 0, 1, 2
LBM_XMIN, LBM_XMAX, LBM_YMIN, LBM_YMAX, LBM_ALL = 1, 2, 4, 8, 15
LBM_BC_PERIODIC, LBM_BC_ZG, LBM_BC_NRBC, LBM_BC_NRBC_A = 0, 1, 2, 3
LBM_DEVICE_PTRS = 1
LBM_DEBUG_POISON = 1
LBM_DEBUG_RANGES = 2

STORAGE = {"f64": LBM_F64, "f32": LBM_F32_DEV, "f16": LBM_F16_DEV}
BC = {"periodic": LBM_BC_PERIODIC, "zg": LBM_BC_ZG, "nrbc": LBM_BC_NRBC, "nrbc_a": LBM_BC_NRBC_A}

# C symbols exported by the library (the header's declarations).
EXPORTED = [
    "lbm_create", "lbm_set_pml", "lbm_set_bc", "lbm_set_nrbc_pml_terms", "lbm_set_debug", "lbm_grid", "lbm_footprint", "lbm_init_fields",
    "lbm_node_classes",
    "lbm_step", "lbm_step_count", "lbm_moments", "lbm_populations", "lbm_pml_q",
    "lbm_velocities", "lbm_error_norms", "lbm_error_norms_noalloc", "lbm_check", "lbm_synchronize", "lbm_set_launch",
    "lbm_get_launch", "lbm_autotune", "lbm_profile", "lbm_profile_read", "lbm_save",
    "lbm_load", "lbm_destroy", "lbm_last_error", "lbm_group_create", "lbm_group_add",
    "lbm_group_remove", "lbm_group_step", "lbm_group_size", "lbm_group_check", "lbm_group_synchronize",
    "lbm_group_set_launch", "lbm_group_get_launch", "lbm_group_autotune", "lbm_group_destroy",
    "lbm_build_flags", "lbm_set_check_interval",
]

ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


class lbm_allocator(ctypes.Structure):
    _fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("ctx", ctypes.c_void_p)]


class lbm_desc(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("tau", ctypes.c_double),
                ("rho0", ctypes.c_double), ("ux0", ctypes.c_double), ("uy0", ctypes.c_double),
                ("T0", ctypes.c_double), ("storage", ctypes.c_int32),
                ("f16_scale", ctypes.c_double), ("allocator", ctypes.POINTER(lbm_allocator)),
                ("stream", ctypes.c_void_p), ("layout", ctypes.c_int32),
                ("row_pad", ctypes.c_int32), ("lattice", ctypes.c_int32)]


class lbm_launch(ctypes.Structure):
    _fields_ = [("bulk_tx", ctypes.c_int32), ("bulk_ty", ctypes.c_int32),
                ("graph_steps", ctypes.c_int32), ("overlap", ctypes.c_int32), ("split", ctypes.c_int32)]


def _launch_dict(c):
    return dict(bulk_tx=c.bulk_tx, bulk_ty=c.bulk_ty, graph_steps=c.graph_steps, overlap=c.overlap,
                split=c.split)


class LbmError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("lbm status %d: %s" % (status, msg))
        self.status = status


_lib = None


def load():
    """Load the HIP library; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("HIP library %s not built: run `python -m paper_2504_20169_amd.build` "
                           "or __graft_entry__.build()" % LIB_PATH)
    lib = ctypes.CDLL(LIB_PATH)
    H = ctypes.c_void_p
    dp = ctypes.POINTER(ctypes.c_double)
    i32p = ctypes.POINTER(ctypes.c_int32)
    i64p = ctypes.POINTER(ctypes.c_int64)
    sig = {
        "lbm_create": [ctypes.POINTER(lbm_desc), ctypes.POINTER(H)],
        "lbm_set_pml": [H, ctypes.c_uint, ctypes.c_int32, ctypes.c_double],
        "lbm_set_bc": [H, ctypes.c_uint, ctypes.c_int],
        "lbm_set_nrbc_pml_terms": [H, ctypes.c_uint],
        "lbm_set_debug": [H, ctypes.c_uint],
        "lbm_grid": [H, i32p, i32p],
        "lbm_footprint": [H, ctypes.POINTER(ctypes.c_size_t)],
        "lbm_node_classes": [H, i64p],
        "lbm_init_fields": [H, dp, dp, dp, dp],
        "lbm_step": [H, ctypes.c_int64],
        "lbm_set_check_interval": [H, ctypes.c_int64],
        "lbm_step_count": [H, i64p],
        "lbm_moments": [H, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                        ctypes.c_uint],
        "lbm_populations": [H, dp],
        "lbm_pml_q": [H, dp],
        "lbm_velocities": [ctypes.c_int32, i32p, dp, dp],
        "lbm_error_norms": [H, dp, dp, dp, dp],
        "lbm_error_norms_noalloc": [H, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                    ctypes.c_void_p],
        "lbm_check": [H],
        "lbm_synchronize": [H],
        "lbm_set_launch": [H, ctypes.POINTER(lbm_launch)],
        "lbm_get_launch": [H, ctypes.POINTER(lbm_launch)],
        "lbm_autotune": [H, ctypes.c_int32, ctypes.c_char_p, ctypes.POINTER(lbm_launch)],
        "lbm_group_set_launch": [H, ctypes.POINTER(lbm_launch)],
        "lbm_group_get_launch": [H, ctypes.POINTER(lbm_launch)],
        "lbm_group_autotune": [H, ctypes.c_int32, ctypes.POINTER(lbm_launch)],
        "lbm_profile": [H, ctypes.c_int],
        "lbm_profile_read": [H, dp, i64p, ctypes.c_int],
        "lbm_save": [H, ctypes.c_char_p],
        "lbm_load": [H, ctypes.c_char_p],
        "lbm_group_create": [ctypes.c_void_p, ctypes.POINTER(lbm_allocator), ctypes.POINTER(H)],
        "lbm_group_add": [H, H],
        "lbm_group_remove": [H, H],
        "lbm_group_step": [H, i64p, ctypes.c_int64],
        "lbm_group_size": [H, i32p],
        "lbm_group_check": [H, i32p],
        "lbm_group_synchronize": [H],
    }
    for name, args in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    lib.lbm_destroy.argtypes = [H]
    lib.lbm_destroy.restype = None
    lib.lbm_group_destroy.argtypes = [H]
    lib.lbm_group_destroy.restype = None
    lib.lbm_last_error.argtypes = []
    lib.lbm_last_error.restype = ctypes.c_char_p
    lib.lbm_build_flags.argtypes = []
    lib.lbm_build_flags.restype = ctypes.c_int32
    _lib = lib
    return lib


def _check(st):
    if st != LBM_OK:
        raise LbmError(st, load().lbm_last_error().decode())
    return st


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


# ---- same-named functions over the C ABI ------------------------------------------------------

LATTICES = (37, 17, 9)


def lbm_build_flags():
    """0 for the normal build, LBM_BUILD_BOUNDS for the bounds-checked debug build."""
    return int(load().lbm_build_flags())


def lbm_velocities(lattice=37):
    """(e [q,2], w [q], r) of the library's velocity order for the D2Q37, D2Q17 or D2Q9
    stencil."""
    q = 37 if int(lattice) == 0 else int(lattice)
    if q not in LATTICES:
        raise LbmError(LBM_ERR_ARG, "lattice must be 37, 17 or 9")
    e = np.zeros((q, 2), dtype=np.int32)
    w = np.zeros(q)
    r = ctypes.c_double()
    _check(load().lbm_velocities(q, e.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), _dp(w),
                                 ctypes.byref(r)))
    return e.astype(np.int64), w, r.value


def torch_allocator(stream=None):
    """Allocator hook that takes device memory from PyTorch's caching allocator.

    The caching allocator hands out a block as soon as its last use has been queued on the stream
    it was allocated on, so the block is safe only for work ordered after that stream's queue.
    With ``stream`` (the torch stream the run or group will use, the same object passed as their
    ``stream=``) the blocks are allocated on that stream, and the library's work on it is ordered
    after every earlier use.  Without it the blocks come from the current stream, which is
    synchronised before the block is handed over, so work queued on any stream may use it.  The
    library frees a block only after its own stream has drained."""
    import torch

    live = {}

    def _alloc(nbytes, ctx):
        try:
            if stream is not None:
                with torch.cuda.stream(stream):
                    t = torch.empty(int(nbytes), dtype=torch.uint8, device="cuda")
            else:
                t = torch.empty(int(nbytes), dtype=torch.uint8, device="cuda")
                torch.cuda.current_stream().synchronize()
        except RuntimeError:
            return None
        ptr = t.data_ptr()
        live[ptr] = t
        return ptr

    def _free(ptr, ctx):
        live.pop(ptr, None)

    a = lbm_allocator(ALLOC_FN(_alloc), FREE_FN(_free), None)
    a._keep = (_alloc, _free, live)
    return a


def _stream_ptr(stream):
    if stream is None:
        return None
    if isinstance(stream, int):
        return stream
    return int(stream.cuda_stream)


class Run:
    """One simulation handle (create -> set_pml / set_bc -> init -> step ...)."""

    def __init__(self, nx, ny, tau=0.8, rho0=1.0, ux0=0.0, uy0=0.0, T0=1.0, storage="f64",
                 f16_scale=0.0, stream=None, allocator=None, layout=0, row_pad=0, lattice=37):
        lib = load()
        self._lib = lib
        self._alloc = allocator
        d = lbm_desc(int(nx), int(ny), float(tau), float(rho0), float(ux0), float(uy0),
                     float(T0), STORAGE[storage] if isinstance(storage, str) else int(storage),
                     float(f16_scale),
                     ctypes.pointer(allocator) if allocator is not None else None,
                     _stream_ptr(stream), int(layout), int(row_pad), int(lattice))
        h = ctypes.c_void_p()
        _check(lib.lbm_create(ctypes.byref(d), ctypes.byref(h)))
        self.h = h
        self.nx, self.ny = int(nx), int(ny)
        self.q = 37 if int(lattice) == 0 else int(lattice)

    def close(self):
        if getattr(self, "h", None):
            self._lib.lbm_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_pml(self, mask, W, sigma_max):
        _check(self._lib.lbm_set_pml(self.h, int(mask), int(W), float(sigma_max)))

    def set_bc(self, mask, kind):
        _check(self._lib.lbm_set_bc(self.h, int(mask), BC[kind] if isinstance(kind, str) else int(kind)))

    def set_nrbc_pml_terms(self, flags):
        """Appendix: PML moments in the characteristic target (bit 0 term I, bit 1 term II,
        bit 2 term III)."""
        _check(self._lib.lbm_set_nrbc_pml_terms(self.h, int(flags)))

    def set_debug(self, flags):
        """Debug flags (LBM_DEBUG_POISON: NaN canary in the buffers each step writes)."""
        _check(self._lib.lbm_set_debug(self.h, int(flags)))

    def grid(self):
        nx, ny = ctypes.c_int32(), ctypes.c_int32()
        _check(self._lib.lbm_grid(self.h, ctypes.byref(nx), ctypes.byref(ny)))
        return nx.value, ny.value

    def footprint(self):
        b = ctypes.c_size_t()
        _check(self._lib.lbm_footprint(self.h, ctypes.byref(b)))
        return b.value

    def node_classes(self):
        """(bulk-kernel nodes, frame-kernel nodes, PML Q-region nodes, characteristic ring nodes)."""
        out = np.zeros(4, dtype=np.int64)
        _check(self._lib.lbm_node_classes(self.h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))))
        return tuple(int(v) for v in out)

    def init(self, rho, ux, uy, T):
        Nx, Ny = self.grid()
        arrs = [np.ascontiguousarray(np.broadcast_to(a, (Ny, Nx)), dtype=np.float64)
                for a in (rho, ux, uy, T)]
        _check(self._lib.lbm_init_fields(self.h, *[_dp(a) for a in arrs]))

    def step(self, n):
        _check(self._lib.lbm_step(self.h, int(n)))

    def set_check_interval(self, every):
        """Check the state every `every` steps inside step(); an unstable state raises
        LbmError (LBM_ERR_UNSTABLE) with the run stopped after the failing chunk.  0: off."""
        _check(self._lib.lbm_set_check_interval(self.h, int(every)))

    @property
    def step_count(self):
        v = ctypes.c_int64()
        _check(self._lib.lbm_step_count(self.h, ctypes.byref(v)))
        return v.value

    def synchronize(self):
        _check(self._lib.lbm_synchronize(self.h))

    def moments(self):
        Nx, Ny = self.grid()
        out = [np.zeros((Ny, Nx)) for _ in range(4)]
        _check(self._lib.lbm_moments(self.h, *[a.ctypes.data for a in out], 0))
        return out

    def moments_device(self, rho=None, ux=None, uy=None, T=None):
        """Stream-ordered moments into device buffers given as integer pointers (or None)."""
        _check(self._lib.lbm_moments(self.h, rho, ux, uy, T, LBM_DEVICE_PTRS))

    def populations(self):
        Nx, Ny = self.grid()
        out = np.zeros((self.q, Ny, Nx))
        _check(self._lib.lbm_populations(self.h, _dp(out)))
        return out

    def pml_q(self):
        Nx, Ny = self.grid()
        out = np.zeros((self.q, Ny, Nx))
        _check(self._lib.lbm_pml_q(self.h, _dp(out)))
        return out

    def error_norms(self, ref_rho, ref_ux, ref_T):
        refs = [np.ascontiguousarray(a, dtype=np.float64) for a in (ref_rho, ref_ux, ref_T)]
        out = np.zeros(3)
        _check(self._lib.lbm_error_norms(self.h, *[_dp(a) for a in refs], _dp(out)))
        return out

    def error_norms_noalloc(self, ref_rho, ref_ux, ref_T, out):
        """lbm_error_norms_noalloc with device pointers (integers): enqueues only; the result lands
        in out (3 doubles) once the run's stream has reached it."""
        _check(self._lib.lbm_error_norms_noalloc(self.h, int(ref_rho), int(ref_ux), int(ref_T),
                                                 int(out)))

    def check(self):
        """LBM_OK or LBM_ERR_UNSTABLE (returned, not raised); in the bounds-checked build an index
        out of range in the run's kernels raises LbmError (LBM_ERR_DEVICE)."""
        st = self._lib.lbm_check(self.h)
        if st not in (LBM_OK, LBM_ERR_UNSTABLE):
            _check(st)
        return st

    def set_launch(self, bulk_tx=64, graph_steps=32, overlap=2, split=-1):
        """overlap: 0 kernels in order, 1 boundary/PML chain on a side stream, 2 phase A fused
        with the bulk tiles in one grid (split: phase-A blocks after split/8 of the tiles, -1 the
        default placement); the same bits in every schedule."""
        c = lbm_launch(int(bulk_tx), 256 // int(bulk_tx), int(graph_steps), int(overlap), int(split))
        _check(self._lib.lbm_set_launch(self.h, ctypes.byref(c)))

    def get_launch(self):
        c = lbm_launch()
        _check(self._lib.lbm_get_launch(self.h, ctypes.byref(c)))
        return _launch_dict(c)

    def autotune(self, steps=10, cache_path=None):
        c = lbm_launch()
        _check(self._lib.lbm_autotune(self.h, int(steps),
                                      cache_path.encode() if cache_path else None, ctypes.byref(c)))
        return _launch_dict(c)

    def profile(self, mode=1):
        """Event timing: 1 (or True) kernel classes in order, 2 bulk kernel in the normal
        schedule, 3 as 2 on the first step of each batch only, 0 (or False) off."""
        _check(self._lib.lbm_profile(self.h, int(mode)))

    def profile_read(self, reset=False):
        ms = np.zeros(3)
        n = np.zeros(3, dtype=np.int64)
        _check(self._lib.lbm_profile_read(self.h, _dp(ms),
                                          n.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                          1 if reset else 0))
        return ms, n

    def save(self, path):
        _check(self._lib.lbm_save(self.h, str(path).encode()))

    def load(self, path):
        _check(self._lib.lbm_load(self.h, str(path).encode()))


class Group:
    """Batched runs advanced by one launch per kernel class and step."""

    def __init__(self, stream=None, allocator=None):
        lib = load()
        self._lib = lib
        self._alloc = allocator
        g = ctypes.c_void_p()
        _check(lib.lbm_group_create(_stream_ptr(stream),
                                    ctypes.pointer(allocator) if allocator is not None else None,
                                    ctypes.byref(g)))
        self.g = g
        self.members = []

    def add(self, run: Run):
        _check(self._lib.lbm_group_add(self.g, run.h))
        self.members.append(run)

    def remove(self, run: Run):
        _check(self._lib.lbm_group_remove(self.g, run.h))
        self.members.remove(run)

    def step(self, steps=None, nsteps=0):
        if steps is None:
            _check(self._lib.lbm_group_step(self.g, None, int(nsteps)))
        else:
            arr = np.ascontiguousarray(steps, dtype=np.int64)
            _check(self._lib.lbm_group_step(self.g, arr.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), 0))

    def synchronize(self):
        _check(self._lib.lbm_group_synchronize(self.g))

    def set_launch(self, bulk_tx=64, graph_steps=32, overlap=2, split=-1):
        """overlap 0 (kernels in order) or 2 (phase A fused with the bulk tiles, split as for a
        run); a group runs on one stream, so the side-stream schedule (1) is refused."""
        c = lbm_launch(int(bulk_tx), 256 // int(bulk_tx), int(graph_steps), int(overlap), int(split))
        _check(self._lib.lbm_group_set_launch(self.g, ctypes.byref(c)))

    def get_launch(self):
        c = lbm_launch()
        _check(self._lib.lbm_group_get_launch(self.g, ctypes.byref(c)))
        return _launch_dict(c)

    def autotune(self, steps=10):
        c = lbm_launch()
        _check(self._lib.lbm_group_autotune(self.g, int(steps), ctypes.byref(c)))
        return _launch_dict(c)

    def size(self):
        n = ctypes.c_int32()
        _check(self._lib.lbm_group_size(self.g, ctypes.byref(n)))
        return n.value

    def check(self):
        """Per-member health flags (member order): 0 healthy, 1 non-finite, rho <= 0 or T <= 0, 2 an
        index out of range in the member's kernels (bounds-checked build only)."""
        out = np.zeros(max(len(self.members), 1), dtype=np.int32)
        _check(self._lib.lbm_group_check(self.g, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))))
        return out[:len(self.members)]

    def close(self):
        if getattr(self, "g", None):
            self._lib.lbm_group_destroy(self.g)
            self.g = None
            self.members = []

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def configure(run: Run, spec):
    """Apply a workload RunSpec's PML and boundary (all four sides)."""
    if spec.bc == "periodic":
        run.set_bc(LBM_ALL, "periodic")
    else:
        run.set_bc(LBM_ALL, spec.bc)
        if spec.W > 0:
            run.set_pml(LBM_ALL, spec.W, spec.sigma_max)
    return run
