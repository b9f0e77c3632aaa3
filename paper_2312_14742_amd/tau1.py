"""Thin ctypes binding of the C ABI in ``include/tau1.h`` (argument marshalling only).

Every step of the update runs in ``libtau1.so``.  PyTorch provides the device
workspace (a uint8 tensor) and the HIP stream; nothing here computes the
method.  The binding raises :class:`Tau1Error` when the library is missing or
a call fails; there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libtau1.so")

LATTICES = (9, 15, 19, 27)       # D2Q9 (validation lattice) and the 3-D sets
PRECISIONS = {"f64": 0, "f32": 1, "f16": 2, "bf16": 3}

TAU1_OK = 0
TAU1_E_INVALID = -1
TAU1_E_NOMEM = -2
TAU1_E_HIP = -3
TAU1_E_UNSUPPORTED = -4
TAU1_E_NONFINITE = -5
TAU1_E_WORKSPACE = -6

# Every function the header declares (checked against include/tau1.h by the tests).
EXPORTS = ("tau1_workspace_size", "tau1_create", "tau1_step", "tau1_sync",
           "tau1_moments", "tau1_moments_drho", "tau1_permeability",
           "tau1_permeability_noalloc", "tau1_autotune",
           "tau1_get_info", "tau1_destroy", "tau1_strerror", "tau1_copy_probe")


class Tau1Error(RuntimeError):
    def __init__(self, status: int, what: str):
        self.status = status
        msg = _lib().tau1_strerror(status).decode() if _LIB is not None else str(status)
        super().__init__(f"{what}: {msg} ({status})")


class tau1_sample(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int64), ("ny", ctypes.c_int64), ("nz", ctypes.c_int64),
                ("solid", ctypes.c_void_p), ("drho0", ctypes.c_void_p),
                ("u0", ctypes.c_void_p)]


class tau1_desc(ctypes.Structure):
    _fields_ = [("lattice", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("n_samples", ctypes.c_int32), ("graph_chunk", ctypes.c_int32),
                ("samples", ctypes.POINTER(tau1_sample)),
                ("g", ctypes.c_double * 3),
                ("hip_stream", ctypes.c_void_p),
                ("workspace", ctypes.c_void_p),
                ("workspace_bytes", ctypes.c_size_t),
                ("kernel", ctypes.c_int32), ("tile", ctypes.c_int32),
                ("f16_log2_scale_rho", ctypes.c_int32),
                ("f16_log2_scale_u", ctypes.c_int32),
                ("tune_cache", ctypes.c_char_p),
                ("layout", ctypes.c_int32),
                ("x_boundary", ctypes.c_int32),
                ("rho_in", ctypes.c_double), ("rho_out", ctypes.c_double),
                ("wall_u", ctypes.c_double * 3),
                ("batch_graph", ctypes.c_int32)]


class tau1_info(ctypes.Structure):
    _fields_ = [("lattice", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("n_samples", ctypes.c_int32), ("kernel", ctypes.c_int32),
                ("tile", ctypes.c_int32), ("graph_chunk", ctypes.c_int32),
                ("layout", ctypes.c_int32),
                ("n_nodes", ctypes.c_int64), ("n_fluid", ctypes.c_int64),
                ("steps_done", ctypes.c_int64), ("bytes_per_step", ctypes.c_double),
                ("work_items", ctypes.c_int64), ("launches_per_step", ctypes.c_int32)]


_LIB = None


def _lib() -> ctypes.CDLL:
    """Load libtau1.so (raises if it has not been built)."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build it with python -m paper_2312_14742_amd.build")
        lib = ctypes.CDLL(LIB_PATH)
        P = ctypes.c_void_p
        st = ctypes.c_int
        lib.tau1_workspace_size.argtypes = [ctypes.POINTER(tau1_desc),
                                            ctypes.POINTER(ctypes.c_size_t)]
        lib.tau1_workspace_size.restype = st
        lib.tau1_create.argtypes = [ctypes.POINTER(tau1_desc), ctypes.POINTER(P)]
        lib.tau1_create.restype = st
        lib.tau1_step.argtypes = [P, ctypes.c_int64]
        lib.tau1_step.restype = st
        lib.tau1_sync.argtypes = [P]
        lib.tau1_sync.restype = st
        lib.tau1_moments.argtypes = [P, ctypes.c_int32, P, P]
        lib.tau1_moments.restype = st
        lib.tau1_moments_drho.argtypes = [P, ctypes.c_int32, P, P]
        lib.tau1_moments_drho.restype = st
        lib.tau1_permeability.argtypes = [P, ctypes.c_int32, ctypes.c_int32,
                                          ctypes.POINTER(ctypes.c_double),
                                          ctypes.POINTER(ctypes.c_double)]
        lib.tau1_permeability.restype = st
        lib.tau1_permeability_noalloc.argtypes = [P, ctypes.c_int32, ctypes.c_int32, P]
        lib.tau1_permeability_noalloc.restype = st
        lib.tau1_autotune.argtypes = [P, ctypes.c_int32]
        lib.tau1_autotune.restype = st
        lib.tau1_get_info.argtypes = [P, ctypes.POINTER(tau1_info)]
        lib.tau1_get_info.restype = st
        lib.tau1_destroy.argtypes = [P]
        lib.tau1_destroy.restype = None
        lib.tau1_strerror.argtypes = [ctypes.c_int]
        lib.tau1_strerror.restype = ctypes.c_char_p
        lib.tau1_copy_probe.argtypes = [P, P, ctypes.c_size_t, ctypes.c_int32,
                                        ctypes.POINTER(ctypes.c_double)]
        lib.tau1_copy_probe.restype = st
        _LIB = lib
    return _LIB


def _check(status: int, what: str):
    if status != TAU1_OK:
        raise Tau1Error(status, what)


def _precision(p) -> int:
    if isinstance(p, str):
        return PRECISIONS[p]
    return int(p)


class Sample:
    """Host inputs of one lattice: solid (nz, ny, nx) uint8, optional drho0 and u0."""

    def __init__(self, solid, drho0=None, u0=None):
        self.solid = np.ascontiguousarray(solid, dtype=np.uint8)
        if self.solid.ndim != 3:
            raise ValueError("solid must have shape (nz, ny, nx)")
        shape = self.solid.shape
        self.drho0 = None if drho0 is None else np.ascontiguousarray(
            np.asarray(drho0, dtype=np.float64).reshape(shape))
        self.u0 = None if u0 is None else np.ascontiguousarray(
            np.asarray(u0, dtype=np.float64).reshape((3,) + shape))

    @property
    def dims(self):
        nz, ny, nx = self.solid.shape
        return nx, ny, nz

    def c_struct(self) -> tau1_sample:
        nx, ny, nz = self.dims
        return tau1_sample(nx, ny, nz, self.solid.ctypes.data,
                           None if self.drho0 is None else self.drho0.ctypes.data,
                           None if self.u0 is None else self.u0.ctypes.data)


def _desc(samples, lattice, precision, g, graph_chunk, kernel, tile, f16_scales,
          tune_cache, layout=-1, x_boundary=0, rho_in=1.0, rho_out=1.0, wall_u=(0.0, 0.0, 0.0),
          batch_graph=0):
    arr = (tau1_sample * len(samples))(*[s.c_struct() for s in samples])
    d = tau1_desc()
    d.lattice = int(lattice)
    d.precision = _precision(precision)
    d.n_samples = len(samples)
    d.graph_chunk = int(graph_chunk)
    d.samples = ctypes.cast(arr, ctypes.POINTER(tau1_sample))
    for a in range(3):
        d.g[a] = float(g[a])
    d.kernel = int(kernel)
    d.tile = int(tile)
    d.f16_log2_scale_rho = int(f16_scales[0])
    d.f16_log2_scale_u = int(f16_scales[1])
    d.tune_cache = None if tune_cache is None else os.fsencode(tune_cache)
    d.layout = int(layout)
    d.x_boundary = int(x_boundary)
    d.rho_in = float(rho_in)
    d.rho_out = float(rho_out)
    for a in range(3):
        d.wall_u[a] = float(wall_u[a]) if a < len(wall_u) else 0.0
    d.batch_graph = int(batch_graph)
    return d, arr


def workspace_size(samples, lattice=19, precision="f32", g=(0.0, 0.0, 0.0),
                   graph_chunk=0, kernel=-1, tile=-1, f16_scales=(0, 0), layout=-1,
                   x_boundary=0, rho_in=1.0, rho_out=1.0, wall_u=(0.0, 0.0, 0.0)) -> int:
    """Device bytes tau1_create needs (host-only call)."""
    samples = [s if isinstance(s, Sample) else Sample(*s) for s in samples]
    d, keep = _desc(samples, lattice, precision, g, graph_chunk, kernel, tile,
                    f16_scales, None, layout, x_boundary, rho_in, rho_out, wall_u)
    n = ctypes.c_size_t(0)
    _check(_lib().tau1_workspace_size(ctypes.byref(d), ctypes.byref(n)),
           "tau1_workspace_size")
    del keep
    return int(n.value)


class Sim:
    """One Tau1 context over one or more samples (batched when several).

    ``precision`` is one of "f64", "f32", "f16", "bf16".  ``kernel`` -1 picks
    automatically, 0 forces the per-node gather kernel, 1 the z-march tiles.
    ``layout`` -1 picks the state layout automatically, 0 is dense, 1 packed
    (all-solid lane chunks not stored).  ``lattice=9`` is the D2Q9 validation
    lattice (samples of shape (1, ny, nx); solid values 0 fluid, 1 wall,
    2 moving wall with velocity ``wall_u``; ``x_boundary=1`` puts Zou-He
    pressure columns at x = 0 (``rho_in``) and x = nx - 1 (``rho_out``)).
    ``batch_graph`` shapes the launches of a batch with several lane layouts:
    1 one chain, 2 a chain per layout side by side, 3 one launch for the
    layouts of rows 64-320 nodes long, 0 automatic (2).
    """

    def __init__(self, samples, lattice=19, precision="f32", g=(0.0, 0.0, 0.0),
                 graph_chunk=0, kernel=-1, tile=-1, f16_scales=(0, 0),
                 tune_cache=None, device="cuda:0", layout=-1, x_boundary=0, rho_in=1.0,
                 rho_out=1.0, wall_u=(0.0, 0.0, 0.0), batch_graph=0):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("Tau1 Sim needs a ROCm GPU (torch.cuda is unavailable)")
        self._torch = torch
        self.device = torch.device(device)
        self.samples = [s if isinstance(s, Sample) else Sample(*s) for s in samples]
        self.lattice = int(lattice)
        self.precision = _precision(precision)
        self.g = tuple(float(x) for x in g)
        lib = _lib()
        d, keep = _desc(self.samples, lattice, precision, g, graph_chunk, kernel, tile,
                        f16_scales, tune_cache, layout, x_boundary, rho_in, rho_out, wall_u,
                        batch_graph)
        n = ctypes.c_size_t(0)
        _check(lib.tau1_workspace_size(ctypes.byref(d), ctypes.byref(n)),
               "tau1_workspace_size")
        with torch.cuda.device(self.device):
            self.workspace = torch.empty(int(n.value) + 256, dtype=torch.uint8,
                                         device=self.device)
            self.stream = torch.cuda.current_stream(self.device)
        ptr = self.workspace.data_ptr()
        aligned = (ptr + 255) // 256 * 256
        d.workspace = aligned
        d.workspace_bytes = int(n.value)
        d.hip_stream = self.stream.cuda_stream
        ctx = ctypes.c_void_p(None)
        with torch.cuda.device(self.device):
            _check(lib.tau1_create(ctypes.byref(d), ctypes.byref(ctx)), "tau1_create")
        self._ctx = ctx
        del keep

    # -- calls -------------------------------------------------------------
    def _c(self):
        if not self._ctx:
            raise RuntimeError("Sim is closed")
        return self._ctx

    def step(self, nsteps: int):
        _check(_lib().tau1_step(self._c(), int(nsteps)), "tau1_step")

    def sync(self):
        _check(_lib().tau1_sync(self._c()), "tau1_sync")

    def _read(self, fn, what, sample, allow_nonfinite):
        s = self.samples[sample]
        shape = s.solid.shape
        first = np.empty(shape, dtype=np.float64)
        u = np.empty((3,) + shape, dtype=np.float64)
        st = fn(self._c(), int(sample), first.ctypes.data, u.ctypes.data)
        if not (allow_nonfinite and st == TAU1_E_NONFINITE):
            _check(st, what)
        return first, u

    def moments(self, sample: int = 0, allow_nonfinite: bool = False):
        """(drho, u) with drho = rho - 1 as stored (tau1_moments_drho), FP64
        numpy arrays of shapes (nz, ny, nx), (3, nz, ny, nx)."""
        return self._read(_lib().tau1_moments_drho, "tau1_moments_drho", sample,
                          allow_nonfinite)

    def rho_u(self, sample: int = 0, allow_nonfinite: bool = False):
        """(rho, u), the physical density and velocity (tau1_moments)."""
        return self._read(_lib().tau1_moments, "tau1_moments", sample, allow_nonfinite)

    def permeability(self, sample: int = 0, axis: int = 0, with_k: bool = True):
        """(k, mass) from the FP64 device reduction (k is None if with_k is False)."""
        k = ctypes.c_double(0.0)
        m = ctypes.c_double(0.0)
        _check(_lib().tau1_permeability(self._c(), int(sample), int(axis),
                                        ctypes.byref(k) if with_k else None,
                                        ctypes.byref(m)), "tau1_permeability")
        return (k.value if with_k else None), m.value

    def permeability_noalloc(self, out, sample: int = 0, axis: int = 0):
        """Enqueue the FP64 reductions with no allocation and no wait; ``out`` is
        a float64 device tensor of at least 4 elements that receives (mass, k,
        fluid count, non-finite count) when the stream gets there."""
        if out.dtype != self._torch.float64 or not out.is_cuda or out.numel() < 4 \
                or not out.is_contiguous():
            raise ValueError("out must be a contiguous float64 device tensor of >= 4 elements")
        _check(_lib().tau1_permeability_noalloc(self._c(), int(sample), int(axis),
                                                out.data_ptr()),
               "tau1_permeability_noalloc")

    def autotune(self, trial_steps: int = 10):
        _check(_lib().tau1_autotune(self._c(), int(trial_steps)), "tau1_autotune")
        return self.info()

    def info(self) -> dict:
        inf = tau1_info()
        _check(_lib().tau1_get_info(self._c(), ctypes.byref(inf)), "tau1_get_info")
        return {f: getattr(inf, f) for f, _ in tau1_info._fields_}

    def close(self):
        if getattr(self, "_ctx", None):
            _lib().tau1_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:   # noqa: BLE001 - interpreter shutdown
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
        return False


def copy_probe(nbytes: int, reps: int = 20, device="cuda:0") -> float:
    """Mean seconds of one copy of nbytes/2 bytes (device copy-bandwidth probe)."""
    import torch
    buf = torch.empty(int(nbytes), dtype=torch.uint8, device=device)
    sec = ctypes.c_double(0.0)
    stream = torch.cuda.current_stream(buf.device).cuda_stream
    _check(_lib().tau1_copy_probe(stream, buf.data_ptr(), int(nbytes), int(reps),
                                  ctypes.byref(sec)), "tau1_copy_probe")
    return sec.value
