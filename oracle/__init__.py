"""FP64 CPU oracle for the Tau1 lattice Boltzmann update (test infrastructure).

Only the test suite, the smoke check and the CPU-baseline leg of the benchmark
may import this package.  It wraps ``tau1_oracle.c`` (plain C, FP64, built with
``-O2 -ffp-contract=off``) through ctypes and shares nothing with the GPU path.

Functions follow the paper's statement of the method:

* :func:`run` -- Eq. (8)-(10) in drho form with halfway bounce-back (Eq. (11)),
  periodic wrap and velocity-shift body forcing; the parity target.
* :func:`bgk_run` -- brute-force standard LBGK, Eq. (4), full populations; at
  omega = 1 it must equal :func:`run` exactly.
* :func:`run_rhoform` -- the same update with rho stored and Eq. (3) evaluated
  as printed.
* :func:`step_nodes` -- one update at chosen nodes from a full state.
* :func:`reduce` -- mass and Darcy permeability.

Two-dimensional validation lattice (``tau1_oracle_2d.c``, a library of its
own): :func:`run_2d` (D2Q9 Tau1 with walls, moving walls and Zou-He pressure
columns), :func:`bgk_run_2d` (its brute-force population counterpart),
:func:`reduce_2d`, :func:`lattice_2d`.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "tau1_oracle.c")
_LIB = os.path.join(_HERE, "libtau1_oracle.so")
_SRC2D = os.path.join(_HERE, "tau1_oracle_2d.c")
_LIB2D = os.path.join(_HERE, "libtau1_oracle_2d.so")

CFLAGS = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
          "-std=c99", "-Wall", "-Wextra", "-shared", "-fPIC"]


def build(force: bool = True) -> str:
    """Compile the oracle libraries with gcc; returns the 3-D library path."""
    for src, lib in ((_SRC, _LIB), (_SRC2D, _LIB2D)):
        if force or not os.path.exists(lib):
            tmp = f"{lib}.{os.getpid()}.tmp"      # concurrent builders never share it
            subprocess.run(["gcc", *CFLAGS, src, "-o", tmp, "-lm"], check=True)
            os.replace(tmp, lib)
    return _LIB


class _Lib:
    """ctypes handle on one build of the oracle library."""

    def __init__(self, path: str):
        lib = ctypes.CDLL(path)
        P = ctypes.c_void_p
        L = ctypes.c_long
        I = ctypes.c_int
        D = ctypes.c_double
        lib.tau1o_lattice.argtypes = [I, P, P, P]
        lib.tau1o_run.argtypes = [I, L, L, L, P, P, P, P, P, P, L, I]
        lib.tau1o_run_rhoform.argtypes = [I, L, L, L, P, P, P, P, P, P, L, I]
        lib.tau1o_bgk_run.argtypes = [I, L, L, L, P, P, P, P, P, P, D, L, I]
        lib.tau1o_step_nodes.argtypes = [I, L, L, L, P, P, P, P, P, P, L, P, P, I]
        lib.tau1o_reduce.argtypes = [L, L, L, P, P, P, P, P, I, D, P, P]
        lib.tau1o_threads.restype = I
        self.lib = lib


_default = None
_override = None


def _load():
    global _default
    if _override is not None:
        return _override.lib
    if _default is None:
        if not os.path.exists(_LIB):
            build(force=True)
        _default = _Lib(_LIB)
    return _default.lib


class use_library:
    """Context manager: route this module's calls to another oracle build
    (used by the mutation tests, which compile deliberately broken copies)."""

    def __init__(self, path: str):
        self._lib = _Lib(path)

    def __enter__(self):
        global _override
        self._prev = _override
        _override = self._lib
        return self

    def __exit__(self, *exc):
        global _override
        _override = self._prev
        return False


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def threads() -> int:
    """OpenMP threads the oracle uses by default."""
    return int(_load().tau1o_threads())


def lattice(q: int):
    """Direction vectors c (q x 3 int), weights w (q) and opposite map (q)."""
    c = np.zeros((q, 3), dtype=np.int32)
    w = np.zeros(q, dtype=np.float64)
    opp = np.zeros(q, dtype=np.int32)
    if _load().tau1o_lattice(q, _ptr(c), _ptr(w), _ptr(opp)) != q:
        raise ValueError(f"unsupported lattice q={q}")
    return c, w, opp


class State:
    """drho = rho - 1 and velocity (ux, uy, uz), FP64, index x + nx*(y + ny*z).

    Arrays are 3-D with shape (nz, ny, nx) so that x is the fastest axis.
    """

    def __init__(self, solid: np.ndarray, drho=None, u=None):
        solid = np.ascontiguousarray(solid, dtype=np.uint8)
        if solid.ndim != 3:
            raise ValueError("solid must be (nz, ny, nx)")
        self.solid = solid
        shape = solid.shape
        self.drho = (np.zeros(shape) if drho is None
                     else np.array(drho, dtype=np.float64, copy=True).reshape(shape))
        if u is None:
            self.u = np.zeros((3,) + shape)
        else:
            self.u = np.array(u, dtype=np.float64, copy=True).reshape((3,) + shape)
        self.drho = np.ascontiguousarray(self.drho)
        self.u = np.ascontiguousarray(self.u)

    @property
    def dims(self):
        nz, ny, nx = self.solid.shape
        return nx, ny, nz

    def copy(self) -> "State":
        return State(self.solid, self.drho, self.u)


def _g(g):
    return np.ascontiguousarray(np.asarray(g, dtype=np.float64).reshape(3))


def run(q: int, st: State, g, nsteps: int, nthreads: int = 0) -> State:
    """Advance a copy of ``st`` by ``nsteps`` Tau1 updates (drho form)."""
    out = st.copy()
    nx, ny, nz = out.dims
    gg = _g(g)
    rc = _load().tau1o_run(q, nx, ny, nz, _ptr(out.solid), _ptr(out.drho),
                           _ptr(out.u[0]), _ptr(out.u[1]), _ptr(out.u[2]),
                           _ptr(gg), nsteps, nthreads)
    if rc != 0:
        raise RuntimeError(f"tau1o_run failed ({rc})")
    return out


def run_rhoform(q: int, st: State, g, nsteps: int, nthreads: int = 0) -> State:
    """Same as :func:`run` but evaluated with rho stored (Eq. (3) as printed)."""
    out = st.copy()
    rho = np.ascontiguousarray(1.0 + out.drho)
    nx, ny, nz = out.dims
    gg = _g(g)
    rc = _load().tau1o_run_rhoform(q, nx, ny, nz, _ptr(out.solid), _ptr(rho),
                                   _ptr(out.u[0]), _ptr(out.u[1]), _ptr(out.u[2]),
                                   _ptr(gg), nsteps, nthreads)
    if rc != 0:
        raise RuntimeError(f"tau1o_run_rhoform failed ({rc})")
    out.drho = rho - 1.0
    return out


def bgk_run(q: int, st: State, g, nsteps: int, omega: float = 1.0,
            nthreads: int = 0) -> State:
    """Brute-force standard LBGK with populations; returns its moments."""
    out = st.copy()
    nx, ny, nz = out.dims
    gg = _g(g)
    rc = _load().tau1o_bgk_run(q, nx, ny, nz, _ptr(out.solid), _ptr(out.drho),
                               _ptr(out.u[0]), _ptr(out.u[1]), _ptr(out.u[2]),
                               _ptr(gg), float(omega), nsteps, nthreads)
    if rc != 0:
        raise RuntimeError(f"tau1o_bgk_run failed ({rc})")
    return out


def step_nodes(q: int, st: State, g, idx, nthreads: int = 0) -> np.ndarray:
    """One update at flat node indices ``idx``; returns (len(idx), 4)."""
    idx = np.ascontiguousarray(np.asarray(idx, dtype=np.int64).ravel())
    out = np.zeros((idx.size, 4), dtype=np.float64)
    nx, ny, nz = st.dims
    gg = _g(g)
    rc = _load().tau1o_step_nodes(q, nx, ny, nz, _ptr(st.solid), _ptr(st.drho),
                                  _ptr(st.u[0]), _ptr(st.u[1]), _ptr(st.u[2]),
                                  _ptr(gg), idx.size, _ptr(idx), _ptr(out),
                                  nthreads)
    if rc != 0:
        raise RuntimeError(f"tau1o_step_nodes failed ({rc})")
    return out


def reduce(st: State, axis: int, g_axis: float):
    """(mass, permeability) of a state; see tau1o_reduce."""
    m = np.zeros(1)
    k = np.zeros(1)
    nx, ny, nz = st.dims
    rc = _load().tau1o_reduce(nx, ny, nz, _ptr(st.solid), _ptr(st.drho),
                              _ptr(st.u[0]), _ptr(st.u[1]), _ptr(st.u[2]),
                              axis, float(g_axis), _ptr(m), _ptr(k))
    if rc != 0:
        raise RuntimeError("tau1o_reduce failed")
    return float(m[0]), float(k[0])


# ---------------------------------------------------------------------------
# Two-dimensional validation lattice (D2Q9)
# ---------------------------------------------------------------------------
_lib2d = None
_override2d = None


def _open2d(path: str):
    lib = ctypes.CDLL(path)
    P, L, I, D = ctypes.c_void_p, ctypes.c_long, ctypes.c_int, ctypes.c_double
    lib.tau1o2_lattice.argtypes = [P, P, P]
    lib.tau1o2_run.argtypes = [L, L, P, P, P, P, P, P, I, D, D, L, I]
    lib.tau1o2_bgk_run.argtypes = [L, L, P, P, P, P, P, P, I, D, D, D, L]
    lib.tau1o2_reduce.argtypes = [L, L, P, P, P, P, P]
    return lib


def _load2d():
    global _lib2d
    if _override2d is not None:
        return _override2d
    if _lib2d is None:
        if not os.path.exists(_LIB2D):
            build(force=True)
        _lib2d = _open2d(_LIB2D)
    return _lib2d


class use_library_2d:
    """Context manager: route the 2-D calls to another build of the 2-D
    oracle (the mutation tests' deliberately broken copies)."""

    def __init__(self, path: str):
        self._lib = _open2d(path)

    def __enter__(self):
        global _override2d
        self._prev = _override2d
        _override2d = self._lib
        return self

    def __exit__(self, *exc):
        global _override2d
        _override2d = self._prev
        return False


def lattice_2d():
    """D2Q9 direction vectors (9 x 2), weights and opposite map."""
    c = np.zeros((9, 2), dtype=np.int32)
    w = np.zeros(9, dtype=np.float64)
    opp = np.zeros(9, dtype=np.int32)
    _load2d().tau1o2_lattice(_ptr(c), _ptr(w), _ptr(opp))
    return c, w, opp


class State2D:
    """Node types (0 fluid, 1 wall, 2 moving wall), drho = rho - 1 and
    velocity (ux, uy), FP64, arrays of shape (ny, nx) (x fastest)."""

    def __init__(self, types: np.ndarray, drho=None, u=None):
        types = np.ascontiguousarray(types, dtype=np.uint8)
        if types.ndim != 2:
            raise ValueError("types must be (ny, nx)")
        self.types = types
        self.drho = (np.zeros(types.shape) if drho is None
                     else np.array(drho, dtype=np.float64, copy=True).reshape(types.shape))
        self.u = (np.zeros((2,) + types.shape) if u is None
                  else np.array(u, dtype=np.float64, copy=True).reshape((2,) + types.shape))

    def copy(self):
        return State2D(self.types, self.drho, self.u)


def _bc_args(g, uw, xbc, rho_in, rho_out):
    return (np.array(g, dtype=np.float64), np.array(uw, dtype=np.float64), int(xbc),
            float(rho_in), float(rho_out))


def run_2d(st: State2D, nsteps: int, g=(0.0, 0.0), uw=(0.0, 0.0), xbc=0, rho_in=1.0,
           rho_out=1.0, nthreads: int = 0) -> State2D:
    """nsteps D2Q9 Tau1 updates of a copy of st (walls, moving walls with
    velocity uw, Zou-He pressure columns at x = 0 and nx - 1 when xbc = 1)."""
    out = st.copy()
    ny, nx = st.types.shape
    ga, ua, xb, ri, ro = _bc_args(g, uw, xbc, rho_in, rho_out)
    ux = np.ascontiguousarray(out.u[0])
    uy = np.ascontiguousarray(out.u[1])
    rc = _load2d().tau1o2_run(nx, ny, _ptr(out.types), _ptr(out.drho), _ptr(ux), _ptr(uy),
                              _ptr(ga), _ptr(ua), xb, ri, ro, int(nsteps), int(nthreads))
    if rc != 0:
        raise RuntimeError(f"tau1o2_run failed ({rc})")
    out.u = np.stack([ux, uy])
    return out


def bgk_run_2d(st: State2D, nsteps: int, omega: float = 1.0, g=(0.0, 0.0), uw=(0.0, 0.0),
               xbc=0, rho_in=1.0, rho_out=1.0) -> State2D:
    """Brute-force D2Q9 LBGK with full populations and the same boundary rules."""
    out = st.copy()
    ny, nx = st.types.shape
    ga, ua, xb, ri, ro = _bc_args(g, uw, xbc, rho_in, rho_out)
    ux = np.ascontiguousarray(out.u[0])
    uy = np.ascontiguousarray(out.u[1])
    rc = _load2d().tau1o2_bgk_run(nx, ny, _ptr(out.types), _ptr(out.drho), _ptr(ux),
                                  _ptr(uy), _ptr(ga), _ptr(ua), xb, ri, ro, float(omega),
                                  int(nsteps))
    if rc != 0:
        raise RuntimeError(f"tau1o2_bgk_run failed ({rc})")
    out.u = np.stack([ux, uy])
    return out


def reduce_2d(st: State2D):
    """(mass = sum of rho over fluid nodes, mean of u_x over all nodes)."""
    ny, nx = st.types.shape
    m = np.zeros(1)
    s = np.zeros(1)
    ux = np.ascontiguousarray(st.u[0])
    _load2d().tau1o2_reduce(nx, ny, _ptr(st.types), _ptr(st.drho), _ptr(ux), _ptr(m), _ptr(s))
    return float(m[0]), float(s[0])
