"""Python access to the FP64 CPU oracle (oracle/oracle.c).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU-baseline
leg of the benchmark may import this module; the product package never does.

Array conventions (the same data format the GPU library exchanges, written out
here on its own):
  * scalar fields have shape (nz, ny, nx) -- x fastest;
  * vector fields have shape (3, nz, ny, nx);
  * populations have shape (2, 19, nz, ny, nx): component, direction, site.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

Q = 19


def build(force: bool = True) -> str:
    """Compile oracle.c with gcc: plain IEEE doubles, no FMA contraction, no
    fast-math; OpenMP over sites."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-fopenmp",
               "-ffp-contract=off", "-fno-fast-math", _SRC, "-o", tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


class _Params(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("eq_kind", ctypes.c_int32),
        ("force_kind", ctypes.c_int32),
        ("wall_kind", ctypes.c_int32),
        ("tau", ctypes.c_double * 2),
        ("G", ctypes.c_double),
        ("g", ctypes.c_double * 3),
        ("rho_s", ctypes.c_double),
        ("solid", ctypes.c_void_p),
    ]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        pp = ctypes.POINTER(_Params)
        lib.ora_lattice.argtypes = [ctypes.POINTER(ctypes.c_int32), dp, ctypes.POINTER(ctypes.c_int32)]
        lib.ora_feq.argtypes = [ctypes.c_int, ctypes.c_double, dp, dp]
        lib.ora_regularize.argtypes = [dp, dp, dp, dp]
        lib.ora_init.argtypes = [pp, dp, dp, dp, dp]
        lib.ora_moments.argtypes = [pp, dp, dp, dp, dp]
        lib.ora_moments.restype = ctypes.c_int
        lib.ora_step.argtypes = [pp, dp, dp]
        lib.ora_step.restype = ctypes.c_int
        lib.ora_run.argtypes = [pp, dp, ctypes.c_int64]
        lib.ora_run.restype = ctypes.c_int
        lib.ora_reduce.argtypes = [pp, dp, dp]
        lib.ora_reduce.restype = ctypes.c_int
        lib.ora_step_sites.argtypes = [pp, dp, ctypes.c_int64, ctypes.POINTER(ctypes.c_int64), dp]
        lib.ora_step_sites.restype = ctypes.c_int
        lib.ora_set_threads.argtypes = [ctypes.c_int]
        lib.ora_get_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def _dp(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


@dataclass
class Params:
    """Problem statement of Section 2: lattice size, per-component relaxation
    times (Eq. 5), coupling G (Eq. 7, paper sign), body acceleration, wall
    parameter rho^s (after Eq. 11), equilibrium kind (0: Eq. 3 as printed),
    forcing kind (0: with its second-order part; 1: first order only)."""
    nx: int
    ny: int
    nz: int
    tau: tuple = (1.0, 1.0)
    G: float = 0.0
    g: tuple = (0.0, 0.0, 0.0)
    rho_s: float = 0.0
    eq_kind: int = 0
    force_kind: int = 0
    wall_kind: int = 0
    solid: np.ndarray | None = None
    _keep: list = field(default_factory=list, repr=False)

    @property
    def shape(self):
        return (self.nz, self.ny, self.nx)

    def c_struct(self) -> _Params:
        s = _Params()
        s.nx, s.ny, s.nz, s.eq_kind = self.nx, self.ny, self.nz, self.eq_kind
        s.force_kind = self.force_kind
        s.wall_kind = self.wall_kind
        s.tau[0], s.tau[1] = self.tau
        s.G = self.G
        for d in range(3):
            s.g[d] = self.g[d]
        s.rho_s = self.rho_s
        if self.solid is not None:
            m = np.ascontiguousarray(self.solid, dtype=np.uint8).reshape(self.shape)
            self._keep = [m]
            s.solid = m.ctypes.data
        else:
            s.solid = None
        return s


def set_threads(n: int) -> None:
    _load().ora_set_threads(int(n))


def get_threads() -> int:
    return int(_load().ora_get_threads())


def lattice():
    """(c[19,3] int, w[19], opp[19]) as the oracle holds them."""
    lib = _load()
    c = np.zeros(Q * 3, np.int32)
    w = np.zeros(Q, np.float64)
    opp = np.zeros(Q, np.int32)
    lib.ora_lattice(c.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), _dp(w),
                    opp.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
    return c.reshape(Q, 3), w, opp


def feq(rho: float, u, eq_kind: int = 0) -> np.ndarray:
    out = np.zeros(Q)
    uu = np.ascontiguousarray(u, dtype=np.float64)
    _load().ora_feq(int(eq_kind), float(rho), _dp(uu), _dp(out))
    return out


def regularize(f, fe):
    f = np.ascontiguousarray(f, dtype=np.float64)
    fe = np.ascontiguousarray(fe, dtype=np.float64)
    fp = np.zeros(Q)
    Pi = np.zeros(9)
    _load().ora_regularize(_dp(f), _dp(fe), _dp(fp), _dp(Pi))
    return fp, Pi.reshape(3, 3)


def init(p: Params, rho1, rho2, u=None) -> np.ndarray:
    r1 = np.ascontiguousarray(rho1, dtype=np.float64).reshape(p.shape)
    r2 = np.ascontiguousarray(rho2, dtype=np.float64).reshape(p.shape)
    f = np.zeros((2, Q) + p.shape)
    up = None
    if u is not None:
        uu = np.ascontiguousarray(u, dtype=np.float64).reshape((3,) + p.shape)
        up = _dp(uu)
    cs = p.c_struct()
    _load().ora_init(ctypes.byref(cs), _dp(r1), _dp(r2), up, _dp(f))
    return f


def step(p: Params, f: np.ndarray) -> np.ndarray:
    f = np.ascontiguousarray(f, dtype=np.float64)
    out = np.zeros_like(f)
    cs = p.c_struct()
    if _load().ora_step(ctypes.byref(cs), _dp(f), _dp(out)) != 0:
        raise MemoryError("oracle step: allocation failed")
    return out


def run(p: Params, f: np.ndarray, n: int) -> np.ndarray:
    g = np.array(f, dtype=np.float64, order="C", copy=True)
    cs = p.c_struct()
    if _load().ora_run(ctypes.byref(cs), _dp(g), int(n)) != 0:
        raise MemoryError("oracle run: allocation failed")
    return g


def moments(p: Params, f: np.ndarray):
    """(rho1, rho2, uF[3]) of the state f; zeros on solid sites."""
    f = np.ascontiguousarray(f, dtype=np.float64)
    r1 = np.zeros(p.shape)
    r2 = np.zeros(p.shape)
    uF = np.zeros((3,) + p.shape)
    cs = p.c_struct()
    if _load().ora_moments(ctypes.byref(cs), _dp(f), _dp(r1), _dp(r2), _dp(uF)) != 0:
        raise MemoryError("oracle moments: allocation failed")
    return r1, r2, uF


def reduce(p: Params, f: np.ndarray) -> np.ndarray:
    """[sum rho1, sum rho2, sum rho uF_x, _y, _z] over fluid sites."""
    f = np.ascontiguousarray(f, dtype=np.float64)
    out = np.zeros(5)
    cs = p.c_struct()
    if _load().ora_reduce(ctypes.byref(cs), _dp(f), _dp(out)) != 0:
        raise MemoryError("oracle reduce: allocation failed")
    return out


def step_sites(p: Params, f: np.ndarray, sites) -> np.ndarray:
    """f(t+1) at the given flat site indices, shape (k, 2, 19)."""
    f = np.ascontiguousarray(f, dtype=np.float64)
    s = np.ascontiguousarray(sites, dtype=np.int64)
    out = np.zeros((len(s), 2, Q))
    cs = p.c_struct()
    rc = _load().ora_step_sites(ctypes.byref(cs), _dp(f), len(s),
                                s.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), _dp(out))
    if rc != 0:
        raise ValueError("oracle step_sites: a requested site is solid")
    return out
