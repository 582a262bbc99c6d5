"""ctypes wrapper of the 3D FP64 oracle (``lbmhd3_oracle.cpp``).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU
baseline of the benchmark may use it; the GPU library never does.

State arrays are (45, nz, ny, nx) float64: planes 0..26 the D3Q27 populations
in the order of ``lattice()``, then the x, y, z components of the six vector
populations.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

from . import oracle as _o

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "lbmhd3_oracle.cpp")
LIB = os.environ.get("LBMHD3_ORACLE_LIB") or os.path.join(HERE, "liblbmhd3_oracle.so")
NPOP = 45
DIAG_NAMES = ("mass", "mom_x", "mom_y", "mom_z", "flux_x", "flux_y", "flux_z", "e_kin",
              "e_mag", "max_abs_divB", "max_u", "nonfinite")


def build(force: bool = False) -> str:
    if os.environ.get("LBMHD3_ORACLE_LIB"):
        return LIB
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        _o.compile_source(SRC, LIB)
    return LIB


class _P(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("nu", ctypes.c_double), ("eta", ctypes.c_double), ("les", ctypes.c_int32),
                ("cs", ctypes.c_double), ("csb", ctypes.c_double), ("delta", ctypes.c_double),
                ("mrt", ctypes.c_int32), ("s5", ctypes.c_double), ("s7", ctypes.c_double),
                ("s8", ctypes.c_double), ("sg", ctypes.c_double), ("szz", ctypes.c_double)]


@dataclass
class Params:
    """Lattice size, nu, eta (tau0 = 3 nu + 1/2, tau_m0 = 3 eta + 1/2), les
    (0 or 1: Smagorinsky-MHD closure), closure constants cs (C_Sv) and csb
    (C_Sb, None for cs) and the filter width delta.  mrt = 1: moment-space
    collision for f with the rates s5 (2D rows 5, 6), s7, s8, sg (the other
    moments varying along c_z) and szz (the z normal stress); the shears
    take 1/tau."""
    nx: int
    ny: int
    nz: int
    nu: float = 0.01
    eta: float = 0.01
    les: int = 0
    cs: float = 0.1
    delta: float = 1.0
    csb: float | None = None
    mrt: int = 0
    s5: float = 1.0
    s7: float = 1.0
    s8: float = 1.0
    sg: float = 1.0
    szz: float = 1.0

    def c(self) -> _P:
        return _P(self.nx, self.ny, self.nz, self.nu, self.eta, int(self.les), self.cs,
                  self.cs if self.csb is None else self.csb, self.delta, int(self.mrt),
                  self.s5, self.s7, self.s8, self.sg, self.szz)


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = ctypes.CDLL(build())
    return _lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _check(rc, what):
    if rc != 0:
        raise ValueError(f"oracle3 {what} rejected its arguments")


def lattice():
    """(c27 (27, 3), w27 (27,), c6 (6, 3), w6 (6,))."""
    c27, w27, c6, w6 = np.zeros(81), np.zeros(27), np.zeros(18), np.zeros(6)
    lib().orc3_lattice(_ptr(c27), _ptr(w27), _ptr(c6), _ptr(w6))
    return c27.reshape(27, 3), w27, c6.reshape(6, 3), w6


def equilibrium(rho, u, B):
    feq, geq = np.zeros(27), np.zeros(18)
    uu = np.ascontiguousarray(u, dtype=np.float64)
    bb = np.ascontiguousarray(B, dtype=np.float64)
    lib().orc3_equilibrium(ctypes.c_double(rho), _ptr(uu), _ptr(bb), _ptr(feq), _ptr(geq))
    return feq, geq.reshape(3, 6)


def _field(p, a):
    return np.ascontiguousarray(np.broadcast_to(np.asarray(a, dtype=np.float64),
                                                (p.nz, p.ny, p.nx)))


def init(p: Params, rho, ux, uy, uz, bx, by, bz) -> np.ndarray:
    fs = [_field(p, a) for a in (rho, ux, uy, uz, bx, by, bz)]
    st = np.zeros((NPOP, p.nz, p.ny, p.nx))
    _check(lib().orc3_init(ctypes.byref(p.c()), *[_ptr(f) for f in fs], _ptr(st)), "init")
    return st


def collide(p: Params, state, return_tau: bool = False):
    st = np.array(state, dtype=np.float64, order="C", copy=True)
    tau = np.zeros((p.nz, p.ny, p.nx))
    taum = np.zeros((p.nz, p.ny, p.nx))
    _check(lib().orc3_collide(ctypes.byref(p.c()), _ptr(st), _ptr(tau), _ptr(taum)), "collide")
    return (st, tau, taum) if return_tau else st


def stream(p: Params, state) -> np.ndarray:
    st = np.ascontiguousarray(state, dtype=np.float64)
    out = np.zeros_like(st)
    _check(lib().orc3_stream(ctypes.byref(p.c()), _ptr(st), _ptr(out)), "stream")
    return out


def run(p: Params, state, nsteps: int) -> np.ndarray:
    st = np.array(state, dtype=np.float64, order="C", copy=True)
    _check(lib().orc3_run(ctypes.byref(p.c()), _ptr(st), ctypes.c_int64(int(nsteps))), "run")
    return st


def macro(p: Params, state) -> dict:
    st = np.ascontiguousarray(state, dtype=np.float64)
    rho = np.zeros((p.nz, p.ny, p.nx))
    u = np.zeros((3, p.nz, p.ny, p.nx))
    B = np.zeros((3, p.nz, p.ny, p.nx))
    _check(lib().orc3_macro(ctypes.byref(p.c()), _ptr(st), _ptr(rho), _ptr(u), _ptr(B)), "macro")
    return dict(rho=rho, ux=u[0], uy=u[1], uz=u[2], bx=B[0], by=B[1], bz=B[2])


def diag(p: Params, state) -> dict:
    st = np.ascontiguousarray(state, dtype=np.float64)
    out = np.zeros(12)
    _check(lib().orc3_diag(ctypes.byref(p.c()), _ptr(st), _ptr(out)), "diag")
    return dict(zip(DIAG_NAMES, out))
