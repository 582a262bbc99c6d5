"""ctypes front end of the FP64 CPU oracle (``lbmhd_oracle.cpp``).

TEST INFRASTRUCTURE ONLY: the GPU library never imports this module.  Only the
test suite, the smoke check and the CPU-baseline leg of the benchmark use it.

The oracle follows Flint & Vahala, arXiv:1607.08675: D2Q9 MRT collision for f
(Sec. 3, eqs. FluidTMatrix and KinMomentEq), D2Q5 single-relaxation collision
for the vector distribution g (eqs. MagTMatrix and MagMomentEq), rates from the
transport coefficients of Sec. 4.3, the Smagorinsky-MHD closures of Sec. 1.1
and collide-then-stream with unit time step (Sec. 1.2).  State arrays are
float64 of shape (19, ny, nx): f_0..f_8, g_x,0..g_x,4, g_y,0..g_y,4, holding the
pre-collision populations at integer time.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "lbmhd_oracle.cpp")
# LBMHD_ORACLE_LIB selects another build of the same source (the mutation tests
# point it at deliberately broken copies to show the pins catch them).
LIB = os.environ.get("LBMHD_ORACLE_LIB") or os.path.join(HERE, "liblbmhd_oracle.so")

NPOP = 19
NDIAG = 14
ND = 16  # tangent directions carried by one dual-number pass

DIAG_NAMES = (
    "mass", "mom_x", "mom_y", "flux_x", "flux_y", "e_kin", "e_mag",
    "cross_helicity", "max_abs_divB", "enstrophy", "current_sq", "nonfinite",
    "max_u", "divB_over_curlB",
)


def compile_source(src: str, out: str) -> str:
    """g++ -O2 -fopenmp (no fast-math) of one oracle source into a shared library."""
    cmd = ["g++", "-std=c++17", "-O2", "-fopenmp", "-fPIC", "-shared", src, "-o", out + ".tmp"]
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


def build(force: bool = False) -> str:
    """Compile the oracle (unless LBMHD_ORACLE_LIB names a prebuilt variant)."""
    if os.environ.get("LBMHD_ORACLE_LIB"):
        return LIB
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        compile_source(SRC, LIB)
    return LIB


class OrcParams(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
        ("nu", ctypes.c_double), ("eta", ctypes.c_double),
        ("s5", ctypes.c_double), ("s6", ctypes.c_double),
        ("s7", ctypes.c_double), ("s8", ctypes.c_double),
        ("les", ctypes.c_int32),
        ("cs", ctypes.c_double), ("csb", ctypes.c_double), ("delta", ctypes.c_double),
    ]


@dataclass
class Params:
    """Physical parameters in lattice units.

    nu, eta: shear viscosity and resistivity (Sec. 4.3 gives s_3 = s_4 and s_m).
    s5..s8: rates of the non-hydrodynamic moments (not fixed by the paper).
    les: bit 0 = Smagorinsky-MHD closure, bit 1 = kinetic closure (filtered
    equilibria), bit 2 = cross-helicity closure (eqs. CHClosureV/B; not with
    bit 0), so 0 plain, 1, 2, 3, 4 or 6; cs: closure constant C_Sv of the eddy
    viscosity; csb: constant C_Sb of the eddy resistivity (eqs.
    SmagorinskyMHDClosureV/B), None for the same as cs; delta: filter width.
    """
    nx: int
    ny: int
    nu: float = 0.01
    eta: float = 0.01
    s5: float = 1.0
    s6: float = 1.0
    s7: float = 1.0
    s8: float = 1.0
    les: int = 0
    cs: float = 0.1
    delta: float = 1.0
    csb: float | None = None

    def c(self) -> OrcParams:
        csb = self.cs if self.csb is None else self.csb
        return OrcParams(self.nx, self.ny, self.nu, self.eta, self.s5, self.s6, self.s7,
                         self.s8, int(self.les), self.cs, csb, self.delta)


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = ctypes.CDLL(LIB)
        P = ctypes.POINTER
        d = ctypes.c_double
        pd = P(d)
        pp = P(OrcParams)
        L.orc_num_threads.restype = ctypes.c_int
        L.orc_lattice.argtypes = [pd] * 6
        L.orc_matrices.argtypes = [pd] * 3
        L.orc_equilibrium.argtypes = [d] * 5 + [pd, pd]
        L.orc_moment_equilibria.argtypes = [d] * 5 + [pd, pd]
        L.orc_init.argtypes = [pp] + [pd] * 6
        L.orc_collide.argtypes = [pp, pd, pd, pd]
        L.orc_stream.argtypes = [pp, pd, pd]
        L.orc_run.argtypes = [pp, pd, ctypes.c_int64]
        L.orc_macro.argtypes = [pp] + [pd] * 6
        L.orc_diag.argtypes = [pp, pd, pd]
        L.orc_energy.argtypes = [pp, pd]
        L.orc_energy.restype = d
        L.orc_tm_inverse.argtypes = [pd]
        L.orc_filter_terms.argtypes = [d] * 4 + [pd] * 4
        L.orc_filtered_moment_corrections.argtypes = [d] * 6 + [pd] * 3
        L.orc_gradients.argtypes = [pp, pd, pd]
        L.orc_gradients.restype = ctypes.c_int
        L.orc_tl_collide.argtypes = [pp, pd, pd, pd, ctypes.c_int]
        L.orc_tl_energy.argtypes = [pp] + [pd] * 7 + [ctypes.c_int, ctypes.c_int64, pd, pd]
        for name in ("orc_init", "orc_collide", "orc_stream", "orc_run", "orc_macro",
                     "orc_diag", "orc_tl_collide", "orc_tl_energy"):
            getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _check(rc: int, what: str):
    if rc != 0:
        raise ValueError(f"oracle {what} rejected its arguments (rc={rc})")


def num_threads() -> int:
    return lib().orc_num_threads()


def lattice():
    """(cx, cy, w, Cx, Cy, w') as float64 arrays."""
    a = [np.zeros(9) for _ in range(3)] + [np.zeros(5) for _ in range(3)]
    lib().orc_lattice(*[_ptr(x) for x in a])
    return tuple(a)


def matrices():
    """(T, T^-1, T_m) as float64 arrays."""
    T, Ti, Tm = np.zeros((9, 9)), np.zeros((9, 9)), np.zeros((5, 5))
    lib().orc_matrices(_ptr(T), _ptr(Ti), _ptr(Tm))
    return T, Ti, Tm


def tm_inverse():
    out = np.zeros((5, 5))
    lib().orc_tm_inverse(_ptr(out))
    return out


def filter_terms(d2, X, Y, Z, dX, dY, dZ):
    """(product term, ratio term) of the filter-width expansions at one point."""
    arrs = [np.ascontiguousarray(a, dtype=np.float64) for a in (dX, dY, dZ)]
    out = np.zeros(2)
    lib().orc_filter_terms(d2, X, Y, Z, *[_ptr(a) for a in arrs], _ptr(out))
    return out[0], out[1]


def filtered_moment_corrections(d2, rho, jx, jy, bx, by, grad):
    """Delta^2 parts (dM^eq (9,), dN^eq (2, 5)) at one site; grad = d_x, d_y of
    (rho, j_x, j_y, B_x, B_y) as 10 values."""
    g = np.ascontiguousarray(grad, dtype=np.float64)
    dm, dn = np.zeros(9), np.zeros(10)
    lib().orc_filtered_moment_corrections(d2, rho, jx, jy, bx, by, _ptr(g), _ptr(dm), _ptr(dn))
    return dm, dn.reshape(2, 5)


def gradients(p: Params, state: np.ndarray) -> np.ndarray:
    """(10, ny, nx): d_x, d_y of rho, j_x, j_y, B_x, B_y (kinetic-closure stencil)."""
    st = np.ascontiguousarray(state, dtype=np.float64)
    out = np.zeros((10, p.ny, p.nx))
    _check(lib().orc_gradients(ctypes.byref(p.c()), _ptr(st), _ptr(out)), "gradients")
    return out


def equilibrium(rho, ux, uy, bx, by):
    """f^eq (9,) and g^eq (2, 5) at one site."""
    feq, geq = np.zeros(9), np.zeros(10)
    lib().orc_equilibrium(rho, ux, uy, bx, by, _ptr(feq), _ptr(geq))
    return feq, geq.reshape(2, 5)


def moment_equilibria(rho, jx, jy, bx, by):
    """M^eq (9,) and N^eq (2, 5) at one site."""
    meq, neq = np.zeros(9), np.zeros(10)
    lib().orc_moment_equilibria(rho, jx, jy, bx, by, _ptr(meq), _ptr(neq))
    return meq, neq.reshape(2, 5)


def _fields(p: Params, *fs):
    out = []
    for f in fs:
        a = np.ascontiguousarray(np.broadcast_to(np.asarray(f, dtype=np.float64),
                                                 (p.ny, p.nx)))
        out.append(a)
    return out


def init(p: Params, rho, ux, uy, bx, by) -> np.ndarray:
    """Equilibrium state (19, ny, nx) for the given macroscopic fields."""
    fs = _fields(p, rho, ux, uy, bx, by)
    st = np.zeros((NPOP, p.ny, p.nx))
    _check(lib().orc_init(ctypes.byref(p.c()), *[_ptr(f) for f in fs], _ptr(st)), "init")
    return st


def collide(p: Params, state: np.ndarray, return_tau: bool = False):
    """One collision at every site (returns a new array)."""
    st = np.array(state, dtype=np.float64, order="C", copy=True)
    tau = np.zeros((p.ny, p.nx))
    taum = np.zeros((p.ny, p.nx))
    _check(lib().orc_collide(ctypes.byref(p.c()), _ptr(st), _ptr(tau), _ptr(taum)), "collide")
    return (st, tau, taum) if return_tau else st


def stream(p: Params, state: np.ndarray) -> np.ndarray:
    st = np.ascontiguousarray(state, dtype=np.float64)
    out = np.zeros_like(st)
    _check(lib().orc_stream(ctypes.byref(p.c()), _ptr(st), _ptr(out)), "stream")
    return out


def run(p: Params, state: np.ndarray, nsteps: int) -> np.ndarray:
    """nsteps collide-then-stream updates (returns a new array)."""
    st = np.array(state, dtype=np.float64, order="C", copy=True)
    _check(lib().orc_run(ctypes.byref(p.c()), _ptr(st), int(nsteps)), "run")
    return st


def macro(p: Params, state: np.ndarray):
    """dict of rho, ux, uy, bx, by (each (ny, nx))."""
    st = np.ascontiguousarray(state, dtype=np.float64)
    out = [np.zeros((p.ny, p.nx)) for _ in range(5)]
    _check(lib().orc_macro(ctypes.byref(p.c()), _ptr(st), *[_ptr(o) for o in out]), "macro")
    return dict(zip(("rho", "ux", "uy", "bx", "by"), out))


def diag(p: Params, state: np.ndarray) -> dict:
    st = np.ascontiguousarray(state, dtype=np.float64)
    out = np.zeros(NDIAG)
    _check(lib().orc_diag(ctypes.byref(p.c()), _ptr(st), _ptr(out)), "diag")
    return dict(zip(DIAG_NAMES, out.tolist()))


def energy(p: Params, state: np.ndarray) -> float:
    st = np.ascontiguousarray(state, dtype=np.float64)
    return float(lib().orc_energy(ctypes.byref(p.c()), _ptr(st)))


def _cs_tangents(dcs, ndir):
    if dcs is None:
        return np.zeros(2 * ndir)
    d = np.asarray(dcs, dtype=np.float64)
    if d.shape == (ndir,):
        d = np.stack([d, d], axis=1)
    if d.shape != (ndir, 2):
        raise ValueError("closure-constant tangents must have shape (ndir,) or (ndir, 2)")
    return np.ascontiguousarray(d.reshape(-1))


def tl_collide(p: Params, state: np.ndarray, dstate: np.ndarray, dcs=None):
    """Tangent-linear collision: returns (state', dstate') for ndir directions.

    dstate has shape (ndir, 19, ny, nx); dcs, the tangents of the closure
    constants, is (ndir, 2) for (C_Sv, C_Sb) or (ndir,) for both moving together.
    """
    st = np.array(state, dtype=np.float64, order="C", copy=True)
    ds = np.array(dstate, dtype=np.float64, order="C", copy=True)
    ndir = ds.shape[0]
    dc = _cs_tangents(dcs, ndir)
    _check(lib().orc_tl_collide(ctypes.byref(p.c()), _ptr(st), _ptr(ds), _ptr(dc), ndir),
           "tl_collide")
    return st, ds


def tl_energy(p: Params, fields, dfields, dcs, nsteps: int):
    """J and <grad J, v_k> for the final total energy after nsteps.

    fields: (rho, ux, uy, bx, by); dfields: (ndir, 4, ny, nx) tangents of
    (ux, uy, bx, by); dcs: tangents of the closure constants, (ndir, 2) for
    (C_Sv, C_Sb) or (ndir,) for both moving together.
    """
    fs = _fields(p, *fields)
    dfl = np.ascontiguousarray(dfields, dtype=np.float64)
    ndir = dfl.shape[0]
    dc = _cs_tangents(dcs, ndir)
    J = np.zeros(1)
    dJ = np.zeros(ndir)
    _check(lib().orc_tl_energy(ctypes.byref(p.c()), *[_ptr(f) for f in fs], _ptr(dfl),
                               _ptr(dc), ndir, int(nsteps), _ptr(J), _ptr(dJ)), "tl_energy")
    return float(J[0]), dJ
