"""Python binding of the 3D lattice (``include/lbmhd3.h``): argument
marshalling only; every step runs in the library's kernels.

Fields are float64 tensors of shape (nz, ny, nx); populations (45, nz, ny, nx)
in the plane order of the header.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import torch

from . import _capi as C


@dataclass
class LBMHD3Config:
    """nx, ny, nz: periodic lattice; nu, eta: viscosity and resistivity
    (tau0 = 3 nu + 1/2, tau_m0 = 3 eta + 1/2); les: 1 for the Smagorinsky-MHD
    closure; cs, cs_b: closure constants C_Sv and C_Sb (None: same as cs);
    delta: filter width; storage: "fp32" or "fp16" (deviation from the rest
    state, FP16 scaled by 2^10).  mrt = 1: moment-space collision for f in the
    tensor-product basis of the paper's D2Q9 rows and (1, c_z, 3 c_z^2 - 1),
    with the rates s5 (2D rows 5, 6), s7, s8, sg (other moments varying along
    c_z) and szz (z normal stress); the shears take 1/tau."""
    nx: int
    ny: int
    nz: int
    nu: float = 0.01
    eta: float = 0.01
    les: int = 1
    cs: float = 0.1
    delta: float = 1.0
    cs_b: float | None = None
    storage: str = "fp32"
    mrt: int = 0
    s5: float = 1.0
    s7: float = 1.0
    s8: float = 1.0
    sg: float = 1.0
    szz: float = 1.0

    def c_params(self) -> C.Params3:
        st = {"fp32": C.LBMHD_FP32, "fp16": C.LBMHD_FP16}[self.storage]
        return C.Params3(self.nx, self.ny, self.nz, self.nu, self.eta, int(self.les), self.cs,
                         self.cs if self.cs_b is None else self.cs_b, self.delta, st,
                         int(self.mrt), self.s5, self.s7, self.s8, self.sg, self.szz)


def _ptr(t: torch.Tensor) -> ctypes.c_void_p:
    return ctypes.c_void_p(t.data_ptr())


class Lattice3:
    """One periodic 3D LB-MHD lattice on the current HIP device and stream."""

    def __init__(self, cfg: LBMHD3Config, device: str | torch.device = "cuda",
                 stream: torch.cuda.Stream | None = None):
        self.cfg = cfg
        self.device = torch.device(device)
        L = C.lib()
        self._L = L
        h = ctypes.c_void_p()
        self._check_rc(L.lbmhd3_create(ctypes.byref(cfg.c_params()), ctypes.byref(h)),
                       "lbmhd3_create", None)
        self._h = h
        lat, ws = ctypes.c_size_t(), ctypes.c_size_t()
        self._check(L.lbmhd3_sizes(h, ctypes.byref(lat), ctypes.byref(ws)), "lbmhd3_sizes")
        self.lattice_bytes, self.workspace_bytes = lat.value, ws.value
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self._a = torch.empty(self.lattice_bytes, dtype=torch.uint8, device=self.device)
        self._b = torch.empty(self.lattice_bytes, dtype=torch.uint8, device=self.device)
        self._ws = torch.empty(self.workspace_bytes, dtype=torch.uint8, device=self.device)
        self._check(L.lbmhd3_bind(h, _ptr(self._a), self.lattice_bytes, _ptr(self._b),
                                  self.lattice_bytes, _ptr(self._ws), self.workspace_bytes,
                                  ctypes.c_void_p(self.stream.cuda_stream)), "lbmhd3_bind")

    def _check_rc(self, rc, what, h):
        C.check(rc, what, h, self._L.lbmhd3_last_error)

    def _check(self, rc, what):
        self._check_rc(rc, what, self._h)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            self._L.lbmhd3_destroy(h)
            self._h = None

    def _field(self, a) -> torch.Tensor:
        shape = (self.cfg.nz, self.cfg.ny, self.cfg.nx)
        t = torch.as_tensor(a, dtype=torch.float64)
        return t.expand(shape).to(self.device).contiguous()

    def init_fields(self, rho, ux, uy, uz, bx, by, bz) -> "Lattice3":
        fs = [self._field(a) for a in (rho, ux, uy, uz, bx, by, bz)]
        self._check(self._L.lbmhd3_init_fields(self._h, *[_ptr(f) for f in fs]),
                    "lbmhd3_init_fields")
        self._keep = fs
        return self

    def step(self, n: int = 1) -> "Lattice3":
        self._check(self._L.lbmhd3_step(self._h, int(n)), "lbmhd3_step")
        return self

    def macro(self) -> dict:
        shape = (self.cfg.nz, self.cfg.ny, self.cfg.nx)
        rho = torch.empty(shape, dtype=torch.float64, device=self.device)
        u = torch.empty((3,) + shape, dtype=torch.float64, device=self.device)
        B = torch.empty((3,) + shape, dtype=torch.float64, device=self.device)
        self._check(self._L.lbmhd3_macro(self._h, _ptr(rho), _ptr(u), _ptr(B)), "lbmhd3_macro")
        return dict(rho=rho, ux=u[0], uy=u[1], uz=u[2], bx=B[0], by=B[1], bz=B[2])

    def diag(self, raise_nonfinite: bool = False) -> dict:
        d = C.Diag3()
        rc = self._L.lbmhd3_diag(self._h, ctypes.byref(d))
        if rc != C.LBMHD_ERR_NONFINITE or raise_nonfinite:
            self._check(rc, "lbmhd3_diag")
        return d.as_dict()

    def populations(self) -> torch.Tensor:
        out = torch.empty((45, self.cfg.nz, self.cfg.ny, self.cfg.nx), dtype=torch.float64,
                          device=self.device)
        self._check(self._L.lbmhd3_get_populations(self._h, _ptr(out)), "lbmhd3_get_populations")
        return out

    def set_populations(self, pops, step: int = 0) -> "Lattice3":
        t = torch.as_tensor(pops, dtype=torch.float64).to(self.device).contiguous()
        if tuple(t.shape) != (45, self.cfg.nz, self.cfg.ny, self.cfg.nx):
            raise ValueError("populations must have shape (45, nz, ny, nx)")
        self._check(self._L.lbmhd3_set_populations(self._h, _ptr(t), int(step)),
                    "lbmhd3_set_populations")
        self._keep = t
        return self
