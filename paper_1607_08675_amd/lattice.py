"""``Lattice``: a thin Python handle over the C ABI of ``liblbmhd.so``.

PyTorch owns every device buffer (two encoded lattices and the workspace) and
supplies the stream; the library runs every step of the update in its own HIP
kernels.  Field arrays are float64 (ny, nx); population arrays are float64
(19, ny, nx) with planes f_0..f_8, g_x,0..4, g_y,0..4 (Flint & Vahala,
arXiv:1607.08675, Sec. 3 velocity order).
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import numpy as np
import torch

from . import _capi as C

FIELDS = ("rho", "ux", "uy", "bx", "by")


@dataclass
class LBMHDConfig:
    """Lattice size and physical parameters (lattice units).

    nu, eta: viscosity and resistivity (tau0 = 3 nu + 1/2, tau_m0 = 3 eta + 1/2).
    s5 (= s6), s7, s8: rates of the non-hydrodynamic moments.
    les: bit mask -- 0 plain, 1 Smagorinsky-MHD closure, 2 kinetic closure
    (filtered equilibria), 3 both, 4 cross-helicity closure (with backscatter),
    6 kinetic and cross-helicity; cs: closure constant C_Sv of the eddy
    viscosity; cs_b: constant C_Sb of the eddy resistivity (None: same as cs);
    delta: filter width.
    storage: "fp32" or "fp16" (deviation from the rest state, FP16 scaled by 2^10).
    inplace: one lattice updated in place (AA pattern) instead of two; not with
    the closures that read neighbours (les = 2, 3, 4, 6).
    steps_per_pass: with two lattices, step() can advance several steps per
    pass over the lattice with the intermediate states kept on chip, equal to
    single steps bit for bit in both storages.  les = 0 or 1: 0 (default)
    takes three per pass with FP32 storage and two with FP16 where the lattice
    is large enough for it to pay; 3: three with FP32, two with FP16; 2: two.
    les = 2, 3, 4, 6: 0 takes two with FP32 storage where the lattice is large
    enough, 2 and 3 two.  1: one.
    """
    nx: int
    ny: int
    nu: float = 0.01
    eta: float = 0.01
    s5: float = 1.0
    s7: float = 1.0
    s8: float = 1.0
    les: int = 1
    cs: float = 0.1
    delta: float = 1.0
    storage: str = "fp32"
    cs_b: float | None = None
    inplace: bool = False
    steps_per_pass: int = 0

    @property
    def csb(self) -> float:
        return self.cs if self.cs_b is None else self.cs_b

    def c_params(self) -> C.Params:
        st = {"fp32": C.LBMHD_FP32, "fp16": C.LBMHD_FP16}[self.storage]
        return C.Params(self.nx, self.ny, self.nu, self.eta, self.s5, self.s5, self.s7,
                        self.s8, int(self.les), self.cs, self.csb, self.delta, st,
                        int(self.inplace), int(self.steps_per_pass))


def _ptr(t: torch.Tensor) -> ctypes.c_void_p:
    return ctypes.c_void_p(t.data_ptr())


class Lattice:
    """One periodic LB-MHD lattice on the current CUDA (HIP) device and stream."""

    def __init__(self, cfg: LBMHDConfig, device: str | torch.device = "cuda",
                 stream: torch.cuda.Stream | None = None):
        self.cfg = cfg
        self.device = torch.device(device)
        L = C.lib()
        self._L = L
        h = ctypes.c_void_p()
        C.check(L.lbmhd_create(ctypes.byref(cfg.c_params()), ctypes.byref(h)), "lbmhd_create")
        self._h = h
        sizes = [ctypes.c_size_t() for _ in range(4)]
        C.check(L.lbmhd_sizes(h, *[ctypes.byref(s) for s in sizes]), "lbmhd_sizes", h)
        (self.lattice_bytes, self.workspace_bytes,
         self.adj_lattice_bytes, self.adj_acc_bytes) = (s.value for s in sizes)
        lay = [ctypes.c_int64() for _ in range(4)]
        C.check(L.lbmhd_layout(h, *[ctypes.byref(v) for v in lay]), "lbmhd_layout", h)
        # elements: population q of site (x, y) at q * plane + y * pitch + x
        self.pitch, self.plane, self.adj_pitch, self.adj_plane = (v.value for v in lay)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self._a = torch.empty(self.lattice_bytes, dtype=torch.uint8, device=self.device)
        self._b = (None if cfg.inplace else
                   torch.empty(self.lattice_bytes, dtype=torch.uint8, device=self.device))
        self._ws = torch.empty(self.workspace_bytes, dtype=torch.uint8, device=self.device)
        b = ctypes.c_void_p(0) if self._b is None else _ptr(self._b)
        C.check(L.lbmhd_bind(h, _ptr(self._a), self.lattice_bytes, b,
                             0 if self._b is None else self.lattice_bytes, _ptr(self._ws),
                             self.workspace_bytes,
                             ctypes.c_void_p(self.stream.cuda_stream)), "lbmhd_bind", h)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            self._L.lbmhd_destroy(h)
            self._h = None

    # ----------------------------------------------------------- helpers
    def _field(self, a) -> torch.Tensor:
        t = torch.as_tensor(a, dtype=torch.float64)
        t = t.expand(self.cfg.ny, self.cfg.nx) if t.dim() == 0 else t
        if tuple(t.shape) != (self.cfg.ny, self.cfg.nx):
            raise ValueError(f"field shape {tuple(t.shape)} != (ny, nx)")
        return t.to(self.device).contiguous()

    def _check(self, rc, what):
        C.check(rc, what, self._h)

    # ------------------------------------------------------------ the ABI
    def init_fields(self, rho, ux, uy, bx, by) -> "Lattice":
        fs = [self._field(a) for a in (rho, ux, uy, bx, by)]
        self._check(self._L.lbmhd_init_fields(self._h, *[_ptr(f) for f in fs]),
                    "lbmhd_init_fields")
        self._keep = fs  # inputs stay alive until the stream has used them
        return self

    def step(self, n: int = 1) -> "Lattice":
        self._check(self._L.lbmhd_step(self._h, int(n)), "lbmhd_step")
        return self

    def step_between(self, src: torch.Tensor, dst: torch.Tensor):
        """One step from encoded lattice src into dst; the current state is untouched."""
        if src.numel() < self.lattice_bytes or dst.numel() < self.lattice_bytes:
            raise ValueError("state buffer too small")
        self._check(self._L.lbmhd_step_between(self._h, _ptr(src), _ptr(dst)),
                    "lbmhd_step_between")

    def step_store(self, src: torch.Tensor, store: torch.Tensor, n: int):
        """n steps from encoded lattice src; state t (1..n) goes to row t - 1 of
        store, a (>= n, lattice_bytes or more) uint8 tensor whose row stride is a
        multiple of 256 bytes.  One library call for all n steps."""
        stride = self._store_stride(store, n)
        if src.numel() < self.lattice_bytes:
            raise ValueError("state buffer too small")
        self._check(self._L.lbmhd_step_store(self._h, _ptr(src),
                                             _ptr(store) if n else ctypes.c_void_p(0),
                                             stride, int(n)), "lbmhd_step_store")

    def step_store_pairs(self, src: torch.Tensor, store: torch.Tensor, npairs: int):
        """npairs pairs of steps from encoded lattice src, one pass each; state
        2k (k = 1..npairs) goes to row k - 1 of store (odd states are not
        kept).  The current state is untouched."""
        stride = self._store_stride(store, npairs)
        if src.numel() < self.lattice_bytes:
            raise ValueError("state buffer too small")
        self._check(self._L.lbmhd_step_store_pairs(self._h, _ptr(src),
                                                   _ptr(store) if npairs else ctypes.c_void_p(0),
                                                   stride, int(npairs)),
                    "lbmhd_step_store_pairs")

    def _store_stride(self, store: torch.Tensor, n: int) -> int:
        if n == 0:
            return self.lattice_bytes
        if store.dim() != 2 or store.dtype != torch.uint8 or store.shape[0] < n:
            raise ValueError("store must be a 2D uint8 tensor with a row per state")
        if store.shape[1] < self.lattice_bytes or store.stride(1) != 1:
            raise ValueError("store rows must hold a lattice each")
        return int(store.stride(0))

    def macro(self) -> dict:
        out = [torch.empty(self.cfg.ny, self.cfg.nx, dtype=torch.float64, device=self.device)
               for _ in FIELDS]
        self._check(self._L.lbmhd_macro(self._h, *[_ptr(o) for o in out]), "lbmhd_macro")
        return dict(zip(FIELDS, out))

    def macro_box(self, w: int) -> dict:
        """rho, u, B averaged over w x w blocks: fields of (ny / w, nx / w)."""
        out = [torch.empty(self.cfg.ny // w, self.cfg.nx // w, dtype=torch.float64,
                           device=self.device) for _ in FIELDS]
        self._check(self._L.lbmhd_macro_box(self._h, int(w), *[_ptr(o) for o in out]),
                    "lbmhd_macro_box")
        return dict(zip(FIELDS, out))

    def mismatch(self, targets, state: torch.Tensor | None = None) -> float:
        """sum |u - u_t|^2 + |B - B_t|^2 for targets (ux, uy, bx, by)."""
        ts = [self._field(t) for t in targets]
        L = ctypes.c_double()
        p = _ptr(state) if state is not None else ctypes.c_void_p(0)
        self._check(self._L.lbmhd_mismatch(self._h, p, *[_ptr(t) for t in ts], ctypes.byref(L)),
                    "lbmhd_mismatch")
        return L.value

    def diag(self, raise_nonfinite: bool = False) -> dict:
        d = C.Diag()
        rc = self._L.lbmhd_diag(self._h, ctypes.byref(d))
        if rc != C.LBMHD_ERR_NONFINITE or raise_nonfinite:
            self._check(rc, "lbmhd_diag")
        return d.as_dict()

    def run(self, n: int, every: int, dev: torch.Tensor = None,
            raise_nonfinite: bool = False) -> list:
        """n steps with the diagnostics of diag() after steps every, 2 every, ...
        (lbmhd_run: no host wait between them, one at the end); returns their
        dicts.  dev: optional device float64 buffer of at least 16 n // every
        elements for the results (allocated here when not given)."""
        nd = n // every if every > 0 else 0
        if nd == 0:
            self.step(n)
            return []
        if dev is None:
            dev = torch.empty(16 * nd, dtype=torch.float64, device=self.device)
        elif dev.dtype != torch.float64 or dev.numel() < 16 * nd or not dev.is_contiguous():
            raise ValueError("dev must be a contiguous float64 tensor of 16 n // every elements")
        out = (C.Diag * nd)()
        rc = self._L.lbmhd_run(self._h, int(n), int(every), _ptr(dev), out, nd)
        if rc != C.LBMHD_ERR_NONFINITE or raise_nonfinite:
            self._check(rc, "lbmhd_run")
        return [d.as_dict() for d in out]

    def diag_noalloc(self, raise_nonfinite: bool = False) -> dict:
        """diag() through lbmhd_diag_noalloc: the reductions' scratch is the
        library's static device array, not the bound workspace."""
        d = C.Diag()
        rc = self._L.lbmhd_diag_noalloc(self._h, ctypes.byref(d))
        if rc != C.LBMHD_ERR_NONFINITE or raise_nonfinite:
            self._check(rc, "lbmhd_diag_noalloc")
        return d.as_dict()

    def populations(self) -> torch.Tensor:
        out = torch.empty(19, self.cfg.ny, self.cfg.nx, dtype=torch.float64, device=self.device)
        self._check(self._L.lbmhd_get_populations(self._h, _ptr(out)), "lbmhd_get_populations")
        return out

    def set_populations(self, pops, step: int = 0) -> "Lattice":
        t = torch.as_tensor(pops, dtype=torch.float64).to(self.device).contiguous()
        if tuple(t.shape) != (19, self.cfg.ny, self.cfg.nx):
            raise ValueError("populations must have shape (19, ny, nx)")
        self._check(self._L.lbmhd_set_populations(self._h, _ptr(t), int(step)),
                    "lbmhd_set_populations")
        self._keep = t
        return self

    def new_state_buffer(self) -> torch.Tensor:
        return torch.empty(self.lattice_bytes, dtype=torch.uint8, device=self.device)

    def save_state(self, dst: torch.Tensor | None = None) -> torch.Tensor:
        dst = self.new_state_buffer() if dst is None else dst
        if dst.numel() < self.lattice_bytes:
            raise ValueError("state buffer too small")
        self._check(self._L.lbmhd_save_state(self._h, _ptr(dst)), "lbmhd_save_state")
        return dst

    def load_state(self, src: torch.Tensor, step: int) -> "Lattice":
        if src.numel() < self.lattice_bytes:
            raise ValueError("state buffer too small")
        self._check(self._L.lbmhd_load_state(self._h, _ptr(src), int(step)), "lbmhd_load_state")
        return self

    @property
    def step_count(self) -> int:
        v = ctypes.c_int64()
        self._check(self._L.lbmhd_get_step(self._h, ctypes.byref(v)), "lbmhd_get_step")
        return v.value

    def current_state(self) -> torch.Tensor:
        """The bound lattice buffer (uint8, lattice_bytes) that holds the current
        state; in place, read it after a call that restores the natural layout
        (diag, macro, save_state)."""
        p = ctypes.c_void_p()
        self._check(self._L.lbmhd_current_state(self._h, ctypes.byref(p)), "lbmhd_current_state")
        for t in (self._a, self._b):
            if t is not None and t.data_ptr() == p.value:
                return t
        raise RuntimeError("the library reports a state outside the bound lattices")

    @property
    def steps_per_pass(self) -> int:
        """Steps one kernel pass covers in step(): 3 (FP32 triples), 2 or 1.
        With 3, a remainder of two steps is one pair and of one step a
        single step."""
        v = ctypes.c_int32()
        self._check(self._L.lbmhd_steps_per_pass(self._h, ctypes.byref(v)),
                    "lbmhd_steps_per_pass")
        return v.value

    def energy(self, state: torch.Tensor | None = None) -> float:
        J = ctypes.c_double()
        p = _ptr(state) if state is not None else ctypes.c_void_p(0)
        self._check(self._L.lbmhd_energy(self._h, p, ctypes.byref(J)), "lbmhd_energy")
        return J.value

    # -------------------------------------------------------------- adjoint
    def new_adj_buffer(self) -> torch.Tensor:
        return torch.empty(self.adj_lattice_bytes // 4, dtype=torch.float32, device=self.device)

    def new_adj_acc(self) -> torch.Tensor:
        return torch.zeros(self.adj_acc_bytes // 8, dtype=torch.float64, device=self.device)

    def adj_seed_energy(self, state: torch.Tensor, lam: torch.Tensor):
        self._check(self._L.lbmhd_adj_seed_energy(self._h, _ptr(state), _ptr(lam)),
                    "lbmhd_adj_seed_energy")

    def adj_seed_mismatch(self, state: torch.Tensor, targets, scale: float, lam: torch.Tensor):
        ts = [self._field(t) for t in targets]
        self._check(self._L.lbmhd_adj_seed_mismatch(self._h, _ptr(state), *[_ptr(t) for t in ts],
                                                     float(scale), _ptr(lam)),
                    "lbmhd_adj_seed_mismatch")
        self._keep = ts

    def adj_step(self, state_n: torch.Tensor, lam_next: torch.Tensor, lam_prev: torch.Tensor,
                 acc: torch.Tensor):
        self._check(self._L.lbmhd_adj_step(self._h, _ptr(state_n), _ptr(lam_next),
                                           _ptr(lam_prev), _ptr(acc)), "lbmhd_adj_step")

    def adj_sweep(self, src: torch.Tensor, store: torch.Tensor | None, n: int,
                  lam: torch.Tensor, tmp: torch.Tensor, acc: torch.Tensor):
        """Reverse sweep over n steps in one library call: x_0 = src, x_t = row
        t - 1 of store (t = 1 .. n - 1); lam holds lam_n on entry and lam_0 on
        return; tmp is scratch."""
        stride = self._store_stride(store, n - 1) if n > 1 else self.lattice_bytes
        sp = _ptr(store) if n > 1 else ctypes.c_void_p(0)
        self._check(self._L.lbmhd_adj_sweep(self._h, _ptr(src), sp, stride, int(n), _ptr(lam),
                                            _ptr(tmp), _ptr(acc)), "lbmhd_adj_sweep")

    def adj_step2(self, state_t: torch.Tensor, lam_next: torch.Tensor, lam_prev: torch.Tensor,
                  acc: torch.Tensor):
        """Two reverse steps from state x_t alone (x_{t+1} recomputed on the
        device): lam_prev = lam_t from lam_next = lam_{t+2}."""
        self._check(self._L.lbmhd_adj_step2(self._h, _ptr(state_t), _ptr(lam_next),
                                            _ptr(lam_prev), _ptr(acc)), "lbmhd_adj_step2")

    def adj_sweep_pairs(self, src: torch.Tensor, store: torch.Tensor | None, n: int,
                        lam: torch.Tensor, tmp: torch.Tensor, acc: torch.Tensor):
        """Reverse sweep over n steps from every other state (the layout of
        step_store_pairs): x_0 = src, x_t = row t / 2 - 1 of store for the even
        t <= n - 1; lam holds lam_n on entry and lam_0 on return."""
        rows = (n - 1) // 2
        stride = self._store_stride(store, rows) if rows > 0 else self.lattice_bytes
        sp = _ptr(store) if rows > 0 else ctypes.c_void_p(0)
        self._check(self._L.lbmhd_adj_sweep_pairs(self._h, _ptr(src), sp, stride, int(n),
                                                  _ptr(lam), _ptr(tmp), _ptr(acc)),
                    "lbmhd_adj_sweep_pairs")

    def adj_acc_total(self, acc: torch.Tensor) -> tuple[float, float]:
        """(sum lam . dx/dC_Sv, sum lam . dx/dC_Sb) accumulated in acc."""
        out = (ctypes.c_double * 2)()
        self._check(self._L.lbmhd_adj_acc_total(self._h, _ptr(acc), out),
                    "lbmhd_adj_acc_total")
        return float(out[0]), float(out[1])

    def adj_fields(self, lam0: torch.Tensor, fields) -> tuple:
        fs = [self._field(a) for a in fields]
        outs = [torch.empty(self.cfg.ny, self.cfg.nx, dtype=torch.float64, device=self.device)
                for _ in range(4)]
        self._check(self._L.lbmhd_adj_fields(self._h, _ptr(lam0), *[_ptr(f) for f in fs],
                                             *[_ptr(o) for o in outs]), "lbmhd_adj_fields")
        return tuple(outs)

    def adj_view(self, lam: torch.Tensor) -> torch.Tensor:
        """(19, ny, nx) view of an adjoint buffer (drops the row padding and the
        gaps between planes).  Entries are in streamed position: plane i at site
        x + c_i holds dJ/dx_i(x)."""
        return lam.as_strided((19, self.cfg.ny, self.cfg.nx), (self.adj_plane, self.adj_pitch, 1))

    def state_view(self, state: torch.Tensor | None = None) -> torch.Tensor:
        """(19, ny, nx) view of the stored elements of an encoded lattice (default:
        the current state, returned to the natural layout): float32 for FP32
        storage, float16 (deviation x 2^10) for FP16."""
        st = self.save_state() if state is None else state
        dt = torch.float32 if self.cfg.storage == "fp32" else torch.float16
        return st[: self.lattice_bytes].view(dt).as_strided(
            (19, self.cfg.ny, self.cfg.nx), (self.plane, self.pitch, 1))
