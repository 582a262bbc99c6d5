"""Fit of the closure constant C_S by the discrete adjoint.

Target: a fine FP32 run box-filtered onto the coarse grid (``reference``).
Model: the coarse LES run from the same initial realisation, with acoustic
scaling (grid spacing and time step both w times larger, so the lattice
velocity is unchanged, the step count is divided by w and the lattice
viscosity and resistivity by w).  Loss: the relative mismatch
L = sum |u - u_t|^2 + |B - B_t|^2 / sum |u_t|^2 + |B_t|^2 of the final coarse
state.  Each iteration runs the coarse model forward with checkpoints and
returns L and dL/dC_S from one adjoint sweep; C_S is updated on log C_S with
sign-based steps (step x1.2 while the sign of dL/dlog C_S holds, x0.5 when it
flips).  The arithmetic runs in the library's kernels; this module orders the
calls and updates one scalar.
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass, field

import torch

from .adjoint import Checkpointed
from .lattice import Lattice, LBMHDConfig


def reference(fields, cfg: LBMHDConfig, steps: int, w: int):
    """Box-filtered (w x w) u and B after `steps` steps of the fine run."""
    lat = Lattice(cfg)
    lat.init_fields(*fields).step(steps)
    m = lat.macro_box(w)
    out = (m["ux"], m["uy"], m["bx"], m["by"])
    del lat
    return out


@dataclass
class FitResult:
    cs: list = field(default_factory=list)
    loss: list = field(default_factory=list)
    grad: list = field(default_factory=list)
    seconds: float = 0.0


def fit_cs(coarse_fields, targets, cfg: LBMHDConfig, steps: int, iters: int = 20,
           every: int = 100, step0: float = 0.5, log=None) -> FitResult:
    """Minimise the relative mismatch over C_S (cfg.cs is the start value)."""
    norm = float(sum(torch.sum(torch.as_tensor(t) ** 2).item() for t in targets))
    res = FitResult()
    theta, step, last_sign = math.log(cfg.cs), step0, 0.0
    t0 = time.perf_counter()
    for it in range(iters):
        cs = math.exp(theta)
        lat = Lattice(LBMHDConfig(**{**cfg.__dict__, "les": True, "cs": cs}))
        run = Checkpointed(lat, every)
        L = run.forward(coarse_fields, steps, targets=targets) / norm
        dcs = run.backward(scale=1.0 / norm)[4]
        g = dcs * cs                            # dL / dlog C_S
        res.cs.append(cs)
        res.loss.append(L)
        res.grad.append(dcs)
        if log:
            log(f"fit iter {it}: C_S = {cs:.5f}  L = {L:.6e}  dL/dC_S = {dcs:.4e}")
        sign = 1.0 if g > 0 else (-1.0 if g < 0 else 0.0)
        if last_sign and sign and sign != last_sign:
            step *= 0.5
        elif last_sign and sign == last_sign:
            step *= 1.2
        theta -= sign * step
        last_sign = sign
        del run, lat
    torch.cuda.synchronize()
    res.seconds = time.perf_counter() - t0
    return res
