"""Fit of the closure constants by the discrete adjoint.

Target: a fine FP32 run box-filtered onto the coarse grid (``reference``).
Model: the coarse LES run from the same initial realisation, with acoustic
scaling (grid spacing and time step both w times larger, so the lattice
velocity is unchanged, the step count is divided by w and the lattice
viscosity and resistivity by w).  Loss: the relative mismatch
L = sum |u - u_t|^2 + |B - B_t|^2 / sum |u_t|^2 + |B_t|^2 of the final coarse
state.  Each iteration runs the coarse model forward with checkpoints and
returns L and dL/dC_Sv, dL/dC_Sb from one adjoint sweep; the constants are
updated on their logs with sign-based steps (step x1.2 while the sign of the
derivative holds, x0.5 when it flips), either tied (C_Sv = C_Sb) or jointly,
one step size per constant.  The model is the Smagorinsky-MHD closure, on its
own or on top of the kinetic closure's filtered equilibria.  The arithmetic runs in the library's kernels; this module
orders the calls and updates the constants.
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
    cs: list = field(default_factory=list)      # C_Sv per iteration
    cs_b: list = field(default_factory=list)    # C_Sb per iteration
    loss: list = field(default_factory=list)
    grad: list = field(default_factory=list)    # (dL/dC_Sv, dL/dC_Sb)
    seconds: float = 0.0


def fit_cs(coarse_fields, targets, cfg: LBMHDConfig, steps: int, iters: int = 20,
           every="auto", step0: float = 0.5, joint: bool = False, log=None) -> FitResult:
    """Minimise the relative mismatch over the closure constants, starting from
    cfg.cs (and cfg.cs_b).  joint=False fits one constant C_Sv = C_Sb; joint=True
    fits C_Sv and C_Sb together, each with its own sign-based step on its log.
    The model carries the Smagorinsky-MHD closure: alone (cfg.les = 0 or 1) or
    measured from the kinetic closure's filtered equilibria (cfg.les = 2 or
    3)."""
    if cfg.les & 4:
        raise ValueError("the cross-helicity closure has no adjoint to fit with")
    les = 3 if cfg.les & 2 else 1
    norm = float(sum(torch.sum(torch.as_tensor(t) ** 2).item() for t in targets))
    res = FitResult()
    theta = [math.log(cfg.cs), math.log(cfg.csb)] if joint else [math.log(cfg.cs)]
    step = [step0] * len(theta)
    last = [0.0] * len(theta)
    t0 = time.perf_counter()
    for it in range(iters):
        csv, csb = math.exp(theta[0]), math.exp(theta[-1])
        lat = Lattice(LBMHDConfig(**{**cfg.__dict__, "les": les, "cs": csv, "cs_b": csb}))
        run = Checkpointed(lat, every)
        L = run.forward(coarse_fields, steps, targets=targets) / norm
        dv, db = run.backward(scale=1.0 / norm)[4:]
        # dL/dlog C: per constant, or along the tied direction
        g = [dv * csv, db * csb] if joint else [dv * csv + db * csb]
        res.cs.append(csv)
        res.cs_b.append(csb)
        res.loss.append(L)
        res.grad.append((dv, db))
        if log:
            log(f"fit iter {it}: C_Sv = {csv:.5f}  C_Sb = {csb:.5f}  L = {L:.6e}  "
                f"dL/dC_Sv = {dv:.4e}  dL/dC_Sb = {db:.4e}")
        for k, gk in enumerate(g):
            sign = 1.0 if gk > 0 else (-1.0 if gk < 0 else 0.0)
            if last[k] and sign and sign != last[k]:
                step[k] *= 0.5
            elif last[k] and sign == last[k]:
                step[k] *= 1.2
            theta[k] -= sign * step[k]
            last[k] = sign
        del run, lat
    torch.cuda.synchronize()
    res.seconds = time.perf_counter() - t0
    return res
