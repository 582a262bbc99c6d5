"""Gradients of the final total energy through the GPU adjoint step.

``LBMHDFunction.apply(ux0, uy0, bx0, by0, cs, cfg, nsteps, every="auto")`` runs
``nsteps`` steps from equilibrium at (rho = 1, u0, B0) and returns
J = sum |rho u|^2 / (2 rho) + |B|^2 / 2 of the final state (FP64).  Its backward
pass is the discrete adjoint: checkpoints of the encoded lattice are kept every
``every`` steps during the forward run (every state when they fit in device
memory); the backward sweep recomputes each segment's states from its
checkpoint straight into one stored block and walks them in reverse, each a
single library call.  Without neighbour terms in the closure (les = 0, 1) the
reverse steps go two per pass from one state (``lbmhd_adj_sweep_pairs``), so
only every other state is kept or recomputed (``lbmhd_step_store_pairs``, one
pass per pair); with the kinetic closure every state is
(``lbmhd_step_store``, ``lbmhd_adj_sweep``).  The result holds the exact
derivative of the FP32 update map (storage rounding counted as the identity)
with respect to the initial fields and the closure constants: ``cs`` is a
scalar (C_Sv = C_Sb = cs) or a pair (C_Sv, C_Sb), and its gradient has the
same shape.
"""
from __future__ import annotations

import torch

from .lattice import LBMHDConfig, Lattice


def states_needed(nsteps: int, every: int, pairs: bool = False) -> int:
    """Lattice-sized buffers a run of nsteps with checkpoints every `every`
    steps holds at once: every state when every == 1; otherwise the
    checkpoints, the final state and the every - 1 recomputed states of one
    segment.  With pairs (reverse steps two per pass, each from one state)
    only the even states of a segment are kept: at every == 1 the initial
    state, the states 2, 4, .. <= nsteps - 1 and the final one; otherwise
    (every - 1) // 2 segment states."""
    if every == 1:
        return (nsteps - 1) // 2 + 2 if pairs and nsteps > 1 else nsteps + 1
    seg = (every - 1) // 2 if pairs else every - 1
    return -(-nsteps // every) + 1 + seg


def choose_interval(nsteps: int, state_bytes: int, budget_bytes: int,
                    pairs: bool = False) -> int:
    """The smallest checkpoint interval whose buffers fit the budget (1 keeps
    every state and makes the backward sweep recompute nothing).  With pairs an
    odd interval k > 1 becomes k + 1: that holds no more buffers (the same
    (k - 1) // 2 segment states, fewer checkpoints) and takes every reverse
    step in a pair, where k leaves one single step per segment.  An even
    interval that is not a multiple of 4 then becomes the next multiple of 4
    where that still fits: a segment's sweep is then an even number of paired
    launches, so it ends in lam without a copy of the adjoint lattice."""
    fit = budget_bytes // max(state_bytes, 1)
    for k in range(1, max(nsteps, 1) + 1):
        if states_needed(nsteps, k, pairs) <= fit:
            if not pairs or k == 1:
                return k
            k += k % 2
            if k % 4 and states_needed(nsteps, k + 2, pairs) <= fit:
                k += 2
            return k
    raise MemoryError("not even one checkpoint segment fits the memory budget")


class Checkpointed:
    """Forward run with checkpoints every ``every`` steps and the matching
    reverse sweep (the C ABI does the arithmetic; this class only orders calls).

    every = "auto" picks the smallest interval whose state buffers fit
    ``budget_bytes`` (default: 70% of the device memory free when the forward
    run starts).  With interval 1 every state the sweep reads is kept (every
    other one with paired reverse steps): the forward steps write straight
    into the stored buffers and the backward sweep recomputes nothing, which
    is the case whenever the run fits in HBM (the 1001 states of 2000 steps
    of a 1024^2 FP32 lattice take 80 GB)."""

    def __init__(self, lat: Lattice, every="auto", budget_bytes: int | None = None):
        if every != "auto" and (not isinstance(every, int) or every < 1):
            raise ValueError("checkpoint interval must be >= 1 or 'auto'")
        self.lat = lat
        self.every = every
        self.budget_bytes = budget_bytes
        self.interval = None
        self.ckpts: list[torch.Tensor] = []
        # reverse steps in pairs, from every other state (closures without
        # neighbour terms)
        self.pairs = lat is not None and (int(lat.cfg.les) & 6) == 0

    def _interval(self, nsteps: int) -> int:
        if self.every != "auto":
            return self.every
        budget = self.budget_bytes
        if budget is None:
            free, _ = torch.cuda.mem_get_info(self.lat.device)
            cached = (torch.cuda.memory_reserved(self.lat.device)
                      - torch.cuda.memory_allocated(self.lat.device))
            budget = int(0.7 * (free + cached))
        return choose_interval(nsteps, self.lat.lattice_bytes, budget, self.pairs)

    def forward(self, fields, nsteps: int, targets=None) -> float:
        """Run nsteps from equilibrium at `fields` (rho, ux, uy, bx, by) keeping
        checkpoints.  Returns the final total energy, or with `targets`
        (ux, uy, bx, by) the mismatch sum |u - u_t|^2 + |B - B_t|^2."""
        lat = self.lat
        self.targets = targets
        lat.init_fields(*fields)
        self.fields = fields
        self.nsteps = nsteps
        self.ckpts, self.final, self.store = [], None, None
        k = self._interval(nsteps)
        store = None
        if k == 1:
            try:
                store = torch.empty(states_needed(nsteps, 1, self.pairs), lat.lattice_bytes,
                                    dtype=torch.uint8, device=lat.device)
            except torch.OutOfMemoryError:
                # the free memory was not in one piece: fall back to checkpoints
                # within half of what every state would have taken
                k = choose_interval(nsteps, lat.lattice_bytes,
                                    states_needed(nsteps, 1, self.pairs) * lat.lattice_bytes // 2,
                                    self.pairs)
        self.interval = k
        if k == 1 and self.pairs and nsteps > 1:
            # the initial state, the even states 2 .. 2m (m = (nsteps - 1) // 2,
            # one library call) and the final state, reached from state 2m by
            # the one or two steps left; the lattice ends on the final state
            m = (nsteps - 1) // 2
            self.store = store
            self.ckpts = [store[0]]
            lat.save_state(store[0])
            lat.step_store_pairs(store[0], store[1:m + 1], m)
            lat.load_state(store[m], lat.step_count + 2 * m)
            lat.step(nsteps - 2 * m)
            self.final = lat.save_state(store[m + 1])
        elif k == 1:
            # every state kept, in one allocation, written by one library call;
            # the lattice ends on the final state
            self.store = store
            self.ckpts = list(store.unbind(0))
            lat.save_state(self.ckpts[0])
            lat.step_store(self.ckpts[0], store[1:], nsteps)
            self.final = self.ckpts[-1]
            lat.load_state(self.final, lat.step_count + nsteps)
        else:
            done = 0
            while done < nsteps:
                self.ckpts.append(lat.save_state())
                step = min(k, nsteps - done)
                lat.step(step)
                done += step
            self.final = lat.save_state()
        return lat.energy(self.final) if targets is None else lat.mismatch(targets, self.final)

    def backward(self, scale: float = 1.0):
        """Returns scale * (dJ/du_x, dJ/du_y, dJ/dB_x, dJ/dB_y, dJ/dC_Sv, dJ/dC_Sb)
        for the functional returned by forward()."""
        lat = self.lat
        lam = lat.new_adj_buffer()
        lam2 = lat.new_adj_buffer()
        acc = lat.new_adj_acc()
        if self.targets is None:
            if scale != 1.0:
                raise ValueError("the energy seed takes no scale")
            lat.adj_seed_energy(self.final, lam)
        else:
            lat.adj_seed_mismatch(self.final, self.targets, scale, lam)
        k = self.interval
        if k == 1 and self.pairs and self.nsteps > 1:
            m = (self.nsteps - 1) // 2
            lat.adj_sweep_pairs(self.ckpts[0], self.store[1:m + 1], self.nsteps, lam, lam2, acc)
        elif k == 1:
            lat.adj_sweep(self.ckpts[0], self.store[1:], self.nsteps, lam, lam2, acc)
        elif self.pairs:
            # per segment, from the last: recompute its even states into one
            # block (one pass per pair), then sweep back over it in pairs
            seg = torch.empty(max((k - 1) // 2, 1), lat.lattice_bytes, dtype=torch.uint8,
                              device=lat.device)
            for s in reversed(range(len(self.ckpts))):
                n = min(k, self.nsteps - s * k)
                lat.step_store_pairs(self.ckpts[s], seg, (n - 1) // 2)
                lat.adj_sweep_pairs(self.ckpts[s], seg, n, lam, lam2, acc)
        else:
            # per segment, from the last: recompute its states into one block,
            # then sweep back over them (lambda stays in lam)
            seg = torch.empty(k - 1, lat.lattice_bytes, dtype=torch.uint8, device=lat.device)
            for s in reversed(range(len(self.ckpts))):
                n = min(k, self.nsteps - s * k)
                lat.step_store(self.ckpts[s], seg, n - 1)
                lat.adj_sweep(self.ckpts[s], seg, n, lam, lam2, acc)
        g = lat.adj_fields(lam, self.fields)
        return (*g, *lat.adj_acc_total(acc))


class LBMHDFunction(torch.autograd.Function):
    """J(u0, B0, C_S) with a hand-written adjoint backward (see module doc)."""

    @staticmethod
    def forward(ctx, ux0, uy0, bx0, by0, cs, cfg: LBMHDConfig, nsteps: int, every="auto"):
        c = cs.detach().to(torch.float64).reshape(-1).cpu()
        if c.numel() not in (1, 2):
            raise ValueError("cs must be a scalar or a pair (C_Sv, C_Sb)")
        csv, csb = float(c[0]), float(c[-1])
        cfg = LBMHDConfig(**{**cfg.__dict__, "cs": csv, "cs_b": csb})
        lat = Lattice(cfg, device=ux0.device)
        rho0 = torch.ones_like(ux0, dtype=torch.float64)
        fields = (rho0, *(t.detach().to(torch.float64) for t in (ux0, uy0, bx0, by0)))
        run = Checkpointed(lat, every)
        J = run.forward(fields, nsteps)
        ctx.run = run
        ctx.dtypes = tuple(t.dtype for t in (ux0, uy0, bx0, by0, cs))
        ctx.cs_shape = cs.shape
        return torch.tensor(J, dtype=torch.float64, device=ux0.device)

    @staticmethod
    def backward(ctx, gJ):
        gux, guy, gbx, gby, gv, gb = ctx.run.backward()
        s = gJ.to(torch.float64)
        outs = [s * g for g in (gux, guy, gbx, gby)]
        outs = [o.to(dt) for o, dt in zip(outs, ctx.dtypes[:4])]
        if ctx.cs_shape.numel() == 1:
            gc = (s * (gv + gb)).reshape(ctx.cs_shape)
        else:
            gc = s * torch.tensor([gv, gb], dtype=torch.float64,
                                  device=s.device).reshape(ctx.cs_shape)
        gc = gc.to(ctx.dtypes[4])
        ctx.run = None
        return (*outs, gc, None, None, None)
