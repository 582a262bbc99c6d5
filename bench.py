#!/usr/bin/env python3
"""Benchmark of the LB-MHD hot path on one MI355X.

Headline (``value``): site updates per second (MLUPS) of the FP32
stream-collide update on a 4096 x 4096 periodic Orszag-Tang vortex
(nu = eta = 1e-5, Smagorinsky-MHD closure with C_S = 0.1), inputs resident in
HBM, K timed steps with the FP64 diagnostics reduction run every 100 steps
inside the timed region (one lbmhd_run call: each diagnostics pass overlaps
the next kernel pass, and the host waits once, at the end, for all results).
Steps go three per pass over the lattice (the
intermediate states stay on chip; the results equal single steps bit for
bit), so the dominant kernel moves 152 B per site per launch for three
updates; the single-step kernel is timed beside it.  The same JSON line also reports the FP16-storage
step on 8192 x 8192 decaying turbulence (nu = eta = 1e-6), the adjoint
(gradient of the final total energy after 2000 steps of a perturbed 1024 x 1024
Orszag-Tang run, checkpoint interval from the free HBM), the adjoint-driven fit of C_S
(2048^2 FP16 LES against a box-filtered 8192^2 FP32 run), the HBM roofline of
the dominant kernel, and the FP64 CPU oracle timed on the host on the headline
workload.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
Progress goes to stderr; stdout carries exactly one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MLUPS + %HBM peak, FP32 vs FP16-store fwd and adjoint, at stated err"
HBM_PEAK_GBS = 8000.0           # MI355X HBM3E, published
FP32_BYTES_PER_SITE = 19 * 4 * 2
FP16_BYTES_PER_SITE = 19 * 2 * 2
ADJ_BYTES_PER_SITE = 19 * 4 * 2 + 3 * 19 * 4  # recompute step + (lam in, state gather, lam out)
COUNTERS_FILE = os.path.join(ROOT, "profiles", "counters_kernels.json")
# VALU issue: 256 CUs x 4 SIMDs x 16 lanes, one lane-operation per lane and cycle, 2.4 GHz
# (an FMA counted once; the 78.6 TFLOP/s FP32 figure counts it twice)
VALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12


def log(msg: str):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1607_08675_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        if name.endswith((".hip", ".h")):
            with open(os.path.join(csrc, name), "rb") as fh:
                h.update(name.encode() + fh.read())
    return h.hexdigest()[:16]


def counters():
    """The committed counter summary, or None if the kernel sources changed
    since it was taken."""
    try:
        with open(COUNTERS_FILE) as fh:
            c = json.load(fh)
    except (OSError, ValueError):
        return None
    return c if c.get("kernel_source_hash") == kernel_source_hash() else None


def measured_traffic():
    """HBM bytes per launch of the headline kernel from the committed counters."""
    c = counters()
    return c.get("headline_bytes_per_launch") if c else None


def valu_frac(key, ms_per_launch):
    """VALU issue time per launch at the chip's peak (from the committed SQ
    counters of kernel `key`) over the launch time measured here."""
    c = counters()
    if not c or key not in c["kernels"]:
        return None
    return round(c["kernels"][key]["valu_time_at_peak_us"] * 1e-3 / ms_per_launch, 4)


def valu_roofline(key, ms_per_launch):
    """Roofline object of a kernel bound by its VALU issue rate: achieved lane
    operations per second (counted instructions x 64 lanes, transcendentals
    at four issue slots) against VALU_PEAK_TOPS."""
    c = counters()
    if not c or key not in c["kernels"]:
        return None
    k = c["kernels"][key]
    ops = (k["valu_insts"] + 3 * k["trans_insts"]) * 64
    achieved = ops / (ms_per_launch * 1e-3) / 1e12
    return {"kernel": k["kernel"], "bound": "alu", "achieved": round(achieved, 2),
            "peak": round(VALU_PEAK_TOPS, 2), "unit": "TOP/s (VALU lane operations)",
            "frac": round(achieved / VALU_PEAK_TOPS, 4), "hbm_frac": round(
                k["algorithmic_bytes"] / (ms_per_launch * 1e-3) / (HBM_PEAK_GBS * 1e9), 4),
            "ms_per_launch": round(ms_per_launch, 5)}


def timed_steps(torch, lat, steps, diag_every):
    """Run `steps` steps with the FP64 diagnostics after every diag_every of
    them (one lbmhd_run call: each diagnostics pass overlaps the next kernel
    pass, and the host waits once, at the end) between two events on the
    lattice's stream; returns milliseconds."""
    s = lat.stream
    dev = torch.empty(16 * max(1, steps // diag_every), dtype=torch.float64, device="cuda")
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(s)
    lat.run(steps, diag_every, dev)
    e1.record(s)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1)


def warm_up(lat, steps):
    """Untimed steps through lbmhd_run with at least one diagnostics pass, so
    that the library's diagnostics stream has run before the timed call (its
    first dispatch costs a few milliseconds once)."""
    if steps > 0:
        lat.run(steps, min(100, steps))


def burst_ms_per_step(torch, lat, steps):
    """Average time per step of `steps` back-to-back steps, from HIP events on
    the lattice's stream (a kernel launch covers lat.steps_per_pass of them
    when `steps` is even)."""
    s = lat.stream
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(s)
    lat.step(steps)
    e1.record(s)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def fp32_leg(torch, args):
    from lbmhd_inputs import orszag_tang
    from paper_1607_08675_amd.lattice import Lattice, LBMHDConfig
    n = 4096
    cfg = LBMHDConfig(nx=n, ny=n, nu=1e-5, eta=1e-5, les=True, cs=0.1, storage="fp32")
    fields = orszag_tang(n, n)
    # the same workload one step per pass (the single-step kernel), timed
    # first: it also brings the chip to its running clocks before the headline
    lat = Lattice(LBMHDConfig(**{**cfg.__dict__, "steps_per_pass": 1}))
    lat.init_fields(*fields).step(args.warmup)
    single = burst_ms_per_step(torch, lat, 200)
    log(f"fp32 one step per pass: {single:.4f} ms/step")
    del lat
    torch.cuda.empty_cache()
    lat = Lattice(cfg)
    lat.init_fields(*fields)
    warm_up(lat, args.warmup)
    torch.cuda.synchronize()
    log(f"fp32 4096^2: warmup {args.warmup} done, timing {args.steps} steps")
    t0 = time.perf_counter()
    ms = timed_steps(torch, lat, args.steps, 100)
    wall = time.perf_counter() - t0
    d = lat.diag()
    spp = lat.steps_per_pass
    per_launch = burst_ms_per_step(torch, lat, 198) * spp   # 198 steps: 66 triples or 99 pairs
    # checkpoint of the final state: one plain copy kernel of lattice_bytes,
    # the reference size for calibrating HBM byte counters
    lat.save_state()
    torch.cuda.synchronize()
    log(f"fp32: {ms / args.steps:.4f} ms/step, burst {per_launch:.4f} ms/launch of {spp} "
        f"steps, nonfinite={d['nonfinite']}")
    del lat
    torch.cuda.empty_cache()
    return dict(ms=ms, wall=wall, per_launch=per_launch, steps_per_pass=spp, single=single,
                sites=n * n, diag=d)


def inplace_leg(torch, args):
    """The headline workload (4096^2 Orszag-Tang, FP32, LES) on one lattice
    updated in place (AA pattern): an even number of back-to-back launches,
    so the timing covers both step kinds equally and no layout pass."""
    from lbmhd_inputs import orszag_tang
    from paper_1607_08675_amd.lattice import Lattice, LBMHDConfig
    n = 4096
    cfg = LBMHDConfig(nx=n, ny=n, nu=1e-5, eta=1e-5, les=1, cs=0.1, storage="fp32",
                      inplace=True)
    lat = Lattice(cfg)
    lat.init_fields(*orszag_tang(n, n))
    lat.step(2 * (args.warmup // 2))
    torch.cuda.synchronize()
    per_launch = burst_ms_per_step(torch, lat, 200)
    d = lat.diag()
    log(f"in-place 4096^2 FP32: {per_launch:.4f} ms/launch, nonfinite={d['nonfinite']}")
    mem = lat.lattice_bytes
    del lat
    torch.cuda.empty_cache()
    return dict(per_launch=per_launch, sites=n * n, nonfinite=d["nonfinite"], lattice_bytes=mem)


def threed_leg(torch, args):
    """The 3D update (D3Q27 + six magnetic vectors, Smagorinsky-MHD closure)
    on a 256^3 Orszag-Tang-type vortex: 45 populations, 360 B per site-step in
    FP32 storage, 180 B in FP16."""
    from lbmhd_inputs import orszag_tang_3d
    from paper_1607_08675_amd.lattice3 import Lattice3, LBMHD3Config
    n = 256
    fields = orszag_tang_3d(n, n, n)
    out = dict(sites=n ** 3)
    # single relaxation in FP32 and FP16, and the moment-space collision
    # (tensor-product basis, unequal rates) in FP32
    mrt = dict(mrt=1, s5=1.3, s7=0.7, s8=1.6, sg=1.1, szz=0.9)
    for key, st, extra in (("fp32", "fp32", {}), ("fp16", "fp16", {}), ("fp32_mrt", "fp32", mrt)):
        lat = Lattice3(LBMHD3Config(nx=n, ny=n, nz=n, nu=1e-5, eta=1e-5, les=1, cs=0.1,
                                    storage=st, **extra))
        lat.init_fields(*fields)
        lat.step(args.warmup)
        torch.cuda.synchronize()
        per_launch = burst_ms_per_step(torch, lat, 100)
        d = lat.diag()
        log(f"3D 256^3 {key}: {per_launch:.4f} ms/launch, nonfinite={d['nonfinite']}")
        out[key] = dict(per_launch=per_launch, nonfinite=d["nonfinite"])
        del lat
        torch.cuda.empty_cache()
    return out


CLOSURES = {2: "kinetic closure", 4: "cross-helicity closure"}


def closure_leg(torch, args, les):
    """FP32 step with one of the paper's neighbour-dependent closures on the
    headline 4096^2 Orszag-Tang workload: les = 2, the kinetic closure
    (filtered equilibria, Delta = 1); les = 4, the cross-helicity closure
    (C_S = 0.1, backscatter clipped at zero total resistivity)."""
    from lbmhd_inputs import orszag_tang
    from paper_1607_08675_amd.lattice import Lattice, LBMHDConfig
    n = 4096
    cfg = LBMHDConfig(nx=n, ny=n, nu=1e-5, eta=1e-5, les=les, cs=0.1, delta=1.0,
                      storage="fp32")
    lat = Lattice(cfg)
    lat.init_fields(*orszag_tang(n, n))
    lat.step(args.warmup)
    torch.cuda.synchronize()
    spp = lat.steps_per_pass
    per_step = burst_ms_per_step(torch, lat, 200)
    d = lat.diag()
    log(f"{CLOSURES[les]} 4096^2 FP32: {per_step:.4f} ms/step, {spp} per pass, "
        f"nonfinite={d['nonfinite']}")
    del lat
    torch.cuda.empty_cache()
    return dict(per_step=per_step, spp=spp, sites=n * n, nonfinite=d["nonfinite"])


def fp16_leg(torch, args):
    """FP16 deviation storage against FP32 storage on the same 8192^2 decaying
    turbulence (nu = eta = 1e-6, LES): each timed for args.fp16_steps steps
    with the diagnostics every 100 steps, and the relative L2 of u and B
    between the two after args.fp16_compare_steps (1000) steps from the same
    initial fields."""
    from lbmhd_inputs import decaying_turbulence
    from paper_1607_08675_amd.lattice import Lattice, LBMHDConfig
    n = 8192
    log("fp16 8192^2: generating decaying-turbulence fields")
    fields = decaying_turbulence(n, n)
    out = dict(sites=n * n)
    snaps = {}
    for st in ("fp16", "fp32"):
        cfg = LBMHDConfig(nx=n, ny=n, nu=1e-6, eta=1e-6, les=True, cs=0.1, storage=st)
        lat = Lattice(cfg)
        lat.init_fields(*fields).step(args.fp16_compare_steps)
        m = lat.macro()
        snaps[st] = torch.stack([m["ux"], m["uy"], m["bx"], m["by"]])
        del m
        lat.init_fields(*fields)
        warm_up(lat, args.warmup)
        torch.cuda.synchronize()
        log(f"{st} 8192^2: timing {args.fp16_steps} steps")
        ms = timed_steps(torch, lat, args.fp16_steps, 100)
        spp = lat.steps_per_pass
        per_launch = burst_ms_per_step(torch, lat, 96) * spp   # 96: 48 pairs or 32 triples
        d = lat.diag()
        log(f"{st}: {ms / args.fp16_steps:.4f} ms/step, burst {per_launch:.4f} ms/launch of "
            f"{spp} steps, nonfinite={d['nonfinite']}")
        out[st] = dict(ms=ms, per_launch=per_launch, steps_per_pass=spp, nonfinite=d["nonfinite"])
        del lat
        torch.cuda.empty_cache()
    a, b = snaps["fp16"], snaps["fp32"]
    out["rel_l2_u_1000"] = float(torch.linalg.vector_norm(a[:2] - b[:2]) /
                                 torch.linalg.vector_norm(b[:2]))
    out["rel_l2_b_1000"] = float(torch.linalg.vector_norm(a[2:] - b[2:]) /
                                 torch.linalg.vector_norm(b[2:]))
    log(f"fp16 vs fp32 at step {args.fp16_compare_steps}: rel-L2 u {out['rel_l2_u_1000']:.3e}, "
        f"B {out['rel_l2_b_1000']:.3e}")
    del snaps, a, b
    torch.cuda.empty_cache()
    return out


def adjoint_leg(torch, args):
    """Gradient of the final total energy after args.adj_steps steps of the
    perturbed 1024^2 Orszag-Tang run: end to end with checkpoints every 100
    steps (the stated workload: recompute each segment, then sweep back), and
    with the interval chosen from the free HBM (every state the sweep reads
    kept, nothing recomputed); then at 4096^2 one 100-step segment, the
    reverse kernels alone, and a run of args.adj_steps steps with the interval
    chosen from the free HBM."""
    from lbmhd_inputs import perturbed_orszag_tang
    from paper_1607_08675_amd.adjoint import Checkpointed
    from paper_1607_08675_amd.lattice import Lattice, LBMHDConfig
    n, nsteps = 1024, args.adj_steps
    cfg = LBMHDConfig(nx=n, ny=n, nu=1e-5, eta=1e-5, les=True, cs=0.1, storage="fp32")
    lat = Lattice(cfg)
    fields = perturbed_orszag_tang(n, n)
    out = dict(sites=n * n, nsteps=nsteps)
    for key, every in (("k100", 100), ("auto", "auto")):
        run = Checkpointed(lat, every)
        # warm-up of both passes at the full length, so that the buffers are
        # allocated once and reused by the timed run (as in a fit loop)
        run.forward(fields, nsteps)
        run.backward()
        torch.cuda.synchronize()
        log(f"adjoint 1024^2, interval {every}: forward + backward of {nsteps} steps")
        t0 = time.perf_counter()
        J = run.forward(fields, nsteps)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        g = run.backward()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        out[key] = dict(J=J, fwd_s=t1 - t0, bwd_s=t2 - t1, interval=run.interval,
                        dJ_dcsv=g[4], dJ_dcsb=g[5])
        log(f"adjoint: J={J:.6e}, interval {run.interval}, forward {t1 - t0:.3f}s, "
            f"backward {t2 - t1:.3f}s")
        if key == "k100":
            out["grad_check"] = {str(nsteps): gradient_check(torch, cfg, fields, nsteps, g,
                                                             (1e-2, 1e-3, 1e-4))}
        del run, g
        torch.cuda.empty_cache()
    # the same check after 500 steps, where central differences converge
    run = Checkpointed(lat, 100)
    run.forward(fields, 500)
    out["grad_check"]["500"] = gradient_check(torch, cfg, fields, 500, run.backward(), (1e-3,))
    del run
    torch.cuda.empty_cache()
    # the forward step as the forward run takes it (steps three per pass)
    out["fwd_ms"] = burst_ms_per_step(torch, lat, 198)
    # one reverse step alone
    st = lat.save_state()
    lam, lam2, acc = lat.new_adj_buffer(), lat.new_adj_buffer(), lat.new_adj_acc()
    lat.adj_seed_energy(st, lam)
    e0, e1 = (torch.cuda.Event(enable_timing=True) for _ in range(2))
    torch.cuda.synchronize()
    e0.record(lat.stream)
    for _ in range(100):
        lat.adj_step(st, lam, lam2, acc)
        lam, lam2 = lam2, lam
    e1.record(lat.stream)
    torch.cuda.synchronize()
    out["adj_kernel_ms"] = e0.elapsed_time(e1) / 100
    log(f"adjoint kernel 1024^2: {out['adj_kernel_ms']:.4f} ms, forward {out['fwd_ms']:.4f} "
        f"ms/step")
    del lat, st, lam, lam2, acc
    torch.cuda.empty_cache()
    # one checkpoint segment of 100 steps at 4096^2, where the working set is
    # far above the caches, as the checkpointed backward takes it: recompute
    # of the 49 even states 2 .. 98 into one stored block (a pass per pair),
    # then 100 reverse steps two per pass; and the reverse step alone, single
    # and paired
    from lbmhd_inputs import orszag_tang
    nb = 4096
    lat = Lattice(LBMHDConfig(nx=nb, ny=nb, nu=1e-5, eta=1e-5, les=True, cs=0.1, storage="fp32"))
    f4096 = orszag_tang(nb, nb)
    lat.init_fields(*f4096).step(10)
    st = lat.save_state()
    seg = torch.empty(49, lat.lattice_bytes, dtype=torch.uint8, device=lat.device)
    lam, lam2, acc = lat.new_adj_buffer(), lat.new_adj_buffer(), lat.new_adj_acc()
    e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
    for _ in range(2):   # the first round warms up
        lat.adj_seed_energy(st, lam)
        torch.cuda.synchronize()
        e0.record(lat.stream)
        lat.step_store_pairs(st, seg, 49)
        e1.record(lat.stream)
        lat.adj_sweep_pairs(st, seg, 100, lam, lam2, acc)
        e2.record(lat.stream)
        torch.cuda.synchronize()
    out["recompute_ms_4096"] = e0.elapsed_time(e1) / 100
    out["adj_ms_4096"] = e1.elapsed_time(e2) / 100
    out["fwd_ms_4096"] = burst_ms_per_step(torch, lat, 198)
    x1 = lat.new_state_buffer()
    lat.step_between(st, x1)
    torch.cuda.synchronize()
    e0.record(lat.stream)
    for _ in range(10):
        lat.adj_step(x1, lam, lam2, acc)
        lat.adj_step(st, lam2, lam, acc)
    e1.record(lat.stream)
    for _ in range(10):
        lat.adj_step2(st, lam, lam2, acc)
        lam, lam2 = lam2, lam
    e2.record(lat.stream)
    torch.cuda.synchronize()
    out["adj_single_ms_4096"] = e0.elapsed_time(e1) / 20
    out["adj_pair_ms_4096"] = e1.elapsed_time(e2) / 20
    log(f"4096^2 segment of 100: recompute {out['recompute_ms_4096']:.4f} ms/step, adjoint "
        f"{out['adj_ms_4096']:.4f} ms/step, forward {out['fwd_ms_4096']:.4f} ms/step; reverse "
        f"step single {out['adj_single_ms_4096']:.4f}, paired {out['adj_pair_ms_4096']:.4f} "
        f"ms/step")
    del st, seg, lam, lam2, acc, x1
    torch.cuda.empty_cache()
    # the stated run length at 4096^2: 2000 steps forward and backward with the
    # interval chosen from the free HBM (a warm-up run allocates the buffers)
    for rnd in range(2):
        run = Checkpointed(lat, "auto")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        J = run.forward(f4096, args.adj_steps)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        g = run.backward()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        if rnd == 0:
            del run, g
            continue
        out["run_4096"] = dict(nsteps=args.adj_steps, interval=run.interval, J=J,
                               fwd_ms=1e3 * (t1 - t0) / args.adj_steps,
                               bwd_ms=1e3 * (t2 - t1) / args.adj_steps, dJ_dcsv=g[4])
        log(f"4096^2 run of {args.adj_steps} steps, interval {run.interval}: forward "
            f"{out['run_4096']['fwd_ms']:.4f} ms/step, backward {out['run_4096']['bwd_ms']:.4f} "
            f"ms/step")
        del run, g
    del lat
    torch.cuda.empty_cache()
    # the reverse step of the kinetic closure (two passes) at the same size
    lat = Lattice(LBMHDConfig(nx=nb, ny=nb, nu=1e-5, eta=1e-5, les=2, cs=0.1, delta=1.0,
                              storage="fp32"))
    lat.init_fields(*orszag_tang(nb, nb)).step(10)
    st = lat.save_state()
    lam, lam2, acc = lat.new_adj_buffer(), lat.new_adj_buffer(), lat.new_adj_acc()
    lat.adj_seed_energy(st, lam)
    lat.adj_step(st, lam, lam2, acc)
    torch.cuda.synchronize()
    e0.record(lat.stream)
    for _ in range(20):
        lat.adj_step(st, lam, lam2, acc)
    e1.record(lat.stream)
    torch.cuda.synchronize()
    out["adj_kin_ms_4096"] = e0.elapsed_time(e1) / 20
    out["fwd_kin_ms_4096"] = burst_ms_per_step(torch, lat, 50)
    log(f"kinetic-closure adjoint 4096^2: {out['adj_kin_ms_4096']:.4f} ms, forward "
        f"{out['fwd_kin_ms_4096']:.4f} ms")
    del lat, st, lam, lam2, acc
    torch.cuda.empty_cache()
    return out


def gradient_check(torch, cfg, fields, nsteps, g, eps_list):
    """Directional derivatives of the adjoint gradient g along seeded
    directions 100 and 107 against central differences (J(p + eps v) -
    J(p - eps v)) / (2 eps) of the FP32 forward run, for each eps."""
    from lbmhd_inputs import directions
    from paper_1607_08675_amd.lattice import Lattice, LBMHDConfig
    n = cfg.nx
    d, dcs = directions(16, n, n, 100, 0.05, 0.05, cfg.cs)
    grads = [t.cpu().numpy() for t in g[:4]]
    rows = {}
    for k in (0, 7):
        adj = sum(float((grads[i] * d[k, i]).sum()) for i in range(4)) + (g[4] + g[5]) * dcs[k]
        fd = {}
        for eps in eps_list:
            J = []
            for sign in (1, -1):
                c = cfg.cs + sign * eps * dcs[k]
                L = Lattice(LBMHDConfig(**{**cfg.__dict__, "cs": c, "cs_b": c}))
                L.init_fields(*([fields[0]] + [fields[1 + i] + sign * eps * d[k, i]
                                               for i in range(4)])).step(nsteps)
                J.append(L.energy())
                del L
            fd[f"{eps:.0e}"] = float(f"{(J[0] - J[1]) / (2 * eps):.6e}")
        rows[f"direction_{100 + k}"] = {"adjoint": float(f"{adj:.6e}"), "central_difference": fd}
        log(f"gradient check, {nsteps} steps, direction {100 + k}: adjoint {adj:.6e}, "
            f"central differences {fd}")
    torch.cuda.empty_cache()
    return rows


def fit_leg(torch, args):
    """Adjoint-driven joint fit of (C_Sv, C_Sb): 8192^2 FP32 LES reference after
    5000 steps, box-filtered (width 4) onto 2048^2; the 2048^2 FP16 model from
    the same realisation runs 1250 steps at nu = eta = 2.5e-7 (acoustic scaling)."""
    from lbmhd_inputs import decaying_turbulence
    from paper_1607_08675_amd.fit import fit_cs, reference
    from paper_1607_08675_amd.lattice import LBMHDConfig
    nf, w = 8192, 4
    log("fit: 8192^2 FP32 reference, 5000 steps")
    t0 = time.perf_counter()
    ref_cfg = LBMHDConfig(nx=nf, ny=nf, nu=1e-6, eta=1e-6, les=True, cs=0.1, storage="fp32")
    targets = reference(decaying_turbulence(nf, nf), ref_cfg, args.fit_ref_steps, w)
    torch.cuda.synchronize()
    t_ref = time.perf_counter() - t0
    torch.cuda.empty_cache()
    nc = nf // w
    cfg = LBMHDConfig(nx=nc, ny=nc, nu=1e-6 / w, eta=1e-6 / w, les=True, cs=0.1, storage="fp16")
    res = fit_cs(decaying_turbulence(nc, nc), targets, cfg, args.fit_ref_steps // w,
                 iters=args.fit_iters, every="auto", joint=True, log=log)
    return dict(t_ref=t_ref, res=res, steps=args.fit_ref_steps // w)


def host_cpu_model() -> str:
    """Model name of the host CPU (from /proc/cpuinfo) and its logical CPU count."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return f"{model} ({os.cpu_count()} logical CPUs on the host)"


def cpu_baseline(seconds: float):
    """The FP64 oracle on the headline workload (4096^2 Orszag-Tang, LES),
    timed on the host cores: whole steps until about `seconds` have passed."""
    from lbmhd_inputs import orszag_tang
    from oracle import oracle as orc
    orc.build()
    n = 4096
    p = orc.Params(n, n, nu=1e-5, eta=1e-5, les=True, cs=0.1)
    st = orc.init(p, *orszag_tang(n, n))
    log(f"cpu baseline: oracle on {n}^2 with {orc.num_threads()} threads")
    steps, t0 = 0, time.perf_counter()
    while True:
        st = orc.run(p, st, 1)
        steps += 1
        el = time.perf_counter() - t0
        log(f"cpu baseline: step {steps} at {el:.1f}s")
        if el >= seconds or steps >= 50:
            break
    return dict(value=n * n * steps / el / 1e6, unit="MLUPS", cores=orc.num_threads(),
                kind="oracle", cpu_model=host_cpu_model(),
                sample=f"FP64 oracle, {steps} step(s) of the 4096x4096 Orszag-Tang LES workload "
                       f"({el:.1f} s wall)")


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--fp16-steps", type=int, default=500)
    ap.add_argument("--fp16-compare-steps", type=int, default=1000)
    ap.add_argument("--adj-steps", type=int, default=2000)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--fit-iters", type=int, default=20)
    ap.add_argument("--fit-ref-steps", type=int, default=5000)
    ap.add_argument("--skip", default="",
                    help="comma list of legs to skip: kinetic,crosshelicity,inplace,3d,fp16,adjoint,fit,cpu")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)
    skip = set(s for s in args.skip.split(",") if s)
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    props = torch.cuda.get_device_properties(0)
    log(f"device: {props.name}, {props.multi_processor_count} CUs")

    r32 = fp32_leg(torch, args)
    rkin = None if "kinetic" in skip else closure_leg(torch, args, 2)
    rch = None if "crosshelicity" in skip else closure_leg(torch, args, 4)
    rin = None if "inplace" in skip else inplace_leg(torch, args)
    r3 = None if "3d" in skip else threed_leg(torch, args)
    r16 = None if "fp16" in skip else fp16_leg(torch, args)
    radj = None if "adjoint" in skip else adjoint_leg(torch, args)
    rfit = None if "fit" in skip else fit_leg(torch, args)
    cpu = None if "cpu" in skip else cpu_baseline(args.cpu_seconds)

    ms_step = r32["ms"] / args.steps
    value = r32["sites"] / (ms_step * 1e-3) / 1e6
    spp = r32["steps_per_pass"]
    # one read and one write of the lattice per launch, whatever it covers
    achieved = FP32_BYTES_PER_SITE * r32["sites"] / (r32["per_launch"] * 1e-3) / 1e9
    single_gbs = FP32_BYTES_PER_SITE * r32["sites"] / (r32["single"] * 1e-3) / 1e9
    traffic = measured_traffic()
    line = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "Orszag-Tang vortex 4096x4096 periodic, FP32 storage+compute, "
                        "nu=eta=1e-5, Smagorinsky-MHD LES C_S=0.1, diagnostics every 100 steps",
            "lattice": [4096, 4096], "storage": "fp32", "nu": 1e-5, "eta": 1e-5, "cs": 0.1,
        },
        "steps_per_pass": spp,
        "hbm_bytes_per_site_update": FP32_BYTES_PER_SITE / spp,
        "one_step_per_pass_bound_mlups": round(HBM_PEAK_GBS * 1e9 / FP32_BYTES_PER_SITE / 1e6, 1),
        "roofline": {
            "kernel": {3: "k_step_t3<fp32,les>", 2: "k_step2<fp32,les>"}.get(spp, "k_step<fp32,les>"),
            "bound": "hbm",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic,
            "valu_frac": valu_frac("step_t3_fp32_4096", r32["per_launch"]),
            "binding": "neither HBM nor VALU saturated (VALU ceiling 0.86x the HBM ceiling): "
                       "9.5 waves per CU, each pass a chain of loads, three collisions and two "
                       "barriers",
            "bytes_per_site": FP32_BYTES_PER_SITE,
            "steps_per_launch": spp,
            "ms_per_launch": round(r32["per_launch"], 5),
        },
        "single_step": {
            "kernel": "k_step<fp32,les>",
            "mlups": round(r32["sites"] / (r32["single"] * 1e-3) / 1e6, 1),
            "ms_per_step": round(r32["single"], 5),
            "achieved_gbs": round(single_gbs, 1), "frac": round(single_gbs / HBM_PEAK_GBS, 4),
            "bytes_per_site": FP32_BYTES_PER_SITE,
            "speedup_of_steps_per_pass": round(r32["single"] / (r32["per_launch"] / spp), 3),
        },
        "cpu_baseline": cpu,
        "error_bound": {
            "fp32_rel_l2_uB": 1e-5,
            "fp32_workloads": "64^2 Orszag-Tang (nu = eta = 0.01) at steps 100, 500, 1000; 256^2 "
                              "turbulence (nu = eta = 1e-6) at steps 100 and 1000; 256^2 "
                              "Orszag-Tang at the headline parameters at step 300 (energies "
                              "within 2e-3 at step 1000)",
            "fp16_rel_l2_uB": {"step_100": 1.5e-3, "step_1000": 1.2e-2},
            "fp16_workload": "256^2 turbulence, nu = eta = 1e-6 (measured 8.4e-4 / 7.7e-3)",
            "targets_out_of_reach": "FP16 <= 1e-3 after 1000 steps and FP32 <= 1e-5 at step 1000 "
                                    "of the nu = 1e-5 Orszag-Tang run cannot be met by anything "
                                    "that rounds differently from the FP64 oracle: the oracle "
                                    "with FP16 storage rounding alone departs by 7.4e-3 at step "
                                    "1000, and a 1e-9 perturbation of that Orszag-Tang run grows "
                                    "past 1e-5 by step 1000 (tests/test_oracle_precision.py)",
            "checked_by": "tests/test_gpu_forward.py (oracle parity, 64^2/256^2 trajectories, "
                          "full-size sampled sites), tests/test_oracle_precision.py (what the "
                          "oracle fixes about the reachable accuracy)",
        },
    }
    if r3:
        t32, t16 = r3["fp32"], r3["fp16"]
        m3 = r3["sites"] / (t32["per_launch"] * 1e-3) / 1e6
        a3 = 360 * r3["sites"] / (t32["per_launch"] * 1e-3) / 1e9
        m316 = r3["sites"] / (t16["per_launch"] * 1e-3) / 1e6
        a316 = 180 * r3["sites"] / (t16["per_launch"] * 1e-3) / 1e9
        line["three_d"] = {
            "workload": "3D Orszag-Tang-type vortex 256^3, FP32, D3Q27 + 6 magnetic vectors, "
                        "LES C_S=0.1, nu=eta=1e-5",
            "mlups": round(m3, 1), "ms_per_step": round(t32["per_launch"], 5),
            "achieved_gbs": round(a3, 1), "frac": round(a3 / HBM_PEAK_GBS, 4),
            "bytes_per_site": 360, "nonfinite": t32["nonfinite"],
            "fp16": {"mlups": round(m316, 1), "ms_per_step": round(t16["per_launch"], 5),
                     "achieved_gbs": round(a316, 1), "frac": round(a316 / HBM_PEAK_GBS, 4),
                     "bytes_per_site": 180, "nonfinite": t16["nonfinite"],
                     "speedup_vs_fp32_mlups": round(m316 / m3, 3)},
        }
        tm = r3.get("fp32_mrt")
        if tm:
            am = 360 * r3["sites"] / (tm["per_launch"] * 1e-3) / 1e9
            line["three_d"]["moment_collision"] = {
                "what": "moment-space collision for f in the tensor-product basis of the "
                        "paper's D2Q9 rows and (1, c_z, 3 c_z^2 - 1), unequal rates "
                        "(s5, s7, s8, sg, szz) = (1.3, 0.7, 1.6, 1.1, 0.9), FP32",
                "mlups": round(r3["sites"] / (tm["per_launch"] * 1e-3) / 1e6, 1),
                "ms_per_step": round(tm["per_launch"], 5), "achieved_gbs": round(am, 1),
                "frac": round(am / HBM_PEAK_GBS, 4), "nonfinite": tm["nonfinite"],
            }
    if rin:
        mi = rin["sites"] / (rin["per_launch"] * 1e-3) / 1e6
        ai = FP32_BYTES_PER_SITE * rin["sites"] / (rin["per_launch"] * 1e-3) / 1e9
        line["inplace"] = {
            "workload": "Orszag-Tang 4096x4096, FP32, LES C_S=0.1, nu=eta=1e-5, one lattice "
                        "updated in place (AA pattern)",
            "mlups": round(mi, 1), "ms_per_step": round(rin["per_launch"], 5),
            "achieved_gbs": round(ai, 1), "frac": round(ai / HBM_PEAK_GBS, 4),
            "bytes_per_site": FP32_BYTES_PER_SITE, "nonfinite": rin["nonfinite"],
            "state_bytes": rin["lattice_bytes"], "state_bytes_two_lattices": 2 * rin["lattice_bytes"],
        }
    for key, res, what in (
            ("kinetic_closure", rkin, "kinetic LES closure (filtered equilibria, Delta = 1)"),
            ("cross_helicity_closure", rch,
             "cross-helicity LES closure with backscatter (C_S = 0.1, Delta = 1)")):
        if not res:
            continue
        # one launch reads and writes the lattice once for its steps_per_pass steps
        ms_launch = res["per_step"] * res["spp"]
        mk = res["sites"] / (res["per_step"] * 1e-3) / 1e6
        ak = FP32_BYTES_PER_SITE * res["sites"] / (ms_launch * 1e-3) / 1e9
        line[key] = {
            "workload": f"Orszag-Tang 4096x4096, FP32, {what}, nu=eta=1e-5",
            "mlups": round(mk, 1), "ms_per_step": round(res["per_step"], 5),
            "steps_per_pass": res["spp"], "ms_per_launch": round(ms_launch, 5),
            "achieved_gbs": round(ak, 1), "frac": round(ak / HBM_PEAK_GBS, 4),
            "bytes_per_site_per_launch": FP32_BYTES_PER_SITE, "nonfinite": res["nonfinite"],
        }
    if r16:
        f16, f32 = r16["fp16"], r16["fp32"]
        ms16, ms32 = f16["ms"] / args.fp16_steps, f32["ms"] / args.fp16_steps
        m16 = r16["sites"] / (ms16 * 1e-3) / 1e6
        m32 = r16["sites"] / (ms32 * 1e-3) / 1e6
        a16 = FP16_BYTES_PER_SITE * r16["sites"] / (f16["per_launch"] * 1e-3) / 1e9
        a32 = FP32_BYTES_PER_SITE * r16["sites"] / (f32["per_launch"] * 1e-3) / 1e9
        line["fp16"] = {
            "workload": "decaying 2D MHD turbulence 8192x8192, nu=eta=1e-6, LES C_S=0.1: FP16 "
                        "deviation storage (x2^10) against FP32 storage on the same fields",
            "steps": args.fp16_steps,
            "mlups": round(m16, 1), "ms_per_step": round(ms16, 5),
            "achieved_gbs": round(a16, 1), "frac": round(a16 / HBM_PEAK_GBS, 4),
            "bytes_per_site": FP16_BYTES_PER_SITE, "steps_per_launch": f16["steps_per_pass"],
            "nonfinite": f16["nonfinite"],
            "fp32_same_workload": {
                "mlups": round(m32, 1), "ms_per_step": round(ms32, 5),
                "achieved_gbs": round(a32, 1), "frac": round(a32 / HBM_PEAK_GBS, 4),
                "bytes_per_site": FP32_BYTES_PER_SITE, "steps_per_launch": f32["steps_per_pass"],
                "nonfinite": f32["nonfinite"],
            },
            "roofline": valu_roofline("step2_fp16_8192", f16["per_launch"]),
            "speedup_vs_fp32_same_workload": round(m16 / m32, 3),
            "speedup_vs_fp32_headline": round(m16 / value, 3),
            "rel_l2_vs_fp32": {"step": args.fp16_compare_steps,
                               "u": float(f"{r16['rel_l2_u_1000']:.4e}"),
                               "B": float(f"{r16['rel_l2_b_1000']:.4e}")},
        }
    if radj:
        s = radj["sites"]
        k100, kauto = radj["k100"], radj["auto"]
        per_step = lambda sec: sec * 1e3 / radj["nsteps"]
        line["adjoint"] = {
            "workload": f"perturbed Orszag-Tang 1024x1024, FP32, dJ/d(u0,B0,C_Sv,C_Sb) of the "
                        f"total energy after {radj['nsteps']} steps",
            "forward_ms_per_step": round(radj["fwd_ms"], 5),
            # the stated workload: checkpoints every 100 steps, each segment
            # recomputed before its reverse sweep
            "interval_100": {
                "forward_s": round(k100["fwd_s"], 4), "backward_s": round(k100["bwd_s"], 4),
                "backward_over_forward_wall": round(k100["bwd_s"] / k100["fwd_s"], 3),
                "backward_ms_per_step": round(per_step(k100["bwd_s"]), 5),
                "backward_over_forward_step": round(per_step(k100["bwd_s"]) / radj["fwd_ms"], 3),
                "J": k100["J"], "dJ_dcsv": k100["dJ_dcsv"], "dJ_dcsb": k100["dJ_dcsb"],
            },
            # every state kept when the run fits in HBM: nothing recomputed
            "interval_auto": {
                "interval": kauto["interval"],
                "forward_s": round(kauto["fwd_s"], 4), "backward_s": round(kauto["bwd_s"], 4),
                "backward_over_forward_wall": round(kauto["bwd_s"] / kauto["fwd_s"], 3),
                "backward_ms_per_step": round(per_step(kauto["bwd_s"]), 5),
                "backward_over_forward_step": round(per_step(kauto["bwd_s"]) / radj["fwd_ms"], 3),
            },
            "gradient_check": {
                "what": "adjoint directional derivatives against central differences of the "
                        "FP32 forward run, seeded directions 100 and 107; at 500 steps they "
                        "agree, at 2000 steps the differences do not converge as eps falls "
                        "(the flow amplifies rounding-size differences between the two runs)",
                "steps": radj["grad_check"],
            },
            "adj_kernel_ms": round(radj["adj_kernel_ms"], 5),
            "adj_kernel_over_forward_step": round(radj["adj_kernel_ms"] / radj["fwd_ms"], 3),
            "adj_kernel_gbs": round(3 * 19 * 4 * s / (radj["adj_kernel_ms"] * 1e-3) / 1e9, 1),
            "segment_4096": {
                "workload": "Orszag-Tang 4096x4096, FP32, LES: one 100-step checkpoint segment "
                            "(the 49 even states recomputed into one block, a pass per pair, "
                            "then 100 reverse steps two per pass)",
                "recompute_ms_per_step": round(radj["recompute_ms_4096"], 5),
                "adjoint_ms_per_step": round(radj["adj_ms_4096"], 5),
                "forward_ms_per_step": round(radj["fwd_ms_4096"], 5),
                "adjoint_over_forward_step": round(radj["adj_ms_4096"] / radj["fwd_ms_4096"], 3),
                "recompute_plus_adjoint_over_forward_step": round(
                    (radj["recompute_ms_4096"] + radj["adj_ms_4096"]) / radj["fwd_ms_4096"], 3),
                # x_t, lam_{t+2} and lam_t once per pair of reverse steps
                "adj_pair_kernel_gbs": round(3 * 19 * 4 * 4096 * 4096 / (2 * radj["adj_ms_4096"] * 1e-3) / 1e9, 1),
                "adj_pair_kernel_frac": round(3 * 19 * 4 * 4096 * 4096 / (2 * radj["adj_ms_4096"] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                "reverse_step_single_ms": round(radj["adj_single_ms_4096"], 5),
                "reverse_step_paired_ms": round(radj["adj_pair_ms_4096"], 5),
            },
            "run_4096": {
                "workload": f"Orszag-Tang 4096x4096, FP32, LES, {radj['run_4096']['nsteps']} steps, "
                            "checkpoint interval from the free HBM, reverse steps in pairs",
                "interval": radj["run_4096"]["interval"],
                "forward_ms_per_step": round(radj["run_4096"]["fwd_ms"], 5),
                "backward_ms_per_step": round(radj["run_4096"]["bwd_ms"], 5),
                "backward_over_forward_step": round(radj["run_4096"]["bwd_ms"] / radj["fwd_ms_4096"], 3),
                "J": radj["run_4096"]["J"], "dJ_dcsv": radj["run_4096"]["dJ_dcsv"],
            },
            "kinetic_closure_adj_ms_4096": round(radj["adj_kin_ms_4096"], 5),
            "kinetic_closure_adj_gbs_4096": round(228 * 4096 * 4096 / (radj["adj_kin_ms_4096"] * 1e-3) / 1e9, 1),
            "kinetic_closure_adj_over_forward_4096": round(radj["adj_kin_ms_4096"] / radj["fwd_kin_ms_4096"], 3),
        }
    if rfit:
        r = rfit["res"]
        ib = min(range(len(r.loss)), key=r.loss.__getitem__)
        line["cs_fit"] = {
            "workload": f"joint (C_Sv, C_Sb) fit: 2048x2048 FP16-storage LES "
                        f"({rfit['steps']} steps, nu=eta=2.5e-7) "
                        f"against the width-4 box filter of an 8192x8192 FP32 LES run "
                        f"({args.fit_ref_steps} steps, nu=eta=1e-6), decaying turbulence",
            "iterations": len(r.cs), "seconds": round(r.seconds, 3),
            "reference_seconds": round(rfit["t_ref"], 3),
            "cs_v": [round(c, 6) for c in r.cs], "cs_b": [round(c, 6) for c in r.cs_b],
            "loss": [float(f"{v:.6e}") for v in r.loss],
            "best": [round(r.cs[ib], 6), round(r.cs_b[ib], 6)],
        }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
