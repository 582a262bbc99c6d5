"""Steps with diagnostics along the way (GPU): lbmhd_run against lbmhd_step and
lbmhd_diag called in turn.

lbmhd_run takes the diagnostics of the states at steps every, 2 every, ... on a
second stream, each overlapping the next kernel pass, and waits on the host once.
Its results must equal those of the plain sequence (step(every), diag(), ...,
then the remaining steps) exactly: the same kernels on the same states in the
same reduction order, the step counts, and the final state bit for bit.  An
interval of one or three steps makes every pass write the lattice that a
diagnostics pass enqueued one or two passes earlier reads, so a missing wait
would show as a differing result at 1024^2, where the passes take tens of
microseconds.  Intervals that end in a single step of FP32 storage take that
step and its diagnostics in one fused pass, also equal bit for bit (the headline
lattice, the plain update, ragged and tiny lattices, every step).  Also: the
in-place lattice, FP16 storage, the kinetic closure, the non-finite count, and
the argument checks (made before anything is enqueued).
"""
import ctypes

import numpy as np
import pytest
import torch

from lbmhd_inputs import orszag_tang
from state_words import stored_words

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lb():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1607_08675_amd import lattice
    return lattice


def pair(lb, n, **kw):
    """Two lattices of the same configuration (n x n, or nx x ny for n a
    pair), both at the Orszag-Tang state."""
    nx, ny = n if isinstance(n, tuple) else (n, n)
    cfg = lb.LBMHDConfig(nx=nx, ny=ny, nu=1e-4, eta=1e-4, les=kw.pop("les", 1), cs=0.1,
                         delta=1.0, **kw)
    a, b = lb.Lattice(cfg), lb.Lattice(cfg)
    f = orszag_tang(nx, ny)
    a.init_fields(*f)
    b.init_fields(*f)
    return a, b


def plain(L, n, every):
    """The reference: step(every) then diag(), as long as whole intervals fit."""
    out = []
    done = 0
    while done + every <= n:
        L.step(every)
        done += every
        out.append(L.diag())
    L.step(n - done)
    return out


CASES = [
    # (name, lattice side, config keywords, steps, interval)
    ("fp32 triples", 512, dict(storage="fp32", steps_per_pass=3), 230, 50),
    ("fp32 interval 7", 256, dict(storage="fp32", steps_per_pass=3), 40, 7),
    ("fp32 pairs", 256, dict(storage="fp32", steps_per_pass=2), 41, 10),
    ("fp32 single", 256, dict(storage="fp32", steps_per_pass=1), 25, 4),
    ("fp16 pairs", 512, dict(storage="fp16", steps_per_pass=2), 101, 20),
    ("kinetic pairs", 256, dict(storage="fp32", steps_per_pass=2, les=2), 30, 6),
    ("in place", 256, dict(storage="fp32", inplace=True), 33, 5),
    ("overlap every pass", 1024, dict(storage="fp32", steps_per_pass=3), 60, 3),
    ("overlap single steps", 1024, dict(storage="fp16", steps_per_pass=2), 12, 1),
    # intervals that end in a single step of FP32 storage: that step and the
    # diagnostics in one pass (k_step_diag)
    ("fused headline chunks", 4096, dict(storage="fp32", steps_per_pass=3), 200, 100),
    ("fused plain", 256, dict(storage="fp32", steps_per_pass=3, les=0), 22, 4),
    ("fused ragged", (300, 70), dict(storage="fp32", steps_per_pass=3), 15, 7),
    ("fused tiny", (5, 3), dict(storage="fp32", steps_per_pass=1), 9, 3),
    ("fused every step", 1024, dict(storage="fp32", steps_per_pass=3), 12, 1),
]


@pytest.mark.parametrize("name,n,kw,steps,every", CASES, ids=[c[0] for c in CASES])
def test_run_equals_steps_then_diag(lb, name, n, kw, steps, every):
    print(f"\nrun {name} {n} steps={steps} every={every}", flush=True)
    a, b = pair(lb, n, **kw)
    got = a.run(steps, every)
    want = plain(b, steps, every)
    assert len(got) == len(want) == steps // every
    for k, (g, w) in enumerate(zip(got, want)):
        assert g["step"] == w["step"] == every * (k + 1)
        for key, v in w.items():
            assert g[key] == v or (np.isnan(v) and np.isnan(g[key])), (k, key, g[key], v)
    assert a.step_count == b.step_count == steps
    assert torch.equal(stored_words(a), stored_words(b))
    # the handle keeps working on its bound stream afterwards
    a.step(3)
    b.step(3)
    assert a.diag() == b.diag()


def test_run_without_whole_interval_is_step(lb):
    a, b = pair(lb, 128, storage="fp32", steps_per_pass=3)
    assert a.run(10, 25) == []
    assert a.run(5, 0) == []
    assert a._L.lbmhd_run(a._h, 4, 5, None, None, 0) == 0
    b.step(19)
    assert a.step_count == 19
    assert torch.equal(stored_words(a), stored_words(b))


def test_run_reports_nonfinite(lb):
    n = 64
    a, _ = pair(lb, n, storage="fp32", steps_per_pass=3)
    pops = a.populations().cpu().numpy()
    pops[4, 10, 20] = np.nan
    a.set_populations(pops)
    got = a.run(9, 3)
    assert len(got) == 3 and all(d["nonfinite"] > 0 for d in got)
    from paper_1607_08675_amd._capi import LbmhdError
    with pytest.raises(LbmhdError):
        a.run(6, 3, raise_nonfinite=True)


def test_run_argument_checks(lb):
    from paper_1607_08675_amd import _capi as C
    a, _ = pair(lb, 64, storage="fp32", steps_per_pass=3)
    L, h = a._L, a._h
    dev = torch.zeros(16 * 4, dtype=torch.float64, device="cuda")
    out = (C.Diag * 4)()
    p = ctypes.c_void_p(dev.data_ptr())
    assert L.lbmhd_run(h, -1, 2, p, out, 4) == C.LBMHD_ERR_INVALID_ARG
    assert L.lbmhd_run(h, 8, -2, p, out, 4) == C.LBMHD_ERR_INVALID_ARG
    assert L.lbmhd_run(h, 8, 2, p, out, 3) == C.LBMHD_ERR_INVALID_ARG      # 4 results
    assert L.lbmhd_run(h, 8, 2, None, out, 4) == C.LBMHD_ERR_INVALID_ARG
    assert L.lbmhd_run(h, 8, 2, p, None, 4) == C.LBMHD_ERR_INVALID_ARG
    unaligned = ctypes.c_void_p(dev.data_ptr() + 4)
    assert L.lbmhd_run(h, 8, 2, unaligned, out, 4) == C.LBMHD_ERR_INVALID_ARG
    state = ctypes.c_void_p()
    assert L.lbmhd_current_state(h, ctypes.byref(state)) == 0
    assert L.lbmhd_run(h, 8, 2, state, out, 4) == C.LBMHD_ERR_INVALID_ARG   # a bound lattice
    assert a.step_count == 0
    assert a.run(8, 2, dev)[-1]["step"] == 8
