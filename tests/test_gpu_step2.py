"""Two and three steps per pass over the lattice (temporal blocking) against
single steps and against the oracle (GPU).

A fused pass keeps the intermediate state on chip in the storage encoding, so
n steps taken several per pass reproduce n single steps bit for bit, in FP32
and in FP16 storage: full and ragged tiles (256 columns FP32, 512 FP16 with nx
even, 256 FP16 with nx odd), ragged strips, tiny periodic lattices where the
halo columns and rows wrap onto the tile itself, odd step counts, rough
fields and the largest headline lattice.  The collision spells out every
fused multiply-add and forbids the compiler any other contraction, so the
copies of it inlined for one and two sites per thread and for the halo
columns round identically.  The oracle comparison repeats the forward parity
bound on the fused path itself.
"""
import numpy as np
import pytest
import torch

from lbmhd_inputs import decaying_turbulence, orszag_tang, random_fields
from state_words import stored_words

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lb():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1607_08675_amd import lattice
    return lattice


def stored(L):
    return stored_words(L)


def same(a, b):
    assert torch.equal(a, b), int((a != b).sum())


def pair(lb, fields, n, **kw):
    out = []
    for spp in (1, 2):
        L = lb.Lattice(lb.LBMHDConfig(steps_per_pass=spp, **kw))
        L.init_fields(*fields).step(n)
        assert L.step_count == n
        out.append(stored(L))
    return out


# (600, 60) FP32 and (1030, 124) FP16 have a multiple of 8 strips with a ragged
# last one and several tiles each: their blocks take the XCD-grouped order
CASES = [
    ("fp32", 256, 64), ("fp32", 300, 70), ("fp32", 2, 2), ("fp32", 3, 5), ("fp32", 513, 9),
    ("fp32", 600, 60), ("fp16", 512, 40), ("fp16", 600, 70), ("fp16", 2, 2),
    ("fp16", 1030, 17), ("fp16", 1030, 124), ("fp16", 301, 33), ("fp16", 3, 3),
]


@pytest.mark.parametrize("storage,nx,ny", CASES)
@pytest.mark.parametrize("les", [0, 1])
@pytest.mark.parametrize("n", [5, 6])
def test_fused_equals_single_steps(lb, storage, nx, ny, les, n):
    fields = random_fields(nx, ny, 7 + nx + ny)
    a, b = pair(lb, fields, n, nx=nx, ny=ny, nu=1e-3, eta=2e-3, les=les, cs=0.15,
                storage=storage)
    assert torch.equal(a, b), int((a != b).sum())


@pytest.mark.parametrize("storage,nx,ny", [("fp32", 1061, 2000), ("fp32", 2048, 1536),
                                           ("fp16", 3000, 8000)])
def test_fused_equals_single_steps_mid_strips(lb, storage, nx, ny):
    """Strip heights between the bounds: 19 rows with a ragged last strip in
    block order; 24 rows in XCD-grouped order; 11 rows, ragged, XCD-grouped."""
    fields = decaying_turbulence(nx, ny, u_rms=0.05, b_rms=0.05)
    a, b = pair(lb, fields, 4, nx=nx, ny=ny, nu=1e-4, eta=1e-4, les=1, cs=0.1,
                storage=storage)
    same(a, b)


@pytest.mark.parametrize("storage", ["fp32", "fp16"])
def test_fused_equals_single_steps_headline_size(lb, storage):
    """4096^2 Orszag-Tang with the Smagorinsky-MHD closure: 128-row strips
    (FP32) and 8-row strips of 512 columns (FP16), XCD-grouped."""
    n = 4096
    fields = orszag_tang(n, n)
    a, b = pair(lb, fields, 4, nx=n, ny=n, nu=1e-5, eta=1e-5, les=1, cs=0.1, storage=storage)
    same(a, b)


@pytest.mark.parametrize("storage,n", [("fp32", 4096), ("fp16", 2048), ("fp16", 4096)])
def test_fused_equals_single_steps_rough_fields(lb, storage, n):
    """Rough random fields, one fused pass, bit for bit in both storages."""
    a, b = pair(lb, random_fields(n, n, 3), 2, nx=n, ny=n, nu=1e-4, eta=1e-4, les=1, cs=0.1,
                storage=storage)
    same(a, b)


@pytest.mark.parametrize("storage,nx,ny,n,deep", [
    ("fp32", 300, 70, 5, 2), ("fp32", 600, 60, 6, 2), ("fp16", 512, 40, 4, 2),
    ("fp16", 301, 33, 5, 2), ("fp32", 1024, 1024, 4, 2), ("fp32", 300, 70, 3, 3),
    ("fp32", 300, 70, 7, 3), ("fp32", 600, 60, 8, 3), ("fp32", 5, 3, 4, 3),
    ("fp32", 1024, 1024, 6, 3)])
def test_stored_trajectory_two_steps_per_pass(lb, storage, nx, ny, n, deep):
    """lbmhd_step_store with two or three steps per pass (the pass also stores
    its intermediate states) writes every state of the one-step trajectory."""
    fields = random_fields(nx, ny, 13)
    rows = []
    for spp in (1, deep):
        L = lb.Lattice(lb.LBMHDConfig(nx=nx, ny=ny, nu=1e-3, eta=2e-3, les=1, cs=0.15,
                                      storage=storage, steps_per_pass=spp))
        L.init_fields(*fields)
        store = torch.zeros(n, L.lattice_bytes, dtype=torch.uint8, device="cuda")
        L.step_store(L.save_state(), store, n)
        rows.append([stored_words(L, store[t]).clone() for t in range(n)])
    for t in range(n):
        assert torch.equal(rows[0][t], rows[1][t]), (t, int((rows[0][t] != rows[1][t]).sum()))


def test_gradient_with_two_steps_per_pass_matches_single(lb):
    """The checkpointed gradient (stored trajectory and checkpointed segments)
    with two or three steps per pass equals the one-step gradient bit for bit
    (FP32)."""
    from paper_1607_08675_amd.adjoint import LBMHDFunction
    n, steps = 64, 30
    fields = decaying_turbulence(n, n, u_rms=0.05, b_rms=0.05)
    out = []
    for spp in (1, 2, 3):
        for every in (1, 7):
            cfg = lb.LBMHDConfig(nx=n, ny=n, nu=1e-4, eta=1e-4, les=1, cs=0.1, cs_b=0.07,
                                 steps_per_pass=spp)
            t = [torch.tensor(f, dtype=torch.float64, device="cuda", requires_grad=True)
                 for f in fields[1:]]
            cs = torch.tensor(0.1, dtype=torch.float64, device="cuda", requires_grad=True)
            J = LBMHDFunction.apply(*t, cs, cfg, steps, every)
            J.backward()
            out.append((float(J), [ti.grad.clone() for ti in t], float(cs.grad)))
    ref = out[0]
    for o in out[1:]:
        assert o[0] == ref[0] and o[2] == ref[2]
        for a, b in zip(o[1], ref[1]):
            assert torch.equal(a, b)


T3_CASES = [(256, 64), (300, 70), (2, 2), (3, 5), (513, 9), (600, 60), (5, 3), (77, 41)]


@pytest.mark.parametrize("nx,ny", T3_CASES)
@pytest.mark.parametrize("les", [0, 1])
@pytest.mark.parametrize("n", [3, 4, 5, 7])
def test_three_steps_per_pass_equal_single_steps(lb, nx, ny, les, n):
    """Three steps per pass (FP32): triples, then a remainder of two as one
    pair and of one as a single step, bit for bit equal to single steps; full
    and ragged tiles and strips, halos wrapping onto tiny lattices."""
    fields = random_fields(nx, ny, 23 + nx + ny)
    out = []
    for spp in (1, 3):
        L = lb.Lattice(lb.LBMHDConfig(nx=nx, ny=ny, nu=1e-3, eta=2e-3, les=les, cs=0.15,
                                      steps_per_pass=spp))
        assert L.steps_per_pass == spp
        L.init_fields(*fields).step(n)
        assert L.step_count == n
        out.append(stored_words(L))
    assert torch.equal(out[0], out[1]), int((out[0] != out[1]).sum())


@pytest.mark.parametrize("nx,ny,gen", [(4096, 4096, "ot"), (4096, 4096, "rough"),
                                       (1061, 2000, "turb"), (2048, 1536, "turb"),
                                       (8192, 4096, "rough")])
def test_three_steps_per_pass_large(lb, nx, ny, gen):
    """The headline lattice (128-row strips, XCD-grouped), rough fields, strip
    heights between the bounds (ragged and XCD-grouped) and a lattice past
    the 128-row bound (32-row strips)."""
    f = {"ot": lambda: orszag_tang(nx, ny), "rough": lambda: random_fields(nx, ny, 3),
         "turb": lambda: decaying_turbulence(nx, ny, u_rms=0.05, b_rms=0.05)}[gen]()
    out = []
    for spp in (1, 3):
        L = lb.Lattice(lb.LBMHDConfig(nx=nx, ny=ny, nu=1e-5, eta=1e-5, les=1, cs=0.1,
                                      steps_per_pass=spp))
        L.init_fields(*f).step(6)
        out.append(stored_words(L))
        del L
    assert torch.equal(out[0], out[1]), int((out[0] != out[1]).sum())


def test_three_steps_per_pass_matches_oracle(lb, orc):
    nx, ny, steps = 300, 70, 12
    fields = decaying_turbulence(nx, ny, u_rms=0.05, b_rms=0.05)
    L = lb.Lattice(lb.LBMHDConfig(nx=nx, ny=ny, nu=1e-3, eta=1e-3, les=1, cs=0.15,
                                  steps_per_pass=3))
    L.init_fields(*fields).step(steps)
    got = {k: v.cpu().numpy() for k, v in L.macro().items()}
    op = orc.Params(nx, ny, nu=1e-3, eta=1e-3, les=True, cs=0.15)
    want = orc.macro(op, orc.run(op, orc.init(op, *fields), steps))
    for k in ("ux", "uy", "bx", "by"):
        err = np.linalg.norm(got[k] - want[k]) / np.linalg.norm(want[k])
        assert err < 1e-5, (k, err)


@pytest.mark.parametrize("spp,n", [(1, 3), (2, 3), (2, 4), (3, 3), (3, 4), (3, 7)])
def test_current_state_follows_the_passes(lb, spp, n):
    """lbmhd_current_state names the lattice that holds the state, whatever
    the number of kernel passes the steps took."""
    nx, ny = 300, 70
    L = lb.Lattice(lb.LBMHDConfig(nx=nx, ny=ny, steps_per_pass=spp))
    L.init_fields(*random_fields(nx, ny, 3)).step(n)
    cur = L.current_state()
    assert torch.equal(stored_words(L, cur), stored_words(L))


@pytest.mark.parametrize("deep", [2, 3])
def test_multi_step_long_run_equals_single_steps(lb, deep):
    """301 steps of 1024^2 Orszag-Tang (FP32, LES) two or three per pass,
    remainders included, against 301 single steps, bit for bit: any
    difference would have been amplified by the flow over that many steps."""
    n = 1024
    fields = orszag_tang(n, n)
    out = []
    for spp in (1, deep):
        L = lb.Lattice(lb.LBMHDConfig(nx=n, ny=n, nu=1e-5, eta=1e-5, les=1, cs=0.1,
                                      steps_per_pass=spp))
        L.init_fields(*fields)
        for chunk in (100, 100, 100, 1):
            L.step(chunk)
        assert L.step_count == 301
        out.append(stored_words(L))
    assert torch.equal(out[0], out[1]), int((out[0] != out[1]).sum())


def test_fused_interleaved_with_stored_steps(lb):
    """Fused steps, single steps into a store, and fused steps again, against
    single steps throughout."""
    nx, ny = 300, 70
    fields = random_fields(nx, ny, 11)
    kw = dict(nx=nx, ny=ny, nu=1e-3, eta=2e-3, les=1, cs=0.15)
    ref = lb.Lattice(lb.LBMHDConfig(steps_per_pass=1, **kw))
    ref.init_fields(*fields).step(9)
    L = lb.Lattice(lb.LBMHDConfig(**kw))
    L.init_fields(*fields).step(4)
    store = torch.empty(3, L.lattice_bytes, dtype=torch.uint8, device="cuda")
    L.step_store(L.save_state(), store, 3)
    L.load_state(store[2], 7).step(2)
    assert L.step_count == 9
    assert torch.equal(stored(L), stored(ref))


@pytest.mark.parametrize("storage,nx,ny", [("fp32", 300, 70), ("fp16", 600, 34), ("fp16", 77, 41)])
def test_fused_path_matches_oracle(lb, orc, storage, nx, ny):
    steps = 12
    fields = decaying_turbulence(nx, ny, u_rms=0.05, b_rms=0.05)
    cfg = lb.LBMHDConfig(nx=nx, ny=ny, nu=1e-3, eta=1e-3, les=1, cs=0.15, storage=storage)
    L = lb.Lattice(cfg)
    L.init_fields(*fields).step(steps)
    got = {k: v.cpu().numpy() for k, v in L.macro().items()}
    op = orc.Params(nx, ny, nu=1e-3, eta=1e-3, les=True, cs=0.15)
    want = orc.macro(op, orc.run(op, orc.init(op, *fields), steps))
    bound = 1e-5 if storage == "fp32" else 1.5e-3
    for k in ("ux", "uy", "bx", "by"):
        err = np.linalg.norm(got[k] - want[k]) / np.linalg.norm(want[k])
        assert err < bound, (k, err)
