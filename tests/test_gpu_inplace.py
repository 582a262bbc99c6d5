"""In-place (AA pattern) update against the two-lattice update.

The in-place steps alternate between a gather/scatter step into reversed
slots and a local step back; each site runs the same collision arithmetic as
the two-lattice step, so after any number of steps the populations must be
bit-identical, whichever layout the lattice is left in (an odd step count
leaves it reversed and the next read turns it back in place).  Uninterrupted
runs alternate both step kinds; runs read after every step repeat the first
kind.  Sizes cover several 256-site tiles, ragged ends, odd widths (the FP16
kernels then take one site per thread) and production lattices.  (The FP16
encoder keeps its FP32 input unfused: a half conversion fused with the
preceding multiply-add rounds once instead of twice and made about 2 in 10^5
stored codes differ between the two kinds of kernel on 8192 x 4096.)
"""
import numpy as np
import pytest
import torch

from lbmhd_inputs import orszag_tang, perturbed_orszag_tang, random_planes

pytestmark = pytest.mark.gpu

W9 = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)
W19 = np.concatenate([W9, np.zeros(10)])


@pytest.fixture(scope="module")
def lb():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1607_08675_amd import lattice
    return lattice


def assert_same(a, b, what=""):
    d = (a - b).abs()
    assert torch.equal(a, b), (what, int((d > 0).sum()), float(d.max()))


def pair(lb, **kw):
    cfg = lb.LBMHDConfig(**kw)
    two = lb.Lattice(cfg)
    one = lb.Lattice(lb.LBMHDConfig(**{**cfg.__dict__, "inplace": True}))
    assert one._b is None
    return two, one


@pytest.mark.parametrize("storage", ["fp32", "fp16"])
@pytest.mark.parametrize("les", [0, 1])
@pytest.mark.parametrize("nx,ny", [(8, 8), (100, 36), (257, 3), (300, 5), (2, 2), (514, 7)])
def test_every_step_count_matches_two_lattices(lb, nx, ny, les, storage):
    two, one = pair(lb, nx=nx, ny=ny, nu=0.01, eta=0.02, s5=1.2, s7=1.5, s8=0.8, les=les,
                    cs=0.15, cs_b=0.1, storage=storage)
    scale = np.concatenate([W9 * 0.02, np.full(10, 0.01)])
    x0 = random_planes(19, nx, ny, nx * 31 + ny, W19, scale)
    two.set_populations(x0)
    one.set_populations(x0)
    for n in range(1, 6):        # odd counts leave the in-place lattice reversed
        two.step(1)
        one.step(1)
        assert_same(two.populations(), one.populations(), f"after {n} steps")
    for n in (2, 5):             # uninterrupted runs alternate both step kinds
        two.set_populations(x0).step(n)
        one.set_populations(x0).step(n)
        assert_same(two.populations(), one.populations(), f"{n} steps at once")


def test_orszag_tang_run_and_diagnostics(lb):
    """64^2 Orszag-Tang, 1001 steps with diagnostics at odd and even counts."""
    n = 64
    two, one = pair(lb, nx=n, ny=n, nu=0.01, eta=0.01, les=1, cs=0.1)
    f = orszag_tang(n, n)
    two.init_fields(*f)
    one.init_fields(*f)
    for k in (1, 100, 400, 500):
        two.step(k)
        one.step(k)
        assert two.diag() == one.diag()
    assert torch.equal(two.populations(), one.populations())
    m2, m1 = two.macro(), one.macro()
    for key in m2:
        assert torch.equal(m2[key], m1[key]), key


def test_checkpoint_and_gradient(lb, orc):
    """Checkpoints saved from an in-place lattice restore it exactly, and the
    adjoint gradient through an in-place forward run equals the two-lattice
    one (the recomputed segments start from the saved natural-layout states)."""
    from paper_1607_08675_amd.adjoint import LBMHDFunction
    n, steps = 32, 37
    two, one = pair(lb, nx=n, ny=n, nu=0.002, eta=0.002, les=1, cs=0.2)
    f = perturbed_orszag_tang(n, n, u0=0.1, b0=0.1)
    one.init_fields(*f).step(7)
    st = one.save_state()
    one.step(5)
    one.load_state(st, 7)
    two.init_fields(*f).step(7)
    # (rows are padded to 256 bytes; the padding is never written, so compare
    # the decoded populations, not the raw bytes)
    assert torch.equal(one.populations(), two.populations())
    dev = torch.device("cuda")
    grads = []
    for inplace in (False, True):
        cfg = lb.LBMHDConfig(nx=n, ny=n, nu=0.002, eta=0.002, les=1, cs=0.2, inplace=inplace)
        t = [torch.tensor(a, dtype=torch.float64, device=dev, requires_grad=True) for a in f[1:]]
        cs = torch.tensor([0.2, 0.2], dtype=torch.float64, device=dev, requires_grad=True)
        J = LBMHDFunction.apply(*t, cs, cfg, steps, 10)
        J.backward()
        grads.append([float(J.detach())] + [ti.grad.cpu().numpy() for ti in t] + [cs.grad.cpu().numpy()])
    assert grads[0][0] == grads[1][0]
    for a, b in zip(grads[0][1:], grads[1][1:]):
        np.testing.assert_array_equal(a, b)


@pytest.mark.parametrize("storage,nx,ny", [("fp32", 4096, 4096), ("fp16", 8192, 4096),
                                           ("fp16", 4097, 2048)])
def test_production_size(lb, storage, nx, ny):
    """Production-size lattices (4096^2 FP32; 8192 x 4096 FP16, two sites per
    thread; an odd FP16 width, one site per thread), 3 and then 4 steps run
    without reads in between."""
    two, one = pair(lb, nx=nx, ny=ny, nu=1e-5, eta=1e-5, les=1, cs=0.1, storage=storage)
    f = orszag_tang(nx, ny)
    two.init_fields(*f)
    one.init_fields(*f)
    for k in (3, 4):
        two.step(k)
        one.step(k)
        assert_same(two.populations(), one.populations(), k)
    del two, one
    torch.cuda.empty_cache()


@pytest.mark.parametrize("storage", ["fp32", "fp16"])
def test_bound_lattice_passed_as_explicit_state(lb, storage):
    """After an odd step count the in-place lattice is reversed; calls given
    the bound lattice itself as their state read it in the natural layout."""
    two, one = pair(lb, nx=40, ny=24, nu=0.01, eta=0.01, les=1, cs=0.1, storage=storage)
    fields = perturbed_orszag_tang(40, 24)
    two.init_fields(*fields).step(3)
    one.init_fields(*fields).step(3)
    assert one.energy(one._a) == two.energy()
    one.step(2)
    two.step(2)
    # zeroed: the kernels leave the row padding alone
    a, b = one.new_state_buffer().zero_(), two.new_state_buffer().zero_()
    one.step_between(one._a, a)
    two.step_between(two.save_state(), b)
    assert torch.equal(a, b)
    lam1, lam2 = one.new_adj_buffer(), two.new_adj_buffer()
    one.step(1)
    two.step(1)
    one.adj_seed_energy(one._a, lam1)
    two.adj_seed_energy(two.save_state(), lam2)
    assert torch.equal(one.adj_view(lam1), two.adj_view(lam2))


def test_load_state_of_the_reversed_lattice_itself(lb):
    """load_state(current_state()) on an in-place lattice left reversed by an
    odd step count turns the layout back before taking it as the state, and a
    buffer that partly overlaps the bound lattice is refused."""
    import ctypes
    n = 64
    two, one = pair(lb, nx=n, ny=n, nu=0.002, eta=0.002, les=1, cs=0.2)
    f = perturbed_orszag_tang(n, n, u0=0.1, b0=0.1)
    one.init_fields(*f).step(7)
    one.load_state(one.current_state(), 7)
    two.init_fields(*f).step(7)
    assert_same(one.populations(), two.populations(), "after load")
    one.step(4)
    two.step(4)
    assert_same(one.populations(), two.populations(), "four steps on")
    # through the C ABI: a source 256 bytes into the bound lattice
    p = ctypes.c_void_p(one.current_state().data_ptr() + 256)
    assert one._L.lbmhd_load_state(one._h, p, ctypes.c_int64(11)) == -1   # LBMHD_ERR_INVALID_ARG
    assert one.step_count == 11
