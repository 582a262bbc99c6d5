"""Two reverse steps per pass (GPU): lbmhd_adj_step2, the paired sweeps and
the every-other-state store, against single reverse steps.

The pass recomputes x_{t+1} = C(S(x_t)) on chip with the forward collision
and the storage codec, so it sees the values a stored x_{t+1} would hold, and
applies the same transposed collision as the single reverse step: lam_t equals
two lbmhd_adj_step calls bit for bit.  The closure-constant derivatives are
summed per block over both steps, in another order than two single steps, so
those agree to 1e-12 relative.  Cases: full and ragged 256-column tiles and
strips, lattices two and three sites wide or high (the halo columns and rows
wrap onto the tile), FP32 and FP16 states, les = 0 and 1, and C_S = 0 with
les = 1 (the forward step then takes the plain collision, the reverse step
still differentiates the closure).  The sweeps: even and odd step counts,
the every-other-state store against lbmhd_step_store, and the full-store
sweep where it takes pairs by itself (1024^2).
"""
import numpy as np
import pytest
import torch

from lbmhd_inputs import perturbed_orszag_tang, random_planes

pytestmark = pytest.mark.gpu

W9 = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)
W19 = np.concatenate([W9, np.zeros(10)])


@pytest.fixture(scope="module")
def lb():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1607_08675_amd import lattice
    return lattice


def random_state(nx, ny, seed):
    scale = np.concatenate([W9 * 0.02, np.full(10, 0.01)])
    return random_planes(19, nx, ny, seed, W19, scale)


def random_adjoint(L, seed):
    g = torch.Generator(device="cuda").manual_seed(seed)
    lam = L.new_adj_buffer()
    lam.copy_(torch.randn(lam.shape, generator=g, device="cuda", dtype=torch.float32))
    return lam


def close(a, b, rel=1e-12):
    for x, y in zip(a, b):
        assert abs(x - y) <= rel * max(abs(y), 1e-300), (a, b)


SIZES = [(256, 64), (300, 70), (2, 2), (3, 5), (5, 3), (513, 9), (600, 60), (77, 41),
         (1030, 17)]
CLOSURES = [(0, 0.1), (1, 0.12), (1, 0.0)]


@pytest.mark.parametrize("storage", ["fp32", "fp16"])
@pytest.mark.parametrize("les,cs", CLOSURES)
@pytest.mark.parametrize("nx,ny", SIZES)
def test_pair_equals_two_single_reverse_steps(lb, nx, ny, les, cs, storage):
    print(f"\nadj pair les={les} cs={cs} {storage} {nx}x{ny}", flush=True)
    cfg = lb.LBMHDConfig(nx=nx, ny=ny, nu=0.01, eta=0.02, s5=1.2, s7=1.5, s8=0.8, les=les,
                         cs=cs, cs_b=0.07 if cs else 0.0, delta=1.3, storage=storage)
    L = lb.Lattice(cfg)
    L.set_populations(random_state(nx, ny, nx * 100 + ny + les))
    x0 = L.save_state()
    x1 = L.new_state_buffer().zero_()
    L.step_between(x0, x1)
    lam = random_adjoint(L, nx + ny)
    # two single reverse steps
    mid, out1, acc1 = L.new_adj_buffer(), L.new_adj_buffer(), L.new_adj_acc()
    L.adj_step(x1, lam, mid, acc1)
    L.adj_step(x0, mid, out1, acc1)
    # one pair
    out2, acc2 = L.new_adj_buffer(), L.new_adj_acc()
    L.adj_step2(x0, lam, out2, acc2)
    a, b = L.adj_view(out1), L.adj_view(out2)
    assert torch.equal(a, b), (int((a != b).sum()), float((a - b).abs().max()),
                               float(a.abs().max()))
    close(L.adj_acc_total(acc2), L.adj_acc_total(acc1))


@pytest.mark.parametrize("n", [1, 2, 5, 6])
@pytest.mark.parametrize("storage", ["fp32", "fp16"])
def test_paired_sweep_over_every_other_state(lb, n, storage):
    """lbmhd_step_store_pairs keeps the even states of lbmhd_step_store bit for
    bit (row stride larger than a lattice); lbmhd_adj_sweep_pairs over them
    leaves the lam_0 of n single reverse steps."""
    nx, ny = 300, 70
    print(f"\nadj sweep pairs n={n} {storage}", flush=True)
    cfg = lb.LBMHDConfig(nx=nx, ny=ny, nu=0.01, eta=0.01, les=1, cs=0.12, cs_b=0.07,
                         storage=storage)
    L = lb.Lattice(cfg)
    L.init_fields(*perturbed_orszag_tang(nx, ny, u0=0.08, b0=0.08)).step(2)
    x0 = L.save_state()
    stride = L.lattice_bytes + 512
    full = torch.zeros(max(n, 1), stride, dtype=torch.uint8, device="cuda")
    L.step_store(x0, full, n)
    m = (n - 1) // 2
    half = torch.zeros(max(n // 2, 1), stride, dtype=torch.uint8, device="cuda")
    L.step_store_pairs(x0, half, n // 2)
    for k in range(n // 2):
        assert torch.equal(half[k, :L.lattice_bytes], full[2 * k + 1, :L.lattice_bytes]), k
    states = [x0] + [full[t - 1] for t in range(1, n)]
    lam_a, tmp_a, acc_a = L.new_adj_buffer(), L.new_adj_buffer(), L.new_adj_acc()
    L.adj_seed_energy(full[n - 1], lam_a)
    lam_b, tmp_b, acc_b = L.new_adj_buffer(), L.new_adj_buffer(), L.new_adj_acc()
    lam_b.copy_(lam_a)
    L.adj_sweep_pairs(x0, half[:max(m, 1)], n, lam_a, tmp_a, acc_a)
    for t in reversed(range(n)):
        L.adj_step(states[t], lam_b, tmp_b, acc_b)
        lam_b, tmp_b = tmp_b, lam_b
    assert torch.equal(L.adj_view(lam_a), L.adj_view(lam_b))
    close(L.adj_acc_total(acc_a), L.adj_acc_total(acc_b))


@pytest.mark.parametrize("n", [5, 6])
def test_full_store_sweep_takes_pairs_where_they_pay(lb, n):
    """At 1024^2 lbmhd_adj_sweep takes the reverse steps in pairs by itself
    (reading the even states of the full store): the same lam_0 as single
    reverse steps."""
    nx = ny = 1024
    print(f"\nadj full-store sweep 1024^2 n={n}", flush=True)
    cfg = lb.LBMHDConfig(nx=nx, ny=ny, nu=1e-4, eta=1e-4, les=1, cs=0.1)
    L = lb.Lattice(cfg)
    L.init_fields(*perturbed_orszag_tang(nx, ny, u0=0.08, b0=0.08)).step(2)
    x0 = L.save_state()
    full = torch.zeros(n, L.lattice_bytes, dtype=torch.uint8, device="cuda")
    L.step_store(x0, full, n)
    states = [x0] + [full[t - 1] for t in range(1, n)]
    lam_a, tmp_a, acc_a = L.new_adj_buffer(), L.new_adj_buffer(), L.new_adj_acc()
    L.adj_seed_energy(full[n - 1], lam_a)
    lam_b, tmp_b, acc_b = L.new_adj_buffer(), L.new_adj_buffer(), L.new_adj_acc()
    lam_b.copy_(lam_a)
    L.adj_sweep(x0, full, n, lam_a, tmp_a, acc_a)
    for t in reversed(range(n)):
        L.adj_step(states[t], lam_b, tmp_b, acc_b)
        lam_b, tmp_b = tmp_b, lam_b
    assert torch.equal(L.adj_view(lam_a), L.adj_view(lam_b))
    close(L.adj_acc_total(acc_a), L.adj_acc_total(acc_b))
    del L, full, states
    torch.cuda.empty_cache()


def test_pairs_refused_for_the_kinetic_closure(lb):
    import ctypes
    from paper_1607_08675_amd import _capi as C
    L = lb.Lattice(lb.LBMHDConfig(nx=16, ny=8, les=2))
    x0 = L.save_state()
    lam, lam2, acc = L.new_adj_buffer(), L.new_adj_buffer(), L.new_adj_acc()
    p = ctypes.c_void_p
    assert L._L.lbmhd_adj_step2(L._h, p(x0.data_ptr()), p(lam.data_ptr()), p(lam2.data_ptr()),
                                p(acc.data_ptr())) == C.LBMHD_ERR_UNSUPPORTED
    assert L._L.lbmhd_adj_sweep_pairs(L._h, p(x0.data_ptr()), p(0), L.lattice_bytes, 2,
                                      p(lam.data_ptr()), p(lam2.data_ptr()),
                                      p(acc.data_ptr())) == C.LBMHD_ERR_UNSUPPORTED
    torch.cuda.synchronize()
