"""Box filter, mismatch functional, its adjoint seed and the C_S fit (GPU).

Reference values: the oracle's macroscopic fields of the same stored state,
box-averaged and differenced in numpy (plain definitions); derivatives against
central differences of the oracle.  The fit is checked as a twin experiment:
targets made by the same coarse model at a known C_S must pull C_S back to it.
"""
import numpy as np
import pytest
import torch

from adjoint_layout import unstreamed
from lbmhd_inputs import decaying_turbulence, orszag_tang, random_fields, random_planes

pytestmark = pytest.mark.gpu

W9 = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)
W19 = np.concatenate([W9, np.zeros(10)])


@pytest.fixture(scope="module")
def lb():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1607_08675_amd import lattice
    return lattice


def stored32(x):
    return W19[:, None, None] + (x - W19[:, None, None]).astype(np.float32).astype(np.float64)


def random_state(nx, ny, seed):
    scale = np.concatenate([W9 * 0.02, np.full(10, 0.01)])
    return random_planes(19, nx, ny, seed, W19, scale)


def _mismatch(m, t):
    return sum(float(np.sum((m[k] - tk) ** 2)) for k, tk in zip(("ux", "uy", "bx", "by"), t))


@pytest.mark.parametrize("w", [1, 2, 4])
def test_macro_box(lb, orc, w):
    nx, ny = 32, 16
    L = lb.Lattice(lb.LBMHDConfig(nx=nx, ny=ny))
    x = random_state(nx, ny, 3)
    L.set_populations(x)
    got = L.macro_box(w)
    m = orc.macro(orc.Params(nx, ny), stored32(x))
    for k in ("rho", "ux", "uy", "bx", "by"):
        want = m[k].reshape(ny // w, w, nx // w, w).mean(axis=(1, 3))
        np.testing.assert_allclose(got[k].cpu().numpy(), want, rtol=0, atol=1e-14)


def test_mismatch_value_and_seed(lb, orc):
    nx, ny = 20, 12
    L = lb.Lattice(lb.LBMHDConfig(nx=nx, ny=ny))
    x = stored32(random_state(nx, ny, 5))
    L.set_populations(x)
    t = random_fields(nx, ny, 9)[1:]
    op = orc.Params(nx, ny)
    want = _mismatch(orc.macro(op, x), t)
    assert abs(L.mismatch(t) - want) <= 1e-12 * want
    lam = L.new_adj_buffer()
    L.adj_seed_mismatch(L.save_state(), t, 0.5, lam)
    got = unstreamed(L.adj_view(lam).double().cpu().numpy())
    rng = np.random.default_rng(2)
    eps = 1e-6
    for _ in range(4):
        v = rng.standard_normal(x.shape)
        fd = (_mismatch(orc.macro(op, x + eps * v), t) - _mismatch(orc.macro(op, x - eps * v), t)) / (2 * eps)
        assert abs(0.5 * fd - np.sum(got * v)) <= 1e-6 * abs(fd) + 1e-6


def test_mismatch_gradient_wrt_cs_matches_oracle_fd(lb, orc):
    """dL/dC_Sv and dL/dC_Sb through 30 steps (checkpoint every 8) against
    central differences of the FP64 oracle in each constant; targets are
    unrelated synthetic fields."""
    from paper_1607_08675_amd.adjoint import Checkpointed
    n, steps, cs, csb = 24, 30, 0.15, 0.1
    fields = orszag_tang(n, n, u0=0.1, b0=0.1)
    targets = decaying_turbulence(n, n)[1:]
    cfg = lb.LBMHDConfig(nx=n, ny=n, nu=1e-3, eta=1e-3, les=True, cs=cs, cs_b=csb)
    run = Checkpointed(lb.Lattice(cfg), 8)
    Lg = run.forward(fields, steps, targets=targets)
    g = run.backward()
    def oracle_L(c, cb):
        op = orc.Params(n, n, nu=1e-3, eta=1e-3, les=True, cs=c, csb=cb)
        return _mismatch(orc.macro(op, orc.run(op, orc.init(op, *fields), steps)), targets)
    assert abs(Lg - oracle_L(cs, csb)) <= 1e-6 * abs(Lg)
    eps = 1e-5
    fdv = (oracle_L(cs + eps, csb) - oracle_L(cs - eps, csb)) / (2 * eps)
    fdb = (oracle_L(cs, csb + eps) - oracle_L(cs, csb - eps)) / (2 * eps)
    assert abs(g[4] - fdv) <= 1e-3 * abs(fdv), (g[4], fdv)
    assert abs(g[5] - fdb) <= 1e-3 * abs(fdb), (g[5], fdb)


@pytest.mark.parametrize("storage", ["fp32", "fp16"])
def test_fit_recovers_known_cs(lb, orc, storage):
    """Twin experiment: targets from the coarse model itself at C_S = 0.2;
    the adjoint-driven fit started at C_S = 0.05 must return to 0.2."""
    from paper_1607_08675_amd.fit import fit_cs
    n, steps = 32, 60
    fields = decaying_turbulence(n, n, u_rms=0.08, b_rms=0.08)
    cfg = lb.LBMHDConfig(nx=n, ny=n, nu=1e-4, eta=1e-4, les=True, cs=0.2, storage=storage)
    L = lb.Lattice(cfg)
    L.init_fields(*fields).step(steps)
    m = L.macro()
    targets = (m["ux"], m["uy"], m["bx"], m["by"])
    start = lb.LBMHDConfig(**{**cfg.__dict__, "cs": 0.05})
    res = fit_cs(fields, targets, start, steps, iters=14, every=16)
    assert res.loss[-1] < 1e-2 * res.loss[0], res.loss
    assert abs(res.cs[-1] - 0.2) < 0.01 * (5 if storage == "fp16" else 1), res.cs


def test_joint_fit_recovers_both_constants(lb, orc):
    """Twin experiment with C_Sv = 0.2, C_Sb = 0.1: the joint fit started at
    0.05 for both returns to the pair."""
    from paper_1607_08675_amd.fit import fit_cs
    n, steps = 32, 60
    fields = decaying_turbulence(n, n, u_rms=0.08, b_rms=0.08)
    cfg = lb.LBMHDConfig(nx=n, ny=n, nu=1e-4, eta=1e-4, les=True, cs=0.2, cs_b=0.1)
    L = lb.Lattice(cfg)
    L.init_fields(*fields).step(steps)
    m = L.macro()
    targets = (m["ux"], m["uy"], m["bx"], m["by"])
    start = lb.LBMHDConfig(**{**cfg.__dict__, "cs": 0.05, "cs_b": 0.05})
    res = fit_cs(fields, targets, start, steps, iters=24, every=16, joint=True)
    assert res.loss[-1] < 1e-2 * res.loss[0], res.loss
    assert abs(res.cs[-1] - 0.2) < 0.02 and abs(res.cs_b[-1] - 0.1) < 0.01, (res.cs, res.cs_b)


def test_fit_with_kinetic_closure_recovers_cs(lb, orc):
    """Twin experiment with the Smagorinsky estimate on top of the kinetic
    closure (les = 3, Delta = 1): targets at C_S = 0.2, the fit started at 0.05
    returns to it through the two-pass kinetic reverse step."""
    from paper_1607_08675_amd.fit import fit_cs
    n, steps = 32, 60
    fields = decaying_turbulence(n, n, u_rms=0.08, b_rms=0.08)
    cfg = lb.LBMHDConfig(nx=n, ny=n, nu=1e-4, eta=1e-4, les=3, cs=0.2, delta=1.0)
    L = lb.Lattice(cfg)
    L.init_fields(*fields).step(steps)
    m = L.macro()
    targets = (m["ux"], m["uy"], m["bx"], m["by"])
    start = lb.LBMHDConfig(**{**cfg.__dict__, "cs": 0.05})
    res = fit_cs(fields, targets, start, steps, iters=14, every=16)
    assert res.loss[-1] < 1e-2 * res.loss[0], res.loss
    assert abs(res.cs[-1] - 0.2) < 0.01, res.cs
