"""GPU parity of the forward path against the FP64 oracle (through the C ABI).

The GPU stores post-collision populations: after n steps it holds
C((S C)^(n-1) S x0) where the oracle's paper-ordered update is (S C)^n x0
(S: streaming, C: collision).  Population-level comparisons therefore apply
one extra oracle collision; macroscopic fields (rho, u, B are collision
invariants) compare directly.

Tolerances: FP32 storage and arithmetic against FP64 -- populations within
5e-7 after one step and 2e-6 after ten (deviations are O(0.1), FP32 ulp
~1e-8, ~50 dependent operations); relative L2 of u and B within 1e-5 after
1000 steps where the flow does not amplify rounding (see the 256^2 case).  FP16 storage: one step from an FP16-representable state
within one half-precision rounding of the output (|dev| * 2^-11, dev =
deviation of the population, plus 1e-6); trajectories within the bounds of
the FP16 noise model stated at test_fp16_turbulence_256.
"""
import numpy as np
import pytest
import torch

from lbmhd_inputs import (decaying_turbulence, orszag_tang, random_planes)
from state_words import stored_words

pytestmark = pytest.mark.gpu

# D2Q9 weights (mean populations of the rest state) used to draw random
# near-equilibrium test states; g is drawn around zero.
W9 = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)
W19 = np.concatenate([W9, np.zeros(10)])


@pytest.fixture(scope="module")
def lb():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1607_08675_amd import lattice
    return lattice


def random_state(nx, ny, seed, famp=0.02, gamp=0.01):
    scale = np.concatenate([W9 * famp, np.full(10, gamp)])
    return random_planes(19, nx, ny, seed, W19, scale)


def make(lb, orc, nx, ny, storage="fp32", **kw):
    cfg = lb.LBMHDConfig(nx=nx, ny=ny, storage=storage, **kw)
    op = orc.Params(nx, ny, nu=cfg.nu, eta=cfg.eta, s5=cfg.s5, s6=cfg.s5, s7=cfg.s7, s8=cfg.s8,
                    les=cfg.les, cs=cfg.cs, delta=cfg.delta)
    return lb.Lattice(cfg), op


def rel_l2(a, b):
    return float(np.sqrt(np.sum((a - b) ** 2)) / np.sqrt(np.sum(b ** 2)))


def uv_err(gm, om):
    g = {k: v.cpu().numpy() for k, v in gm.items()}
    eu = rel_l2(np.stack([g["ux"], g["uy"]]), np.stack([om["ux"], om["uy"]]))
    eb = rel_l2(np.stack([g["bx"], g["by"]]), np.stack([om["bx"], om["by"]]))
    return eu, eb


def _oracle_gpu_state(orc, op, x0, n):
    # (C S)^n x0 = C (S C)^(n-1) S x0
    st = orc.stream(op, x0)
    st = orc.run(op, st, n - 1)
    return orc.collide(op, st)


# ------------------------------------------------------------------- init
@pytest.mark.parametrize("storage,tol", [("fp32", 1e-8), ("fp16", 3e-5)])
def test_init_matches_oracle_equilibrium(lb, orc, storage, tol):
    nx, ny = 100, 36
    L, op = make(lb, orc, nx, ny, storage)
    fields = orszag_tang(nx, ny)
    L.init_fields(*fields)
    got = L.populations().cpu().numpy()
    np.testing.assert_allclose(got, orc.init(op, *fields), rtol=0, atol=tol)
    m = L.macro()
    for k, f in zip(("rho", "ux", "uy", "bx", "by"), fields):
        np.testing.assert_allclose(m[k].cpu().numpy(), f, rtol=0, atol=10 * tol)
    assert L.step_count == 0


# --------------------------------------------------------------- one step
SIZES = [(8, 8), (100, 36), (64, 64), (300, 5), (2, 2), (257, 3)]


@pytest.mark.parametrize("les", [False, True])
@pytest.mark.parametrize("nx,ny", SIZES)
def test_one_step_fp32(lb, orc, nx, ny, les):
    L, op = make(lb, orc, nx, ny, "fp32", nu=0.01, eta=0.02, s5=1.2, s7=1.5, s8=0.8, les=les,
                 cs=0.15)
    x0 = random_state(nx, ny, seed=nx * 1000 + ny)
    L.set_populations(x0)
    L.step(1)
    got = L.populations().cpu().numpy()
    want = orc.collide(op, orc.stream(op, x0))
    err = np.abs(got - want).max()
    assert err < 5e-7, err
    assert L.step_count == 1


@pytest.mark.parametrize("les", [False, True])
def test_ten_steps_fp32(lb, orc, les):
    nx, ny = 100, 36
    L, op = make(lb, orc, nx, ny, "fp32", nu=0.005, eta=0.01, s5=1.1, s7=1.3, s8=1.2, les=les,
                 cs=0.2)
    x0 = random_state(nx, ny, seed=7)
    L.set_populations(x0).step(10)
    got = L.populations().cpu().numpy()
    want = _oracle_gpu_state(orc, op, x0, 10)
    err = np.abs(got - want).max()
    assert err < 2e-6, err


def _fp16_representable(x0):
    dev = x0 - W19[:, None, None]
    h = (dev.astype(np.float32) * np.float32(1024)).astype(np.float16)
    return W19[:, None, None] + h.astype(np.float64) / 1024.0


@pytest.mark.parametrize("les", [False, True])
@pytest.mark.parametrize("nx,ny", [(8, 8), (100, 36), (300, 5), (257, 3), (2, 2), (1030, 4)])
def test_one_step_fp16(lb, orc, nx, ny, les):
    L, op = make(lb, orc, nx, ny, "fp16", nu=0.01, eta=0.02, les=les, cs=0.15)
    x0 = _fp16_representable(random_state(nx, ny, seed=3 + nx))
    L.set_populations(x0)
    np.testing.assert_array_equal(L.populations().cpu().numpy(), x0)  # exact encode
    L.step(1)
    got = L.populations().cpu().numpy()
    want = orc.collide(op, orc.stream(op, x0))
    dev = np.abs(want - W19[:, None, None])
    assert np.all(np.abs(got - want) <= dev * 2.0 ** -11 + 1e-6)


def test_fp16_codec_is_round_to_nearest_even(lb, orc):
    """Stored half = RNE(float32(f - w) * 2^10), compared bit for bit with
    numpy's IEEE conversion, including subnormals, ties and overflow to inf."""
    nx, ny = 64, 2
    L, _ = make(lb, orc, nx, ny, "fp16", les=False)
    rng = np.random.default_rng(0)
    dev = np.concatenate([
        rng.standard_normal(19 * nx * ny // 2) * 0.05,
        rng.standard_normal(19 * nx * ny // 2) * 1e-7,     # subnormal halves
    ]).reshape(19, ny, nx)
    # exact ties of the half grid (g planes: w = 0, so f - w is exact): normal
    # ties 1 + 2^-11, 1 + 3 * 2^-11 and subnormal ties k * 2^-25, all / 2^10
    ties = np.array([1 + 2.0 ** -11, 1 + 3 * 2.0 ** -11, -(1 + 2.0 ** -11), 2.0 ** -25,
                     3 * 2.0 ** -25, 5 * 2.0 ** -25, -(3 * 2.0 ** -25), 7 * 2.0 ** -25])
    dev[9, 0, :8] = ties / 1024.0
    dev[10, 0, :2] = [70.0, -70.0]                                       # overflow -> +-inf
    x = W19[:, None, None] + dev
    L.set_populations(x)
    got = L.state_view().cpu().numpy()
    want = (np.float32(1024) * (x - W19[:, None, None]).astype(np.float32)).astype(np.float16)
    np.testing.assert_array_equal(got.view(np.uint16), want.view(np.uint16))


# ------------------------------------------------------------ trajectories
def test_orszag_tang_64_config(lb, orc):
    """64x64 Orszag-Tang, nu = eta = 0.01, LES C_S = 0.1: relative L2 of u and
    B within 1e-5 at steps 100, 500 and 1000."""
    n = 64
    L, op = make(lb, orc, n, n, "fp32", nu=0.01, eta=0.01, les=True, cs=0.1)
    fields = orszag_tang(n, n)
    L.init_fields(*fields)
    st = orc.init(op, *fields)
    done = 0
    for target in (100, 500, 1000):
        L.step(target - done)
        st = orc.run(op, st, target - done)
        done = target
        eu, eb = uv_err(L.macro(), orc.macro(op, st))
        assert eu < 1e-5 and eb < 1e-5, (target, eu, eb)


def test_orszag_tang_256_low_viscosity(lb, orc):
    """256x256 Orszag-Tang with the 4096^2 production parameters (nu = eta =
    1e-5, LES C_S = 0.1).  This flow amplifies any rounding difference
    exponentially after ~400 steps (two FP64 runs whose rounding differs
    separate from 1e-14 to 1e-11 between steps 100 and 700), so pointwise
    parity is checked at step 300 (<= 1e-5) and the global energies and
    cross helicity at step 1000 (<= 2e-3, the decorrelated small scales carry
    little energy).  The oracle alone fixes this: a 1e-9 perturbation of u is
    below 1e-8 at step 300 and above 1e-5 at step 1000
    (test_oracle_precision.py::test_orszag_tang_low_viscosity_amplifies_perturbations_at_256)."""
    n = 256
    L, op = make(lb, orc, n, n, "fp32", nu=1e-5, eta=1e-5, les=True, cs=0.1)
    fields = orszag_tang(n, n)
    L.init_fields(*fields).step(300)
    st = orc.run(op, orc.init(op, *fields), 300)
    eu, eb = uv_err(L.macro(), orc.macro(op, st))
    assert eu < 1e-5 and eb < 1e-5, (eu, eb)
    L.step(700)
    st = orc.run(op, st, 700)
    g, o = L.diag(), orc.diag(op, st)
    for key in ("e_kin", "e_mag", "cross_helicity"):
        assert abs(g[key] - o[key]) < 2e-3 * abs(o[key]), (key, g[key], o[key])
    assert abs(g["mass"] - o["mass"]) < 1e-6 * o["mass"]


@pytest.fixture(scope="module")
def turb256(orc):
    """Oracle macros of 256^2 decaying turbulence (nu = eta = 1e-6, LES) at
    steps 100 and 1000."""
    n = 256
    op = orc.Params(n, n, nu=1e-6, eta=1e-6, les=True, cs=0.1)
    fields = decaying_turbulence(n, n)
    st = orc.run(op, orc.init(op, *fields), 100)
    m100 = orc.macro(op, st)
    st = orc.run(op, st, 900)
    return fields, {100: m100, 1000: orc.macro(op, st)}


def test_fp32_turbulence_256(lb, orc, turb256):
    """FP32: relative L2 of u and B within 1e-5 after 1000 steps."""
    fields, ref = turb256
    L, _ = make(lb, orc, 256, 256, "fp32", nu=1e-6, eta=1e-6, les=True, cs=0.1)
    L.init_fields(*fields)
    for n_done, target in ((0, 100), (100, 1000)):
        L.step(target - n_done)
        eu, eb = uv_err(L.macro(), ref[target])
        assert eu < 1e-5 and eb < 1e-5, (target, eu, eb)


def test_fp16_turbulence_256(lb, orc, turb256):
    """FP16 deviation storage.  Each stored deviation carries an RNE error of
    up to 2^-12 of itself, and the first-order part 3 w_i c_i . u of the
    deviations dominates, so the update accumulates small-scale noise: a
    the oracle stepped with its state rounded to FP16 storage between steps
    (exact arithmetic otherwise) departs by 8.4e-4 (u) after 100 steps and
    7.4e-3 after 1000 (test_oracle_precision.py::
    test_fp16_storage_rounding_alone_departs_beyond_1e3_at_256), so no FP16
    run meets 1e-3 at step 1000.  Bounds: 1.5e-3 and 1.2e-2."""
    fields, ref = turb256
    L, _ = make(lb, orc, 256, 256, "fp16", nu=1e-6, eta=1e-6, les=True, cs=0.1)
    L.init_fields(*fields)
    for n_done, target, tol in ((0, 100, 1.5e-3), (100, 1000, 1.2e-2)):
        L.step(target - n_done)
        eu, eb = uv_err(L.macro(), ref[target])
        print(f"fp16 turbulence step {target}: rel-L2 u {eu:.3e}, B {eb:.3e}")
        assert eu < tol and eb < tol, (target, eu, eb)


# ---------------------------------------------------- full-size, sampled
def _patch(fields, cx, cy, r):
    ny, nx = fields[0].shape
    ys = (np.arange(cy - r, cy + r + 1)) % ny
    xs = (np.arange(cx - r, cx + r + 1)) % nx
    return [f[np.ix_(ys, xs)] for f in fields]


@pytest.mark.parametrize("storage,n,gen,nu,tol", [
    ("fp32", 4096, "ot", 1e-5, 1e-6),
    ("fp16", 8192, "turb", 1e-6, 1e-4),
])
def test_full_size_sampled_sites(lb, orc, storage, n, gen, nu, tol):
    """Production sizes and launch configuration: k = 3 steps on the GPU, then
    the oracle recomputes sampled sites one by one on (2k+3)^2 patches (after k
    steps a site depends only on sites within distance k)."""
    k, r = 3, 4
    fields = orszag_tang(n, n) if gen == "ot" else decaying_turbulence(n, n)
    L, _ = make(lb, orc, n, n, storage, nu=nu, eta=nu, les=True, cs=0.1)
    L.init_fields(*fields).step(k)
    pops = L.populations()
    rng = np.random.default_rng(5)
    sites = [(0, 0), (n - 1, n - 1), (0, n - 1), (n - 1, 0), (n // 2, 1)]
    sites += [tuple(int(v) for v in rng.integers(0, n, 2)) for _ in range(27)]
    op = orc.Params(2 * r + 1, 2 * r + 1, nu=nu, eta=nu, les=True, cs=0.1)
    for (x, y) in sites:
        st = orc.init(op, *_patch(fields, x, y, r))
        want = _oracle_gpu_state(orc, op, st, k)[:, r, r]
        got = pops[:, y, x].cpu().numpy()
        err = np.abs(got - want).max()
        assert err < tol, (x, y, err)
    del pops, L
    torch.cuda.empty_cache()


# ------------------------------------------------------- invariants & state
def test_conservation_fp32(lb, orc):
    n = 128
    L, op = make(lb, orc, n, n, "fp32", nu=1e-4, eta=1e-4, les=True, cs=0.1)
    L.init_fields(*decaying_turbulence(n, n))
    d0 = L.diag()
    L.step(1000)
    d1 = L.diag()
    assert abs(d1["mass"] - d0["mass"]) < 1e-6 * d0["mass"]
    for key in ("mom_x", "mom_y", "flux_x", "flux_y"):
        assert abs(d1[key] - d0[key]) < 1e-7 * n * n, key
    assert d1["nonfinite"] == 0 and d1["step"] == 1000


def test_diag_matches_oracle(lb, orc):
    nx, ny = 100, 36
    L, op = make(lb, orc, nx, ny, "fp32", les=True)
    x0 = random_state(nx, ny, seed=11)
    L.set_populations(x0)
    g = L.diag()
    o = orc.diag(op, x0)
    for key in ("mass", "mom_x", "mom_y", "flux_x", "flux_y", "e_kin", "e_mag",
                "cross_helicity", "max_abs_divB", "enstrophy", "current_sq", "max_u"):
        assert abs(g[key] - o[key]) <= 1e-7 * max(abs(o[key]), 1e-3), (key, g[key], o[key])
    assert g["nonfinite"] == 0


def test_diag_counts_nonfinite(lb, orc):
    nx, ny = 16, 8
    L, _ = make(lb, orc, nx, ny, "fp32")
    x0 = random_state(nx, ny, seed=1)
    x0[3, 2, 5] = np.nan
    x0[12, 7, 0] = np.inf
    L.set_populations(x0)
    assert L.diag()["nonfinite"] == 2
    from paper_1607_08675_amd._capi import LbmhdError
    with pytest.raises(LbmhdError):
        L.diag(raise_nonfinite=True)


def test_checkpoint_resume_bit_exact(lb, orc):
    n = 96
    L, _ = make(lb, orc, n, n, "fp32", nu=1e-4, eta=1e-4, les=True)
    L.init_fields(*orszag_tang(n, n)).step(50)
    ck = L.save_state().clone()
    L.step(50)
    ref = stored_words(L).clone()
    L.load_state(ck, 50).step(50)
    assert L.step_count == 100
    assert torch.equal(stored_words(L), ref)


def test_les_off_matches_zero_constant_bitwise(lb, orc):
    n = 64
    L0, _ = make(lb, orc, n, n, "fp32", les=False)
    L1, _ = make(lb, orc, n, n, "fp32", les=True, cs=0.0)
    f = orszag_tang(n, n)
    L0.init_fields(*f).step(20)
    L1.init_fields(*f).step(20)
    assert torch.equal(stored_words(L0), stored_words(L1))
