"""What the FP64 oracle fixes about the reachable accuracy of the GPU runs.

Two GPU parity tests use bounds other than the relative-L2 figures asked of
them: FP16 storage on 256^2 decaying turbulence (nu = eta = 1e-6, LES) is held
to 1.5e-3 at step 100 and 1.2e-2 at step 1000, not 1e-3 at step 1000
(``test_gpu_forward.py::test_fp16_turbulence_256``), and the FP32 256^2
Orszag-Tang run at the 4096^2 production parameters (nu = eta = 1e-5) is
compared pointwise at step 300 and through its energies at step 1000
(``test_gpu_forward.py::test_orszag_tang_256_low_viscosity``).  The pins here
show, with the oracle alone, that those targets are out of reach for any
implementation that rounds differently from the oracle:

* FP16 storage: the oracle stepped one update at a time with its state rounded
  between updates exactly as the GPU stores it, half(float32(f - w) * 2^10)
  for every population (w = 0 for g), departs from the unrounded oracle by
  more than 1e-3 by step 1000.  The rounding sits on the test side; the
  oracle itself is unchanged.  Rounding the post-stream state is rounding the
  post-collision state moved by a permutation, so this is the GPU's storage.
* The low-viscosity Orszag-Tang flow amplifies perturbations: a relative
  1e-9 white-noise perturbation of u grows beyond 1e-5 by step 1000, while it
  is still below 1e-8 at step 300, where the GPU run is compared pointwise.

The 1024^2 versions (configuration of the FP16 accuracy statement: 1024^2
decaying turbulence, nu = eta = 1e-6, 1000 steps) take about ten minutes with
eight threads and run only with LBMHD_SLOW_PINS=1.
"""
import os

import numpy as np
import pytest

from lbmhd_inputs import decaying_turbulence, orszag_tang

# rest-state populations (D2Q9 weights; g has rest state 0): the offsets the
# GPU subtracts before encoding
W19 = np.concatenate([[4 / 9] + [1 / 9] * 4 + [1 / 36] * 4, np.zeros(10)])[:, None, None]

slow = pytest.mark.skipif(os.environ.get("LBMHD_SLOW_PINS") != "1",
                          reason="1024^2 oracle pins take ~10 min; set LBMHD_SLOW_PINS=1")


def fp16_storage(state):
    """The state as FP16 deviation storage holds it: RNE to half of the FP32
    deviation scaled by 2^10, decoded back exactly."""
    h = ((state - W19).astype(np.float32) * np.float32(1024.0)).astype(np.float16)
    return W19 + h.astype(np.float64) / 1024.0


def rel_l2(a, b, keys):
    x = np.stack([a[k] for k in keys])
    y = np.stack([b[k] for k in keys])
    return float(np.linalg.norm(x - y) / np.linalg.norm(y))


def fp16_departure(orc, n, checkpoints):
    """rel-L2 of u and B between the FP16-stored and the plain oracle run of
    n^2 decaying turbulence (nu = eta = 1e-6, LES C_S = 0.1) at each checkpoint."""
    op = orc.Params(n, n, nu=1e-6, eta=1e-6, les=True, cs=0.1)
    x0 = orc.init(op, *decaying_turbulence(n, n))
    ref, q, done, out = x0, fp16_storage(x0), 0, {}
    for target in checkpoints:
        ref = orc.run(op, ref, target - done)
        for _ in range(target - done):
            q = fp16_storage(orc.run(op, q, 1))
        done = target
        a, b = orc.macro(op, q), orc.macro(op, ref)
        out[target] = (rel_l2(a, b, ("ux", "uy")), rel_l2(a, b, ("bx", "by")))
    return out


def perturbation_growth(orc, n, gen, nu, checkpoints, rel=1e-9, seed=9):
    """rel-L2 of u and B between the oracle run from the fields of `gen` and
    the run whose u carries a relative white-noise perturbation `rel`."""
    op = orc.Params(n, n, nu=nu, eta=nu, les=True, cs=0.1)
    f = list(gen(n, n))
    g = list(f)
    rng = np.random.default_rng(seed)
    for k in (1, 2):
        g[k] = f[k] * (1.0 + rel * rng.standard_normal(f[k].shape))
    a, b, done, out = orc.init(op, *f), orc.init(op, *g), 0, {}
    for target in checkpoints:
        a = orc.run(op, a, target - done)
        b = orc.run(op, b, target - done)
        done = target
        ma, mb = orc.macro(op, a), orc.macro(op, b)
        out[target] = (rel_l2(mb, ma, ("ux", "uy")), rel_l2(mb, ma, ("bx", "by")))
    return out


def test_fp16_storage_rounding_alone_departs_beyond_1e3_at_256(orc):
    """FP16 storage with exact arithmetic otherwise: 8.4e-4 (u) after 100
    steps and 7.4e-3 after 1000 (measured), so the 1e-3-after-1000-steps
    target cannot be met by this storage; the GPU's FP16 run measures 8.4e-4
    and 7.7e-3 and is bounded at 1.5e-3 and 1.2e-2."""
    e = fp16_departure(orc, 256, (100, 1000))
    (u100, b100), (u1000, b1000) = e[100], e[1000]
    assert 5e-4 < u100 < 1.2e-3 and 5e-4 < b100 < 1.2e-3, e
    assert 4e-3 < u1000 < 1e-2 and 4e-3 < b1000 < 1e-2, e
    # the GPU bounds are less than twice the departure of the storage alone
    assert 1.5e-3 < 2.0 * u100 and 1.2e-2 < 2.0 * u1000


def test_orszag_tang_low_viscosity_amplifies_perturbations_at_256(orc):
    """256^2 Orszag-Tang at nu = eta = 1e-5: a 1e-9 perturbation of u is
    damped at first (2.6e-10 at step 100, 4.6e-10 at 300) and then grows
    exponentially (1.7e-6 at step 800, 4.2e-5 at 1000): pointwise parity of
    two runs whose rounding differs holds at step 300 and fails at step 1000
    for any implementation but the oracle's own."""
    e = perturbation_growth(orc, 256, orszag_tang, 1e-5, (300, 1000))
    assert e[300][0] < 1e-8 and e[300][1] < 1e-8, e
    assert e[1000][0] > 1e-5 and e[1000][1] > 1e-5, e


@slow
def test_turbulence_1024_amplifies_perturbations(orc):
    """1024^2 decaying turbulence at nu = eta = 1e-6 amplifies perturbations:
    a 1e-9 perturbation of u is damped to 2.5e-10 by step 100 and then grows
    to 1.3e-7 at step 500 and 1.1e-6 at step 1000 (measured), a factor of
    4500 in 900 steps; storage rounding, injected at every step, is
    amplified likewise."""
    e = perturbation_growth(orc, 1024, decaying_turbulence, 1e-6, (100, 1000))
    assert e[100][0] < 1e-9, e
    assert e[1000][0] > 1000 * e[100][0] and e[1000][0] > 1e-7, e


@slow
def test_fp16_storage_rounding_alone_at_1024(orc):
    """FP16 storage with exact arithmetic on 1024^2 decaying turbulence: the
    departure at step 1000 is far above 1e-3 (the GPU measures 6.7e-2)."""
    e = fp16_departure(orc, 1024, (100, 1000))
    assert e[100][0] < 2e-3, e
    assert e[1000][0] > 1e-2, e
