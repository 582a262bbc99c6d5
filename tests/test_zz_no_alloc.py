"""lbmhd_diag_noalloc against lbmhd_diag, through the C ABI.

The allocation-free variant runs the same diagnostics kernels with its block
partials and result slots in the library's static device array instead of the
bound workspace, so on the same state the two must agree bit for bit.  Two
calls in a row on one GPU, the second on a smaller lattice (fewer partials),
check that the shared array carries nothing from one call into the next; a
state holding non-finite populations checks the error path.
"""
import ctypes

import numpy as np
import pytest
import torch

from lbmhd_inputs import decaying_turbulence, orszag_tang

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lb():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1607_08675_amd import lattice
    return lattice


def both(L):
    from paper_1607_08675_amd._capi import Diag
    a, b = Diag(), Diag()
    ra = L._L.lbmhd_diag(L._h, ctypes.byref(a))
    rb = L._L.lbmhd_diag_noalloc(L._h, ctypes.byref(b))
    return (ra, a.as_dict()), (rb, b.as_dict())


def same(a, b):
    (ra, da), (rb, db) = a, b
    assert ra == rb, (ra, rb)
    for k in da:
        assert da[k] == db[k] or (np.isnan(da[k]) and np.isnan(db[k])), (k, da[k], db[k])


@pytest.mark.parametrize("storage", ["fp32", "fp16"])
def test_noalloc_diag_equals_diag_on_two_calls_in_a_row(lb, storage):
    big = lb.Lattice(lb.LBMHDConfig(nx=2048, ny=1536, nu=1e-4, eta=1e-4, les=True, cs=0.1,
                                    storage=storage))
    big.init_fields(*decaying_turbulence(2048, 1536)).step(7)
    r_big = both(big)
    same(*r_big)
    assert r_big[0][0] == 0 and r_big[0][1]["step"] == 7
    small = lb.Lattice(lb.LBMHDConfig(nx=100, ny=36, nu=0.01, eta=0.01, les=True, cs=0.1,
                                      storage=storage))
    small.init_fields(*orszag_tang(100, 36)).step(3)
    r_small = both(small)
    same(*r_small)
    assert r_small[0][1]["mass"] != r_big[0][1]["mass"]
    # the first lattice again after the small one
    same(*both(big))


def test_noalloc_diag_reports_nonfinite(lb):
    from paper_1607_08675_amd._capi import LBMHD_ERR_NONFINITE
    L = lb.Lattice(lb.LBMHDConfig(nx=64, ny=40, storage="fp32"))
    rng = np.random.default_rng(3)
    w = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4 + [0.0] * 10)
    x = w[:, None, None] + 1e-3 * rng.standard_normal((19, 40, 64))
    x[5, 7, 9] = np.inf
    x[12, 0, 63] = np.nan
    L.set_populations(x)
    a, b = both(L)
    same(a, b)
    assert a[0] == LBMHD_ERR_NONFINITE and a[1]["nonfinite"] == 2
