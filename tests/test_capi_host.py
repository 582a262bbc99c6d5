"""Host-only checks of the C ABI (no GPU work is launched).

The library loads, exports every function include/lbmhd.h declares, validates
parameters in lbmhd_create, reports sizes, and refuses device calls before
lbmhd_bind.
"""
import ctypes
import os
import re
import subprocess

import pytest

from conftest import ROOT


@pytest.fixture(scope="module")
def capi():
    from paper_1607_08675_amd import _capi
    if not os.path.exists(_capi.LIB_PATH):
        from paper_1607_08675_amd import build
        build.build()
    return _capi


def _header_functions(name="lbmhd.h", prefix="lbmhd_"):
    text = open(os.path.join(ROOT, "include", name)).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(" + prefix + r"[a-z_0-9]+)\s*\(", text)))


def test_every_declared_function_is_exported(capi):
    declared = _header_functions() + _header_functions("lbmhd3.h", "lbmhd3_")
    assert len(declared) >= 30
    assert set(declared) == set(capi.EXPORTS) | set(capi.EXPORTS3)
    out = subprocess.run(["nm", "-D", "--defined-only", capi.LIB_PATH], check=True,
                         capture_output=True, text=True).stdout
    exported = set(re.findall(r"\bT (lbmhd3?_\w+)", out))
    missing = set(declared) - exported
    assert not missing, missing
    L = capi.lib()
    for name in declared:
        assert hasattr(L, name)


def _params(capi, **kw):
    base = dict(nx=64, ny=48, nu=0.01, eta=0.02, s5=1.0, s6=1.0, s7=1.1, s8=0.9, les=1,
                cs=0.1, cs_b=0.1, delta=1.0, storage=capi.LBMHD_FP32, inplace=0,
                steps_per_pass=0)
    base.update(kw)
    return capi.Params(*[base[n] for n, _ in capi.Params._fields_])


def _create(capi, p):
    h = ctypes.c_void_p()
    rc = capi.lib().lbmhd_create(ctypes.byref(p), ctypes.byref(h))
    return rc, h


@pytest.mark.parametrize("bad", [
    dict(nx=1), dict(ny=0), dict(nu=0.0), dict(eta=-1.0), dict(nu=float("nan")),
    dict(s5=2.0), dict(s7=0.0), dict(s8=-0.5), dict(s5=1.1, s6=1.2), dict(les=5), dict(les=7), dict(les=-1),
    dict(cs=-0.1), dict(cs_b=-0.1), dict(cs_b=float("inf")), dict(delta=0.0),
    dict(inplace=2), dict(steps_per_pass=4), dict(steps_per_pass=-1), dict(inplace=1, les=2), dict(inplace=1, les=4), dict(inplace=1, les=6), dict(storage=7), dict(nx=70000, ny=70000),
])
def test_create_rejects_invalid_parameters(capi, bad):
    rc, h = _create(capi, _params(capi, **bad))
    assert rc == capi.LBMHD_ERR_INVALID_ARG
    assert not h.value


@pytest.mark.parametrize("les", [4, 6])
def test_create_refuses_crosshelicity_beyond_eta_one_quarter(capi, les):
    """The clip of the cross-helicity closure's magnetic relaxation time
    nears a double root of its cubic as tau_m0 = 3 eta + 1/2 nears 3/2; the
    library refuses the closure beyond tau_m0 = 5/4 and accepts it up to
    there (any nu)."""
    rc, h = _create(capi, _params(capi, les=les, eta=0.2501))
    assert rc == capi.LBMHD_ERR_UNSUPPORTED and not h.value
    rc, h = _create(capi, _params(capi, les=les, eta=0.25, nu=2.0))
    assert rc == 0
    assert capi.lib().lbmhd_destroy(h) == 0


def test_sizes_and_layout(capi):
    L = capi.lib()
    for storage, esize in ((capi.LBMHD_FP32, 4), (capi.LBMHD_FP16, 2)):
        rc, h = _create(capi, _params(capi, nx=100, ny=36, storage=storage))
        assert rc == 0
        s = [ctypes.c_size_t() for _ in range(4)]
        assert L.lbmhd_sizes(h, *[ctypes.byref(x) for x in s]) == 0
        lat, ws, adj, acc = (x.value for x in s)
        pitch = -(-100 * esize // 256) * 256 // esize   # rows padded to 256 bytes
        plane = 36 * pitch + 768 // esize                # and a 768-byte gap between planes
        assert lat == 19 * plane * esize
        assert adj == 19 * (36 * 128 + 192) * 4
        lay = [ctypes.c_int64() for _ in range(4)]
        assert L.lbmhd_layout(h, *[ctypes.byref(x) for x in lay]) == 0
        assert [x.value for x in lay] == [pitch, plane, 128, 36 * 128 + 192]
        assert L.lbmhd_layout(h, None, None, None, None) == 0
        assert L.lbmhd_layout(None, None, None, None, None) == capi.LBMHD_ERR_INVALID_ARG
        assert ws >= 16 * 8 and ws % 256 == 0   # reduction partials and results only
        assert acc % 256 == 0 and acc >= 2 * 8 * 36   # two slot arrays, >= 1 block per row
        assert L.lbmhd_destroy(h) == 0


@pytest.mark.parametrize("kw,want", [
    (dict(nx=4096, ny=4096), 3), (dict(nx=1024, ny=1024), 3), (dict(nx=512, ny=512), 1),
    (dict(nx=2048, ny=2048, storage=1), 2), (dict(nx=1024, ny=1024, storage=1), 1),
    (dict(nx=1023, ny=1024, storage=1), 2), (dict(nx=64, ny=48, steps_per_pass=2), 2),
    (dict(nx=4096, ny=4096, steps_per_pass=2), 2),
    (dict(nx=4096, ny=4096, steps_per_pass=1), 1), (dict(nx=4096, ny=4096, les=0), 3),
    (dict(nx=4096, ny=4096, les=2), 2), (dict(nx=4096, ny=4096, les=4), 2),
    (dict(nx=4096, ny=4096, les=4, cs=0.0, cs_b=0.0), 3), (dict(nx=512, ny=512, les=2), 1),
    (dict(nx=4096, ny=4096, les=6, storage=1), 1), (dict(nx=4096, ny=4096, les=3, steps_per_pass=1), 1),
    (dict(nx=4096, ny=4096, les=3), 2), (dict(nx=4096, ny=4096, les=6), 2),
    (dict(nx=4096, ny=4096, les=2, storage=1), 1), (dict(nx=4096, ny=4096, les=6, steps_per_pass=2), 2),
    (dict(nx=4096, ny=4096, inplace=1), 1), (dict(nx=64, ny=48, inplace=1, steps_per_pass=2), 1),
    (dict(nx=64, ny=48, steps_per_pass=3), 3), (dict(nx=64, ny=48, steps_per_pass=3, storage=1), 2),
    (dict(nx=64, ny=48, steps_per_pass=3, les=2), 2), (dict(nx=64, ny=48, steps_per_pass=2, les=4), 2),
])
def test_steps_per_pass_selection(capi, kw, want):
    """Several steps per pass only for two lattices: for the closures without
    neighbour terms automatically from 512 tiles of 8 rows (256 FP32 or
    FP16-odd-nx columns, 512 FP16 columns) up, triples for FP32 and pairs for
    FP16, triples with 3 for FP32 (pairs for FP16), pairs with 2; for the
    closures that read the neighbours' moments pairs with 2 or 3, and
    automatically from 512 tiles of 256 columns by 8 rows with FP32 storage
    (pairs measured no faster with FP16 storage); single steps with 1.  The
    cross-helicity
    closure at C_S = 0 is the plain update and takes its kernels."""
    rc, h = _create(capi, _params(capi, **kw))
    assert rc == 0
    try:
        v = ctypes.c_int32()
        assert capi.lib().lbmhd_steps_per_pass(h, ctypes.byref(v)) == 0
        assert v.value == want
        assert capi.lib().lbmhd_steps_per_pass(h, None) == capi.LBMHD_ERR_INVALID_ARG
    finally:
        capi.lib().lbmhd_destroy(h)


def test_calls_before_bind_are_refused(capi):
    L = capi.lib()
    rc, h = _create(capi, _params(capi))
    assert rc == 0
    assert L.lbmhd_step(h, 1) == capi.LBMHD_ERR_NOT_BOUND
    assert b"bind" in L.lbmhd_last_error(h)
    d = capi.Diag()
    assert L.lbmhd_diag(h, ctypes.byref(d)) == capi.LBMHD_ERR_NOT_BOUND
    assert L.lbmhd_run(h, 10, 5, None, ctypes.byref(d), 2) == capi.LBMHD_ERR_NOT_BOUND
    assert L.lbmhd_bind(h, None, 0, None, 0, None, 0, None) == capi.LBMHD_ERR_INVALID_ARG
    step = ctypes.c_int64(-1)
    assert L.lbmhd_get_step(h, ctypes.byref(step)) == 0 and step.value == 0
    ptr = ctypes.c_void_p()
    assert L.lbmhd_current_state(h, ctypes.byref(ptr)) == capi.LBMHD_ERR_NOT_BOUND
    assert L.lbmhd_current_state(h, None) == capi.LBMHD_ERR_INVALID_ARG
    assert L.lbmhd_destroy(h) == 0
    assert L.lbmhd_destroy(None) == 0


def test_strerror_covers_codes(capi):
    for code in (0, -1, -2, -3, -4, -5):
        assert capi.strerror(code) not in ("", "unknown status")
    assert capi.strerror(-99) == "unknown status"


def test_product_path_fails_loudly_without_library(tmp_path, monkeypatch):
    from paper_1607_08675_amd import _capi
    monkeypatch.setattr(_capi, "_lib", None)
    monkeypatch.setattr(_capi, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(RuntimeError, match="no non-GPU fallback"):
        _capi.lib()


def _params3(capi, **kw):
    base = dict(nx=16, ny=8, nz=4, nu=0.01, eta=0.02, les=1, cs=0.1, cs_b=0.1, delta=1.0,
                storage=capi.LBMHD_FP32, mrt=0, s5=1.0, s7=1.0, s8=1.0, sg=1.0, szz=1.0)
    base.update(kw)
    return capi.Params3(*[base[n] for n, _ in capi.Params3._fields_])


@pytest.mark.parametrize("bad", [
    dict(nx=0), dict(nz=0), dict(nu=0.0), dict(eta=float("nan")), dict(les=2), dict(cs=-1.0),
    dict(cs_b=-1.0), dict(delta=0.0), dict(nx=1 << 14, ny=1 << 14, nz=8), dict(storage=5),
    dict(nx=1 << 14, ny=1 << 14, nz=16, storage=1), dict(mrt=2), dict(mrt=1, s5=0.0),
    dict(mrt=1, s7=2.0), dict(mrt=1, s8=float("nan")), dict(mrt=1, sg=-0.5), dict(mrt=1, szz=2.5),
])
def test_3d_create_rejects_invalid_parameters(capi, bad):
    h = ctypes.c_void_p()
    rc = capi.lib().lbmhd3_create(ctypes.byref(_params3(capi, **bad)), ctypes.byref(h))
    assert rc == capi.LBMHD_ERR_INVALID_ARG and not h.value


def test_3d_sizes_and_unbound_calls(capi):
    L = capi.lib()
    h = ctypes.c_void_p()
    assert L.lbmhd3_create(ctypes.byref(_params3(capi, nx=100, ny=6, nz=5)), ctypes.byref(h)) == 0
    lat, ws = ctypes.c_size_t(), ctypes.c_size_t()
    assert L.lbmhd3_sizes(h, ctypes.byref(lat), ctypes.byref(ws)) == 0
    assert lat.value == 45 * (5 * 6 * 128 + 192) * 4   # rows padded to 256 bytes, 768-byte gaps
    assert ws.value >= 7 * 100 * 6 * 5 * 8 and ws.value % 256 == 0
    assert L.lbmhd3_step(h, 1) == capi.LBMHD_ERR_NOT_BOUND
    assert b"bind" in L.lbmhd3_last_error(h)
    assert L.lbmhd3_destroy(h) == 0 and L.lbmhd3_destroy(None) == 0
    p16 = _params3(capi, nx=100, ny=6, nz=5, storage=capi.LBMHD_FP16)
    assert L.lbmhd3_create(ctypes.byref(p16), ctypes.byref(h)) == 0
    assert L.lbmhd3_sizes(h, ctypes.byref(lat), None) == 0
    assert lat.value == 45 * (5 * 6 * 128 + 384) * 2   # 128 halves = 256 bytes per row
    assert L.lbmhd3_destroy(h) == 0
    # a plane of 2^14 x 2^14 x 4 sites takes 4 GiB in FP32 (refused: in-plane
    # byte offsets are 32-bit) and 2 GiB in FP16 (accepted)
    big = dict(nx=1 << 14, ny=1 << 14, nz=4)
    assert L.lbmhd3_create(ctypes.byref(_params3(capi, **big)), ctypes.byref(h)) == \
        capi.LBMHD_ERR_INVALID_ARG
    p16 = _params3(capi, storage=capi.LBMHD_FP16, **big)
    assert L.lbmhd3_create(ctypes.byref(p16), ctypes.byref(h)) == 0
    assert L.lbmhd3_destroy(h) == 0
