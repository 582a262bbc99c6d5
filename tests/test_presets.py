"""Workload presets and the runner's command line (host side, no GPU).

Every preset must describe a lattice the library accepts (lbmhd_create /
lbmhd3_create validate on the host), name a known field generator with
arguments it takes, and state its readings."""
import ctypes
import inspect

import pytest

import lbmhd_inputs
from paper_1607_08675_amd import _capi, run


def test_presets_present():
    assert set(run.names()) >= {"orszag_tang_64", "orszag_tang_4096", "turbulence_8192_fp16",
                                "adjoint_1024", "cs_fit_2048", "kinetic_4096",
                                "crosshelicity_4096", "inplace_4096", "orszag_tang_3d_256"}


@pytest.mark.parametrize("name", run.names())
def test_preset_is_accepted_by_the_library(name):
    p = run.load(name)
    assert p.name == name and p.description and p.readings
    assert p.steps > 0 and p.diag_every > 0
    assert p.fields["generator"] in run.GENERATORS
    gen = getattr(lbmhd_inputs, p.fields["generator"])
    size = [p.lattice[k] for k in ("nx", "ny", "nz") if k in p.lattice]
    inspect.signature(gen).bind(*size, **p.fields.get("args", {}))
    cfg = p.config()
    L = _capi.lib()
    h = ctypes.c_void_p()
    if p.three_d:
        assert L.lbmhd3_create(ctypes.byref(cfg.c_params()), ctypes.byref(h)) == 0
        assert L.lbmhd3_destroy(h) == 0
    else:
        assert L.lbmhd_create(ctypes.byref(cfg.c_params()), ctypes.byref(h)) == 0
        assert L.lbmhd_destroy(h) == 0


def test_small_preset_fields():
    p = run.load("orszag_tang_64")
    rho, ux, uy, bx, by = p.initial_fields()
    assert rho.shape == (64, 64) and float(rho.min()) == 1.0
    assert abs(float(ux.max()) - 0.05) < 1e-12 and abs(float(by.max()) - 0.05) < 1e-3


def test_unknown_preset_and_generator_rejected():
    with pytest.raises(ValueError, match="no preset"):
        run.load("no_such_workload")
    p = run.load("orszag_tang_64")
    p.fields = {"generator": "eval", "args": {}}
    with pytest.raises(ValueError, match="unknown field generator"):
        p.initial_fields()


def test_list_on_the_command_line(capsys):
    assert run.main(["--list"]) == 0
    out = capsys.readouterr().out
    assert "orszag_tang_64" in out and "turbulence_8192_fp16" in out
