"""The preset runner on the GPU: JSON-lines diagnostics of the 64^2
Orszag-Tang workload against the oracle's diagnostics of the same steps, and
a short 3D run."""
import json

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def test_orszag_tang_64_log_matches_oracle(gpu, orc, tmp_path):
    from paper_1607_08675_amd import run
    p = run.load("orszag_tang_64")
    path = str(tmp_path / "ot64.jsonl")
    recs = run.run(p, steps=30, every=10, log=path)
    lines = [json.loads(s) for s in open(path)]
    assert lines == recs
    assert [r["step"] for r in recs] == [0, 10, 20, 30]
    cfg = p.config()
    op = orc.Params(cfg.nx, cfg.ny, nu=cfg.nu, eta=cfg.eta, s5=cfg.s5, s6=cfg.s5, s7=cfg.s7,
                    s8=cfg.s8, les=cfg.les, cs=cfg.cs)
    st = orc.init(op, *p.initial_fields())
    for r in recs:
        if r["step"]:
            st = orc.run(op, st, 10)
        d = orc.diag(op, st)
        assert abs(r["mass"] - d["mass"]) <= 1e-9 * d["mass"]   # FP32 storage of f - w
        for k in ("e_kin", "e_mag"):
            assert abs(r[k] - d[k]) <= 1e-5 * abs(d[k]), (r["step"], k, r[k], d[k])
        assert r["nonfinite"] == 0


def test_3d_preset_runs(gpu):
    from paper_1607_08675_amd import run
    recs = run.run(run.load("orszag_tang_3d_256"), steps=2, every=1)
    assert [r["step"] for r in recs] == [0, 1, 2]
    m = [r["mass"] for r in recs]
    assert max(abs(x - m[0]) for x in m) <= 1e-6 * m[0]
    assert all(r["nonfinite"] == 0 for r in recs)
