"""The oracle's pins catch plausible mistakes.

Each case plants one mistake in a copy of ``oracle/lbmhd_oracle.cpp`` (a
wrong weight, a flipped sign, a dropped factor, a transposed inverse, the
wrong streaming direction, a wrong closure constant, a wrong rate index, a
wrong root or sign in a closure, a broken dual-number rule), builds it with the same flags into a temporary
library, and runs the pin suites (tables, physics, kinetic and cross-helicity
closures; the 3D suite for the 3D oracle) against it in a subprocess.  Every mutant must make at least one pin fail; the
unmodified source must pass.  Everything runs on the CPU.
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

import pytest

from conftest import ROOT

SRC = os.path.join(ROOT, "oracle", "lbmhd_oracle.cpp")
SRC3 = os.path.join(ROOT, "oracle", "lbmhd3_oracle.cpp")
PINS3 = [os.path.join(ROOT, "tests", "test_oracle3.py")]
PINS = [os.path.join(ROOT, "tests", "test_oracle_tables.py"),
        os.path.join(ROOT, "tests", "test_oracle_physics.py"),
        os.path.join(ROOT, "tests", "test_oracle_kinetic.py"),
        os.path.join(ROOT, "tests", "test_oracle_crosshelicity.py")]

MUTANTS = {
    "diagonal weight 1/36 -> 1/18": ("1.0 / 9.0 : 1.0 / 36.0)", "1.0 / 9.0 : 1.0 / 18.0)"),
    "T row 7 drops a factor 2": ("4.0 - 9.0 * (cx2 + cy2 - 2.0 * cx2 * cy2)",
                                 "4.0 - 9.0 * (cx2 + cy2 - cx2 * cy2)"),
    "Maxwell stress sign": ("4.5 * w * (0.5 * b2 * c2 - cb * cb)",
                            "4.5 * w * (0.5 * b2 * c2 + cb * cb)"),
    "Maxwell stress half": ("4.5 * w * (0.5 * b2 * c2 - cb * cb)",
                            "4.5 * w * (1.0 * b2 * c2 - cb * cb)"),
    "g^eq u x B sign": ("geq[k] = w * (bx + 3.0 * (cu * bx - cb * ux));",
                        "geq[k] = w * (bx + 3.0 * (cu * bx + cb * ux));"),
    "M3^eq Lorentz sign": ("meq[3] = jx * jy / rho - bx * by;", "meq[3] = jx * jy / rho + bx * by;"),
    "M8^eq coefficient": ("meq[8] = (5.0 / 3.0) * rho", "meq[8] = (4.0 / 3.0) * rho"),
    "T inverse transposed": ("Tinv[i][r] = T[r][i] / n2;", "Tinv[r][i] = T[r][i] / n2;"),
    "tau0 offset": ("r.tau0 = 3.0 * p.nu + 0.5;", "r.tau0 = 3.0 * p.nu + 1.0;"),
    "eta mapping uses nu": ("r.taum0 = 3.0 * p.eta + 0.5;", "r.taum0 = 3.0 * p.nu + 0.5;"),
    "closure factor 18 -> 9": ("18.0 * d2 * cs * Q / rho", "9.0 * d2 * cs * Q / rho"),
    "closure Q drops factor 4": ("R Q = root(n4 * n4 + 4.0 * n3 * n3);", "R Q = root(n4 * n4 + n3 * n3);"),
    "magnetic closure sign of A": ("R A = (N[5 + 1] - neq[5 + 1]) - (N[0 + 2] - neq[0 + 2]);",
                                   "R A = (N[5 + 1] - neq[5 + 1]) + (N[0 + 2] - neq[0 + 2]);"),
    "magnetic closure factor 36 -> 18": ("36.0 * d2 * csb * magnitude(A)", "18.0 * d2 * csb * magnitude(A)"),
    "eddy resistivity takes C_Sv": ("36.0 * d2 * csb * magnitude(A)", "36.0 * d2 * cs * magnitude(A)"),
    "cross-helicity resistivity takes C_Sv": ("d2 * csb * sign_of(value(X))", "d2 * cs * sign_of(value(X))"),
    "eddy viscosity takes C_Sb": ("18.0 * d2 * cs * Q / rho", "18.0 * d2 * csb * Q / rho"),
    "shear rate s4 takes s5": ("  s[4] = 1.0 / tau;\n", "  s[4] = R(rt.s[5]);\n"),
    "relaxation sign": ("Mstar[r] = M[r] - s[r] * (M[r] - meq[r]);",
                        "Mstar[r] = M[r] + s[r] * (M[r] - meq[r]);"),
    "magnetic rate uses tau": ("R sm = 1.0 / taum;", "R sm = 1.0 / tau;"),
    "streaming direction of f": ("int64_t xd = wrap(x + CX[i], nx), yd = wrap(y + CY[i], ny);",
                                 "int64_t xd = wrap(x - CX[i], nx), yd = wrap(y - CY[i], ny);"),
    "dual product rule": ("r.d[k] = a.d[k] * b.v + a.v * b.d[k];", "r.d[k] = a.d[k] * b.v;"),
    "ratio rule sign": ("acc = acc + dX[b] * dY[b] - (dZ[b] / Z) * (X * dY[b] + Y * dX[b] - X * Y * dZ[b] / Z);",
                        "acc = acc + dX[b] * dY[b] + (dZ[b] / Z) * (X * dY[b] + Y * dX[b] - X * Y * dZ[b] / Z);"),
    "product rule 1/12 -> 1/24": ("return (d2 / 12.0) * (dX[0] * dY[0] + dX[1] * dY[1]);",
                                  "return (d2 / 24.0) * (dX[0] * dY[0] + dX[1] * dY[1]);"),
    "M4 correction magnetic sign": ("- filtered_product_term(d2, gbx, gbx) + filtered_product_term(d2, gby, gby);",
                                    "+ filtered_product_term(d2, gbx, gbx) - filtered_product_term(d2, gby, gby);"),
    "M8 correction dropped": ("  dmeq[8] = -3.0 * (jxjx + jyjy);", "  dmeq[8] = 0.0 * (jxjx + jyjy);"),
    "N correction sign": ("    dneq[5 * a + 1] = filtered_ratio_term(d2, jx, b[a], rho, gjx, gb[a], gr) -",
                          "    dneq[5 * a + 1] = filtered_ratio_term(d2, jx, b[a], rho, gjx, gb[a], gr) +"),
    "gradient stencil weight": ("3.0 * weight9(i) * double(CX[i]) * mac[m * n + t];",
                                "2.0 * weight9(i) * double(CX[i]) * mac[m * n + t];"),
    "T_m inverse transposed in use": ("acc = acc + tb.Tminv[k][r] * dneq[5 * a + r];",
                                      "acc = acc + tb.Tminv[r][k] * dneq[5 * a + r];"),
    "cross-helicity contraction drops factor 2": ("R P = n4 * dL + 2.0 * n3 * sL;",
                                                 "R P = n4 * dL + n3 * sL;"),
    "cross-helicity S^b takes the antisymmetric part": (
        "R sL = (N[5 + 1] - neq[5 + 1]) + (N[0 + 2] - neq[0 + 2]);",
        "R sL = (N[5 + 1] - neq[5 + 1]) - (N[0 + 2] - neq[0 + 2]);"),
    "cross-helicity normal strain of B summed": (
        "R dL = (N[0 + 1] - neq[0 + 1]) - (N[5 + 2] - neq[5 + 2]);",
        "R dL = (N[0 + 1] - neq[0 + 1]) + (N[5 + 2] - neq[5 + 2]);"),
    "cross-helicity sign of the backscatter": ("R qb = -3.0 * std::sqrt(3.0) * d2",
                                               "R qb = 3.0 * std::sqrt(3.0) * d2"),
    "vorticity sign of d_y u_x": ("R omega = ((grad[4] - uy * grad[0]) - (grad[3] - ux * grad[1])) / rho;",
                                  "R omega = ((grad[4] - uy * grad[0]) + (grad[3] - ux * grad[1])) / rho;"),
    "cross-helicity resistivity not clipped": ("if (tm < std::sqrt(0.5)) {", "if (tm < 0.0) {"),
    "cubic takes the middle root": ("return 2.0 * r * std::cos(std::acos(h) / 3.0);",
                                    "return 2.0 * r * std::cos((std::acos(h) - 2.0 * M_PI) / 3.0);"),
    "Cardano sign": ("return std::cbrt(0.5 * q + d) + std::cbrt(0.5 * q - d);",
                     "return std::cbrt(0.5 * q + d) - std::cbrt(0.5 * q - d);"),
    "cross-helicity viscosity factor 9/2 -> 3": ("R qv = 4.5 * d2 * cs", "R qv = 3.0 * d2 * cs"),
    "dual sqrt rule": ("double g = r.v > 0.0 ? 0.5 / r.v : 0.0;", "double g = r.v > 0.0 ? 1.0 / r.v : 0.0;"),
}


MUTANTS3 = {
    "3D lattice weights 2/3, 1/6 -> 1/2, 1/4": ("C27[i][a] == 0 ? 2.0 / 3.0 : 1.0 / 6.0",
                                               "C27[i][a] == 0 ? 1.0 / 2.0 : 1.0 / 4.0"),
    "3D Maxwell stress sign": ("(a == b ? 0.5 * b2 : 0.0) - B[a] * B[b];",
                               "(a == b ? 0.5 * b2 : 0.0) + B[a] * B[b];"),
    "3D Hermite trace 1/3 -> 1/2": ("(C27[i][a] * C27[i][b] - (a == b ? 1.0 / 3.0 : 0.0))",
                                    "(C27[i][a] * C27[i][b] - (a == b ? 0.5 : 0.0))"),
    "3D g^eq induction sign": ("(B[b] + 3.0 * (cu * B[b] - cb * u[b])) / 6.0",
                               "(B[b] + 3.0 * (cu * B[b] + cb * u[b])) / 6.0"),
    "3D streaming along z reversed": ("wrap(z + c[2], nz)", "wrap(z - c[2], nz)"),
    "3D current from the symmetric part": ("L[0][1] - L[1][0]", "L[0][1] + L[1][0]"),
    "3D closure factor 36 -> 18": ("36.0 * d2 * p.csb * An", "18.0 * d2 * p.csb * An"),
    "3D eddy viscosity takes C_Sb": ("18.0 * d2 * p.cs * Q / rho", "18.0 * d2 * p.csb * Q / rho"),
    "3D strain drops the factor 2": ("std::sqrt(2.0 * ss)", "std::sqrt(ss)"),
}


def _run_pins(lib_path, pins=PINS, var="LBMHD_ORACLE_LIB"):
    env = dict(os.environ, OMP_NUM_THREADS="2")
    env[var] = lib_path
    return subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                           *pins], cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)


def _build(tmp_path, text, name):
    from oracle import oracle
    src = tmp_path / f"{name}.cpp"
    src.write_text(text)
    return oracle.compile_source(str(src), str(tmp_path / f"lib{name}.so"))


def _case(d, key):
    """Build one oracle variant in directory d and run its pin suite:
    (return code, output tail)."""
    kind, name = key
    src, pins, var = (SRC3, PINS3, "LBMHD3_ORACLE_LIB") if kind.endswith("3") else \
        (SRC, PINS, "LBMHD_ORACLE_LIB")
    text = open(src).read()
    if kind.startswith("mut"):
        old, new = (MUTANTS3 if kind.endswith("3") else MUTANTS)[name]
        assert text.count(old) >= 1, f"mutation site not found: {old}"
        text = text.replace(old, new, 1)
    d.mkdir()
    r = _run_pins(_build(d, text, "v"), pins, var)
    return r.returncode, r.stdout[-2000:]


@pytest.fixture(scope="module")
def outcomes(tmp_path_factory):
    """Every variant built and checked once, four at a time (each pin run uses
    two threads): the unmodified sources and every mutant."""
    keys = [("orig", ""), ("orig3", "")] + [("mut", k) for k in sorted(MUTANTS)] + \
        [("mut3", k) for k in sorted(MUTANTS3)]
    tmp = tmp_path_factory.mktemp("mutants")
    with ThreadPoolExecutor(max_workers=4) as ex:
        futs = {k: ex.submit(_case, tmp / f"v{i}", k) for i, k in enumerate(keys)}
        return {k: f.result() for k, f in futs.items()}


def test_unmodified_oracle_passes_pins(outcomes):
    rc, out = outcomes[("orig", "")]
    assert rc == 0, out


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(outcomes, name):
    rc, _ = outcomes[("mut", name)]
    assert rc != 0, f"mutant '{name}' passed every pin"


def test_unmodified_3d_oracle_passes_pins(outcomes):
    rc, out = outcomes[("orig3", "")]
    assert rc == 0, out


@pytest.mark.parametrize("name", sorted(MUTANTS3))
def test_3d_mutant_is_caught(outcomes, name):
    rc, _ = outcomes[("mut3", name)]
    assert rc != 0, f"mutant '{name}' passed every pin"
