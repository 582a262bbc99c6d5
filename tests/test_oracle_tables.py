"""Pins of the oracle's lattice data against what the paper prints.

Flint & Vahala, arXiv:1607.08675, Sec. 3: the velocity lists, the matrices T
(eq. FluidTMatrix) and T_m (eq. MagTMatrix), the equilibrium moment tables
(eqs. KinMomentEq, MagMomentEq) and the D2Q9 / D2Q5 relaxation distributions.
The two tables and the two distributions are stated independently in the paper,
so T f^eq = M^eq and T_m g^eq = N^eq pin both the weights (which the paper never
states) and every term of f^eq and g^eq.
"""
import numpy as np
import pytest

from conftest import load_golden


def _matrix(name):
    return np.array([[float(v) for v in r.split()] for r in load_golden(name)])


def test_velocity_lists_match_paper(orc):
    rows = {r.split()[0]: np.array([float(v) for v in r.split()[1:]])
            for r in load_golden("paper_velocities.txt")}
    cx, cy, w, Cx, Cy, wm = orc.lattice()
    np.testing.assert_array_equal(cx, rows["c_x"])
    np.testing.assert_array_equal(cy, rows["c_y"])
    np.testing.assert_array_equal(Cx, rows["C_x"])
    np.testing.assert_array_equal(Cy, rows["C_y"])


def test_T_rows_match_printed_matrix(orc):
    T, Ti, Tm = orc.matrices()
    np.testing.assert_array_equal(T, _matrix("paper_T_matrix.txt"))
    np.testing.assert_array_equal(Tm, _matrix("paper_Tm_matrix.txt"))


def test_T_rows_orthogonal_and_inverse(orc):
    T, Ti, _ = orc.matrices()
    G = T @ T.T
    np.testing.assert_array_equal(G, np.diag(np.diag(G)))
    np.testing.assert_array_equal(np.diag(G), [9, 6, 6, 4, 4, 12, 12, 180, 20])
    np.testing.assert_allclose(Ti @ T, np.eye(9), atol=1e-15)
    np.testing.assert_allclose(T @ Ti, np.eye(9), atol=1e-15)
    np.testing.assert_allclose(Ti, np.linalg.inv(T), atol=1e-15)


def test_weights_isotropy(orc):
    """Textbook D2Q9 / D2Q5 lattice moments: sum w = 1, sum w c c = delta / 3,
    D2Q9 fourth moment = (delta delta + perms) / 9."""
    cx, cy, w, Cx, Cy, wm = orc.lattice()
    c = np.stack([cx, cy], 1)
    C = np.stack([Cx, Cy], 1)
    assert abs(w.sum() - 1) < 1e-15 and abs(wm.sum() - 1) < 1e-15
    np.testing.assert_allclose(np.einsum("i,ia,ib->ab", w, c, c), np.eye(2) / 3, atol=1e-15)
    np.testing.assert_allclose(np.einsum("i,ia,ib->ab", wm, C, C), np.eye(2) / 3, atol=1e-15)
    d = np.eye(2)
    iso = (np.einsum("ab,cd->abcd", d, d) + np.einsum("ac,bd->abcd", d, d)
           + np.einsum("ad,bc->abcd", d, d)) / 9
    np.testing.assert_allclose(np.einsum("i,ia,ib,ic,id->abcd", w, c, c, c, c), iso, atol=1e-15)


def _printed_meq(rho, jx, jy, bx, by):
    # eq. KinMomentEq, term by term as printed (written with rho u).
    return np.array([
        rho, jx, jy,
        jx * jy / rho - bx * by,
        (jx ** 2 - jy ** 2) / rho - bx ** 2 + by ** 2,
        -jx, -jy,
        -3 * (jx ** 2 + jy ** 2) / rho,
        5 / 3 * rho - 3 * (jx ** 2 + jy ** 2) / rho,
    ])


def _printed_neq(rho, jx, jy, bx, by):
    # eq. MagMomentEq, read with u = (rho u) / rho.
    ux, uy = jx / rho, jy / rho
    out = []
    for b, u in ((bx, ux), (by, uy)):
        out.append([b, ux * b - u * bx, uy * b - u * by, b / 3, b / 3])
    return np.array(out)


@pytest.mark.parametrize("seed", range(5))
def test_feq_moments_reproduce_paper_table(orc, seed):
    rng = np.random.default_rng(seed)
    rho = 1 + 0.2 * rng.standard_normal()
    ux, uy, bx, by = 0.1 * rng.standard_normal(4)
    T, _, Tm = orc.matrices()
    feq, geq = orc.equilibrium(rho, ux, uy, bx, by)
    jx, jy = rho * ux, rho * uy
    np.testing.assert_allclose(T @ feq, _printed_meq(rho, jx, jy, bx, by), atol=2e-15)
    np.testing.assert_allclose(geq @ Tm.T, _printed_neq(rho, jx, jy, bx, by), atol=2e-16)
    meq, neq = orc.moment_equilibria(rho, jx, jy, bx, by)
    np.testing.assert_allclose(meq, T @ feq, atol=2e-15)
    np.testing.assert_allclose(neq, geq @ Tm.T, atol=2e-16)


def test_conserved_moments_are_rho_j_B(orc):
    """Sec. 3: sum f = rho, sum c f = rho u, sum g = B; the first three fluid
    moments and the first magnetic moment are the collision invariants."""
    feq, geq = orc.equilibrium(1.3, 0.04, -0.07, 0.02, 0.09)
    cx, cy, *_ = orc.lattice()
    assert abs(feq.sum() - 1.3) < 1e-15
    assert abs((cx * feq).sum() - 1.3 * 0.04) < 1e-15
    assert abs((cy * feq).sum() + 1.3 * 0.07) < 1e-15
    np.testing.assert_allclose(geq.sum(1), [0.02, 0.09], atol=1e-16)


def test_maxwell_stress_in_second_moment(orc):
    """The B terms of f^eq give the momentum flux B^2/2 delta - B B, the Lorentz
    force of the filtered momentum equation (eq. FinalMomentum)."""
    cx, cy, *_ = orc.lattice()
    rho, bx, by = 1.0, 0.3, -0.2
    feq, _ = orc.equilibrium(rho, 0.0, 0.0, bx, by)
    c = np.stack([cx, cy], 1)
    Pi = np.einsum("i,ia,ib->ab", feq, c, c)
    B = np.array([bx, by])
    expect = rho / 3 * np.eye(2) + 0.5 * B @ B * np.eye(2) - np.outer(B, B)
    np.testing.assert_allclose(Pi, expect, atol=1e-15)
