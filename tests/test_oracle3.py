"""Pins of the 3D oracle (``oracle/lbmhd3_oracle.cpp``).

The paper defines the method in 2D and states that it extends to 3D with
more lattice velocities.  The 3D oracle's lattice, equilibria and closure are
pinned here by what fixes them: the isotropy of D3Q27 and of the six-vector
magnetic lattice, the equilibrium moments (the 3D form of eqs. KinMomentEq
and MagMomentEq), the exact reduction to the paper's 2D update for fields
that do not depend on one coordinate (checked against the 2D oracle along
two different axes), conservation, transport coefficients along z, the
closure against resolved strain and current, cube rotations.
"""
import numpy as np
import pytest

from lbmhd_inputs import random_fields

D2_CX = [0, 1, 0, -1, 0, 1, -1, -1, 1]
D2_CY = [0, 0, 1, 0, -1, 1, 1, -1, -1]
D2_MX = [0, 1, 0, -1, 0]
D2_MY = [0, 0, 1, 0, -1]


@pytest.fixture(scope="module")
def o3():
    from oracle import oracle3
    oracle3.build()
    return oracle3


def test_lattice_isotropy(o3):
    c, w, C, W = o3.lattice()
    assert len({tuple(v) for v in c}) == 27 and len({tuple(v) for v in C}) == 6
    assert abs(w.sum() - 1) < 1e-15 and abs(W.sum() - 1) < 1e-15
    d = np.eye(3)
    np.testing.assert_allclose(np.einsum("i,ia->a", w, c), 0, atol=1e-16)
    np.testing.assert_allclose(np.einsum("i,ia,ib->ab", w, c, c), d / 3, atol=1e-16)
    np.testing.assert_allclose(np.einsum("i,ia,ib,ic->abc", w, c, c, c), 0, atol=1e-16)
    four = (np.einsum("ab,cd->abcd", d, d) + np.einsum("ac,bd->abcd", d, d) +
            np.einsum("ad,bc->abcd", d, d)) / 9
    np.testing.assert_allclose(np.einsum("i,ia,ib,ic,id->abcd", w, c, c, c, c), four, atol=1e-16)
    np.testing.assert_allclose(np.einsum("k,ka,kb->ab", W, C, C), d / 3, atol=1e-16)
    for i in range(1, 27, 2):        # opposite velocities adjacent
        np.testing.assert_array_equal(c[i], -c[i + 1])


def test_z_sums_give_the_paper_2d_weights(o3):
    """Summing D3Q27 over c_z gives the D2Q9 weights (4/9, 1/9, 1/36); the six
    magnetic vectors give the D2Q5 weights (1/3 at rest from +-z, 1/6)."""
    c, w, C, W = o3.lattice()
    for i2 in range(9):
        s = sum(w[i] for i in range(27) if (c[i][0], c[i][1]) == (D2_CX[i2], D2_CY[i2]))
        want = 4 / 9 if i2 == 0 else (1 / 9 if i2 < 5 else 1 / 36)
        assert abs(s - want) < 1e-15, i2
    for k2 in range(5):
        s = sum(W[k] for k in range(6) if (C[k][0], C[k][1]) == (D2_MX[k2], D2_MY[k2]))
        assert abs(s - (1 / 3 if k2 == 0 else 1 / 6)) < 1e-15


def test_equilibrium_moments(o3):
    """rho, j, the momentum flux rho I/3 + j j / rho + |B|^2 I / 2 - B B and the
    third moment (delta j + ...)/3 of f^eq; B, the induction flux
    u_a B_b - B_a u_b and B delta / 3 of g^eq."""
    c, w, C, W = o3.lattice()
    rng = np.random.default_rng(3)
    d = np.eye(3)
    for _ in range(5):
        rho = 1 + 0.1 * rng.standard_normal()
        u, B = 0.1 * rng.standard_normal(3), 0.1 * rng.standard_normal(3)
        feq, geq = o3.equilibrium(rho, u, B)
        j = rho * u
        assert abs(feq.sum() - rho) < 1e-15
        np.testing.assert_allclose(c.T @ feq, j, atol=1e-16)
        Pi = rho * d / 3 + np.outer(j, j) / rho + 0.5 * (B @ B) * d - np.outer(B, B)
        np.testing.assert_allclose(np.einsum("ia,ib,i->ab", c, c, feq), Pi, atol=1e-15)
        third = (np.einsum("ab,c->abc", d, j) + np.einsum("ac,b->abc", d, j) +
                 np.einsum("bc,a->abc", d, j)) / 3
        np.testing.assert_allclose(np.einsum("ia,ib,ic,i->abc", c, c, c, feq), third, atol=1e-15)
        np.testing.assert_allclose(geq.sum(axis=1), B, atol=1e-16)
        np.testing.assert_allclose(np.einsum("ka,bk->ab", C, geq), np.outer(u, B) - np.outer(B, u),
                                   atol=1e-16)
        np.testing.assert_allclose(np.einsum("ka,kc,bk->acb", C, C, geq),
                                   np.einsum("ac,b->acb", d, B) / 3, atol=1e-16)


def _project(st3, c, C, axis):
    """Sum the 3D populations of a state invariant along `axis` over that
    velocity component: a 2D state in the two remaining coordinates, in the
    2D oracle's plane order (f_0..f_8, g_x(5), g_y(5))."""
    keep = [a for a in range(3) if a != axis]
    sl = [slice(None)] * 3
    sl[2 - axis] = 0                                   # arrays are [z][y][x]
    planes = st3[(slice(None), *sl)]                   # (45, n1, n0) of the kept axes
    out = np.zeros((19,) + planes.shape[1:])
    for i in range(27):
        i2 = [(D2_CX[t], D2_CY[t]) for t in range(9)].index((c[i][keep[0]], c[i][keep[1]]))
        out[i2] += planes[i]
    for k in range(6):
        k2 = [(D2_MX[t], D2_MY[t]) for t in range(5)].index((C[k][keep[0]], C[k][keep[1]]))
        for b2, b in enumerate(keep):
            out[9 + 5 * b2 + k2] += planes[27 + 6 * b + k]
    return out


@pytest.mark.parametrize("axis", [2, 1])
def test_reduces_to_the_paper_2d_update(o3, orc, axis):
    """Fields independent of one coordinate, with no velocity or field along
    it: the 3D update summed over that velocity component is the paper's 2D
    update with all moment rates equal to 1/tau0 (its BGK limit), step by
    step, to rounding.  axis = 2: fields in (x, y); axis = 1: fields in
    (x, z), so streaming along z is checked too."""
    c, w, C, W = o3.lattice()
    n0, n1, nu, eta = 12, 10, 0.02, 0.03
    rho, ux, uy, bx, by = random_fields(n0, n1, 5, u_amp=0.05, b_amp=0.05)
    zero = np.zeros_like(ux)
    keep = [a for a in range(3) if a != axis]
    u3 = [zero, zero, zero]
    b3 = [zero, zero, zero]
    u3[keep[0]], u3[keep[1]], b3[keep[0]], b3[keep[1]] = ux, uy, bx, by
    shape = {2: (1, n1, n0), 1: (n1, 3, n0)}[axis]
    def lift(a):
        a = np.asarray(a, dtype=np.float64)
        return np.broadcast_to(a[None] if axis == 2 else a[:, None, :], shape).copy()
    p3 = o3.Params(shape[2], shape[1], shape[0], nu=nu, eta=eta, les=0)
    st3 = o3.init(p3, *[lift(a) for a in [rho] + u3 + b3])
    s = 1 / (3 * nu + 0.5)
    p2 = orc.Params(n0, n1, nu=nu, eta=eta, s5=s, s6=s, s7=s, s8=s, les=0)
    st2 = orc.init(p2, rho, ux, uy, bx, by)
    np.testing.assert_allclose(_project(st3, c, C, axis), st2, atol=1e-15)
    for _ in range(3):
        st3, st2 = o3.run(p3, st3, 4), orc.run(p2, st2, 4)
        np.testing.assert_allclose(_project(st3, c, C, axis), st2, atol=2e-15)


@pytest.mark.parametrize("rates", [(1.3, 0.7, 1.6, 1.1, 0.9), (0.6, 1.8, 0.5, 1.9, 1.4)])
def test_moment_collision_reduces_to_the_paper_2d_mrt(o3, orc, rates):
    """The moment-space collision (mrt = 1) with unequal rates: for fields
    independent of z, with no velocity or field along z, the 3D update summed
    over c_z is the paper's 2D update with the same s5 = s6, s7, s8 (shear
    1/tau0), step by step, to rounding, whatever the rates sg and szz of the
    moments that vary along c_z.  The two sets differ from each other and
    from 1/tau0 = 1.79 in every rate, so a 3D rate table that mixed the z
    sums with those moments, or a 2D row taken wrong, shows here."""
    c, w, C, W = o3.lattice()
    n0, n1, nu, eta = 12, 10, 0.02, 0.03
    s5, s7, s8, sg, szz = rates
    rho, ux, uy, bx, by = random_fields(n0, n1, 7, u_amp=0.05, b_amp=0.05)
    zero = np.zeros_like(ux)
    def lift(a):
        return np.broadcast_to(np.asarray(a, dtype=np.float64)[None], (2, n1, n0)).copy()
    p3 = o3.Params(n0, n1, 2, nu=nu, eta=eta, les=0, mrt=1, s5=s5, s7=s7, s8=s8, sg=sg,
                   szz=szz)
    st3 = o3.init(p3, *[lift(a) for a in (rho, ux, uy, zero, bx, by, zero)])
    p2 = orc.Params(n0, n1, nu=nu, eta=eta, s5=s5, s6=s5, s7=s7, s8=s8, les=0)
    st2 = orc.init(p2, rho, ux, uy, bx, by)
    # a non-equilibrium start: the same perturbation of every z layer, even
    # in c_z (u_z and B_z stay zero), none on the g_z planes
    rng = np.random.default_rng(3)
    dz = 1e-3 * rng.standard_normal((45, 1, n1, n0)) * np.concatenate(
        [w, np.full(18, 0.2)])[:, None, None, None]
    mirror = [next(j for j in range(27) if list(c[j]) == [c[i][0], c[i][1], -c[i][2]])
              for i in range(27)]
    mirror += [27 + 6 * (q // 6) + next(j for j in range(6) if list(C[j]) == [
        C[q % 6][0], C[q % 6][1], -C[q % 6][2]]) for q in range(18)]
    dz = 0.5 * (dz + dz[mirror])
    dz[39:45] = 0.0
    st3 = st3 + dz
    st2 = st2 + _project(dz * np.ones((1, 2, 1, 1)), c, C, 2)
    np.testing.assert_allclose(_project(st3, c, C, 2), st2, atol=1e-15)
    for _ in range(3):
        st3, st2 = o3.run(p3, st3, 4), orc.run(p2, st2, 4)
        np.testing.assert_allclose(_project(st3, c, C, 2), st2, atol=2e-15)
    # the 3D update is not the BGK one at these rates
    pb = o3.Params(n0, n1, 2, nu=nu, eta=eta, les=0)
    assert np.abs(o3.run(pb, st3, 1) - o3.run(p3, st3, 1)).max() > 1e-6


def test_moment_collision_with_every_rate_one_over_tau_is_bgk(o3):
    """mrt = 1 with every rate 1/tau (per site, with the closure) is the
    single-relaxation update: T^-1 S T = I / tau."""
    p = o3.Params(5, 4, 3, nu=0.02, eta=0.01, les=1, cs=0.2, csb=0.15)
    rng = np.random.default_rng(4)
    f = [1 + 0.01 * rng.standard_normal((3, 4, 5))] + [0.05 * rng.standard_normal((3, 4, 5))
                                                       for _ in range(6)]
    st = o3.init(p, *f) + 1e-3 * rng.standard_normal((45, 3, 4, 5))
    s0 = 1 / (3 * p.nu + 0.5)
    pm = o3.Params(5, 4, 3, nu=0.02, eta=0.01, les=0, mrt=1, s5=s0, s7=s0, s8=s0, sg=s0, szz=s0)
    p0 = o3.Params(5, 4, 3, nu=0.02, eta=0.01, les=0)
    np.testing.assert_allclose(o3.collide(pm, st), o3.collide(p0, st), atol=1e-16)


def test_moment_collision_conserves_and_keeps_equilibria(o3):
    p = o3.Params(6, 5, 4, nu=0.02, eta=0.01, les=1, cs=0.2, csb=0.15, mrt=1, s5=1.3,
                  s7=0.7, s8=1.6, sg=1.1, szz=0.9)
    rng = np.random.default_rng(1)
    f = [1 + 0.01 * rng.standard_normal((4, 5, 6))] + [0.05 * rng.standard_normal((4, 5, 6))
                                                       for _ in range(6)]
    st = o3.init(p, *f) + 1e-3 * rng.standard_normal((45, 4, 5, 6))
    d0, d1 = o3.diag(p, st), o3.diag(p, o3.run(p, st, 10))
    assert abs(d1["mass"] - d0["mass"]) < 1e-14 * d0["mass"]
    for k in ("mom_x", "mom_y", "mom_z", "flux_x", "flux_y", "flux_z"):
        assert abs(d1[k] - d0[k]) < 1e-14, k
    eq = o3.init(p, *f)
    np.testing.assert_allclose(o3.collide(p, eq), eq, atol=1e-16)


def test_conservation_and_fixed_point(o3):
    p = o3.Params(6, 5, 4, nu=0.02, eta=0.01, les=1, cs=0.2, csb=0.15)
    rng = np.random.default_rng(1)
    f = [1 + 0.01 * rng.standard_normal((4, 5, 6))] + [0.05 * rng.standard_normal((4, 5, 6))
                                                       for _ in range(6)]
    st = o3.init(p, *f) + 1e-3 * rng.standard_normal((45, 4, 5, 6))
    d0, d1 = o3.diag(p, st), o3.diag(p, o3.run(p, st, 10))
    assert abs(d1["mass"] - d0["mass"]) < 1e-14 * d0["mass"]
    for k in ("mom_x", "mom_y", "mom_z", "flux_x", "flux_y", "flux_z"):
        assert abs(d1[k] - d0[k]) < 1e-14, k
    uni = o3.init(p, 1.1, 0.02, -0.03, 0.01, 0.04, 0.02, -0.05)
    np.testing.assert_allclose(o3.run(p, uni, 5), uni, atol=1e-16)


def _decay(o3, p, f, key, k, coord, t0=100, t1=1100):
    st = o3.run(p, o3.init(p, *f), t0)
    a0 = 2 * np.mean(o3.macro(p, st)[key] * np.sin(k * coord))
    st = o3.run(p, st, t1 - t0)
    a1 = 2 * np.mean(o3.macro(p, st)[key] * np.sin(k * coord))
    return -np.log(a1 / a0) / (t1 - t0)


def test_transport_coefficients_along_z(o3):
    """u_x = U sin(k z) decays at nu k^2; B_y = B0 sin(k z) at eta k^2 (to
    the O(k^2) lattice correction, 0.08% at this k)."""
    n = 64
    k = 2 * np.pi / n
    z = np.arange(n)[:, None, None] * np.ones((1, 2, 2))
    zero = np.zeros_like(z)
    p = o3.Params(2, 2, n, nu=0.02, eta=0.04, les=0)
    r = _decay(o3, p, (1.0, 1e-4 * np.sin(k * z), zero, zero, zero, zero, zero), "ux", k, z)
    assert abs(r / (p.nu * k * k) - 1) < 2e-3, r / (p.nu * k * k)
    r = _decay(o3, p, (1.0, zero, zero, zero, zero, 1e-4 * np.sin(k * z), zero), "by", k, z)
    assert abs(r / (p.eta * k * k) - 1) < 2e-3, r / (p.eta * k * k)


def test_moment_collision_transport_along_z(o3):
    """With the moment-space collision at unequal rates the shears xz and yz
    still relax at 1/tau: u_x = U sin(k z) decays at nu k^2 and B_y = B0
    sin(k z) at eta k^2, as with single relaxation."""
    n = 64
    k = 2 * np.pi / n
    z = np.arange(n)[:, None, None] * np.ones((1, 2, 2))
    zero = np.zeros_like(z)
    p = o3.Params(2, 2, n, nu=0.02, eta=0.04, les=0, mrt=1, s5=1.3, s7=0.7, s8=1.6, sg=1.1,
                  szz=0.9)
    r = _decay(o3, p, (1.0, 1e-4 * np.sin(k * z), zero, zero, zero, zero, zero), "ux", k, z)
    assert abs(r / (p.nu * k * k) - 1) < 2e-3, r / (p.nu * k * k)
    r = _decay(o3, p, (1.0, zero, zero, zero, zero, 1e-4 * np.sin(k * z), zero), "by", k, z)
    assert abs(r / (p.eta * k * k) - 1) < 2e-3, r / (p.eta * k * k)


def _d(a, axis):
    return 0.5 * (np.roll(a, -1, axis) - np.roll(a, 1, axis))


def test_closure_matches_resolved_strain(o3):
    """u_x = U sin(k z): tau = tau0 + 3 C_Sv |d u_x / d z| (eq. SmagorinskyClosure)."""
    n, U, cs = 64, 0.01, 0.1
    k = 2 * np.pi / n
    z = np.arange(n)[:, None, None] * np.ones((1, 2, 2))
    zero = np.zeros_like(z)
    p = o3.Params(2, 2, n, nu=0.01, eta=0.01, les=1, cs=cs, csb=0.2)
    st = o3.run(p, o3.init(p, 1.0, U * np.sin(k * z), zero, zero, zero, zero, zero), 60)
    dudz = _d(o3.macro(p, st)["ux"], 0)
    _, tau, _ = o3.collide(p, st, return_tau=True)
    sel = np.abs(dudz) > 0.3 * np.abs(dudz).max()
    rel = np.abs(tau - 3 * p.nu - 0.5 - 3 * cs * np.abs(dudz))[sel] / (3 * cs * np.abs(dudz[sel]))
    assert rel.max() < 0.03, rel.max()


def test_closure_matches_resolved_current(o3):
    """B = B0 (sin k y, sin k x, 0) has both d_x B_y and d_y B_x: tau_m =
    tau_m0 + 3 C_Sb |j| with j_z = d_x B_y - d_y B_x (eq.
    SmagorinskyMHDClosureB); a symmetric-part mix-up would give |d_x B_y +
    d_y B_x| instead."""
    n, B0, csb = 64, 0.01, 0.2
    k = 2 * np.pi / n
    y, x = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    y, x = np.broadcast_to(y, (2, n, n)), np.broadcast_to(x, (2, n, n))
    zero = np.zeros((2, n, n))
    p = o3.Params(n, n, 2, nu=0.01, eta=0.01, les=1, cs=0.1, csb=csb)
    st = o3.run(p, o3.init(p, 1.0, zero, zero, zero, B0 * np.sin(k * y), B0 * np.sin(k * x), zero),
                60)
    m = o3.macro(p, st)
    jz = _d(m["by"], 2) - _d(m["bx"], 1)
    _, _, taum = o3.collide(p, st, return_tau=True)
    sel = np.abs(jz) > 0.3 * np.abs(jz).max()
    rel = np.abs(taum - 3 * p.eta - 0.5 - 3 * csb * np.abs(jz))[sel] / (3 * csb * np.abs(jz[sel]))
    assert rel.max() < 0.03, rel.max()


def _rotate(o3, st):
    """Cyclic axis permutation (x, y, z) -> (y, z, x) of a state: site
    (x, y, z) moves to (z, x, y) and velocity (a, b, c) becomes (c, a, b)."""
    c, _, C, _ = o3.lattice()
    out = np.empty_like(st)
    moved = np.transpose(st, (0, 2, 1, 3))               # [q][z][y][x] -> ...
    moved = np.transpose(st, (0, 2, 3, 1))               # new [z'][y'][x'] = old [y][x][z]
    idx27 = {tuple(v): i for i, v in enumerate(c)}
    idx6 = {tuple(v): i for i, v in enumerate(C)}
    for i, v in enumerate(c):
        out[idx27[(v[2], v[0], v[1])]] = moved[i]
    for b in range(3):
        for k, v in enumerate(C):
            out[27 + 6 * ((b + 1) % 3) + idx6[(v[2], v[0], v[1])]] = moved[27 + 6 * b + k]
    return out


def test_update_commutes_with_cube_rotation(o3):
    n = 5
    p = o3.Params(n, n, n, nu=0.02, eta=0.01, les=1, cs=0.2)
    rng = np.random.default_rng(8)
    f = [1 + 0.01 * rng.standard_normal((n, n, n))] + [0.05 * rng.standard_normal((n, n, n))
                                                       for _ in range(6)]
    st = o3.init(p, *f) + 1e-3 * rng.standard_normal((45, n, n, n))
    a = _rotate(o3, o3.run(p, st, 3))
    b = o3.run(p, _rotate(o3, st), 3)
    np.testing.assert_allclose(a, b, atol=1e-15)
