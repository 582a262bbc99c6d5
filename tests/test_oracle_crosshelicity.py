"""Pins of the oracle's cross-helicity closure (les = 4, and 6 with the
kinetic closure) against the paper's definitions, eqs. CHClosureV/B:

    nu_t  = C_S Delta^2 |S^v : S^b|^(1/2),
    eta_t = C_S Delta^2 sgn(j . omega) |j . omega|^(1/2),

with S^v the strain of u, S^b the symmetrised gradient of B, j the current
and omega the vorticity of the resolved fields.  The oracle reads S^v, S^b
and j from non-equilibrium moments and omega from lattice differences; the
checks below compare its relaxation times with these quantities taken from
the macroscopic fields by centred differences, so a wrong factor, sign or
index in the moment algebra fails them.  Backscatter (j . omega < 0) lowers
eta; the total resistivity is clipped at zero (tau_m >= 1/2).
"""
import numpy as np
import pytest

from test_oracle_physics import _mirror_x, _random_state, _rotate


def _cellular_fields(p, U, B0):
    """Solenoidal cellular flow and field with different wave numbers:
    u = curl of U (sin(kx) sin(ky) + 0.8 sin(ky + 0.5)) / k (cells plus a
    shear), B = curl of B0 sin(kx + 1) sin(2ky + 2) / k, so both strains have
    normal and shear parts, S^b_xy differs from j / 2, and S^v : S^b and
    j . omega change sign across the lattice."""
    k = 2 * np.pi / p.nx
    y, x = np.meshgrid(np.arange(p.ny), np.arange(p.nx), indexing="ij")
    ux = U * (np.sin(k * x) * np.cos(k * y) + 0.8 * np.cos(k * y + 0.5))
    uy = -U * np.cos(k * x) * np.sin(k * y)
    bx = 2 * B0 * np.sin(k * x + 1) * np.cos(2 * k * y + 2)
    by = -B0 * np.cos(k * x + 1) * np.sin(2 * k * y + 2)
    return 1.0, ux, uy, bx, by


def _dx(a):
    return 0.5 * (np.roll(a, -1, 1) - np.roll(a, 1, 1))


def _dy(a):
    return 0.5 * (np.roll(a, -1, 0) - np.roll(a, 1, 0))


def _evolved(orc, eta, U=0.01, B0=0.01, cs=0.1, steps=60):
    p = orc.Params(64, 64, nu=0.01, eta=eta, les=4, cs=cs)
    st = orc.run(p, orc.init(p, *_cellular_fields(p, U, B0)), steps)
    m = orc.macro(p, st)
    _, tau, taum = orc.collide(p, st, return_tau=True)
    return p, m, tau, taum


def _resolved(m):
    """S^v : S^b (traceless parts) and j . omega by centred differences."""
    ux, uy, bx, by = m["ux"], m["uy"], m["bx"], m["by"]
    svd, svs = _dx(ux) - _dy(uy), 0.5 * (_dy(ux) + _dx(uy))
    sbd, sbs = _dx(bx) - _dy(by), 0.5 * (_dy(bx) + _dx(by))
    ss = 0.5 * svd * sbd + 2 * svs * sbs
    jw = (_dx(by) - _dy(bx)) * (_dx(uy) - _dy(ux))
    return ss, jw


def test_eddy_viscosity_matches_cross_strain(orc):
    """nu_t = C_S Delta^2 |S^v : S^b|^(1/2) with the contraction of the
    traceless strains, (1/2)(S_xx - S_yy)^v (S_xx - S_yy)^b + 2 S^v_xy S^b_xy."""
    p, m, tau, _ = _evolved(orc, eta=0.01)
    ss, _ = _resolved(m)
    expect = 3 * p.cs * np.sqrt(np.abs(ss))
    sel = np.abs(ss) > 0.3 * np.abs(ss).max()
    assert np.any(ss[sel] > 0) and np.any(ss[sel] < 0)
    rel = np.abs((tau - (3 * p.nu + 0.5)) - expect)[sel] / expect[sel]
    assert rel.max() < 0.03, rel.max()


def test_eddy_resistivity_follows_cross_helicity_with_its_sign(orc):
    """eta_t = C_S Delta^2 sgn(j omega) |j omega|^(1/2), negative
    (backscatter) where j omega < 0."""
    p, m, _, taum = _evolved(orc, eta=0.01)
    _, jw = _resolved(m)
    expect = 3 * p.cs * np.sign(jw) * np.sqrt(np.abs(jw))
    sel = np.abs(jw) > 0.3 * np.abs(jw).max()
    assert np.any(jw[sel] > 0) and np.any(jw[sel] < 0)
    got = taum - (3 * p.eta + 0.5)
    assert np.all(np.sign(got[sel]) == np.sign(jw[sel]))
    rel = np.abs(got - expect)[sel] / np.abs(expect[sel])
    assert rel.max() < 0.03, rel.max()
    assert np.all(taum > 0.5)          # eta = 0.01 is far above |eta_t|: nothing clipped


def test_backscatter_beyond_the_resistivity_is_clipped(orc):
    """A state evolved at eta = 0.01 (non-equilibrium well damped) collided
    with eta = 1e-4: where the backscatter C_S |j omega|^(1/2) exceeds 4 eta,
    tau_m = 1/2 exactly (zero total resistivity); where j omega > 0 well
    away from its zeros, tau_m > tau_m0; nowhere below 1/2.  (Along a run at
    eta = 1e-4 a clipped site relaxes g with s_m = 2, which mirrors its
    non-equilibrium part instead of damping it, so the current read from it
    alternates in sign; the comparison therefore uses one collision.)"""
    p = orc.Params(64, 64, nu=0.01, eta=0.01, les=4, cs=0.5)
    st = orc.run(p, orc.init(p, *_cellular_fields(p, 0.02, 0.02)), 60)
    q = orc.Params(64, 64, nu=0.01, eta=1e-4, les=4, cs=0.5)
    _, _, taum = orc.collide(q, st, return_tau=True)
    _, jw = _resolved(orc.macro(p, st))
    eta_t = q.cs * np.sign(jw) * np.sqrt(np.abs(jw))
    assert np.all(taum >= 0.5)
    strong = eta_t < -4 * q.eta
    assert strong.sum() > 100
    assert np.all(taum[strong] == 0.5)
    assert np.all(taum[eta_t > 4 * q.eta] > 3 * q.eta + 0.5)


def test_without_vorticity_there_is_no_eddy_resistivity(orc):
    """u = 0 initially and B_x = B_x(y): every field stays a function of y with
    u_x = 0, so omega vanishes identically and tau_m = tau_m0."""
    p = orc.Params(6, 64, nu=0.01, eta=0.02, les=4, cs=0.2)
    k = 2 * np.pi / p.ny
    y = np.arange(p.ny)[:, None] * np.ones((1, p.nx))
    st = orc.run(p, orc.init(p, 1.0, 0.0, 0.0, 0.02 * np.sin(k * y), 0.0), 50)
    _, _, taum = orc.collide(p, st, return_tau=True)
    np.testing.assert_allclose(taum, 3 * p.eta + 0.5, rtol=0, atol=1e-15)


@pytest.mark.parametrize("les,base", [(4, 0), (6, 2)])
def test_zero_constant_gives_the_closure_free_update(orc, les, base):
    p0 = orc.Params(9, 7, nu=0.01, eta=0.02, les=base, cs=0.0)
    p1 = orc.Params(9, 7, nu=0.01, eta=0.02, les=les, cs=0.0)
    st = _random_state(orc, p0, 8)
    np.testing.assert_allclose(orc.run(p1, st, 5), orc.run(p0, st, 5), rtol=0, atol=1e-15)


def test_relaxation_times_continuous_and_monotone_in_the_constant(orc):
    """tau grows with C_S (its cubic's root moves right as q grows); tau_m
    moves away from tau_m0 in the direction of sgn(j omega), stopping at 1/2;
    the roots stay smooth across the switch between the trigonometric and
    Cardano forms."""
    p = orc.Params(8, 8, nu=0.01, eta=0.3, les=4, cs=0.0)
    st = _random_state(orc, p, 4, amp=5e-3)
    cs_grid = np.linspace(0.0, 60.0, 241)
    taus, taums = [], []
    for cs in cs_grid:
        q = orc.Params(8, 8, nu=0.01, eta=0.3, les=4, cs=cs)
        _, tau, taum = orc.collide(q, st, return_tau=True)
        taus.append(tau)
        taums.append(taum)
    taus, taums = np.array(taus), np.array(taums)
    assert np.all(np.diff(taus, axis=0) >= 0)
    assert np.all(taums >= 0.5)
    up = taums[-1] > taums[0]
    assert np.all(np.diff(taums[:, up], axis=0) >= 0)
    assert np.all(np.diff(taums[:, ~up], axis=0) <= 0)
    assert np.any(taums == 0.5) and up.sum() > 8
    # Where j omega > 0 nothing is clipped and tau, tau_m are smooth in C_S;
    # there the largest eddy part crosses the switch q = 2 (tau0/3)^(3/2)
    # between the two root formulas without a jump in the increments.
    t0 = 3 * p.nu + 0.5
    tu = taus[:, up]
    q = tu[-1] ** 1.5 - t0 * tu[-1] ** 0.5
    assert q.max() > 2 * (t0 / 3) ** 1.5
    for a in (tu, taums[:, up]):
        d1 = np.diff(a, axis=0)
        d2 = np.abs(np.diff(d1, axis=0))
        assert np.all(d2 <= 0.1 * np.abs(d1[1:]) + 1e-12)


@pytest.mark.parametrize("les", [4, 6])
def test_conservation(orc, les):
    p = orc.Params(12, 10, nu=0.02, eta=0.02, les=les, cs=0.2)
    st = _random_state(orc, p, 31, amp=3e-3)
    m0 = orc.macro(p, st)
    m1 = orc.macro(p, orc.run(p, st, 20))
    for key in ("rho",):
        assert abs(m1[key].sum() - m0[key].sum()) < 1e-12
    for key in ("bx", "by"):
        assert abs(m1[key].sum() - m0[key].sum()) < 1e-13
    for a in ("ux", "uy"):
        j0 = (m0["rho"] * m0[a]).sum()
        j1 = (m1["rho"] * m1[a]).sum()
        assert abs(j1 - j0) < 1e-13


@pytest.mark.parametrize("les", [4, 6])
@pytest.mark.parametrize("op", [_rotate, _mirror_x])
def test_update_commutes_with_lattice_symmetries(orc, op, les):
    """Under a mirror j and omega both change sign, so j . omega and the
    closure are unchanged; the update commutes with the lattice symmetries."""
    p = orc.Params(8, 8, nu=0.02, eta=0.01, s5=1.3, s6=1.3, s7=1.1, s8=0.7, les=les, cs=0.2)
    st = _random_state(orc, p, 21, amp=3e-3)
    a = op(orc.run(p, st, 3))
    b = orc.run(p, op(st), 3)
    np.testing.assert_allclose(a, b, atol=1e-15)
