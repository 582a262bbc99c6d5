"""Pins of the oracle's update against what the paper and the mathematics fix.

Flint & Vahala, arXiv:1607.08675:
* collision invariants (Sec. 3, after eq. MagMomentEq's preamble; eq. Density);
* single-relaxation limit: equal rates give the BGK update of Sec. 1.2;
* transport coefficients (Sec. 4.3): nu = 1/(3 s_3) - 1/6, eta = 1/(3 s_m) - 1/6,
  xi = -1/9 - 1/(9 s_4) - 1/(15 s_7) + 2/(5 s_8), p = rho / 3 -- checked as
  decay rates, sound speed and sound damping of linear waves of the filtered
  MHD equations (eqs. FinalMomentum, FinalMagnetic at Delta = 0);
* MHD coupling: Alfven waves at v_A = B0 / sqrt(rho); advection by a uniform
  flow (streaming direction and the sign of the u x B terms);
* div B (Sec. 1.2, eq. Density): exact to roundoff when tau_m = 1, otherwise a
  second-order truncation error;
* Smagorinsky closures (eqs. SmagorinskyClosure, SmagorinskyMHDClosureB): the
  per-site relaxation times carry nu + C_S Delta^2 |S| and eta + C_S Delta^2 |j|
  with |S| and |j| of the resolved fields;
* brute force: an independent numpy transcription (printed matrices,
  numpy.linalg.inv, numpy.roll) on 8x8 lattices;
* symmetry: the lattice update commutes with 90-degree rotations and mirrors.
"""
import numpy as np
import pytest
from scipy.optimize import curve_fit

from lbmhd_inputs import orszag_tang, random_fields, random_planes


def _proj(a, k, c):
    return 2 * np.mean(a * np.sin(k * c)), 2 * np.mean(a * np.cos(k * c))


def _random_state(orc, p, seed, amp=1e-3):
    st = orc.init(p, *random_fields(p.nx, p.ny, seed))
    return st + random_planes(19, p.nx, p.ny, seed + 100, np.zeros(19), np.full(19, amp))


# ----------------------------------------------------------------- invariants
@pytest.mark.parametrize("les", [False, True])
def test_conservation(orc, les):
    p = orc.Params(12, 10, nu=0.01, eta=0.02, s5=1.1, s6=1.1, s7=1.3, s8=0.9, les=les, cs=0.2)
    st = _random_state(orc, p, 3)
    d0 = orc.diag(p, st)
    st = orc.run(p, st, 200)
    d1 = orc.diag(p, st)
    assert abs(d1["mass"] - d0["mass"]) < 1e-13 * d0["mass"]
    for k in ("mom_x", "mom_y", "flux_x", "flux_y"):
        assert abs(d1[k] - d0[k]) < 1e-14 * p.nx * p.ny, k


def test_uniform_state_is_fixed_point(orc):
    p = orc.Params(6, 5, les=True, cs=0.3)
    st = orc.init(p, 1.1, 0.04, -0.03, 0.05, 0.02)
    np.testing.assert_allclose(orc.run(p, st, 20), st, atol=2e-16)


def test_equal_rates_reduce_to_bgk(orc):
    """All rates equal 1/tau: the MRT collision is f - (f - f^eq) / tau."""
    tau = 0.8
    nu = (tau - 0.5) / 3
    p = orc.Params(7, 6, nu=nu, eta=0.05, s5=1 / tau, s6=1 / tau, s7=1 / tau, s8=1 / tau)
    st = _random_state(orc, p, 11, amp=1e-2)
    m = orc.macro(p, st)
    out = orc.collide(p, st)
    for y in range(p.ny):
        for x in range(p.nx):
            feq, _ = orc.equilibrium(*(m[k][y, x] for k in ("rho", "ux", "uy", "bx", "by")))
            f = st[:9, y, x]
            np.testing.assert_allclose(out[:9, y, x], f - (f - feq) / tau, atol=2e-16)


def test_brute_force_agreement(orc):
    from oracle import brute
    p = orc.Params(8, 8, nu=0.01, eta=0.02, s5=1.2, s6=1.2, s7=1.5, s8=0.8, les=True, cs=0.1)
    st = _random_state(orc, p, 5)
    kw = dict(nu=p.nu, eta=p.eta, s5=p.s5, s6=p.s6, s7=p.s7, s8=p.s8, les=True, cs=p.cs)
    for n in (1, 10):
        np.testing.assert_allclose(orc.run(p, st, n), brute.run(st, n, **kw), rtol=0, atol=1e-13)


# ------------------------------------------------------------------ symmetry
def _rotate(st):
    """Rotate the lattice by +90 degrees: site (x, y) -> (-y, x), velocity
    (c_x, c_y) -> (-c_y, c_x), vector components (g_x, g_y) -> (-g_y, g_x)."""
    n = st.shape[1]
    out = np.empty_like(st)
    perm9 = {0: 0, 1: 2, 2: 3, 3: 4, 4: 1, 5: 6, 6: 7, 7: 8, 8: 5}
    perm5 = {0: 0, 1: 2, 2: 3, 3: 4, 4: 1}
    ys, xs = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    def rot_plane(a):
        b = np.empty_like(a)
        b[xs, (-ys) % n] = a[ys, xs]
        return b
    for i, j in perm9.items():
        out[j] = rot_plane(st[i])
    for k, j in perm5.items():
        out[9 + j] = -rot_plane(st[14 + k])
        out[14 + j] = rot_plane(st[9 + k])
    return out


def _mirror_x(st):
    out = np.empty_like(st)
    perm9 = {0: 0, 1: 3, 2: 2, 3: 1, 4: 4, 5: 6, 6: 5, 7: 8, 8: 7}
    perm5 = {0: 0, 1: 3, 2: 2, 3: 1, 4: 4}
    def mir(a):
        return np.roll(a[:, ::-1], 1, axis=1)  # x -> -x mod n
    for i, j in perm9.items():
        out[j] = mir(st[i])
    for k, j in perm5.items():
        out[9 + j] = -mir(st[9 + k])
        out[14 + j] = mir(st[14 + k])
    return out


@pytest.mark.parametrize("op", [_rotate, _mirror_x])
def test_update_commutes_with_lattice_symmetries(orc, op):
    p = orc.Params(8, 8, nu=0.02, eta=0.01, s5=1.3, s6=1.3, s7=1.1, s8=0.7, les=True, cs=0.2)
    st = _random_state(orc, p, 21, amp=3e-3)
    a = op(orc.run(p, st, 3))
    b = orc.run(p, op(st), 3)
    np.testing.assert_allclose(a, b, atol=1e-15)


# ------------------------------------------------------- transport coefficients
def _decay_rate(orc, p, field, key, k, coord, t0=200, t1=2200):
    st = orc.init(p, *field)
    st = orc.run(p, st, t0)
    a0 = _proj(orc.macro(p, st)[key], k, coord)[0]
    st = orc.run(p, st, t1 - t0)
    a1 = _proj(orc.macro(p, st)[key], k, coord)[0]
    return -np.log(a1 / a0) / (t1 - t0)


def test_shear_wave_decays_at_nu_k2(orc):
    """u_x = U sin(k y): amplitude decays at nu k^2 with nu = 1/(3 s_3) - 1/6."""
    ny, nx = 128, 4
    for nu, eta in ((0.01, 0.03), (0.002, 0.05)):
        p = orc.Params(nx, ny, nu=nu, eta=eta)
        y = np.arange(ny)[:, None] * np.ones((1, nx))
        k = 2 * np.pi / ny
        rate = _decay_rate(orc, p, (1.0, 1e-4 * np.sin(k * y), 0.0, 0.0, 0.0), "ux", k, y)
        assert abs(rate / (nu * k * k) - 1) < 4e-4, (nu, rate / (nu * k * k))


def test_magnetic_sine_decays_at_eta_k2(orc):
    """B_x = B0 sin(k y), u = 0: amplitude decays at eta k^2, eta = 1/(3 s_m) - 1/6."""
    ny, nx = 128, 4
    for nu, eta in ((0.02, 0.01), (0.05, 0.003)):
        p = orc.Params(nx, ny, nu=nu, eta=eta)
        y = np.arange(ny)[:, None] * np.ones((1, nx))
        k = 2 * np.pi / ny
        rate = _decay_rate(orc, p, (1.0, 0.0, 0.0, 1e-4 * np.sin(k * y), 0.0), "bx", k, y)
        assert abs(rate / (eta * k * k) - 1) < 4e-4, (eta, rate / (eta * k * k))


def _fit_wave(ts, a, G0, w0):
    f = lambda t, A, G, w, ph: A * np.exp(-G * t) * np.cos(w * t + ph)
    popt, _ = curve_fit(f, ts, a, p0=[1.0, G0, w0, 0.0])
    return popt[1], popt[2]


@pytest.mark.parametrize("s5,s7,s8", [(1.2, 1.6, 1.1), (1.0, 1.0, 1.0), (1.7, 0.8, 1.4)])
def test_sound_speed_and_bulk_damping(orc, s5, s7, s8):
    """Density wave: frequency c_s k with c_s^2 = 1/3 (p = rho/3) and damping
    (nu + xi + nu/3) k^2 / 2 with the paper's xi(s_4, s_7, s_8)."""
    ny, nx, nu, eps = 128, 4, 0.01, 1e-6
    p = orc.Params(nx, ny, nu=nu, eta=0.01, s5=s5, s6=s5, s7=s7, s8=s8)
    y = np.arange(ny)[:, None] * np.ones((1, nx))
    k = 2 * np.pi / ny
    st = orc.init(p, 1 + eps * np.sin(k * y), 0.0, 0.0, 0.0, 0.0)
    ts, a = [], []
    for t in range(0, 3000, 10):
        if t >= 100:
            ts.append(t)
            a.append(_proj(orc.macro(p, st)["rho"] - 1, k, y)[0] / eps)
        st = orc.run(p, st, 10)
    s4 = 1 / (3 * nu + 0.5)
    xi = -1 / 9 - 1 / (9 * s4) - 1 / (15 * s7) + 2 / (5 * s8)
    G0, w0 = 0.5 * (nu + xi + nu / 3) * k * k, k / np.sqrt(3)
    G, w = _fit_wave(np.array(ts), np.array(a), G0, w0)
    assert abs(w / w0 - 1) < 2e-4
    assert abs(G / G0 - 1) < 5e-4


def test_alfven_wave(orc):
    """k parallel to a uniform B0: frequency B0 k / sqrt(rho), damping
    (nu + eta) k^2 / 2 (an O(B0^2) lattice deficit is visible at B0 = 0.05)."""
    nx, ny, eps = 64, 4, 1e-6
    k = 2 * np.pi / nx
    x = np.ones((ny, 1)) * np.arange(nx)[None, :]
    for B0, T, tol_g in ((0.05, 3000, 1e-2), (0.02, 6000, 2e-3)):
        p = orc.Params(nx, ny, nu=0.01, eta=0.01)
        st = orc.init(p, 1.0, 0.0, 0.0, B0, eps * np.sin(k * x))
        ts, a = [], []
        for t in range(0, T, 10):
            if t >= 100:
                ts.append(t)
                a.append(_proj(orc.macro(p, st)["by"], k, x)[0] / eps)
            st = orc.run(p, st, 10)
        G0, w0 = 0.5 * (p.nu + p.eta) * k * k, B0 * k
        G, w = _fit_wave(np.array(ts), np.array(a), G0, w0)
        assert abs(w / w0 - 1) < 2e-4, (B0, w / w0)
        assert abs(G / G0 - 1) < tol_g, (B0, G / G0)


def test_advection_by_uniform_flow(orc):
    """u = (U, 0) carries a transverse velocity and field pattern to x + U t:
    fixes the streaming direction and the sign of the u x B terms of g^eq."""
    nx, ny, U, T, eps = 64, 4, 0.05, 400, 1e-6
    k = 2 * np.pi / nx
    x = np.ones((ny, 1)) * np.arange(nx)[None, :]
    p = orc.Params(nx, ny, nu=0.01, eta=0.01)
    st = orc.init(p, 1.0, U, eps * np.sin(k * x), 0.0, eps * np.sin(k * x))
    m = orc.macro(p, orc.run(p, st, T))
    for key in ("uy", "by"):
        s, c = _proj(m[key], k, x)
        phase = np.arctan2(-c, s)
        assert abs(phase - k * U * T) < 1e-3, (key, phase, k * U * T)


# ---------------------------------------------------------------------- div B
def test_divB_roundoff_when_tau_m_is_one(orc):
    p = orc.Params(64, 64, nu=0.01, eta=1 / 6)
    st = orc.init(p, *orszag_tang(64, 64))
    assert orc.diag(p, st)["max_abs_divB"] < 1e-16
    d = orc.diag(p, orc.run(p, st, 300))
    assert d["max_abs_divB"] < 1e-15


def test_divB_second_order_otherwise(orc):
    """tau_m != 1: div B is a truncation error falling 4x per grid doubling
    (diffusive scaling: N -> 2N, t -> 4t, amplitudes halved)."""
    eta = 0.1
    r = []
    for N, T, a in ((32, 100, 0.04), (64, 400, 0.02)):
        p = orc.Params(N, N, nu=eta, eta=eta)
        st = orc.run(p, orc.init(p, *orszag_tang(N, N, u0=a, b0=a)), T)
        r.append(orc.diag(p, st)["divB_over_curlB"])
    assert 3.5 < r[0] / r[1] < 4.5, r


# ------------------------------------------------------------------ LES closure
def test_les_with_zero_constant_is_the_plain_method(orc):
    p0 = orc.Params(9, 7, nu=0.01, eta=0.02, les=False)
    p1 = orc.Params(9, 7, nu=0.01, eta=0.02, les=True, cs=0.0)
    st = _random_state(orc, p0, 8)
    np.testing.assert_array_equal(orc.run(p0, st, 5), orc.run(p1, st, 5))


def test_les_relaxation_times_bounded_and_monotone(orc):
    st = None
    prev = None
    for cs in (0.0, 0.05, 0.1, 0.3):
        p = orc.Params(8, 8, nu=0.01, eta=0.02, les=True, cs=cs)
        if st is None:
            st = _random_state(orc, p, 4, amp=5e-3)
        _, tau, taum = orc.collide(p, st, return_tau=True)
        assert np.all(tau >= 3 * p.nu + 0.5 - 1e-15)
        assert np.all(taum >= 3 * p.eta + 0.5 - 1e-15)
        if prev is not None:
            assert np.all(tau >= prev[0]) and np.all(taum >= prev[1])
        prev = (tau, taum)


def test_les_eddy_viscosity_matches_resolved_strain(orc):
    """Shear flow u_x = U sin(k y): the closure's tau equals
    tau0 + 3 C_S Delta^2 |S| with |S| = sqrt(2 S:S) = |d u_x / d y| of the
    resolved field (eq. SmagorinskyClosure with the Sec. 1.2 strain relation)."""
    ny, nx, U, cs = 128, 4, 0.01, 0.1
    p = orc.Params(nx, ny, nu=0.01, eta=0.01, les=True, cs=cs)
    k = 2 * np.pi / ny
    y = np.arange(ny)[:, None] * np.ones((1, nx))
    st = orc.run(p, orc.init(p, 1.0, U * np.sin(k * y), 0.0, 0.0, 0.0), 100)
    m = orc.macro(p, st)
    ux = m["ux"]
    dudy = 0.5 * (np.roll(ux, -1, 0) - np.roll(ux, 1, 0))
    _, tau, _ = orc.collide(p, st, return_tau=True)
    expect = 3 * p.nu + 0.5 + 3 * cs * np.abs(dudy)
    sel = np.abs(dudy) > 0.3 * np.abs(dudy).max()
    rel = np.abs((tau - expect)[sel]) / (3 * cs * np.abs(dudy[sel]))
    assert rel.max() < 0.02, rel.max()


def test_les_eddy_resistivity_matches_resolved_current(orc):
    """B_x = B0 sin(k y), u = 0: tau_m = tau_m0 + 3 C_S Delta^2 |j| with
    j = d_x B_y - d_y B_x of the resolved field (eq. SmagorinskyMHDClosureB)."""
    ny, nx, B0, cs = 128, 4, 0.01, 0.1
    p = orc.Params(nx, ny, nu=0.01, eta=0.01, les=True, cs=cs)
    k = 2 * np.pi / ny
    y = np.arange(ny)[:, None] * np.ones((1, nx))
    st = orc.run(p, orc.init(p, 1.0, 0.0, 0.0, B0 * np.sin(k * y), 0.0), 100)
    bx = orc.macro(p, st)["bx"]
    j = -0.5 * (np.roll(bx, -1, 0) - np.roll(bx, 1, 0))
    _, _, taum = orc.collide(p, st, return_tau=True)
    expect = 3 * p.eta + 0.5 + 3 * cs * np.abs(j)
    sel = np.abs(j) > 0.3 * np.abs(j).max()
    rel = np.abs((taum - expect)[sel]) / (3 * cs * np.abs(j[sel]))
    assert rel.max() < 0.02, rel.max()


def test_les_relaxation_time_solves_its_quadratic(orc):
    """Self-consistency reading: tau = tau0 + 3 C_S Delta^2 |S| with |S| from
    the non-equilibrium M3, M4 relaxed with that same tau."""
    p = orc.Params(8, 8, nu=0.01, eta=0.02, les=True, cs=0.15, delta=1.3)
    st = _random_state(orc, p, 9, amp=5e-3)
    T, _, Tm = orc.matrices()
    m = orc.macro(p, st)
    _, tau, taum = orc.collide(p, st, return_tau=True)
    for y in range(p.ny):
        for x in range(p.nx):
            rho, ux, uy, bx, by = (m[k][y, x] for k in ("rho", "ux", "uy", "bx", "by"))
            feq, geq = orc.equilibrium(rho, ux, uy, bx, by)
            dM = T @ (st[:9, y, x] - feq)
            S = 3 / (2 * rho * tau[y, x]) * np.hypot(dM[4], 2 * dM[3])
            assert abs(tau[y, x] - (3 * p.nu + 0.5 + 3 * p.cs * p.delta ** 2 * S)) < 1e-14
            dN = Tm @ (st[9:].reshape(2, 5, p.ny, p.nx)[:, :, y, x] - geq).T
            jz = -3 / taum[y, x] * (dN[1, 1] - dN[2, 0])
            assert abs(taum[y, x] - (3 * p.eta + 0.5 + 3 * p.cs * p.delta ** 2 * abs(jz))) < 1e-14


# ------------------------------------------------------------- tangent-linear
def test_tangent_matches_central_differences(orc):
    from lbmhd_inputs import directions
    n, steps = 12, 15
    p = orc.Params(n, n, nu=0.01, eta=0.01, les=True, cs=0.1)
    fields = orszag_tang(n, n, u0=0.08, b0=0.08)
    d, dcs = directions(3, n, n, 100, 0.05, 0.05, 0.1)
    J, dJ = orc.tl_energy(p, fields, d, dcs, steps)
    eps = 1e-5
    for k in range(3):
        Js = []
        for sgn in (1, -1):
            f = list(fields)
            for c in range(4):
                f[1 + c] = fields[1 + c] + sgn * eps * d[k, c]
            q = orc.Params(n, n, nu=0.01, eta=0.01, les=True, cs=p.cs + sgn * eps * dcs[k])
            Js.append(orc.energy(q, orc.run(q, orc.init(q, *f), steps)))
        fd = (Js[0] - Js[1]) / (2 * eps)
        assert abs(fd - dJ[k]) < 1e-7 * abs(dJ[k]) + 1e-12, (k, fd, dJ[k])
    assert abs(J - orc.energy(p, orc.run(p, orc.init(p, *fields), steps))) < 1e-13


@pytest.mark.parametrize("les", [1, 4])
def test_each_constant_drives_its_own_rate(orc, les):
    """Eqs. SmagorinskyMHDClosureV/B (and CHClosureV/B): C_Sv sets the eddy
    viscosity, C_Sb the eddy resistivity.  With one of them zero its
    relaxation time is the molecular one, and the other matches the run
    with both constants equal."""
    p = orc.Params(10, 8, nu=0.01, eta=0.02, les=les, cs=0.2)
    st = _random_state(orc, p, 6, amp=5e-3)
    _, tau, taum = orc.collide(p, st, return_tau=True)
    _, tv, tmv = orc.collide(orc.Params(10, 8, nu=0.01, eta=0.02, les=les, cs=0.2, csb=0.0), st,
                             return_tau=True)
    _, tb, tmb = orc.collide(orc.Params(10, 8, nu=0.01, eta=0.02, les=les, cs=0.0, csb=0.2), st,
                             return_tau=True)
    np.testing.assert_allclose(tmv, 3 * p.eta + 0.5, rtol=0, atol=1e-15)
    np.testing.assert_allclose(tb, 3 * p.nu + 0.5, rtol=0, atol=1e-15)
    np.testing.assert_allclose(tmb, taum, rtol=0, atol=1e-15)
    if les == 1:   # the Smagorinsky fluid rate does not depend on tau_m
        np.testing.assert_allclose(tv, tau, rtol=0, atol=1e-15)
    assert np.all(tv > 3 * p.nu + 0.5) and np.all(np.abs(tmb - (3 * p.eta + 0.5)) > 0)


def test_tangent_splits_over_the_two_constants(orc):
    """d/dC_Sv + d/dC_Sb = d/dC_S (both moving), each against central
    differences in its own constant."""
    n, steps = 10, 12
    p = orc.Params(n, n, nu=0.01, eta=0.01, les=1, cs=0.1, csb=0.15)
    fields = orszag_tang(n, n, u0=0.08, b0=0.08)
    d = np.zeros((3, 4, n, n))
    J, dJ = orc.tl_energy(p, fields, d, np.array([[1.0, 0.0], [0.0, 1.0], [1.0, 1.0]]), steps)
    assert abs(dJ[0] + dJ[1] - dJ[2]) < 1e-12 * abs(dJ[2])
    eps = 1e-5
    for k, key in ((0, "cs"), (1, "csb")):
        Js = []
        for sgn in (1, -1):
            kw = dict(cs=p.cs, csb=p.csb)
            kw[key] += sgn * eps
            q = orc.Params(n, n, nu=0.01, eta=0.01, les=1, **kw)
            Js.append(orc.energy(q, orc.run(q, orc.init(q, *fields), steps)))
        fd = (Js[0] - Js[1]) / (2 * eps)
        assert abs(fd - dJ[k]) < 1e-6 * abs(dJ[k]) + 1e-12, (key, fd, dJ[k])
        assert abs(dJ[k]) > 1e-6


def test_tangent_collide_is_linear_in_direction(orc):
    p = orc.Params(6, 6, nu=0.01, eta=0.02, les=True, cs=0.2)
    st = _random_state(orc, p, 2, amp=3e-3)
    rng = np.random.default_rng(0)
    d = rng.standard_normal((2, 19, 6, 6))
    _, t = orc.tl_collide(p, st, np.stack([d[0], d[1], d[0] + 2 * d[1]]), np.array([0.3, 0.0, 0.3]))
    np.testing.assert_allclose(t[2], t[0] + 2 * t[1], atol=1e-14)
