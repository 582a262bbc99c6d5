"""Brute-force numpy cross-check of the C oracle (TEST INFRASTRUCTURE ONLY).

A second, independently written transcription of the same update, used only
on tiny lattices: it takes the 9x9 matrix T and the 5x5 matrix T_m exactly as
printed (Sec. 3, eqs. FluidTMatrix and MagTMatrix), inverts T with
``numpy.linalg.inv``, builds the equilibria in distribution space (Sec. 3, the
D2Q9 and D2Q5 relaxation distributions), relaxes the full moment vector
M* = M - S (M - T f^eq) with S = diag(s_i), and streams with ``numpy.roll``.
The Smagorinsky-MHD closure enters as in the C oracle: per-site relaxation
times from the non-equilibrium moments T f - T f^eq and T_m g - T_m g^eq.
"""
from __future__ import annotations

import numpy as np

# Eq. FluidTMatrix, as printed.
T_PRINTED = np.array([
    [1, 1, 1, 1, 1, 1, 1, 1, 1],
    [0, 1, 0, -1, 0, 1, -1, -1, 1],
    [0, 0, 1, 0, -1, 1, 1, -1, -1],
    [0, 0, 0, 0, 0, 1, -1, 1, -1],
    [0, 1, -1, 1, -1, 0, 0, 0, 0],
    [0, -2, 0, 2, 0, 1, -1, -1, 1],
    [0, 0, -2, 0, 2, 1, 1, -1, -1],
    [4, -5, -5, -5, -5, 4, 4, 4, 4],
    [4, 0, 0, 0, 0, -1, -1, -1, -1],
], dtype=np.float64)

# Eq. MagTMatrix, as printed.
TM_PRINTED = np.array([
    [1, 1, 1, 1, 1],
    [0, 1, 0, -1, 0],
    [0, 0, 1, 0, -1],
    [0, 1, 0, 1, 0],
    [0, 0, 1, 0, 1],
], dtype=np.float64)

CX = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1], dtype=np.float64)
CY = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1], dtype=np.float64)
MCX = np.array([0, 1, 0, -1, 0], dtype=np.float64)
MCY = np.array([0, 0, 1, 0, -1], dtype=np.float64)
W9 = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)
W5 = np.array([1 / 3] + [1 / 6] * 4)


def feq(rho, ux, uy, bx, by):
    cu = CX[:, None, None] * ux + CY[:, None, None] * uy
    cb = CX[:, None, None] * bx + CY[:, None, None] * by
    c2 = (CX ** 2 + CY ** 2)[:, None, None]
    u2, b2 = ux ** 2 + uy ** 2, bx ** 2 + by ** 2
    w = W9[:, None, None]
    return w * rho * (1 + 3 * cu + 4.5 * cu ** 2 - 1.5 * u2) + 4.5 * w * (0.5 * b2 * c2 - cb ** 2)


def geq(ux, uy, bx, by):
    cu = MCX[:, None, None] * ux + MCY[:, None, None] * uy
    cb = MCX[:, None, None] * bx + MCY[:, None, None] * by
    w = W5[:, None, None]
    gx = w * (bx + 3 * (cu * bx - cb * ux))
    gy = w * (by + 3 * (cu * by - cb * uy))
    return np.concatenate([gx, gy], axis=0)


def collide(state, nu, eta, s5, s6, s7, s8, les=False, cs=0.0, delta=1.0):
    f, g = state[:9], state[9:]
    rho = f.sum(0)
    ux = (CX[:, None, None] * f).sum(0) / rho
    uy = (CY[:, None, None] * f).sum(0) / rho
    bx, by = g[:5].sum(0), g[5:].sum(0)
    fe = feq(rho, ux, uy, bx, by)
    ge = geq(ux, uy, bx, by)
    M = np.einsum("ij,jyx->iyx", T_PRINTED, f)
    Me = np.einsum("ij,jyx->iyx", T_PRINTED, fe)
    tau0, taum0 = 3 * nu + 0.5, 3 * eta + 0.5
    if les:
        Q = np.sqrt((M[4] - Me[4]) ** 2 + 4 * (M[3] - Me[3]) ** 2)
        tau = 0.5 * (tau0 + np.sqrt(tau0 ** 2 + 18 * cs * delta ** 2 * Q / rho))
        N = np.einsum("ij,jyx->iyx", TM_PRINTED, g[:5]), np.einsum("ij,jyx->iyx", TM_PRINTED, g[5:])
        Ne = np.einsum("ij,jyx->iyx", TM_PRINTED, ge[:5]), np.einsum("ij,jyx->iyx", TM_PRINTED, ge[5:])
        A = (N[1][1] - Ne[1][1]) - (N[0][2] - Ne[0][2])
        taum = 0.5 * (taum0 + np.sqrt(taum0 ** 2 + 36 * cs * delta ** 2 * np.abs(A)))
    else:
        tau = np.full_like(rho, tau0)
        taum = np.full_like(rho, taum0)
    S = np.zeros((9,) + rho.shape)
    S[3] = S[4] = 1 / tau
    S[5], S[6], S[7], S[8] = s5, s6, s7, s8
    Mstar = M - S * (M - Me)
    fstar = np.einsum("ij,jyx->iyx", np.linalg.inv(T_PRINTED), Mstar)
    gstar = g - (g - ge) / taum
    return np.concatenate([fstar, gstar], axis=0)


def stream(state):
    out = np.empty_like(state)
    for i in range(9):
        out[i] = np.roll(state[i], shift=(int(CY[i]), int(CX[i])), axis=(0, 1))
    for a in range(2):
        for k in range(5):
            q = 9 + 5 * a + k
            out[q] = np.roll(state[q], shift=(int(MCY[k]), int(MCX[k])), axis=(0, 1))
    return out


def run(state, nsteps, **kw):
    st = np.array(state, dtype=np.float64, copy=True)
    for _ in range(nsteps):
        st = stream(collide(st, **kw))
    return st
