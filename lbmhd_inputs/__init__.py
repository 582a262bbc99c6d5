"""Seeded synthetic inputs shared by the GPU library's tests/benchmark and the oracle.

This module produces macroscopic initial fields and random arrays only.  It
holds none of the lattice Boltzmann method's arithmetic (no equilibria, no
moments, no weights): whatever a caller needs of the method it computes on its
own side.  All arrays are float64 with shape (ny, nx), x fastest, on the grid
x_i = 2 pi i / nx, y_j = 2 pi j / ny.
"""
from __future__ import annotations

import numpy as np


def grid(nx: int, ny: int):
    """Node coordinates on [0, 2 pi)^2: x_i = 2 pi i / nx, y_j = 2 pi j / ny."""
    x = 2.0 * np.pi * np.arange(nx) / nx
    y = 2.0 * np.pi * np.arange(ny) / ny
    return np.meshgrid(x, y, indexing="xy")


def orszag_tang(nx: int, ny: int, u0: float = 0.05, b0: float = 0.05):
    """Orszag-Tang vortex: rho = 1, u = u0 (-sin y, sin x), B = b0 (-sin y, sin 2x).

    B_x depends on y only and B_y on x only, so the centred discrete
    divergence of B is exactly zero.
    """
    X, Y = grid(nx, ny)
    rho = np.ones((ny, nx))
    ux = -u0 * np.sin(Y)
    uy = u0 * np.sin(X)
    bx = -b0 * np.sin(Y)
    by = b0 * np.sin(2.0 * X)
    return rho, ux, uy, bx, by


def _centred(a: np.ndarray, axis: int) -> np.ndarray:
    return 0.5 * (np.roll(a, -1, axis=axis) - np.roll(a, 1, axis=axis))


def _potential(n_x: int, n_y: int, seed: int, kmax: int, kpeak: float) -> np.ndarray:
    """Random-phase scalar potential with |phi_k| ~ sqrt(E(k) / (pi k)) / k,
    E(k) = k^4 exp(-(k / kpeak)^2), drawn on a fixed |k| <= kmax grid so the
    same realisation is reproduced at every lattice size (modes the lattice
    cannot hold are dropped)."""
    rng = np.random.default_rng(seed)
    m = 2 * kmax + 1
    phase = rng.uniform(0.0, 2.0 * np.pi, size=(m, m))
    k1 = np.arange(-kmax, kmax + 1)
    KX, KY = np.meshgrid(k1, k1, indexing="xy")
    K = np.sqrt(KX ** 2 + KY ** 2)
    amp = np.zeros_like(K)
    nz = (K > 0) & (K <= kmax)
    E = K[nz] ** 4 * np.exp(-(K[nz] / kpeak) ** 2)
    amp[nz] = np.sqrt(E / (np.pi * K[nz])) / K[nz]
    keep = (np.abs(KX) < n_x // 2) & (np.abs(KY) < n_y // 2) & nz
    spec = np.zeros((n_y, n_x), dtype=np.complex128)
    spec[KY[keep] % n_y, KX[keep] % n_x] = amp[keep] * np.exp(1j * phase[keep])
    return np.real(np.fft.ifft2(spec)) * (n_x * n_y)


def solenoidal(nx: int, ny: int, seed: int, rms: float, kmax: int = 64, kpeak: float = 8.0):
    """Divergence-free 2D vector field (a_x, a_y) = (d_y phi, -d_x phi), with
    centred differences, rescaled so sqrt(<a_x^2 + a_y^2>) = rms."""
    phi = _potential(nx, ny, seed, kmax, kpeak)
    ax = _centred(phi, axis=0)
    ay = -_centred(phi, axis=1)
    norm = np.sqrt(np.mean(ax ** 2 + ay ** 2))
    return ax * (rms / norm), ay * (rms / norm)


def decaying_turbulence(nx: int, ny: int, seed_u: int = 1, seed_b: int = 2,
                        u_rms: float = 0.04, b_rms: float = 0.04):
    """Decaying 2D MHD turbulence: rho = 1, u and B solenoidal from seeded
    random-phase stream and flux functions with E(k) ~ k^4 exp(-(k/8)^2)."""
    ux, uy = solenoidal(nx, ny, seed_u, u_rms)
    bx, by = solenoidal(nx, ny, seed_b, b_rms)
    return np.ones((ny, nx)), ux, uy, bx, by


def perturbed_orszag_tang(nx: int, ny: int, seed_u: int = 3, seed_b: int = 4,
                          rel: float = 0.01, u0: float = 0.05, b0: float = 0.05):
    """Orszag-Tang plus a seeded solenoidal perturbation of rms rel * u0 (rel * b0)."""
    rho, ux, uy, bx, by = orszag_tang(nx, ny, u0, b0)
    dux, duy = solenoidal(nx, ny, seed_u, rel * u0)
    dbx, dby = solenoidal(nx, ny, seed_b, rel * b0)
    return rho, ux + dux, uy + duy, bx + dbx, by + dby


def random_planes(nplanes: int, nx: int, ny: int, seed: int, mean, scale) -> np.ndarray:
    """Array (nplanes, ny, nx) with plane q = mean[q] + scale[q] * N(0, 1)."""
    rng = np.random.default_rng(seed)
    mean = np.asarray(mean, dtype=np.float64).reshape(nplanes, 1, 1)
    scale = np.asarray(scale, dtype=np.float64).reshape(nplanes, 1, 1)
    return mean + scale * rng.standard_normal((nplanes, ny, nx))


def random_fields(nx: int, ny: int, seed: int, rho_amp: float = 0.01, u_amp: float = 0.03,
                  b_amp: float = 0.03):
    """Uncorrelated random macroscopic fields (rho near 1) for tiny-lattice tests."""
    rng = np.random.default_rng(seed)
    rho = 1.0 + rho_amp * rng.standard_normal((ny, nx))
    ux, uy, bx, by = (a * rng.standard_normal((ny, nx)) for a in (u_amp, u_amp, b_amp, b_amp))
    return rho, ux, uy, bx, by


def directions(ndir: int, nx: int, ny: int, seed0: int, rms_u: float, rms_b: float,
               cs_scale: float):
    """ndir seeded perturbation directions: solenoidal (du, dB) with the given
    rms and a C_S tangent cs_scale * N(0, 1).  Returns (dfields (ndir, 4, ny, nx),
    dcs (ndir,))."""
    d = np.zeros((ndir, 4, ny, nx))
    dcs = np.zeros(ndir)
    for k in range(ndir):
        s = seed0 + k
        d[k, 0], d[k, 1] = solenoidal(nx, ny, 2 * s, rms_u, kmax=min(64, nx // 2 - 1))
        d[k, 2], d[k, 3] = solenoidal(nx, ny, 2 * s + 1, rms_b, kmax=min(64, nx // 2 - 1))
        dcs[k] = cs_scale * np.random.default_rng(s).standard_normal()
    return d, dcs


def orszag_tang_3d(nx: int, ny: int, nz: int, u0: float = 0.05, b0: float = 0.05):
    """A 3D Orszag-Tang-type vortex on the nodes of [0, 2 pi)^3, arrays [z][y][x]:
    rho = 1, u = u0 (-sin y + 0.2 sin z, sin x + 0.2 sin z, 0.2 (sin x + sin y)),
    B = b0 (-sin y + 0.5 sin z, sin 2x + 0.5 sin z, 0.5 (sin x + sin y)).
    Each component is independent of its own coordinate, so the centred
    discrete divergence of u and of B is exactly zero."""
    z, y, x = np.meshgrid(2 * np.pi * np.arange(nz) / nz, 2 * np.pi * np.arange(ny) / ny,
                          2 * np.pi * np.arange(nx) / nx, indexing="ij")
    rho = np.ones_like(x)
    ux = u0 * (-np.sin(y) + 0.2 * np.sin(z))
    uy = u0 * (np.sin(x) + 0.2 * np.sin(z))
    uz = u0 * 0.2 * (np.sin(x) + np.sin(y))
    bx = b0 * (-np.sin(y) + 0.5 * np.sin(z))
    by = b0 * (np.sin(2 * x) + 0.5 * np.sin(z))
    bz = b0 * 0.5 * (np.sin(x) + np.sin(y))
    return rho, ux, uy, uz, bx, by, bz
