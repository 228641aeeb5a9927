"""Closed-form and boundary-value reference solutions from Sec. 3 of Liu & He.

TEST INFRASTRUCTURE ONLY (part of the oracle). Positions are in lattice
units with walls at y = 0 and y = L; lattice node j sits at y = j + 1/2.
"""
from __future__ import annotations

import numpy as np


def theta(phi, K, nu, J):
    """vartheta = sqrt(phi nu / (K nu_e)) with nu_e = J nu (after Eq. 24)."""
    return np.sqrt(phi * nu / (K * J * nu))


def brinkman_poiseuille(y, L, ax, phi, K, nu, J=1.0):
    """Eq. (23) with F_phi = 0, solved in closed form.

    The centreline value is Eq. (24), whose printed "cosh^-1" is the
    reciprocal 1/cosh (the only reading under which the profile vanishes on
    both walls):
        u(y) = (a K / nu) [1 - cosh(th (y - L/2)) / cosh(th L/2)].
    """
    th = theta(phi, K, nu, J)
    return ax * K / nu * (1.0 - np.cosh(th * (y - 0.5 * L)) / np.cosh(0.5 * th * L))


def poiseuille_u0(L, ax, phi, K, nu, J=1.0):
    """Eq. (24): centreline velocity of the Brinkman (F_phi = 0) profile."""
    th = theta(phi, K, nu, J)
    return ax * K / nu * (1.0 - 1.0 / np.cosh(0.5 * th * L))


def free_poiseuille(y, L, ax, nu, J=1.0):
    """phi = 1, K -> infinity: (nu_e) u'' + a = 0, u(0) = u(L) = 0."""
    return ax / (2.0 * J * nu) * y * (L - y)


def porous_couette(y, L, u0, phi, K, nu, J=1.0):
    """Eq. (23) with a_x = 0 and F_phi = 0, u(0) = 0, u(L) = u0 (Sec. 3.2)."""
    th = theta(phi, K, nu, J)
    return u0 * np.sinh(th * y) / np.sinh(th * L)


def partial_couette(y, L, u0, phi, Da, J=1.0):
    """Eq. (25): Couette flow over a porous layer filling 0 <= y <= L/2 (Brinkman
    model, F_phi = 0) under free fluid (phi = 1, nu_e = nu) up to the lid y = L.

    In the layer u'' = (phi / (J Da)) u in y/L, so u = d0 sinh(th y/L)/sinh(th/2)
    with th = sqrt(phi / (J Da)) (the paper's vartheta with K = Da L^2 and
    nu_e = J nu); above it u is linear. Continuity of u and of the viscous flux
    nu_e du/dy at y = L/2 and u(L) = u0 fix
        d1 = J th coth(th/2) d0,   d0 = u0 / (1 + J th coth(th/2) / 2).
    The printed d0 and d1 are the limit coth -> 1 of a layer many times thicker
    than sqrt(J Da / phi) L; this finite-layer form is exact for the setup.
    """
    th = np.sqrt(phi / (J * Da))
    ct = 1.0 / np.tanh(0.5 * th)
    d0 = u0 / (1.0 + 0.5 * J * th * ct)
    d1 = J * th * ct * d0
    yh = np.asarray(y, dtype=np.float64) / L
    return np.where(yh > 0.5, d0 + d1 * (yh - 0.5), d0 * np.sinh(th * yh) / np.sinh(0.5 * th))


def _cheb(n):
    """Chebyshev differentiation matrix and points on [-1, 1] (Trefethen, 'Spectral
    Methods in MATLAB', program cheb)."""
    x = np.cos(np.pi * np.arange(n + 1) / n)
    c = np.ones(n + 1); c[0] = c[-1] = 2.0
    c *= (-1.0) ** np.arange(n + 1)
    X = np.tile(x, (n + 1, 1)).T
    dX = X - X.T
    D = np.outer(c, 1.0 / c) / (dX + np.eye(n + 1))
    D -= np.diag(D.sum(axis=1))
    return D, x


def bf_poiseuille(y, L, ax, phi, K, nu, Fphi, J=1.0, n=96):
    """Eq. (23), Brinkman-Forchheimer channel flow, by Chebyshev collocation and
    Newton iteration (converged to round-off); evaluated at the points y.

        (nu_e/phi) u'' - (nu/K) u - (F_phi/sqrt K) u^2 + a = 0,  u(0) = u(L) = 0.
    """
    D, xc = _cheb(n)
    s = 2.0 / L                      # d/dy = s d/dx for y = (x + 1) L / 2
    D2 = (s * s) * (D @ D)
    yc = (xc + 1.0) * 0.5 * L
    nu_e = J * nu
    u = brinkman_poiseuille(yc, L, ax, phi, K, nu, J)
    inner = slice(1, n)
    for _ in range(50):
        R = nu_e / phi * (D2 @ u) - nu / K * u - Fphi / np.sqrt(K) * u * u + ax
        Jm = nu_e / phi * D2 - np.diag(nu / K + 2.0 * Fphi / np.sqrt(K) * u)
        du = np.zeros_like(u)
        du[inner] = np.linalg.solve(Jm[inner, inner], -R[inner])
        u = u + du
        if np.max(np.abs(du)) <= 1e-15 * max(np.max(np.abs(u)), 1e-300):
            break
    # exact polynomial interpolant through the collocation values
    coef = np.polynomial.chebyshev.chebfit(xc, u, n)
    return np.polynomial.chebyshev.chebval(2.0 * np.asarray(y) / L - 1.0, coef)
