"""Closed forms used to pin the FP64 oracle.  TEST INFRASTRUCTURE ONLY.

Each function is a textbook or paper formula that does not go through the
oracle's step code:

* ``sphere_moments``     homogeneous radiating sphere, Sec. 4.2.2
                         (distribution function f(r, mu) and its moments
                         eqs. radsph_1 and radsph_2);
* ``monomial_average``   (1/4pi) int x^a y^b z^c dOmega, the continuous
                         integrals that a degree-p rule must reproduce
                         (Sec. 3.2.1, eq. sph-quad-cond);
* ``binomial_green``     n steps of pure streaming from a point source: the
                         trilinear pull of eq. (interp) is a product of three
                         independent two-point kernels, so its n-fold power is
                         a product of three binomial laws;
* ``diffusion_x_moments`` exact first and second x-moments of the energy for
                         pure isotropic scattering on an unbounded lattice,
                         obtained by propagating the per-direction moments
                         sum_x x^k I_i through one stream and one implicit
                         collision at a time.
"""
from __future__ import annotations

import math
from typing import Sequence, Tuple

import numpy as np


def _double_factorial(n: int) -> int:
    if n <= 0:
        return 1
    out = 1
    while n > 1:
        out *= n
        n -= 2
    return out


def monomial_average(a: int, b: int, c: int) -> float:
    """(1/4pi) int_{S^2} x^a y^b z^c dOmega."""
    if a % 2 or b % 2 or c % 2:
        return 0.0
    return (_double_factorial(a - 1) * _double_factorial(b - 1) * _double_factorial(c - 1)
            / _double_factorial(a + b + c + 1))


def sphere_distribution(r: float, mu: np.ndarray, R: float, kappa: float, b: float = 1.0):
    """f(r, mu) = b (1 - exp(-kappa s(r, mu))) of Sec. 4.2.2, with
    mu the cosine between the direction and the radial vector and b = eta/kappa."""
    mu = np.asarray(mu, dtype=np.float64)
    if r < R:
        g = np.sqrt(np.maximum(0.0, 1.0 - (r * r) / (R * R) * (1.0 - mu * mu)))
        s = r * mu + R * g
    else:
        mu0 = math.sqrt(max(0.0, 1.0 - R * R / (r * r)))
        g = np.sqrt(np.maximum(0.0, 1.0 - (r * r) / (R * R) * (1.0 - mu * mu)))
        s = np.where(mu > mu0, 2.0 * R * g, 0.0)
    return b * (1.0 - np.exp(-kappa * s))


def sphere_moments(r: float, R: float, kappa: float, b: float = 1.0) -> Tuple[float, float]:
    """E(r) = 1/2 int f dmu and F(r) = 1/2 int mu f dmu (eqs. radsph_1, radsph_2)."""
    from scipy.integrate import quad
    brk = []
    if r >= R and r > 0:
        brk = [math.sqrt(max(0.0, 1.0 - R * R / (r * r)))]
    fE = lambda m: float(sphere_distribution(r, np.array([m]), R, kappa, b)[0])
    fF = lambda m: m * fE(m)
    E = 0.5 * quad(fE, -1.0, 1.0, points=brk or None, limit=400, epsabs=1e-13, epsrel=1e-12)[0]
    F = 0.5 * quad(fF, -1.0, 1.0, points=brk or None, limit=400, epsabs=1e-13, epsrel=1e-12)[0]
    return E, F


def binomial_green(nsteps: int, n: Sequence[float], dt: float, dx: float,
                   shape: Tuple[int, int, int], origin: Tuple[int, int, int]) -> np.ndarray:
    """Field ``[z, y, x]`` after ``nsteps`` pure-streaming steps of a unit
    point source at ``origin = (z, y, x)`` along direction ``n``: along each
    axis the mass moves k cells in direction sgn(n^a) with probability
    Binomial(nsteps, dt |n^a| / dx).  ``shape`` must be large enough that
    nothing reaches the box edge."""
    from scipy.stats import binom
    out = np.ones(shape)
    axes = [(0, n[2]), (1, n[1]), (2, n[0])]
    for ax, comp in axes:
        p = dt * abs(comp) / dx
        sgn = -1 if comp < 0 else 1
        k = np.arange(shape[ax]) - origin[ax]
        pmf = np.where(sgn * k >= 0, binom.pmf(np.abs(k), nsteps, p), 0.0)
        if p == 0.0:
            pmf = (k == 0).astype(np.float64)
        sh = [1, 1, 1]
        sh[ax] = shape[ax]
        out = out * pmf.reshape(sh)
    return out


def diffusion_x_moments(nsteps: int, dirs: np.ndarray, w: np.ndarray, dt: float,
                        dx: float, kappa0: float, T: float, X1: float, X2: float
                        ) -> np.ndarray:
    """Exact (sum E, sum x E, sum x^2 E) after each step for pure isotropic
    scattering (kappa_a = eta = 0, lambda = 0, uniform kappa0) on an unbounded
    lattice, starting from an isotropic state I_i = w_i E0 with total T and
    x-moments X1, X2.

    Per direction the moments m_k = sum_x x^k I_i change under the two-point
    x pull (fraction p = dt |n^x| / dx taken from x - s) as
        m0 -> m0,  m1 -> m1 + p s m0,  m2 -> m2 + 2 p s m1 + p m0,
    (the y and z pulls leave x-moments alone), and under the implicit
    collision I_i -> c I*_i + (1 - c) w_i E* with c = 1 / (1 + dt kappa0).
    Returns an array ``(nsteps + 1, 3)``."""
    N = len(w)
    c = 1.0 / (1.0 + dt * kappa0)
    m0 = w * T
    m1 = w * X1
    m2 = w * X2
    out = np.zeros((nsteps + 1, 3))
    out[0] = (m0.sum(), m1.sum(), m2.sum())
    p = dt * np.abs(dirs[:, 0]) / dx
    s = np.where(dirs[:, 0] < 0, -1.0, 1.0)
    for k in range(nsteps):
        m2 = m2 + 2.0 * p * s * m1 + p * m0
        m1 = m1 + p * s * m0
        T0, T1, T2 = m0.sum(), m1.sum(), m2.sum()
        m0 = c * m0 + (1.0 - c) * w * T0
        m1 = c * m1 + (1.0 - c) * w * T1
        m2 = c * m2 + (1.0 - c) * w * T2
        out[k + 1] = (m0.sum(), m1.sum(), m2.sum())
    return out
