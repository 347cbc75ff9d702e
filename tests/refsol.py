"""Deterministic reference solutions used to pin the oracle (test infrastructure).

These solve the linearized, steady, one-dimensional Boltzmann equation in the
relaxation-time approximation by independent means (integral equations in
exponential-integral kernels, solved by product-integration Nystrom), not by
Monte Carlo.  They know nothing of the oracle's code.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import expn


def _E(n, x):
    return expn(n, np.maximum(x, 0.0))


def gray_slab(sL: float, dT1: float = 0.5, dT2: float = -0.5, M: int = 1600, n_bins: int = 20):
    """Gray slab of optical thickness sL between black (isothermal) walls.

    Unknown: the emissive temperature T(s) (equal to the energy temperature
    for a gray medium) on M uniform cells; the integral equation

        T(s) = 1/2 [dT1 E2(s) + dT2 E2(sL - s)] + 1/2 int_0^sL T(s') E1(|s - s'|) ds'

    is collocated at cell centres with the kernel integrated exactly over each
    cell (cell integrals of E1 are differences of E2).  Returns
    (bin averages of T over n_bins bins, Psi = q / (C v (dT1 - dT2) / 4)).
    """
    edges = np.linspace(0.0, sL, M + 1)
    s = 0.5 * (edges[1:] + edges[:-1])
    a = edges[None, :-1]
    b = edges[None, 1:]
    x = s[:, None]
    # int_a^b E1(|x - s'|) ds'
    left = _E(2, x - b) - _E(2, x - a)  # cells entirely below x: int E1(x - s') = E2(x-b) - E2(x-a)
    right = _E(2, a - x) - _E(2, b - x)  # cells entirely above x
    inside = (1.0 - _E(2, x - a)) + (1.0 - _E(2, b - x))
    Kmat = np.where(b <= x, left, np.where(a >= x, right, inside))
    rhs = 0.5 * (dT1 * _E(2, s) + dT2 * _E(2, sL - s))
    A = np.eye(M) - 0.5 * Kmat
    T = np.linalg.solve(A, rhs)
    # heat flux at s = 0: (Cv/2)[dT1 E3(0) - dT2 E3(sL) - int_0^sL T E2(s') ds'] ; E3(0) = 1/2
    integ = np.sum(T * (_E(3, edges[:-1]) - _E(3, edges[1:])))
    q = 0.5 * (dT1 * 0.5 - dT2 * _E(3, sL) - integ)
    psi = q / ((dT1 - dT2) / 4.0)
    per = M // n_bins
    bins = T[: per * n_bins].reshape(n_bins, per).mean(axis=1)
    return bins, float(psi)


def gray_slab_richardson(sL: float, n_bins: int = 20, M: int = 1600):
    """Two-grid Richardson extrapolation (second order) of ``gray_slab``."""
    b1, p1 = gray_slab(sL, M=M, n_bins=n_bins)
    b2, p2 = gray_slab(sL, M=2 * M, n_bins=n_bins)
    return (4 * b2 - b1) / 3.0, (4 * p2 - p1) / 3.0


def milne_psi(sL: float, z0: float = 0.7104) -> float:
    """Diffusion limit of the gray-slab transmission with the Milne extrapolation length."""
    return (4.0 / 3.0) / (sL + 2.0 * z0)


def fuchs_sondheimer_S(delta, p: float, n: int = 4000):
    """In-plane conductivity reduction of a film of thickness delta mean free paths with
    specularity p:  S = 1 - 3(1-p)/(2 delta) int_0^1 (mu - mu^3)(1 - e^{-delta/mu}) /
    (1 - p e^{-delta/mu}) d mu   (Gauss-Legendre on [0, 1]).  ``delta`` may be an array."""
    x, w = np.polynomial.legendre.leggauss(n)
    mu = 0.5 * (x + 1.0)
    w = 0.5 * w
    d = np.atleast_1d(np.asarray(delta, dtype=np.float64))[:, None]
    e = np.exp(-d / mu[None, :])
    integ = np.sum(w * (mu - mu ** 3) * (1.0 - e) / (1.0 - p * e), axis=1)
    S = 1.0 - 3.0 * (1.0 - p) / (2.0 * d[:, 0]) * integ
    return float(S[0]) if np.ndim(delta) == 0 else S
