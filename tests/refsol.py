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


# --------------------------------------------------------------------------
# Frequency-dependent slab: the pseudo-temperature integral equation
# --------------------------------------------------------------------------


def _H(u, lam):
    """Second antiderivative of E1(|u| / lam) / lam that is smooth at u = 0:
    lam E3(|u| / lam) + |u|."""
    a = np.abs(u)
    return lam * _E(3, a / lam) + a


def _pair_integral(a, b, c, d, lam):
    """int_a^b dx int_c^d dx' E1(|x - x'| / lam) / lam (intervals as arrays,
    broadcast against each other)."""
    return _H(b - c, lam) - _H(a - c, lam) - _H(b - d, lam) + _H(a - d, lam)


def graded_mesh(L: float, n_bins: int, per_bin: int, h_min: float, ratio: float = 1.25):
    """Cell edges on [0, L] that contain every bin edge: each bin is cut into
    per_bin uniform cells, and the two wall bins are cut geometrically toward the
    wall down to cells of h_min (ratio between neighbours)."""
    w = L / n_bins
    pts = set(np.linspace(0.0, L, n_bins * per_bin + 1).tolist())
    h, x = h_min, 0.0
    while x + h < w:
        x += h
        pts.add(x)
        pts.add(L - x)
        h *= ratio
    e = np.array(sorted(pts))
    return e[np.concatenate([[True], np.diff(e) > 1e-15 * L])]


def nongray_slab(C, v, tau, L: float, dT1: float = 0.5, dT2: float = -0.5, n_bins: int = 20,
                 per_bin: int = 8, h_min: float = None, ratio: float = 1.25):
    """Steady frequency-dependent slab between black (isothermal) walls at dT1
    (x = 0) and dT2 (x = L), relaxation-time approximation, states m with heat
    capacity C_m, speed v_m and relaxation time tau_m (free path lam_m = v_m tau_m).

    Along each characteristic the intensity relaxes toward C_m psi, psi being the
    pseudo-temperature; angular averaging gives the angle-averaged deviational
    energy of state m,

        <e_m>(x) / C_m = 1/2 dT1 E2(x / lam_m) + 1/2 dT2 E2((L - x) / lam_m)
                         + 1/(2 lam_m) int_0^L psi(x') E1(|x - x'| / lam_m) dx',

    and energy conservation in scattering fixes psi as the (C_m / tau_m)-weighted
    mean of <e_m> / C_m over states.  psi is taken piecewise constant on a mesh
    that is refined toward the walls, and the equation is imposed on cell averages
    (every kernel and source term integrated exactly with E2 / E3).  The cells
    must not be much wider than the free paths that carry the gain weight: for
    cells wider than a free path, cell averages exchange energy at a rate set by
    the cell width instead of the free path.  Returns bin averages of the energy
    temperature T = sum_m <e_m> / C_tot, of the pseudo-temperature psi, and the
    heat flux

        q = sum_m v_m C_m / 2 [dT1 E3(x / lam) - dT2 E3((L - x) / lam)
                               + (1/lam) (int_0^x psi E2((x - x') / lam) dx'
                                          - int_x^L psi E2((x' - x) / lam) dx')],

    evaluated at both walls (equal by energy conservation)."""
    C, v, tau = (np.asarray(a, dtype=np.float64) for a in (C, v, tau))
    lam = v * tau
    w = (C / tau) / np.sum(C / tau)
    if h_min is None:
        h_min = 0.05 * float(lam.min())
    e = graded_mesh(L, n_bins, per_bin, h_min, ratio)
    a, b = e[:-1], e[1:]
    dx = b - a
    n = a.shape[0]
    A = np.zeros((n, n))  # sum_m w_m / 2 <pair integral> / dx_i   (psi -> psi)
    B = np.zeros((n, n))  # sum_m C_m / 2 <pair integral> / dx_i   (psi -> sum_m <e_m>)
    rhs = np.zeros(n)
    src_T = np.zeros(n)
    iu = np.triu_indices(n + 1)
    for m in range(lam.shape[0]):
        lm = lam[m]
        # H(e_p - e_q) for every pair of edges (symmetric); the pair integral of cells i, j
        # is H(b_i - a_j) - H(a_i - a_j) - H(b_i - b_j) + H(a_i - b_j)
        Hm = np.zeros((n + 1, n + 1))
        Hm[iu] = _H(e[iu[0]] - e[iu[1]], lm)
        Hm = Hm + np.triu(Hm, 1).T
        P = Hm[1:, :-1] - Hm[:-1, :-1] - Hm[1:, 1:] + Hm[:-1, 1:]
        P /= dx[:, None]
        src = (0.5 * dT1 * lm * (_E(3, a / lm) - _E(3, b / lm))
               + 0.5 * dT2 * lm * (_E(3, (L - b) / lm) - _E(3, (L - a) / lm))) / dx
        rhs += w[m] * src
        src_T += C[m] * src
        A += (0.5 * w[m]) * P
        B += (0.5 * C[m]) * P
    psi = np.linalg.solve(np.eye(n) - A, rhs)
    T_cell = (src_T + B @ psi) / np.sum(C)
    edges = np.linspace(0.0, L, n_bins + 1)
    k = np.clip(np.searchsorted(edges, 0.5 * (a + b)) - 1, 0, n_bins - 1)
    T_bin = np.bincount(k, weights=T_cell * dx, minlength=n_bins) / np.diff(edges)
    psi_bin = np.bincount(k, weights=psi * dx, minlength=n_bins) / np.diff(edges)

    def flux_at(x):
        q = 0.0
        left = a < x
        for m in range(lam.shape[0]):
            lm = lam[m]
            # int over a cell of psi E2(|x - x'| / lam) dx' / lam = E3 differences, per side
            il = np.sum(psi[left] * (_E(3, np.maximum(x - b[left], 0.0) / lm) - _E(3, (x - a[left]) / lm)))
            ir = np.sum(psi[~left] * (_E(3, (a[~left] - x) / lm) - _E(3, (b[~left] - x) / lm)))
            q += 0.5 * v[m] * C[m] * (dT1 * _E(3, x / lm) - dT2 * _E(3, (L - x) / lm) + il - ir)
        return q

    return T_bin, psi_bin, flux_at(0.0), flux_at(L)


# --------------------------------------------------------------------------
# Heated spot: ballistic and diffusive references averaged over grid cells
# --------------------------------------------------------------------------


def gaussian_spherical_mean(rho, R, r0):
    """Mean of exp(-|y|^2 / r0^2) over the sphere |y - x| = R with |x| = rho:
    exp(-(rho^2 + R^2) / r0^2) sinh(2 rho R / r0^2) / (2 rho R / r0^2),
    written with exp of non-positive arguments only."""
    rho = np.asarray(rho, dtype=np.float64)
    a = 2.0 * rho * R / (r0 * r0)
    base = np.exp(-(rho - R) ** 2 / (r0 * r0))  # exp(-(rho^2 + R^2)/r0^2 + a)
    with np.errstate(invalid="ignore", divide="ignore"):
        ratio = np.where(a > 1e-8, (1.0 - np.exp(-2.0 * a)) / (2.0 * np.where(a > 1e-8, a, 1.0)), 1.0 - a)
    return base * ratio


def cell_averages(f, grid, lo, hi, nq: int = 6):
    """Average of f(x, y, z) over every cell of a grid (x fastest), by
    Gauss-Legendre quadrature with nq points per axis in each cell."""
    g = np.polynomial.legendre.leggauss(nq)
    out = np.zeros((grid[2], grid[1], grid[0]))
    axes = []
    for d in range(3):
        w = (hi[d] - lo[d]) / grid[d]
        c = lo[d] + w * (np.arange(grid[d])[:, None] + 0.5 * (g[0][None, :] + 1.0))  # (cells, nq)
        axes.append((c, 0.5 * g[1]))
    (cx, wx), (cy, wy), (cz, wz) = axes
    X = cx[None, None, :, None, None, :]
    Y = cy[None, :, None, None, :, None]
    Z = cz[:, None, None, :, None, None]
    W = wz[None, None, None, :, None, None] * wy[None, None, None, None, :, None] * wx[None, None, None, None, None, :]
    vals = f(X, Y, Z) * W
    return vals.sum(axis=(3, 4, 5))


def ballistic_spot_cells(grid, lo, hi, v: float, t: float, r0: float, dT: float = 1.0, nq: int = 6):
    """Free streaming (no scattering) from dT exp(-|x|^2 / r0^2) on the half space
    z >= 0 with a specular surface, i.e. the full-space problem with the mirrored
    (whole) Gaussian: dT(x, t) is the Gaussian's mean over the sphere of radius
    v t about x.  Cell averages."""
    return cell_averages(lambda X, Y, Z: dT * gaussian_spherical_mean(np.sqrt(X * X + Y * Y + Z * Z), v * t, r0),
                         grid, lo, hi, nq)


def diffusive_spot_cells(grid, lo, hi, alpha: float, t: float, r0: float, dT: float = 1.0, nq: int = 6):
    """Fourier diffusion of dT exp(-|x|^2 / r0^2) on the half space with an
    adiabatic surface (the full-space solution, by image symmetry):
    dT (r0^2 / s)^(3/2) exp(-|x|^2 / s), s = r0^2 + 4 alpha t.  Cell averages."""
    s = r0 * r0 + 4.0 * alpha * t
    return cell_averages(lambda X, Y, Z: dT * (r0 * r0 / s) ** 1.5 * np.exp(-(X * X + Y * Y + Z * Z) / s),
                         grid, lo, hi, nq)
