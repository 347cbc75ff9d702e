"""Seeded synthetic inputs for the linearized deviational phonon Monte Carlo.

This module is shared by the FP64 CPU oracle (``oracle/``) and by the GPU
library's tests and benchmark.  It only *describes* problems: material
property tables (a dispersion relation and a relaxation-time law, i.e. the
D(omega,p), V_g(omega,p), tau(omega,p,T_eq) inputs of the paper's Eq. (1)),
geometries, sources, tally grids and workload lists.  No step of the Monte
Carlo method (heat capacities, source normalisation, sampling, transport,
scoring) is computed here.

Units are SI throughout: rad/s, s/m^3 per rad/s (density of states per unit
volume and angular frequency, one polarization), m/s, s, K, m.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

import numpy as np

# --------------------------------------------------------------------------
# Materials
# --------------------------------------------------------------------------


@dataclass
class Branch:
    """One polarization branch tabulated on frequency bins."""

    omega: np.ndarray  # bin centres [rad/s]
    domega: np.ndarray  # bin widths [rad/s]
    dos: np.ndarray  # D(omega) per polarization [s/m^3]
    vg: np.ndarray  # group-velocity magnitude [m/s]
    tau: np.ndarray  # relaxation time at T_eq [s]
    degeneracy: float = 1.0  # number of identical polarizations in the branch

    def __post_init__(self):
        for name in ("omega", "domega", "dos", "vg", "tau"):
            setattr(self, name, np.ascontiguousarray(getattr(self, name), dtype=np.float64))
        n = self.omega.shape[0]
        for name in ("domega", "dos", "vg", "tau"):
            if getattr(self, name).shape != (n,):
                raise ValueError(f"branch array {name} has shape {getattr(self, name).shape}, expected ({n},)")


@dataclass
class Material:
    branches: List[Branch]
    T_eq: float = 300.0
    name: str = ""
    # mean cosine of the angle between the directions before and after a
    # scattering event (Henyey-Greenstein phase function); 0: isotropic
    scatter_g: float = 0.0

    @property
    def n_states(self) -> int:
        return int(sum(b.omega.shape[0] for b in self.branches))

    def flat(self):
        """Concatenate the branches in order: (omega, domega, dos, vg, tau, degeneracy)."""
        cat = lambda a: np.concatenate([getattr(b, a) for b in self.branches])
        deg = np.concatenate([np.full(b.omega.shape[0], b.degeneracy) for b in self.branches])
        return cat("omega"), cat("domega"), cat("dos"), cat("vg"), cat("tau"), deg


def gray_material(vg: float = 6000.0, tau: float = 16.7e-12, omega: float = 1.0e13,
                  T_eq: float = 300.0, dos_domega: float = 7.25e28, scatter_g: float = 0.0) -> Material:
    """A single-mode (gray) material: one state with the given speed and relaxation time.

    D*domega defaults to about 1e6 / k_B so the mode's heat capacity is of
    order 1e6 J/m^3/K; gray results are reported non-dimensionally, so its
    exact value does not matter.
    """
    b = Branch(omega=[omega], domega=[1.0], dos=[dos_domega], vg=[vg], tau=[tau], degeneracy=1.0)
    return Material([b], T_eq=T_eq, name="gray", scatter_g=scatter_g)


SILICON_LATTICE = 5.431e-10  # m


def silicon_like(n_bins: int = 1000, T_eq: float = 300.0,
                 omega_max=(7.7e13, 3.0e13), degeneracy=(1.0, 2.0),
                 A: float = 1.3e-45, B: float = 9e-19, C: float = 190.0,
                 L_b: float = math.inf, lattice: float = SILICON_LATTICE,
                 tau_scale: float = 1.0, scatter_g: float = 0.0) -> Material:
    """Silicon-like material: isotropic sine dispersion, LA + doubly-degenerate TA.

    omega(k) = omega_max sin(pi k / (2 k_max)), k_max = 2 pi / a.
    v_g = d omega / d k, D = k^2 / (2 pi^2 v_g) per polarization.
    tau^-1 = A omega^4 + B omega^2 T exp(-C/T) + v_g / L_b, at T = T_eq.
    ``n_bins`` uniform bins per branch on [0, omega_max], properties at the
    bin midpoints.  ``tau_scale`` multiplies every relaxation time (used to
    push the material into the diffusive limit for tests).
    """
    kmax = 2.0 * math.pi / lattice
    branches = []
    for wmax, g in zip(omega_max, degeneracy):
        edges = np.linspace(0.0, wmax, n_bins + 1)
        w = 0.5 * (edges[1:] + edges[:-1])
        dw = np.diff(edges)
        k = (2.0 * kmax / math.pi) * np.arcsin(w / wmax)
        vg = (math.pi / (2.0 * kmax)) * np.sqrt(wmax * wmax - w * w)
        dos = k * k / (2.0 * math.pi ** 2 * vg)
        inv_tau = A * w ** 4 + B * w ** 2 * T_eq * math.exp(-C / T_eq)
        if math.isfinite(L_b):
            inv_tau = inv_tau + vg / L_b
        tau = tau_scale / inv_tau
        branches.append(Branch(w, dw, dos, vg, tau, g))
    return Material(branches, T_eq=T_eq, name="silicon_like", scatter_g=scatter_g)


# --------------------------------------------------------------------------
# Geometry, sources, tallies
# --------------------------------------------------------------------------

GEOMETRY_KINDS = ("slab_z", "film_x", "pore_cell_xz", "halfspace_z")
WALL_TYPES = ("isothermal", "adiabatic", "periodic")
SOURCE_KINDS = ("walls", "gaussian", "gradient")


@dataclass
class Wall:
    type: str = "isothermal"
    temperature: float = 300.0  # isothermal walls only
    specularity: float = 0.0  # adiabatic walls only, probability of a specular reflection


@dataclass
class Geometry:
    """Simulation domain.

    slab_z        walls at z = 0 (walls[0]) and z = length (walls[1]); infinite in x, y.
    film_x        walls at x = 0 (walls[0]) and x = length (walls[1]); infinite in y, z.
    pore_cell_xz  periodic unit cell [0, length)^2 in (x, z), infinite in y, with a
                  cylindrical pore (axis along y) of ``radius`` at the cell centre;
                  walls[0] describes the pore surface (adiabatic).
    halfspace_z   solid for z >= 0, surface z = 0 described by walls[0].
    """

    kind: str
    length: float = 0.0
    radius: float = 0.0
    walls: List[Wall] = field(default_factory=list)


@dataclass
class Source:
    """Particle source.

    walls     every isothermal wall whose temperature differs from T_eq emits its
              deviational flux (steady problem).
    gaussian  initial condition T_i - T_eq = dT exp(-|x|^2 / radius^2) centred at the
              origin (transient problem, half-space z >= 0).
    gradient  uniform volumetric source of an imposed temperature gradient dT/dz =
              ``gradient`` [K/m] (steady, periodic problems).
    """

    kind: str
    dT: float = 0.0
    radius: float = 0.0
    gradient: float = 0.0


@dataclass
class Tally:
    n_bins: int = 0  # 1-D bins along the geometry's confining axis (slab: z, film: x)
    n_batches: int = 16  # batch replicas (batch = pid mod n_batches) for standard errors
    kmax: int = -1  # stop a particle after this many scattering events (-1: never)
    n_hj: int = 0  # record the per-scattering-index flux contributions H_j, j < n_hj
    times: Tuple[float, ...] = ()  # transient snapshot times (empty: steady problem)
    grid: Tuple[int, int, int] = (0, 0, 0)  # snapshot grid cells along x, y, z
    grid_lo: Tuple[float, float, float] = (0.0, 0.0, 0.0)
    grid_hi: Tuple[float, float, float] = (0.0, 0.0, 0.0)
    first_event: bool = False  # in-plane films: end at the first scattering event or diffuse reflection
    # transient jobs: time-windowed track-length temperature and z heat flux in the
    # z-aligned cylinder (cx, cy, radius, z_lo, z_hi), windows between snapshot times
    region: Optional[Tuple[float, float, float, float, float]] = None


@dataclass
class Job:
    material: Material
    geometry: Geometry
    source: Source
    tally: Tally
    n_particles: int
    seed: int
    name: str = ""
    first_particle: int = 0   # simulate pids first_particle .. first_particle + n_particles - 1


# --------------------------------------------------------------------------
# Workloads
# --------------------------------------------------------------------------

T_EQ = 300.0


def slab_job(material: Material, L: float, n: int, seed: int, n_bins: int = 20,
             dT: float = 0.5, name: str = "") -> Job:
    """Cross-plane slab: isothermal walls at T_eq + dT (z = 0) and T_eq - dT (z = L)."""
    T = material.T_eq
    geom = Geometry("slab_z", length=L, walls=[Wall("isothermal", T + dT), Wall("isothermal", T - dT)])
    return Job(material, geom, Source("walls"), Tally(n_bins=n_bins), int(n), int(seed), name or f"slab_L{L:.3g}")


def gray_slab(n: int = 100_000, seed: int = 1, L: float = 100e-9, tau: float = 16.7e-12,
              vg: float = 6000.0, n_bins: int = 20) -> Job:
    """Gray 1-D slab: walls at T_eq +- 0.5 K, L = 100 nm, v = 6000 m/s, tau = 16.7 ps."""
    return slab_job(gray_material(vg=vg, tau=tau), L, n, seed, n_bins, name="gray_slab")


def film_thicknesses(n: int = 12, lo: float = 10e-9, hi: float = 10e-6) -> np.ndarray:
    """Log-spaced film thicknesses lo .. hi (inclusive)."""
    return lo * (hi / lo) ** (np.arange(n) / (n - 1))


def cross_plane_films(n_per_film: int = 100_000_000, n_films: int = 12, n_bins: int = 20,
                      material: Optional[Material] = None, seed0: int = 100) -> List[Job]:
    """Silicon-like cross-plane films, 12 thicknesses log-spaced 10 nm - 10 um, seed 100 + j."""
    mat = material or silicon_like()
    return [slab_job(mat, float(L), n_per_film, seed0 + j, n_bins, name=f"film_{j}_L{L:.3g}")
            for j, L in enumerate(film_thicknesses(n_films))]


TTR_PROBE = (0.0, 0.0, 10e-6, 0.0, 5e-9)  # surface cylinder of radius 10 um, 5 nm deep


def heated_spot(n: int = 1_000_000_000, seed: int = 7, material: Optional[Material] = None,
                grid: int = 64, n_times: int = 50, r0: float = 1e-6, dT: float = 1.0,
                specularity: float = 0.0, probe: Optional[Tuple[float, float, float, float, float]] = None) -> Job:
    """Transient heated spot on a semi-infinite substrate.

    Gaussian initial temperature of radius r0 and amplitude dT at the origin of the
    adiabatic surface z = 0; snapshot grid x, y in [-4, 4] um, z in [0, 8] um;
    times log-spaced 1 ps .. 10 ns (both ends included).  ``probe`` adds the
    windowed track-length tally in a surface cylinder (e.g. TTR_PROBE).
    """
    mat = material or silicon_like()
    times = tuple(float(t) for t in 10.0 ** (-12.0 + 4.0 * np.arange(n_times) / (n_times - 1)))
    geom = Geometry("halfspace_z", walls=[Wall("adiabatic", specularity=specularity)])
    tally = Tally(n_bins=0, times=times, grid=(grid, grid, grid),
                  grid_lo=(-4e-6, -4e-6, 0.0), grid_hi=(4e-6, 4e-6, 8e-6), region=probe)
    return Job(mat, geom, Source("gaussian", dT=dT, radius=r0), tally, int(n), int(seed), "heated_spot")


def in_plane_film(d: float, specularity: float, n: int, seed: int, material: Optional[Material] = None,
                  gradient: float = -1e6, kmax: int = 40, n_hj: int = 40, n_bins: int = 0,
                  first_event: bool = False) -> Job:
    mat = material or silicon_like()
    w = Wall("adiabatic", specularity=specularity)
    geom = Geometry("film_x", length=d, walls=[w, Wall("adiabatic", specularity=specularity)])
    tally = Tally(n_bins=n_bins, kmax=kmax, n_hj=n_hj, first_event=first_event)
    return Job(mat, geom, Source("gradient", gradient=gradient), tally, int(n), int(seed),
               f"film_d{d:.3g}_p{specularity}" + ("_first" if first_event else ""))


def pore_cell(period: float, porosity: float, n: int, seed: int, material: Optional[Material] = None,
              gradient: float = -1e6, kmax: int = 40, n_hj: int = 40, specularity: float = 0.0,
              field: Optional[Tuple[int, int]] = None) -> Job:
    """Square-lattice unit cell with a centred cylindrical pore of porosity pi r^2 / P^2.
    ``field`` = (nx, nz) adds the steady temperature and z heat-flux fields on an
    nx x nz grid over the unit cell."""
    mat = material or silicon_like()
    r = period * math.sqrt(porosity / math.pi)
    geom = Geometry("pore_cell_xz", length=period, radius=r, walls=[Wall("adiabatic", specularity=specularity)])
    tally = Tally(kmax=kmax, n_hj=n_hj)
    if field is not None:
        tally.grid = (int(field[0]), 1, int(field[1]))
        tally.grid_lo = (0.0, 0.0, 0.0)
        tally.grid_hi = (float(period), 1.0, float(period))
    return Job(mat, geom, Source("gradient", gradient=gradient), tally,
               int(n), int(seed), f"pore_P{period:.3g}_phi{porosity}" + ("_field" if field else ""))


def batched_nanostructures(n_scale: float = 1.0, seed: int = 4, material: Optional[Material] = None,
                           n_min: float = 1e6, n_max: float = 1e8, first_event_films: bool = False) -> List[Job]:
    """64 instances: 24 in-plane films (8 thicknesses 20-500 nm x p in {0, .5, .9}) and
    40 pore cells (porosity {.1,.2,.3,.4} x 10 periods 50-500 nm).  Particle counts are
    log-uniform in [n_min, n_max] (numpy PCG64 with ``seed``), times ``n_scale``."""
    mat = material or silicon_like()
    rng = np.random.Generator(np.random.PCG64(seed))
    counts = np.exp(rng.uniform(math.log(n_min), math.log(n_max), size=64))
    jobs: List[Job] = []
    i = 0
    for d in 20e-9 * (500 / 20) ** (np.arange(8) / 7):
        for p in (0.0, 0.5, 0.9):
            jobs.append(in_plane_film(float(d), p, max(1, int(counts[i] * n_scale)), 1000 + i, mat,
                                      first_event=first_event_films))
            i += 1
    for phi in (0.1, 0.2, 0.3, 0.4):
        for P in 50e-9 * (500 / 50) ** (np.arange(10) / 9):
            jobs.append(pore_cell(float(P), phi, max(1, int(counts[i] * n_scale)), 1000 + i, mat))
            i += 1
    return jobs


def serving_stream(n_requests: int = 500, seed: int = 5, n_min: float = 1e5, n_max: float = 1e8,
                   material: Optional[Material] = None) -> List[Tuple[str, Job]]:
    """Request mix: uniform over {cross-plane film (random thickness index), heated spot,
    pore cell}; particle counts log-uniform in [n_min, n_max]; request seed 10^6 + id."""
    mat = material or silicon_like()
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    Ls = film_thicknesses()
    for rid in range(n_requests):
        kind = int(rng.integers(0, 3))
        n = int(math.exp(rng.uniform(math.log(n_min), math.log(n_max))))
        s = 1_000_000 + rid
        if kind == 0:
            j = int(rng.integers(0, len(Ls)))
            out.append(("film", slab_job(mat, float(Ls[j]), n, s, 20, name=f"req{rid}_film{j}")))
        elif kind == 1:
            job = heated_spot(n=n, seed=s, material=mat, grid=32, n_times=10)
            job.name = f"req{rid}_spot"
            out.append(("spot", job))
        else:
            phi = float(rng.choice([0.1, 0.2, 0.3, 0.4]))
            P = float(50e-9 * 10 ** rng.uniform(0, 1))
            job = pore_cell(P, phi, n, s, mat)
            job.name = f"req{rid}_pore"
            out.append(("pore", job))
    return out


def poisson_arrivals(n: int, rate: float, seed: int = 5) -> np.ndarray:
    """Arrival times [s] of a Poisson process of the given rate."""
    rng = np.random.Generator(np.random.PCG64(seed + 1))
    return np.cumsum(rng.exponential(1.0 / rate, size=n))
