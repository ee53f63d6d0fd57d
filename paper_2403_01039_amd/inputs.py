"""Seeded synthetic problem generators for the 3D-RISM solver.

This module only *draws and lays out inputs*: solute atoms (positions, LJ sigma /
epsilon, partial charges), solvent site tables (charges, LJ parameters, number
densities, intramolecular geometry), grids and solver options.  It holds none
of the method's arithmetic (no potential, no closure, no transform, no
correlation function), so both the FP64 CPU oracle and the HIP path may import
it without sharing any of the computation.

Units: Angstrom, kcal/mol, elementary charge, Kelvin.

Workloads (the paper's own RBD-ACE2 system, section "Example", is not
available, so these seeded stand-ins of the same kind are used):

* ``single_site``    one neutral LJ sphere (sigma 3.73, eps 0.294) on the box
                     centre in 3-site water, 64^3 at 0.5 A.
* ``solute_200``     200 atoms uniform in a 14 A sphere, >= 1.2 A apart,
                     sigma in {2.0, 3.0, 3.5}, eps ~ U(0.05, 0.2),
                     q ~ N(0, 0.3) shifted to net charge 0; 128^3 at 0.5 A.
                     Solvent: water + 0.1 M NaCl (5 sites) or water (3 sites).
* ``globule_4000``   4000 atoms in a 22 A ellipsoid (axes 1 : 0.8 : 0.7), net
                     charge +4, water, 256^3 at 0.4 A, PSE-3, MDIIS depth 10.
* ``batch_uneven``   64 solutes of 20..300 atoms, grid per solute from
                     {64, 96, 128}^3 at 0.5 A keeping >= 12 A of solvent.

Draw order inside one solute is fixed: positions, then sigma choices, then
epsilon, then charges (numpy PCG64 via ``default_rng(seed)``).
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional, Sequence

import numpy as np

# ---------------------------------------------------------------------------
# Solvent description (inputs only)
# ---------------------------------------------------------------------------


@dataclasses.dataclass(frozen=True)
class Site:
    name: str
    q: float        # e
    sigma: float    # A
    eps: float      # kcal/mol


@dataclasses.dataclass(frozen=True)
class Species:
    """A solvent molecule: its sites, their coordinates in a molecular frame
    (Angstrom) and the molecular number density (A^-3)."""
    name: str
    sites: Sequence[Site]
    coords: np.ndarray   # [n_sites][3]
    density: float


@dataclasses.dataclass(frozen=True)
class Solvent:
    species: Sequence[Species]
    temperature: float = 298.15
    dielectric: float = 78.4        # used only by the 1D DRISM solvent solve

    @property
    def sites(self) -> List[Site]:
        return [s for sp in self.species for s in sp.sites]

    @property
    def n_sites(self) -> int:
        return len(self.sites)

    def site_arrays(self):
        """(q, sigma, eps, rho) per solvent site, float64."""
        q, sig, eps, rho = [], [], [], []
        for sp in self.species:
            for s in sp.sites:
                q.append(s.q)
                sig.append(s.sigma)
                eps.append(s.eps)
                rho.append(sp.density)
        return (np.array(q), np.array(sig), np.array(eps), np.array(rho))

    def site_names(self) -> List[str]:
        return [s.name for s in self.sites]


WATER_DENSITY = 0.0334           # molecules / A^3
AVOGADRO = 6.02214076e23
ION_DENSITY_0P1M = 0.1 * AVOGADRO * 1e-27   # 0.1 mol/L in A^-3 = 6.0221e-5


def water_species(density: float = WATER_DENSITY) -> Species:
    """SPC/E-like 3-site water: O q -0.8476 sigma 3.166 eps 0.1553,
    H q +0.4238 sigma 0.4 eps 0.046, O-H 1.0 A, H-O-H 109.47 degrees.
    Frame: O at the origin, H atoms in the xz plane, bisector along +z."""
    half = np.deg2rad(109.47) / 2.0
    r_oh = 1.0
    coords = np.array([
        [0.0, 0.0, 0.0],
        [+r_oh * np.sin(half), 0.0, r_oh * np.cos(half)],
        [-r_oh * np.sin(half), 0.0, r_oh * np.cos(half)],
    ])
    sites = (Site("O", -0.8476, 3.166, 0.1553),
             Site("H1", 0.4238, 0.4, 0.046),
             Site("H2", 0.4238, 0.4, 0.046))
    return Species("water", sites, coords, density)


def sodium(density: float = ION_DENSITY_0P1M) -> Species:
    return Species("Na+", (Site("Na", 1.0, 2.35, 0.13),), np.zeros((1, 3)), density)


def chloride(density: float = ION_DENSITY_0P1M) -> Species:
    return Species("Cl-", (Site("Cl", -1.0, 4.40, 0.10),), np.zeros((1, 3)), density)


def water_solvent() -> Solvent:
    return Solvent((water_species(),))


def saline_solvent() -> Solvent:
    """Water + 0.1 M NaCl: 5 sites O, H1, H2, Na, Cl."""
    return Solvent((water_species(), sodium(), chloride()))


def single_site_solvent(density: float, q: float = 0.0, sigma: float = 3.0,
                        eps: float = 0.2) -> Solvent:
    """One spherical site (used for reductions and closed-form checks)."""
    return Solvent((Species("X", (Site("X", q, sigma, eps),), np.zeros((1, 3)), density),))


# ---------------------------------------------------------------------------
# Solute description
# ---------------------------------------------------------------------------


@dataclasses.dataclass
class Solute:
    xyz: np.ndarray      # [n][3] A
    q: np.ndarray        # [n] e
    sigma: np.ndarray    # [n] A
    eps: np.ndarray      # [n] kcal/mol

    @property
    def n_atoms(self) -> int:
        return int(self.xyz.shape[0])


@dataclasses.dataclass
class Grid:
    nx: int
    ny: int
    nz: int
    spacing: float
    center: tuple = (0.0, 0.0, 0.0)   # sits on grid index (nx/2, ny/2, nz/2)

    @property
    def shape(self):
        return (self.nz, self.ny, self.nx)

    @property
    def n_points(self) -> int:
        return self.nx * self.ny * self.nz


@dataclasses.dataclass
class Options:
    closure: str = "kh"          # "kh" | "hnc" | "pse"
    pse_order: int = 3
    tol: float = 1e-6
    max_iter: int = 5000
    mdiis_depth: int = 5
    mdiis_eta: float = 0.6         # MDIIS damping, or the modified-Anderson mixing b
    eta_dynamic: bool = False
    accelerator: str = "mdiis"     # "mdiis" | "anderson" (modified Anderson, two histories)
    anderson_s1: float = 0.2
    anderson_s2: float = 0.0


@dataclasses.dataclass
class Problem:
    name: str
    solute: Solute
    solvent: Solvent
    grid: Grid
    options: Options
    seed: Optional[int] = None


SIGMA_CHOICES = np.array([2.0, 3.0, 3.5])


def _rejection_points(rng, n: int, semi_axes, min_sep: float) -> np.ndarray:
    """n points uniform in an axis-aligned ellipsoid, pairwise >= min_sep apart.
    Candidates are drawn uniformly in the bounding box and accepted if inside
    the ellipsoid and far enough from every accepted point."""
    a = np.asarray(semi_axes, dtype=np.float64)
    pts = np.empty((n, 3))
    k = 0
    tries = 0
    while k < n:
        tries += 1
        if tries > 2000 * n + 100000:
            raise RuntimeError("rejection sampling did not place all atoms")
        p = rng.uniform(-a, a)
        if np.sum((p / a) ** 2) > 1.0:
            continue
        if k and np.min(np.sum((pts[:k] - p) ** 2, axis=1)) < min_sep * min_sep:
            continue
        pts[k] = p
        k += 1
    return pts


def random_solute(seed: int, n_atoms: int, semi_axes, net_charge: float = 0.0,
                  min_sep: float = 1.2) -> Solute:
    rng = np.random.default_rng(seed)
    xyz = _rejection_points(rng, n_atoms, semi_axes, min_sep)
    sigma = SIGMA_CHOICES[rng.integers(0, len(SIGMA_CHOICES), size=n_atoms)]
    eps = rng.uniform(0.05, 0.2, size=n_atoms)
    q = rng.normal(0.0, 0.3, size=n_atoms)
    q = q - q.mean() + net_charge / n_atoms
    xyz = xyz - xyz.mean(axis=0)      # centroid on the box centre (origin)
    return Solute(xyz=xyz, q=q, sigma=sigma, eps=eps)


# ---------------------------------------------------------------------------
# Named workloads
# ---------------------------------------------------------------------------


def single_site_problem(n: int = 64, spacing: float = 0.5, solvent: Optional[Solvent] = None,
                        closure: str = "kh") -> Problem:
    """One LJ site (sigma 3.73 A, eps 0.294 kcal/mol, q 0) on the centre grid
    point, in 3-site water; KH, MDIIS depth 5, rms 1e-6."""
    sol = Solute(xyz=np.zeros((1, 3)), q=np.zeros(1), sigma=np.array([3.73]),
                 eps=np.array([0.294]))
    return Problem("single_site", sol, solvent or water_solvent(), Grid(n, n, n, spacing),
                   Options(closure=closure, mdiis_depth=5))


def solute_200_problem(seed: int = 1, saline: bool = True, n: int = 128,
                       spacing: float = 0.5, n_atoms: int = 200,
                       radius: float = 14.0) -> Problem:
    sol = random_solute(seed, n_atoms, (radius, radius, radius))
    solvent = saline_solvent() if saline else water_solvent()
    return Problem("solute_200" + ("_saline" if saline else "_water"), sol, solvent,
                   Grid(n, n, n, spacing), Options(closure="kh", mdiis_depth=5), seed)


def globule_4000_problem(seed: int = 2, n: int = 256, spacing: float = 0.4,
                         n_atoms: int = 4000) -> Problem:
    sol = random_solute(seed, n_atoms, (22.0, 17.6, 15.4), net_charge=4.0)
    return Problem("globule_4000", sol, water_solvent(), Grid(n, n, n, spacing),
                   Options(closure="pse", pse_order=3, mdiis_depth=10), seed)


def globule_12877_problem(seed: int = 3, n: int = 512, spacing: float = 0.5) -> Problem:
    """Stand-in at the paper's demonstration scale (12877 atoms on 512^3 over a
    256 A box): a globule at the 4000-atom globule's packing (semi-axes scaled
    by (12877/4000)^(1/3)), net charge +13, in water + 0.1 M NaCl (5 sites),
    KH, MDIIS 5."""
    f = (12877 / 4000.0) ** (1.0 / 3.0)
    sol = random_solute(seed, 12877, (22.0 * f, 17.6 * f, 15.4 * f), net_charge=13.0)
    return Problem("globule_12877", sol, saline_solvent(), Grid(n, n, n, spacing),
                   Options(closure="kh", mdiis_depth=5), seed)


BATCH_GRID_CHOICES = (64, 96, 128)


def batch_member_problem(seed: int, spacing: float = 0.5, margin: float = 12.0) -> Problem:
    """One member of the uneven batch: n_atoms ~ U{20..300}; sphere radius
    14 (n/200)^(1/3) A (the 200-atom density); the smallest grid of
    {64, 96, 128}^3 that leaves >= margin A from the outermost atom centre to
    every box face."""
    rng = np.random.default_rng(seed)
    n_atoms = int(rng.integers(20, 301))
    radius = 14.0 * (n_atoms / 200.0) ** (1.0 / 3.0)
    sol = random_solute(seed + 7919, n_atoms, (radius, radius, radius))
    extent = float(np.max(np.abs(sol.xyz)))
    n = None
    for cand in BATCH_GRID_CHOICES:
        half = (cand / 2.0) * spacing       # box spans centre +- n/2 spacings
        if half - extent >= margin:
            n = cand
            break
    if n is None:
        n = BATCH_GRID_CHOICES[-1]
    return Problem(f"batch_{seed}", sol, water_solvent(), Grid(n, n, n, spacing),
                   Options(closure="kh", mdiis_depth=5), seed)


def batch_uneven_problems(first_seed: int = 1000, count: int = 64) -> List[Problem]:
    return [batch_member_problem(first_seed + i) for i in range(count)]


def warmstart_problem(seed: int, n: int = 128, spacing: float = 0.5) -> Problem:
    """200-atom solute in water (3 sites), 128^3 at 0.5 A, KH, depth 5."""
    p = solute_200_problem(seed, saline=False, n=n, spacing=spacing)
    p.name = f"warm_{seed}"
    return p


def small_problem(seed: int, n_atoms: int = 12, shape=(24, 20, 18), spacing: float = 0.5,
                  saline: bool = False, closure: str = "kh", radius: float = 3.0,
                  mdiis_depth: int = 5, charge_scale: float = 1.0) -> Problem:
    """A small charged solute on a small (possibly non-cubic) grid, for parity
    tests that the oracle finishes in seconds.  ``charge_scale`` multiplies
    the drawn charges (HNC and PSE-n diverge for the full N(0, 0.3) charges on
    a compact solute, in FP64 as well)."""
    sol = random_solute(seed, n_atoms, (radius, radius, radius))
    sol.q = sol.q * charge_scale
    solvent = saline_solvent() if saline else water_solvent()
    nz, ny, nx = shape
    return Problem(f"small_{seed}", sol, solvent, Grid(nx, ny, nz, spacing),
                   Options(closure=closure, mdiis_depth=mdiis_depth), seed)


def synthetic_distribution(problem: Problem, seed: int, exclusion: float = 2.0,
                           spread: float = 0.3) -> np.ndarray:
    """A seeded stand-in for a solvent distribution g [n_v, nz, ny, nx] (float32):
    0 within ``exclusion`` A of any atom centre (the excluded core), elsewhere
    max(0, 1 + spread * N(0, 1)).  Grid point (ix, iy, iz) sits at
    centre + ((ix, iy, iz) - (nx, ny, nz) div 2) * spacing."""
    gr = problem.grid
    rng = np.random.default_rng(seed)
    nv = len(problem.solvent.site_names())
    g = np.maximum(0.0, 1.0 + spread * rng.standard_normal((nv, gr.nz, gr.ny, gr.nx)))
    axes = [gr.center[i] + (np.arange(n) - n // 2) * gr.spacing
            for i, n in enumerate((gr.nx, gr.ny, gr.nz))]
    zz, yy, xx = np.meshgrid(axes[2], axes[1], axes[0], indexing="ij")
    core = np.zeros(zz.shape, dtype=bool)
    for a in range(problem.solute.n_atoms):
        x, y, z = problem.solute.xyz[a]
        core |= (xx - x) ** 2 + (yy - y) ** 2 + (zz - z) ** 2 < exclusion ** 2
    g[:, core] = 0.0
    return g.astype(np.float32)


# ---------------------------------------------------------------------------
# Solvent susceptibility tables (data files, read-only)
# ---------------------------------------------------------------------------

import os as _os

SOLVENT_TABLE_DIR = _os.path.join(_os.path.dirname(_os.path.dirname(_os.path.abspath(__file__))),
                                  "tests", "golden", "solvent")


def solvent_table(name: str):
    """(chi [n_v][n_v][n_k] float64, dk) for a stored solvent ('water' or
    'saline').  chi_ab(m dk) = w_ab + rho_a h_ab from a 1D DRISM/KH solve; the
    site order is that of ``water_solvent()`` / ``saline_solvent()``."""
    with np.load(_os.path.join(SOLVENT_TABLE_DIR, f"{name}.npz"), allow_pickle=False) as z:
        return np.array(z["chi"]), float(z["dk"])


def solvent_bulk(name: str):
    """(compressibility chi_T [A^3 mol/kcal], pressure [kcal/(mol A^3)]) of a
    stored solvent, from the same 1D solve as its table."""
    import json
    with open(_os.path.join(SOLVENT_TABLE_DIR, f"{name}_bulk.json")) as f:
        b = json.load(f)
    return float(b["compressibility"]), float(b["pressure"])


def solvent_name(solvent: Solvent) -> str:
    names = solvent.site_names()
    if names == water_solvent().site_names():
        return "water"
    if names == saline_solvent().site_names():
        return "saline"
    raise KeyError(f"no stored solvent with sites {names}")


def solvent_table_for(solvent: Solvent):
    """The stored table whose site list matches ``solvent``."""
    names = solvent.site_names()
    if names == water_solvent().site_names():
        return solvent_table("water")
    if names == saline_solvent().site_names():
        return solvent_table("saline")
    raise KeyError(f"no stored susceptibility table for sites {names}")


# ---------------------------------------------------------------------------
# Warm-start network parameters (seeded initial values; both sides take them
# as inputs)
# ---------------------------------------------------------------------------

def unet_init_params(layers, seed: int, slope: float = 0.1, scale: float = 1.0) -> np.ndarray:
    """Flat FP32 parameter vector for the convolution list ``layers`` =
    [(name, C_in, C_out), ...]: per layer W[C_out, 27, C_in] then b[C_out].
    He-normal weights for a leaky slope (fan-in 27 C_in) times ``scale``, zero
    biases, and a zero output layer (named "out")."""
    rng = np.random.default_rng(seed)
    parts = []
    for name, ci, co in layers:
        if name == "out":
            W = np.zeros((co, 27, ci))
        else:
            std = scale * np.sqrt(2.0 / (1.0 + slope ** 2) / (27 * ci))
            W = rng.standard_normal((co, 27, ci)) * std
        parts += [W.ravel(), np.zeros(co)]
    return np.concatenate(parts).astype(np.float32)


def unet_random_params(layers, seed: int, scale: float = 0.5) -> np.ndarray:
    """Random parameters for gradient checks: every layer (the output layer
    and the biases too) drawn N(0, scale^2 / (27 C_in))."""
    rng = np.random.default_rng(seed)
    parts = []
    for name, ci, co in layers:
        std = scale / np.sqrt(27 * ci)
        parts += [rng.standard_normal(co * 27 * ci) * std, rng.standard_normal(co) * std]
    return np.concatenate(parts).astype(np.float32)
