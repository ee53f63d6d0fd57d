"""FP64 1D RISM oracle: solvent-solvent XRISM / DRISM and solute-solvent RISM
(test infrastructure only).

* Solvent-solvent: the RISM equation Eq 4, h = w * c * (w + rho h), closed with
  KH (Eq 6-7, KH reading: exp for d <= 0, 1 + d above) or HNC (Eq 5), solved on
  the radial grid r_i = i dr (i = 1..N-1) with k_j = j pi / (N dr) by
  Fourier-Bessel transforms written as a sine-matrix product (DST-I).  Its
  output is the solvent susceptibility chi = w + rho h (the quantity the 3D
  equation Eq 13 consumes).  The paper defers the 1D solution to Kinoshita
  and does not use a dielectric correction; the optional dielectrically
  consistent form (DRISM, Perkyns & Pettitt, Chem. Phys. Lett. 190, 626 (1992))
  replaces w by w + rho zeta with
      zeta_ab(k) = hc(k) u_a(k) u_b(k),  u_a = j0(k x_a) j0(k y_a) j1(k z_a),
      hc(k) = hc0 exp(-k^2 a^2 / 4),     hc0 = ((eps_r - 1)/y - 3) / rho_d,
      y = 4 pi beta C sum_s rho_s mu_s^2 / 9,
  for the sites of dipolar species, in a molecular frame centred on the site
  centroid with the dipole along z.  hc0 is fixed by requiring that the
  k -> 0 limit of the charge-charge susceptibility reproduce eps_r (XRISM
  alone gives 1 + 3y).
* The Coulomb tail is split as in Eq 29-30 with l = 1 A: the iteration
  variable is tau = t - beta C q_a q_b (1 - e^{-r})/r, whose transform is
  h~ - c~sr; the analytic long-range transform 4 pi / (k^2 (k^2 + 1)) enters
  c~ = c~sr - f~ (Eq 32's 1D analogue).
* Solute-solvent (Eq 8 with a single spherical solute site):
  h_g = sum_g' c_g' * chi_g'g, used for the 3D -> 1D reduction check, with the
  1D free energy Eq 9 / Eq 10 (rho_g restored, as in Eq 17-18).
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

from .rism3d import (COULOMB, SCREEN, beta_of, closure, mdiis_solve, sfe_density)

N_RADIAL = 4096
DR_RADIAL = 0.025


@dataclasses.dataclass
class RadialGrid:
    n: int = N_RADIAL
    dr: float = DR_RADIAL

    @property
    def r(self) -> np.ndarray:
        return self.dr * np.arange(1, self.n)

    @property
    def dk(self) -> float:
        return math.pi / (self.n * self.dr)

    @property
    def k(self) -> np.ndarray:
        return self.dk * np.arange(1, self.n)

    def sine_matrix(self) -> np.ndarray:
        """S_ij = sin(pi i j / N), i, j = 1..N-1, with exact argument reduction."""
        i = np.arange(1, self.n, dtype=np.int64)
        arg = np.outer(i, i) % (2 * self.n)
        return np.sin(np.pi * arg / self.n)


class Hankel:
    """3D radial Fourier transform pair on the DST-I grid:
        f~(k_j) = (4 pi dr / k_j) sum_i r_i f(r_i) sin(k_j r_i)
        f(r_i)  = (dk / (2 pi^2 r_i)) sum_j k_j f~(k_j) sin(k_j r_i)."""

    def __init__(self, grid: RadialGrid):
        self.grid = grid
        self.S = grid.sine_matrix()
        self.r = grid.r
        self.k = grid.k

    def forward(self, f: np.ndarray) -> np.ndarray:
        return (4.0 * math.pi * self.grid.dr / self.k) * ((f * self.r) @ self.S)

    def inverse(self, fk: np.ndarray) -> np.ndarray:
        return (self.grid.dk / (2.0 * math.pi ** 2 * self.r)) * ((fk * self.k) @ self.S)


def j0(x):
    x = np.asarray(x, dtype=np.float64)
    out = np.ones_like(x)
    nz = np.abs(x) > 1e-8
    out[nz] = np.sin(x[nz]) / x[nz]
    return out


def j1(x):
    x = np.asarray(x, dtype=np.float64)
    out = x / 3.0
    nz = np.abs(x) > 1e-3
    xs = x[nz]
    out[nz] = np.sin(xs) / xs ** 2 - np.cos(xs) / xs
    return out


def lr_kernel_k(k: np.ndarray) -> np.ndarray:
    """Transform of (1 - exp(-r/l))/r: 4 pi l^-2 / (k^2 (k^2 + l^-2)) (Eq 30)."""
    return 4.0 * math.pi / SCREEN ** 2 / (k * k * (k * k + 1.0 / SCREEN ** 2))


def _dipole_frame(coords: np.ndarray, q: np.ndarray):
    """Site coordinates about the site centroid, rotated so the dipole is +z."""
    xyz = coords - coords.mean(axis=0)
    mu = (q[:, None] * xyz).sum(axis=0)
    mu_len = float(np.linalg.norm(mu))
    if mu_len < 1e-12:
        return xyz, 0.0
    a = mu / mu_len
    z = np.array([0.0, 0.0, 1.0])
    v = np.cross(a, z)
    s = float(np.linalg.norm(v))
    cth = float(a @ z)
    if s < 1e-14:
        rot = np.eye(3) if cth > 0 else np.diag([1.0, -1.0, -1.0])
    else:
        vx = np.array([[0, -v[2], v[1]], [v[2], 0, -v[0]], [-v[1], v[0], 0]])
        rot = np.eye(3) + vx + vx @ vx * ((1 - cth) / s ** 2)
    return xyz @ rot.T, mu_len


@dataclasses.dataclass
class SolventResult:
    grid: RadialGrid
    chi: np.ndarray          # [n_s, n_s, N-1]  chi_ab(k_j), j = 1..N-1
    h: np.ndarray            # [n_s, n_s, N-1]  real space
    c: np.ndarray            # [n_s, n_s, N-1]  real space (full c)
    iterations: int
    rms: float
    closure: str
    drism: bool
    dielectric: Optional[float]
    smear: float

    def chi_table(self) -> np.ndarray:
        """chi on m = 0..N-1 (k_m = m dk); m = 0 by the even quadratic
        extrapolation chi(0) = (4 chi(k_1) - chi(k_2)) / 3."""
        out = np.empty(self.chi.shape[:2] + (self.grid.n,))
        out[:, :, 1:] = self.chi
        out[:, :, 0] = (4.0 * self.chi[:, :, 0] - self.chi[:, :, 1]) / 3.0
        return out


def solvent_setup(solvent, grid: RadialGrid, drism: bool, smear: float = 1.0):
    """Intramolecular w(k), DRISM zeta(k), densities, pair potentials."""
    q, sig, eps, rho = solvent.site_arrays()
    ns = len(q)
    k = grid.k
    beta = beta_of(solvent.temperature)
    w = np.zeros((ns, ns, len(k)))
    zeta = np.zeros((ns, ns, len(k)))
    idx = 0
    dip_sites = []
    y = 0.0
    rho_d = 0.0
    frames = {}
    for sp in solvent.species:
        n = len(sp.sites)
        coords = np.asarray(sp.coords, dtype=np.float64)
        for a in range(n):
            for b in range(n):
                if a == b:
                    w[idx + a, idx + b] = 1.0
                else:
                    l_ab = float(np.linalg.norm(coords[a] - coords[b]))
                    w[idx + a, idx + b] = j0(k * l_ab)
        qs = np.array([s.q for s in sp.sites])
        frame, mu = _dipole_frame(coords, qs)
        if mu > 1e-12:
            y += 4.0 * math.pi * beta * COULOMB * sp.density * mu * mu / 9.0
            rho_d += sp.density
            for a in range(n):
                dip_sites.append(idx + a)
                frames[idx + a] = frame[a]
        idx += n
    if drism and dip_sites:
        hc0 = ((solvent.dielectric - 1.0) / y - 3.0) / rho_d
        hck = hc0 * np.exp(-k * k * smear * smear / 4.0)
        u = {a: j0(k * frames[a][0]) * j0(k * frames[a][1]) * j1(k * frames[a][2])
             for a in dip_sites}
        for a in dip_sites:
            for b in dip_sites:
                zeta[a, b] = hck * u[a] * u[b]
    r = grid.r
    sig_ab = 0.5 * (sig[:, None] + sig[None, :])
    eps_ab = np.sqrt(eps[:, None] * eps[None, :])
    s6 = (sig_ab[:, :, None] / r) ** 6
    u_lj = 4.0 * eps_ab[:, :, None] * (s6 * s6 - s6)
    qq = q[:, None] * q[None, :]
    # beta u - f: LJ plus the screened (short-range) Coulomb part
    beta_u_sr = beta * (u_lj + COULOMB * qq[:, :, None] * np.exp(-r / SCREEN) / r)
    f_k = beta * COULOMB * qq[:, :, None] * lr_kernel_k(k)
    return dict(q=q, rho=rho, w=w, zeta=zeta, beta=beta, beta_u_sr=beta_u_sr, f_k=f_k,
                y=y, rho_d=rho_d)


def _scaled_charges(solvent, lam: float):
    """Charges scaled by lam; the target dielectric constant scaled as
    1 + lam^2 (eps_r - 1), which keeps the DRISM amplitude hc0 fixed (y ~ lam^2)."""
    species = []
    for sp in solvent.species:
        sites = tuple(dataclasses.replace(st, q=st.q * lam) for st in sp.sites)
        species.append(dataclasses.replace(sp, sites=sites))
    return dataclasses.replace(solvent, species=tuple(species),
                               dielectric=1.0 + lam * lam * (solvent.dielectric - 1.0))


def solve_solvent(solvent, grid: Optional[RadialGrid] = None, closure_kind: str = "kh",
                  drism: bool = True, smear: float = 1.0, tol: float = 1e-12,
                  max_iter: int = 3000, depth: int = 10, eta: float = 0.3,
                  ramp=tuple(round(0.1 * i, 1) for i in range(1, 11)), ramp_tol: float = 1e-6,
                  callback=None) -> SolventResult:
    """Solve the solvent-solvent RISM (XRISM, or DRISM when ``drism``).

    A strongly polar solvent does not converge from tau = 0 at full charge, so
    the charges are switched on in the steps of ``ramp`` (each step starts
    from the previous solution; intermediate steps stop at ``ramp_tol``).  Only
    the last step, at full charge, defines the result."""
    grid = grid or RadialGrid()
    hk = Hankel(grid)
    tau = None
    total_iter = 0
    for step, lam in enumerate(ramp):
        last = step == len(ramp) - 1
        sv = solvent if last else _scaled_charges(solvent, lam)
        st = solvent_setup(sv, grid, drism, smear)
        ns = len(st["q"])
        wbar = st["w"] + st["rho"][:, None, None] * st["zeta"]          # w + rho zeta
        wbar_k = np.moveaxis(wbar, -1, 0)                                 # [K, ns, ns]
        rho_m = np.diag(st["rho"])
        eye = np.eye(ns)

        def rism_k(ck_full):
            """h~bar = (I - wbar c rho)^-1 wbar c wbar for each k (Eq 4 with wbar)."""
            c_k = np.moveaxis(ck_full, -1, 0)
            lhs = eye - wbar_k @ c_k @ rho_m
            rhs = wbar_k @ c_k @ wbar_k
            hbar = np.linalg.solve(lhs, rhs)
            hbar = 0.5 * (hbar + np.swapaxes(hbar, 1, 2))
            return np.moveaxis(hbar, 0, -1)

        def residual(tau_in):
            d = -st["beta_u_sr"] + tau_in
            g = closure(d, closure_kind)
            csr = g - 1.0 - tau_in
            csr_k = hk.forward(csr)
            c_k = csr_k - st["f_k"]
            hbar_k = rism_k(c_k)
            tau_new = hk.inverse(hbar_k + st["zeta"] - csr_k)
            return tau_new - tau_in, g, csr

        tau0 = np.zeros((ns, ns, grid.n - 1)) if tau is None else tau
        res = mdiis_solve(residual, tau0, tol if last else ramp_tol, depth, eta, max_iter,
                          callback=callback)
        if not res.converged:
            raise RuntimeError(f"1D RISM did not converge at charge scale {lam}: rms {res.rms}")
        tau = res.t
        total_iter += res.iterations
    d = -st["beta_u_sr"] + tau
    g = closure(d, closure_kind)
    csr = g - 1.0 - tau
    c_k = hk.forward(csr) - st["f_k"]
    hbar_k = rism_k(c_k)
    chi = wbar + st["rho"][:, None, None] * hbar_k
    # full c = csr - f with f = beta C q q (1 - e^{-r})/r
    r = grid.r
    f_r = st["beta"] * COULOMB * (st["q"][:, None] * st["q"][None, :])[:, :, None] \
        * (-np.expm1(-r / SCREEN) / r)
    return SolventResult(grid, chi, g - 1.0, csr - f_r, total_iter, res.rms,
                         closure_kind, drism, solvent.dielectric if drism else None, smear)


def bulk_pressure(solvent, res: SolventResult) -> float:
    """Eq 20, the pressure of the bulk solvent in kcal/(mol A^3):
        P = sum_G rho_G (n_G + 1) / (2 beta)
            - (2 pi / beta) sum_{g,l} rho_g rho_l int_0^inf c_gl(r) r^2 dr,
    G over species (molecular density rho_G, n_G sites), g and l over sites,
    c the full direct correlation of the 1D solution.  The radial integral is
    the sum dr sum_i c(r_i) r_i^2 over the grid (the end point r = 0 adds
    nothing).  The Coulomb tails -beta C q_g q_l (1 - e^{-r})/r of c cancel in
    the double sum of an electroneutral solvent, sum_g rho_g q_g = 0."""
    beta = beta_of(solvent.temperature)
    rho = solvent.site_arrays()[3]
    r = res.grid.r
    integral = res.grid.dr * np.sum(res.c * r * r, axis=-1)
    ideal = sum(sp.density * (len(sp.sites) + 1) for sp in solvent.species) / (2.0 * beta)
    return float(ideal - (2.0 * math.pi / beta) * np.einsum("a,b,ab->", rho, rho, integral))


def compressibility(solvent, res: SolventResult) -> float:
    """Isothermal compressibility chi_T of the solvent (the input of Eq 19), in
    A^3 mol / kcal, from the k -> 0 limit of the site-site structure of its
    first species G: rho_G k_B T chi_T = S(0), with S(k) the mean over the
    site pairs of G of chi_gl(k) = w_gl + rho h_gl, extrapolated to k = 0 as
    (4 S(k_1) - S(k_2)) / 3 (S is even in k).  For one species this is the
    compressibility route 1 + rho h~(0); with dissolved ions it is read as
    the compressibility of the first (solvent) species."""
    beta = beta_of(solvent.temperature)
    n = len(solvent.species[0].sites)
    s1 = float(np.mean(res.chi[:n, :n, 0]))
    s2 = float(np.mean(res.chi[:n, :n, 1]))
    return ((4.0 * s1 - s2) / 3.0) * beta / solvent.species[0].density


def charge_structure(solvent, chi: np.ndarray) -> np.ndarray:
    """S_qq(k) = sum_ab q_a rho_b chi_ab(k) q_b (chi_ab = w_ab + rho_a h_ab)."""
    q, _, _, rho = solvent.site_arrays()
    return np.einsum("a,b,abk,b->k", q, rho, chi, q)


def dielectric_from_chi(solvent, chi: np.ndarray, k: np.ndarray) -> float:
    """eps from the k -> 0 charge-charge structure factor
    S_qq = sum_ab q_a q_b (rho_a w_ab + rho_a rho_b h_ab) = sum_ab q_a rho_b chi_ab q_b:
    (eps - 1)/eps = lim 4 pi beta C S_qq / k^2, evaluated at k_1 and k_2 and
    extrapolated quadratically to k = 0."""
    s = charge_structure(solvent, chi[:, :, :2])
    beta = beta_of(solvent.temperature)
    x = 4.0 * math.pi * beta * COULOMB * s / k[:2] ** 2
    x0 = (4.0 * x[0] - x[1]) / 3.0
    return 1.0 / (1.0 - x0)


# ---------------------------------------------------------------------------
# Solute-solvent 1D RISM (Eq 8, one spherical solute site) and Eq 9/10
# ---------------------------------------------------------------------------


@dataclasses.dataclass
class SoluteSolventResult:
    r: np.ndarray
    g: np.ndarray     # [n_v, N-1]
    h: np.ndarray
    c: np.ndarray     # full c
    sfe: float
    sfe_site: np.ndarray
    iterations: int
    rms: float


def solve_solute_1d(solute_q: float, solute_sigma: float, solute_eps: float, solvent,
                    chi_table: np.ndarray, grid: Optional[RadialGrid] = None,
                    closure_kind: str = "kh", pse_order: int = 3, tol: float = 1e-12,
                    max_iter: int = 2000, depth: int = 5, eta: float = 0.7):
    """h_g = sum_g' c_g' * chi_g'g for one spherical solute site; chi_table on
    k_m = m dk, m = 0..N-1 (the table is read at m = 1..N-1, the DST grid)."""
    grid = grid or RadialGrid()
    hk = Hankel(grid)
    q, sig, eps, rho = solvent.site_arrays()
    beta = beta_of(solvent.temperature)
    r = grid.r
    sig_g = 0.5 * (solute_sigma + sig)
    eps_g = np.sqrt(solute_eps * eps)
    s6 = (sig_g[:, None] / r) ** 6
    u = 4.0 * eps_g[:, None] * (s6 * s6 - s6) + COULOMB * solute_q * q[:, None] / r
    f = beta * COULOMB * solute_q * q[:, None] * (-np.expm1(-r / SCREEN) / r)
    f_k = beta * COULOMB * solute_q * q[:, None] * lr_kernel_k(grid.k)
    beta_u = np.minimum(beta * u, 1.0e4)
    chi = chi_table[:, :, 1:]

    def residual(tau):
        t = tau + f
        d = -beta_u + t
        g = closure(d, closure_kind, pse_order)
        csr = g - 1.0 - tau
        c_k = hk.forward(csr) - f_k
        h_k = np.einsum("ak,abk->bk", c_k, chi)
        h = hk.inverse(h_k)
        return h + 1.0 - g, g, h

    tau0 = np.zeros((len(q), grid.n - 1))
    res = mdiis_solve(residual, tau0, tol, depth, eta, max_iter)
    t = res.t + f
    d = -beta_u + t
    g = closure(d, closure_kind, pse_order)
    h = g - 1.0
    c = g - 1.0 - t
    phi = sfe_density(h, c, d, closure_kind, pse_order)
    per_site = rho * 4.0 * math.pi * grid.dr * np.sum(phi * r * r, axis=1) / beta
    return SoluteSolventResult(r, g, h, c, float(per_site.sum()), per_site,
                               res.iterations, res.rms)
