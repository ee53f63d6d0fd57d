"""FP64 3D-RISM oracle (test infrastructure only; never called by the library).

Follows arXiv 2403.01039, sections "Theory" (3D-RISM equation Eq 13, closures
Eq 14-16, solvation free energy Eq 17-18), "Hybrid implementation" (MM
solute-solvent potential Eq 22) and "Numerical procedure" (long-range split
Eq 29-30, half-integer k grid, solution steps 1-7 with Eq 31-33), plus the
MDIIS accelerator of "Convergence acceleration" (Eq 40, read as the
Kovalenko-Ten-no-Hirata form below).

Readings where the paper is silent or garbled:
* KH closure: g = exp(d) for d <= 0 and 1 + d for d > 0 (the printed Eq 15
  has the two branches swapped; Eq 6 uses the threshold 1).
* Units: kcal/mol, Angstrom, e; Coulomb factor C = 332.0637133 kcal A/(mol e^2)
  (absent from Eq 22); k_B = 0.0019872043 kcal/(mol K).
* LJ mixing (Eq 22 "usual meanings"): Lorentz-Berthelot.
* Screening length of Eq 29-30: l = 1 A.
* Distances are clamped at 0.01 A in the potential and beta*u is capped at
  1e4 before the long-range part is subtracted.
* Grid: r_a = r0 + a dr with r0 = centre - (n div 2) dr; k_j = (j + 1/2) dk
  for j < n/2 and (j + 1/2 - n) dk otherwise, dk = 2 pi / (n dr).
* The RMS of Eq 41 is taken as the true root-mean-square of the residual
  R = t' - t of step 5 (Eq 33), over all grid points and solvent sites.
* MDIIS: keep up to M pairs (t_i, R_i); minimise |sum c_i R_i|^2 subject to
  sum c_i = 1 (Lagrange multiplier, Gram matrix normalised by its largest
  diagonal, FP64 Gaussian elimination with partial pivoting); next
  t = sum c_i (t_i + eta R_i); first step Picard; ring buffer; restart
  (keep the stored pair of smallest RMS) when a pivot is below 1e-12 or the
  new RMS exceeds 10x the smallest stored RMS (the new pair is then dropped).
* chi_{g'g}(|k|) is linearly interpolated from a uniform radial k table;
  beyond the table the last value is held.
* PSE-n (Kast & Kloss, J. Chem. Phys. 129, 236101 (2008); not in the paper):
  g = exp(d) for d <= 0, sum_{i<=n} d^i / i! for d > 0, with free-energy
  density -c - hc/2 + h^2/2 - Theta(h) d^(n+1)/(n+1)!.
* Free energy: box sum dV * sum_n, h = g - 1, c = g - 1 - t (full c), no tail
  correction.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

from . import fft as offt

COULOMB = 332.0637133        # kcal A / (mol e^2)
KBOLTZ = 0.0019872043        # kcal / (mol K)
SCREEN = 1.0                 # A, screening length l of Eq 29-30
D_MIN = 0.01                 # A, distance clamp in Eq 22
BETA_U_CAP = 1.0e4           # cap on beta*u before f is subtracted


def beta_of(temperature: float) -> float:
    return 1.0 / (KBOLTZ * temperature)


# ---------------------------------------------------------------------------
# Grid (section "Numerical procedure": k at half-integer points, r at integers)
# ---------------------------------------------------------------------------


def axis_r(n: int, dr: float, centre: float) -> np.ndarray:
    return centre - (n // 2) * dr + dr * np.arange(n)


def axis_k(n: int, dr: float) -> np.ndarray:
    dk = 2.0 * np.pi / (n * dr)
    j = np.arange(n)
    return np.where(j < n / 2.0, (j + 0.5) * dk, (j + 0.5 - n) * dk)


def grid_points(grid) -> np.ndarray:
    """All r-grid points as [nz, ny, nx, 3] (x, y, z)."""
    x = axis_r(grid.nx, grid.spacing, grid.center[0])
    y = axis_r(grid.ny, grid.spacing, grid.center[1])
    z = axis_r(grid.nz, grid.spacing, grid.center[2])
    zz, yy, xx = np.meshgrid(z, y, x, indexing="ij")
    return np.stack([xx, yy, zz], axis=-1)


def k_components(grid):
    kx = axis_k(grid.nx, grid.spacing)[None, None, :]
    ky = axis_k(grid.ny, grid.spacing)[None, :, None]
    kz = axis_k(grid.nz, grid.spacing)[:, None, None]
    return kx, ky, kz


def k_magnitude(grid) -> np.ndarray:
    kx, ky, kz = k_components(grid)
    return np.sqrt(kx * kx + ky * ky + kz * kz)


# ---------------------------------------------------------------------------
# Eq 22 (solute-solvent potential) and Eq 29 (long-range part)
# ---------------------------------------------------------------------------


def lr_kernel(d: np.ndarray) -> np.ndarray:
    """(1 - exp(-d/l)) / d, with its limit 1/l at d = 0 (Eq 29)."""
    d = np.asarray(d, dtype=np.float64)
    out = np.empty_like(d)
    small = d < 1e-300
    out[small] = 1.0 / SCREEN
    ds = d[~small]
    out[~small] = -np.expm1(-ds / SCREEN) / ds
    return out


def potential_at(solute, solvent, points: np.ndarray):
    """Eq 22 and Eq 29 at arbitrary points [..., 3].

    Returns (u [n_v, ...] kcal/mol, phi_lr [...] e/A) where
      u_g(r)  = sum_a [ C q_a q_g / d + 4 eps_ag ((sig_ag/d)^12 - (sig_ag/d)^6) ],
                d = max(|r - R_a|, 0.01 A), sig_ag = (sig_a + sig_g)/2,
                eps_ag = sqrt(eps_a eps_g);
      phi_lr  = sum_a q_a (1 - exp(-|r - R_a|/l)) / |r - R_a|,
    so that f_g = beta C q_g phi_lr."""
    q_v, sig_v, eps_v, _ = solvent.site_arrays()
    pts = np.asarray(points, dtype=np.float64)
    shape = pts.shape[:-1]
    u = np.zeros((len(q_v),) + shape)
    phi = np.zeros(shape)
    for a in range(solute.n_atoms):
        diff = pts - solute.xyz[a]
        dist = np.sqrt(np.sum(diff * diff, axis=-1))
        dc = np.maximum(dist, D_MIN)
        for g in range(len(q_v)):
            sig = 0.5 * (solute.sigma[a] + sig_v[g])
            eps = math.sqrt(solute.eps[a] * eps_v[g])
            s6 = (sig / dc) ** 6
            u[g] += COULOMB * solute.q[a] * q_v[g] / dc + 4.0 * eps * (s6 * s6 - s6)
        phi += solute.q[a] * lr_kernel(dist)
    return u, phi


def ftilde_unit(solute, grid, beta: float) -> np.ndarray:
    """Eq 30 without the solvent charge: F(k) = (4 pi beta C / l^2) sum_a q_a
    exp(-i k . (R_a - r0)) / (|k|^2 (|k|^2 + l^-2)), so f~_g = q_g F.  The phase
    is taken relative to the grid corner r0, the origin of the discrete
    transform."""
    kx, ky, kz = k_components(grid)
    k2 = kx * kx + ky * ky + kz * kz
    r0 = np.array([axis_r(grid.nx, grid.spacing, grid.center[0])[0],
                   axis_r(grid.ny, grid.spacing, grid.center[1])[0],
                   axis_r(grid.nz, grid.spacing, grid.center[2])[0]])
    s = np.zeros(k2.shape, dtype=np.complex128)
    for a in range(solute.n_atoms):
        rel = solute.xyz[a] - r0
        s += solute.q[a] * np.exp(-1j * (kx * rel[0] + ky * rel[1] + kz * rel[2]))
    return (4.0 * np.pi * beta * COULOMB / SCREEN ** 2) * s / (k2 * (k2 + 1.0 / SCREEN ** 2))


# ---------------------------------------------------------------------------
# Closures (Eq 14-16, KH reading, PSE-n) and free-energy densities (Eq 17-18)
# ---------------------------------------------------------------------------


def closure(d: np.ndarray, kind: str, order: int = 3) -> np.ndarray:
    d = np.asarray(d, dtype=np.float64)
    e = np.exp(np.minimum(d, 0.0))
    if kind == "hnc":
        return np.exp(d)
    if kind == "kh":
        return np.where(d <= 0.0, e, 1.0 + d)
    if kind == "pse":
        series = np.zeros_like(d)
        term = np.ones_like(d)
        for i in range(order + 1):
            if i:
                term = term * d / i
            series = series + term
        return np.where(d <= 0.0, e, series)
    raise ValueError(kind)


def sfe_density(h, c, d, kind: str, order: int = 3) -> np.ndarray:
    """The bracket of Eq 17 (HNC), Eq 18 (KH) and its PSE-n analogue."""
    base = -c - 0.5 * h * c
    if kind == "hnc":
        return base + 0.5 * h * h
    if kind == "kh":
        return base + 0.5 * h * h * (h < 0.0)
    if kind == "pse":
        return base + 0.5 * h * h - (h > 0.0) * d ** (order + 1) / math.factorial(order + 1)
    raise ValueError(kind)


# ---------------------------------------------------------------------------
# The discretised 3D-RISM map (steps 2-5, Eq 31-33)
# ---------------------------------------------------------------------------


def chi_interp(chi_table: np.ndarray, dk_table: float, kmag: np.ndarray) -> np.ndarray:
    """chi_{g'g}(|k|) by linear interpolation on the uniform table
    chi_table[g'][g][m] = chi_{g'g}(m dk_table); the last value is held beyond
    the table.  Returns [n_v, n_v, *kmag.shape]."""
    n_k = chi_table.shape[-1]
    x = np.minimum(kmag / dk_table, n_k - 1.0)
    m = np.minimum(np.floor(x).astype(np.int64), n_k - 2)
    fr = x - m
    return chi_table[:, :, m] * (1.0 - fr) + chi_table[:, :, m + 1] * fr


@dataclasses.dataclass
class System:
    """Everything the map F of steps 2-5 needs, for one solute on one grid."""
    problem: object
    beta: float
    dv: float
    beta_u: np.ndarray       # [n_v, nz, ny, nx], capped at 1e4
    f: np.ndarray            # [n_v, nz, ny, nx]  Eq 29
    ftilde: np.ndarray       # [n_v, nz, ny, nx]  Eq 30 (complex, relative to r0)
    chi: np.ndarray          # [n_v, n_v, nz, ny, nx] chi_{g'g}(|k|)
    kind: str
    order: int

    @property
    def n_sites(self) -> int:
        return self.beta_u.shape[0]


def build_system(problem, chi_table: np.ndarray, dk_table: float) -> System:
    grid = problem.grid
    solvent = problem.solvent
    beta = beta_of(solvent.temperature)
    q_v = solvent.site_arrays()[0]
    u, phi = potential_at(problem.solute, solvent, grid_points(grid))
    beta_u = np.minimum(beta * u, BETA_U_CAP)
    f = beta * COULOMB * q_v[:, None, None, None] * phi[None]
    fu = ftilde_unit(problem.solute, grid, beta)
    ftilde = q_v[:, None, None, None] * fu[None]
    chi = chi_interp(np.asarray(chi_table, dtype=np.float64), dk_table, k_magnitude(grid))
    dv = grid.spacing ** 3
    opts = problem.options
    return System(problem, beta, dv, beta_u, f, ftilde, chi, opts.closure, opts.pse_order)


def rism_map(sys_: System, t: np.ndarray):
    """One pass of steps 2-5 on t (t-form).  Returns (R, g, h) with
    R = t' - t = h + 1 - g (Eq 33)."""
    d = -sys_.beta_u + t                                # Eq 16
    g = closure(d, sys_.kind, sys_.order)               # Eq 14 / KH / PSE-n
    csr = g - 1.0 - t + sys_.f                          # Eq 31
    ck = offt.forward3(csr, sys_.dv) - sys_.ftilde      # Eq 32
    hk = np.einsum("ab...,a...->b...", sys_.chi, ck)    # Eq 13: h_g = sum_g' c_g' chi_g'g
    h = offt.inverse3(hk, sys_.dv).real
    R = h + 1.0 - g                                     # Eq 33: t' - t
    return R, g, h


def rms_of(R: np.ndarray) -> float:
    """Root-mean-square residual over grid points and sites (Eq 41 reading)."""
    return float(np.sqrt(np.sum(R * R) / R.size))


# ---------------------------------------------------------------------------
# MDIIS (Eq 40, Kovalenko-Ten-no-Hirata reading)
# ---------------------------------------------------------------------------


def mdiis_coefficients(residuals):
    """Minimise |sum c_i R_i|^2 subject to sum c_i = 1.  Solves the bordered
    system [[B, -1], [-1^T, 0]] [c; lam] = [0; -1] with B_ij = <R_i, R_j>
    normalised by max_i B_ii, by Gaussian elimination with partial pivoting.
    Returns (c, min_abs_pivot)."""
    m = len(residuals)
    B = np.empty((m, m))
    for i in range(m):
        for j in range(m):
            B[i, j] = float(np.sum(residuals[i] * residuals[j]))
    return solve_bordered(B)


def solve_bordered(B: np.ndarray):
    m = B.shape[0]
    scale = float(np.max(np.diag(B)))
    if not scale > 0.0:
        return np.full(m, 1.0 / m), 0.0
    A = np.zeros((m + 1, m + 1))
    A[:m, :m] = B / scale
    A[:m, m] = -1.0
    A[m, :m] = -1.0
    rhs = np.zeros(m + 1)
    rhs[m] = -1.0
    n = m + 1
    min_piv = np.inf
    for col in range(n):
        piv = col + int(np.argmax(np.abs(A[col:, col])))
        if piv != col:
            A[[col, piv]] = A[[piv, col]]
            rhs[[col, piv]] = rhs[[piv, col]]
        p = A[col, col]
        min_piv = min(min_piv, abs(p))
        if abs(p) < 1e-300:
            return np.full(m, 1.0 / m), 0.0
        for row in range(col + 1, n):
            fac = A[row, col] / p
            A[row, col:] -= fac * A[col, col:]
            rhs[row] -= fac * rhs[col]
    sol = np.zeros(n)
    for row in range(n - 1, -1, -1):
        sol[row] = (rhs[row] - A[row, row + 1:] @ sol[row + 1:]) / A[row, row]
    return sol[:m], min_piv


@dataclasses.dataclass
class SolveResult:
    t: np.ndarray
    R: np.ndarray
    g: np.ndarray
    h: np.ndarray
    iterations: int
    rms: float
    restarts: int
    converged: bool
    rms_history: list


def mdiis_solve(residual_fn, x0: np.ndarray, tol: float, depth: int, eta: float,
                max_iter: int, eta_dynamic: bool = False, callback=None) -> SolveResult:
    """Generic MDIIS iteration x -> x' on R(x) = F(x) - x (steps 6-7).
    ``residual_fn(x)`` returns (R, *extras).  Stops when RMS(R) < tol and
    returns the iterate whose residual passed."""
    hist = []          # list of [x, R, rms]
    x = x0
    restarts = 0
    history = []
    for it in range(1, max_iter + 1):
        out = residual_fn(x)
        R = out[0]
        rms = rms_of(R)
        history.append(rms)
        if callback is not None:
            callback(it, rms)
        if not np.isfinite(rms):
            raise FloatingPointError(f"non-finite residual at iteration {it}")
        if rms < tol:
            return SolveResult(x, R, out[1], out[2], it, rms, restarts, True, history)
        if it == max_iter:
            return SolveResult(x, R, out[1], out[2], it, rms, restarts, False, history)
        if hist and rms > 10.0 * min(hp[2] for hp in hist):
            best = min(hist, key=lambda hp: hp[2])
            hist = [best]
            restarts += 1
        else:
            hist.append([x, R, rms])
            if len(hist) > depth:
                hist.pop(0)
        c, piv = mdiis_coefficients([hp[1] for hp in hist])
        if len(hist) > 1 and piv < 1e-12:
            best = min(hist, key=lambda hp: hp[2])
            hist = [best]
            restarts += 1
            c = np.ones(1)
        step = eta
        if eta_dynamic:
            step = min(max(-0.2 * math.log(rms), 0.1), 1.0)
        x = sum(ci * (hp[0] + step * hp[1]) for ci, hp in zip(c, hist))
    raise AssertionError("unreachable")


# ---------------------------------------------------------------------------
# Modified Anderson with two histories (Eq 34-39), the paper's GPU accelerator
# ---------------------------------------------------------------------------


def anderson_theta(R0, R1, R2, weight):
    """theta of Eq 36, read as the normal equations of the least-squares
    problem min |R0 - sum_i theta_i (R0 - R_i)| in the weighted inner product
    of Eq 38: sum_j (D_j, D_i) theta_j = (R0, D_i), D_i = R0 - R_i.  Returns
    None when the 2x2 system is singular (relative determinant < 1e-12)."""
    ip = lambda a, b: float(np.sum(a * b * weight))
    D1, D2 = R0 - R1, R0 - R2
    a11, a12, a22 = ip(D1, D1), ip(D1, D2), ip(D2, D2)
    r1, r2 = ip(R0, D1), ip(R0, D2)
    det = a11 * a22 - a12 * a12
    if not abs(det) > 1e-12 * max(a11 * a22, 1e-300):
        return None
    return np.array([(r1 * a22 - r2 * a12) / det, (a11 * r2 - a12 * r1) / det])


def anderson_solve(residual_fn, x0: np.ndarray, tol: float, s, b: float, weight,
                   max_iter: int, callback=None) -> SolveResult:
    """Modified Anderson iteration on R(X) = Y - X with Y = F(X) (Eq 37):
    Picard X <- X + b R for the first two steps, then with the three newest
    inputs X^(n-1), X^(n-2), X^(n-3) and their outputs
        u = X^(n-1) + sum_i (theta_i + s_i) (X^(n-i-1) - X^(n-1))     (Eq 34)
        v = Y^(n)   + sum_i (theta_i + s_i) (Y^(n-i)   - Y^(n))        (Eq 35)
        X^(n) = u + b (v - u)                                          (Eq 39)
    A singular theta system falls back to a Picard step.  Stops when RMS(R)
    < tol and returns the iterate whose residual passed."""
    hist = []          # [x, R], newest last
    x = x0
    history = []
    for it in range(1, max_iter + 1):
        out = residual_fn(x)
        R = out[0]
        rms = rms_of(R)
        history.append(rms)
        if callback is not None:
            callback(it, rms)
        if not np.isfinite(rms):
            raise FloatingPointError(f"non-finite residual at iteration {it}")
        if rms < tol:
            return SolveResult(x, R, out[1], out[2], it, rms, 0, True, history)
        if it == max_iter:
            return SolveResult(x, R, out[1], out[2], it, rms, 0, False, history)
        hist.append([x, R])
        if len(hist) > 3:
            hist.pop(0)
        theta = None
        if len(hist) == 3:
            (X2, R2), (X1, R1), (X0, R0) = hist
            theta = anderson_theta(R0, R1, R2, weight)
        if theta is None:
            x = x + b * R
            continue
        Y0, Y1, Y2 = X0 + R0, X1 + R1, X2 + R2
        k1, k2 = theta[0] + s[0], theta[1] + s[1]
        u = X0 + k1 * (X1 - X0) + k2 * (X2 - X0)
        v = Y0 + k1 * (Y1 - Y0) + k2 * (Y2 - Y0)
        x = u + b * (v - u)
    raise AssertionError("unreachable")


# ---------------------------------------------------------------------------
# Solve (steps 1-7) and thermodynamics (Eq 17-18)
# ---------------------------------------------------------------------------


@dataclasses.dataclass
class Solution:
    system: System
    t: np.ndarray
    g: np.ndarray
    h: np.ndarray
    c: np.ndarray
    iterations: int
    rms: float
    restarts: int
    converged: bool
    rms_history: list

    @property
    def tau(self) -> np.ndarray:
        """t - f, the short-range indirect correlation."""
        return self.t - self.system.f


def solve(sys_: System, tol: Optional[float] = None, tau0: Optional[np.ndarray] = None,
          max_iter: Optional[int] = None, depth: Optional[int] = None,
          eta: Optional[float] = None, callback=None) -> Solution:
    """Step 1: t0 = f (tau0 = t0 - f = 0 unless a start is supplied); steps 2-7
    with MDIIS, or with modified Anderson when the options ask for it.  Returns the converged t together with g, h = g - 1 and
    c = g - 1 - t."""
    opts = sys_.problem.options
    tol = opts.tol if tol is None else tol
    t0 = sys_.f.copy() if tau0 is None else sys_.f + tau0
    if getattr(opts, "accelerator", "mdiis") == "anderson":
        # Eq 38: inner product weighted by 1 / rho of each solvent site
        rho = sys_.problem.solvent.site_arrays()[3]
        weight = (1.0 / rho)[:, None, None, None]
        res = anderson_solve(lambda t: rism_map(sys_, t), t0, tol,
                             (opts.anderson_s1, opts.anderson_s2),
                             opts.mdiis_eta if eta is None else eta, weight,
                             opts.max_iter if max_iter is None else max_iter, callback)
    else:
        res = mdiis_solve(lambda t: rism_map(sys_, t), t0, tol,
                          opts.mdiis_depth if depth is None else depth,
                          opts.mdiis_eta if eta is None else eta,
                          opts.max_iter if max_iter is None else max_iter,
                          opts.eta_dynamic, callback)
    d = -sys_.beta_u + res.t
    g = closure(d, sys_.kind, sys_.order)
    h = g - 1.0
    c = g - 1.0 - res.t
    return Solution(sys_, res.t, g, h, c, res.iterations, res.rms, res.restarts,
                    res.converged, res.rms_history)


def sfe_gradient(problem, g: np.ndarray, atoms=None) -> np.ndarray:
    """Solvent term of the derivative of the MM/3D-RISM free energy with
    respect to a solute atom position (section "Hybrid implementation", the
    derivative of Eq 23):

        d(dmu)/dR_a = sum_g rho_g int g_g(r) du_g(r)/dR_a dr,

    u_g from Eq 22 (pairs inside the 0.01 A clamp contribute nothing, since
    the clamped pair term does not depend on R_a there), the integral as the
    box sum dV sum_n.  g is any distribution [n_v, nz, ny, nx].  Returns
    [n_atoms, 3] in kcal/(mol A) (or the rows of the listed ``atoms``); the
    solvation force is its negative."""
    solute = problem.solute
    q_v, sig_v, eps_v, rho = problem.solvent.site_arrays()
    pts = grid_points(problem.grid)
    dv = problem.grid.spacing ** 3
    g = np.asarray(g, dtype=np.float64)
    atoms = range(solute.n_atoms) if atoms is None else list(atoms)
    out = np.zeros((len(atoms), 3))
    for row, a in enumerate(atoms):
        diff = pts - solute.xyz[a]                       # r - R_a
        dist = np.sqrt(np.sum(diff * diff, axis=-1))
        live = dist >= D_MIN
        d = np.where(live, dist, 1.0)
        weight = np.zeros(dist.shape)                    # sum_g rho_g g_g (du_g/dd) / d
        for s_ in range(len(q_v)):
            sig = 0.5 * (solute.sigma[a] + sig_v[s_])
            eps = math.sqrt(solute.eps[a] * eps_v[s_])
            sr6 = (sig / d) ** 6
            # derivative in d of the pair term of Eq 22
            du_dd = (-COULOMB * solute.q[a] * q_v[s_] / (d * d)
                     + 4.0 * eps * (-12.0 * sr6 * sr6 + 6.0 * sr6) / d)
            weight += rho[s_] * g[s_] * du_dd / d
        weight = np.where(live, weight, 0.0)
        # du/dR_a = (du/dd) (R_a - r) / d
        out[row] = -dv * np.sum(weight[..., None] * diff, axis=(0, 1, 2))
    return out


def pmv(sol: Solution, compressibility: float):
    """Eq 19: the partial molar volume k_B T chi_T (1 - sum_g rho_g int c_g dr)
    in A^3, with c = g - 1 - t (full c) and the integral as the box sum
    dV sum_n.  Returns (pmv, per-site rho_g int c_g dr)."""
    sys_ = sol.system
    rho = sys_.problem.solvent.site_arrays()[3]
    rho_int_c = np.array([rho[g] * sys_.dv * float(np.sum(sol.c[g]))
                          for g in range(sys_.n_sites)])
    return compressibility / sys_.beta * (1.0 - float(np.sum(rho_int_c))), rho_int_c


def pressure_correction(pmv_value: float, pressure: float) -> float:
    """Eq 21: the PC term -P V of the free energy, kcal/mol (P in kcal/(mol A^3))."""
    return -pressure * pmv_value


def sfe(sol: Solution):
    """Eq 17 / 18 (and the PSE-n form): k_B T sum_g rho_g dV sum_n Phi.
    Returns (total, per_site) in kcal/mol."""
    sys_ = sol.system
    rho = sys_.problem.solvent.site_arrays()[3]
    d = -sys_.beta_u + sol.t
    phi = sfe_density(sol.h, sol.c, d, sys_.kind, sys_.order)
    per_site = np.array([rho[g] * sys_.dv * float(np.sum(phi[g])) for g in range(sys_.n_sites)])
    per_site /= sys_.beta
    return float(np.sum(per_site)), per_site
