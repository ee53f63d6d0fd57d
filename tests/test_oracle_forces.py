"""Pins of the oracle's solvation free-energy gradient (the solvent term of
the derivative of the MM/3D-RISM free energy, Eq 23): it must be the
derivative of quantities the oracle computes independently."""
import copy
import math

import numpy as np
import pytest

from oracle import rism3d as O
from paper_2403_01039_amd import inputs as I


def _energy(prob, g):
    """sum_g rho_g dV sum_n g_g(r_n) u_g(r_n) with g held fixed (Eq 22 via the
    oracle's potential, pinned by its own tests)."""
    rho = prob.solvent.site_arrays()[3]
    u, _ = O.potential_at(prob.solute, prob.solvent, O.grid_points(prob.grid))
    return float(sum(rho[s] * np.sum(g[s] * u[s]) for s in range(len(rho)))) * prob.grid.spacing ** 3


def test_gradient_is_the_derivative_of_the_potential_energy_in_a_fixed_distribution():
    """For a fixed g the gradient equals d/dR_a of sum rho dV sum g u: central
    differences of the oracle potential, charged atoms in saline (five sites
    with two densities), every atom and component."""
    prob = I.small_problem(41, n_atoms=4, shape=(14, 12, 10), radius=1.5, saline=True)
    g = I.synthetic_distribution(prob, 7).astype(np.float64)
    grad = O.sfe_gradient(prob, g)
    h = 1e-5
    fd = np.zeros_like(grad)
    for a in range(prob.solute.n_atoms):
        for k in range(3):
            pp, pm = copy.deepcopy(prob), copy.deepcopy(prob)
            pp.solute.xyz[a, k] += h
            pm.solute.xyz[a, k] -= h
            fd[a, k] = (_energy(pp, g) - _energy(pm, g)) / (2 * h)
    assert np.abs(grad - fd).max() <= 1e-7 * np.abs(fd).max()


def _stationarity_deviation(kind, order=3, eta=0.7, components=((0, 0), (0, 2), (1, 1))):
    """Largest |dF/dR_a - grad_a| / max|grad| over the listed components, with
    F the oracle's free energy (Eq 17, Eq 18 or PSE-n) of whole solves of an
    uncharged two-atom solute in water and grad the gradient formula at the
    solved g."""
    prob = I.small_problem(12, n_atoms=2, shape=(14, 14, 14), radius=1.2, closure=kind)
    prob.solute.q[:] = 0.0
    prob.options.pse_order = order
    prob.options.mdiis_eta = eta
    chi, dk = I.solvent_table("water")

    def solved(p):
        sol = O.solve(O.build_system(p, chi, dk), tol=1e-12, max_iter=5000)
        return O.sfe(sol)[0], sol

    _, sol = solved(prob)
    grad = O.sfe_gradient(prob, sol.g)
    h = 1e-4
    worst = 0.0
    for a, k in components:
        pp, pm = copy.deepcopy(prob), copy.deepcopy(prob)
        pp.solute.xyz[a, k] += h
        pm.solute.xyz[a, k] -= h
        fd = (solved(pp)[0] - solved(pm)[0]) / (2 * h)
        worst = max(worst, abs(grad[a, k] - fd) / np.abs(grad).max())
    return worst


@pytest.mark.parametrize("kind,order,eta", [("kh", 1, 0.7), ("hnc", 1, 0.4), ("pse", 3, 0.7),
                                            ("pse", 2, 0.7)])
def test_gradient_is_the_derivative_of_the_free_energy_for_a_neutral_solute(kind, order, eta):
    """For an uncharged solute each closure's discrete free energy (Eq 18 for
    KH, Eq 17 for HNC, the Kast-Kloss form for PSE-n) is stationary in h and c
    at its fixed point (the OZ operator with the symmetric water table is
    self-adjoint), so its derivative in R_a is exactly the gradient formula at
    the solved g: central differences of whole solves agree to the
    finite-difference error (measured 5e-9 to 3e-8 relative).  This pins the
    factors 1/2 of Eq 17-18 and the PSE-n term Theta(h) d^(n+1)/(n+1)!."""
    assert _stationarity_deviation(kind, order, eta) <= 1e-6


def _planted_hnc(h, c, d, kind, order=3):
    """Eq 17 without its factors 1/2 (h = c only in the chi = 1 limit, where the
    two mistakes cancel)."""
    return -c - h * c + h * h


def _planted_pse_power(h, c, d, kind, order=3):
    """The PSE-n term with d^n / n! in place of d^(n+1) / (n+1)!."""
    return -c - 0.5 * h * c + 0.5 * h * h - (h > 0.0) * d ** order / math.factorial(order)


def _planted_pse_factorial(h, c, d, kind, order=3):
    """The PSE-n term with the power right and the factorial one order low."""
    return -c - 0.5 * h * c + 0.5 * h * h - (h > 0.0) * d ** (order + 1) / math.factorial(order)


@pytest.mark.parametrize("kind,planted", [("hnc", _planted_hnc), ("pse", _planted_pse_power),
                                          ("pse", _planted_pse_factorial)])
def test_stationarity_pin_catches_planted_free_energy_mistakes(monkeypatch, kind, planted):
    """Each planted mistake in the free-energy density breaks the stationarity
    pin above by orders of magnitude (measured 2e-2 to 0.15 relative against
    the 1e-6 bar)."""
    monkeypatch.setattr(O, "sfe_density", planted)
    assert _stationarity_deviation(kind, 3, 0.4 if kind == "hnc" else 0.7,
                                   components=((0, 0),)) > 1e-3


def test_symmetric_distribution_exerts_no_net_gradient():
    """One charged atom at the centre of the grid's point symmetry (half a
    spacing below the centre point on each axis) in a g that is 1 beyond 1.5 A
    and 0 inside: the pair terms cancel in mirror pairs, while the same g
    about an atom moved by 0.1 A does not."""
    prob = I.small_problem(1, n_atoms=1, shape=(12, 12, 12))
    centre = np.array(prob.grid.center) - 0.5 * prob.grid.spacing
    prob.solute.xyz[0] = centre
    prob.solute.q[0] = 0.7
    d = np.sqrt(np.sum((O.grid_points(prob.grid) - centre) ** 2, axis=-1))
    g = np.broadcast_to((d >= 1.5).astype(np.float64), (3,) + prob.grid.shape)
    grad = O.sfe_gradient(prob, g)
    prob.solute.xyz[0] = centre + np.array([0.1, 0.0, 0.0])
    moved = O.sfe_gradient(prob, g)
    assert abs(moved[0, 0]) > 1e-3
    assert np.abs(grad).max() <= 1e-12 * abs(moved[0, 0])


def test_clamped_pairs_do_not_contribute():
    """An atom exactly on a grid point: that pair sits inside the 0.01 A clamp,
    where the potential does not depend on R_a; the gradient equals the one
    with g zeroed at that point."""
    prob = I.small_problem(3, n_atoms=1, shape=(10, 10, 10))
    prob.solute.xyz[0] = np.array(prob.grid.center) + np.array([1.0, -0.5, 0.5])
    g = I.synthetic_distribution(prob, 3, exclusion=0.0).astype(np.float64)
    ix, iy, iz = 5 + 2, 5 - 1, 5 + 1
    assert g[:, iz, iy, ix].min() > 0.0
    a = O.sfe_gradient(prob, g)
    g[:, iz, iy, ix] = 0.0
    b = O.sfe_gradient(prob, g)
    assert np.array_equal(a, b)
