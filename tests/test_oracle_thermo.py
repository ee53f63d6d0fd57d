"""Pins of the oracle's bulk pressure (Eq 20), compressibility, partial molar
volume (Eq 19) and PC term (Eq 21) against the ideal gas, the second virial
coefficient and closed forms of the whole 3D loop."""
import json
import math
import os

import numpy as np
import pytest
from scipy import integrate

from oracle import rism1d, rism3d as O
from paper_2403_01039_amd import inputs as I

BULK_DIR = os.path.join(os.path.dirname(__file__), "golden", "solvent")


def _second_virial(sigma, eps, beta):
    """B2 = -2 pi \\int (e^{-beta u} - 1) r^2 dr for one LJ site (quadrature)."""
    def mayer(r):
        s6 = (sigma / r) ** 6
        return math.expm1(-beta * 4.0 * eps * (s6 * s6 - s6)) * r * r
    core = 0.5 * sigma
    tot = -core ** 3 / 3.0   # e^{-beta u} = 0 to double precision below sigma / 2
    for a, b in ((core, sigma), (sigma, 2 * sigma), (2 * sigma, 6 * sigma), (6 * sigma, 60.0)):
        tot += integrate.quad(mayer, a, b, epsabs=0, epsrel=1e-12, limit=200)[0]
    return -2.0 * math.pi * tot


def test_ideal_gas_pressure_and_compressibility():
    """No interactions: c = 0, so P = rho k_B T and rho k_B T chi_T = 1."""
    sv = I.single_site_solvent(0.01, q=0.0, sigma=0.0, eps=0.0)
    res = rism1d.solve_solvent(sv, drism=False, closure_kind="kh", ramp=(1.0,))
    kt = 1.0 / O.beta_of(sv.temperature)
    assert abs(rism1d.bulk_pressure(sv, res) - 0.01 * kt) <= 1e-15
    assert abs(rism1d.compressibility(sv, res) * 0.01 * kt - 1.0) <= 1e-12


def test_low_density_virial_limits():
    """A dilute LJ fluid under HNC: c -> the Mayer function e^{-beta u} - 1
    (KH would linearise it in the well), so Eq 20 gives
    P / (rho k_B T) = 1 + B2 rho and the compressibility route
    rho k_B T chi_T = 1 - 2 B2 rho, to first order in rho."""
    rho = 1e-5
    sv = I.single_site_solvent(rho, q=0.0, sigma=3.2, eps=0.3)
    res = rism1d.solve_solvent(sv, drism=False, closure_kind="hnc", ramp=(1.0,))
    beta = O.beta_of(sv.temperature)
    b2 = _second_virial(3.2, 0.3, beta)
    p = rism1d.bulk_pressure(sv, res)
    x = rism1d.compressibility(sv, res) * rho / beta
    assert abs((p * beta / rho - 1.0) / (b2 * rho) - 1.0) <= 2e-3
    assert abs((1.0 - x) / (2.0 * b2 * rho) - 1.0) <= 2e-3


@pytest.mark.parametrize("name", ["water", "saline"])
def test_stored_bulk_values(name):
    """The stored values come from the stored tables' solve: compressibility
    near water's 4.6e-5 / bar (the DRISM/KH value), a positive pressure."""
    with open(os.path.join(BULK_DIR, f"{name}_bulk.json")) as f:
        b = json.load(f)
    assert b["table_max_diff"] <= 1e-10
    per_bar = b["compressibility"] / 69476.95   # 1 kcal/(mol A^3) = 69476.95 bar
    assert 3e-5 < per_bar < 7e-5
    assert b["pressure"] > 0.0


def test_pmv_without_solute_is_the_ideal_volume():
    """No atoms: c = 0 and Eq 19 gives k_B T chi_T."""
    prob = I.small_problem(1, n_atoms=1, shape=(8, 8, 8))
    prob.solute = I.Solute(np.zeros((0, 3)), np.zeros(0), np.zeros(0), np.zeros(0))
    chi, dk = I.solvent_table("water")
    sol = O.solve(O.build_system(prob, chi, dk), tol=1e-12)
    v, per = O.pmv(sol, 3.2)
    assert np.all(per == 0.0)
    assert v == 3.2 / sol.system.beta


def test_pmv_low_density_closed_form():
    """chi = 1, neutral solute, HNC: c = e^{-beta u} - 1 (the closed form of the
    whole loop), so rho \\int c = rho dV sum (e^{-beta u} - 1)."""
    prob = I.small_problem(2, n_atoms=3, shape=(10, 12, 14), closure="hnc")
    prob.solute.q[:] = 0.0
    prob.solvent = I.single_site_solvent(0.03, q=0.0, sigma=3.0, eps=0.2)
    s = O.build_system(prob, np.ones((1, 1, 4096)), 0.05)
    sol = O.solve(s, tol=1e-12)
    v, per = O.pmv(sol, 2.5)
    ref = 0.03 * s.dv * np.sum(np.exp(-s.beta_u) - 1.0)
    assert abs(per[0] - ref) <= 1e-12 * abs(ref)
    assert abs(v - 2.5 / s.beta * (1.0 - ref)) <= 1e-12 * abs(v)
    assert O.pressure_correction(v, 0.2) == -0.2 * v


def test_charged_solute_long_range_cancels_in_electroneutral_solvent():
    """sum_g rho_g f_g = beta C phi_lr sum_g rho_g q_g = 0 point by point, so
    the full-c sum equals the short-range one for a charged solute in saline."""
    prob = I.small_problem(6, n_atoms=3, shape=(8, 8, 8), radius=1.5, saline=True)
    chi, dk = I.solvent_table("saline")
    s = O.build_system(prob, chi, dk)
    sol = O.solve(s, tol=1e-9)
    rho = prob.solvent.site_arrays()[3]
    weighted = lambda x: np.tensordot(rho, x, axes=(0, 0))
    full = float(weighted(sol.c).sum())
    short = float(weighted(sol.c + s.f).sum())
    assert np.abs(weighted(s.f)).max() <= 1e-12 * np.abs(s.f).max()
    assert abs(full - short) <= 1e-10 * abs(full)
