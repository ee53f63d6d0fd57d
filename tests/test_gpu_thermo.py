"""Partial molar volume (Eq 19) and the PC term (Eq 21) through the C-ABI
against the FP64 oracle.  rho_g \\int c_g comes from the same float64 pass as
the free energy, so it shares its bar: 1e-3 relative to the oracle converged
to rms 1e-10, plus the oracle's own stopping error."""
import math

import numpy as np
import pytest
import torch

from paper_2403_01039_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def R():
    from paper_2403_01039_amd import rism3d
    return rism3d


@pytest.fixture(scope="module")
def O():
    from oracle import rism3d
    return rism3d


CASES = [
    dict(seed=7, shape=(24, 20, 18), saline=False, closure="kh"),
    dict(seed=35, shape=(64, 24, 32), saline=True, closure="kh"),
    dict(seed=9, shape=(24, 20, 18), saline=False, closure="hnc", q=0.3, eta=0.4, n=8),
    dict(seed=10, shape=(24, 20, 18), saline=False, closure="pse", q=0.5, n=8),
]


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"{c['closure']}_{c['shape']}")
def test_pmv_and_pc_match_oracle(R, O, case):
    prob = inputs.small_problem(case["seed"], n_atoms=case.get("n", 6), shape=case["shape"],
                                radius=2.5,
                                saline=case["saline"], closure=case["closure"],
                                charge_scale=case.get("q", 1.0))
    name = inputs.solvent_name(prob.solvent)
    chi, dk = inputs.solvent_table(name)
    bulk = inputs.solvent_bulk(name)
    print(f"pmv: {case}", flush=True)
    dp = R.DeviceProblem(prob, chi, dk, bulk=bulk)
    if "eta" in case:
        prob.options.mdiis_eta = case["eta"]
    s = R.Solver(dp, R.make_opts(prob.options))
    s.potential()
    assert s.solve().rms < 1e-6
    th = s.thermo_all()
    system = O.build_system(prob, chi, dk)
    ref_v, ref_c = O.pmv(O.solve(system, tol=1e-10), bulk[0])
    stop_v, stop_c = O.pmv(O.solve(system, tol=1e-6), bulk[0])
    err_c = np.abs(th["rho_int_c"] - ref_c).max()
    bar_c = 1e-3 * np.abs(ref_c).max() + 1.5 * np.abs(stop_c - ref_c).max()
    print(f"  rho int c {th['rho_int_c']} vs {ref_c} (diff {err_c:.2e}, bar {bar_c:.2e}); "
          f"pmv {th['pmv']:.4f} vs {ref_v:.4f} A^3", flush=True)
    assert err_c <= bar_c
    assert abs(th["pmv"] - ref_v) <= 1e-3 * abs(ref_v) + 1.5 * abs(stop_v - ref_v)
    assert abs(th["rho_int_c_total"] - th["rho_int_c"].sum()) <= 1e-12 * abs(th["rho_int_c_total"])
    assert th["pc"] == O.pressure_correction(th["pmv"], bulk[1])
    assert th["sfe_pc"] == th["sfe"] + th["pc"]


def test_no_bulk_values_leave_pmv_undefined(R):
    prob = inputs.small_problem(7, n_atoms=6, shape=(24, 20, 18), radius=2.5)
    chi, dk = inputs.solvent_table_for(prob.solvent)
    s = R.Solver(R.DeviceProblem(prob, chi, dk), R.make_opts(prob.options))
    s.potential()
    s.solve()
    th = s.thermo_all()
    assert math.isnan(th["pmv"]) and math.isnan(th["pc"]) and math.isnan(th["sfe_pc"])
    assert np.isfinite(th["rho_int_c"]).all()

