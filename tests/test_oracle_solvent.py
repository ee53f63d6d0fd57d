"""Pins of the oracle's 1D solvent solver and of the stored susceptibility
tables both sides read, plus the 3D -> 1D reduction of the 3D oracle."""
import json
import math
import os

import numpy as np
import pytest

from oracle import rism1d, rism3d as O
from paper_2403_01039_amd import inputs as I

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _meta(name):
    with np.load(os.path.join(GOLDEN, "solvent", f"{name}.npz"), allow_pickle=False) as z:
        return json.loads(str(z["meta"])), np.array(z["chi"]), float(z["dk"])


@pytest.mark.parametrize("name", ["water", "saline"])
def test_stored_tables_are_converged_drism(name):
    meta, chi, dk = _meta(name)
    assert meta["rms"] < 1e-10
    assert meta["drism"] and meta["closure"] == "kh"
    assert chi.shape[-1] == 4096
    assert abs(dk - math.pi / (4096 * 0.025)) < 1e-15


def test_water_dielectric_constant_recovered():
    """DRISM fixes eps_r through the k -> 0 charge structure (P&P 1992); the
    stored water table reproduces eps_r = 78.4 to 1e-3 relative."""
    meta, chi, dk = _meta("water")
    sv = I.water_solvent()
    k = dk * np.arange(1, 4096)
    eps = rism1d.dielectric_from_chi(sv, chi[:, :, 1:], k)
    assert abs(eps - 78.4) / 78.4 < 1e-3
    assert abs(meta["eps_recovered"] - 78.4) / 78.4 < 1e-3


def test_water_table_symmetries():
    """Equal site densities make chi symmetric; the two H sites are identical."""
    _, chi, _ = _meta("water")
    assert np.abs(chi - np.swapaxes(chi, 0, 1)).max() < 1e-10
    assert np.abs(chi[1] - chi[2][[0, 2, 1]]).max() < 1e-10
    assert np.allclose(chi[:, :, -1], np.eye(3) + (1 - np.eye(3)) * chi[:, :, -1], atol=1e-12)


def test_saline_perfect_screening():
    """Stillinger-Lovett: an electrolyte screens perfectly, so
    4 pi beta C S_qq(k) / k^2 -> 1 as k -> 0."""
    _, chi, dk = _meta("saline")
    sv = I.saline_solvent()
    k = dk * np.arange(1, 4)
    s = rism1d.charge_structure(sv, chi[:, :, 1:4])
    x = 4 * math.pi * O.beta_of(298.15) * O.COULOMB * s / k ** 2
    assert abs(x[0] - 1.0) < 2e-3


def test_xrism_gives_ideal_dielectric():
    """Without the dielectric correction the RISM dielectric constant is the
    ideal-dipole value 1 + 3y, y = 4 pi beta C rho mu^2 / 9."""
    sv = I.water_solvent()
    res = rism1d.solve_solvent(sv, grid=rism1d.RadialGrid(1024, 0.05), drism=False, tol=1e-10)
    st = rism1d.solvent_setup(sv, res.grid, False)
    eps = rism1d.dielectric_from_chi(sv, res.chi, res.grid.k)
    assert abs(eps - (1 + 3 * st["y"])) / (1 + 3 * st["y"]) < 1e-4


def test_hankel_pair_is_inverse_and_exact_for_gaussian():
    g = rism1d.RadialGrid()
    hk = rism1d.Hankel(g)
    f = np.exp(-0.7 * g.r ** 2)
    ft = hk.forward(f)
    exact = (math.pi / 0.7) ** 1.5 * np.exp(-g.k ** 2 / (4 * 0.7))
    assert np.abs(ft - exact).max() < 1e-12 * exact.max()
    assert np.abs(hk.inverse(ft) - f).max() < 1e-12


def test_reduction_3d_to_1d_single_site():
    """A single spherical LJ site: the 3D solution (stored line through the box
    centre of the 64^3 run) against the 1D solute-solvent RISM with the same
    chi.  Agreement is limited by the 0.5 A grid and the 32 A box."""
    ref = np.load(os.path.join(GOLDEN, "single_site.npz"), allow_pickle=False)
    prob = I.single_site_problem()
    chi, dk = I.solvent_table("water")
    one = rism1d.solve_solute_1d(0.0, 3.73, 0.294, prob.solvent, chi, tol=1e-11)
    idx = ref["idx"]
    n = prob.grid.nx
    line = (n // 2 * n + n // 2) * n + np.arange(n)
    pos = np.searchsorted(idx, line)
    g3 = ref["g_ref"][:, pos]
    r3 = np.abs(np.arange(n) - n // 2) * prob.grid.spacing
    sel = (r3 > 0) & (r3 <= 12.0)
    i1 = np.rint(r3[sel] / 0.025).astype(int) - 1
    g1 = one.g[:, i1]
    err = np.abs(g3[:, sel] - g1)
    # the 0.5 A grid resolves the steep contact edges (r < 4.5 A) only to ~0.1
    assert err.max() < 0.1, err.max()
    assert err[:, r3[sel] >= 4.5].max() < 0.05
    sfe3 = float(ref["sfe_ref"])
    assert abs(sfe3 - one.sfe) / abs(one.sfe) < 0.01, (sfe3, one.sfe)
