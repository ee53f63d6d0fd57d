"""Solvation free-energy gradient (the solvent term of the derivative of the
MM/3D-RISM free energy, Eq 23) through the C-ABI against the FP64 oracle.

On a given distribution both sides evaluate the same float32 g in FP64, so
they agree to FP64 summation-order round-off (bar 1e-10 of the largest
component).  After a solve the GPU's g carries the FP32 path's and the
stopping rule's error; the bar there is 1e-3 of the largest component (the
relative bar of the free energy) plus the oracle's own stopping error."""
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


def _solver(R, prob):
    chi, dk = inputs.solvent_table_for(prob.solvent)
    dp = R.DeviceProblem(prob, chi, dk)
    s = R.Solver(dp, R.make_opts(prob.options))
    s.potential()
    return s, chi, dk


GIVEN = [
    dict(seed=51, n_atoms=6, shape=(24, 20, 18), saline=False, radius=2.5),   # ragged last tile
    dict(seed=52, n_atoms=70, shape=(64, 24, 32), saline=True, radius=5.0),   # two atom groups, 5 sites
    dict(seed=53, n_atoms=1, shape=(16, 16, 16), saline=False, radius=0.5),
    dict(seed=54, n_atoms=130, shape=(32, 32, 32), saline=False, radius=6.0),  # three, the last ragged
]


@pytest.mark.parametrize("case", GIVEN, ids=lambda c: f"{c['n_atoms']}atoms_{c['shape']}")
def test_gradient_on_a_given_distribution(R, O, case):
    prob = inputs.small_problem(case["seed"], n_atoms=case["n_atoms"], shape=case["shape"],
                                radius=case["radius"], saline=case["saline"])
    print(f"gradient: {case}", flush=True)
    s, _, _ = _solver(R, prob)
    g = inputs.synthetic_distribution(prob, case["seed"])
    got = s.sfe_gradient(torch.tensor(g, device="cuda")).cpu().numpy()
    ref = O.sfe_gradient(prob, g.astype(np.float64))
    err = np.abs(got - ref).max()
    print(f"  max|grad| {np.abs(ref).max():.4e}, max|diff| {err:.3e}", flush=True)
    assert err <= 1e-10 * np.abs(ref).max()


def test_atom_on_a_grid_point(R, O):
    """The pair inside the 0.01 A clamp adds nothing on either side."""
    prob = inputs.small_problem(3, n_atoms=2, shape=(16, 16, 16), radius=1.5)
    prob.solute.xyz[0] = np.array(prob.grid.center) + np.array([1.0, -0.5, 0.5])
    s, _, _ = _solver(R, prob)
    g = inputs.synthetic_distribution(prob, 3, exclusion=0.0)
    assert g[:, 8 + 1, 8 - 1, 8 + 2].min() > 0.0
    got = s.sfe_gradient(torch.tensor(g, device="cuda")).cpu().numpy()
    ref = O.sfe_gradient(prob, g.astype(np.float64))
    assert np.abs(got - ref).max() <= 1e-10 * np.abs(ref).max()


def test_no_atoms_and_bad_arguments(R):
    prob = inputs.small_problem(4, n_atoms=3, shape=(16, 16, 16), radius=1.5)
    chi, dk = inputs.solvent_table_for(prob.solvent)
    dp = R.DeviceProblem(prob, chi, dk)
    s = R.Solver(dp, R.make_opts(prob.options))
    s.ws.zero_()   # a fresh allocation may hold an earlier workspace's state
    g = torch.ones(dp.shape, dtype=torch.float32, device="cuda")
    with pytest.raises(R.RismError, match="not prepared"):
        s.sfe_gradient(g)
    s.potential()
    with pytest.raises(ValueError):
        s.sfe_gradient(g[:, :8])
    empty = inputs.small_problem(4, n_atoms=3, shape=(16, 16, 16), radius=1.5)
    empty.solute = inputs.Solute(np.zeros((0, 3)), np.zeros(0), np.zeros(0), np.zeros(0))
    e, _, _ = _solver(R, empty)
    assert tuple(e.sfe_gradient(g).shape) == (0, 3)


SOLVED = [
    dict(seed=7, n_atoms=6, shape=(24, 20, 18), saline=False),
    dict(seed=35, n_atoms=6, shape=(64, 24, 32), saline=True),
]


@pytest.mark.parametrize("case", SOLVED, ids=lambda c: f"{'saline' if c['saline'] else 'water'}_{c['shape']}")
def test_gradient_after_a_solve(R, O, case):
    """GPU solve (rms 1e-6) and gradient against the oracle's solve converged
    to rms 1e-10 and its gradient."""
    prob = inputs.small_problem(case["seed"], n_atoms=case["n_atoms"], shape=case["shape"],
                                radius=2.5, saline=case["saline"])
    print(f"solve + gradient: {case}", flush=True)
    s, chi, dk = _solver(R, prob)
    g = torch.empty(s.dp.shape, dtype=torch.float32, device="cuda")
    info = s.solve(g_out=g)
    assert info.rms < 1e-6
    got = s.sfe_gradient(g).cpu().numpy()
    system = O.build_system(prob, chi, dk)
    ref = O.sfe_gradient(prob, O.solve(system, tol=1e-10).g)
    stop = np.abs(O.sfe_gradient(prob, O.solve(system, tol=1e-6).g) - ref).max()
    err = np.abs(got - ref).max()
    scale = np.abs(ref).max()
    print(f"  max|grad| {scale:.4e}, max|diff| {err:.3e} (oracle stopping error {stop:.3e})",
          flush=True)
    assert err <= 1e-3 * scale + 1.5 * stop


def test_full_size_sampled_atoms(R, O):
    """The benchmark's 128^3 saline problem (200 atoms, five sites) with a
    given distribution: 16 sampled atoms against the oracle."""
    prob = inputs.solute_200_problem(1, saline=True)
    print("gradient at 128^3, 200 atoms, 5 sites", flush=True)
    s, _, _ = _solver(R, prob)
    g = inputs.synthetic_distribution(prob, 11)
    got = s.sfe_gradient(torch.tensor(g, device="cuda")).cpu().numpy()
    atoms = np.random.default_rng(5).choice(200, 16, replace=False)
    ref = O.sfe_gradient(prob, g.astype(np.float64), atoms=atoms)
    err = np.abs(got[atoms] - ref).max()
    print(f"  max|grad| {np.abs(ref).max():.4e}, max|diff| {err:.3e}", flush=True)
    assert err <= 1e-10 * np.abs(ref).max()
