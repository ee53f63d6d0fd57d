"""Pins of the FP64 3D-RISM oracle against closed forms, special cases and
brute force (nothing here re-types the formula under test)."""
import math

import numpy as np
import pytest

from oracle import fft as offt
from oracle import rism3d as O
from paper_2403_01039_amd import inputs as I


def _one_atom(q=0.0, sigma=3.0, eps=0.25, pos=(0.0, 0.0, 0.0)):
    return I.Solute(np.array([pos], dtype=float), np.array([q]), np.array([sigma]), np.array([eps]))


# --- Eq 22: potential ---------------------------------------------------------


def test_lj_minimum_and_zero_crossing():
    """With Lorentz-Berthelot mixing of equal parameters, the LJ pair has its
    zero at d = sigma and its minimum -eps at d = 2^(1/6) sigma."""
    sv = I.single_site_solvent(0.03, q=0.0, sigma=3.0, eps=0.25)
    sol = _one_atom(sigma=3.0, eps=0.25)
    pts = np.array([[3.0, 0, 0], [0, 2 ** (1 / 6) * 3.0, 0], [0, 0, 2 ** (1 / 6) * 3.0 * 1.001]])
    u, phi = O.potential_at(sol, sv, pts)
    assert abs(u[0, 0]) < 1e-12
    assert abs(u[0, 1] + 0.25) < 1e-12
    assert u[0, 2] > -0.25
    assert np.all(phi == 0.0)


def test_coulomb_pair_and_clamp():
    """Unit charges 2 A apart: u = -C/2; inside 0.01 A the clamp holds u fixed."""
    sv = I.single_site_solvent(0.03, q=-1.0, sigma=0.0, eps=0.0)
    sol = _one_atom(q=1.0, sigma=0.0, eps=0.0)
    u, phi = O.potential_at(sol, sv, np.array([[2.0, 0, 0], [0.005, 0, 0], [0.01, 0, 0]]))
    assert abs(u[0, 0] + O.COULOMB / 2.0) < 1e-10
    assert u[0, 1] == u[0, 2]
    # Eq 29 kernel: (1 - e^{-d})/d -> 1 at d = 0 and ~ 1/d far away
    assert abs(O.lr_kernel(np.array([0.0]))[0] - 1.0) < 1e-15
    assert abs(O.lr_kernel(np.array([40.0]))[0] * 40.0 - 1.0) < 1e-15
    assert abs(phi[0] - (1 - math.exp(-2.0)) / 2.0) < 1e-15


def test_potential_translates_with_the_grid():
    prob = I.small_problem(4, n_atoms=5, shape=(12, 10, 8))
    pts = O.grid_points(prob.grid)
    u0, _ = O.potential_at(prob.solute, prob.solvent, pts)
    shifted = I.Solute(prob.solute.xyz + np.array([0.0, 2 * prob.grid.spacing, 0.0]),
                       prob.solute.q, prob.solute.sigma, prob.solute.eps)
    u1, _ = O.potential_at(shifted, prob.solvent, pts + np.array([0.0, 2 * prob.grid.spacing, 0.0]))
    assert np.allclose(u0, u1, rtol=1e-12, atol=1e-9)


def test_neutral_solute_has_no_long_range_part():
    prob = I.single_site_problem(n=16)
    chi, dk = I.solvent_table("water")
    s = O.build_system(prob, chi, dk)
    assert np.all(s.f == 0.0) and np.all(s.ftilde == 0.0)


# --- Eq 29 <-> Eq 30 ------------------------------------------------------------


def test_long_range_kernel_by_quadrature():
    """FT[(1 - e^{-r})/r] = FT[1/r] - FT[e^{-r}/r]: the Coulomb transform 4 pi/k^2
    minus the screened part, here integrated numerically
    (4 pi / k) int_0^inf e^{-r} sin(kr) dr."""
    from scipy.integrate import quad
    from oracle.rism1d import lr_kernel_k
    for k in (0.05, 0.3, 1.0, 4.0, 12.0):
        screened = 4 * math.pi / k * quad(lambda r: math.exp(-r), 0, np.inf, weight="sin",
                                          wvar=k)[0]
        assert abs(lr_kernel_k(np.array([k]))[0] - (4 * math.pi / k ** 2 - screened)) \
            <= 1e-8 * 4 * math.pi / k ** 2


def test_long_range_phase_and_grid_convention():
    """The analytic spectrum carries exp(-i k.(R - r0)) relative to the grid
    corner: compared through a Gaussian charge, whose discrete shifted
    transform is exact to the aliasing level.  F(k) / kernel(k) equals the
    transform of a unit point charge; smearing it with a Gaussian of known
    transform must match forward3 of the sampled Gaussian."""
    n, dr, a = 40, 0.2, 2.0
    grid = I.Grid(n, n, n, dr)
    R = np.array([[0.31, -0.2, 0.17]])
    sol = I.Solute(R, np.array([1.0]), np.array([0.0]), np.array([0.0]))
    beta = O.beta_of(298.15)
    F = O.ftilde_unit(sol, grid, beta)
    kx, ky, kz = O.k_components(grid)
    k2 = kx * kx + ky * ky + kz * kz
    from oracle.rism1d import lr_kernel_k
    point = F / (beta * O.COULOMB * lr_kernel_k(np.sqrt(k2)))
    gauss_k = (np.pi / a) ** 1.5 * np.exp(-k2 / (4 * a))
    pts = O.grid_points(grid)
    x = np.exp(-a * np.sum((pts - R[0]) ** 2, axis=-1))
    X = offt.forward3(x, dr ** 3)
    assert np.abs(point * gauss_k - X).max() <= 1e-10 * np.abs(X).max()


# --- closures and free-energy densities ------------------------------------------


def test_closures():
    d = np.linspace(-5, 5, 2001)
    assert np.array_equal(O.closure(d, "pse", 1), O.closure(d, "kh"))
    assert np.allclose(O.closure(d, "pse", 40), np.exp(d), rtol=1e-12)
    assert np.array_equal(O.closure(d, "hnc"), np.exp(d))
    eps = 1e-7
    kh = lambda v: O.closure(np.array([v]), "kh")[0]
    assert abs(kh(eps) - kh(-eps)) < 3e-7
    assert abs((kh(eps) - 1) / eps - (1 - kh(-eps)) / eps) < 1e-6
    assert kh(0.0) == 1.0


def test_free_energy_density_forms():
    rng = np.random.default_rng(2)
    h = rng.uniform(-1, 3, 1000)
    c = rng.uniform(-2, 2, 1000)
    d = rng.uniform(-1, 3, 1000)
    assert np.array_equal(O.sfe_density(h, c, d, "pse", 1) + 0.0,
                          O.sfe_density(h, c, d, "pse", 1))
    neg = h <= 0
    assert np.allclose(O.sfe_density(h[neg], c[neg], d[neg], "kh"),
                       O.sfe_density(h[neg], c[neg], d[neg], "hnc"), rtol=0, atol=1e-15)
    # PSE-1 equals KH where the closure is linear (h = d on that branch)
    pos = d > 0
    assert np.allclose(O.sfe_density(d[pos], c[pos], d[pos], "pse", 1),
                       O.sfe_density(d[pos], c[pos], d[pos], "kh"), atol=1e-12)


# --- Eq 13: chi(|k|) on the 3D grid by linear interpolation of the radial table ---


def _chi_interp_shifted(chi_table, dk_table, kmag, shift=1):
    """The table read one node off (a planted mistake for the pin below)."""
    n_k = chi_table.shape[-1]
    x = np.minimum(kmag / dk_table, n_k - 1.0)
    m = np.clip(np.floor(x).astype(np.int64) + shift, 0, n_k - 2)
    fr = x - np.floor(x)
    return chi_table[:, :, m] * (1.0 - fr) + chi_table[:, :, m + 1] * fr


def _chi_pin_errors(fn):
    """Errors of an interpolation routine against what linear interpolation on
    a uniform table fixes independently of any implementation:
      nodes   -- at k = m dk the table value itself;
      linear  -- a table sampled from a + b k is reproduced exactly anywhere;
      midpoint-- for f = k^2 the error at (m + 1/2) dk is exactly dk^2 / 4
                 (the chord of a parabola over one interval);
      held    -- beyond the table the last value;
      order   -- entry [g', g] of the result comes from table row [g', g]."""
    dk, n_k = 0.0306796, 64
    k = dk * np.arange(n_k)
    table = np.empty((2, 3, n_k))
    for a in range(2):
        for b in range(3):
            table[a, b] = (10 * a + b + 1) + (a - b + 0.5) * k   # distinct line per entry
    rng = np.random.default_rng(5)
    kq = rng.uniform(0.0, (n_k - 1) * dk, 500)
    err = {}
    exact = (10 * np.arange(2)[:, None, None] + np.arange(3)[None, :, None] + 1
             + (np.arange(2)[:, None, None] - np.arange(3)[None, :, None] + 0.5) * kq[None, None])
    err["linear"] = float(np.abs(fn(table, dk, kq) - exact).max())
    m = np.arange(n_k)
    err["nodes"] = float(np.abs(fn(table, dk, m * dk) - table).max())
    par = np.broadcast_to(k * k, (1, 1, n_k)).copy()
    mid = (np.arange(n_k - 1) + 0.5) * dk
    err["midpoint"] = float(np.abs(fn(par, dk, mid)[0, 0] - mid * mid - dk * dk / 4).max())
    far = np.array([(n_k - 1) * dk * 1.0001, 10.0 * n_k * dk])
    err["held"] = float(np.abs(fn(table, dk, far) - table[:, :, -1:]).max())
    return err


def test_chi_interpolation_pins():
    err = _chi_pin_errors(O.chi_interp)
    assert err["linear"] <= 1e-12, err
    assert err["nodes"] <= 1e-12, err
    assert err["midpoint"] <= 1e-14, err
    assert err["held"] <= 1e-12, err


@pytest.mark.parametrize("shift", [1, -1])
def test_chi_pin_catches_a_one_node_shift(shift):
    """Reading the table one node off (0.031 A^-1) fails the pin."""
    err = _chi_pin_errors(lambda t, dk, km: _chi_interp_shifted(t, dk, km, shift))
    assert max(err["nodes"], err["midpoint"]) > 1e-4, err


# --- the map and the solve ------------------------------------------------------------


def test_oz_step_with_bruteforce_transforms(monkeypatch):
    """Steps 2-5 with the FFT replaced by the brute-force shifted DFT agree to 1e-12."""
    prob = I.small_problem(6, n_atoms=3, shape=(8, 8, 8), radius=1.5, saline=True)
    chi, dk = I.solvent_table("saline")
    s = O.build_system(prob, chi, dk)
    rng = np.random.default_rng(1)
    t = s.f + 0.1 * rng.standard_normal(s.f.shape)
    R1, _, _ = O.rism_map(s, t)
    monkeypatch.setattr(offt, "forward3", offt.forward3_bruteforce)
    monkeypatch.setattr(offt, "inverse3", offt.inverse3_bruteforce)
    R2, _, _ = O.rism_map(s, t)
    assert np.abs(R1 - R2).max() <= 1e-12 * max(1.0, np.abs(R1).max())


def _ideal_solvent_system(prob, q_site=0.0):
    """A one-site solvent with chi = 1 (the zero-density limit, where h = c)."""
    prob.solvent = I.single_site_solvent(0.03, q=q_site, sigma=3.0, eps=0.2)
    chi = np.ones((1, 1, 4096))
    return O.build_system(prob, chi, 0.05)


def test_low_density_closed_form_hnc():
    """chi = 1: R(t) = -t for a neutral solute, so t* = 0, g = exp(-beta u) and the
    HNC free energy is the second-virial sum -kT rho dV sum (e^{-beta u} - 1)."""
    prob = I.small_problem(2, n_atoms=3, shape=(10, 12, 14), closure="hnc")
    prob.solute.q[:] = 0.0
    s = _ideal_solvent_system(prob)
    sol = O.solve(s, tol=1e-12)
    assert sol.iterations == 1
    assert np.array_equal(sol.g, np.exp(-s.beta_u))
    total, _ = O.sfe(sol)
    ref = -(1 / s.beta) * 0.03 * s.dv * np.sum(np.exp(-s.beta_u) - 1.0)
    assert abs(total - ref) <= 1e-12 * abs(ref)


def test_low_density_charged_fixed_point():
    """chi = 1 with charges: h = c gives t* = f - FT^-1[f~] exactly, whatever g is."""
    prob = I.small_problem(3, n_atoms=4, shape=(12, 12, 12), radius=1.5)
    s = _ideal_solvent_system(prob, q_site=0.5)
    sol = O.solve(s, tol=1e-11, eta=1.0)
    expect = s.f - offt.inverse3(s.ftilde, s.dv).real
    assert np.abs(sol.t - expect).max() <= 1e-9
    R, _, _ = O.rism_map(s, expect)
    assert O.rms_of(R) <= 1e-12


def test_fixed_point_and_start_independence():
    prob = I.small_problem(8, n_atoms=6, shape=(16, 14, 12), radius=2.0)
    chi, dk = I.solvent_table("water")
    s = O.build_system(prob, chi, dk)
    a = O.solve(s, tol=1e-10)
    R, _, _ = O.rism_map(s, a.t)
    assert O.rms_of(R) <= 1e-10
    rng = np.random.default_rng(4)
    b = O.solve(s, tol=1e-10, tau0=0.2 * rng.standard_normal(s.f.shape))
    assert np.abs(a.g - b.g).max() <= 1e-7
    # t - f is what the GPU iterates: the identity t_k = tau_k + f of the tau-form
    assert np.allclose(a.tau + s.f, a.t)


def test_site_symmetries():
    """H1 and H2 are identical sites; a permutation of the solute axes (on a
    cubic grid) permutes the field axes."""
    prob = I.small_problem(9, n_atoms=5, shape=(12, 12, 12), radius=1.5)
    chi, dk = I.solvent_table("water")
    s = O.build_system(prob, chi, dk)
    sol = O.solve(s, tol=1e-11)
    assert np.abs(sol.g[1] - sol.g[2]).max() <= 1e-12
    perm = I.Solute(prob.solute.xyz[:, [1, 0, 2]], prob.solute.q, prob.solute.sigma,
                    prob.solute.eps)
    prob2 = I.Problem("perm", perm, prob.solvent, prob.grid, prob.options)
    sol2 = O.solve(O.build_system(prob2, chi, dk), tol=1e-11)
    assert np.abs(sol2.g - np.swapaxes(sol.g, 2, 3)).max() <= 1e-8


def test_merged_hydrogens_equal_three_site_run():
    """Merging H1 and H2 into one site of density 2 rho (chi rows/columns summed
    accordingly) leaves g_O and g_H unchanged."""
    prob = I.small_problem(10, n_atoms=4, shape=(12, 10, 8), radius=1.5)
    chi, dk = I.solvent_table("water")
    s3 = O.build_system(prob, chi, dk)
    sol3 = O.solve(s3, tol=1e-11)
    w = I.water_species()
    merged = I.Solvent((I.Species("w2", (w.sites[0], w.sites[1]), w.coords[:2], w.density),))
    # chi'_{g'g}: summing over the two H of the *source* index (h_g = sum_g' c_g' chi_g'g)
    chi2 = np.empty((2, 2, chi.shape[-1]))
    chi2[0, 0] = chi[0, 0]
    chi2[0, 1] = chi[0, 1]
    chi2[1, 0] = chi[1, 0] + chi[2, 0]
    chi2[1, 1] = chi[1, 1] + chi[2, 1]
    prob2 = I.Problem("merged", prob.solute, merged, prob.grid, prob.options)
    sol2 = O.solve(O.build_system(prob2, chi2, dk), tol=1e-11)
    assert np.abs(sol2.g[0] - sol3.g[0]).max() <= 1e-8
    assert np.abs(sol2.g[1] - sol3.g[1]).max() <= 1e-8


# --- MDIIS ------------------------------------------------------------------------


def test_mdiis_on_linear_contraction():
    rng = np.random.default_rng(5)
    n = 30
    A = rng.standard_normal((n, n))
    A *= 0.9 / np.max(np.abs(np.linalg.eigvals(A)))
    b = rng.standard_normal(n)
    exact = np.linalg.solve(np.eye(n) - A, b)
    res = O.mdiis_solve(lambda x: (A @ x + b - x, None, None), np.zeros(n), 1e-13, 8, 0.7, 500)
    assert res.converged
    assert np.abs(res.t - exact).max() <= 1e-11


def test_mdiis_depth_one_is_damped_picard():
    rng = np.random.default_rng(6)
    A = 0.3 * rng.standard_normal((5, 5))
    b = rng.standard_normal(5)
    seen = []

    def F(x):
        seen.append(x.copy())
        return A @ x + b - x, None, None

    O.mdiis_solve(F, np.zeros(5), 1e-30, 1, 0.5, 6)
    x = np.zeros(5)
    for k in range(6):
        assert np.allclose(seen[k], x, atol=1e-14)
        x = x + 0.5 * (A @ x + b - x)


# ---------------------------------------------------------------------------
# Modified Anderson (Eq 34-39)
# ---------------------------------------------------------------------------

def test_anderson_first_two_steps_are_picard():
    """Steps 1 and 2 are X <- X + b R; the third uses theta."""
    A = np.array([[0.5, 0.1, 0.0], [0.0, 0.3, 0.2], [0.1, 0.0, 0.4]])
    c = np.array([1.0, -2.0, 0.5])
    seen = []

    def F(x):
        seen.append(x.copy())
        R = A @ x + c - x
        return R, None, None

    O.anderson_solve(F, np.zeros(3), 1e-30, (0.2, 0.0), 0.6, 1.0, 3)
    x0 = np.zeros(3)
    x1 = x0 + 0.6 * (A @ x0 + c - x0)
    x2 = x1 + 0.6 * (A @ x1 + c - x1)
    assert np.allclose(seen[1], x1, rtol=0, atol=1e-15)
    assert np.allclose(seen[2], x2, rtol=0, atol=1e-15)


def test_anderson_solves_a_two_dimensional_linear_map_exactly():
    """With s = 0 and b = 1, Anderson with two histories on an affine map of
    a 2-dimensional space reaches the fixed point exactly at its first
    Anderson step: the two residual differences span the space, so the
    least-squares combination has zero residual."""
    A = np.array([[0.6, 0.3], [-0.2, 0.5]])
    c = np.array([1.0, 2.0])
    xstar = np.linalg.solve(np.eye(2) - A, c)
    seen = []

    def F(x):
        seen.append(x.copy())
        return A @ x + c - x, None, None

    res = O.anderson_solve(F, np.zeros(2), 1e-13, (0.0, 0.0), 1.0, 1.0, 10)
    assert res.converged and res.iterations <= 4
    assert np.abs(seen[3] - xstar).max() < 1e-12


def test_anderson_converges_to_the_linear_fixed_point():
    """Paper parameters (s1 0.2, s2 0, b 0.6) on a contraction of R^20."""
    rng = np.random.default_rng(4)
    A = rng.standard_normal((20, 20))
    A *= 0.8 / np.max(np.abs(np.linalg.eigvals(A)))
    c = rng.standard_normal(20)
    xstar = np.linalg.solve(np.eye(20) - A, c)
    res = O.anderson_solve(lambda x: (A @ x + c - x, None, None), np.zeros(20), 1e-12,
                           (0.2, 0.0), 0.6, 1.0, 2000)
    assert res.converged
    assert np.abs(res.t - xstar).max() < 1e-10


def test_anderson_and_mdiis_reach_the_same_3d_fixed_point():
    """The accelerator changes only the path: both reach the same discrete
    fixed point (water, KH), and the inner-product weights 1/rho enter only
    the choice of theta."""
    import copy
    prob = I.small_problem(5, n_atoms=6, shape=(16, 16, 16), radius=2.5)
    chi, dk = I.solvent_table_for(prob.solvent)
    sys_ = O.build_system(prob, chi, dk)
    a = O.solve(sys_, tol=1e-10)
    p2 = copy.deepcopy(prob)
    p2.options.accelerator = "anderson"
    p2.options.mdiis_eta = 0.6
    sys2 = O.build_system(p2, chi, dk)
    b = O.solve(sys2, tol=1e-10)
    assert a.converged and b.converged
    assert np.abs(a.g - b.g).max() < 1e-8


def test_anderson_theta_is_the_weighted_least_squares_solution():
    """theta minimises |sqrt(w) (R0 - sum_i theta_i (R0 - R_i))|: compare with
    numpy's least-squares solver on the weight-scaled vectors (per-site weights
    1/rho differ for an electrolyte)."""
    rng = np.random.default_rng(11)
    R0, R1, R2 = (rng.standard_normal((5, 4, 4, 4)) for _ in range(3))
    w = (1.0 / np.array([0.0334, 0.0334, 0.0334, 6.0e-5, 6.0e-5]))[:, None, None, None]
    theta = O.anderson_theta(R0, R1, R2, w)
    sw = np.sqrt(w) * np.ones_like(R0)
    M = np.stack([(sw * (R0 - R1)).ravel(), (sw * (R0 - R2)).ravel()], axis=1)
    ref, *_ = np.linalg.lstsq(M, (sw * R0).ravel(), rcond=None)
    assert np.allclose(theta, ref, rtol=1e-10, atol=1e-12)


def test_anderson_shifts_and_mixing_closed_form():
    """For an affine map F(x) = A x + c the residual is affine in x, so with
    sum c_k = 1 the first Anderson step X3 = sum c_k (X_k + b R_k) has
    R(X3) = (I + b (A - I)) sum c_k R_k.  In two dimensions the optimal theta
    makes the unshifted combination vanish, leaving
        sum c_k R_k = s1 (R^(n-2) - R^(n-1)) + s2 (R^(n-3) - R^(n-1)),
    so R(X3) pins which shift pairs with which history and the role of b."""
    A = np.array([[0.6, 0.3], [-0.2, 0.5]])
    c = np.array([1.0, 2.0])
    b, s = 0.6, (0.2, 0.05)
    seen = []

    def F(x):
        seen.append(x.copy())
        return A @ x + c - x, None, None

    O.anderson_solve(F, np.zeros(2), 1e-30, s, b, 1.0, 4)
    R = [A @ x + c - x for x in seen]
    expect = (np.eye(2) + b * (A - np.eye(2))) @ (s[0] * (R[1] - R[2]) + s[1] * (R[0] - R[2]))
    assert np.abs(R[3] - expect).max() < 1e-12
