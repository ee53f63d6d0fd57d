"""GPU parity: the HIP library (through the C-ABI) against the FP64 oracle.

Bars: max |g_gpu - g_oracle| <= 1e-4 against the
oracle converged to rms 1e-10, and |dSFE| / |SFE| <= 1e-3.  Stage checks
(transform, potential, one map evaluation) use FP32 round-off bounds, derived
where each test states them.
"""
import numpy as np
import pytest
import torch

from paper_2403_01039_amd import inputs

pytestmark = pytest.mark.gpu

G_TOL = 1e-4
SFE_RTOL = 1e-3


@pytest.fixture(scope="module")
def R():
    from paper_2403_01039_amd import rism3d
    return rism3d


@pytest.fixture(scope="module")
def O():
    from oracle import rism3d
    return rism3d


def _run(R, prob, **override):
    chi, dk = inputs.solvent_table_for(prob.solvent)
    dp = R.DeviceProblem(prob, chi, dk)
    opts = R.make_opts(prob.options, **override)
    s = R.Solver(dp, opts)
    s.potential()
    return s, chi, dk


@pytest.mark.parametrize("shape,count", [((8, 8, 8), 1), ((18, 20, 24), 2), ((12, 96, 16), 1),
                                          ((64, 64, 64), 2), ((30, 6, 40), 3),
                                          ((32, 128, 96), 1), ((256, 8, 192), 1),
                                          ((128, 128, 20), 2), ((512, 4, 32), 1)])
def test_transform_matches_oracle(R, shape, count):
    from oracle import fft as offt
    print(f"transform {shape} x{count}", flush=True)
    rng = np.random.default_rng(sum(shape) + count)
    x = rng.standard_normal((count,) + shape) + 1j * rng.standard_normal((count,) + shape)
    ref = offt.forward3(x, 1.0)
    d = torch.tensor(x, dtype=torch.complex64, device="cuda")
    R.rism3d_transform(d, True)
    got = d.cpu().numpy()
    scale = np.abs(ref).max()
    assert np.abs(got - ref).max() / scale < 2e-6
    R.rism3d_transform(d, False)
    back = d.cpu().numpy() / np.prod(shape)
    assert np.abs(back - x).max() / np.abs(x).max() < 2e-6


@pytest.mark.parametrize("name", ["water", "saline", "single"])
def test_potential_matches_oracle(R, O, name):
    if name == "single":
        prob = inputs.single_site_problem(n=32)
    else:
        prob = inputs.small_problem(3, n_atoms=14, shape=(20, 24, 18), saline=(name == "saline"))
    print(f"potential {prob.name}", flush=True)
    s, chi, dk = _run(R, prob)
    w, phi = s.fields()
    sys_ = O.build_system(prob, chi, dk)
    w_ref = sys_.beta_u - sys_.f
    q_v = prob.solvent.site_arrays()[0]
    phi_ref = None
    k = int(np.argmax(np.abs(q_v)))
    if abs(q_v[k]) > 0:
        phi_ref = sys_.f[k] / (sys_.beta * O.COULOMB * q_v[k])
    w = w.cpu().numpy()
    rel = np.abs(w - w_ref) / np.maximum(1.0, np.abs(w_ref))
    # Where w < 5 (g not negligible) the FP32 sum must be tight; deeper inside the
    # repulsive core large LJ and Coulomb terms cancel in FP32, and an error of
    # 1e-3 relative there changes g = O(e^-5) by far less than the 1e-4 bar.
    soft = w_ref < 5.0
    print(f"  max rel err w<5: {rel[soft].max():.2e}  elsewhere: {rel[~soft].max():.2e}")
    assert rel[soft].max() < 2e-5
    assert rel[~soft].max() < 1e-3
    if phi_ref is not None:
        phi = phi.cpu().numpy()
        assert np.abs(phi - phi_ref).max() / max(1.0, np.abs(phi_ref).max()) < 2e-5


# (saline, (nz, ny, nx)): the generic path, the fused x kernels with the fused
# z transform + contraction, and every fused instantiation the workloads reach
# at full size: x and z lengths 96 (96^3 batch members), x 256 and z 256 (the
# 256^3 globule), x 512 (the 512^3 stand-in), y 128, 256 and 512, and z 512
# (separate z passes and contraction).
MAP_SHAPES = [(False, (18, 20, 24)), (True, (18, 20, 24)), (True, (64, 24, 32)),
              (False, (32, 16, 64)), (True, (512, 8, 32)), (False, (256, 8, 256)),
              (False, (96, 96, 96)), (True, (64, 8, 512)), (False, (64, 512, 32)),
              (False, (16, 256, 16)), (True, (16, 128, 16))]


def _map_case(R, O, saline, shape, closure="kh"):
    prob = inputs.small_problem(5, n_atoms=10, shape=shape, saline=saline, closure=closure)
    s, chi, dk = _run(R, prob)
    sys_ = O.build_system(prob, chi, dk)
    return prob, s, sys_


@pytest.mark.parametrize("saline,shape", MAP_SHAPES)
def test_map_matches_oracle(R, O, saline, shape):
    """One exact (FP64) evaluation of steps 2-5 at the same tau on both sides.
    Bar: the GPU takes w = beta u - f as an FP32 field and returns R in FP32,
    so its error is a few FP32 roundings of max(1, |R|); 2e-6 relative."""
    prob, s, sys_ = _map_case(R, O, saline, shape)
    print(f"map {prob.name} saline={saline}", flush=True)
    rng = np.random.default_rng(11)
    tau = (0.05 * rng.standard_normal(sys_.f.shape)).astype(np.float32).astype(np.float64)
    res_ref, _, _ = O.rism_map(sys_, tau + sys_.f)
    res, rms = s.map(torch.tensor(tau, dtype=torch.float32, device="cuda"))
    res = res.cpu().numpy()
    scale = max(1.0, np.abs(res_ref).max())
    err = np.abs(res - res_ref).max()
    print(f"  max|dR| {err:.2e} ({err / scale:.2e} of max(1, |R|)); rms {rms:.6e} vs "
          f"{O.rms_of(res_ref):.6e}", flush=True)
    assert err < 2e-6 * scale, err
    assert abs(rms - O.rms_of(res_ref)) / O.rms_of(res_ref) < 1e-6


@pytest.mark.parametrize("saline,shape,closure",
                         [(sal, shp, "kh") for sal, shp in MAP_SHAPES]
                         + [(False, (64, 24, 32), "pse"), (True, (32, 16, 64), "hnc"),
                            (False, (18, 20, 24), "pse")])
def test_map_increment_matches_oracle(R, O, saline, shape, closure):
    """The FP32 kernels of the bulk iterations, at the tile widths a solve of
    the shape runs: an FP64 anchor at tau_ref, then the FP32 evaluation of
    the increment delta (R = R_ref + dh - dg), element by element against the
    oracle's exact map at tau_ref + delta.  Bar: R_ref is stored in FP32
    (2^-24 |R|) and the FP32 transforms of dc = dg - delta (|dc| <= ~0.2
    here) add about 2^-24 log2(N) |chi| |dc|; 2e-6 of max(1, |R|) covers both,
    while a wrong index, twiddle or table entry in an FP32 kernel moves R by
    O(|dc|)."""
    prob, s, sys_ = _map_case(R, O, saline, shape, closure)
    print(f"map increment {prob.name} saline={saline} {closure}", flush=True)
    rng = np.random.default_rng(17)
    tau_ref = (0.05 * rng.standard_normal(sys_.f.shape)).astype(np.float32)
    delta = (0.02 * rng.standard_normal(sys_.f.shape)).astype(np.float32)
    tau = tau_ref.astype(np.float64) + delta.astype(np.float64)
    res_ref, _, _ = O.rism_map(sys_, tau + sys_.f)
    res0_ref, _, _ = O.rism_map(sys_, tau_ref.astype(np.float64) + sys_.f)
    t_ref = torch.tensor(tau_ref, device="cuda")
    res, rms = s.map_increment(t_ref, torch.tensor(delta, device="cuda"))
    res = res.cpu().numpy()
    scale = max(1.0, np.abs(res_ref).max())
    err = np.abs(res - res_ref).max()
    d_ref = np.abs(res_ref - res0_ref).max()
    print(f"  max|dR| {err:.2e} ({err / scale:.2e} of max(1, |R|)); the increment moves R by "
          f"up to {d_ref:.2e}; rms {rms:.6e} vs {O.rms_of(res_ref):.6e}", flush=True)
    assert err < 2e-6 * scale, err
    assert abs(rms - O.rms_of(res_ref)) / O.rms_of(res_ref) < 1e-5


CASES = [
    dict(seed=7, saline=False, closure="kh", q=1.0, shape=(24, 20, 18)),
    dict(seed=8, saline=True, closure="kh", q=1.0, shape=(24, 20, 18)),
    dict(seed=21, saline=False, closure="kh", q=1.0, shape=(36, 32, 30)),
    dict(seed=9, saline=False, closure="hnc", q=0.3, shape=(24, 20, 18), eta=0.4),
    dict(seed=10, saline=False, closure="pse", q=0.5, shape=(24, 20, 18)),
    dict(seed=11, saline=True, closure="pse", q=0.5, shape=(30, 24, 20)),
    # fused paths: x transform fused with update/residual, z transform + contraction fused
    dict(seed=31, saline=False, closure="kh", q=1.0, shape=(64, 24, 32)),
    dict(seed=32, saline=True, closure="kh", q=1.0, shape=(32, 16, 64)),
    dict(seed=33, saline=False, closure="pse", q=0.5, shape=(96, 20, 32)),
    # the 4000-atom globule's settings (PSE-3, MDIIS depth 10) on a fused grid
    dict(seed=34, saline=False, closure="pse", q=0.5, shape=(64, 32, 32), depth=10),
    # modified Anderson (s1 0.2, s2 0, b 0.6): generic grid in water, fused grid in
    # saline (Gram weights 1/rho differ by a factor of ~550 between sites)
    dict(seed=7, saline=False, closure="kh", q=1.0, shape=(24, 20, 18), accel="anderson"),
    dict(seed=35, saline=True, closure="kh", q=1.0, shape=(64, 24, 32), accel="anderson"),
]


def _case_id(c):
    return (f"{c['closure']}-{'saline' if c['saline'] else 'water'}-q{c['q']}-"
            f"{'x'.join(map(str, c['shape']))}" + (f"-m{c['depth']}" if "depth" in c else "")
            + (f"-{c['accel']}" if "accel" in c else ""))


def _case_problem(c):
    prob = inputs.small_problem(c["seed"], n_atoms=8, shape=c["shape"], radius=2.5,
                                saline=c["saline"], closure=c["closure"], charge_scale=c["q"],
                                mdiis_depth=c.get("depth", 5))
    prob.options.mdiis_eta = c.get("eta", prob.options.mdiis_eta)
    if c.get("accel") == "anderson":
        prob.options.accelerator = "anderson"
        prob.options.mdiis_eta = 0.6
    return prob


@pytest.mark.parametrize("case", CASES, ids=_case_id)
def test_solve_matches_oracle(R, O, case):
    """Full solve at the paper's default rms 1e-6 against the oracle converged to
    rms 1e-10.  The 1e-6 stopping rule itself moves g by up to a few 1e-4 near
    the solute (the oracle stopped at 1e-6 differs that much from its own
    rms-1e-10 solution), so the bar on g is the larger of 1e-4 and 1.5x that
    oracle stopping error; the SFE bar is 1e-3 relative."""
    prob = _case_problem(case)
    print(f"solve {prob.name} {case}", flush=True)
    s, chi, dk = _run(R, prob)
    g = torch.empty(s.dp.shape, dtype=torch.float32, device="cuda")
    info = s.solve(g_out=g)
    sfe, sfe_site = s.thermo()
    sys_ = O.build_system(prob, chi, dk)
    ref = O.solve(sys_, tol=1e-10)
    at6 = O.solve(sys_, tol=1e-6)
    stop_err = np.abs(at6.g - ref.g).max()
    sfe_ref, site_ref = O.sfe(ref)
    err = np.abs(g.cpu().numpy() - ref.g).max()
    print(f"  iterations gpu {info.iterations} oracle {at6.iterations}; max|dg| {err:.2e} "
          f"(oracle stopping error {stop_err:.2e}); sfe {sfe:.6f} vs {sfe_ref:.6f}", flush=True)
    assert info.rms < prob.options.tol
    assert err <= max(G_TOL, 1.5 * stop_err)
    assert abs(sfe - sfe_ref) <= SFE_RTOL * abs(sfe_ref)
    assert np.allclose(sfe_site, site_ref, rtol=SFE_RTOL, atol=SFE_RTOL * abs(sfe_ref))
    # the stopping rule is decided on an exact residual: one FP64 evaluation of
    # the map at the held solution reproduces info.rms (the reference it is
    # held on moves by 2^-48 at that evaluation) and is below the tolerance
    _, rms_held = s.map(None)
    print(f"  FP64 map at the returned iterate: rms {rms_held:.6e} (info {info.rms:.6e})",
          flush=True)
    assert rms_held < prob.options.tol
    assert abs(rms_held - info.rms) <= 1e-6 * info.rms
    if case.get("accel") == "anderson":
        # the same accelerator as the oracle's: the RMS after each of the first
        # iterations (Picard, Picard, then Anderson steps) follows the oracle's
        # history before FP32 and FP64 trajectories part (late in a solve they
        # do: the iteration counts differ by up to a quarter)
        for k in range(1, 9):
            s.opts.max_iter = k
            info_k = s.solve(allow_noconv=True)
            ref_k = at6.rms_history[k - 1]
            print(f"    iteration {k}: rms {info_k.rms:.6e} oracle {ref_k:.6e}", flush=True)
            assert abs(info_k.rms - ref_k) <= 1e-4 * ref_k


def test_below_the_fp32_transform_floor(R, O):
    """A plain FP32 transform of c_sr has a residual floor of ~1.3e-6 on this
    compact charged solute in saline (measured at the exact fixed point); the
    FP64 anchors take the FP32 iteration to rms 5e-7, where the remaining floor
    is the FP32 representation of tau itself."""
    prob = inputs.small_problem(8, n_atoms=8, shape=(24, 20, 18), radius=2.5, saline=True)
    s, chi, dk = _run(R, prob, tol=5e-7)
    g = torch.empty(s.dp.shape, dtype=torch.float32, device="cuda")
    info = s.solve(g_out=g)
    sol = O.solve(O.build_system(prob, chi, dk), tol=1e-11)
    err = np.abs(g.cpu().numpy() - sol.g).max()
    print(f"  below floor: iterations {info.iterations} rms {info.rms:.2e} max|dg| {err:.2e}",
          flush=True)
    assert info.rms < 5e-7
    assert err <= G_TOL


def test_single_site_64_golden(R):
    """The 64^3 single-LJ-site workload against stored oracle values."""
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "single_site.npz")
    ref = np.load(path)
    prob = inputs.single_site_problem()
    s, _, _ = _run(R, prob)
    g = torch.empty(s.dp.shape, dtype=torch.float32, device="cuda")
    info = s.solve(g_out=g)
    sfe, _ = s.thermo()
    gs = g.reshape(g.shape[0], -1)[:, torch.as_tensor(ref["idx"], device="cuda")].cpu().numpy()
    err = np.abs(gs - ref["g_ref"]).max()
    print(f"single_site: it {info.iterations} (oracle {int(ref['iterations_tol'])}) "
          f"max|dg| {err:.2e} sfe {sfe:.6f} vs {float(ref['sfe_ref']):.6f}", flush=True)
    assert err <= G_TOL
    assert abs(sfe - ref["sfe_ref"]) <= SFE_RTOL * abs(ref["sfe_ref"])


@pytest.mark.parametrize("name", ["solute_200_saline", "warm_20000"])
def test_full_size_golden(R, name):
    """The 128^3 workloads (200-atom solute in water + 0.1 M NaCl, and in
    water) at full size, in the launch configuration the benchmark times
    (graph replay of anchor periods), against stored oracle values on the
    sampled points (a seeded choice, the centre line, the oracle's contact
    peaks and the points where its own rms-1e-6 solution is furthest from the
    fixed point): the potential w and phi, the SFE, and g.
      * At the paper's rms 1e-6 the oracle's own iterate is up to
        stop_err_tol (a few 1e-3, over the whole grid) from its rms-1e-10
        solution; the GPU's must be within 1.5 x that, and its iteration
        count within 25% of the oracle's (same MDIIS depth and damping).
      * At rms 1e-8 both are close to the one fixed point: max |dg| <= 1e-4,
        the bar of the benchmark spec, with no allowance."""
    import os
    ref = np.load(os.path.join(os.path.dirname(__file__), "golden", f"{name}.npz"))
    seed = 1 if name == "solute_200_saline" else int(name.split("_")[1])
    prob = (inputs.solute_200_problem(seed, saline=True) if name == "solute_200_saline"
            else inputs.warmstart_problem(seed))
    print(f"full-size golden {name}", flush=True)
    R.use_graphs(True)
    s, _, _ = _run(R, prob)
    idx = torch.as_tensor(ref["idx"], device="cuda")
    w, phi = s.fields()
    w_s = w.reshape(w.shape[0], -1)[:, idx].cpu().numpy().astype(np.float64)
    phi_s = phi.reshape(-1)[idx].cpu().numpy().astype(np.float64)
    w_ref = ref["w_ref"]
    rel = np.abs(w_s - w_ref) / np.maximum(1.0, np.abs(w_ref))
    soft = w_ref < 5.0
    assert rel[soft].max() < 2e-5
    assert rel[~soft].max() < 1e-3 if (~soft).any() else True
    assert np.abs(phi_s - ref["phi_ref"]).max() / max(1.0, np.abs(ref["phi_ref"]).max()) < 2e-5
    g = torch.empty(s.dp.shape, dtype=torch.float32, device="cuda")
    info = s.solve(g_out=g)
    sfe, _ = s.thermo()
    gs = g.reshape(g.shape[0], -1)[:, idx].cpu().numpy()
    err = np.abs(gs - ref["g_ref"]).max()
    stop = float(ref["stop_err_tol"])
    it_ref = int(ref["iterations_tol"])
    print(f"  rms 1e-6: it {info.iterations} (oracle {it_ref}) rms {info.rms:.2e} max|dg| "
          f"{err:.2e} (oracle stopping error {stop:.2e}) sfe {sfe:.4f} vs "
          f"{float(ref['sfe_ref']):.4f}", flush=True)
    assert info.rms < 1e-6
    assert err <= max(G_TOL, 1.5 * stop)
    assert abs(sfe - ref["sfe_ref"]) <= SFE_RTOL * abs(ref["sfe_ref"])
    assert abs(info.iterations - it_ref) <= 0.25 * it_ref
    s.opts = R.make_opts(prob.options, tol=1e-8)
    info = s.solve(g_out=g)
    sfe, _ = s.thermo()
    gs = g.reshape(g.shape[0], -1)[:, idx].cpu().numpy()
    err = np.abs(gs - ref["g_ref"]).max()
    print(f"  rms 1e-8: it {info.iterations} rms {info.rms:.2e} max|dg| {err:.2e} sfe "
          f"{sfe:.4f}", flush=True)
    assert info.rms < 1e-8
    assert err <= G_TOL
    assert abs(sfe - ref["sfe_ref"]) <= SFE_RTOL * abs(ref["sfe_ref"])


def test_globule_4000_at_256(R, O):
    """The 4000-atom globule (net +4, water, 256^3 at 0.4 A) as specified:
    PSE-3, MDIIS depth 10, rms 1e-6.  The potential at 2000 sampled points
    against the oracle's pair sums; then the closure ladder KH -> PSE-2 ->
    PSE-3 (PSE-3 started from t = f diverges on this densely charged globule:
    its cubic branch turns the strong Coulomb wells into g ~ d^3/6, and the
    first Picard step overshoots by orders of magnitude).  Damping 0.3 for KH
    and PSE-2 (the paper advises b <= 0.4 for closures stiffer than KH).  On
    this stiff problem the depth-10 MDIIS tail is erratic: the iteration count
    of one stage moves several-fold with the damping and even with the FP64
    rounding order of the Gram sums, so the PSE-3 stage is a short sequence
    of restarts with damping 0.35, 0.5, 0.3 and 0.45 (each restart keeps the
    last iterate and clears the MDIIS history; a stage short of its
    tolerance hands its iterate on).  The PSE-3 iterate returned has an
    exact FP64 residual below 1e-6: one FP64 evaluation of the map at it
    reproduces info.rms."""
    import time
    prob = inputs.globule_4000_problem()
    assert prob.options.closure == "pse" and prob.options.pse_order == 3
    assert prob.options.mdiis_depth == 10
    print("globule_4000 256^3", flush=True)
    s, chi, dk = _run(R, prob)
    w, phi = s.fields()
    rng = np.random.default_rng(3)
    idx = rng.choice(prob.grid.n_points, 2000, replace=False)
    pts = O.grid_points(prob.grid).reshape(-1, 3)[idx]
    u, phi_ref = O.potential_at(prob.solute, prob.solvent, pts)
    beta = O.beta_of(prob.solvent.temperature)
    q_v = prob.solvent.site_arrays()[0]
    w_ref = np.minimum(beta * u, O.BETA_U_CAP) - beta * O.COULOMB * q_v[:, None] * phi_ref[None]
    w_s = w.reshape(3, -1)[:, torch.as_tensor(idx, device="cuda")].cpu().numpy()
    rel = np.abs(w_s - w_ref) / np.maximum(1.0, np.abs(w_ref))
    soft = w_ref < 5.0
    assert rel[soft].max() < 2e-5 and rel[~soft].max() < 1e-3
    stages = [R.make_opts(prob.options, closure="kh", tol=1e-5, mdiis_eta=0.3, max_iter=4000),
              R.make_opts(prob.options, pse_order=2, tol=1e-6, mdiis_eta=0.3, max_iter=4000)]
    stages += [R.make_opts(prob.options, tol=1e-6, mdiis_eta=eta, max_iter=n)
               for eta, n in ((0.35, 2500), (0.5, 2500), (0.3, 4000), (0.45, 4000))]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = s.solve_ladder(stages)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    th = s.thermo_all()
    res, rms = s.map(None)
    del res
    its = [i.iterations for i in infos]
    print(f"  KH -> PSE-2 -> PSE-3: {its} iterations, rms {[f'{i.rms:.2e}' for i in infos]}, "
          f"{el:.2f} s; FP64 map rms at the returned iterate {rms:.3e}; sfe {th['sfe']:.2f}",
          flush=True)
    assert infos[1].status == 0 and infos[-1].status == 0
    assert infos[-1].rms < 1e-6 and rms < 1e-6
    assert abs(rms - infos[-1].rms) <= 1e-6 * infos[-1].rms
    assert np.isfinite(th["sfe"])


def test_globule_12877_at_512(R, O):
    """The paper-scale stand-in: 12877 atoms (net +13) in water + 0.1 M NaCl on
    512^3 at 0.5 A, one GPU.  The potential at 2000 sampled points against the
    oracle's pair sums, a KH solve with modified Anderson (the paper's GPU
    accelerator) to the paper's rms 1e-6 through the 512-point transforms,
    the returned tau's residual under one FP64 evaluation of the map, and
    finite SFE and PMV.  |tau| reaches ~1.6e3 in the core: the iterate is held
    as a reference plus an increment, so updates far below the FP32 spacing
    of tau itself still accumulate; the returned tau is rounded to FP32,
    which adds ~3e-7 to its FP64 residual."""
    import time
    prob = inputs.globule_12877_problem()
    print("globule_12877 512^3, 5 sites", flush=True)
    chi, dk = inputs.solvent_table_for(prob.solvent)
    dp = R.DeviceProblem(prob, chi, dk, bulk=inputs.solvent_bulk("saline"))
    s = R.Solver(dp, R.make_opts(prob.options, accelerator="anderson", mdiis_eta=0.6,
                                 tol=1e-6, max_iter=3000))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.potential()
    torch.cuda.synchronize()
    t_pot = time.perf_counter() - t0
    w, phi = s.fields()
    rng = np.random.default_rng(4)
    idx = rng.choice(prob.grid.n_points, 2000, replace=False)
    pts = O.grid_points(prob.grid).reshape(-1, 3)[idx]
    u, phi_ref = O.potential_at(prob.solute, prob.solvent, pts)
    beta = O.beta_of(prob.solvent.temperature)
    q_v = prob.solvent.site_arrays()[0]
    w_ref = np.minimum(beta * u, O.BETA_U_CAP) - beta * O.COULOMB * q_v[:, None] * phi_ref[None]
    w_s = w.reshape(5, -1)[:, torch.as_tensor(idx, device="cuda")].cpu().numpy()
    del w, phi
    rel = np.abs(w_s - w_ref) / np.maximum(1.0, np.abs(w_ref))
    soft = w_ref < 5.0
    assert rel[soft].max() < 2e-5 and rel[~soft].max() < 1e-3
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    info = s.solve()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    th = s.thermo_all()
    res, rms = s.map(None)
    del res
    print(f"  potential {t_pot:.2f} s; Anderson: {info.iterations} iterations, rms {info.rms:.2e}, "
          f"{el:.2f} s ({el / info.iterations * 1e3:.1f} ms each); FP64 map rms {rms:.2e}; "
          f"sfe {th['sfe']:.1f} kcal/mol, pmv {th['pmv']:.0f} A^3", flush=True)
    assert info.rms < 1e-6 and info.status == 0
    assert rms < 1e-6
    assert np.isfinite(th["sfe"]) and th["pmv"] > 0.0


def test_z512_solve_has_the_fp64_residual(R):
    """A solve with 512-point z columns (FP32 increments, five sites) stops
    where one FP64 evaluation of the map (checked against the oracle at this
    shape by test_map_matches_oracle) agrees that the residual is below the
    tolerance."""
    prob = inputs.small_problem(36, n_atoms=6, shape=(512, 8, 32), radius=1.5, saline=True,
                                charge_scale=0.5)
    print("z 512 solve", flush=True)
    s, _, _ = _run(R, prob)
    info = s.solve()
    res, rms = s.map(None)
    print(f"  {info.iterations} iterations, rms {info.rms:.2e}; FP64 map rms {rms:.2e}", flush=True)
    assert info.rms < 1e-6
    assert rms < 1e-6


def test_empty_solute_is_bulk(R):
    """No solute atoms: u = 0, so g = 1, h = c = 0 is the fixed point (one map)."""
    prob = inputs.small_problem(1, n_atoms=3, shape=(16, 16, 16))
    prob.solute = inputs.Solute(np.zeros((0, 3)), np.zeros(0), np.zeros(0), np.zeros(0))
    s, _, _ = _run(R, prob)
    g = torch.empty(s.dp.shape, dtype=torch.float32, device="cuda")
    info = s.solve(g_out=g)
    assert info.iterations == 1
    assert torch.all(g == 1.0)
    sfe, _ = s.thermo()
    assert sfe == 0.0


def test_warm_start_from_solution(R):
    """Restarting from a converged tau takes one map evaluation and returns
    the same g up to the rounding of tau to float32 (the iterate is held as
    an FP32 reference plus an FP32 increment, and rism3d_get_tau returns their
    sum rounded to FP32).  The first solve goes to rms 3e-7, so that this
    rounding cannot lift the restarted residual above the 1e-6 of the
    second."""
    prob = inputs.small_problem(12, n_atoms=8, shape=(20, 20, 20), radius=2.5)
    s, _, _ = _run(R, prob)
    g1 = torch.empty(s.dp.shape, dtype=torch.float32, device="cuda")
    s.opts = R.make_opts(prob.options, tol=3e-7)
    s.solve(g_out=g1)
    s.opts = R.make_opts(prob.options)
    tau = s.tau()
    g2 = torch.empty_like(g1)
    info = s.solve(tau0=tau, g_out=g2)
    assert info.warm_start_used == 1
    assert info.iterations == 1
    assert torch.allclose(g1, g2, rtol=2e-6, atol=1e-7)


def test_noconv_and_bad_args(R):
    prob = inputs.small_problem(13, n_atoms=8, shape=(20, 20, 20), radius=2.5)
    s, _, _ = _run(R, prob)
    s.opts.max_iter = 3
    info = s.solve(allow_noconv=True)
    assert info.status == 3 and info.iterations == 3 and info.rms > 0
    bad = R.make_opts(prob.options, mdiis_depth=99)
    with pytest.raises(R.RismError) as e:
        R.rism3d_workspace_bytes(s.dp, bad)
    assert e.value.status == 1


def test_workspace_prepared_under_other_options_is_refused(R):
    """A workspace laid out for MDIIS depth 10 and prepared under it is large
    enough for depth 5, but its offsets differ: a solve with depth-5 options
    must be refused rather than read the potential at the wrong offsets."""
    prob = inputs.small_problem(13, n_atoms=8, shape=(20, 20, 20), radius=2.5)
    s, _, _ = _run(R, prob, mdiis_depth=10)
    s.opts = R.make_opts(prob.options, mdiis_depth=5)
    assert R.rism3d_workspace_bytes(s.dp, s.opts) < s.nbytes
    with pytest.raises(R.RismError) as e:
        s.solve()
    assert e.value.status == 5 and "another layout" in str(e.value)
    s.potential()
    info = s.solve()
    assert info.status == 0


def test_residual_history(R):
    """The recorded history: one RMS per evaluation, the last one exact (FP64)
    and equal to info.rms, every anchor_every-th evaluation exact."""
    prob = inputs.small_problem(13, n_atoms=8, shape=(20, 20, 20), radius=2.5)
    s, _, _ = _run(R, prob, anchor_every=4)
    info = s.solve()
    rms, exact = s.history()
    print(f"history: {info.iterations} iterations, {exact.sum()} exact", flush=True)
    assert len(rms) == info.iterations
    assert exact[-1] and rms[-1] == info.rms and rms[-1] < prob.options.tol
    # an exact evaluation below tol ends the solve, so no earlier one is
    assert (rms[:-1][exact[:-1]] >= prob.options.tol).all()
    pos = np.nonzero(exact)[0]
    assert pos[0] == 0 and np.diff(pos).max() <= 4
    assert np.isfinite(rms).all() and (rms > 0).all()
