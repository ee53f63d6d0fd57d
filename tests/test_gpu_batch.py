"""Batched solves (many solutes, uneven grids) through rism3d_solve_batch.

Every member of a batch runs the same kernels as its single solve, with the
member selected by the launch's second grid dimension, and every reduction
has a fixed order; so each member's g, iteration count and SFE must equal
those of its single solve bit for bit.  The single-solve path is itself held
to the oracle by the parity tests."""
import numpy as np
import pytest
import torch

from paper_2403_01039_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def R():
    from paper_2403_01039_amd import rism3d
    return rism3d


def _single(R, prob, opts):
    chi, dk = inputs.solvent_table_for(prob.solvent)
    dp = R.DeviceProblem(prob, chi, dk)
    s = R.Solver(dp, opts)
    s.potential()
    g = torch.empty(dp.shape, dtype=torch.float32, device="cuda")
    info = s.solve(g_out=g)
    sfe, site = s.thermo()
    return g, info, sfe, site


def _batch(R, probs, opts):
    dps = []
    for p in probs:
        chi, dk = inputs.solvent_table_for(p.solvent)
        dps.append(R.DeviceProblem(p, chi, dk))
    nbytes = R.rism3d_batch_workspace_bytes(dps, opts)
    ws = R.alloc_workspace(nbytes)
    gs = [torch.empty(dp.shape, dtype=torch.float32, device="cuda") for dp in dps]
    infos, sfe = R.rism3d_solve_batch(dps, opts, ws, g_out=gs)
    torch.cuda.synchronize()
    return gs, infos, sfe


def _compare(R, probs, opts, members):
    gs, infos, sfe = _batch(R, probs, opts)
    for i in members:
        g1, info1, sfe1, site1 = _single(R, probs[i], opts)
        print(f"  member {i} {probs[i].grid.nx}x{probs[i].grid.ny}x{probs[i].grid.nz} "
              f"atoms {probs[i].solute.n_atoms}: it {infos[i].iterations} (single "
              f"{info1.iterations}) sfe {sfe[i][0]:.6f} (single {sfe1:.6f})", flush=True)
        assert infos[i].iterations == info1.iterations
        assert infos[i].rms == info1.rms
        assert torch.equal(gs[i], g1)
        assert sfe[i][0] == sfe1
        assert np.array_equal(sfe[i][1], site1)
    return infos


@pytest.mark.parametrize("graphs", [True, False])
def test_mixed_batch_equals_single_solves(R, graphs):
    """Two members share a batched group (same grid, different solutes), one
    has its own batched grid, one grid has no fused kernels (a group of one)."""
    print(f"mixed batch, graphs={graphs}", flush=True)
    R.use_graphs(graphs)
    try:
        probs = [inputs.small_problem(21, n_atoms=6, shape=(64, 24, 32), radius=2.5),
                 inputs.small_problem(22, n_atoms=10, shape=(64, 24, 32), radius=3.0),
                 inputs.small_problem(23, n_atoms=8, shape=(96, 20, 32), radius=2.5),
                 inputs.small_problem(24, n_atoms=5, shape=(24, 20, 18), radius=2.5)]
        opts = R.make_opts(probs[0].options)
        _compare(R, probs, opts, range(len(probs)))
    finally:
        R.use_graphs(True)


def test_uneven_batch_64_solutes(R):
    """The 64-solute uneven batch (20-300 atoms, 96^3 / 128^3 grids, water):
    every member converges; sampled members of both grids equal their single
    solves bit for bit."""
    probs = inputs.batch_uneven_problems()
    sizes = [p.grid.nx for p in probs]
    print(f"uneven batch: {sizes.count(96)} x 96^3, {sizes.count(128)} x 128^3", flush=True)
    opts = R.make_opts(probs[0].options)
    first96 = sizes.index(96)
    first128 = sizes.index(128)
    infos = _compare(R, probs, opts, [first96, first128, len(probs) - 1])
    assert all(inf.rms < 1e-6 for inf in infos)


@pytest.mark.parametrize("tol", [1e-6, 1e-8])
def test_batch_members_against_the_oracle(R, tol):
    """Members of the uneven batch against stored FP64 oracle values (seed
    1000 on 96^3, seed 1001 on 128^3; oracle at rms 1e-10, sampled at a
    seeded choice, the contact peaks and its worst stopping-error points), in
    one batched call with four more members of both grids.  At rms 1e-6 the
    allowance is 1.5 x the oracle's own stopping error over the whole grid
    and the iteration count is within 25% of the oracle's; at rms 1e-8 the
    bar is 1e-4 with no allowance."""
    import os
    probs = [inputs.batch_member_problem(sd) for sd in (1000, 1001, 1002, 1003, 1004, 1005)]
    opts = R.make_opts(probs[0].options, tol=tol)
    gs, infos, sfe = _batch(R, probs, opts)
    for k, sd in enumerate((1000, 1001)):
        ref = np.load(os.path.join(os.path.dirname(__file__), "golden", f"batch_{sd}.npz"))
        idx = torch.as_tensor(ref["idx"], device="cuda")
        got = gs[k].reshape(gs[k].shape[0], -1)[:, idx].cpu().numpy()
        err = np.abs(got - ref["g_ref"]).max()
        stop = float(ref["stop_err_tol"])
        it_ref = int(ref["iterations_tol"])
        print(f"  batch member {sd} ({probs[k].grid.nx}^3, {probs[k].solute.n_atoms} atoms) at "
              f"rms {tol}: it {infos[k].iterations} (oracle {it_ref} at 1e-6) max|dg| {err:.2e} "
              f"(oracle stopping error {stop:.2e}) sfe {sfe[k][0]:.4f} vs "
              f"{float(ref['sfe_ref']):.4f}", flush=True)
        assert infos[k].rms < tol
        assert abs(sfe[k][0] - ref["sfe_ref"]) <= 1e-3 * abs(ref["sfe_ref"])
        if tol == 1e-6:
            assert err <= max(1e-4, 1.5 * stop)
            assert abs(infos[k].iterations - it_ref) <= 0.25 * it_ref
        else:
            assert err <= 1e-4


def test_anderson_batch_equals_single_solves(R):
    """Modified Anderson in a batch: members in water and in saline (different
    Gram weights, so different groups) equal their single solves bit for bit."""
    probs = [inputs.small_problem(26, n_atoms=6, shape=(64, 24, 32), radius=2.5),
             inputs.small_problem(27, n_atoms=8, shape=(64, 24, 32), radius=2.5),
             inputs.small_problem(28, n_atoms=6, shape=(64, 24, 32), radius=2.5, saline=True)]
    opts = R.make_opts(probs[0].options, accelerator="anderson", mdiis_eta=0.6)
    _compare(R, probs, opts, range(len(probs)))


def test_batch_thermo_includes_pmv(R):
    """The batch's thermodynamics carry the PMV and PC term of each member
    (its own solvent's bulk values), equal to the single solves'."""
    probs = [inputs.small_problem(41, n_atoms=6, shape=(64, 24, 32), radius=2.5),
             inputs.small_problem(42, n_atoms=6, shape=(64, 24, 32), radius=2.5, saline=True)]
    opts = R.make_opts(probs[0].options)
    dps = []
    for p in probs:
        name = inputs.solvent_name(p.solvent)
        dps.append(R.DeviceProblem(p, *inputs.solvent_table(name), bulk=inputs.solvent_bulk(name)))
    ws = R.alloc_workspace(R.rism3d_batch_workspace_bytes(dps, opts))
    _, th = R.rism3d_solve_batch(dps, opts, ws, full_thermo=True)
    for dp, t in zip(dps, th):
        s = R.Solver(dp, opts)
        s.potential()
        s.solve()
        one = s.thermo_all()
        print(f"  pmv {t['pmv']:.4f} (single {one['pmv']:.4f}), pc {t['pc']:.4f}", flush=True)
        assert t["pmv"] == one["pmv"] and t["pc"] == one["pc"]
        assert np.array_equal(t["rho_int_c"], one["rho_int_c"])


def test_batch_nonconvergence_reports_member(R):
    probs = [inputs.small_problem(31, n_atoms=6, shape=(64, 24, 32), radius=2.5),
             inputs.small_problem(32, n_atoms=6, shape=(64, 24, 32), radius=2.5)]
    opts = R.make_opts(probs[0].options, max_iter=5)
    dps = [R.DeviceProblem(p, *inputs.solvent_table_for(p.solvent)) for p in probs]
    ws = R.alloc_workspace(R.rism3d_batch_workspace_bytes(dps, opts))
    infos, sfe = R.rism3d_solve_batch(dps, opts, ws, allow_noconv=True)
    assert infos[0].status == 3
    assert all(inf.iterations == 5 for inf in infos)
    assert "batch member" in R.last_error()


def test_tile_widths_change_no_result(R):
    """Every y-pass and z-kernel width the autotuner can choose, and its own
    choice, converge to the default solve's fixed point: the widths change
    which workgroup transforms a line, not the operations on it, so the
    results agree to round-off (separately compiled variants may fuse
    multiply-adds differently, and MDIIS can turn that into an iteration
    more or less)."""
    prob = inputs.small_problem(51, n_atoms=8, shape=(64, 32, 64), radius=3.0)
    opts = R.make_opts(prob.options)
    dp = R.DeviceProblem(prob, *inputs.solvent_table_for(prob.solvent))
    R.tune_reset()
    g0, i0, s0, _ = _single(R, prob, opts)
    try:
        for y, z, x in [(8, 4, 8), (16, 8, 16), (32, 16, 32), (64, 0, 0), (0, 16, 8)]:
            R.tune_set(dp, opts, y, z, x)
            g, info, sfe, _ = _single(R, prob, opts)
            dg = (g - g0).abs().max().item()
            print(f"  widths y {y} z {z} x {x}: it {info.iterations} (default {i0.iterations}), "
                  f"max|dg| {dg:.2e}", flush=True)
            assert abs(info.iterations - i0.iterations) <= 5 and info.rms < 1e-6
            assert dg <= 1e-3 and abs(sfe - s0) <= 1e-4 * abs(s0)
        s = R.Solver(dp, opts)
        s.potential()
        res = R.rism3d_autotune(dp, opts, s.ws)
        print(f"  autotune: {res}", flush=True)
        assert res["y_us"] <= res["y_default_us"] and res["z_us"] <= res["z_default_us"]
        assert res["x_us"] <= res["x_default_us"]
        g, info, sfe, _ = _single(R, prob, opts)
        assert (g - g0).abs().max().item() <= 1e-3 and abs(sfe - s0) <= 1e-4 * abs(s0)
    finally:
        R.tune_reset()


def test_autotune_keeps_the_prepared_potential(R):
    """A solve right after rism3d_autotune on the same workspace (no second
    rism3d_potential) reaches the same fixed point as an untuned solve."""
    prob = inputs.small_problem(52, n_atoms=8, shape=(64, 32, 64), radius=3.0)
    opts = R.make_opts(prob.options)
    g0, i0, s0, _ = _single(R, prob, opts)
    dp = R.DeviceProblem(prob, *inputs.solvent_table_for(prob.solvent))
    s = R.Solver(dp, opts)
    s.potential()
    try:
        R.rism3d_autotune(dp, opts, s.ws)
        g = torch.empty(dp.shape, dtype=torch.float32, device="cuda")
        info = s.solve(g_out=g)
        sfe, _ = s.thermo()
        assert info.rms < 1e-6
        assert (g - g0).abs().max().item() <= 1e-3 and abs(sfe - s0) <= 1e-4 * abs(s0)
    finally:
        R.tune_reset()


def test_reused_workspace_with_another_spacing(R):
    """The HIP graphs cached for a workspace are keyed on everything their
    launches hold, the grid spacing (the k-vectors of the contraction)
    included: a workspace that solved one problem and is then prepared for
    the same solute on a grid of another spacing (same dimensions, atoms and
    solvent) solves it exactly as a fresh workspace does."""
    pa = inputs.small_problem(61, n_atoms=6, shape=(64, 32, 64), radius=3.0)
    pb = inputs.small_problem(61, n_atoms=6, shape=(64, 32, 64), radius=3.0, spacing=0.55)
    opts = R.make_opts(pa.options)
    dpa = R.DeviceProblem(pa, *inputs.solvent_table_for(pa.solvent))
    dpb = R.DeviceProblem(pb, *inputs.solvent_table_for(pb.solvent))
    ws = R.alloc_workspace(max(R.rism3d_workspace_bytes(dpa, opts),
                               R.rism3d_workspace_bytes(dpb, opts)))
    R.rism3d_potential(dpa, opts, ws)
    ia = R.rism3d_solve(dpa, opts, ws)
    R.rism3d_potential(dpb, opts, ws)
    g1 = torch.empty(dpb.shape, dtype=torch.float32, device="cuda")
    i1 = R.rism3d_solve(dpb, opts, ws, None, g1)
    g2, i2, _, _ = _single(R, pb, opts)
    print(f"  spacing 0.5: it {ia.iterations}; spacing 0.55 reused workspace: it {i1.iterations}, "
          f"fresh: it {i2.iterations}", flush=True)
    assert i1.iterations == i2.iterations and i1.rms == i2.rms
    assert torch.equal(g1, g2)
