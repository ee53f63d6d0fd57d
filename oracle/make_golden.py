"""Write stored expected values for full-size parity tests (test infrastructure;
calls only the oracle and the input generators).

    python -m oracle.make_golden single_site solute_200_saline warm_20000 batch_1000

For each named workload it runs the FP64 oracle solve to the workload's own
tolerance, continues it to rms 1e-7 and to rms 1e-10 (standing in for the
exact fixed point), and stores in ``tests/golden/<name>.npz``:
  * ``idx``         flat grid indices of the sampled points: a seeded choice,
                    the full x line through the box centre, the points where
                    the tolerance-level solution is furthest from the rms-1e-10
                    one (the stopping rule's worst points) and the highest
                    peaks of g (contact peaks),
  * ``g_ref``       g at those points, per site, at rms <= 1e-10,
  * ``g_tol``       the same at the workload tolerance (stopping-rule error),
  * ``g_tight``     the same at rms <= 1e-7, and ``stop_err_tol`` /
                    ``stop_err_tight``: max |g - g_ref| over the whole grid at
                    the two tolerances,
  * ``w_ref``       beta*u - f at those points (capped as the solver does),
  * ``phi_ref``     sum_a q_a (1 - e^{-d})/d at those points,
  * ``sfe_ref``, ``sfe_site_ref``, ``sfe_tol``: free energies (kcal/mol),
  * ``iterations``, ``iterations_tol``: oracle MDIIS iteration counts.
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(_HERE))

from paper_2403_01039_amd import inputs  # noqa: E402
from oracle import rism3d  # noqa: E402

OUT_DIR = os.path.join(os.path.dirname(_HERE), "tests", "golden")


def workload(name: str):
    if name == "single_site":
        return inputs.single_site_problem()
    if name == "solute_200_saline":
        return inputs.solute_200_problem(1, saline=True)
    if name.startswith("warm_"):
        return inputs.warmstart_problem(int(name.split("_")[1]))
    if name.startswith("small_"):
        return inputs.small_problem(int(name.split("_")[1]))
    if name.startswith("batch_"):
        return inputs.batch_member_problem(int(name.split("_")[1]))
    raise KeyError(name)


def sample_indices(grid, g_ref=None, g_tol=None, count: int = 6000, worst: int = 1500,
                   seed: int = 12345) -> np.ndarray:
    rng = np.random.default_rng(seed)
    n = grid.n_points
    pick = rng.choice(n, size=min(count, n), replace=False)
    cz, cy = grid.nz // 2, grid.ny // 2
    line = (cz * grid.ny + cy) * grid.nx + np.arange(grid.nx)
    parts = [pick, line]
    if g_ref is not None:
        nv = g_ref.shape[0]
        peak = g_ref.reshape(nv, -1).max(axis=0)
        parts.append(np.argsort(peak)[-worst:])
        if g_tol is not None:
            err = np.abs(g_tol - g_ref).reshape(nv, -1).max(axis=0)
            parts.append(np.argsort(err)[-worst:])
    return np.unique(np.concatenate(parts)).astype(np.int64)


def make(name: str, out_dir: str = OUT_DIR, log=print) -> str:
    prob = workload(name)
    chi, dk = inputs.solvent_table_for(prob.solvent)
    t0 = time.time()
    sys_ = rism3d.build_system(prob, chi, dk)
    log(f"{name}: system built in {time.time() - t0:.1f} s")

    def cb(it, rms):
        if it % 10 == 0:
            log(f"{name}: it {it} rms {rms:.3e} ({time.time() - t0:.0f} s)")

    tol = prob.options.tol
    sol_tol = rism3d.solve(sys_, tol=tol, callback=cb)
    sfe_tol, _ = rism3d.sfe(sol_tol)
    log(f"{name}: tol {tol} reached in {sol_tol.iterations} iterations")
    sol_tight = rism3d.solve(sys_, tol=1e-7, tau0=sol_tol.tau, callback=cb)
    sol = rism3d.solve(sys_, tol=1e-10, tau0=sol_tight.tau, callback=cb)
    sfe_ref, sfe_site = rism3d.sfe(sol)
    idx = sample_indices(prob.grid, sol.g, sol_tol.g)
    nv = sys_.n_sites
    g_ref = sol.g.reshape(nv, -1)[:, idx]
    g_tol = sol_tol.g.reshape(nv, -1)[:, idx]
    g_tight = sol_tight.g.reshape(nv, -1)[:, idx]
    stop_err_tol = float(np.abs(sol_tol.g - sol.g).max())
    stop_err_tight = float(np.abs(sol_tight.g - sol.g).max())
    log(f"{name}: oracle stopping error {stop_err_tol:.2e} at rms {tol}, "
        f"{stop_err_tight:.2e} at rms 1e-7")
    w_ref = (sys_.beta_u - sys_.f).reshape(nv, -1)[:, idx]
    q_v = prob.solvent.site_arrays()[0]
    k = int(np.argmax(np.abs(q_v)))
    phi_ref = (sys_.f[k] / (sys_.beta * rism3d.COULOMB * q_v[k])).reshape(-1)[idx]
    meta = dict(name=name, tol=tol, mdiis_eta=prob.options.mdiis_eta,
                mdiis_depth=prob.options.mdiis_depth, rms_tol=sol_tol.rms,
                rms_tight=sol_tight.rms, rms_ref=sol.rms,
                restarts=sol_tol.restarts, seconds=time.time() - t0,
                iterations_tight_from_tol=sol_tight.iterations,
                iterations_ref_from_tight=sol.iterations)
    os.makedirs(out_dir, exist_ok=True)
    path = os.path.join(out_dir, f"{name}.npz")
    np.savez_compressed(path, idx=idx, g_ref=g_ref, g_tol=g_tol, g_tight=g_tight,
                        stop_err_tol=np.float64(stop_err_tol),
                        stop_err_tight=np.float64(stop_err_tight), w_ref=w_ref, phi_ref=phi_ref,
                        sfe_ref=np.float64(sfe_ref), sfe_site_ref=sfe_site,
                        sfe_tol=np.float64(sfe_tol), iterations=np.int64(sol.iterations),
                        iterations_tol=np.int64(sol_tol.iterations),
                        rms_history=np.array(sol_tol.rms_history),
                        meta=np.array(json.dumps(meta)))
    log(f"{name}: wrote {path} ({time.time() - t0:.0f} s)")
    return path


if __name__ == "__main__":
    for nm in sys.argv[1:]:
        make(nm, log=lambda s: print(s, flush=True))
