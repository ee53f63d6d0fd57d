"""Benchmark: converged 3D-RISM solves per second on one MI355X.

One step = one whole solve of the hot path on inputs already resident in HBM:
rism3d_potential (Eq 22 potential, Eq 30 long-range spectrum, tables) +
rism3d_solve (MDIIS iterations to rms 1e-6) + rism3d_thermo (Eq 18 SFE).

Workload: the seeded 200-atom solute (14 A sphere, sigma in {2, 3, 3.5} A,
eps ~ U(0.05, 0.2), q ~ N(0, 0.3) net 0) in water + 0.1 M NaCl (5 sites),
128^3 grid at 0.5 A, KH closure, MDIIS depth 5, rms 1e-6.

Prints one JSON line with the solves/s, the roofline of the dominant kernel
(its algorithmic bytes per launch over its mean duration, from HIP events
recorded by the library during the timed region) and the FP64 CPU oracle timed
on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "converged 3D-RISM solves/s @128^3, resid 1e-6: plain vs warm-start; HBM GB/s"
HBM_PEAK_GBPS = 8000.0
PROFILE_TRAFFIC = os.path.join(ROOT, "profiles", "traffic.json")


def kernel_bytes(nv: int, N: int, M: int, m_avg: float, fam: str) -> float:
    """Algorithmic HBM bytes of one launch of a kernel family: the bytes the
    method's steps move (FP32 = 4 B, complex FP32 = 8 B, complex FP64 = 16 B;
    P = ceil(nv/2) packed pairs).  For the fused update + closure + forward x
    transform: read the m_avg stored tau_i and R_i and w, write the new tau and
    the packed spectra.  The FP32 increment scheme moves more than that (see
    increment_overhead_bytes)."""
    P = (nv + 1) // 2
    if fam == "update_closure_f32":   # read m tau_i, m R_i, w; write tau; write spectra
        return nv * N * 4 * (2 * m_avg + 2) + 8 * P * N
    if fam == "update_closure_f64":   # read m tau_i, m R_i, w, tau_ref; write tau; FP64 spectra
        return nv * N * 4 * (2 * m_avg + 3) + 16 * P * N
    if fam.startswith("fft_") and fam.endswith("_f32") or fam in ("contract_f32",
                                                                   "zfft_contract_f32"):
        return 16 * P * N
    if fam.startswith("fft_") and fam.endswith("_f64") or fam in ("contract_f64",
                                                                   "zfft_contract_f64"):
        return 32 * P * N
    if fam == "update_fftx_f32":      # update + closure, spectra written once after the x pass
        return nv * N * 4 * (2 * m_avg + 2) + 8 * P * N
    if fam == "update_fftx_f64":
        return nv * N * 4 * (2 * m_avg + 3) + 16 * P * N
    if fam == "fftx_residual_f32":    # spectra read once, then the residual + Gram row
        return 8 * P * N + nv * N * 4 * (2 + max(m_avg - 1, 0) + 1)
    if fam == "fftx_residual_f64":    # as residual_gram_f64 below, spectra read once
        return 16 * P * N + nv * N * 4 * (8 + 3 * max(m_avg - 1, 0))
    if fam == "residual_gram_f32":    # read spectra, R_ref, dg, (m-1) R_i; write R
        return 8 * P * N + nv * N * 4 * (2 + max(m_avg - 1, 0) + 1)
    if fam == "residual_gram_f64":    # read FP64 spectra, delta, tau_ref, w, (m-1) R_i; write R,
        # delta, tau_ref, R_ref, d_ref; read and write the other (m-1) stored deltas
        return 16 * P * N + nv * N * 4 * (8 + 3 * max(m_avg - 1, 0))
    return 0.0


def increment_overhead_bytes(nv: int, N: int, fam: str) -> float:
    """Bytes a launch moves beyond the method's because the FP32 iterations
    transform increments over an FP64 anchor: the update writes the closure
    increment dg (read back by the residual in place of tau and w, so the
    residual's count is unchanged; the update reads the anchor's closure
    argument d_ref in place of w)."""
    if fam in ("update_fftx_f32", "update_closure_f32"):
        return 4.0 * nv * N
    return 0.0


ITERATION_FAMILIES = ("update_fftx_f32", "fft_y_f32", "zfft_contract_f32", "fftx_residual_f32",
                      "update_closure_f32", "fft_x_f32", "fft_z_f32", "contract_f32",
                      "residual_gram_f32")


def host_cpu():
    """CPU model and logical CPU count of the host the benchmark runs on."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return model, os.cpu_count()


def source_digest() -> str:
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2403_01039_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        with open(os.path.join(csrc, name), "rb") as f:
            h.update(name.encode())
            h.update(f.read())
    return h.hexdigest()[:16]


def cpu_baseline(prob, chi, dk, iterations: int):
    """The FP64 oracle on a bounded sample of the workload: its potential on
    1/16 of the grid points and its long-range spectrum for 1/4 of the atoms
    (both scaled up), plus three full-size evaluations of the 3D-RISM map
    (their mean scaled by the iteration count of a solve).  Single-threaded
    numpy."""
    import numpy as np
    from threadpoolctl import threadpool_limits
    from oracle import rism3d as O
    from paper_2403_01039_amd import inputs

    with threadpool_limits(limits=1):
        t_start = time.perf_counter()
        grid = prob.grid
        pts = O.grid_points(grid).reshape(-1, 3)
        rng = np.random.default_rng(0)
        sample = pts[rng.choice(len(pts), size=len(pts) // 16, replace=False)]
        t0 = time.perf_counter()
        O.potential_at(prob.solute, prob.solvent, sample)
        t_pot = (time.perf_counter() - t0) * 16
        sub = inputs.Solute(prob.solute.xyz[::4], prob.solute.q[::4], prob.solute.sigma[::4],
                            prob.solute.eps[::4])
        t0 = time.perf_counter()
        beta = O.beta_of(prob.solvent.temperature)
        O.ftilde_unit(sub, grid, beta)
        t_ft = (time.perf_counter() - t0) * prob.solute.n_atoms / sub.n_atoms
        nv = prob.solvent.n_sites
        shape = (nv,) + grid.shape
        t0 = time.perf_counter()
        chi3 = O.chi_interp(chi, dk, O.k_magnitude(grid))
        t_chi = time.perf_counter() - t0
        system = O.System(prob, beta, grid.spacing ** 3, np.zeros(shape), np.zeros(shape),
                          np.zeros(shape, dtype=np.complex128), chi3, "kh", 1)
        t = 0.01 * rng.standard_normal(shape)
        t0 = time.perf_counter()
        for _ in range(3):
            O.rism_map(system, t)
        t_map = (time.perf_counter() - t0) / 3
        wall = time.perf_counter() - t_start
        # a measured point: the whole 64^3 single-site solve (potential,
        # spectrum, chi, MDIIS iterations to rms 1e-6, SFE)
        c0 = inputs.single_site_problem()
        chi0, dk0 = inputs.solvent_table_for(c0.solvent)
        t0 = time.perf_counter()
        sol0 = O.solve(O.build_system(c0, chi0, dk0))
        O.sfe(sol0)
        t_c0 = time.perf_counter() - t0
    per_solve = t_pot + t_ft + t_chi + iterations * t_map
    model, nproc = host_cpu()
    return {
        "value": 1.0 / per_solve, "unit": "solves/s", "cores": 1, "kind": "oracle",
        "extrapolated": True,
        "sample": (f"FP64 numpy oracle, 1 thread: potential on 1/16 of the grid points (x16), "
                   f"long-range spectrum for 1/4 of the atoms (x4), chi interpolation, and the "
                   f"full-size map evaluation (mean of 3: {t_map:.2f} s) x {iterations} "
                   f"iterations (the GPU's count; the oracle's MDIIS step itself not timed); "
                   f"{wall - t_c0:.1f} s of CPU work"),
        "seconds_per_solve": per_solve,
        "host_cpu": model, "host_nproc": nproc,
        "measured_c0": {"workload": "single_site: 1 LJ site in 3-site water, 64^3 at 0.5 A, KH, "
                                    "MDIIS 5, rms 1e-6, whole solve",
                        "seconds": t_c0, "solves_per_s": 1.0 / t_c0,
                        "iterations": int(sol0.iterations), "cores": 1},
    }


# Kernel-name patterns of the iteration kernels -> timing family names.
FAMILY_PATTERNS = [
    (r"k_update_fftx<false", "update_fftx_f32"), (r"k_update_fftx<true", "update_fftx_f64"),
    (r"k_fftx_residual<false", "fftx_residual_f32"), (r"k_fftx_residual<true", "fftx_residual_f64"),
    (r"k_zcz<HIP_vector_type<float, 2u>|k_zcz<float2", "zfft_contract_f32"),
    (r"k_zcz<HIP_vector_type<double, 2u>|k_zcz<double2", "zfft_contract_f64"),
    (r"k_fft_fixed<HIP_vector_type<float, 2u>, \d+, 1|k_fft_fixed<float2, \d+, 1", "fft_y_f32"),
    (r"k_fft_fixed<HIP_vector_type<double, 2u>, \d+, 1|k_fft_fixed<double2, \d+, 1",
     "fft_y_f64"),
    (r"k_control", "mdiis_control"), (r"k_potential", "potential"),
    (r"k_ftilde", "long_range_spectrum"),
    (r"elementwise_kernel", "copy_calibration"),
]


def family_of(kernel_name: str):
    import re
    for pat, fam in FAMILY_PATTERNS:
        if re.search(pat, kernel_name):
            return fam
    return None


def summarize_counters(fetch_csv: str, write_csv: str, copy_bytes: int, out_path: str):
    """HBM bytes per launch of each kernel family from two rocprofv3 --pmc
    runs (FETCH_SIZE, WRITE_SIZE; KiB per dispatch), each scaled by what the
    same counter reads for the plain copy of copy_bytes bytes in that run."""
    import csv
    import numpy as np

    def load(path, counter):
        per = {}
        with open(path) as f:
            for row in csv.DictReader(f):
                if row.get("Counter_Name") != counter:
                    continue
                fam = family_of(row["Kernel_Name"])
                if fam:
                    per.setdefault(fam, []).append(float(row["Counter_Value"]))
        return per

    def active(per):
        # Launches that follow convergence inside a replayed anchor period exit
        # at once and move (almost) no bytes; they are not launches of the step.
        return {f: [v for v in vals if v >= 0.01 * max(vals)] for f, vals in per.items()}

    fetch = active(load(fetch_csv, "FETCH_SIZE"))
    write = active(load(write_csv, "WRITE_SIZE"))
    # the calibration copy is the elementwise dispatch with the largest fetch
    # (torch.ones before it only writes)
    f_copy = max(fetch["copy_calibration"]) * 1024.0
    w_copy = max(write["copy_calibration"]) * 1024.0
    f_scale, w_scale = copy_bytes / f_copy, copy_bytes / w_copy
    out = {"source_digest": source_digest(), "copy_bytes": copy_bytes,
           "fetch_scale": f_scale, "write_scale": w_scale, "kernels": {}}
    for fam in sorted(set(fetch) & set(write)):
        if fam == "copy_calibration":
            continue
        fb = float(np.mean(fetch[fam])) * 1024.0 * f_scale
        wb = float(np.mean(write[fam])) * 1024.0 * w_scale
        out["kernels"][fam] = {"dispatches": len(fetch[fam]), "write_dispatches": len(write[fam]),
                               "fetch_bytes": fb,
                               "write_bytes": wb, "bytes_per_launch": fb + wb}
    with open(out_path, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out, indent=1))


def warm_start_comparison(R, inputs, n_seeds: int):
    """Plain vs warm-started solves on held-out seeds of the warm-start
    workload (200-atom solutes in water, 128^3 at 0.5 A, KH, MDIIS 5, rms
    1e-6), and the same two with modified Anderson.  One solve = potential +
    [network inference + OZ half-step] + iterations + SFE; inputs resident on
    the device."""
    import numpy as np
    import torch
    if not os.path.exists(R.WEIGHTS_PATH):
        return {"error": "no trained warm-start weights"}
    net = R.WarmStart()
    chi, dk = inputs.solvent_table("water")
    seeds = list(range(20000, 20000 + n_seeds))
    probs = [inputs.warmstart_problem(s) for s in seeds]
    dps = [R.DeviceProblem(p, chi, dk) for p in probs]
    opts = R.make_opts(probs[0].options)
    ws = R.alloc_workspace(max(R.rism3d_workspace_bytes(dp, opts) for dp in dps))
    tau0 = torch.empty(dps[0].shape, dtype=torch.float32, device="cuda")

    def plain(dp):
        R.rism3d_potential(dp, opts, ws)
        info = R.rism3d_solve(dp, opts, ws)
        R.rism3d_thermo(dp, opts, ws)
        return info

    def warm(dp):
        R.rism3d_potential(dp, opts, ws)
        net.tau0(dp, opts, ws, tau0)
        info = R.rism3d_solve(dp, opts, ws, tau0)
        R.rism3d_thermo(dp, opts, ws)
        return info

    R.rism3d_potential(dps[0], opts, ws)
    R.rism3d_autotune(dps[0], opts, ws)  # this grid's tile widths, as for the headline
    opts_a = R.make_opts(probs[0].options, accelerator="anderson", mdiis_eta=0.6,
                         anderson_s1=0.2, anderson_s2=0.0)

    def warm_anderson(dp):
        R.rism3d_potential(dp, opts_a, ws)
        net.tau0(dp, opts_a, ws, tau0)
        info = R.rism3d_solve(dp, opts_a, ws, tau0)
        R.rism3d_thermo(dp, opts_a, ws)
        return info

    def plain_anderson(dp):
        R.rism3d_potential(dp, opts_a, ws)
        info = R.rism3d_solve(dp, opts_a, ws)
        R.rism3d_thermo(dp, opts_a, ws)
        return info

    R.rism3d_autotune(dps[0], opts_a, ws)
    plain(dps[0]); warm(dps[0])          # warm-up (graph capture, workspaces)
    plain_anderson(dps[0]); warm_anderson(dps[0])
    out = {}
    for name, fn in (("plain", plain), ("warm", warm), ("plain_anderson", plain_anderson),
                     ("warm_anderson", warm_anderson)):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        its = [fn(dp).iterations for dp in dps]
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        out[name] = {"solves_per_s": len(dps) / el, "iterations_mean": float(np.mean(its))}
    # the warm-started batched solver: per member the potential and the
    # network's tau0 on a single workspace, then the members in
    # rism3d_solve_batch calls of up to `chunk` (which repeat each potential)
    chunk = 50
    bws = R.alloc_workspace(R.rism3d_batch_workspace_bytes(dps[:chunk], opts))
    taus = [torch.empty(dps[0].shape, dtype=torch.float32, device="cuda")
            for _ in range(min(chunk, len(dps)))]

    def warm_batch(group):
        for dp, t in zip(group, taus):
            R.rism3d_potential(dp, opts, ws)
            net.tau0(dp, opts, ws, t)
        infos, _ = R.rism3d_solve_batch(group, opts, bws, tau0=taus[:len(group)])
        return [i.iterations for i in infos]

    warm_batch(dps[:min(chunk, len(dps))])   # warm-up (graph capture)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    its = []
    for i in range(0, len(dps), chunk):
        its += warm_batch(dps[i:i + chunk])
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    out["warm_batch"] = {"solves_per_s": len(dps) / el, "iterations_mean": float(np.mean(its)),
                         "batch_size": chunk}
    del bws
    out["speedup"] = out["warm"]["solves_per_s"] / out["plain"]["solves_per_s"]
    out["speedup_warm_batch_vs_plain"] = (out["warm_batch"]["solves_per_s"]
                                          / out["plain"]["solves_per_s"])
    out["speedup_warm_anderson_vs_plain_mdiis"] = (out["warm_anderson"]["solves_per_s"]
                                                  / out["plain"]["solves_per_s"])
    out["workload"] = (f"warm_start: held-out seeds {seeds[0]}..{seeds[-1]}, 200-atom solutes in "
                       f"water (3 sites), 128^3 at 0.5 A, KH, MDIIS 5, rms 1e-6")
    return out


def anderson_comparison(R, prob, dp, stream, n: int):
    """The headline workload with the paper's GPU accelerator (modified
    Anderson, two histories, s1 0.2, s2 0, b 0.6) instead of MDIIS."""
    import torch
    opts = R.make_opts(prob.options, accelerator="anderson", mdiis_eta=0.6,
                       anderson_s1=0.2, anderson_s2=0.0)
    solver = R.Solver(dp, opts)
    R.rism3d_potential(dp, opts, solver.ws, stream)
    R.rism3d_autotune(dp, opts, solver.ws, stream)

    def step():
        solver.potential(stream)
        info = solver.solve(stream=stream)
        solver.thermo(stream)
        return info

    step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    its = [step().iterations for _ in range(n)]
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    return {"solves_per_s": n / el, "iterations_mean": sum(its) / n,
            "accelerator": "modified Anderson (s1 0.2, s2 0, b 0.6)"}


def batch_comparison(R, inputs, count: int):
    """The uneven batch (count solutes of 20-300 atoms in water on 96^3 /
    128^3 grids at 0.5 A, KH, MDIIS 5, rms 1e-6) in one rism3d_solve_batch
    call: potentials, solves and SFEs of every member; solves/s = count /
    wall time (inputs resident on the device)."""
    import torch
    probs = inputs.batch_uneven_problems(count=count)
    chi, dk = inputs.solvent_table("water")
    dps = [R.DeviceProblem(p, chi, dk) for p in probs]
    opts = R.make_opts(probs[0].options)
    ws = R.alloc_workspace(R.rism3d_batch_workspace_bytes(dps, opts))
    for shape in sorted({dp.shape for dp in dps}):   # tile widths per grid, as elsewhere
        dp = next(d for d in dps if d.shape == shape)
        one = R.alloc_workspace(R.rism3d_workspace_bytes(dp, opts))
        R.rism3d_potential(dp, opts, one)
        R.rism3d_autotune(dp, opts, one)
        del one
    R.rism3d_solve_batch(dps, opts, ws)          # warm-up (graph capture)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos, _ = R.rism3d_solve_batch(dps, opts, ws)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    del ws
    # the same problems one after another (potential + solve + SFE each, one
    # workspace per grid, graphs captured in a warm-up pass)
    one = {}
    for shape in {dp.shape for dp in dps}:   # sized for the largest solute of the grid
        one[shape] = R.alloc_workspace(max(R.rism3d_workspace_bytes(dp, opts)
                                           for dp in dps if dp.shape == shape))

    def single(dp):
        w = one[dp.shape]
        R.rism3d_potential(dp, opts, w)
        info = R.rism3d_solve(dp, opts, w)
        R.rism3d_thermo(dp, opts, w)
        return info

    for shape in one:
        single(next(d for d in dps if d.shape == shape))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    its = [single(dp).iterations for dp in dps]
    torch.cuda.synchronize()
    el_seq = time.perf_counter() - t0
    sizes = [p.grid.nx for p in probs]
    return {"solves_per_s": count / el, "seconds": el,
            "iterations_mean": sum(i.iterations for i in infos) / count,
            "sequential_solves_per_s": count / el_seq, "sequential_seconds": el_seq,
            "sequential_iterations_mean": sum(its) / count,
            "speedup_vs_sequential": el_seq / el,
            "workload": (f"batch_uneven: {count} solutes (seeds 1000..{999 + count}), "
                         f"{sizes.count(96)} x 96^3 + {sizes.count(128)} x 128^3, water, KH, "
                         f"MDIIS 5, rms 1e-6, one rism3d_solve_batch call vs the same solves "
                         f"one by one")}


def gradient_leg(R, prob, solver, stream, reps: int):
    """The solvation free-energy gradient with respect to the 200 atom
    positions (the solvent term of the derivative of Eq 23) at the solved g of
    the headline problem: reps calls, kernel time from HIP events on the
    call's stream."""
    import torch
    g = torch.empty(solver.dp.shape, dtype=torch.float32, device=solver.ws.device)
    solver.potential(stream)
    solver.solve(g_out=g, stream=stream)
    solver.sfe_gradient(g, stream)               # warm-up
    torch.cuda.synchronize()
    R.timing_reset()
    R.timing_select("sfe_gradient")
    R.timing_enable(True)
    t0 = time.perf_counter()
    for _ in range(reps):
        grad = solver.sfe_gradient(g, stream)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    R.timing_enable(False)
    R.timing_select(None)
    cnt, ms = R.timing_read()["sfe_gradient"]
    kernel_s = ms / cnt * 1e-3
    pairs = prob.solute.n_atoms * prob.grid.n_points
    return {"ms_per_call": el / reps * 1e3, "kernel_us": kernel_s * 1e6,
            "atom_point_pairs_per_s": pairs / kernel_s,
            "max_abs_kcal_mol_A": float(grad.abs().max()),
            "workload": "d(dmu)/dR for the 200 atoms of solute_200_saline at its solved g "
                        "(128^3, 5 sites), FP64 pair terms"}


def network_leg(R, inputs, steps: int):
    """The warm-start network of the learned part (4 levels, 16-128 channels,
    3^3 convolutions, BF16 on the matrix cores with FP32 accumulation) at the
    128^3 grid: one training step (forward, loss, backward, Adam) and one
    inference, on seeded He-normal parameters and seeded synthetic input and
    target.  TFLOP/s counts the convolutions' multiply-adds (2 flops each):
    forward 2 N 27 C_in C_out per layer at its level's N voxels, backward
    twice that (data and weight gradients); the peak is the dense BF16 MFMA
    rate."""
    import numpy as np
    import torch
    shape = (128, 128, 128)
    cfg = R.unet_config(3, 3, levels=4, base=16)
    layers = R.unet_layers(cfg)
    theta = torch.tensor(inputs.unet_init_params(layers, 7), dtype=torch.float32, device="cuda")
    rng = np.random.default_rng(8)
    x = torch.tensor(rng.standard_normal((3,) + shape), dtype=torch.float32, device="cuda")
    y = torch.tensor(rng.standard_normal((3,) + shape), dtype=torch.float32, device="cuda")
    grad = torch.empty_like(theta)
    m = torch.zeros_like(theta)
    v = torch.zeros_like(theta)
    out = torch.empty_like(x)
    ws_t = R.alloc_workspace(R.unet_workspace_bytes(cfg, shape, True))
    scratch = R.unet_adam_scratch()
    n0 = shape[0] * shape[1] * shape[2]
    level = {}
    for name, ci, co in layers:
        lv = int(name[3]) if name.startswith(("enc", "dec")) else 0
        level[name] = n0 >> (3 * lv)
    fwd = sum(2.0 * level[n] * 27 * ci * co for n, ci, co in layers)

    def train_step(k):
        R.unet_gradient(cfg, theta, x, y, grad, ws_t)
        R.unet_adam(theta, m, v, grad, k + 1, 1e-4, clip_norm=1.0, scratch=scratch)

    train_step(0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        train_step(k + 1)
    torch.cuda.synchronize()
    t_train = (time.perf_counter() - t0) / steps
    R.unet_forward(cfg, theta, x, out, ws_t)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        R.unet_forward(cfg, theta, x, out, ws_t)
    torch.cuda.synchronize()
    t_fwd = (time.perf_counter() - t0) / steps
    peak = 2500.0
    return {"train_step_ms": t_train * 1e3, "forward_ms": t_fwd * 1e3,
            "forward_tflop": fwd / 1e12, "train_step_tflop": 3.0 * fwd / 1e12,
            "train_tflops": 3.0 * fwd / t_train / 1e12, "forward_tflops": fwd / t_fwd / 1e12,
            "bf16_mfma_peak_tflops": peak,
            "train_frac": 3.0 * fwd / t_train / 1e12 / peak,
            "forward_frac": fwd / t_fwd / 1e12 / peak,
            "parameters": int(theta.numel()),
            "workload": "warm-start network, 4 levels, 16-128 channels, 3 -> 3 channels, 128^3 "
                        "voxels, seeded synthetic input and target, one solute per step"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--gradient-reps", type=int, default=5,
                    help="calls of the free-energy gradient leg (0: skip)")
    ap.add_argument("--batch-solutes", type=int, default=64,
                    help="solutes of the batched-solve leg (0: skip)")
    ap.add_argument("--anderson-steps", type=int, default=2,
                    help="solves of the headline workload with modified Anderson (0: skip)")
    ap.add_argument("--warm-seeds", type=int, default=200,
                    help="held-out seeds of the plain vs warm-start comparison (0: skip)")
    ap.add_argument("--network-steps", type=int, default=5,
                    help="timed training steps and inferences of the warm-start network (0: skip)")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="first run one plain device copy of this many MiB (the reference "
                         "dispatch for scaling HBM counters)")
    ap.add_argument("--summarize-counters", nargs=3, metavar=("FETCH_CSV", "WRITE_CSV", "OUT"),
                    help="write per-family HBM bytes from two rocprofv3 --pmc runs and exit")
    args = ap.parse_args()
    if args.summarize_counters:
        summarize_counters(*args.summarize_counters[:2], args.copy_calibration_mib << 20,
                           args.summarize_counters[2])
        return
    if args.gpus != 1:
        print(json.dumps({"error": "the solver runs on one GPU per process; --gpus must be 1 "
                                   "(independent solves shard across GPUs by process)"}))
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2403_01039_amd import inputs
    from paper_2403_01039_amd import rism3d as R

    dev = torch.device("cuda:0")
    if args.copy_calibration_mib:
        n = (args.copy_calibration_mib << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.mul(src, 1.0, out=dst)   # one elementwise kernel: reads and writes n floats
        torch.cuda.synchronize()
        del src, dst
    prob = inputs.solute_200_problem(1, saline=True)
    chi, dk = inputs.solvent_table_for(prob.solvent)
    dp = R.DeviceProblem(prob, chi, dk, device=dev,
                         bulk=inputs.solvent_bulk(inputs.solvent_name(prob.solvent)))
    opts = R.make_opts(prob.options)
    solver = R.Solver(dp, opts)
    stream = torch.cuda.current_stream(dev)

    def step():
        solver.potential(stream)
        info = solver.solve(stream=stream)
        sfe, _ = solver.thermo(stream)
        return info, sfe

    # Warmup.  One-time set-up outside the timed region: pick the tile widths
    # of the FP32 iteration kernels for this grid (no effect on results).  One
    # warmup step then times every kernel family (the per-family breakdown,
    # which names the dominant family); the timed region records events around
    # that family only, since every event record also orders the stream and
    # timing all families would slow the solve.
    step()
    tuning = R.rism3d_autotune(dp, opts, solver.ws, stream)
    R.timing_reset()
    R.timing_enable(True)
    step()
    torch.cuda.synchronize()
    R.timing_enable(False)
    breakdown = R.timing_read()
    for _ in range(max(args.warmup - 2, 0)):
        step()
    torch.cuda.synchronize()
    dominant = max((f for f, (c, ms) in breakdown.items() if c and kernel_bytes(
        prob.solvent.n_sites, prob.grid.n_points, 1, 1.0, f)), key=lambda f: breakdown[f][1])
    R.timing_reset()
    R.timing_select(dominant)
    R.timing_enable(True)
    iters = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        info, sfe = step()
        iters.append(info.iterations)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    R.timing_enable(False)
    R.timing_select(None)
    timing = R.timing_read()

    nv = prob.solvent.n_sites
    N = prob.grid.n_points
    M = prob.options.mdiis_depth
    it_mean = float(np.mean(iters))
    m_avg = float(np.mean([min(k, M) for k in range(int(round(it_mean)))]))
    def table(tm):
        out = {}
        for fam, (cnt, ms) in tm.items():
            if cnt == 0:
                continue
            avg_s = ms / cnt * 1e-3
            b = kernel_bytes(nv, N, M, m_avg, fam)
            ov = increment_overhead_bytes(nv, N, fam)
            out[fam] = {"launches": cnt, "total_ms": round(ms, 3),
                        "avg_us": round(avg_s * 1e6, 2), "bytes_per_launch": b,
                        "gbps": round(b / avg_s / 1e9, 1) if b else None,
                        "frac": round(b / avg_s / 1e9 / HBM_PEAK_GBPS, 4) if b else None}
            if ov:
                out[fam]["increment_overhead_bytes"] = ov
                out[fam]["gbps_incl_overhead"] = round((b + ov) / avg_s / 1e9, 1)
        return out

    kernels = table(breakdown)
    timed = table(timing)[dominant]
    achieved = timed["gbps"]
    # the FP32 iteration's kernels together: their algorithmic bytes over
    # their summed time (traffic-weighted fraction of the HBM peak)
    it_fams = [f for f in ITERATION_FAMILIES if f in kernels]
    it_bytes = sum(kernels[f]["bytes_per_launch"] * kernels[f]["launches"] for f in it_fams)
    it_s = sum(kernels[f]["total_ms"] for f in it_fams) * 1e-3
    fp32_iteration = {"families": it_fams,
                      "gbps": round(it_bytes / it_s / 1e9, 1) if it_s else None,
                      "frac": round(it_bytes / it_s / 1e9 / HBM_PEAK_GBPS, 4) if it_s else None,
                      "control_us_per_iteration": (kernels["mdiis_control"]["avg_us"]
                                                   if "mdiis_control" in kernels else None)}
    traffic = None
    if os.path.exists(PROFILE_TRAFFIC):
        with open(PROFILE_TRAFFIC) as f:
            tr = json.load(f)
        ent = tr.get("kernels", {}).get(dominant)
        if ent and tr.get("source_digest") == source_digest():
            traffic = ent.get("bytes_per_launch")
    b_min_iter = 4.0 * nv * N * (3 * M + 3)
    ms_per_step = elapsed / args.steps * 1e3
    out = {
        "metric": METRIC,
        "value": args.steps / elapsed,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": ("solute_200_saline: seeded 200-atom solute in water + 0.1 M NaCl "
                                "(5 sites), 128^3 grid at 0.5 A, KH, MDIIS depth 5, rms 1e-6, "
                                "plain start"),
                   "grid": [prob.grid.nx, prob.grid.ny, prob.grid.nz], "n_sites": nv,
                   "n_atoms": prob.solute.n_atoms, "start": "plain"},
        "iterations_mean": it_mean,
        "sfe_kcal_mol": sfe,
        "hbm_gbps_effective": b_min_iter * it_mean / (elapsed / args.steps) / 1e9,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBPS, "traffic": traffic, "kernel": dominant,
                     "launches": timed["launches"], "avg_us": timed["avg_us"],
                     "bytes_per_launch": timed["bytes_per_launch"],
                     "increment_overhead_bytes": timed.get("increment_overhead_bytes", 0.0),
                     "achieved_incl_overhead": timed.get("gbps_incl_overhead", achieved)},
        "kernels_tuned_step": kernels,
        "fp32_iteration_kernels": fp32_iteration,
        "tuning": tuning,
    }
    th = solver.thermo_all(stream)   # the last timed solve's thermodynamics
    out["thermo"] = {"sfe_kcal_mol": th["sfe"], "pmv_A3": th["pmv"], "pc_kcal_mol": th["pc"],
                     "sfe_pc_kcal_mol": th["sfe_pc"], "rho_int_c_total": th["rho_int_c_total"]}
    if args.gradient_reps > 0:
        out["sfe_gradient"] = gradient_leg(R, prob, solver, stream, args.gradient_reps)
    if args.batch_solutes > 0:
        out["batch"] = batch_comparison(R, inputs, args.batch_solutes)
    if args.anderson_steps > 0:
        out["anderson"] = anderson_comparison(R, prob, dp, stream, args.anderson_steps)
    if args.warm_seeds > 0:
        out["warm_start"] = warm_start_comparison(R, inputs, args.warm_seeds)
    if args.network_steps > 0:
        out["network"] = network_leg(R, inputs, args.network_steps)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(prob, chi, dk, int(round(it_mean)))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
