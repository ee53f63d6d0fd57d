"""Python binding of librism3d.so (argument marshalling only).

Every step of the computation runs in the library's HIP kernels; this module
only builds the C structs of ``include/rism3d.h``, passes torch device pointers
and the current HIP stream, and converts status codes into exceptions.  The
function names follow the C entry points.  There is no fallback: if the
library is not built, importing the binding raises.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_lib", "librism3d.so")
MAX_SITES = 8
MAX_DEPTH = 16

STATUS = {0: "OK", 1: "E_ARG", 2: "E_DEVICE", 3: "E_NOCONV", 4: "E_NONFINITE", 5: "E_WORKSPACE"}
CLOSURES = {"kh": 0, "hnc": 1, "pse": 2}
ACCELERATORS = {"mdiis": 0, "anderson": 1}


class RismError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status


class Problem(ctypes.Structure):
    _fields_ = [
        ("n_atoms", ctypes.c_int),
        ("xyz", ctypes.c_void_p), ("q", ctypes.c_void_p),
        ("sigma", ctypes.c_void_p), ("eps", ctypes.c_void_p),
        ("n_sites", ctypes.c_int),
        ("site_q", ctypes.c_void_p), ("site_sigma", ctypes.c_void_p),
        ("site_eps", ctypes.c_void_p), ("site_rho", ctypes.c_void_p),
        ("n_k", ctypes.c_int), ("dk", ctypes.c_double), ("chi", ctypes.c_void_p),
        ("temperature", ctypes.c_double),
        ("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
        ("spacing", ctypes.c_double), ("center", ctypes.c_double * 3),
        ("compressibility", ctypes.c_double), ("pressure", ctypes.c_double),
    ]


class Opts(ctypes.Structure):
    _fields_ = [
        ("closure", ctypes.c_int), ("pse_order", ctypes.c_int), ("tol", ctypes.c_double),
        ("max_iter", ctypes.c_int), ("mdiis_depth", ctypes.c_int),
        ("mdiis_eta", ctypes.c_double), ("eta_dynamic", ctypes.c_int),
        ("check_every", ctypes.c_int), ("anchor_every", ctypes.c_int),
        ("accelerator", ctypes.c_int), ("anderson_s1", ctypes.c_double),
        ("anderson_s2", ctypes.c_double),
    ]


class Info(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int), ("rms", ctypes.c_double),
                ("restarts", ctypes.c_int), ("warm_start_used", ctypes.c_int)]


class ThermoOut(ctypes.Structure):
    _fields_ = [("sfe", ctypes.c_double), ("sfe_site", ctypes.c_double * MAX_SITES),
                ("rho_int_c", ctypes.c_double * MAX_SITES), ("rho_int_c_total", ctypes.c_double),
                ("pmv", ctypes.c_double), ("pc", ctypes.c_double), ("sfe_pc", ctypes.c_double)]


class Tuning(ctypes.Structure):
    _fields_ = [("y_lines", ctypes.c_int), ("z_cols", ctypes.c_int), ("x_lines", ctypes.c_int),
                ("y_us", ctypes.c_double), ("z_us", ctypes.c_double), ("x_us", ctypes.c_double),
                ("y_default_us", ctypes.c_double), ("z_default_us", ctypes.c_double),
                ("x_default_us", ctypes.c_double)]


class UnetConfig(ctypes.Structure):
    _fields_ = [("levels", ctypes.c_int), ("base", ctypes.c_int), ("in_channels", ctypes.c_int),
                ("out_channels", ctypes.c_int), ("slope", ctypes.c_float)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() first")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER
    vp, sz, st = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p
    sig = {
        "rism3d_workspace_bytes": (sz, [P(Problem), P(Opts)]),
        "rism3d_potential": (ctypes.c_int, [P(Problem), P(Opts), vp, sz, st]),
        "rism3d_solve": (ctypes.c_int, [P(Problem), P(Opts), vp, vp, sz, vp, P(Info), st]),
        "rism3d_solve_ladder": (ctypes.c_int, [P(Problem), vp, ctypes.c_int, vp, vp, sz, vp,
                                               vp, st]),
        "rism3d_thermo": (ctypes.c_int, [P(Problem), P(Opts), vp, sz, P(ThermoOut), st]),
        "rism3d_sfe_gradient": (ctypes.c_int, [P(Problem), P(Opts), vp, vp, sz, vp, st]),
        "rism3d_get_tau": (ctypes.c_int, [P(Problem), P(Opts), vp, sz, vp, st]),
        "rism3d_map": (ctypes.c_int, [P(Problem), P(Opts), vp, vp, sz, vp,
                                      P(ctypes.c_double), st]),
        "rism3d_map_increment": (ctypes.c_int, [P(Problem), P(Opts), vp, vp, vp, sz, vp,
                                                P(ctypes.c_double), st]),
        "rism3d_get_potential": (ctypes.c_int, [P(Problem), P(Opts), vp, sz, vp, vp, st]),
        "rism3d_get_history": (ctypes.c_int, [P(Problem), P(Opts), vp, sz, ctypes.c_int,
                                              P(ctypes.c_double), P(ctypes.c_int),
                                              P(ctypes.c_int), st]),
        "rism3d_transform_workspace_bytes": (sz, [ctypes.c_int] * 3),
        "rism3d_transform": (ctypes.c_int, [ctypes.c_int] * 4 + [vp, ctypes.c_int, vp, sz, st]),
        "rism3d_transform_noalloc": (ctypes.c_int, [ctypes.c_int] * 4 + [vp, ctypes.c_int, st]),
        "rism3d_timing_enable": (None, [ctypes.c_int]),
        "rism3d_timing_reset": (None, []),
        "rism3d_timing_read": (ctypes.c_int, [ctypes.c_int, P(ctypes.c_char_p), P(ctypes.c_long),
                                              P(ctypes.c_double)]),
        "rism3d_batch_workspace_bytes": (ctypes.c_size_t, [ctypes.c_int, ctypes.c_void_p, P(Opts)]),
        "rism3d_solve_batch": (ctypes.c_int, [ctypes.c_int, ctypes.c_void_p, P(Opts), ctypes.c_void_p,
                                              ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p,
                                              ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
        "rism3d_timing_select": (ctypes.c_int, [ctypes.c_char_p]),
        "rism3d_autotune": (ctypes.c_int, [P(Problem), P(Opts), vp, sz, P(Tuning), st]),
        "rism3d_tune_reset": (None, []),
        "rism3d_tune_set": (ctypes.c_int, [P(Problem), P(Opts), ctypes.c_int, ctypes.c_int,
                                           ctypes.c_int]),
        "rism3d_unet_param_count": (sz, [P(UnetConfig)]),
        "rism3d_unet_workspace_bytes": (sz, [P(UnetConfig), ctypes.c_int, ctypes.c_int,
                                             ctypes.c_int, ctypes.c_int]),
        "rism3d_unet_forward": (ctypes.c_int, [P(UnetConfig), ctypes.c_int, ctypes.c_int,
                                               ctypes.c_int, vp, vp, vp, vp, sz, st]),
        "rism3d_unet_gradient": (ctypes.c_int, [P(UnetConfig), ctypes.c_int, ctypes.c_int,
                                                ctypes.c_int, vp, vp, vp, vp, vp, vp, sz, st]),
        "rism3d_unet_adam_scratch_bytes": (sz, []),
        "rism3d_unet_adam": (ctypes.c_int, [sz, vp, vp, vp, vp, ctypes.c_int, ctypes.c_float,
                                            ctypes.c_float, ctypes.c_float, ctypes.c_float,
                                            ctypes.c_float, vp, st]),
        "rism3d_net_input": (ctypes.c_int, [P(Problem), P(Opts), vp, sz, vp, st]),
        "rism3d_csr": (ctypes.c_int, [P(Problem), P(Opts), vp, sz, vp, st]),
        "rism3d_oz_half_step": (ctypes.c_int, [P(Problem), P(Opts), vp, ctypes.c_float, vp, sz,
                                               vp, st]),
        "rism3d_warmstart": (ctypes.c_int, [P(Problem), P(Opts), P(UnetConfig), vp,
                                            ctypes.c_float, vp, sz, vp, sz, vp, st]),
        "rism3d_use_graphs": (None, [ctypes.c_int]),
        "rism3d_release_graphs": (None, []),
        "rism3d_last_error": (ctypes.c_char_p, []),
        "rism3d_constants": (None, [P(ctypes.c_double)] * 5),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


LIB = _load()
EXPORTED = ("rism3d_workspace_bytes", "rism3d_potential", "rism3d_solve", "rism3d_solve_ladder",
            "rism3d_thermo",
            "rism3d_sfe_gradient",
            "rism3d_get_tau", "rism3d_get_history", "rism3d_map", "rism3d_map_increment", "rism3d_get_potential",
            "rism3d_transform_workspace_bytes", "rism3d_transform", "rism3d_transform_noalloc",
            "rism3d_timing_enable",
            "rism3d_timing_reset", "rism3d_timing_read", "rism3d_use_graphs",
            "rism3d_release_graphs", "rism3d_timing_select",
            "rism3d_batch_workspace_bytes", "rism3d_solve_batch", "rism3d_unet_param_count",
            "rism3d_unet_workspace_bytes", "rism3d_unet_forward", "rism3d_unet_gradient",
            "rism3d_unet_adam", "rism3d_unet_adam_scratch_bytes", "rism3d_net_input", "rism3d_csr", "rism3d_oz_half_step",
            "rism3d_warmstart", "rism3d_autotune", "rism3d_tune_reset",
            "rism3d_tune_set", "rism3d_last_error", "rism3d_constants")


def last_error() -> str:
    return LIB.rism3d_last_error().decode()


def _check(status: int, allow=()):
    if status != 0 and status not in allow:
        raise RismError(status, last_error())
    return status


def constants():
    vals = [ctypes.c_double() for _ in range(5)]
    LIB.rism3d_constants(*[ctypes.byref(v) for v in vals])
    return dict(zip(("coulomb", "kboltz", "screen", "d_min", "beta_u_cap"),
                    (v.value for v in vals)))


def use_graphs(on: bool = True):
    LIB.rism3d_use_graphs(int(bool(on)))


def release_graphs():
    LIB.rism3d_release_graphs()


def timing_enable(on: bool = True):
    LIB.rism3d_timing_enable(int(bool(on)))


def timing_select(family: Optional[str] = None):
    """Restrict kernel timing to one family (None: every family)."""
    _check(LIB.rism3d_timing_select(family.encode() if family else None))


def timing_reset():
    LIB.rism3d_timing_reset()


def timing_read() -> dict:
    """{family: (launches, total_ms)} of the kernel timing collected on this thread."""
    n = LIB.rism3d_timing_read(-1, None, None, None)
    out = {}
    for i in range(n):
        name = ctypes.c_char_p()
        cnt = ctypes.c_long()
        ms = ctypes.c_double()
        LIB.rism3d_timing_read(i, ctypes.byref(name), ctypes.byref(cnt), ctypes.byref(ms))
        out[name.value.decode()] = (int(cnt.value), float(ms.value))
    return out


def _stream(stream=None) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


def _ptr(t: Optional[torch.Tensor]) -> Optional[int]:
    return None if t is None else int(t.data_ptr())


class DeviceProblem:
    """The problem statement of ``include/rism3d.h`` with its large arrays on
    the device (float64 torch tensors) and the per-site arrays on the host."""

    def __init__(self, problem, chi: np.ndarray, dk: float, device="cuda", bulk=None):
        """bulk: (compressibility [A^3 mol/kcal], pressure [kcal/(mol A^3)]) of the
        solvent, for the PMV and PC term of rism3d_thermo (None: not computed)."""
        sol = problem.solute
        dev = torch.device(device)
        f64 = torch.float64
        self.problem = problem
        self.n_atoms = sol.n_atoms
        self.xyz = torch.as_tensor(np.ascontiguousarray(sol.xyz), dtype=f64).to(dev)
        self.q = torch.as_tensor(np.ascontiguousarray(sol.q), dtype=f64).to(dev)
        self.sigma = torch.as_tensor(np.ascontiguousarray(sol.sigma), dtype=f64).to(dev)
        self.eps = torch.as_tensor(np.ascontiguousarray(sol.eps), dtype=f64).to(dev)
        self.chi = torch.as_tensor(np.ascontiguousarray(chi), dtype=f64).to(dev)
        q, sg, ep, rho = (np.ascontiguousarray(a, dtype=np.float64)
                          for a in problem.solvent.site_arrays())
        self._host = (q, sg, ep, rho)
        g = problem.grid
        self.shape = (len(q), g.nz, g.ny, g.nx)
        s = Problem()
        s.n_atoms = self.n_atoms
        s.xyz, s.q, s.sigma, s.eps = (_ptr(t) if self.n_atoms else None
                                      for t in (self.xyz, self.q, self.sigma, self.eps))
        s.n_sites = len(q)
        s.site_q, s.site_sigma, s.site_eps, s.site_rho = (a.ctypes.data for a in self._host)
        s.n_k = int(chi.shape[-1])
        s.dk = float(dk)
        s.chi = _ptr(self.chi)
        s.temperature = float(problem.solvent.temperature)
        s.nx, s.ny, s.nz = g.nx, g.ny, g.nz
        s.spacing = float(g.spacing)
        s.center[:] = [float(c) for c in g.center]
        if bulk is not None:
            s.compressibility, s.pressure = float(bulk[0]), float(bulk[1])
        self.struct = s


def make_opts(options, check_every: int = 0, anchor_every: int = 0, **override) -> Opts:
    o = Opts()
    o.closure = CLOSURES[override.get("closure", options.closure)]
    o.pse_order = int(override.get("pse_order", options.pse_order))
    o.tol = float(override.get("tol", options.tol))
    o.max_iter = int(override.get("max_iter", options.max_iter))
    o.mdiis_depth = int(override.get("mdiis_depth", options.mdiis_depth))
    o.mdiis_eta = float(override.get("mdiis_eta", options.mdiis_eta))
    o.eta_dynamic = int(bool(override.get("eta_dynamic", options.eta_dynamic)))
    o.check_every = int(check_every)
    o.anchor_every = int(anchor_every)
    o.accelerator = ACCELERATORS[override.get("accelerator",
                                              getattr(options, "accelerator", "mdiis"))]
    o.anderson_s1 = float(override.get("anderson_s1", getattr(options, "anderson_s1", 0.2)))
    o.anderson_s2 = float(override.get("anderson_s2", getattr(options, "anderson_s2", 0.0)))
    return o


# --- thin wrappers with the C names ---------------------------------------


def rism3d_workspace_bytes(dp: DeviceProblem, opts: Opts) -> int:
    n = LIB.rism3d_workspace_bytes(ctypes.byref(dp.struct), ctypes.byref(opts))
    if n == 0:
        raise RismError(1, last_error())
    return int(n)


def rism3d_potential(dp, opts, ws: torch.Tensor, stream=None):
    _check(LIB.rism3d_potential(ctypes.byref(dp.struct), ctypes.byref(opts), _ptr(ws),
                                ws.numel() * ws.element_size(), _stream(stream)))


def rism3d_solve(dp, opts, ws, tau0=None, g_out=None, stream=None, allow_noconv=False) -> Info:
    info = Info()
    allow = (3,) if allow_noconv else ()
    info.status = _check(LIB.rism3d_solve(ctypes.byref(dp.struct), ctypes.byref(opts), _ptr(tau0),
                                          _ptr(ws), ws.numel() * ws.element_size(), _ptr(g_out),
                                          ctypes.byref(info), _stream(stream)), allow)
    return info


def rism3d_solve_ladder(dp, stages, ws, tau0=None, g_out=None, stream=None):
    """Closure ladder: a list of Opts run in order, each stage from the last
    one's iterate; returns the list of Info of the stages (a failing last
    stage, or a stage failing otherwise than by reaching max_iter, raises)."""
    n = len(stages)
    arr = (Opts * n)(*stages)
    infos = (Info * n)()
    status = LIB.rism3d_solve_ladder(ctypes.byref(dp.struct), ctypes.cast(arr, ctypes.c_void_p), n,
                                     _ptr(tau0), _ptr(ws), ws.numel() * ws.element_size(),
                                     _ptr(g_out), ctypes.cast(infos, ctypes.c_void_p),
                                     _stream(stream))
    _check(status)
    out = list(infos)
    for inf, op in zip(out, stages):   # a stage short of its tolerance hands on (E_NOCONV)
        inf.status = 0 if inf.rms < op.tol else 3
    return out


def rism3d_thermo(dp, opts, ws, stream=None):
    out = ThermoOut()
    _check(LIB.rism3d_thermo(ctypes.byref(dp.struct), ctypes.byref(opts), _ptr(ws),
                             ws.numel() * ws.element_size(), ctypes.byref(out), _stream(stream)))
    nv = dp.struct.n_sites
    return out.sfe, np.array(out.sfe_site[:nv])


def rism3d_sfe_gradient(dp, opts, ws, g: torch.Tensor, out: Optional[torch.Tensor] = None,
                        stream=None) -> torch.Tensor:
    """d(dmu)/dR_a [n_atoms, 3] (float64, kcal/(mol A)) for the distribution g."""
    n = dp.struct.n_atoms
    gc = g.contiguous()
    if gc.dtype != torch.float32 or tuple(gc.shape) != tuple(dp.shape):
        raise ValueError(f"g must be float32 {tuple(dp.shape)}")
    if out is None:
        out = torch.empty((n, 3), dtype=torch.float64, device=ws.device)
    _check(LIB.rism3d_sfe_gradient(ctypes.byref(dp.struct), ctypes.byref(opts), _ptr(gc),
                                   _ptr(ws), ws.numel() * ws.element_size(),
                                   _ptr(out) if n > 0 else None, _stream(stream)))
    return out


def rism3d_thermo_all(dp, opts, ws, stream=None) -> dict:
    """Every field of rism3d_thermo_out: SFE (total, per site), rho_g int c_g,
    PMV (Eq 19), PC term (Eq 21) and SFE + PC."""
    out = ThermoOut()
    _check(LIB.rism3d_thermo(ctypes.byref(dp.struct), ctypes.byref(opts), _ptr(ws),
                             ws.numel() * ws.element_size(), ctypes.byref(out), _stream(stream)))
    return _thermo_dict(out, dp.struct.n_sites)


def _thermo_dict(out, nv: int) -> dict:
    return {"sfe": out.sfe, "sfe_site": np.array(out.sfe_site[:nv]),
            "rho_int_c": np.array(out.rho_int_c[:nv]), "rho_int_c_total": out.rho_int_c_total,
            "pmv": out.pmv, "pc": out.pc, "sfe_pc": out.sfe_pc}


def rism3d_get_tau(dp, opts, ws, tau_out, stream=None):
    _check(LIB.rism3d_get_tau(ctypes.byref(dp.struct), ctypes.byref(opts), _ptr(ws),
                              ws.numel() * ws.element_size(), _ptr(tau_out), _stream(stream)))


def rism3d_get_history(dp, opts, ws, stream=None):
    """(rms [n] float64, exact [n] bool) of every evaluation of the last solve."""
    count = ctypes.c_int()
    _check(LIB.rism3d_get_history(ctypes.byref(dp.struct), ctypes.byref(opts), _ptr(ws),
                                  ws.numel() * ws.element_size(), 0, None, None,
                                  ctypes.byref(count), _stream(stream)))
    n = count.value
    rms = np.zeros(n, dtype=np.float64)
    exact = np.zeros(n, dtype=np.int32)
    if n:
        _check(LIB.rism3d_get_history(
            ctypes.byref(dp.struct), ctypes.byref(opts), _ptr(ws), ws.numel() * ws.element_size(),
            n, rms.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
            exact.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), ctypes.byref(count),
            _stream(stream)))
    return rms, exact.astype(bool)


def rism3d_map(dp, opts, ws, tau, res_out, stream=None) -> float:
    """tau None: the iterate the last solve on ws returned, as it is held."""
    rms = ctypes.c_double()
    _check(LIB.rism3d_map(ctypes.byref(dp.struct), ctypes.byref(opts), _ptr(tau), _ptr(ws),
                          ws.numel() * ws.element_size(), _ptr(res_out), ctypes.byref(rms),
                          _stream(stream)))
    return rms.value


def rism3d_map_increment(dp, opts, ws, tau_ref, delta, res_out, stream=None) -> float:
    rms = ctypes.c_double()
    _check(LIB.rism3d_map_increment(ctypes.byref(dp.struct), ctypes.byref(opts), _ptr(tau_ref),
                                    _ptr(delta), _ptr(ws), ws.numel() * ws.element_size(),
                                    _ptr(res_out), ctypes.byref(rms), _stream(stream)))
    return rms.value


def rism3d_get_potential(dp, opts, ws, w_out=None, phi_out=None, stream=None):
    _check(LIB.rism3d_get_potential(ctypes.byref(dp.struct), ctypes.byref(opts), _ptr(ws),
                                    ws.numel() * ws.element_size(), _ptr(w_out), _ptr(phi_out),
                                    _stream(stream)))


def rism3d_transform(data: torch.Tensor, forward: bool, ws: Optional[torch.Tensor] = None,
                     stream=None):
    """In-place shifted 3D transform of complex64 data [count, nz, ny, nx]."""
    assert data.dtype == torch.complex64 and data.is_contiguous() and data.dim() == 4
    count, nz, ny, nx = data.shape
    need = LIB.rism3d_transform_workspace_bytes(nx, ny, nz)
    if need == 0:
        raise RismError(1, last_error())
    if ws is None:
        ws = torch.empty(need, dtype=torch.uint8, device=data.device)
    _check(LIB.rism3d_transform(nx, ny, nz, count, _ptr(data), int(bool(forward)), _ptr(ws),
                                ws.numel(), _stream(stream)))
    return data


def rism3d_transform_noalloc(data: torch.Tensor, forward: bool, stream=None):
    """rism3d_transform with the library's static twiddle scratch (no workspace)."""
    assert data.dtype == torch.complex64 and data.is_contiguous() and data.dim() == 4
    count, nz, ny, nx = data.shape
    _check(LIB.rism3d_transform_noalloc(nx, ny, nz, count, _ptr(data), int(bool(forward)),
                                        _stream(stream)))
    return data


def _problem_array(dps):
    arr = (Problem * len(dps))()
    for i, dp in enumerate(dps):
        arr[i] = dp.struct
    return arr


def rism3d_batch_workspace_bytes(dps, opts: Opts) -> int:
    arr = _problem_array(dps)
    n = LIB.rism3d_batch_workspace_bytes(len(dps), ctypes.cast(arr, ctypes.c_void_p),
                                         ctypes.byref(opts))
    if n == 0:
        raise RismError(1, last_error())
    return n


def rism3d_solve_batch(dps, opts: Opts, ws: torch.Tensor, tau0=None, g_out=None, stream=None,
                       allow_noconv=False, thermo=True, full_thermo=False):
    """Batched potential + solve (+ SFE) of several problems; returns the list of
    Info and the list of (sfe, per-site sfe), or of rism3d_thermo_all's
    dictionaries when full_thermo, or None."""
    n = len(dps)
    arr = _problem_array(dps)
    ptrs = lambda ts: (None if ts is None else
                       (ctypes.c_void_p * n)(*[_ptr(t) if t is not None else None for t in ts]))
    tau_arr, g_arr = ptrs(tau0), ptrs(g_out)
    infos = (Info * n)()
    th = (ThermoOut * n)() if thermo else None
    status = LIB.rism3d_solve_batch(n, ctypes.cast(arr, ctypes.c_void_p), ctypes.byref(opts),
                                    tau_arr and ctypes.cast(tau_arr, ctypes.c_void_p), _ptr(ws),
                                    ws.numel(), g_arr and ctypes.cast(g_arr, ctypes.c_void_p),
                                    ctypes.cast(infos, ctypes.c_void_p),
                                    th and ctypes.cast(th, ctypes.c_void_p), _stream(stream))
    _check(status, allow=(3, 4) if allow_noconv else ())
    out_info = list(infos)
    for inf in out_info:
        inf.status = status
    sfe = None
    if thermo and full_thermo:
        sfe = [_thermo_dict(t, dp.shape[0]) for t, dp in zip(th, dps)]
    elif thermo:
        sfe = [(t.sfe, np.array(t.sfe_site[:dp.shape[0]])) for t, dp in zip(th, dps)]
    return out_info, sfe


def rism3d_autotune(dp, opts, ws, stream=None) -> dict:
    t = Tuning()
    _check(LIB.rism3d_autotune(ctypes.byref(dp.struct), ctypes.byref(opts), _ptr(ws), ws.numel(),
                               ctypes.byref(t), _stream(stream)))
    return {f: getattr(t, f) for f, _ in Tuning._fields_}


def tune_reset():
    LIB.rism3d_tune_reset()


def tune_set(dp, opts, y_lines: int, z_cols: int, x_lines: int = 0):
    _check(LIB.rism3d_tune_set(ctypes.byref(dp.struct), ctypes.byref(opts), int(y_lines),
                               int(z_cols), int(x_lines)))


# --- warm-start network ------------------------------------------------------


def unet_config(in_channels: int, out_channels: int, levels: int = 4, base: int = 16,
                slope: float = 0.1) -> UnetConfig:
    c = UnetConfig()
    c.levels, c.base, c.in_channels, c.out_channels, c.slope = (
        levels, base, in_channels, out_channels, slope)
    return c


def unet_layers(cfg: UnetConfig):
    """(name, C_in, C_out) of every convolution, in parameter order."""
    ch = lambda l: cfg.base << l
    out = []
    for l in range(cfg.levels):
        out += [(f"enc{l}a", cfg.in_channels if l == 0 else ch(l - 1), ch(l)),
                (f"enc{l}b", ch(l), ch(l))]
    for l in range(cfg.levels - 2, -1, -1):
        out += [(f"dec{l}a", ch(l + 1) + ch(l), ch(l)), (f"dec{l}b", ch(l), ch(l))]
    return out + [("out", ch(0), cfg.out_channels)]


def unet_param_count(cfg: UnetConfig) -> int:
    n = LIB.rism3d_unet_param_count(ctypes.byref(cfg))
    if n == 0:
        raise RismError(1, last_error())
    return n


def unet_workspace_bytes(cfg: UnetConfig, shape, training: bool) -> int:
    nz, ny, nx = shape
    n = LIB.rism3d_unet_workspace_bytes(ctypes.byref(cfg), nx, ny, nz, int(bool(training)))
    if n == 0:
        raise RismError(1, last_error())
    return n


def unet_forward(cfg, params: torch.Tensor, x: torch.Tensor, out: torch.Tensor, ws, stream=None):
    nz, ny, nx = x.shape[1:]
    _check(LIB.rism3d_unet_forward(ctypes.byref(cfg), nx, ny, nz, _ptr(params), _ptr(x),
                                   _ptr(out), _ptr(ws), ws.numel(), _stream(stream)))
    return out


def unet_gradient(cfg, params, x, target, grad, ws, loss: Optional[torch.Tensor] = None,
                  stream=None):
    nz, ny, nx = x.shape[1:]
    _check(LIB.rism3d_unet_gradient(ctypes.byref(cfg), nx, ny, nz, _ptr(params), _ptr(x),
                                    _ptr(target), _ptr(grad), _ptr(loss), _ptr(ws), ws.numel(),
                                    _stream(stream)))
    return grad


def unet_adam_scratch(device="cuda") -> torch.Tensor:
    return torch.zeros(LIB.rism3d_unet_adam_scratch_bytes() // 8, dtype=torch.float64,
                       device=device)


def unet_adam(params, m, v, grad, step: int, lr: float, beta1=0.9, beta2=0.999, eps=1e-8,
              clip_norm: float = 0.0, scratch: Optional[torch.Tensor] = None, stream=None):
    """One Adam step; clip_norm > 0 clips the global gradient norm (scratch from
    unet_adam_scratch(); its last two entries receive |g| and the scale)."""
    _check(LIB.rism3d_unet_adam(params.numel(), _ptr(params), _ptr(m), _ptr(v), _ptr(grad),
                                int(step), lr, beta1, beta2, eps, float(clip_norm), _ptr(scratch),
                                _stream(stream)))


def rism3d_net_input(dp, opts, ws, x, stream=None):
    _check(LIB.rism3d_net_input(ctypes.byref(dp.struct), ctypes.byref(opts), _ptr(ws),
                                ws.numel(), _ptr(x), _stream(stream)))
    return x


def rism3d_csr(dp, opts, ws, c, stream=None):
    _check(LIB.rism3d_csr(ctypes.byref(dp.struct), ctypes.byref(opts), _ptr(ws), ws.numel(),
                          _ptr(c), _stream(stream)))
    return c


def rism3d_oz_half_step(dp, opts, ws, c0, tau0, c_scale: float = 1.0, stream=None):
    _check(LIB.rism3d_oz_half_step(ctypes.byref(dp.struct), ctypes.byref(opts), _ptr(c0),
                                   float(c_scale), _ptr(ws), ws.numel(), _ptr(tau0),
                                   _stream(stream)))
    return tau0


def rism3d_warmstart(dp, opts, cfg, params, ws, net_ws, tau0, c_scale: float = 1.0, stream=None):
    _check(LIB.rism3d_warmstart(ctypes.byref(dp.struct), ctypes.byref(opts), ctypes.byref(cfg),
                                _ptr(params), float(c_scale), _ptr(ws), ws.numel(), _ptr(net_ws),
                                net_ws.numel(), _ptr(tau0), _stream(stream)))
    return tau0


WEIGHTS_PATH = os.path.join(_HERE, "weights", "warmstart_unet.npz")


class WarmStart:
    """Trained warm-start network: configuration, FP32 parameters on the
    device, the output scale c_scale and an inference workspace."""

    def __init__(self, path: str = WEIGHTS_PATH, device="cuda"):
        with np.load(path, allow_pickle=False) as z:
            self.cfg = unet_config(int(z["in_channels"]), int(z["out_channels"]),
                                   levels=int(z["levels"]), base=int(z["base"]),
                                   slope=float(z["slope"]))
            self.params = torch.tensor(np.asarray(z["params"], dtype=np.float32), device=device)
            self.c_scale = float(z["c_scale"])
        if self.params.numel() != unet_param_count(self.cfg):
            raise ValueError(f"{path}: parameter count does not match the configuration")
        self.device = device
        self._ws = {}

    def tau0(self, dp, opts, ws, out: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
        """Starting tau of a prepared workspace (after rism3d_potential)."""
        shape = dp.shape[1:]
        if shape not in self._ws:
            self._ws[shape] = alloc_workspace(unet_workspace_bytes(self.cfg, shape, False),
                                              self.device)
        if out is None:
            out = torch.empty(dp.shape, dtype=torch.float32, device=self.device)
        return rism3d_warmstart(dp, opts, self.cfg, self.params, ws, self._ws[shape], out,
                                self.c_scale, stream)


# --- convenience -------------------------------------------------------------


def alloc_workspace(nbytes: int, device="cuda") -> torch.Tensor:
    ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
    off = (-ws.data_ptr()) % 256
    return ws[off:off + nbytes]


class Solver:
    """Owns a workspace for one problem and runs potential -> solve -> thermo."""

    def __init__(self, dp: DeviceProblem, opts: Opts):
        self.dp = dp
        self.opts = opts
        self.nbytes = rism3d_workspace_bytes(dp, opts)
        self.ws = alloc_workspace(self.nbytes, dp.xyz.device)

    def potential(self, stream=None):
        rism3d_potential(self.dp, self.opts, self.ws, stream)

    def solve(self, tau0=None, g_out=None, stream=None, allow_noconv=False) -> Info:
        return rism3d_solve(self.dp, self.opts, self.ws, tau0, g_out, stream, allow_noconv)

    def solve_ladder(self, stages, tau0=None, g_out=None, stream=None):
        """Runs the stages (Opts) in order; self.opts becomes the last stage's
        (for thermo and map calls that follow)."""
        infos = rism3d_solve_ladder(self.dp, stages, self.ws, tau0, g_out, stream)
        self.opts = stages[-1]
        return infos

    def thermo(self, stream=None):
        return rism3d_thermo(self.dp, self.opts, self.ws, stream)

    def thermo_all(self, stream=None) -> dict:
        return rism3d_thermo_all(self.dp, self.opts, self.ws, stream)

    def sfe_gradient(self, g: torch.Tensor, stream=None) -> torch.Tensor:
        return rism3d_sfe_gradient(self.dp, self.opts, self.ws, g, stream=stream)

    def history(self, stream=None):
        return rism3d_get_history(self.dp, self.opts, self.ws, stream)

    def tau(self) -> torch.Tensor:
        t = torch.empty(self.dp.shape, dtype=torch.float32, device=self.ws.device)
        rism3d_get_tau(self.dp, self.opts, self.ws, t)
        return t

    def fields(self):
        w = torch.empty(self.dp.shape, dtype=torch.float32, device=self.ws.device)
        phi = torch.empty(self.dp.shape[1:], dtype=torch.float32, device=self.ws.device)
        rism3d_get_potential(self.dp, self.opts, self.ws, w, phi)
        return w, phi

    def map(self, tau: Optional[torch.Tensor]):
        """Exact evaluation of the map at tau (None: at the held solution)."""
        res = torch.empty(self.dp.shape, dtype=torch.float32, device=self.ws.device)
        rms = rism3d_map(self.dp, self.opts, self.ws, None if tau is None else tau.contiguous(),
                         res)
        return res, rms

    def map_increment(self, tau_ref: torch.Tensor, delta: torch.Tensor):
        """The map at tau_ref + delta through the FP32 increment kernels."""
        res = torch.empty(self.dp.shape, dtype=torch.float32, device=self.ws.device)
        rms = rism3d_map_increment(self.dp, self.opts, self.ws, tau_ref.contiguous(),
                                   delta.contiguous(), res)
        return res, rms
