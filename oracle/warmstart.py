"""FP64 oracle of the warm start around the network (test infrastructure
only; never called by the library).

The network maps a transform of the solute potential to an initial
short-range direct correlation c0 (not in the paper, which starts at t = f).
The starting tau then follows from one Ornstein-Zernike half-step: with c0 in
place of the closure's c_sr, steps 3-5 of "Numerical procedure" (Eq 32, then
Eq 13, then the inverse transform) give h0, and since the update of Eq 33 is
t' = t + h + 1 - g = h - c_sr + f, the starting iterate is
    tau0 = t0 - f = h0 - c0.
At the fixed point this returns tau* itself (tau* = h* - c*).
"""
from __future__ import annotations

import numpy as np

from oracle import fft as offt
from oracle import rism3d as O


def symlog(v: np.ndarray) -> np.ndarray:
    """sign(v) log(1 + |v|): compresses the capped beta*u (up to 1e4)."""
    return np.sign(v) * np.log1p(np.abs(v))


def net_input(sys_: O.System) -> np.ndarray:
    """Network input, channels last: x[z, y, x, g] = symlog(beta u_g)."""
    return np.moveaxis(symlog(sys_.beta_u), 0, -1)


def csr_of(sys_: O.System, tau: np.ndarray) -> np.ndarray:
    """Short-range direct correlation of Eq 31 in tau-form, channels last:
    c_sr = g - 1 - tau with g = closure(-w + tau), w = beta u - f."""
    d = -(sys_.beta_u - sys_.f) + tau
    g = O.closure(d, sys_.kind, sys_.order)
    return np.moveaxis(g - 1.0 - tau, 0, -1)


def oz_half_step(sys_: O.System, c0: np.ndarray) -> np.ndarray:
    """tau0 = h0 - c0 with h0 = IFT[ sum_g' (FT[c0_g'] - ftilde_g') chi_g'g ]
    (Eq 32, Eq 13); c0 channels last, tau0 site-major like the solver."""
    c = np.moveaxis(c0, -1, 0)
    ck = offt.forward3(c, sys_.dv) - sys_.ftilde
    hk = np.einsum("ab...,a...->b...", sys_.chi, ck)
    h = offt.inverse3(hk, sys_.dv).real
    return h - c
