"""FP64 oracle of the warm-start network (test infrastructure only; never
called by the library).

The warm start is not in the paper (the paper starts every solve at t = f,
"Numerical procedure", step 1); it is the learned initial guess of the
solver's specification: a 3D convolutional encoder-decoder that maps the
solute potential of each solvent site to an initial short-range direct
correlation c_sr.  This module is the plain definition of that network, its
gradients and its optimiser, written as directly as numpy allows:

* tensors are one sample, channels last: x[z, y, x, c];
* conv3(x, W, b): 3x3x3 cross-correlation with zero padding one voxel wide,
      y[v, o] = b[o] + sum_{k, i} x[v + off(k), i] W[o, k, i],
  where k = (dz * 3 + dy) * 3 + dx indexes the offsets off(k) = (dz-1, dy-1, dx-1);
* leaky(x) = x for x > 0, slope * x otherwise;
* pool2: mean over 2x2x2 blocks; up2: nearest-neighbour copy into 2x2x2 blocks;
* U-Net with L levels and channels C_l = base * 2^l:
      encoder level l:  a = leaky(conv3(in_l)), e_l = leaky(conv3(a)),
                        in_0 = input, in_{l+1} = pool2(e_l);
      decoder level l (L-2 .. 0):  in = concat(up2(d_{l+1}), e_l) (upsampled
                        channels first), a = leaky(conv3(in)), d_l = leaky(conv3(a)),
                        with d_{L-1} = e_{L-1};
      output = conv3(d_0) (no activation);
  parameters in that order (enc0a, enc0b, ..., dec_{L-2}a, dec_{L-2}b, ...,
  dec0a, dec0b, out), each W[C_out, 27, C_in] then b[C_out];
* loss = mean over voxels and output channels of (output - target)^2;
* Adam (Kingma & Ba 2015) with bias correction, optionally after scaling the
  gradient to a global L2 norm of at most `clip`.
"""
from __future__ import annotations

import dataclasses
from typing import List, Tuple

import numpy as np

OFFSETS = [(dz - 1, dy - 1, dx - 1) for dz in range(3) for dy in range(3) for dx in range(3)]


# ---------------------------------------------------------------------------
# Layers
# ---------------------------------------------------------------------------

def _shifted(xp: np.ndarray, off, shape) -> np.ndarray:
    """Window of the one-voxel zero-padded array xp at offset off."""
    dz, dy, dx = off
    nz, ny, nx = shape
    return xp[1 + dz:1 + dz + nz, 1 + dy:1 + dy + ny, 1 + dx:1 + dx + nx]


def conv3(x: np.ndarray, W: np.ndarray, b: np.ndarray) -> np.ndarray:
    """y[v, o] = b[o] + sum_k sum_i x[v + off(k), i] W[o, k, i] (zero outside)."""
    shape = x.shape[:3]
    xp = np.pad(x, ((1, 1), (1, 1), (1, 1), (0, 0)))
    y = np.broadcast_to(b, shape + (W.shape[0],)).astype(np.float64).copy()
    for k, off in enumerate(OFFSETS):
        y += _shifted(xp, off, shape) @ W[:, k, :].T
    return y


def conv3_backward(x: np.ndarray, W: np.ndarray, dy: np.ndarray):
    """Gradients of sum(dy * conv3(x, W, b)) with respect to x, W and b."""
    shape = x.shape[:3]
    xp = np.pad(x, ((1, 1), (1, 1), (1, 1), (0, 0)))
    dxp = np.zeros_like(xp)
    dW = np.zeros_like(W)
    for k, off in enumerate(OFFSETS):
        dz, dy_, dx_ = off
        win = (slice(1 + dz, 1 + dz + shape[0]), slice(1 + dy_, 1 + dy_ + shape[1]),
               slice(1 + dx_, 1 + dx_ + shape[2]))
        dxp[win] += dy @ W[:, k, :]
        dW[:, k, :] = np.einsum("zyxo,zyxi->oi", dy, xp[win])
    db = dy.sum(axis=(0, 1, 2))
    return dxp[1:-1, 1:-1, 1:-1], dW, db


def leaky(x: np.ndarray, slope: float) -> np.ndarray:
    return np.where(x > 0, x, slope * x)


def leaky_backward(y: np.ndarray, dy: np.ndarray, slope: float) -> np.ndarray:
    """Derivative through leaky, taken from the sign of its output y."""
    return np.where(y > 0, dy, slope * dy)


def pool2(x: np.ndarray) -> np.ndarray:
    nz, ny, nx, c = x.shape
    return x.reshape(nz // 2, 2, ny // 2, 2, nx // 2, 2, c).mean(axis=(1, 3, 5))


def pool2_backward(dy: np.ndarray) -> np.ndarray:
    return up2(dy) / 8.0


def up2(x: np.ndarray) -> np.ndarray:
    return x.repeat(2, axis=0).repeat(2, axis=1).repeat(2, axis=2)


def up2_backward(dy: np.ndarray) -> np.ndarray:
    nz, ny, nx, c = dy.shape
    return dy.reshape(nz // 2, 2, ny // 2, 2, nx // 2, 2, c).sum(axis=(1, 3, 5))


# ---------------------------------------------------------------------------
# Network
# ---------------------------------------------------------------------------

@dataclasses.dataclass(frozen=True)
class Config:
    levels: int = 4
    base: int = 16
    in_channels: int = 3
    out_channels: int = 3
    slope: float = 0.1

    def channels(self, level: int) -> int:
        return self.base << level

    def layers(self) -> List[Tuple[str, int, int]]:
        """(name, C_in, C_out) of every convolution in parameter order."""
        out = []
        for l in range(self.levels):
            cin = self.in_channels if l == 0 else self.channels(l - 1)
            out.append((f"enc{l}a", cin, self.channels(l)))
            out.append((f"enc{l}b", self.channels(l), self.channels(l)))
        for l in range(self.levels - 2, -1, -1):
            out.append((f"dec{l}a", self.channels(l + 1) + self.channels(l), self.channels(l)))
            out.append((f"dec{l}b", self.channels(l), self.channels(l)))
        out.append(("out", self.channels(0), self.out_channels))
        return out

    def param_count(self) -> int:
        return sum(co * 27 * ci + co for _, ci, co in self.layers())


def unpack(cfg: Config, theta: np.ndarray):
    """Flat parameter vector -> list of (W[C_out, 27, C_in], b[C_out])."""
    params, off = [], 0
    for _, ci, co in cfg.layers():
        W = theta[off:off + co * 27 * ci].reshape(co, 27, ci)
        off += co * 27 * ci
        b = theta[off:off + co]
        off += co
        params.append((W, b))
    assert off == theta.size
    return params


def forward(cfg: Config, theta: np.ndarray, x: np.ndarray):
    """Network output and the activations the backward pass needs."""
    P = unpack(cfg, theta)
    acts = {}
    h = x
    j = 0
    enc = []
    for l in range(cfg.levels):
        if l > 0:
            h = pool2(enc[-1])
        acts[j] = h
        a = leaky(conv3(h, *P[j]), cfg.slope)
        j += 1
        acts[j] = a
        e = leaky(conv3(a, *P[j]), cfg.slope)
        j += 1
        acts[("y", j - 2)] = a
        acts[("y", j - 1)] = e
        enc.append(e)
    d = enc[-1]
    for l in range(cfg.levels - 2, -1, -1):
        inp = np.concatenate([up2(d), enc[l]], axis=-1)
        acts[j] = inp
        a = leaky(conv3(inp, *P[j]), cfg.slope)
        acts[("y", j)] = a
        j += 1
        acts[j] = a
        d = leaky(conv3(a, *P[j]), cfg.slope)
        acts[("y", j)] = d
        j += 1
    acts[j] = d
    out = conv3(d, *P[j])
    return out, acts


def backward(cfg: Config, theta: np.ndarray, acts, dout: np.ndarray):
    """Gradient of sum(dout * forward(theta, x)) with respect to theta and x."""
    P = unpack(cfg, theta)
    L = cfg.levels
    grads = [None] * len(P)
    j = len(P) - 1
    dx, dW, db = conv3_backward(acts[j], P[j][0], dout)
    grads[j] = (dW, db)
    d_d = dx                                    # gradient at d_0
    d_enc = [None] * L
    for l in range(0, L - 1):
        # decoder level l, walked from the output back towards the bottleneck
        jb = len(P) - 2 - 2 * l                 # dec_l b
        ja = jb - 1                             # dec_l a
        dpre = leaky_backward(acts[("y", jb)], d_d, cfg.slope)
        dx, dW, db = conv3_backward(acts[jb], P[jb][0], dpre)
        grads[jb] = (dW, db)
        dpre = leaky_backward(acts[("y", ja)], dx, cfg.slope)
        dx, dW, db = conv3_backward(acts[ja], P[ja][0], dpre)
        grads[ja] = (dW, db)
        cu = cfg.channels(l + 1)
        d_enc[l] = dx[..., cu:]                 # skip branch
        d_d = up2_backward(dx[..., :cu])        # to d_{l+1}
    d_enc[L - 1] = d_d
    dinput = None
    for l in range(L - 1, -1, -1):
        g = d_enc[l]
        jb = 2 * l + 1
        ja = 2 * l
        dpre = leaky_backward(acts[("y", jb)], g, cfg.slope)
        dx, dW, db = conv3_backward(acts[jb], P[jb][0], dpre)
        grads[jb] = (dW, db)
        dpre = leaky_backward(acts[("y", ja)], dx, cfg.slope)
        dx, dW, db = conv3_backward(acts[ja], P[ja][0], dpre)
        grads[ja] = (dW, db)
        if l > 0:
            d_enc[l - 1] = d_enc[l - 1] + pool2_backward(dx)
        else:
            dinput = dx
    flat = np.concatenate([np.concatenate([dW.ravel(), db]) for dW, db in grads])
    return flat, dinput


def mse(out: np.ndarray, target: np.ndarray):
    """Mean squared error over voxels and channels, and its gradient."""
    diff = out - target
    return float(np.mean(diff * diff)), 2.0 * diff / diff.size


def loss_and_grad(cfg: Config, theta: np.ndarray, x: np.ndarray, target: np.ndarray):
    out, acts = forward(cfg, theta, x)
    loss, dout = mse(out, target)
    g, _ = backward(cfg, theta, acts, dout)
    return loss, g


@dataclasses.dataclass
class Adam:
    lr: float = 1e-3
    beta1: float = 0.9
    beta2: float = 0.999
    eps: float = 1e-8

    clip: float = 0.0        # > 0: scale the gradient to global L2 norm <= clip first

    def step(self, theta, grad, m, v, t: int):
        """One update at step t >= 1; returns (theta, m, v)."""
        if self.clip > 0.0:
            norm = float(np.sqrt(np.sum(grad * grad)))
            if norm > self.clip:
                grad = grad * (self.clip / norm)
        m = self.beta1 * m + (1.0 - self.beta1) * grad
        v = self.beta2 * v + (1.0 - self.beta2) * grad * grad
        mhat = m / (1.0 - self.beta1 ** t)
        vhat = v / (1.0 - self.beta2 ** t)
        return theta - self.lr * mhat / (np.sqrt(vhat) + self.eps), m, v

