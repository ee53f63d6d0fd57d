"""Pins of the warm-start network oracle (oracle/unet.py) and of the
warm-start half-step (oracle/warmstart.py), each against something other
than the oracle itself: brute-force sums, identities, central finite
differences, the closed form of Adam under a constant gradient, and the
Ornstein-Zernike relation at the converged fixed point."""
import itertools

import numpy as np
import pytest

from oracle import unet as U
from oracle import warmstart as WS
from oracle import rism3d as O
from paper_2403_01039_amd import inputs


def _conv_bruteforce(x, W, b):
    nz, ny, nx, ci = x.shape
    co = W.shape[0]
    y = np.zeros((nz, ny, nx, co))
    for z, yy, xx, o in itertools.product(range(nz), range(ny), range(nx), range(co)):
        s = b[o]
        for dz, dy, dx in itertools.product(range(3), repeat=3):
            zz, y2, x2 = z + dz - 1, yy + dy - 1, xx + dx - 1
            if 0 <= zz < nz and 0 <= y2 < ny and 0 <= x2 < nx:
                for i in range(ci):
                    s += x[zz, y2, x2, i] * W[o, (dz * 3 + dy) * 3 + dx, i]
        y[z, yy, xx, o] = s
    return y


def test_conv3_equals_bruteforce_sum():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((3, 4, 5, 2))
    W = rng.standard_normal((3, 27, 2))
    b = rng.standard_normal(3)
    assert np.abs(U.conv3(x, W, b) - _conv_bruteforce(x, W, b)).max() < 1e-12


def test_conv3_delta_kernels():
    """The centre tap is the identity; the tap at offset (0, 0, +1) shifts by
    one voxel along x with a zero fill at the far face."""
    rng = np.random.default_rng(1)
    x = rng.standard_normal((4, 4, 6, 3))
    W = np.zeros((3, 27, 3))
    W[:, 13, :] = np.eye(3)
    assert np.array_equal(U.conv3(x, W, np.zeros(3)), x)
    W = np.zeros((3, 27, 3))
    W[:, 14, :] = np.eye(3)                      # (dz, dy, dx) = (0, 0, +1)
    y = U.conv3(x, W, np.zeros(3))
    assert np.array_equal(y[:, :, :-1], x[:, :, 1:])
    assert np.all(y[:, :, -1] == 0)


def _fd(f, v, idx, h):
    e = np.zeros_like(v)
    e.flat[idx] = h
    return (f(v + e) - f(v - e)) / (2 * h)


def test_conv3_backward_matches_finite_differences():
    rng = np.random.default_rng(2)
    x = rng.standard_normal((4, 3, 4, 3))
    W = rng.standard_normal((2, 27, 3))
    b = rng.standard_normal(2)
    dy = rng.standard_normal((4, 3, 4, 2))
    dx, dW, db = U.conv3_backward(x, W, dy)
    L = lambda x_, W_, b_: float(np.sum(dy * U.conv3(x_, W_, b_)))
    for idx in rng.choice(x.size, 12, replace=False):
        assert abs(_fd(lambda v: L(v, W, b), x, idx, 1e-3) - dx.flat[idx]) < 1e-9
    for idx in rng.choice(W.size, 12, replace=False):
        assert abs(_fd(lambda v: L(x, v, b), W, idx, 1e-3) - dW.flat[idx]) < 1e-9
    for idx in range(2):
        assert abs(_fd(lambda v: L(x, W, v), b, idx, 1e-3) - db[idx]) < 1e-9


def test_pool_and_upsample_are_adjoint_pairs():
    rng = np.random.default_rng(3)
    a = rng.standard_normal((4, 6, 8, 3))
    c = rng.standard_normal((2, 3, 4, 3))
    assert abs(np.sum(U.up2(c) * a) - np.sum(c * U.up2_backward(a))) < 1e-12
    assert abs(np.sum(U.pool2(a) * c) - np.sum(a * U.pool2_backward(c))) < 1e-12
    assert np.allclose(U.pool2(U.up2(c)), c, atol=1e-15)
    assert U.pool2(a)[1, 2, 3, 1] == pytest.approx(a[2:4, 4:6, 6:8, 1].mean(), abs=1e-15)


def test_leaky_backward_matches_finite_differences():
    x = np.array([-2.0, -0.3, 0.4, 3.0])
    y = U.leaky(x, 0.1)
    g = U.leaky_backward(y, np.ones(4), 0.1)
    fd = (U.leaky(x + 1e-6, 0.1) - U.leaky(x - 1e-6, 0.1)) / 2e-6
    assert np.allclose(g, fd, atol=1e-9)


def test_default_network_size():
    """4 levels, 16..128 channels, 3 -> 3 channels: 15 convolutions."""
    cfg = U.Config()
    layers = cfg.layers()
    assert len(layers) == 15
    assert [c for _, _, c in layers] == [16, 16, 32, 32, 64, 64, 128, 128, 64, 64, 32, 32, 16, 16, 3]
    assert layers[8] == ("dec2a", 192, 64) and layers[12] == ("dec0a", 48, 16)
    n = sum(co * (27 * ci + 1) for _, ci, co in layers)
    assert cfg.param_count() == n == 1461731   # summed by hand layer by layer


def test_network_composition_with_delta_kernels():
    """Two levels, one channel, every convolution a centre-tap identity on a
    positive input (leaky is then the identity): the output is
    a * up2(pool2(x)) + b * x, where a and b are the centre taps of the first
    decoder convolution on its first upsampled channel (index 0; two follow
    from level 1) and on its skip channel (index 2)."""
    cfg = U.Config(levels=2, base=1, in_channels=1, out_channels=1)
    rng = np.random.default_rng(4)
    x = rng.uniform(0.5, 2.0, (4, 4, 4, 1))
    for a, b, expect in [(1.0, 0.0, U.up2(U.pool2(x))), (0.0, 1.0, x),
                         (0.5, 2.0, 0.5 * U.up2(U.pool2(x)) + 2.0 * x)]:
        parts = []
        for name, ci, co in cfg.layers():
            W = np.zeros((co, 27, ci))
            if name == "dec0a":
                W[0, 13, 0], W[0, 13, cfg.channels(1)] = a, b
            else:
                W[0, 13, 0] = 1.0
            parts += [W.ravel(), np.zeros(co)]
        out, _ = U.forward(cfg, np.concatenate(parts), x)
        assert np.allclose(out, expect, rtol=0, atol=1e-14)


def test_network_gradient_matches_finite_differences():
    """Whole-network gradient (3 levels, 2..8 channels, 8^3) of the MSE loss
    against central differences, for parameters of every layer and for the
    input."""
    cfg = U.Config(levels=3, base=2, in_channels=3, out_channels=3)
    theta = inputs.unet_random_params(cfg.layers(), 5, scale=1.0).astype(np.float64)
    rng = np.random.default_rng(6)
    x = rng.standard_normal((8, 8, 8, 3))
    target = rng.standard_normal((8, 8, 8, 3))
    loss, g = U.loss_and_grad(cfg, theta, x, target)
    f = lambda th: U.loss_and_grad(cfg, th, x, target)[0]
    offs = np.cumsum([0] + [co * 27 * ci + co for _, ci, co in cfg.layers()])
    picks = [int(rng.integers(offs[i], offs[i + 1])) for i in range(len(offs) - 1)]
    picks += [int(offs[i + 1] - 1) for i in range(len(offs) - 1)]          # a bias of each layer
    for idx in picks:
        fd = _fd(f, theta, idx, 1e-5)
        assert abs(fd - g[idx]) <= 1e-6 * max(1e-3, abs(g[idx])) + 1e-10, (idx, fd, g[idx])
    out, acts = U.forward(cfg, theta, x)
    _, dout = U.mse(out, target)
    _, dinput = U.backward(cfg, theta, acts, dout)
    fx = lambda v: U.mse(U.forward(cfg, theta, v)[0], target)[0]
    for idx in rng.choice(x.size, 6, replace=False):
        fd = _fd(fx, x, idx, 1e-5)
        assert abs(fd - dinput.flat[idx]) <= 1e-6 * max(1e-3, abs(dinput.flat[idx])) + 1e-10


def test_adam_constant_gradient_closed_form():
    """With a constant gradient g the bias-corrected moments are exactly g and
    g^2, so every step moves theta by lr * g / (|g| + eps)."""
    opt = U.Adam(lr=0.01)
    g = np.array([0.5, -2.0, 1e-3])
    theta, m, v = np.zeros(3), np.zeros(3), np.zeros(3)
    for t in range(1, 6):
        theta, m, v = opt.step(theta, g, m, v, t)
        assert np.allclose(theta, -t * 0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=1e-15)


def test_adam_clipping_scales_the_first_moment():
    """With clipping the first step stores m = (1 - beta1) g c / |g| when
    |g| > c, and the unclipped m when |g| <= c."""
    g = np.array([3.0, -4.0])                    # |g| = 5
    for clip, expect in [(1.0, 0.1 * g / 5.0), (10.0, 0.1 * g)]:
        opt = U.Adam(lr=0.01, clip=clip)
        _, m, v = opt.step(np.zeros(2), g, np.zeros(2), np.zeros(2), 1)
        assert np.allclose(m, expect, rtol=1e-15)
        assert np.allclose(v, 0.001 * (expect / 0.1) ** 2, rtol=1e-12)


def test_oz_half_step_returns_the_fixed_point():
    """At the converged solution c* = g* - 1 - tau*, the half-step gives
    h* - c* = tau* (the residual h + 1 - g vanishes there)."""
    prob = inputs.small_problem(7, n_atoms=6, shape=(16, 16, 16), radius=2.5)
    chi, dk = inputs.solvent_table_for(prob.solvent)
    sys_ = O.build_system(prob, chi, dk)
    sol = O.solve(sys_, tol=1e-11)
    tau = sol.tau
    c = WS.csr_of(sys_, tau)
    tau0 = WS.oz_half_step(sys_, c)
    assert np.abs(tau0 - tau).max() < 1e-8
    # and a perturbed c moves tau0 linearly (the half-step is affine in c)
    rng = np.random.default_rng(8)
    dc = 1e-3 * rng.standard_normal(c.shape)
    t1 = WS.oz_half_step(sys_, c + dc)
    t2 = WS.oz_half_step(sys_, c + 2 * dc)
    assert np.abs((t2 - t1) - (t1 - tau0)).max() < 1e-10


def test_net_input_is_symlog_of_capped_beta_u():
    prob = inputs.small_problem(9, n_atoms=4, shape=(8, 8, 8), radius=1.5)
    chi, dk = inputs.solvent_table_for(prob.solvent)
    sys_ = O.build_system(prob, chi, dk)
    x = WS.net_input(sys_)
    assert x.shape == (8, 8, 8, prob.solvent.n_sites)
    bu = np.moveaxis(sys_.beta_u, 0, -1)
    assert np.allclose(np.sign(x) * np.expm1(np.abs(x)), bu, rtol=1e-12, atol=1e-12)
    assert x.max() <= np.log1p(1e4) + 1e-12
