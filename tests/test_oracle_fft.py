"""Pins of the oracle's own FFT and of the half-integer-shifted 3D transforms
(section "Numerical procedure": k at half-integer points, r at integers)."""
import numpy as np
import pytest

from oracle import fft as offt


@pytest.mark.parametrize("n", [1, 2, 3, 5, 7, 8, 12, 16, 17, 30, 34, 96, 128])
def test_fft_equals_bruteforce_dft(n):
    rng = np.random.default_rng(n)
    x = rng.standard_normal((3, n)) + 1j * rng.standard_normal((3, n))
    for sign in (-1, 1):
        ref = offt.dft_axis(x, sign=sign)
        got = offt.fft_axis(x, sign=sign)
        assert np.abs(got - ref).max() <= 1e-12 * max(1.0, np.abs(ref).max())


@pytest.mark.parametrize("shape", [(8, 8, 8), (6, 6, 6), (12, 12, 12), (6, 8, 10)])
def test_shifted_3d_equals_bruteforce(shape):
    rng = np.random.default_rng(sum(shape))
    x = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    dv = 0.125
    X = offt.forward3(x, dv)
    Xb = offt.forward3_bruteforce(x, dv)
    assert np.abs(X - Xb).max() <= 1e-12 * np.abs(Xb).max()
    xb = offt.inverse3_bruteforce(X, dv)
    assert np.abs(offt.inverse3(X, dv) - xb).max() <= 1e-12 * np.abs(x).max()
    assert np.abs(xb - x).max() <= 1e-12 * np.abs(x).max()
    # Parseval for the shifted (unitary up to scale) transform
    assert abs(np.sum(np.abs(X) ** 2) - x.size * dv * dv * np.sum(np.abs(x) ** 2)) \
        <= 1e-12 * np.sum(np.abs(X) ** 2)


def test_real_field_conjugate_mirror():
    """For real x: X(n-1-j) = conj X(j) per axis, the property that lets two
    real sites share one complex transform."""
    rng = np.random.default_rng(3)
    x = rng.standard_normal((6, 10, 8))
    X = offt.forward3(x, 1.0)
    mirror = X[::-1, ::-1, ::-1]
    assert np.abs(mirror - np.conj(X)).max() <= 1e-12 * np.abs(X).max()


def test_gaussian_closed_form():
    """FT of exp(-a |r - c|^2) is (pi/a)^{3/2} exp(-k^2/4a) exp(-i k.(c - r0)).
    On a fine, large grid the discrete shifted transform reproduces it to the
    aliasing level (exp(-32) here)."""
    from oracle import rism3d as O
    from paper_2403_01039_amd.inputs import Grid
    n, dr, a = 40, 0.2, 2.0
    grid = Grid(n, n, n, dr)
    pts = O.grid_points(grid)
    c = np.array([0.13, -0.07, 0.21])
    x = np.exp(-a * np.sum((pts - c) ** 2, axis=-1))
    X = offt.forward3(x, dr ** 3)
    kx, ky, kz = O.k_components(grid)
    r0 = np.array([O.axis_r(n, dr, 0.0)[0]] * 3)
    k2 = kx * kx + ky * ky + kz * kz
    ref = (np.pi / a) ** 1.5 * np.exp(-k2 / (4 * a)) \
        * np.exp(-1j * (kx * (c[0] - r0[0]) + ky * (c[1] - r0[1]) + kz * (c[2] - r0[2])))
    assert np.abs(X - ref).max() <= 1e-10 * np.abs(ref).max()
