"""Pins of the oracle's Fourier-pseudospectral Laplacian (Sec. 3).

The reference is the discrete formula of eq. discrete:laplace and eq.
discrete:fourier written out as explicit sums over p = -n/2..n/2-1 (O(n^2) per
axis, no FFT), applied axis by axis on tensor grids; plus plane-wave eigenpairs
and Parseval.
"""
import itertools

import numpy as np
import pytest

import oracle
from oracle.model import make_problem


def naive_dxx(phi, a, b, axis):
    """d_xx^f phi along ``axis`` by the explicit sums of eq. discrete:laplace."""
    n = phi.shape[axis]
    j = np.arange(n)
    p = np.arange(-n // 2, n // 2)
    lam = 2 * np.pi * p / (b - a)
    fwd = np.exp(-2j * np.pi * np.outer(p, j) / n)       # tilde phi_p = sum_j phi_j e^{-i2pi jp/n}
    inv = np.exp(2j * np.pi * np.outer(j, p) / n)        # sum_p ... e^{i 2 pi j p / n}
    ph = np.moveaxis(phi, axis, -1)
    tilde = ph @ fwd.T
    out = -(1.0 / n) * ((tilde * lam ** 2) @ inv.T)
    return np.moveaxis(out, -1, axis)


@pytest.mark.parametrize("n", [(4,), (6,), (8,), (12,), (8, 6), (4, 12), (4, 6, 8), (6, 6, 4)])
def test_laplacian_matches_naive_dft(n):
    rng = np.random.default_rng(sum(n))
    lo = tuple(-1.0 - 0.5 * i for i in range(len(n)))
    hi = tuple(2.0 + 0.25 * i for i in range(len(n)))
    prob = make_problem(1, n, lo, hi, np.zeros(tuple(reversed(n))), (0, 0), 0.5)
    X = rng.standard_normal((3,) + prob.shape) + 1j * rng.standard_normal((3,) + prob.shape)
    ref = np.zeros_like(X)
    for ax in range(len(n)):                    # L = -sum_alpha d_alpha alpha
        arr_axis = len(n) - ax                  # x is the last array axis
        ref -= naive_dxx(X, lo[ax], hi[ax], arr_axis)
    got = oracle.laplacian(prob, X)
    assert np.linalg.norm(got - ref) <= 1e-13 * np.linalg.norm(ref)


@pytest.mark.parametrize("n,p", [(16, 3), (16, -8), (12, 5), (32, -16), (10, 0)])
def test_plane_waves_are_eigenvectors(n, p):
    a, b = -3.0, 5.0
    prob = make_problem(1, (n,), (a,), (b,), np.zeros(n), (0, 0), 0.5)
    j = np.arange(n)
    w = np.exp(2j * np.pi * j * p / n)
    X = np.stack([w, 2 * w, -w])
    lam2 = (2 * np.pi * p / (b - a)) ** 2       # Nyquist p = -n/2 is kept (eq. discrete:fourier)
    assert np.allclose(oracle.laplacian(prob, X), lam2 * X, atol=1e-12 * max(1, lam2))


def test_parseval_kinetic_energy():
    n = (8, 12)
    prob = make_problem(2, n, (-2, -3), (2, 3), np.zeros((12, 8)), (0, 0, 0), 0.3)
    rng = np.random.default_rng(7)
    X = rng.standard_normal((5, 12, 8)) + 1j * rng.standard_normal((5, 12, 8))
    LX = oracle.laplacian(prob, X)
    lhs = 0.5 * np.real(np.vdot(X, LX))
    Xh = np.fft.fftn(X, axes=(1, 2))
    lam = [(2 * np.pi * np.fft.fftfreq(m, d=1.0 / m) / (b - a)) ** 2 for m, a, b in zip(n, prob.lo, prob.hi)]
    lam[0][n[0] // 2] = (np.pi * n[0] / (prob.hi[0] - prob.lo[0])) ** 2
    lam[1][n[1] // 2] = (np.pi * n[1] / (prob.hi[1] - prob.lo[1])) ** 2
    Lam = lam[1][:, None] + lam[0][None, :]
    rhs = 0.5 / np.prod(n) * np.sum(Lam * np.abs(Xh) ** 2)
    assert abs(lhs - rhs) <= 1e-13 * abs(rhs)
