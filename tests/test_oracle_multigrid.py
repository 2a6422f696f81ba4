"""Pins of the oracle's mesh transfer for the cascadic multigrid (Sec. 5):
Fourier interpolation keeps the coarse nodes, is exact on trigonometric
polynomials of the coarse mesh (Nyquist cosine included), and preserves the
discrete mass of data without a Nyquist component."""
import numpy as np
import pytest

from oracle.model import make_problem, mesh
from oracle.multigrid import prolong, restrict


def _probs(n, L=3.0, dim=1):
    lo, hi = (-L,) * dim, (1.7 * L,) * dim
    pc = make_problem(1, n, lo, hi, np.zeros(tuple(reversed(n))), (0, 0), 0.2)
    pf = make_problem(1, tuple(2 * m for m in n), lo, hi, np.zeros(tuple(2 * m for m in reversed(n))), (0, 0), 0.2)
    return pc, pf


@pytest.mark.parametrize("n", [(8,), (6, 10), (4, 6, 8)])
def test_prolong_keeps_coarse_nodes_and_restrict_inverts(n):
    pc, pf = _probs(n, dim=len(n))
    rng = np.random.default_rng(1)
    Xc = rng.standard_normal((3,) + pc.shape) + 1j * rng.standard_normal((3,) + pc.shape)
    Xf = prolong(pc, Xc)
    assert np.allclose(restrict(pf, Xf), Xc, atol=1e-13)


@pytest.mark.parametrize("n", [(8,), (12, 6), (6, 4, 8)])
def test_prolong_exact_on_trig_polynomials(n):
    pc, pf = _probs(n, dim=len(n))
    xc = mesh(pc)
    xf = mesh(pf)
    L = [b - a for a, b in zip(pc.lo, pc.hi)]
    a = pc.lo
    rng = np.random.default_rng(2)

    def f(xs, ps):
        v = 1.0
        for x, p, Lk, ak, m in zip(xs, ps, L, a, n):
            if abs(p) == m // 2:
                v = v * np.cos(2 * np.pi * p * (x - ak) / Lk)       # Nyquist: the cosine survives
            else:
                v = v * np.exp(2j * np.pi * p * (x - ak) / Lk)
        return v

    for _ in range(5):
        ps = [int(rng.integers(-m // 2, m // 2 + 1)) for m in n]
        Xc = np.stack([f(xc, ps)] * 3)
        Xf = prolong(pc, Xc) * 2.0 ** (len(n) / 2)
        assert np.allclose(Xf, np.stack([f(xf, ps)] * 3), atol=1e-12)


def test_prolong_preserves_mass_without_nyquist():
    pc, pf = _probs((16, 12), dim=2)
    rng = np.random.default_rng(3)
    Xc = rng.standard_normal((3,) + pc.shape) + 1j * rng.standard_normal((3,) + pc.shape)
    H = np.fft.fftn(Xc, axes=(1, 2))
    H[:, 6, :] = 0
    H[:, :, 8] = 0
    Xc = np.fft.ifftn(H, axes=(1, 2))
    Xf = prolong(pc, Xc)
    assert abs(np.vdot(Xf, Xf).real - np.vdot(Xc, Xc).real) <= 1e-12 * np.vdot(Xc, Xc).real
