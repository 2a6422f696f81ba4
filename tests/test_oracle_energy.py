"""Pins of the oracle's E_h, grad E_h and Hessian-vector product (Sec. 3).

* Closed form: with beta = 0 and V = 1/2 sum gamma_a^2 x_a^2 the harmonic ground
  state gives E = sum(gamma_a)/2, grad E = (sum gamma_a) X and a zero Riemannian
  gradient, for any spinor U of unit mass (spectrally exact on these boxes).
* Exact identities of the energy's invariances: global phase, spin rotation
  about z, and degree-2/degree-4 homogeneity; symmetry of the Hessian.
* Central finite differences of E and of grad E.
"""
import numpy as np
import pytest

import oracle
from oracle.model import make_problem, mesh
from paper_1907_01194_amd import workloads as W
from helpers import oracle_problem, small_spec, rel


def harmonic_state(prob, gam, U):
    xs = mesh(prob)
    phi = np.ones(prob.shape)
    for g, x in zip(gam, xs):
        phi = phi * (g / np.pi) ** 0.25 * np.exp(-g * x * x / 2)
    U = np.asarray(U, float).reshape((-1,) + (1,) * prob.dim)
    return (U * phi[None] * np.sqrt(prob.h)).astype(complex)


@pytest.mark.parametrize("F,n,L,gam,M", [
    (1, (128,), 16.0, (1.0,), 0.5),
    (2, (48, 48), 8.0, (1.0, 1.5), 0.3),
    (3, (48, 48, 64), 8.0, (1.0, 1.0, 2.0), 0.2),
])
def test_harmonic_closed_form(F, n, L, gam, M):
    dim = len(n)
    V = lambda *xs: 0.5 * sum((g * x) ** 2 for g, x in zip(gam, xs))
    prob = make_problem(F, n, (-L,) * dim, (L,) * dim, V, (0, 0, 0, 0), M)
    K = 2 * F + 1
    rng = np.random.default_rng(F)
    U = rng.random(K)
    l = prob.lvals
    # fix mass 1 and magnetization M by scaling the top and bottom components
    U = U / np.sqrt(np.sum(U ** 2))
    X = harmonic_state(prob, gam, U)
    X = oracle.retraction.psi(prob, X, 1)      # only rescales components
    E = oracle.energy(prob, X)
    assert abs(E - sum(gam) / 2) <= 1e-12
    G = oracle.grad(prob, X)
    assert rel(G, sum(gam) * X) <= 1e-12
    g = oracle.rgrad(prob, X)[0]
    assert np.sqrt(oracle.inner(g, g)) <= 1e-12


def _point(F, n=(16, 12), seed=0, p=0.0, q=0.0):
    spec = small_spec(F, n, p=p, q=q)
    prob = oracle_problem(spec)
    X = W.noisy_envelope_state(spec, seed, (0.3,) * len(n))
    X = oracle.retraction.psi(prob, X, 1)
    Z = W.random_direction(spec, seed + 100) * 1e-2
    return prob, X, Z


def _E2grad(prob, X):
    """Gradient of the quadratic part: L X + 2 V X + 2 X B."""
    l = prob.zeeman.reshape((-1,) + (1,) * prob.dim)
    return oracle.laplacian(prob, X) + 2 * prob.V[None] * X + 2 * l * X


@pytest.mark.parametrize("F", [1, 2, 3])
def test_hvp_invariance_identities(F):
    prob, X, Z = _point(F, p=0.3, q=0.7)
    G = oracle.grad(prob, X)
    nG = np.linalg.norm(G)
    # global phase: H[iX] = i grad E
    assert np.linalg.norm(oracle.hvp(prob, X, 1j * X) - 1j * G) <= 1e-12 * nG
    # spin rotation about z: H[i Gamma X] = i Gamma grad E
    GX = oracle.manifold.gamma(prob, X)
    assert np.linalg.norm(oracle.hvp(prob, X, 1j * GX) - 1j * oracle.manifold.gamma(prob, G)) <= 1e-12 * nG
    # homogeneity: H[X] = 3 grad E - 2 grad E_2
    E2g = _E2grad(prob, X)
    assert np.linalg.norm(oracle.hvp(prob, X, X) - (3 * G - 2 * E2g)) <= 1e-12 * nG
    # Euler: Re<grad E, X> = 2 E_2 + 4 E_4
    E = oracle.energy(prob, X)
    E2 = 0.5 * oracle.inner(E2g, X)
    E4 = E - E2
    assert abs(oracle.inner(G, X) - (2 * E2 + 4 * E4)) <= 1e-12 * abs(E)


@pytest.mark.parametrize("F", [1, 2, 3])
def test_hvp_symmetric(F):
    prob, X, Z = _point(F, seed=3)
    Z2 = W.random_direction(small_spec(F, (16, 12)), 77)
    a = oracle.inner(oracle.hvp(prob, X, Z), Z2)
    b = oracle.inner(Z, oracle.hvp(prob, X, Z2))
    assert abs(a - b) <= 1e-12 * max(abs(a), 1.0)


@pytest.mark.parametrize("F", [1, 2, 3])
def test_finite_differences(F):
    prob, X, Z = _point(F, seed=5, p=0.2, q=-0.1)
    eps = 1e-6
    d_fd = (oracle.energy(prob, X + eps * Z) - oracle.energy(prob, X - eps * Z)) / (2 * eps)
    d = oracle.inner(oracle.grad(prob, X), Z)
    assert abs(d_fd - d) <= 1e-7 * max(abs(d), 1e-3)
    H_fd = (oracle.grad(prob, X + eps * Z) - oracle.grad(prob, X - eps * Z)) / (2 * eps)
    assert rel(oracle.hvp(prob, X, Z), H_fd) <= 1e-7


def test_hvp_is_real_linear_not_complex_linear():
    prob, X, Z = _point(3, seed=9)
    H1 = oracle.hvp(prob, X, 1j * Z)
    H2 = 1j * oracle.hvp(prob, X, Z)
    assert rel(H1, H2) > 1e-3          # the conj(Z) terms break C-linearity
    assert rel(oracle.hvp(prob, X, 2.5 * Z), 2.5 * oracle.hvp(prob, X, Z)) <= 1e-14
