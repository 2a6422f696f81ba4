"""Pins of the oracle's projection, Riemannian gradient and Hessian (Sec. 4)."""
import numpy as np
import pytest

import oracle
from oracle.manifold import gamma, inner, project, project_closed_form
from paper_1907_01194_amd import workloads as W
from helpers import oracle_problem, small_spec, rel


def _setup(F, seed=0, n=(12, 10)):
    spec = small_spec(F, n)
    prob = oracle_problem(spec)
    u = oracle.retraction.psi(prob, W.noisy_envelope_state(spec, seed, (0.3, 0.3)), 1)
    w = W.random_direction(spec, seed + 1)
    return prob, spec, u, w


@pytest.mark.parametrize("F", [1, 2, 3])
def test_projection_tangent_idempotent_orthogonal(F):
    prob, spec, u, w = _setup(F)
    Pw = project(prob, u, w)
    s = np.sqrt(inner(w, w))
    assert abs(inner(u, Pw)) <= 1e-13 * s
    assert abs(inner(gamma(prob, u), Pw)) <= 1e-13 * s
    assert rel(project(prob, u, Pw), Pw) <= 1e-13
    # w - Pw lies in span{u, Gamma u}: orthogonal to any tangent vector
    t = project(prob, u, W.random_direction(spec, 99))
    assert abs(inner(w - Pw, t)) <= 1e-13 * s * np.sqrt(inner(t, t))


@pytest.mark.parametrize("F", [1, 2, 3])
def test_projection_matches_lemma_closed_form(F):
    prob, spec, u, w = _setup(F, seed=4)
    assert rel(project(prob, u, w), project_closed_form(prob, u, w)) <= 1e-12


@pytest.mark.parametrize("F", [1, 2, 3])
def test_hessian_matches_lemma_explicit_formula(F):
    """eq. Hess0 (the explicit expansion) against P_u(h_e - a_g xi - b_g Gamma xi)."""
    prob, spec, u, w = _setup(F, seed=6)
    xi = project(prob, u, w)
    G = oracle.grad(prob, u)
    M = prob.M
    Gu = gamma(prob, u)
    au = inner(Gu, Gu) - M * M
    ag = (1 + M * M / au) * inner(u, G) - M / au * inner(Gu, G)
    bg = -M / au * inner(u, G) + 1 / au * inner(Gu, G)
    he = oracle.hvp(prob, u, xi)
    bu = inner(Gu, he) - bg * inner(Gu, gamma(prob, xi))
    g2 = inner(Gu, Gu)
    ref = (he - ag * xi - bg * gamma(prob, xi) - (g2 * inner(u, he) - M * bu) / au * u
           + (M * inner(u, he) - bu) / au * Gu)
    assert rel(oracle.rhess(prob, u, xi), ref) <= 1e-12


@pytest.mark.parametrize("F", [2, 3])
def test_rhess_symmetric_on_tangent_space(F):
    prob, spec, u, w = _setup(F, seed=8)
    a = project(prob, u, w)
    b = project(prob, u, W.random_direction(spec, 123))
    x = inner(oracle.rhess(prob, u, a, sigma=0.3), b)
    y = inner(a, oracle.rhess(prob, u, b, sigma=0.3))
    assert abs(x - y) <= 1e-11 * max(abs(x), 1)


def test_rgrad_matches_directional_derivative_along_curve():
    """<grad f(u), xi> = d/dt E(R_u(t xi)) at t = 0 for tangent xi."""
    prob, spec, u, w = _setup(2, seed=10)
    xi = project(prob, u, w) * 1e-1
    g = oracle.rgrad(prob, u)[0]
    eps = 1e-6
    fd = (oracle.energy(prob, oracle.retract(prob, u, xi, eps)) -
          oracle.energy(prob, oracle.retract(prob, u, xi, -eps))) / (2 * eps)
    assert abs(fd - inner(g, xi)) <= 1e-6 * max(abs(fd), 1e-3)


def test_rhess_matches_second_derivative_along_projective_curve():
    """For the projective retraction (second order), d^2/dt^2 E(R_u(t xi)) = <Hess[xi], xi>."""
    prob, spec, u, w = _setup(3, seed=12)
    xi = project(prob, u, w) * 3e-2
    eps = 1e-4
    E = lambda t: oracle.energy(prob, oracle.retract(prob, u, xi, t, 1))
    fd = (E(eps) - 2 * E(0.0) + E(-eps)) / eps ** 2
    exact = inner(oracle.rhess(prob, u, xi), xi)
    assert abs(fd - exact) <= 1e-4 * abs(exact)
