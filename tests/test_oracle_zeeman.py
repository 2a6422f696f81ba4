"""Pin of the oracle's Zeeman term b_l = -p l + q l^2 (Sec. 2 energy, Sec. 3
definition of B) by a closed form on the manifold.

With beta = 0 and V = |x|^2/2 every component sees the same harmonic
oscillator, so on {sum ||X_l||^2 = 1, sum l ||X_l||^2 = M} the energy of the
state X_l = sqrt(m_l) X_0 (X_0 the oscillator ground state, unit mass) is

    E = d/2 + sum_l b_l m_l = d/2 - p M + q sum_l l^2 m_l,

and its minimum over the component masses m_l >= 0 is a linear programme:
the term in p is fixed by the magnetization; for q >= 0 and 0 < M < 1 the
convexity of l^2 puts the mass on l = 0 and l = 1 (sum l^2 m_l = M), for q < 0
on l = +-F (sum l^2 m_l = F^2).  So

    q >= 0:  E* = d/2 - p M + q M,       q < 0:  E* = d/2 - p M + q F^2.

A sign slip in p or q, the component order (storage index i holds l = F - i)
or a dropped factor changes these values.  The oracle's energy at the
two-component minimiser, its Riemannian gradient there (zero: Lemma 4.1's
multipliers fit any two components), and its solver started from a random
state must all reach them.
"""
import numpy as np
import pytest

import oracle
from oracle.model import make_problem, mesh


def ground_mix(prob, masses):
    """sqrt(h) sqrt(m_l) phi_0 with phi_0 = pi^(-d/4) exp(-|x|^2/2)."""
    xs = mesh(prob)
    phi = np.ones(prob.shape)
    for x in xs:
        phi = phi * np.pi ** -0.25 * np.exp(-x * x / 2)
    m = np.asarray(masses, float).reshape((-1,) + (1,) * prob.dim)
    return (np.sqrt(m) * phi[None] * np.sqrt(prob.h)).astype(complex)


def closed_form(F, d, p, q, M):
    return d / 2 - p * M + (q * M if q >= 0 else q * F * F)


def minimiser_masses(F, q, M):
    K = 2 * F + 1
    m = np.zeros(K)
    if q >= 0:
        m[F - 1] = M          # l = 1
        m[F] = 1.0 - M        # l = 0
    else:
        m[0] = 0.5 * (1 + M / F)     # l = F
        m[K - 1] = 0.5 * (1 - M / F)  # l = -F
    return m


CASES = [(F, p, q) for F in (1, 2, 3) for p, q in ((0.3, 0.7), (-0.4, 0.25), (0.5, -0.3), (-0.2, -0.6))]


def _problem(F, n, L, p, q, M):
    dim = len(n)
    V = lambda *xs: 0.5 * sum(x * x for x in xs)
    return make_problem(F, n, (-L,) * dim, (L,) * dim, V, (0, 0, 0, 0), M, p=p, q=q)


@pytest.mark.parametrize("F,p,q", CASES)
@pytest.mark.parametrize("n", [(64,), (48, 48)])
def test_zeeman_closed_form_energy(F, p, q, n):
    M = 0.35
    prob = _problem(F, n, 10.0, p, q, M)
    X = ground_mix(prob, minimiser_masses(F, q, M))
    mass, mag = oracle.constraints(prob, X)
    assert abs(mass - 1) <= 1e-12 and abs(mag - M) <= 1e-12
    E = oracle.energy(prob, X)
    assert abs(E - closed_form(F, len(n), p, q, M)) <= 1e-12
    g = oracle.rgrad(prob, X)[0]
    assert np.sqrt(oracle.inner(g, g)) <= 1e-12
    # any other feasible two-level split costs more (strict convexity in l^2 / linearity)
    K = 2 * F + 1
    other = np.zeros(K)
    if q >= 0:
        # mass on l = -1 and l = +1 with the same magnetization: sum l^2 m = 1 > M
        other[F - 1] = 0.5 * (1 + M)
        other[F + 1] = 0.5 * (1 - M)
    else:
        other[F - 1] = M
        other[F] = 1 - M
    E_other = oracle.energy(prob, ground_mix(prob, other))
    assert E_other > E + 1e-3 * abs(q)


@pytest.mark.slow
@pytest.mark.parametrize("F,p,q", [(1, 0.3, 0.7), (2, -0.4, 0.25), (3, 0.5, -0.3), (2, 0.2, -0.6)])
def test_zeeman_solver_reaches_closed_form(F, p, q):
    """Algorithm 1 from a random spinor finds the linear programme's minimum."""
    M = 0.35
    prob = _problem(F, (64,), 10.0, p, q, M)
    rng = np.random.default_rng(7 + F)
    xs = mesh(prob)
    X0 = (rng.standard_normal((2 * F + 1, 1)) + 1j * rng.standard_normal((2 * F + 1, 1))) * np.exp(-xs[0] ** 2 / 2)
    u, st = oracle.solve(prob, X0, oracle.SolveOpts(tol=1e-9))
    assert st.converged
    assert abs(st.E - closed_form(F, 1, p, q, M)) <= 1e-10
