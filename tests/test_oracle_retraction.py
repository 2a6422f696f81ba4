"""Pins of the oracle's retractions (Sec. 6)."""
import numpy as np
import pytest
from scipy.optimize import minimize

import oracle
from oracle.manifold import constraints, inner, project
from oracle.retraction import comp_norms, psi, sigma_r2
from oracle.model import make_problem
from paper_1907_01194_amd import workloads as W
from helpers import oracle_problem, small_spec, rel


def _setup(F, seed=0, n=(12, 10), M=None):
    spec = small_spec(F, n, M=M)
    prob = oracle_problem(spec)
    u = psi(prob, W.noisy_envelope_state(spec, seed, (0.3, 0.3)), 1)
    xi = project(prob, u, W.random_direction(spec, seed + 1))
    xi *= 0.3 / np.sqrt(inner(xi, xi))
    return prob, spec, u, xi


@pytest.mark.parametrize("kind", [1, 2, 3])
@pytest.mark.parametrize("F,M", [(1, 0.5), (2, 0.3), (3, 0.2), (3, 0.0), (2, 1.0)])
def test_constraints_exact(kind, F, M):
    prob, spec, u, xi = _setup(F, M=M)
    for t in (1.0, 0.1, 1e-3):
        z = oracle.retract(prob, u, xi, t, kind)
        mass, mag = constraints(prob, z)
        assert abs(mass - 1) <= 1e-12 and abs(mag - M) <= 1e-12


@pytest.mark.parametrize("kind", [1, 2, 3])
def test_zero_step_and_second_order(kind):
    prob, spec, u, xi = _setup(3, seed=2)
    assert rel(oracle.retract(prob, u, xi, 0.0, kind), u) <= 1e-14
    ts = np.array([1e-1, 3e-2, 1e-2, 3e-3])
    err = [np.sqrt(inner(d, d)) for d in (oracle.retract(prob, u, xi, t, kind) - (u + t * xi) for t in ts)]
    slope = np.polyfit(np.log(ts), np.log(err), 1)[0]
    assert 1.9 <= slope <= 2.1          # R(t xi) = u + t xi + O(t^2): DR_u(0) = id


def test_r3_approximates_r1_to_second_order():
    prob, spec, u, xi = _setup(2, seed=3)
    ts = np.array([1e-1, 3e-2, 1e-2])
    d = [rel(oracle.retract(prob, u, xi, t, 3), oracle.retract(prob, u, xi, t, 1)) for t in ts]
    slope = np.polyfit(np.log(ts), np.log(d), 1)[0]
    assert slope >= 1.9


def test_r2_coefficients_satisfy_defining_conditions():
    prob, spec, u, xi = _setup(3, seed=4)
    a = comp_norms(prob, u + xi)
    s, r = sigma_r2(prob, a)
    sig = dict(zip(prob.lvals, s))
    for l in range(1, prob.F):
        assert abs(sig[l - 1] * sig[l + 1] - sig[l] ** 2) <= 1e-13
    for l in range(1, prob.F + 1):
        assert abs(sig[l] * sig[-l] - sig[0] ** 2) <= 1e-13


@pytest.mark.parametrize("F,M,seed", [(1, 0.4, 0), (2, 0.7, 1), (3, 1.3, 2), (2, 0.0, 3)])
def test_r1_is_the_nearest_point_brute_force(F, M, seed):
    """Minimise ||z - w|| over the manifold with a generic constrained optimiser from
    many starts; the projective retraction must be at least as close, and equal."""
    n = (4,)
    prob = make_problem(F, n, (-2.0,), (2.0,), np.zeros(4), (0, 0, 0, 0), M)
    K = 2 * F + 1
    rng = np.random.default_rng(seed)
    w = rng.standard_normal((K, 4)) + 1j * rng.standard_normal((K, 4))
    w *= 0.8
    z1 = psi(prob, w, 1)
    lv = prob.lvals.repeat(8)
    wv = np.concatenate([np.r_[c.real, c.imag] for c in w])
    cons = [{"type": "eq", "fun": lambda v: v @ v - 1},
            {"type": "eq", "fun": lambda v: v @ (lv * v) - M}]
    best = np.inf
    for k in range(12):
        v0 = rng.standard_normal(wv.size)
        r = minimize(lambda v: 0.5 * np.sum((v - wv) ** 2), v0, jac=lambda v: v - wv,
                     constraints=cons, method="SLSQP", options={"ftol": 1e-14, "maxiter": 500})
        if r.success and abs(r.x @ r.x - 1) < 1e-9 and abs(r.x @ (lv * r.x) - M) < 1e-9:
            best = min(best, np.linalg.norm(r.x - wv))
    d1 = np.linalg.norm(z1 - w)
    assert np.isfinite(best)
    assert d1 <= best + 1e-9
    assert abs(d1 - best) <= 1e-6
    # and no random feasible point is closer
    for k in range(200):
        v = psi(prob, rng.standard_normal((K, 4)) + 1j * rng.standard_normal((K, 4)), 1)
        assert np.linalg.norm(v - w) >= d1 - 1e-12


def _spin1_prob(M):
    return make_problem(1, (6,), (-1.0,), (1.0,), np.zeros(6), (0, 0), M)


def test_r1_spin1_closed_form_case1():
    """Spin-1 closed form, case (1): M = 0."""
    prob = _spin1_prob(0.0)
    rng = np.random.default_rng(0)
    w = rng.standard_normal((3, 6)) + 1j * rng.standard_normal((3, 6))
    nw = np.sqrt(comp_norms(prob, w))
    t = np.sqrt(nw[1] ** 2 + (nw[0] + nw[2]) ** 2 / 2)
    ref = np.stack([(nw[0] + nw[2]) / (2 * t * nw[0]) * w[0], w[1] / t,
                    (nw[0] + nw[2]) / (2 * t * nw[2]) * w[2]])
    assert rel(psi(prob, w, 1), ref) <= 1e-13


def test_r1_spin1_closed_form_case2():
    """Spin-1 closed form, case (2): M > 0, w_0 = 0."""
    M = 0.35
    prob = _spin1_prob(M)
    rng = np.random.default_rng(1)
    w = rng.standard_normal((3, 6)) + 1j * rng.standard_normal((3, 6))
    w[1] = 0
    nw = np.sqrt(comp_norms(prob, w))
    ref = np.stack([np.sqrt(1 + M) / (np.sqrt(2) * nw[0]) * w[0], 0 * w[1],
                    np.sqrt(1 - M) / (np.sqrt(2) * nw[2]) * w[2]])
    assert rel(psi(prob, w, 1), ref) <= 1e-13


def test_r1_spin1_closed_form_case3():
    """Spin-1 closed form, case (3): M > 0, w_{-1} = 0."""
    M = 0.6
    prob = _spin1_prob(M)
    rng = np.random.default_rng(2)
    w = rng.standard_normal((3, 6)) + 1j * rng.standard_normal((3, 6))
    w[2] = 0
    nw = np.sqrt(comp_norms(prob, w))
    ref = np.stack([np.sqrt(M) / nw[0] * w[0], np.sqrt(1 - M) / nw[1] * w[1], 0 * w[2]])
    assert rel(psi(prob, w, 1), ref) <= 1e-13


def test_domain_errors():
    prob = _spin1_prob(0.5)
    w = np.zeros((3, 6), complex)
    w[2] = 1.0                       # all mass below M: outside Omega
    for kind in (1, 2, 3):
        with pytest.raises(ValueError):
            psi(prob, w, kind)
