"""Parity of the HIP library (through the C ABI) with the FP64 oracle.

Per call: energy (Sec. 3), Euclidean and Riemannian gradient (Sec. 3, Sec. 4),
Euclidean and Riemannian Hessian-vector products (Sec. 3, Lemma 4.2) and the
three retractions (Sec. 6), on seeded inputs, for F = 1, 2, 3 in 1D/2D/3D on
grids that span several workgroups with ragged tails, plus the full-size
spin-3 128^3 workload.  Tolerances: FP64 1e-10 relative on energies (the
stated bar) and 1e-11 relative 2-norm on fields; mixed (c64) HVPs 1e-5.
"""
import numpy as np
import pytest

import oracle
from paper_1907_01194_amd import workloads as W
from helpers import oracle_problem, small_spec

pytestmark = pytest.mark.gpu

CASES = [
    (1, (4,)), (1, (24,)), (1, (128,)), (1, (512,)),
    (2, (12, 16)), (2, (96, 6)), (2, (64, 48)),
    (3, (8, 12, 16)), (3, (16, 6, 4)), (3, (24, 32, 12)),
    (2, (192, 4, 4)), (1, (384, 6, 4)),
]


def ids(c):
    return "F%d-%s" % (c[0], "x".join(map(str, c[1])))


@pytest.fixture(scope="module")
def torch():
    import torch
    assert torch.cuda.is_available()
    return torch


def setup_case(F, n, seed=0, precision="fp64", p=0.0, q=0.0):
    from paper_1907_01194_amd.binding import Problem
    spec = small_spec(F, n, p=p, q=q)
    prob = oracle_problem(spec)
    w = W.noisy_envelope_state(spec, seed, (0.2,) * len(n))
    u = oracle.retraction.psi(prob, w, 1)
    return spec, prob, u, Problem(spec, precision)


@pytest.mark.parametrize("case", CASES, ids=ids)
def test_energy_grad_parity(torch, case):
    from gpu_util import dev, host, relnorm
    F, n = case
    print("energy/grad parity", case, flush=True)
    spec, prob, u, gp = setup_case(F, n, p=0.1, q=0.05)
    X = dev(u)
    E = gp.energy(X)
    E_or = oracle.energy(prob, u)
    assert abs(E - E_or) <= 1e-10 * abs(E_or)
    G, E2, gn = gp.grad(X, riemannian=False)
    assert relnorm(host(G), oracle.grad(prob, u)) <= 1e-11
    assert abs(gn - np.linalg.norm(oracle.grad(prob, u))) <= 1e-11 * gn
    gR, E3, gnR = gp.grad(X, riemannian=True)
    g_or = oracle.rgrad(prob, u)[0]
    assert relnorm(host(gR), g_or) <= 1e-11
    assert abs(gnR - np.sqrt(oracle.inner(g_or, g_or))) <= 1e-11 * gnR
    assert abs(E2 - E_or) <= 1e-10 * abs(E_or) and abs(E3 - E_or) <= 1e-10 * abs(E_or)


@pytest.mark.parametrize("case", CASES, ids=ids)
def test_hvp_parity(torch, case):
    from gpu_util import dev, host, relnorm
    F, n = case
    print("hvp parity", case, flush=True)
    spec, prob, u, gp = setup_case(F, n, seed=1, p=-0.2, q=0.1)
    Z = W.random_direction(spec, 11) * 1e-2
    gp.set_point(dev(u))
    H = gp.hvp(dev(Z), riemannian=False)
    assert relnorm(host(H), oracle.hvp(prob, u, Z)) <= 1e-11
    xi = oracle.project(prob, u, Z)
    sigma = 0.3
    HR = gp.hvp(dev(xi), riemannian=True, sigma=sigma)
    HR_or = oracle.rhess(prob, u, xi, sigma=sigma)
    assert relnorm(host(HR), HR_or) <= 1e-11
    HR2, kappa = gp.hvp_dot(dev(xi), sigma)
    k_or = oracle.inner(xi, HR_or)
    assert abs(kappa - k_or) <= 1e-10 * abs(k_or) + 1e-13


@pytest.mark.parametrize("case", [(1, (24,)), (2, (12, 16)), (3, (8, 12, 16)), (3, (24, 32, 12))], ids=ids)
def test_hvp_mixed_precision(torch, case):
    from gpu_util import dev, host, relnorm
    F, n = case
    print("hvp mixed", case, flush=True)
    spec, prob, u, gp = setup_case(F, n, seed=2, precision="mixed")
    xi = oracle.project(prob, u, W.random_direction(spec, 12))
    gp.set_point(dev(u))
    H = gp.hvp(dev(xi, torch.complex64), riemannian=False)
    assert relnorm(host(H), oracle.hvp(prob, u, xi)) <= 1e-5
    HR = gp.hvp(dev(xi, torch.complex64), riemannian=True, sigma=0.1)
    assert relnorm(host(HR), oracle.rhess(prob, u, xi, sigma=0.1)) <= 1e-5


@pytest.mark.parametrize("kind", [1, 2, 3])
@pytest.mark.parametrize("case", [(1, (24,)), (2, (12, 16)), (3, (8, 12, 16))], ids=ids)
def test_retraction_parity(torch, case, kind):
    from gpu_util import dev, host, relnorm
    F, n = case
    print("retract", case, kind, flush=True)
    spec, prob, u, gp = setup_case(F, n, seed=3)
    xi = oracle.project(prob, u, W.random_direction(spec, 13))
    xi *= 0.2 / np.sqrt(oracle.inner(xi, xi))
    for t in (1.0, 0.3, 0.0):
        Z = gp.retract(dev(u), dev(xi), t, kind)
        ref = oracle.retract(prob, u, xi, t, kind)
        assert relnorm(host(Z), ref) <= 1e-12
        mass, mag = gp.constraints(Z)
        assert abs(mass - 1) <= 1e-12 and abs(mag - spec.M) <= 1e-12


def test_retraction_domain_error(torch):
    from paper_1907_01194_amd.binding import GpeError
    from gpu_util import dev
    spec, prob, u, gp = setup_case(1, (16,), seed=4)
    w = np.zeros_like(u)
    w[2] = u[2]                       # all mass on l = -1 < M: outside Omega
    with pytest.raises(GpeError) as e:
        gp.retract(dev(w), None, 0.0, 1)
    assert e.value.status == 2


def test_hvp_requires_set_point(torch):
    from paper_1907_01194_amd.binding import GpeError
    spec, prob, u, gp = setup_case(2, (8, 8), seed=5)
    with pytest.raises(GpeError) as e:
        gp.hvp(gp.empty(work=True))
    assert e.value.status == 1


def test_full_size_spin3_128(torch):
    """spin-3 128^3 workload (the benchmark's configuration): energy, Riemannian
    gradient and Riemannian HVP against the oracle, FP64 and mixed."""
    from paper_1907_01194_amd.binding import Problem
    from gpu_util import dev, host, relnorm
    print("full size spin-3 128^3", flush=True)
    spec = W.spin3_3d(128)
    prob = oracle_problem(spec)
    u = oracle.retraction.psi(prob, W.initial_state(spec, 3), 1)
    xi = oracle.project(prob, u, W.random_direction(spec, 103))
    xi /= np.sqrt(oracle.inner(xi, xi))
    g_or, G_or, ag, bg = oracle.rgrad(prob, u)
    E_or = oracle.energy(prob, u)
    H_or = oracle.rhess(prob, u, xi, ag, bg, 1e-2)
    for prec, tol in (("fp64", 1e-11), ("mixed", 1e-5)):
        gp = Problem(spec, prec)
        X = dev(u)
        assert abs(gp.energy(X) - E_or) <= 1e-10 * abs(E_or)
        gR, E, gn = gp.grad(X, riemannian=True)
        assert relnorm(host(gR), g_or) <= 1e-11
        gp.set_point(X)
        Z = dev(xi, gp.work_dtype)
        HR = gp.hvp(Z, riemannian=True, sigma=1e-2)
        assert relnorm(host(HR), H_or) <= tol, prec
        del gp
        torch.cuda.empty_cache()
