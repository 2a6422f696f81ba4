"""Batched form: many spin-1 2D problems of uneven grids and parameters run
in lock step through gpe_batch_* (one launch per kernel stage for all of
them).  Parity: the batched HVP against the single-problem HVP and the
oracle's Riemannian Hessian, the batched Newton solve against the oracle's
energies (FP64: 1e-10 relative, mixed: 1e-5) and against the same problems
solved one at a time."""
import numpy as np
import pytest

import oracle
from paper_1907_01194_amd import workloads as W
from helpers import oracle_problem, rel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch
    assert torch.cuda.is_available()
    return torch


def _points(batch, specs, seed0):
    """Set points psi(X0) (C1's initial recipe) and unit tangent directions."""
    from gpu_util import dev
    pts, dirs = [], []
    for i, (p, sp) in enumerate(zip(batch.problems, specs)):
        X = p.retract(dev(W.initial_state(sp, seed0 + i)), None)
        D = p.project(X, dev(W.random_direction(sp, 100 + seed0 + i)))
        D = D / float(D.abs().pow(2).sum().sqrt())
        pts.append(X)
        dirs.append(D)
    return pts, dirs


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_batch_hvp_matches_single_and_oracle(torch, precision):
    from paper_1907_01194_amd.binding import Batch
    from gpu_util import host
    specs = W.spin1_2d_batch(count=7, seed=11, sizes=(16, 32, 64))
    print("batch hvp", precision, [s.n for s in specs], flush=True)
    b = Batch(specs, precision)
    pts, dirs = _points(b, specs, 40)
    wd = b.problems[0].work_dtype
    Z = [d.to(wd) for d in dirs]
    sig = [1e-2 * (i + 1) for i in range(len(specs))]
    for p, X in zip(b.problems, pts):
        p.set_point(X)
    for riem in (True, False):
        HB, kap = b.hvp(Z, riemannian=riem, sigma=sig)
        # without kappa: same products, no kappa finalize, no synchronisation
        HB0, k0 = b.hvp(Z, riemannian=riem, sigma=sig, kappa=False)
        torch.cuda.synchronize()
        assert k0 is None
        for i in range(len(specs)):
            assert torch.equal(HB0[i], HB[i]), (i, riem)
        for i, (p, sp) in enumerate(zip(b.problems, specs)):
            HS = p.hvp(Z[i], riemannian=riem, sigma=sig[i])
            tol_s = 1e-12 if precision == "fp64" else 2e-6
            assert rel(host(HB[i]), host(HS)) <= tol_s, (i, riem)
            op = oracle_problem(sp)
            u, z = host(pts[i]), host(Z[i])
            ref = oracle.rhess(op, u, z, sigma=sig[i]) if riem else oracle.hvp(op, u, z)
            tol_o = 1e-10 if precision == "fp64" else 1e-5
            assert rel(host(HB[i]), ref) <= tol_o, (i, riem)
            k_ref = float(np.real(np.vdot(z, ref)))
            assert abs(kap[i] - k_ref) <= tol_o * max(abs(k_ref), 1.0), (i, riem)
    b.close()


def _pick(pairs, sizes=(16, 32, 64)):
    """Problems (and their initial-state seeds) picked from seeded batches:
    pairs of (batch seed, index).  The picks are ones whose oracle solve takes
    seconds, not minutes (problems with soft modes need thousands of HVPs)."""
    specs, seeds = [], []
    for seed, i in pairs:
        specs.append(W.spin1_2d_batch(count=6, seed=seed, sizes=sizes)[i])
        seeds.append(60 + i)
    return specs, seeds


def test_batch_solve_fp64_matches_oracle_and_single(torch):
    from paper_1907_01194_amd.binding import Batch, Problem
    from gpu_util import dev
    specs, seeds = _pick([(8, 1), (8, 2), (8, 3), (8, 5), (0, 0)])
    print("batch solve fp64", [(s.n, s.beta[1], s.M) for s in specs], flush=True)
    X0 = [W.initial_state(sp, sd) for sp, sd in zip(specs, seeds)]
    # tol 1e-7: the 64^2 pick has a soft mode (small M) whose last factor of
    # ten sits at FP64 resolution, where rounding decides whether a trial lowers
    # the gradient norm (the batched and single runs round differently)
    b = Batch(specs, "fp64")
    Xs, stats = b.newton_solve([dev(x) for x in X0], tol=1e-7)
    for i, sp in enumerate(specs):
        st = stats[i]
        assert st["converged"], (i, st)
        assert st["gnorm"] <= 1e-7
        assert st["mass_err"] <= 1e-12 and st["mag_err"] <= 1e-12
        _, so = oracle.solve(oracle_problem(sp), X0[i], oracle.SolveOpts(tol=1e-7))
        assert so.converged
        assert st["gnorm"] <= max(10 * so.gnorm, 1e-7)   # the last step lands anywhere below tol
        assert abs(st["E"] - so.E) <= 1e-10 * abs(so.E), (i, st["E"], so.E)
        ps = Problem(sp, "fp64")
        _, s1 = ps.newton_solve(dev(X0[i]), tol=1e-7)
        assert abs(st["E"] - s1["E"]) <= 1e-11 * abs(s1["E"])
        ps.close()
    b.close()


def test_batch_solve_mixed_uneven_grids(torch):
    from paper_1907_01194_amd.binding import Batch
    from gpu_util import dev
    specs, seeds = _pick([(5, 1), (5, 2), (5, 3), (5, 4), (8, 3)])
    print("batch solve mixed", [(s.n, s.beta[1], s.M) for s in specs], flush=True)
    X0 = [W.initial_state(sp, sd) for sp, sd in zip(specs, seeds)]
    b = Batch(specs, "mixed")
    v, us = b.schedule()
    assert 0 <= v < 3 and us[v] > 0
    Xs, stats = b.newton_solve([dev(x) for x in X0], tol=1e-6)
    for i, sp in enumerate(specs):
        st = stats[i]
        assert st["converged"], (i, st)
        assert st["mass_err"] <= 1e-12 and st["mag_err"] <= 1e-12
        _, so = oracle.solve(oracle_problem(sp), X0[i], oracle.SolveOpts(tol=1e-6))
        assert abs(st["E"] - so.E) <= 1e-5 * abs(so.E), (i, st["E"], so.E)
    b.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_batch_cascadic_solve_matches_single(torch, precision):
    """The batch through the cascadic hierarchy (one coarser mesh per problem,
    every coarse level a lock-step batch of its own) against each problem's
    own cascadic solve: same energies, constraints exact."""
    from paper_1907_01194_amd.binding import Batch, Problem
    from gpu_util import dev
    specs = W.spin1_2d_batch(count=5, seed=8, sizes=(32, 64))
    X0 = [W.initial_state(sp, 60 + i) for i, sp in enumerate(specs)]
    print("batch cascadic", precision, [(s.n, s.beta[1], s.M) for s in specs], flush=True)
    b = Batch(specs, precision)
    _, stats = b.newton_solve([dev(x) for x in X0], tol=1e-6, mg_levels=1, time_limit=100.0)
    b.close()
    tol_e = 1e-10 if precision == "fp64" else 1e-6
    for i, sp in enumerate(specs):
        st = stats[i]
        assert st["converged"] and st["mg_levels"] == 1 and st["t_coarse"] > 0, (i, st)
        assert st["mass_err"] <= 1e-12 and st["mag_err"] <= 1e-12
        p = Problem(sp, precision)
        _, s1 = p.newton_solve(dev(X0[i]), tol=1e-6, mg_levels=1, time_limit=100.0)
        p.close()
        assert s1["converged"] and s1["mg_levels"] == 1
        assert abs(st["E"] - s1["E"]) <= tol_e * abs(s1["E"]), (i, st["E"], s1["E"])


def test_batch_cascadic_levels_limited_by_smallest_grid(torch):
    """A batch with a 32^2 problem can take one coarser level (16^2), not two."""
    from paper_1907_01194_amd.binding import Batch
    from gpu_util import dev
    specs = W.spin1_2d_batch(count=3, seed=9, sizes=(32, 64))
    specs = [sp for sp in specs] + [W.spin1_2d_batch(count=1, seed=3, sizes=(32,))[0]]
    X0 = [W.initial_state(sp, 70 + i) for i, sp in enumerate(specs)]
    print("batch cascadic levels", [s.n for s in specs], flush=True)
    b = Batch(specs, "fp64")
    _, stats = b.newton_solve([dev(x) for x in X0], check=False, tol=1e-6, mg_levels=3, time_limit=100.0)
    b.close()
    assert all(st["mg_levels"] == 1 for st in stats)


def test_batch_solve_small_cg_cap(torch):
    """Every truncated CG of the run stops at a cap of 4 iterations or earlier
    (the cap stop updates z but not p, in the closing step of the iteration
    that hit it): the batched solve still matches the same problems solved one
    at a time with the same options, and the oracle's ground-state energy."""
    from paper_1907_01194_amd.binding import Batch, Problem
    from gpu_util import dev
    specs, seeds = _pick([(8, 1), (8, 2), (8, 3)])
    print("batch solve fp64 cg cap 4", [(s.n, s.beta[1], s.M) for s in specs], flush=True)
    X0 = [W.initial_state(sp, sd) for sp, sd in zip(specs, seeds)]
    opts = dict(tol=1e-6, cg_maxit=4, cg_per_digit=0.0)
    b = Batch(specs, "fp64")
    Xs, stats = b.newton_solve([dev(x) for x in X0], **opts)
    for i, sp in enumerate(specs):
        st = stats[i]
        assert st["converged"], (i, st)
        assert st["cg_total"] <= 4 * st["outer"]
        assert st["mass_err"] <= 1e-12 and st["mag_err"] <= 1e-12
        ps = Problem(sp, "fp64")
        _, s1 = ps.newton_solve(dev(X0[i]), **opts)
        assert s1["converged"] and s1["cg_total"] <= 4 * s1["outer"]   # (counts differ: batched kernels round differently)
        assert abs(st["E"] - s1["E"]) <= 1e-11 * abs(s1["E"])
        ps.close()
        _, so = oracle.solve(oracle_problem(sp), X0[i], oracle.SolveOpts(tol=1e-6))
        assert abs(st["E"] - so.E) <= 1e-9 * abs(so.E), (i, st["E"], so.E)
    b.close()


def test_batch_rejects_unsupported(torch):
    from paper_1907_01194_amd.binding import Batch, GpeError
    specs = W.spin1_2d_batch(count=2, seed=1, sizes=(16,))
    bad = W.make_spec("odd", 1, (24, 24), (-12, -12), (12, 12), W.lattice(10.0, np.pi / 4), (100, 0.5), 0.3)
    with pytest.raises(GpeError):
        Batch(specs + [bad], "mixed")
    other = W.spin2_2d()
    with pytest.raises(GpeError):
        Batch(specs + [other], "mixed")


@pytest.mark.parametrize("F,dim,sizes", [(2, 3, (16, 32)), (3, 2, (32, 64)), (1, 1, (64, 128))])
def test_batch_hvp_other_spins_and_dims(torch, F, dim, sizes):
    """Batched HVPs (FP64, Riemannian and Euclidean) for spin-2 3D, spin-3 2D and
    spin-1 1D batches of uneven grids against the single-problem HVP."""
    from paper_1907_01194_amd.binding import Batch
    from gpu_util import host
    beta = {1: (100, -0.5), 2: (100, 1, -1), 3: (100, 1, 10, 1)}[F]
    rng = np.random.default_rng(F * 10 + dim)
    specs = []
    for i in range(5):
        n = int(sizes[i % len(sizes)])
        specs.append(W.make_spec("b%d" % i, F, (n,) * dim, (-8.0,) * dim, (8.0,) * dim, W.lattice(10.0, np.pi / 2),
                                 beta, float(rng.uniform(0.1, 0.5))))
    print("batch hvp F=%d dim=%d" % (F, dim), [s.n for s in specs], flush=True)
    b = Batch(specs, "fp64")
    pts, dirs = _points(b, specs, 300)
    for p, X in zip(b.problems, pts):
        p.set_point(X)
    sig = [0.05] * len(specs)
    for riem in (True, False):
        HB, kap = b.hvp(dirs, riemannian=riem, sigma=sig)
        HB0, _ = b.hvp(dirs, riemannian=riem, sigma=sig, kappa=False)
        torch.cuda.synchronize()
        for i, p in enumerate(b.problems):
            assert torch.equal(HB0[i], HB[i]), (i, riem)
            HS, k1 = p.hvp_dot(dirs[i], sigma=sig[i]) if riem else (p.hvp(dirs[i]), None)
            assert rel(host(HB[i]), host(HS)) <= 1e-12, (i, riem)
            if riem:
                assert abs(kap[i] - k1) <= 1e-12 * max(abs(k1), 1.0)
    b.close()
