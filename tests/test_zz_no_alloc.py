"""The no-allocation entry point gpe_retract_noalloc (static device scratch)
against gpe_retract on a handle: two calls in a row, the second on a smaller
problem, every retraction; results identical (the same kernels run)."""
import numpy as np
import pytest

import oracle
from paper_1907_01194_amd import workloads as W
from helpers import oracle_problem, small_spec

pytestmark = pytest.mark.gpu


def _case(F, n, seed):
    spec = small_spec(F, n)
    prob = oracle_problem(spec)
    u = oracle.retraction.psi(prob, W.noisy_envelope_state(spec, seed, (0.2,) * len(n)), 1)
    xi = oracle.project(prob, u, W.random_direction(spec, seed + 1))
    xi *= 0.3 / np.sqrt(oracle.inner(xi, xi))
    return spec, u, xi


@pytest.mark.parametrize("kind", [1, 2, 3])
def test_retract_noalloc_matches_retract(kind):
    import torch
    from paper_1907_01194_amd.binding import Problem, retract_noalloc
    from gpu_util import dev
    print("retract_noalloc kind", kind, flush=True)
    # large first (many workgroups fill the scratch), then a smaller problem
    for F, n, seed, t in ((3, (48, 32, 24), 40, 0.7), (1, (24,), 41, 0.4)):
        spec, u, xi = _case(F, n, seed)
        gp = Problem(spec, "fp64")
        X, Xi = dev(u), dev(xi)
        ref = gp.retract(X, Xi, t, kind)
        got = retract_noalloc(spec, X, Xi, t, kind)
        torch.cuda.synchronize()
        assert torch.equal(got, ref), (F, n, kind)
        got0 = retract_noalloc(spec, X, None, 0.0, kind)
        assert torch.equal(got0, gp.retract(X, None, 0.0, kind))
        mass, mag = gp.constraints(got)
        assert abs(mass - 1) <= 1e-12 and abs(mag - spec.M) <= 1e-12
        gp.close()


def test_retract_noalloc_errors():
    from paper_1907_01194_amd.binding import GpeError, retract_noalloc
    from gpu_util import dev
    spec, u, xi = _case(1, (16,), 50)
    w = np.zeros_like(u)
    w[2] = u[2]                       # all mass on l = -1 < M: outside Omega
    with pytest.raises(GpeError) as e:
        retract_noalloc(spec, dev(w), None, 0.0, 1)
    assert e.value.status == 2
    with pytest.raises(GpeError) as e:
        retract_noalloc(spec, dev(u), None, 0.0, 9)
    assert e.value.status == 1
    # the scratch is reused correctly after the failed calls
    from paper_1907_01194_amd.binding import Problem
    got = retract_noalloc(spec, dev(u), dev(xi), 0.5, 1)
    ref = Problem(spec, "fp64").retract(dev(u), dev(xi), 0.5, 1)
    import torch
    assert torch.equal(got, ref)
