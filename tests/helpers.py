"""Test-side glue: build oracle problems from the shared workload specs."""
import numpy as np

import oracle
from paper_1907_01194_amd import workloads as W


def oracle_problem(spec, a20_variant="paper"):
    return oracle.make_problem(spec.F, spec.n, spec.lo, spec.hi, spec.V, spec.beta, spec.M,
                               spec.p, spec.q, a20_variant=a20_variant)


def small_spec(F, n, dim_box=None, beta=None, M=None, potential=None, p=0.0, q=0.0):
    """A small problem on a box of half-width 8 (or dim_box) with a harmonic-plus-lattice V."""
    dim = len(n)
    L = dim_box or 8.0
    beta = beta or {1: (100, -0.5), 2: (100, 1, -1), 3: (500, 5, -5, 2)}[F]
    M = {1: 0.5, 2: 0.3, 3: 0.2}[F] if M is None else M
    potential = potential or W.lattice(10.0, np.pi / 4)
    return W.make_spec("small", F, n, (-L,) * dim, (L,) * dim, potential, beta, M, p, q)


def rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(np.asarray(b).ravel()), 1e-300))
