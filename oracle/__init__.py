"""FP64 CPU oracle for the spin-F BEC ground-state hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library, its
Python binding) may import, call or link this package; only the tests, the
smoke check and the CPU-baseline leg of the benchmark do.  It shares no code
with the GPU path: it keeps its own spin tables, grid, Laplacian, energy,
gradient, Hessian-vector product, manifold projection, retractions and
solver, all written from the paper (Tian, Cai, Wu, Wen, "Ground states and
their characterization of spin-F Bose-Einstein condensates") in complex128 /
float64 with NumPy and scipy.fft.

Each function cites the passage of the paper it follows.  Everything here is
the plain definition: the matrix forms of Sec. 3 (with dense spin matrices),
the projection and Hessian lemmas of Sec. 4, the projective, orthogonal
and closed-form retractions of Sec. 6, Algorithm 1 of Sec. 5 and its mesh
transfer (multigrid.py).  No blocking, fusion or reordering
beyond what those definitions state.

Parity status of each part is listed in ``PINS``; a part without a pin to
something other than itself says "parity unpinned".
"""

from .model import Problem, make_problem
from .spin import spin_tables
from .energy import laplacian, energy, grad, hvp, densities
from .manifold import inner, proj_coeffs, project, rgrad, rhess, constraints
from .retraction import retract_r1, retract_r2, retract_r3, retract
from .solver import SolveOpts, solve, rgbb, arnt, tcg

PINS = {
    "laplacian": "naive DFT of the discrete Laplace formula; plane-wave eigenpairs",
    "energy/grad": "harmonic closed form (E = sum(gamma)/2); finite differences",
    "zeeman term": "closed form on the manifold with beta = 0: E* = d/2 - p M + q M (q >= 0), "
                   "d/2 - p M + q F^2 (q < 0), reached by the solver",
    "hvp": "finite differences; phase/spin-rotation/homogeneity identities; symmetry",
    "projection/rgrad/rhess": "tangency, idempotence, Lemma 4.1 closed form",
    "retractions": "constraints exact; R(0)=u; second order; R1 = brute-force nearest point; "
                   "spin-1 closed-form cases 1-3 (Sec. 6.1)",
    "solver": "paper Table 3-1 / Table 4-1 printed ground-state energies (1D); Zeeman closed form",
    "multigrid transfer": "coarse nodes kept; exact on trigonometric polynomials; mass preserved",
}

__all__ = [
    "Problem", "make_problem", "spin_tables", "laplacian", "energy", "grad", "hvp",
    "densities", "inner", "proj_coeffs", "project", "rgrad", "rhess", "constraints",
    "retract_r1", "retract_r2", "retract_r3", "retract", "SolveOpts", "solve", "rgbb",
    "arnt", "tcg", "PINS",
]
