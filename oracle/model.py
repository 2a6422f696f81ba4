"""Problem description and the Fourier-pseudospectral grid (Sec. 3).

Grid (Sec. 3, first paragraph, extended to tensor grids as the paper says it
extends): on each axis alpha the box is [a_alpha, b_alpha), the mesh size is
h_alpha = (b_alpha - a_alpha)/n_alpha with n_alpha even, and the nodes are
x_j = a_alpha + j h_alpha, j = 0..n_alpha-1.  The unknown is the sqrt(h)-scaled
matrix X = (sqrt(h) phi_jl) with h = prod_alpha h_alpha.

Wavenumbers (eq. discrete:fourier): lambda_p = 2 pi p / (b - a) for
p = -n/2 .. n/2-1; Nyquist p = -n/2 is kept.  In d dimensions the symbol of the
discrete negative Laplacian is Lambda = sum_alpha lambda_alpha^2.

Array layout shared with the tests: a wave function is a complex128 array of
shape (K, n_z, n_y, n_x) (trailing axes dropped in 1D/2D), component index 0
holding l = F; x is the last (fastest) axis.
"""

from dataclasses import dataclass, field
import numpy as np


@dataclass
class Problem:
    F: int
    n: tuple            # (n_x[, n_y[, n_z]])
    lo: tuple           # (a_x, ...)
    hi: tuple           # (b_x, ...)
    V: np.ndarray       # potential on the grid, shape = reversed(n)
    beta: tuple         # (beta0, beta1[, beta2[, beta3]])
    M: float
    p: float = 0.0
    q: float = 0.0
    a20_variant: str = "paper"
    _cache: dict = field(default_factory=dict, repr=False)

    @property
    def dim(self):
        return len(self.n)

    @property
    def K(self):
        return 2 * self.F + 1

    @property
    def shape(self):
        return tuple(reversed(self.n))

    @property
    def h_axes(self):
        return tuple((b - a) / m for a, b, m in zip(self.lo, self.hi, self.n))

    @property
    def h(self):
        return float(np.prod(self.h_axes))

    @property
    def npts(self):
        return int(np.prod(self.n))

    @property
    def lvals(self):
        """Magnetic quantum numbers in storage order: F, F-1, ..., -F."""
        return np.arange(self.F, -self.F - 1, -1)

    @property
    def zeeman(self):
        """b_l = -p l + q l^2 (Sec. 3, definition of B)."""
        l = self.lvals.astype(float)
        return -self.p * l + self.q * l * l

    def betas(self):
        b = list(self.beta) + [0.0] * (4 - len(self.beta))
        return b[:4]


def axis_nodes(a, b, n):
    """x_j = a + j h, j = 0..n-1 (Sec. 3)."""
    h = (b - a) / n
    return a + h * np.arange(n)


def lambda2_axis(a, b, n):
    """lambda_p^2 in numpy FFT order: index k holds p = k (k < n/2) or k - n."""
    k = np.arange(n)
    p = np.where(k < n // 2, k, k - n)
    lam = 2 * np.pi * p / (b - a)
    return lam * lam


def mesh(prob):
    """Coordinate arrays (x, y, z) each broadcast to prob.shape."""
    axes = [axis_nodes(a, b, m) for a, b, m in zip(prob.lo, prob.hi, prob.n)]
    grids = np.meshgrid(*reversed(axes), indexing="ij")  # arrays ordered (z, y, x)
    return list(reversed(grids))  # x, y, z


def symbol(prob):
    """Lambda = sum_alpha lambda_alpha^2 on the FFT grid, shape prob.shape."""
    if "Lambda" not in prob._cache:
        lam = [lambda2_axis(a, b, m) for a, b, m in zip(prob.lo, prob.hi, prob.n)]
        grids = np.meshgrid(*reversed(lam), indexing="ij")
        prob._cache["Lambda"] = sum(grids)
    return prob._cache["Lambda"]


def make_problem(F, n, lo, hi, potential, beta, M, p=0.0, q=0.0, a20_variant="paper"):
    """Build a Problem; ``potential`` is a callable V(x[, y[, z]]) evaluated on the
    nodes x_j = a + j h, or an array of the grid's shape."""
    n = tuple(int(v) for v in n)
    for m in n:
        if m % 2:
            raise ValueError("n must be even (Sec. 3)")
    prob = Problem(F=F, n=n, lo=tuple(float(v) for v in lo), hi=tuple(float(v) for v in hi),
                   V=None, beta=tuple(beta), M=float(M), p=p, q=q, a20_variant=a20_variant)
    if callable(potential):
        prob.V = np.asarray(potential(*mesh(prob)), dtype=float)
    else:
        prob.V = np.asarray(potential, dtype=float).reshape(prob.shape)
    return prob
