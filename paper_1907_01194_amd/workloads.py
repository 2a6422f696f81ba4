"""Problem specifications and seeded synthetic inputs.

This module holds no arithmetic of the method (no Laplacian, energy,
projection or retraction): it only samples potentials and initial data on the
grid nodes x_j = a + j h (j = 0..n-1, h = (b - a)/n) and draws seeded random
numbers.  Both the GPU path and the CPU oracle consume exactly the arrays it
returns.

Array layout: a wave function is complex128 with shape (K, n_z, n_y, n_x)
(trailing spatial axes dropped in 1D/2D), component 0 holding l = F; the
potential has shape (n_z, n_y, n_x).
"""

from dataclasses import dataclass
import numpy as np


@dataclass
class Spec:
    """One problem: spin F, grid n = (n_x[, n_y[, n_z]]) on [lo, hi) per axis,
    potential V on the grid, interaction strengths beta = (beta0..beta3),
    magnetization M and Zeeman shifts p, q."""
    name: str
    F: int
    n: tuple
    lo: tuple
    hi: tuple
    V: np.ndarray
    beta: tuple
    M: float
    p: float = 0.0
    q: float = 0.0

    @property
    def K(self):
        return 2 * self.F + 1

    @property
    def dim(self):
        return len(self.n)

    @property
    def shape(self):
        return tuple(reversed(self.n))

    @property
    def field_shape(self):
        return (self.K,) + self.shape

    @property
    def h(self):
        return float(np.prod([(b - a) / m for a, b, m in zip(self.lo, self.hi, self.n)]))


def coords(n, lo, hi):
    """Node coordinates (x, y, z) broadcast to the grid shape (z, y, x)."""
    axes = [a + (b - a) / m * np.arange(m) for a, b, m in zip(lo, hi, n)]
    g = np.meshgrid(*reversed(axes), indexing="ij")
    return list(reversed(g))


def harmonic(gam):
    """V = 1/2 sum gamma_a^2 x_a^2 (trap frequencies gamma_a)."""
    def V(*xs):
        return 0.5 * sum((g * x) ** 2 for g, x in zip(gam, xs))
    return V


def lattice(amp, k):
    """V = 1/2 |x|^2 + amp * sum sin^2(k x_a)."""
    def V(*xs):
        return 0.5 * sum(x * x for x in xs) + amp * sum(np.sin(k * x) ** 2 for x in xs)
    return V


def make_spec(name, F, n, lo, hi, potential, beta, M, p=0.0, q=0.0):
    n = tuple(int(v) for v in n)
    lo = tuple(float(v) for v in lo)
    hi = tuple(float(v) for v in hi)
    V = np.ascontiguousarray(potential(*coords(n, lo, hi)), dtype=np.float64)
    beta = tuple(float(b) for b in beta) + (0.0,) * (4 - len(beta))
    return Spec(name, F, n, lo, hi, V, beta, float(M), float(p), float(q))


# ---------------------------------------------------------------- workloads

def spin1_1d():
    """Spin-1, 1D, 128 points on [-16,16], V = x^2/2, beta = (100, -0.5), M = 0.5."""
    return make_spec("spin1-1d-128", 1, (128,), (-16,), (16,), harmonic((1.0,)), (100, -0.5), 0.5)


def spin2_2d():
    """Spin-2, 2D, 256^2 on [-12,12]^2, V = |x|^2/2 + 10 sum sin^2(pi x_a/4),
    beta = (100, 1, -1), M = 0.3."""
    return make_spec("spin2-2d-256", 2, (256, 256), (-12, -12), (12, 12),
                     lattice(10.0, np.pi / 4), (100, 1, -1), 0.3)


def spin3_3d(n=128):
    """Spin-3, 3D, n^3 on [-8,8]^3, V = 1/2 (x^2 + y^2 + 4 z^2) (trap gamma = (1,1,2)),
    beta = (500, 5, -5, 2), M = 0.2."""
    return make_spec("spin3-3d-%d" % n, 3, (n, n, n), (-8, -8, -8), (8, 8, 8),
                     harmonic((1.0, 1.0, 2.0)), (500, 5, -5, 2), 0.2)


def spin3_3d_paper(n=128, case="II", M=0.5):
    """The paper's spin-3 3D workload (Sec. 7.3, Tables 1-3-3 and 4-1): [-8,8]^3,
    V = |x|^2/2 + 100 sum sin^2(pi x_a/2), Case I beta = (100, 1, -10, -1),
    Case II beta = (100, 1, 10, 1)."""
    beta = {"I": (100, 1, -10, -1), "II": (100, 1, 10, 1)}[case]
    return make_spec("spin3-3d-%d-paper-case%s-M%g" % (n, case, M), 3, (n, n, n), (-8, -8, -8), (8, 8, 8),
                     lattice(100.0, np.pi / 2), beta, M)


def spin2_3d(n=96):
    """Spin-2, 3D, n^3 on [-12,12]^3, V = |x|^2/2, beta = (100, 1, -1), M = 0.3."""
    return make_spec("spin2-3d-%d" % n, 2, (n, n, n), (-12, -12, -12), (12, 12, 12),
                     harmonic((1.0, 1.0, 1.0)), (100, 1, -1), 0.3)


def spin1_2d_batch(count=64, seed=5, sizes=(64, 128, 256)):
    """Batched workload: `count` spin-1 2D problems, n x n with n drawn from
    `sizes`, on spin2_2d's box and potential ([-12,12]^2, |x|^2/2 + 10 sum
    sin^2(pi x_a/4)), beta = (100, beta1) with beta1 ~ U[-1, 1] and M ~
    U[0, 0.9] (seeded)."""
    rng = np.random.default_rng(seed)
    specs = []
    for i in range(count):
        n = int(rng.choice(np.asarray(sizes)))
        b1 = float(rng.uniform(-1.0, 1.0))
        M = float(rng.uniform(0.0, 0.9))
        specs.append(make_spec("spin1-2d-%d-b%d" % (n, i), 1, (n, n), (-12, -12), (12, 12),
                               lattice(10.0, np.pi / 4), (100, b1), M))
    return specs


def _lat(amp, k, half=False):
    """V = 1/2 |x|^2 + amp sum sin^2(k x_a) (half: the lattice term also halved)."""
    a = 0.5 * amp if half else amp
    def V(*xs):
        return 0.5 * sum(x * x for x in xs) + a * sum(np.sin(k * x) ** 2 for x in xs)
    return V


# The performance workloads of Sec. 7.1 (Tables 1-1-2 .. 1-3-3): spin F, grid
# points per axis, half-width of the box, potential, interaction strengths, the
# Sec. 7 initial spinor's phase, and the magnetizations with the ARNT energies
# the tables print.  The spin-1 2D case is printed with the lattice term
# 10 sum sin^2(pi x_a / 4), but its table's energies are those of
# 10 sum sin^2(pi x_a / 2) (the lattice of the spin-2 and spin-3 2D cases): the
# oracle gives 15.14106 at M = 0.2 with the latter (table: 15.1411) and 14.77136
# with the former.  The table is taken to be right.
PAPER_TABLES = {
    "1-1-2": dict(F=1, dim=2, n=512, L=16, V=_lat(10.0, np.pi / 2), beta=(300, 100), phase="antiferro",
                  E={0.0: 15.1032, 0.2: 15.1411, 0.5: 15.3436, 0.9: 15.9621}),
    "1-1-3": dict(F=1, dim=3, n=256, L=16, V=_lat(200.0, np.pi / 2, half=True), beta=(880, -4.1), phase="ferro",
                  E={0.0: 55.4362, 0.2: 55.4362, 0.5: 55.4362, 0.9: 55.4362}),
    "1-2-2": dict(F=2, dim=2, n=256, L=8, V=_lat(10.0, np.pi / 2), beta=(243, 12.1, -13), phase="nematic",
                  E={0.0: 14.3386, 0.5: 14.3730, 1.5: 14.6754}),
    "1-2-3": dict(F=2, dim=3, n=256, L=16, V=_lat(100.0, np.pi / 2), beta=(183.9, 26.8, 134.7), phase="cyclic",
                  E={0.0: 46.2917, 0.5: 45.7403, 1.5: 46.8619}),
    "1-3-2": dict(F=3, dim=2, n=256, L=8, V=_lat(10.0, np.pi / 2), beta=(100, 1, 10, 1), phase=None,
                  E={0.0: 11.8279, 0.5: 11.8334, 1.5: 11.8780}),
    "1-3-3": dict(F=3, dim=3, n=128, L=8, V=_lat(100.0, np.pi / 2), beta=(100, 1, 10, 1), phase=None,
                  E={0.0: 42.9752, 0.5: 42.9822, 1.5: 43.0399}),
}


def paper_table_case(table, M, n=None, seed=0):
    """(spec, X0) of one row of a Sec. 7.1 table: the Sec. 7 initial data U phi0
    (U of the table's phase; seeded uniform in R^7 for spin-3).  n overrides the
    grid points per axis (a smaller mesh of the same problem)."""
    t = PAPER_TABLES[table]
    m = n or t["n"]
    spec = make_spec("table%s-M%g-n%d" % (table, M, m), t["F"], (m,) * t["dim"], (-t["L"],) * t["dim"],
                     (t["L"],) * t["dim"], t["V"], t["beta"], M)
    return spec, paper_initial(spec, paper_U(t["F"], t["phase"], M, seed))


# ---------------------------------------------------------------- inputs

def cn(rng, shape):
    """iid standard complex normal, E|z|^2 = 1."""
    return (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) / np.sqrt(2.0)


def gaussian_phase_state(spec, seed):
    """phi_l = exp(-|x|^2/2) exp(i theta_l), theta_l ~ U[0, 2 pi) per component."""
    rng = np.random.default_rng(seed)
    xs = coords(spec.n, spec.lo, spec.hi)
    env = np.exp(-0.5 * sum(x * x for x in xs))
    th = rng.uniform(0, 2 * np.pi, spec.K)
    return np.ascontiguousarray(np.exp(1j * th).reshape((-1,) + (1,) * spec.dim) * env[None])


def noisy_envelope_state(spec, seed, widths=None):
    """iid CN(0,1) per point and component times exp(-sum w_a x_a^2 / 2)."""
    rng = np.random.default_rng(seed)
    xs = coords(spec.n, spec.lo, spec.hi)
    widths = widths or (1.0,) * spec.dim
    env = np.exp(-0.5 * sum(w * x * x for w, x in zip(widths, xs)))
    return np.ascontiguousarray(cn(rng, spec.field_shape) * env[None])


def random_direction(spec, seed):
    """iid CN(0,1) field (not normalised, not tangent)."""
    return np.ascontiguousarray(cn(np.random.default_rng(seed), spec.field_shape))


def initial_state(spec, seed):
    """The seeded initial state of each workload (before it is mapped onto the manifold)."""
    if spec.dim == 1:
        return gaussian_phase_state(spec, seed)
    if spec.F == 3 and spec.dim == 3:
        return noisy_envelope_state(spec, seed, (1.0, 1.0, 2.0))
    return noisy_envelope_state(spec, seed)


def paper_initial(spec, U):
    """Phi_0 = U phi_0 with phi_0 = pi^{-d/4} exp(-|x|^2/2), returned as the
    sqrt(h)-scaled X (Sec. 7, initial data)."""
    xs = coords(spec.n, spec.lo, spec.hi)
    phi0 = np.pi ** (-spec.dim / 4) * np.exp(-0.5 * sum(x * x for x in xs))
    U = np.asarray(U, dtype=float).reshape((-1,) + (1,) * spec.dim)
    return np.ascontiguousarray((U * phi0[None] * np.sqrt(spec.h)).astype(np.complex128))


def paper_U(F, phase, M, seed=0):
    """Initial spinor U of Sec. 7 for the given phase."""
    s = np.sqrt
    if F == 1:
        if phase == "ferro":
            return [s(1 + 3 * M) / 2, s((1 - M) / 2), s(1 - M) / 2]
        return [s((1 + M) / 2), 0.0, s((1 - M) / 2)]
    if F == 2:
        if phase == "ferro":
            m1, m2 = s(2 + M), s(2 - M)
            return [m1 ** 4 / 16, m1 ** 3 * m2 / 8, s(6) * m1 ** 2 * m2 ** 2 / 16,
                    m1 * m2 ** 3 / 8, m2 ** 4 / 16]
        if phase == "nematic":
            return [s(2 + M) / 2, 0, 0, 0, s(2 - M) / 2]
        if phase == "cyclic":
            return [s((M + 1) / 3), 0, 0, s((2 - M) / 3), 0]
    if F == 3:
        return list(np.random.default_rng(seed).random(7))
    raise ValueError("unknown phase")
