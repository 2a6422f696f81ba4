"""Ground states of Sec. 7.2 (Table 3-1, spin-2) and Sec. 7.3 (Table 4-1,
spin-3) on the GPU, every printed row: the paper's potentials, boxes, grids,
interaction strengths and initial data (Sec. 7), ||grad|| <= 1e-6.

* Table 3-1 prints 10-digit energies for 1D, 2D and 3D (commented-out
  versions of the table): matched to 1e-8.
* Table 4-1 prints 4 decimals: matched to +-5e-5.
* Readings, each pinned here:
  - cyclic spin-2 at M = 0 (Table 3-1, 1D and 2D): beta1, beta2 > 0 bound every
    state's energy below by the scalar GPE with the same beta0, and the cyclic
    spinor attains that bound, below the printed value: the printed entry is
    not the minimum of the stated problem;
  - Table 3-1 3D Case I: the printed energy is that of [-8,8]^3 with n = 128
    (mesh 1/8 on every axis); the printed box [-8,8]x[-16,16]^2 with n = 2^7
    would have mesh 1/4 on two axes and a larger energy;
  - Table 4-1 3D, Case I at M = 0 and Case II at M = 1.5: a converged state with
    exact constraints lies below the printed energy (by 8e-5 and 1.4e-4), so
    the printed state is not the minimum; the test asks for at most the printed
    energy (+5e-5) and no more than 5e-4 below it.  Case II at M = 1.5 (also
    Table 1-3-3's last row) is the state the cascadic hierarchy of Algorithm 1
    reaches from two coarser meshes (32^3, 64^3): that solve gives the printed
    energy.
The 3D cases run in mixed precision (c64 Hessian products; energies,
gradients and retractions in FP64)."""
import os

import numpy as np
import pytest

from paper_1907_01194_amd import workloads as W

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))


def lattice(amp, k):
    return lambda *xs: 0.5 * sum(x * x for x in xs) + amp * sum(np.sin(k * x) ** 2 for x in xs)


def golden(name):
    rows = []
    for line in open(os.path.join(HERE, "golden", name)):
        r = line.split()
        if r and not r[0].startswith("#"):
            rows.append(r)
    return rows


SPIN2_PHASE = {"I": "ferro", "II": "nematic", "III": "cyclic"}


@pytest.fixture(scope="module")
def torch():
    import torch
    assert torch.cuda.is_available()
    return torch


def solve(torch, spec, U, prec="fp64", limit=200.0, mg=0):
    from paper_1907_01194_amd.binding import Problem
    X0 = W.paper_initial(spec, U)
    gp = Problem(spec, prec)
    X, st = gp.newton_solve(torch.from_numpy(X0).cuda(), check=False, tol=1e-6, time_limit=limit, mg_levels=mg)
    gp.close()
    del X
    torch.cuda.empty_cache()
    return st


def check_converged(st):
    assert st["converged"] and st["gnorm"] <= 1e-6
    assert st["mass_err"] <= 1e-12 and st["mag_err"] <= 1e-12


def scalar_bound(torch, spec, U):
    """Ground-state energy of the same problem with beta1 = beta2 = beta3 = 0."""
    s = W.make_spec(spec.name + "-scalar", spec.F, spec.n, spec.lo, spec.hi, lambda *xs: spec.V,
                    (spec.beta[0], 0.0, 0.0, 0.0), spec.M)
    st = solve(torch, s, U)
    check_converged(st)
    return st["E"]


T31_1D = [r for r in golden("table3_1_spin2_1d.txt")]


@pytest.mark.parametrize("row", T31_1D, ids=lambda r: "%s-M%s" % (r[0], r[7]))
def test_table3_1_1d(torch, row):
    case, b0, b1, b2, a, b, n, M, E = row
    M, E = float(M), float(E)
    print("table 3-1 1D", case, M, flush=True)
    spec = W.make_spec("t31-1d", 2, (int(n),), (float(a),), (float(b),), lattice(25, np.pi / 4),
                       (float(b0), float(b1), float(b2)), M)
    U = W.paper_U(2, SPIN2_PHASE[case], M)
    st = solve(torch, spec, U)
    check_converged(st)
    if case == "III" and M == 0.0:
        Eb = scalar_bound(torch, spec, U)
        assert abs(st["E"] - Eb) <= 1e-9 * Eb and st["E"] < E - 1.0
    else:
        assert abs(st["E"] - E) <= 1e-8


T31 = golden("table3_1_spin2_2d3d.txt")


@pytest.mark.parametrize("row", [r for r in T31 if r[0] == "2"], ids=lambda r: "%s-M%s" % (r[1], r[5]))
def test_table3_1_2d(torch, row):
    _, case, b0, b1, b2, M, E = row
    M, E = float(M), float(E)
    print("table 3-1 2D", case, M, flush=True)
    spec = W.make_spec("t31-2d", 2, (256, 256), (-8, -8), (8, 8), lattice(10, np.pi / 2),
                       (float(b0), float(b1), float(b2)), M)
    U = W.paper_U(2, SPIN2_PHASE[case], M)
    st = solve(torch, spec, U)
    check_converged(st)
    if case == "III" and M == 0.0:
        Eb = scalar_bound(torch, spec, U)
        assert abs(st["E"] - Eb) <= 1e-9 * Eb and st["E"] < E - 0.1
    else:
        assert abs(st["E"] - E) <= 1e-8


@pytest.mark.parametrize("row", [r for r in T31 if r[0] == "3" and (r[1] == "II" or (r[1] == "I" and r[5] != "0.5"))],
                         ids=lambda r: "%s-M%s" % (r[1], r[5]))
def test_table3_1_3d(torch, row):
    """Case I on [-8,8]^3 with n = 128 (see the module notes); Case II on
    [-16,16]^3 with n = 256.  Case III is Table 1-2-3 (test_gpu_paper_tables)."""
    _, case, b0, b1, b2, M, E = row
    M, E = float(M), float(E)
    print("table 3-1 3D", case, M, flush=True)
    L, n = (8, 128) if case == "I" else (16, 256)
    spec = W.make_spec("t31-3d", 2, (n,) * 3, (-L,) * 3, (L,) * 3, lattice(100, np.pi / 2),
                       (float(b0), float(b1), float(b2)), M)
    st = solve(torch, spec, W.paper_U(2, SPIN2_PHASE[case], M), "mixed")
    check_converged(st)
    assert abs(st["E"] - E) <= 1e-8


def test_table3_1_3d_case1_printed_box_is_coarser(torch):
    """The printed box of Table 3-1's 3D Case I with n = 2^7 gives a mesh of 1/4
    on two axes and an energy well above the printed one; keeping the mesh 1/8
    on those axes (n = 256 there) recovers it."""
    b = (130.6, -25.4, -125.3)
    U = W.paper_U(2, "ferro", 0.0)
    V = lattice(100, np.pi / 2)
    coarse = W.make_spec("t31-3d-I-box", 2, (128, 128, 128), (-8, -16, -16), (8, 16, 16), V, b, 0.0)
    fine = W.make_spec("t31-3d-I-box-fine", 2, (128, 256, 256), (-8, -16, -16), (8, 16, 16), V, b, 0.0)
    Ec, Ef = solve(torch, coarse, U, "mixed")["E"], solve(torch, fine, U, "mixed")["E"]
    assert Ec - 39.0044828481 > 0.03
    assert abs(Ef - 39.0044828481) <= 1e-8


T41_1D = golden("table4_1_spin3_1d.txt")
T41_2D = golden("table4_1_spin3_2d.txt")
T41_3D = golden("table4_1_spin3_3d.txt")


@pytest.mark.parametrize("row", T41_1D, ids=lambda r: "%s-M%s" % (r[0], r[5]))
def test_table4_1_1d(torch, row):
    case, b0, b1, b2, b3, M, E = row
    M, E = float(M), float(E)
    print("table 4-1 1D", case, M, flush=True)
    spec = W.make_spec("t41-1d", 3, (256,), (-8,), (8,), lattice(25, np.pi / 4),
                       tuple(float(v) for v in (b0, b1, b2, b3)), M)
    st = solve(torch, spec, W.paper_U(3, None, M, 0))
    check_converged(st)
    assert abs(st["E"] - E) <= 5e-5


@pytest.mark.parametrize("row", [r for r in T41_2D if r[0] == "I"], ids=lambda r: "%s-M%s" % (r[0], r[5]))
def test_table4_1_2d(torch, row):
    """Case I (Case II is Table 1-3-2, test_gpu_paper_tables)."""
    case, b0, b1, b2, b3, M, E = row
    M, E = float(M), float(E)
    print("table 4-1 2D", case, M, flush=True)
    spec = W.make_spec("t41-2d", 3, (256, 256), (-8, -8), (8, 8), lattice(10, np.pi / 2),
                       tuple(float(v) for v in (b0, b1, b2, b3)), M)
    st = solve(torch, spec, W.paper_U(3, None, M, 0))
    check_converged(st)
    assert abs(st["E"] - E) <= 5e-5


@pytest.mark.parametrize("row", [r for r in T41_3D if r[5] != "0.5"], ids=lambda r: "%s-M%s" % (r[0], r[5]))
def test_table4_1_3d(torch, row):
    """M = 0 and 1.5 for both cases (M = 0.5: test_gpu_solve)."""
    case, b0, b1, b2, b3, M, E = row
    M, E = float(M), float(E)
    print("table 4-1 3D", case, M, flush=True)
    spec = W.make_spec("t41-3d", 3, (128,) * 3, (-8,) * 3, (8,) * 3, lattice(100, np.pi / 2),
                       tuple(float(v) for v in (b0, b1, b2, b3)), M)
    st = solve(torch, spec, W.paper_U(3, None, M, 0), "mixed", limit=240.0)
    check_converged(st)
    if (case, M) in (("I", 0.0), ("II", 1.5)):
        assert -5e-4 <= st["E"] - E <= 5e-5        # below the printed value (module notes)
    else:
        assert abs(st["E"] - E) <= 5e-5


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_table4_1_3d_case2_m15_cascadic(torch, prec):
    """Case II at M = 1.5 through the cascadic hierarchy (Algorithm 1, two
    coarser meshes): the printed 43.0399, which the one-mesh solve passes below."""
    print("table 4-1 3D II M=1.5 cascadic", prec, flush=True)
    spec = W.make_spec("t41-3d", 3, (128,) * 3, (-8,) * 3, (8,) * 3, lattice(100, np.pi / 2), (100, 1, 10, 1), 1.5)
    st = solve(torch, spec, W.paper_U(3, None, 1.5, 0), prec, limit=120.0, mg=2)
    check_converged(st)
    assert st["mg_levels"] == 2
    assert abs(st["E"] - 43.0399) <= 5e-5
