"""Spin matrices and pair-amplitude matrices, entered as the paper prints them.

Component order everywhere is l = F, F-1, ..., -F (row/column 0 is l = F).

* Spin-1: f_x, f_y, f_z (Sec. 2, eq. spin1m).
* Spin-2: f_x, f_y, f_z = diag(2..-2) and the singlet matrix A (Sec. 2, spin-2
  paragraph, the 5x5 matrices and eq. A:spin2).
* Spin-3: f_x, f_y, f_z = diag(3..-3), the singlet matrix A, the quintet matrix
  A_0, and A_{+-1}, A_{+-2} given through the vectors a_{+-1}, a_{+-2} whose
  entries sit on the anti-diagonals j + k = 8 - l (1-based indices; Sec. 2,
  spin-3 paragraph).

Reading (recorded in the design notes): the spin-3 matrices as printed govern
the energy, gradient and Hessian of Sec. 3.  The printed A_0 centre entry
sqrt(2/3)/sqrt(7) gives a psi_0^2 coefficient sqrt(2)/sqrt(21) in A_20 (the
printed explicit A_20 agrees); a Clebsch-Gordan normalised amplitude would
have 2/sqrt(21).  ``a20_variant="cg"`` switches that single entry to
(2/sqrt(3))/sqrt(7) so that the paper's Table 4-1 energies can decide between
the two.  The printed explicit A_{2,+-2} has sqrt(2) psi_{+-1}^2 where the
printed vector a_{+-2} gives sqrt(6); the matrix (vector) form is used.
"""

import numpy as np

SQ = np.sqrt


def _spin1():
    # eq. spin1m
    fx = (1 / SQ(2)) * np.array([[0, 1, 0], [1, 0, 1], [0, 1, 0]], dtype=complex)
    fy = (1j / SQ(2)) * np.array([[0, -1, 0], [1, 0, -1], [0, 1, 0]], dtype=complex)
    fz = np.diag([1, 0, -1]).astype(complex)
    return [fx, fy, fz], None, []


def _spin2():
    r = SQ(3 / 2)
    fx = np.array([[0, 1, 0, 0, 0],
                   [1, 0, r, 0, 0],
                   [0, r, 0, r, 0],
                   [0, 0, r, 0, 1],
                   [0, 0, 0, 1, 0]], dtype=complex)
    fy = 1j * np.array([[0, -1, 0, 0, 0],
                        [1, 0, -r, 0, 0],
                        [0, r, 0, -r, 0],
                        [0, 0, r, 0, -1],
                        [0, 0, 0, 1, 0]], dtype=complex)
    fz = np.diag([2, 1, 0, -1, -2]).astype(complex)
    A = (1 / SQ(5)) * np.array([[0, 0, 0, 0, 1],
                                [0, 0, 0, -1, 0],
                                [0, 0, 1, 0, 0],
                                [0, -1, 0, 0, 0],
                                [1, 0, 0, 0, 0]], dtype=complex)
    return [fx, fy, fz], A, []


def _antidiag_matrix(l, vec):
    """A_l = (a_{l,jk}) with nonzeros only where j + k = 8 - l (1-based).

    For l = 1, 2 the vector lists a_{l,1(7-l)}, a_{l,2(6-l)}, ..., a_{l,(7-l)1};
    for l = -1, -2 it lists a_{l,(1-l)7}, a_{l,(2-l)6}, ..., a_{l,7(1-l)}.
    """
    M = np.zeros((7, 7), dtype=complex)
    s = 8 - l
    if l > 0:
        rows = range(1, 7 - l + 1)
    else:
        rows = range(1 - l, 7 + 1)
    rows = list(rows)
    assert len(rows) == len(vec)
    for v, j in zip(vec, rows):
        k = s - j
        M[j - 1, k - 1] = v
    return M


def _spin3(a20_variant="paper"):
    fx = np.zeros((7, 7))
    off = [SQ(3 / 2), SQ(5 / 2), SQ(3), SQ(3), SQ(5 / 2), SQ(3 / 2)]
    for i, v in enumerate(off):
        fx[i, i + 1] = v
        fx[i + 1, i] = v
    fy = np.zeros((7, 7))
    for i, v in enumerate(off):
        fy[i, i + 1] = -v
        fy[i + 1, i] = v
    fx = fx.astype(complex)
    fy = 1j * fy.astype(complex)
    fz = np.diag([3, 2, 1, 0, -1, -2, -3]).astype(complex)

    A = np.zeros((7, 7), dtype=complex)
    for j in range(7):
        A[j, 6 - j] = (-1) ** j
    A /= SQ(7)

    A0 = np.zeros((7, 7), dtype=complex)
    A0[0, 6] = A0[6, 0] = 5 / (2 * SQ(3))
    A0[2, 4] = A0[4, 2] = -SQ(3) / 2
    if a20_variant == "paper":
        A0[3, 3] = SQ(2 / 3)
    elif a20_variant == "cg":
        A0[3, 3] = 2 / SQ(3)
    else:
        raise ValueError("a20_variant must be 'paper' or 'cg'")
    A0 /= SQ(7)

    a1 = np.array([5 / (2 * SQ(3)), -SQ(5) / 2, 1 / SQ(6), 1 / SQ(6), -SQ(5) / 2,
                   5 / (2 * SQ(3))]) / SQ(7)
    a2 = np.array([SQ(5 / 6), -SQ(5 / 3), SQ(2), -SQ(5 / 3), SQ(5 / 6)]) / SQ(7)
    Al = {0: A0,
          1: _antidiag_matrix(1, a1), -1: _antidiag_matrix(-1, a1),
          2: _antidiag_matrix(2, a2), -2: _antidiag_matrix(-2, a2)}
    # order l = -2..2 as in the sum over A_{2l}
    return [fx, fy, fz], A, [Al[l] for l in (-2, -1, 0, 1, 2)]


def spin_tables(F, a20_variant="paper"):
    """Return (f, A, Alist): f = [f_x, f_y, f_z]; A the singlet matrix (None for
    F = 1); Alist the quintet matrices A_l, l = -2..2 (empty unless F = 3)."""
    if F == 1:
        return _spin1()
    if F == 2:
        return _spin2()
    if F == 3:
        return _spin3(a20_variant)
    raise ValueError("F must be 1, 2 or 3")
