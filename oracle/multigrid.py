"""Mesh transfer for the cascadic multigrid of Algorithm 1 (Sec. 5, outer loop).

The paper refines "uniformly" and says no more (reading, in the design notes):
the coarse mesh has half the points per axis on the same box, so coarse node j
coincides with fine node 2j; the fine-mesh initial guess is the Fourier
(trigonometric) interpolant of the coarse solution, which is the natural
refinement of the Fourier-pseudospectral discretisation of Sec. 3.

Interpolant of a periodic sample phi_k, k = 0..n-1 (n even), at any x:
  phi(x) = (1/n) sum_{p=-n/2}^{n/2} c_p phi~_p exp(i 2 pi p (x - a)/(b - a)),
  phi~_p = sum_k phi_k exp(-i 2 pi k p / n),  c_{+-n/2} = 1/2, c_p = 1 otherwise
(the Nyquist coefficient is split evenly between +-n/2 so that real data stay
real).  With X = sqrt(h) phi, the fine X is 2^{-d/2} times the interpolant of
the coarse X (h_fine = h_coarse / 2^d).
"""

import numpy as np


def interp_axis(a, axis):
    """Values of the trigonometric interpolant at the 2n nodes of the refined axis."""
    n = a.shape[axis]
    A = np.fft.fft(a, axis=axis)
    shape = list(a.shape)
    shape[axis] = 2 * n
    B = np.zeros(shape, dtype=complex)
    idx = [slice(None)] * a.ndim
    # p = 0 .. n/2-1
    idx[axis] = slice(0, n // 2)
    src = [slice(None)] * a.ndim
    src[axis] = slice(0, n // 2)
    B[tuple(idx)] = A[tuple(src)]
    # p = -n/2+1 .. -1
    idx[axis] = slice(2 * n - (n // 2 - 1), 2 * n)
    src[axis] = slice(n // 2 + 1, n)
    B[tuple(idx)] = A[tuple(src)]
    # Nyquist split between p = +n/2 and p = -n/2
    src[axis] = slice(n // 2, n // 2 + 1)
    idx[axis] = slice(n // 2, n // 2 + 1)
    B[tuple(idx)] = 0.5 * A[tuple(src)]
    idx[axis] = slice(2 * n - n // 2, 2 * n - n // 2 + 1)
    B[tuple(idx)] = 0.5 * A[tuple(src)]
    return np.fft.ifft(B, axis=axis) * 2          # ifft over 2n carries 1/(2n); the interpolant has 1/n


def prolong(prob_coarse, Xc):
    """Fine-mesh X (2n per axis) from the coarse X, layout (K, *grid)."""
    out = np.asarray(Xc, dtype=complex)
    for ax in range(1, out.ndim):
        out = interp_axis(out, ax)
    return out * 2.0 ** (-prob_coarse.dim / 2)


def restrict(prob_fine, Xf):
    """Coarse-mesh X by injection (coarse node j = fine node 2j), times 2^{d/2}."""
    sl = (slice(None),) + (slice(None, None, 2),) * prob_fine.dim
    return np.ascontiguousarray(np.asarray(Xf)[sl]) * 2.0 ** (prob_fine.dim / 2)
