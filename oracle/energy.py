"""Discrete energy E_h, its gradient and its Hessian-vector product (Sec. 3).

All three are written in the paper's matrix form with X in C^{n x (2F+1)}
(rows = grid points, columns = components l = F..-F):

* energy, eq. discrete:energy:
    E_h(X) = 1/2 tr(X* L X) + tr(X* V X) + tr(X B X*) + beta0/(2h) rho^T rho
             + beta1/(2h) sum_a F_a^T F_a + beta2/(2h) A00* A00
             + beta3/(2h) sum_l A2l* A2l,
  rho = diag(X X*), F_a = diag(X f_a^T X*), A00 = diag(X A X^T),
  A2l = diag(X A_l X^T);
* gradient (the formula following the second-order Taylor expansion),
  for the convention E(X + D) = E(X) + Re<grad, D> + ..., <X, Y> = sum X conj(Y);
* Hessian-vector product (the formula after it).

L is the Fourier-pseudospectral negative Laplacian of eq. discrete:laplace,
per component and in d dimensions with symbol sum_alpha lambda_alpha^2.  The
paper writes L = C* Lambda C; with its C (entries e^{-i 2 pi j p/n}) that is n
times the operator of eq. discrete:laplace, so the 1/n of eq. discrete:laplace
is kept (reading recorded in the design notes).  scipy's ifftn carries exactly
that 1/n.
"""

import numpy as np
import scipy.fft as sfft

from .model import symbol
from .spin import spin_tables

FFT_WORKERS = None  # None -> scipy default (1); the CPU-baseline timing sets os.cpu_count()


def _mat(prob, X):
    """(K, *grid) array -> X in C^{n x K} (a view, rows = points)."""
    return X.reshape(prob.K, prob.npts).T


def _unmat(prob, Xm):
    return np.ascontiguousarray(Xm.T).reshape((prob.K,) + prob.shape)


def laplacian(prob, X):
    """(L X)_l = ifftn(Lambda * fftn(X_l)) for every component (eq. discrete:laplace)."""
    Lam = symbol(prob)
    axes = tuple(range(1, prob.dim + 1))
    Xh = sfft.fftn(X, axes=axes, workers=FFT_WORKERS)
    Xh *= Lam
    return sfft.ifftn(Xh, axes=axes, workers=FFT_WORKERS)


def _tables(prob):
    key = ("tables", prob.a20_variant)
    if key not in prob._cache:
        prob._cache[key] = spin_tables(prob.F, prob.a20_variant)
    return prob._cache[key]


def densities(prob, X):
    """rho, [F_x, F_y, F_z], A00, [A2l for l=-2..2] as column vectors (Sec. 3)."""
    Xm = _mat(prob, X)
    f, A, Al = _tables(prob)
    rho = (Xm * Xm.conj()).sum(1).real
    Fa = [((Xm @ fa.T) * Xm.conj()).sum(1).real for fa in f]
    A00 = ((Xm @ A) * Xm).sum(1) if A is not None else None
    A2 = [((Xm @ Am) * Xm).sum(1) for Am in Al]
    return rho, Fa, A00, A2


def energy(prob, X, LX=None):
    """E_h(X), eq. discrete:energy."""
    Xm = _mat(prob, X)
    if LX is None:
        LX = laplacian(prob, X)
    LXm = _mat(prob, LX)
    b0, b1, b2, b3 = prob.betas()
    h = prob.h
    V = prob.V.reshape(-1)
    rho, Fa, A00, A2 = densities(prob, X)
    E = 0.5 * np.real(np.sum(Xm.conj() * LXm))             # 1/2 tr(X* L X)
    E += np.sum(V[:, None] * np.abs(Xm) ** 2)               # tr(X* V X)
    E += np.sum(np.abs(Xm) ** 2 * prob.zeeman[None, :])     # tr(X B X*)
    E += b0 / (2 * h) * np.dot(rho, rho)
    E += b1 / (2 * h) * sum(np.dot(Fv, Fv) for Fv in Fa)
    if A00 is not None:
        E += b2 / (2 * h) * np.real(np.vdot(A00, A00))
    for a in A2:
        E += b3 / (2 * h) * np.real(np.vdot(a, a))
    return float(E)


def grad(prob, X, LX=None):
    """Euclidean gradient nabla E_h(X) (Sec. 3)."""
    Xm = _mat(prob, X)
    if LX is None:
        LX = laplacian(prob, X)
    G = _mat(prob, LX).copy()
    f, A, Al = _tables(prob)
    b0, b1, b2, b3 = prob.betas()
    h = prob.h
    V = prob.V.reshape(-1)
    rho, Fa, A00, A2 = densities(prob, X)
    G += 2 * V[:, None] * Xm + 2 * Xm * prob.zeeman[None, :]
    G += (2 * b0 / h) * rho[:, None] * Xm
    for fa, Fv in zip(f, Fa):
        G += (2 * b1 / h) * Fv[:, None] * (Xm @ fa.T)
    if A is not None:
        G += (2 * b2 / h) * A00[:, None] * (Xm.conj() @ A)
    for Am, a in zip(Al, A2):
        G += (2 * b3 / h) * a[:, None] * (Xm.conj() @ Am)
    return _unmat(prob, G)


def hvp(prob, X, Z, LZ=None):
    """Euclidean Hessian-vector product nabla^2 E_h(X)[Z] (Sec. 3).  R-linear in Z."""
    Xm = _mat(prob, X)
    Zm = _mat(prob, Z)
    if LZ is None:
        LZ = laplacian(prob, Z)
    H = _mat(prob, LZ).copy()
    f, A, Al = _tables(prob)
    b0, b1, b2, b3 = prob.betas()
    h = prob.h
    V = prob.V.reshape(-1)
    rho, Fa, A00, A2 = densities(prob, X)
    H += 2 * V[:, None] * Zm + 2 * Zm * prob.zeeman[None, :]
    reZX = np.real((Zm * Xm.conj()).sum(1))                     # diag(Re(Z X*))
    H += (2 * b0 / h) * (rho[:, None] * Zm + 2 * reZX[:, None] * Xm)
    for fa, Fv in zip(f, Fa):
        dF = np.real(((Zm @ fa.T) * Xm.conj()).sum(1))          # diag(Re(Z f^T X*))
        H += (2 * b1 / h) * (Fv[:, None] * (Zm @ fa.T) + 2 * dF[:, None] * (Xm @ fa.T))
    if A is not None:
        dA = ((Zm @ A) * Xm).sum(1)                              # diag(Z A X^T)
        H += (2 * b2 / h) * (A00[:, None] * (Zm.conj() @ A) + 2 * dA[:, None] * (Xm.conj() @ A))
    for Am, a in zip(Al, A2):
        dA = ((Zm @ Am) * Xm).sum(1)
        H += (2 * b3 / h) * (a[:, None] * (Zm.conj() @ Am) + 2 * dA[:, None] * (Xm.conj() @ Am))
    return _unmat(prob, H)
