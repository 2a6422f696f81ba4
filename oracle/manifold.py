"""Manifold geometry of the two constraints (Sec. 4).

The real vector u of the paper stacks (Re X_l; Im X_l) per component, so for two
wave functions a, b in the (K, *grid) layout u_a^T u_b = Re sum a conj(b), and
Gamma multiplies component l by l (definition of Gamma, Sec. 4).

* Tangent space, eq. tspace: {xi : u^T xi = 0, u^T Gamma xi = 0}.
* Projection, Lemma 4.1: P_u w = w - alpha_w u - beta_w Gamma u, with
  (alpha_w, beta_w) solving the 2x2 system of the lemma's proof (eq. TM1).
  The proof then substitutes u^T u = 1 and u^T Gamma u = M; the oracle keeps
  the measured values (identical on the manifold, and the exact orthogonal
  projection everywhere -- reading recorded in the design notes).
* Riemannian gradient, eq. grad2: grad f = P_u grad_E f.
* Riemannian Hessian, Lemma 4.2 / eq. hess-l1:
  Hess f(u)[xi] = P_u(h_e - alpha_g xi - beta_g Gamma xi), h_e = H xi.
"""

import numpy as np

from .energy import grad as egrad, hvp as ehvp


def inner(a, b):
    """u_a^T u_b = Re sum a conj(b)."""
    return float(np.real(np.vdot(b, a)))


def gamma(prob, X):
    """Gamma applied to X: component l scaled by l."""
    l = prob.lvals.astype(float).reshape((-1,) + (1,) * prob.dim)
    return X * l


def constraints(prob, u):
    """(mass, magnetization) = (u^T u, u^T Gamma u) (eq. dcon)."""
    return inner(u, u), inner(u, gamma(prob, u))


def proj_coeffs(prob, u, w):
    """(alpha_w, beta_w) of Lemma 4.1 from the system eq. TM1."""
    Gu = gamma(prob, u)
    a11 = inner(u, u)
    a12 = inner(u, Gu)
    a22 = inner(Gu, Gu)             # u^T Gamma^2 u
    r1 = inner(u, w)
    r2 = inner(Gu, w)               # u^T Gamma w
    det = a11 * a22 - a12 * a12
    if not det > 0:
        raise ValueError("degenerate Gram system: u^T Gamma^2 u <= M^2")
    alpha = (a22 * r1 - a12 * r2) / det
    beta = (a11 * r2 - a12 * r1) / det
    return alpha, beta


def project(prob, u, w):
    """P_u w (Lemma 4.1)."""
    alpha, beta = proj_coeffs(prob, u, w)
    return w - alpha * u - beta * gamma(prob, u)


def project_closed_form(prob, u, w):
    """eq. Pz0 verbatim (assumes u on the manifold: u^T u = 1, u^T Gamma u = M)."""
    M = prob.M
    Gu = gamma(prob, u)
    g2 = inner(Gu, Gu)
    uw = inner(u, w)
    uGw = inner(Gu, w)
    return w - (g2 * uw - M * uGw) / (g2 - M * M) * u + (M * uw - uGw) / (g2 - M * M) * Gu


def rgrad(prob, u, G=None):
    """Riemannian gradient P_u grad_E (eq. grad2).  Returns (grad, G, alpha_g, beta_g)."""
    if G is None:
        G = egrad(prob, u)
    ag, bg = proj_coeffs(prob, u, G)
    return G - ag * u - bg * gamma(prob, u), G, ag, bg


def rhess(prob, u, xi, ag=None, bg=None, sigma=0.0):
    """Hess f(u)[xi] + sigma xi with Hess from Lemma 4.2 (eq. hess-l1)."""
    if ag is None:
        ag, bg = proj_coeffs(prob, u, egrad(prob, u))
    he = ehvp(prob, u, xi)
    w = he - ag * xi - bg * gamma(prob, xi)
    return project(prob, u, w) + sigma * xi
