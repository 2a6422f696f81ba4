"""Retractions R_u(xi) = psi(u + xi) onto the two-constraint manifold (Sec. 6).

Every psi here scales each component: psi(w)_l = sigma_l w_l, with sigma_l fixed
by the component norms a_l = ||w_l||^2 alone.

* Projective (Sec. 6.1, projective-retraction lemma): the nearest point of the manifold.  With f1, f2 the
  lowest/highest l carrying a nonzero component, r is the unique zero of
  h1(t) = sum_{l=f1}^{f2} (l-M) a_l / [1-(l-M)t]^2 on (1/(f1-M), 1/(f2-M)),
  s = sum a_l / [1-(l-M)r]^2, and psi(w)_l = w_l / (sqrt(s) (1-(l-M)r)) for
  f1 <= l <= f2, 0 otherwise.  (This is w_l/(1-mu-l lambda) with the lemma's
  lambda = r sqrt(s), mu = 1-(1+Mr) sqrt(s).)
* Orthogonal (Sec. 6.2, orthogonal-retraction lemma): sigma_l = sqrt(r^l / sum_k a_k r^k) with r the unique
  positive zero of h2(t) = sum_{l=0}^{2F} (l-F-M) a_{l-F} t^l.  The lemma's
  denominator prints ||w_l|| inside the sum over k; the sum is over a_k (the
  proof's eq. orth-3 has it so).
* Closed form (Sec. 6.3, closed-form lemma, eq. retract3):
  sigma_l = sqrt[(w^T G^2 w - (M+l) w^T G w + M l w^T w) / (w^T w w^T G^2 w - (w^T G w)^2)].

Domains: Omega (Sec. 6, before Sec. 6.1) for the first two, S (Sec. 6.3) for
the third; outside them a ValueError is raised.
"""

import numpy as np


def comp_norms(prob, w):
    """a_l = ||w_l||^2 in storage order l = F..-F."""
    return np.array([float(np.real(np.vdot(w[i], w[i]))) for i in range(prob.K)])


def _omega_check(prob, a):
    l = prob.lvals
    M = prob.M
    if not (a[l < M].sum() > 0 and a[l > M].sum() > 0):
        raise ValueError("point outside Omega: no mass on one side of M")


def sigma_r1(prob, a):
    """Scaling factors of the projective retraction (Sec. 6.1)."""
    _omega_check(prob, a)
    l = prob.lvals.astype(float)
    M = prob.M
    nz = a > 0
    f1 = l[nz].min()
    f2 = l[nz].max()
    lo, hi = 1.0 / (f1 - M), 1.0 / (f2 - M)
    c = (l - M)[nz]
    an = a[nz]

    def h1(t):
        d = 1.0 - c * t
        return np.sum(c * an / d ** 2), np.sum(2 * c * c * an / d ** 3)  # eq. h1, eq. hderi

    t = 0.0
    for _ in range(400):
        hv, dh = h1(t)
        if hv == 0.0:
            break
        if hv > 0:
            hi = t
        else:
            lo = t
        tn = t - hv / dh
        if not (lo < tn < hi):
            tn = 0.5 * (lo + hi)
        if abs(tn - t) <= 2e-16 * max(abs(t), 1e-300) or hi - lo <= 2e-16 * max(abs(lo), abs(hi)):
            t = tn
            break
        t = tn
    r = t
    d = 1.0 - (l - M) * r
    s = np.sum(np.where(nz, a / d ** 2, 0.0))
    sig = np.where((l >= f1) & (l <= f2), 1.0 / (np.sqrt(s) * d), 0.0)
    return sig, r


def sigma_r2(prob, a):
    """Scaling factors of the orthogonal retraction (Sec. 6.2)."""
    _omega_check(prob, a)
    l = prob.lvals.astype(float)
    M = prob.M

    # h2(t) t^{-F} = sum_l (l-M) a_l t^l has the same positive zero; in s = ln t it is
    # negative for s -> -inf (f1 < M) and positive for s -> +inf (f2 > M), with
    # exactly one sign change (proof of the orthogonal-retraction lemma).  Bisection on s.
    def g(s):
        e = (l - M) * a * np.exp(l * s - np.max(l * s))
        return np.sum(e)

    lo, hi = -1.0, 1.0
    while g(lo) > 0:
        lo *= 2
    while g(hi) < 0:
        hi *= 2
    for _ in range(300):
        mid = 0.5 * (lo + hi)
        if mid == lo or mid == hi:
            break
        if g(mid) > 0:
            hi = mid
        else:
            lo = mid
    r = np.exp(0.5 * (lo + hi))
    rl = r ** l
    sig0sq = 1.0 / np.sum(a * rl)
    return np.sqrt(rl * sig0sq), r


def sigma_r3(prob, a):
    """Scaling factors of the closed-form retraction (Sec. 6.3)."""
    l = prob.lvals.astype(float)
    M = prob.M
    F = prob.F
    ww = a.sum()
    wGw = np.sum(l * a)
    wG2w = np.sum(l * l * a)
    num = lambda ll: wG2w - (M + ll) * wGw + M * ll * ww
    den = ww * wG2w - wGw ** 2
    if not (num(F) > 0 and num(-F) > 0 and den > 0):
        raise ValueError("point outside S (closed-form retraction domain)")
    return np.sqrt(num(l) / den), None


_SIG = {1: sigma_r1, 2: sigma_r2, 3: sigma_r3}


def psi(prob, w, kind=1):
    sig, _ = _SIG[kind](prob, comp_norms(prob, w))
    return w * sig.reshape((-1,) + (1,) * prob.dim)


def retract(prob, u, xi, t=1.0, kind=1):
    """R_u(t xi) = psi(u + t xi) (eq. oretr0)."""
    return psi(prob, u + t * xi, kind)


def retract_r1(prob, u, xi, t=1.0):
    return retract(prob, u, xi, t, 1)


def retract_r2(prob, u, xi, t=1.0):
    return retract(prob, u, xi, t, 2)


def retract_r3(prob, u, xi, t=1.0):
    return retract(prob, u, xi, t, 3)
