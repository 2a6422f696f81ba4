"""Algorithm 1 on one mesh: RGBB warm start, then the modified ARNT (Sec. 5).

RGBB (Sec. 5, eq. NMN and the text around it): steepest descent on the
manifold with the Barzilai-Borwein step gamma_k = |<s,v>| / <v,v>, a
nonmonotone Armijo test against C_k with the Zhang-Hager update
C_{k+1} = (varrho Q_k C_k + E_{k+1}) / Q_{k+1}, Q_{k+1} = varrho Q_k + 1.

ARNT (Sec. 5, eq. prob-sub .. eq. ratio, Algorithm 1): at u_k the model
m_k(u) = <g, u-u_k> + 1/2 <H (u-u_k), u-u_k> + sigma_k/2 ||u-u_k||^2
(g, H the Euclidean gradient and Hessian) is reduced by a truncated CG on
grad m_k + Hess m_k[xi] = 0 that stops on accuracy or on negative curvature and
returns s_k, d_k; the direction is xi_k = s_k + tau_k d_k (eq. xi); a monotone
Armijo curvilinear search on m_k along R_{u_k}(alpha0 delta^j xi_k)
(eq. tp1, tp2) gives the trial point z_k; the ratio rho_k of eq. ratio decides
acceptance and the update of sigma (Algorithm 1); sigma_k = sigma_hat_k ||grad||
with sigma_hat_0 = 1 and the sigma_est reset of Sec. 7.1.

Parameters the paper leaves open are taken as follows (readings, listed in the
design notes): the truncated CG itself is not printed (it is the one of the
cited ARNT paper); it is plain CG from 0 with stopping rule
||r|| <= min(T, ||g||^theta) ||g||, T = 0.1, theta = 1, and stops on curvature
kappa = <p, A p> <= 1e-12 max(1, ||g||) ||p||^2, returning s = z (or -g at the
first iteration), d = p when kappa < 0, sigma_est = |kappa| / ||p||^2.
alpha0 = 1, rho = 1e-4, delta = 0.2, at most 30 backtracks.  sigma_hat is
multiplied by gamma0 = 0.2 when rho_k >= eta2, by gamma1 = 1 when
eta1 <= rho_k < eta2, by gamma2 = 10 on rejection.  RGBB: rho = 1e-4,
delta = 0.2, varrho = 0.85, first step 0.1/||grad||, BB step clamped to
[1e-20, 1e20].  The inner iterations of a subproblem are capped, as Sec. 7.1
says, by a rule in ||grad||: 80 iterations per decimal digit the CG residual
must gain, ceil(80 log10(1 / min(T, ||g||^theta))), and never more than 500.
When both the energy change
and the model value are below 16 eps |E| neither can rank the two points: the
trial is then accepted (ratio 1) if and only if it lowers the Riemannian
gradient norm; and when the predicted decrease |<grad, xi>| is itself below
16 eps |E| the Armijo search (whose model values are then rounding noise) is
skipped and the full step alpha0 xi is tried; that trial has no model value,
so unless its energy change is also below 16 eps |E| (the gradient-norm rule
above) it is accepted if and only if the energy decreases.  A trial step whose
point u + t xi lies outside the retraction's domain (Omega for R1 and R2, S for
R3, Sec. 6) counts as a failed trial of its line search (t is reduced); RGBB
ends if no trial of a search can be retracted.  Thirty rejections
in a row end
the run unconverged.  sigma_hat never drops below 1e-8 (repeated very
successful steps would otherwise drive it to underflow, after which the
increases on rejection can no longer restore any regularisation).  The
gradient given to the truncated CG is projected onto the tangent space twice
(tangent_grad): with one projection its normal rounding noise, eps ||grad E||,
bounds the CG residual from below and the CG breaks down once the residual
tolerance ||grad||^2 falls under it.
"""

from dataclasses import dataclass, field
import numpy as np

from .energy import energy, grad as egrad, hvp as ehvp, laplacian
from .manifold import inner, rgrad, rhess, project
from .retraction import retract, psi


@dataclass
class SolveOpts:
    tol: float = 1e-6
    maxit: int = 10000
    retraction: int = 1
    # RGBB warm start (Algorithm 1, first loop; stop rules of Sec. 7.1)
    rgbb_tol: float = 1e-2
    rgbb_maxit: int = 2000
    rgbb_rho: float = 1e-4
    rgbb_delta: float = 0.2
    rgbb_varrho: float = 0.85
    rgbb_step0: float = 0.1
    # ARNT (Sec. 7.1 constants)
    eta1: float = 0.01
    eta2: float = 0.9
    gamma0: float = 0.2
    gamma1: float = 1.0
    gamma2: float = 10.0
    sigma_hat0: float = 1.0
    rho: float = 1e-4
    delta: float = 0.2
    alpha0: float = 1.0
    ls_max: int = 30
    cg_maxit: int = 500
    cg_per_digit: float = 80.0   # 0: the fixed cap cg_maxit
    cg_T: float = 0.1
    cg_theta: float = 1.0
    sigma_hat_min: float = 1e-8
    max_reject_streak: int = 30


@dataclass
class SolveStats:
    E: float = 0.0
    gnorm: float = 0.0
    rgbb_iters: int = 0
    outer: int = 0
    cg_total: int = 0
    hvp_calls: int = 0
    ls_trials: int = 0
    rejected: int = 0
    converged: bool = False
    history: list = field(default_factory=list)


def _norm(a):
    return np.sqrt(inner(a, a))


def energy_grad(prob, X):
    LX = laplacian(prob, X)
    return energy(prob, X, LX), egrad(prob, X, LX)


def _try_retract(prob, u, xi, t, kind):
    """R_u(t xi), or None when u + t xi lies outside the retraction's domain."""
    try:
        return retract(prob, u, xi, t, kind)
    except ValueError:
        return None


def rgbb(prob, u, opts, stats):
    """Riemannian gradient method with BB step and nonmonotone search (eq. NMN)."""
    E, G = energy_grad(prob, u)
    gR = rgrad(prob, u, G)[0]
    gn = _norm(gR)
    C, Q = E, 1.0
    step = opts.rgbb_step0 / max(gn, 1e-300)
    for k in range(opts.rgbb_maxit):
        if gn <= opts.rgbb_tol:
            break
        eta = -gR
        slope = inner(gR, eta)
        t = step
        z = None
        for _ in range(opts.ls_max):
            stats.ls_trials += 1
            zt = _try_retract(prob, u, eta, t, opts.retraction)
            if zt is None:                      # outside the retraction's domain: a failed trial
                t *= opts.rgbb_delta
                continue
            z = zt
            Ez = energy(prob, z)
            if Ez <= C + opts.rgbb_rho * t * slope:
                break
            t *= opts.rgbb_delta
        if z is None:
            break                               # no trial step could be retracted
        Ez, Gz = energy_grad(prob, z)
        gz = rgrad(prob, z, Gz)[0]
        s = z - u
        v = gz - gR
        vv = inner(v, v)
        step = abs(inner(s, v)) / vv if vv > 0 else step
        step = min(max(step, 1e-20), 1e20)
        Qn = opts.rgbb_varrho * Q + 1.0
        C = (opts.rgbb_varrho * Q * C + Ez) / Qn
        Q = Qn
        u, E, gR, gn = z, Ez, gz, _norm(gz)
        stats.rgbb_iters += 1
    return u


def cg_cap(opts, gn):
    """Inner-iteration cap of a subproblem at ||grad|| = gn (Sec. 7.1: adaptive in
    ||grad||; reading: cg_per_digit iterations per decimal digit the residual
    must gain, at most cg_maxit; cg_per_digit = 0 gives the fixed cap)."""
    if opts.cg_per_digit <= 0:
        return opts.cg_maxit
    digits = np.log10(1.0 / min(opts.cg_T, gn ** opts.cg_theta))
    return int(min(opts.cg_maxit, max(1.0, np.ceil(opts.cg_per_digit * digits))))


def tcg(prob, u, gR, ag, bg, sigma, opts, stats):
    """Truncated CG on Hess m_k[xi] = -grad m_k.  Returns (s, d, A d, sigma_est)."""
    gn = _norm(gR)
    tol = min(opts.cg_T, gn ** opts.cg_theta) * gn
    eps_c = 1e-12 * max(1.0, gn)
    z = np.zeros_like(gR)
    r = gR.copy()
    p = -r
    rr = inner(r, r)
    for i in range(cg_cap(opts, gn)):
        Ap = rhess(prob, u, p, ag, bg, sigma)
        stats.hvp_calls += 1
        stats.cg_total += 1
        kappa = inner(p, Ap)
        pp = inner(p, p)
        if kappa <= eps_c * pp:
            s = -gR if i == 0 else z
            if kappa < 0:
                return s, p, Ap, abs(kappa) / pp
            return s, None, None, None
        alpha = rr / kappa
        z = z + alpha * p
        r = r + alpha * Ap
        rr_new = inner(r, r)
        if np.sqrt(rr_new) <= tol:
            return z, None, None, None
        p = -r + (rr_new / rr) * p
        rr = rr_new
    return z, None, None, None


def tangent_grad(prob, u, G):
    """Riemannian gradient for the Newton subproblem: P_u applied twice.  One
    projection of G leaves a normal component of the size of its rounding,
    eps ||G||, and ||G|| stays O(E) at a critical point while ||grad|| -> 0; the
    truncated CG cannot reduce a normal residual (its operator maps into the
    tangent space), so that noise would bound the CG residual from below.
    Projecting the (small) result again leaves eps ||grad||.  Returns
    (grad, alpha_g, beta_g) with the multipliers of the first projection
    (those of Lemma 4.2's Hessian)."""
    gR, _, ag, bg = rgrad(prob, u, G)
    return project(prob, u, gR), ag, bg


def arnt(prob, u, opts, stats):
    """Modified adaptive regularized Newton method (Algorithm 1, second loop)."""
    eps = np.finfo(float).eps
    E, G = energy_grad(prob, u)
    gR, ag, bg = tangent_grad(prob, u, G)
    gn = _norm(gR)
    shat = opts.sigma_hat0
    streak = 0
    for k in range(opts.maxit):
        stats.history.append((E, gn))
        if gn <= opts.tol:
            stats.converged = True
            break
        if streak >= opts.max_reject_streak:
            break                                   # stagnation below FP64 resolution
        sigma = shat * gn
        s, d, Ad, sest = tcg(prob, u, gR, ag, bg, sigma, opts, stats)
        if d is not None:
            tau = inner(d, gR) / inner(d, Ad)       # eq. xi
            xi = s + tau * d
        else:
            xi = s
        slope = inner(gR, xi)
        t = opts.alpha0
        ok = False
        # Near FP64 resolution the model and the energy cannot rank points: take
        # the full step and let the gradient norm decide (reading, see header).
        resolved = abs(slope) > 16 * eps * abs(E)
        for _ in range(opts.ls_max if resolved else 0):
            z = _try_retract(prob, u, xi, t, opts.retraction)
            if z is None:                       # outside the retraction's domain: a failed trial
                stats.ls_trials += 1
                t *= opts.delta
                continue
            dz = z - u
            m = inner(G, dz) + 0.5 * inner(ehvp(prob, u, dz), dz) + 0.5 * sigma * inner(dz, dz)
            stats.hvp_calls += 1
            stats.ls_trials += 1
            if m <= opts.rho * t * slope:
                ok = True
                break
            t *= opts.delta
        if not resolved:
            z = _try_retract(prob, u, xi, t, opts.retraction)
            ok = z is not None
            m = 0.0
        ratio = -np.inf
        if ok:
            Ez, Gz = energy_grad(prob, z)
            dE = Ez - E
            if abs(dE) <= 16 * eps * abs(E) and abs(m) <= 16 * eps * abs(E):
                gz = rgrad(prob, z, Gz)[0]
                ratio = 1.0 if np.sqrt(inner(gz, gz)) < gn else -np.inf
            elif not resolved:
                # the model value was not evaluated (m = 0): the energy alone decides
                ratio = 1.0 if dE < 0 else -np.inf
            else:
                ratio = dE / m
        stats.outer += 1
        if ratio >= opts.eta1:
            u, E, G = z, Ez, Gz
            gR, ag, bg = tangent_grad(prob, u, G)
            gn = _norm(gR)
            shat = max(shat * (opts.gamma0 if ratio >= opts.eta2 else opts.gamma1), opts.sigma_hat_min)
            streak = 0
        else:
            stats.rejected += 1
            streak += 1
            shat *= opts.gamma2
        if sest is not None and gn > 0:
            shat = max(shat * gn, sest) / gn
    stats.E, stats.gnorm = E, gn
    return u


def solve(prob, X0, opts=None):
    """Ground state from X0 on one mesh: u0 = psi(X0) (projective), RGBB, ARNT."""
    opts = opts or SolveOpts()
    stats = SolveStats()
    u = psi(prob, X0, 1)
    u = rgbb(prob, u, opts, stats)
    u = arnt(prob, u, opts, stats)
    return u, stats
