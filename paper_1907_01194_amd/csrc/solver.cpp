// Newton driver: Algorithm 1 of Sec. 5 on one mesh -- RGBB warm start, then
// the modified adaptive regularized Newton method with a truncated CG on the
// regularised model, an Armijo curvilinear search on the model and the
// trust-region-like ratio test.  Every field operation runs on the device
// through the handle's operations; only scalars (inner products, norms,
// energies) come back to the host, in FP64.
//
// Choices the paper leaves open (its CG is the one of the cited ARNT work;
// its "default parameters" of RGBB are not printed):
//   * CG from 0, stop when ||r|| <= min(T, ||g||^theta) ||g|| (T = 0.1,
//     theta = 1); on curvature kappa = <p, A p> <= 1e-12 max(1, ||g||) ||p||^2
//     stop with s = z (or -g at the first iteration), d = p if kappa < 0,
//     sigma_est = |kappa| / ||p||^2;
//   * sigma_hat *= gamma0 if rho_k >= eta2, *= gamma1 if eta1 <= rho_k < eta2,
//     *= gamma2 on rejection; sigma = sigma_hat ||grad||; after a subproblem
//     that produced sigma_est, sigma_{k+1} = max(sigma_{k+1}, sigma_est);
//   * Armijo on the model with alpha0 = 1, rho = 1e-4, delta = 0.2, 30 trials;
//   * RGBB: first step 0.1/||grad||, BB step |<s,v>|/<v,v> clamped to
//     [1e-20, 1e20], rho = 1e-4, delta = 0.2, varrho = 0.85;
//   * when the energy change and the model value are both below 16 eps |E|
//     the trial is accepted (ratio 1) iff it lowers the Riemannian gradient
//     norm; when |<grad, xi>| <= 16 eps |E| the Armijo search is skipped and
//     the full step is tried, and if its energy change is resolved it is
//     accepted iff the energy decreases; 30 rejections in a row end the run
//     (each multiplies sigma by 10: by then a trial is a short gradient step);
//   * a trial step whose point lies outside the retraction's domain (Omega
//     for R1/R2, S for R3, Sec. 6) is a failed trial of its line search;
//     RGBB ends when no trial of a search can be retracted;
//   * sigma_hat is kept >= sigma_hat_min (1e-8): a run of very successful
//     steps would otherwise drive it to underflow, and the x10 increases on
//     rejection could then never restore any regularisation.
//   * the Riemannian gradient handed to the CG is projected twice: one
//     projection of the Euclidean gradient (of norm O(E) at a critical point)
//     leaves normal rounding noise eps ||grad E||, which the CG cannot reduce
//     (its operator maps into the tangent space); once the residual tolerance
//     ||grad||^2 falls below that noise the CG stalls and breaks down.
// In a mixed-precision handle the CG vectors, the Hessian products and the
// model evaluations are c64 with FP64 reductions; energies, gradients,
// retractions and the ratio are FP64.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <utility>
#include <vector>
#include <string>

#include "sched.h"

namespace gpe {

namespace {

struct Clock {
  std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();
  double sec() const {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
};

// solver workspace, allocated once per handle
enum {
  B_Z = 0,   // trial point (c128)
  B_GZ,      // gradient at the trial point (c128)
  B_GR,      // Riemannian gradient at u (c128)
  B_GRZ,     // Riemannian gradient at the trial point (c128)
  B_T1,      // scratch (c128)
  B_T2,      // scratch (c128)
  B_R,       // CG residual (work)
  B_P,       // CG direction (work)
  B_AP,      // Hess p (work)
  B_CZ,      // CG iterate (work)
  B_XI,      // search direction (work)
  B_DZ,      // z - u for the model (work)
  B_HDZ,     // H (z - u) (work)
  B_GW,      // Riemannian gradient in the work precision
  B_COUNT
};

gpe_status ensure_bufs(gpe_handle* h) {
  if ((int)h->solver_bufs.size() == B_COUNT) return GPE_OK;
  // work buffers take c128 in a mixed handle too: an FP64 polish reuses them
  const size_t f64 = h->nel * 16;
  h->solver_bufs.assign(B_COUNT, nullptr);
  for (int b = 0; b < B_COUNT; ++b) GPE_TRY(alloc_field(h, &h->solver_bufs[b], f64));
  return GPE_OK;
}

}  // namespace

// ---------------------------------------------------------------- requests
// Builders of the queued operations (sched.h); a driver pushes them and
// awaits a Round before reading results.
namespace {

Req rq_eval(const void* X, void* G, double* gram) {
  Req r;
  r.kind = RQ_EVAL;
  r.a = X;
  r.c = G;
  r.gram = gram;
  return r;
}
Req rq_pgrad(const void* X, const void* G, void* gR, double ag, double bg) {
  Req r;
  r.kind = RQ_PGRAD;
  r.a = X;
  r.b = G;
  r.c = gR;
  r.s0 = ag;
  r.s1 = bg;
  return r;
}
Req rq_norms(const void* u, const void* xi, bool xi32) {
  Req r;
  r.kind = RQ_NORMS;
  r.a = u;
  r.b = xi;
  r.b32 = xi32;
  return r;
}
Req rq_scale(const void* u, const void* xi, bool xi32, double t, const double* sig, void* out) {
  Req r;
  r.kind = RQ_SCALE;
  r.a = u;
  r.b = xi;
  r.b32 = xi32;
  r.c = out;
  r.s0 = t;
  for (int i = 0; i < 7; ++i) r.sig[i] = sig[i];
  return r;
}
Req rq_dot(const void* a, bool a32, const void* b, bool b32, size_t n) {
  Req r;
  r.kind = RQ_DOT;
  r.a = a;
  r.a32 = a32;
  r.b = b;
  r.b32 = b32;
  r.n = n;
  return r;
}
Req rq_diff(const void* a, const void* b, void* out, bool out32, size_t n) {
  Req r;
  r.kind = RQ_DIFF;
  r.a = a;
  r.b = b;
  r.c = out;
  r.c32 = out32;
  r.n = n;
  return r;
}
Req rq_axpby(double a, const void* x, double b, void* y, bool w32, size_t n) {
  Req r;
  r.kind = RQ_AXPBY;
  r.s0 = a;
  r.a = x;
  r.s1 = b;
  r.c = y;
  r.a32 = r.c32 = w32;
  r.n = n;
  return r;
}
Req rq_copy(const void* src, bool src32, void* dst, bool dst32, size_t n) {
  Req r;
  r.kind = RQ_COPY;
  r.a = src;
  r.a32 = src32;
  r.c = dst;
  r.c32 = dst32;
  r.n = n;
  return r;
}
Req rq_lap(const void* in, void* out, bool w32) {
  Req r;
  r.kind = RQ_LAP;
  r.a = in;
  r.c = out;
  r.a32 = r.c32 = w32;
  return r;
}
Req rq_hvp(const void* Z, void* HZ, bool riem, double sigma, bool w32) {
  Req r;
  r.kind = RQ_HVP;
  r.a = Z;
  r.c = HZ;
  r.flag = riem;
  r.s0 = sigma;
  r.a32 = r.c32 = w32;
  return r;
}
// One iteration (number iter from 0) of the device-resident truncated CG:
// A p, the update of r with the tests, then z += alpha p and the new direction
// p = -r + beta p in one pass over p.
void push_cg_iteration(Ctx& c, void* p, void* Ap, void* z, void* r, double sigma, bool w32, int iter) {
  Req h;
  h.kind = RQ_HVP;
  h.a = p;
  h.c = Ap;
  h.flag = true;
  h.cg = true;
  h.s0 = sigma;
  h.a32 = h.c32 = w32;
  c.push(h);
  Req u;
  u.kind = RQ_CG;
  u.a = z;
  u.b = Ap;
  u.c = p;
  u.d = r;
  u.s0 = iter;
  u.n = c.h->nel;
  u.a32 = u.c32 = w32;
  u.cg = true;
  c.push(u);
}

Req rq_cginit(double tol, double eps, int maxit) {
  Req r;
  r.kind = RQ_CGINIT;
  r.s0 = tol;
  r.s1 = eps;
  r.n = (size_t)(maxit > 0 ? maxit : 0);
  r.cg = true;
  return r;
}

// Make the handle's current point (Xp) the set point of its HVPs: the HVP
// needs L X_p for <X_i, (LZ)_i> = <(LX)_i, Z_i>.
void push_adopt(Ctx& c) {
  gpe_handle* h = c.h;
  if (work32(h)) {
    c.push(rq_copy(h->Xp, false, h->Xp32, true, h->nel));
    c.push(rq_lap(h->Xp32, h->LX32, true));
  } else {
    c.push(rq_lap(h->Xp, h->LX64, false));
  }
  h->has_point = true;
}

}  // namespace

#define CO_TRY(call)                 \
  do {                               \
    gpe_status s_ = (call);          \
    if (s_ != GPE_OK) co_return s_;  \
  } while (0)
#define ROUND co_await Round{}
// Project gR onto the tangent space at u once more (in place) and read its
// norm into gn.  One projection of G leaves a normal component of the size of
// its rounding, eps ||G||, with ||G|| = O(E) at a critical point; the CG cannot
// reduce a normal residual, so the second projection (leaving eps ||gR||)
// keeps that noise below every residual tolerance.
#define REPROJECT_GRAD()                                   \
  do {                                                     \
    RetractNorms rg_;                                      \
    double a_, b_;                                         \
    c.push(rq_norms(u, gR, false));                        \
    ROUND;                                                 \
    CO_TRY(norms_read(h, true, &rg_));                     \
    CO_TRY(proj_coeffs(h, rg_, &a_, &b_));                 \
    c.push(rq_pgrad(u, gR, gR, a_, b_));                   \
    ROUND;                                                 \
    CO_TRY(pgrad_read(h, &gn));                            \
  } while (0)

// One row of the optional solve trace (gpe_solve_opts.trace, GPE_TRACE_COLS columns).
static void trace_row(const gpe_solve_opts* o, gpe_solve_stats* st, double t, double E, double gn, double sigma,
                      double ratio, int cg, int reason, double step, int accepted) {
  if (!o->trace || st->trace_len >= o->trace_cap) return;
  double* r = o->trace + (size_t)st->trace_len * GPE_TRACE_COLS;
  const double v[GPE_TRACE_COLS] = {t, E, gn, (double)st->hvp_calls, sigma, ratio, (double)cg, (double)reason,
                                    step, (double)accepted};
  for (int i = 0; i < GPE_TRACE_COLS; ++i) r[i] = v[i];
  st->trace_len++;
}

SolveTask solve_task(Ctx& c, void* Xio, const gpe_solve_opts* o, gpe_solve_stats* st) {
  gpe_handle* h = c.h;
  Clock clk;
  CO_TRY(ensure_bufs(h));
  auto& B = h->solver_bufs;
  h->polish = false;
  bool w32 = work32(h);
  st->polish_at = -1;
  const size_t n = h->nel;
  const double eps = 2.220446049250313e-16;
  double sig[7];

  // u = psi(X0) (projective) into the set-point buffer
  {
    RetractNorms rn;
    c.push(rq_norms(Xio, nullptr, false));
    ROUND;
    CO_TRY(norms_read(h, false, &rn));
    CO_TRY(retract_sigma_at(h, rn, 0.0, GPE_R1_PROJECTIVE, sig));
    c.push(rq_scale(Xio, nullptr, false, 0.0, sig, h->Xp));
  }
  void* u = h->Xp;
  void* G = h->Gp;
  void* gR = B[B_GR];
  double E, ag, bg, gn;
  c.push(rq_eval(u, G, h->gram_pt));
  ROUND;
  CO_TRY(eval_read(h, true, &E, &ag, &bg));
  c.push(rq_pgrad(u, G, gR, ag, bg));
  ROUND;
  CO_TRY(pgrad_read(h, &gn));

  // ------------------------------------------------------------ RGBB
  Clock crg;
  {
    double C = E, Q = 1.0;
    double step = o->rgbb_step0 / std::fmax(gn, 1e-300);
    for (int k = 0; k < o->rgbb_maxit && gn > o->rgbb_tol; ++k) {
      if (o->time_limit > 0 && clk.sec() > o->time_limit) break;
      RetractNorms rn;
      c.push(rq_norms(u, gR, false));
      ROUND;
      CO_TRY(norms_read(h, true, &rn));
      double t = step, Ez = 0, agz = 0, bgz = 0;
      bool have_z = false;
      for (int ls = 0; ls < o->ls_max; ++ls) {
        st->ls_trials++;
        const gpe_status rs = retract_sigma_at(h, rn, -t, o->retraction, sig);
        if (rs == GPE_EDOMAIN) {          // outside the retraction's domain: a failed trial
          t *= o->rgbb_delta;
          continue;
        }
        CO_TRY(rs);
        c.push(rq_scale(u, gR, false, -t, sig, B[B_Z]));
        c.push(rq_eval(B[B_Z], B[B_GZ], h->gram_tmp));
        ROUND;
        CO_TRY(eval_read(h, true, &Ez, &agz, &bgz));
        have_z = true;
        if (Ez <= C - o->rgbb_rho * t * gn * gn) break;
        t *= o->rgbb_delta;
      }
      if (!have_z) break;                 // no trial step could be retracted
      double gnz;
      c.push(rq_pgrad(B[B_Z], B[B_GZ], B[B_GRZ], agz, bgz));
      ROUND;
      CO_TRY(pgrad_read(h, &gnz));
      c.push(rq_diff(B[B_Z], u, B[B_T1], false, n));
      c.push(rq_diff(B[B_GRZ], gR, B[B_T2], false, n));
      c.push(rq_dot(B[B_T1], false, B[B_T2], false, n));
      ROUND;
      double sv, vv;
      CO_TRY(dot_read(h, &sv));
      c.push(rq_dot(B[B_T2], false, B[B_T2], false, n));
      ROUND;
      CO_TRY(dot_read(h, &vv));
      if (vv > 0) step = std::fabs(sv) / vv;
      step = std::fmin(std::fmax(step, 1e-20), 1e20);
      const double Qn = o->rgbb_varrho * Q + 1.0;
      C = (o->rgbb_varrho * Q * C + Ez) / Qn;
      Q = Qn;
      std::swap(h->Xp, B[B_Z]);
      std::swap(h->Gp, B[B_GZ]);
      std::swap(B[B_GR], B[B_GRZ]);
      std::swap(h->gram_pt, h->gram_tmp);
      u = h->Xp;
      G = h->Gp;
      gR = B[B_GR];
      E = Ez;
      ag = agz;
      bg = bgz;
      gn = gnz;
      st->rgbb_iters++;
      if (o->verbose > 1) std::fprintf(stderr, "rgbb %d E=%.12f |g|=%.3e step=%.3e\n", k, E, gn, t);
    }
  }
  st->t_rgbb = crg.sec();
  trace_row(o, st, clk.sec(), E, gn, 0.0, NAN, 0, -1, 0.0, 1);

  // ------------------------------------------------------------ ARNT
  Clock carnt;
  REPROJECT_GRAD();
  h->E_pt = E;
  h->alpha_g = ag;
  h->beta_g = bg;
  push_adopt(c);
  double shat = o->sigma_hat0;
  int streak = 0;
  bool converged = false;
  double best_gn = gn;   // for the stagnation test of the FP64 polish
  int best_k = 0;
  for (int k = 0; k < o->maxit; ++k) {
    if (gn <= o->tol) {
      converged = true;
      break;
    }
    if (gn < 0.5 * best_gn) {
      best_gn = gn;
      best_k = k;
    }
    // FP64 polish of a mixed solve: below polish_tol, or when polish_window
    // outer iterations have not halved ||grad|| (the c64 Hessian cannot
    // resolve the soft directions that remain)
    if (w32 && ((o->polish_tol > 0 && gn <= o->polish_tol) ||
                (o->polish_window > 0 && k - best_k >= o->polish_window))) {
      if (!h->LX64) CO_TRY(alloc_field(h, &h->LX64, h->nel * 16));
      h->polish = true;
      w32 = false;
      push_adopt(c);
      st->polish_at = k;
      if (o->verbose) std::fprintf(stderr, "arnt %d: FP64 polish from |g|=%.3e\n", k, gn);
    }
    if (streak >= o->max_reject_streak) break;
    if (o->time_limit > 0 && clk.sec() > o->time_limit) break;
    const double sigma = shat * gn;

    // ---- truncated CG on Hess m_k [xi] = -grad m_k.  Its scalars (alpha, beta,
    // the curvature, residual and cap tests) live on the device, so a round
    // queues several iterations; launches after the stop return at once.
    void* r = B[B_R];
    void* p = B[B_P];
    void* Ap = B[B_AP];
    void* cz = B[B_CZ];
    void* xi = B[B_XI];
    c.push(rq_copy(gR, false, B[B_GW], w32, n));
    c.push(rq_copy(gR, false, r, w32, n));
    c.push(rq_copy(nullptr, w32, cz, w32, n));
    c.push(rq_axpby(-1.0, r, 0.0, p, w32, n));
    c.push(rq_dot(r, w32, r, w32, n));
    const double cg_tol = std::fmin(o->cg_T, std::pow(gn, o->cg_theta)) * gn;
    const double eps_c = 1e-12 * std::fmax(1.0, gn);
    int cg_cap = o->cg_maxit;
    if (o->cg_per_digit > 0) {
      const double digits = std::log10(1.0 / std::fmin(o->cg_T, std::pow(gn, o->cg_theta)));
      cg_cap = (int)std::fmin((double)o->cg_maxit, std::fmax(1.0, std::ceil(o->cg_per_digit * digits)));
    }
    c.push(rq_cginit(cg_tol, eps_c, cg_cap));
    CgState cs{};
    int queued = 0;
    for (int kstep = 2;; kstep = std::min(2 * kstep, 16)) {
      for (int j = 0; j < kstep; ++j) push_cg_iteration(c, p, Ap, cz, r, sigma, w32, queued++);
      ROUND;
      CO_TRY(cg_state_read(h, &cs));
      if (cs.done) break;
    }
    st->hvp_calls += cs.iters;
    st->cg_total += cs.iters;
    bool have_d = false, s_is_mg = false;
    double kappa_d = 0, sigma_est = -1.0;
    int it = cs.iters;
    if (cs.reason == CG_STOP_CURVATURE) {
      it = cs.iters - 1;                    // the iteration whose curvature stopped the CG
      if (it == 0) s_is_mg = true;
      if (cs.kappa < 0) {
        have_d = true;
        kappa_d = cs.kappa;
        sigma_est = std::fabs(cs.kappa) / cs.pp;
      }
    }
    // ---- direction xi = s + tau d (eq. xi)
    if (s_is_mg) c.push(rq_axpby(-1.0, B[B_GW], 0.0, xi, w32, n));
    else c.push(rq_copy(cz, w32, xi, w32, n));
    if (have_d) {
      double dg;
      c.push(rq_dot(p, w32, B[B_GW], w32, n));
      ROUND;
      CO_TRY(dot_read(h, &dg));
      c.push(rq_axpby(dg / kappa_d, p, 1.0, xi, w32, n));
    }
    double slope;
    c.push(rq_dot(gR, false, xi, w32, n));
    ROUND;
    CO_TRY(dot_read(h, &slope));

    // ---- Armijo curvilinear search on the model (eq. tp1, tp2).  Near FP64
    // resolution (|<grad, xi>| <= 16 eps |E|) model values are rounding noise:
    // the full step is tried and the gradient norm decides below.
    RetractNorms rn;
    c.push(rq_norms(u, xi, w32));
    ROUND;
    CO_TRY(norms_read(h, true, &rn));
    const bool resolved = std::fabs(slope) > 16 * eps * std::fabs(E);
    double t = o->alpha0, m = 0;
    bool ok = false;
    for (int ls = 0; resolved && ls < o->ls_max; ++ls) {
      const gpe_status rs = retract_sigma_at(h, rn, t, o->retraction, sig);
      if (rs == GPE_EDOMAIN) {            // outside the retraction's domain: a failed trial
        st->ls_trials++;
        t *= o->delta;
        continue;
      }
      CO_TRY(rs);
      c.push(rq_scale(u, xi, w32, t, sig, B[B_Z]));
      c.push(rq_diff(B[B_Z], u, B[B_DZ], w32, n));
      c.push(rq_hvp(B[B_DZ], B[B_HDZ], false, 0.0, w32));
      ROUND;
      double dHd, dd, gd;
      CO_TRY(hvp_read(h, &dHd, &dd));
      c.push(rq_dot(G, false, B[B_DZ], w32, n));
      ROUND;
      CO_TRY(dot_read(h, &gd));
      m = gd + 0.5 * dHd + 0.5 * sigma * dd;
      st->hvp_calls++;
      st->ls_trials++;
      if (m <= o->rho * t * slope) {
        ok = true;
        break;
      }
      t *= o->delta;
    }
    if (!resolved) {
      const gpe_status rs = retract_sigma_at(h, rn, t, o->retraction, sig);
      if (rs != GPE_EDOMAIN) {
        CO_TRY(rs);
        c.push(rq_scale(u, xi, w32, t, sig, B[B_Z]));
        ok = true;
      }
      m = 0.0;
    }
    double ratio = -INFINITY, Ez = 0, agz = 0, bgz = 0, gnz = -1.0;
    if (ok) {
      c.push(rq_eval(B[B_Z], B[B_GZ], h->gram_tmp));
      ROUND;
      CO_TRY(eval_read(h, true, &Ez, &agz, &bgz));
      const double dE = Ez - E;
      if (std::fabs(dE) <= 16 * eps * std::fabs(E) && std::fabs(m) <= 16 * eps * std::fabs(E)) {
        // energies cannot rank u and z: the Riemannian gradient norm does
        c.push(rq_pgrad(B[B_Z], B[B_GZ], B[B_GRZ], agz, bgz));
        ROUND;
        CO_TRY(pgrad_read(h, &gnz));
        ratio = gnz < gn ? 1.0 : -INFINITY;
      } else if (!resolved) {
        ratio = dE < 0 ? 1.0 : -INFINITY;   // the model was not evaluated: the energy decides
      } else {
        ratio = dE / m;
      }
    }
    st->outer++;
    if (o->verbose)
      std::fprintf(stderr, "arnt %d E=%.14f |g|=%.3e sigma=%.3e cg=%d t=%.2e ratio=%.3f\n", k, E, gn, sigma, it, t,
                   ratio);
    if (ratio >= o->eta1) {
      std::swap(h->Xp, B[B_Z]);
      std::swap(h->Gp, B[B_GZ]);
      std::swap(h->gram_pt, h->gram_tmp);
      u = h->Xp;
      G = h->Gp;
      E = Ez;
      ag = agz;
      bg = bgz;
      c.push(rq_pgrad(u, G, gR, ag, bg));
      ROUND;
      CO_TRY(pgrad_read(h, &gn));
      REPROJECT_GRAD();
      h->E_pt = E;
      h->alpha_g = ag;
      h->beta_g = bg;
      push_adopt(c);
      shat = std::fmax(shat * (ratio >= o->eta2 ? o->gamma0 : o->gamma1), o->sigma_hat_min);
      streak = 0;
    } else {
      st->rejected++;
      streak++;
      shat *= o->gamma2;
    }
    if (sigma_est >= 0 && gn > 0) shat = std::fmax(shat * gn, sigma_est) / gn;
    trace_row(o, st, clk.sec(), E, gn, sigma, ratio, it, cs.reason, t, ratio >= o->eta1 ? 1 : 0);
  }
  st->t_arnt = carnt.sec();
  if (h->polish) {   // leave the handle's HVPs in its own precision at the final point
    h->polish = false;
    push_adopt(c);
  }

  c.push(rq_copy(u, false, Xio, false, n));
  c.push(rq_norms(u, nullptr, false));
  ROUND;
  RetractNorms fin;
  CO_TRY(norms_read(h, false, &fin));
  double mass = 0, mag = 0;
  for (int i = 0; i < h->K; ++i) {
    mass += fin.uu[i];
    mag += (h->F - i) * fin.uu[i];
  }
  st->E = E;
  st->gnorm = gn;
  st->converged = converged;
  st->mass_err = std::fabs(mass - 1.0);
  st->mag_err = std::fabs(mag - h->M);
  st->t_total = clk.sec();
  if (!converged) co_return fail(h, GPE_ENOTCONV, "tolerance not reached");
  co_return GPE_OK;
}

#undef REPROJECT_GRAD
#undef CO_TRY
#undef ROUND

// Cascadic multigrid (Algorithm 1, outer loop): solve on the coarsest of
// mg_levels nested meshes (every axis halved per level, same box, V and the
// initial state injected), then prolong each solution as the next finer
// mesh's initial guess (Fourier interpolation); coarse meshes stop at
// mg_coarse_tol (Sec. 7.1: 1e-5), the finest at tol.
gpe_status newton_solve(gpe_handle* h, void* Xio, const gpe_solve_opts* o, gpe_solve_stats* st) {
  int L = o->mg_levels;
  // the coarsest admissible level: every used axis stays even, supported, >= 8
  for (int l = 1; l <= L; ++l)
    for (int a = 0; a < h->dim; ++a) {
      const int m = h->n[a] >> l;
      if ((h->n[a] % (1 << l)) || m < 8 || m % 2 || !lap_size_supported(m)) {
        L = l - 1;
        break;
      }
    }
  if (L <= 0) {
    gpe_status r = solve_single(h, Xio, o, st);
    st->mg_levels = 0;
    return r;
  }
  Clock clk;
  std::vector<gpe_handle*> hs(L + 1, nullptr);
  std::vector<void*> xs(L + 1, nullptr);
  hs[0] = h;
  xs[0] = Xio;
  gpe_status rs = GPE_OK;
  for (int l = 1; l <= L && rs == GPE_OK; ++l) {
    const gpe_handle* f = hs[l - 1];
    gpe_problem pc = f->prob;
    std::vector<double> Vc;
    int nc[3] = {1, 1, 1};
    for (int a = 0; a < f->dim; ++a) {
      pc.n[a] = f->n[a] / 2;
      nc[a] = pc.n[a];
    }
    Vc.resize((size_t)nc[0] * nc[1] * nc[2]);
    const int sy = f->dim > 1 ? 2 : 1, sz = f->dim > 2 ? 2 : 1;
    for (int z = 0; z < nc[2]; ++z)
      for (int y = 0; y < nc[1]; ++y)
        for (int x = 0; x < nc[0]; ++x)
          Vc[((size_t)z * nc[1] + y) * nc[0] + x] =
              f->Vhost[((size_t)(z * sz) * f->n[1] + (size_t)(y * sy)) * f->n[0] + 2 * x];
    rs = gpe_create(&pc, Vc.data(), h->prec, h->st, &hs[l]);
    if (rs != GPE_OK) {
      fail(h, rs, std::string("multigrid: coarse handle: ") + gpe_last_error(nullptr));
      hs[l] = nullptr;
      break;
    }
    rs = alloc_field(h, &xs[l], hs[l]->nel * 16);
    if (rs != GPE_OK) break;
    hipError_t e = restrict_inject(xs[l - 1], xs[l], h->K, h->dim, nc, std::pow(2.0, 0.5 * h->dim), h->st);
    if (e != hipSuccess) rs = hip_fail(h, e, "restrict_inject");
  }
  double t_coarse = 0.0;
  for (int l = L; l >= 1 && rs == GPE_OK; --l) {
    gpe_solve_opts oc = *o;
    oc.tol = o->mg_coarse_tol;
    oc.mg_levels = 0;
    oc.trace = nullptr;   // the trace follows the finest mesh only
    oc.trace_cap = 0;
    if (o->time_limit > 0) oc.time_limit = std::fmax(o->time_limit - clk.sec(), 1e-3);
    gpe_solve_stats sc;
    std::memset(&sc, 0, sizeof(sc));
    gpe_status r = solve_single(hs[l], xs[l], &oc, &sc);
    if (r != GPE_OK && r != GPE_ENOTCONV) {
      rs = fail(h, r, std::string("multigrid: coarse solve: ") + hs[l]->err);
      break;
    }
    if (o->verbose)
      std::fprintf(stderr, "mg level %d (%dx%dx%d): E=%.12f |g|=%.3e outer=%d cg=%d %.2fs\n", l, hs[l]->n[0],
                   hs[l]->n[1], hs[l]->n[2], sc.E, sc.gnorm, sc.outer, sc.cg_total, sc.t_total);
    rs = prolong(hs[l], xs[l], hs[l - 1], xs[l - 1]);
    if (rs != GPE_OK && hs[l - 1] != h) h->err = hs[l - 1]->err;
  }
  t_coarse = clk.sec();
  for (int l = 1; l <= L; ++l) {
    if (xs[l]) (void)hipFree(xs[l]);
    if (hs[l]) gpe_destroy(hs[l]);
  }
  if (rs != GPE_OK) return rs;
  gpe_solve_opts of = *o;
  of.mg_levels = 0;
  if (o->time_limit > 0) of.time_limit = std::fmax(o->time_limit - clk.sec(), 1e-3);
  gpe_status r = solve_single(h, Xio, &of, st);   // counters: finest mesh only
  st->mg_levels = L;
  st->t_coarse = t_coarse;
  st->t_total += t_coarse;
  return r;
}

}  // namespace gpe
