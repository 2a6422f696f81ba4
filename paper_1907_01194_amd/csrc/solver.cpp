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
//     the full step is tried; 12 rejections in a row end the run;
//   * sigma_hat is kept >= sigma_hat_min (1e-8): a run of very successful
//     steps would otherwise drive it to underflow, and the x10 increases on
//     rejection could then never restore any regularisation.
// In a mixed-precision handle the CG vectors, the Hessian products and the
// model evaluations are c64 with FP64 reductions; energies, gradients,
// retractions and the ratio are FP64.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <utility>
#include <vector>
#include <string>

#include "runtime.h"

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
  const size_t f64 = h->nel * 16;
  const size_t fw = h->nel * (h->prec == GPE_FP64 ? 16 : 8);
  h->solver_bufs.assign(B_COUNT, nullptr);
  for (int b = 0; b < B_COUNT; ++b) GPE_TRY(alloc_field(h, &h->solver_bufs[b], b < B_R ? f64 : fw));
  return GPE_OK;
}

}  // namespace

static gpe_status newton_solve_one(gpe_handle* h, void* Xio, const gpe_solve_opts* o, gpe_solve_stats* st) {
  Clock clk;
  GPE_TRY(ensure_bufs(h));
  auto& B = h->solver_bufs;
  const bool w32 = h->prec == GPE_MIXED;
  const size_t n = h->nel;
  const double eps = 2.220446049250313e-16;
  hipStream_t s = h->st;

  // u = psi(X0) (projective) into the set-point buffer
  {
    RetractNorms rn;
    GPE_TRY(retract_norms(h, Xio, nullptr, false, &rn));
    GPE_TRY(retract_apply(h, rn, Xio, nullptr, false, 0.0, GPE_R1_PROJECTIVE, h->Xp));
  }
  void* u = h->Xp;
  void* G = h->Gp;
  void* gR = B[B_GR];
  double E, ag, bg, gn;
  GPE_TRY(eval_point(h, u, G, h->gram_pt, &E, &ag, &bg));
  GPE_TRY(project_grad(h, u, G, gR, ag, bg, &gn));

  // ------------------------------------------------------------ RGBB
  Clock crg;
  {
    double C = E, Q = 1.0;
    double step = o->rgbb_step0 / std::fmax(gn, 1e-300);
    for (int k = 0; k < o->rgbb_maxit && gn > o->rgbb_tol; ++k) {
      if (o->time_limit > 0 && clk.sec() > o->time_limit) break;
      RetractNorms rn;
      GPE_TRY(retract_norms(h, u, gR, false, &rn));
      double t = step, Ez = 0, agz = 0, bgz = 0;
      for (int ls = 0; ls < o->ls_max; ++ls) {
        GPE_TRY(retract_apply(h, rn, u, gR, false, -t, o->retraction, B[B_Z]));
        GPE_TRY(eval_point(h, B[B_Z], B[B_GZ], h->gram_tmp, &Ez, &agz, &bgz));
        st->ls_trials++;
        if (Ez <= C - o->rgbb_rho * t * gn * gn) break;
        t *= o->rgbb_delta;
      }
      double gnz;
      GPE_TRY(project_grad(h, B[B_Z], B[B_GZ], B[B_GRZ], agz, bgz, &gnz));
      GPE_HIP(h, (diff<double, double, double>(B[B_Z], u, B[B_T1], n, s)));
      GPE_HIP(h, (diff<double, double, double>(B[B_GRZ], gR, B[B_T2], n, s)));
      double sv, vv;
      GPE_TRY(dot_host(h, B[B_T1], false, B[B_T2], false, n, &sv));
      GPE_TRY(dot_host(h, B[B_T2], false, B[B_T2], false, n, &vv));
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

  // ------------------------------------------------------------ ARNT
  Clock carnt;
  h->E_pt = E;
  h->alpha_g = ag;
  h->beta_g = bg;
  GPE_TRY(adopt_point(h));
  double shat = o->sigma_hat0;
  int streak = 0;
  auto to_work = [&](const void* src, void* dst) -> gpe_status {
    if (w32) GPE_HIP(h, to_c64(src, dst, n, s));
    else GPE_HIP(h, hipMemcpyAsync(dst, src, n * 16, hipMemcpyDeviceToDevice, s));
    return GPE_OK;
  };
  auto axpby_w = [&](double a, const void* x, double b, void* y) -> gpe_status {
    if (w32) GPE_HIP(h, axpby<float>(a, x, b, y, n, s));
    else GPE_HIP(h, axpby<double>(a, x, b, y, n, s));
    return GPE_OK;
  };
  bool converged = false;
  for (int k = 0; k < o->maxit; ++k) {
    if (gn <= o->tol) {
      converged = true;
      break;
    }
    if (streak >= o->max_reject_streak) break;
    if (o->time_limit > 0 && clk.sec() > o->time_limit) break;
    const double sigma = shat * gn;

    // ---- truncated CG on Hess m_k [xi] = -grad m_k
    void* r = B[B_R];
    void* p = B[B_P];
    void* Ap = B[B_AP];
    void* cz = B[B_CZ];
    void* xi = B[B_XI];
    GPE_TRY(to_work(gR, B[B_GW]));
    GPE_TRY(to_work(gR, r));
    GPE_HIP(h, hipMemsetAsync(cz, 0, n * (w32 ? 8 : 16), s));
    GPE_HIP(h, hipMemsetAsync(p, 0, n * (w32 ? 8 : 16), s));
    GPE_TRY(axpby_w(-1.0, r, 0.0, p));
    double rr;
    GPE_TRY(dot_host(h, r, w32, r, w32, n, &rr));
    const double cg_tol = std::fmin(o->cg_T, std::pow(gn, o->cg_theta)) * gn;
    const double eps_c = 1e-12 * std::fmax(1.0, gn);
    bool have_d = false, s_is_mg = false;
    double kappa_d = 0, sigma_est = -1.0;
    int it = 0;
    for (; it < o->cg_maxit; ++it) {
      double kappa, pp;
      GPE_TRY(hvp(h, p, Ap, true, sigma, &kappa, &pp));
      st->hvp_calls++;
      st->cg_total++;
      if (kappa <= eps_c * pp) {
        if (it == 0) s_is_mg = true;
        if (kappa < 0) {
          have_d = true;
          kappa_d = kappa;
          sigma_est = std::fabs(kappa) / pp;
        }
        break;
      }
      const double alpha = rr / kappa;
      if (w32) GPE_HIP(h, cg_update<float>(alpha, p, Ap, cz, r, h->part, h->nblk, n, s));
      else GPE_HIP(h, cg_update<double>(alpha, p, Ap, cz, r, h->part, h->nblk, n, s));
      GPE_TRY(reduce_to_host(h, 1, POST_NONE, nullptr, 1));
      const double rr_new = h->hres[0];
      if (std::sqrt(rr_new) <= cg_tol) {
        ++it;
        break;
      }
      GPE_TRY(axpby_w(-1.0, r, rr_new / rr, p));
      rr = rr_new;
    }
    // ---- direction xi = s + tau d (eq. xi)
    if (s_is_mg) GPE_TRY(axpby_w(-1.0, B[B_GW], 0.0, xi));
    else GPE_HIP(h, hipMemcpyAsync(xi, cz, n * (w32 ? 8 : 16), hipMemcpyDeviceToDevice, s));
    if (have_d) {
      double dg;
      GPE_TRY(dot_host(h, p, w32, B[B_GW], w32, n, &dg));
      GPE_TRY(axpby_w(dg / kappa_d, p, 1.0, xi));
    }
    double slope;
    GPE_TRY(dot_host(h, gR, false, xi, w32, n, &slope));

    // ---- Armijo curvilinear search on the model (eq. tp1, tp2).  Near FP64
    // resolution (|<grad, xi>| <= 16 eps |E|) model values are rounding noise:
    // the full step is tried and the gradient norm decides below.
    RetractNorms rn;
    GPE_TRY(retract_norms(h, u, xi, w32, &rn));
    const bool resolved = std::fabs(slope) > 16 * eps * std::fabs(E);
    double t = o->alpha0, m = 0;
    bool ok = false;
    for (int ls = 0; resolved && ls < o->ls_max; ++ls) {
      GPE_TRY(retract_apply(h, rn, u, xi, w32, t, o->retraction, B[B_Z]));
      if (w32) GPE_HIP(h, (diff<double, double, float>(B[B_Z], u, B[B_DZ], n, s)));
      else GPE_HIP(h, (diff<double, double, double>(B[B_Z], u, B[B_DZ], n, s)));
      double dHd, dd, gd;
      GPE_TRY(hvp(h, B[B_DZ], B[B_HDZ], false, 0.0, &dHd, &dd));
      GPE_TRY(dot_host(h, G, false, B[B_DZ], w32, n, &gd));
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
      GPE_TRY(retract_apply(h, rn, u, xi, w32, t, o->retraction, B[B_Z]));
      ok = true;
      m = 0.0;
    }
    double ratio = -INFINITY, Ez = 0, agz = 0, bgz = 0, gnz = -1.0;
    if (ok) {
      GPE_TRY(eval_point(h, B[B_Z], B[B_GZ], h->gram_tmp, &Ez, &agz, &bgz));
      const double dE = Ez - E;
      if (std::fabs(dE) <= 16 * eps * std::fabs(E) && std::fabs(m) <= 16 * eps * std::fabs(E)) {
        // energies cannot rank u and z: the Riemannian gradient norm does
        GPE_TRY(project_grad(h, B[B_Z], B[B_GZ], B[B_GRZ], agz, bgz, &gnz));
        ratio = gnz < gn ? 1.0 : -INFINITY;
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
      GPE_TRY(project_grad(h, u, G, gR, ag, bg, &gn));
      h->E_pt = E;
      h->alpha_g = ag;
      h->beta_g = bg;
      GPE_TRY(adopt_point(h));
      shat = std::fmax(shat * (ratio >= o->eta2 ? o->gamma0 : o->gamma1), o->sigma_hat_min);
      streak = 0;
    } else {
      st->rejected++;
      streak++;
      shat *= o->gamma2;
    }
    if (sigma_est >= 0 && gn > 0) shat = std::fmax(shat * gn, sigma_est) / gn;
  }
  st->t_arnt = carnt.sec();

  GPE_HIP(h, hipMemcpyAsync(Xio, u, n * 16, hipMemcpyDeviceToDevice, s));
  double mass, mag;
  GPE_TRY(gpe_constraints(h, u, &mass, &mag));
  st->E = E;
  st->gnorm = gn;
  st->converged = converged;
  st->mass_err = std::fabs(mass - 1.0);
  st->mag_err = std::fabs(mag - h->M);
  st->t_total = clk.sec();
  if (!converged) return fail(h, GPE_ENOTCONV, "tolerance not reached");
  return GPE_OK;
}

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
    gpe_status r = newton_solve_one(h, Xio, o, st);
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
    if (o->time_limit > 0) oc.time_limit = std::fmax(o->time_limit - clk.sec(), 1e-3);
    gpe_solve_stats sc;
    std::memset(&sc, 0, sizeof(sc));
    gpe_status r = newton_solve_one(hs[l], xs[l], &oc, &sc);
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
  gpe_status r = newton_solve_one(h, Xio, &of, st);   // counters: finest mesh only
  st->mg_levels = L;
  st->t_coarse = t_coarse;
  st->t_total += t_coarse;
  return r;
}

}  // namespace gpe
