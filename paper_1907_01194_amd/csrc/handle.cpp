// C ABI entry points (include/gpe.h) and the device operations they are
// built from.  Host code only: every kernel is launched through kernels.h.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>

#include "common.h"
#include "retract_scalar.h"
#include "runtime.h"

static std::string g_create_error;

namespace gpe {

gpe_status fail(gpe_handle* h, gpe_status s, const std::string& msg) {
  if (h) h->err = msg;
  else g_create_error = msg;
  return s;
}

gpe_status hip_fail(gpe_handle* h, hipError_t e, const char* where) {
  std::string m = std::string("HIP error '") + hipGetErrorString(e) + "' in " + where;
  return fail(h, e == hipErrorOutOfMemory ? GPE_ENOMEM : GPE_EHIP, m);
}

const char* const kKernelNames[KK_COUNT] = {"lap_axis_x", "lap_axis_y", "lap_axis_z", "hvp_xpass",
                                            "pw_grad", "finalize", "project", "comp_norms",
                                            "scale_comps", "vector_ops"};

hipEvent_t timing_event(gpe_handle* h) {
  if (!h->event_pool.empty()) {
    hipEvent_t e = h->event_pool.back();
    h->event_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  (void)hipEventCreate(&e);
  return e;
}

gpe_status alloc_field(gpe_handle* h, void** p, size_t bytes) {
  hipError_t e = hipMalloc(p, bytes);
  if (e != hipSuccess) {
    *p = nullptr;
    (void)hipGetLastError();
    return fail(h, GPE_ENOMEM, "device allocation of " + std::to_string(bytes) + " bytes failed");
  }
  return GPE_OK;
}

template <typename T>
gpe_status laplacian(gpe_handle* h, const void* in, void* out) {
  for (int a = 0; a < h->dim; ++a) GPE_KT(h, KK_LAP_X + a, lap_axis<T>(h->ax[a], in, a == 0 ? nullptr : out, out, h->st));
  return GPE_OK;
}
template gpe_status laplacian<double>(gpe_handle*, const void*, void*);
template gpe_status laplacian<float>(gpe_handle*, const void*, void*);

gpe_status finalize_enq(gpe_handle* h, int nq, int post, double* gram) {
  SlotCounts nb;
  for (int q = 0; q < kMaxQ; ++q) nb.nb[q] = h->nblk;
  GPE_KT(h, KK_FINALIZE, finalize(h->part, h->nblk, nb, nq, h->res, post, h->F, gram, h->ticket, nullptr, h->st));
  return GPE_OK;
}

gpe_status fetch(gpe_handle* h) {
  GPE_HIP(h, hipMemcpyAsync(h->hres, h->res, sizeof(double) * kResDoubles, hipMemcpyDeviceToHost, h->st));
  GPE_HIP(h, hipStreamSynchronize(h->st));
  return GPE_OK;
}

static gpe_status finite(gpe_handle* h, const double* v, int n, const char* what) {
  for (int i = 0; i < n; ++i)
    if (!std::isfinite(v[i])) return fail(h, GPE_ENUMERIC, std::string("NaN or Inf in ") + what);
  return GPE_OK;
}

gpe_status reduce_to_host(gpe_handle* h, int nq, int post, double* gram, int nout) {
  GPE_TRY(finalize_enq(h, nq, post, gram));
  GPE_TRY(fetch(h));
  return finite(h, h->hres, nout, "a reduction");
}

gpe_status eval_enq(gpe_handle* h, const void* X, void* G, double* gram) {
  GPE_TRY(laplacian<double>(h, X, h->T64));
  GPE_KT(h, KK_PW_GRAD, pw_grad<double>(h->F, X, h->T64, h->V64, G, h->part, h->nblk, h->npts, h->pw, h->st));
  return finalize_enq(h, 1 + 2 * h->K, G ? POST_GRAD : POST_NONE, G ? gram : nullptr);
}

gpe_status eval_read(gpe_handle* h, bool grad, double* E, double* ag, double* bg) {
  const int nq = 1 + 2 * h->K;
  const double* r = h->hres;
  // the reductions first; the multipliers after the degeneracy test (a
  // singular Gram system gives NaN multipliers, which is GPE_EDEGEN)
  GPE_TRY(finite(h, r, grad ? nq : 1, "the energy or gradient"));
  if (grad) {
    double a11 = 0, a12 = 0, a22 = 0;
    for (int i = 0; i < h->K; ++i) {
      const double l = h->F - i;
      a11 += r[1 + h->K + i];
      a12 += l * r[1 + h->K + i];
      a22 += l * l * r[1 + h->K + i];
    }
    if (!(a11 * a22 - a12 * a12 > 0))
      return fail(h, GPE_EDEGEN, "degenerate point: u^T Gamma^2 u u^T u - (u^T Gamma u)^2 <= 0");
    GPE_TRY(finite(h, r + nq, 2, "the gradient's multipliers"));
    if (ag) *ag = r[nq];
    if (bg) *bg = r[nq + 1];
  }
  if (E) *E = r[0];
  return GPE_OK;
}

gpe_status eval_point(gpe_handle* h, const void* X, void* G, double* gram, double* E, double* ag, double* bg) {
  GPE_TRY(eval_enq(h, X, G, gram));
  GPE_TRY(fetch(h));
  return eval_read(h, G != nullptr, E, ag, bg);
}

gpe_status pgrad_enq(gpe_handle* h, const void* X, const void* G, void* gR, double ag, double bg) {
  GPE_KT(h, KK_PROJECT,
         launch_single(ProjArgs<double, double, true>{X, G, gR, nullptr, ag, bg, h->part, h->npts, h->F}, h->nblk,
                       h->st));
  return finalize_enq(h, 1, POST_NONE, nullptr);
}

gpe_status pgrad_read(gpe_handle* h, double* gnorm) {
  GPE_TRY(finite(h, h->hres, 1, "the gradient norm"));
  if (gnorm) *gnorm = std::sqrt(h->hres[0]);
  return GPE_OK;
}

gpe_status project_grad(gpe_handle* h, const void* X, const void* G, void* gR, double ag, double bg,
                        double* gnorm) {
  GPE_TRY(pgrad_enq(h, X, G, gR, ag, bg));
  GPE_TRY(fetch(h));
  return pgrad_read(h, gnorm);
}

gpe_status adopt_point(gpe_handle* h) {
  // the HVP needs L X_p for <X_i, (LZ)_i> = <(LX)_i, Z_i>
  if (work32(h)) {
    GPE_HIP(h, to_c64(h->Xp, h->Xp32, h->nel, h->st));
    GPE_TRY(laplacian<float>(h, h->Xp32, h->LX32));
  } else {
    GPE_TRY(laplacian<double>(h, h->Xp, h->LX64));
  }
  h->has_point = true;
  return GPE_OK;
}

// cg: one iteration of the device-resident truncated CG (the launches are
// skipped once the CG has stopped, and the last finalize runs its tests).
// kappa: form <Z, HZ> and ||Z||^2 (res[34..35]) in a last finalize; gpe_hvp
// without scalar outputs skips that launch.
template <typename T>
static gpe_status hvp_t(gpe_handle* h, const void* Z, void* HZ, bool riem, const PwParams& p, bool cg,
                        bool kappa) {
  const void* Xw = sizeof(T) == 8 ? h->Xp : h->Xp32;
  const void* Yw = sizeof(T) == 8 ? h->LX64 : h->LX32;
  const T* Vw = reinterpret_cast<const T*>(sizeof(T) == 8 ? (const void*)h->V64 : (const void*)h->V32);
  const double* skip = cg ? h->res + CG_DONE : nullptr;
  SlotCounts nb;
  for (int q = 0; q < kMaxQ; ++q) nb.nb[q] = 0;
  int nbx = 0;
  GPE_KT(h, KK_HVP_XPASS,
         hvp_xpass<T>(h->F, h->ax[0], h->npts, Xw, Z, Yw, Vw, HZ, p, h->part, h->pstride, &nbx, h->xvar, skip, h->st));
  for (int q = 0; q < 7; ++q) nb.nb[q] = nbx;
  double* coef = h->res + 32;
  // Projection coefficients (Lemma 4.1) from the x pass's partials: with few
  // x-pass workgroups every workgroup of the last axis pass forms them itself;
  // in 3D otherwise one extra workgroup of the y pass does; else a finalize.
  const bool ab_local = riem && h->dim >= 2 && nbx <= kAbLocalMax;
  const bool ab_ypass = riem && !ab_local && h->dim == 3;
  if (riem && !ab_local && !ab_ypass)
    GPE_KT(h, KK_FINALIZE,
           finalize(h->part, h->pstride, nb, 7, h->res, POST_HVP_AB, h->F, h->gram_pt, h->ticket, skip, h->st));
  int nq = 7;
  if (h->dim == 1) {
    // (after a CG stop this projection still runs, on an HZ that nothing reads any more)
    if (riem)
      GPE_KT(h, KK_PROJECT,
             launch_single(ProjArgs<T, T, false>{Xw, HZ, HZ, coef, 0.0, 0.0, nullptr, h->npts, h->F}, h->nblk, h->st));
  } else {
    for (int a = 1; a < h->dim; ++a) {
      const bool proj = riem && a == h->dim - 1;
      AbSrc ab, fin;
      if (proj && ab_local) ab = AbSrc{h->part, h->pstride, nbx, h->gram_pt, h->res};
      if (a == 1 && ab_ypass) fin = AbSrc{h->part, h->pstride, nbx, h->gram_pt, h->res};
      GPE_KT(h, KK_LAP_X + a,
             lap_axis_ex<T>(h->ax[a], Z, HZ, HZ, h->F, h->npts, proj ? Xw : nullptr, coef, h->part, h->pstride,
                            6 + a, &nb.nb[6 + a], skip, a == 1, ab.part ? &ab : nullptr, fin.part ? &fin : nullptr,
                            h->st));
      nq = 7 + a;
    }
  }
  if (!cg && !kappa) return GPE_OK;
  const int post = cg ? POST_CG_KAPPA : riem ? POST_HVP_KAPPA : POST_HVP_KAPPA_E;
  GPE_KT(h, KK_FINALIZE, finalize(h->part, h->pstride, nb, nq, h->res, post, h->F, h->gram_pt, h->ticket, skip, h->st));
  return GPE_OK;
}

// Pick the fused x pass's rows-per-workgroup by timing each variant on the
// handle's own grid.  The fields hold pseudo-random values rather than zeros:
// the cost does not depend on the values, but the power drawn (and so the
// clock the chip sustains) does.
template <typename T>
static gpe_status tune_xpass_t(gpe_handle* h) {
  const int nv = xpass_variants(h->n[0]);
  if (nv <= 1 || h->npts < (1u << 15)) return GPE_OK;
  // three distinct fields for X, Z, LX (aliasing them would hide memory traffic)
  void* A = sizeof(T) == 8 ? h->T64 : h->T32;
  void* Bz = sizeof(T) == 8 ? h->Xp : h->Xp32;
  void* C = sizeof(T) == 8 ? h->LX64 : h->LX32;
  void* Wt = h->Gp;                                // scratch output (c128, large enough)
  const T* Vw = reinterpret_cast<const T*>(sizeof(T) == 8 ? (const void*)h->V64 : (const void*)h->V32);
  unsigned seed = 1;
  for (void* b : {A, Bz, C})
    GPE_HIP(h, launch_single(FillArgs<T>{b, h->nel, seed++}, elementwise_blocks(h->nel), h->st));
  hipEvent_t e0, e1;
  GPE_HIP(h, hipEventCreate(&e0));
  GPE_HIP(h, hipEventCreate(&e1));
  float best = 1e30f;
  int bestv = 1;
  for (int v = 0; v < nv; ++v) {
    int nb = 0;
    GPE_HIP(h, hvp_xpass<T>(h->F, h->ax[0], h->npts, A, Bz, C, Vw, Wt, h->pw, h->part, h->pstride, &nb, v, nullptr,
                            h->st));
    float tmin = 1e30f;
    for (int rep = 0; rep < 3; ++rep) {
      GPE_HIP(h, hipEventRecord(e0, h->st));
      GPE_HIP(h, hvp_xpass<T>(h->F, h->ax[0], h->npts, A, Bz, C, Vw, Wt, h->pw, h->part, h->pstride, &nb, v,
                              nullptr, h->st));
      GPE_HIP(h, hipEventRecord(e1, h->st));
      GPE_HIP(h, hipEventSynchronize(e1));
      float ms = 0.f;
      GPE_HIP(h, hipEventElapsedTime(&ms, e0, e1));
      tmin = std::fmin(tmin, ms);
    }
    h->xvar_us[v] = 1e3f * tmin;
    if (tmin < best) {
      best = tmin;
      bestv = v;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  h->xvar = bestv;
  return GPE_OK;
}

gpe_status tune_xpass(gpe_handle* h) {
  return h->prec == GPE_FP64 ? tune_xpass_t<double>(h) : tune_xpass_t<float>(h);
}

PwParams hvp_params(const gpe_handle* h, bool riem, double sigma) {
  PwParams p = h->pw;
  for (int i = 0; i < 7; ++i) p.zc[i] = (riem && i < h->K) ? sigma - h->alpha_g - h->beta_g * (h->F - i) : 0.0;
  return p;
}

gpe_status hvp_enq(gpe_handle* h, const void* Z, void* HZ, bool riem, double sigma, bool cg, bool kappa) {
  if (!h->has_point) return fail(h, GPE_EINVAL, "gpe_hvp before gpe_set_point");
  if (cg && !riem) return fail(h, GPE_EINVAL, "the device-resident CG takes the Riemannian HVP");
  const PwParams p = hvp_params(h, riem, sigma);
  if (!work32(h)) return hvp_t<double>(h, Z, HZ, riem, p, cg, kappa);
  return hvp_t<float>(h, Z, HZ, riem, p, cg, kappa);
}

gpe_status hvp_read(gpe_handle* h, double* kappa, double* zz) {
  GPE_TRY(finite(h, h->hres + 34, 2, "the Hessian-vector product"));
  if (kappa) *kappa = h->hres[34];
  if (zz) *zz = h->hres[35];
  return GPE_OK;
}

gpe_status hvp(gpe_handle* h, const void* Z, void* HZ, bool riem, double sigma, double* kappa, double* zz) {
  GPE_TRY(hvp_enq(h, Z, HZ, riem, sigma, false, kappa || zz));
  if (!kappa && !zz) return GPE_OK;
  GPE_TRY(fetch(h));
  return hvp_read(h, kappa, zz);
}

gpe_status norms_enq(gpe_handle* h, const void* u, const void* xi, bool xi32) {
  if (xi32)
    GPE_KT(h, KK_NORMS, (comp_norms<double, float>(h->K, u, xi, h->part, h->nblk, h->npts, h->st)));
  else
    GPE_KT(h, KK_NORMS, (comp_norms<double, double>(h->K, u, xi, h->part, h->nblk, h->npts, h->st)));
  // without xi only the K slots of ||u_i||^2 are written, so only they are summed
  return finalize_enq(h, xi ? 3 * h->K : h->K, POST_NONE, nullptr);
}

gpe_status norms_read(gpe_handle* h, bool has_xi, RetractNorms* rn) {
  const int K = h->K;
  GPE_TRY(finite(h, h->hres, has_xi ? 3 * K : K, "the component norms"));
  for (int i = 0; i < K; ++i) {
    rn->uu[i] = h->hres[i];
    rn->ux[i] = has_xi ? h->hres[K + i] : 0.0;
    rn->xx[i] = has_xi ? h->hres[2 * K + i] : 0.0;
  }
  return GPE_OK;
}

gpe_status retract_norms(gpe_handle* h, const void* u, const void* xi, bool xi32, RetractNorms* rn) {
  GPE_TRY(norms_enq(h, u, xi, xi32));
  GPE_TRY(fetch(h));
  return norms_read(h, xi != nullptr, rn);
}

gpe_status retraction_sigma(gpe_handle* h, const double* a, int kind, double* sig) {
  int r;
  switch (kind) {
    case GPE_R1_PROJECTIVE: r = sigma_projective(h->F, h->M, a, sig); break;
    case GPE_R2_ORTHOGONAL: r = sigma_orthogonal(h->F, h->M, a, sig); break;
    case GPE_R3_CLOSED: r = sigma_closed(h->F, h->M, a, sig); break;
    default: return fail(h, GPE_EINVAL, "unknown retraction kind");
  }
  if (r != SIGMA_OK)
    return fail(h, GPE_EDOMAIN, kind == GPE_R3_CLOSED ? "retraction argument outside S"
                                                      : "retraction argument outside Omega");
  return GPE_OK;
}

gpe_status proj_coeffs(gpe_handle* h, const RetractNorms& rn, double* alpha, double* beta) {
  double a11 = 0, a12 = 0, a22 = 0, r1 = 0, r2 = 0;
  for (int i = 0; i < h->K; ++i) {
    const double l = h->F - i;
    a11 += rn.uu[i];
    a12 += l * rn.uu[i];
    a22 += l * l * rn.uu[i];
    r1 += rn.ux[i];
    r2 += l * rn.ux[i];
  }
  const double det = a11 * a22 - a12 * a12;
  if (!(det > 0)) return fail(h, GPE_EDEGEN, "degenerate Gram system in the projection");
  *alpha = (a22 * r1 - a12 * r2) / det;
  *beta = (a11 * r2 - a12 * r1) / det;
  return GPE_OK;
}

gpe_status retract_sigma_at(gpe_handle* h, const RetractNorms& rn, double t, int kind, double* sig) {
  double a[7];
  for (int i = 0; i < h->K; ++i) {
    a[i] = rn.uu[i] + 2.0 * t * rn.ux[i] + t * t * rn.xx[i];   // ||u_i + t xi_i||^2
    if (a[i] < 0) a[i] = 0;
  }
  return retraction_sigma(h, a, kind, sig);
}

gpe_status retract_apply(gpe_handle* h, const RetractNorms& rn, const void* u, const void* xi, bool xi32, double t,
                         int kind, void* out) {
  double sig[7];
  GPE_TRY(retract_sigma_at(h, rn, t, kind, sig));
  if (xi32)
    GPE_KT(h, KK_SCALE, (scale_comps<double, float, double>(h->K, u, xi, t, sig, out, h->npts, h->st)));
  else
    GPE_KT(h, KK_SCALE, (scale_comps<double, double, double>(h->K, u, xi, t, sig, out, h->npts, h->st)));
  return GPE_OK;
}

gpe_status dot_enq(gpe_handle* h, const void* a, bool a32, const void* b, bool b32, size_t n) {
  if (!a32 && !b32) GPE_KT(h, KK_VECTOR, (dot<double, double>(a, b, h->part, h->nblk, n, h->st)));
  else if (a32 && b32) GPE_KT(h, KK_VECTOR, (dot<float, float>(a, b, h->part, h->nblk, n, h->st)));
  else if (!a32 && b32) GPE_KT(h, KK_VECTOR, (dot<double, float>(a, b, h->part, h->nblk, n, h->st)));
  else GPE_KT(h, KK_VECTOR, (dot<double, float>(b, a, h->part, h->nblk, n, h->st)));
  return finalize_enq(h, 1, POST_NONE, nullptr);
}

gpe_status dot_read(gpe_handle* h, double* out) {
  GPE_TRY(finite(h, h->hres, 1, "an inner product"));
  *out = h->hres[0];
  return GPE_OK;
}

gpe_status dot_host(gpe_handle* h, const void* a, bool a32, const void* b, bool b32, size_t n, double* out) {
  GPE_TRY(dot_enq(h, a, a32, b, b32, n));
  GPE_TRY(fetch(h));
  return dot_read(h, out);
}

gpe_status cg_init_enq(gpe_handle* h, double tol, double eps, int maxit) {
  GPE_KT(h, KK_VECTOR, launch_single(CgInitArgs{h->res, tol, eps, maxit}, 1, h->st));
  return GPE_OK;
}

// Small fields: the CG's closing step applies the residual and cap tests from
// the update's partials itself (every one of its workgroups sums them), and
// the update needs no finalize launch.
bool cg_local_step(const gpe_handle* h) {
  return h->nblk <= 256 && (size_t)h->nblk * (size_t)elementwise_blocks(h->nel) <= (size_t)1 << 20;
}

template <typename T>
static gpe_status cg_step_t(gpe_handle* h, const void* p, const void* q, void* z, void* r) {
  CgArgs<T> a{p, q, z, r, h->part, 0.0, h->nel};
  a.adev = h->res + CG_ALPHA;
  a.skip = h->res + CG_DONE;
  GPE_KT(h, KK_VECTOR, launch_single(a, h->nblk, h->st));
  if (cg_local_step(h)) return GPE_OK;
  SlotCounts nb;
  for (int k = 0; k < kMaxQ; ++k) nb.nb[k] = h->nblk;
  GPE_KT(h, KK_FINALIZE, finalize(h->part, h->nblk, nb, 1, h->res, POST_CG_STEP, h->F, nullptr, h->ticket,
                                  h->res + CG_DONE, h->st));
  return GPE_OK;
}

template <typename T>
static gpe_status cg_dir_t(gpe_handle* h, const void* r, void* p, void* z, int iter) {
  CgDirArgs<T> a{r, p, z, h->res, iter, h->nel};
  if (cg_local_step(h)) {
    a.part = h->part;
    a.nb = h->nblk;
  }
  GPE_KT(h, KK_VECTOR, launch_single(a, elementwise_blocks(h->nel), h->st));
  return GPE_OK;
}

gpe_status cg_dir_enq(gpe_handle* h, const void* r, void* p, void* z, int iter) {
  return work32(h) ? cg_dir_t<float>(h, r, p, z, iter) : cg_dir_t<double>(h, r, p, z, iter);
}

gpe_status cg_step_enq(gpe_handle* h, const void* p, const void* q, void* z, void* r) {
  return work32(h) ? cg_step_t<float>(h, p, q, z, r) : cg_step_t<double>(h, p, q, z, r);
}


gpe_status cg_state_read(gpe_handle* h, CgState* cs) {
  const double* c = h->hres;
  cs->done = c[CG_DONE] != 0.0;
  cs->reason = (int)c[CG_REASON];
  cs->iters = (int)c[CG_IT];
  cs->kappa = c[CG_KAPPA];
  cs->pp = c[CG_PP];
  if (cs->done && cs->reason == CG_STOP_CURVATURE) GPE_TRY(finite(h, c + CG_KAPPA, 2, "the CG curvature"));
  GPE_TRY(finite(h, c + CG_RR, 1, "the CG residual"));
  GPE_TRY(finite(h, c + CG_RR1, 1, "the CG residual"));
  return GPE_OK;
}

// Interpolation matrix of the Fourier interpolant from n nodes to the 2n nodes
// of the refined axis: P[j'][k] = (1/n) sum_{p=-n/2}^{n/2} c_p e^{i 2 pi p (j'/(2n) - k/n)},
// c_{+-n/2} = 1/2 (real: the sum pairs p and -p).
static std::vector<double> interp_matrix(int n) {
  std::vector<double> P((size_t)2 * n * n);
  for (int jp = 0; jp < 2 * n; ++jp)
    for (int k = 0; k < n; ++k) {
      const double th = M_PI * (double)(jp - 2 * k) / (double)n;
      double s = 1.0 + std::cos(0.5 * n * th);
      for (int p = 1; p < n / 2; ++p) s += 2.0 * std::cos(p * th);
      P[(size_t)jp * n + k] = s / n;
    }
  return P;
}

gpe_status prolong(const gpe_handle* c, const void* Xc, gpe_handle* f, void* Xf) {
  if (c->F != f->F || c->dim != f->dim) return fail(f, GPE_EINVAL, "prolong: problems differ");
  for (int a = 0; a < c->dim; ++a)
    if (f->n[a] != 2 * c->n[a]) return fail(f, GPE_EINVAL, "prolong: fine grid must have 2n points per axis");
  // ping-pong through the fine handle's scratch (T64, Gp); the set point is lost
  f->has_point = false;
  const void* src = Xc;
  size_t sizes[3] = {(size_t)c->n[0], (size_t)c->n[1], (size_t)c->n[2]};
  std::vector<double*> mats;
  gpe_status rs = GPE_OK;
  for (int a = 0; a < c->dim && rs == GPE_OK; ++a) {
    const int n = c->n[a];
    std::vector<double> P = interp_matrix(n);
    double* dP = nullptr;
    rs = alloc_field(f, (void**)&dP, P.size() * sizeof(double));
    if (rs != GPE_OK) break;
    mats.push_back(dP);
    hipError_t e = hipMemcpyAsync(dP, P.data(), P.size() * sizeof(double), hipMemcpyHostToDevice, f->st);
    if (e == hipSuccess) e = hipStreamSynchronize(f->st);   // P is a stack vector
    if (e != hipSuccess) { rs = hip_fail(f, e, "copy interpolation matrix"); break; }
    size_t inner = 1, outer = (size_t)c->K;
    for (int b = 0; b < a; ++b) inner *= sizes[b];
    for (int b = a + 1; b < c->dim; ++b) outer *= sizes[b];
    const bool last = a == c->dim - 1;
    void* dst = last ? Xf : (a == 0 ? f->T64 : f->Gp);
    const double scale = last ? std::pow(2.0, -0.5 * c->dim) : 1.0;
    e = prolong_axis(src, dst, dP, n, inner, outer, scale, f->st);
    if (e != hipSuccess) { rs = hip_fail(f, e, "prolong_axis"); break; }
    sizes[a] = 2 * (size_t)n;
    src = dst;
  }
  hipError_t e = hipStreamSynchronize(f->st);
  for (double* m : mats) (void)hipFree(m);
  if (rs != GPE_OK) return rs;
  if (e != hipSuccess) return hip_fail(f, e, "prolong sync");
  return GPE_OK;
}

}  // namespace gpe

using namespace gpe;

// ----------------------------------------------------------------- C ABI


// Validation of a problem statement (gpe_problem's contract); "" if valid.
static std::string problem_error(const gpe_problem* pr) {
  if (pr->F < 1 || pr->F > 3) return "F must be 1, 2 or 3";
  if (pr->dim < 1 || pr->dim > 3) return "dim must be 1, 2 or 3";
  if (!(std::fabs(pr->M) < pr->F)) return "|M| must be < F";
  if (pr->M < 0) return "M < 0: reverse the component order and pass -M";
  for (int a = 0; a < pr->dim; ++a) {
    const int n = pr->n[a];
    if (!lap_size_supported(n))
      return "n[" + std::to_string(a) + "] = " + std::to_string(n) + " unsupported (2^k or 3*2^k, 4..512)";
    if (!(pr->hi[a] > pr->lo[a])) return "empty box";
  }
  return "";
}

// ----------------------------------------------------------------- scratch of gpe_retract_noalloc
// The retraction's partial sums (3K slots of at most kMaxRedBlocks workgroups),
// the finalize's results and its ticket, for every admissible problem.  One
// copy per GPU, at a device address found once per device.
namespace {
constexpr size_t kNaPart = 3 * 7 * (size_t)kMaxRedBlocks;
constexpr size_t kNaRes = 64;
constexpr size_t kNaDoubles = kNaPart + kNaRes + 2;   // + the ticket (first 4 bytes of the last 16)
constexpr int kNaMaxDevices = 64;
}  // namespace
static __device__ __align__(256) double scratch[kNaDoubles];
static double* g_scratch_ptr[kNaMaxDevices];
static std::mutex g_scratch_mu;

// Device address of `scratch` on the current device (resolved once per device).
static gpe_status scratch_on_device(double** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(nullptr, e, "hipGetDevice");
  if (dev < 0 || dev >= kNaMaxDevices) return fail(nullptr, GPE_EINVAL, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return hip_fail(nullptr, e != hipSuccess ? e : hipErrorInvalidSymbol,
                                               "hipGetSymbolAddress(scratch)");
    g_scratch_ptr[dev] = static_cast<double*>(p);
  }
  *out = g_scratch_ptr[dev];
  return GPE_OK;
}

extern "C" {

const char* gpe_version(void) { return "gpe 0.1 (gfx950)"; }

void gpe_solve_opts_default(gpe_solve_opts* o) {
  if (!o) return;
  o->tol = 1e-6;
  o->maxit = 10000;
  o->retraction = GPE_R1_PROJECTIVE;
  o->rgbb_tol = 1e-2;
  o->rgbb_maxit = 2000;
  o->rgbb_rho = 1e-4;
  o->rgbb_delta = 0.2;
  o->rgbb_varrho = 0.85;
  o->rgbb_step0 = 0.1;
  o->eta1 = 0.01;
  o->eta2 = 0.9;
  o->gamma0 = 0.2;
  o->gamma1 = 1.0;
  o->gamma2 = 10.0;
  o->sigma_hat0 = 1.0;
  o->rho = 1e-4;
  o->delta = 0.2;
  o->alpha0 = 1.0;
  o->ls_max = 30;
  o->cg_maxit = 500;
  o->cg_T = 0.1;
  o->cg_theta = 1.0;
  o->max_reject_streak = 30;
  o->sigma_hat_min = 1e-8;
  o->verbose = 0;
  o->time_limit = 0.0;
  o->mg_levels = 0;
  o->mg_coarse_tol = 1e-5;
  o->polish_tol = 0.0;
  o->polish_window = 0;
  o->cg_per_digit = 80.0;
  o->trace = nullptr;
  o->trace_cap = 0;
}

const char* gpe_last_error(const gpe_handle* h) { return h ? h->err.c_str() : g_create_error.c_str(); }

gpe_status gpe_destroy(gpe_handle* h) {
  if (!h) return GPE_OK;
  (void)hipSetDevice(h->device);
  if (h->st) (void)hipStreamSynchronize(h->st);
  if (!h->res_shared) {
    if (h->res) (void)hipFree(h->res);
    if (h->hres) (void)hipHostFree(h->hres);
  }
  void* bufs[] = {h->ticket, h->V64, h->V32, h->part, h->gram_pt, h->gram_tmp, h->T64, h->T32, h->Xp, h->Gp, h->Xp32,
                  h->LX64, h->LX32,
                  h->tw[0], h->tw[1], h->tw[2], h->tw[3], h->tw[4], h->tw[5]};
  for (void* b : bufs)
    if (b) (void)hipFree(b);
  for (void* b : h->solver_bufs)
    if (b) (void)hipFree(b);
  for (auto& r : h->recs) {
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  for (auto e : h->event_pool) (void)hipEventDestroy(e);
  delete h;
  return GPE_OK;
}

gpe_status gpe_create(const gpe_problem* pr, const double* V, int precision, void* stream, gpe_handle** out) {
  if (!out) return fail(nullptr, GPE_EINVAL, "out is NULL");
  *out = nullptr;
  if (!pr || !V) return fail(nullptr, GPE_EINVAL, "problem or potential is NULL");
  if (precision != GPE_FP64 && precision != GPE_MIXED) return fail(nullptr, GPE_EINVAL, "bad precision");
  {
    const std::string err = problem_error(pr);
    if (!err.empty()) return fail(nullptr, GPE_EINVAL, err);
  }
  gpe_handle* h = new gpe_handle();
  h->prob = *pr;
  h->F = pr->F;
  h->K = 2 * pr->F + 1;
  h->dim = pr->dim;
  h->prec = precision;
  h->st = reinterpret_cast<hipStream_t>(stream);
  h->p = pr->p;
  h->q = pr->q;
  h->M = pr->M;
  for (int k = 0; k < 4; ++k) h->beta[k] = pr->beta[k];
  if (h->F < 3) h->beta[3] = 0;
  if (h->F < 2) h->beta[2] = 0;
  h->npts = 1;
  h->h = 1.0;
  for (int a = 0; a < h->dim; ++a) {
    h->n[a] = pr->n[a];
    h->lo[a] = pr->lo[a];
    h->hi[a] = pr->hi[a];
    h->npts *= (size_t)pr->n[a];
    h->h *= (pr->hi[a] - pr->lo[a]) / pr->n[a];
  }
  h->nel = h->npts * h->K;
  (void)hipGetDevice(&h->device);
  {
    // V may live in host or device memory: a device (or managed) pointer is
    // copied to the host mirror first; anything else is read as host memory
    hipPointerAttribute_t attr;
    bool on_device = false;
    if (hipPointerGetAttributes(&attr, V) == hipSuccess)
      on_device = attr.type == hipMemoryTypeDevice || attr.type == hipMemoryTypeManaged;
    else
      (void)hipGetLastError();
    h->Vhost.resize(h->npts);
    if (on_device) {
      const hipError_t ev = hipMemcpy(h->Vhost.data(), V, h->npts * sizeof(double), hipMemcpyDeviceToHost);
      if (ev != hipSuccess) {
        hip_fail(h, ev, "copy of the device potential");
        g_create_error = h->err;
        delete h;
        return GPE_EHIP;
      }
    } else {
      std::memcpy(h->Vhost.data(), V, h->npts * sizeof(double));
    }
  }
  const double* V_host = h->Vhost.data();

  // pointwise constants
  for (int i = 0; i < 7; ++i) {
    const double l = h->F - i;
    h->pw.zee[i] = i < h->K ? -h->p * l + h->q * l * l : 0.0;
    h->pw.zc[i] = 0.0;
  }
  for (int k = 0; k < 4; ++k) {
    h->pw.g[k] = 2.0 * h->beta[k] / h->h;
    h->pw.e[k] = h->beta[k] / (2.0 * h->h);
  }
  h->nblk = red_blocks(h->npts);

  gpe_status s;
#define GPE_ALLOC(ptr, bytes)                                              \
  do {                                                                     \
    s = alloc_field(h, (void**)&(ptr), (bytes));                           \
    if (s != GPE_OK) { g_create_error = h->err; gpe_destroy(h); return s; } \
  } while (0)
  const size_t f64 = h->nel * 16, f32 = h->nel * 8;
  GPE_ALLOC(h->V64, h->npts * sizeof(double));
  {
    size_t ps = kMaxRedBlocks;
    size_t inner = 1;
    for (int a = 0; a < h->dim; ++a) {
      LapAxis ax;
      ax.n = pr->n[a];
      ax.inner = (int)inner;
      ax.nlines = (long)(h->nel / pr->n[a]);
      const size_t m = lap_max_blocks(ax, h->K);
      if (m > ps) ps = m;
      inner *= (size_t)pr->n[a];
    }
    h->pstride = ps;
  }
  GPE_ALLOC(h->part, sizeof(double) * kMaxQ * h->pstride);
  GPE_ALLOC(h->res, sizeof(double) * kResDoubles);
  GPE_ALLOC(h->gram_pt, sizeof(double) * 8);
  GPE_ALLOC(h->gram_tmp, sizeof(double) * 8);
  GPE_ALLOC(h->ticket, sizeof(unsigned int) * 4);
  GPE_ALLOC(h->T64, f64);
  GPE_ALLOC(h->Xp, f64);
  GPE_ALLOC(h->Gp, f64);
  if (precision == GPE_FP64) GPE_ALLOC(h->LX64, f64);
  if (precision == GPE_MIXED) {
    GPE_ALLOC(h->LX32, f32);
    GPE_ALLOC(h->V32, h->npts * sizeof(float));
    GPE_ALLOC(h->T32, f32);
    GPE_ALLOC(h->Xp32, f32);
  }
  if (hipHostMalloc((void**)&h->hres, sizeof(double) * kResDoubles, hipHostMallocDefault) != hipSuccess) {
    g_create_error = "pinned host allocation failed";
    gpe_destroy(h);
    return GPE_ENOMEM;
  }
  auto bail = [&](hipError_t e, const char* w) {
    hip_fail(h, e, w);
    g_create_error = h->err;
    gpe_destroy(h);
    return GPE_EHIP;
  };
  hipError_t e = hipMemsetAsync(h->ticket, 0, sizeof(unsigned int) * 4, h->st);
  if (e != hipSuccess) return bail(e, "clear ticket");
  e = hipMemcpyAsync(h->V64, V_host, h->npts * sizeof(double), hipMemcpyHostToDevice, h->st);
  if (e != hipSuccess) return bail(e, "copy V");
  if (precision == GPE_MIXED) {
    std::vector<float> v32(h->npts);
    for (size_t j = 0; j < h->npts; ++j) v32[j] = (float)V_host[j];
    e = hipMemcpyAsync(h->V32, v32.data(), h->npts * sizeof(float), hipMemcpyHostToDevice, h->st);
    if (e != hipSuccess) return bail(e, "copy V32");
    e = hipStreamSynchronize(h->st);
    if (e != hipSuccess) return bail(e, "sync");
  }
  // Laplacian axes: axis a has lines of length n[a] at stride prod_{b<a} n[b]
  size_t inner = 1;
  for (int a = 0; a < h->dim; ++a) {
    const int n = h->n[a];
    LapAxis& ax = h->ax[a];
    ax.n = n;
    ax.inner = (int)inner;
    ax.nlines = (long)(h->nel / n);
    ax.lamc = 2.0 * M_PI / (h->hi[a] - h->lo[a]);
    std::vector<double> t64(2 * n);
    std::vector<float> t32(2 * n);
    for (int m = 0; m < n; ++m) {
      // exp(-2 pi i m / n), argument reduced exactly through m/n
      const double ang = -2.0 * M_PI * (double)m / (double)n;
      t64[2 * m] = std::cos(ang);
      t64[2 * m + 1] = std::sin(ang);
      t32[2 * m] = (float)t64[2 * m];
      t32[2 * m + 1] = (float)t64[2 * m + 1];
    }
    GPE_ALLOC(h->tw[2 * a], n * 16);
    GPE_ALLOC(h->tw[2 * a + 1], n * 8);
    e = hipMemcpy(h->tw[2 * a], t64.data(), n * 16, hipMemcpyHostToDevice);
    if (e != hipSuccess) return bail(e, "copy twiddles");
    e = hipMemcpy(h->tw[2 * a + 1], t32.data(), n * 8, hipMemcpyHostToDevice);
    if (e != hipSuccess) return bail(e, "copy twiddles");
    ax.tw64 = h->tw[2 * a];
    ax.tw32 = h->tw[2 * a + 1];
    inner *= (size_t)n;
  }
#undef GPE_ALLOC
  e = hipStreamSynchronize(h->st);
  if (e != hipSuccess) return bail(e, "sync");
  if (tune_xpass(h) != GPE_OK) {
    g_create_error = h->err;
    gpe_destroy(h);
    return GPE_EHIP;
  }
  *out = h;
  return GPE_OK;
}

gpe_status gpe_energy(gpe_handle* h, const void* X, double* E) {
  if (!h || !X || !E) return fail(h, GPE_EINVAL, "NULL argument");
  return eval_point(h, X, nullptr, nullptr, E, nullptr, nullptr);
}

gpe_status gpe_grad(gpe_handle* h, const void* X, void* G, int riemannian, double* E, double* gnorm) {
  if (!h || !X || !G) return fail(h, GPE_EINVAL, "NULL argument");
  if (X == G) return fail(h, GPE_EINVAL, "X and G must be distinct");
  double e, ag, bg;
  GPE_TRY(eval_point(h, X, G, h->gram_tmp, &e, &ag, &bg));
  if (E) *E = e;
  if (riemannian) {
    double gn;
    GPE_TRY(project_grad(h, X, G, G, ag, bg, &gn));
    if (gnorm) *gnorm = gn;
  } else if (gnorm) {
    double g2;
    GPE_TRY(dot_host(h, G, false, G, false, h->nel, &g2));
    *gnorm = std::sqrt(g2);
  }
  return GPE_OK;
}

gpe_status gpe_set_point(gpe_handle* h, const void* X) {
  if (!h || !X) return fail(h, GPE_EINVAL, "NULL argument");
  GPE_HIP(h, hipMemcpyAsync(h->Xp, X, h->nel * 16, hipMemcpyDeviceToDevice, h->st));
  GPE_TRY(eval_point(h, h->Xp, h->Gp, h->gram_pt, &h->E_pt, &h->alpha_g, &h->beta_g));
  return adopt_point(h);
}

gpe_status gpe_hvp(gpe_handle* h, const void* Z, void* HZ, int riemannian, double sigma) {
  if (!h || !Z || !HZ) return fail(h, GPE_EINVAL, "NULL argument");
  if (Z == HZ) return fail(h, GPE_EINVAL, "Z and HZ must be distinct");
  return hvp(h, Z, HZ, riemannian != 0, sigma, nullptr, nullptr);
}

gpe_status gpe_hvp_dot(gpe_handle* h, const void* Z, void* HZ, double sigma, double* kappa) {
  if (!h || !Z || !HZ || !kappa) return fail(h, GPE_EINVAL, "NULL argument");
  if (Z == HZ) return fail(h, GPE_EINVAL, "Z and HZ must be distinct");
  return hvp(h, Z, HZ, true, sigma, kappa, nullptr);
}

gpe_status gpe_retract(gpe_handle* h, const void* X, const void* Xi, double t, int kind, void* Xout) {
  if (!h || !X || !Xout) return fail(h, GPE_EINVAL, "NULL argument");
  RetractNorms rn;
  GPE_TRY(retract_norms(h, X, Xi, false, &rn));
  GPE_TRY(retract_apply(h, rn, X, Xi, false, Xi ? t : 0.0, kind, Xout));
  GPE_HIP(h, hipStreamSynchronize(h->st));
  return GPE_OK;
}

gpe_status gpe_constraints(gpe_handle* h, const void* X, double* mass, double* mag) {
  if (!h || !X) return fail(h, GPE_EINVAL, "NULL argument");
  RetractNorms rn;
  GPE_TRY(retract_norms(h, X, nullptr, false, &rn));
  double m = 0, g = 0;
  for (int i = 0; i < h->K; ++i) {
    m += rn.uu[i];
    g += (h->F - i) * rn.uu[i];
  }
  if (mass) *mass = m;
  if (mag) *mag = g;
  return GPE_OK;
}

gpe_status gpe_project(gpe_handle* h, const void* X, const void* W, void* out) {
  if (!h || !X || !W || !out) return fail(h, GPE_EINVAL, "NULL argument");
  RetractNorms rn;
  GPE_TRY(retract_norms(h, X, W, false, &rn));
  double alpha, beta;
  GPE_TRY(proj_coeffs(h, rn, &alpha, &beta));
  double gn;
  GPE_TRY(project_grad(h, X, W, out, alpha, beta, &gn));
  return GPE_OK;
}

gpe_status gpe_prolong(const gpe_handle* coarse, const void* Xc, gpe_handle* fine, void* Xf) {
  if (!coarse || !fine || !Xc || !Xf) return fail(fine, GPE_EINVAL, "NULL argument");
  return gpe::prolong(coarse, Xc, fine, Xf);
}

gpe_status gpe_schedule(const gpe_handle* h, int* xpass_variant, float* variant_us, int nvariants) {
  if (!h) return fail(nullptr, GPE_EINVAL, "NULL handle");
  if (xpass_variant) *xpass_variant = h->xvar;
  for (int v = 0; v < nvariants && v < 3; ++v)
    if (variant_us) variant_us[v] = h->xvar_us[v];
  return GPE_OK;
}

gpe_status gpe_set_schedule(gpe_handle* h, int xpass_variant) {
  if (!h) return fail(nullptr, GPE_EINVAL, "NULL handle");
  const int nv = xpass_variants(h->n[0]);
  if (xpass_variant < 0 || xpass_variant >= nv)
    return fail(h, GPE_EINVAL, "x-pass variant " + std::to_string(xpass_variant) + " out of range: this grid has " +
                                   std::to_string(nv));
  h->xvar = xpass_variant;
  return GPE_OK;
}

gpe_status gpe_schedule_count(const gpe_handle* h, int* nvariants) {
  if (!h || !nvariants) return fail(nullptr, GPE_EINVAL, "NULL argument");
  *nvariants = xpass_variants(h->n[0]);
  return GPE_OK;
}

gpe_status gpe_timing_enable(gpe_handle* h, int enable) {
  if (!h) return fail(h, GPE_EINVAL, "NULL handle");
  GPE_HIP(h, hipStreamSynchronize(h->st));
  for (auto& r : h->recs) {
    h->event_pool.push_back(r.a);
    h->event_pool.push_back(r.b);
  }
  h->recs.clear();
  h->timing = enable != 0;
  return GPE_OK;
}

gpe_status gpe_timing_read(gpe_handle* h, int max, const char** names, int* counts, double* ms, int* nkinds) {
  if (!h) return fail(h, GPE_EINVAL, "NULL handle");
  GPE_HIP(h, hipStreamSynchronize(h->st));
  double tot[KK_COUNT] = {0};
  int cnt[KK_COUNT] = {0};
  for (auto& r : h->recs) {
    float t = 0.f;
    GPE_HIP(h, hipEventElapsedTime(&t, r.a, r.b));
    tot[r.kind] += t;
    cnt[r.kind] += 1;
  }
  int k = 0;
  for (int i = 0; i < KK_COUNT; ++i) {
    if (!cnt[i]) continue;
    if (k < max) {
      if (names) names[k] = kKernelNames[i];
      if (counts) counts[k] = cnt[i];
      if (ms) ms[k] = tot[i];
    }
    ++k;
  }
  if (nkinds) *nkinds = k;
  return GPE_OK;
}

gpe_status gpe_retract_noalloc(const gpe_problem* pr, const void* X, const void* Xi, double t, int kind, void* Xout,
                               void* stream) {
  if (!pr || !X || !Xout) return fail(nullptr, GPE_EINVAL, "NULL argument");
  {
    const std::string err = problem_error(pr);
    if (!err.empty()) return fail(nullptr, GPE_EINVAL, err);
  }
  if (kind != GPE_R1_PROJECTIVE && kind != GPE_R2_ORTHOGONAL && kind != GPE_R3_CLOSED)
    return fail(nullptr, GPE_EINVAL, "unknown retraction kind");
  const int F = pr->F, K = 2 * F + 1;
  size_t npts = 1;
  for (int a = 0; a < pr->dim; ++a) npts *= (size_t)pr->n[a];
  const int nblk = red_blocks(npts);
  const int nq = Xi ? 3 * K : K;   // without Xi the norms kernel writes the K slots of ||X_i||^2 only
  if ((size_t)3 * K * (size_t)nblk > kNaPart) return fail(nullptr, GPE_EINVAL, "problem exceeds the static scratch");
  double* base = nullptr;
  GPE_TRY(scratch_on_device(&base));
  double* part = base;
  double* res = base + kNaPart;
  unsigned int* ticket = reinterpret_cast<unsigned int*>(base + kNaPart + kNaRes);
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
#define NA_HIP(call)                                                  \
  do {                                                                \
    hipError_t e_ = (call);                                           \
    if (e_ != hipSuccess) return hip_fail(nullptr, e_, #call);        \
  } while (0)
  // the ticket starts at 0 (a finalize leaves it there; an interrupted call might not)
  NA_HIP(hipMemsetAsync(ticket, 0, sizeof(unsigned int), st));
  NA_HIP((comp_norms<double, double>(K, X, Xi, part, nblk, npts, st)));
  SlotCounts nb;
  for (int q = 0; q < kMaxQ; ++q) nb.nb[q] = nblk;
  NA_HIP(finalize(part, nblk, nb, nq, res, POST_NONE, F, nullptr, ticket, nullptr, st));
  double r[3 * 7];
  NA_HIP(hipMemcpyAsync(r, res, sizeof(double) * nq, hipMemcpyDeviceToHost, st));
  NA_HIP(hipStreamSynchronize(st));
  for (int i = 0; i < nq; ++i)
    if (!std::isfinite(r[i])) return fail(nullptr, GPE_ENUMERIC, "NaN or Inf in the component norms");
  double a[7], sig[7];
  for (int i = 0; i < K; ++i) {
    const double ux = Xi ? r[K + i] : 0.0, xx = Xi ? r[2 * K + i] : 0.0;
    a[i] = r[i] + 2.0 * t * ux + t * t * xx;   // ||u_i + t xi_i||^2
    if (a[i] < 0) a[i] = 0;
  }
  const int rs = kind == GPE_R1_PROJECTIVE ? sigma_projective(F, pr->M, a, sig)
               : kind == GPE_R2_ORTHOGONAL ? sigma_orthogonal(F, pr->M, a, sig)
                                           : sigma_closed(F, pr->M, a, sig);
  if (rs != SIGMA_OK)
    return fail(nullptr, GPE_EDOMAIN, kind == GPE_R3_CLOSED ? "retraction argument outside S"
                                                            : "retraction argument outside Omega");
  NA_HIP((scale_comps<double, double, double>(K, X, Xi, t, sig, Xout, npts, st)));
#undef NA_HIP
  return GPE_OK;
}

gpe_status gpe_newton_solve(gpe_handle* h, void* X, const gpe_solve_opts* opts, gpe_solve_stats* stats) {
  if (!h || !X) return fail(h, GPE_EINVAL, "NULL argument");
  gpe_solve_opts o;
  if (opts) o = *opts;
  else gpe_solve_opts_default(&o);
  gpe_solve_stats s;
  std::memset(&s, 0, sizeof(s));
  gpe_status r = newton_solve(h, X, &o, &s);
  if (stats) *stats = s;
  return r;
}

}  // extern "C"
