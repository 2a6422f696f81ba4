// Batched solves: the lock-step scheduler of sched.h, the executors that turn
// the queued operations of many problems into batched launches, and the
// gpe_batch_* entry points of the C ABI.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "common.h"
#include "sched.h"

struct gpe_batch {
  std::vector<gpe_handle*> hs;
  hipStream_t st = nullptr;
  int F = 0, dim = 0, prec = GPE_FP64;
  double* res = nullptr;    // hs.size() * kResDoubles, the handles' res slices
  double* hres = nullptr;   // pinned mirror, the handles' hres slices
  gpe::Stager sg;
  int xvar = 1;             // schedule variant of the batched fused x pass (autotuned)
  float xvar_us[3] = {0, 0, 0};
  std::string err;
};

namespace gpe {

namespace {

constexpr size_t kAlign = 256;

struct Item {
  Ctx* c;
  Req* r;
};

// --------------------------------------------------------------- launch helpers
// Stage one record per problem plus the workgroup offsets and launch.
template <typename A, typename Fn>
gpe_status launch_records(gpe_batch* b, const std::vector<A>& recs, const std::vector<int>& nblk, Fn&& fn) {
  gpe_handle* h0 = b->hs[0];
  std::vector<int> blk0(recs.size() + 1, 0);
  for (size_t i = 0; i < recs.size(); ++i) {
    if (nblk[i] < 1) return fail(h0, GPE_EINVAL, "batched launch: empty problem");
    blk0[i + 1] = blk0[i] + nblk[i];
  }
  const void* da = nullptr;
  const void* db = nullptr;
  GPE_TRY(b->sg.put2(h0, b->st, recs.data(), sizeof(A) * recs.size(), blk0.data(), sizeof(int) * blk0.size(), &da,
                     &db));
  const Span sp{reinterpret_cast<const int*>(db), (int)recs.size(), blk0.back()};
  GPE_HIP(h0, fn(reinterpret_cast<const A*>(da), sp));
  return GPE_OK;
}

template <typename A>
gpe_status ops(gpe_batch* b, const std::vector<A>& recs, const std::vector<int>& nblk) {
  return launch_records(b, recs, nblk, [&](const A* d, const Span& sp) { return launch_batched<A>(d, sp, b->st); });
}

// Finalize records of every problem of g (slot counts checked against the stride).
gpe_status fin_records(gpe_batch* b, const std::vector<Item>& g, int nq, const std::vector<double*>& gram,
                       const std::vector<SlotCounts>& nb, bool pstride, bool cg, std::vector<FinArgs>* recs) {
  gpe_handle* h0 = b->hs[0];
  recs->resize(g.size());
  for (size_t i = 0; i < g.size(); ++i) {
    gpe_handle* h = g[i].c->h;
    const size_t stride = pstride ? h->pstride : (size_t)h->nblk;
    for (int q = 0; q < nq; ++q)
      if (nb[i].nb[q] < 0 || (size_t)nb[i].nb[q] > stride) return fail(h0, GPE_EINVAL, "finalize: slot count");
    (*recs)[i] = FinArgs{h->part, h->res, gram[i], stride, nb[i], cg ? h->res + CG_DONE : nullptr};
  }
  return GPE_OK;
}

gpe_status fin(gpe_batch* b, const std::vector<Item>& g, int nq, int post, const std::vector<double*>& gram,
               const std::vector<SlotCounts>& nb, bool pstride, bool cg = false) {
  gpe_handle* h0 = b->hs[0];
  std::vector<FinArgs> recs;
  GPE_TRY(fin_records(b, g, nq, gram, nb, pstride, cg, &recs));
  const void* d = nullptr;
  GPE_TRY(b->sg.put(h0, b->st, recs.data(), sizeof(FinArgs) * recs.size(), &d));
  GPE_HIP(h0, finalize_batched(reinterpret_cast<const FinArgs*>(d), (int)recs.size(), nq, post, b->F, b->st));
  return GPE_OK;
}

// Workgroup offsets of a batched launch (nblk[i] workgroups for problem i).
gpe_status offsets(gpe_handle* h0, const std::vector<int>& nblk, std::vector<int>* blk0) {
  blk0->assign(nblk.size() + 1, 0);
  for (size_t i = 0; i < nblk.size(); ++i) {
    if (nblk[i] < 1) return fail(h0, GPE_EINVAL, "batched launch: empty problem");
    (*blk0)[i + 1] = (*blk0)[i] + nblk[i];
  }
  return GPE_OK;
}

template <typename A> Stager::Seg seg(const std::vector<A>& v, const void** d) {
  return Stager::Seg{v.data(), sizeof(A) * v.size(), d};
}

SlotCounts all_slots(int v) {
  SlotCounts s;
  for (int q = 0; q < kMaxQ; ++q) s.nb[q] = v;
  return s;
}

// finalize over each problem's nblk reduction workgroups
gpe_status fin_nblk(gpe_batch* b, const std::vector<Item>& g, int nq, int post, const std::vector<double*>& gram,
                    bool cg = false) {
  std::vector<SlotCounts> nb(g.size());
  for (size_t i = 0; i < g.size(); ++i) nb[i] = all_slots(g[i].c->h->nblk);
  return fin(b, g, nq, post, gram, nb, false, cg);
}

std::vector<double*> no_gram(size_t n) { return std::vector<double*>(n, nullptr); }

// work-precision helpers
template <typename T> const void* twid(const LapAxis& ax) { return sizeof(T) == 8 ? ax.tw64 : ax.tw32; }

// Every axis pass of L for each problem: c = L a (precision T), Parseval off.
template <typename T>
gpe_status lap_all(gpe_batch* b, const std::vector<Item>& g, const std::vector<const void*>& in,
                   const std::vector<void*>& out) {
  for (int a = 0; a < b->dim; ++a) {
    std::vector<LapArgs<T>> recs(g.size());
    std::vector<int> nb(g.size());
    for (size_t i = 0; i < g.size(); ++i) {
      const gpe_handle* h = g[i].c->h;
      const LapAxis& ax = h->ax[a];
      recs[i] = LapArgs<T>{in[i], a == 0 ? nullptr : out[i], out[i], twid<T>(ax), nullptr, nullptr, nullptr,
                           ax.lamc, ax.nlines, h->npts, 0, ax.inner, ax.n, nullptr};
      nb[i] = lap_batch_blocks(ax.n, ax.nlines);
    }
    GPE_TRY(launch_records(b, recs, nb, [&](const LapArgs<T>* d, const Span& sp) {
      return lap_batched<T>(d, sp, b->F, 0, b->st);
    }));
  }
  return GPE_OK;
}

// --------------------------------------------------------------- executors
// Each takes a group of problems that queued the same operation (same
// operand precisions); a lone problem takes the single-launch path.

gpe_status ex_eval(gpe_batch* b, std::vector<Item>& g) {
  if (!b || g.size() == 1) {
    for (auto& it : g) GPE_TRY(eval_enq(it.c->h, it.r->a, it.r->c, it.r->gram));
    return GPE_OK;
  }
  std::vector<const void*> in(g.size());
  std::vector<void*> t(g.size());
  for (size_t i = 0; i < g.size(); ++i) {
    in[i] = g[i].r->a;
    t[i] = g[i].c->h->T64;
  }
  GPE_TRY(lap_all<double>(b, g, in, t));
  const bool grad = g[0].r->c != nullptr;
  std::vector<int> nb(g.size());
  for (size_t i = 0; i < g.size(); ++i) nb[i] = g[i].c->h->nblk;
  auto pw = [&](auto tag) -> gpe_status {
    using A = decltype(tag);
    std::vector<A> recs(g.size());
    for (size_t i = 0; i < g.size(); ++i) {
      const gpe_handle* h = g[i].c->h;
      recs[i] = A{g[i].r->a, h->T64, h->V64, g[i].r->c, h->part, h->npts, h->pw};
    }
    return ops(b, recs, nb);
  };
  gpe_status s = GPE_EINVAL;
  switch (b->F * 2 + (grad ? 1 : 0)) {
    case 2: s = pw(PwGradArgs<double, 1, false>{}); break;
    case 3: s = pw(PwGradArgs<double, 1, true>{}); break;
    case 4: s = pw(PwGradArgs<double, 2, false>{}); break;
    case 5: s = pw(PwGradArgs<double, 2, true>{}); break;
    case 6: s = pw(PwGradArgs<double, 3, false>{}); break;
    case 7: s = pw(PwGradArgs<double, 3, true>{}); break;
  }
  GPE_TRY(s);
  std::vector<double*> gram(g.size());
  for (size_t i = 0; i < g.size(); ++i) gram[i] = grad ? g[i].r->gram : nullptr;
  return fin_nblk(b, g, 1 + 2 * (2 * b->F + 1), grad ? POST_GRAD : POST_NONE, gram);
}

gpe_status ex_pgrad(gpe_batch* b, std::vector<Item>& g) {
  if (!b || g.size() == 1) {
    for (auto& it : g) GPE_TRY(pgrad_enq(it.c->h, it.r->a, it.r->b, it.r->c, it.r->s0, it.r->s1));
    return GPE_OK;
  }
  std::vector<ProjArgs<double, double, true>> recs(g.size());
  std::vector<int> nb(g.size());
  for (size_t i = 0; i < g.size(); ++i) {
    const gpe_handle* h = g[i].c->h;
    const Req& r = *g[i].r;
    recs[i] = ProjArgs<double, double, true>{r.a, r.b, r.c, nullptr, r.s0, r.s1, h->part, h->npts, h->F};
    nb[i] = h->nblk;
  }
  GPE_TRY(ops(b, recs, nb));
  return fin_nblk(b, g, 1, POST_NONE, no_gram(g.size()));
}

gpe_status ex_norms(gpe_batch* b, std::vector<Item>& g) {
  if (!b || g.size() == 1) {
    for (auto& it : g) GPE_TRY(norms_enq(it.c->h, it.r->a, it.r->b, it.r->b32));
    return GPE_OK;
  }
  std::vector<int> nb(g.size());
  for (size_t i = 0; i < g.size(); ++i) nb[i] = g[i].c->h->nblk;
  auto run = [&](auto tag) -> gpe_status {
    using A = decltype(tag);
    std::vector<A> recs(g.size());
    for (size_t i = 0; i < g.size(); ++i) recs[i] = A{g[i].r->a, g[i].r->b, g[i].c->h->part, g[i].c->h->npts};
    return ops(b, recs, nb);
  };
  gpe_status s = GPE_EINVAL;
  const bool x32 = g[0].r->b32;
  switch (b->F * 2 + (x32 ? 1 : 0)) {
    case 2: s = run(NormsArgs<double, double, 3>{}); break;
    case 3: s = run(NormsArgs<double, float, 3>{}); break;
    case 4: s = run(NormsArgs<double, double, 5>{}); break;
    case 5: s = run(NormsArgs<double, float, 5>{}); break;
    case 6: s = run(NormsArgs<double, double, 7>{}); break;
    case 7: s = run(NormsArgs<double, float, 7>{}); break;
  }
  GPE_TRY(s);
  // the slots of <u_i, xi_i> and ||xi_i||^2 only where some problem has a xi
  // (a problem without one reads only its ||u_i||^2)
  bool any_xi = false;
  for (auto& it : g) any_xi = any_xi || it.r->b != nullptr;
  return fin_nblk(b, g, (any_xi ? 3 : 1) * (2 * b->F + 1), POST_NONE, no_gram(g.size()));
}

gpe_status ex_scale(gpe_batch* b, std::vector<Item>& g) {
  auto rec = [](const gpe_handle* h, const Req& r, auto tag) {
    using A = decltype(tag);
    A a{r.a, r.b, r.c, r.s0, {0, 0, 0, 0, 0, 0, 0}, h->npts, h->K};
    for (int i = 0; i < 7; ++i) a.s[i] = r.sig[i];
    return a;
  };
  auto run = [&](auto tag) -> gpe_status {
    using A = decltype(tag);
    if (!b || g.size() == 1) {
      for (auto& it : g) {
        gpe_handle* h = it.c->h;
        GPE_KT(h, KK_SCALE, launch_single(rec(h, *it.r, tag), elementwise_blocks(h->nel), h->st));
      }
      return GPE_OK;
    }
    std::vector<A> recs(g.size());
    std::vector<int> nb(g.size());
    for (size_t i = 0; i < g.size(); ++i) {
      recs[i] = rec(g[i].c->h, *g[i].r, tag);
      nb[i] = elementwise_blocks(g[i].c->h->nel);
    }
    return ops(b, recs, nb);
  };
  if (g[0].r->b32) return run(ScaleArgs<double, float, double>{});
  return run(ScaleArgs<double, double, double>{});
}

gpe_status ex_dot(gpe_batch* b, std::vector<Item>& g) {
  if (!b || g.size() == 1) {
    for (auto& it : g) GPE_TRY(dot_enq(it.c->h, it.r->a, it.r->a32, it.r->b, it.r->b32, it.r->n));
    return GPE_OK;
  }
  std::vector<int> nb(g.size());
  for (size_t i = 0; i < g.size(); ++i) nb[i] = g[i].c->h->nblk;
  auto run = [&](auto tag, bool swap) -> gpe_status {
    using A = decltype(tag);
    std::vector<A> recs(g.size());
    for (size_t i = 0; i < g.size(); ++i) {
      const Req& r = *g[i].r;
      recs[i] = swap ? A{r.b, r.a, g[i].c->h->part, r.n} : A{r.a, r.b, g[i].c->h->part, r.n};
    }
    return ops(b, recs, nb);
  };
  const bool a32 = g[0].r->a32, b32 = g[0].r->b32;
  gpe_status s;
  if (!a32 && !b32) s = run(DotArgs<double, double>{}, false);
  else if (a32 && b32) s = run(DotArgs<float, float>{}, false);
  else s = run(DotArgs<double, float>{}, a32);
  GPE_TRY(s);
  return fin_nblk(b, g, 1, POST_NONE, no_gram(g.size()));
}

template <typename A>
gpe_status elementwise(gpe_batch* b, std::vector<Item>& g, A (*rec)(const Req&), int kind) {
  if (!b || g.size() == 1) {
    for (auto& it : g) {
      gpe_handle* h = it.c->h;
      GPE_KT(h, kind, launch_single(rec(*it.r), elementwise_blocks(it.r->n), h->st));
    }
    return GPE_OK;
  }
  std::vector<A> recs(g.size());
  std::vector<int> nb(g.size());
  for (size_t i = 0; i < g.size(); ++i) {
    recs[i] = rec(*g[i].r);
    nb[i] = elementwise_blocks(g[i].r->n);
  }
  return ops(b, recs, nb);
}

template <typename TO> DiffArgs<double, double, TO> diff_rec(const Req& r) { return {r.a, r.b, r.c, r.n}; }
template <typename T> AxpbyArgs<T> axpby_rec(const Req& r) { return {r.a, r.c, r.s0, r.s1, r.n}; }
template <typename TI, typename TO> ConvArgs<TI, TO> copy_rec(const Req& r) { return {r.a, r.c, r.n}; }

gpe_status ex_diff(gpe_batch* b, std::vector<Item>& g) {
  if (g[0].r->c32) return elementwise(b, g, &diff_rec<float>, KK_VECTOR);
  return elementwise(b, g, &diff_rec<double>, KK_VECTOR);
}

gpe_status ex_axpby(gpe_batch* b, std::vector<Item>& g) {
  if (g[0].r->a32) return elementwise(b, g, &axpby_rec<float>, KK_VECTOR);
  return elementwise(b, g, &axpby_rec<double>, KK_VECTOR);
}

gpe_status ex_copy(gpe_batch* b, std::vector<Item>& g) {
  const bool a32 = g[0].r->a32 && g[0].r->a, c32 = g[0].r->c32;
  if (!a32 && !c32) return elementwise(b, g, &copy_rec<double, double>, KK_VECTOR);
  if (!a32 && c32) return elementwise(b, g, &copy_rec<double, float>, KK_VECTOR);
  if (a32 && c32) return elementwise(b, g, &copy_rec<float, float>, KK_VECTOR);
  return elementwise(b, g, &copy_rec<float, double>, KK_VECTOR);
}

gpe_status ex_lap(gpe_batch* b, std::vector<Item>& g) {
  const bool w32 = g[0].r->a32;
  if (!b || g.size() == 1) {
    for (auto& it : g) {
      if (w32) GPE_TRY(laplacian<float>(it.c->h, it.r->a, it.r->c));
      else GPE_TRY(laplacian<double>(it.c->h, it.r->a, it.r->c));
    }
    return GPE_OK;
  }
  std::vector<const void*> in(g.size());
  std::vector<void*> out(g.size());
  for (size_t i = 0; i < g.size(); ++i) {
    in[i] = g[i].r->a;
    out[i] = g[i].r->c;
  }
  return w32 ? lap_all<float>(b, g, in, out) : lap_all<double>(b, g, in, out);
}

// Batched HVP: fused x pass, projection coefficients, remaining axis passes
// with the projection in the last one, kappa where wanted (same stages as
// hvp_enq).  Every
// launch's records are built first and staged with one copy.
template <typename T>
gpe_status hvp_batched(gpe_batch* b, std::vector<Item>& g, bool riem, bool cg, bool kappa) {
  gpe_handle* h0 = b->hs[0];
  const size_t m = g.size();
  std::vector<XpassArgs<T>> xr(m);
  std::vector<int> xb(m), x0;
  std::vector<SlotCounts> nb(m, all_slots(0));
  for (size_t i = 0; i < m; ++i) {
    gpe_handle* h = g[i].c->h;
    if (!h->has_point) return fail(h, GPE_EINVAL, "batched HVP before the set point");
    const Req& r = *g[i].r;
    const bool w64 = sizeof(T) == 8;
    xr[i] = XpassArgs<T>{w64 ? h->Xp : h->Xp32, r.a, w64 ? h->LX64 : h->LX32,
                         w64 ? (const void*)h->V64 : (const void*)h->V32, r.c, twid<T>(h->ax[0]), h->part,
                         h->ax[0].lamc, h->npts, h->pstride, h->ax[0].n, hvp_params(h, riem, r.s0),
                         cg ? h->res + CG_DONE : nullptr};
    xb[i] = xpass_batch_blocks(h->ax[0].n, h->F, b->xvar, h->npts);
    for (int q = 0; q < 7; ++q) nb[i].nb[q] = xb[i];
  }
  GPE_TRY(offsets(h0, xb, &x0));
  std::vector<double*> gram(m);
  for (size_t i = 0; i < m; ++i) gram[i] = g[i].c->h->gram_pt;
  // few x-pass workgroups everywhere: the last axis pass forms the projection coefficients
  bool ab_local = riem && b->dim >= 2;
  for (size_t i = 0; i < m; ++i) ab_local = ab_local && xb[i] <= kAbLocalMax;
  std::vector<FinArgs> fab;
  if (riem && !ab_local) GPE_TRY(fin_records(b, g, 7, gram, nb, true, cg, &fab));
  // remaining stages: the 1-D projection, or the other axis passes
  std::vector<ProjArgs<T, T, false>> pr;
  std::vector<int> pb, p0;
  std::vector<std::vector<LapArgs<T>>> lr(b->dim);
  std::vector<std::vector<int>> l0(b->dim);
  int nq = 7;
  if (b->dim == 1) {
    if (riem) {
      pr.resize(m);
      pb.resize(m);
      for (size_t i = 0; i < m; ++i) {
        const gpe_handle* h = g[i].c->h;
        pr[i] = ProjArgs<T, T, false>{sizeof(T) == 8 ? h->Xp : h->Xp32, g[i].r->c, g[i].r->c, h->res + 32, 0.0, 0.0,
                                      nullptr, h->npts, h->F};
        pb[i] = h->nblk;
      }
      GPE_TRY(offsets(h0, pb, &p0));
    }
  } else {
    for (int a = 1; a < b->dim; ++a) {
      const bool proj = riem && a == b->dim - 1;
      lr[a].resize(m);
      std::vector<int> lb(m);
      for (size_t i = 0; i < m; ++i) {
        const gpe_handle* h = g[i].c->h;
        const LapAxis& ax = h->ax[a];
        const Req& r = *g[i].r;
        lr[a][i] = LapArgs<T>{r.a, r.c, r.c, twid<T>(ax), proj ? (sizeof(T) == 8 ? h->Xp : h->Xp32) : nullptr,
                              h->res + 32, h->part, ax.lamc, ax.nlines, h->npts, h->pstride, ax.inner, ax.n,
                              cg ? h->res + CG_DONE : nullptr};
        if (proj && ab_local) lr[a][i].ab = AbSrc{h->part, h->pstride, xb[i], h->gram_pt, h->res};
        lb[i] = lap_batch_blocks(ax.n, ax.nlines);
        nb[i].nb[6 + a] = lb[i];
      }
      GPE_TRY(offsets(h0, lb, &l0[a]));
      nq = 7 + a;
    }
  }
  std::vector<FinArgs> fk;   // the kappa finalize, where anyone reads kappa
  if (kappa) GPE_TRY(fin_records(b, g, nq, gram, nb, true, cg, &fk));

  // one staging copy for every launch below
  const void *dx = nullptr, *dx0 = nullptr, *dab = nullptr, *dp = nullptr, *dp0 = nullptr, *dk = nullptr;
  const void* dl[3] = {nullptr, nullptr, nullptr};
  const void* dl0[3] = {nullptr, nullptr, nullptr};
  std::vector<Stager::Seg> segs = {seg(xr, &dx), seg(x0, &dx0)};
  if (!fab.empty()) segs.push_back(seg(fab, &dab));
  if (!pr.empty()) {
    segs.push_back(seg(pr, &dp));
    segs.push_back(seg(p0, &dp0));
  }
  for (int a = 1; a < b->dim; ++a) {
    segs.push_back(seg(lr[a], &dl[a]));
    segs.push_back(seg(l0[a], &dl0[a]));
  }
  if (kappa) segs.push_back(seg(fk, &dk));
  GPE_TRY(b->sg.put_all(h0, b->st, segs.data(), segs.size()));

  const int n = (int)m;
  GPE_HIP(h0, xpass_batched<T>(b->F, b->xvar, reinterpret_cast<const XpassArgs<T>*>(dx),
                               Span{reinterpret_cast<const int*>(dx0), n, x0.back()}, b->st));
  if (!fab.empty())
    GPE_HIP(h0, finalize_batched(reinterpret_cast<const FinArgs*>(dab), n, 7, POST_HVP_AB, b->F, b->st));
  using PA = ProjArgs<T, T, false>;
  if (!pr.empty())
    GPE_HIP(h0, launch_batched<PA>(reinterpret_cast<const PA*>(dp), Span{reinterpret_cast<const int*>(dp0), n, p0.back()},
                                   b->st));
  for (int a = 1; a < b->dim; ++a)
    GPE_HIP(h0, lap_batched<T>(reinterpret_cast<const LapArgs<T>*>(dl[a]),
                               Span{reinterpret_cast<const int*>(dl0[a]), n, l0[a].back()}, b->F, 6 + a, b->st));
  if (!kappa) return GPE_OK;
  const int post = cg ? POST_CG_KAPPA : riem ? POST_HVP_KAPPA : POST_HVP_KAPPA_E;
  GPE_HIP(h0, finalize_batched(reinterpret_cast<const FinArgs*>(dk), n, nq, post, b->F, b->st));
  return GPE_OK;
}

gpe_status ex_hvp(gpe_batch* b, std::vector<Item>& g) {
  if (!b || g.size() == 1) {
    for (auto& it : g) GPE_TRY(hvp_enq(it.c->h, it.r->a, it.r->c, it.r->flag, it.r->s0, it.r->cg, it.r->kappa));
    return GPE_OK;
  }
  const bool riem = g[0].r->flag, cg = g[0].r->cg;
  if (cg && !riem) return fail(g[0].c->h, GPE_EINVAL, "the device-resident CG takes the Riemannian HVP");
  bool kappa = cg;
  for (auto& it : g) kappa = kappa || it.r->kappa;
  return g[0].r->a32 ? hvp_batched<float>(b, g, riem, cg, kappa) : hvp_batched<double>(b, g, riem, cg, kappa);
}

gpe_status ex_cg(gpe_batch* b, std::vector<Item>& g) {
  if (!b || g.size() == 1) {
    for (auto& it : g) {
      const Req& r = *it.r;
      GPE_TRY(cg_step_enq(it.c->h, nullptr, r.b, nullptr, r.d));
      GPE_TRY(cg_dir_enq(it.c->h, r.d, r.c, const_cast<void*>(r.a), (int)r.s0));
    }
    return GPE_OK;
  }
  // the update, its finalize (none where every problem is small: the closing
  // step applies the tests) and the closing step staged with one copy
  gpe_handle* h0 = b->hs[0];
  bool local = true;
  for (size_t i = 0; i < g.size(); ++i) local = local && cg_local_step(g[i].c->h);
  std::vector<SlotCounts> sc(g.size());
  for (size_t i = 0; i < g.size(); ++i) sc[i] = all_slots(g[i].c->h->nblk);
  std::vector<FinArgs> fr;
  if (!local) GPE_TRY(fin_records(b, g, 1, no_gram(g.size()), sc, false, true, &fr));
  auto run = [&](auto tag, auto dtag) -> gpe_status {
    using A = decltype(tag);
    using D = decltype(dtag);
    std::vector<A> recs(g.size());
    std::vector<D> drecs(g.size());
    std::vector<int> nb(g.size()), b0, nd(g.size()), d0;
    for (size_t i = 0; i < g.size(); ++i) {
      gpe_handle* h = g[i].c->h;
      const Req& r = *g[i].r;
      recs[i] = A{nullptr, r.b, nullptr, r.d, h->part, 0.0, h->nel, h->res + CG_ALPHA, h->res + CG_DONE};
      drecs[i] = D{r.d, r.c, const_cast<void*>(r.a), h->res, (int)r.s0, r.n};
      if (local) {
        drecs[i].part = h->part;
        drecs[i].nb = h->nblk;
      }
      nb[i] = h->nblk;
      nd[i] = elementwise_blocks(r.n);
    }
    GPE_TRY(offsets(h0, nb, &b0));
    GPE_TRY(offsets(h0, nd, &d0));
    const void *dr = nullptr, *db0 = nullptr, *df = nullptr, *dd = nullptr, *dd0 = nullptr;
    std::vector<Stager::Seg> segs = {seg(recs, &dr), seg(b0, &db0), seg(drecs, &dd), seg(d0, &dd0)};
    if (!local) segs.push_back(seg(fr, &df));
    GPE_TRY(b->sg.put_all(h0, b->st, segs.data(), segs.size()));
    const int n = (int)g.size();
    GPE_HIP(h0, launch_batched<A>(reinterpret_cast<const A*>(dr), Span{reinterpret_cast<const int*>(db0), n, b0.back()},
                                  b->st));
    if (!local) GPE_HIP(h0, finalize_batched(reinterpret_cast<const FinArgs*>(df), n, 1, POST_CG_STEP, b->F, b->st));
    GPE_HIP(h0, launch_batched<D>(reinterpret_cast<const D*>(dd), Span{reinterpret_cast<const int*>(dd0), n, d0.back()},
                                  b->st));
    return GPE_OK;
  };
  return g[0].r->a32 ? run(CgArgs<float>{}, CgDirArgs<float>{}) : run(CgArgs<double>{}, CgDirArgs<double>{});
}

gpe_status ex_cginit(gpe_batch* b, std::vector<Item>& g) {
  if (!b || g.size() == 1) {
    for (auto& it : g) GPE_TRY(cg_init_enq(it.c->h, it.r->s0, it.r->s1, (int)it.r->n));
    return GPE_OK;
  }
  std::vector<CgInitArgs> recs(g.size());
  std::vector<int> nb(g.size(), 1);
  for (size_t i = 0; i < g.size(); ++i) recs[i] = CgInitArgs{g[i].c->h->res, g[i].r->s0, g[i].r->s1, (int)g[i].r->n};
  return ops(b, recs, nb);
}

gpe_status execute(gpe_batch* b, int kind, std::vector<Item>& g) {
  switch (kind) {
    case RQ_EVAL: return ex_eval(b, g);
    case RQ_PGRAD: return ex_pgrad(b, g);
    case RQ_NORMS: return ex_norms(b, g);
    case RQ_SCALE: return ex_scale(b, g);
    case RQ_DOT: return ex_dot(b, g);
    case RQ_DIFF: return ex_diff(b, g);
    case RQ_AXPBY: return ex_axpby(b, g);
    case RQ_COPY: return ex_copy(b, g);
    case RQ_LAP: return ex_lap(b, g);
    case RQ_HVP: return ex_hvp(b, g);
    case RQ_CG: return ex_cg(b, g);
    case RQ_CGINIT: return ex_cginit(b, g);
    default: return fail(g[0].c->h, GPE_EINVAL, "unknown queued operation");
  }
}

// Requests with the same key can share one batched launch.
unsigned key_of(const Req& r) {
  return (unsigned)r.kind | (r.a32 << 8) | (r.b32 << 9) | (r.c32 << 10) | (r.flag << 11) | ((r.a != nullptr) << 12) |
         ((r.b != nullptr) << 13) | ((r.c != nullptr) << 14) | (r.cg << 15);
}

void resume(Ctx* c) {
  c->task.co.resume();
  if (c->task.co.done()) {
    c->done = true;
    c->status = c->task.co.promise().status;
  }
}

}  // namespace

gpe_status Stager::put(gpe_handle* h, hipStream_t st, const void* src, size_t bytes, const void** dptr) {
  const size_t need = (bytes + kAlign - 1) / kAlign * kAlign;
  if (need > cap) return fail(h, GPE_ENOMEM, "batched launch records exceed the staging arena");
  if (off + need > cap) {
    GPE_HIP(h, hipStreamSynchronize(st));   // every staged record has been consumed
    off = 0;
  }
  std::memcpy(host + off, src, bytes);
  GPE_HIP(h, hipMemcpyAsync(dev + off, host + off, bytes, hipMemcpyHostToDevice, st));
  *dptr = dev + off;
  off += need;
  return GPE_OK;
}

gpe_status Stager::put2(gpe_handle* h, hipStream_t st, const void* a, size_t na, const void* b, size_t nb,
                        const void** da, const void** db) {
  const Seg s[2] = {{a, na, da}, {b, nb, db}};
  return put_all(h, st, s, 2);
}

gpe_status Stager::put_all(gpe_handle* h, hipStream_t st, const Seg* segs, size_t n) {
  size_t bytes = 0;
  for (size_t k = 0; k < n; ++k) bytes = (bytes + 15) / 16 * 16 + segs[k].bytes;
  const size_t need = (bytes + kAlign - 1) / kAlign * kAlign;
  if (need > cap) return fail(h, GPE_ENOMEM, "batched launch records exceed the staging arena");
  if (off + need > cap) {
    GPE_HIP(h, hipStreamSynchronize(st));   // every staged record has been consumed
    off = 0;
  }
  size_t o = 0;
  for (size_t k = 0; k < n; ++k) {
    o = (o + 15) / 16 * 16;
    std::memcpy(host + off + o, segs[k].src, segs[k].bytes);
    *segs[k].dptr = dev + off + o;
    o += segs[k].bytes;
  }
  GPE_HIP(h, hipMemcpyAsync(dev + off, host + off, bytes, hipMemcpyHostToDevice, st));
  off += need;
  return GPE_OK;
}

gpe_status Lockstep::round(std::vector<Ctx*>& cs, bool sync) {
  // Run the queues head by head, each step taking the operation that heads
  // the most queues: a problem's own order is kept and launches are shared.
  std::vector<size_t> head(cs.size(), 0);
  for (;;) {
    unsigned best = 0;
    int best_n = 0;
    for (size_t i = 0; i < cs.size(); ++i) {
      if (head[i] >= cs[i]->q.size()) continue;
      const unsigned k = key_of(cs[i]->q[head[i]]);
      int n = 0;
      for (size_t j = 0; j < cs.size(); ++j)
        if (head[j] < cs[j]->q.size() && key_of(cs[j]->q[head[j]]) == k) ++n;
      if (n > best_n) {
        best_n = n;
        best = k;
      }
    }
    if (best_n == 0) break;
    std::vector<Item> g;
    for (size_t i = 0; i < cs.size(); ++i)
      if (head[i] < cs[i]->q.size() && key_of(cs[i]->q[head[i]]) == best) g.push_back({cs[i], &cs[i]->q[head[i]++]});
    const gpe_status s = execute(b_, g[0].r->kind, g);
    if (s != GPE_OK) {
      if (b_) b_->err = g[0].c->h->err;
      return s;
    }
  }
  for (Ctx* c : cs) c->q.clear();
  if (!sync) return GPE_OK;   // the staging arena keeps its place: its records may not be consumed yet
  gpe_handle* h0 = cs[0]->h;
  if (b_) {
    GPE_HIP(h0, hipMemcpyAsync(b_->hres, b_->res, sizeof(double) * kResDoubles * b_->hs.size(),
                               hipMemcpyDeviceToHost, b_->st));
  } else {
    for (Ctx* c : cs)
      GPE_HIP(c->h, hipMemcpyAsync(c->h->hres, c->h->res, sizeof(double) * kResDoubles, hipMemcpyDeviceToHost,
                                   c->h->st));
  }
  for (Ctx* c : cs) {
    if (c != cs[0] && c->h->st == h0->st) continue;
    GPE_HIP(c->h, hipStreamSynchronize(c->h->st));
  }
  if (b_) b_->sg.off = 0;
  return GPE_OK;
}

gpe_status Lockstep::run(std::vector<Ctx*>& cs) {
  for (Ctx* c : cs) resume(c);
  for (;;) {
    bool pending = false;
    for (Ctx* c : cs) pending = pending || !c->done || !c->q.empty();
    if (!pending) return GPE_OK;
    GPE_TRY(round(cs));
    for (Ctx* c : cs)
      if (!c->done) resume(c);
  }
}

// One driver on a lone handle (no batch): every operation is a single launch.
gpe_status solve_single(gpe_handle* h, void* X, const gpe_solve_opts* o, gpe_solve_stats* st) {
  Ctx c;
  c.h = h;
  c.task = solve_task(c, X, o, st);
  std::vector<Ctx*> cs{&c};
  Lockstep ls(nullptr);
  GPE_TRY(ls.run(cs));
  return c.status;
}

// Time the batched fused x pass per schedule variant on pseudo-random fields
// (three distinct buffers per problem, as at handle creation) and keep the
// fastest.
static gpe_status tune_batch(gpe_batch* b) {
  if (b->hs.size() < 2) return GPE_OK;
  gpe_handle* h0 = b->hs[0];
  const int nv = b->F == 3 ? 2 : 3;
  const bool w32 = b->prec == GPE_MIXED;
  for (gpe_handle* h : b->hs) {
    void* bufs[3] = {w32 ? h->Xp32 : h->Xp, w32 ? h->LX32 : h->LX64, w32 ? h->T32 : h->T64};
    unsigned seed = 1;
    for (void* p : bufs) {
      if (w32) GPE_HIP(h, launch_single(FillArgs<float>{p, h->nel, seed++}, elementwise_blocks(h->nel), b->st));
      else GPE_HIP(h, launch_single(FillArgs<double>{p, h->nel, seed++}, elementwise_blocks(h->nel), b->st));
    }
  }
  hipEvent_t e0, e1;
  GPE_HIP(h0, hipEventCreate(&e0));
  GPE_HIP(h0, hipEventCreate(&e1));
  float best = 1e30f;
  int bestv = 1;
  gpe_status s = GPE_OK;
  for (int v = 0; v < nv && s == GPE_OK; ++v) {
    b->xvar = v;
    float tmin = 1e30f;
    for (int rep = 0; rep < 4 && s == GPE_OK; ++rep) {
      if (hipEventRecord(e0, b->st) != hipSuccess) s = GPE_EHIP;
      auto one = [&](auto tag) -> gpe_status {
        using T = decltype(tag);
        std::vector<XpassArgs<T>> xr(b->hs.size());
        std::vector<int> xb(b->hs.size());
        for (size_t i = 0; i < b->hs.size(); ++i) {
          gpe_handle* h = b->hs[i];
          const bool w64 = sizeof(T) == 8;
          xr[i] = XpassArgs<T>{w64 ? h->Xp : h->Xp32, w64 ? h->T64 : h->T32, w64 ? h->LX64 : h->LX32,
                               w64 ? (const void*)h->V64 : (const void*)h->V32, h->Gp, twid<T>(h->ax[0]), h->part,
                               h->ax[0].lamc, h->npts, h->pstride, h->ax[0].n, h->pw, nullptr};
          xb[i] = xpass_batch_blocks(h->ax[0].n, h->F, v, h->npts);
        }
        return launch_records(b, xr, xb, [&](const XpassArgs<T>* d, const Span& sp) {
          return xpass_batched<T>(b->F, v, d, sp, b->st);
        });
      };
      if (s == GPE_OK) s = b->prec == GPE_MIXED ? one(0.0f) : one(0.0);
      if (s == GPE_OK && hipEventRecord(e1, b->st) != hipSuccess) s = GPE_EHIP;
      if (s == GPE_OK && hipEventSynchronize(e1) != hipSuccess) s = GPE_EHIP;
      float ms = 0.f;
      if (s == GPE_OK && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) s = GPE_EHIP;
      b->sg.off = 0;
      if (rep > 0) tmin = std::fmin(tmin, ms);   // the first launch is a warm-up
    }
    b->xvar_us[v] = 1e3f * tmin;
    if (tmin < best) {
      best = tmin;
      bestv = v;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (s != GPE_OK) {
    b->err = h0->err.empty() ? "batched x-pass autotune failed" : h0->err;
    return s;
  }
  b->xvar = bestv;
  return GPE_OK;
}

}  // namespace gpe

using namespace gpe;

// ----------------------------------------------------------------- C ABI

static std::string g_batch_error;

static gpe_status batch_fail(gpe_batch* b, gpe_status s, const std::string& m) {
  if (b) b->err = m;
  else g_batch_error = m;
  return s;
}

extern "C" {

const char* gpe_batch_last_error(const gpe_batch* b) { return b ? b->err.c_str() : g_batch_error.c_str(); }

gpe_status gpe_batch_destroy(gpe_batch* b) {
  if (!b) return GPE_OK;
  if (b->st) (void)hipStreamSynchronize(b->st);
  for (gpe_handle* h : b->hs) gpe_destroy(h);
  if (b->res) (void)hipFree(b->res);
  if (b->hres) (void)hipHostFree(b->hres);
  if (b->sg.dev) (void)hipFree(b->sg.dev);
  if (b->sg.host) (void)hipHostFree(b->sg.host);
  delete b;
  return GPE_OK;
}

gpe_status gpe_batch_create(const gpe_problem* probs, const double* const* V_host, int count, int precision,
                            void* stream, gpe_batch** out) {
  if (!out) return batch_fail(nullptr, GPE_EINVAL, "out is NULL");
  *out = nullptr;
  if (!probs || !V_host || count < 1 || count > 65535) return batch_fail(nullptr, GPE_EINVAL, "bad problem list");
  for (int i = 0; i < count; ++i) {
    const gpe_problem& p = probs[i];
    if (p.F != probs[0].F || p.dim != probs[0].dim)
      return batch_fail(nullptr, GPE_EINVAL, "every problem of a batch needs the same F and dim");
    for (int a = 0; a < p.dim && a < 3; ++a)
      if (!batch_size_supported(p.n[a]))
        return batch_fail(nullptr, GPE_EINVAL, "problem " + std::to_string(i) + ": n[" + std::to_string(a) +
                                                   "] = " + std::to_string(p.n[a]) +
                                                   " (a batch takes powers of two 16..512)");
  }
  gpe_batch* b = new gpe_batch();
  b->st = reinterpret_cast<hipStream_t>(stream);
  b->F = probs[0].F;
  b->dim = probs[0].dim;
  b->prec = precision;
  for (int i = 0; i < count; ++i) {
    gpe_handle* h = nullptr;
    const gpe_status s = gpe_create(&probs[i], V_host[i], precision, stream, &h);
    if (s != GPE_OK) {
      const std::string m = "problem " + std::to_string(i) + ": " + gpe_last_error(nullptr);
      gpe_batch_destroy(b);
      return batch_fail(nullptr, s, m);
    }
    b->hs.push_back(h);
  }
  auto bail = [&](gpe_status s, const std::string& m) {
    gpe_batch_destroy(b);
    return batch_fail(nullptr, s, m);
  };
  const size_t nres = sizeof(double) * kResDoubles * count;
  if (hipMalloc((void**)&b->res, nres) != hipSuccess) return bail(GPE_ENOMEM, "batch result array");
  if (hipHostMalloc((void**)&b->hres, nres, hipHostMallocDefault) != hipSuccess)
    return bail(GPE_ENOMEM, "batch pinned result array");
  b->sg.cap = std::max<size_t>((size_t)1 << 20, (size_t)count * 8192);
  if (hipMalloc((void**)&b->sg.dev, b->sg.cap) != hipSuccess) return bail(GPE_ENOMEM, "batch staging arena");
  if (hipHostMalloc((void**)&b->sg.host, b->sg.cap, hipHostMallocDefault) != hipSuccess)
    return bail(GPE_ENOMEM, "batch pinned staging arena");
  // every handle reports into its slice of the batch's arrays
  for (int i = 0; i < count; ++i) {
    gpe_handle* h = b->hs[i];
    (void)hipFree(h->res);
    (void)hipHostFree(h->hres);
    h->res = b->res + (size_t)kResDoubles * i;
    h->hres = b->hres + (size_t)kResDoubles * i;
    h->res_shared = true;
  }
  const gpe_status ts = tune_batch(b);
  if (ts != GPE_OK) return bail(ts, b->err);
  *out = b;
  return GPE_OK;
}

gpe_status gpe_batch_size(const gpe_batch* b, int* count) {
  if (!b || !count) return batch_fail(nullptr, GPE_EINVAL, "NULL argument");
  *count = (int)b->hs.size();
  return GPE_OK;
}

gpe_status gpe_batch_handle(gpe_batch* b, int i, gpe_handle** h) {
  if (!b || !h) return batch_fail(b, GPE_EINVAL, "NULL argument");
  if (i < 0 || i >= (int)b->hs.size()) return batch_fail(b, GPE_EINVAL, "problem index out of range");
  *h = b->hs[i];
  return GPE_OK;
}

gpe_status gpe_batch_schedule(const gpe_batch* b, int* xpass_variant, float* variant_us, int nvariants) {
  if (!b) return batch_fail(nullptr, GPE_EINVAL, "NULL batch");
  if (xpass_variant) *xpass_variant = b->xvar;
  for (int v = 0; v < nvariants && v < 3; ++v)
    if (variant_us) variant_us[v] = b->xvar_us[v];
  return GPE_OK;
}

gpe_status gpe_batch_hvp(gpe_batch* b, const void* const* Z, void* const* HZ, int riemannian, const double* sigma,
                         double* kappa) {
  if (!b || !Z || !HZ) return batch_fail(b, GPE_EINVAL, "NULL argument");
  const size_t m = b->hs.size();
  std::vector<Ctx> cs(m);
  std::vector<Ctx*> cp(m);
  for (size_t i = 0; i < m; ++i) {
    if (!Z[i] || !HZ[i] || Z[i] == HZ[i]) return batch_fail(b, GPE_EINVAL, "Z and HZ must be distinct and non-NULL");
    if (!b->hs[i]->has_point) return batch_fail(b, GPE_EINVAL, "problem " + std::to_string(i) + " has no set point");
    cs[i].h = b->hs[i];
    Req r;
    r.kind = RQ_HVP;
    r.a = Z[i];
    r.c = HZ[i];
    r.flag = riemannian != 0;
    r.s0 = sigma ? sigma[i] : 0.0;
    r.a32 = r.c32 = b->prec == GPE_MIXED;
    r.kappa = kappa != nullptr;
    cs[i].push(r);
    cp[i] = &cs[i];
  }
  Lockstep ls(b);
  const gpe_status s = ls.round(cp, kappa != nullptr);
  if (s != GPE_OK) return batch_fail(b, s, b->err.empty() ? b->hs[0]->err : b->err);
  if (kappa)
    for (size_t i = 0; i < m; ++i) {
      const gpe_status r = hvp_read(b->hs[i], &kappa[i], nullptr);
      if (r != GPE_OK) return batch_fail(b, r, "problem " + std::to_string(i) + ": " + b->hs[i]->err);
    }
  return GPE_OK;
}

}  // extern "C"

namespace gpe {
namespace {

// One lock-step solve of every problem of b on its own mesh (opts->mg_levels
// is ignored).  status[i]: problem i's own outcome.
gpe_status lockstep_solve(gpe_batch* b, void* const* X, const gpe_solve_opts& o, gpe_solve_stats* st,
                          std::vector<gpe_status>* status) {
  const size_t m = b->hs.size();
  gpe_solve_opts oo = o;
  oo.mg_levels = 0;
  oo.trace = nullptr;   // one trace buffer cannot serve many problems
  oo.trace_cap = 0;
  std::vector<Ctx> cs(m);
  std::vector<Ctx*> cp(m);
  for (size_t i = 0; i < m; ++i) {
    std::memset(&st[i], 0, sizeof(st[i]));
    cs[i].h = b->hs[i];
    cp[i] = &cs[i];
  }
  for (size_t i = 0; i < m; ++i) cs[i].task = solve_task(cs[i], X[i], &oo, &st[i]);
  Lockstep ls(b);
  const gpe_status rs = ls.run(cp);
  status->resize(m);
  for (size_t i = 0; i < m; ++i) (*status)[i] = cs[i].status;
  return rs;
}

// Coarse levels of the cascadic hierarchy (Algorithm 1, outer loop) for a
// whole batch: level l halves every axis of level l - 1, with V and the
// initial states injected; each level is a batch of its own, solved in lock
// step to the coarse tolerance, and every problem's solution is prolonged to
// the next finer level.  On return X holds the prolonged states on b's grids.
gpe_status cascadic_levels(gpe_batch* b, void* const* X, const gpe_solve_opts& o, int L, double* t_coarse) {
  using clock = std::chrono::steady_clock;
  const auto t0 = clock::now();
  const size_t m = b->hs.size();
  std::vector<gpe_batch*> bs(L + 1, nullptr);
  std::vector<std::vector<void*>> xs(L + 1, std::vector<void*>(m, nullptr));
  bs[0] = b;
  for (size_t i = 0; i < m; ++i) xs[0][i] = X[i];
  gpe_status rs = GPE_OK;
  for (int l = 1; l <= L && rs == GPE_OK; ++l) {
    const gpe_batch* f = bs[l - 1];
    std::vector<gpe_problem> pc(m);
    std::vector<std::vector<double>> Vc(m);
    std::vector<const double*> vp(m);
    for (size_t i = 0; i < m; ++i) {
      const gpe_handle* h = f->hs[i];
      pc[i] = h->prob;
      int nc[3] = {1, 1, 1};
      for (int a = 0; a < h->dim; ++a) nc[a] = pc[i].n[a] = h->n[a] / 2;
      Vc[i].resize((size_t)nc[0] * nc[1] * nc[2]);
      const int sy = h->dim > 1 ? 2 : 1, sz = h->dim > 2 ? 2 : 1;
      for (int z = 0; z < nc[2]; ++z)
        for (int y = 0; y < nc[1]; ++y)
          for (int x = 0; x < nc[0]; ++x)
            Vc[i][((size_t)z * nc[1] + y) * nc[0] + x] =
                h->Vhost[((size_t)(z * sz) * h->n[1] + (size_t)(y * sy)) * h->n[0] + 2 * x];
      vp[i] = Vc[i].data();
    }
    rs = gpe_batch_create(pc.data(), vp.data(), (int)m, b->prec, b->st, &bs[l]);
    if (rs != GPE_OK) {
      b->err = std::string("multigrid: coarse batch: ") + gpe_batch_last_error(nullptr);
      bs[l] = nullptr;
      break;
    }
    for (size_t i = 0; i < m && rs == GPE_OK; ++i) {
      const gpe_handle* hc = bs[l]->hs[i];
      rs = alloc_field(b->hs[i], &xs[l][i], hc->nel * 16);
      if (rs != GPE_OK) {
        b->err = b->hs[i]->err;
        break;
      }
      int nc[3] = {hc->n[0], hc->n[1], hc->n[2]};
      const hipError_t e = restrict_inject(xs[l - 1][i], xs[l][i], hc->K, hc->dim, nc, std::pow(2.0, 0.5 * hc->dim),
                                           b->st);
      if (e != hipSuccess) {
        rs = hip_fail(b->hs[i], e, "restrict_inject");
        b->err = b->hs[i]->err;
      }
    }
  }
  for (int l = L; l >= 1 && rs == GPE_OK; --l) {
    gpe_solve_opts oc = o;
    oc.tol = o.mg_coarse_tol;
    if (o.time_limit > 0)
      oc.time_limit = std::fmax(o.time_limit - std::chrono::duration<double>(clock::now() - t0).count(), 1e-3);
    std::vector<gpe_solve_stats> sc(m);
    std::vector<gpe_status> stat;
    rs = lockstep_solve(bs[l], xs[l].data(), oc, sc.data(), &stat);
    if (rs != GPE_OK) {
      b->err = "multigrid: coarse solve: " + (bs[l]->err.empty() ? bs[l]->hs[0]->err : bs[l]->err);
      break;
    }
    for (size_t i = 0; i < m && rs == GPE_OK; ++i)
      if (stat[i] != GPE_OK && stat[i] != GPE_ENOTCONV) {
        rs = stat[i];
        b->err = "multigrid: coarse solve of problem " + std::to_string(i) + ": " + bs[l]->hs[i]->err;
      }
    for (size_t i = 0; i < m && rs == GPE_OK; ++i) {
      rs = prolong(bs[l]->hs[i], xs[l][i], bs[l - 1]->hs[i], xs[l - 1][i]);
      if (rs != GPE_OK) b->err = "multigrid: prolong problem " + std::to_string(i) + ": " + bs[l - 1]->hs[i]->err;
    }
  }
  if (b->st) (void)hipStreamSynchronize(b->st);
  for (int l = 1; l <= L; ++l) {
    for (void* p : xs[l])
      if (p) (void)hipFree(p);
    if (bs[l]) gpe_batch_destroy(bs[l]);
  }
  *t_coarse = std::chrono::duration<double>(clock::now() - t0).count();
  return rs;
}

}  // namespace
}  // namespace gpe

extern "C" {

gpe_status gpe_batch_newton_solve(gpe_batch* b, void* const* X_inout, const gpe_solve_opts* opts,
                                  gpe_solve_stats* stats) {
  if (!b || !X_inout) return batch_fail(b, GPE_EINVAL, "NULL argument");
  gpe_solve_opts o;
  if (opts) o = *opts;
  else gpe_solve_opts_default(&o);
  if (o.mg_levels < 0) return batch_fail(b, GPE_EINVAL, "mg_levels must be >= 0");
  const size_t m = b->hs.size();
  for (size_t i = 0; i < m; ++i)
    if (!X_inout[i]) return batch_fail(b, GPE_EINVAL, "NULL field");
  // the coarsest admissible level: every axis of every problem stays a batch size (a power of two >= 16)
  int L = o.mg_levels;
  for (size_t i = 0; i < m; ++i)
    for (int a = 0; a < b->dim; ++a)
      while (L > 0 && !batch_size_supported(b->hs[i]->n[a] >> L)) --L;
  double t_coarse = 0.0;
  b->err.clear();
  if (L > 0) {
    const gpe_status r = cascadic_levels(b, X_inout, o, L, &t_coarse);
    if (r != GPE_OK) return batch_fail(b, r, b->err.empty() ? "multigrid failed" : b->err);
    if (o.time_limit > 0) o.time_limit = std::fmax(o.time_limit - t_coarse, 1e-3);
  }
  std::vector<gpe_solve_stats> st(m);
  std::vector<gpe_status> stat;
  const gpe_status rs = lockstep_solve(b, X_inout, o, st.data(), &stat);
  for (size_t i = 0; i < m; ++i) {   // counters: finest mesh only
    st[i].mg_levels = L;
    st[i].t_coarse = t_coarse;
    st[i].t_total += t_coarse;
  }
  if (stats)
    for (size_t i = 0; i < m; ++i) stats[i] = st[i];
  if (rs != GPE_OK) return batch_fail(b, rs, b->err.empty() ? b->hs[0]->err : b->err);
  gpe_status agg = GPE_OK;
  for (size_t i = 0; i < m && agg == GPE_OK; ++i)
    if (stat[i] != GPE_OK && stat[i] != GPE_ENOTCONV) {
      agg = stat[i];
      b->err = "problem " + std::to_string(i) + ": " + b->hs[i]->err;
    }
  if (agg == GPE_OK)
    for (size_t i = 0; i < m; ++i)
      if (stat[i] == GPE_ENOTCONV) {
        agg = GPE_ENOTCONV;
        b->err = "problem " + std::to_string(i) + ": tolerance not reached";
        break;
      }
  return agg;
}

}  // extern "C"
