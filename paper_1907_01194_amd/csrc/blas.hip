// Field-level kernels: deterministic FP64 reductions (block partial sums, one
// single-block finalize), the tangent-space projection of Lemma 4.1, the
// componentwise scaling of the retractions (Sec. 6), CG vector updates and
// precision conversions.  All reductions accumulate in FP64 whatever the
// field precision.
#include "batch_ops.h"

namespace gpe {

// ----------------------------------------------------------------- finalize
// Two forms, both summing in a fixed order (bitwise reproducible):
// * one workgroup (ticket null): its waves split the slots (several waves per
//   slot when there are fewer slots than waves); each lane sums a fixed strided
//   subset of a slot's partials, each wave a fixed shuffle tree, and thread 0
//   adds the waves of a slot in order, stores the sums and applies the
//   post-operation.  No atomics, no cross-workgroup fence.
// * one workgroup per slot (ticket non-null, slot q = the workgroup's index):
//   for many partials, where one workgroup cannot fetch them fast enough.  The
//   last workgroup to finish (counted with the atomic ticket, which it resets)
//   applies the post-operation.
constexpr int kFinThreads = 1024;   // up to 16k partials per slot: 16 loads per thread
constexpr int kFinWaves = kFinThreads / kWave;
constexpr int kFinOneBlockMax = 1024;   // partials per slot up to which one workgroup does all

__device__ void finalize_body(const double* __restrict__ part, size_t stride, const SlotCounts& nb, int nq,
                              double* __restrict__ res, int post, int F, double* gram, unsigned int* ticket,
                              const double* skip) {
  __shared__ double red[kMaxQ > kFinWaves ? kMaxQ : kFinWaves];
  __shared__ bool last;
  if (skip && *skip != 0.0) return;   // uniform over the launch: no ticket is taken
  const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
  if (ticket) {
    const int q = blockIdx.x;
    const double* pq = part + (size_t)q * stride;
    const int n = nb.nb[q];
    double s0 = 0, s1 = 0, s2 = 0, s3 = 0;
    int b = threadIdx.x;
    for (; b + 3 * kFinThreads < n; b += 4 * kFinThreads) {
      s0 += pq[b];
      s1 += pq[b + kFinThreads];
      s2 += pq[b + 2 * kFinThreads];
      s3 += pq[b + 3 * kFinThreads];
    }
    for (; b < n; b += kFinThreads) s0 += pq[b];
    const double s = wave_sum((s0 + s1) + (s2 + s3));
    if (lane == 0) red[w] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
      double t = 0.0;
      for (int u = 0; u < kFinWaves; ++u) t += red[u];
      res[q] = t;
      __threadfence();
      last = atomicAdd(ticket, 1u) == (unsigned)(nq - 1);
    }
    __syncthreads();
    if (!last || threadIdx.x != 0) return;
    *ticket = 0u;   // every workgroup of this launch has taken its ticket
    __threadfence();
  } else {
    const int wps = nq < kFinWaves ? kFinWaves / nq : 1;   // waves per slot; nq * wps <= max(nq, kFinWaves)
    for (int q = w / wps; q < nq; q += kFinWaves / wps) {
      const int sub = w % wps;
      const double* pq = part + (size_t)q * stride;
      const int n = nb.nb[q];
      const int step = wps * kWave;
      double s0 = 0, s1 = 0, s2 = 0, s3 = 0;
      int b = sub * kWave + lane;
      for (; b + 3 * step < n; b += 4 * step) {
        s0 += pq[b];
        s1 += pq[b + step];
        s2 += pq[b + 2 * step];
        s3 += pq[b + 3 * step];
      }
      for (; b < n; b += step) s0 += pq[b];
      const double s = wave_sum((s0 + s1) + (s2 + s3));
      if (lane == 0) red[q * wps + sub] = s;
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    for (int q = 0; q < nq; ++q) {
      double t = 0.0;
      for (int u = 0; u < wps; ++u) t += red[q * wps + u];
      res[q] = t;
    }
  }
  const volatile double* out = res;   // (slots written by other workgroups in the ticket form)
  const int K = 2 * F + 1;
  if (post == POST_GRAD) {
    // Gram system of Lemma 4.1 (proof) with the measured u^T u, u^T G u, u^T G^2 u
    double a11 = 0, a12 = 0, a22 = 0, r1 = 0, r2 = 0;
    for (int i = 0; i < K; ++i) {
      const double l = F - i, nrm = out[1 + K + i];
      a11 += nrm;
      a12 += l * nrm;
      a22 += l * l * nrm;
      r1 += out[1 + i];
      r2 += l * out[1 + i];
    }
    const double det = a11 * a22 - a12 * a12;
    res[nq] = (a22 * r1 - a12 * r2) / det;
    res[nq + 1] = (a11 * r2 - a12 * r1) / det;
    if (gram)
      for (int i = 0; i < K; ++i) gram[i] = out[1 + K + i];
  } else if (post == POST_HVP_AB) {
    double a11 = 0, a12 = 0, a22 = 0;
    for (int i = 0; i < K; ++i) {
      const double l = F - i;
      a11 += gram[i];
      a12 += l * gram[i];
      a22 += l * l * gram[i];
    }
    const double det = a11 * a22 - a12 * a12;
    res[32] = (a22 * out[0] - a12 * out[1]) / det;
    res[33] = (a11 * out[1] - a12 * out[0]) / det;
  } else if (post == POST_HVP_KAPPA || post == POST_HVP_KAPPA_E || post == POST_CG_KAPPA) {
    double zlz = 0.0;
    for (int k = 6; k < nq; ++k) zlz += out[k];
    const double kappa = post == POST_HVP_KAPPA_E ? out[4] + zlz
                                                  : out[4] + zlz - out[32] * out[2] - out[33] * out[3];
    const double pp = out[5];
    res[34] = kappa;
    res[35] = pp;
    if (post == POST_CG_KAPPA) {
      res[CG_IT] = out[CG_IT] + 1.0;
      if (!(kappa > out[CG_EPS] * pp)) {   // curvature stop (a NaN stops too)
        res[CG_KAPPA] = kappa;
        res[CG_PP] = pp;
        res[CG_REASON] = CG_STOP_CURVATURE;
        res[CG_CURV] = 1.0;
        res[CG_DONE] = 1.0;
      } else {
        res[CG_ALPHA] = out[cg_rr_slot((int)out[CG_IT] - 1)] / kappa;   // (CG_IT counts this iteration already)
      }
    }
  } else if (post == POST_CG_STEP) {
    const double rr = out[0];
    const int it = (int)out[CG_IT];   // iterations done, this one included
    if (sqrt(rr) <= out[CG_TOL]) {
      res[CG_REASON] = CG_STOP_RESIDUAL;
      res[CG_DONE] = 1.0;
    } else {
      res[CG_BETA] = rr / out[cg_rr_slot(it - 1)];
      res[cg_rr_slot(it)] = rr;
      if (out[CG_IT] >= out[CG_MAXIT]) {
        res[CG_REASON] = CG_STOP_CAP;
        res[CG_DONE] = 1.0;
      }
    }
  }
}

__global__ void __launch_bounds__(kFinThreads)
finalize_kernel(const double* __restrict__ part, size_t stride, SlotCounts nb, int nq, double* __restrict__ res,
                int post, int F, double* gram, unsigned int* ticket, const double* skip) {
  finalize_body(part, stride, nb, nq, res, post, F, gram, ticket, skip);
}

__global__ void __launch_bounds__(kFinThreads)
finalize_batched_kernel(const FinArgs* __restrict__ args, int nq, int post, int F) {
  const FinArgs& a = args[blockIdx.x];
  finalize_body(a.part, a.stride, a.nb, nq, a.res, post, F, a.gram, nullptr, a.skip);
}

static bool counts_ok(const SlotCounts& nb, int nq, size_t stride) {
  if (nq < 1 || nq > kMaxQ || nq > (int)(sizeof(nb.nb) / sizeof(nb.nb[0]))) return false;
  for (int q = 0; q < nq; ++q)
    if (nb.nb[q] < 0 || (size_t)nb.nb[q] > stride) return false;
  return true;
}

hipError_t finalize(const double* part, size_t stride, const SlotCounts& nb, int nq, double* res, int post, int F,
                    double* gram, unsigned int* ticket, const double* skip, hipStream_t st) {
  if (!counts_ok(nb, nq, stride)) return hipErrorInvalidValue;
  int most = 0;
  for (int q = 0; q < nq; ++q) most = nb.nb[q] > most ? nb.nb[q] : most;
  const bool split = ticket && most > kFinOneBlockMax;
  hipLaunchKernelGGL(finalize_kernel, dim3(split ? nq : 1), dim3(kFinThreads), 0, st, part, stride, nb, nq, res, post,
                     F, gram, split ? ticket : nullptr, skip);
  return hipGetLastError();
}

// The slot counts of the records are checked where the host builds them.
hipError_t finalize_batched(const FinArgs* args, int nprob, int nq, int post, int F, hipStream_t st) {
  if (nq < 1 || nq > kMaxQ || nprob < 1 || nprob > 65535) return hipErrorInvalidValue;
  hipLaunchKernelGGL(finalize_batched_kernel, dim3(nprob), dim3(kFinThreads), 0, st, args, nq, post, F);
  return hipGetLastError();
}

// ----------------------------------------------------------------- projection
template <typename T, typename TX, bool NORM>
__device__ void run_op(const ProjArgs<T, TX, NORM>& a, int blk, int nblk) {
  const double alpha = a.coef ? a.coef[0] : a.c0, beta = a.coef ? a.coef[1] : a.c1;
  auto X = reinterpret_cast<const c_t<TX>*>(a.X);
  auto W = reinterpret_cast<const c_t<T>*>(a.W);
  auto out = reinterpret_cast<c_t<T>*>(a.out);
  const size_t n = a.npts;
  double acc[1] = {0.0};
  const size_t total = (size_t)(2 * a.F + 1) * n;
  for (size_t e = (size_t)blk * blockDim.x + threadIdx.x; e < total; e += (size_t)nblk * blockDim.x) {
    const int i = (int)(e / n);
    const T c = (T)(alpha + beta * (double)(a.F - i));
    const c_t<TX> x = X[e];
    c_t<T> w = W[e];
    w.x -= c * (T)x.x;
    w.y -= c * (T)x.y;
    out[e] = w;
    if (NORM) acc[0] += (double)cabs2(w);
  }
  if (NORM) block_partials_any<1>(acc, a.part, nblk, blk);
}

template <typename T, typename TX>
hipError_t project(int F, const void* X, const void* W, void* out, const double* coef, double* part, int nblk,
                   size_t npts, hipStream_t st) {
  if (part) return launch_single(ProjArgs<T, TX, true>{X, W, out, coef, 0.0, 0.0, part, npts, F}, nblk, st);
  return launch_single(ProjArgs<T, TX, false>{X, W, out, coef, 0.0, 0.0, nullptr, npts, F}, nblk, st);
}

// ----------------------------------------------------------------- retraction support
template <typename TU, typename TXI, int K>
__device__ void run_op(const NormsArgs<TU, TXI, K>& a, int blk, int nblk) {
  auto u = reinterpret_cast<const c_t<TU>*>(a.u);
  auto xi = reinterpret_cast<const c_t<TXI>*>(a.xi);
  const size_t n = a.npts;
  double acc[3 * K];
#pragma unroll
  for (int q = 0; q < 3 * K; ++q) acc[q] = 0.0;
  for (size_t j = (size_t)blk * blockDim.x + threadIdx.x; j < n; j += (size_t)nblk * blockDim.x) {
#pragma unroll
    for (int i = 0; i < K; ++i) {
      const c_t<TU> av = u[i * n + j];
      const double ax = av.x, ay = av.y;
      acc[i] += ax * ax + ay * ay;
      if (xi) {
        const c_t<TXI> b = xi[i * n + j];
        const double bx = b.x, by = b.y;
        acc[K + i] += ax * bx + ay * by;
        acc[2 * K + i] += bx * bx + by * by;
      }
    }
  }
  block_partials_any<3 * K>(acc, a.part, nblk, blk);
}

template <typename TU, typename TXI>
hipError_t comp_norms(int K, const void* u, const void* xi, double* part, int nblk, size_t npts, hipStream_t st) {
  switch (K) {
    case 3: return launch_single(NormsArgs<TU, TXI, 3>{u, xi, part, npts}, nblk, st);
    case 5: return launch_single(NormsArgs<TU, TXI, 5>{u, xi, part, npts}, nblk, st);
    case 7: return launch_single(NormsArgs<TU, TXI, 7>{u, xi, part, npts}, nblk, st);
    default: return hipErrorInvalidValue;
  }
}

template <typename TU, typename TXI, typename TO>
__device__ void run_op(const ScaleArgs<TU, TXI, TO>& a, int blk, int nblk) {
  auto u = reinterpret_cast<const c_t<TU>*>(a.u);
  auto xi = reinterpret_cast<const c_t<TXI>*>(a.xi);
  auto out = reinterpret_cast<c_t<TO>*>(a.out);
  const size_t n = a.npts;
  const size_t total = (size_t)a.K * n;
  for (size_t e = (size_t)blk * blockDim.x + threadIdx.x; e < total; e += (size_t)nblk * blockDim.x) {
    const int i = (int)(e / n);
    const double si = a.s[i];
    const c_t<TU> av = u[e];
    double re = av.x, im = av.y;
    if (xi) {
      const c_t<TXI> b = xi[e];
      re += a.t * (double)b.x;
      im += a.t * (double)b.y;
    }
    c_t<TO> r;
    r.x = (TO)(si * re);
    r.y = (TO)(si * im);
    out[e] = r;
  }
}

int elementwise_blocks(size_t total) {
  size_t g = (total + kRedThreads - 1) / kRedThreads;
  if (g > 8192) g = 8192;
  if (g < 1) g = 1;
  return (int)g;
}

template <typename TU, typename TXI, typename TO>
hipError_t scale_comps(int K, const void* u, const void* xi, double t, const double* s, void* out, size_t npts,
                       hipStream_t st) {
  ScaleArgs<TU, TXI, TO> a{u, xi, out, t, {0, 0, 0, 0, 0, 0, 0}, npts, K};
  for (int i = 0; i < K && i < 7; ++i) a.s[i] = s[i];
  return launch_single(a, elementwise_blocks((size_t)K * npts), st);
}

// ----------------------------------------------------------------- vector updates
template <typename T>
__device__ void run_op(const AxpbyArgs<T>& a, int blk, int nblk) {
  auto x = reinterpret_cast<const c_t<T>*>(a.x);
  auto y = reinterpret_cast<c_t<T>*>(a.y);
  const T ca = (T)a.a, cb = (T)a.b;
  const bool keep = a.b != 0.0;
  for (size_t e = (size_t)blk * blockDim.x + threadIdx.x; e < a.n; e += (size_t)nblk * blockDim.x) {
    const c_t<T> xv = x[e];
    c_t<T> yv;
    yv.x = ca * xv.x;
    yv.y = ca * xv.y;
    if (keep) {
      const c_t<T> old = y[e];
      yv.x += cb * old.x;
      yv.y += cb * old.y;
    }
    y[e] = yv;
  }
}

template <typename T>
hipError_t axpby(double a, const void* x, double b, void* y, size_t n, hipStream_t st) {
  return launch_single(AxpbyArgs<T>{x, y, a, b, n}, elementwise_blocks(n), st);
}

template <typename T>
__device__ void run_op(const CgArgs<T>& a, int blk, int nblk) {
  if (a.skip && *a.skip != 0.0) return;
  auto p = reinterpret_cast<const c_t<T>*>(a.p);
  auto q = reinterpret_cast<const c_t<T>*>(a.q);
  auto z = reinterpret_cast<c_t<T>*>(a.z);
  auto r = reinterpret_cast<c_t<T>*>(a.r);
  const T ca = (T)(a.adev ? *a.adev : a.a);
  double acc[1] = {0.0};
  // last element first: the HVP before this update ends on the last component
  for (size_t f = (size_t)blk * blockDim.x + threadIdx.x; f < a.n; f += (size_t)nblk * blockDim.x) {
    const size_t e = a.n - 1 - f;
    const c_t<T> qv = q[e];
    c_t<T> rv = r[e];
    if (z) {
      const c_t<T> pv = p[e];
      c_t<T> zv = z[e];
      zv.x += ca * pv.x;
      zv.y += ca * pv.y;
      z[e] = zv;
    }
    rv.x += ca * qv.x;
    rv.y += ca * qv.y;
    r[e] = rv;
    acc[0] += (double)rv.x * (double)rv.x + (double)rv.y * (double)rv.y;
  }
  block_partials_any<1>(acc, a.part, nblk, blk);
}

template <typename T>
__device__ void run_op(const CgDirArgs<T>& a, int blk, int nblk) {
  double* c = a.res;
  if (c[CG_IT] != (double)(a.iter + 1)) return;   // the iteration stopped before its update, or never ran
  const bool zupd = c[CG_CURV] == 0.0;
  if (!zupd) return;   // a curvature stop: neither z nor p changes
  bool pupd;
  double bv;
  if (a.part) {
    // the residual and cap tests from the update's partials (uniform: every
    // workgroup sums them in the same order; workgroup 0 stores the outcome,
    // in slots no workgroup of this launch reads: CG_REASON, CG_DONE, CG_BETA
    // and the next iteration's ||r||^2 slot)
    __shared__ double red[kRedThreads / kWave];
    double s = 0.0;
    for (int b = threadIdx.x; b < a.nb; b += blockDim.x) s += a.part[b];
    s = wave_sum(s);
    if (threadIdx.x % kWave == 0) red[threadIdx.x / kWave] = s;
    __syncthreads();
    double rr = 0.0;
    for (int w = 0; w < (int)(blockDim.x + kWave - 1) / kWave; ++w) rr += red[w];
    const int it = a.iter + 1;
    const bool res_stop = sqrt(rr) <= c[CG_TOL];
    bv = res_stop ? 0.0 : rr / c[cg_rr_slot(a.iter)];
    const bool cap_stop = !res_stop && (double)it >= c[CG_MAXIT];
    pupd = !res_stop && !cap_stop;
    if (blk == 0 && threadIdx.x == 0) {
      if (res_stop) {
        c[CG_REASON] = CG_STOP_RESIDUAL;
        c[CG_DONE] = 1.0;
      } else {
        c[CG_BETA] = bv;
        c[cg_rr_slot(it)] = rr;
        if (cap_stop) {
          c[CG_REASON] = CG_STOP_CAP;
          c[CG_DONE] = 1.0;
        }
      }
    }
  } else {
    pupd = c[CG_DONE] == 0.0;
    bv = c[CG_BETA];
  }
  auto r = reinterpret_cast<const c_t<T>*>(a.r);
  auto p = reinterpret_cast<c_t<T>*>(a.p);
  auto z = reinterpret_cast<c_t<T>*>(a.z);
  const T ca = (T)c[CG_ALPHA];
  const T cm = T(-1), cb = (T)bv;
  const bool keep = bv != 0.0;
  for (size_t e = (size_t)blk * blockDim.x + threadIdx.x; e < a.n; e += (size_t)nblk * blockDim.x) {
    const c_t<T> pv = p[e];
    if (zupd) {
      c_t<T> zv = z[e];
      zv.x += ca * pv.x;
      zv.y += ca * pv.y;
      z[e] = zv;
    }
    if (pupd) {
      const c_t<T> rv = r[e];
      c_t<T> v;
      v.x = cm * rv.x;
      v.y = cm * rv.y;
      if (keep) {
        v.x += cb * pv.x;
        v.y += cb * pv.y;
      }
      p[e] = v;
    }
  }
}

template <typename T>
hipError_t cg_update(double a, const void* p, const void* q, void* z, void* r, double* part, int nblk, size_t n,
                     hipStream_t st) {
  return launch_single(CgArgs<T>{p, q, z, r, part, a, n}, nblk, st);
}

__device__ void run_op(const CgInitArgs& a, int blk, int nblk) {
  if (blk != 0 || threadIdx.x != 0) return;
  double* c = a.res;
  c[CG_RR] = c[0];
  c[CG_RR1] = 0.0;
  c[CG_CURV] = 0.0;
  c[CG_IT] = 0.0;
  c[CG_TOL] = a.tol;
  c[CG_EPS] = a.eps;
  c[CG_MAXIT] = (double)a.maxit;
  c[CG_REASON] = a.maxit > 0 ? CG_STOP_NONE : CG_STOP_CAP;
  c[CG_DONE] = a.maxit > 0 ? 0.0 : 1.0;
}

template <typename TA, typename TB>
__device__ void run_op(const DotArgs<TA, TB>& a, int blk, int nblk) {
  auto x = reinterpret_cast<const c_t<TA>*>(a.a);
  auto y = reinterpret_cast<const c_t<TB>*>(a.b);
  double acc[1] = {0.0};
  for (size_t e = (size_t)blk * blockDim.x + threadIdx.x; e < a.n; e += (size_t)nblk * blockDim.x) {
    const c_t<TA> av = x[e];
    const c_t<TB> bv = y[e];
    acc[0] += (double)av.x * (double)bv.x + (double)av.y * (double)bv.y;
  }
  block_partials_any<1>(acc, a.part, nblk, blk);
}

template <typename TA, typename TB>
hipError_t dot(const void* a, const void* b, double* part, int nblk, size_t n, hipStream_t st) {
  return launch_single(DotArgs<TA, TB>{a, b, part, n}, nblk, st);
}

template <typename TA, typename TB, typename TO>
__device__ void run_op(const DiffArgs<TA, TB, TO>& a, int blk, int nblk) {
  auto x = reinterpret_cast<const c_t<TA>*>(a.a);
  auto y = reinterpret_cast<const c_t<TB>*>(a.b);
  auto o = reinterpret_cast<c_t<TO>*>(a.out);
  for (size_t e = (size_t)blk * blockDim.x + threadIdx.x; e < a.n; e += (size_t)nblk * blockDim.x) {
    const c_t<TA> av = x[e];
    const c_t<TB> bv = y[e];
    c_t<TO> r;
    r.x = (TO)((double)av.x - (double)bv.x);
    r.y = (TO)((double)av.y - (double)bv.y);
    o[e] = r;
  }
}

template <typename TA, typename TB, typename TO>
hipError_t diff(const void* a, const void* b, void* out, size_t n, hipStream_t st) {
  return launch_single(DiffArgs<TA, TB, TO>{a, b, out, n}, elementwise_blocks(n), st);
}

// Values for timing runs only: each element's index is mixed with the
// 32-bit finaliser of MurmurHash3 (the published constants), and the two
// 16-bit halves give the real and imaginary parts.
template <typename T>
__device__ void run_op(const FillArgs<T>& a, int blk, int nblk) {
  auto o = reinterpret_cast<c_t<T>*>(a.out);
  for (size_t e = (size_t)blk * blockDim.x + threadIdx.x; e < a.n; e += (size_t)nblk * blockDim.x) {
    uint32_t h = (uint32_t)e ^ (uint32_t)(e >> 32) * 0x9e3779b9u ^ a.seed;
    h ^= h >> 16;
    h *= 0x85ebca6bu;
    h ^= h >> 13;
    h *= 0xc2b2ae35u;
    h ^= h >> 16;
    c_t<T> r;
    r.x = (T)((int)(h & 0xffffu) - 32768) * (T)(1.0 / 32768);
    r.y = (T)((int)(h >> 16) - 32768) * (T)(1.0 / 32768);
    o[e] = r;
  }
}

template <typename TI, typename TO>
__device__ void run_op(const ConvArgs<TI, TO>& a, int blk, int nblk) {
  auto x = reinterpret_cast<const c_t<TI>*>(a.src);
  auto o = reinterpret_cast<c_t<TO>*>(a.dst);
  for (size_t e = (size_t)blk * blockDim.x + threadIdx.x; e < a.n; e += (size_t)nblk * blockDim.x) {
    c_t<TO> r;
    if (x) {
      const c_t<TI> v = x[e];
      r.x = (TO)v.x;
      r.y = (TO)v.y;
    } else {
      r.x = TO(0);
      r.y = TO(0);
    }
    o[e] = r;
  }
}

hipError_t to_c64(const void* src, void* dst, size_t n, hipStream_t st) {
  return launch_single(ConvArgs<double, float>{src, dst, n}, elementwise_blocks(n), st);
}

hipError_t to_c128(const void* src, void* dst, size_t n, hipStream_t st) {
  return launch_single(ConvArgs<float, double>{src, dst, n}, elementwise_blocks(n), st);
}

// ----------------------------------------------------------------- instantiations
GPE_OP(ProjArgs<double, double, true>)
GPE_OP(ProjArgs<double, double, false>)
GPE_OP(ProjArgs<float, float, true>)
GPE_OP(ProjArgs<float, float, false>)
GPE_OP(NormsArgs<double, double, 3>)
GPE_OP(NormsArgs<double, double, 5>)
GPE_OP(NormsArgs<double, double, 7>)
GPE_OP(NormsArgs<double, float, 3>)
GPE_OP(NormsArgs<double, float, 5>)
GPE_OP(NormsArgs<double, float, 7>)
GPE_OP(NormsArgs<float, float, 3>)
GPE_OP(NormsArgs<float, float, 5>)
GPE_OP(NormsArgs<float, float, 7>)
GPE_OP(ScaleArgs<double, double, double>)
GPE_OP(ScaleArgs<double, float, double>)
GPE_OP(ScaleArgs<float, float, float>)
GPE_OP(AxpbyArgs<double>)
GPE_OP(AxpbyArgs<float>)
GPE_OP(CgArgs<double>)
GPE_OP(CgArgs<float>)
GPE_OP(CgDirArgs<double>)
GPE_OP(CgDirArgs<float>)
GPE_OP(DotArgs<double, double>)
GPE_OP(DotArgs<float, float>)
GPE_OP(DotArgs<double, float>)
GPE_OP(DiffArgs<double, double, double>)
GPE_OP(DiffArgs<double, double, float>)
GPE_OP(ConvArgs<double, float>)
GPE_OP(ConvArgs<float, double>)
GPE_OP(ConvArgs<double, double>)
GPE_OP(ConvArgs<float, float>)
GPE_OP(CgInitArgs)
GPE_OP(FillArgs<double>)
GPE_OP(FillArgs<float>)

template hipError_t project<double, double>(int, const void*, const void*, void*, const double*, double*, int, size_t, hipStream_t);
template hipError_t project<float, float>(int, const void*, const void*, void*, const double*, double*, int, size_t, hipStream_t);
template hipError_t comp_norms<double, double>(int, const void*, const void*, double*, int, size_t, hipStream_t);
template hipError_t comp_norms<double, float>(int, const void*, const void*, double*, int, size_t, hipStream_t);
template hipError_t comp_norms<float, float>(int, const void*, const void*, double*, int, size_t, hipStream_t);
template hipError_t scale_comps<double, double, double>(int, const void*, const void*, double, const double*, void*, size_t, hipStream_t);
template hipError_t scale_comps<double, float, double>(int, const void*, const void*, double, const double*, void*, size_t, hipStream_t);
template hipError_t scale_comps<float, float, float>(int, const void*, const void*, double, const double*, void*, size_t, hipStream_t);
template hipError_t axpby<double>(double, const void*, double, void*, size_t, hipStream_t);
template hipError_t axpby<float>(double, const void*, double, void*, size_t, hipStream_t);
template hipError_t cg_update<double>(double, const void*, const void*, void*, void*, double*, int, size_t, hipStream_t);
template hipError_t cg_update<float>(double, const void*, const void*, void*, void*, double*, int, size_t, hipStream_t);
template hipError_t dot<double, double>(const void*, const void*, double*, int, size_t, hipStream_t);
template hipError_t dot<float, float>(const void*, const void*, double*, int, size_t, hipStream_t);
template hipError_t dot<double, float>(const void*, const void*, double*, int, size_t, hipStream_t);
template hipError_t diff<double, double, double>(const void*, const void*, void*, size_t, hipStream_t);
template hipError_t diff<double, double, float>(const void*, const void*, void*, size_t, hipStream_t);

}  // namespace gpe
