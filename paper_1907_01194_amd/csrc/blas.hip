// Field-level kernels: deterministic FP64 reductions (block partial sums, one
// single-block finalize), the tangent-space projection of Lemma 4.1, the
// componentwise scaling of the retractions (Sec. 6), CG vector updates and
// precision conversions.  All reductions accumulate in FP64 whatever the
// field precision.
#include "common.h"
#include "kernels.h"

namespace gpe {

template <typename T> struct C7 { T v[7]; };

// ----------------------------------------------------------------- finalize
// One block per slot sums that slot's partials in a fixed order (so results
// are bitwise reproducible); the last block to finish (counted with an atomic
// ticket, which it resets) applies the post-operation.
constexpr int kFinThreads = 256;

__global__ void __launch_bounds__(kFinThreads)
finalize_kernel(const double* __restrict__ part, size_t stride, SlotCounts nb, int nq, double* __restrict__ res,
                int post, int F, double* gram, unsigned int* ticket) {
  __shared__ double red[kFinThreads / kWave];
  __shared__ bool last;
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
  double s = wave_sum((s0 + s1) + (s2 + s3));
  if (threadIdx.x % kWave == 0) red[threadIdx.x / kWave] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < kFinThreads / kWave; ++w) t += red[w];
    res[q] = t;
    __threadfence();
    last = atomicAdd(ticket, 1u) == (unsigned)(nq - 1);
  }
  __syncthreads();
  if (!last || threadIdx.x != 0) return;
  *ticket = 0u;   // every block of this launch has taken its ticket
  __threadfence();
  const volatile double* out = res;
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
  } else if (post == POST_HVP_KAPPA) {
    double zlz = 0.0;
    for (int k = 6; k < nq; ++k) zlz += out[k];
    res[34] = out[4] + zlz - out[32] * out[2] - out[33] * out[3];
    res[35] = out[5];
  }
}

hipError_t finalize(const double* part, size_t stride, const SlotCounts& nb, int nq, double* res, int post, int F,
                    double* gram, unsigned int* ticket, hipStream_t st) {
  if (nq < 1 || nq > kMaxQ || nq > (int)(sizeof(nb.nb) / sizeof(nb.nb[0]))) return hipErrorInvalidValue;
  for (int q = 0; q < nq; ++q)
    if (nb.nb[q] < 0 || (size_t)nb.nb[q] > stride) return hipErrorInvalidValue;
  hipLaunchKernelGGL(finalize_kernel, dim3(nq), dim3(kFinThreads), 0, st, part, stride, nb, nq, res, post, F, gram,
                     ticket);
  return hipGetLastError();
}

// ----------------------------------------------------------------- projection
template <typename T, typename TX, bool NORM>
__global__ void __launch_bounds__(kRedThreads)
project_kernel(int K, int F, const c_t<TX>* __restrict__ X, const c_t<T>* W, c_t<T>* out,
               const double* __restrict__ coef, double* __restrict__ part, int nblk, size_t n) {
  const double alpha = coef[0], beta = coef[1];
  double acc[1] = {0.0};
  const size_t total = (size_t)K * n;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
    const int i = (int)(e / n);
    const T c = (T)(alpha + beta * (double)(F - i));
    const c_t<TX> x = X[e];
    c_t<T> w = W[e];
    w.x -= c * (T)x.x;
    w.y -= c * (T)x.y;
    out[e] = w;
    if (NORM) acc[0] += (double)cabs2(w);
  }
  if (NORM) block_partials<1>(acc, part, nblk);
}

template <typename T, typename TX>
hipError_t project(int F, const void* X, const void* W, void* out, const double* coef, double* part, int nblk,
                   size_t npts, hipStream_t st) {
  const int K = 2 * F + 1;
  auto x = reinterpret_cast<const c_t<TX>*>(X);
  auto w = reinterpret_cast<const c_t<T>*>(W);
  auto o = reinterpret_cast<c_t<T>*>(out);
  if (part)
    hipLaunchKernelGGL((project_kernel<T, TX, true>), dim3(nblk), dim3(kRedThreads), 0, st, K, F, x, w, o, coef,
                       part, nblk, npts);
  else
    hipLaunchKernelGGL((project_kernel<T, TX, false>), dim3(nblk), dim3(kRedThreads), 0, st, K, F, x, w, o, coef,
                       part, nblk, npts);
  return hipGetLastError();
}

// ----------------------------------------------------------------- retraction support
template <typename TU, typename TXI, int K>
__global__ void __launch_bounds__(kRedThreads)
comp_norms_kernel(const c_t<TU>* __restrict__ u, const c_t<TXI>* __restrict__ xi, double* __restrict__ part,
                  int nblk, size_t n) {
  double acc[3 * K];
#pragma unroll
  for (int q = 0; q < 3 * K; ++q) acc[q] = 0.0;
  for (size_t j = (size_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += (size_t)gridDim.x * blockDim.x) {
#pragma unroll
    for (int i = 0; i < K; ++i) {
      const c_t<TU> a = u[i * n + j];
      const double ax = a.x, ay = a.y;
      acc[i] += ax * ax + ay * ay;
      if (xi) {
        const c_t<TXI> b = xi[i * n + j];
        const double bx = b.x, by = b.y;
        acc[K + i] += ax * bx + ay * by;
        acc[2 * K + i] += bx * bx + by * by;
      }
    }
  }
  block_partials<3 * K>(acc, part, nblk);
}

template <typename TU, typename TXI>
hipError_t comp_norms(int K, const void* u, const void* xi, double* part, int nblk, size_t npts, hipStream_t st) {
  auto a = reinterpret_cast<const c_t<TU>*>(u);
  auto b = reinterpret_cast<const c_t<TXI>*>(xi);
  switch (K) {
    case 3: hipLaunchKernelGGL((comp_norms_kernel<TU, TXI, 3>), dim3(nblk), dim3(kRedThreads), 0, st, a, b, part, nblk, npts); break;
    case 5: hipLaunchKernelGGL((comp_norms_kernel<TU, TXI, 5>), dim3(nblk), dim3(kRedThreads), 0, st, a, b, part, nblk, npts); break;
    case 7: hipLaunchKernelGGL((comp_norms_kernel<TU, TXI, 7>), dim3(nblk), dim3(kRedThreads), 0, st, a, b, part, nblk, npts); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename TU, typename TXI, typename TO>
__global__ void scale_comps_kernel(int K, const c_t<TU>* u, const c_t<TXI>* __restrict__ xi, double t, C7<double> s,
                                   c_t<TO>* out, size_t n) {
  const size_t total = (size_t)K * n;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
    const int i = (int)(e / n);
    const double si = s.v[i];
    const c_t<TU> a = u[e];
    double re = a.x, im = a.y;
    if (xi) {
      const c_t<TXI> b = xi[e];
      re += t * (double)b.x;
      im += t * (double)b.y;
    }
    c_t<TO> r;
    r.x = (TO)(si * re);
    r.y = (TO)(si * im);
    out[e] = r;
  }
}

static inline int grid_for(size_t total, int threads = 256) {
  size_t g = (total + threads - 1) / threads;
  if (g > 8192) g = 8192;
  if (g < 1) g = 1;
  return (int)g;
}

template <typename TU, typename TXI, typename TO>
hipError_t scale_comps(int K, const void* u, const void* xi, double t, const double* s, void* out, size_t npts,
                       hipStream_t st) {
  C7<double> sv;
  for (int i = 0; i < 7; ++i) sv.v[i] = i < K ? s[i] : 0.0;
  hipLaunchKernelGGL((scale_comps_kernel<TU, TXI, TO>), dim3(grid_for((size_t)K * npts)), dim3(256), 0, st, K,
                     reinterpret_cast<const c_t<TU>*>(u), reinterpret_cast<const c_t<TXI>*>(xi), t, sv,
                     reinterpret_cast<c_t<TO>*>(out), npts);
  return hipGetLastError();
}

// ----------------------------------------------------------------- vector updates
template <typename T>
__global__ void axpby_kernel(T a, const c_t<T>* __restrict__ x, T b, c_t<T>* y, size_t n) {
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x) {
    const c_t<T> xv = x[e];
    c_t<T> yv = y[e];
    yv.x = a * xv.x + b * yv.x;
    yv.y = a * xv.y + b * yv.y;
    y[e] = yv;
  }
}

template <typename T>
hipError_t axpby(double a, const void* x, double b, void* y, size_t n, hipStream_t st) {
  hipLaunchKernelGGL((axpby_kernel<T>), dim3(grid_for(n)), dim3(256), 0, st, (T)a,
                     reinterpret_cast<const c_t<T>*>(x), (T)b, reinterpret_cast<c_t<T>*>(y), n);
  return hipGetLastError();
}

template <typename T>
__global__ void __launch_bounds__(kRedThreads)
cg_update_kernel(T a, const c_t<T>* __restrict__ p, const c_t<T>* __restrict__ q, c_t<T>* __restrict__ z,
                 c_t<T>* __restrict__ r, double* __restrict__ part, int nblk, size_t n) {
  double acc[1] = {0.0};
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x) {
    const c_t<T> pv = p[e], qv = q[e];
    c_t<T> zv = z[e], rv = r[e];
    zv.x += a * pv.x;
    zv.y += a * pv.y;
    rv.x += a * qv.x;
    rv.y += a * qv.y;
    z[e] = zv;
    r[e] = rv;
    acc[0] += (double)rv.x * (double)rv.x + (double)rv.y * (double)rv.y;
  }
  block_partials<1>(acc, part, nblk);
}

template <typename T>
hipError_t cg_update(double a, const void* p, const void* q, void* z, void* r, double* part, int nblk, size_t n,
                     hipStream_t st) {
  hipLaunchKernelGGL((cg_update_kernel<T>), dim3(nblk), dim3(kRedThreads), 0, st, (T)a,
                     reinterpret_cast<const c_t<T>*>(p), reinterpret_cast<const c_t<T>*>(q),
                     reinterpret_cast<c_t<T>*>(z), reinterpret_cast<c_t<T>*>(r), part, nblk, n);
  return hipGetLastError();
}

template <typename TA, typename TB>
__global__ void __launch_bounds__(kRedThreads)
dot_kernel(const c_t<TA>* __restrict__ a, const c_t<TB>* __restrict__ b, double* __restrict__ part, int nblk,
           size_t n) {
  double acc[1] = {0.0};
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x) {
    const c_t<TA> av = a[e];
    const c_t<TB> bv = b[e];
    acc[0] += (double)av.x * (double)bv.x + (double)av.y * (double)bv.y;
  }
  block_partials<1>(acc, part, nblk);
}

template <typename TA, typename TB>
hipError_t dot(const void* a, const void* b, double* part, int nblk, size_t n, hipStream_t st) {
  hipLaunchKernelGGL((dot_kernel<TA, TB>), dim3(nblk), dim3(kRedThreads), 0, st,
                     reinterpret_cast<const c_t<TA>*>(a), reinterpret_cast<const c_t<TB>*>(b), part, nblk, n);
  return hipGetLastError();
}

template <typename TA, typename TB, typename TO>
__global__ void diff_kernel(const c_t<TA>* __restrict__ a, const c_t<TB>* __restrict__ b, c_t<TO>* __restrict__ o,
                            size_t n) {
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x) {
    const c_t<TA> av = a[e];
    const c_t<TB> bv = b[e];
    c_t<TO> r;
    r.x = (TO)((double)av.x - (double)bv.x);
    r.y = (TO)((double)av.y - (double)bv.y);
    o[e] = r;
  }
}

template <typename TA, typename TB, typename TO>
hipError_t diff(const void* a, const void* b, void* out, size_t n, hipStream_t st) {
  hipLaunchKernelGGL((diff_kernel<TA, TB, TO>), dim3(grid_for(n)), dim3(256), 0, st,
                     reinterpret_cast<const c_t<TA>*>(a), reinterpret_cast<const c_t<TB>*>(b),
                     reinterpret_cast<c_t<TO>*>(out), n);
  return hipGetLastError();
}

template <typename TI, typename TO>
__global__ void convert_kernel(const c_t<TI>* __restrict__ a, c_t<TO>* __restrict__ o, size_t n) {
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x) {
    const c_t<TI> v = a[e];
    c_t<TO> r;
    r.x = (TO)v.x;
    r.y = (TO)v.y;
    o[e] = r;
  }
}

hipError_t to_c64(const void* src, void* dst, size_t n, hipStream_t st) {
  hipLaunchKernelGGL((convert_kernel<double, float>), dim3(grid_for(n)), dim3(256), 0, st,
                     reinterpret_cast<const double2*>(src), reinterpret_cast<float2*>(dst), n);
  return hipGetLastError();
}

hipError_t to_c128(const void* src, void* dst, size_t n, hipStream_t st) {
  hipLaunchKernelGGL((convert_kernel<float, double>), dim3(grid_for(n)), dim3(256), 0, st,
                     reinterpret_cast<const float2*>(src), reinterpret_cast<double2*>(dst), n);
  return hipGetLastError();
}

// ----------------------------------------------------------------- instantiations
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
