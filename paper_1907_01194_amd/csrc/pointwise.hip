// Pointwise energy density and gradient kernels (Sec. 3 discrete energy and
// gradient), built on the spin algebra of spin.h.  The pointwise part of the
// Hessian-vector product is fused into the x-axis Laplacian pass (lap.hip).
#include "spin.h"
#include "batch_ops.h"

namespace gpe {

template <typename T, int F, bool GRAD>
__device__ void run_op(const PwGradArgs<T, F, GRAD>& a, int blk, int nblk) {
  using T2 = c_t<T>;
  auto X = reinterpret_cast<const T2*>(a.X);
  auto LX = reinterpret_cast<const T2*>(a.LX);
  auto V = reinterpret_cast<const T*>(a.V);
  auto G = reinterpret_cast<T2*>(a.G);
  const size_t n = a.npts;
  const PwParams& p = a.p;
  constexpr int K = 2 * F + 1;
  constexpr int NQ = 1 + 2 * K;
  double acc[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) acc[q] = 0.0;
  for (size_t j = (size_t)blk * blockDim.x + threadIdx.x; j < n; j += (size_t)nblk * blockDim.x) {
    T2 x[K], lx[K];
#pragma unroll
    for (int i = 0; i < K; ++i) {
      x[i] = X[i * n + j];
      lx[i] = LX[i * n + j];
    }
    const T v = V[j];
    Dens<T, F> d;
    densities<T, F>(x, d);
    T e = 0;
#pragma unroll
    for (int i = 0; i < K; ++i) e += T(0.5) * cdotr(lx[i], x[i]) + (v + (T)p.zee[i]) * cabs2(x[i]);
    T inter = (T)p.e[0] * d.rho * d.rho + (T)p.e[1] * (d.fz * d.fz + cabs2(d.fp));
    if constexpr (F >= 2) inter += (T)p.e[2] * cabs2(d.a00);
    if constexpr (F == 3) {
      T s = 0;
#pragma unroll
      for (int mi = 0; mi < 5; ++mi) s += cabs2(d.a2[mi]);
      inter += (T)p.e[3] * s;
    }
    acc[0] += (double)e + (double)inter;
#pragma unroll
    for (int i = 0; i < K; ++i) acc[1 + K + i] += (double)cabs2(x[i]);
    if constexpr (GRAD) {
#pragma unroll
      for (int i = 0; i < K; ++i) {
        T2 g = cadd(lx[i], cscale(x[i], T(2) * (v + (T)p.zee[i])));
        T2 nl = cscale(x[i], (T)p.g[0] * d.rho);
        nl = cadd(nl, cscale(ffy<T, F>(d.fz, d.fp, x, i), (T)p.g[1]));
        if constexpr (F >= 2)
          nl = cadd(nl, cscale(cmulc(x[K - 1 - i], d.a00), (T)p.g[2] * (T)singlet_s<F>(i)));
        if constexpr (F == 3) {
#pragma unroll
          for (int mi = 0; mi < 5; ++mi) {
            const int k = 8 - mi - i;
            if (k >= 0 && k < 7) nl = cadd(nl, cscale(cmulc(x[k], d.a2[mi]), (T)p.g[3] * (T)a2coef(mi, i)));
          }
        }
        g = cadd(g, nl);
        G[i * n + j] = g;
        acc[1 + i] += (double)cdotr(x[i], g);
      }
    }
  }
  block_partials_any<NQ>(acc, a.part, nblk, blk);
}

template <typename T>
hipError_t pw_grad(int F, const void* X, const void* LX, const T* V, void* G, double* part, int nblk,
                   size_t npts, const PwParams& p, hipStream_t st) {
#define GPE_LAUNCH(FF)                                                                             \
  return G ? launch_single(PwGradArgs<T, FF, true>{X, LX, V, G, part, npts, p}, nblk, st)         \
           : launch_single(PwGradArgs<T, FF, false>{X, LX, V, G, part, npts, p}, nblk, st);
  switch (F) {
    case 1: GPE_LAUNCH(1)
    case 2: GPE_LAUNCH(2)
    case 3: GPE_LAUNCH(3)
    default: return hipErrorInvalidValue;
  }
#undef GPE_LAUNCH
}

GPE_OP(PwGradArgs<double, 1, true>)
GPE_OP(PwGradArgs<double, 2, true>)
GPE_OP(PwGradArgs<double, 3, true>)
GPE_OP(PwGradArgs<double, 1, false>)
GPE_OP(PwGradArgs<double, 2, false>)
GPE_OP(PwGradArgs<double, 3, false>)
GPE_OP(PwGradArgs<float, 1, true>)
GPE_OP(PwGradArgs<float, 2, true>)
GPE_OP(PwGradArgs<float, 3, true>)
GPE_OP(PwGradArgs<float, 1, false>)
GPE_OP(PwGradArgs<float, 2, false>)
GPE_OP(PwGradArgs<float, 3, false>)
template hipError_t pw_grad<double>(int, const void*, const void*, const double*, void*, double*, int, size_t,
                                    const PwParams&, hipStream_t);
template hipError_t pw_grad<float>(int, const void*, const void*, const float*, void*, double*, int, size_t,
                                   const PwParams&, hipStream_t);
}  // namespace gpe
