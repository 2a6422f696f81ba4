// Pointwise spin-F algebra shared by the pointwise kernels and the fused
// x-pass (Sec. 2 energies, Sec. 3 discrete forms).
//
// Per grid point the K = 2F+1 components are held in registers and the
// sparse structure of the spin matrices replaces dense K x K products:
//   rho  = sum |X_i|^2,  F_z = sum l_i |X_i|^2,
//   F_+  = F_x + i F_y = sum_i cr_i conj(X_{i-1}) X_i   (raising operator,
//          cr_i = sqrt(F(F+1) - m(m+1)) for m = l_i),
//   (F.f Y)_i = F_z l_i Y_i + 1/2 [conj(F_+) cr_{i+1} Y_{i+1} + F_+ cr_i Y_{i-1}],
//   A00  = X^T A X = sum_i s_i X_i X_{K-1-i},  s_i = (-1)^i / sqrt(K)   (F = 2, 3),
//   A2m  = X^T A_m X = sum_i a_m(i) X_i X_{6-m-i},  m = -2..2            (F = 3),
// where a_m are the anti-diagonal entries of the spin-3 matrices A_0, A_{+-1},
// A_{+-2} exactly as printed in Sec. 2 (A_0 centre entry sqrt(2/3)/sqrt(7)).
// Storage index i holds l_i = F - i.
#pragma once
#include "common.h"
#include "kernels.h"

namespace gpe {

template <int F> struct Spin;

template <> struct Spin<1> {
  static constexpr int K = 3;
};
template <> struct Spin<2> {
  static constexpr int K = 5;
};
template <> struct Spin<3> {
  static constexpr int K = 7;
};

// raising-operator coefficient cr_i (i = 1..K-1), couples storage i-1 <- i
template <int F> __host__ __device__ constexpr double raise_c(int i) {
  // F(F+1) - m(m+1) with m = F - i
  return (F == 1) ? 1.4142135623730950488
       : (F == 2) ? ((i == 1 || i == 4) ? 2.0 : 2.4494897427831780982)
       : ((i == 1 || i == 6) ? 2.4494897427831780982
          : (i == 2 || i == 5) ? 3.1622776601683793320 : 3.4641016151377545871);
}

// spin-3 quintet anti-diagonal coefficients a[m+2][i], pair partner 6 - m - i
// (entries of the printed matrices A_{-2}, A_{-1}, A_0, A_1, A_2, including their 1/sqrt 7)
__host__ __device__ constexpr double a2coef(int mi, int i) {
  constexpr double t[5][7] = {
      // m = -2: entries on i = 2..6: sqrt(5/6), -sqrt(5/3), sqrt(2), -sqrt(5/3), sqrt(5/6)
      {0.0, 0.0, 0.34503277967117707, -0.48795003647426659, 0.53452248382484879,
       -0.48795003647426659, 0.34503277967117707},
      // m = -1: i = 1..6: 5/(2 sqrt 3), -sqrt5/2, 1/sqrt6, 1/sqrt6, -sqrt5/2, 5/(2 sqrt 3)
      {0.0, 0.54554472558998102, -0.42257712736425829, 0.15430334996209191, 0.15430334996209191,
       -0.42257712736425829, 0.54554472558998102},
      // m = 0: i = 0..6: 5/(2 sqrt 3), 0, -sqrt3/2, sqrt(2/3), -sqrt3/2, 0, 5/(2 sqrt 3)
      {0.54554472558998102, 0.0, -0.32732683535398857, 0.30860669992418382, -0.32732683535398857,
       0.0, 0.54554472558998102},
      // m = 1: i = 0..5
      {0.54554472558998102, -0.42257712736425829, 0.15430334996209191, 0.15430334996209191,
       -0.42257712736425829, 0.54554472558998102, 0.0},
      // m = 2: i = 0..4
      {0.34503277967117707, -0.48795003647426659, 0.53452248382484879, -0.48795003647426659,
       0.34503277967117707, 0.0, 0.0}};
  return t[mi][i];
}

template <int F> __device__ constexpr double singlet_s(int i) {
  return ((i & 1) ? -1.0 : 1.0) / (F == 2 ? 2.2360679774997896964 : 2.6457513110645905905);
}

// Spin densities of one point.
template <typename T, int F> struct Dens {
  using T2 = c_t<T>;
  T rho, fz;
  T2 fp;        // F_+
  T2 a00;       // singlet pair amplitude
  T2 a2[5];     // quintet amplitudes (F = 3)
};

template <typename T, int F>
__device__ __forceinline__ void densities(const c_t<T> (&x)[2 * F + 1], Dens<T, F>& d) {
  using T2 = c_t<T>;
  constexpr int K = 2 * F + 1;
  d.rho = 0;
  d.fz = 0;
#pragma unroll
  for (int i = 0; i < K; ++i) {
    const T a = cabs2(x[i]);
    d.rho += a;
    d.fz += T(F - i) * a;
  }
  d.fp = mk<T2>(0, 0);
#pragma unroll
  for (int i = 1; i < K; ++i) {
    const T c = (T)raise_c<F>(i);
    d.fp = cadd(d.fp, cscale(cmulc(x[i - 1], x[i]), c));
  }
  if constexpr (F >= 2) {
    d.a00 = mk<T2>(0, 0);
#pragma unroll
    for (int i = 0; i < K; ++i) d.a00 = cadd(d.a00, cscale(cmul(x[i], x[K - 1 - i]), (T)singlet_s<F>(i)));
  }
  if constexpr (F == 3) {
#pragma unroll
    for (int mi = 0; mi < 5; ++mi) {
      T2 s = mk<T2>(0, 0);
#pragma unroll
      for (int i = 0; i < 7; ++i) {
        const int k = 8 - mi - i;
        if (k >= 0 && k < 7) s = cadd(s, cscale(cmul(x[i], x[k]), (T)a2coef(mi, i)));
      }
      d.a2[mi] = s;
    }
  }
}

// (F.f Y)_i with spin vector given by (fz, fp)
template <typename T, int F>
__device__ __forceinline__ c_t<T> ffy(T fz, c_t<T> fp, const c_t<T> (&y)[2 * F + 1], int i) {
  using T2 = c_t<T>;
  constexpr int K = 2 * F + 1;
  T2 r = cscale(y[i], fz * T(F - i));
  if (i + 1 < K) r = cadd(r, cscale(cmulc(fp, y[i + 1]), (T)(0.5 * raise_c<F>(i + 1))));
  if (i >= 1) r = cadd(r, cscale(cmul(fp, y[i - 1]), (T)(0.5 * raise_c<F>(i))));
  return r;
}


// Pointwise Hessian terms of the Sec. 3 HVP formula at one point, for all
// components: q_i = 2 (V + b_i) Z_i + zc_i Z_i + (2/h)[beta0 ... + beta3 ...]
// (the Laplacian term is added by the caller); sink(i, q_i) receives each.
template <typename T, int F, typename Sink>
__device__ __forceinline__ void hvp_point(const c_t<T> (&x)[2 * F + 1], const c_t<T> (&z)[2 * F + 1], T v,
                                          const PwParams& p, const T (&zcoef)[2 * F + 1], Sink&& sink) {
  using T2 = c_t<T>;
  constexpr int K = 2 * F + 1;
  Dens<T, F> d;
  densities<T, F>(x, d);
  T drho = 0, dfz = 0;
#pragma unroll
  for (int i = 0; i < K; ++i) {
    const T r = cdotr(z[i], x[i]);
    drho += r;
    dfz += T(F - i) * r;
  }
  drho *= T(2);
  dfz *= T(2);
  T2 dfp = mk<T2>(0, 0);
#pragma unroll
  for (int i = 1; i < K; ++i)
    dfp = cadd(dfp, cscale(cadd(cmulc(z[i - 1], x[i]), cmulc(x[i - 1], z[i])), (T)raise_c<F>(i)));
  T2 da00 = mk<T2>(0, 0);
  if constexpr (F >= 2) {
#pragma unroll
    for (int i = 0; i < K; ++i) da00 = cadd(da00, cscale(cmul(x[i], z[K - 1 - i]), T(2) * (T)singlet_s<F>(i)));
  }
  T2 da2[5];
  if constexpr (F == 3) {
#pragma unroll
    for (int mi = 0; mi < 5; ++mi) {
      T2 s = mk<T2>(0, 0);
#pragma unroll
      for (int i = 0; i < 7; ++i) {
        const int k = 8 - mi - i;
        if (k >= 0 && k < 7) s = cadd(s, cscale(cmul(x[i], z[k]), T(2) * (T)a2coef(mi, i)));
      }
      da2[mi] = s;
    }
  }
#pragma unroll
  for (int i = 0; i < K; ++i) {
    T2 w = cscale(z[i], T(2) * (v + (T)p.zee[i]) + zcoef[i]);
    T2 nl = cadd(cscale(z[i], (T)p.g[0] * d.rho), cscale(x[i], (T)p.g[0] * drho));
    nl = cadd(nl, cscale(cadd(ffy<T, F>(d.fz, d.fp, z, i), ffy<T, F>(dfz, dfp, x, i)), (T)p.g[1]));
    if constexpr (F >= 2) {
      const T sc = (T)p.g[2] * (T)singlet_s<F>(i);
      nl = cadd(nl, cscale(cadd(cmulc(z[K - 1 - i], d.a00), cmulc(x[K - 1 - i], da00)), sc));
    }
    if constexpr (F == 3) {
#pragma unroll
      for (int mi = 0; mi < 5; ++mi) {
        const int k = 8 - mi - i;
        if (k >= 0 && k < 7) {
          const T sc = (T)p.g[3] * (T)a2coef(mi, i);
          nl = cadd(nl, cscale(cadd(cmulc(z[k], d.a2[mi]), cmulc(x[k], da2[mi])), sc));
        }
      }
    }
    sink(i, cadd(w, nl));   // q_i is consumed at once, never held for all i
  }
}

}  // namespace gpe
