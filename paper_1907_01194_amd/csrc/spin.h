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
#include <type_traits>

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


// Compile-time loop: fn(std::integral_constant<int, I>) for I = B .. E-1.
template <int B, int E, typename Fn> __device__ __forceinline__ void sfor(Fn&& fn) {
  if constexpr (B < E) {
    fn(std::integral_constant<int, B>{});
    sfor<B + 1, E>(fn);
  }
}

// acc += s conj(a) b and acc += s a b for real s (FMA-shaped).
template <typename T2, typename S> __device__ __forceinline__ void acc_cjmul(T2& acc, T2 a, T2 b, S s) {
  acc.x += s * (a.x * b.x + a.y * b.y);
  acc.y += s * (a.x * b.y - a.y * b.x);
}
template <typename T2, typename S> __device__ __forceinline__ void acc_mul(T2& acc, T2 a, T2 b, S s) {
  acc.x += s * (a.x * b.x - a.y * b.y);
  acc.y += s * (a.x * b.y + a.y * b.x);
}
// s (a b + c d)
template <typename T2, typename S> __device__ __forceinline__ void acc_mul2(T2& acc, T2 a, T2 b, T2 c, T2 d, S s) {
  acc.x += s * ((a.x * b.x - a.y * b.y) + (c.x * d.x - c.y * d.y));
  acc.y += s * ((a.x * b.y + a.y * b.x) + (c.x * d.y + c.y * d.x));
}
// s (conj(a) b + conj(c) d)
template <typename T2, typename S> __device__ __forceinline__ void acc_cjmul2(T2& acc, T2 a, T2 b, T2 c, T2 d, S s) {
  acc.x += s * ((a.x * b.x + a.y * b.y) + (c.x * d.x + c.y * d.y));
  acc.y += s * ((a.x * b.y - a.y * b.x) + (c.x * d.y - c.y * d.x));
}

// Pointwise Hessian terms of the Sec. 3 HVP formula at one point, for all
// components: q_i = 2 (V + b_i) Z_i + zc_i Z_i + (2/h)[beta0 ... + beta3 ...]
// (the Laplacian term is added by the caller); sink(i, q_i) receives each.
//
// Written for few operations: the densities of X and their derivatives along
// Z are scaled once by their coupling constants; the pair amplitudes use the
// symmetry of the singlet vector and of the matrices A_m (entry (i, k) equals
// entry (k, i), so each unordered pair is formed once), and zero matrix
// entries are skipped at compile time.  The algebra is the formula's own.
template <typename T, int F, typename Sink>
__device__ __forceinline__ void hvp_point(const c_t<T> (&x)[2 * F + 1], const c_t<T> (&z)[2 * F + 1], T v,
                                          const PwParams& p, const T (&zcoef)[2 * F + 1], Sink&& sink) {
  using T2 = c_t<T>;
  constexpr int K = 2 * F + 1;
  // rho, F_z and their derivatives d rho = 2 Re sum Z conj X, d F_z likewise
  T rho = 0, fz = 0, drho = 0, dfz = 0;
#pragma unroll
  for (int i = 0; i < K; ++i) {
    const T a = x[i].x * x[i].x + x[i].y * x[i].y;
    const T r = z[i].x * x[i].x + z[i].y * x[i].y;
    rho += a;
    fz += T(F - i) * a;
    drho += r;
    dfz += T(F - i) * r;
  }
  // F_+ = sum cr_i conj(X_{i-1}) X_i and its derivative, both times g1 / 2
  T2 hfp = mk<T2>(0, 0), hdfp = mk<T2>(0, 0);
  sfor<1, K>([&](auto I) {
    constexpr int i = I;
    constexpr double c = raise_c<F>(i);
    acc_cjmul(hfp, x[i - 1], x[i], (T)c);
    acc_cjmul2(hdfp, z[i - 1], x[i], x[i - 1], z[i], (T)c);
  });
  const T g1h = T(0.5) * (T)p.g[1];
  hfp = cscale(hfp, g1h);
  hdfp = cscale(hdfp, g1h);
  const T cz0 = (T)p.g[0] * rho, cfz = (T)p.g[1] * fz;
  const T cx0 = T(2) * (T)p.g[0] * drho, cdfz = T(2) * (T)p.g[1] * dfz;
  // singlet amplitude A00 = sum s_i X_i X_{K-1-i} and dA00 = 2 sum s_i X_i Z_{K-1-i}, times g2
  T2 sa = mk<T2>(0, 0), sda = mk<T2>(0, 0);
  if constexpr (F >= 2) {
    sfor<0, F>([&](auto I) {
      constexpr int i = I;
      constexpr double s2 = 2.0 * singlet_s<F>(i);
      acc_mul(sa, x[i], x[K - 1 - i], (T)s2);
      acc_mul2(sda, x[i], z[K - 1 - i], x[K - 1 - i], z[i], (T)s2);
    });
    constexpr double sm = singlet_s<F>(F);
    acc_mul(sa, x[F], x[F], (T)sm);
    acc_mul(sda, x[F], z[F], (T)(2.0 * sm));
    sa = cscale(sa, (T)p.g[2]);
    sda = cscale(sda, (T)p.g[2]);
  }
  // quintet amplitudes A2m = sum a_m(i) X_i X_k (k = 8 - mi - i) and dA2m = 2 sum a_m(i) X_i Z_k, times g3
  T2 b2[5], db2[5];
  if constexpr (F == 3) {
    sfor<0, 5>([&](auto MI) {
      constexpr int mi = MI;
      T2 b = mk<T2>(0, 0), db = mk<T2>(0, 0);
      sfor<0, 7>([&](auto I) {
        constexpr int i = I;
        constexpr int k = 8 - mi - i;
        if constexpr (k >= 0 && k < 7 && i <= k && a2coef(mi, i) != 0.0) {
          constexpr double a = a2coef(mi, i);
          if constexpr (i < k) {
            acc_mul(b, x[i], x[k], (T)(2.0 * a));
            acc_mul2(db, x[i], z[k], x[k], z[i], (T)(2.0 * a));
          } else {
            acc_mul(b, x[i], x[i], (T)a);
            acc_mul(db, x[i], z[i], (T)(2.0 * a));
          }
        }
      });
      b2[mi] = cscale(b, (T)p.g[3]);
      db2[mi] = cscale(db, (T)p.g[3]);
    });
  }
  sfor<0, K>([&](auto I) {
    constexpr int i = I;
    constexpr T l = T(F - i);
    const T cz = T(2) * (v + (T)p.zee[i]) + zcoef[i] + cz0 + l * cfz;
    const T cx = cx0 + l * cdfz;
    T2 q = mk<T2>(cz * z[i].x + cx * x[i].x, cz * z[i].y + cx * x[i].y);
    // spin-density terms: ((F.f) Z + (dF.f) X)_i, the F_z part folded into cz and cx above
    if constexpr (i + 1 < K) acc_cjmul2(q, hfp, z[i + 1], hdfp, x[i + 1], (T)raise_c<F>(i + 1));
    if constexpr (i >= 1) acc_mul2(q, hfp, z[i - 1], hdfp, x[i - 1], (T)raise_c<F>(i));
    if constexpr (F >= 2) acc_cjmul2(q, z[K - 1 - i], sa, x[K - 1 - i], sda, (T)singlet_s<F>(i));
    if constexpr (F == 3) {
      sfor<0, 5>([&](auto MI) {
        constexpr int mi = MI;
        constexpr int k = 8 - mi - i;
        if constexpr (k >= 0 && k < 7 && a2coef(mi, i) != 0.0)
          acc_cjmul2(q, z[k], b2[mi], x[k], db2[mi], (T)a2coef(mi, i));
      });
    }
    sink(i, q);   // q_i is consumed at once, never held for all i
  });
}

}  // namespace gpe
