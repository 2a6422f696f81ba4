// Scalar part of the retractions of Sec. 6 (see retract_scalar.h).
#include "retract_scalar.h"

#include <cmath>

namespace gpe {

// h1(t) = sum (l-M) a_l / (1-(l-M)t)^2 increases on the interval between its
// poles 1/(f1-M) < 0 < 1/(f2-M).  The zero is sought in w = t - 1/(fa-M), the
// offset from one pole (fa = f2 if the mass below M outweighs the mass above,
// else f1: the zero then lies nearer that pole), with
//   d_l = 1 - (l-M) t = (1 - (l-M)/(fa-M)) - (l-M) w,   d_fa = -(fa-M) w,
// so that the d_l of the components next to the pole keep their relative
// accuracy even when the norms on one side of M are tiny.  A safeguarded
// Newton iteration (bisection whenever the Newton point leaves the bracket)
// finds the zero to the last bits.
int sigma_projective(int F, double M, const double* a, double* sig) {
  const int K = 2 * F + 1;
  int f1 = 1 << 20, f2 = -(1 << 20);
  double below = 0.0, above = 0.0;
  for (int i = 0; i < K; ++i)
    if (a[i] > 0) {
      const int l = F - i;
      if (l < f1) f1 = l;
      if (l > f2) f2 = l;
      if (l < M) below += a[i];
      if (l > M) above += a[i];
    }
  if (!(f1 < M && f2 > M)) return SIGMA_DOMAIN;
  const int fa = below >= above ? f2 : f1;
  const double ca = fa - M;
  double off[7];   // 1 - (l-M)/(fa-M), exactly 0 at the anchor
  for (int i = 0; i < K; ++i) off[i] = (F - i) == fa ? 0.0 : 1.0 - ((F - i) - M) / ca;
  auto dl = [&](int i, double w) { return off[i] - ((F - i) - M) * w; };
  // bracket in w: t in (1/(f1-M), 1/(f2-M)), open at both poles
  double lo = fa == f2 ? 1.0 / (f1 - M) - 1.0 / ca : 0.0;
  double hi = fa == f2 ? 0.0 : 1.0 / (f2 - M) - 1.0 / ca;
  double w = 0.5 * (lo + hi);
  for (int it = 0; it < 400; ++it) {
    double f = 0.0, df = 0.0;
    for (int i = 0; i < K; ++i) {
      if (!(a[i] > 0)) continue;
      const double c = (F - i) - M;
      const double d = dl(i, w);
      f += c * a[i] / (d * d);
      df += 2.0 * c * c * a[i] / (d * d * d);
    }
    if (f == 0.0) break;
    if (f > 0) hi = w;
    else lo = w;
    double wn = w - f / df;
    if (!(wn > lo && wn < hi)) wn = 0.5 * (lo + hi);
    const bool done = std::fabs(wn - w) <= 4e-16 * std::fabs(w);
    w = wn;
    if (done || hi - lo <= 4e-16 * std::fmax(std::fabs(lo), std::fabs(hi))) break;
  }
  double s = 0.0;
  for (int i = 0; i < K; ++i) {
    if (!(a[i] > 0)) continue;
    const double d = dl(i, w);
    s += a[i] / (d * d);
  }
  const double rs = 1.0 / std::sqrt(s);
  for (int i = 0; i < K; ++i) {
    const int l = F - i;
    sig[i] = (l >= f1 && l <= f2) ? rs / dl(i, w) : 0.0;
  }
  return SIGMA_OK;
}

// h2(t) t^{-F} has the same positive zero as sum (l-M) a_l t^l; in s = ln t
// that sum changes sign exactly once, so bisection on s finds it.  Every term
// is formed in the log domain, a_l e^{l s} = exp(ln a_l + l s), scaled by the
// largest exponent, so that neither the norms' range nor s over- or
// underflows.
int sigma_orthogonal(int F, double M, const double* a, double* sig) {
  const int K = 2 * F + 1;
  double below = 0, above = 0;
  for (int i = 0; i < K; ++i) {
    if ((F - i) < M) below += a[i];
    if ((F - i) > M) above += a[i];
  }
  if (!(below > 0 && above > 0)) return SIGMA_DOMAIN;
  double la[7];
  for (int i = 0; i < K; ++i) la[i] = a[i] > 0 ? std::log(a[i]) : -INFINITY;
  auto top = [&](double s) {
    double mx = -INFINITY;
    for (int i = 0; i < K; ++i)
      if (a[i] > 0) mx = std::fmax(mx, la[i] + (F - i) * s);
    return mx;
  };
  auto g = [&](double s) {
    const double mx = top(s);
    double v = 0.0;
    for (int i = 0; i < K; ++i)
      if (a[i] > 0) v += ((F - i) - M) * std::exp(la[i] + (F - i) * s - mx);
    return v;
  };
  double lo = -1.0, hi = 1.0;
  while (g(lo) > 0 && lo > -1e6) lo *= 2;
  while (g(hi) < 0 && hi < 1e6) hi *= 2;
  for (int it = 0; it < 200; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (mid == lo || mid == hi) break;
    if (g(mid) > 0) hi = mid;
    else lo = mid;
  }
  const double s = 0.5 * (lo + hi);
  // sigma_l^2 = e^{l s} / sum_k a_k e^{k s} = exp(l s - mx - ln sum_k exp(ln a_k + k s - mx))
  const double mx = top(s);
  double den = 0.0;
  for (int i = 0; i < K; ++i)
    if (a[i] > 0) den += std::exp(la[i] + (F - i) * s - mx);
  const double lden = mx + std::log(den);
  // an empty component stays empty: its factor is set to 0, never to a value
  // that could overflow and turn 0 * inf into NaN in the scaling kernel
  for (int i = 0; i < K; ++i) sig[i] = a[i] > 0 ? std::exp(0.5 * ((F - i) * s - lden)) : 0.0;
  return SIGMA_OK;
}

// eq. retract3 with its sums regrouped so that no large terms cancel:
//   w^T w w^T G^2 w - (w^T G w)^2 = sum_{j<k} a_j a_k (l_j - l_k)^2   (Lagrange's identity),
//   w^T G^2 w - (M+l) w^T G w + M l w^T w = sum_k a_k (l_k - M)(l_k - l),
// the same values, but accurate when one component carries almost all the mass.
int sigma_closed(int F, double M, const double* a, double* sig) {
  const int K = 2 * F + 1;
  double den = 0.0;
  for (int j = 0; j < K; ++j)
    for (int k = j + 1; k < K; ++k) den += a[j] * a[k] * double((k - j) * (k - j));
  auto num = [&](double l) {
    double v = 0.0;
    for (int k = 0; k < K; ++k) v += a[k] * (((F - k) - M) * ((F - k) - l));
    return v;
  };
  if (!(num(F) > 0 && num(-F) > 0 && den > 0)) return SIGMA_DOMAIN;
  for (int i = 0; i < K; ++i) sig[i] = std::sqrt(num(F - i) / den);
  return SIGMA_OK;
}

}  // namespace gpe
