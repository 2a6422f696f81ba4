// Host-only driver of the retraction scalar solves (retract_scalar.cpp) for
// the sanitizer test: each input line "kind F M a_0 .. a_{2F}" gives one line
// "status sigma_0 .. sigma_{2F}" (17 significant digits).
#include <cstdio>

#include "retract_scalar.h"

int main() {
  int kind, F;
  double M;
  while (std::scanf("%d %d %lf", &kind, &F, &M) == 3) {
    if (F < 1 || F > 3) return 2;
    const int K = 2 * F + 1;
    double a[7], sig[7] = {0, 0, 0, 0, 0, 0, 0};
    for (int i = 0; i < K; ++i)
      if (std::scanf("%lf", &a[i]) != 1) return 2;
    int st = kind == 1 ? gpe::sigma_projective(F, M, a, sig)
           : kind == 2 ? gpe::sigma_orthogonal(F, M, a, sig)
                       : gpe::sigma_closed(F, M, a, sig);
    std::printf("%d", st);
    for (int i = 0; i < K; ++i) std::printf(" %.17g", sig[i]);
    std::printf("\n");
  }
  return 0;
}
