// Host check of the padded LDS index shortcuts of the Stockham passes: for
// both element sizes, every radix (2, 3, 4, 8), every supported line length
// and every stride a plan can reach, wherever read_split / write_split allow
// the shortcut it must equal the padded index computed in full.  Prints the
// number of violations and exits non-zero if there are any.
#include <cstdio>

#include "fft.h"

template <typename T>
static long check() {
  using gpe::lpad;
  long bad = 0, used = 0;
  const int sizes[] = {4, 6, 8, 12, 16, 24, 32, 48, 64, 96, 128, 192, 256, 384, 512};
  const int radices[] = {2, 3, 4, 8};
  for (int N : sizes)
    for (int R : radices) {
      if (N % R) continue;
      const int B = N / R;
      for (int Ns = 1; Ns * R <= N; ++Ns) {
        if (N % (Ns * R)) continue;
        const bool rs = gpe::read_split<T>(B), ws = gpe::write_split<T>(Ns, R);
        for (int b = 0; b < B; ++b) {
          const int base = (b / Ns) * Ns * R + b % Ns;
          for (int r = 0; r < R; ++r) {
            if (rs) {
              ++used;
              bad += lpad<T>(b + r * B) != lpad<T>(b) + lpad<T>(r * B);
            }
            if (ws) {
              ++used;
              bad += lpad<T>(base + r * Ns) != lpad<T>(base) + (Ns == 1 ? r : lpad<T>(r * Ns));
            }
          }
        }
      }
    }
  std::printf("pad run %d: %ld shortcut indices checked, %ld violations\n", gpe::pad_run<T>(), used, bad);
  return bad;
}

int main() {
  const long bad = check<float>() + check<double>();
  std::printf("violations %ld\n", bad);
  return bad != 0;
}
