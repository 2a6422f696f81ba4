// Spectral negative Laplacian, one axis per launch (Sec. 3, eq. discrete:laplace).
//
// On a tensor grid L = sum_alpha L_alpha, where L_alpha is: DFT along axis
// alpha, multiply by lambda_alpha(p)^2 / n_alpha (p = -n/2..n/2-1, Nyquist kept),
// inverse DFT.  Each launch applies one L_alpha to every line of every
// component and writes out = acc + L_alpha(in) (acc may be null or alias out).
//
// A workgroup owns LPB whole lines.  The forward and inverse transforms are
// self-sorting (Stockham) mixed radix-8/4/3/2 passes on the lines held in LDS:
// the first forward pass reads global memory directly, the last inverse pass
// writes global memory directly, the lambda^2 scaling is folded into the last
// forward pass.  Lines along x are contiguous; lines along y and z are taken
// LPB at a time at consecutive x so that every global access is coalesced.
#include "fft.h"

namespace gpe {

// fin.part non-null: the launch has one more workgroup, dispatched first,
// that forms the HVP's projection coefficients from the x pass's partials
// into fin.res[32..33] for a later pass (instead of a finalize launch).
template <typename T, int N>
__global__ void __launch_bounds__(Geo<N>::THREADS)
lap_axis_kernel(const c_t<T>* __restrict__ in, const c_t<T>* acc, c_t<T>* out,
                const c_t<T>* __restrict__ twg, long nlines, int inner, T lamc, int F, size_t npts,
                const c_t<T>* __restrict__ X, const double* __restrict__ coef, double* __restrict__ part,
                size_t stride, int slot, const double* skip, int rev, AbSrc ab, AbSrc fin) {
  // c64 lines: consecutive workgroups on one XCD (measured faster for c64
  // and slower for c128, whose line segments already fill the cache lines)
  long b = sizeof(T) == 4 ? (long)xcd_local_block((int)blockIdx.x, (int)gridDim.x) : (long)blockIdx.x;
  long nb = (long)gridDim.x;
  if (fin.part) {
    if (b == 0) {
      if (skip && *skip != 0.0) return;
      double cf[2];
      ab_coeffs(fin, F, true, cf);
      return;
    }
    --b;
    --nb;
  }
  const long blk = rev ? nb - 1 - b : b;
  lap_body<T, N>(in, acc, out, twg, nlines, inner, lamc, F, npts, X, coef, part, stride, slot, blk, skip, ab);
}

template <typename T, int N, int F, int VAR>
__global__ void __launch_bounds__((XGeo<N, 2 * F + 1, VAR>::THREADS))
hvp_xpass_kernel(const c_t<T>* __restrict__ X, const c_t<T>* __restrict__ Z, const c_t<T>* __restrict__ Y,
                 const T* __restrict__ V, c_t<T>* __restrict__ W, const c_t<T>* __restrict__ twg, long nrows,
                 size_t npts, T lamc, PwParams p, double* __restrict__ part, size_t stride, const double* skip) {
  const long blk = sizeof(T) == 4 ? (long)xcd_local_block((int)blockIdx.x, (int)gridDim.x) : (long)blockIdx.x;
  xpass_body<T, N, F, VAR>(X, Z, Y, V, W, twg, nrows, npts, lamc, p, part, stride, blk, skip);
}

template <typename T, int N>
static void launch_lap(const LapAxis& ax, const void* in, const void* acc, void* out, int F, size_t npts,
                       const void* X, const double* coef, double* part, size_t stride, int slot, int* nb,
                       const double* skip, int rev, const AbSrc* ab, const AbSrc* fin, hipStream_t st) {
  using T2 = c_t<T>;
  constexpr int LPB = Geo<N>::LPB;
  const long nlines = ax.nlines;
  const int grid = (int)((nlines + LPB - 1) / LPB);
  const size_t lds = sizeof(T2) * (size_t)(N + LPB * (N + 1));
  const T2* tw = reinterpret_cast<const T2*>(sizeof(T) == 8 ? ax.tw64 : ax.tw32);
  hipLaunchKernelGGL((lap_axis_kernel<T, N>), dim3(grid + (fin ? 1 : 0)), dim3(Geo<N>::THREADS), lds, st,
                     reinterpret_cast<const T2*>(in), reinterpret_cast<const T2*>(acc),
                     reinterpret_cast<T2*>(out), tw, nlines, ax.inner, (T)ax.lamc, F, npts,
                     reinterpret_cast<const T2*>(X), coef, part, stride, slot, skip, rev, ab ? *ab : AbSrc{},
                     fin ? *fin : AbSrc{});
  if (nb) *nb = grid;   // partials of the pass itself (the extra workgroup writes none)
}

#define GPE_SIZES(M) M(4) M(6) M(8) M(12) M(16) M(24) M(32) M(48) M(64) M(96) M(128) M(192) M(256) M(384) M(512)

template <typename T>
hipError_t lap_axis(const LapAxis& ax, const void* in, const void* acc, void* out, hipStream_t st) {
  switch (ax.n) {
#define GPE_CASE(NN) \
  case NN:                                                                                                       \
    launch_lap<T, NN>(ax, in, acc, out, 0, 1, nullptr, nullptr, nullptr, 0, 0, nullptr, nullptr, 0, nullptr,     \
                      nullptr, st);                                                                               \
    break;
    GPE_SIZES(GPE_CASE)
#undef GPE_CASE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename T>
hipError_t lap_axis_ex(const LapAxis& ax, const void* in, const void* acc, void* out, int F, size_t npts,
                       const void* X, const double* coef, double* part, size_t stride, int slot, int* nb,
                       const double* skip, int rev, const AbSrc* ab, const AbSrc* fin, hipStream_t st) {
  switch (ax.n) {
#define GPE_CASE(NN)                                                                                          \
  case NN: launch_lap<T, NN>(ax, in, acc, out, F, npts, X, coef, part, stride, slot, nb, skip, rev, ab, fin, st); \
    break;
    GPE_SIZES(GPE_CASE)
#undef GPE_CASE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename T, int N, int F, int VAR>
static void launch_xpass(const LapAxis& ax, size_t npts, const void* X, const void* Z, const void* Y, const T* V,
                         void* W, const PwParams& p, double* part, size_t stride, int* nb, const double* skip,
                         hipStream_t st) {
  using T2 = c_t<T>;
  constexpr int K = 2 * F + 1;
  using G = XGeo<N, K, VAR>;
  const long nrows = (long)(npts / N);
  const int grid = (int)((nrows + G::RPB - 1) / G::RPB);
  const size_t lds = sizeof(T2) * G::template lds_elems<T>();
  const T2* tw = reinterpret_cast<const T2*>(sizeof(T) == 8 ? ax.tw64 : ax.tw32);
  if (lds > 65536)
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&hvp_xpass_kernel<T, N, F, VAR>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  hipLaunchKernelGGL((hvp_xpass_kernel<T, N, F, VAR>), dim3(grid), dim3(G::THREADS), lds, st,
                     reinterpret_cast<const T2*>(X), reinterpret_cast<const T2*>(Z),
                     reinterpret_cast<const T2*>(Y), V, reinterpret_cast<T2*>(W), tw, nrows, npts, (T)ax.lamc, p,
                     part, stride, skip);
  *nb = grid;
}

// the line lengths that get all three schedule variants (the others use the default)
static constexpr bool tuned_size(int n) { return n == 64 || n == 96 || n == 128 || n == 256; }

template <typename T, int N, int F>
static void launch_xpass_var(int var, const LapAxis& ax, size_t npts, const void* X, const void* Z, const void* Y,
                             const T* V, void* W, const PwParams& p, double* part, size_t stride, int* nb,
                             const double* skip, hipStream_t st) {
  if constexpr (tuned_size(N)) {
    if (var == 0) return launch_xpass<T, N, F, 0>(ax, npts, X, Z, Y, V, W, p, part, stride, nb, skip, st);
    if (var == 2) return launch_xpass<T, N, F, 2>(ax, npts, X, Z, Y, V, W, p, part, stride, nb, skip, st);
  }
  launch_xpass<T, N, F, 1>(ax, npts, X, Z, Y, V, W, p, part, stride, nb, skip, st);
}

int xpass_variants(int n) { return tuned_size(n) ? 3 : 1; }

template <typename T>
hipError_t hvp_xpass(int F, const LapAxis& ax, size_t npts, const void* X, const void* Z, const void* Y,
                     const T* V, void* W, const PwParams& p, double* part, size_t stride, int* nb, int var,
                     const double* skip, hipStream_t st) {
  switch (ax.n * 4 + F) {
#define GPE_CASE(NN)                                                                                          \
  case NN * 4 + 1: launch_xpass_var<T, NN, 1>(var, ax, npts, X, Z, Y, V, W, p, part, stride, nb, skip, st); \
    break;                                                                                                    \
  case NN * 4 + 2: launch_xpass_var<T, NN, 2>(var, ax, npts, X, Z, Y, V, W, p, part, stride, nb, skip, st); \
    break;                                                                                                    \
  case NN * 4 + 3: launch_xpass_var<T, NN, 3>(var, ax, npts, X, Z, Y, V, W, p, part, stride, nb, skip, st); \
    break;
    GPE_SIZES(GPE_CASE)
#undef GPE_CASE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

size_t lap_max_blocks(const LapAxis& ax, int K) {
  size_t lpb = 1, rpb = 1;
  switch (ax.n) {
#define GPE_CASE(NN)                                                                       \
  case NN:                                                                                 \
    lpb = Geo<NN>::LPB;                                                                    \
    rpb = 1; /* the smallest rows-per-workgroup of any schedule variant */               \
    break;
    GPE_SIZES(GPE_CASE)
#undef GPE_CASE
  }
  const size_t a = (ax.nlines + lpb - 1) / lpb;
  const size_t b = ((size_t)ax.nlines / K + rpb - 1) / rpb;
  return a > b ? a : b;
}

bool lap_size_supported(int n) {
  switch (n) {
    case 4: case 6: case 8: case 12: case 16: case 24: case 32: case 48: case 64: case 96:
    case 128: case 192: case 256: case 384: case 512: return true;
    default: return false;
  }
}

template hipError_t lap_axis<double>(const LapAxis&, const void*, const void*, void*, hipStream_t);
template hipError_t lap_axis<float>(const LapAxis&, const void*, const void*, void*, hipStream_t);
template hipError_t lap_axis_ex<double>(const LapAxis&, const void*, const void*, void*, int, size_t, const void*,
                                        const double*, double*, size_t, int, int*, const double*, int,
                                        const AbSrc*, const AbSrc*, hipStream_t);
template hipError_t lap_axis_ex<float>(const LapAxis&, const void*, const void*, void*, int, size_t, const void*,
                                       const double*, double*, size_t, int, int*, const double*, int,
                                       const AbSrc*, const AbSrc*, hipStream_t);
template hipError_t hvp_xpass<double>(int, const LapAxis&, size_t, const void*, const void*, const void*,
                                      const double*, void*, const PwParams&, double*, size_t, int*, int,
                                      const double*, hipStream_t);
template hipError_t hvp_xpass<float>(int, const LapAxis&, size_t, const void*, const void*, const void*,
                                     const float*, void*, const PwParams&, double*, size_t, int*, int,
                                     const double*, hipStream_t);

}  // namespace gpe
