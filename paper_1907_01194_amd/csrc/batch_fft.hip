// Batched spectral Laplacian axis pass and batched fused HVP x pass: one
// launch covers every problem of a batch, whatever its grid.  A workgroup
// finds its problem from the workgroup offsets, then runs the same device
// body as the single-problem kernels (fft.h) for that problem's line length,
// chosen at run time among the powers of two 16..512.  All those lengths give
// the same axis-pass workgroup size, and a fused x pass is launched with the
// largest workgroup any of them needs (the bodies leave the extra threads
// idle), so one launch can hold all of them; the dynamic LDS is the largest
// any of them needs.
#include "fft.h"
#include "batch_ops.h"

namespace gpe {

#define GPE_BSIZES(M) M(16) M(32) M(64) M(128) M(256) M(512)

bool batch_size_supported(int n) {
  switch (n) {
#define GPE_CASE(NN) case NN:
    GPE_BSIZES(GPE_CASE)
#undef GPE_CASE
    return true;
    default: return false;
  }
}

// ---------------------------------------------------------------- axis pass
template <int... Ns> struct LapBatchGeo {
  static constexpr int THREADS = Geo<16>::THREADS;
  static constexpr bool uniform = ((Geo<Ns>::THREADS == THREADS) && ...);
  static constexpr size_t lds_elems() {
    size_t m = 0;
    ((m = (size_t)(Ns + Geo<Ns>::LPB * (Ns + 1)) > m ? (size_t)(Ns + Geo<Ns>::LPB * (Ns + 1)) : m), ...);
    return m;
  }
};
using LapB = LapBatchGeo<16, 32, 64, 128, 256, 512>;
static_assert(LapB::uniform, "batched axis pass needs one workgroup size for every line length");

template <typename T>
__global__ void __launch_bounds__(LapB::THREADS)
lap_batched_kernel(const LapArgs<T>* __restrict__ args, const int* __restrict__ blk0, int nprob, int F, int slot) {
  using T2 = c_t<T>;
  const int gb = sizeof(T) == 4 ? xcd_local_block((int)blockIdx.x, (int)gridDim.x) : (int)blockIdx.x;
  const int pb = batch_problem(blk0, nprob, gb);
  const LapArgs<T>& a = args[pb];
  const long blk = (long)gb - blk0[pb];
  switch (a.n) {
#define GPE_CASE(NN)                                                                                          \
  case NN:                                                                                                    \
    lap_body<T, NN>(reinterpret_cast<const T2*>(a.in), reinterpret_cast<const T2*>(a.acc),                    \
                    reinterpret_cast<T2*>(a.out), reinterpret_cast<const T2*>(a.tw), a.nlines, a.inner,       \
                    (T)a.lamc, F, a.npts, reinterpret_cast<const T2*>(a.X), a.coef, a.part, a.stride, slot,   \
                    blk, a.skip, a.ab);                                                                       \
    break;
    GPE_BSIZES(GPE_CASE)
#undef GPE_CASE
    default: break;
  }
}

int lap_batch_blocks(int n, long nlines) {
  int lpb = 0;
  switch (n) {
#define GPE_CASE(NN) case NN: lpb = Geo<NN>::LPB; break;
    GPE_BSIZES(GPE_CASE)
#undef GPE_CASE
    default: return -1;
  }
  return (int)((nlines + lpb - 1) / lpb);
}

template <typename T>
hipError_t lap_batched(const LapArgs<T>* args, const Span& sp, int F, int slot, hipStream_t st) {
  if (sp.nprob < 1 || sp.nblocks < 1) return hipErrorInvalidValue;
  const size_t lds = sizeof(c_t<T>) * LapB::lds_elems();
  if (lds > 65536)
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&lap_batched_kernel<T>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  hipLaunchKernelGGL((lap_batched_kernel<T>), dim3(sp.nblocks), dim3(LapB::THREADS), lds, st, args, sp.blk0,
                     sp.nprob, F, slot);
  return hipGetLastError();
}

// ---------------------------------------------------------------- fused x pass
template <int K, int VAR, int... Ns> struct XBatchGeo {
  static constexpr int THREADS = [] {
    int m = 0;
    ((m = XGeo<Ns, K, VAR>::THREADS > m ? XGeo<Ns, K, VAR>::THREADS : m), ...);
    return m;
  }();
  template <typename T> static constexpr size_t lds_elems() {
    size_t m = 0;
    ((m = XGeo<Ns, K, VAR>::template lds_elems<T>() > m ? XGeo<Ns, K, VAR>::template lds_elems<T>() : m), ...);
    return m;
  }
};
template <int K, int VAR> using XB = XBatchGeo<K, VAR, 16, 32, 64, 128, 256, 512>;

template <typename T, int F, int VAR>
__global__ void __launch_bounds__((XB<2 * F + 1, VAR>::THREADS))
xpass_batched_kernel(const XpassArgs<T>* __restrict__ args, const int* __restrict__ blk0, int nprob) {
  using T2 = c_t<T>;
  const int gb = sizeof(T) == 4 ? xcd_local_block((int)blockIdx.x, (int)gridDim.x) : (int)blockIdx.x;
  const int pb = batch_problem(blk0, nprob, gb);
  const XpassArgs<T>& a = args[pb];
  const long blk = (long)gb - blk0[pb];
  switch (a.n) {
#define GPE_CASE(NN)                                                                                              \
  case NN:                                                                                                        \
    xpass_body<T, NN, F, VAR>(reinterpret_cast<const T2*>(a.X), reinterpret_cast<const T2*>(a.Z),                \
                              reinterpret_cast<const T2*>(a.Y), reinterpret_cast<const T*>(a.V),                  \
                              reinterpret_cast<T2*>(a.W), reinterpret_cast<const T2*>(a.tw), (long)(a.npts / NN), \
                              a.npts, (T)a.lamc, a.p, a.part, a.stride, blk, a.skip);                             \
    break;
    GPE_BSIZES(GPE_CASE)
#undef GPE_CASE
    default: break;
  }
}

int xpass_batch_blocks(int n, int F, int var, size_t npts) {
  int rpb = 0;
  switch (n * 16 + F * 4 + var) {
#define GPE_CASE(NN)                                                   \
  case NN * 16 + 4 + 0: rpb = XGeo<NN, 3, 0>::RPB; break;             \
  case NN * 16 + 4 + 1: rpb = XGeo<NN, 3, 1>::RPB; break;             \
  case NN * 16 + 4 + 2: rpb = XGeo<NN, 3, 2>::RPB; break;             \
  case NN * 16 + 8 + 0: rpb = XGeo<NN, 5, 0>::RPB; break;             \
  case NN * 16 + 8 + 1: rpb = XGeo<NN, 5, 1>::RPB; break;             \
  case NN * 16 + 8 + 2: rpb = XGeo<NN, 5, 2>::RPB; break;             \
  case NN * 16 + 12 + 0: rpb = XGeo<NN, 7, 0>::RPB; break;            \
  case NN * 16 + 12 + 1: rpb = XGeo<NN, 7, 1>::RPB; break;            \
  case NN * 16 + 12 + 2: rpb = XGeo<NN, 7, 2>::RPB; break;
    GPE_BSIZES(GPE_CASE)
#undef GPE_CASE
    default: return -1;
  }
  const size_t nrows = npts / (size_t)n;
  return (int)((nrows + rpb - 1) / rpb);
}

template <typename T, int F, int VAR>
static hipError_t launch_xb(const XpassArgs<T>* args, const Span& sp, hipStream_t st) {
  using G = XB<2 * F + 1, VAR>;
  const size_t lds = sizeof(c_t<T>) * G::template lds_elems<T>();
  if (lds > 65536)
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&xpass_batched_kernel<T, F, VAR>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  hipLaunchKernelGGL((xpass_batched_kernel<T, F, VAR>), dim3(sp.nblocks), dim3(G::THREADS), lds, st, args, sp.blk0,
                     sp.nprob);
  return hipGetLastError();
}

template <typename T>
hipError_t xpass_batched(int F, int var, const XpassArgs<T>* args, const Span& sp, hipStream_t st) {
  if (sp.nprob < 1 || sp.nblocks < 1) return hipErrorInvalidValue;
  switch (F * 4 + var) {
    case 4 + 0: return launch_xb<T, 1, 0>(args, sp, st);
    case 4 + 1: return launch_xb<T, 1, 1>(args, sp, st);
    case 4 + 2: return launch_xb<T, 1, 2>(args, sp, st);
    case 8 + 0: return launch_xb<T, 2, 0>(args, sp, st);
    case 8 + 1: return launch_xb<T, 2, 1>(args, sp, st);
    case 8 + 2: return launch_xb<T, 2, 2>(args, sp, st);
    case 12 + 0: return launch_xb<T, 3, 0>(args, sp, st);
    case 12 + 1: return launch_xb<T, 3, 1>(args, sp, st);
    case 12 + 2: return launch_xb<T, 3, 2>(args, sp, st);
    default: return hipErrorInvalidValue;
  }
}

template hipError_t lap_batched<double>(const LapArgs<double>*, const Span&, int, int, hipStream_t);
template hipError_t lap_batched<float>(const LapArgs<float>*, const Span&, int, int, hipStream_t);
template hipError_t xpass_batched<double>(int, int, const XpassArgs<double>*, const Span&, hipStream_t);
template hipError_t xpass_batched<float>(int, int, const XpassArgs<float>*, const Span&, hipStream_t);

}  // namespace gpe
