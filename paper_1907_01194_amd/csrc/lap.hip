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
#include "common.h"
#include "kernels.h"

namespace gpe {

struct RadixPlan {
  int S;
  int r[12];
  int maxr;
};

constexpr RadixPlan make_plan(int N) {
  RadixPlan p{0, {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0}, 1};
  int m = N;
  while (m % 3 == 0) { p.r[p.S++] = 3; m /= 3; }
  while (m % 8 == 0) { p.r[p.S++] = 8; m /= 8; }
  if (m % 4 == 0) { p.r[p.S++] = 4; m /= 4; }
  if (m % 2 == 0) { p.r[p.S++] = 2; m /= 2; }
  for (int i = 0; i < p.S; ++i)
    if (p.r[i] > p.maxr) p.maxr = p.r[i];
  return p;
}

constexpr int plan_prefix(RadixPlan p, int s) {
  int v = 1;
  for (int i = 0; i < s; ++i) v *= p.r[i];
  return v;
}

template <int N> struct Geo {
  static constexpr RadixPlan P = make_plan(N);
  static constexpr int TPL = N / P.maxr;                       // threads per line
  static constexpr int LPB0 = (256 / TPL) > 0 ? 256 / TPL : 1;
  static constexpr int LPB = LPB0 >= 128 ? 128 : LPB0 >= 64 ? 64 : LPB0 >= 32 ? 32 : LPB0 >= 16 ? 16
                           : LPB0 >= 8 ? 8 : LPB0 >= 4 ? 4 : LPB0 >= 2 ? 2 : 1;   // power of two
  static constexpr int THREADS = LPB * TPL;
};

// multiply by -i (forward) or +i (inverse)
template <bool FWD, typename T2> __device__ __forceinline__ T2 mul_mi(T2 a) {
  return FWD ? mk<T2>(a.y, -a.x) : mk<T2>(-a.y, a.x);
}

template <int R, bool FWD, typename T2> struct Dft;

template <bool FWD, typename T2> struct Dft<2, FWD, T2> {
  __device__ static __forceinline__ void run(T2* a) {
    T2 t = a[0];
    a[0] = cadd(t, a[1]);
    a[1] = csub(t, a[1]);
  }
};

template <bool FWD, typename T2> struct Dft<4, FWD, T2> {
  __device__ static __forceinline__ void run(T2* a) {
    T2 t0 = cadd(a[0], a[2]), t1 = csub(a[0], a[2]);
    T2 t2 = cadd(a[1], a[3]), t3 = mul_mi<FWD>(csub(a[1], a[3]));
    a[0] = cadd(t0, t2);
    a[2] = csub(t0, t2);
    a[1] = cadd(t1, t3);
    a[3] = csub(t1, t3);
  }
};

template <bool FWD, typename T2> struct Dft<8, FWD, T2> {
  __device__ static __forceinline__ void run(T2* a) {
    using T = decltype(T2::x);
    T2 e[4] = {a[0], a[2], a[4], a[6]};
    T2 o[4] = {a[1], a[3], a[5], a[7]};
    Dft<4, FWD, T2>::run(e);
    Dft<4, FWD, T2>::run(o);
    const T s = (T)0.70710678118654752440;
    // o1 *= W8, o2 *= W8^2 = -+i, o3 *= W8^3
    T2 o1 = FWD ? mk<T2>(s * (o[1].x + o[1].y), s * (o[1].y - o[1].x))
                : mk<T2>(s * (o[1].x - o[1].y), s * (o[1].y + o[1].x));
    T2 o2 = mul_mi<FWD>(o[2]);
    T2 o3 = FWD ? mk<T2>(s * (o[3].y - o[3].x), -s * (o[3].x + o[3].y))
                : mk<T2>(-s * (o[3].x + o[3].y), s * (o[3].x - o[3].y));
    a[0] = cadd(e[0], o[0]);
    a[4] = csub(e[0], o[0]);
    a[1] = cadd(e[1], o1);
    a[5] = csub(e[1], o1);
    a[2] = cadd(e[2], o2);
    a[6] = csub(e[2], o2);
    a[3] = cadd(e[3], o3);
    a[7] = csub(e[3], o3);
  }
};

template <bool FWD, typename T2> struct Dft<3, FWD, T2> {
  __device__ static __forceinline__ void run(T2* a) {
    using T = decltype(T2::x);
    const T c = (T)0.86602540378443864676;  // sqrt(3)/2
    T2 s = cadd(a[1], a[2]);
    T2 d = csub(a[1], a[2]);
    T2 m = mk<T2>(a[0].x - (T)0.5 * s.x, a[0].y - (T)0.5 * s.y);
    T2 jd = mul_mi<FWD>(mk<T2>(c * d.x, c * d.y));   // -+ i sqrt(3)/2 d
    a[0] = cadd(a[0], s);
    a[1] = cadd(m, jd);
    a[2] = csub(m, jd);
  }
};

enum { SRC_GLOBAL = 0, SRC_LDS = 1 };
enum { DST_LDS = 0, DST_GLOBAL = 1 };

struct LineCtx {
  size_t goff;      // global element offset of this thread's line
  int gstride;      // element stride along the line in global memory
  int lbase;        // LDS element offset of this thread's line
  int lstride;      // element stride along the line in LDS
  int tl;           // thread index within the line
  bool valid;       // line exists
};

template <typename T, int N, int s, bool FWD, int SRC, int DST>
__device__ __forceinline__ void stage(const c_t<T>* __restrict__ gin, c_t<T>* lds,
                                      const c_t<T>* tw, c_t<T>* __restrict__ gout,
                                      const c_t<T>* gacc, const LineCtx& lc, T lamc, T invn) {
  using T2 = c_t<T>;
  constexpr RadixPlan P = Geo<N>::P;
  constexpr int R = P.r[s];
  constexpr int Ns = plan_prefix(P, s);
  constexpr int B = N / R;
  constexpr int TPL = Geo<N>::TPL;
  constexpr int NB = (B + TPL - 1) / TPL;
  constexpr bool LAST_FWD = FWD && (s == P.S - 1);
  T2 v[NB][R];
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    const int b = lc.tl + i * TPL;
    if (lc.valid && (B % TPL == 0 || b < B)) {
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int j = b + r * B;
        v[i][r] = (SRC == SRC_GLOBAL) ? gin[lc.goff + (size_t)j * lc.gstride] : lds[lc.lbase + j * lc.lstride];
      }
    }
  }
  if (SRC == SRC_LDS) __syncthreads();
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    const int b = lc.tl + i * TPL;
    if (lc.valid && (B % TPL == 0 || b < B)) {
      const int k = b % Ns;
      if (Ns > 1) {
#pragma unroll
        for (int r = 1; r < R; ++r) {
          T2 w = tw[(r * k * (N / (Ns * R))) % N];
          if (!FWD) w.y = -w.y;
          v[i][r] = cmul(v[i][r], w);
        }
      }
      Dft<R, FWD, T2>::run(v[i]);
      const int base = (b / Ns) * Ns * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int idx = base + r * Ns;
        T2 val = v[i][r];
        if (LAST_FWD) {
          const int p = idx < N / 2 ? idx : idx - N;
          const T lam = lamc * (T)p;
          val = cscale(val, lam * lam * invn);
        }
        if (DST == DST_LDS) {
          lds[lc.lbase + idx * lc.lstride] = val;
        } else {
          const size_t g = lc.goff + (size_t)idx * lc.gstride;
          gout[g] = gacc ? cadd(gacc[g], val) : val;
        }
      }
    }
  }
  if (DST == DST_LDS) __syncthreads();
}

template <typename T, int N, int s>
__device__ __forceinline__ void fwd_stages(const c_t<T>* gin, c_t<T>* lds, const c_t<T>* tw,
                                           const LineCtx& lc, T lamc, T invn) {
  constexpr int S = Geo<N>::P.S;
  if constexpr (s < S) {
    if constexpr (s == 0)
      stage<T, N, 0, true, SRC_GLOBAL, DST_LDS>(gin, lds, tw, nullptr, nullptr, lc, lamc, invn);
    else
      stage<T, N, s, true, SRC_LDS, DST_LDS>(nullptr, lds, tw, nullptr, nullptr, lc, lamc, invn);
    fwd_stages<T, N, s + 1>(gin, lds, tw, lc, lamc, invn);
  }
}

template <typename T, int N, int s>
__device__ __forceinline__ void inv_stages(c_t<T>* lds, const c_t<T>* tw, c_t<T>* gout,
                                           const c_t<T>* gacc, const LineCtx& lc) {
  constexpr int S = Geo<N>::P.S;
  if constexpr (s < S) {
    if constexpr (s == S - 1)
      stage<T, N, s, false, SRC_LDS, DST_GLOBAL>(nullptr, lds, tw, gout, gacc, lc, T(0), T(0));
    else
      stage<T, N, s, false, SRC_LDS, DST_LDS>(nullptr, lds, tw, nullptr, nullptr, lc, T(0), T(0));
    inv_stages<T, N, s + 1>(lds, tw, gout, gacc, lc);
  }
}

template <typename T, int N>
__global__ void __launch_bounds__(Geo<N>::THREADS)
lap_axis_kernel(const c_t<T>* __restrict__ in, const c_t<T>* acc, c_t<T>* out,
                const c_t<T>* __restrict__ twg, long nlines, int inner, T lamc) {
  using T2 = c_t<T>;
  constexpr int TPL = Geo<N>::TPL;
  constexpr int LPB = Geo<N>::LPB;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T2* tw = reinterpret_cast<T2*>(smem_raw);
  T2* lds = tw + N;

  const int t = threadIdx.x;
  for (int m = t; m < N; m += blockDim.x) tw[m] = twg[m];

  LineCtx lc;
  int ln;
  if (inner == 1) {
    lc.tl = t % TPL;
    ln = t / TPL;
    lc.lstride = 1;
    lc.lbase = ln * (N + 1);
  } else {
    ln = t % LPB;
    lc.tl = t / LPB;
    lc.lstride = LPB;
    lc.lbase = ln;
  }
  const long L = (long)blockIdx.x * LPB + ln;
  lc.valid = L < nlines;
  const long o = L / inner;
  const long i = L % inner;
  lc.goff = (size_t)o * N * inner + i;
  lc.gstride = inner;
  const T invn = T(1) / T(N);
  // Stage 0 reads global memory and uses no twiddles; the barrier that ends it
  // also publishes the twiddle table.
  fwd_stages<T, N, 0>(in, lds, tw, lc, lamc, invn);
  inv_stages<T, N, 0>(lds, tw, out, acc, lc);
}

template <typename T, int N>
static void launch_lap(const LapAxis& ax, const void* in, const void* acc, void* out, hipStream_t st) {
  using T2 = c_t<T>;
  constexpr int LPB = Geo<N>::LPB;
  const long nlines = ax.nlines;
  const int grid = (int)((nlines + LPB - 1) / LPB);
  const size_t lds = sizeof(T2) * (size_t)(N + LPB * (N + 1));
  const T2* tw = reinterpret_cast<const T2*>(sizeof(T) == 8 ? ax.tw64 : ax.tw32);
  hipLaunchKernelGGL((lap_axis_kernel<T, N>), dim3(grid), dim3(Geo<N>::THREADS), lds, st,
                     reinterpret_cast<const T2*>(in), reinterpret_cast<const T2*>(acc),
                     reinterpret_cast<T2*>(out), tw, nlines, ax.inner, (T)ax.lamc);
}

template <typename T>
hipError_t lap_axis(const LapAxis& ax, const void* in, const void* acc, void* out, hipStream_t st) {
  switch (ax.n) {
#define GPE_CASE(NN) case NN: launch_lap<T, NN>(ax, in, acc, out, st); break;
    GPE_CASE(4) GPE_CASE(6) GPE_CASE(8) GPE_CASE(12) GPE_CASE(16) GPE_CASE(24) GPE_CASE(32)
    GPE_CASE(48) GPE_CASE(64) GPE_CASE(96) GPE_CASE(128) GPE_CASE(192) GPE_CASE(256)
    GPE_CASE(384) GPE_CASE(512)
#undef GPE_CASE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
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

}  // namespace gpe
