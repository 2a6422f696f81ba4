// Device building blocks of the spectral Laplacian passes (Sec. 3, eq.
// discrete:laplace): the mixed radix-8/4/3/2 Stockham line transforms in LDS,
// one axis pass over a block of lines, and the fused x pass of the
// Hessian-vector product (pointwise Hessian terms of Sec. 3 plus L_x).  The
// bodies take their workgroup index explicitly so that one batched launch
// can run them for many problems (batch_fft.hip) as well as one (lap.hip).
#pragma once

#include "common.h"
#include "kernels.h"
#include "spin.h"

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
  int lstride;      // element stride along the line in LDS (unpadded layouts)
  int tl;           // thread index within the line
  bool valid;       // line exists
};

// Padded LDS layout of a line held contiguously: element j sits at
// j + (j >> pad_shift<T>()), one pad per pad_run<T>() elements: 16 for c64
// lines, 8 for c128 lines (the run with the fewest bank conflicts for each
// element size).  The Stockham passes access a line at strides R (the first
// pass's writes: 8 for radix 8) and 2rk (twiddles); the pads spread every such
// group of lanes over distinct banks.
template <typename T> __host__ __device__ constexpr int pad_shift() { return sizeof(T) == 4 ? 4 : 3; }
template <typename T> __host__ __device__ constexpr int pad_run() { return 1 << pad_shift<T>(); }
template <typename T> __host__ __device__ constexpr int lpad(int j) { return j + (j >> pad_shift<T>()); }
// LDS elements a padded line (or twiddle table) of length N occupies
template <typename T> __host__ __device__ constexpr int padded_len(int N) { return N + (N >> pad_shift<T>()) + 1; }
// Index shortcuts of a padded pass with B = N / R butterflies and stride Ns:
// reads at b + r B may be taken as lpad(b) + lpad(r B) when B is a multiple of
// the pad run; writes at base + r Ns (base = (b / Ns) Ns R + b % Ns) as
// lpad(base) + lpad(r Ns) when Ns is, or as lpad(base) + r when Ns = 1 and R
// divides the pad run (base + r then never carries into the pad count).
template <typename T> __host__ __device__ constexpr bool read_split(int B) { return B % pad_run<T>() == 0; }
template <typename T> __host__ __device__ constexpr bool write_split(int Ns, int R) {
  return Ns % pad_run<T>() == 0 || (Ns == 1 && pad_run<T>() % R == 0);
}

// Epilogue of the last inverse pass: out = acc + val - pc * X (pc = 0: no projection).
template <typename T> struct Epi {
  const c_t<T>* acc;
  const c_t<T>* X;
  T pc;
};

// PAD: the line is contiguous in LDS in the padded layout (lpad), and so is
// the twiddle table; otherwise element j of the line is at lbase + j lstride
// and twiddle m at m.  raw (first pass only, may be null): the line as read
// from global memory is also stored there, in the line's own LDS layout.
template <typename T, bool PAD> __device__ __forceinline__ int lidx(const LineCtx& lc, int j) {
  return PAD ? lc.lbase + lpad<T>(j) : lc.lbase + j * lc.lstride;
}

template <typename T, int N, int s, bool FWD, int SRC, int DST, bool PAD>
__device__ __forceinline__ void stage(const c_t<T>* __restrict__ gin, c_t<T>* lds,
                                      const c_t<T>* tw, c_t<T>* __restrict__ gout,
                                      const Epi<T>& epi, const LineCtx& lc, T lamc, T invn, double& pars,
                                      c_t<T>* raw = nullptr) {
  using T2 = c_t<T>;
  constexpr RadixPlan P = Geo<N>::P;
  constexpr int R = P.r[s];
  constexpr int Ns = plan_prefix(P, s);
  constexpr int B = N / R;
  constexpr int TPL = Geo<N>::TPL;
  constexpr int NB = (B + TPL - 1) / TPL;
  constexpr bool LAST_FWD = FWD && (s == P.S - 1);
  T2 v[NB][R];
  constexpr bool kReadSplit = PAD && read_split<T>(B);
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    const int b = lc.tl + i * TPL;
    if (lc.valid && (B % TPL == 0 || b < B)) {
      const int pb = lc.lbase + lpad<T>(b);
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int j = b + r * B;
        const int li = kReadSplit ? pb + lpad<T>(r * B) : lidx<T, PAD>(lc, j);
        v[i][r] = (SRC == SRC_GLOBAL) ? gin[lc.goff + (size_t)j * lc.gstride] : lds[li];
        if (SRC == SRC_GLOBAL && raw) raw[li] = v[i][r];
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
          const int m = (r * k * (N / (Ns * R))) % N;
          T2 w = tw[PAD ? lpad<T>(m) : m];
          if (!FWD) w.y = -w.y;
          v[i][r] = cmul(v[i][r], w);
        }
      }
      Dft<R, FWD, T2>::run(v[i]);
      const int base = (b / Ns) * Ns * R + k;
      constexpr bool kWriteSplit = PAD && write_split<T>(Ns, R);
      const int pbase = lc.lbase + lpad<T>(base);
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int idx = base + r * Ns;
        const int lw = kWriteSplit ? pbase + (Ns == 1 ? r : lpad<T>(r * Ns)) : lidx<T, PAD>(lc, idx);
        T2 val = v[i][r];
        if (LAST_FWD) {
          const int p = idx < N / 2 ? idx : idx - N;
          const T lam = lamc * (T)p;
          const T sc = lam * lam * invn;
          pars += (double)sc * (double)cabs2(val);   // Parseval: <Z, L_a Z> = sum lambda^2/n |Z^|^2
          val = cscale(val, sc);
        }
        if (DST == DST_LDS) {
          lds[lw] = val;
        } else {
          const size_t g = lc.goff + (size_t)idx * lc.gstride;
          T2 o = epi.acc ? cadd(epi.acc[g], val) : val;
          if (epi.X) {
            const T2 xv = epi.X[g];
            o.x -= epi.pc * xv.x;
            o.y -= epi.pc * xv.y;
          }
          gout[g] = o;
        }
      }
    }
  }
  if (DST == DST_LDS) __syncthreads();
}

template <typename T, int N, int s, bool PAD = false>
__device__ __forceinline__ void fwd_stages(const c_t<T>* gin, c_t<T>* lds, const c_t<T>* tw,
                                           const LineCtx& lc, T lamc, T invn, double& pars,
                                           c_t<T>* raw = nullptr) {
  constexpr int S = Geo<N>::P.S;
  const Epi<T> none{nullptr, nullptr, T(0)};
  if constexpr (s < S) {
    if constexpr (s == 0)
      stage<T, N, 0, true, SRC_GLOBAL, DST_LDS, PAD>(gin, lds, tw, nullptr, none, lc, lamc, invn, pars, raw);
    else
      stage<T, N, s, true, SRC_LDS, DST_LDS, PAD>(nullptr, lds, tw, nullptr, none, lc, lamc, invn, pars);
    fwd_stages<T, N, s + 1, PAD>(gin, lds, tw, lc, lamc, invn, pars);
  }
}

// LAST_TO_GLOBAL: the last inverse pass writes global memory through the
// epilogue; otherwise it writes the result back to LDS.
template <typename T, int N, int s, bool LAST_TO_GLOBAL, bool PAD = false>
__device__ __forceinline__ void inv_stages(c_t<T>* lds, const c_t<T>* tw, c_t<T>* gout, const Epi<T>& epi,
                                           const LineCtx& lc) {
  constexpr int S = Geo<N>::P.S;
  const Epi<T> none{nullptr, nullptr, T(0)};
  double dummy = 0.0;
  if constexpr (s < S) {
    if constexpr (s == S - 1 && LAST_TO_GLOBAL)
      stage<T, N, s, false, SRC_LDS, DST_GLOBAL, PAD>(nullptr, lds, tw, gout, epi, lc, T(0), T(0), dummy);
    else
      stage<T, N, s, false, SRC_LDS, DST_LDS, PAD>(nullptr, lds, tw, nullptr, none, lc, T(0), T(0), dummy);
    inv_stages<T, N, s + 1, LAST_TO_GLOBAL, PAD>(lds, tw, gout, epi, lc);
  }
}

// Projection coefficients of the HVP (Lemma 4.1 with the measured Gram
// system): sums slots 0 and 1 of the x pass's partials (ab.n per slot,
// ab.stride apart) in a fixed order over the workgroup, solves the 2x2 Gram
// system with the set point's component norms ab.gram and returns the
// coefficients in c[0..1] (every thread); res: also stored in ab.res[32..33].
__device__ inline void ab_coeffs(const AbSrc& ab, int F, bool store, double* c) {
  __shared__ double red2[2][1024 / kWave];
  __shared__ double cf[2];
  const int t = threadIdx.x;
  double s0 = 0.0, s1 = 0.0;
  for (int b = t; b < ab.n; b += blockDim.x) {
    s0 += ab.part[b];
    s1 += ab.part[ab.stride + b];
  }
  s0 = wave_sum(s0);
  s1 = wave_sum(s1);
  if (t % kWave == 0) {
    red2[0][t / kWave] = s0;
    red2[1][t / kWave] = s1;
  }
  __syncthreads();
  if (t == 0) {
    double w0 = 0.0, w1 = 0.0;
    for (int w = 0; w < ((int)blockDim.x + kWave - 1) / kWave; ++w) {
      w0 += red2[0][w];
      w1 += red2[1][w];
    }
    double a11 = 0, a12 = 0, a22 = 0;
    for (int q = 0; q < 2 * F + 1; ++q) {
      const double l = F - q;
      a11 += ab.gram[q];
      a12 += l * ab.gram[q];
      a22 += l * l * ab.gram[q];
    }
    const double det = a11 * a22 - a12 * a12;
    cf[0] = (a22 * w0 - a12 * w1) / det;
    cf[1] = (a11 * w1 - a12 * w0) / det;
    if (store) {
      ab.res[32] = cf[0];
      ab.res[33] = cf[1];
    }
  }
  __syncthreads();
  c[0] = cf[0];
  c[1] = cf[1];
}

// One axis pass for every line of every component: out = acc + L_a(in)
// [- (coef[0] + coef[1] l) X], with the Parseval sum <in, L_a in> per workgroup
// in part[slot * stride + wg] when part != null.
// Threads at or beyond Geo<N>::THREADS (a batched launch sized for another
// N) take no line.
template <typename T, int N>
__device__ __forceinline__ void lap_body(const c_t<T>* __restrict__ in, const c_t<T>* acc, c_t<T>* out,
                                         const c_t<T>* __restrict__ twg, long nlines, int inner, T lamc, int F,
                                         size_t npts, const c_t<T>* __restrict__ X, const double* __restrict__ coef,
                                         double* __restrict__ part, size_t stride, int slot, long blk,
                                         const double* skip, const AbSrc& ab) {
  if (skip && *skip != 0.0) return;   // uniform over the workgroup
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
  const long L = blk * LPB + ln;
  lc.valid = t < Geo<N>::THREADS && L < nlines;
  const long o = L / inner;
  const long i = L % inner;
  lc.goff = (size_t)o * N * inner + i;
  lc.gstride = inner;
  const T invn = T(1) / T(N);
  Epi<T> epi{acc, nullptr, T(0)};
  double c0 = 0.0, c1 = 0.0;
  if (X && ab.part) {   // uniform: the coefficients from the x pass's partials
    double cf[2];
    ab_coeffs(ab, F, blk == 0, cf);
    c0 = cf[0];
    c1 = cf[1];
  } else if (X) {
    c0 = coef[0];
    c1 = coef[1];
  }
  if (X && lc.valid) {
    const int comp = (int)(lc.goff / npts);          // a line never crosses a component
    epi.X = X;
    epi.pc = (T)(c0 + c1 * (double)(F - comp));
  }
  double pars = 0.0;
  // Stage 0 reads global memory and uses no twiddles; the barrier that ends it
  // also publishes the twiddle table.
  fwd_stages<T, N, 0>(in, lds, tw, lc, lamc, invn, pars);
  inv_stages<T, N, 0, true>(lds, tw, out, epi, lc);
  if (part) {
    double a[1] = {pars};
    block_partials_any<1>(a, part + (size_t)slot * stride, 0, blk);
  }
}

// Fused x pass of the Hessian-vector product: RPB x-rows, all K components.
// Schedule variant VAR: 0 = half the default rows per workgroup, 1 = default
// (about 256 threads), 2 = twice the default (if it fits 1024 threads).
template <int N, int K, int VAR = 1> struct XGeo {
  static constexpr int TPL = Geo<N>::TPL;
  static constexpr int R0 = 256 / (K * TPL);
  static constexpr int RD = R0 >= 16 ? 16 : R0 >= 8 ? 8 : R0 >= 4 ? 4 : R0 >= 2 ? 2 : 1;
  static constexpr int RPB = VAR == 0 ? (RD > 1 ? RD / 2 : 1)
                           : VAR == 1 ? RD
                           : (2 * RD * K * TPL <= 1024 ? 2 * RD : RD);
  static constexpr int LINES = RPB * K;
  static constexpr int THREADS = ((LINES * TPL + 63) / 64) * 64;
  // LDS: the padded twiddle table, then LINES padded lines, then (FP64 only)
  // LINES more holding the rows of Z as read (the pointwise terms take Z
  // from there instead of reading global memory a second time)
  template <typename T> static constexpr int lstr() { return padded_len<T>(N); }
  template <typename T> static constexpr bool stash() {
    return sizeof(T) == 8 && 2 * sizeof(T) * ((size_t)lstr<T>() + 2 * (size_t)LINES * lstr<T>()) <= 150 * 1024;
  }
  template <typename T> static constexpr size_t lds_elems() {
    return (size_t)lstr<T>() + (size_t)LINES * lstr<T>() * (stash<T>() ? 2 : 1);
  }
};

template <typename T, int N, int F, int VAR>
__device__ __forceinline__ void xpass_body(const c_t<T>* __restrict__ X, const c_t<T>* __restrict__ Z,
                                           const c_t<T>* __restrict__ Y, const T* __restrict__ V,
                                           c_t<T>* __restrict__ W, const c_t<T>* __restrict__ twg, long nrows,
                                           size_t npts, T lamc, const PwParams& p, double* __restrict__ part,
                                           size_t stride, long blk, const double* skip) {
  if (skip && *skip != 0.0) return;   // uniform over the workgroup
  using T2 = c_t<T>;
  constexpr int K = 2 * F + 1;
  constexpr int TPL = Geo<N>::TPL;
  using G = XGeo<N, K, VAR>;
  constexpr int RPB = G::RPB;
  constexpr int LINES = G::LINES;
  constexpr int LSTR = G::template lstr<T>();
  constexpr bool kStash = G::template stash<T>();
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T2* tw = reinterpret_cast<T2*>(smem_raw);
  T2* lds = tw + LSTR;
  T2* zraw = kStash ? lds + LINES * LSTR : nullptr;
  const int t = threadIdx.x;
  for (int m = t; m < N; m += blockDim.x) tw[lpad<T>(m)] = twg[m];
  const long row0 = blk * RPB;

  // ---- prefetch the global pointwise operands of this thread's first point
  // (X, L X, V, and Z where it is not kept in LDS) so that their latency
  // hides behind the transforms below.  FP64 keeps the rows of Z in LDS as
  // the first transform pass reads them (an FP64 row block's traffic evicts Z
  // from L2 before the pointwise loop would re-read it); they are taken from
  // there once the transforms are done.
  int pt = t;
  bool have = pt < RPB * N && row0 + pt / N < nrows;
  T2 x[K], z[K], y[K];
  T vj = T(0);
  size_t j = have ? (size_t)(row0 + pt / N) * N + pt % N : 0;
  auto load_global = [&]() {
#pragma unroll
    for (int i = 0; i < K; ++i) {
      x[i] = X[i * npts + j];
      if constexpr (!kStash) z[i] = Z[i * npts + j];
      y[i] = Y[i * npts + j];
    }
    vj = V[j];
  };
  auto load_stashed = [&]() {
    if constexpr (kStash) {
#pragma unroll
      for (int i = 0; i < K; ++i) z[i] = zraw[(i * RPB + pt / N) * LSTR + lpad<T>(pt % N)];
    }
  };
  if (have) load_global();

  // ---- L_x Z for the RPB rows of every component, left in LDS
  LineCtx lc;
  const int ls = t / TPL;                 // line slot = comp * RPB + row
  lc.tl = t % TPL;
  const int comp = ls / RPB, r = ls % RPB;
  lc.valid = ls < LINES && row0 + r < nrows;
  lc.goff = (size_t)comp * npts + (size_t)(row0 + r) * N;
  lc.gstride = 1;
  lc.lbase = ls * LSTR;
  lc.lstride = 1;
  const T invn = T(1) / T(N);
  double pars = 0.0;
  const Epi<T> none{nullptr, nullptr, T(0)};
  fwd_stages<T, N, 0, true>(Z, lds, tw, lc, lamc, invn, pars, zraw);
  inv_stages<T, N, 0, false, true>(lds, tw, nullptr, none, lc);

  // ---- pointwise Hessian terms, W = L_x Z + q
  T zcoef[K];
#pragma unroll
  for (int i = 0; i < K; ++i) zcoef[i] = (T)p.zc[i];
  double acc[7] = {0, 0, 0, 0, 0, 0, pars};
  // Per point the partial sums run over the K components in the work
  // precision; the sums over points accumulate in FP64.
  auto point = [&](int rr, int xx) {
    T s_xw = 0, s_lxw = 0, s_xz = 0, s_lxz = 0, s_zq = 0, s_zz = 0;
#pragma unroll
    for (int i = 0; i < K; ++i) {
      const T c = cdotr(y[i], z[i]);     // <(LX)_i, Z_i> = <X_i, (LZ)_i>
      const T xz = cdotr(x[i], z[i]);
      s_xw += c;
      s_lxw += T(F - i) * c;
      s_xz += xz;
      s_lxz += T(F - i) * xz;
      s_zz += cabs2(z[i]);
    }
    hvp_point<T, F>(x, z, vj, p, zcoef, [&](int i, T2 qi) {
      const T2 lz = lds[(i * RPB + rr) * LSTR + lpad<T>(xx)];
      W[i * npts + j] = cadd(lz, qi);
      const T xq = cdotr(x[i], qi);
      s_xw += xq;
      s_lxw += T(F - i) * xq;
      s_zq += cdotr(z[i], qi);
    });
    acc[0] += (double)s_xw;
    acc[1] += (double)s_lxw;
    acc[2] += (double)s_xz;
    acc[3] += (double)s_lxz;
    acc[4] += (double)s_zq;
    acc[5] += (double)s_zz;
  };
  while (have) {
    load_stashed();
    point(pt / N, pt % N);
    pt += blockDim.x;
    have = pt < RPB * N && row0 + pt / N < nrows;
    if (have) {
      j = (size_t)(row0 + pt / N) * N + pt % N;
      load_global();
    }
  }
  block_partials_any<7>(acc, part, stride, blk);
}

}  // namespace gpe
