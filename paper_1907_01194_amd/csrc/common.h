// Shared device/host helpers of the HIP library: complex arithmetic on the
// interleaved (re, im) storage, wavefront reductions and launch constants.
#pragma once

#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>

namespace gpe {

template <typename T> struct cplx;
template <> struct cplx<double> { using type = double2; };
template <> struct cplx<float> { using type = float2; };
template <typename T> using c_t = typename cplx<T>::type;

template <typename T2> __host__ __device__ inline T2 mk(decltype(T2::x) re, decltype(T2::x) im) {
  T2 r; r.x = re; r.y = im; return r;
}
template <typename T2> __device__ __forceinline__ T2 cadd(T2 a, T2 b) { return mk<T2>(a.x + b.x, a.y + b.y); }
template <typename T2> __device__ __forceinline__ T2 csub(T2 a, T2 b) { return mk<T2>(a.x - b.x, a.y - b.y); }
template <typename T2> __device__ __forceinline__ T2 cmul(T2 a, T2 b) {
  return mk<T2>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// conj(a) * b
template <typename T2> __device__ __forceinline__ T2 cmulc(T2 a, T2 b) {
  return mk<T2>(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
template <typename T2> __device__ __forceinline__ T2 cconj(T2 a) { return mk<T2>(a.x, -a.y); }
template <typename T2, typename S> __device__ __forceinline__ T2 cscale(T2 a, S s) {
  return mk<T2>(a.x * s, a.y * s);
}
template <typename T2> __device__ __forceinline__ decltype(T2::x) cabs2(T2 a) { return a.x * a.x + a.y * a.y; }
// Re(a * conj(b))
template <typename T2> __device__ __forceinline__ decltype(T2::x) cdotr(T2 a, T2 b) { return a.x * b.x + a.y * b.y; }

// Loads/stores of one complex element, both precisions.
template <typename T2> __device__ __forceinline__ T2 ld(const T2* p) { return *p; }

constexpr int kWave = 64;          // CDNA wavefront width
constexpr int kRedThreads = 256;   // block size of reduction-producing kernels
constexpr int kMaxQ = 32;          // partial sums per reduction launch (max)
constexpr int kMaxRedBlocks = 2048;
constexpr int kXcds = 8;           // accelerator dies (XCDs), each with its own L2

// The hardware hands workgroup b of a launch to XCD b % kXcds.  Renumbered
// this way, consecutive numbers share an XCD and its L2: workgroups that read
// neighbouring parts of the same cache lines then find them there.  A
// bijection on [0, nb) for any nb; workgroup 0 keeps number 0.
__device__ __forceinline__ int xcd_local_block(int b, int nb) {
  const int x = b % kXcds, i = b / kXcds, q = nb / kXcds, rem = nb % kXcds;
  return x * q + (x < rem ? x : rem) + i;
}

// Sum of a double over the wavefront (shuffle tree).
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}

// Block-reduce NQ per-thread doubles and write the block's partial sums to
// part[q * nblk + blockIdx.x].  blockDim.x must be kRedThreads.
template <int NQ>
__device__ inline void block_partials(double (&acc)[NQ], double* __restrict__ part, int nblk) {
  __shared__ double red[kRedThreads / kWave][NQ > 0 ? NQ : 1];
  const int lane = threadIdx.x % kWave;
  const int wid = threadIdx.x / kWave;
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    double v = wave_sum(acc[q]);
    if (lane == 0) red[wid][q] = v;
  }
  __syncthreads();
  if (threadIdx.x < NQ) {
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < kRedThreads / kWave; ++w) s += red[w][threadIdx.x];
    part[(size_t)threadIdx.x * nblk + blockIdx.x] = s;
  }
}

// Same for any blockDim.x <= 1024 (a multiple of the wave size): block sums go
// to part[q * stride + blk].
template <int NQ>
__device__ inline void block_partials_any(const double (&acc)[NQ], double* __restrict__ part, size_t stride,
                                          size_t blk) {
  __shared__ double red[1024 / kWave][NQ > 0 ? NQ : 1];
  const int lane = threadIdx.x % kWave;
  const int wid = threadIdx.x / kWave;
  const int nw = (blockDim.x + kWave - 1) / kWave;
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    double v = wave_sum(acc[q]);
    if (lane == 0) red[wid][q] = v;
  }
  __syncthreads();
  if (threadIdx.x < NQ) {
    double s = 0.0;
    for (int w = 0; w < nw; ++w) s += red[w][threadIdx.x];
    part[(size_t)threadIdx.x * stride + blk] = s;
  }
}

inline int red_blocks(size_t npts) {
  size_t b = (npts + kRedThreads * 4 - 1) / (kRedThreads * 4);
  if (b < 1) b = 1;
  if (b > (size_t)kMaxRedBlocks) b = kMaxRedBlocks;
  return (int)b;
}

}  // namespace gpe
