// Single and batched launches of the elementwise and reduction operations.
// Each operation is an argument record (kernels.h) with a device overload
//   run_op(const Args&, int blk, int nblk)
// that does the work of workgroup blk of nblk.  A single launch runs it with
// blk = blockIdx.x; a batched launch first finds the problem that owns the
// workgroup, then runs that problem's record with its local index.  A source
// file that defines run_op overloads instantiates launch_single and
// launch_batched for its records.
#pragma once

#include "common.h"
#include "kernels.h"

namespace gpe {

// Problem owning workgroup b (default: this one): the last p with
// blk0[p] <= b (one ballot per 64 problems).
__device__ __forceinline__ int batch_problem(const int* __restrict__ blk0, int nprob, int b = -1) {
  if (b < 0) b = (int)blockIdx.x;
  const int lane = threadIdx.x % kWave;
  int cnt = 0;
  for (int base = 0; base < nprob; base += kWave) {
    const int i = base + lane;
    const bool le = i < nprob && blk0[i] <= b;
    cnt += __popcll(__ballot(le));
  }
  return cnt - 1;
}


template <typename A>
__global__ void __launch_bounds__(kRedThreads) op_kernel(A a) {
  run_op(a, blockIdx.x, gridDim.x);
}

template <typename A>
__global__ void __launch_bounds__(kRedThreads)
op_batched_kernel(const A* __restrict__ args, const int* __restrict__ blk0, int nprob) {
  const int p = batch_problem(blk0, nprob);
  run_op(args[p], (int)blockIdx.x - blk0[p], blk0[p + 1] - blk0[p]);
}

template <typename A>
hipError_t launch_single(const A& a, int nblk, hipStream_t st) {
  if (nblk < 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL((op_kernel<A>), dim3(nblk), dim3(kRedThreads), 0, st, a);
  return hipGetLastError();
}

template <typename A>
hipError_t launch_batched(const A* args, const Span& sp, hipStream_t st) {
  if (sp.nprob < 1 || sp.nblocks < 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL((op_batched_kernel<A>), dim3(sp.nblocks), dim3(kRedThreads), 0, st, args, sp.blk0, sp.nprob);
  return hipGetLastError();
}

#define GPE_OP(...)                                                                              \
  template hipError_t launch_single<__VA_ARGS__>(const __VA_ARGS__&, int, hipStream_t);          \
  template hipError_t launch_batched<__VA_ARGS__>(const __VA_ARGS__*, const Span&, hipStream_t);

}  // namespace gpe
