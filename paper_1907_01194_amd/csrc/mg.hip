// Mesh transfer for the cascadic multigrid of Algorithm 1 (Sec. 5): the
// coarse mesh halves every axis of the same box (coarse node j = fine node
// 2j).  Prolongation is the Fourier (trigonometric) interpolant of the coarse
// samples, applied axis by axis as a real 2n x n matrix; restriction is
// injection.  Both act on c128 fields of K components.
#include "common.h"
#include "kernels.h"

namespace gpe {

// out[o][j'][i] = scale * sum_k P[j'][k] in[o][k][i]
__global__ void prolong_axis_kernel(const double2* __restrict__ in, double2* __restrict__ out,
                                    const double* __restrict__ P, int n, size_t inner, size_t total, double scale) {
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
    const size_t i = e % inner;
    const size_t jo = e / inner;
    const int jp = (int)(jo % (size_t)(2 * n));
    const size_t o = jo / (size_t)(2 * n);
    const double* prow = P + (size_t)jp * n;
    const double2* src = in + o * (size_t)n * inner + i;
    double re = 0.0, im = 0.0;
    for (int k = 0; k < n; ++k) {
      const double pk = prow[k];
      const double2 v = src[(size_t)k * inner];
      re += pk * v.x;
      im += pk * v.y;
    }
    double2 r;
    r.x = scale * re;
    r.y = scale * im;
    out[e] = r;
  }
}

hipError_t prolong_axis(const void* in, void* out, const double* P, int n, size_t inner, size_t outer, double scale,
                        hipStream_t st) {
  const size_t total = outer * (size_t)(2 * n) * inner;
  size_t g = (total + 255) / 256;
  if (g > 65536) g = 65536;
  hipLaunchKernelGGL(prolong_axis_kernel, dim3((unsigned)g), dim3(256), 0, st, reinterpret_cast<const double2*>(in),
                     reinterpret_cast<double2*>(out), P, n, inner, total, scale);
  return hipGetLastError();
}

// coarse[c][z][y][x] = scale * fine[c][2z][2y][2x]; nc = coarse sizes (x, y, z), unused axes 1
__global__ void restrict_kernel(const double2* __restrict__ fine, double2* __restrict__ coarse, int K, int ncx,
                                int ncy, int ncz, int sy, int sz, double scale) {
  const size_t npc = (size_t)ncx * ncy * ncz;
  const size_t total = npc * K;
  const size_t npf = (size_t)(ncx * 2) * (ncy * sy) * (ncz * sz);
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
    const int c = (int)(e / npc);
    size_t r = e % npc;
    const int x = (int)(r % ncx);
    r /= ncx;
    const int y = (int)(r % ncy);
    const int z = (int)(r / ncy);
    const size_t nfx = (size_t)ncx * 2, nfy = (size_t)ncy * sy;
    const size_t jf = ((size_t)(z * sz) * nfy + (size_t)(y * sy)) * nfx + (size_t)(2 * x);
    double2 v = fine[(size_t)c * npf + jf];
    v.x *= scale;
    v.y *= scale;
    coarse[e] = v;
  }
}

hipError_t restrict_inject(const void* fine, void* coarse, int K, int dim, const int* nc, double scale,
                           hipStream_t st) {
  const int ncx = nc[0], ncy = dim > 1 ? nc[1] : 1, ncz = dim > 2 ? nc[2] : 1;
  const size_t total = (size_t)K * ncx * ncy * ncz;
  size_t g = (total + 255) / 256;
  if (g > 65536) g = 65536;
  hipLaunchKernelGGL(restrict_kernel, dim3((unsigned)g), dim3(256), 0, st, reinterpret_cast<const double2*>(fine),
                     reinterpret_cast<double2*>(coarse), K, ncx, ncy, ncz, dim > 1 ? 2 : 1, dim > 2 ? 2 : 1, scale);
  return hipGetLastError();
}

}  // namespace gpe
