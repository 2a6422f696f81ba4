// Internal launch interface between the host runtime (handle, solver) and the
// HIP kernels.  Nothing here is part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <cstddef>

namespace gpe {

// One axis of the spectral Laplacian: lines of length n at stride `inner`,
// nlines = K * npts / n of them; lamc = 2 pi / (hi - lo) of that axis;
// twiddle tables exp(-2 pi i m / n), m = 0..n-1, in both precisions.
struct LapAxis {
  int n;
  int inner;
  long nlines;
  double lamc;
  const void* tw64;
  const void* tw32;
};

template <typename T>
hipError_t lap_axis(const LapAxis& ax, const void* in, const void* acc, void* out, hipStream_t st);
bool lap_size_supported(int n);

// Partial sums per reduction slot (finalize).
struct SlotCounts {
  int nb[32];   // kMaxQ
};

// Projection coefficients formed inside an axis pass instead of by a finalize
// launch: every workgroup sums slots 0 and 1 of the x pass's n partials
// (stride apart) in the same order and solves Lemma 4.1's 2x2 Gram system with
// the set point's component norms gram; workgroup 0 also stores the two
// coefficients in res[32..33] (part null: off).
struct AbSrc {
  const double* part = nullptr;
  size_t stride = 0;
  int n = 0;
  const double* gram = nullptr;
  double* res = nullptr;
};
// Largest x-pass workgroup count for which the last axis pass forms the
// projection coefficients itself.
constexpr int kAbLocalMax = 1024;

// Physical constants of the pointwise terms, already combined with h:
// zee[l] = b_l (storage order), c0 = 2 beta0 / h, ... (gradient factors)
// and e0 = beta0 / (2h), ... (energy factors).
struct PwParams {
  double zee[7];
  double g[4];   // 2 beta_k / h
  double e[4];   // beta_k / (2h)
  double zc[7];  // HVP only: extra multiple of Z_i added to W_i
};

// Energy density (+ gradient).  Partials layout (nq = 1 + 2K):
//   [0] sum of the energy density, [1+i] <X_i, G_i>, [1+K+i] ||X_i||^2.
// G may be null (energy only; then [1+i] is 0).
template <typename T>
hipError_t pw_grad(int F, const void* X, const void* LX, const T* V, void* G, double* part,
                   int nblk, size_t npts, const PwParams& p, hipStream_t st);

// Fused x-axis pass of the HVP (all components of RPB x-rows per workgroup):
//   W = L_x Z + (pointwise Hessian terms of Sec. 3) + p.zc[i] Z_i,
// with FP64 partial sums (one per workgroup, slots of stride `stride`):
//   [0] sum_i <X_i, W_i>  [1] sum_i l_i <X_i, W_i>  (both through <(LX)_i, Z_i> = <X_i, (LZ)_i>,
//   Y = L X), [2] sum <X_i,Z_i>, [3] sum l_i <X_i,Z_i>, [4] <Z, W - LZ>, [5] ||Z||^2,
//   [6] <Z, L_x Z> (Parseval).
// Returns the number of workgroups (partials per slot) in *nblk_out.
// var: schedule variant (rows per workgroup), 0 .. xpass_variants(n)-1; 1 is the default.
// skip (all the launches below that take one): a device flag; when it is
// nonzero at launch time every workgroup returns at once (null: never).
template <typename T>
hipError_t hvp_xpass(int F, const LapAxis& ax, size_t npts, const void* X, const void* Z, const void* Y,
                     const T* V, void* W, const PwParams& p, double* part, size_t stride, int* nblk_out, int var,
                     const double* skip, hipStream_t st);
int xpass_variants(int n);

// Axis pass with Parseval partial <Z, L_a Z> into part[slot * stride + wg] and,
// if coef != null, the projection epilogue out -= (coef[0] + coef[1] l) X
// (coefficients from coef, or formed in the pass from ab).  fin non-null: one
// more workgroup forms the projection coefficients from fin's partials into
// fin->res[32..33] for a later pass of the same HVP.
template <typename T>
hipError_t lap_axis_ex(const LapAxis& ax, const void* in, const void* acc, void* out, int F, size_t npts,
                       const void* X, const double* coef, double* part, size_t stride, int slot, int* nblk_out,
                       const double* skip, int rev, const AbSrc* ab, const AbSrc* fin, hipStream_t st);
size_t lap_max_blocks(const LapAxis& ax, int K);

// Post-processing done by the single-block finalize kernel after summing the
// partial sums into res[0..nq).
enum PostOp {
  POST_NONE = 0,
  // res = [e, <X_i,G_i>, ||X_i||^2]: writes alpha_g, beta_g to res[nq], res[nq+1]
  // and copies ||X_i||^2 into gram[0..K).
  POST_GRAD = 1,
  // res = HVP slots 0..6 (see hvp_xpass), gram = ||X_i||^2 of the point:
  // writes the projection coefficients alpha_w, beta_w to res[32], res[33].
  POST_HVP_AB = 2,
  // res = HVP slots 0..8 (x, y, z Parseval in 6, 7, 8), projection
  // coefficients in res[32..33] (zero for a Euclidean HVP):
  // writes kappa = <Z, HZ> to res[34] and ||Z||^2 to res[35].
  POST_HVP_KAPPA = 3,
  // as POST_HVP_KAPPA for a Euclidean HVP: no projection, res[32..33] unused
  POST_HVP_KAPPA_E = 4,
  // truncated CG on the device (state in res[CG_*]): POST_HVP_KAPPA, then one
  // more HVP is counted and either the curvature test stops the CG or
  // alpha = rr / kappa
  POST_CG_KAPPA = 5,
  // after the CG update (res[0] = ||r||^2): the residual test stops the CG,
  // else beta = ||r||^2 / rr, rr = ||r||^2, and the iteration cap stops it
  POST_CG_STEP = 6
};

// Device-resident state of the truncated CG of the Newton model, in a
// handle's res array (doubles): the stop flag doubles as the skip flag of every
// launch of the CG iteration, so the host can queue several iterations at once.
enum CgSlot {
  CG_RR = 40,     // ||r||^2 at the start of an even iteration (CG_RR1: odd), so that
                  // the step that stores the next one never overwrites the one being read
  CG_ALPHA,       // step of the last CG update
  CG_BETA,        // direction coefficient of the last update
  CG_DONE,        // 0 while running, 1 once stopped
  CG_IT,          // HVPs done (one per iteration)
  CG_KAPPA,       // kappa and ||p||^2 at a curvature stop
  CG_PP,
  CG_REASON,      // CG_STOP_*
  CG_TOL,         // residual tolerance
  CG_EPS,         // curvature threshold factor: stop when kappa <= eps ||p||^2
  CG_MAXIT,       // iteration cap
  CG_RR1,
  CG_CURV         // 1 once the curvature test stopped the CG (written only by the kappa finalize,
                  // so the closing step can read it while its workgroup 0 writes CG_REASON)
};
// ||r||^2 at the start of iteration i (0-based) of the CG
__host__ __device__ inline int cg_rr_slot(int i) { return (i & 1) ? CG_RR1 : CG_RR; }
enum CgStop { CG_STOP_NONE = 0, CG_STOP_CURVATURE = 1, CG_STOP_RESIDUAL = 2, CG_STOP_CAP = 3 };
// Sum partials part[q * stride + b], b < nb[q], for q < nq into res[q]
// (deterministic), then apply `post`.  One workgroup, or with many partials
// one per slot; ticket (may be null: always one workgroup) is a device counter
// that is 0 between launches (the launch leaves it at 0).
hipError_t finalize(const double* part, size_t stride, const SlotCounts& nb, int nq, double* res, int post,
                    int F, double* gram, unsigned int* ticket, const double* skip, hipStream_t st);

// out_i = W_i - (coef[0] + coef[1] l_i) X_i (coef on the device).  X is c128
// or c64 as TX; W/out in T.  If part != null, partial sums of ||out||^2 (nq = 1).
template <typename T, typename TX>
hipError_t project(int F, const void* X, const void* W, void* out, const double* coef,
                   double* part, int nblk, size_t npts, hipStream_t st);

// Per-component sums for the retraction: [i] ||u_i||^2, [K+i] <u_i, xi_i>,
// [2K+i] ||xi_i||^2 (nq = 3K).  xi may be null (then only the first K are set).
template <typename TU, typename TXI>
hipError_t comp_norms(int K, const void* u, const void* xi, double* part, int nblk,
                      size_t npts, hipStream_t st);

// out_i = s_i (u_i + t xi_i), i = 0..K-1.  out may alias u.
template <typename TU, typename TXI, typename TO>
hipError_t scale_comps(int K, const void* u, const void* xi, double t, const double* s,
                       void* out, size_t npts, hipStream_t st);

// y = a x + b y (complex fields of n elements of type T, real scalars);
// b == 0 gives y = a x without reading y.
template <typename T>
hipError_t axpby(double a, const void* x, double b, void* y, size_t n, hipStream_t st);

// z += a p; r += a q; partial sums of ||r||^2 (nq = 1).
template <typename T>
hipError_t cg_update(double a, const void* p, const void* q, void* z, void* r, double* part,
                     int nblk, size_t n, hipStream_t st);

// Partial sums of <a, b> = Re sum a conj(b) (nq = 1), a in TA, b in TB.
template <typename TA, typename TB>
hipError_t dot(const void* a, const void* b, double* part, int nblk, size_t n, hipStream_t st);

// Precision conversion of complex fields.
hipError_t to_c64(const void* src, void* dst, size_t n, hipStream_t st);
hipError_t to_c128(const void* src, void* dst, size_t n, hipStream_t st);

// out = a - b (complex fields) in T.
template <typename TA, typename TB, typename TO>
hipError_t diff(const void* a, const void* b, void* out, size_t n, hipStream_t st);

// ---------------------------------------------------------------- batched launches
// One launch runs an operation for nprob problems: problem p owns the
// workgroups blk0[p] .. blk0[p+1]-1 (blk0: nprob + 1 non-decreasing ints in
// device memory, blk0[0] = 0) and takes its arguments from args[p] (device
// memory).  Within its range a problem's workgroups do exactly what a single
// launch of that many workgroups does for it.
struct Span {
  const int* blk0;
  int nprob;
  int nblocks;   // blk0[nprob]
};

// Argument records of the elementwise and reduction operations above.
// Reductions write partial sums part[q * nblk + wg] for their nblk
// workgroups; elementwise operations take any workgroup count.
template <typename T> struct AxpbyArgs {   // y = a x + b y; b == 0: y = a x (y not read)
  const void* x;
  void* y;
  double a, b;
  size_t n;
};
template <typename T> struct CgArgs {      // z += a p (z null: skipped, p not read); r += a q; partials of ||r||^2
  const void* p;
  const void* q;
  void* z;
  void* r;
  double* part;
  double a;
  size_t n;
  const double* adev = nullptr;   // a from device memory when set
  const double* skip = nullptr;
};
// Closing step of iteration iter of a device-resident CG (state in res[CG_*]):
// if that iteration reached its update (res[CG_IT] == iter + 1), z += alpha p
// unless it stopped on curvature, then p = -r + beta p unless the CG has
// stopped.  Reads p before overwriting it; r is not read once stopped.
template <typename T> struct CgDirArgs {
  const void* r;
  void* p;
  void* z;
  double* res;
  int iter;
  size_t n;
  // part non-null: the CG update's nb partials of ||r||^2 (no finalize launch);
  // every workgroup sums them in the same order and applies the residual and
  // cap tests itself, and workgroup 0 stores the outcome in res
  const double* part = nullptr;
  int nb = 0;
};
// Start of a device-resident CG: rr = res[0] (the preceding reduction), not
// stopped, no iteration yet, with the given tolerance, curvature factor and cap.
struct CgInitArgs {
  double* res;
  double tol, eps;
  int maxit;
};
template <typename TA, typename TB> struct DotArgs {   // partials of <a, b>
  const void* a;
  const void* b;
  double* part;
  size_t n;
};
template <typename TA, typename TB, typename TO> struct DiffArgs {   // out = a - b
  const void* a;
  const void* b;
  void* out;
  size_t n;
};
template <typename T> struct FillArgs {   // out = pseudo-random complex values in [-1, 1) (timing data)
  void* out;
  size_t n;
  unsigned seed;
};
template <typename TI, typename TO> struct ConvArgs {   // dst = src (converted); src null: dst = 0
  const void* src;
  void* dst;
  size_t n;
};
template <typename TU, typename TXI, typename TO> struct ScaleArgs {   // out_i = s_i (u_i + t xi_i)
  const void* u;
  const void* xi;
  void* out;
  double t;
  double s[7];
  size_t npts;
  int K;
};
template <typename TU, typename TXI, int K> struct NormsArgs {   // retraction norms (see comp_norms)
  const void* u;
  const void* xi;
  double* part;
  size_t npts;
};
// out_i = W_i - (c0 + c1 l_i) X_i with (c0, c1) = coef[0..1] (device) or, if
// coef is null, the values given; NORM: partials of ||out||^2.
template <typename T, typename TX, bool NORM> struct ProjArgs {
  const void* X;
  const void* W;
  void* out;
  const double* coef;
  double c0, c1;
  double* part;
  size_t npts;
  int F;
};
template <typename T, int F, bool GRAD> struct PwGradArgs {   // see pw_grad
  const void* X;
  const void* LX;
  const void* V;
  void* G;
  double* part;
  size_t npts;
  PwParams p;
};

// Single launch with nblk workgroups, and batched launch.
template <typename A> hipError_t launch_single(const A& a, int nblk, hipStream_t st);
template <typename A> hipError_t launch_batched(const A* args, const Span& sp, hipStream_t st);
// Workgroups an elementwise operation over `total` elements uses.
int elementwise_blocks(size_t total);

// Batched finalize: problem p sums args[p].part (stride args[p].stride, counts
// args[p].nb) into args[p].res with its own gram; one workgroup per problem.
struct FinArgs {
  const double* part;
  double* res;
  double* gram;
  size_t stride;
  SlotCounts nb;
  const double* skip;
};
hipError_t finalize_batched(const FinArgs* args, int nprob, int nq, int post, int F, hipStream_t st);

// Batched axis pass (lap_axis_ex for every problem; line length n of each
// problem's axis a power of two in 16..512, see batch_size_supported).
template <typename T> struct LapArgs {
  const void* in;
  const void* acc;
  void* out;
  const void* tw;       // twiddles of that axis in precision T
  const void* X;        // projection epilogue (null: none)
  const double* coef;
  double* part;         // Parseval partials (null: none)
  double lamc;
  long nlines;
  size_t npts;
  size_t stride;
  int inner;
  int n;
  const double* skip;
  AbSrc ab;             // projection coefficients formed in the pass (part null: from coef)
};
template <typename T>
hipError_t lap_batched(const LapArgs<T>* args, const Span& sp, int F, int slot, hipStream_t st);
int lap_batch_blocks(int n, long nlines);
bool batch_size_supported(int n);

// Batched fused x pass (hvp_xpass for every problem with schedule variant var).
template <typename T> struct XpassArgs {
  const void* X;
  const void* Z;
  const void* Y;
  const void* V;
  void* W;
  const void* tw;
  double* part;
  double lamc;
  size_t npts;
  size_t stride;
  int n;
  PwParams p;
  const double* skip;
};
template <typename T>
hipError_t xpass_batched(int F, int var, const XpassArgs<T>* args, const Span& sp, hipStream_t st);
int xpass_batch_blocks(int n, int F, int var, size_t npts);

// Multigrid transfer (c128 fields).  prolong_axis: out[o][j'][i] = scale *
// sum_k P[j' n + k] in[o][k][i] with j' < 2n (P real, on the device).
// restrict_inject: coarse[c][z][y][x] = scale * fine[c][2z][2y][2x] (nc = coarse
// sizes, x first).
hipError_t prolong_axis(const void* in, void* out, const double* P, int n, size_t inner, size_t outer, double scale,
                        hipStream_t st);
hipError_t restrict_inject(const void* fine, void* coarse, int K, int dim, const int* nc, double scale,
                           hipStream_t st);

}  // namespace gpe
