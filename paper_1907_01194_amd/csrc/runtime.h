// Host runtime: the handle behind the C ABI and the device operations the
// C entry points and the Newton driver are built from.
#pragma once

#include <string>
#include <vector>

#include "../../include/gpe.h"
#include "kernels.h"

struct gpe_handle {
  // problem (Sec. 2, Sec. 3)
  int F = 0, K = 0, dim = 0;
  int n[3] = {1, 1, 1};
  double lo[3] = {0, 0, 0}, hi[3] = {1, 1, 1};
  double beta[4] = {0, 0, 0, 0};
  double p = 0, q = 0, M = 0;
  size_t npts = 0;   // grid points
  size_t nel = 0;    // K * npts complex elements per field
  double h = 0;      // prod_a h_a
  int prec = GPE_FP64;
  gpe_problem prob;                 // as given at creation
  std::vector<double> Vhost;        // potential on the grid (host copy, for coarse meshes)
  hipStream_t st = nullptr;
  int device = 0;

  // device constants and scratch
  double* V64 = nullptr;
  float* V32 = nullptr;
  gpe::LapAxis ax[3];
  void* tw[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
  double* part = nullptr;      // kMaxQ slots of pstride (>= kMaxRedBlocks) partial sums
  size_t pstride = 0;
  double* res = nullptr;       // kResDoubles doubles
  double* gram_pt = nullptr;   // ||u_i||^2 of the set point (7)
  double* gram_tmp = nullptr;  // scratch gram (7)
  unsigned int* ticket = nullptr;  // finalize completion counter (0 between launches)
  double* hres = nullptr;      // pinned host mirror of res
  bool res_shared = false;     // res / hres are slices of a batch's arrays (not owned)
  int nblk = 1;
  int xvar = 1;                // schedule variant of the fused x pass (autotuned)
  float xvar_us[3] = {0, 0, 0};  // measured microseconds per variant (0: not measured)
  gpe::PwParams pw;

  // owned fields
  void* T64 = nullptr;   // Laplacian scratch, c128
  void* T32 = nullptr;   // Laplacian scratch, c64 (mixed)
  void* Xp = nullptr;    // set point, c128
  void* Gp = nullptr;    // Euclidean gradient at the set point, c128
  void* Xp32 = nullptr;  // c64 copy of the set point (mixed)
  void* LX64 = nullptr;  // L X_p (FP64 handle)
  void* LX32 = nullptr;  // L X_p in c64 (mixed handle)
  std::vector<void*> solver_bufs;  // lazily allocated by the Newton driver

  // set-point state
  bool has_point = false;
  bool polish = false;   // a mixed handle's HVPs and CG run in FP64 (FP64 polish of a solve)
  double E_pt = 0, alpha_g = 0, beta_g = 0;

  // per-kernel event timing (gpe_timing_enable)
  struct TimingRec {
    int kind;
    hipEvent_t a, b;
  };
  bool timing = false;
  std::vector<TimingRec> recs;
  std::vector<hipEvent_t> event_pool;

  std::string err;
};

namespace gpe {

constexpr int kResDoubles = 64;   // reduction results per handle (res, hres)

// Status helpers: record a message on the handle and return the status.
gpe_status fail(gpe_handle* h, gpe_status s, const std::string& msg);
gpe_status hip_fail(gpe_handle* h, hipError_t e, const char* where);

#define GPE_HIP(h, call)                                   \
  do {                                                     \
    hipError_t e_ = (call);                                \
    if (e_ != hipSuccess) return gpe::hip_fail(h, e_, #call); \
  } while (0)

// Kernel kinds of the timing record.
enum KernelKind {
  KK_LAP_X = 0, KK_LAP_Y, KK_LAP_Z, KK_HVP_XPASS, KK_PW_GRAD, KK_FINALIZE, KK_PROJECT, KK_NORMS,
  KK_SCALE, KK_VECTOR, KK_COUNT
};
extern const char* const kKernelNames[KK_COUNT];
hipEvent_t timing_event(gpe_handle* h);

// Launch `call` (returning hipError_t) and, when timing is on, bracket it
// with events on the handle's stream.
#define GPE_KT(h, kind, call)                                           \
  do {                                                                  \
    hipEvent_t a_ = nullptr, b_ = nullptr;                              \
    if ((h)->timing) {                                                  \
      a_ = gpe::timing_event(h);                                        \
      b_ = gpe::timing_event(h);                                        \
      (void)hipEventRecord(a_, (h)->st);                                \
    }                                                                   \
    hipError_t e_ = (call);                                             \
    if ((h)->timing) {                                                  \
      (void)hipEventRecord(b_, (h)->st);                                \
      (h)->recs.push_back({(int)(kind), a_, b_});                       \
    }                                                                   \
    if (e_ != hipSuccess) return gpe::hip_fail(h, e_, #call);           \
  } while (0)

#define GPE_TRY(call)                  \
  do {                                 \
    gpe_status s_ = (call);            \
    if (s_ != GPE_OK) return s_;       \
  } while (0)

gpe_status alloc_field(gpe_handle* h, void** p, size_t bytes);

// Work precision of HVPs and CG vectors: c64 for a mixed handle unless it polishes in FP64.
inline bool work32(const gpe_handle* h) { return h->prec == GPE_MIXED && !h->polish; }

// out = L in (all axes), field precision T.
template <typename T>
gpe_status laplacian(gpe_handle* h, const void* in, void* out);

// Operations that end in a reduction come in two halves: *_enq launches the
// kernels and the finalize into h->res (stream-ordered, no synchronisation);
// after h->res has reached h->hres (fetch, or a lock-step round of a batch)
// *_read checks and returns the values.  The plain forms do both.
gpe_status finalize_enq(gpe_handle* h, int nq, int post, double* gram);
gpe_status fetch(gpe_handle* h);   // h->res -> h->hres, synchronises
gpe_status reduce_to_host(gpe_handle* h, int nq, int post, double* gram, int nout);

// Energy, gradient G (may be null), alpha_g/beta_g of G and ||X_i||^2 into gram.
gpe_status eval_enq(gpe_handle* h, const void* X, void* G, double* gram);
gpe_status eval_read(gpe_handle* h, bool grad, double* E, double* ag, double* bg);
gpe_status eval_point(gpe_handle* h, const void* X, void* G, double* gram, double* E, double* ag,
                      double* bg);

// gR = P_X G with the multipliers (ag, bg) already known; returns ||gR||.
gpe_status pgrad_enq(gpe_handle* h, const void* X, const void* G, void* gR, double ag, double bg);
gpe_status pgrad_read(gpe_handle* h, double* gnorm);
gpe_status project_grad(gpe_handle* h, const void* X, const void* G, void* gR, double ag, double bg,
                        double* gnorm);

// Make (X, G, E, ag, bg, gram) the set point without recomputing anything.
gpe_status adopt_point(gpe_handle* h);

// HVP at the set point in the work precision; if kappa != null also
// returns <Z, HZ> and ||Z||^2 (synchronises).
PwParams hvp_params(const gpe_handle* h, bool riemannian, double sigma);
gpe_status hvp_enq(gpe_handle* h, const void* Z, void* HZ, bool riemannian, double sigma, bool cg,
                   bool kappa = true);
gpe_status hvp_read(gpe_handle* h, double* kappa, double* zz);
gpe_status hvp(gpe_handle* h, const void* Z, void* HZ, bool riemannian, double sigma, double* kappa,
               double* zz);

// Retraction in two steps: norms of u and xi (xi in the precision xi32 ? c64 : c128),
// then the scaled combination for a given t.
struct RetractNorms {
  double uu[7], ux[7], xx[7];
};
gpe_status norms_enq(gpe_handle* h, const void* u, const void* xi, bool xi32);
gpe_status norms_read(gpe_handle* h, bool has_xi, RetractNorms* rn);
gpe_status retract_norms(gpe_handle* h, const void* u, const void* xi, bool xi32, RetractNorms* rn);
// Coefficients (alpha, beta) of the projection of xi onto the tangent space at
// u (Lemma 4.1 with the measured Gram system) from the norms of u and xi.
gpe_status proj_coeffs(gpe_handle* h, const RetractNorms& rn, double* alpha, double* beta);
// sigma_i of retraction `kind` at u + t xi, from the norms (host, FP64).
gpe_status retract_sigma_at(gpe_handle* h, const RetractNorms& rn, double t, int kind, double* sig);
gpe_status retract_apply(gpe_handle* h, const RetractNorms& rn, const void* u, const void* xi, bool xi32,
                         double t, int kind, void* out);
// Scalar part of the retractions (host, FP64): sigma_i from component norms a_i.
gpe_status retraction_sigma(gpe_handle* h, const double* a, int kind, double* sig);

// <a, b> with a c128 and b in (b32 ? c64 : c128), or both in the work precision.
gpe_status dot_enq(gpe_handle* h, const void* a, bool a32, const void* b, bool b32, size_t n);
gpe_status dot_read(gpe_handle* h, double* out);
gpe_status dot_host(gpe_handle* h, const void* a, bool a32, const void* b, bool b32, size_t n, double* out);

// Device-resident truncated CG (state in h->res[CG_*], see kernels.h), work
// precision: cg_init_enq after a reduction of ||r||^2 into res[0]; per
// iteration i (from 0) hvp_enq(..., cg = true), cg_step_enq (r += alpha q,
// residual and cap tests; z null) and cg_dir_enq (z += alpha p, then
// p = -r + beta p, see CgDirArgs).  After a fetch cg_state_read reports where
// the CG stands.
struct CgState {
  bool done;
  int reason;    // CG_STOP_*
  int iters;     // HVPs done
  double kappa, pp;   // at a curvature stop
};
gpe_status cg_init_enq(gpe_handle* h, double tol, double eps, int maxit);
gpe_status cg_step_enq(gpe_handle* h, const void* p, const void* q, void* z, void* r);
gpe_status cg_dir_enq(gpe_handle* h, const void* r, void* p, void* z, int iter);
bool cg_local_step(const gpe_handle* h);
gpe_status cg_state_read(gpe_handle* h, CgState* cs);

gpe_status newton_solve(gpe_handle* h, void* X, const gpe_solve_opts* o, gpe_solve_stats* st);
gpe_status tune_xpass(gpe_handle* h);
// Fourier prolongation of a c128 field from `coarse` to `fine` (2n per axis).
gpe_status prolong(const gpe_handle* coarse, const void* Xc, gpe_handle* fine, void* Xf);

}  // namespace gpe
