// Lock-step execution of Newton drivers.
//
// The driver of Algorithm 1 (solver.cpp) is written once, as a C++20
// coroutine per problem.  Instead of launching kernels and waiting for
// scalars itself, it queues device operations (Req) and suspends at the end
// of each step that needs a scalar back (Round).  The scheduler resumes every
// problem's coroutine until each has suspended, runs all queued operations
// (one batched launch per operation and stage for all problems that queued
// the same operation, single launches for a lone problem), copies every
// problem's reduction results to the host once and synchronises once, then
// resumes them all again.  A single solve is the one-problem case.
#pragma once

#include <coroutine>
#include <vector>

#include "runtime.h"

namespace gpe {

// Queued device operations.  Operand precisions: a32/b32/c32 select c64
// (true) or c128 (false); "work" is the handle's work precision.
enum ReqKind {
  RQ_EVAL = 0,   // energy and gradient: a = X, c = G (or null), gram; read with eval_read
  RQ_PGRAD,      // c = P_a b with multipliers (s0, s1), all c128; read with pgrad_read
  RQ_NORMS,      // retraction norms of a (c128) and b (b32, or null); read with norms_read
  RQ_SCALE,      // c (c128) = sig_i (a_i + s0 b_i), a c128, b in b32 or null
  RQ_DOT,        // <a, b> over n elements (a32, b32); read with dot_read
  RQ_DIFF,       // c (c32) = a - b (both c128), n elements
  RQ_AXPBY,      // c = s0 a + s1 c over n elements, precision a32 (s1 == 0: c not read)
  RQ_COPY,       // c (c32) = a (a32), or 0 if a is null, n elements
  RQ_LAP,        // c = L a, precision a32 (every axis)
  RQ_HVP,        // c = Hess a (work precision) at the set point, flag: Riemannian, s0 = sigma;
                 // read with hvp_read; cg: an iteration of the device-resident CG
  RQ_CG,         // rest of device-resident CG iteration (int)s0: r = d += alpha b with the
                 // tests, then z = a += alpha c and c = -d + beta c (see CgDirArgs)
  RQ_CGINIT,     // start the device-resident CG: tolerance s0, curvature factor s1, cap n
  RQ_COUNT
};

struct Req {
  int kind = RQ_EVAL;
  const void* a = nullptr;
  const void* b = nullptr;
  void* c = nullptr;
  void* d = nullptr;
  double s0 = 0.0, s1 = 0.0;
  double sig[7] = {0, 0, 0, 0, 0, 0, 0};
  double* gram = nullptr;
  size_t n = 0;
  bool a32 = false, b32 = false, c32 = false, flag = false, cg = false;
  bool kappa = true;   // RQ_HVP: form kappa = <Z, HZ> (always with cg)
};

// Coroutine of one problem's driver; its value is the problem's status.
struct SolveTask {
  struct promise_type {
    gpe_status status = GPE_OK;
    SolveTask get_return_object() {
      return SolveTask(std::coroutine_handle<promise_type>::from_promise(*this));
    }
    std::suspend_always initial_suspend() noexcept { return {}; }
    std::suspend_always final_suspend() noexcept { return {}; }
    void return_value(gpe_status s) { status = s; }
    void unhandled_exception() { status = GPE_ENOMEM; }   // host allocation failure
  };
  SolveTask() = default;
  explicit SolveTask(std::coroutine_handle<promise_type> c) : co(c) {}
  SolveTask(SolveTask&& o) noexcept : co(o.co) { o.co = {}; }
  SolveTask& operator=(SolveTask&& o) noexcept {
    if (this != &o) {
      if (co) co.destroy();
      co = o.co;
      o.co = {};
    }
    return *this;
  }
  SolveTask(const SolveTask&) = delete;
  SolveTask& operator=(const SolveTask&) = delete;
  ~SolveTask() {
    if (co) co.destroy();
  }
  std::coroutine_handle<promise_type> co;
};

// One problem in a lock-step run.
struct Ctx {
  gpe_handle* h = nullptr;
  std::vector<Req> q;      // operations queued since the last round, in order
  SolveTask task;
  gpe_status status = GPE_OK;
  bool done = false;
  void push(const Req& r) { q.push_back(r); }
};

// Awaited by a driver when it needs the results of its queued operations.
struct Round {
  bool await_ready() const noexcept { return false; }
  void await_suspend(std::coroutine_handle<>) const noexcept {}
  void await_resume() const noexcept {}
};

// Pinned host / device staging of the argument records of batched launches.
struct Stager {
  char* host = nullptr;
  char* dev = nullptr;
  size_t cap = 0, off = 0;
  // Copy bytes to the device (stream-ordered) and return the device address.
  // When the arena is full the stream is synchronised and it starts over.
  gpe_status put(gpe_handle* h, hipStream_t st, const void* src, size_t bytes, const void** dptr);
  // Two arrays staged back to back with one copy: the second starts at the
  // first's size rounded up to 16 bytes.
  gpe_status put2(gpe_handle* h, hipStream_t st, const void* a, size_t na, const void* b, size_t nb,
                  const void** da, const void** db);
  // Any number of arrays staged back to back (16-byte aligned) with one copy.
  struct Seg {
    const void* src;
    size_t bytes;
    const void** dptr;
  };
  gpe_status put_all(gpe_handle* h, hipStream_t st, const Seg* segs, size_t n);
};

// Run queued operations and the rounds of lock-step drivers.
class Lockstep {
 public:
  // batch: the batch the problems belong to (null for a lone handle).
  explicit Lockstep(::gpe_batch* batch) : b_(batch) {}
  // Execute every queued request; with sync, bring all results to the host
  // and synchronise, else leave the launches queued on the stream.
  gpe_status round(std::vector<Ctx*>& cs, bool sync = true);
  // Resume the drivers round after round until every one has returned.
  gpe_status run(std::vector<Ctx*>& cs);

 private:
  ::gpe_batch* b_;
};

// The driver (solver.cpp): Algorithm 1 on one mesh for the problem of c,
// X_inout c128 on the device.
SolveTask solve_task(Ctx& c, void* X_inout, const gpe_solve_opts* o, gpe_solve_stats* st);

// The driver run alone on a handle (batch.cpp).
gpe_status solve_single(gpe_handle* h, void* X_inout, const gpe_solve_opts* o, gpe_solve_stats* st);

}  // namespace gpe
