"""ctypes binding of libgpe.so (C ABI in include/gpe.h).

Argument marshalling only: every computation runs in the HIP library.  PyTorch
provides device memory and the stream.  Fields are torch tensors on the GPU,
contiguous, of shape (K, n_z, n_y, n_x) (trailing spatial axes dropped in
1D/2D), dtype complex128 for master fields and complex128/complex64 (the
handle's work precision) for HVP directions.

The library is loaded on first use and a missing build raises RuntimeError:
there is no fallback path.
"""

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgpe.so")

c_int = ctypes.c_int
c_double = ctypes.c_double
c_void_p = ctypes.c_void_p

STATUS = {0: "GPE_OK", 1: "GPE_EINVAL", 2: "GPE_EDOMAIN", 3: "GPE_EDEGEN", 4: "GPE_ENUMERIC",
          5: "GPE_ENOTCONV", 6: "GPE_ENOMEM", 7: "GPE_EHIP"}
FP64, MIXED = 0, 1
R1, R2, R3 = 1, 2, 3


class gpe_problem(ctypes.Structure):
    _fields_ = [("F", c_int), ("dim", c_int), ("n", c_int * 3), ("lo", c_double * 3),
                ("hi", c_double * 3), ("beta", c_double * 4), ("p", c_double), ("q", c_double),
                ("M", c_double)]


class gpe_solve_opts(ctypes.Structure):
    _fields_ = [("tol", c_double), ("maxit", c_int), ("retraction", c_int),
                ("rgbb_tol", c_double), ("rgbb_maxit", c_int),
                ("rgbb_rho", c_double), ("rgbb_delta", c_double), ("rgbb_varrho", c_double),
                ("rgbb_step0", c_double),
                ("eta1", c_double), ("eta2", c_double), ("gamma0", c_double), ("gamma1", c_double),
                ("gamma2", c_double), ("sigma_hat0", c_double),
                ("rho", c_double), ("delta", c_double), ("alpha0", c_double),
                ("ls_max", c_int), ("cg_maxit", c_int), ("cg_T", c_double), ("cg_theta", c_double),
                ("max_reject_streak", c_int), ("sigma_hat_min", c_double), ("verbose", c_int), ("time_limit", c_double),
                ("mg_levels", c_int), ("mg_coarse_tol", c_double), ("polish_tol", c_double),
                ("polish_window", c_int), ("cg_per_digit", c_double),
                ("trace", ctypes.POINTER(c_double)), ("trace_cap", c_int)]

TRACE_COLS = 10
TRACE_NAMES = ("t", "E", "gnorm", "hvp_calls", "sigma", "ratio", "cg_iters", "cg_reason", "step", "accepted")


class gpe_solve_stats(ctypes.Structure):
    _fields_ = [("E", c_double), ("gnorm", c_double), ("converged", c_int), ("rgbb_iters", c_int),
                ("outer", c_int), ("cg_total", c_int), ("hvp_calls", c_int), ("ls_trials", c_int),
                ("rejected", c_int), ("t_total", c_double), ("t_rgbb", c_double),
                ("t_arnt", c_double), ("mass_err", c_double), ("mag_err", c_double),
                ("mg_levels", c_int), ("t_coarse", c_double), ("polish_at", c_int), ("trace_len", c_int)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


# name -> (restype, argtypes); the list mirrors include/gpe.h
SIGNATURES = {
    "gpe_solve_opts_default": (None, [ctypes.POINTER(gpe_solve_opts)]),
    "gpe_create": (c_int, [ctypes.POINTER(gpe_problem), c_void_p, c_int, c_void_p, ctypes.POINTER(c_void_p)]),
    "gpe_destroy": (c_int, [c_void_p]),
    "gpe_energy": (c_int, [c_void_p, c_void_p, ctypes.POINTER(c_double)]),
    "gpe_grad": (c_int, [c_void_p, c_void_p, c_void_p, c_int, ctypes.POINTER(c_double),
                         ctypes.POINTER(c_double)]),
    "gpe_set_point": (c_int, [c_void_p, c_void_p]),
    "gpe_hvp": (c_int, [c_void_p, c_void_p, c_void_p, c_int, c_double]),
    "gpe_hvp_dot": (c_int, [c_void_p, c_void_p, c_void_p, c_double, ctypes.POINTER(c_double)]),
    "gpe_retract": (c_int, [c_void_p, c_void_p, c_void_p, c_double, c_int, c_void_p]),
    "gpe_constraints": (c_int, [c_void_p, c_void_p, ctypes.POINTER(c_double), ctypes.POINTER(c_double)]),
    "gpe_retract_noalloc": (c_int, [ctypes.POINTER(gpe_problem), c_void_p, c_void_p, c_double, c_int, c_void_p,
                                    c_void_p]),
    "gpe_newton_solve": (c_int, [c_void_p, c_void_p, ctypes.POINTER(gpe_solve_opts),
                                 ctypes.POINTER(gpe_solve_stats)]),
    "gpe_project": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p]),
    "gpe_prolong": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p]),
    "gpe_schedule": (c_int, [c_void_p, ctypes.POINTER(c_int), ctypes.POINTER(ctypes.c_float), c_int]),
    "gpe_set_schedule": (c_int, [c_void_p, c_int]),
    "gpe_schedule_count": (c_int, [c_void_p, ctypes.POINTER(c_int)]),
    "gpe_timing_enable": (c_int, [c_void_p, c_int]),
    "gpe_timing_read": (c_int, [c_void_p, c_int, ctypes.POINTER(ctypes.c_char_p), ctypes.POINTER(c_int),
                                ctypes.POINTER(c_double), ctypes.POINTER(c_int)]),
    "gpe_last_error": (ctypes.c_char_p, [c_void_p]),
    "gpe_version": (ctypes.c_char_p, []),
    "gpe_batch_create": (c_int, [ctypes.POINTER(gpe_problem), ctypes.POINTER(c_void_p), c_int, c_int, c_void_p,
                                 ctypes.POINTER(c_void_p)]),
    "gpe_batch_destroy": (c_int, [c_void_p]),
    "gpe_batch_size": (c_int, [c_void_p, ctypes.POINTER(c_int)]),
    "gpe_batch_handle": (c_int, [c_void_p, c_int, ctypes.POINTER(c_void_p)]),
    "gpe_batch_hvp": (c_int, [c_void_p, ctypes.POINTER(c_void_p), ctypes.POINTER(c_void_p), c_int,
                              ctypes.POINTER(c_double), ctypes.POINTER(c_double)]),
    "gpe_batch_newton_solve": (c_int, [c_void_p, ctypes.POINTER(c_void_p), ctypes.POINTER(gpe_solve_opts),
                                       ctypes.POINTER(gpe_solve_stats)]),
    "gpe_batch_schedule": (c_int, [c_void_p, ctypes.POINTER(c_int), ctypes.POINTER(ctypes.c_float), c_int]),
    "gpe_batch_last_error": (ctypes.c_char_p, [c_void_p]),
}

_lib = None


def lib():
    """Load libgpe.so (once).  Raises RuntimeError if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libgpe.so is not built (run `python -m paper_1907_01194_amd.build`); "
                               "there is no fallback implementation")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


class GpeError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s: %s" % (STATUS.get(status, status), msg))
        self.status = status


def default_opts(**kw):
    o = gpe_solve_opts()
    lib().gpe_solve_opts_default(ctypes.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o


def _ptr(t, dtype, shape):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("expected a CUDA tensor")
    if t.dtype != dtype:
        raise TypeError("expected dtype %s, got %s" % (dtype, t.dtype))
    if tuple(t.shape) != tuple(shape):
        raise ValueError("expected shape %s, got %s" % (tuple(shape), tuple(t.shape)))
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return c_void_p(t.data_ptr())


def problem_struct(spec):
    """gpe_problem of a spec (F, n with x first, lo, hi, beta, M, p, q)."""
    pr = gpe_problem()
    pr.F = int(spec.F)
    pr.dim = len(spec.n)
    for a in range(3):
        pr.n[a] = int(spec.n[a]) if a < pr.dim else 1
        pr.lo[a] = float(spec.lo[a]) if a < pr.dim else 0.0
        pr.hi[a] = float(spec.hi[a]) if a < pr.dim else 1.0
    beta = list(spec.beta) + [0.0] * (4 - len(spec.beta))
    for k in range(4):
        pr.beta[k] = float(beta[k])
    pr.p, pr.q, pr.M = float(spec.p), float(spec.q), float(spec.M)
    return pr


def retract_noalloc(spec, X, Xi, t=1.0, kind=R1, out=None):
    """gpe_retract_noalloc: Xout = psi(X + t Xi) with no handle and no device
    allocation by the library (X, Xi, out: complex128 CUDA tensors of the
    problem's field shape; Xi may be None).  Runs on torch's current stream."""
    import torch
    shape = (2 * int(spec.F) + 1,) + tuple(reversed(tuple(spec.n)))
    Xo = out if out is not None else torch.empty(shape, dtype=torch.complex128, device=X.device)
    pr = problem_struct(spec)
    xi = _ptr(Xi, torch.complex128, shape) if Xi is not None else None
    st = lib().gpe_retract_noalloc(ctypes.byref(pr), _ptr(X, torch.complex128, shape), xi, float(t), int(kind),
                                   _ptr(Xo, torch.complex128, shape),
                                   c_void_p(torch.cuda.current_stream(X.device).cuda_stream))
    if st != 0:
        raise GpeError(st, lib().gpe_last_error(None).decode())
    return Xo


def potential(spec, grid_shape):
    V = np.ascontiguousarray(spec.V, dtype=np.float64)
    if V.shape != tuple(grid_shape):
        raise ValueError("potential has shape %s, grid is %s" % (V.shape, tuple(grid_shape)))
    return V


class Problem:
    """One gpe handle.

    spec: an object with F, n (x first), lo, hi, V (numpy, grid shape), beta
    (4 values), M, p, q -- e.g. workloads.Spec.  precision: "fp64" or "mixed".
    All calls are ordered on torch's current stream of ``device``.
    """

    def __init__(self, spec, precision="fp64", device=0, _handle=None):
        import torch
        self.torch = torch
        self.device = torch.device("cuda", device)
        torch.cuda.set_device(self.device)
        self.spec = spec
        self.F = int(spec.F)
        self.K = 2 * self.F + 1
        self.shape = (self.K,) + tuple(reversed(tuple(spec.n)))
        self.precision = {"fp64": FP64, "mixed": MIXED}[precision]
        self.work_dtype = torch.complex128 if self.precision == FP64 else torch.complex64
        self.stream = torch.cuda.current_stream(self.device)
        self._owned = _handle is None
        if _handle is not None:        # a batch's handle: the batch owns it
            self.h = _handle
            return
        pr = problem_struct(spec)
        V = potential(spec, self.shape[1:])
        h = c_void_p()
        st = lib().gpe_create(ctypes.byref(pr), V.ctypes.data_as(c_void_p), self.precision,
                              c_void_p(self.stream.cuda_stream), ctypes.byref(h))
        if st != 0:
            raise GpeError(st, lib().gpe_last_error(None).decode())
        self.h = h

    # ------------------------------------------------------------ helpers
    def _check(self, st):
        if st != 0:
            raise GpeError(st, lib().gpe_last_error(self.h).decode())

    def empty(self, work=False):
        dt = self.work_dtype if work else self.torch.complex128
        return self.torch.empty(self.shape, dtype=dt, device=self.device)

    def _m(self, X):
        return _ptr(X, self.torch.complex128, self.shape)

    def _w(self, Z):
        return _ptr(Z, self.work_dtype, self.shape)

    def close(self):
        if getattr(self, "h", None):
            if self._owned:
                lib().gpe_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------ C ABI calls
    def energy(self, X):
        E = c_double()
        self._check(lib().gpe_energy(self.h, self._m(X), ctypes.byref(E)))
        return E.value

    def grad(self, X, riemannian=False, out=None):
        G = out if out is not None else self.empty()
        E, gn = c_double(), c_double()
        self._check(lib().gpe_grad(self.h, self._m(X), self._m(G), int(bool(riemannian)),
                                   ctypes.byref(E), ctypes.byref(gn)))
        return G, E.value, gn.value

    def set_point(self, X):
        self._check(lib().gpe_set_point(self.h, self._m(X)))

    def hvp(self, Z, riemannian=False, sigma=0.0, out=None):
        HZ = out if out is not None else self.empty(work=True)
        self._check(lib().gpe_hvp(self.h, self._w(Z), self._w(HZ), int(bool(riemannian)), float(sigma)))
        return HZ

    def hvp_dot(self, Z, sigma=0.0, out=None):
        HZ = out if out is not None else self.empty(work=True)
        k = c_double()
        self._check(lib().gpe_hvp_dot(self.h, self._w(Z), self._w(HZ), float(sigma), ctypes.byref(k)))
        return HZ, k.value

    def retract(self, X, Xi, t=1.0, kind=R1, out=None):
        Xo = out if out is not None else self.empty()
        xi = self._m(Xi) if Xi is not None else None
        self._check(lib().gpe_retract(self.h, self._m(X), xi, float(t), int(kind), self._m(Xo)))
        return Xo

    def project(self, X, W, out=None):
        O = out if out is not None else self.empty()
        self._check(lib().gpe_project(self.h, self._m(X), self._m(W), self._m(O)))
        return O

    def prolong(self, Xc, fine, out=None):
        """Fourier prolongation of Xc (this handle's mesh) onto ``fine`` (2n per axis)."""
        Xf = out if out is not None else fine.empty()
        self._check(lib().gpe_prolong(self.h, self._m(Xc), fine.h, fine._m(Xf)))
        return Xf

    def schedule(self):
        """(chosen x-pass variant, measured microseconds per variant)."""
        v = c_int()
        us = (ctypes.c_float * 3)()
        self._check(lib().gpe_schedule(self.h, ctypes.byref(v), us, 3))
        return v.value, list(us)

    def set_schedule(self, variant):
        """Force x-pass schedule variant ``variant`` (see schedule_count)."""
        self._check(lib().gpe_set_schedule(self.h, int(variant)))

    def schedule_count(self):
        n = c_int()
        self._check(lib().gpe_schedule_count(self.h, ctypes.byref(n)))
        return n.value

    def timing(self, enable=True):
        self._check(lib().gpe_timing_enable(self.h, int(bool(enable))))

    def timing_read(self):
        """{kernel kind: (launches, total ms)} since timing(True)."""
        m = 16
        names = (ctypes.c_char_p * m)()
        counts = (c_int * m)()
        ms = (c_double * m)()
        nk = c_int()
        self._check(lib().gpe_timing_read(self.h, m, names, counts, ms, ctypes.byref(nk)))
        return {names[i].decode(): (counts[i], ms[i]) for i in range(min(nk.value, m))}

    def constraints(self, X):
        m, g = c_double(), c_double()
        self._check(lib().gpe_constraints(self.h, self._m(X), ctypes.byref(m), ctypes.byref(g)))
        return m.value, g.value

    def newton_solve(self, X, check=True, trace=0, **opts):
        """Algorithm 1 from X (overwritten).  trace > 0 asks for up to `trace`
        rows of the per-iteration trace, returned as stats["trace"] (a numpy
        array with columns TRACE_NAMES)."""
        o = default_opts(**opts)
        buf = None
        if trace:
            buf = np.zeros((int(trace), TRACE_COLS))
            o.trace = buf.ctypes.data_as(ctypes.POINTER(c_double))
            o.trace_cap = int(trace)
        s = gpe_solve_stats()
        st = lib().gpe_newton_solve(self.h, self._m(X), ctypes.byref(o), ctypes.byref(s))
        if st != 0 and (check or st != 5):
            self._check(st)
        out = s.as_dict()
        if buf is not None:
            out["trace"] = buf[:s.trace_len].copy()
        return X, out


class Batch:
    """A gpe_batch: problems of one spin F and dimension (any grids, boxes,
    potentials and parameters) whose HVPs and Newton solves run in lock step,
    one launch per kernel stage for all of them.  ``problems[i]`` is a
    Problem view of problem i's handle (owned by the batch)."""

    def __init__(self, specs, precision="mixed", device=0):
        import torch
        self.torch = torch
        self.device = torch.device("cuda", device)
        torch.cuda.set_device(self.device)
        self.stream = torch.cuda.current_stream(self.device)
        m = len(specs)
        probs = (gpe_problem * m)(*[problem_struct(sp) for sp in specs])
        shapes = [tuple(reversed(tuple(sp.n))) for sp in specs]
        self._V = [potential(sp, sh) for sp, sh in zip(specs, shapes)]
        Vp = (c_void_p * m)(*[V.ctypes.data for V in self._V])
        b = c_void_p()
        st = lib().gpe_batch_create(probs, Vp, m, {"fp64": FP64, "mixed": MIXED}[precision],
                                    c_void_p(self.stream.cuda_stream), ctypes.byref(b))
        if st != 0:
            raise GpeError(st, lib().gpe_batch_last_error(None).decode())
        self.b = b
        self.problems = []
        for i, sp in enumerate(specs):
            h = c_void_p()
            self._check(lib().gpe_batch_handle(self.b, i, ctypes.byref(h)))
            self.problems.append(Problem(sp, precision, device, _handle=h))

    def __len__(self):
        return len(self.problems)

    def _check(self, st):
        if st != 0:
            raise GpeError(st, lib().gpe_batch_last_error(self.b).decode())

    def close(self):
        if getattr(self, "b", None):
            for p in self.problems:
                p.h = None
            lib().gpe_batch_destroy(self.b)
            self.b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def hvp(self, Zs, riemannian=False, sigma=None, outs=None, kappa=True):
        """HZ_i = Hess(Z_i) for every problem at its set point; returns (HZs, kappas).
        kappa=False: no kappas (None) and no synchronisation."""
        m = len(self.problems)
        outs = outs if outs is not None else [p.empty(work=True) for p in self.problems]
        zp = (c_void_p * m)(*[p._w(Z).value for p, Z in zip(self.problems, Zs)])
        hp = (c_void_p * m)(*[p._w(H).value for p, H in zip(self.problems, outs)])
        sg = (c_double * m)(*([0.0] * m if sigma is None else [float(x) for x in sigma]))
        kap = (c_double * m)() if kappa else None
        self._check(lib().gpe_batch_hvp(self.b, zp, hp, int(bool(riemannian)), sg, kap))
        return outs, (list(kap) if kappa else None)

    def newton_solve(self, Xs, check=True, **opts):
        """Lock-step gpe_newton_solve of every problem; returns (Xs, [stats dicts])."""
        m = len(self.problems)
        o = default_opts(**opts)
        xp = (c_void_p * m)(*[p._m(X).value for p, X in zip(self.problems, Xs)])
        stats = (gpe_solve_stats * m)()
        st = lib().gpe_batch_newton_solve(self.b, xp, ctypes.byref(o), stats)
        if st != 0 and (check or st != 5):
            self._check(st)
        return Xs, [s.as_dict() for s in stats]

    def schedule(self):
        """(chosen batched x-pass variant, measured microseconds per variant)."""
        v = c_int()
        us = (ctypes.c_float * 3)()
        self._check(lib().gpe_batch_schedule(self.b, ctypes.byref(v), us, 3))
        return v.value, list(us)
