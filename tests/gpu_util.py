"""Helpers of the GPU tests: move numpy fields to the device and back, and
compare fields both in norm and element by element."""
import numpy as np


def dev(a, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def host(t):
    return t.detach().cpu().numpy().astype(np.complex128)


def relnorm(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


def comp_maxerr(a, b):
    """Largest per-component max|a_l - b_l| / max|b_l| (component = leading
    axis); a component's scale is floored at 1e-3 of the field's largest
    magnitude so that (nearly) empty components do not divide by ~0."""
    a = np.asarray(a)
    b = np.asarray(b)
    big = max(float(np.max(np.abs(b))), 1e-300)
    worst = 0.0
    for l in range(b.shape[0]):
        scale = max(float(np.max(np.abs(b[l]))), 1e-3 * big)
        worst = max(worst, float(np.max(np.abs(a[l] - b[l]))) / scale)
    return worst


def assert_field(got, ref, tol, what=""):
    """Both the relative 2-norm and every component's relative max error within tol."""
    r = relnorm(got, ref)
    m = comp_maxerr(got, ref)
    assert r <= tol and m <= tol, "%s: relnorm %.3e, per-component max %.3e, tol %.1e" % (what, r, m, tol)
    return r, m
