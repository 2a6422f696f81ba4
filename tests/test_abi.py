"""CPU checks of the C ABI: the library loads, exports every entry point that
include/gpe.h declares, and the ctypes structures match the C layout."""
import ctypes
import os
import re
import subprocess

import pytest

from paper_1907_01194_amd import binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gpe.h")


def header_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gpe_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = header_functions()
    for required in ("gpe_create", "gpe_destroy", "gpe_energy", "gpe_grad", "gpe_set_point", "gpe_hvp",
                     "gpe_retract", "gpe_newton_solve", "gpe_last_error"):
        assert required in names


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(binding.LIB_PATH):
        pytest.fail("libgpe.so not built: run `python -m paper_1907_01194_amd.build`")
    return binding.lib()


def test_library_exports_every_declared_symbol(lib):
    for name in header_functions():
        assert hasattr(lib, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", binding.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(l.split()[-1] for l in out.splitlines() if l.strip())
    assert set(header_functions()) <= exported


def test_binding_covers_header(lib):
    assert set(header_functions()) == set(binding.SIGNATURES)


def test_default_options_are_the_papers(lib):
    o = binding.default_opts()
    assert o.tol == 1e-6 and o.maxit == 10000 and o.retraction == 1
    assert (o.eta1, o.eta2, o.gamma0, o.gamma1, o.gamma2, o.sigma_hat0) == (0.01, 0.9, 0.2, 1.0, 10.0, 1.0)
    assert o.rgbb_tol == 1e-2 and o.rgbb_maxit == 2000
    assert lib.gpe_version().startswith(b"gpe")


def test_struct_layout_matches_c(tmp_path):
    """Compile a C program against the header and compare sizeof/offsetof with ctypes."""
    src = tmp_path / "layout.c"
    fields = {"gpe_problem": binding.gpe_problem, "gpe_solve_opts": binding.gpe_solve_opts,
              "gpe_solve_stats": binding.gpe_solve_stats}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "gpe.h"', "int main(void){"]
    for sname, cls in fields.items():
        lines.append('printf("%s %%zu\\n", sizeof(%s));' % (sname, sname))
        for f, _ in cls._fields_:
            lines.append('printf("%s.%s %%zu\\n", offsetof(%s, %s));' % (sname, f, sname, f))
    lines.append("return 0;}")
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = dict(l.split() for l in subprocess.run([str(exe)], capture_output=True, text=True).stdout.splitlines())
    for sname, cls in fields.items():
        assert int(got[sname]) == ctypes.sizeof(cls), sname
        for f, _ in cls._fields_:
            assert int(got[sname + "." + f]) == getattr(cls, f).offset, (sname, f)


def _bad_problem(**kw):
    pr = binding.gpe_problem()
    pr.F, pr.dim = 2, 2
    for a in range(3):
        pr.n[a], pr.lo[a], pr.hi[a] = (16, -4.0, 4.0) if a < 2 else (1, 0.0, 1.0)
    pr.beta[0], pr.beta[1], pr.beta[2] = 100.0, 1.0, -1.0
    pr.M = 0.3
    for k, v in kw.items():
        if k in ("n", "lo", "hi"):
            for a, x in enumerate(v):
                getattr(pr, k)[a] = x
        else:
            setattr(pr, k, v)
    return pr


@pytest.mark.parametrize("what,kw", [
    ("|M| = F", dict(M=2.0)), ("|M| > F", dict(M=3.5)), ("M < 0", dict(M=-0.3)),
    ("F = 0", dict(F=0)), ("F = 4", dict(F=4)), ("dim = 0", dict(dim=0)), ("dim = 4", dict(dim=4)),
    ("odd n", dict(n=(15, 16, 1))), ("n = 36 (2^2 3^2)", dict(n=(36, 16, 1))), ("n = 10", dict(n=(16, 10, 1))),
    ("n = 2", dict(n=(2, 16, 1))), ("n = 1024", dict(n=(1024, 16, 1))), ("empty box", dict(hi=(-4.0, 4.0, 1.0))),
])
def test_create_rejects_invalid_problems(lib, what, kw):
    """gpe_create validates the problem before touching the device (Sec. 2
    constraint |M| < F, Sec. 3 even n; the library's size list), so these run
    without a GPU: GPE_EINVAL, NULL handle, a message naming the fault."""
    pr = _bad_problem(**kw)
    V = (ctypes.c_double * (16 * 16 * 36))()
    h = ctypes.c_void_p(12345)
    st = lib.gpe_create(ctypes.byref(pr), ctypes.cast(V, ctypes.c_void_p), binding.FP64, None, ctypes.byref(h))
    assert st == 1, what
    assert h.value is None
    assert lib.gpe_last_error(None), what


def test_create_rejects_null_arguments(lib):
    pr = _bad_problem()
    h = ctypes.c_void_p()
    assert lib.gpe_create(ctypes.byref(pr), None, binding.FP64, None, ctypes.byref(h)) == 1
    assert b"NULL" in lib.gpe_last_error(None)
    V = (ctypes.c_double * 256)()
    assert lib.gpe_create(None, ctypes.cast(V, ctypes.c_void_p), binding.FP64, None, ctypes.byref(h)) == 1
    assert lib.gpe_create(ctypes.byref(pr), ctypes.cast(V, ctypes.c_void_p), 7, None, ctypes.byref(h)) == 1
    assert lib.gpe_create(ctypes.byref(pr), ctypes.cast(V, ctypes.c_void_p), binding.FP64, None, None) == 1


def test_calls_reject_null_handles(lib):
    """Entry points given a NULL handle or NULL buffers fail with GPE_EINVAL
    (no device access happens)."""
    E = ctypes.c_double()
    assert lib.gpe_energy(None, None, ctypes.byref(E)) == 1
    assert lib.gpe_set_schedule(None, 0) == 1
    n = ctypes.c_int()
    assert lib.gpe_schedule_count(None, ctypes.byref(n)) == 1
    assert lib.gpe_destroy(None) == 0
