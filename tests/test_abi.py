"""CPU checks of the C ABI: libgl.so loads, exports every function include/gl.h
declares, the Python structs match the C layout, and argument validation
(pure host code, no GPU call) returns the documented error codes."""
import ctypes as C
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gl.h")
LIB = os.path.join(ROOT, "paper_1004_5128_amd", "libgl.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gl_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_1004_5128_amd import build
        build.build()
    return C.CDLL(LIB)


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("gl_init", "gl_step_n", "gl_adjoint", "gl_free", "gl_last_error"):
        assert required in names


def test_library_exports_every_declared_symbol(lib):
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True,
                         check=True).stdout
    exported = set(re.findall(r" T (gl_\w+)", out))
    missing = [n for n in declared_functions() if n not in exported]
    assert not missing, missing
    for n in declared_functions():
        getattr(lib, n)


def test_python_binding_names_match_header():
    from paper_1004_5128_amd import gl
    assert sorted(gl.EXPORTS) == declared_functions()
    for n in declared_functions():
        assert callable(getattr(gl, n))


def test_struct_layout_matches_c(tmp_path):
    probe = tmp_path / "probe.c"
    probe.write_text("""
#include <stdio.h>
#include <stddef.h>
#include "gl.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu %zu\\n", sizeof(gl_problem), offsetof(gl_problem, nz),
         offsetof(gl_problem, dx),
         offsetof(gl_problem, rxn_rate), sizeof(gl_options), offsetof(gl_options, stream));
  printf("%zu %zu %zu\\n", offsetof(gl_options, short_L), offsetof(gl_options, max_steps),
         offsetof(gl_options, ckpt_every));
  return 0;
}
""")
    exe = tmp_path / "probe"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(probe), "-o", str(exe)],
                   check=True)
    vals = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True,
                                           check=True).stdout.split()]
    from paper_1004_5128_amd.gl import gl_options, gl_problem
    assert vals == [C.sizeof(gl_problem), gl_problem.nz.offset, gl_problem.dx.offset,
                    gl_problem.rxn_rate.offset,
                    C.sizeof(gl_options), gl_options.stream.offset, gl_options.short_L.offset,
                    gl_options.max_steps.offset, gl_options.ckpt_every.offset]


def _init(lib, prob_kw, opt_kw, nprob=1):
    from paper_1004_5128_amd.gl import gl_options, gl_problem
    base = dict(ndim=2, nx=8, ny=8, nz=1, rxn=0, dx=1 / 9, dt=1e-4, gamma=0.8, alpha=1.0, rxn_rate=0.0)
    base.update(prob_kw)
    probs = (gl_problem * max(nprob, 1))(*[gl_problem(**base)] * max(nprob, 1))
    o = dict(mem_mode=0, adapt_rule=0, short_L=0, adapt_a=2, sum_path=0, block_B=0,
             check_finite=0, max_steps=10, ckpt_every=0, stream=None)
    o.update(opt_kw)
    opts = gl_options(**o)
    ctx = C.c_void_p()
    lib.gl_init.restype = C.c_int32
    lib.gl_last_error.restype = C.c_char_p
    lib.gl_last_error.argtypes = [C.c_void_p]
    dummy = C.c_void_p(0x1000)   # never dereferenced: validation fails first
    st = lib.gl_init(probs, nprob, C.byref(opts), dummy, C.byref(ctx))
    return st, lib.gl_last_error(None).decode(), ctx


@pytest.mark.parametrize("prob_kw,opt_kw,code", [
    ({"ndim": 4}, {}, -1),
    ({"ndim": 0}, {}, -1),
    ({"nx": 0}, {}, -1),
    ({"ndim": 3, "nz": 0}, {}, -1),
    ({"ndim": 3, "nx": 1024, "ny": 1024, "nz": 257}, {}, -1),   # more than 2^28 points
    ({"gamma": 0.0}, {}, -1),
    ({"gamma": 2.01}, {}, -1),
    ({"alpha": -1.0}, {}, -1),
    ({"dt": 0.0}, {}, -1),
    ({"rxn": 7}, {}, -1),
    ({}, {"mem_mode": 5}, -1),
    ({}, {"mem_mode": 2, "adapt_a": 1}, -1),
    ({}, {"mem_mode": 2, "adapt_rule": 9}, -1),
    ({}, {"mem_mode": 1, "short_L": -1}, -1),
    ({}, {"max_steps": 0}, -1),
    ({}, {"sum_path": 4}, -1),
    ({"dt": 1e-2}, {}, -2),       # r = 0.01^0.8 * 81 = 2.04 > 2^0.8 / 8
    ({"ndim": 3, "nz": 8, "dt": 4.8e-4}, {}, -2),   # r = 0.179: under 2^0.8 / 8, over 2^0.8 / 12
    ({"gamma": 1.5, "dt": 0.03}, {}, -2),           # r = 0.42 > 2^1.5 / 8
])
def test_validation_errors(lib, prob_kw, opt_kw, code):
    st, msg, ctx = _init(lib, prob_kw, opt_kw)
    assert st == code, msg
    assert msg and ctx.value is None


def test_autotune_rejects_null_context(lib):
    lib.gl_autotune.restype = C.c_int32
    lib.gl_autotune.argtypes = [C.c_void_p, C.c_int32, C.c_void_p]
    assert lib.gl_autotune(None, 0, None) == -1


def test_nprob_zero_and_free_null(lib):
    st, msg, _ = _init(lib, {}, {}, nprob=0)
    assert st == -1 and "nprob" in msg
    lib.gl_free(None)   # no-op
    lib.gl_steps_done.restype = C.c_int64
    lib.gl_steps_done.argtypes = [C.c_void_p]
    assert lib.gl_steps_done(None) == -1
