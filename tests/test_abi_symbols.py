"""CPU checks of the built C-ABI library: it loads, exports every function
include/crsht.h declares, and rejects invalid plan arguments before touching
a device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "crsht.h")
LIB = os.path.join(ROOT, "paper_2306_15511_amd", "libcrsht.so")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?(?:int|void|char)\s*\*?\s*(\w+)\s*\(", text, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libcrsht.so not built; run python -m paper_2306_15511_amd.build")
    return ctypes.CDLL(LIB)


def test_header_declares_the_boundary():
    names = _declared()
    for required in ("sht_synth", "sht_synth_adjoint", "sht_analysis", "cr_solve", "joint_cl_step",
                     "crsht_plan_create", "crsht_plan_destroy", "crsht_strerror", "cr_apply", "cr_rhs",
                     "cr_precond", "cr_lnpi"):
        assert required in names


def test_every_declared_symbol_is_exported(lib):
    for name in _declared():
        assert hasattr(lib, name), name


def test_binding_covers_every_symbol():
    src = open(os.path.join(ROOT, "paper_2306_15511_amd", "crsht.py")).read()
    for name in _declared():
        assert '"%s"' % name in src, name


def test_invalid_plan_arguments_rejected_without_device(lib):
    f = lib.crsht_plan_create
    f.argtypes = [ctypes.c_int] * 5 + [ctypes.POINTER(ctypes.c_void_p)]
    f.restype = ctypes.c_int
    h = ctypes.c_void_p()
    assert f(0, 10, -1, 1, 1, ctypes.byref(h)) == -1          # nside < 1
    assert f(4, -1, -1, 1, 1, ctypes.byref(h)) == -1          # lmax < 0
    assert f(4, 10, 11, 1, 1, ctypes.byref(h)) == -1          # mmax > lmax
    assert f(4, 10, -1, 1, 0, ctypes.byref(h)) == -1          # nrhs_max < 1
    assert f(4, 10, -1, 2, 1, ctypes.byref(h)) == -1          # ncomp 2
    assert f(4, 10, -1, 1, 1, None) == -1                     # NULL out
    assert h.value is None
    rc = f(4, 10, -1, 3, 1, ctypes.byref(h))                  # ncomp 3 (T, Q, U) passes the checks
    if rc == 0:
        lib.crsht_plan_destroy.argtypes = [ctypes.c_void_p]
        lib.crsht_plan_destroy(h)
    assert rc in (0, -3)                                      # -3: no HIP device here


def test_strerror(lib):
    lib.crsht_strerror.restype = ctypes.c_char_p
    lib.crsht_strerror.argtypes = [ctypes.c_int]
    assert lib.crsht_strerror(0) == b"success"
    assert b"invalid" in lib.crsht_strerror(-1)
    assert lib.crsht_strerror(12345) == b"unknown status"


def test_binding_struct_layouts_match_header(tmp_path):
    # every struct the binding passes through the boundary has the size and
    # field offsets the C compiler gives the header's declaration
    import shutil
    import subprocess
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    from paper_2306_15511_amd import crsht
    pairs = {"crsht_info": crsht._Info, "cr_problem": crsht._Problem, "cr_opts": crsht._Opts,
             "cr_stats": crsht._Stats, "cr_chain": crsht._Chain, "cr_draws": crsht._Draws,
             "cr_step_out": crsht._StepOut, "cr_gibbs_out": crsht._GibbsOut, "cr_bin_chain": crsht._BinChain,
             "cr_hmc_draws": crsht._HmcDraws, "cr_hmc_out": crsht._HmcOut}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "crsht.h"', "int main(void) {"]
    for cname, py in pairs.items():
        lines.append('  printf("%s %%zu\\n", sizeof(%s));' % (cname, cname))
        for fname, _ in py._fields_:
            lines.append('  printf("%s.%s %%zu\\n", offsetof(%s, %s));' % (cname, fname, cname, fname))
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = dict(l.split() for l in subprocess.run([str(exe)], check=True, capture_output=True,
                                                 text=True).stdout.splitlines())
    for cname, py in pairs.items():
        assert int(got[cname]) == ctypes.sizeof(py), cname
        for fname, _ in py._fields_:
            assert int(got["%s.%s" % (cname, fname)]) == getattr(py, fname).offset, (cname, fname)
