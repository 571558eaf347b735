"""C-ABI checks that need no GPU: the library builds, loads and exports every
function include/lpdense.h declares; host-side validation rejects bad
arguments before any device call."""
import ctypes
import os
import re

import pytest

from paper_1804_04737_amd import lpdense

HEADER = os.path.join(os.path.dirname(os.path.dirname(__file__)), "include", "lpdense.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^[A-Za-z_][\w \*]*?\b(l[a-z_]+)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_header_declares_expected_entry_points():
    names = declared_functions()
    for want in ("lp_solve_dense", "lp_solve_dense_ex", "lpd_workspace_bytes",
                 "lpd_error_string", "lpd_status_string", "lpd_version"):
        assert want in names
    assert set(names) == set(lpdense.EXPORTS)


def test_library_exports_every_declared_symbol():
    lib = lpdense.load()
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_strings_and_version():
    lib = lpdense.load()
    assert lib.lpd_version() >= 100
    assert lpdense.error_string(0) == "success"
    assert lpdense.error_string(-2) == "null pointer"
    assert lpdense.error_string(12345) == "unknown"
    for s, name in enumerate(lpdense.STATUS_NAMES):
        assert lib.lpd_status_string(s).decode() == name
    assert lib.lpd_status_string(99).decode() == "unknown"


def test_host_validation_without_device():
    """Invalid arguments are rejected on the host, before any HIP call."""
    lib = lpdense.load()
    dummy = ctypes.c_void_p(0x1000)
    assert lib.lp_solve_dense(0, 3, dummy, dummy, dummy, dummy, dummy, dummy, None) == -1
    assert lib.lp_solve_dense(3, -1, dummy, dummy, dummy, dummy, dummy, dummy, None) == -1
    assert lib.lp_solve_dense(3, 3, None, dummy, dummy, dummy, dummy, dummy, None) == -2
    assert lib.lp_solve_dense(3, 3, dummy, dummy, dummy, None, dummy, dummy, None) == -2
    assert lib.lp_solve_dense(1 << 40, 3, dummy, dummy, dummy, dummy, dummy, dummy, None) == -3
    assert lib.lp_solve_dense_ex(None, None, None, None) == -2
    p = lpdense.Problem(2, 2, 0x1000, 0x1000, 0x1000)
    o = lpdense.Outputs(0x1000, 0x1000, 0x1000, None, None, None, 5, None, None)
    assert lib.lp_solve_dense_ex(ctypes.byref(p), None, ctypes.byref(o), None) == -2  # trace_cap > 0, no trace
    o.trace_cap = -1
    assert lib.lp_solve_dense_ex(ctypes.byref(p), None, ctypes.byref(o), None) == -1
    # Schedules 0..5 (the last: two pivots per sweep of the condensed tableau);
    # anything else is an argument error, found before any device call.
    o.trace_cap = 0
    assert lpdense.SCHED_GRID_CONDENSED_PAIRED == 5
    for bad in (-1, 6):
        opts = lpdense.Options(0.0, 0.0, -1, bad, 0)
        assert lib.lp_solve_dense_ex(ctypes.byref(p), ctypes.byref(opts), ctypes.byref(o), None) == -1


def test_tableau_and_noalloc_host_validation_without_device():
    """lp_solve_tableau and lp_solve_dense_noalloc reject bad arguments on
    the host, before any HIP call (no GPU here)."""
    import numpy as np
    lib = lpdense.load()
    d = 0x1000
    o = lpdense.Outputs(d, d, d, None, None, None, 0, None, None, None, 0)
    basis = np.array([0, 1], dtype=np.int64)
    bp = basis.ctypes.data_as(ctypes.c_void_p)
    f = lib.lp_solve_tableau
    assert f(0, 3, ctypes.c_void_p(d), bp, None, ctypes.byref(o), None) == -1   # m < 1
    assert f(3, 2, ctypes.c_void_p(d), bp, None, ctypes.byref(o), None) == -1   # ncols < m
    assert f(2, 4, None, bp, None, ctypes.byref(o), None) == -2                  # no tableau
    assert f(2, 4, ctypes.c_void_p(d), None, None, ctypes.byref(o), None) == -2  # no basis
    for bad in ([0, 0], [0, 4], [-1, 1]):
        bb = np.array(bad, dtype=np.int64)
        assert f(2, 4, ctypes.c_void_p(d), bb.ctypes.data_as(ctypes.c_void_p), None, ctypes.byref(o), None) == -1
    oy = lpdense.Outputs(d, d, d, d, None, None, 0, None, None, None, 0)      # y is not an output here
    assert f(2, 4, ctypes.c_void_p(d), bp, None, ctypes.byref(oy), None) == -1
    assert lib.lp_solve_dense_noalloc(None, None, None, None) == -2
    p = lpdense.Problem(0, 2, d, d, d)
    assert lib.lp_solve_dense_noalloc(ctypes.byref(p), None, ctypes.byref(o), None) == -1


def test_batch_host_validation_without_device():
    lib = lpdense.load()
    import numpy as np
    d = ctypes.c_void_p(0x1000)
    one = np.array([3], dtype=np.int64)
    zero = np.array([0], dtype=np.int64)
    neg = np.array([-1], dtype=np.int64)
    p = lambda a: a.ctypes.data_as(ctypes.c_void_p)
    f = lib.lp_solve_batch
    assert f(0, p(one), p(one), d, p(zero), d, p(zero), d, p(zero), d, p(zero), d, d, None, None) == -1
    assert f(1, p(zero), p(one), d, p(zero), d, p(zero), d, p(zero), d, p(zero), d, d, None, None) == -1
    assert f(1, p(one), p(one), None, p(zero), d, p(zero), d, p(zero), d, p(zero), d, d, None, None) == -2
    assert f(1, p(one), p(one), d, p(neg), d, p(zero), d, p(zero), d, p(zero), d, d, None, None) == -1


def test_server_host_validation_without_device():
    lib = lpdense.load()
    d = ctypes.c_void_p(0x1000)
    assert lib.lpd_server_submit(None, 3, 3, d, d, d, d) == -8
    assert lib.lpd_server_poll(None, None, 0) == -1
    assert lib.lpd_server_get_stats(None, None) == -2
    lib.lpd_server_destroy(None)


def _c_layout(structs):
    """sizeof and field offsets of header structs, from a C compiler."""
    import shutil
    import subprocess
    import tempfile
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "lpdense.h"', "int main(void) {"]
    for cname, fields in structs:
        lines.append(f'printf("%zu\\n", sizeof({cname}));')
        for f in fields:
            lines.append(f'printf("%zu\\n", offsetof({cname}, {f}));')
    lines.append("return 0; }")
    with tempfile.TemporaryDirectory() as d:
        src, exe = os.path.join(d, "l.c"), os.path.join(d, "l")
        open(src, "w").write("\n".join(lines))
        r = subprocess.run([cc, "-D__HIP_PLATFORM_AMD__", f"-I{os.path.dirname(HEADER)}",
                            "-I/opt/rocm/include", src, "-o", exe], capture_output=True, text=True)
        if r.returncode != 0:
            pytest.skip("header does not compile with the host C compiler: " + r.stderr[-300:])
        return [int(v) for v in subprocess.run([exe], capture_output=True, text=True).stdout.split()]


def test_python_struct_mirrors_match_the_header():
    mirrors = [("lpd_problem", lpdense.Problem), ("lpd_options", lpdense.Options),
               ("lpd_outputs", lpdense.Outputs), ("lpd_batch_options", lpdense.BatchOptions),
               ("lpd_server_options", lpdense.ServerOptions), ("lpd_completion", lpdense.Completion),
               ("lpd_server_stats", lpdense.ServerStats)]
    structs = [(cname, [f for f, _ in py._fields_]) for cname, py in mirrors]
    got = _c_layout(structs)
    want = []
    for _, py in mirrors:
        want.append(ctypes.sizeof(py))
        want += [getattr(py, f).offset for f, _ in py._fields_]
    assert got == want


def test_schedule_constants_match_header():
    """The binding's schedule numbers are the header's enum values."""
    with open(HEADER) as f:
        text = re.sub(r"/\*.*?\*/", "", f.read(), flags=re.S)
    enum = dict((k, int(v)) for k, v in re.findall(r"\b(LPD_SCHED_\w+)\s*=\s*(\d+)", text))
    assert enum == {
        "LPD_SCHED_AUTO": lpdense.SCHED_AUTO,
        "LPD_SCHED_WORKGROUP": lpdense.SCHED_WORKGROUP,
        "LPD_SCHED_GRID": lpdense.SCHED_GRID,
        "LPD_SCHED_GRID_CONDENSED": lpdense.SCHED_GRID_CONDENSED,
        "LPD_SCHED_GRID_PAIRED": lpdense.SCHED_GRID_PAIRED,
        "LPD_SCHED_GRID_CONDENSED_PAIRED": lpdense.SCHED_GRID_CONDENSED_PAIRED,
    }


@pytest.mark.parametrize("lang,std", [("c", "c99"), ("c++", "c++11")])
def test_header_compiles_standalone(lang, std):
    """The public header builds on its own as C99 and as C++11 with warnings as errors,
    and lpd_result names the outputs struct."""
    import shutil
    import subprocess
    import tempfile
    cc = shutil.which("gcc")
    if cc is None:
        pytest.skip("no C compiler")
    code = ('#include "lpdense.h"\n'
            "int main(void) { lpd_result r; lpd_outputs *o = &r; (void)o;\n"
            "  int (*f)(const lpd_problem*, const lpd_options*, const lpd_outputs*, hipStream_t)"
            " = lp_solve_dense_ex; (void)f; return 0; }\n")
    with tempfile.TemporaryDirectory() as d:
        src = os.path.join(d, "h.c")
        open(src, "w").write(code)
        r = subprocess.run([cc, "-x", lang, f"-std={std}", "-Wall", "-Wextra", "-Werror",
                            "-D__HIP_PLATFORM_AMD__", f"-I{os.path.dirname(HEADER)}",
                            "-I/opt/rocm/include", "-c", src, "-o", os.path.join(d, "h.o")],
                           capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-2000:]
