"""The C-ABI library loads and exports every entry point include/fsi.h
declares (no device calls), and the binding declares the same set."""
import ctypes
import os
import re
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fsi.h")
LIB = os.path.join(ROOT, "paper_1801_05648_amd", "libfsi.so")


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fsi_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        import __graft_entry__
        __graft_entry__.build()
    return ctypes.CDLL(LIB)


def test_header_declares_the_documented_calls():
    names = declared()
    for n in ("fsi_create", "fsi_destroy", "fsi_setup_blocks", "fsi_build_precond", "fsi_solve",
              "fsi_spmv", "fsi_apply_precond", "fsi_vcycle", "fsi_set_hierarchy", "fsi_last_error"):
        assert n in names


def test_every_declared_symbol_is_exported(lib):
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True, check=True).stdout
    exported = set(re.findall(r"\sT\s(fsi_\w+)", out))
    missing = [n for n in declared() if n not in exported]
    assert not missing, missing
    for n in declared():
        getattr(lib, n)  # resolvable through the dynamic loader


def test_binding_declares_every_header_symbol():
    from paper_1801_05648_amd import fsi
    assert sorted(fsi.exported_symbols()) == declared()


def test_default_options_without_a_device(lib):
    from paper_1801_05648_amd import fsi
    o = fsi.CSolveOpts()
    lib.fsi_default_solve_opts(ctypes.byref(o))
    assert (o.tol, o.restart, o.maxit, o.timing) == (1e-8, 50, 2000, 0)
    p = fsi.CPrecondOpts()
    lib.fsi_default_precond_opts(ctypes.byref(p))
    assert (p.precision, p.max_coarse, p.max_levels, p.strength0) == (0, 500, 10, 0.08)
    # the pressure Schur approximation SIMPLE, the fluid inverse the Uzawa-like step alone
    assert (p.schur, p.fluid_inner, p.fluid_inner_pc, p.poly_ratio) == (0, 0, 0, 8.0)
    assert fsi.SCHUR["simple"] == 0 and fsi.INNER_PC == {"uzawa": 0, "triangular": 1}


def test_null_context_arguments_are_rejected(lib):
    """Argument checks that need no device: NULL context -> FSI_ERR_ARG."""
    from paper_1801_05648_amd import fsi
    L = fsi.load()
    assert L.fsi_create(None, 0, None) == -1
    assert L.fsi_build_precond(None, None) == -1
    assert L.fsi_solve(None, None, None, None, None) == -1
    assert L.fsi_spmv(None, None, None) == -1
    assert L.fsi_fe_setup(None, None) == -1
    assert L.fsi_fe_residual(None, None, None) == -1
    assert L.fsi_fe_jacobian(None, None, 0) == -1
    assert L.fsi_newton(None, None, None, None) == -1
    assert L.fsi_fe_advance(None, None) == -1
    assert L.fsi_time_step(None, None, None) == -1
    assert L.fsi_fe_get_fields(None, None, None, None) == -1
    assert L.fsi_destroy(None) == 0


def test_default_newton_options_follow_section_6(lib):
    """The quasi-Newton defaults: reassemble when the last step cut the
    max-norm residual by less than ten, stop at a 1e-6 reduction, GMRES to a
    reduction of 1e3 per step."""
    from paper_1801_05648_amd import fsi
    o = fsi.CNewtonOpts()
    lib.fsi_default_newton_opts(ctypes.byref(o))
    assert (o.rtol, o.reassemble_ratio, o.lin_tol) == (1e-6, 0.1, 1e-3)
    assert (o.max_steps, o.precond, o.restart, o.maxit) == (25, fsi.NEWTON_PC["rebuild"], 50, 2000)


STRUCTS = [("fsi_csr", "CCsr"), ("fsi_layout", "CLayout"), ("fsi_precond_opts", "CPrecondOpts"),
           ("fsi_solve_opts", "CSolveOpts"), ("fsi_solve_info", "CSolveInfo"),
           ("fsi_mlp_train_opts", "CMlpTrainOpts"), ("fsi_mlp_train_info", "CMlpTrainInfo"),
           ("fsi_fe_mesh", "CFeMesh"), ("fsi_newton_opts", "CNewtonOpts"), ("fsi_newton_info", "CNewtonInfo")]


def test_ctypes_structs_match_the_header_layout(tmp_path):
    """Size and every field offset of the binding's structs equal what a C
    compiler makes of the header."""
    from paper_1801_05648_amd import fsi
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "fsi.h"', 'int main(void) {']
    for cname, pname in STRUCTS:
        lines.append(f'  printf("{pname} size %zu\\n", sizeof({cname}));')
        for f, _ in getattr(fsi, pname)._fields_:
            lines.append(f'  printf("{pname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines += ['  return 0;', '}']
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l.strip()}
    for _, pname in STRUCTS:
        cls = getattr(fsi, pname)
        assert got[(pname, "size")] == ctypes.sizeof(cls), pname
        for f, _ in cls._fields_:
            assert got[(pname, f)] == getattr(cls, f).offset, (pname, f)


def test_header_compiles_as_c99(tmp_path):
    src = tmp_path / "t.c"
    src.write_text('#include "fsi.h"\nint main(void) { fsi_solve_opts o; fsi_default_solve_opts(&o); return 0; }\n')
    subprocess.run(["gcc", "-std=c99", "-Wall", "-Werror", "-fsyntax-only", "-I", os.path.join(ROOT, "include"),
                    str(src)], check=True)


def test_bench_refuses_more_than_one_gpu():
    """The benchmark runs on one GPU; asked for more it exits with a message
    (before touching a device)."""
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
