"""The C ABI library loads and exports every function include/pr.h declares
(no device calls: runs without a GPU)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "pr.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(pr_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_the_four_method_calls():
    names = _declared()
    for n in ("pr_solve", "pr_prox", "pr_dual_bound", "pr_solve_batch"):
        assert n in names


def test_library_exports_every_declared_symbol():
    import paper_2603_01306_amd as pr
    lib = pr.load()
    for name in _declared():
        assert hasattr(lib, name), name
        getattr(lib, name)
    assert set(pr.EXPORTS) <= set(_declared())


def test_strerror_and_defaults_without_device():
    import paper_2603_01306_amd as pr
    lib = pr.load()
    assert lib.pr_strerror(0) == b"ok"
    assert lib.pr_strerror(-2) == b"J0 and J1 overlap"
    o = pr.default_opts()
    assert o.rel_gap_tol == 1e-6 and abs(o.eta - 20.085536923187668) < 1e-12 and o.max_iter > 0


def test_struct_layouts_match_header(tmp_path):
    """sizeof and every field offset of the header's structs, as a C compiler
    lays them out, equal the ctypes mirrors of the binding."""
    import subprocess
    import paper_2603_01306_amd._binding as b
    structs = {"pr_problem": b.PrProblem, "pr_node": b.PrNode, "pr_opts": b.PrOpts, "pr_result": b.PrResult,
               "pr_bnb_opts": b.PrBnbOpts, "pr_bnb_result": b.PrBnbResult, "pr_lasso": b.PrLasso}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "pr.h"', "int main(void) {"]
    for cname, cls in structs.items():
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in cls._fields_:
            lines.append(f'  printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines.append("  return 0;\n}")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    got = {}
    for line in subprocess.check_output([str(exe)]).decode().splitlines():
        a, f, v = line.split()
        got[(a, f)] = int(v)
    for cname, cls in structs.items():
        assert got[(cname, "size")] == ctypes.sizeof(cls), cname
        for fname, _ in cls._fields_:
            assert got[(cname, fname)] == getattr(cls, fname).offset, (cname, fname)
