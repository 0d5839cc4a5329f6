"""The C-ABI library loads without a GPU, exports every declared symbol, and the
Python structures match the C layout (checked by compiling the header)."""
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "qcdw.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(qcdw_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_what_the_binding_lists():
    import paper_2411_08461_amd as q

    assert _declared_functions() == sorted(q.EXPORTED)


def test_library_exports_every_declared_symbol():
    import paper_2411_08461_amd as q

    if not os.path.exists(q.LIB_PATH):
        pytest.fail("libqcdw.so is not built; run __graft_entry__.build()")
    lib = q.load_library()
    missing = [n for n in _declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    out = subprocess.run(["nm", "-D", "--defined-only", q.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\bT (qcdw_\w+)", out))
    assert set(_declared_functions()) <= exported


def test_struct_layout_matches_header(tmp_path):
    import ctypes

    import paper_2411_08461_amd as q

    src = tmp_path / "layout.c"
    src.write_text(
        '#include <stdio.h>\n#include <stddef.h>\n#include "qcdw.h"\n'
        "int main(void){\n"
        'printf("%zu %zu %zu\\n", sizeof(qcdw_lattice), sizeof(qcdw_solver_params), sizeof(qcdw_solve_info));\n'
        'printf("%zu %zu %zu %zu\\n", offsetof(qcdw_solver_params, delta), offsetof(qcdw_solver_params, fault_inject),'
        " offsetof(qcdw_solve_info, true_res), offsetof(qcdw_solve_info, res_hist));\n"
        'printf("%zu %zu %zu %zu\\n", sizeof(qcdw_mg_params), offsetof(qcdw_mg_params, seed),'
        " offsetof(qcdw_mg_params, coarse_tol), offsetof(qcdw_mg_params, smooth_iters));\n"
        "return 0;}\n"
    )
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    lines = subprocess.check_output([str(exe)], text=True).split("\n")
    sizes = [int(v) for v in lines[0].split()]
    offs = [int(v) for v in lines[1].split()]
    assert sizes == [ctypes.sizeof(q.qcdw_lattice), ctypes.sizeof(q.qcdw_solver_params),
                     ctypes.sizeof(q.qcdw_solve_info)]
    assert offs == [q.qcdw_solver_params.delta.offset, q.qcdw_solver_params.fault_inject.offset,
                    q.qcdw_solve_info.true_res.offset, q.qcdw_solve_info.res_hist.offset]
    mg = [int(v) for v in lines[2].split()]
    assert mg == [ctypes.sizeof(q.qcdw_mg_params), q.qcdw_mg_params.seed.offset, q.qcdw_mg_params.coarse_tol.offset,
                  q.qcdw_mg_params.smooth_iters.offset]


def test_calls_without_gpu_fail_loudly():
    import torch

    import paper_2411_08461_amd as q

    if torch.cuda.is_available():
        pytest.skip("GPU present")
    with pytest.raises(RuntimeError):
        q.Context(0)


def test_product_package_never_touches_the_oracle():
    pkg = os.path.join(ROOT, "paper_2411_08461_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                text = open(os.path.join(dirpath, f)).read()
                for bad in ("import oracle", "from oracle", "liboracle", "orc_"):
                    assert bad not in text, (f, bad)


def test_binding_orders_object_destruction():
    """Children (nets, batches, operators) are closed before their context."""
    import paper_2411_08461_amd as q

    assert q.Net._rank < q.Batch._rank < q.Operator._rank
