"""CPU checks of the C ABI boundary: the library loads and exports every
function that include/idq.h declares, and the ctypes structs match the header."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "idq.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[a-z_ ]+\**\s*\**\s*(idq_\w+)\s*\(", src, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_api():
    names = declared_functions()
    for must in ["idq_solve", "idq_grad_reg", "idq_apply_A", "idq_apply_AT", "idq_backward",
                 "idq_ws_forward", "idq_ws_train_step"]:
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_2605_19705_amd import _lib
    L = _lib.lib()
    for name in declared_functions():
        assert hasattr(L, name), name
    assert set(declared_functions()) == set(_lib.EXPORTED)


def test_version_and_defaults_without_gpu():
    from paper_2605_19705_amd import _lib
    L = _lib.lib()
    assert L.idq_version() >= 10000
    o = _lib.SolveOpts()
    L.idq_solve_opts_default(C.byref(o))
    assert o.beta == 0.5 and o.lambda_ == 1.0 and o.tol == 1e-4 and o.conv_prec == _lib.IDQ_F32
    assert o.switch_tol == 2e-3 and o.switch_patience == 5 and o.refine_prec == _lib.IDQ_F32
    assert o.power_iters == 30 and o.init == _lib.IDQ_INIT_Y


STRUCTS = {"NetDesc": "idq_net_desc", "OpDesc": "idq_op_desc", "SolveOpts": "idq_solve_opts",
           "SolveInfo": "idq_solve_info", "BwdOpts": "idq_bwd_opts", "BwdInfo": "idq_bwd_info",
           "TrainOpts": "idq_train_opts"}


def test_struct_layouts_match_the_header(tmp_path):
    """Compile the header with gcc and compare sizeof/offsetof with ctypes."""
    import subprocess
    from paper_2605_19705_amd import _lib
    lines = ['#include <stdio.h>', '#include <stddef.h>', f'#include "{HEADER}"', "int main(void){"]
    for py, cname in STRUCTS.items():
        lines.append(f'printf("{py} %zu\\n", sizeof({cname}));')
        for fname, _ in getattr(_lib, py)._fields_:
            cf = "lambda" if fname == "lambda_" else fname
            lines.append(f'printf("{py}.{fname} %zu\\n", offsetof({cname}, {cf}));')
    lines.append("return 0;}")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", str(src), "-o", str(exe)], check=True)
    got = dict(l.split() for l in subprocess.run([str(exe)], capture_output=True, text=True,
                                                  check=True).stdout.splitlines())
    for py in STRUCTS:
        T = getattr(_lib, py)
        assert int(got[py]) == C.sizeof(T), py
        for fname, _ in T._fields_:
            assert int(got[f"{py}.{fname}"]) == getattr(T, fname).offset, (py, fname)


def test_missing_library_fails_loudly():
    """Without libidq.so the package raises instead of computing anything on the
    CPU: constructing a solver context or a warm-start network is an error."""
    import subprocess
    import sys
    code = "\n".join([
        "import numpy as np",
        "import paper_2605_19705_amd as P",
        "P._lib.LIB_PATH = '/nonexistent/libidq.so'",
        "layers = [(np.zeros((3, 3, 3, 3)), np.zeros(3))]",
        "for make in (lambda: P.IDQ(layers, op_kind='identity'), lambda: P.WarmStart(layers)):",
        "    try:",
        "        make()",
        "    except ImportError as e:",
        "        assert 'libidq.so is missing' in str(e), e",
        "        print('raised')",
        "    else:",
        "        raise SystemExit('no error')",
    ])
    r = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True,
                       timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
    assert r.stdout.split() == ["raised", "raised"], r.stdout
