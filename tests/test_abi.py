"""Host-side checks of the C ABI (no GPU needed): exports, struct layout, argument errors."""
import ctypes
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "snmf.h")


@pytest.fixture(scope="module")
def S():
    from paper_2606_02887_amd import snmf
    return snmf


def _declared_functions():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:snmf_status|double|const char\*|int32_t|size_t)\s+(snmf_\w+)\s*\(",
                                 txt, re.M)))


def test_library_exports_every_declared_function(S):
    names = _declared_functions()
    assert len(names) >= 14
    lib = ctypes.CDLL(S.LIB_PATH)
    for nm in names:
        assert hasattr(lib, nm), nm
    assert set(S.EXPORTS) == set(names)


def test_struct_layout_matches_c(S, tmp_path):
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("gcc not available")
    src = tmp_path / "layout.c"
    checks = {
        "snmf_matrix": ["n", "dense", "ld", "rowptr", "val", "nnz", "U", "ell", "lam"],
        "snmf_params": ["gamma", "L", "eta", "beta_shrink", "max_ls", "check_every",
                        "target_res", "prec", "use_graph", "check_symmetry", "naive",
                        "tuning"],
        "snmf_batch_tuning": ["tiles_per_wg", "spmm_rows_per_wg", "reserved"],
        "snmf_info": ["inner_total", "ls_exhausted", "res_WH", "seconds_to_target", "normA2"],
        "snmf_mlp": ["hidden", "M1", "b1", "M2", "b2", "M1h", "M2h", "adam_m", "adam_v"],
    }
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "snmf.h"', 'int main(void){']
    for st, fields in checks.items():
        lines.append(f'printf("{st} %zu\\n", sizeof({st}));')
        for f in fields:
            lines.append(f'printf("{st}.{f} %zu\\n", offsetof({st}, {f}));')
    lines.append("return 0;}")
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.check_call([gcc, "-I", os.path.dirname(HEADER), str(src), "-o", str(exe)])
    out = dict(l.split() for l in subprocess.check_output([str(exe)]).decode().splitlines())
    py = {"snmf_matrix": S.Matrix, "snmf_params": S.Params, "snmf_info": S.Info,
          "snmf_mlp": S.MlpC, "snmf_batch_tuning": S.Tuning}
    for st, cls in py.items():
        assert int(out[st]) == ctypes.sizeof(cls)
        for f in checks[st]:
            pyf = "lambda_" if f == "lambda" else f
            assert int(out[f"{st}.{f}"]) == getattr(cls, pyf).offset, (st, f)


def test_abi_version_matches_the_binding(S):
    assert S.abi_version() == S.ABI_VERSION


def test_naive_and_nmf_arguments_are_rejected_before_any_device_work(S):
    A = S.Matrix(fmt=S.DENSE, n=10, dense=1, ld=10)  # never dereferenced
    p = S.params(naive=1, lam=0.5)
    st, h = _create(S, A, 3, p)
    assert st == 1 and not h.value                     # the naive variant needs lambda = 0
    info = S.Info()
    V = S.Matrix(fmt=S.LOWRANK, n=10, U=1, ell=2, lam=None)
    assert S._lib.snmf_nmf_solve(ctypes.byref(V), 8, 3, 1, 1, ctypes.byref(S.params(lam=0.0)),
                                 1, 1, ctypes.byref(info), None, None) != 0
    V = S.Matrix(fmt=S.DENSE, n=10, dense=1, ld=8)
    assert S._lib.snmf_nmf_solve(ctypes.byref(V), 8, 3, 1, 1, ctypes.byref(S.params(lam=0.3)),
                                 1, 1, ctypes.byref(info), None, None) == 1   # lambda != 0
    assert S._lib.snmf_nmf_solve(ctypes.byref(V), 9, 3, 1, 1, ctypes.byref(S.params(lam=0.0)),
                                 1, 1, ctypes.byref(info), None, None) == 2   # ld < n_cols


def test_bad_batch_tuning_is_rejected(S):
    p = S.params(tuning={"tiles_per_wg": [4, 0, 4, 4], "spmm_rows_per_wg": 16})
    A = (S.Matrix * 1)(S.Matrix(fmt=S.CSR, n=10, rowptr=1, col=1, val=1, nnz=4))
    r = (ctypes.c_int32 * 1)(3)
    h = ctypes.c_void_p()
    st = S._lib.snmf_batch_create(1, A, r, None, 1, ctypes.byref(p), None, ctypes.byref(h))
    assert st == 1 and not h.value and "tuning" in S._lib.snmf_last_error().decode()


def test_params_default(S):
    p = S.params()
    assert (p.eta, p.theta, p.phi, p.alpha_min, p.alpha_max) == (0.85, 1e-3, 1.7, 1e-10, 1e10)
    assert (p.beta_shrink, p.max_ls, p.inner_iters, p.prec) == (0.5, 20, 5, S.F32)
    assert p.project_update == 1 and p.accept_at_relaxed == 0 and p.validate == 1


def _create(S, A, r, p):
    h = ctypes.c_void_p()
    st = S._lib.snmf_plan_create(None if A is None else ctypes.byref(A), r,
                                 None if p is None else ctypes.byref(p), None, ctypes.byref(h))
    return st, h


@pytest.mark.parametrize("field,value", [("lambda_", -1.0), ("eta", 1.0), ("theta", 0.0),
                                         ("phi", 0.0), ("alpha_min", 2e10), ("beta_shrink", 1.0),
                                         ("max_ls", -1), ("inner_iters", 0), ("max_outer", 0),
                                         ("prec", 7)])
def test_bad_parameters_are_rejected_before_any_device_work(S, field, value):
    A = S.Matrix(fmt=S.DENSE, n=10, dense=1, ld=10)  # never dereferenced
    p = S.params()
    setattr(p, field, value)
    st, h = _create(S, A, 3, p)
    assert st == 1 and not h.value
    assert S._lib.snmf_last_error().decode()


def test_bad_shapes_and_combinations(S):
    p = S.params()
    assert _create(S, None, 3, p)[0] == 1
    assert _create(S, S.Matrix(fmt=S.DENSE, n=10, dense=1, ld=10), 3, None)[0] == 1
    assert _create(S, S.Matrix(fmt=S.DENSE, n=10, dense=1, ld=10), 0, p)[0] == 2
    assert _create(S, S.Matrix(fmt=S.DENSE, n=10, dense=1, ld=10), 11, p)[0] == 2
    assert _create(S, S.Matrix(fmt=S.DENSE, n=100, dense=1, ld=100), 65, p)[0] == 2
    assert _create(S, S.Matrix(fmt=S.DENSE, n=10, dense=1, ld=9), 3, p)[0] == 2
    assert _create(S, S.Matrix(fmt=S.DENSE, n=10, dense=None, ld=10), 3, p)[0] == 1
    assert _create(S, S.Matrix(fmt=S.LOWRANK, n=10, U=1, ell=200, lam=1), 3, p)[0] == 2
    pb = S.params(prec=S.BF16X3)
    assert _create(S, S.Matrix(fmt=S.CSR, n=10, rowptr=1, col=1, val=1, nnz=5), 3, pb)[0] == 8
    pr = S.params(accept_at_relaxed=1)
    assert _create(S, S.Matrix(fmt=S.DENSE, n=10, dense=1, ld=10), 3, pr)[0] == 8


def test_null_outputs_rejected(S):
    assert S._lib.snmf_rho(None, 3, None, None) == 1
    assert S._lib.snmf_split_bf16(None, 4, None, None, None) == 1
    assert S._lib.snmf_plan_solve(None, None, None, None, None, None, None) == 1
