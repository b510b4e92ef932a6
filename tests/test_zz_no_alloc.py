"""The allocation-free solve (snmf_solve_noalloc) against snmf_solve, through the C ABI.

The allocation-free entry point runs the same kernels as snmf_solve, launched directly
instead of from a captured graph (graph replay equals direct launches bitwise), with its
scratch in the library's static device array.  Two calls in a row, the second on a
smaller problem (so stale contents of the shared array from the first call would show),
must return factors, monitor records and trace bitwise equal to snmf_solve's; a third
call solves a graph problem with its Laplacian.  Problems whose scratch exceeds the
array, and the split-BF16 form, are refused with a message.
"""
import numpy as np
import pytest

import oracle as O
from paper_2606_02887_amd import gen

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
DEV = "cuda"


@pytest.fixture(scope="module")
def S():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2606_02887_amd import snmf
    return snmf


def _same(S, A, W0, prm_kw, L=None):
    W1, H1, i1 = S.solve(A, W0, S.params(**prm_kw), L)
    W2, H2, i2 = S.solve_noalloc(A, W0, S.params(**prm_kw), L)
    assert torch.equal(W1, W2) and torch.equal(H1, H2)
    for k in ("status", "outer", "res_WH", "res_WWt", "sym_gap", "pg_norm", "objective",
              "inner_total", "ls_evals"):
        assert i1[k] == i2[k], k
    assert np.array_equal(i1["trace"][:, :5], i2["trace"][:, :5])
    return i2


def test_noalloc_equals_solve_on_consecutive_calls(S):
    p0 = gen.planted_dense(500, 10, 1000)                 # the config-0 workload
    A0 = torch.from_numpy(p0["A"]).to(DEV, torch.float32)
    i = _same(S, S.dense(A0), torch.from_numpy(p0["W0"]).to(DEV, torch.float32),
              dict(lam=O.default_lambda(p0["A"]), max_outer=30))
    assert i["status"] == 0 and i["outer"] == 30
    p1 = gen.planted_dense(300, 6, 77)                    # smaller, FP64
    A1 = torch.from_numpy(p1["A"]).to(DEV, torch.float64)
    _same(S, S.dense(A1), torch.from_numpy(p1["W0"]).to(DEV, torch.float64),
          dict(lam=O.default_lambda(p1["A"]), max_outer=12, prec=S.F64))
    g = gen.sbm_problem(n=1000, k=5, r=5, p_in=0.08, p_out=0.004, seed=23)
    Ag = S.csr_from_scipy(g["A"], torch.float32)
    Lg = S.csr_from_scipy(O.knn_laplacian(g["X"], g["knn"]), torch.float32)
    _same(S, Ag, torch.from_numpy(g["W0"]).to(DEV, torch.float32),
          dict(lam=O.default_lambda(g["A"]), gamma=0.2, max_outer=10), Lg)


def test_noalloc_refuses_what_does_not_fit(S):
    n = 4096
    A = torch.rand((n, n), dtype=torch.float32, device=DEV)
    A = (A + A.T).contiguous()
    W0 = torch.rand((n, 64), dtype=torch.float32, device=DEV)
    with pytest.raises(S.SnmfError) as e:                 # 6 n r doubles alone are 12 MiB; F64
        big = torch.rand((20000, 64), dtype=torch.float64, device=DEV)
        S.solve_noalloc(S.dense(torch.eye(20000, dtype=torch.float64, device=DEV)), big,
                        S.params(prec=S.F64, max_outer=1))
    assert e.value.name == "E_SHAPE" and "static array" in str(e.value)
    with pytest.raises(S.SnmfError) as e:
        S.solve_noalloc(S.dense(A), W0, S.params(prec=S.BF16X3, max_outer=1))
    assert e.value.name == "E_UNSUPPORTED"
