"""ctypes binding of the HIP SNMPBB library (``libsnmf.so``, C ABI in include/snmf.h).

Argument marshalling only: every step of the solve runs in the library's kernels.
PyTorch provides device memory (tensors) and the current HIP stream.  Importing this
module loads the library and raises if it has not been built -- there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_double, c_int32, c_int64, c_void_p

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsnmf.so")

DENSE, CSR, LOWRANK = 0, 1, 2
F64, F32, BF16X3 = 0, 1, 2
TRACE_FIELDS = 10
TRACE_NAMES = ("res_WH", "res_WWt", "sym_gap", "pg_norm", "objective", "ticks", "ls_evals",
               "ls_exhausted", "alpha", "inner_total")
STATUS = {0: "OK", 1: "E_ARG", 2: "E_SHAPE", 3: "E_NOT_SYMMETRIC", 4: "E_NEGATIVE",
          5: "E_NONFINITE", 6: "E_OOM", 7: "E_DEVICE", 8: "E_UNSUPPORTED", 9: "E_BREAKDOWN"}


class SnmfError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"snmf {STATUS.get(status, status)}: {msg}")
        self.status = status
        self.name = STATUS.get(status, str(status))


class Matrix(ctypes.Structure):
    _fields_ = [("fmt", c_int32), ("reserved", c_int32), ("n", c_int64), ("dense", c_void_p),
                ("ld", c_int64), ("rowptr", c_void_p), ("col", c_void_p), ("val", c_void_p),
                ("nnz", c_int64), ("U", c_void_p), ("ell", c_int64), ("lam", c_void_p)]


class Tuning(ctypes.Structure):
    _fields_ = [("tiles_per_wg", c_int32 * 4), ("spmm_rows_per_wg", c_int32),
                ("reserved", c_int32 * 3)]


class Params(ctypes.Structure):
    _fields_ = [("lambda_", c_double), ("gamma", c_double), ("L", POINTER(Matrix)),
                ("eta", c_double), ("theta", c_double), ("phi", c_double),
                ("alpha_min", c_double), ("alpha_max", c_double), ("beta_shrink", c_double),
                ("max_ls", c_int32), ("inner_iters", c_int32), ("max_outer", c_int32),
                ("check_every", c_int32), ("target_res", c_double), ("prec", c_int32),
                ("accept_at_relaxed", c_int32), ("project_update", c_int32),
                ("validate", c_int32), ("use_graph", c_int32), ("check_symmetry", c_int32),
                ("naive", c_int32), ("fuse_inner", c_int32), ("tuning", POINTER(Tuning))]


class Info(ctypes.Structure):
    _fields_ = [("status", c_int32), ("outer", c_int32), ("converged_at", c_int32),
                ("reserved", c_int32), ("inner_total", c_int64), ("ls_evals", c_int64),
                ("ls_exhausted", c_int64), ("res_WH", c_double), ("res_WWt", c_double),
                ("sym_gap", c_double), ("pg_norm", c_double), ("objective", c_double),
                ("seconds", c_double), ("seconds_to_target", c_double), ("normA2", c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved"}


class MlpC(ctypes.Structure):
    _fields_ = [("r", c_int32), ("hidden", c_int32), ("M1", c_void_p), ("b1", c_void_p),
                ("M2", c_void_p), ("b2", c_void_p), ("M1h", c_void_p), ("M2h", c_void_p),
                ("adam_m", c_void_p), ("adam_v", c_void_p)]


ABI_VERSION = 4
EXPORTS = ("snmf_params_default", "snmf_solve", "snmf_solve_noalloc", "snmf_plan_create",
           "snmf_plan_solve",
           "snmf_plan_destroy", "snmf_plan_half_step", "snmf_plan_apass", "snmf_plan_gram",
           "snmf_plan_time_apass", "snmf_rho", "snmf_spmm", "snmf_split_bf16",
           "snmf_batch_create", "snmf_batch_solve", "snmf_batch_destroy", "snmf_solve_batched",
           "snmf_batch_apass", "snmf_batch_time_apass", "snmf_batch_size", "snmf_mlp_sync",
           "snmf_mlp_forward", "snmf_mlp_workspace_bytes", "snmf_mlp_train_step", "snmf_batch_frame",
           "snmf_batch_targets", "snmf_batch_warmstart", "snmf_warmstart", "snmf_lai_sketch",
           "snmf_svd_start", "snmf_knn", "snmf_knn_graph", "snmf_nmf_solve", "snmf_clock_rate_hz",
           "snmf_last_error", "snmf_abi_version")


def load_library(path: str = LIB_PATH):
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with __graft_entry__.build()")
    lib = ctypes.CDLL(path)
    vp = c_void_p
    sig = {
        "snmf_params_default": ([POINTER(Params)], c_int32),
        "snmf_solve": ([POINTER(Matrix), c_int32, vp, POINTER(Params), vp, vp, POINTER(Info), vp,
                        POINTER(c_double)], c_int32),
        "snmf_solve_noalloc": ([POINTER(Matrix), c_int32, vp, POINTER(Params), vp, vp,
                                POINTER(Info), vp, POINTER(c_double)], c_int32),
        "snmf_plan_create": ([POINTER(Matrix), c_int32, POINTER(Params), vp, POINTER(vp)], c_int32),
        "snmf_plan_solve": ([vp, vp, vp, vp, POINTER(Info), vp, POINTER(c_double)], c_int32),
        "snmf_plan_destroy": ([vp], c_int32),
        "snmf_plan_half_step": ([vp, vp, vp, c_int32, vp, POINTER(c_double)], c_int32),
        "snmf_plan_apass": ([vp, vp, vp, vp], c_int32),
        "snmf_plan_gram": ([vp, vp, vp, vp], c_int32),
        "snmf_plan_time_apass": ([vp, vp, c_int32, POINTER(c_double)], c_int32),
        "snmf_rho": ([vp, c_int32, POINTER(c_double), vp], c_int32),
        "snmf_spmm": ([POINTER(Matrix), c_int32, vp, c_int32, vp, vp], c_int32),
        "snmf_split_bf16": ([vp, c_int64, vp, vp, vp], c_int32),
        "snmf_batch_create": ([c_int32, POINTER(Matrix), POINTER(c_int32), POINTER(c_double),
                               c_int32, POINTER(Params), vp, POINTER(vp)], c_int32),
        "snmf_batch_solve": ([vp, POINTER(vp), POINTER(vp), POINTER(vp), POINTER(Info), vp,
                              POINTER(c_double)], c_int32),
        "snmf_batch_destroy": ([vp], c_int32),
        "snmf_solve_batched": ([c_int32, POINTER(Matrix), POINTER(c_int32), POINTER(c_double),
                                c_int32, POINTER(vp), POINTER(Params), POINTER(vp), POINTER(vp),
                                POINTER(Info), vp, POINTER(c_double)], c_int32),
        "snmf_batch_apass": ([vp, vp, vp, vp], c_int32),
        "snmf_batch_time_apass": ([vp, vp, c_int32, POINTER(c_double)], c_int32),
        "snmf_batch_size": ([vp, POINTER(c_int32), POINTER(c_int64)], c_int32),
        "snmf_mlp_sync": ([POINTER(MlpC), vp], c_int32),
        "snmf_mlp_forward": ([POINTER(MlpC), c_int64, vp, vp, vp, vp], c_int32),
        "snmf_mlp_workspace_bytes": ([c_int32, c_int64], ctypes.c_size_t),
        "snmf_mlp_train_step": ([POINTER(MlpC), c_int64, vp, vp, vp, c_int64, ctypes.c_float,
                                 ctypes.c_float, c_int32, vp, ctypes.c_size_t, vp,
                                 POINTER(c_double)], c_int32),
        "snmf_batch_frame": ([vp, vp, vp, vp, vp, vp], c_int32),
        "snmf_batch_targets": ([vp, vp, vp, vp, vp, vp], c_int32),
        "snmf_batch_warmstart": ([vp, c_int32, POINTER(MlpC), vp, vp, vp], c_int32),
        "snmf_warmstart": ([POINTER(MlpC), POINTER(Matrix), c_int32, c_int32, vp, vp, vp], c_int32),
        "snmf_lai_sketch": ([POINTER(Matrix), c_int32, c_int32, c_int32, c_int32, vp, vp, vp, vp],
                            c_int32),
        "snmf_svd_start": ([POINTER(Matrix), c_int32, c_int32, c_int32, c_int32, vp, vp, vp],
                           c_int32),
        "snmf_knn": ([vp, c_int64, c_int32, c_int32, c_int32, vp, vp], c_int32),
        "snmf_knn_graph": ([vp, c_int64, c_int32, c_int32, c_double, c_int32, c_int32, vp, vp, vp,
                            c_int64, POINTER(c_int64), vp], c_int32),
        "snmf_nmf_solve": ([POINTER(Matrix), c_int64, c_int32, vp, vp, POINTER(Params), vp, vp,
                            POINTER(Info), vp, POINTER(c_double)], c_int32),
        "snmf_clock_rate_hz": ([], c_double),
        "snmf_last_error": ([], ctypes.c_char_p),
        "snmf_abi_version": ([], c_int32),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    if lib.snmf_abi_version() != ABI_VERSION:   # the structs above follow this version
        raise ImportError(f"{path} has ABI {lib.snmf_abi_version()}, the binding {ABI_VERSION}:"
                          " rebuild it with __graft_entry__.build()")
    return lib


_lib = load_library()


def _check(status):
    if status != 0:
        raise SnmfError(status, _lib.snmf_last_error().decode())


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def prec_of(dtype) -> int:
    import torch
    return F64 if dtype == torch.float64 else F32


# ------------------------------------------------------------------ matrix descriptors
class MatrixRef:
    """A Matrix descriptor plus the tensors it points to (kept alive with it)."""

    def __init__(self, desc: Matrix, keep):
        self.desc = desc
        self.keep = keep
        self.n = desc.n


def dense(A) -> MatrixRef:
    assert A.is_cuda and A.dim() == 2 and A.stride(1) == 1
    d = Matrix(fmt=DENSE, n=A.shape[0], dense=A.data_ptr(), ld=A.stride(0))
    return MatrixRef(d, [A])


def csr(rowptr, col, val, n: int) -> MatrixRef:
    d = Matrix(fmt=CSR, n=n, rowptr=rowptr.data_ptr(), col=col.data_ptr() if col.numel() else 0,
               val=val.data_ptr() if val.numel() else 0, nnz=val.numel())
    return MatrixRef(d, [rowptr, col, val])


def lowrank(U, lam) -> MatrixRef:
    d = Matrix(fmt=LOWRANK, n=U.shape[0], U=U.data_ptr(), ell=U.shape[1], lam=lam.data_ptr())
    return MatrixRef(d, [U, lam])


def csr_from_scipy(a, dtype, device="cuda"):
    """Upload a scipy CSR matrix (sorted indices) as a MatrixRef of the given dtype."""
    import torch
    a = a.tocsr()
    a.sort_indices()
    rowptr = torch.from_numpy(np.ascontiguousarray(a.indptr, dtype=np.int64)).to(device)
    col = torch.from_numpy(np.ascontiguousarray(a.indices, dtype=np.int32)).to(device)
    val = torch.from_numpy(np.ascontiguousarray(a.data)).to(device=device, dtype=dtype)
    return csr(rowptr, col, val, a.shape[0])


# ------------------------------------------------------------------ parameters
def tuning(tiles_per_wg=(4, 4, 4, 4), spmm_rows_per_wg: int = 16) -> Tuning:
    """Launch shape of a batched solve (rank classes r <= 8, 16, 32, 64)."""
    t = Tuning()
    for q, v in enumerate(tiles_per_wg):
        t.tiles_per_wg[q] = int(v)
    t.spmm_rows_per_wg = int(spmm_rows_per_wg)
    return t


def params(**kw) -> Params:
    p = Params()
    _check(_lib.snmf_params_default(ctypes.byref(p)))
    for k, v in kw.items():
        if k == "lam":
            k = "lambda_"
        if k == "L":
            continue
        if k == "tuning":                 # a Tuning, a dict of its fields, or None
            if isinstance(v, dict):
                v = tuning(**v)
            p.tuning = ctypes.pointer(v) if v is not None else None
            continue
        if not hasattr(p, k):
            raise KeyError(k)
        setattr(p, k, v)
    return p


# ------------------------------------------------------------------ plans
class Plan:
    """Owns a library plan: repeated solves of one A (and L) with reused scratch memory."""

    def __init__(self, A: MatrixRef, r: int, prm: Params, L: MatrixRef | None = None):
        self._A, self._L = A, L
        self._prm = prm
        if L is not None:
            prm.L = ctypes.pointer(L.desc)
        self.max_outer = prm.max_outer
        self.r = r
        self.n = A.n
        h = ctypes.c_void_p()
        _check(_lib.snmf_plan_create(ctypes.byref(A.desc), r, ctypes.byref(prm), _stream(),
                                     ctypes.byref(h)))
        self._h = h

    def solve(self, W0, W_out=None, Ht_out=None, trace: bool = True):
        import torch
        W_out = torch.empty_like(W0) if W_out is None else W_out
        Ht_out = torch.empty_like(W0) if Ht_out is None else Ht_out
        info = Info()
        tr = (c_double * (self.max_outer * TRACE_FIELDS))() if trace else None
        st = _lib.snmf_plan_solve(self._h, _ptr(W0), _ptr(W_out), _ptr(Ht_out),
                                  ctypes.byref(info), _stream(), tr)
        _check(st)
        out = info.as_dict()
        if trace:
            arr = np.frombuffer(tr, dtype=np.float64).reshape(self.max_outer, TRACE_FIELDS)
            out["trace"] = arr[: info.outer].copy()
        return W_out, Ht_out, out

    def half_step(self, X, P, is_hstep: bool):
        sc = (c_double * 8)()
        _check(_lib.snmf_plan_half_step(self._h, _ptr(X), _ptr(P), int(is_hstep), _stream(), sc))
        keys = ("rho", "alpha", "beta", "e", "ss", "sy", "ls_evals", "inner_done")
        return dict(zip(keys, list(sc)))

    def apass(self, P, B):
        _check(_lib.snmf_plan_apass(self._h, _ptr(P), _ptr(B), _stream()))
        return B

    def time_apass(self, P, reps: int = 50) -> float:
        """Average A-pass kernel time in ms (HIP events on the plan's stream)."""
        import torch
        torch.cuda.synchronize()
        ms = c_double()
        _check(_lib.snmf_plan_time_apass(self._h, _ptr(P), int(reps), ctypes.byref(ms)))
        return ms.value

    def gram(self, P):
        import torch
        G = torch.empty((self.r, self.r), dtype=torch.float64, device=P.device)
        _check(_lib.snmf_plan_gram(self._h, _ptr(P), _ptr(G), _stream()))
        return G

    def close(self):
        if getattr(self, "_h", None):
            _lib.snmf_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


class Batch:
    """Batched solves (snmf_batch_*): problems As[g] with ranks r[g], each from `restarts`
    starts.  Starts and results are per-problem tensors of shape (restarts, n_g, r_g)."""

    def __init__(self, As, r, prm: Params, restarts: int = 1, lam=None):
        self._As = list(As)
        self.nprob = len(self._As)
        self.r = [int(x) for x in r]
        self.n = [int(a.n) for a in self._As]
        self.S = int(restarts)
        self.max_outer = prm.max_outer
        self._prm = prm
        self._descs = (Matrix * self.nprob)(*[a.desc for a in self._As])
        self._r = (c_int32 * self.nprob)(*self.r)
        self._lam = None if lam is None else (c_double * self.nprob)(*[float(x) for x in lam])
        h = ctypes.c_void_p()
        _check(_lib.snmf_batch_create(self.nprob, self._descs, self._r, self._lam, self.S,
                                      ctypes.byref(prm), _stream(), ctypes.byref(h)))
        self._h = h
        ni, ne = c_int32(), c_int64()
        _check(_lib.snmf_batch_size(self._h, ctypes.byref(ni), ctypes.byref(ne)))
        self.ninst, self.elements = ni.value, ne.value

    def solve(self, W0s, trace: bool = False):
        import torch
        Ws = [torch.empty_like(w) for w in W0s]
        Hs = [torch.empty_like(w) for w in W0s]
        vpa = ctypes.c_void_p * self.nprob
        infos = (Info * self.ninst)()
        tr = (c_double * (self.ninst * self.max_outer * TRACE_FIELDS))() if trace else None
        _check(_lib.snmf_batch_solve(self._h, vpa(*[w.data_ptr() for w in W0s]),
                                     vpa(*[w.data_ptr() for w in Ws]),
                                     vpa(*[w.data_ptr() for w in Hs]), infos, _stream(), tr))
        out = [i.as_dict() for i in infos]
        traces = None
        if trace:
            traces = np.frombuffer(tr, dtype=np.float64).reshape(self.ninst, self.max_outer,
                                                                 TRACE_FIELDS).copy()
        return Ws, Hs, out, traces

    def apass(self, P, B):
        _check(_lib.snmf_batch_apass(self._h, _ptr(P), _ptr(B), _stream()))
        return B

    def time_apass(self, P, reps: int = 20) -> float:
        """Average time in ms of the batch's A-pass launches (HIP events on its stream)."""
        import torch
        torch.cuda.synchronize()
        ms = c_double()
        _check(_lib.snmf_batch_time_apass(self._h, _ptr(P), int(reps), ctypes.byref(ms)))
        return ms.value

    def offsets(self):
        """Element offset of every problem's block (restart 0) in a batch buffer."""
        out, at = [], 0
        for n, r in zip(self.n, self.r):
            out.append(at)
            at += self.S * n * r
        return out

    def split(self, buf):
        """Per-problem (S, n_g, r_g) views of a batch buffer."""
        return [buf[o: o + self.S * n * r].view(self.S, n, r)
                for o, n, r in zip(self.offsets(), self.n, self.r)]

    def frame(self, Omega):
        """Sketch Y = A Omega and anchor-frame coordinates C (batch buffers), anchors."""
        import torch
        Y = torch.empty_like(Omega)
        C = torch.empty_like(Omega)
        anc = torch.empty((self.ninst, 64), dtype=torch.int32, device=Omega.device)
        _check(_lib.snmf_batch_frame(self._h, _ptr(Omega), _ptr(Y), _ptr(C), _ptr(anc),
                                     _stream()))
        return Y, C, anc

    def targets(self, C, Ht):
        import torch
        T = torch.empty_like(C)
        perm = torch.empty((self.ninst, 64), dtype=torch.int32, device=C.device)
        _check(_lib.snmf_batch_targets(self._h, _ptr(C), _ptr(Ht), _ptr(T), _ptr(perm),
                                       _stream()))
        return T, perm

    def warmstart(self, models, Omega):
        import torch
        W0 = torch.empty_like(Omega)
        arr = (MlpC * len(models))(*[m.desc for m in models]) if models else None
        _check(_lib.snmf_batch_warmstart(self._h, len(models), arr, _ptr(Omega), _ptr(W0),
                                         _stream()))
        return W0

    def close(self):
        if getattr(self, "_h", None):
            _lib.snmf_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


class Mlp:
    """A warm-start network r -> 128 -> r in device memory (FP32 masters, BF16 copies,
    Adam moments), initialised from host arrays {M1, b1, M2, b2}."""

    def __init__(self, init, device="cuda"):
        import torch
        M1 = np.asarray(init["M1"], dtype=np.float32)
        self.r = int(M1.shape[1])
        self.hidden = int(M1.shape[0])
        f = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(device)
        self.M1, self.b1, self.M2, self.b2 = f(init["M1"]), f(init["b1"]), f(init["M2"]), f(init["b2"])
        self.M1h = torch.empty(self.M1.shape, dtype=torch.int16, device=device)
        self.M2h = torch.empty(self.M2.shape, dtype=torch.int16, device=device)
        n = 2 * self.hidden * self.r + self.hidden + self.r
        self.adam_m = torch.zeros(n, dtype=torch.float32, device=device)
        self.adam_v = torch.zeros(n, dtype=torch.float32, device=device)
        self.desc = MlpC(self.r, self.hidden, self.M1.data_ptr(), self.b1.data_ptr(),
                         self.M2.data_ptr(), self.b2.data_ptr(), self.M1h.data_ptr(),
                         self.M2h.data_ptr(), self.adam_m.data_ptr(), self.adam_v.data_ptr())
        self.step = 0
        self._work = None
        _check(_lib.snmf_mlp_sync(ctypes.byref(self.desc), _stream()))

    def params(self):
        return {k: getattr(self, k).double().cpu().numpy() for k in ("M1", "b1", "M2", "b2")}

    def forward(self, C, row_scale=None):
        import torch
        Y = torch.empty_like(C)
        _check(_lib.snmf_mlp_forward(ctypes.byref(self.desc), C.shape[0], _ptr(C),
                                     _ptr(row_scale), _ptr(Y), _stream()))
        return Y

    def train_step(self, C, T, idx, mu, lr, want_loss=False):
        import torch
        B = int(idx.numel())
        need = _lib.snmf_mlp_workspace_bytes(self.r, B)
        if self._work is None or self._work.numel() < need:
            self._work = torch.empty(need, dtype=torch.uint8, device=C.device)
        self.step += 1
        loss = c_double(0.0)
        _check(_lib.snmf_mlp_train_step(ctypes.byref(self.desc), C.shape[0], _ptr(C), _ptr(T),
                                        _ptr(idx), B,
                                        float(mu), float(lr), self.step, _ptr(self._work),
                                        self._work.numel(), _stream(),
                                        ctypes.byref(loss) if want_loss else None))
        return loss.value if want_loss else None


def solve(A: MatrixRef, W0, prm: Params, L: MatrixRef | None = None, trace: bool = True):
    with Plan(A, W0.shape[1], prm, L) as pl:
        return pl.solve(W0, trace=trace)


def solve_noalloc(A: MatrixRef, W0, prm: Params, L: MatrixRef | None = None, W_out=None,
                  Ht_out=None, trace: bool = True):
    """snmf_solve_noalloc: the solve with the library's static scratch (no allocation in
    the library; the outputs are the caller's)."""
    import torch
    if L is not None:
        prm.L = ctypes.pointer(L.desc)
    W_out = torch.empty_like(W0) if W_out is None else W_out
    Ht_out = torch.empty_like(W0) if Ht_out is None else Ht_out
    info = Info()
    tr = (c_double * (prm.max_outer * TRACE_FIELDS))() if trace else None
    _check(_lib.snmf_solve_noalloc(ctypes.byref(A.desc), W0.shape[1], _ptr(W0), ctypes.byref(prm),
                                   _ptr(W_out), _ptr(Ht_out), ctypes.byref(info), _stream(), tr))
    out = info.as_dict()
    if trace:
        arr = np.frombuffer(tr, dtype=np.float64).reshape(prm.max_outer, TRACE_FIELDS)
        out["trace"] = arr[: info.outer].copy()
    return W_out, Ht_out, out


def warmstart(A: MatrixRef, Omega, mlp: "Mlp | None" = None):
    """The warm start of one problem (snmf_warmstart): W0 from the sketch matrix Omega
    (n x r, float32 or float64) through the frame and, if given, the network."""
    import torch
    W0 = torch.empty_like(Omega)
    _check(_lib.snmf_warmstart(ctypes.byref(mlp.desc) if mlp is not None else None,
                               ctypes.byref(A.desc), Omega.shape[1], prec_of(Omega.dtype),
                               _ptr(Omega), _ptr(W0), _stream()))
    return W0


def lai_sketch(A: MatrixRef, rank: int, power_iters: int, Omega):
    """Range finder (snmf_lai_sketch): U (n x rank) and lam (rank, float64) from the
    Gaussian sketch matrix Omega (n x (rank + oversample), float32 or float64)."""
    import torch
    U = torch.empty((Omega.shape[0], rank), dtype=Omega.dtype, device=Omega.device)
    lam = torch.empty(rank, dtype=torch.float64, device=Omega.device)
    _check(_lib.snmf_lai_sketch(ctypes.byref(A.desc), int(rank), Omega.shape[1] - int(rank),
                                int(power_iters), prec_of(Omega.dtype), _ptr(Omega), _ptr(U),
                                _ptr(lam), _stream()))
    return U, lam


def svd_start(A: MatrixRef, r: int, power_iters: int, Omega):
    """SVD-based start W0 = |U E^(1/2)| (snmf_svd_start); Omega is n x (r + oversample)."""
    import torch
    W0 = torch.empty((Omega.shape[0], r), dtype=Omega.dtype, device=Omega.device)
    _check(_lib.snmf_svd_start(ctypes.byref(A.desc), int(r), Omega.shape[1] - int(r),
                               int(power_iters), prec_of(Omega.dtype), _ptr(Omega), _ptr(W0),
                               _stream()))
    return W0


def knn(X, K: int):
    """Neighbour lists (n x K int32) of the rows of X (snmf_knn)."""
    import torch
    nbr = torch.empty((X.shape[0], K), dtype=torch.int32, device=X.device)
    _check(_lib.snmf_knn(_ptr(X), X.shape[0], X.shape[1], int(K), prec_of(X.dtype), _ptr(nbr),
                         _stream()))
    return nbr


def knn_graph(X, K: int, sigma: float = 0.0, laplacian: bool = True) -> MatrixRef:
    """The K-nearest-neighbour similarity (or its normalised Laplacian) of the rows of X
    as a CSR MatrixRef (snmf_knn_graph)."""
    import torch
    n, dim = X.shape
    cap = n * (2 * int(K) + (1 if laplacian else 0))
    rowptr = torch.empty(n + 1, dtype=torch.int64, device=X.device)
    col = torch.empty(cap, dtype=torch.int32, device=X.device)
    val = torch.empty(cap, dtype=X.dtype, device=X.device)
    nnz = c_int64()
    _check(_lib.snmf_knn_graph(_ptr(X), n, dim, int(K), float(sigma), int(bool(laplacian)),
                               prec_of(X.dtype), _ptr(rowptr), _ptr(col), _ptr(val), cap,
                               ctypes.byref(nnz), _stream()))
    return csr(rowptr, col[: nnz.value], val[: nnz.value], n)


def rho(G) -> float:
    out = c_double()
    _check(_lib.snmf_rho(_ptr(G), G.shape[0], ctypes.byref(out), _stream()))
    return out.value


def spmm(M: MatrixRef, X, Y=None):
    import torch
    Y = torch.empty_like(X) if Y is None else Y
    _check(_lib.snmf_spmm(ctypes.byref(M.desc), prec_of(X.dtype), _ptr(X), X.shape[1], _ptr(Y),
                          _stream()))
    return Y


def split_bf16(x):
    import torch
    hi = torch.empty(x.shape, dtype=torch.int16, device=x.device)
    lo = torch.empty(x.shape, dtype=torch.int16, device=x.device)
    _check(_lib.snmf_split_bf16(_ptr(x), x.numel(), _ptr(hi), _ptr(lo), _stream()))
    return hi, lo


def clock_rate_hz() -> float:
    return _lib.snmf_clock_rate_hz()


def abi_version() -> int:
    return _lib.snmf_abi_version()


def nmf_solve(V: MatrixRef, n_cols: int, W0, Ht0, prm: Params, trace: bool = True):
    """NMPBB for rectangular NMF (snmf_nmf_solve): V is m x n_cols (dense or CSR), W0 is
    m x r, Ht0 n_cols x r; returns W, Ht and the info dict (with the trace)."""
    import torch
    W_out, Ht_out = torch.empty_like(W0), torch.empty_like(Ht0)
    info = Info()
    tr = (c_double * (prm.max_outer * TRACE_FIELDS))() if trace else None
    _check(_lib.snmf_nmf_solve(ctypes.byref(V.desc), int(n_cols), W0.shape[1], _ptr(W0),
                               _ptr(Ht0), ctypes.byref(prm), _ptr(W_out), _ptr(Ht_out),
                               ctypes.byref(info), _stream(), tr))
    out = info.as_dict()
    if trace:
        arr = np.frombuffer(tr, dtype=np.float64).reshape(prm.max_outer, TRACE_FIELDS)
        out["trace"] = arr[: info.outer].copy()
    return W_out, Ht_out, out
