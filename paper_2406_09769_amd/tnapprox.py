"""ctypes binding of libtnapprox.so (include/tnapprox.h); argument marshalling only.

Every step of the contraction runs inside the library. If the library has not been
built the import of this module raises: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import json
import math
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtnapprox.so")

TN_OK, TN_EINVAL, TN_ENOMEM, TN_EDEVICE, TN_ENUMERIC, TN_EUNSUPPORTED = range(6)
TN_FP64, TN_SPLIT_BF16X3, TN_SPLIT_FP16X3, TN_SPLIT_BF16X3_ALL, TN_SPLIT_FP16X3_ALL = range(5)
TN_EIG_EXACT, TN_EIG_LEARNED = range(2)
TN_TRIDIAG_AUTO, TN_TRIDIAG_QL = range(2)


class TnError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"[{status}] {msg}")
        self.status = status


class tn_tensor(C.Structure):
    _fields_ = [("order", C.c_int32), ("dims", C.POINTER(C.c_int64)), ("data", C.POINTER(C.c_double))]


class tn_edge(C.Structure):
    _fields_ = [("t0", C.c_int32), ("m0", C.c_int32), ("t1", C.c_int32), ("m1", C.c_int32)]


class tn_path(C.Structure):
    _fields_ = [("n_slices", C.c_int32), ("slice_ptr", C.POINTER(C.c_int32)),
                ("slice_vertices", C.POINTER(C.c_int32))]


PROGRESS = C.CFUNCTYPE(None, C.c_void_p, C.c_int32, C.c_int32)


class tn_options(C.Structure):
    _fields_ = [("precision", C.c_int32), ("eig", C.c_int32), ("residual_tol", C.c_double),
                ("tau_rel", C.c_double), ("tau_deg", C.c_double), ("hip_stream", C.c_void_p),
                ("model", C.c_void_p), ("gemm_config", C.c_int32 * 3), ("chunks", C.c_int32),
                ("progress", PROGRESS), ("progress_ctx", C.c_void_p), ("tridiag", C.c_int32)]


class tn_result(C.Structure):
    _fields_ = [("log_abs", C.c_double), ("sign", C.c_int32), ("_pad", C.c_int32),
                ("seconds", C.c_double), ("flops", C.c_int64), ("eig_flops", C.c_int64),
                ("n_eig", C.c_int64), ("n_fallback", C.c_int64), ("max_residual", C.c_double),
                ("n_learned", C.c_int64), ("split_flops", C.c_int64)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run paper_2406_09769_amd/build.py "
                          "(or __graft_entry__.build()) first")
    lib = C.CDLL(LIB_PATH)
    P = C.POINTER
    sig = {
        "tn_create": (C.c_int, [P(tn_tensor), C.c_int32, P(tn_edge), C.c_int32, P(C.c_void_p)]),
        "tn_contract_approx": (C.c_int, [C.c_void_p, P(tn_path), C.c_int32, C.c_int32, P(tn_options), P(tn_result)]),
        "tn_contract_approx_batch": (C.c_int, [P(C.c_void_p), P(tn_path), P(C.c_int32), P(C.c_int32), C.c_int32,
                                              P(tn_options), P(tn_result)]),
        "tn_contract_approx_noalloc": (C.c_int, [C.c_void_p, P(tn_path), C.c_int32, C.c_int32, P(tn_options),
                                                P(tn_result)]),
        "tn_plan_json": (C.c_int, [P(C.c_int64), P(C.c_int32), C.c_int32, P(tn_edge), C.c_int32, P(tn_path),
                                   C.c_int32, C.c_char_p, P(C.c_int64)]),
        "tn_destroy": (None, [C.c_void_p]),
        "tn_error_string": (C.c_char_p, [C.c_int]),
        "tn_last_error": (C.c_char_p, []),
        "tn_plan_stats": (C.c_int, [C.c_void_p, P(tn_path), C.c_int32, C.c_int32, P(C.c_int64)]),
        "tn_debug_gemm": (C.c_int, [P(C.c_double), C.c_int64, C.c_int64, P(C.c_double), C.c_int64, C.c_int64,
                                    P(C.c_double), C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_int32,
                                    C.c_int32]),
        "tn_debug_eig": (C.c_int, [P(C.c_double), C.c_int32, C.c_int32, C.c_int32, P(tn_options),
                                   P(C.c_double), P(C.c_int64)]),
        "tn_debug_rescale": (C.c_int, [P(C.c_double), C.c_int64, P(C.c_int64)]),
        "tn_profile_last": (C.c_int, [C.c_void_p, P(C.c_double)]),
        "tn_model_create": (C.c_int, [C.c_uint64, P(C.c_void_p)]),
        "tn_model_set": (C.c_int, [C.c_void_p, P(C.c_float), C.c_int64]),
        "tn_model_get": (C.c_int, [C.c_void_p, P(C.c_float), C.c_int64]),
        "tn_model_grad": (C.c_int, [C.c_void_p, P(C.c_float), P(C.c_float), C.c_int32, P(C.c_float),
                                    P(C.c_double)]),
        "tn_model_train": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, C.c_int32, C.c_double, C.c_uint64,
                                     P(C.c_double)]),
        "tn_model_destroy": (None, [C.c_void_p]),
        "tn_dataset_create": (C.c_int, [C.c_int64, P(C.c_void_p)]),
        "tn_dataset_size": (C.c_int, [C.c_void_p, P(C.c_int64)]),
        "tn_dataset_read": (C.c_int, [C.c_void_p, P(C.c_float), P(C.c_float), C.c_int64]),
        "tn_dataset_destroy": (None, [C.c_void_p]),
        "tn_harvest": (C.c_int, [C.c_void_p, P(tn_path), C.c_int32, C.c_int32, C.c_void_p, P(tn_result)]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


LIB = _load()


def _check(rc: int):
    if rc != TN_OK:
        raise TnError(rc, f"{LIB.tn_error_string(rc).decode()}: {LIB.tn_last_error().decode()}")


def _dptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


# ---------------------------------------------------------------- marshalling

class _NetArgs:
    """Keeps the ctypes views of one network alive for the duration of a call."""

    def __init__(self, tensors, edges):
        self.data = [np.array(t, dtype=np.float64, order="C") for t in tensors]   # keeps 0-d scalars 0-d
        self.dims = [np.array(t.shape, dtype=np.int64) for t in self.data]
        n = len(self.data)
        self.tensors = (tn_tensor * n)()
        for i, (d, s) in enumerate(zip(self.data, self.dims)):
            self.tensors[i].order = d.ndim
            self.tensors[i].dims = s.ctypes.data_as(C.POINTER(C.c_int64)) if d.ndim else None
            self.tensors[i].data = _dptr(d) if d.size else None
        ne = len(edges)
        self.edges = (tn_edge * max(ne, 1))()
        for i, (t0, m0, t1, m1) in enumerate(edges):
            self.edges[i] = tn_edge(int(t0), int(m0), int(t1), int(m1))
        self.n = n
        self.ne = ne


class _PathArgs:
    def __init__(self, slices):
        ptr = [0]
        flat = []
        for s in slices:
            flat.extend(int(v) for v in s)
            ptr.append(len(flat))
        self.ptr = np.array(ptr, dtype=np.int32)
        self.flat = np.array(flat if flat else [0], dtype=np.int32)
        self.path = tn_path(len(slices), self.ptr.ctypes.data_as(C.POINTER(C.c_int32)),
                            self.flat.ctypes.data_as(C.POINTER(C.c_int32)))


_LIVE = []   # the progress callback of the call in flight (kept alive across it)


def _options(precision=TN_FP64, eig=TN_EIG_EXACT, residual_tol=1e-6, tau_rel=1e-12, tau_deg=0.1,
             stream=None, model=None, gemm_config=(0, 0, 0), chunks=0, progress=None, tridiag=0):
    """progress: a Python callable (done, total) called after each part when chunks > 1."""
    cb = PROGRESS(lambda ctx, done, total: progress(int(done), int(total))) if progress else PROGRESS()
    _LIVE[:] = [cb]
    return tn_options(int(precision), int(eig), float(residual_tol), float(tau_rel), float(tau_deg),
                      C.c_void_p(stream) if stream else None, model.ptr if model is not None else None,
                      (C.c_int32 * 3)(*[int(x) for x in gemm_config]), int(chunks), cb, None, int(tridiag))


@dataclass
class Result:
    log_abs: float
    sign: int
    seconds: float
    flops: int
    eig_flops: int
    n_eig: int
    n_fallback: int
    max_residual: float
    n_learned: int
    split_flops: int


def _result(r: tn_result) -> Result:
    return Result(r.log_abs, r.sign, r.seconds, r.flops, r.eig_flops, r.n_eig, r.n_fallback, r.max_residual,
                  r.n_learned, r.split_flops)


# ---------------------------------------------------------------- the calls

class Handle:
    """Owns a tn_net; destroyed with the object."""

    def __init__(self, ptr):
        self.ptr = ptr

    def __del__(self):
        if getattr(self, "ptr", None):
            LIB.tn_destroy(self.ptr)
            self.ptr = None


def tn_create(tensors, edges) -> Handle:
    a = _NetArgs(tensors, edges)
    out = C.c_void_p()
    _check(LIB.tn_create(a.tensors, a.n, a.edges, a.ne, C.byref(out)))
    return Handle(out)


def tn_contract_approx(h: Handle, slices, max_rank: int, env_size: int, **opt) -> Result:
    p = _PathArgs(slices)
    o = _options(**opt)
    r = tn_result()
    _check(LIB.tn_contract_approx(h.ptr, C.byref(p.path), int(max_rank), int(env_size), C.byref(o), C.byref(r)))
    return _result(r)


def tn_contract_approx_noalloc(h: Handle, slices, max_rank: int, env_size: int, **opt) -> Result:
    p = _PathArgs(slices)
    o = _options(**opt)
    r = tn_result()
    _check(LIB.tn_contract_approx_noalloc(h.ptr, C.byref(p.path), int(max_rank), int(env_size), C.byref(o),
                                          C.byref(r)))
    return _result(r)


def tn_contract_approx_batch(handles, slices_list, max_rank, env_size, **opt):
    """max_rank and env_size: one int for every network, or one per network."""
    n = len(handles)
    hs = (C.c_void_p * n)(*[h.ptr.value for h in handles])
    ps = [_PathArgs(s) for s in slices_list]
    paths = (tn_path * n)(*[p.path for p in ps])
    mr = [int(max_rank)] * n if np.isscalar(max_rank) else [int(x) for x in max_rank]
    es = [int(env_size)] * n if np.isscalar(env_size) else [int(x) for x in env_size]
    mra = (C.c_int32 * n)(*mr)
    esa = (C.c_int32 * n)(*es)
    o = _options(**opt)
    rs = (tn_result * n)()
    _check(LIB.tn_contract_approx_batch(hs, paths, mra, esa, n, C.byref(o), rs))
    return [_result(r) for r in rs]


def tn_plan_json(tensors_or_shapes, edges, slices, env_size: int) -> dict:
    shapes = [tuple(np.shape(t)) if not isinstance(t, tuple) else t for t in tensors_or_shapes]
    orders = np.array([len(s) for s in shapes], dtype=np.int32)
    flat = np.array([d for s in shapes for d in s] or [1], dtype=np.int64)
    ne = len(edges)
    ed = (tn_edge * max(ne, 1))()
    for i, (t0, m0, t1, m1) in enumerate(edges):
        ed[i] = tn_edge(int(t0), int(m0), int(t1), int(m1))
    p = _PathArgs(slices)
    ln = C.c_int64(0)
    args = (flat.ctypes.data_as(C.POINTER(C.c_int64)), orders.ctypes.data_as(C.POINTER(C.c_int32)),
            len(shapes), ed, ne, C.byref(p.path), int(env_size))
    rc = LIB.tn_plan_json(*args, None, C.byref(ln))
    _check(rc)
    buf = C.create_string_buffer(ln.value)
    _check(LIB.tn_plan_json(*args, buf, C.byref(ln)))
    return json.loads(buf.value.decode())


def tn_plan_stats(h: Handle, slices, max_rank: int, env_size: int) -> dict:
    p = _PathArgs(slices)
    st = (C.c_int64 * 9)()
    _check(LIB.tn_plan_stats(h.ptr, C.byref(p.path), int(max_rank), int(env_size), st))
    keys = ["ops", "table_entries", "ws_doubles", "flops", "eig_flops", "n_eig", "max_eig_dim", "grid_ops", "qr_svd"]
    return dict(zip(keys, list(st)))


def tn_profile_last(h: Handle) -> dict:
    out = (C.c_double * 18)()
    _check(LIB.tn_profile_last(h.ptr, out))
    return {"gemm": out[1], "eig": out[2], "rescale": out[3], "scalar": out[4], "ident": out[5],
            "eig_reduce": out[0], "eig_ql": out[6], "eig_back": out[7], "ql_rotations": out[8],
            "learned_rejected": {"size": int(out[9]), "dependent": int(out[10]), "cut": int(out[11]),
                                 "residual": int(out[12])},
            "learned_time": {"start": out[13], "products": out[14], "small_eig": out[15], "ritz": out[16]},
            "qr": out[17]}


def tn_debug_gemm(A: np.ndarray, B: np.ndarray, lo_split: int = 1 << 30, precision: int = TN_FP64,
                  chip_wide: bool = False) -> np.ndarray:
    A = np.asarray(A, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64)
    M, K = A.shape
    K2, N = B.shape
    assert K == K2
    sam, sak = (s // 8 for s in A.strides)
    sbk, sbn = (s // 8 for s in B.strides)
    Cm = np.zeros((M, N))
    _check(LIB.tn_debug_gemm(_dptr(A), sam, sak, _dptr(B), sbk, sbn, _dptr(Cm), M, N, K, int(lo_split),
                             int(precision), int(bool(chip_wide))))
    return Cm


def tn_debug_eig(L: np.ndarray, ucols: int, tau_rel=1e-12, tau_deg=0.1, rest: int = 0, model=None,
                 residual_tol=1e-6, stats: bool = False, tridiag: int = 0):
    """Kept eigenvectors (n x ucols, zero past the kept rank) and the fallback flag;
    with stats=True also the dict of the learned warm start's outcome."""
    L = np.ascontiguousarray(L, dtype=np.float64)
    n = L.shape[0]
    U = np.zeros((n, ucols))
    st = (C.c_int64 * 8)()
    o = _options(tau_rel=tau_rel, tau_deg=tau_deg, residual_tol=residual_tol,
                 eig=TN_EIG_LEARNED if model is not None else TN_EIG_EXACT, model=model, tridiag=tridiag)
    _check(LIB.tn_debug_eig(_dptr(L), n, int(ucols), int(rest), C.byref(o), _dptr(U), st))
    if not stats:
        return U, int(st[0])
    return U, int(st[0]), {"learned": int(st[1]), "kept": int(st[2]), "rejected": [int(x) for x in st[3:7]]}


def tn_debug_rescale(x: np.ndarray):
    x = np.ascontiguousarray(x, dtype=np.float64).copy()
    e = C.c_int64(0)
    _check(LIB.tn_debug_rescale(_dptr(x), x.size, C.byref(e)))
    return x, int(e.value)


# ---------------------------------------------------------------- learned warm start

N_PARAMS = 8 * 32 + 32 + 32 * 32 + 32 + 32 + 1


class Model:
    """Owns a tn_model (the warm-start MLP on the device)."""

    def __init__(self, seed: int = 0):
        self.ptr = C.c_void_p()
        _check(LIB.tn_model_create(C.c_uint64(seed), C.byref(self.ptr)))

    def __del__(self):
        if getattr(self, "ptr", None):
            LIB.tn_model_destroy(self.ptr)
            self.ptr = None

    def set(self, w):
        w = np.ascontiguousarray(w, dtype=np.float32)
        _check(LIB.tn_model_set(self.ptr, w.ctypes.data_as(C.POINTER(C.c_float)), w.size))

    def get(self):
        w = np.zeros(N_PARAMS, dtype=np.float32)
        _check(LIB.tn_model_get(self.ptr, w.ctypes.data_as(C.POINTER(C.c_float)), N_PARAMS))
        return w

    def grad(self, X, y):
        X = np.ascontiguousarray(X, dtype=np.float32)
        y = np.ascontiguousarray(y, dtype=np.float32)
        g = np.zeros(N_PARAMS, dtype=np.float32)
        loss = C.c_double()
        fp = C.POINTER(C.c_float)
        _check(LIB.tn_model_grad(self.ptr, X.ctypes.data_as(fp), y.ctypes.data_as(fp), len(y), g.ctypes.data_as(fp),
                                 C.byref(loss)))
        return loss.value, g

    def train(self, ds, steps: int, batch: int = 128, lr: float = 3e-3, seed: int = 1) -> float:
        loss = C.c_double()
        _check(LIB.tn_model_train(self.ptr, ds.ptr, int(steps), int(batch), float(lr), C.c_uint64(seed),
                                  C.byref(loss)))
        return loss.value


class Dataset:
    """Owns a tn_dataset (harvested training rows on the device)."""

    def __init__(self, capacity: int):
        self.ptr = C.c_void_p()
        _check(LIB.tn_dataset_create(int(capacity), C.byref(self.ptr)))

    def __del__(self):
        if getattr(self, "ptr", None):
            LIB.tn_dataset_destroy(self.ptr)
            self.ptr = None

    def size(self) -> int:
        n = C.c_int64()
        _check(LIB.tn_dataset_size(self.ptr, C.byref(n)))
        return n.value

    def read(self):
        n = self.size()
        X = np.zeros((n, 8), dtype=np.float32)
        y = np.zeros(n, dtype=np.float32)
        fp = C.POINTER(C.c_float)
        _check(LIB.tn_dataset_read(self.ptr, X.ctypes.data_as(fp), y.ctypes.data_as(fp), n))
        return X, y


def tn_harvest(h: Handle, slices, max_rank: int, env_size: int, ds: Dataset) -> Result:
    p = _PathArgs(slices)
    r = tn_result()
    _check(LIB.tn_harvest(h.ptr, C.byref(p.path), int(max_rank), int(env_size), ds.ptr, C.byref(r)))
    return _result(r)


# ---------------------------------------------------------------- conveniences

def create_network(net) -> Handle:
    """tn_create on a paper_2406_09769_amd.inputs.Network."""
    return tn_create(net.tensors, net.edges)


def lnz(h: Handle, net, max_rank: int, env_size: int, **opt) -> Result:
    return tn_contract_approx(h, net.slices, max_rank, env_size, **opt)
