"""Python binding of libmpchol (include/mpchol.h): argument marshalling only.

Every step of the factorization and solve runs in the library's HIP kernels;
torch provides device memory and the stream.  There is no CPU fallback: if the
shared library is missing, importing this module raises.

Storage convention.  The C-ABI is column-major (LAPACK).  A column-major
``ld x n`` matrix is handed over as a contiguous float64 CUDA tensor of shape
``(n, ld)`` whose row j holds column j (i.e. the transpose view).  For a
symmetric input with ``ld == n`` that is the matrix itself; the factor comes back
in the same layout, so ``L_cm.T`` (a view) is the lower-triangular factor in
row-major indexing.  ``to_device_cm`` / ``from_device_cm`` convert between numpy
Fortran arrays and this layout.
"""
from __future__ import annotations

import ctypes as ct
import os
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np

E4M3, F16, F32, F64 = 0, 1, 2, 3
OK, NOT_SPD, NONFINITE, NOT_CONVERGED, HIP_ERROR, NOT_SUPPORTED = 0, 1, 2, 3, 4, 5
PROF_KINDS = ["gemm_e4m3", "gemm_f16", "gemm_f32", "gemm_f64", "cast", "maxabs", "potrf", "trsm",
              "trsv", "residual", "trinv"]
ABI_VERSION = 2
PREC_LABELS = {0: "E4M3", 1: "F16", 2: "F32", 3: "F64"}
MAX_LEVELS = 24

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmpchol.so")


class CTree(ct.Structure):
    _fields_ = [
        ("abi_version", ct.c_int32),
        ("leaf", ct.c_int32),
        ("split_align", ct.c_int32),
        ("nlevels", ct.c_int32),
        ("offdiag", ct.c_int32 * MAX_LEVELS),
        ("leaf_prec", ct.c_int32),
        ("syrk_leaf_mode", ct.c_int32),
        ("scale_mode", ct.c_int32),
        ("scale_tile", ct.c_int32),
        ("leaf_trsm", ct.c_int32),
        ("node_prec", ct.POINTER(ct.c_int8)),
        ("n_nodes", ct.c_int64),
    ]


class CInfo(ct.Structure):
    _fields_ = [
        ("status", ct.c_int32),
        ("ir_iters", ct.c_int32),
        ("failed_index", ct.c_int64),
        ("final_rel_corr", ct.c_double),
        ("ms_factor", ct.c_double),
        ("ms_solve", ct.c_double),
    ]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


class CTuneEntry(ct.Structure):
    _fields_ = [("nmax", ct.c_int32), ("leaf", ct.c_int32), ("split_align", ct.c_int32),
                ("tile", ct.c_int32)]


def _load() -> ct.CDLL:
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            f"{LIB_PATH} is missing: build it with paper_2601_08082_amd/build.py "
            "(hipcc, gfx950); there is no CPU fallback")
    # torch ships its own HIP runtime under the same soname; load it first so
    # that this library binds to the runtime that owns torch's allocations
    import torch  # noqa: F401
    lib = ct.CDLL(LIB_PATH)
    vp, i64, i32, dbl = ct.c_void_p, ct.c_int64, ct.c_int32, ct.c_double
    lib.mpchol_create.argtypes = [ct.POINTER(vp), ct.c_int]
    lib.mpchol_destroy.argtypes = [vp]
    lib.mpchol_factor.argtypes = [vp, i64, vp, i64, vp, i64, ct.POINTER(CTree), vp,
                                  ct.POINTER(CInfo)]
    lib.mpchol_solve.argtypes = [vp, i64, i64, vp, i64, vp, i64, vp, i64, vp, i64, dbl, i32, vp,
                                 ct.POINTER(CInfo)]
    lib.mpchol_trsm.argtypes = [vp, i64, i64, vp, i64, ct.POINTER(CTree), vp, ct.POINTER(CInfo)]
    lib.mpchol_syrk.argtypes = [vp, i64, i64, vp, i64, ct.POINTER(CTree), vp, ct.POINTER(CInfo)]
    lib.mpchol_solve_noalloc.argtypes = [ct.c_int, i64, i64, vp, i64, vp, i64, vp, i64, vp, i64,
                                         dbl, i32, vp, ct.POINTER(CInfo)]
    lib.mpchol_factor_batched.argtypes = [vp, i64, ct.POINTER(i64), ct.POINTER(vp),
                                          ct.POINTER(i64), ct.POINTER(vp), ct.POINTER(i64), i64,
                                          ct.POINTER(vp), ct.POINTER(vp), dbl, i32,
                                          ct.POINTER(CTree), vp, ct.POINTER(CInfo)]
    lib.mpchol_plan_stats.argtypes = [i64, i64, ct.POINTER(CTree), ct.POINTER(dbl),
                                      ct.POINTER(dbl), ct.POINTER(dbl), ct.POINTER(i64),
                                      ct.POINTER(i64)]
    lib.mpchol_quantize.argtypes = [vp, i64, i64, vp, i64, i32, i32, vp, i64,
                                    ct.POINTER(dbl), vp]
    lib.mpchol_set_tune_table.argtypes = [vp, i32, ct.POINTER(CTuneEntry)]
    lib.mpchol_profile.argtypes = [vp, ct.c_uint32]
    lib.mpchol_profile_read.argtypes = [vp, ct.POINTER(dbl), ct.POINTER(dbl), ct.POINTER(i64)]
    lib.mpchol_backward_error.argtypes = [vp, i64, vp, i64, vp, i64, ct.POINTER(dbl), vp]
    lib.mpchol_policy_nodes.argtypes = [i64, ct.POINTER(CTree), ct.POINTER(i64)]
    lib.mpchol_policy_nodes.restype = i64
    lib.mpchol_policy_features.argtypes = [vp, i64, vp, i64, ct.POINTER(CTree), vp, vp]
    lib.mpchol_policy_labels.argtypes = [vp, i64, vp, i64, vp, i64, ct.POINTER(CTree), dbl, i32,
                                         i32, vp, vp, vp]
    lib.mpchol_mlp_forward.argtypes = [vp, i64, vp, vp, vp, vp, vp]
    lib.mpchol_mlp_train_step.argtypes = [vp, i64, vp, vp, vp, vp, vp, i32, ct.c_float, vp, vp,
                                          vp]
    lib.mpchol_policy_choose.argtypes = [vp, i64, vp, i64, ct.POINTER(CTree), vp,
                                         ct.POINTER(ct.c_int8), vp]
    lib.mpchol_version.restype = ct.c_char_p
    return lib


lib = _load()


@dataclass
class Tree:
    """Precision-tree descriptor (see include/mpchol.h, mpchol_tree)."""
    leaf: int = 64
    offdiag: Sequence[int] = (F16,)
    leaf_prec: int = F64
    split_align: int = 1
    syrk_leaf_mode: int = 0
    scale_mode: int = 0
    node_prec: Optional[Sequence[int]] = None
    leaf_trsm: int = 0          # 0: FP64 leaf TRSM through the leaf inverse; 1: substitution

    def to_c(self):
        t = CTree()
        t.abi_version = ABI_VERSION
        t.leaf = self.leaf
        t.split_align = self.split_align
        t.nlevels = len(self.offdiag)
        for i, p in enumerate(self.offdiag):
            t.offdiag[i] = p
        t.leaf_prec = self.leaf_prec
        t.syrk_leaf_mode = self.syrk_leaf_mode
        t.scale_mode = self.scale_mode
        t.scale_tile = 0
        t.leaf_trsm = self.leaf_trsm
        keep = None
        if self.node_prec is not None and len(self.node_prec):
            keep = (ct.c_int8 * len(self.node_prec))(*self.node_prec)
            t.node_prec = ct.cast(keep, ct.POINTER(ct.c_int8))
            t.n_nodes = len(self.node_prec)
        else:
            t.node_prec = None
            t.n_nodes = 0
        return t, keep


def _stream_handle(stream) -> Optional[int]:
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream


def _ptr(t) -> Optional[int]:
    return None if t is None else t.data_ptr()


def _check_cm(t, name: str):
    import torch
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64
            and t.dim() == 2 and t.is_contiguous()):
        raise TypeError(f"{name} must be a contiguous float64 CUDA tensor of shape (n, ld)")


def to_device_cm(M: np.ndarray, device="cuda"):
    """numpy Fortran array (ld x n) -> device tensor (n, ld) (column-major storage)."""
    import torch
    M = np.asfortranarray(M, dtype=np.float64)
    return torch.from_numpy(np.ascontiguousarray(M.T)).to(device)


def from_device_cm(T) -> np.ndarray:
    """device tensor (n, ld) -> numpy Fortran array (ld x n)."""
    return np.asfortranarray(T.detach().cpu().numpy().T)


def plan_stats(n: int, tree: Tree, ldl: Optional[int] = None) -> dict:
    """Host-only plan introspection: flops by precision, launches, workspace."""
    t, keep = tree.to_c()
    f4 = (ct.c_double * 4)()
    lf, cb = ct.c_double(), ct.c_double()
    nl, ws = ct.c_int64(), ct.c_int64()
    r = lib.mpchol_plan_stats(n, ldl or max(1, n), ct.byref(t), f4, ct.byref(lf), ct.byref(cb),
                              ct.byref(nl), ct.byref(ws))
    if r != 0:
        raise ValueError(f"mpchol_plan_stats returned {r}")
    return {"flops": {"E4M3": f4[0], "F16": f4[1], "F32": f4[2], "F64": f4[3]},
            "leaf_flops": lf.value, "cast_bytes": cb.value, "launches": nl.value,
            "ws_bytes": ws.value}


class Context:
    """Owns an mpchol_ctx (plans, workspace, status words) on one device."""

    def __init__(self, device: int = 0):
        self._h = ct.c_void_p()
        r = lib.mpchol_create(ct.byref(self._h), device)
        if r != 0:
            raise RuntimeError(f"mpchol_create failed ({r})")

    def close(self):
        if self._h:
            lib.mpchol_destroy(self._h)
            self._h = ct.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def factor(self, A_cm, n: int, tree: Tree, L_cm=None, stream=None, sync: bool = True):
        """Factor; returns (L_cm, info dict or None).  L_cm may be A_cm (in place)."""
        import torch
        _check_cm(A_cm, "A")
        lda = A_cm.shape[1]
        if L_cm is None:
            L_cm = torch.zeros_like(A_cm)
        _check_cm(L_cm, "L")
        t, keep = tree.to_c()
        info = CInfo()
        r = lib.mpchol_factor(self._h, n, _ptr(A_cm), lda, _ptr(L_cm), L_cm.shape[1],
                              ct.byref(t), _stream_handle(stream),
                              ct.byref(info) if sync else None)
        if r < 0:
            raise ValueError(f"mpchol_factor: invalid argument {-r}")
        if r == HIP_ERROR:
            raise RuntimeError("mpchol_factor: HIP error")
        if r == NOT_SUPPORTED:
            raise NotImplementedError("mpchol_factor: descriptor feature not supported")
        return L_cm, (info.as_dict() if sync else None)

    def solve(self, L_cm, B_cm, n: int, A_cm=None, tol: float = 1e-13, max_iter: int = 20,
              X_cm=None, stream=None):
        """Solve (+ refinement when A_cm is given); returns (X_cm, info dict)."""
        import torch
        _check_cm(L_cm, "L")
        _check_cm(B_cm, "B")
        if A_cm is not None:
            _check_cm(A_cm, "A")
        nrhs = B_cm.shape[0]
        if X_cm is None:
            X_cm = torch.zeros_like(B_cm)
        _check_cm(X_cm, "X")
        info = CInfo()
        r = lib.mpchol_solve(self._h, n, nrhs, _ptr(A_cm),
                             A_cm.shape[1] if A_cm is not None else max(1, n),
                             _ptr(L_cm), L_cm.shape[1], _ptr(B_cm), B_cm.shape[1], _ptr(X_cm),
                             X_cm.shape[1], tol, max_iter, _stream_handle(stream),
                             ct.byref(info))
        if r < 0:
            raise ValueError(f"mpchol_solve: invalid argument {-r}")
        if r == HIP_ERROR:
            raise RuntimeError("mpchol_solve: HIP error")
        return X_cm, info.as_dict()

    def _sub(self, fn, name, A_cm, a: int, k: int, tree: Tree, stream, sync: bool):
        _check_cm(A_cm, "A")
        t, keep = tree.to_c()
        info = CInfo()
        r = fn(self._h, a, k, _ptr(A_cm), A_cm.shape[1], ct.byref(t), _stream_handle(stream),
               ct.byref(info) if sync else None)
        if r < 0:
            raise ValueError(f"{name}: invalid argument {-r}")
        if r == HIP_ERROR:
            raise RuntimeError(f"{name}: HIP error")
        if r == NOT_SUPPORTED:
            raise NotImplementedError(f"{name}: descriptor feature not supported")
        return info.as_dict() if sync else None

    def trsm(self, A_cm, m: int, k: int, tree: Tree, stream=None, sync: bool = True):
        """Tree-TRSM in place on blocks of A: A[k:k+m, :k] <- A[k:k+m, :k] L^-T with
        L the lower triangle of A[:k, :k] (indices in the column-major matrix)."""
        return self._sub(lib.mpchol_trsm, "mpchol_trsm", A_cm, m, k, tree, stream, sync)

    def syrk(self, A_cm, n: int, k: int, tree: Tree, stream=None, sync: bool = True):
        """Tree-SYRK in place on blocks of A: lower A[k:k+n, k:k+n] -=
        A[k:k+n, :k] A[k:k+n, :k]^T."""
        return self._sub(lib.mpchol_syrk, "mpchol_syrk", A_cm, n, k, tree, stream, sync)

    def quantize(self, X_cm, rows: int, cols: int, prec: int, scale_mode: int = 0,
                 stream=None):
        """Quantize a column-major block; returns (codes uint16/uint8 tensor of
        shape (rows, ldq), scale, status)."""
        import torch
        _check_cm(X_cm, "X")
        ldq = max(16, (cols + 15) // 16 * 16)
        dt = torch.int16 if prec == F16 else torch.uint8
        out = torch.zeros((max(rows, 1), ldq), dtype=dt, device=X_cm.device)
        sc = ct.c_double(0.0)
        r = lib.mpchol_quantize(self._h, rows, cols, _ptr(X_cm), X_cm.shape[1], prec, scale_mode,
                                _ptr(out), ldq, ct.byref(sc), _stream_handle(stream))
        if r < 0:
            raise ValueError(f"mpchol_quantize: invalid argument {-r}")
        if r == HIP_ERROR:
            raise RuntimeError("mpchol_quantize: HIP error")
        return out, sc.value, r

    def profile(self, kinds: Sequence[str]):
        """Time every later launch of the given classes with HIP events."""
        mask = 0
        for k in kinds:
            mask |= 1 << PROF_KINDS.index(k)
        if lib.mpchol_profile(self._h, mask) != 0:
            raise RuntimeError("mpchol_profile failed")

    def profile_read(self) -> dict:
        """{class: (ms, work, launches)} accumulated since profile()."""
        n = len(PROF_KINDS)
        ms, wk, nl = (ct.c_double * n)(), (ct.c_double * n)(), (ct.c_int64 * n)()
        if lib.mpchol_profile_read(self._h, ms, wk, nl) != 0:
            raise RuntimeError("mpchol_profile_read failed")
        return {k: (ms[i], wk[i], nl[i]) for i, k in enumerate(PROF_KINDS)}

    def backward_error(self, A_cm, L_cm, n: int, stream=None):
        """(||A - L L^T||_F / ||A||_F, ||A - L L^T||_F, ||A||_F) computed on the device."""
        out = (ct.c_double * 2)()
        r = lib.mpchol_backward_error(self._h, n, _ptr(A_cm), A_cm.shape[1], _ptr(L_cm),
                                      L_cm.shape[1], out, _stream_handle(stream))
        _raise(r, "mpchol_backward_error")
        return (out[0] / out[1] if out[1] > 0 else 0.0), out[0], out[1]

    # ------------------------------------------------------------ learned policy
    def policy_features(self, A_cm, n: int, tree: Tree, stream=None):
        """(nodes, MLP_IN) float32 device tensor of per-node features."""
        import torch
        _check_cm(A_cm, "A")
        nn = policy_nodes(n, tree).shape[0]
        feat = torch.empty((max(nn, 1), MLP_IN), dtype=torch.float32, device=A_cm.device)
        t, keep = tree.to_c()
        r = lib.mpchol_policy_features(self._h, n, _ptr(A_cm), A_cm.shape[1], ct.byref(t),
                                       feat.data_ptr(), _stream_handle(stream))
        _raise(r, "mpchol_policy_features")
        return feat[:nn]

    def policy_labels(self, A_cm, L_cm, n: int, tree: Tree, tau: float = 1e-4,
                      scale_mode: int = 1, min_prec: int = E4M3, stream=None):
        """(labels int32 (nodes,), errors float64 (nodes, 3)) device tensors."""
        import torch
        nn = policy_nodes(n, tree).shape[0]
        lab = torch.empty(max(nn, 1), dtype=torch.int32, device=A_cm.device)
        err = torch.empty((max(nn, 1), 3), dtype=torch.float64, device=A_cm.device)
        t, keep = tree.to_c()
        r = lib.mpchol_policy_labels(self._h, n, _ptr(A_cm), A_cm.shape[1], _ptr(L_cm),
                                     L_cm.shape[1], ct.byref(t), tau, scale_mode, min_prec,
                                     err.data_ptr(), lab.data_ptr(), _stream_handle(stream))
        _raise(r, "mpchol_policy_labels")
        return lab[:nn], err[:nn]

    def mlp_forward(self, X, params, stream=None):
        """(probs (rows, 4), classes (rows,)) for float32 features X (rows, MLP_IN)."""
        import torch
        rows = X.shape[0]
        probs = torch.empty((max(rows, 1), MLP_OUT), dtype=torch.float32, device=X.device)
        cls = torch.empty(max(rows, 1), dtype=torch.int32, device=X.device)
        r = lib.mpchol_mlp_forward(self._h, rows, X.data_ptr(), params.data_ptr(),
                                   probs.data_ptr(), cls.data_ptr(), _stream_handle(stream))
        _raise(r, "mpchol_mlp_forward")
        return probs[:rows], cls[:rows]

    def mlp_train_step(self, X, y, params, m, v, step: int, lr: float, want_grad: bool = False,
                       stream=None):
        """One gradient (+ Adam when lr > 0) step in place on params/m/v;
        returns (loss tensor (1,), grad tensor or None)."""
        import torch
        loss = torch.empty(1, dtype=torch.float32, device=X.device)
        grad = torch.empty(MLP_PARAMS, dtype=torch.float32, device=X.device) if want_grad else None
        r = lib.mpchol_mlp_train_step(self._h, X.shape[0], X.data_ptr(), y.data_ptr(),
                                      params.data_ptr(), m.data_ptr() if m is not None else None,
                                      v.data_ptr() if v is not None else None, step, lr,
                                      loss.data_ptr(), grad.data_ptr() if want_grad else None,
                                      _stream_handle(stream))
        _raise(r, "mpchol_mlp_train_step")
        return loss, grad

    def policy_choose(self, A_cm, n: int, tree: Tree, params, stream=None) -> list:
        """Per-node precisions chosen by the perceptron (preorder node list)."""
        nn = policy_nodes(n, tree).shape[0]
        out = (ct.c_int8 * max(nn, 1))()
        t, keep = tree.to_c()
        r = lib.mpchol_policy_choose(self._h, n, _ptr(A_cm), A_cm.shape[1], ct.byref(t),
                                     params.data_ptr(), out, _stream_handle(stream))
        _raise(r, "mpchol_policy_choose")
        return [int(out[i]) for i in range(nn)]

    def set_tune_table(self, entries):
        """Per-size plan choices for factor_batched: a list of
        (nmax, leaf, split_align, tile) tuples (0 = the descriptor's / automatic),
        nmax strictly increasing; [] clears the table."""
        k = len(entries)
        arr = (CTuneEntry * max(k, 1))(*[CTuneEntry(*map(int, e)) for e in entries])
        r = lib.mpchol_set_tune_table(self._h, k, arr)
        if r != 0:
            raise ValueError(f"mpchol_set_tune_table: invalid argument {-r}")

    def load_tune_table(self, path: str):
        """Install a table written by the autotuner (JSON)."""
        import json
        with open(path) as f:
            tab = json.load(f)
        self.set_tune_table([(e["nmax"], e["leaf"], e.get("split_align", 0), e.get("tile", 0))
                             for e in tab["entries"]])

    def factor_batched(self, A_list, L_list, ns, tree: Tree, B_list=None, X_list=None,
                       tol: float = 1e-13, max_iter: int = 20, stream=None):
        """Factor (+ solve and refine when B_list/X_list are given) independent
        systems in one persistent launch; returns (worst status, info dicts).
        B_i / X_i: tensors of shape (nrhs, n_i) (column-major n_i x nrhs)."""
        batch = len(A_list)
        nrhs = B_list[0].shape[0] if B_list else 0
        n_arr = (ct.c_int64 * batch)(*ns)
        lda = (ct.c_int64 * batch)(*[a.shape[1] for a in A_list])
        ldl = (ct.c_int64 * batch)(*[l.shape[1] for l in L_list])
        Ap = (ct.c_void_p * batch)(*[a.data_ptr() for a in A_list])
        Lp = (ct.c_void_p * batch)(*[l.data_ptr() for l in L_list])
        Bp = (ct.c_void_p * batch)(*[b.data_ptr() for b in B_list]) if B_list else None
        Xp = (ct.c_void_p * batch)(*[x.data_ptr() for x in X_list]) if X_list else None
        infos = (CInfo * batch)()
        t, keep = tree.to_c()
        r = lib.mpchol_factor_batched(self._h, batch, n_arr, Ap, lda, Lp, ldl, nrhs, Bp, Xp, tol,
                                      max_iter, ct.byref(t), _stream_handle(stream), infos)
        if r < 0:
            raise ValueError(f"mpchol_factor_batched: invalid argument {-r}")
        if r == HIP_ERROR:
            raise RuntimeError("mpchol_factor_batched: HIP error")
        return r, [infos[i].as_dict() for i in range(batch)]


MLP_IN, MLP_H, MLP_OUT = 6, 64, 4
MLP_PARAMS = 4880


NOALLOC_MAX_N = 16384
NOALLOC_MAX_RHS = 16


def solve_noalloc(L_cm, B_cm, n: int, A_cm=None, tol: float = 1e-13, max_iter: int = 20,
                  X_cm=None, device: int = 0, stream=None):
    """mpchol_solve_noalloc: the solve + refinement of Context.solve on the
    library's fixed per-GPU scratch (n <= NOALLOC_MAX_N, nrhs <=
    NOALLOC_MAX_RHS); returns (X_cm, info dict).  X_cm must be given by a
    caller that cannot allocate."""
    import torch
    _check_cm(L_cm, "L")
    _check_cm(B_cm, "B")
    if A_cm is not None:
        _check_cm(A_cm, "A")
    nrhs = B_cm.shape[0]
    if X_cm is None:
        X_cm = torch.zeros_like(B_cm)
    _check_cm(X_cm, "X")
    info = CInfo()
    r = lib.mpchol_solve_noalloc(device, n, nrhs, _ptr(A_cm),
                                 A_cm.shape[1] if A_cm is not None else max(1, n),
                                 _ptr(L_cm), L_cm.shape[1], _ptr(B_cm), B_cm.shape[1],
                                 _ptr(X_cm), X_cm.shape[1], tol, max_iter,
                                 _stream_handle(stream), ct.byref(info))
    if r < 0:
        raise ValueError(f"mpchol_solve_noalloc: invalid argument {-r}")
    if r == HIP_ERROR:
        raise RuntimeError("mpchol_solve_noalloc: HIP error")
    return X_cm, info.as_dict()


def _raise(r: int, name: str):
    if r < 0:
        raise ValueError(f"{name}: invalid argument {-r}")
    if r == HIP_ERROR:
        raise RuntimeError(f"{name}: HIP error")
    if r != 0:
        raise RuntimeError(f"{name}: status {r}")


def policy_nodes(n: int, tree: Tree):
    """(nodes, 4) int64 array: i0, m, m1, depth of each internal node (preorder)."""
    t, keep = tree.to_c()
    k = lib.mpchol_policy_nodes(n, ct.byref(t), None)
    if k < 0:
        raise ValueError(f"mpchol_policy_nodes: invalid argument {-k}")
    tab = (ct.c_int64 * max(4 * k, 1))()
    lib.mpchol_policy_nodes(n, ct.byref(t), tab)
    return np.array(tab[:4 * k], dtype=np.int64).reshape(k, 4)


def version() -> str:
    return lib.mpchol_version().decode()
