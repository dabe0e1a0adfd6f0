"""GPU fill for the seeded input generator (libspdgen.so, csrc/spdgen.hip).

Same definition as ``spdgen.py`` (bitwise-identical output); used to create
large inputs directly in device memory.  Input generation only.
"""
from __future__ import annotations

import ctypes as ct
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libspdgen.so")


def _load():
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build with paper_2601_08082_amd/build.py")
    # torch ships its own HIP runtime under the same soname; load it first so
    # that this library binds to the runtime that owns torch's allocations
    import torch  # noqa: F401
    lib = ct.CDLL(LIB_PATH)
    lib.spdgen_fill.argtypes = [ct.c_int64, ct.c_int64, ct.c_double, ct.c_double, ct.c_uint64,
                                ct.c_void_p, ct.c_void_p]
    lib.spdgen_kernel_fill.argtypes = [ct.c_int64, ct.c_int64, ct.c_double, ct.c_double,
                                       ct.c_uint64, ct.c_void_p, ct.c_void_p]
    lib.spdgen_rhs.argtypes = [ct.c_int64, ct.c_int64, ct.c_int64, ct.c_uint64, ct.c_void_p,
                               ct.c_void_p]
    return lib


_lib = None


def _get():
    global _lib
    if _lib is None:
        _lib = _load()
    return _lib


def gen_spd(n: int, ratio: float, shift: float = 0.0, seed: int = 1, lda: int | None = None,
            device="cuda"):
    """Device tensor (n, lda): column-major storage of the generator's matrix."""
    import torch
    lda = n if lda is None else lda
    A = torch.empty((max(n, 1), lda), dtype=torch.float64, device=device)
    r = _get().spdgen_fill(n, lda, ratio, shift, seed, A.data_ptr(),
                           torch.cuda.current_stream().cuda_stream)
    if r != 0:
        raise RuntimeError(f"spdgen_fill failed ({r})")
    return A


def gen_kernel(n: int, ell: float, nugget: float, seed: int = 1, lda: int | None = None,
               device="cuda"):
    """Device tensor (n, lda): the squared-exponential kernel matrix plus nugget."""
    import torch
    lda = n if lda is None else lda
    A = torch.empty((max(n, 1), lda), dtype=torch.float64, device=device)
    r = _get().spdgen_kernel_fill(n, lda, ell, nugget, seed, A.data_ptr(),
                                  torch.cuda.current_stream().cuda_stream)
    if r != 0:
        raise RuntimeError(f"spdgen_kernel_fill failed ({r})")
    return A


def gen_rhs(n: int, nrhs: int, seed: int = 101, ldb: int | None = None, device="cuda"):
    import torch
    ldb = n if ldb is None else ldb
    B = torch.empty((max(nrhs, 1), ldb), dtype=torch.float64, device=device)
    r = _get().spdgen_rhs(n, nrhs, ldb, seed, B.data_ptr(), torch.cuda.current_stream().cuda_stream)
    if r != 0:
        raise RuntimeError(f"spdgen_rhs failed ({r})")
    return B
