"""The paper's CPU method (batched B = 8 CLT H.x with OpenMP, Sec. 2,
"Computational setup") for the CPU baseline only -- TEST INFRASTRUCTURE,
not one of the oracle's definitions (paper_cpu.c)."""
import ctypes

import numpy as np

from . import lib as _lib_base, _ptr, _bonds

B = 8


def hv_clt_b8(bonds, basis_arr, mask, prefix, x, row0=0, nrows=None):
    """Rows [row0, row0 + nrows) of H x for the 8 columns of x [D][8] (FP64)."""
    L = _lib_base()
    vp, u64, i32 = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int
    L.pcpu_hv_clt_b8.restype = None
    L.pcpu_hv_clt_b8.argtypes = [i32, vp, vp, vp, vp, vp, vp, vp, vp, u64, u64]
    bi, bj, J = _bonds(bonds)
    x = np.ascontiguousarray(x, dtype=np.float64)
    assert x.ndim == 2 and x.shape[1] == B
    nrows = x.shape[0] - row0 if nrows is None else nrows
    y = np.empty((nrows, B), dtype=np.float64)
    L.pcpu_hv_clt_b8(len(bonds), _ptr(bi), _ptr(bj), _ptr(J), _ptr(basis_arr), _ptr(mask), _ptr(prefix), _ptr(x),
                     _ptr(y), row0, nrows)
    return y
