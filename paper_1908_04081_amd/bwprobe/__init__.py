"""ctypes binding of the bandwidth probes (bwprobe.h): the streaming read,
streaming copy and cache-resident read ceilings that the solver's kernels
are measured against.  Buffers are torch CUDA tensors."""
from __future__ import annotations

import ctypes as C
import os

_DIR = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_DIR, "libassg_bwprobe.so")
PIECE = 32768
_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} not built (python -m paper_1908_04081_amd.build)")
        L = C.CDLL(LIB_PATH)
        L.assg_bw_read.restype = C.c_int
        L.assg_bw_read.argtypes = [C.c_void_p, C.c_size_t, C.c_int, C.c_int, C.c_void_p,
                                   C.POINTER(C.c_float)]
        L.assg_bw_copy.restype = C.c_int
        L.assg_bw_copy.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t, C.c_int,
                                   C.POINTER(C.c_float)]
        _lib = L
    return _lib


def read_gbps(buf, nontemporal=True, iters=20, partial=None) -> tuple[float, float]:
    """(GB/s, ms per pass) of reading the whole tensor ``buf`` (its size a
    multiple of 32 KiB)."""
    import torch
    nbytes = buf.numel() * buf.element_size()
    if partial is None:
        partial = torch.empty(nbytes // PIECE, dtype=torch.float64, device=buf.device)
    ms = C.c_float()
    rc = lib().assg_bw_read(C.c_void_p(buf.data_ptr()), nbytes, int(nontemporal), iters,
                            C.c_void_p(partial.data_ptr()), C.byref(ms))
    if rc != 0:
        raise RuntimeError(f"assg_bw_read failed ({rc})")
    return nbytes / (ms.value * 1e-3) / 1e9, ms.value


def copy_gbps(src, dst, iters=20) -> tuple[float, float]:
    """(GB/s counting read + write bytes, ms per pass) of copying src to dst."""
    nbytes = src.numel() * src.element_size()
    assert dst.numel() * dst.element_size() >= nbytes
    ms = C.c_float()
    rc = lib().assg_bw_copy(C.c_void_p(src.data_ptr()), C.c_void_p(dst.data_ptr()), nbytes,
                            iters, C.byref(ms))
    if rc != 0:
        raise RuntimeError(f"assg_bw_copy failed ({rc})")
    return 2 * nbytes / (ms.value * 1e-3) / 1e9, ms.value
