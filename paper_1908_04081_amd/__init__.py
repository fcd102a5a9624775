"""Python binding of libassg (adaptive s-step CG for MI355X / gfx950).

Argument marshalling only: every step of a solve runs in the library's HIP
kernels.  Functions carry the names of the C entry points in
``include/assg.h``; device arrays are torch CUDA tensors (float64 vectors,
int32/float64 CSR arrays) passed by pointer, torch's current stream orders
the library's work.  A missing library is an error, never a fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libassg.so")
# the same sources built with -DASSG_DEBUG (index checks in the kernels)
DEBUG_LIB_PATH = os.path.join(_PKG, "libassg_debug.so")

MAX_S = 16
MAX_COLS = 2 * MAX_S + 1

OK, ERR_INVALID_ARG, ERR_HIP, ERR_ALLOC, ERR_UNSUPPORTED, ERR_NOT_ANALYZED = 0, -1, -2, -3, -4, -5
CONVERGED, STAGNATED, DIVERGED, BREAKDOWN, MAX_ITER, RUNNING = 0, 1, 2, 3, 4, 5
OUTCOME_NAMES = {0: "CONVERGED", 1: "STAGNATED", 2: "DIVERGED", 3: "BREAKDOWN", 4: "MAX_ITER",
                 5: "RUNNING"}
BASIS = {"monomial": 0, "newton": 1, "chebyshev": 2}
VARIANT = {"improved": 0, "improved_c_ratio": 1, "improved_c_one": 2, "old": 3, "fixed": 4}
FORMAT = {"auto": 0, "csr": 1, "dia": 2}
FORMAT_NAMES = {v: k for k, v in FORMAT.items()}


class AssgCsr(C.Structure):
    _fields_ = [("n", C.c_int64), ("nnz", C.c_int64), ("row_ptr", C.c_void_p),
                ("col_idx", C.c_void_p), ("val", C.c_void_p)]


class AssgOpts(C.Structure):
    _fields_ = [("s_max", C.c_int32), ("s_init", C.c_int32), ("growth", C.c_int32),
                ("basis", C.c_int32), ("tol", C.c_double), ("max_outer", C.c_int64),
                ("max_iters", C.c_int64), ("record_trace", C.c_int32),
                ("time_kernels", C.c_int32), ("variant", C.c_int32), ("pad0", C.c_int32),
                ("c_const", C.c_double)]


class AssgInfo(C.Structure):
    _fields_ = [("outcome", C.c_int32), ("pad0", C.c_int32), ("outer_iters", C.c_int64),
                ("total_iters", C.c_int64), ("relres_updated", C.c_double),
                ("relres_true", C.c_double), ("lambda_min_est", C.c_double),
                ("lambda_max_est", C.c_double), ("c_last", C.c_double),
                ("solve_ms", C.c_double), ("sweep_ms", C.c_double),
                ("sweep_launches", C.c_int64), ("sweep1_ms", C.c_double),
                ("sweep1_launches", C.c_int64), ("last_gram_ms", C.c_double),
                ("last_gram_launches", C.c_int64), ("other_ms", C.c_double)]


class AssgTrace(C.Structure):
    _fields_ = [("k", C.c_int32), ("sbar", C.c_int32), ("stilde", C.c_int32), ("sk", C.c_int32),
                ("m", C.c_int64), ("candidate", C.c_int32), ("flags", C.c_int32),
                ("c_in", C.c_double), ("thr", C.c_double), ("rho_m", C.c_double),
                ("phi", C.c_double), ("c", C.c_double), ("lmin", C.c_double),
                ("lmax", C.c_double), ("psi", C.c_double), ("relres_updated", C.c_double),
                ("relres_true", C.c_double), ("kappa", C.c_double * MAX_S)]


class AssgBlockState(C.Structure):
    _fields_ = [("m", C.c_int64), ("c", C.c_double), ("psi", C.c_double),
                ("alpha_prev", C.c_double), ("beta_prev", C.c_double),
                ("mt_max_omega", C.c_double), ("mt_max_h", C.c_double),
                ("mt_max_zeta", C.c_double), ("mt_min_omega", C.c_double),
                ("mt_min_a", C.c_double), ("mt_min_d", C.c_double), ("mt_min_g", C.c_double),
                ("mt_min_h", C.c_double), ("lmin", C.c_double), ("lmax", C.c_double),
                ("theta", C.c_double * MAX_S), ("gamma", C.c_double * MAX_S),
                ("mu", C.c_double * MAX_S)]


class AssgBlockResult(C.Structure):
    _fields_ = [("stilde", C.c_int32), ("sk", C.c_int32), ("candidate", C.c_int32),
                ("flags", C.c_int32), ("thr", C.c_double), ("rho_m", C.c_double),
                ("phi", C.c_double), ("relres_updated", C.c_double),
                ("kappa", C.c_double * MAX_S), ("alpha", C.c_double * MAX_S),
                ("beta", C.c_double * MAX_S), ("coef_x", C.c_double * MAX_COLS),
                ("coef_r", C.c_double * MAX_COLS), ("coef_p", C.c_double * MAX_COLS)]


TUNE_CLASSES = 4
TUNE_SHAPES = [(256, 2048), (256, 1024), (128, 2048), (128, 1024), (64, 1024), (64, 512)]


class AssgTuneClass(C.Structure):
    _fields_ = [("systems", C.c_int32), ("rows", C.c_int32), ("nnz_cap", C.c_int32),
                ("cached", C.c_int32), ("candidate_us", C.c_double * len(TUNE_SHAPES))]


_STRUCTS = [AssgOpts, AssgInfo, AssgTrace, AssgBlockState, AssgBlockResult, AssgCsr, AssgTuneClass]

EXPORTS = [
    "assg_default_opts", "assg_status_string", "assg_last_error", "assg_struct_sizes",
    "assg_create", "assg_destroy", "assg_set_stream", "assg_basis_params",
    "assg_workspace_size", "assg_analyze", "assg_solve", "assg_hscg_solve", "assg_get_trace",
    "assg_spmv", "assg_basis_gram", "assg_block_controller", "assg_solve_forced_schedule",
    "assg_solve_noalloc", "assg_set_format", "assg_get_format",
]

_lib = None


def load(path: str = LIB_PATH):
    """Loads the library at ``path`` (LIB_PATH, or DEBUG_LIB_PATH for the
    build with kernel index checks) for this process; must come before the
    first call.  Returns the library."""
    global _lib
    if _lib is not None:
        if getattr(_lib, "_path", None) == path:
            return _lib
        raise RuntimeError(f"another library is already loaded ({_lib._path})")
    if not os.path.exists(path):
        raise RuntimeError(f"{os.path.basename(path)} not found at {path}: build it with "
                           "`python -m paper_1908_04081_amd.build` (no CPU fallback exists)")
    L = C.CDLL(path)
    L._path = path
    P, I32, I64, D = C.c_void_p, C.c_int32, C.c_int64, C.c_double
    sig = {
        "assg_default_opts": (I32, [C.POINTER(AssgOpts)]),
        "assg_status_string": (C.c_char_p, [I32]),
        "assg_last_error": (C.c_char_p, [P]),
        "assg_struct_sizes": (I32, [C.POINTER(C.c_int64), I32]),
        "assg_create": (I32, [C.POINTER(C.c_void_p), P]),
        "assg_destroy": (I32, [P]),
        "assg_set_stream": (I32, [P, P]),
        "assg_basis_params": (I32, [I32, D, D, I32, C.POINTER(D), C.POINTER(D), C.POINTER(D)]),
        "assg_workspace_size": (I32, [I64, I32, C.POINTER(C.c_size_t)]),
        "assg_analyze": (I32, [P, C.POINTER(AssgCsr)]),
        "assg_set_format": (I32, [P, I32]),
        "assg_get_format": (I32, [P, C.POINTER(I32)]),
        "assg_batch_format": (I32, [P, C.POINTER(I32)]),
        "assg_solve": (I32, [P, C.POINTER(AssgCsr), P, P, C.POINTER(AssgOpts), P, C.c_size_t,
                             C.POINTER(AssgInfo)]),
        "assg_solve_noalloc": (I32, [P, C.POINTER(AssgCsr), P, P, C.POINTER(AssgOpts),
                                     C.POINTER(AssgInfo)]),
        "assg_solve_forced_schedule": (I32, [P, C.POINTER(AssgCsr), P, P, C.POINTER(AssgOpts),
                                             C.POINTER(I32), I64, P, C.c_size_t,
                                             C.POINTER(AssgInfo)]),
        "assg_hscg_solve": (I32, [P, C.POINTER(AssgCsr), P, P, D, I64, P, C.c_size_t,
                                  C.POINTER(AssgInfo)]),
        "assg_get_trace": (I32, [P, C.POINTER(AssgTrace), I64, C.POINTER(C.c_int64)]),
        "assg_spmv": (I32, [P, C.POINTER(AssgCsr), P, P]),
        "assg_csr_outer_on_pattern": (I32, [P, C.POINTER(AssgCsr), P, P, D, P]),
        "assg_batch_analyze": (I32, [P, I32, C.POINTER(AssgCsr)]),
        "assg_batch_solve": (I32, [P, I32, C.POINTER(AssgCsr), C.POINTER(C.c_void_p),
                                   C.POINTER(C.c_void_p), C.POINTER(AssgOpts),
                                   C.POINTER(AssgInfo)]),
        "assg_batch_tuning": (I32, [P, C.POINTER(AssgTuneClass)]),
        "assg_basis_gram": (I32, [P, C.POINTER(AssgCsr), P, P, I32, C.POINTER(D), C.POINTER(D),
                                  C.POINTER(D), P, C.POINTER(D)]),
        "assg_block_controller": (I32, [P, C.POINTER(D), I32, D, D, I32, I32,
                                        C.POINTER(AssgBlockState), C.POINTER(AssgBlockResult)]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    sizes = (C.c_int64 * len(_STRUCTS))()
    L.assg_struct_sizes(sizes, len(_STRUCTS))
    for st, sz in zip(_STRUCTS, sizes):
        if C.sizeof(st) != sz:
            raise RuntimeError(f"ABI mismatch: {st.__name__} is {C.sizeof(st)} bytes here, "
                               f"{sz} in the library")
    _lib = L
    return L


def lib():
    """The loaded library (libassg.so unless load() chose another); raises if
    it has not been built."""
    return _lib if _lib is not None else load(LIB_PATH)


class AssgError(RuntimeError):
    pass


def _check(st, h=None):
    if st != OK:
        L = lib()
        msg = L.assg_status_string(st).decode()
        detail = L.assg_last_error(h).decode() if h else ""
        raise AssgError(f"{msg} ({st}): {detail}")


def _dptr(t, numel=None, dtype=None, what="tensor"):
    """Device pointer of a contiguous CUDA tensor; with ``numel``/``dtype``
    also checks the element count and type the C ABI will assume (a wrong
    size would make the kernels read or write past the buffer)."""
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{what}: expected a CUDA tensor")
    if not t.is_contiguous():
        raise ValueError(f"{what}: tensor must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{what}: expected {dtype}, got {t.dtype}")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{what}: expected {numel} elements, got {t.numel()}")
    return C.c_void_p(t.data_ptr())


def _f64(t, numel, what):
    import torch
    return _dptr(t, numel, torch.float64, what)


def _stream_ptr():
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


# ----------------------------------------------------------------- host-only
def assg_default_opts(**overrides) -> AssgOpts:
    """The library's default options with the given fields replaced; an
    unknown field name raises TypeError (a typo would otherwise be ignored)."""
    o = AssgOpts()
    _check(lib().assg_default_opts(C.byref(o)))
    names = {f for f, _ in AssgOpts._fields_ if not f.startswith("pad")}
    for k, v in overrides.items():
        if k not in names:
            raise TypeError(f"unknown option {k!r}; options: {sorted(names)}")
        if k == "basis" and isinstance(v, str):
            v = BASIS[v]
        if k == "variant" and isinstance(v, str):
            v = VARIANT[v]
        setattr(o, k, v)
    return o


def assg_basis_params(kind, lmin: float, lmax: float, s: int):
    if isinstance(kind, str):
        kind = BASIS[kind]
    th = (C.c_double * MAX_S)(); ga = (C.c_double * MAX_S)(); mu = (C.c_double * MAX_S)()
    _check(lib().assg_basis_params(kind, lmin, lmax, s, th, ga, mu))
    return np.array(th[:s]), np.array(ga[:s]), np.array(mu[:max(s - 1, 0)])


def assg_workspace_size(n: int, s_max: int) -> int:
    v = C.c_size_t()
    _check(lib().assg_workspace_size(n, s_max, C.byref(v)))
    return v.value


def assg_struct_sizes():
    sizes = (C.c_int64 * len(_STRUCTS))()
    k = lib().assg_struct_sizes(sizes, len(_STRUCTS))
    return list(sizes[:k])


# ----------------------------------------------------------------- device
@dataclass
class DeviceCSR:
    """CSR arrays on the GPU (torch tensors) plus the C descriptor."""
    row_ptr: "object"
    col_idx: "object"
    val: "object"
    n: int
    nnz: int

    def c(self) -> AssgCsr:
        import torch
        return AssgCsr(self.n, self.nnz,
                       _dptr(self.row_ptr, self.n + 1, torch.int32, "row_ptr").value,
                       _dptr(self.col_idx, self.nnz, torch.int32, "col_idx").value,
                       _dptr(self.val, self.nnz, torch.float64, "val").value)


def csr_to_device(A, device="cuda") -> DeviceCSR:
    """Copies a scipy CSR matrix (int32 indices, float64 values) to the GPU."""
    import torch
    rp = torch.from_numpy(np.ascontiguousarray(A.indptr, dtype=np.int32)).to(device)
    ci = torch.from_numpy(np.ascontiguousarray(A.indices, dtype=np.int32)).to(device)
    va = torch.from_numpy(np.ascontiguousarray(A.data, dtype=np.float64)).to(device)
    return DeviceCSR(rp, ci, va, int(A.shape[0]), int(A.nnz))


class Handle:
    def __init__(self, ptr):
        self.ptr = ptr

    def __del__(self):
        if getattr(self, "ptr", None):
            try:
                lib().assg_destroy(self.ptr)
            except Exception:
                pass
            self.ptr = None


def assg_create(stream=None) -> Handle:
    p = C.c_void_p()
    s = _stream_ptr() if stream is None else C.c_void_p(stream)
    _check(lib().assg_create(C.byref(p), s))
    return Handle(p)


def assg_destroy(h: Handle):
    if h.ptr:
        _check(lib().assg_destroy(h.ptr))
        h.ptr = None


def assg_set_stream(h: Handle, stream=None):
    s = _stream_ptr() if stream is None else C.c_void_p(stream)
    _check(lib().assg_set_stream(h.ptr, s), h.ptr)


def assg_analyze(h: Handle, A: DeviceCSR):
    d = A.c()
    _check(lib().assg_analyze(h.ptr, C.byref(d)), h.ptr)


def assg_set_format(h: Handle, fmt: str = "auto"):
    """Storage of A for the matrix-powers kernels, used from the next
    assg_analyze: "auto", "csr" or "dia"."""
    _check(lib().assg_set_format(h.ptr, FORMAT[fmt]), h.ptr)


def assg_get_format(h: Handle) -> str:
    """"csr" or "dia": the storage the last analysis chose."""
    f = C.c_int32()
    _check(lib().assg_get_format(h.ptr, C.byref(f)), h.ptr)
    return FORMAT_NAMES[f.value]


def assg_batch_format(h: Handle) -> str:
    """"csr" or "dia": the storage the last batch analysis chose."""
    f = C.c_int32()
    _check(lib().assg_batch_format(h.ptr, C.byref(f)), h.ptr)
    return FORMAT_NAMES[f.value]


def _info_dict(info: AssgInfo) -> dict:
    d = {name: getattr(info, name) for name, _ in AssgInfo._fields_ if name != "pad0"}
    d["outcome_name"] = OUTCOME_NAMES.get(info.outcome, "?")
    return d


def assg_solve(h: Handle, A: DeviceCSR, b, x, opts: AssgOpts | None = None, workspace=None) -> dict:
    """Algorithm 5; x (CUDA float64) holds x0 on entry and the solution on return."""
    opts = opts or assg_default_opts()
    info = AssgInfo()
    d = A.c()
    ws, wsb = (None, 0) if workspace is None else (_dptr(workspace), workspace.numel() * workspace.element_size())
    _check(lib().assg_solve(h.ptr, C.byref(d), _f64(b, A.n, "b"), _f64(x, A.n, "x"),
                            C.byref(opts), ws, wsb,
                            C.byref(info)), h.ptr)
    return _info_dict(info)


def solve(A, b, x0=None, format: str = "auto", **opts):
    """One call: analysis and Algorithm 5 on a handle of its own.  A: a
    DeviceCSR or a scipy CSR matrix (copied to the GPU); b and x0: CUDA
    float64 tensors or arrays (copied to the GPU); x0 = None starts from 0.
    ``opts`` are assg_default_opts' keywords.  Returns (x, info) with x a
    CUDA tensor.  For repeated solves with one pattern keep a handle
    (assg_create, assg_analyze once, assg_solve per right-hand side)."""
    import torch
    if not isinstance(A, DeviceCSR):
        A = csr_to_device(A)
    dev = A.val.device

    def on_dev(v):
        v = torch.as_tensor(v, dtype=torch.float64)
        return v.to(dev).contiguous()

    b = on_dev(b)
    x = torch.zeros_like(b) if x0 is None else on_dev(x0).clone()
    h = assg_create()
    try:
        assg_set_format(h, format)
        assg_analyze(h, A)
        info = assg_solve(h, A, b, x, assg_default_opts(**opts))
    finally:
        assg_destroy(h)
    return x, info


NOALLOC_SCRATCH_BYTES = 64 << 20


def assg_solve_noalloc(h: Handle, A: DeviceCSR, b, x, opts: AssgOpts | None = None) -> dict:
    """assg_solve with its workspace in the library's static per-device
    scratch (no allocation inside the call; n limited by the scratch size)."""
    opts = opts or assg_default_opts()
    info = AssgInfo()
    d = A.c()
    _check(lib().assg_solve_noalloc(h.ptr, C.byref(d), _f64(b, A.n, "b"), _f64(x, A.n, "x"),
                                    C.byref(opts), C.byref(info)), h.ptr)
    return _info_dict(info)


def assg_solve_forced_schedule(h: Handle, A: DeviceCSR, b, x, sk, opts: AssgOpts | None = None,
                               workspace=None) -> dict:
    """assg_solve with loop k running exactly sk[k] inner steps (a schedule
    taken from another run, e.g. the oracle's trace)."""
    opts = opts or assg_default_opts()
    sk = np.ascontiguousarray(sk, dtype=np.int32)
    info = AssgInfo()
    d = A.c()
    ws, wsb = (None, 0) if workspace is None else (_dptr(workspace), workspace.numel() * workspace.element_size())
    _check(lib().assg_solve_forced_schedule(
        h.ptr, C.byref(d), _f64(b, A.n, "b"), _f64(x, A.n, "x"), C.byref(opts),
        sk.ctypes.data_as(C.POINTER(C.c_int32)), int(sk.size), ws, wsb, C.byref(info)), h.ptr)
    return _info_dict(info)


def assg_hscg_solve(h: Handle, A: DeviceCSR, b, x, tol=1e-10, max_iters=0, workspace=None) -> dict:
    info = AssgInfo()
    d = A.c()
    ws, wsb = (None, 0) if workspace is None else (_dptr(workspace), workspace.numel() * workspace.element_size())
    _check(lib().assg_hscg_solve(h.ptr, C.byref(d), _f64(b, A.n, "b"), _f64(x, A.n, "x"), tol,
                                 max_iters, ws, wsb,
                                 C.byref(info)), h.ptr)
    return _info_dict(info)


def assg_get_trace(h: Handle) -> list:
    cnt = C.c_int64()
    _check(lib().assg_get_trace(h.ptr, None, 0, C.byref(cnt)), h.ptr)
    buf = (AssgTrace * max(cnt.value, 1))()
    _check(lib().assg_get_trace(h.ptr, buf, cnt.value, C.byref(cnt)), h.ptr)
    out = []
    for t in buf[:cnt.value]:
        d = {name: getattr(t, name) for name, _ in AssgTrace._fields_ if name != "kappa"}
        d["kappa"] = list(t.kappa[:t.sbar])
        out.append(d)
    return out


def assg_spmv(h: Handle, A: DeviceCSR, x, y):
    d = A.c()
    _check(lib().assg_spmv(h.ptr, C.byref(d), _f64(x, A.n, "x"), _f64(y, A.n, "y")), h.ptr)


def assg_batch_analyze(h: Handle, As: list):
    """Prepares a batch of systems (DeviceCSR each) for assg_batch_solve."""
    arr = (AssgCsr * len(As))(*[A.c() for A in As])
    _check(lib().assg_batch_analyze(h.ptr, len(As), arr), h.ptr)


def assg_batch_solve(h: Handle, As: list, bs: list, xs: list, opts: AssgOpts | None = None) -> list:
    """Algorithm 5 on every system of the analyzed batch; xs[i] (CUDA float64)
    holds x0_i on entry and the solution on return.  One info dict per system."""
    n = len(As)
    if not (len(bs) == len(xs) == n):
        raise ValueError("As, bs and xs must have the same length")
    opts = opts or assg_default_opts()
    arr = (AssgCsr * n)(*[A.c() for A in As])
    bp = (C.c_void_p * n)(*[_f64(b, A.n, f"b[{i}]").value for i, (A, b) in enumerate(zip(As, bs))])
    xp = (C.c_void_p * n)(*[_f64(x, A.n, f"x[{i}]").value for i, (A, x) in enumerate(zip(As, xs))])
    infos = (AssgInfo * n)()
    _check(lib().assg_batch_solve(h.ptr, n, arr, bp, xp, C.byref(opts), infos), h.ptr)
    return [_info_dict(i) for i in infos]


def assg_batch_tuning(h: Handle) -> list:
    """The batch tuner's choice per size class (rows < 4096, < 65536,
    < 1048576, larger): systems, rows per block, nonzero cap, whether it came
    from the process cache, and each candidate shape's product time (us)."""
    arr = (AssgTuneClass * TUNE_CLASSES)()
    _check(lib().assg_batch_tuning(h.ptr, arr), h.ptr)
    return [{"systems": t.systems, "rows": t.rows, "nnz_cap": t.nnz_cap, "cached": bool(t.cached),
             "candidates_us": {f"{r}x{c}": t.candidate_us[i] for i, (r, c) in enumerate(TUNE_SHAPES)}}
            for t in arr]


def assg_csr_outer_on_pattern(h: Handle, A: DeviceCSR, u, v, alpha: float, out):
    """out[k] = alpha * u[row(k)] * v[col(k)] on A's pattern (CUDA float64)."""
    d = A.c()
    _check(lib().assg_csr_outer_on_pattern(h.ptr, C.byref(d), _f64(u, A.n, "u"), _f64(v, A.n, "v"),
                                           float(alpha), _f64(out, A.nnz, "out")), h.ptr)


def assg_basis_gram(h: Handle, A: DeviceCSR, p, r, s: int, theta, gamma, mu, Y_out=None):
    """Returns the (2s+1)^2 Gram matrix (interleaved order); fills Y_out
    (CUDA float64, (2s+1) x n, column c contiguous) when given."""
    th = (C.c_double * MAX_S)(*list(theta)[:s])
    ga = (C.c_double * MAX_S)(*list(gamma)[:s])
    mu_ = (C.c_double * MAX_S)(*list(mu)[:max(s - 1, 0)])
    G = (C.c_double * ((2 * s + 1) ** 2))()
    d = A.c()
    yp = None if Y_out is None else _f64(Y_out, (2 * s + 1) * A.n, "Y_out")
    _check(lib().assg_basis_gram(h.ptr, C.byref(d), _f64(p, A.n, "p"), _f64(r, A.n, "r"), s, th,
                                 ga, mu_, yp, G),
           h.ptr)
    return np.array(G[:]).reshape(2 * s + 1, 2 * s + 1)


def assg_block_controller(h: Handle, G, sbar: int, nb: float, tol: float, basis, s_max: int,
                          state: AssgBlockState):
    if isinstance(basis, str):
        basis = BASIS[basis]
    G = np.ascontiguousarray(G, dtype=np.float64)
    assert G.shape == (2 * sbar + 1, 2 * sbar + 1)
    Gc = G.ctypes.data_as(C.POINTER(C.c_double))
    res = AssgBlockResult()
    _check(lib().assg_block_controller(h.ptr, Gc, sbar, nb, tol, basis, s_max, C.byref(state),
                                       C.byref(res)), h.ptr)
    return res
