"""The C ABI without a GPU: the library loads, exports every function that
include/assg.h declares, agrees with the Python mirrors of its structs, and
its host-only entry points (defaults, basis parameters of (2.7)/(2.8),
workspace sizes, status strings) work."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "assg.h")


def _lib():
    import paper_1908_04081_amd as L
    if not os.path.exists(L.LIB_PATH):
        from paper_1908_04081_amd import build
        build.build()
    return L, L.lib()


def declared_functions():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:assg_status_t|const char\*|int32_t)\s+(assg_\w+)\s*\(",
                                 text, flags=re.M)))


def test_header_declares_the_api():
    names = declared_functions()
    for must in ("assg_solve", "assg_hscg_solve", "assg_analyze", "assg_batch_solve",
                 "assg_csr_outer_on_pattern", "assg_basis_gram", "assg_block_controller"):
        assert must in names
    assert len(names) >= 20


def test_library_exports_every_declared_function():
    _, lib = _lib()
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_debug_build_exports_every_declared_function():
    """libassg_debug.so (the same sources with -DASSG_DEBUG: index checks in
    the kernels) exports the same ABI with the same struct layouts."""
    L, _ = _lib()
    if not os.path.exists(L.DEBUG_LIB_PATH):
        from paper_1908_04081_amd import build
        build.build()
    dbg = C.CDLL(L.DEBUG_LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(dbg, n)]
    assert not missing, missing
    dbg.assg_struct_sizes.restype = C.c_int32
    sizes = (C.c_int64 * 7)()
    assert dbg.assg_struct_sizes(sizes, 7) == 7
    assert [C.sizeof(m) for m in (L.AssgOpts, L.AssgInfo, L.AssgTrace, L.AssgBlockState,
                                  L.AssgBlockResult, L.AssgCsr, L.AssgTuneClass)] == list(sizes)


def test_struct_sizes_match_the_python_mirrors():
    L, lib = _lib()
    sizes = (C.c_int64 * 7)()
    assert lib.assg_struct_sizes(sizes, 7) == 7
    mirrors = [L.AssgOpts, L.AssgInfo, L.AssgTrace, L.AssgBlockState, L.AssgBlockResult,
               L.AssgCsr, L.AssgTuneClass]
    assert [C.sizeof(m) for m in mirrors] == list(sizes)


def test_host_only_entry_points():
    L, lib = _lib()
    o = L.assg_default_opts()
    assert (o.s_max, o.s_init, o.growth, o.basis, o.tol, o.variant, o.c_const) == \
        (10, 0, 0, 2, 1e-10, 0, 1.0)   # s_init = growth = 0: both follow s_max
    assert lib.assg_status_string(0) == b"ok"
    assert L.assg_workspace_size(1000, 10) > 21 * 1000 * 8
    # Chebyshev (2.8) as read here: theta = centre, gamma_0 = d/2, gamma_l = mu_l = d/4
    th, ga, mu = L.assg_basis_params("chebyshev", 0.5, 2.5, 4)
    assert np.allclose(th, 1.5) and ga[0] == 1.0 and np.allclose(ga[1:], 0.5)
    assert np.allclose(mu, 0.5)
    # Newton (2.7): theta_0 = lmax, theta_1 = lmin, Leja order inside
    th, ga, mu = L.assg_basis_params("newton", 1.0, 3.0, 3)
    assert th[0] == 3.0 and th[1] == 1.0 and abs(th[2] - 2.0) < 1e-15
    assert np.all(ga == 1.0) and np.all(mu == 0.0)
    with pytest.raises(L.AssgError):
        L.assg_basis_params("newton", 2.0, 1.0, 3)


def test_c_example_compiles_against_the_header(tmp_path):
    """The public header is ISO C (C99, pedantic, on its own) and the
    library's exports link from C: the C example builds with warnings as
    errors (no GPU needed to build)."""
    import subprocess

    import paper_1908_04081_amd.build as B
    src = tmp_path / "only_header.c"
    src.write_text('#include "assg.h"\nint main(void) { return ASSG_OK; }\n')
    r = subprocess.run([B.CC, "-std=c99", "-pedantic", "-Wall", "-Wextra", "-Werror",
                        f"-I{B.INCLUDE}", str(src), "-o", str(tmp_path / "only_header")],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    out = str(tmp_path / "poisson2d")
    r = subprocess.run(B.example_cmd(out, extra=("-Werror",)), capture_output=True, text=True)
    assert r.returncode == 0, r.stderr


def test_unknown_option_is_refused():
    L, _ = _lib()
    with pytest.raises(TypeError):
        L.assg_default_opts(smax=5)
    assert L.assg_default_opts(s_max=5).s_max == 5
