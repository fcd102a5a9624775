"""The stored expected values under tests/golden/ (written from the oracle by
tests/golden/make_golden.py): the oracle still reproduces them, and the
library's own Leja table (bisection of the logarithmic derivative, host
code) agrees with the oracle's (roots of the derivative, numpy)."""
import os

import numpy as np

import oracle as O
import spd_problems as P

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _rows(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return [ln.split() for ln in f if ln.strip() and not ln.startswith("#")]


def _header(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return [ln for ln in f if ln.startswith("# outcome")][0].split()


def test_oracle_reproduces_leja_table():
    t = np.array([float(r[0]) for r in _rows("leja_points_16.txt")])
    assert np.allclose(O.leja_reference_points(16), t, rtol=0, atol=1e-15)


def test_library_leja_table_matches_golden():
    from test_abi import _lib
    L, _ = _lib()
    t = np.array([float(r[0]) for r in _rows("leja_points_16.txt")])
    th, _, _ = L.assg_basis_params("newton", -1.0, 1.0, 16)
    assert np.allclose(th, t, rtol=0, atol=4e-16)


def test_oracle_reproduces_cfg1_trace():
    rows = _rows("poisson2d_64_chebyshev_s10.txt")
    hdr = _header("poisson2d_64_chebyshev_s10.txt")
    pr = P.make_config("poisson2d_64")
    _, info = O.adaptive_sstep_cg(pr.A, pr.b, pr.x0, s_max=10, tol=1e-10, basis="chebyshev")
    assert info["outcome"].name == hdr[2] and info["outer"] == int(hdr[4])
    assert info["iters"] == int(hdr[6])
    for t, r in zip(info["trace"], rows):
        assert (t["k"], t["sbar"], t["stilde"], t["sk"]) == tuple(int(v) for v in r[:4])
        assert abs(t["relres_updated"] - float(r[4])) <= 1e-9 * float(r[4])
