"""The plain C example (paper_1908_04081_amd/examples/poisson2d.c) run on
the GPU: a consumer of the C ABI with no Python in between solves the 2-D
Poisson problem and checks the residual on the host (exit status 0)."""
import os
import subprocess

import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def binary():
    import paper_1908_04081_amd.build as B
    if not os.path.exists(B.EXAMPLE_BIN):
        B.build_example()
    return B.EXAMPLE_BIN


@pytest.mark.parametrize("args", [("64", "c", "10"), ("48", "n", "10"), ("100", "c", "16"),
                                  ("1", "c", "10")])
def test_c_example_solves(binary, args):
    r = subprocess.run([binary, *args], capture_output=True, text=True, timeout=100)
    print(r.stdout, r.stderr)
    assert r.returncode == 0, (r.stdout, r.stderr)
    assert "outcome=CONVERGED" in r.stdout
