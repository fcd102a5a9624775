"""The host partitioners every kernel indexes through (row blocks of the
CSR-stream kernels, reduction chunks of the fused last sweep and the grid
reductions), built on their own with g++ under the address and
undefined-behaviour sanitizers and checked for their invariants on random
row-length patterns and batches: the blocks cover the rows in order, each
holds at most ``rows`` rows and at most ``cap`` nonzeros or is a single
row, no block or chunk straddles a system, the chunk count is a multiple of
8 and at most 4096 (the size of the partial-sum buffers).  Also the host
part of the diagonal-storage choice: the sampled rows and the candidate
diagonals taken from them, with the limits that reject a matrix."""
import os
import shutil
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1908_04081_amd", "csrc")
HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    out = str(tmp_path_factory.mktemp("part") / "partition_driver")
    cmd = [gxx, "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", f"-I{CSRC}", os.path.join(HERE, "partition_driver.cpp"),
           os.path.join(CSRC, "partition.cpp"), "-o", out]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    return out


def _run(driver, text):
    # the environment is passed on unchanged; ASan is told not to insist on
    # coming first among the loaded libraries
    env = dict(os.environ,
               ASAN_OPTIONS="detect_leaks=1:abort_on_error=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([driver], input=text, capture_output=True, text=True, env=env)
    assert r.returncode == 0, r.stderr[-3000:]
    return r.stdout.splitlines()


def _blocks(driver, lengths, rows, cap):
    rp = np.concatenate([[0], np.cumsum(lengths)]).astype(np.int64)
    line = _run(driver, f"B {len(lengths)} {rows} {cap}\n" + " ".join(map(str, rp)) + "\n")[0]
    return rp, np.array(line.split(), dtype=np.int64)


def _check_blocks(rp, blk, rows, cap):
    n = rp.size - 1
    assert blk[0] == 0 and blk[-1] == n
    assert np.all(np.diff(blk) >= 1)
    for b0, b1 in zip(blk[:-1], blk[1:]):
        assert b1 - b0 <= rows
        assert rp[b1] - rp[b0] <= cap or b1 - b0 == 1, (b0, b1, rp[b1] - rp[b0])
        # greedy: the next row would have broken a limit
        if b1 < n:
            assert b1 - b0 == rows or rp[b1 + 1] - rp[b0] > cap or rp[b0 + 1] - rp[b0] > cap


@pytest.mark.parametrize("seed", range(8))
@pytest.mark.parametrize("shape", [(256, 2048), (128, 1024), (64, 512)])
def test_row_blocks(driver, seed, shape):
    rows, cap = shape
    rng = np.random.default_rng(seed)
    n = int(rng.integers(1, 20000))
    lengths = rng.integers(0, 40, n)                       # empty rows included
    long = rng.integers(0, n, max(1, n // 2000))
    lengths[long] = rng.integers(cap - 2, 3 * cap, long.size)   # rows around and past the cap
    rp, blk = _blocks(driver, lengths, rows, cap)
    _check_blocks(rp, blk, rows, cap)


def test_row_blocks_edge_cases(driver):
    for lengths in ([1], [0], [5000], [2048], [2049], [2048, 1], [1] * 257, [0] * 1000,
                    [8] * 256 + [2048] + [8] * 300):
        rp, blk = _blocks(driver, np.array(lengths), 256, 2048)
        _check_blocks(rp, blk, 256, 2048)


@pytest.mark.parametrize("seed", range(12))
def test_chunks(driver, seed):
    rng = np.random.default_rng(100 + seed)
    nsys = int(rng.choice([1, 2, 7, 64, 700, 2048]))
    per = rng.integers(1, 400 if nsys < 100 else 6, nsys)       # blocks per system
    if seed % 3 == 0:
        per[rng.integers(0, nsys)] = int(rng.integers(1000, 5000))
    sys_blk = np.concatenate([[0], np.cumsum(per)]).astype(np.int64)
    target = int(rng.choice([8, 512, 768, 1024, 4096]))
    line = _run(driver, f"C {nsys} {target}\n" + " ".join(map(str, sys_blk)) + "\n")[0]
    a, b, c = line.split("|")
    cblk = np.array(a.split(), dtype=np.int64)
    csys = np.array(b.split(), dtype=np.int64)
    sys_chunk = np.array(c.split(), dtype=np.int64)
    nchunk = cblk.size - 1
    assert nchunk % 8 == 0 and csys.size == nchunk and sys_chunk.size == nsys + 1
    assert cblk[0] == 0 and cblk[-1] == sys_blk[-1] and np.all(np.diff(cblk) >= 0)
    assert sys_chunk[0] == 0 and np.all(np.diff(sys_chunk) >= 1)    # at least one per system
    for i in range(nsys):
        c0, c1 = sys_chunk[i], sys_chunk[i + 1]
        assert np.all(csys[c0:c1] == i)
        assert cblk[c0] == sys_blk[i] and cblk[c1] == sys_blk[i + 1]   # no straddling
    assert np.all(cblk[sys_chunk[-1]:] == sys_blk[-1])               # padding chunks are empty
    if target >= nsys:
        assert nchunk <= max(target, nsys) + 8 + nsys
    if nsys <= 2048 and target <= 768:
        assert nchunk <= 4096


# ---- candidate diagonals of the diagonal storage (host part of the choice)

def _dia(driver, A, check_fill=True):
    A = A.tocsr()
    A.sort_indices()
    n = A.shape[0]
    text = (f"D {n} {A.nnz} {int(check_fill)}\n" + " ".join(map(str, A.indptr)) + "\n"
            + " ".join(map(str, A.indices)) + "\n")
    out = _run(driver, text)[0].strip()
    rows, res = out.split("|")
    rows = [int(v) for v in rows.split()]
    res = res.split()
    return rows, (res[0] == "ok"), ([int(v) for v in res[1:]] if res[0] == "ok" else " ".join(res[1:]))


def _stencil(shape, offsets):
    import spd_problems as P
    return P._stencil_csr(shape, offsets, [1.0] * len(offsets))


def test_dia_sample_rows_spread(driver):
    """64 rows inside [0, n), distinct once n leaves room (the first 64
    golden-ratio fractions lie at least 1/200 apart), and on a 64^3 grid
    mostly interior rows: the fractions spread over the range instead of
    hitting multiples of n/64, every one of which is a boundary row there."""
    import scipy.sparse as sp
    for n in (1, 5, 64, 4096, 262144, 3001):
        rows, _, _ = _dia(driver, sp.identity(n, format="csr"))
        assert len(rows) == 64 and min(rows) >= 0 and max(rows) < n
        if n >= 4096:
            assert len(set(rows)) == 64
    g = 64
    rows, _, _ = _dia(driver, sp.identity(g ** 3, format="csr"))
    interior = [r for r in rows if 0 < r // (g * g) < g - 1 and 0 < (r // g) % g < g - 1
                and 0 < r % g < g - 1]
    assert len(interior) >= 48


@pytest.mark.parametrize("g", [16, 64])
def test_dia_offsets_of_stencils(driver, g):
    """The 7- and 27-point stencils give their 7 and 27 offsets, sorted; the
    27-point stencil on a small grid exceeds the fill limit (its boundary
    rows leave many positions empty) unless the check is off."""
    seven = [(-1, 0, 0), (0, -1, 0), (0, 0, -1), (0, 0, 0), (0, 0, 1), (0, 1, 0), (1, 0, 0)]
    _, ok, offs = _dia(driver, _stencil((g, g, g), seven))
    assert ok and offs == [-g * g, -g, -1, 0, 1, g, g * g]
    full = [(a, b, c) for a in (-1, 0, 1) for b in (-1, 0, 1) for c in (-1, 0, 1)]
    A = _stencil((g, g, g), full)
    lin = sorted(a * g * g + b * g + c for a, b, c in full)
    rows, ok, offs = _dia(driver, A, check_fill=(g == 64))
    assert ok and offs == lin
    if g == 16:
        _, ok, why = _dia(driver, A, check_fill=True)
        fill = 27 * g ** 3 / A.nnz
        assert (not ok and "15%" in why) == (fill > 1.15), fill


def test_dia_offsets_rejections(driver):
    """More than 32 entries in a sampled row, more than 32 diagonals over the
    sampled rows, and a matrix without entries in its sampled rows."""
    import scipy.sparse as sp
    n = 4000
    dense_row = sp.lil_matrix((n, n))
    dense_row.setdiag(1.0)
    rows, _, _ = _dia(driver, sp.identity(n, format="csr"))
    for c in range(40):
        dense_row[rows[3], (rows[3] + 1 + c) % n] = 1.0
    _, ok, why = _dia(driver, dense_row.tocsr())
    assert not ok and "more than 32 entries" in why
    # each sampled row on its own offset: 64 diagonals
    A = sp.lil_matrix((n, n))
    for k, r in enumerate(rows):
        A[r, (r + 7 * k + 1) % n] = 1.0
    _, ok, why = _dia(driver, A.tocsr(), check_fill=False)
    assert not ok and "more than 32 diagonals" in why
    _, ok, why = _dia(driver, sp.csr_matrix((n, n)), check_fill=False)
    assert not ok
