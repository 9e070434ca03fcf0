"""Host-side checks of the benchmark script (no GPU): the one-GPU contract
and the algorithmic byte counts its roofline uses."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode != 0
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def test_spmv_algorithmic_bytes_per_unit():
    """Per alive bond: its 6x6 block once (36 values) and two 4-byte column
    indices; per particle: the 21 packed values of the diagonal block, u read
    once and w written once (6 FP64 each)."""
    for elt in (4, 8):
        base = bench.spmv_algorithmic_bytes(0, 0, elt)
        assert base == 0
        assert bench.spmv_algorithmic_bytes(0, 1, elt) == 36 * elt + 8
        assert bench.spmv_algorithmic_bytes(1, 0, elt) == 21 * elt + 96
    # the 219,024-particle plate after its impact step (1,336,336 alive bonds)
    assert bench.spmv_algorithmic_bytes(219024, 1336336, 4) == 242547392


def test_bond_algorithmic_bytes_per_unit():
    """The bond-evaluation (K1) figure of the measurement plan: per particle
    the state read once (p and q: 56 B), the diagonal block (21 values) and
    the FP64 gradient (48 B); per bond its topology and rest data (i, j, l0,
    d0: 24 B) and its block (36 values); the row-parallel kernel also writes
    the block-Jacobi inverse (21 values per particle)."""
    for elt in (4, 8):
        assert bench.bond_algorithmic_bytes(1, 0, elt) == 56 + 21 * elt + 48
        assert bench.bond_algorithmic_bytes(0, 1, elt) == 24 + 36 * elt
        assert bench.bond_algorithmic_bytes(1, 0, elt, inverse=True) == 56 + 42 * elt + 48
    # the 219,024-particle plate, 1,336,336 alive bonds, FP32 blocks: 265.7 MB
    assert bench.bond_algorithmic_bytes(219024, 1336336, 4) == 265_680_960


def test_counter_figures_are_tied_to_the_kernel_source():
    """A counter summary names the digest of the kernel source it was taken
    on; a different digest means the figures are stale and are not reported."""
    for k in ("k_spmv<float>", "k_rows_eval<float>"):
        d = bench.source_digest(k)
        assert len(d) == 16 and d == bench.source_digest(k)
    assert bench.source_digest("k_spmv<float>") != bench.source_digest("k_rows_eval<float>")
