"""The bytes model that prices the MTTKRP kernel against HBM peak (host logic only)."""
import os

import bench

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_table2_memory_access_formula():
    """Section 5.2, Table 2: MTTKRP memory access 12 nnz R + 16 nnz bytes at order 3,
    32-bit indices and fp32 values."""
    g = {}
    for line in open(os.path.join(GOLDEN, "table2_mttkrp.txt")):
        if line.strip() and not line.startswith("#"):
            k, v = line.split()
            g[k] = int(v)
    for R in (1, 16, 32, 64):
        assert bench.bytes_paper(3, R, 4) == g["memory_bytes_per_nnz"] + g["memory_bytes_per_nnzR"] * R


def test_alg_and_compulsory_bytes():
    # 50K x 40K x 30K, 50M nonzeros, R = 32, fp32: 272 B per nonzero
    assert bench.bytes_alg_per_nnz(3, 32, 4) == 272
    assert bench.bytes_alg(3, 32, 4, 50_000_000, 50_000) == 50_000_000 * 272 + 4 * 32 * 50_000
    # order 4, R = 64: 788 B; order 5, R = 64, fp32 / bf16: 1048 / 536 B
    assert bench.bytes_alg_per_nnz(4, 64, 4) == 788
    assert bench.bytes_alg_per_nnz(5, 64, 4) == 1048
    assert bench.bytes_alg_per_nnz(5, 64, 2) == 536
    dims = (50_000, 40_000, 30_000)
    q = bench.bytes_compulsory(dims, 32, 4, 50_000_000, 0)
    assert q == 50_000_000 * 16 + 4 * 32 * 70_000 + 4 * 32 * 50_000
    assert q < bench.bytes_alg(3, 32, 4, 50_000_000, 50_000)


def test_multi_gpu_request_is_refused():
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(os.path.dirname(GOLDEN), "..", "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True)
    assert r.returncode == 2 and "one GPU" in r.stderr
