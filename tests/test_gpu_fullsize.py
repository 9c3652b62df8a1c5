"""Parity at the full 50Kx40Kx30K / 50M-nonzero Zipf(1.1) size, in the launch
configuration the benchmark times (R = 32, fp32 and bf16 factors).

The oracle computes sampled output rows one by one (the hottest row of every
mode, rows that cross chunk edges and random rows); properties that hold at
any size are checked on whole outputs: the all-ones invariant against the
mode marginals, and the defining property of each mode's order.
"""
import os

import numpy as np
import pytest
import torch

import oracle
from helpers import DEV, factors_dev, oracle_factors, rel, upload
from paper_1902_03317_amd import synth

pytestmark = pytest.mark.gpu

CACHE = os.environ.get("PASTA_BENCH_CACHE", "/tmp/pasta_cache")


@pytest.fixture(scope="module")
def full():
    spec = synth.CONFIGS[2]
    coo = synth.load_or_make_coo(spec, CACHE)
    X = upload(coo)
    return spec, coo, X


def _row_oracle(coo, U64, n, r):
    """MTTKRP row r of mode n from the nonzeros of that row only."""
    sel = np.flatnonzero(coo.inds[n] == r)
    inds = coo.inds[:, sel].copy()
    inds[n] = 0
    dims = list(coo.dims)
    dims[n] = 1
    return oracle.mttkrp(dims, inds, coo.vals[sel], U64, n)[0]


def test_mode_orders_full_size(full):
    """Each mode's permutation is a permutation, and the keys it produces are strictly
    increasing in (i_n, i_{n-1}, ..., i_0, [i_{N-1}], caller position), which fixes it."""
    spec, coo, X = full
    N = coo.order
    for n in range(N):
        perm, rowptr, sinds, svals = X.mode_view(n)
        p = perm.cpu().numpy().view(np.uint32).astype(np.int64)
        assert np.array_equal(np.bincount(p, minlength=coo.nnz), np.ones(coo.nnz, np.int64))
        keys = list(range(n, -1, -1)) + ([N - 1] if n < N - 1 else [])
        cols = [coo.inds[k][p].astype(np.int64) for k in keys] + [p]
        less = np.zeros(coo.nnz - 1, bool)
        equal = np.ones(coo.nnz - 1, bool)
        for c in cols:
            less |= equal & (c[:-1] < c[1:])
            equal &= c[:-1] == c[1:]
        assert less.all()
        rp = rowptr.cpu().numpy().view(np.uint32)
        assert np.array_equal(rp, np.searchsorted(coo.inds[n][p], np.arange(coo.dims[n] + 1)))
        assert np.array_equal(sinds[n].cpu().numpy().view(np.uint32), coo.inds[n][p])
        assert np.array_equal(svals.cpu().numpy(), coo.vals[p])


@pytest.mark.parametrize("dtype", [torch.float32, torch.bfloat16])
def test_sampled_rows_full_size(full, dtype):
    spec, coo, X = full
    U = synth.make_factors(spec)
    fd = factors_dev(U, dtype)
    U64 = oracle_factors(U, bf16=dtype == torch.bfloat16)
    rng = np.random.default_rng(31)
    C = 256 * 64 // (8 if dtype == torch.float32 else 4)  # nonzeros per chunk of this launch shape
    for n in range(coo.order):
        out = torch.empty((coo.dims[n], spec.rank), device=DEV)
        from paper_1902_03317_amd import api
        api.mttkrp(X, fd, n, out=out)
        got = out.cpu().numpy().astype(np.float64)
        counts = np.bincount(coo.inds[n], minlength=coo.dims[n])
        starts = np.concatenate([[0], np.cumsum(counts)])
        crossing = np.flatnonzero(((starts[:-1] // C) != ((starts[1:] - 1) // C)) & (counts > 0))
        rows = {int(np.argmax(counts))} | set(int(r) for r in rng.choice(coo.dims[n], 12, replace=False))
        rows |= set(int(r) for r in rng.choice(crossing, min(8, crossing.size), replace=False))
        for r in sorted(rows):
            want = _row_oracle(coo, U64, n, r)
            if not np.any(want):
                assert not np.any(got[r])
                continue
            assert rel(got[r], want) <= 1e-5, f"mode {n} row {r} ({counts[r]} nonzeros)"


def test_all_ones_marginals_full_size(full):
    """With all-ones factors every output row is the mode-n marginal sum of the values."""
    spec, coo, X = full
    from paper_1902_03317_amd import api
    ones = [torch.ones((d, spec.rank), device=DEV) for d in coo.dims]
    for n in range(coo.order):
        got = api.mttkrp(X, ones, n).cpu().numpy().astype(np.float64)
        marg = np.bincount(coo.inds[n], weights=coo.vals.astype(np.float64), minlength=coo.dims[n])
        assert rel(got, np.repeat(marg[:, None], spec.rank, axis=1)) <= 1e-6
        assert np.all(got == got[:, :1])  # every column of a row is the same number
