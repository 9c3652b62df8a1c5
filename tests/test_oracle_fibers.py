"""Pins of the FP64 oracle's fiber, TTM and TTV functions against what the paper
and the mathematics fix: the fiber definition on the paper's COO example, the
dense definitions of eq. ttm and the TTV equation (Sections 4.3 and 4.4), the
matricized form Y_(n) = U^T X_(n) of eq. moden-mat (in the paper's I_n x R
orientation of U), the identity matrix, brute-force orders on tiny inputs, and
the R = 1 MTTKRP as a chain of TTVs.
"""
import os

import numpy as np
import pytest

import oracle
from oracle import brute

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def rand_coo(rng, dims, nnz, dup=False):
    inds = np.stack([rng.integers(0, d, nnz) for d in dims]).astype(np.uint32)
    if dup and nnz > 2:
        inds[:, nnz // 2] = inds[:, 0]
    return inds, rng.standard_normal(nnz)


def dense_ttm(X, U, n):
    """eq. ttm on a dense tensor: contract mode n with the rows of U; the R axis takes mode n's place."""
    return np.moveaxis(np.tensordot(X, U, axes=([n], [0])), -1, n)


def scatter_fibers(dims, n, coords, Y):
    """Dense tensor of a semi-sparse TTM result (mode n of size R)."""
    R = Y.shape[1]
    out_dims = list(dims)
    out_dims[n] = R
    D = np.zeros(out_dims)
    other = [k for k in range(len(dims)) if k != n]
    for f in range(Y.shape[0]):
        idx = [0] * len(dims)
        for q, k in enumerate(other):
            idx[k] = int(coords[q, f])
        for r in range(R):
            idx[n] = r
            D[tuple(idx)] += Y[f, r]
    return D


def _golden_fibers():
    lines = [l.split("#")[0].strip() for l in open(os.path.join(GOLDEN, "fibers_example.txt"))]
    lines = [l for l in lines if l]
    out, i = {}, 0
    while i < len(lines):
        _, n, _, cnt = lines[i].split()
        n, cnt = int(n), int(cnt)
        fibs = []
        for l in lines[i + 1:i + 1 + cnt]:
            c, m = l.split(":")
            fibs.append((tuple(int(x) for x in c.split()), [int(x) for x in m.split()]))
        out[n] = fibs
        i += 1 + cnt
    return out


def _coo_example():
    lines = [l.split("#")[0].strip() for l in open(os.path.join(GOLDEN, "coo_example.txt"))]
    lines = [l for l in lines if l]
    dims = [int(x) for x in lines[0].split()[1:]]
    inds = np.array([[int(x) for x in l.split()] for l in lines[1:]], dtype=np.uint32).T
    return dims, inds


def test_golden_fibers_of_the_coo_example():
    """The fibers of the Section 5.1 example, worked out by hand from the Section 3 definition."""
    dims, inds = _coo_example()
    want = _golden_fibers()
    for n in range(3):
        o, fptr, coords = oracle.fibers(inds, n)
        assert fptr.size - 1 == len(want[n])
        for f, (c, members) in enumerate(want[n]):
            assert tuple(int(x) for x in coords[:, f]) == c
            assert sorted(int(m) for m in o[fptr[f]:fptr[f + 1]]) == members


def test_golden_lexicographic_order_is_the_last_mode_fiber_order():
    """For the last mode the fiber order is the paper's lexicographic order (Section 5.2 example)."""
    lines = [l.split("#")[0].strip() for l in open(os.path.join(GOLDEN, "lexicographic_order.txt"))]
    tuples = [tuple(int(x) for x in l.split()) for l in lines if l]  # largest first
    inds = np.array(tuples, dtype=np.uint32).T
    o = oracle.fiber_order(inds, 2)
    assert [tuples[i] for i in o] == sorted(tuples)
    assert [tuples[i] for i in o] == tuples[::-1]


@pytest.mark.parametrize("N", [2, 3, 4, 5])
def test_fiber_order_brute_force(N):
    """The order against a Python sort by (other indices in mode order, i_n, position), and
    fptr/coords against a brute-force grouping; duplicates included."""
    rng = np.random.default_rng(200 + N)
    dims = [int(x) for x in rng.integers(1, 5, N)]
    inds, _ = rand_coo(rng, dims, 60, dup=True)
    M = inds.shape[1]
    for n in range(N):
        other = [k for k in range(N) if k != n]
        key = lambda m: (tuple(int(inds[k, m]) for k in other), int(inds[n, m]), m)
        want = sorted(range(M), key=key)
        o, fptr, coords = oracle.fibers(inds, n)
        assert list(o) == want
        groups = {}
        for m in range(M):
            groups.setdefault(tuple(int(inds[k, m]) for k in other), []).append(m)
        keys = sorted(groups)
        assert fptr.size - 1 == len(keys)
        for f, k in enumerate(keys):
            assert tuple(int(x) for x in coords[:, f]) == k
            assert sorted(int(x) for x in o[fptr[f]:fptr[f + 1]]) == groups[k]


@pytest.mark.parametrize("N", [2, 3, 4, 5])
def test_ttm_dense_definition(N):
    """eq. ttm on the dense tensor equals the semi-sparse result scattered back, and is zero
    wherever no fiber holds a nonzero."""
    rng = np.random.default_rng(300 + N)
    dims = [int(x) for x in rng.integers(2, 6, N)]
    inds, vals = rand_coo(rng, dims, 50, dup=True)
    X = brute.dense(dims, inds, vals)
    for n in range(N):
        for R in (1, 3, 5):
            U = rng.standard_normal((dims[n], R))
            fptr, coords, Y = oracle.ttm(dims, inds, vals, U, n)
            assert Y.shape == (fptr.size - 1, R)
            D = scatter_fibers(dims, n, coords, Y)
            assert np.max(np.abs(D - dense_ttm(X, U, n))) <= 1e-12 * max(1.0, np.max(np.abs(D)))


def test_ttm_matricized_form():
    """eq. moden-mat with U of shape I_n x R: Y_(n) = U^T X_(n) (unfoldings with the same column order)."""
    rng = np.random.default_rng(41)
    dims = (4, 5, 3, 2)
    inds, vals = rand_coo(rng, dims, 70)
    X = brute.dense(dims, inds, vals)
    for n in range(4):
        U = rng.standard_normal((dims[n], 6))
        fptr, coords, Y = oracle.ttm(dims, inds, vals, U, n)
        D = scatter_fibers(dims, n, coords, Y)
        assert np.allclose(brute.unfold(D, n), U.T @ brute.unfold(X, n), rtol=0, atol=1e-12)


def test_ttm_identity_matrix_returns_the_tensor():
    """U = I (R = I_n): Y is X itself, each fiber's entries at their own i_n."""
    rng = np.random.default_rng(42)
    dims = (6, 4, 5)
    inds, vals = rand_coo(rng, dims, 40, dup=True)
    X = brute.dense(dims, inds, vals)
    for n in range(3):
        fptr, coords, Y = oracle.ttm(dims, inds, vals, np.eye(dims[n]), n)
        assert np.array_equal(scatter_fibers(dims, n, coords, Y), X)


def test_ttv_dense_definition_and_ttm_r1():
    """The TTV equation on the dense tensor; TTV equals TTM with the vector as an I_n x 1 matrix."""
    rng = np.random.default_rng(43)
    dims = (5, 3, 4, 2)
    inds, vals = rand_coo(rng, dims, 45)
    X = brute.dense(dims, inds, vals)
    for n in range(4):
        v = rng.standard_normal(dims[n])
        fptr, coords, y = oracle.ttv(dims, inds, vals, v, n)
        Dy = np.tensordot(X, v, axes=([n], [0]))
        other = [k for k in range(4) if k != n]
        S = np.zeros([dims[k] for k in other])
        for f in range(y.size):
            S[tuple(int(c) for c in coords[:, f])] += y[f]
        assert np.max(np.abs(S - Dy)) <= 1e-12
        assert np.array_equal(oracle.ttm(dims, inds, vals, v[:, None], n)[2][:, 0], y)


def test_rank1_mttkrp_is_a_chain_of_sparse_ttvs(oracle_lib):
    """R = 1: MTTKRP_n = X x_{k != n} u_k evaluated as sparse TTVs, each feeding the next."""
    rng = np.random.default_rng(44)
    dims = [5, 4, 6, 3]
    inds, vals = rand_coo(rng, dims, 90, dup=True)
    U = [rng.standard_normal((d, 1)) for d in dims]
    for n in range(4):
        cur_dims, cur_inds, cur_vals, modes = list(dims), inds, vals, list(range(4))
        for k in reversed(range(4)):
            if k == n:
                continue
            pos = modes.index(k)
            _, coords, y = oracle.ttv(cur_dims, cur_inds, cur_vals, U[k][:, 0], pos)
            cur_inds, cur_vals = coords, y
            del cur_dims[pos]
            modes.remove(k)
        got = np.zeros(dims[n])
        np.add.at(got, cur_inds[0].astype(np.int64), cur_vals)
        assert oracle.rel_fro(got, oracle.mttkrp(dims, inds, vals, U, n)[:, 0]) <= 1e-13


def test_degenerate_fibers():
    """No nonzeros: no fibers; a size-1 mode: every nonzero is its own fiber along it unless
    coordinates repeat; all other modes of size 1: one fiber."""
    o, fptr, coords = oracle.fibers(np.zeros((3, 0), np.uint32), 1)
    assert o.size == 0 and list(fptr) == [0] and coords.shape == (2, 0)
    _, _, Y = oracle.ttm([3, 4, 5], np.zeros((3, 0), np.uint32), np.zeros(0), np.ones((4, 2)), 1)
    assert Y.shape == (0, 2)
    rng = np.random.default_rng(45)
    inds = np.stack([np.zeros(30, np.uint32), rng.integers(0, 7, 30).astype(np.uint32)])
    vals = rng.standard_normal(30)
    fptr, coords, y = oracle.ttv([1, 7], inds, vals, np.arange(7.0), 1)
    assert fptr.tolist() == [0, 30] and coords.tolist() == [[0]]
    assert abs(y[0] - np.sum(vals * inds[1])) <= 1e-12


def _ttm_mutant(dims, inds, vals, U, n, mutant):
    """Alg. 5 with plain loops over the oracle's fibers; ``mutant`` plants one mistake."""
    o, fptr, coords = oracle.fibers(inds, n)
    nf = fptr.size - 1
    Y = np.zeros((nf, U.shape[1]))
    for f in range(nf - (mutant == "drop_last_fiber")):
        for p in range(fptr[f], fptr[f + 1] - (mutant == "drop_last_entry")):
            m = o[p]
            i = inds[(n + 1) % len(dims), m] % dims[n] if mutant == "wrong_mode" else inds[n, m]
            row = U.reshape(U.shape[1], U.shape[0])[:, i] if mutant == "transposed" else U[i]  # R x I_n reading
            Y[f] += vals[m] * row
    return fptr, coords, Y


@pytest.mark.parametrize("mutant", [None, "drop_last_fiber", "drop_last_entry", "wrong_mode", "transposed"])
def test_pins_reject_planted_mistakes(mutant):
    """The dense-definition pin catches each planted mistake and passes the clean loops."""
    rng = np.random.default_rng(46)
    dims = (4, 4, 4)
    inds, vals = rand_coo(rng, dims, 40)
    X = brute.dense(dims, inds, vals)
    ok = True
    for n in range(3):
        U = rng.standard_normal((4, 3))
        _, coords, Y = _ttm_mutant(dims, inds, vals, U, n, mutant)
        ok &= np.allclose(scatter_fibers(dims, n, coords, Y), dense_ttm(X, U, n), rtol=0, atol=1e-12)
    assert ok == (mutant is None)
