"""Pins of the FP64 oracle's element-wise (TEW-eq, TEW) and tensor-scalar (TS)
functions against what the paper and the mathematics fix: the element-wise
definition on dense tensors (Section 4.1), the scalar definition on the
nonzeros (Section 4.2) with the paper's equivalences X x s = X / s^-1 and
X + s = X - (-s), the union / intersection structure of the general merge
(Alg. 2) with its output shape and lexicographic order, and the paper's own
ordering example (tests/golden/).
"""
import os

import numpy as np
import pytest

import oracle
from oracle import brute

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def distinct_coo(rng, dims, nnz):
    cells = int(np.prod(dims))
    flat = rng.choice(cells, size=min(nnz, cells), replace=False)
    inds = np.stack(np.unravel_index(flat, dims)).astype(np.uint32)
    return inds, rng.standard_normal(inds.shape[1])


def dense_at(dims, inds, vals):
    return brute.dense(dims, inds, vals)


@pytest.mark.parametrize("op", ["add", "sub", "mul", "div"])
def test_tew_eq_is_the_elementwise_definition(op):
    """Same pattern: z at each nonzero is the dense element-wise result there."""
    rng = np.random.default_rng(1)
    dims = (7, 5, 6)
    inds, x = distinct_coo(rng, dims, 90)
    y = rng.standard_normal(x.size) + 3.0
    z = oracle.tew_eq(op, x, y)
    X, Y = dense_at(dims, inds, x), dense_at(dims, inds, y)
    D = {"add": X + Y, "sub": X - Y, "mul": X * Y}.get(op)
    if op == "div":
        D = np.divide(X, Y, out=np.zeros_like(X), where=Y != 0)
    assert np.array_equal(z, D[tuple(inds.astype(np.int64))])


def test_tew_eq_inverse_pairs():
    rng = np.random.default_rng(2)
    x, y = rng.standard_normal(1000), rng.standard_normal(1000) + 4.0
    assert np.allclose(oracle.tew_eq("sub", oracle.tew_eq("add", x, y), y), x, rtol=0, atol=1e-14)
    assert np.allclose(oracle.tew_eq("div", oracle.tew_eq("mul", x, y), y), x, rtol=1e-15, atol=0)
    assert np.isinf(oracle.tew_eq("div", np.array([1.0]), np.array([0.0]))[0])


def test_ts_definition_and_the_papers_equivalences():
    """Section 4.2: the scalar acts on every nonzero; X x s equals X / s^-1 (to rounding) and
    X + s equals X - (-s) exactly; implicit zeros stay zero (the pattern is kept)."""
    rng = np.random.default_rng(3)
    dims = (6, 4, 5)
    inds, x = distinct_coo(rng, dims, 50)
    s = 1.75
    ym, ya = oracle.ts("mul", x, s), oracle.ts("add", x, s)
    X = dense_at(dims, inds, x)
    assert np.array_equal(ym, (X * s)[tuple(inds.astype(np.int64))])
    assert np.array_equal(ya, X[tuple(inds.astype(np.int64))] + s)
    assert np.allclose(oracle.ts("div", x, 1.0 / s), ym, rtol=1e-15, atol=0)
    assert np.array_equal(oracle.ts("sub", x, -s), ya)
    assert ym.shape == x.shape


@pytest.mark.parametrize("op", ["add", "sub", "mul"])
@pytest.mark.parametrize("N", [2, 3, 4])
def test_tew_general_against_dense(op, N):
    """Alg. 2 on overlapping patterns and different shapes: scattered into the unified
    (element-wise maximum) shape, the result is the dense element-wise result."""
    rng = np.random.default_rng(10 + N)
    dx = [int(d) for d in rng.integers(2, 7, N)]
    dy = [int(d) for d in rng.integers(2, 7, N)]
    ix, vx = distinct_coo(rng, dx, 40)
    iy, vy = distinct_coo(rng, dy, 40)
    iy[:, :10] = ix[:, :10] % np.array(dy, dtype=np.uint32)[:, None]  # force overlaps
    iy, keep = np.unique(iy, axis=1, return_index=True)
    vy = vy[keep]
    dims_z, iz, vz = oracle.tew(op, dx, ix, vx, dy, iy, vy)
    assert dims_z == tuple(max(a, b) for a, b in zip(dx, dy))
    X, Y, Z = dense_at(dims_z, ix, vx), dense_at(dims_z, iy, vy), dense_at(dims_z, iz, vz)
    want = {"add": X + Y, "sub": X - Y, "mul": X * Y}[op]
    assert np.max(np.abs(Z - want)) <= 1e-14
    # structure: the union (add, sub) or the intersection (mul) of the patterns, lexicographic
    sx = {tuple(c) for c in ix.T.tolist()}
    sy = {tuple(c) for c in iy.T.tolist()}
    want_set = sx & sy if op == "mul" else sx | sy
    got = [tuple(c) for c in iz.T.tolist()]
    assert got == sorted(want_set)


def test_tew_general_special_cases():
    rng = np.random.default_rng(20)
    dims = (5, 6, 7)
    ix, vx = distinct_coo(rng, dims, 60)
    vy = rng.standard_normal(vx.size)
    # the same pattern: the merge equals the same-pattern operation, in lexicographic order
    o = oracle.lex_order(ix)
    _, iz, vz = oracle.tew("add", dims, ix, vx, dims, ix, vy)
    assert np.array_equal(iz, ix[:, o]) and np.array_equal(vz, oracle.tew_eq("add", vx, vy)[o])
    # disjoint patterns: the sorted union with -y for subtraction, nothing for multiplication
    iy = ix.copy()
    iy[0] += np.uint32(dims[0])
    _, iz, vz = oracle.tew("sub", dims, ix, vx, (10, 6, 7), iy, vy)
    assert iz.shape[1] == 2 * vx.size
    assert np.array_equal(vz, np.concatenate([vx[o], -vy[o]]))
    assert oracle.tew("mul", dims, ix, vx, (10, 6, 7), iy, vy)[1].shape == (3, 0)
    # repeated coordinates inside one input count as their sum
    ixd = np.concatenate([ix, ix[:, :5]], axis=1)
    vxd = np.concatenate([vx, np.ones(5)])
    _, izd, vzd = oracle.tew("add", dims, ixd, vxd, dims, np.zeros((3, 0), np.uint32), np.zeros(0))
    want = vx.copy()
    want[:5] += 1.0
    assert np.array_equal(izd, ix[:, o]) and np.allclose(vzd, want[o], rtol=0, atol=1e-15)
    # empty inputs
    assert oracle.tew("add", dims, np.zeros((3, 0), np.uint32), [], dims, np.zeros((3, 0), np.uint32), [])[1].shape \
        == (3, 0)


def test_golden_lexicographic_merge_order():
    """The Section 5.2 example: (1,1,1) < (1,1,2) < (2,1,1), with the tuples split over the two inputs."""
    lines = [l.split("#")[0].strip() for l in open(os.path.join(GOLDEN, "lexicographic_order.txt"))]
    tuples = [tuple(int(x) for x in l.split()) for l in lines if l]  # largest first
    X = np.array([tuples[0], tuples[2]], dtype=np.uint32).T  # (2,1,1) and (1,1,1)
    Y = np.array([tuples[1]], dtype=np.uint32).T  # (1,1,2)
    _, iz, vz = oracle.tew("add", (3, 2, 3), X, [1.0, 3.0], (3, 2, 3), Y, [2.0])
    assert [tuple(c) for c in iz.T.tolist()] == tuples[::-1]
    assert vz.tolist() == [3.0, 2.0, 1.0]


def _merge_loops(op, ix, vx, iy, vy, mutant=None):
    """Alg. 2 with plain loops over lexicographically sorted distinct inputs; ``mutant``
    plants one mistake."""
    ox, oy = oracle.lex_order(ix), oracle.lex_order(iy)
    X = [(tuple(ix[:, i].tolist()), vx[i]) for i in ox]
    Y = [(tuple(iy[:, i].tolist()), vy[i]) for i in oy]
    a = b = 0
    out = []
    while a < len(X) and b < len(Y):
        if X[a][0] == Y[b][0]:
            z = {"add": X[a][1] + Y[b][1], "sub": X[a][1] - Y[b][1], "mul": X[a][1] * Y[b][1]}[op]
            out.append((X[a][0], z))
            a, b = a + 1, b + 1
        elif X[a][0] < Y[b][0]:
            if op != "mul" or mutant == "mul_keeps_one_sided":
                out.append(X[a])
            a += 1
        else:
            if op != "mul" or mutant == "mul_keeps_one_sided":
                out.append((Y[b][0], -Y[b][1] if op == "sub" and mutant != "no_negation" else Y[b][1]))
            b += 1
    if op != "mul" and mutant != "drop_tail":
        out += X[a:]
        out += [(c, -v if op == "sub" and mutant != "no_negation" else v) for c, v in Y[b:]]
    return out


@pytest.mark.parametrize("mutant", [None, "drop_tail", "no_negation", "mul_keeps_one_sided"])
def test_pins_reject_planted_mistakes(mutant):
    rng = np.random.default_rng(30)
    dims = (5, 5, 5)
    ix, vx = distinct_coo(rng, dims, 40)
    iy, vy = distinct_coo(rng, dims, 40)
    ok = True
    for op in ("add", "sub", "mul"):
        out = _merge_loops(op, ix, vx, iy, vy, mutant)
        Z = np.zeros(dims)
        for c, v in out:
            Z[c] += v
        X, Y = dense_at(dims, ix, vx), dense_at(dims, iy, vy)
        want = {"add": X + Y, "sub": X - Y, "mul": X * Y}[op]
        sx = {tuple(c) for c in ix.T.tolist()}
        sy = {tuple(c) for c in iy.T.tolist()}
        keys = sorted(sx & sy if op == "mul" else sx | sy)
        ok &= np.max(np.abs(Z - want)) <= 1e-14 and [c for c, _ in out] == keys
    assert ok == (mutant is None)
