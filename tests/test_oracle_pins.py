"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test compares the oracle with something that is not the oracle: the dense
matrix formulation of eq. mttkrp-init (unfolding times Khatri-Rao product),
closed forms, library routines for special cases, invariants and the paper's
own printed examples (tests/golden/).
"""
import os

import numpy as np
import pytest
import scipy.sparse as sp

import oracle
from oracle import brute
from paper_1902_03317_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def rand_coo(rng, dims, nnz, dup=False):
    inds = np.stack([rng.integers(0, d, nnz) for d in dims]).astype(np.uint32)
    if dup and nnz > 2:
        inds[:, nnz // 2] = inds[:, 0]  # one repeated coordinate
    vals = rng.standard_normal(nnz)
    return inds, vals


def rand_factors(rng, dims, R):
    return [rng.standard_normal((d, R)) for d in dims]


def rel(a, b):
    return oracle.rel_fro(a, b)


@pytest.mark.parametrize("N", [2, 3, 4, 5])
@pytest.mark.parametrize("strategy", ["seq", "priv", "atomic"])
def test_brute_force_random(oracle_lib, N, strategy):
    """p1: oracle == X_(n) (KRP of the others) on random tiny tensors, every mode."""
    rng = np.random.default_rng(100 + N)
    dims = [int(x) for x in rng.integers(2, 7, N)]
    nnz = int(min(np.prod(dims), 40))
    inds, vals = rand_coo(rng, dims, nnz, dup=True)
    for R in (1, 3, 7):
        U = rand_factors(rng, dims, R)
        X = brute.dense(dims, inds, vals)
        for n in range(N):
            got = oracle.mttkrp(dims, inds, vals, U, n, strategy)
            want = brute.mttkrp_dense(X, U, n)
            assert got.shape == (dims[n], R)
            assert rel(got, want) <= 1e-12
            # the C-order unfolding with forward operand order gives the same matrix
            assert rel(brute.mttkrp_dense_c_order(X, U, n), want) <= 1e-12


def test_brute_force_small_workload(oracle_lib):
    """p1 on the full 100x80x60 / 20K-nonzero / R=16 workload, all modes."""
    spec = synth.CONFIGS[1]
    coo = synth.make_coo(spec)
    U = [f.astype(np.float64) for f in synth.make_factors(spec)]
    X = brute.dense(coo.dims, coo.inds, coo.vals)
    for n in range(3):
        got = oracle.mttkrp(coo.dims, coo.inds, coo.vals, U, n)
        assert rel(got, brute.mttkrp_dense(X, U, n)) <= 1e-12


def test_kronecker_khatri_rao_definitions():
    """Section 4.5 definitions against numpy's kron (a library routine)."""
    rng = np.random.default_rng(7)
    U, V = rng.standard_normal((3, 4)), rng.standard_normal((2, 5))
    assert np.array_equal(brute.kronecker(U, V), np.kron(U, V))
    A, B = rng.standard_normal((3, 4)), rng.standard_normal((5, 4))
    K = brute.khatri_rao(A, B)
    assert K.shape == (15, 4)
    for r in range(4):
        assert np.array_equal(K[:, r], np.kron(A[:, r], B[:, r]))
    # row (i, j) of A (.) B is the Hadamard product of row i of A and row j of B
    assert np.allclose(K[2 * 5 + 3], A[2] * B[3])


def test_unfolding_shape_and_order():
    """Reading of the matricization: I_n rows; column j = sum_k i_k * prod_{k'<k, k'!=n} I_k'."""
    X = np.arange(2 * 3 * 4, dtype=np.float64).reshape(2, 3, 4)
    X1 = brute.unfold(X, 1)
    assert X1.shape == (3, 8)
    for i0 in range(2):
        for i1 in range(3):
            for i2 in range(4):
                assert X1[i1, i0 + 2 * i2] == X[i0, i1, i2]


@pytest.mark.parametrize("R", [1, 4, 16])
def test_all_ones_marginals(oracle_lib, R):
    """p2: all-ones factors turn MTTKRP into the mode-n marginal sums of the values."""
    rng = np.random.default_rng(11)
    dims = [9, 7, 5, 4]
    inds, _ = rand_coo(rng, dims, 300, dup=True)
    vals = rng.integers(0, 8, 300).astype(np.float64)
    U = [np.ones((d, R)) for d in dims]
    for n in range(4):
        got = oracle.mttkrp(dims, inds, vals, U, n)
        marg = np.bincount(inds[n], weights=vals, minlength=dims[n])
        assert np.array_equal(got, np.repeat(marg[:, None], R, axis=1))


def test_planted_dense_closed_form(oracle_lib):
    """p3: X = [[A1..AN]] stored densely as COO => MTTKRP_n(U) = A_n * (Hadamard_k A_k^T U_k)."""
    rng = np.random.default_rng(12)
    dims, Rp, R = (6, 5, 4), 3, 2
    A = rand_factors(rng, dims, Rp)
    U = rand_factors(rng, dims, R)
    X = brute.cp_full(A)
    inds = np.stack(np.unravel_index(np.arange(X.size), dims)).astype(np.uint32)
    vals = X.reshape(-1)
    for n in range(3):
        H = np.ones((Rp, R))
        for k in range(3):
            if k != n:
                H *= A[k].T @ U[k]
        want = A[n] @ H
        assert rel(oracle.mttkrp(dims, inds, vals, U, n), want) <= 1e-12


def test_order2_is_sparse_times_dense(oracle_lib):
    """p5: N=2: MTTKRP_0 = X U1 and MTTKRP_1 = X^T U0 (scipy sparse product)."""
    rng = np.random.default_rng(13)
    dims = (30, 20)
    inds, vals = rand_coo(rng, dims, 150, dup=True)
    U = rand_factors(rng, dims, 5)
    Xs = sp.coo_matrix((vals, (inds[0], inds[1])), shape=dims).tocsr()
    assert rel(oracle.mttkrp(dims, inds, vals, U, 0), Xs @ U[1]) <= 1e-13
    assert rel(oracle.mttkrp(dims, inds, vals, U, 1), Xs.T @ U[0]) <= 1e-13


def test_rank1_is_ttv_chain(oracle_lib):
    """p6: R=1: MTTKRP_n = X x_{k!=n} u_k, a chain of tensor-times-vector products (Section 4.4)."""
    rng = np.random.default_rng(14)
    dims = (5, 4, 6, 3)
    inds, vals = rand_coo(rng, dims, 80)
    U = rand_factors(rng, dims, 1)
    X = brute.dense(dims, inds, vals)
    for n in range(4):
        Y = X
        for k in reversed(range(4)):  # contract the highest modes first so axis numbers stay valid
            if k != n:
                Y = np.tensordot(Y, U[k][:, 0], axes=([k], [0]))
        assert rel(oracle.mttkrp(dims, inds, vals, U, n)[:, 0], Y) <= 1e-13


def test_invariants(oracle_lib):
    """p7: linearity, scaling, independence of U_n, nonzero order, duplicates, empty rows."""
    rng = np.random.default_rng(15)
    dims = (12, 9, 7)
    inds, vals = rand_coo(rng, dims, 120)
    vals2 = rng.standard_normal(120)
    U = rand_factors(rng, dims, 6)
    for n in range(3):
        base = oracle.mttkrp(dims, inds, vals, U, n)
        lin = oracle.mttkrp(dims, inds, 2.0 * vals - 3.0 * vals2, U, n)
        assert rel(lin, 2.0 * base - 3.0 * oracle.mttkrp(dims, inds, vals2, U, n)) <= 1e-13
        k = (n + 1) % 3
        Us = [u.copy() for u in U]
        Us[k] *= -2.5
        assert rel(oracle.mttkrp(dims, inds, vals, Us, n), -2.5 * base) <= 1e-13
        Ug = [u.copy() for u in U]
        Ug[n] = np.full_like(U[n], np.nan)  # never read
        assert np.array_equal(oracle.mttkrp(dims, inds, vals, Ug, n), base)
        p = rng.permutation(120)
        assert rel(oracle.mttkrp(dims, inds[:, p], vals[p], U, n), base) <= 1e-13
        empty = np.setdiff1d(np.arange(dims[n]), inds[n])
        assert np.all(base[empty] == 0.0)
    # duplicates are summed: two copies of x equal one copy of 2x
    d_inds = np.concatenate([inds, inds], axis=1)
    d_vals = np.concatenate([vals, vals])
    for n in range(3):
        assert rel(oracle.mttkrp(dims, d_inds, d_vals, U, n), oracle.mttkrp(dims, inds, 2 * vals, U, n)) <= 1e-13


def test_degenerate_shapes(oracle_lib):
    """nnz = 0 gives zeros; a mode of size 1; an order-2 tensor with one nonzero."""
    dims = (4, 1, 3)
    U = [np.ones((d, 2)) for d in dims]
    z = oracle.mttkrp(dims, np.zeros((3, 0), np.uint32), np.zeros(0), U, 0)
    assert z.shape == (4, 2) and np.all(z == 0)
    inds = np.array([[1, 3], [0, 0], [2, 2]], np.uint32)
    out = oracle.mttkrp(dims, inds, np.array([2.0, 5.0]), U, 1)
    assert np.array_equal(out, [[7.0, 7.0]])
    with pytest.raises(ValueError):
        oracle.mttkrp(dims, np.array([[4], [0], [0]], np.uint32), np.ones(1), U, 0)


def test_cp_sample_matches_dense_model(oracle_lib):
    """p4: sampling [[A]] at a sparse pattern equals the dense outer-product model there."""
    rng = np.random.default_rng(16)
    dims = (7, 6, 5, 4)
    A = rand_factors(rng, dims, 3)
    inds, _ = rand_coo(rng, dims, 60)
    Xf = brute.cp_full(A)
    want = Xf[tuple(inds.astype(np.int64))]
    assert rel(oracle.cp_sample(dims, inds, A), want) <= 1e-14
    loss, resid = oracle.cp_loss(dims, inds, want, A)
    assert loss <= 1e-28 and np.max(np.abs(resid)) <= 1e-14
    _, grads = oracle.cp_grad(dims, inds, want, A)
    for g in grads:
        assert np.max(np.abs(g)) <= 1e-13


def test_cp_gradient_finite_differences(oracle_lib):
    """p8(i): central differences of the FP64 loss match the residual-weighted MTTKRP."""
    rng = np.random.default_rng(17)
    dims = (6, 5, 4)
    U = rand_factors(rng, dims, 3)
    inds, vals = rand_coo(rng, dims, 50)
    _, grads = oracle.cp_grad(dims, inds, vals, U)
    for n in range(3):
        for (i, r) in [(0, 0), (3, 2), (dims[n] - 1, 1)]:
            h = 1e-6 * max(1.0, abs(U[n][i, r]))
            Up = [u.copy() for u in U]
            Um = [u.copy() for u in U]
            Up[n][i, r] += h
            Um[n][i, r] -= h
            fd = (oracle.cp_loss(dims, inds, vals, Up)[0] - oracle.cp_loss(dims, inds, vals, Um)[0]) / (2 * h)
            assert abs(fd - grads[n][i, r]) <= 1e-6 * max(1.0, abs(fd))


def test_cp_gradient_dense_closed_form(oracle_lib):
    """p8(ii): on a fully observed tensor the masked loss is the full CP loss, whose
    gradient is U_n (Hadamard_k U_k^T U_k) - X_(n) (KRP of the others)."""
    rng = np.random.default_rng(18)
    dims = (5, 4, 3)
    U = rand_factors(rng, dims, 2)
    X = rng.standard_normal(dims)
    inds = np.stack(np.unravel_index(np.arange(X.size), dims)).astype(np.uint32)
    _, grads = oracle.cp_grad(dims, inds, X.reshape(-1), U)
    for n in range(3):
        G = np.ones((2, 2))
        for k in range(3):
            if k != n:
                G *= U[k].T @ U[k]
        want = U[n] @ G - brute.mttkrp_dense(X, U, n)
        assert rel(grads[n], want) <= 1e-12


def test_sort_perm_and_rowptr(oracle_lib):
    """p9: the stable mode-n order against Python's stable sort; rowptr against counting."""
    rng = np.random.default_rng(19)
    rows = rng.integers(0, 9, 200)
    rows[50:90] = 4  # a long run of ties
    perm = oracle.sort_perm(rows)
    assert list(perm) == sorted(range(200), key=lambda m: rows[m])
    rp = oracle.rowptr(rows[perm], 12)
    counts = [int(np.sum(rows == i)) for i in range(12)]
    assert list(rp) == [sum(counts[:i]) for i in range(13)]


def test_mode_orders_are_cyclic_lexicographic(oracle_lib):
    """The chained per-mode orders equal a lexicographic sort on (i_n, i_{n-1}, ..., i_0),
    then i_{N-1} (for n < N-1), then caller position, checked with Python's own sort."""
    rng = np.random.default_rng(22)
    for dims in [(4, 3), (5, 4, 3), (3, 4, 2, 3)]:
        N = len(dims)
        inds, _ = rand_coo(rng, dims, 90, dup=True)
        orders = oracle.mode_orders(inds)
        for n in range(N):
            cyc = list(range(n, -1, -1)) + ([N - 1] if n < N - 1 else [])
            want = sorted(range(90), key=lambda m: tuple(int(inds[k, m]) for k in cyc) + (m,))
            assert list(orders[n]) == want
        # the same orders as a chain of stable single-key sorts: mode N-1 by i_{N-1} out of
        # caller order, then each mode n by i_n out of mode n-1's order
        prev = np.argsort(inds[N - 1], kind="stable")
        for n in range(N):
            prev = prev[np.argsort(inds[n][prev], kind="stable")]
            assert np.array_equal(orders[n], prev)


def test_golden_lexicographic_order(oracle_lib):
    """Section 5.2 example (2,1,1) > (1,1,2) > (1,1,1): composing stable single-mode
    sorts from the last mode to the first yields that lexicographic order."""
    lines = [l.split() for l in open(os.path.join(GOLDEN, "lexicographic_order.txt")) if l.strip()
             and not l.startswith("#")]
    desc = np.array([[int(x) for x in l] for l in lines])
    shuffled = desc[[1, 2, 0]]
    perm = np.arange(3)
    for k in reversed(range(3)):
        perm = perm[oracle.sort_perm(shuffled[perm, k])]
    assert np.array_equal(shuffled[perm], desc[::-1])


def test_golden_coo_example_zero_based(oracle_lib):
    """Section 5.1 example: 0-based coordinates of a 4x4x3 tensor; the two entries that
    share (i, j) = (1, 0) land in the same mode-0 and mode-1 output rows."""
    lines = [l.split() for l in open(os.path.join(GOLDEN, "coo_example.txt")) if l.strip()
             and not l.startswith("#")]
    dims = tuple(int(x) for x in lines[0][1:])
    inds = np.array([[int(x) for x in l] for l in lines[1:]], dtype=np.uint32).T
    U = [np.ones((d, 1)) for d in dims]
    out0 = oracle.mttkrp(dims, inds, [1.0, 2.0], U, 0)
    assert out0[:, 0].tolist() == [0.0, 3.0, 0.0, 0.0]
    out2 = oracle.mttkrp(dims, inds, [1.0, 2.0], U, 2)
    assert out2[:, 0].tolist() == [1.0, 0.0, 2.0]


def test_bf16_round(oracle_lib):
    """Round to nearest even against torch's CPU float32 -> bfloat16 conversion and hand cases."""
    import torch
    rng = np.random.default_rng(20)
    x = np.concatenate([rng.standard_normal(10000).astype(np.float32),
                        np.array([1.0, -2.5, 3.0e-38, 1.0e38], np.float32)])
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float32).numpy()
    assert np.array_equal(oracle.bf16_round(x), ref)
    ties = np.array([0x3F808000, 0x3F818000, 0x3F807FFF, 0x3F808001], np.uint32).view(np.float32)
    got = oracle.bf16_round(ties).view(np.uint32)
    assert got.tolist() == [0x3F800000, 0x3F820000, 0x3F800000, 0x3F810000]


def _mttkrp_loops(dims, inds, vals, U, n, mutant=None):
    """Alg. 6 generalised, written with plain loops; ``mutant`` plants one mistake."""
    N = len(dims)
    R = U[(n + 1) % N].shape[1]
    out = np.zeros((dims[n], R))
    for m in range(inds.shape[1]):
        for r in range(R):
            t = vals[m]
            for k in range(N):
                if k == n:
                    continue
                if mutant == "drop_term" and k == N - 1 - (n == N - 1):
                    continue
                idx = inds[k, m]
                if mutant == "wrong_index":
                    idx = inds[(k + 1) % N, m] % dims[k]
                if mutant == "transposed":
                    t *= U[k].reshape(-1)[(r * dims[k] + idx) % U[k].size]
                else:
                    t *= U[k][idx, r]
            row = inds[n, m] if mutant != "wrong_output" else inds[(n + 1) % N, m] % dims[n]
            out[row, r] += -t if mutant == "sign" else t
    return out


@pytest.mark.parametrize("mutant", [None, "drop_term", "wrong_index", "transposed", "wrong_output", "sign"])
def test_pins_reject_planted_mistakes(mutant):
    """The brute-force and marginal pins reject each plausible mistake planted in a
    loop version of the definition, and accept the correct one."""
    rng = np.random.default_rng(21)
    dims = (5, 4, 3)
    inds, vals = rand_coo(rng, dims, 30)
    U = rand_factors(rng, dims, 3)
    X = brute.dense(dims, inds, vals)
    ok = True
    for n in range(3):
        ok &= rel(_mttkrp_loops(dims, inds, vals, U, n, mutant), brute.mttkrp_dense(X, U, n)) <= 1e-12
    ones = [np.ones((d, 3)) for d in dims]
    for n in range(3):
        marg = np.bincount(inds[n], weights=vals, minlength=dims[n])
        ok &= np.allclose(_mttkrp_loops(dims, inds, vals, ones, n, mutant)[:, 0], marg)
    assert ok == (mutant is None)


def test_cp_als_update_is_the_least_squares_solution(oracle_lib):
    """Each mode update of the ALS sweep solves min ||X_(n) - U_n (KRP of the others)^T||_F:
    checked against numpy lstsq on the dense unfolding and the explicit Khatri-Rao product."""
    rng = np.random.default_rng(23)
    dims = (6, 5, 4)
    lin = rng.choice(120, 70, replace=False)  # distinct coordinates: the fit's norm is the dense one
    inds = np.stack(np.unravel_index(lin, dims)).astype(np.uint32)
    vals = rng.standard_normal(70)
    U0 = rand_factors(rng, dims, 3)
    X = brute.dense(dims, inds, vals)
    U, lam, fit = oracle.cp_als_sweep(dims, inds, vals, U0)
    # replay the sweep mode by mode with lstsq on the unfolding
    W = [u.copy() for u in U0]
    for n in range(3):
        K = brute.khatri_rao_chain([W[k] for k in reversed(range(3)) if k != n])
        Un = np.linalg.lstsq(K, brute.unfold(X, n).T, rcond=None)[0].T
        ln = np.linalg.norm(Un, axis=0)
        W[n] = Un / ln
    for n in range(3):
        assert rel(U[n], W[n]) <= 1e-10
    assert rel(lam, ln) <= 1e-10
    # the fit formula against the dense residual
    model = brute.cp_full([W[0], W[1], W[2] * ln[None, :]])
    want = 1.0 - np.linalg.norm(X - model) / np.linalg.norm(X)
    assert abs(fit - want) <= 1e-10


def test_cp_als_recovers_a_planted_model(oracle_lib):
    """A fully observed exact rank-3 tensor: a few sweeps from a random start drive the
    fit to 1 (the model is recovered)."""
    rng = np.random.default_rng(24)
    dims = (8, 7, 6)
    A = rand_factors(rng, dims, 3)
    X = brute.cp_full(A)
    inds = np.stack(np.unravel_index(np.arange(X.size), dims)).astype(np.uint32)
    U = rand_factors(rng, dims, 3)
    fit = 0.0
    for _ in range(60):
        U, lam, fit = oracle.cp_als_sweep(dims, inds, X.reshape(-1), U)
    assert fit > 1 - 1e-6


def test_cp_fit_is_the_dense_relative_residual(oracle_lib):
    """cp_fit on distinct coordinates equals 1 - ||X - [[lambda; U]]||_F / ||X||_F with the
    model built densely (outer products) and X zero off the nonzeros."""
    rng = np.random.default_rng(25)
    dims = (5, 6, 4)
    lin = rng.choice(120, 50, replace=False)
    inds = np.stack(np.unravel_index(lin, dims)).astype(np.uint32)
    vals = rng.standard_normal(50)
    U = rand_factors(rng, dims, 3)
    lam = rng.uniform(0.5, 2.0, 3)
    X = brute.dense(dims, inds, vals)
    model = brute.cp_full([U[0] * lam[None, :], U[1], U[2]])
    want = 1.0 - np.linalg.norm(X - model) / np.linalg.norm(X)
    assert abs(oracle.cp_fit(dims, inds, vals, U, lam) - want) <= 1e-12


def test_cp_als_update_condition_number(oracle_lib):
    """With orthonormal columns in every other factor, V = Hadamard of identities = I, so
    the reported condition number is 1 and the update is MTTKRP scaled to unit columns."""
    rng = np.random.default_rng(26)
    dims = (7, 6, 5)
    inds, vals = rand_coo(rng, dims, 40)
    U = [np.linalg.qr(rng.standard_normal((d, 3)))[0] for d in dims]
    Un, lam, M, kappa = oracle.cp_als_update(dims, inds, vals, U, 0)
    assert abs(kappa - 1.0) <= 1e-12
    assert rel(Un * lam[None, :], M) <= 1e-12
    assert rel(M, brute.mttkrp_dense(brute.dense(dims, inds, vals), U, 0)) <= 1e-12
