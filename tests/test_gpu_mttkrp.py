"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Preprocessing (sort permutation, row offsets, sorted copies) must be bit-exact;
MTTKRP must match the oracle to a relative Frobenius error of 1e-5 with fp32
factors and 1e-2 with bf16 factors, per mode; integer-valued cases must be
bit-exact in any summation order.
"""
import numpy as np
import pytest
import torch

import oracle
from helpers import DEV, coo_from_arrays, factors_dev, oracle_factors, rel, to_dev, upload
from paper_1902_03317_amd import synth

pytestmark = [pytest.mark.gpu, pytest.mark.usefixtures("mttkrp_form")]

TOL_F32 = 1e-5
TOL_BF16 = 1e-2


def api():
    from paper_1902_03317_amd import api as a
    return a


def check_preprocess(coo, X):
    orders = oracle.mode_orders(coo.inds)
    for n in range(coo.order):
        perm, rowptr, sinds, svals = X.mode_view(n)
        want = orders[n]
        got = perm.cpu().numpy().view(np.uint32)
        assert np.array_equal(got, want), f"mode {n}: permutation differs"
        assert np.array_equal(rowptr.cpu().numpy().view(np.uint32),
                              oracle.rowptr(coo.inds[n][want], coo.dims[n])), f"mode {n}: rowptr differs"
        for k in range(coo.order):
            assert np.array_equal(sinds[k].cpu().numpy().view(np.uint32), coo.inds[k][want])
        assert np.array_equal(svals.cpu().numpy(), coo.vals[want])


def check_mttkrp(coo, X, factors, tol, dtype=torch.float32, modes=None, ld=None, ldo=None):
    fd = factors_dev(factors, dtype, ld)
    fo = oracle_factors(factors, bf16=dtype == torch.bfloat16)
    errs = []
    for n in (range(coo.order) if modes is None else modes):
        R = factors[0].shape[1]
        out = None
        if ldo is not None:
            out = torch.full((coo.dims[n], ldo), float("nan"), device=DEV)[:, :R]
        got = api().mttkrp(X, fd, n, out=out).cpu().numpy().astype(np.float64)
        want = oracle.mttkrp(coo.dims, coo.inds, coo.vals, fo, n, "priv")
        e = rel(got, want)
        errs.append(e)
        assert e <= tol, f"mode {n}: rel-Fro {e:.3e} > {tol}"
    X.check()  # no kernel found a sorted stream out of order
    return errs


def small_zipf(nnz=300_000, dims=(5000, 4000, 3000), seed=None, spec=2, values=None):
    base = synth.CONFIGS[spec]
    sp = base.scaled(nnz, dims=dims, seed=seed)
    if values:
        from dataclasses import replace
        sp = replace(sp, values=values)
    return sp, synth.make_coo(sp)


def test_small_uniform_workload_all_modes():
    spec = synth.CONFIGS[1]
    coo = synth.make_coo(spec)
    X = upload(coo)
    check_preprocess(coo, X)
    check_mttkrp(coo, X, synth.make_factors(spec), TOL_F32)


@pytest.mark.parametrize("R", [16, 32, 64])
def test_zipf_order3(R):
    sp, coo = small_zipf()
    X = upload(coo)
    check_preprocess(coo, X)
    check_mttkrp(coo, X, synth.make_factors(sp, rank=R), TOL_F32)


def test_zipf_order4_and_order5():
    for cfg, dims, nnz in [(3, (20_000, 2000, 1000, 200), 400_000), (5, (100_000, 100_000, 10_000, 1000, 100), 300_000)]:
        sp = synth.CONFIGS[cfg].scaled(nnz, dims=dims)
        coo = synth.make_coo(sp)
        X = upload(coo)
        check_preprocess(coo, X)
        f = synth.make_factors(sp)
        check_mttkrp(coo, X, f, TOL_F32)
        check_mttkrp(coo, X, f, TOL_BF16, dtype=torch.bfloat16)


@pytest.mark.parametrize("dims", [(3000, 2000), (40, 30, 20, 10, 8, 6), (20, 16, 12, 10, 8, 6, 5),
                                  (12, 10, 8, 7, 6, 5, 4, 3)])
def test_orders_2_and_6_to_8(dims):
    """The smallest order and the largest ones the library takes (2 <= N <= 8), each with
    its own compiled kernels: uniform distinct coordinates (long rows for the small modes,
    so the wave-run form also runs), fp32 and bf16 factors, every mode, and the fused CP
    gradient, against the oracle."""
    from paper_1902_03317_amd.synth import TensorSpec
    N = len(dims)
    cells = int(np.prod(dims))
    sp = TensorSpec(f"uniform-order{N}", dims, min(300_000, cells // 3), 32, (None,) * N, "uniform", True,
                    synth.BASE_SEED + 100 + N)
    coo = synth.make_coo(sp)
    X = upload(coo)
    check_preprocess(coo, X)
    f = synth.make_factors(sp, scale=synth.cp_planted_scale(32, N))
    check_mttkrp(coo, X, f, TOL_F32)
    check_mttkrp(coo, X, f, TOL_BF16, dtype=torch.bfloat16)
    loss, grads = api().cp_grad(X, factors_dev(f))
    wl, wg = oracle.cp_grad(coo.dims, coo.inds, coo.vals, oracle_factors(f), "priv")
    assert abs(loss.item() - wl) <= 1e-5 * wl
    for n in range(N):
        assert rel(grads[n].cpu().numpy(), wg[n]) <= TOL_F32, n


@pytest.mark.parametrize("cfg,dims,R", [(3, (30_000, 3000, 208, 209), 64), (3, (30_000, 3000, 416, 417), 32),
                                         (2, (5000, 416, 417), 32), (5, (20_000, 2000, 1000, 208, 100), 64)])
def test_lds_factor_at_its_size_limit(cfg, dims, R):
    """Both kernel forms (orders 3-5) read the smallest factor after the second key from LDS
    when its rows fit 52 KiB: 208 rows of 256 bytes (fp32, R = 64) or 416 of 128 bytes (fp32
    R = 32, bf16 R = 64); one row more takes the global path. The factor that qualifies
    differs by mode; fp32 and bf16 factors, every mode, and the fused CP gradient (whose
    kernels stage the factor the same way), against the oracle."""
    sp = synth.CONFIGS[cfg].scaled(400_000, dims=dims)
    coo = synth.make_coo(sp)
    X = upload(coo)
    f = synth.make_factors(sp, rank=R)
    check_mttkrp(coo, X, f, TOL_F32)
    check_mttkrp(coo, X, f, TOL_BF16, dtype=torch.bfloat16)
    fd = factors_dev(f, torch.bfloat16)
    fo = oracle_factors(f, bf16=True)
    for n in range(coo.order):  # accumulation only: the fp32 bar against the bf16-rounded factors
        got = api().mttkrp(X, fd, n).cpu().numpy().astype(np.float64)
        assert rel(got, oracle.mttkrp(coo.dims, coo.inds, coo.vals, fo, n, "priv")) <= TOL_F32
    loss, grads = api().cp_grad(X, factors_dev(f))
    wl, wg = oracle.cp_grad(coo.dims, coo.inds, coo.vals, oracle_factors(f), "priv")
    assert abs(loss.item() - wl) <= 1e-5 * wl
    for n in range(coo.order):
        assert rel(grads[n].cpu().numpy(), wg[n]) <= TOL_F32, n


@pytest.mark.parametrize("R", [1, 3, 8, 24, 48, 100, 256])
def test_rank_generality(R):
    sp, coo = small_zipf(nnz=50_000, dims=(700, 500, 300))
    X = upload(coo)
    check_mttkrp(coo, X, synth.make_factors(sp, rank=R), TOL_F32)


@pytest.mark.parametrize("R", [8, 24, 64, 128, 5])
def test_bf16_factors(R):
    sp, coo = small_zipf(nnz=100_000, dims=(2000, 1500, 1000))
    X = upload(coo)
    check_mttkrp(coo, X, synth.make_factors(sp, rank=R), TOL_BF16, dtype=torch.bfloat16)
    # against the oracle on the bf16-rounded factors the error is fp32 accumulation only
    f = synth.make_factors(sp, rank=R)
    fd = factors_dev(f, torch.bfloat16)
    fo = oracle_factors(f, bf16=True)
    for n in range(3):
        got = api().mttkrp(X, fd, n).cpu().numpy()
        assert rel(got, oracle.mttkrp(coo.dims, coo.inds, coo.vals, fo, n)) <= TOL_F32


def test_leading_dimensions():
    sp, coo = small_zipf(nnz=60_000, dims=(900, 800, 700))
    X = upload(coo)
    f = synth.make_factors(sp, rank=32)
    check_mttkrp(coo, X, f, TOL_F32, ld=40, ldo=36)
    check_mttkrp(coo, X, f, TOL_F32, ld=33, ldo=35)  # misaligned rows take the generic path
    check_mttkrp(coo, X, f, TOL_BF16, dtype=torch.bfloat16, ld=40, ldo=36)


def test_integer_values_bit_exact():
    """Small-integer values and factors: every partial sum is an exact fp32 integer,
    so any summation order gives the oracle's value exactly."""
    rng = np.random.default_rng(5)
    sp, coo = small_zipf(nnz=200_000, dims=(3000, 2000, 1000), values="ints")
    X = upload(coo)
    for R in (16, 32, 64, 7):
        f = [rng.integers(-2, 3, (d, R)).astype(np.float32) for d in coo.dims]
        fd = factors_dev(f)
        for n in range(3):
            got = api().mttkrp(X, fd, n).cpu().numpy()
            want = oracle.mttkrp(coo.dims, coo.inds, coo.vals, oracle_factors(f), n)
            assert np.max(np.abs(want)) < 2 ** 24
            assert np.array_equal(got.astype(np.float64), want), f"R={R} mode {n}"
    ones = [np.ones((d, 32), np.float32) for d in coo.dims]
    for n in range(3):
        got = api().mttkrp(X, factors_dev(ones), n).cpu().numpy()
        marg = np.bincount(coo.inds[n], weights=coo.vals.astype(np.float64), minlength=coo.dims[n])
        assert np.array_equal(got, np.repeat(marg[:, None], 32, axis=1).astype(np.float32))


def _layout(rows_per_nnz, dims, seed):
    rng = np.random.default_rng(seed)
    M = rows_per_nnz.size
    inds = np.stack([rows_per_nnz] + [rng.integers(0, d, M) for d in dims[1:]]).astype(np.uint32)
    vals = rng.random(M).astype(np.float32)
    return coo_from_arrays(dims, inds, vals)


@pytest.mark.parametrize("case", ["one_row", "every_nnz_own_row", "chunk_aligned", "chunk_plus_one",
                                  "chunk_minus_one", "sub_run_edges", "tail_only", "single_nnz", "empty_rows",
                                  "lone_split_row_high_lane", "long_row_mid_chunk", "short_mixed",
                                  "tile_edges"])
@pytest.mark.parametrize("R", [32, 64, 100])
def test_adversarial_layouts(case, R, mttkrp_form):
    """Row layouts that stress the chunk, tile and lane-group edges of the kernel form under
    test (mode 0 carries the layout)."""
    rng = np.random.default_rng(sum(map(ord, case)))
    if mttkrp_form == "wave" and R != 100:
        C = 2048  # nonzeros per chunk of the wave-run form (R = 100 takes the strided run form)
    else:
        C = 256 * (64 // (8 if R == 32 else 16)) if R != 100 else 256  # nonzeros per chunk of mode 0
    if case == "one_row":
        rows = np.full(50_000, 7)
        dims = (10, 300, 200)
    elif case == "every_nnz_own_row":
        rows = rng.permutation(40_000)
        dims = (40_000, 300, 200)
    elif case == "chunk_aligned":
        rows = np.repeat(np.arange(20), C)
        dims = (20, 300, 200)
    elif case == "chunk_plus_one":
        rows = np.repeat(np.arange(20), C + 1)
        dims = (25, 300, 200)
    elif case == "chunk_minus_one":
        rows = np.repeat(np.arange(20), C - 1)
        dims = (20, 300, 200)
    elif case == "sub_run_edges":
        rows = np.repeat(np.arange(300), np.resize([1, 255, 256, 257, 2, 511, 3], 300))
        dims = (300, 300, 200)
    elif case == "tail_only":
        rows = np.sort(rng.integers(0, 5, C * 3 + 17))
        dims = (9, 300, 200)
    elif case == "lone_split_row_high_lane":
        # rows 0..62 hold one nonzero each, row 63 crosses the first chunk edge: the fixup
        # sees one light split row, held by the last lane of its 64-row tile
        rows = np.concatenate([np.arange(63), np.full(C + 10, 63), np.arange(64, 200)])
        dims = (200, 300, 200)
    elif case == "long_row_mid_chunk":
        # one row over ~150 chunks (level-one fixup blocks), ending inside a chunk
        rows = np.concatenate([np.zeros(100, int), np.ones(C * 147 + 123, int), np.full(50, 2)])
        dims = (3, 300, 200)
    elif case == "short_mixed":
        # rows of 1..20 nonzeros: several rows end inside most steps of a lane group
        rows = np.repeat(np.arange(3000), rng.integers(1, 21, 3000))
        dims = (3000, 300, 200)
    elif case == "tile_edges":
        # row lengths around 64 and around the steps of a lane group
        rows = np.repeat(np.arange(400), np.resize([64, 63, 65, 8, 16, 7, 9, 128, 1, 127], 400))
        dims = (400, 300, 200)
    elif case == "single_nnz":
        rows = np.array([3])
        dims = (6, 5, 4)
    else:  # most rows empty
        rows = rng.choice([0, 17, 999], 5000)
        dims = (1000, 30, 20)
    coo = _layout(np.asarray(rows), dims, 11)
    X = upload(coo)
    check_preprocess(coo, X)
    f = synth.make_factors(synth.TensorSpec("adv", dims, coo.nnz, R, seed=3), rank=R)
    check_mttkrp(coo, X, f, TOL_F32)


def test_empty_tensor_and_unit_mode():
    coo = coo_from_arrays((5, 1, 3), np.zeros((3, 0), np.uint32), np.zeros(0, np.float32))
    X = upload(coo)
    f = factors_dev([np.ones((d, 16), np.float32) for d in (5, 1, 3)])
    for n in range(3):
        out = torch.full((coo.dims[n], 16), 7.0, device=DEV)
        api().mttkrp(X, f, n, out=out)
        assert torch.count_nonzero(out).item() == 0
    rng = np.random.default_rng(2)
    inds = np.stack([rng.integers(0, 5, 3000), np.zeros(3000, int), rng.integers(0, 3, 3000)])
    coo = coo_from_arrays((5, 1, 3), inds, rng.random(3000))
    X = upload(coo)
    check_preprocess(coo, X)
    check_mttkrp(coo, X, [rng.standard_normal((d, 16)).astype(np.float32) for d in (5, 1, 3)], TOL_F32)


def test_deterministic_and_stream_ordered():
    sp, coo = small_zipf(nnz=200_000)
    X = upload(coo)
    fd = factors_dev(synth.make_factors(sp))
    a = api().mttkrp(X, fd, 1)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        b = api().mttkrp(X, fd, 1)
    s.synchronize()
    assert torch.equal(a, b)


def test_forced_form_is_the_one_launched(mttkrp_form):
    import ctypes
    from paper_1902_03317_amd._lib import lib
    sp, coo = small_zipf(nnz=50_000)
    X = upload(coo)
    fd = factors_dev(synth.make_factors(sp))
    f = ctypes.c_int(-1)
    want = {"run": 1, "wave": 2}[mttkrp_form]
    w = to_dev(np.ones(coo.nnz, np.float32))
    for n in range(coo.order):
        for call in (lambda: api().mttkrp(X, fd, n), lambda: api().mttkrp(X, fd, n, vals=w)):
            f.value = -1
            call()
            assert lib.pasta_last_mttkrp_form(ctypes.byref(f)) == 0
            assert f.value == want
    f.value = -1
    api().cp_grad(X, fd)  # the fused gradient
    assert lib.pasta_last_mttkrp_form(ctypes.byref(f)) == 0 and f.value == want
    assert lib.pasta_last_mttkrp_form(None) != 0


def test_values_override_and_alpha():
    sp, coo = small_zipf(nnz=100_000)
    X = upload(coo)
    f = synth.make_factors(sp)
    w = np.random.default_rng(4).standard_normal(coo.nnz).astype(np.float32)
    for n in range(3):
        got = api().mttkrp(X, factors_dev(f), n, vals=to_dev(w), alpha=-0.5).cpu().numpy()
        want = -0.5 * oracle.mttkrp(coo.dims, coo.inds, w, oracle_factors(f), n)
        assert rel(got, want) <= TOL_F32


def test_atomic_variant():
    sp, coo = small_zipf(nnz=100_000)
    X = upload(coo)
    f = synth.make_factors(sp)
    for n in range(3):
        got = api().mttkrp_atomic(X, factors_dev(f), n).cpu().numpy()
        assert rel(got, oracle.mttkrp(coo.dims, coo.inds, coo.vals, oracle_factors(f), n)) <= TOL_F32


def test_cast_bf16_bit_exact():
    rng = np.random.default_rng(8)
    x = np.concatenate([rng.standard_normal(100_003).astype(np.float32),
                        np.array([0x3F808000, 0x3F818000, 0x7F7FFFFF], np.uint32).view(np.float32)])
    got = api().cast_bf16(to_dev(x)).view(torch.int16).cpu().numpy().view(np.uint16)
    assert np.array_equal(got, oracle.bf16_bits(x))


def test_status_codes():
    """Argument errors come back as documented status codes through the raw C ABI."""
    import ctypes
    from paper_1902_03317_amd._lib import PastaError, lib, ptr_array
    coo = coo_from_arrays((4, 3, 2), np.array([[0, 3], [1, 2], [1, 0]]), np.ones(2))
    X = upload(coo)
    f = factors_dev([np.ones((d, 8), np.float32) for d in (4, 3, 2)])
    out = torch.zeros((4, 8), device=DEV)
    ws = torch.empty(1 << 16, dtype=torch.uint8, device=DEV)
    fp = ptr_array([t.data_ptr() for t in f])
    s0 = ctypes.c_void_p(0)

    def call(mode=0, factors=fp, rank=8, ldf=8, ldo=8, work=ws.data_ptr(), nbytes=ws.numel()):
        return lib.pasta_mttkrp(X.handle, mode, factors, 0, rank, ldf, None, 1.0, out.data_ptr(), ldo, work,
                                nbytes, s0)

    assert call() == 0
    assert call(mode=3) == 1  # mode >= order
    assert call(rank=0) == 1
    assert call(ldf=4) == 1  # ldf < rank
    assert call(ldo=4) == 1
    assert call(factors=ptr_array([f[0].data_ptr(), 0, f[2].data_ptr()])) == 1  # a needed factor is NULL
    assert call(factors=ptr_array([0, f[1].data_ptr(), f[2].data_ptr()])) == 0  # factors[mode] is not read
    assert call(rank=300, ldf=300, ldo=300) == 3
    assert call(work=0, nbytes=0) == 4
    assert call(work=ws.data_ptr() + 16) == 4  # misaligned workspace
    torch.cuda.synchronize()
    bad = coo_from_arrays((4, 3, 2), np.array([[0, 4], [1, 2], [1, 0]]), np.ones(2))
    with pytest.raises(PastaError, match="ERANGE"):
        upload(bad)
