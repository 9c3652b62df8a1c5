"""Parity of the element-wise (TEW-eq, general TEW) and tensor-scalar (TS)
operations (through the C ABI) with the FP64 oracle.

Each output value is one correctly rounded fp32 operation on fp32 inputs, so
it must equal the FP64 oracle's result rounded to fp32 bit for bit (rounding
an FP64 sum, difference, product or quotient of two fp32 numbers to fp32 gives
the correctly rounded fp32 result). Coordinates, shapes and counts are exact.
Inputs with repeated coordinates sum in fp32: rel-Fro <= 1e-6 there.
"""
import numpy as np
import pytest
import torch

import oracle
from helpers import DEV, to_dev
from paper_1902_03317_amd import synth

pytestmark = pytest.mark.gpu


def api():
    from paper_1902_03317_amd import api as a
    return a


def f32(a):
    return np.asarray(a, dtype=np.float64).astype(np.float32)


def same_bits(got, want):
    g = np.ascontiguousarray(got, np.float32).view(np.uint32)
    w = np.ascontiguousarray(want, np.float32).view(np.uint32)
    return np.array_equal(g, w)


@pytest.mark.parametrize("op", ["add", "sub", "mul", "div"])
@pytest.mark.parametrize("n", [1, 3, 4, 1001, 262_147])
def test_tew_eq_and_ts_bit_exact(op, n):
    rng = np.random.default_rng(n)
    x = rng.standard_normal(n).astype(np.float32)
    y = (rng.standard_normal(n) + 0.5).astype(np.float32)
    xd, yd = to_dev(x), to_dev(y)
    got = api().tew_eq(op, xd, yd).cpu().numpy()
    assert same_bits(got, f32(oracle.tew_eq(op, x, y)))
    s = np.float32(-1.37)
    got = api().ts(op, xd, float(s)).cpu().numpy()
    assert same_bits(got, f32(oracle.ts(op, x, s)))


def test_unaligned_views_aliasing_and_empty():
    rng = np.random.default_rng(5)
    x = rng.standard_normal(10_001).astype(np.float32)
    y = rng.standard_normal(10_001).astype(np.float32)
    xd, yd = to_dev(x), to_dev(y)
    xv, yv = xd[1:], yd[1:]  # 4-byte aligned only: the scalar kernel
    out = torch.empty(10_001, device=DEV)[1:]
    api().tew_eq("mul", xv, yv, out=out)
    assert same_bits(out.cpu().numpy(), f32(oracle.tew_eq("mul", x[1:], y[1:])))
    z = xd.clone()
    api().tew_eq("sub", z, yd, out=z)  # in place
    assert same_bits(z.cpu().numpy(), f32(oracle.tew_eq("sub", x, y)))
    api().ts("add", z, 2.0, out=z)
    assert same_bits(z.cpu().numpy(), f32(oracle.ts("add", f32(oracle.tew_eq("sub", x, y)), 2.0)))
    e = torch.empty(0, device=DEV)
    assert api().tew_eq("add", e, e).numel() == 0 and api().ts("mul", e, 3.0).numel() == 0
    special = to_dev(np.array([1.0, -1.0, 0.0, np.inf], np.float32))
    zero = to_dev(np.zeros(4, np.float32))
    got = api().tew_eq("div", special, zero).cpu().numpy()
    assert np.isposinf(got[0]) and np.isneginf(got[1]) and np.isnan(got[2]) and np.isposinf(got[3])


def rand_distinct(rng, dims, nnz):
    cells = int(np.prod(np.array(dims, dtype=np.float64)))
    if cells < 4 * nnz:
        flat = rng.choice(cells, size=min(nnz, cells), replace=False)
        return np.stack(np.unravel_index(flat, dims)).astype(np.uint32)
    inds = np.stack([rng.integers(0, d, 2 * nnz) for d in dims]).astype(np.uint32)
    _, first = np.unique(inds, axis=1, return_index=True)
    return inds[:, np.sort(first)[:nnz]]


def check_tew(op, dx, ix, vx, dy, iy, vy, exact=True):
    dz, iz, vz = api().tew(op, dx, to_dev(ix), to_dev(f32(vx)), dy, to_dev(iy), to_dev(f32(vy)))
    wd, wi, wv = oracle.tew(op, dx, ix, f32(vx).astype(np.float64), dy, iy, f32(vy).astype(np.float64))
    assert dz == wd
    assert np.array_equal(iz.cpu().numpy().view(np.uint32), wi)
    got = vz.cpu().numpy()
    if exact:
        assert same_bits(got, f32(wv))
    else:
        assert oracle.rel_fro(got, wv) <= 1e-6
    return got


@pytest.mark.parametrize("op", ["add", "sub", "mul"])
@pytest.mark.parametrize("N", [1, 2, 3, 5])
def test_tew_general_overlapping_patterns(op, N):
    """Different shapes, partly shared coordinates, sizes spanning many sort tiles."""
    rng = np.random.default_rng(40 + N)
    dx = [int(d) for d in rng.integers(20, 60, N)]
    dy = [int(d) for d in rng.integers(20, 60, N)]
    nnz = min(60_000, int(np.prod(dx)) // 3)
    ix = rand_distinct(rng, dx, nnz)
    iy = rand_distinct(rng, dy, nnz // 2 + 7)
    share = iy.shape[1] // 3  # a third of Y's coordinates taken from X (where they fit)
    cand = ix[:, :share]
    fits = np.all(cand < np.array(dy, np.uint32)[:, None], axis=0)
    iy[:, :share][:, fits] = cand[:, fits]
    _, keep = np.unique(iy, axis=1, return_index=True)
    iy = iy[:, np.sort(keep)]
    vx = rng.standard_normal(ix.shape[1])
    vy = rng.standard_normal(iy.shape[1])
    check_tew(op, dx, ix, vx, dy, iy, vy)


def test_tew_general_special_cases():
    rng = np.random.default_rng(50)
    dims = (30, 40, 50)
    ix = rand_distinct(rng, dims, 20_000)
    vx = rng.standard_normal(ix.shape[1])
    vy = rng.standard_normal(ix.shape[1])
    # the same pattern (the paper's setup): the same-pattern result in lexicographic order
    check_tew("add", dims, ix, vx, dims, ix, vy)
    check_tew("mul", dims, ix, vx, dims, ix, vy)
    # disjoint patterns
    iy = ix.copy()
    iy[2] += np.uint32(50)
    got = check_tew("sub", dims, ix, vx, (30, 40, 100), iy, vy)
    assert got.size == 2 * ix.shape[1]
    assert check_tew("mul", dims, ix, vx, (30, 40, 100), iy, vy).size == 0
    # repeated coordinates inside the inputs: summed (fp32 sums)
    ixd = np.concatenate([ix, ix[:, :3000], ix[:, :1000]], axis=1)
    vxd = rng.standard_normal(ixd.shape[1])
    check_tew("add", dims, ixd, vxd, dims, ix[:, 5000:9000], vy[5000:9000], exact=False)
    # empty inputs, and one-cell shapes where every entry has the same coordinate
    e = np.zeros((3, 0), np.uint32)
    check_tew("add", dims, e, np.zeros(0), dims, ix, vy)
    check_tew("sub", dims, ix, vx, dims, e, np.zeros(0))
    dz, iz, vz = api().tew("add", dims, to_dev(e), to_dev(np.zeros(0, np.float32)), dims, to_dev(e),
                           to_dev(np.zeros(0, np.float32)))
    assert dz == dims and vz.numel() == 0
    ones = np.zeros((2, 500), np.uint32)
    check_tew("add", (1, 1), ones, rng.integers(0, 4, 500), (1, 1), ones[:, :300], rng.integers(0, 4, 300))


def test_tew_status_codes():
    import ctypes
    from paper_1902_03317_amd._lib import PastaError, lib
    ix = to_dev(np.array([[0, 1], [2, 0]], np.uint32))
    v = to_dev(np.ones(2, np.float32))
    with pytest.raises(PastaError, match="EUNSUPPORTED"):
        api().tew("div", (2, 3), ix, v, (2, 3), ix, v)
    bad = to_dev(np.array([[0, 1], [3, 0]], np.uint32))  # 3 >= dims[1]
    with pytest.raises(PastaError, match="ERANGE"):
        api().tew("add", (2, 3), bad, v, (2, 3), ix, v)
    assert lib.pasta_tew_eq(9, 2, v.data_ptr(), v.data_ptr(), v.data_ptr(), ctypes.c_void_p(0)) == 1
    assert lib.pasta_ts(1, 2, None, 1.0, v.data_ptr(), ctypes.c_void_p(0)) == 1
    nb = ctypes.c_size_t()
    assert lib.pasta_tew_workspace_bytes(9, 10, 10, ctypes.byref(nb)) == 3


def test_full_size_tensor():
    """On the 50M-nonzero Zipf tensor: TEW-eq and TS against the oracle everywhere (bit-exact),
    and the general TEW of the tensor with itself (the paper's setup): 2x in lexicographic order."""
    import os
    spec = synth.CONFIGS[2]
    coo = synth.load_or_make_coo(spec, os.environ.get("PASTA_BENCH_CACHE", "/tmp/pasta_cache"))
    x = coo.vals
    y = synth.make_factors(spec)[0].ravel()[: x.size]  # any second value array
    y = np.resize(y, x.size).astype(np.float32)
    xd, yd = to_dev(x), to_dev(y)
    assert same_bits(api().tew_eq("add", xd, yd).cpu().numpy(), f32(oracle.tew_eq("add", x, y)))
    assert same_bits(api().ts("mul", xd, 0.3).cpu().numpy(), f32(oracle.ts("mul", x, np.float32(0.3))))
    idx = to_dev(coo.inds)
    dz, iz, vz = api().tew("add", coo.dims, idx, xd, coo.dims, idx, xd)
    o = oracle.lex_order(coo.inds)
    assert dz == coo.dims and vz.numel() == coo.nnz
    assert np.array_equal(iz.cpu().numpy().view(np.uint32), coo.inds[:, o])
    assert same_bits(vz.cpu().numpy(), 2.0 * x[o])
