"""Parity at the full sizes of the measured workloads, in the launch configurations
the benchmark times: the 50Kx40Kx30K / 50M-nonzero Zipf(1.1) tensor (R = 32, fp32
and bf16 factors; the CP fit on its planted values), the 100M-nonzero order-4 and
the 200M-nonzero order-5 tensors (R = 64).

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


def _rows_to_check(coo, n, C, rng):
    """The longest row of mode n, 12 random rows and 8 rows that cross a chunk edge
    (chunks of C nonzeros of the sorted stream)."""
    counts = np.bincount(coo.inds[n], minlength=coo.dims[n])
    starts = np.concatenate([[0], np.cumsum(counts)])
    crossing = np.flatnonzero(((starts[:-1] // C) != ((starts[1:] - 1) // C)) & (counts > 0))
    rows = {int(np.argmax(counts))} | set(int(r) for r in rng.choice(coo.dims[n], 12, replace=False))
    rows |= set(int(r) for r in rng.choice(crossing, min(8, crossing.size), replace=False))
    return sorted(rows), counts


def _chunk(form, dtype):
    """Nonzeros per chunk of the kernel form at rank 32."""
    return 2048 if form == "wave" else 256 * 64 // (8 if dtype == torch.float32 else 4)


@pytest.mark.parametrize("dtype", [torch.float32, torch.bfloat16])
def test_sampled_rows_full_size(full, dtype, mttkrp_form):
    """Both kernel forms; rows crossing the chunk edges of either form are sampled."""
    spec, coo, X = full
    U = synth.make_factors(spec)
    fd = factors_dev(U, dtype)
    U64 = oracle_factors(U, bf16=dtype == torch.bfloat16)
    rng = np.random.default_rng(31)
    for n in range(coo.order):
        out = torch.empty((coo.dims[n], spec.rank), device=DEV)
        from paper_1902_03317_amd import api
        api.mttkrp(X, fd, n, out=out)
        got = out.cpu().numpy().astype(np.float64)
        rows, counts = _rows_to_check(coo, n, _chunk(mttkrp_form, dtype), rng)
        for r in rows:
            want = _row_oracle(coo, U64, n, r)
            if not np.any(want):
                assert not np.any(got[r])
                continue
            assert rel(got[r], want) <= 1e-5, f"mode {n} row {r} ({counts[r]} nonzeros)"


def test_whole_output_full_size(full):
    """Every output row of every mode at full size (the bench's launch configuration,
    R = 32) against the FP64 oracle over all 50M nonzeros: fp32 factors at the fp32 bar;
    bf16 factors at the fp32 bar against the oracle on the bf16-rounded factors
    (accumulation only) and at the bf16 bar end to end (against the fp32 factors)."""
    spec, coo, X = full
    from paper_1902_03317_amd import api
    U = synth.make_factors(spec)
    f32, f16 = factors_dev(U), factors_dev(U, torch.bfloat16)
    U64, U16 = oracle_factors(U), oracle_factors(U, bf16=True)
    vals = coo.vals.astype(np.float64)
    for n in range(coo.order):
        want = oracle.mttkrp(coo.dims, coo.inds, vals, U64, n, "priv")
        want16 = oracle.mttkrp(coo.dims, coo.inds, vals, U16, n, "priv")
        e32 = rel(api.mttkrp(X, f32, n).cpu().numpy().astype(np.float64), want)
        got16 = api.mttkrp(X, f16, n).cpu().numpy().astype(np.float64)
        e16a, e16 = rel(got16, want16), rel(got16, want)
        print(f"mode {n}: fp32 {e32:.2e}, bf16 accumulation {e16a:.2e}, bf16 end to end {e16:.2e}")
        assert e32 <= 1e-5 and e16a <= 1e-5 and e16 <= 1e-2, (n, e32, e16a, e16)


@pytest.mark.parametrize("dtype", [torch.float32, torch.bfloat16])
def test_cp_grad_full_size(full, dtype, mttkrp_form):
    """The fused CP gradient at full size, both kernel forms: the loss against the oracle's
    over all 50M nonzeros, and sampled gradient rows (the residual-weighted MTTKRP of the
    row's own nonzeros, residuals from the oracle)."""
    spec, coo, X = full
    from paper_1902_03317_amd import api
    U = synth.make_factors(spec)
    fd = factors_dev(U, dtype)
    U64 = oracle_factors(U, bf16=dtype == torch.bfloat16)
    loss, grads = api.cp_grad(X, fd)
    wl, resid = oracle.cp_loss(coo.dims, coo.inds, coo.vals, U64)
    assert abs(loss.item() - wl) <= 1e-5 * wl
    rng = np.random.default_rng(37)
    for n in range(coo.order):
        got = grads[n].cpu().numpy().astype(np.float64)
        rows, counts = _rows_to_check(coo, n, _chunk(mttkrp_form, dtype), rng)
        for r in rows:
            sel = np.flatnonzero(coo.inds[n] == r)
            inds = coo.inds[:, sel].copy()
            inds[n] = 0
            dims = list(coo.dims)
            dims[n] = 1
            want = oracle.mttkrp(dims, inds, resid[sel], U64, n)[0]
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


def _sub_oracle(coo, rows, fn, operand, n):
    """The oracle on the sub-tensor made of the given nonzeros only (whole fibers)."""
    return fn(coo.dims, coo.inds[:, rows], coo.vals[rows], operand, n)[2]


@pytest.mark.parametrize("n", [0, 1, 2])
def test_fibers_ttv_ttm_full_size(full, n):
    """Mode-n fibers of the full tensor: the order is fixed by its keys (other modes in
    order, then i_n, then caller position), fptr and coordinates follow from it; TTV and
    TTM (R = 32, fp32 and bf16) on sampled fibers (the longest, fibers crossing chunk
    edges, random ones) against the oracle, and TTV with a ones vector against the
    per-fiber value sums on every fiber."""
    spec, coo, X = full
    from paper_1902_03317_amd import api
    N, M = coo.order, coo.nnz
    F = api.Fibers(X, n)
    gfptr, gcoords, gperm, gfid = F.view()
    p = gperm.cpu().numpy().view(np.uint32).astype(np.int64)
    assert np.array_equal(np.bincount(p, minlength=M), np.ones(M, np.int64))
    other = [k for k in range(N) if k != n]
    cols = [coo.inds[k][p] for k in other + [n]] + [p]
    less = np.zeros(M - 1, bool)
    equal = np.ones(M - 1, bool)
    for c in cols:
        less |= equal & (c[:-1] < c[1:])
        equal &= c[:-1] == c[1:]
    assert less.all()
    new = np.ones(M, bool)
    new[1:] = np.any([c[1:] != c[:-1] for c in cols[:N - 1]], axis=0)
    fptr = np.append(np.flatnonzero(new), M)
    del cols, less, equal, new
    assert F.nfibs == fptr.size - 1
    assert np.array_equal(gfptr.cpu().numpy().view(np.uint32), fptr)
    for q, k in enumerate(other):
        assert np.array_equal(gcoords[q].cpu().numpy().view(np.uint32), coo.inds[k][p[fptr[:-1]]])
    lens = np.diff(fptr)
    assert np.array_equal(gfid.cpu().numpy().view(np.uint32), np.repeat(np.arange(F.nfibs, dtype=np.uint32), lens))

    # every fiber: TTV with a ones vector is the fiber's value sum
    ones = torch.ones(coo.dims[n], device=DEV)
    got1 = api.ttv(F, ones).cpu().numpy().astype(np.float64)
    sums = np.add.reduceat(coo.vals[p].astype(np.float64), fptr[:-1])
    assert rel(got1, sums) <= 1e-6

    U = synth.make_factors(spec)[n]
    rng = np.random.default_rng(40 + n)
    v = U[:, 0].copy()
    gotv = api.ttv(F, torch.from_numpy(v).to(DEV)).cpu().numpy().astype(np.float64)
    got32 = api.ttm(F, torch.from_numpy(U).to(DEV)).cpu().numpy().astype(np.float64)
    got16 = api.ttm(F, torch.from_numpy(U).to(DEV).to(torch.bfloat16)).cpu().numpy().astype(np.float64)
    picks = {int(np.argmax(lens))} | set(int(f) for f in rng.choice(F.nfibs, 12, replace=False))
    for C in (1024, 2048):  # TTV chunk; TTM chunk at R = 32 fp32
        cross = np.flatnonzero((fptr[:-1] // C) != ((fptr[1:] - 1) // C))
        picks |= set(int(f) for f in rng.choice(cross, min(8, cross.size), replace=False))
    picks = sorted(picks)
    rows = np.concatenate([p[fptr[f]:fptr[f + 1]] for f in picks])
    want_v = _sub_oracle(coo, rows, oracle.ttv, v.astype(np.float64), n)
    want_m = _sub_oracle(coo, rows, oracle.ttm, U.astype(np.float64), n)
    want_b = _sub_oracle(coo, rows, oracle.ttm, oracle.bf16_round(U).astype(np.float64), n)
    assert want_m.shape[0] == len(picks)
    assert rel(gotv[picks], want_v) <= 1e-5
    for i, f in enumerate(picks):
        assert rel(got32[f], want_m[i]) <= 1e-5, f"ttm fiber {f} ({lens[f]} nonzeros)"
        assert rel(got16[f], want_b[i]) <= 1e-5, f"ttm bf16 fiber {f} ({lens[f]} nonzeros)"


# ---- the order-4 (100M nonzeros, R = 64) and order-5 (200M nonzeros, R = 64) workloads ----

def _load(cfg):
    spec = synth.CONFIGS[cfg]
    coo = synth.load_or_make_coo(spec, CACHE)
    return spec, coo, upload(coo)


@pytest.fixture(scope="module")
def order4():
    return _load(3)


@pytest.fixture(scope="module")
def order5():
    return _load(5)


def _sampled_rows(spec, coo, X, dtype, seed, nrand=6, ncross=4):
    """MTTKRP of every mode at full size, checked on the hottest row, rows crossing chunk
    edges and random non-empty rows, each computed by the oracle from that row's nonzeros."""
    from paper_1902_03317_amd import api
    U = synth.make_factors(spec)
    fd = factors_dev(U, dtype)
    U64 = oracle_factors(U, bf16=dtype == torch.bfloat16)
    rng = np.random.default_rng(seed)
    R = spec.rank
    lanes = max(1, R * (2 if dtype == torch.bfloat16 else 4) // 16)
    Cs = (256 * (64 // lanes), 2048)  # nonzeros per chunk of the run form and of the wave-run form
    worst = 0.0
    for n in range(coo.order):
        out = api.mttkrp(X, fd, n).cpu().numpy().astype(np.float64)
        counts = np.bincount(coo.inds[n], minlength=coo.dims[n])
        starts = np.concatenate([[0], np.cumsum(counts)])
        nonempty = np.flatnonzero(counts)
        crossing = np.flatnonzero(np.logical_or.reduce([(starts[:-1] // C) != ((starts[1:] - 1) // C) for C in Cs])
                                  & (counts > 0))
        rows = {int(np.argmax(counts))} | set(int(r) for r in rng.choice(nonempty, min(nrand, nonempty.size),
                                                                        replace=False))
        rows |= set(int(r) for r in rng.choice(crossing, min(ncross, crossing.size), replace=False))
        empty = np.flatnonzero(counts == 0)
        if empty.size:
            assert not np.any(out[empty[: 1000]])
        for r in sorted(rows):
            want = _row_oracle(coo, U64, n, r)
            e = rel(out[r], want)
            worst = max(worst, e)
            assert e <= 1e-5, f"mode {n} row {r} ({counts[r]} nonzeros): {e:.3e}"
        del out
    return worst


def test_order4_full_size_sampled_rows(order4):
    spec, coo, X = order4
    _sampled_rows(spec, coo, X, torch.float32, 51)


def test_order4_full_size_all_ones_marginals(order4):
    spec, coo, X = order4
    from paper_1902_03317_amd import api
    for n in range(coo.order):
        ones = [torch.ones((d, 8), device=DEV) for d in coo.dims]
        got = api.mttkrp(X, ones, n).cpu().numpy().astype(np.float64)
        marg = np.bincount(coo.inds[n], weights=coo.vals.astype(np.float64), minlength=coo.dims[n])
        assert rel(got, np.repeat(marg[:, None], 8, axis=1)) <= 1e-6


@pytest.mark.parametrize("dtype", [torch.float32, torch.bfloat16])
def test_order5_full_size_sampled_rows(order5, dtype):
    """fp32 and bf16 factor storage; with bf16 the rows are compared with the oracle on the
    bf16-rounded factors (fp32 accumulation error only, the fp32 bar)."""
    spec, coo, X = order5
    _sampled_rows(spec, coo, X, dtype, 52 if dtype == torch.float32 else 53, nrand=4, ncross=3)


def test_order5_full_size_all_ones_marginals(order5):
    spec, coo, X = order5
    from paper_1902_03317_amd import api
    for n in range(coo.order):
        ones = [torch.ones((d, 4), device=DEV) for d in coo.dims]
        got = api.mttkrp(X, ones, n).cpu().numpy().astype(np.float64)
        marg = np.bincount(coo.inds[n], weights=coo.vals.astype(np.float64), minlength=coo.dims[n])
        assert rel(got, np.repeat(marg[:, None], 4, axis=1)) <= 1e-6


@pytest.mark.parametrize("dtype", [torch.float32, torch.bfloat16])
def test_order5_full_size_cp_grad(order5, dtype):
    """The fused CP gradient on the 200M-nonzero order-5 tensor (R = 64): its loss against
    the FP64 oracle's over all 200M nonzeros, sampled residuals against the oracle, and
    gradient rows (the hottest row of every mode, 21M to 44M nonzeros, plus random and
    chunk-edge-crossing rows) against the oracle's residual-weighted MTTKRP of that row's
    nonzeros. bf16 factors are compared with the oracle on the bf16-rounded factors."""
    spec, coo, X = order5
    from paper_1902_03317_amd import api
    U = synth.make_factors(spec)
    fd = factors_dev(U, dtype)
    U64 = oracle_factors(U, bf16=dtype == torch.bfloat16)
    loss, grads = api.cp_grad(X, fd)
    wl, _ = oracle.cp_loss(coo.dims, coo.inds, coo.vals, U64)
    print(f"loss rel error {abs(loss.item() - wl) / wl:.2e}")
    assert abs(loss.item() - wl) <= 1e-5 * wl
    resid, loss_r = api.cp_residual_loss(X, fd)
    assert abs(loss_r.item() - wl) <= 1e-5 * wl
    rng = np.random.default_rng(61 if dtype == torch.float32 else 62)
    pick = rng.choice(coo.nnz, 100_000, replace=False)
    _, want_res = oracle.cp_loss(coo.dims, coo.inds[:, pick], coo.vals[pick], U64)
    assert rel(resid.cpu().numpy()[pick].astype(np.float64), want_res) <= 1e-5
    del resid
    lanes = max(1, spec.rank * (2 if dtype == torch.bfloat16 else 4) // 16)
    Cs = (256 * (64 // lanes), 2048)
    for n in range(coo.order):
        got = grads[n].cpu().numpy().astype(np.float64)
        counts = np.bincount(coo.inds[n], minlength=coo.dims[n])
        starts = np.concatenate([[0], np.cumsum(counts)])
        crossing = np.flatnonzero(np.logical_or.reduce([(starts[:-1] // C) != ((starts[1:] - 1) // C) for C in Cs])
                                  & (counts > 0))
        cand = np.flatnonzero(counts > 0)
        rows = {int(np.argmax(counts))}
        rows |= set(int(r) for r in rng.choice(cand, min(3, cand.size), replace=False))
        rows |= set(int(r) for r in rng.choice(crossing, min(2, crossing.size), replace=False))
        for r in sorted(rows):
            sel = np.flatnonzero(coo.inds[n] == r)
            _, res = oracle.cp_loss(coo.dims, coo.inds[:, sel], coo.vals[sel], U64)
            inds = coo.inds[:, sel].copy()
            inds[n] = 0
            dims = list(coo.dims)
            dims[n] = 1
            want = oracle.mttkrp(dims, inds, res, U64, n, "priv")[0]
            e = rel(got[r], want)
            print(f"mode {n} row {r} ({counts[r]} nonzeros): rel-Fro {e:.2e}")
            assert e <= 1e-5, f"mode {n} row {r} ({counts[r]} nonzeros): {e:.3e}"
        del got


# ---- the CP fit at its stated size: 50 Adam steps on the 50M-nonzero planted tensor ----

@pytest.fixture(scope="module")
def planted_full(full):
    """The coordinates of the 50M-nonzero tensor with planted rank-32 CP values plus 1%
    Gaussian noise (its rms times N(0,1)); the fit starts from an independent draw."""
    spec, coo, _ = full
    cspec = synth.CONFIGS[4]
    R = cspec.rank
    sc = synth.cp_planted_scale(R, 3)
    A = synth.make_factors(cspec, rank=R, scale=sc)
    x = oracle.cp_sample(coo.dims, coo.inds, oracle_factors(A))
    x = x + 0.01 * np.sqrt(np.mean(x * x)) * synth.make_noise(cspec, coo.nnz)
    pc = synth.CooTensor(coo.dims, coo.inds, x.astype(np.float32), cspec)
    return cspec, pc, upload(pc), synth.make_init(cspec, rank=R, scale=sc)


@pytest.mark.parametrize("dtype", [torch.float32, torch.bfloat16])
def test_cp_fit_50_adam_steps_full_size(planted_full, dtype):
    """50 Adam steps (lr 1e-2) of the fused CP gradient on the full 50M-nonzero planted
    tensor: the loss falls; at the final factors the loss over all nonzeros and sampled
    gradient rows (each mode's hottest row, random and chunk-edge-crossing rows) match the
    FP64 oracle (bf16: on the bf16 shadows the step read, and end to end at the bf16 bar)."""
    from paper_1902_03317_amd import api
    from paper_1902_03317_amd.autograd import adam_step
    cspec, pc, X, init = planted_full
    masters = factors_dev(init)
    shadows = [api.cast_bf16(m) for m in masters] if dtype == torch.bfloat16 else None
    ms = [torch.zeros_like(m) for m in masters]
    vs = [torch.zeros_like(m) for m in masters]
    losses = []
    for t in range(1, 51):
        loss, grads = api.cp_grad(X, shadows if shadows is not None else masters)
        losses.append(loss.item())
        adam_step(masters, grads, ms, vs, t, lr=1e-2, shadows=shadows)
    print("loss", losses[0], "->", losses[-1])
    assert all(np.isfinite(losses))
    assert losses[-1] < 0.7 * losses[0]
    final = [m.cpu().numpy() for m in masters]
    fo = oracle_factors(final, bf16=dtype == torch.bfloat16)
    loss, grads = api.cp_grad(X, shadows if shadows is not None else masters)
    wl, resid = oracle.cp_loss(pc.dims, pc.inds, pc.vals, fo)
    assert abs(loss.item() - wl) <= 1e-5 * wl
    rng = np.random.default_rng(71)
    f32 = oracle_factors(final)
    for n in range(pc.order):
        got = grads[n].cpu().numpy().astype(np.float64)
        rows, counts = _rows_to_check(pc, n, 2048, rng)
        hot = int(np.argmax(counts))
        for r in [hot] + [r for r in rows if r != hot and counts[r] > 0][:7]:
            sel = np.flatnonzero(pc.inds[n] == r)
            inds = pc.inds[:, sel].copy()
            inds[n] = 0
            dims = list(pc.dims)
            dims[n] = 1
            want = oracle.mttkrp(dims, inds, resid[sel], fo, n)[0]
            assert rel(got[r], want) <= 1e-5, f"mode {n} row {r} ({counts[r]} nonzeros)"
            if dtype == torch.bfloat16:
                _, r32 = oracle.cp_loss(dims, inds, pc.vals[sel], [f if k != n else f[r:r + 1]
                                                                 for k, f in enumerate(f32)])
                want32 = oracle.mttkrp(dims, inds, r32, f32, n)[0]
                assert rel(got[r], want32) <= 1e-2, f"mode {n} row {r} end to end"
