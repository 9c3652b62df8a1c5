"""Sampled CP model, its residual loss and the residual-weighted MTTKRP gradient on
the GPU against the FP64 oracle; autograd against finite differences and a dense
reference gradient on a fully observed 30x20x10 head block."""
import numpy as np
import pytest
import torch

import oracle
from oracle import brute
from helpers import DEV, coo_from_arrays, factors_dev, oracle_factors, rel, to_dev, upload
from paper_1902_03317_amd import synth

pytestmark = [pytest.mark.gpu, pytest.mark.usefixtures("mttkrp_form")]


def api():
    from paper_1902_03317_amd import api as a
    return a


def planted(nnz=200_000, dims=(5000, 4000, 3000), R=32, noise=0.0):
    sp = synth.CONFIGS[4].scaled(nnz, dims=dims)
    coo = synth.make_coo(sp)
    A = synth.make_factors(sp, rank=R, scale=synth.cp_planted_scale(R, 3))
    x = oracle.cp_sample(coo.dims, coo.inds, oracle_factors(A))
    if noise:
        x = x + noise * np.sqrt(np.mean(x * x)) * synth.make_noise(sp, coo.nnz)
    coo.vals = x.astype(np.float32)
    return sp, coo, A


@pytest.mark.parametrize("dtype", [torch.float32, torch.bfloat16])
def test_cp_sample_and_loss(dtype):
    sp, coo, A = planted(noise=0.01)
    X = upload(coo)
    U = synth.make_init(sp, rank=32, scale=synth.cp_planted_scale(32, 3))
    fd = factors_dev(U, dtype)
    fo = oracle_factors(U, bf16=dtype == torch.bfloat16)
    tol = 1e-5 if dtype == torch.float32 else 1e-5  # vs the oracle on the same (rounded) factors
    mhat = api().cp_sample(X, fd).cpu().numpy()
    want = oracle.cp_sample(coo.dims, coo.inds, fo)
    assert rel(mhat, want) <= tol
    resid, loss = api().cp_residual_loss(X, fd)
    wl, wr = oracle.cp_loss(coo.dims, coo.inds, coo.vals, fo)
    assert rel(resid.cpu().numpy(), wr) <= tol
    assert abs(loss.item() - wl) <= 1e-5 * wl


def test_planted_factors_reproduce_values():
    sp, coo, A = planted()
    X = upload(coo)
    mhat = api().cp_sample(X, factors_dev(A)).cpu().numpy()
    assert rel(mhat, coo.vals) <= 1e-6


@pytest.mark.parametrize("dtype", [torch.float32, torch.bfloat16])
def test_cp_grad_fused(dtype):
    sp, coo, A = planted(noise=0.01)
    X = upload(coo)
    U = synth.make_init(sp, rank=32, scale=synth.cp_planted_scale(32, 3))
    fd = factors_dev(U, dtype)
    loss, grads = api().cp_grad(X, fd)
    fo = oracle_factors(U, bf16=dtype == torch.bfloat16)
    wl, wg = oracle.cp_grad(coo.dims, coo.inds, coo.vals, fo, "priv")
    assert abs(loss.item() - wl) <= 1e-5 * wl
    for n in range(3):
        assert rel(grads[n].cpu().numpy(), wg[n]) <= 1e-5
    # end to end against fp32 factors in fp64: the bf16 error bar
    if dtype == torch.bfloat16:
        _, wg32 = oracle.cp_grad(coo.dims, coo.inds, coo.vals, oracle_factors(U), "priv")
        for n in range(3):
            assert rel(grads[n].cpu().numpy(), wg32[n]) <= 1e-2


@pytest.mark.parametrize("dtype", [torch.float32, torch.bfloat16])
@pytest.mark.parametrize("order", [4, 5])
def test_cp_grad_orders_4_5_and_residual_path_agree(order, dtype):
    """R = 64 at orders 4 and 5 (each has its own gather-group size in the fused kernel):
    the fused gradient and the residual-weighted MTTKRP against the oracle."""
    if order == 5:
        sp = synth.CONFIGS[5].scaled(200_000, dims=(50_000, 50_000, 5000, 1000, 100))
    else:
        sp = synth.CONFIGS[3].scaled(200_000, dims=(20_000, 5000, 1000, 200))
    coo = synth.make_coo(sp)
    X = upload(coo)
    U = synth.make_factors(sp, rank=64, scale=synth.cp_planted_scale(64, order))
    fd = factors_dev(U, dtype)
    loss, grads = api().cp_grad(X, fd)
    U64 = oracle_factors(U, bf16=dtype == torch.bfloat16)
    wl, wg = oracle.cp_grad(coo.dims, coo.inds, coo.vals, U64, "priv")
    assert abs(loss.item() - wl) <= 1e-5 * wl
    resid, _ = api().cp_residual_loss(X, fd)
    for n in range(order):
        assert rel(grads[n].cpu().numpy(), wg[n]) <= 1e-5
        g2 = api().mttkrp(X, fd, n, vals=resid).cpu().numpy()
        assert rel(g2, wg[n]) <= 1e-5


def _head_block():
    """The 30x20x10 head block of the full 50Kx40Kx30K / 50M-nonzero Zipf(1.1) tensor:
    at that size every one of its 6000 cells is present."""
    sp = synth.CONFIGS[4]
    coo = synth.make_coo(sp)
    blk = synth.head_block(coo, sp, (30, 20, 10))
    return sp, blk


@pytest.mark.parametrize("R", [8, 32])
def test_autograd_finite_differences_and_dense_gradient(R):
    """R = 32 is the CP fit's rank; the entries are scaled so the model's values are O(1)."""
    from paper_1902_03317_amd.autograd import cp_loss
    sp, blk = _head_block()
    assert blk.nnz == 6000  # every cell of the block is present
    rng = np.random.default_rng(9)
    A = [rng.standard_normal((d, R)).astype(np.float32) * np.float32(R ** (-1.0 / 6.0)) for d in blk.dims]
    X = upload(blk)
    masters = [t.clone().requires_grad_(True) for t in factors_dev(A)]
    loss = cp_loss(X, masters)
    loss.backward()
    g = [m.grad.cpu().numpy().astype(np.float64) for m in masters]
    fo = oracle_factors(A)
    # (i) central differences of the fp64 oracle loss at 200 random entries
    for _ in range(200):
        n = int(rng.integers(0, 3))
        i = int(rng.integers(0, blk.dims[n]))
        r = int(rng.integers(0, R))
        h = 1e-6 * max(1.0, abs(fo[n][i, r]))
        up = [f.copy() for f in fo]
        dn = [f.copy() for f in fo]
        up[n][i, r] += h
        dn[n][i, r] -= h
        fd = (oracle.cp_loss(blk.dims, blk.inds, blk.vals, up)[0] -
              oracle.cp_loss(blk.dims, blk.inds, blk.vals, dn)[0]) / (2 * h)
        assert abs(g[n][i, r] - fd) <= 1e-4 * max(1.0, abs(fd))
    # (ii) dense reference: full CP gradient U_n (*_k U_k^T U_k) - X_(n) KRP
    Xd = brute.dense(blk.dims, blk.inds, blk.vals)
    for n in range(3):
        G = np.ones((R, R))
        for k in range(3):
            if k != n:
                G *= fo[k].T @ fo[k]
        want = fo[n] @ G - brute.mttkrp_dense(Xd, fo, n)
        assert rel(g[n], want) <= 1e-5
    # (iii) the unfused autograd path (residual forward, residual-weighted MTTKRP backward)
    masters2 = [t.clone().requires_grad_(True) for t in factors_dev(A)]
    loss2 = cp_loss(X, masters2, fused=False)
    loss2.backward()
    assert abs(loss2.item() - loss.item()) <= 1e-6 * loss.item()
    for n in range(3):
        assert rel(masters2[n].grad.cpu().numpy(), g[n]) <= 1e-5


def test_cp_sample_autograd_backward_is_mttkrp():
    from paper_1902_03317_amd.autograd import CPSample
    sp, coo, A = planted(nnz=50_000, dims=(800, 600, 400), R=16)
    X = upload(coo)
    U = [t.requires_grad_(True) for t in factors_dev(synth.make_init(sp, rank=16))]
    mhat = CPSample.apply(X, *U)
    w = torch.from_numpy(np.random.default_rng(3).standard_normal(coo.nnz).astype(np.float32)).to(DEV)
    mhat.backward(w)
    fo = oracle_factors([u.detach().cpu().numpy() for u in U])
    for n in range(3):
        want = oracle.mttkrp(coo.dims, coo.inds, w.cpu().numpy(), fo, n)
        assert rel(U[n].grad.cpu().numpy(), want) <= 1e-5


def test_bf16_mixed_precision_loss_uses_fp32_masters():
    from paper_1902_03317_amd.autograd import cp_loss
    sp, coo, A = planted(nnz=100_000, noise=0.01)
    X = upload(coo)
    U = synth.make_init(sp, rank=32, scale=synth.cp_planted_scale(32, 3))
    masters = [t.requires_grad_(True) for t in factors_dev(U)]
    shadows = [api().cast_bf16(m.detach()) for m in masters]
    loss = cp_loss(X, masters, shadows=shadows)
    loss.backward()
    _, wg = oracle.cp_grad(coo.dims, coo.inds, coo.vals, oracle_factors(U), "priv")
    for n in range(3):
        assert masters[n].grad.dtype == torch.float32
        assert rel(masters[n].grad.cpu().numpy(), wg[n]) <= 1e-2


def test_adam_step_matches_torch_adam():
    """The fused Adam kernel against torch.optim.Adam (fp64, CPU) over three steps; the
    bf16 copy it writes equals round-to-nearest-even of the updated parameters."""
    from paper_1902_03317_amd.autograd import adam_step
    rng = np.random.default_rng(41)
    p0 = rng.standard_normal((1000, 32)).astype(np.float32)
    grads = [rng.standard_normal((1000, 32)).astype(np.float32) for _ in range(3)]
    p = torch.from_numpy(p0.copy()).to(DEV)
    m, v = torch.zeros_like(p), torch.zeros_like(p)
    sh = torch.empty(p.shape, dtype=torch.bfloat16, device=DEV)
    ref = torch.from_numpy(p0.astype(np.float64)).requires_grad_(True)
    opt = torch.optim.Adam([ref], lr=1e-2, betas=(0.9, 0.999), eps=1e-8)
    for t, g in enumerate(grads, start=1):
        adam_step([p], [torch.from_numpy(g).to(DEV)], [m], [v], t, lr=1e-2, shadows=[sh])
        ref.grad = torch.from_numpy(g.astype(np.float64))
        opt.step()
    got = p.cpu().numpy()
    assert rel(got, ref.detach().numpy()) <= 1e-6
    assert np.array_equal(sh.view(torch.int16).cpu().numpy().view(np.uint16), oracle.bf16_bits(got))


@pytest.mark.parametrize("dtype", [torch.float32, torch.bfloat16])
def test_cp_fit_50_adam_steps(dtype):
    """50 Adam steps of the fused CP gradient on a planted rank-32 tensor with 1% noise:
    the loss falls, and the final gradient matches the FP64 oracle's at the same factors."""
    from paper_1902_03317_amd import api
    from paper_1902_03317_amd.autograd import adam_step
    sp, coo, A = planted(nnz=400_000, dims=(4000, 3000, 2000), R=32, noise=0.01)
    X = upload(coo)
    U = synth.make_init(sp, rank=32, scale=synth.cp_planted_scale(32, 3))
    masters = factors_dev(U)
    shadows = [api.cast_bf16(m) for m in masters] if dtype == torch.bfloat16 else None
    ms = [torch.zeros_like(m) for m in masters]
    vs = [torch.zeros_like(m) for m in masters]
    losses = []
    for t in range(1, 51):
        loss, grads = api.cp_grad(X, shadows if shadows is not None else masters)
        losses.append(loss.item())
        adam_step(masters, grads, ms, vs, t, lr=1e-2, shadows=shadows)
    assert losses[-1] < 0.5 * losses[0]
    assert all(np.isfinite(losses))
    final = [m.cpu().numpy() for m in masters]
    fo = oracle_factors(final, bf16=dtype == torch.bfloat16)
    loss, grads = api.cp_grad(X, shadows if shadows is not None else masters)
    wl, wg = oracle.cp_grad(coo.dims, coo.inds, coo.vals, fo, "priv")
    assert abs(loss.item() - wl) <= 1e-5 * wl
    for n in range(3):
        assert rel(grads[n].cpu().numpy(), wg[n]) <= 1e-5
    if dtype == torch.bfloat16:  # end to end against the fp32 masters in fp64
        _, wg32 = oracle.cp_grad(coo.dims, coo.inds, coo.vals, oracle_factors(final), "priv")
        for n in range(3):
            assert rel(grads[n].cpu().numpy(), wg32[n]) <= 1e-2
