"""CP-ALS sweeps on the GPU against the FP64 oracle.

Each mode's update is checked on its own: after a GPU sweep, the oracle redoes the
update of mode n from the factors that update saw (modes before n as the GPU left
them, modes after n as they started), so one mode's rounding does not compound into
the next mode's check. The bar of an update is max(1e-5, 1e-6 * cond(V_n)): the
update solves V_n U_n^T = M^T in fp32, whose inputs (the MTTKRP and the Gram
matrices) carry relative errors of order 1e-7 .. 1e-6, and a solve passes its
inputs' relative error on amplified by up to the condition number of V_n."""
import numpy as np
import pytest

import oracle
from helpers import factors_dev, rel, upload
from paper_1902_03317_amd import synth

pytestmark = [pytest.mark.gpu, pytest.mark.usefixtures("mttkrp_form")]


def api():
    from paper_1902_03317_amd import api as a
    return a


ORDER3 = (2, (3000, 2000, 1000), 200_000)
ORDER4 = (3, (20_000, 2000, 1000, 200), 300_000)
ORDER5 = (5, (50_000, 50_000, 5000, 1000, 100), 200_000)


@pytest.mark.parametrize("shape,R", [(ORDER3, 16), (ORDER3, 48), (ORDER3, 64), (ORDER4, 32), (ORDER4, 64),
                                     (ORDER5, 8), (ORDER5, 48), (ORDER5, 64)])
def test_one_sweep_matches_oracle(shape, R):
    cfg, dims, nnz = shape
    sp = synth.CONFIGS[cfg].scaled(nnz, dims=dims)
    coo = synth.make_coo(sp)
    X = upload(coo)
    U0 = [u.astype(np.float64) for u in synth.make_factors(sp, rank=R)]
    U = factors_dev(U0)
    lam, fit, info = api().cp_als_sweep(X, U)
    assert int(info.item()) == 0
    got = [u.cpu().numpy().astype(np.float64) for u in U]
    N = coo.order
    for n in range(N):
        seen = [got[k] if k < n else U0[k] for k in range(N)]
        Un, ln, _, kappa = oracle.cp_als_update(coo.dims, coo.inds, coo.vals, seen, n, "priv")
        tol = max(1e-5, 1e-6 * kappa)
        e = rel(got[n], Un)
        print(f"R={R} order {N} mode {n}: cond(V) {kappa:.3g}, rel-Fro {e:.2e} (bar {tol:.1e})")
        assert e <= tol, (n, e, kappa)
        if n == N - 1:
            assert rel(lam.cpu().numpy(), ln) <= tol
    # the fit the GPU reports, against the fit's definition at the GPU's final factors
    want = oracle.cp_fit(coo.dims, coo.inds, coo.vals, got, lam.cpu().numpy().astype(np.float64))
    assert abs(fit.item() - want) <= 1e-5, (fit.item(), want)


def test_sweeps_recover_planted_model():
    """Planted rank-8 values on a Zipf pattern: repeated sweeps raise the fit at every
    sweep, and the fit the GPU reports is the fit of the factors it returns."""
    sp = synth.CONFIGS[4].scaled(300_000, dims=(3000, 2000, 1000))
    coo = synth.make_coo(sp)
    A = synth.make_factors(sp, rank=8, scale=synth.cp_planted_scale(8, 3))
    coo.vals = oracle.cp_sample(coo.dims, coo.inds, [a.astype(np.float64) for a in A]).astype(np.float32)
    X = upload(coo)
    U = factors_dev(synth.make_init(sp, rank=8))
    fits = []
    for _ in range(15):
        lam, fit, info = api().cp_als_sweep(X, U)
        fits.append(fit.item())
    # each ALS update minimises the residual over one factor, so the fit never falls (to
    # rounding); the tensor is zero off its nonzeros, so it rises slowly from a random start
    assert fits[-1] > fits[0] and np.all(np.diff(fits) > -1e-6), fits
    # the fit reported on the GPU is the fit's definition at the factors it returned
    want = oracle.cp_fit(coo.dims, coo.inds, coo.vals, [u.cpu().numpy().astype(np.float64) for u in U],
                         lam.cpu().numpy().astype(np.float64))
    assert abs(fits[-1] - want) <= 1e-5, (fits[-1], want)
