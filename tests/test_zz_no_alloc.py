"""pasta_mttkrp_static, the MTTKRP entry point that allocates nothing (its scratch is a
fixed array inside the library), called through the C ABI: its output equals
pasta_mttkrp's with a caller workspace, bit for bit (the same kernels in the same
order), and both are within the fp32 bar of the FP64 oracle, on two calls in a row
with the second on a smaller tensor (the array keeps the first call's contents). A
call that needs more scratch than the array holds is refused before any launch."""
import ctypes

import numpy as np
import pytest
import torch

import oracle
from helpers import DEV, factors_dev, oracle_factors, rel, upload
from paper_1902_03317_amd import synth

pytestmark = pytest.mark.gpu


def _static(X, U, n, out, stream):
    from paper_1902_03317_amd import api
    from paper_1902_03317_amd._lib import lib, ptr_array
    facs = [None if k == n else f for k, f in enumerate(U)]
    ptrs = ptr_array([0 if f is None else f.data_ptr() for f in facs])
    dt = 0 if U[0].dtype == torch.float32 else 1
    return lib.pasta_mttkrp_static(X.handle, n, ptrs, dt, U[0].shape[1], U[0].stride(0), None, 1.0,
                                   out.data_ptr(), out.stride(0), api._stream(stream))


def _one_tensor(nnz, dims, R, dtype, form):
    from paper_1902_03317_amd import api
    from paper_1902_03317_amd._lib import lib
    lib.pasta_set_mttkrp_form(form)
    try:
        sp = synth.CONFIGS[2].scaled(nnz, dims=dims)
        coo = synth.make_coo(sp)
        X = upload(coo)
        U = synth.make_factors(sp, rank=R)
        fd = factors_dev(U, dtype)
        fo = oracle_factors(U, bf16=dtype == torch.bfloat16)
        s = torch.cuda.current_stream()
        for n in range(coo.order):
            got = torch.full((coo.dims[n], R), float("nan"), device=DEV)
            assert _static(X, fd, n, got, s) == 0
            ref = api.mttkrp(X, fd, n)
            torch.cuda.synchronize()
            assert torch.equal(got, ref), f"mode {n}: static scratch and workspace differ"
            want = oracle.mttkrp(coo.dims, coo.inds, coo.vals, fo, n, "priv")
            assert rel(got.cpu().numpy().astype(np.float64), want) <= 1e-5
        X.check()
    finally:
        lib.pasta_set_mttkrp_form(0)


@pytest.mark.parametrize("form", [1, 2])  # run form, wave-run form
def test_static_scratch_two_calls_second_smaller(form):
    _one_tensor(2_000_000, (20_000, 15_000, 10_000), 32, torch.float32, form)
    _one_tensor(150_000, (3000, 2000, 1000), 32, torch.float32, form)
    _one_tensor(100_000, (2000, 1500, 1000), 64, torch.bfloat16, form)


def test_static_scratch_refuses_calls_that_need_more():
    """R = 256 in fp32 takes the strided shape: 256 nonzeros per chunk and two 1 KiB
    partial rows per chunk, so 9M nonzeros need more than the 64 MiB array."""
    from paper_1902_03317_amd import api
    from paper_1902_03317_amd._lib import lib
    nnz = 9_000_000
    sp = synth.CONFIGS[2].scaled(nnz, dims=(4000, 3000, 2000))
    X = upload(synth.make_coo(sp))
    need = api.mttkrp_workspace_bytes(X, 0, 256)
    assert need > (64 << 20)
    U = [torch.zeros((d, 256), device=DEV) for d in sp.dims]
    out = torch.empty((sp.dims[0], 256), device=DEV)
    assert _static(X, U, 0, out, torch.cuda.current_stream()) == 4  # PASTA_EWORKSPACE
    assert lib.pasta_status_str(4) == b"workspace too small or misaligned"
