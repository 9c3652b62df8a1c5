"""Shared helpers for the GPU parity tests (uploading synthetic tensors and
running the oracle on the same inputs)."""
import numpy as np
import torch

import oracle
from paper_1902_03317_amd import synth

DEV = "cuda:0"


def to_dev(a: np.ndarray) -> torch.Tensor:
    if a.dtype == np.uint32:
        a = a.view(np.int32)
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def upload(coo: synth.CooTensor):
    from paper_1902_03317_amd import api
    return api.Coo(coo.dims, to_dev(coo.inds), to_dev(coo.vals))


def factors_dev(factors, dtype=torch.float32, ld=None):
    out = []
    for f in factors:
        t = torch.from_numpy(np.ascontiguousarray(f, dtype=np.float32))
        if ld is not None and ld > f.shape[1]:
            pad = torch.zeros((f.shape[0], ld), dtype=torch.float32)
            pad[:, : f.shape[1]] = t
            t = pad[:, : f.shape[1]]
        out.append(t.to(DEV).to(dtype) if dtype != torch.float32 else t.to(DEV))
    return out


def oracle_factors(factors, bf16=False):
    """FP64 copies of the factors the GPU sees (bf16-rounded by the oracle's own rule if asked)."""
    return [(oracle.bf16_round(f) if bf16 else np.asarray(f, np.float32)).astype(np.float64) for f in factors]


def coo_from_arrays(dims, inds, vals):
    return synth.CooTensor(tuple(int(d) for d in dims), np.ascontiguousarray(inds, dtype=np.uint32),
                           np.ascontiguousarray(vals, dtype=np.float32))


def rel(a, b):
    return oracle.rel_fro(a, b)
