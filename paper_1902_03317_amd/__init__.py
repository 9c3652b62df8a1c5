"""MI355X-native COO MTTKRP (mode-n matricized tensor times Khatri-Rao product),
with the CP model and CP-ALS built on it, the fiber-based sparse TTM / TTV and
the element-wise (TEW) and tensor-scalar (TS) operations.

The compute path lives in ``libpasta.so`` (HIP kernels for gfx950 behind a
C ABI, declared in ``include/pasta.h``); this package is its thin Python
binding. The binding is loaded on first use of the API, so the input
generator in :mod:`.synth` can be imported without it.
"""

__all__ = ["Coo", "mttkrp", "mttkrp_workspace_bytes", "cp_sample", "cp_residual_loss", "cast_bf16", "cp_grad",
           "cp_als_sweep", "mttkrp_atomic", "Fibers", "ttm", "ttv",
           "tew_eq", "ts", "tew", "CPSample", "CPLoss", "lib"]


def __getattr__(name):
    if name in ("Coo", "mttkrp", "mttkrp_workspace_bytes", "cp_sample", "cp_residual_loss", "cast_bf16",
                "cp_grad", "cp_als_sweep", "mttkrp_atomic", "Fibers", "ttm", "ttv",
                "tew_eq", "ts", "tew"):
        from . import api
        return getattr(api, name)
    if name in ("CPSample", "CPLoss"):
        from . import autograd
        return getattr(autograd, name)
    if name == "lib":
        from . import _lib
        return _lib
    raise AttributeError(name)
