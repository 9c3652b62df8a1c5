"""Python API over libpasta. torch supplies device memory and streams; every
computation is a call into the HIP library through the C ABI."""
from __future__ import annotations

import ctypes
from typing import List, Optional, Sequence

import torch

from . import _lib
from ._lib import check, lib, ptr_array

_DT = {torch.float32: _lib.PASTA_F32, torch.bfloat16: _lib.PASTA_BF16}


def _stream(stream=None) -> ctypes.c_void_p:
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _scratch(nbytes: int, device, stream=None) -> torch.Tensor:
    """Device scratch for one call. It is allocated while the call's stream is current, so
    torch's caching allocator hands the block to other work only in that stream's order
    (a block taken on another stream could be reused while the call's kernels still run)."""
    n = max(int(nbytes), 256)
    if stream is None:
        return torch.empty(n, dtype=torch.uint8, device=device)
    with torch.cuda.stream(stream):
        return torch.empty(n, dtype=torch.uint8, device=device)


class Coo:
    """A COO tensor preprocessed for MTTKRP on one GPU.

    ``inds`` is an int32/uint32-valued tensor [N, nnz] (or N tensors [nnz])
    of 0-based coordinates and ``vals`` float32 [nnz], both on the GPU. For
    every mode the library keeps a copy of the nonzeros sorted stably by that
    mode's index, in a workspace this object owns.
    """

    def __init__(self, dims: Sequence[int], inds, vals: torch.Tensor, stream=None,
                 workspace: Optional[torch.Tensor] = None):
        self.dims = tuple(int(d) for d in dims)
        self.order = len(self.dims)
        rows = list(inds) if not isinstance(inds, torch.Tensor) else [inds[k] for k in range(inds.shape[0])]
        if len(rows) != self.order:
            raise ValueError(f"need {self.order} index arrays, got {len(rows)}")
        self.inds = [r.contiguous() for r in rows]
        for r in self.inds:
            if r.dtype != torch.int32 or not r.is_cuda:
                raise TypeError("indices must be int32 CUDA tensors (uint32 bit patterns)")
        self.vals = vals.contiguous()
        if self.vals.dtype != torch.float32 or not self.vals.is_cuda:
            raise TypeError("values must be a float32 CUDA tensor")
        self.nnz = int(self.vals.numel())
        if any(int(r.numel()) != self.nnz for r in self.inds):
            raise ValueError("index arrays and values differ in length")
        self.device = self.vals.device
        self._dims_c = (ctypes.c_uint64 * self.order)(*self.dims)
        nbytes = ctypes.c_size_t()
        check(lib.pasta_coo_workspace_bytes(self.order, self._dims_c, self.nnz, ctypes.byref(nbytes)),
              "pasta_coo_workspace_bytes")
        if workspace is not None and workspace.dtype == torch.uint8 and workspace.numel() >= nbytes.value:
            self.workspace = workspace
        else:
            self.workspace = _scratch(nbytes.value, self.device, stream)
        self._ind_ptrs = ptr_array([r.data_ptr() for r in self.inds])
        h = ctypes.c_void_p()
        check(lib.pasta_coo_create(self.order, self._dims_c, self.nnz, self._ind_ptrs, self.vals.data_ptr(),
                                   self.workspace.data_ptr(), self.workspace.numel(), _stream(stream),
                                   ctypes.byref(h)), "pasta_coo_create")
        self._h = h
        self._destroy = lib.pasta_coo_destroy  # still reachable while the interpreter shuts down

    @property
    def handle(self) -> ctypes.c_void_p:
        return self._h

    def check(self, stream=None) -> None:
        """Wait for the stream and raise if a kernel found this tensor's sorted streams
        out of order (pasta_coo_check; the affected outputs are undefined)."""
        check(lib.pasta_coo_check(self._h, _stream(stream)), "pasta_coo_check")

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            self._destroy(h)
            self._h = None

    def _view(self, ptr: int, count: int, dtype) -> torch.Tensor:
        off = ptr - self.workspace.data_ptr()
        esz = torch.tensor([], dtype=dtype).element_size()
        return self.workspace[off: off + count * esz].view(dtype)

    def mode_view(self, mode: int):
        """(perm, rowptr, sorted index arrays [N], sorted values) of one mode, as views."""
        perm, rowptr, vals = ctypes.c_void_p(), ctypes.c_void_p(), ctypes.c_void_p()
        sinds = (ctypes.c_void_p * self.order)()
        check(lib.pasta_coo_mode_view(self._h, int(mode), ctypes.byref(perm), ctypes.byref(rowptr), sinds,
                                      ctypes.byref(vals)), "pasta_coo_mode_view")
        M = self.nnz
        return (self._view(perm.value, M, torch.int32), self._view(rowptr.value, self.dims[mode] + 1, torch.int32),
                [self._view(sinds[k], M, torch.int32) for k in range(self.order)],
                self._view(vals.value, M, torch.float32))


def _factor_args(X: Coo, factors: Sequence[Optional[torch.Tensor]], skip: Optional[int]):
    ref = None
    for k, f in enumerate(factors):
        if f is None:
            if k != skip:
                raise ValueError(f"factor {k} is required")
            continue
        if not f.is_cuda or f.dim() != 2 or f.stride(1) != 1:
            raise ValueError(f"factor {k} must be a 2-D CUDA tensor with unit column stride")
        if f.shape[0] != X.dims[k]:
            raise ValueError(f"factor {k} has {f.shape[0]} rows, mode size is {X.dims[k]}")
        if ref is None:
            ref = f
        elif f.dtype != ref.dtype or f.shape[1] != ref.shape[1] or f.stride(0) != ref.stride(0):
            raise ValueError("all factors need the same dtype, rank and row stride")
    if ref is None:
        raise ValueError("no factor given")
    if ref.dtype not in _DT:
        raise TypeError("factors must be float32 or bfloat16")
    ptrs = ptr_array([0 if f is None else f.data_ptr() for f in factors])
    return ptrs, _DT[ref.dtype], int(ref.shape[1]), int(max(ref.stride(0), ref.shape[1]))


def coo_workspace_bytes(dims: Sequence[int], nnz: int) -> int:
    d = (ctypes.c_uint64 * len(dims))(*[int(x) for x in dims])
    n = ctypes.c_size_t()
    check(lib.pasta_coo_workspace_bytes(len(dims), d, int(nnz), ctypes.byref(n)), "pasta_coo_workspace_bytes")
    return n.value


def mttkrp_workspace_bytes(X: Coo, mode: int, rank: int, dtype=torch.float32) -> int:
    n = ctypes.c_size_t()
    check(lib.pasta_mttkrp_workspace_bytes(X.handle, int(mode), int(rank), _DT[dtype], ctypes.byref(n)),
          "pasta_mttkrp_workspace_bytes")
    return n.value


def mttkrp(X: Coo, factors: Sequence[Optional[torch.Tensor]], mode: int, out: Optional[torch.Tensor] = None,
           vals: Optional[torch.Tensor] = None, alpha: float = 1.0, workspace: Optional[torch.Tensor] = None,
           stream=None) -> torch.Tensor:
    """out = alpha * MTTKRP_mode(X; factors), fp32 [dims[mode], R]; factors[mode] is not read.

    ``vals`` (float32 [nnz], caller order) replaces the tensor's values."""
    facs = list(factors)
    if not (0 <= mode < X.order):
        raise ValueError("mode out of range")
    facs[mode] = None if facs[mode] is None else facs[mode]
    ptrs, dt, R, ldf = _factor_args(X, [None if k == mode else f for k, f in enumerate(facs)], mode)
    if out is None:
        out = torch.empty((X.dims[mode], R), dtype=torch.float32, device=X.device)
    if out.dtype != torch.float32 or out.dim() != 2 or out.shape[0] != X.dims[mode] or out.shape[1] < R \
            or out.stride(1) != 1:
        raise ValueError("out must be float32 [dims[mode], >=R] with unit column stride")
    vptr = None
    if vals is not None:
        if vals.dtype != torch.float32 or vals.numel() != X.nnz or not vals.is_contiguous():
            raise ValueError("vals must be a contiguous float32 tensor of nnz entries")
        vptr = vals.data_ptr()
    if workspace is None:
        workspace = _scratch(mttkrp_workspace_bytes(X, mode, R, facs[(mode + 1) % X.order].dtype), X.device,
                             stream)
    check(lib.pasta_mttkrp(X.handle, int(mode), ptrs, dt, R, ldf, vptr, float(alpha), out.data_ptr(),
                           int(out.stride(0)), workspace.data_ptr(), workspace.numel(), _stream(stream)),
          "pasta_mttkrp")
    return out


def mttkrp_atomic(X: Coo, factors, mode: int, out: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    """The nonzero-parallel atomic-update form of MTTKRP (for comparison)."""
    ptrs, dt, R, ldf = _factor_args(X, [None if k == mode else f for k, f in enumerate(factors)], mode)
    if out is None:
        out = torch.empty((X.dims[mode], R), dtype=torch.float32, device=X.device)
    check(lib.pasta_mttkrp_atomic(X.handle, int(mode), ptrs, dt, R, ldf, out.data_ptr(), int(out.stride(0)),
                                  _stream(stream)), "pasta_mttkrp_atomic")
    return out


def cp_sample(X: Coo, factors, out: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    """mhat[m] = sum_r prod_k U_k[i_k(m), r] at every nonzero, caller order, fp32."""
    ptrs, dt, R, ldf = _factor_args(X, factors, None)
    if out is None:
        out = torch.empty(X.nnz, dtype=torch.float32, device=X.device)
    check(lib.pasta_cp_sample(X.handle, ptrs, dt, R, ldf, out.data_ptr(), _stream(stream)), "pasta_cp_sample")
    return out


def cp_residual_loss(X: Coo, factors, resid: Optional[torch.Tensor] = None, want_resid: bool = True,
                     stream=None):
    """(resid = mhat - x [fp32, caller order] or None, loss = 1/2 sum resid^2 [fp64 scalar tensor])."""
    ptrs, dt, R, ldf = _factor_args(X, factors, None)
    if resid is None and want_resid:
        resid = torch.empty(X.nnz, dtype=torch.float32, device=X.device)
    loss = torch.empty((), dtype=torch.float64, device=X.device)
    n = ctypes.c_size_t()
    check(lib.pasta_cp_workspace_bytes(X.handle, R, dt, ctypes.byref(n)), "pasta_cp_workspace_bytes")
    ws = _scratch(n.value, X.device, stream)
    check(lib.pasta_cp_residual_loss(X.handle, ptrs, dt, R, ldf, None if resid is None else resid.data_ptr(),
                                     loss.data_ptr(), ws.data_ptr(), ws.numel(), _stream(stream)),
          "pasta_cp_residual_loss")
    return resid, loss


def cp_grad_workspace_bytes(X: Coo, rank: int, dtype=torch.float32) -> int:
    n = ctypes.c_size_t()
    check(lib.pasta_cp_grad_workspace_bytes(X.handle, int(rank), _DT[dtype], ctypes.byref(n)),
          "pasta_cp_grad_workspace_bytes")
    return n.value


def cp_grad(X: Coo, factors, grads: Optional[List[torch.Tensor]] = None, alpha: float = 1.0,
            want_loss: bool = True, workspace: Optional[torch.Tensor] = None, stream=None):
    """(loss [fp64 scalar tensor or None], [alpha * dL/dU_n]) for L = 1/2 sum_m (mhat_m - x_m)^2."""
    ptrs, dt, R, ldf = _factor_args(X, factors, None)
    if grads is None:
        grads = [torch.empty((d, R), dtype=torch.float32, device=X.device) for d in X.dims]
    ldg = int(grads[0].stride(0))
    for n, g in enumerate(grads):
        if g.dtype != torch.float32 or g.shape[0] != X.dims[n] or g.shape[1] < R or g.stride(1) != 1 \
                or int(g.stride(0)) != ldg:
            raise ValueError("grads must be float32 [dims[n], >=R] sharing one row stride")
    loss = torch.empty((), dtype=torch.float64, device=X.device) if want_loss else None
    if workspace is None:
        workspace = _scratch(cp_grad_workspace_bytes(X, R, factors[0].dtype), X.device, stream)
    check(lib.pasta_cp_grad(X.handle, ptrs, dt, R, ldf, float(alpha), ptr_array([g.data_ptr() for g in grads]),
                            ldg, None if loss is None else loss.data_ptr(), workspace.data_ptr(), workspace.numel(),
                            _stream(stream)), "pasta_cp_grad")
    return loss, grads


def cast_bf16(src: torch.Tensor, out: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    """fp32 -> bf16 (round to nearest even) with the library's cast kernel."""
    if src.dtype != torch.float32 or not src.is_contiguous():
        raise ValueError("src must be contiguous float32")
    if out is None:
        out = torch.empty(src.shape, dtype=torch.bfloat16, device=src.device)
    check(lib.pasta_cast_f32_to_bf16(src.data_ptr(), out.data_ptr(), src.numel(), _stream(stream)),
          "pasta_cast_f32_to_bf16")
    return out


def cp_als_sweep(X: Coo, factors: List[torch.Tensor], lam: Optional[torch.Tensor] = None, want_fit: bool = True,
                 workspace: Optional[torch.Tensor] = None, stream=None):
    """One CP-ALS sweep over every mode, updating the fp32 ``factors`` in place.

    Returns (lambda [R] fp32, fit fp64 scalar tensor or None, info uint32 tensor:
    1 if some normal-equation matrix was not positive definite)."""
    ptrs, dt, R, ldf = _factor_args(X, factors, None)
    if dt != _lib.PASTA_F32:
        raise TypeError("CP-ALS updates fp32 factors")
    if lam is None:
        lam = torch.empty(R, dtype=torch.float32, device=X.device)
    fit = torch.empty((), dtype=torch.float64, device=X.device) if want_fit else None
    info = torch.empty(1, dtype=torch.int32, device=X.device)
    if workspace is None:
        n = ctypes.c_size_t()
        check(lib.pasta_cp_als_workspace_bytes(X.handle, R, ctypes.byref(n)), "pasta_cp_als_workspace_bytes")
        workspace = _scratch(n.value, X.device, stream)
    check(lib.pasta_cp_als_sweep(X.handle, ptrs, R, ldf, lam.data_ptr(), None if fit is None else fit.data_ptr(),
                                 info.data_ptr(), workspace.data_ptr(), workspace.numel(), _stream(stream)),
          "pasta_cp_als_sweep")
    return lam, fit, info


class Fibers:
    """The mode-``mode`` fibers of a preprocessed tensor (Algs. 4 and 5's
    pre-processing): the nonzeros reordered so that each fiber (every index
    fixed but i_mode) is one run, numbered in lexicographic order of the other
    modes' indices. Owns its workspace; does not keep ``X`` alive."""

    def __init__(self, X: Coo, mode: int, stream=None, workspace: Optional[torch.Tensor] = None):
        if not (0 <= mode < X.order):
            raise ValueError("mode out of range")
        self.mode = int(mode)
        self.order = X.order
        self.dims = X.dims
        self.nnz = X.nnz
        self.device = X.device
        nbytes = ctypes.c_size_t()
        check(lib.pasta_fibers_workspace_bytes(X.handle, self.mode, ctypes.byref(nbytes)),
              "pasta_fibers_workspace_bytes")
        if workspace is not None and workspace.dtype == torch.uint8 and workspace.numel() >= nbytes.value:
            self.workspace = workspace
        else:
            self.workspace = _scratch(nbytes.value, self.device, stream)
        h = ctypes.c_void_p()
        check(lib.pasta_fibers_create(X.handle, self.mode, self.workspace.data_ptr(), self.workspace.numel(),
                                      _stream(stream), ctypes.byref(h)), "pasta_fibers_create")
        self._h = h
        self._destroy = lib.pasta_fibers_destroy
        nf = ctypes.c_uint64()
        check(lib.pasta_fibers_info(h, None, ctypes.byref(nf)), "pasta_fibers_info")
        self.nfibs = int(nf.value)

    @property
    def handle(self) -> ctypes.c_void_p:
        return self._h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            self._destroy(h)
            self._h = None

    def _view(self, ptr: int, count: int, dtype) -> torch.Tensor:
        off = ptr - self.workspace.data_ptr()
        esz = torch.tensor([], dtype=dtype).element_size()
        return self.workspace[off: off + count * esz].view(dtype)

    def view(self):
        """(fptr [nfibs+1], coords [order-1 tensors of nfibs], perm [nnz], fid [nnz]) as int32 views."""
        fptr, perm, fid = ctypes.c_void_p(), ctypes.c_void_p(), ctypes.c_void_p()
        coords = (ctypes.c_void_p * max(1, self.order - 1))()
        check(lib.pasta_fibers_view(self._h, ctypes.byref(fptr), coords, ctypes.byref(perm), ctypes.byref(fid)),
              "pasta_fibers_view")
        nf, M = self.nfibs, self.nnz
        return (self._view(fptr.value, nf + 1, torch.int32),
                [self._view(coords[q], nf, torch.int32) for q in range(self.order - 1)],
                self._view(perm.value, M, torch.int32), self._view(fid.value, M, torch.int32))


def ttm_workspace_bytes(F: Fibers, rank: int, dtype=torch.float32) -> int:
    n = ctypes.c_size_t()
    check(lib.pasta_ttm_workspace_bytes(F.handle, int(rank), _DT[dtype], ctypes.byref(n)), "pasta_ttm_workspace_bytes")
    return n.value


def ttm(F: Fibers, U: torch.Tensor, out: Optional[torch.Tensor] = None, workspace: Optional[torch.Tensor] = None,
        stream=None) -> torch.Tensor:
    """Sparse TTM (Alg. 5): out[f, :] = sum over fiber f's nonzeros of x * U[i_mode, :]; fp32 [nfibs, R].
    U is [dims[mode], R] (fp32 or bf16, unit column stride)."""
    if not U.is_cuda or U.dim() != 2 or U.stride(1) != 1 or U.dtype not in _DT:
        raise ValueError("U must be a 2-D float32/bfloat16 CUDA tensor with unit column stride")
    if U.shape[0] != F.dims[F.mode]:
        raise ValueError(f"U has {U.shape[0]} rows, mode size is {F.dims[F.mode]}")
    R = int(U.shape[1])
    ldu = int(max(U.stride(0), R))
    if out is None:
        out = torch.empty((F.nfibs, R), dtype=torch.float32, device=F.device)
    if out.dtype != torch.float32 or out.dim() != 2 or out.shape[0] != F.nfibs or out.shape[1] < R \
            or out.stride(1) != 1:
        raise ValueError("out must be float32 [nfibs, >= R] with unit column stride")
    ws = workspace if workspace is not None else _scratch(ttm_workspace_bytes(F, R, U.dtype), F.device, stream)
    check(lib.pasta_ttm(F.handle, U.data_ptr(), _DT[U.dtype], R, ldu, out.data_ptr(),
                        int(max(out.stride(0), out.shape[1])), ws.data_ptr(), ws.numel(), _stream(stream)),
          "pasta_ttm")
    return out


def ttv_workspace_bytes(F: Fibers) -> int:
    n = ctypes.c_size_t()
    check(lib.pasta_ttv_workspace_bytes(F.handle, ctypes.byref(n)), "pasta_ttv_workspace_bytes")
    return n.value


def ttv(F: Fibers, v: torch.Tensor, out: Optional[torch.Tensor] = None, workspace: Optional[torch.Tensor] = None,
        stream=None) -> torch.Tensor:
    """Sparse TTV (Alg. 4): out[f] = sum over fiber f's nonzeros of x * v[i_mode]; fp32 [nfibs]."""
    if not v.is_cuda or v.dtype != torch.float32 or v.dim() != 1 or not v.is_contiguous():
        raise ValueError("v must be a contiguous float32 CUDA vector")
    if v.numel() != F.dims[F.mode]:
        raise ValueError(f"v has {v.numel()} entries, mode size is {F.dims[F.mode]}")
    if out is None:
        out = torch.empty(F.nfibs, dtype=torch.float32, device=F.device)
    if out.dtype != torch.float32 or out.numel() != F.nfibs or not out.is_contiguous():
        raise ValueError("out must be a contiguous float32 [nfibs] tensor")
    ws = workspace if workspace is not None else _scratch(ttv_workspace_bytes(F), F.device, stream)
    check(lib.pasta_ttv(F.handle, v.data_ptr(), out.data_ptr(), ws.data_ptr(), ws.numel(), _stream(stream)),
          "pasta_ttv")
    return out


def _values(t: torch.Tensor, name: str) -> torch.Tensor:
    if not t.is_cuda or t.dtype != torch.float32 or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous float32 CUDA tensor")
    return t


def tew_eq(op: str, x: torch.Tensor, y: torch.Tensor, out: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    """Same-pattern element-wise operation (Alg. 1): out = x op y on the value arrays; op in add/sub/mul/div."""
    _values(x, "x")
    _values(y, "y")
    if x.numel() != y.numel():
        raise ValueError("same pattern: x and y need the same length")
    out = torch.empty_like(x) if out is None else _values(out, "out")
    check(lib.pasta_tew_eq(_lib.EWOP[op], x.numel(), x.data_ptr(), y.data_ptr(), out.data_ptr(), _stream(stream)),
          "pasta_tew_eq")
    return out


def ts(op: str, x: torch.Tensor, s: float, out: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    """Tensor-scalar operation on every nonzero (Alg. 3): out = x op s; op in add/sub/mul/div."""
    _values(x, "x")
    out = torch.empty_like(x) if out is None else _values(out, "out")
    check(lib.pasta_ts(_lib.EWOP[op], x.numel(), x.data_ptr(), float(s), out.data_ptr(), _stream(stream)), "pasta_ts")
    return out


def tew_workspace_bytes(order: int, nnz_x: int, nnz_y: int) -> int:
    n = ctypes.c_size_t()
    check(lib.pasta_tew_workspace_bytes(int(order), int(nnz_x), int(nnz_y), ctypes.byref(n)),
          "pasta_tew_workspace_bytes")
    return n.value


def tew(op: str, dims_x: Sequence[int], inds_x: torch.Tensor, vals_x: torch.Tensor, dims_y: Sequence[int],
        inds_y: torch.Tensor, vals_y: torch.Tensor, workspace: Optional[torch.Tensor] = None, stream=None):
    """General element-wise operation of two sparse tensors of the same order (Alg. 2).

    inds_* are int32 CUDA tensors [N, nnz]; returns (dims_z, inds_z [N, nnz_z] int32, vals_z [nnz_z]) with the
    output in lexicographic order; op in add/sub/mul."""
    N = len(dims_x)
    if len(dims_y) != N or inds_x.shape[0] != N or inds_y.shape[0] != N:
        raise ValueError("the two tensors need the same order")
    for t, name in ((inds_x, "inds_x"), (inds_y, "inds_y")):
        if not t.is_cuda or t.dtype != torch.int32:
            raise TypeError(f"{name} must be an int32 CUDA tensor")
    _values(vals_x, "vals_x")
    _values(vals_y, "vals_y")
    nx, ny = int(vals_x.numel()), int(vals_y.numel())
    ix = [inds_x[k].contiguous() for k in range(N)]
    iy = [inds_y[k].contiguous() for k in range(N)]
    cap = max(nx + ny, 1)
    iz = torch.empty((N, cap), dtype=torch.int32, device=vals_x.device)
    vz = torch.empty(cap, dtype=torch.float32, device=vals_x.device)
    ws = workspace if workspace is not None else _scratch(tew_workspace_bytes(N, nx, ny), vals_x.device, stream)
    dx = (ctypes.c_uint64 * N)(*[int(d) for d in dims_x])
    dy = (ctypes.c_uint64 * N)(*[int(d) for d in dims_y])
    dz = (ctypes.c_uint64 * N)()
    nz = ctypes.c_uint64()
    check(lib.pasta_tew(N, _lib.EWOP[op], dx, nx, ptr_array([t.data_ptr() for t in ix]), vals_x.data_ptr(), dy, ny,
                        ptr_array([t.data_ptr() for t in iy]), vals_y.data_ptr(), dz,
                        ptr_array([iz[k].data_ptr() for k in range(N)]), vz.data_ptr(), ctypes.byref(nz),
                        ws.data_ptr(), ws.numel(), _stream(stream)), "pasta_tew")
    n = int(nz.value)
    return tuple(int(d) for d in dz), iz[:, :n], vz[:n]
