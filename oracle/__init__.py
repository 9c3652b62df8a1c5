"""FP64 CPU oracle for COO MTTKRP and the sampled CP model.

TEST INFRASTRUCTURE ONLY. Only the test suite, the smoke check and the
CPU-baseline leg of ``bench.py`` may import this package. The product path
(``paper_1902_03317_amd``) never imports it, and the two share no code:
the oracle is plain C (``mttkrp_oracle.c``, FP64, OpenMP) plus the numpy
definitions in :mod:`oracle.brute`.

What it computes (the plain definitions, Section 4.6 eq. mttkrp-init and
Section 5.2 Alg. 6 of the suite):
  * ``mttkrp``: out[i, r] = sum_{m: i_n(m)=i} x_m prod_{k!=n} U_k[i_k(m), r];
  * ``cp_sample``: mhat_m = sum_r prod_k U_k[i_k(m), r];
  * ``cp_loss``: 1/2 sum_m (mhat_m - x_m)^2 and its residuals;
  * ``cp_grad``: d loss / d U_n = MTTKRP_n with the residuals as values;
  * ``sort_perm`` / ``mode_orders`` / ``rowptr``: stable orders of the
    nonzeros by one mode, the chained per-mode orders, and the row offsets of
    a sorted stream (a library sort as the step);
  * ``bf16_round``: float32 -> bfloat16, round to nearest, ties to even;
  * ``fiber_order`` / ``fibers``: the mode-n fibers (Section 3: every index
    fixed except i_n) that hold nonzeros, and the order that makes each one a
    contiguous run (the pre-processing step of Algs. 4 and 5);
  * ``ttm``: Y = X x_n U (Section 4.4, eq. ttm, U of shape I_n x R), kept
    semi-sparse as one dense R-vector per fiber (Alg. 5);
  * ``ttv``: Y = X x_n v (Section 4.3), one value per fiber (Alg. 4);
  * ``tew_eq`` / ``ts``: element-wise operations of two tensors with the same
    nonzero pattern, and tensor-scalar operations (Section 4.1-4.2, Algs. 1
    and 3);
  * ``tew``: the general element-wise operation of two tensors of the same
    order, by the sorted merge of Alg. 2.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import List, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mttkrp_oracle.c")
_SO = os.path.join(_HERE, "liboracle.so")


def build(force: bool = False) -> str:
    """Compile the C oracle into ``oracle/liboracle.so`` with gcc."""
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        tmp = _SO + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O3", "-std=c11", "-fopenmp", "-fPIC", "-shared", _SRC, "-o", tmp])
        os.replace(tmp, _SO)
    return _SO


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_SO)
        P = ctypes.c_void_p
        sig = [ctypes.c_int, P, ctypes.c_uint64, P, P, P, ctypes.c_int, ctypes.c_int, ctypes.c_int, P]
        for name in ("oracle_mttkrp_seq", "oracle_mttkrp_priv", "oracle_mttkrp_atomic"):
            f = getattr(L, name)
            f.argtypes = sig
            f.restype = ctypes.c_int
        L.oracle_cp_sample.argtypes = [ctypes.c_int, P, ctypes.c_uint64, P, P, ctypes.c_int, ctypes.c_int, P]
        L.oracle_cp_sample.restype = ctypes.c_int
        L.oracle_cp_loss.argtypes = [ctypes.c_int, P, ctypes.c_uint64, P, P, P, ctypes.c_int, ctypes.c_int, P, P]
        L.oracle_cp_loss.restype = ctypes.c_int
        L.oracle_max_threads.restype = ctypes.c_int
        L.oracle_tew_merge.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_uint64, P, P, ctypes.c_uint64, P, P,
                                       ctypes.c_uint64, P, P]
        L.oracle_tew_merge.restype = ctypes.c_int64
        _lib = L
    return _lib


def max_threads() -> int:
    return int(lib().oracle_max_threads())


class _Args:
    """Marshal numpy arrays into the C oracle's argument layout (keeps refs alive)."""

    def __init__(self, dims, inds, factors, rank=None):
        self.N = len(dims)
        self.dims = np.ascontiguousarray(np.asarray(dims, dtype=np.uint64))
        inds = np.asarray(inds)
        if inds.ndim != 2 or inds.shape[0] != self.N:
            raise ValueError("inds must be [N, nnz]")
        self.inds = np.ascontiguousarray(inds, dtype=np.uint32)
        self.M = int(self.inds.shape[1])
        self.keep = []
        ptrs = (ctypes.c_void_p * self.N)()
        R = None
        ldf = None
        for k in range(self.N):
            f = factors[k]
            if f is None:
                ptrs[k] = None
                continue
            f = np.ascontiguousarray(np.asarray(f), dtype=np.float64)
            if f.ndim != 2 or f.shape[0] != dims[k]:
                raise ValueError(f"factor {k} must be [{dims[k]}, R]")
            self.keep.append(f)
            ptrs[k] = f.ctypes.data
            R = f.shape[1] if R is None else R
            ldf = f.shape[1]
            if f.shape[1] != R:
                raise ValueError("all factors must have R columns")
        self.R = int(rank if rank is not None else R)
        self.ldf = int(ldf if ldf is not None else self.R)
        self.ptrs = ptrs


_ERR = {-1: "bad argument", -2: "index out of range", -3: "out of memory"}


def _check(rc):
    if rc != 0:
        raise ValueError(f"oracle: {_ERR.get(rc, rc)}")


def mttkrp(dims: Sequence[int], inds, vals, factors: List, mode: int, strategy: str = "seq") -> np.ndarray:
    """Mode-``mode`` MTTKRP in FP64; ``factors[mode]`` is ignored (may be None).

    strategy: "seq" (Alg. 6 generalised), "priv" (per-thread buffers, Section
    5.3), "atomic" (atomic updates, Section 5.3) or "auto" (privatisation
    while the private buffers fit in 16 GB, else atomics).
    """
    facs = [None if k == mode else factors[k] for k in range(len(dims))]
    if all(f is None for f in facs):  # order 1: no factor, R from the caller is required
        raise ValueError("order-1 MTTKRP needs a rank")
    a = _Args(dims, inds, facs)
    v = np.ascontiguousarray(np.asarray(vals), dtype=np.float64)
    if v.shape != (a.M,):
        raise ValueError("vals must be [nnz]")
    out = np.empty((int(dims[mode]), a.R), dtype=np.float64)
    if strategy == "auto":
        strategy = "priv" if max_threads() * int(dims[mode]) * a.R * 8 <= (16 << 30) else "atomic"
    fn = {"seq": lib().oracle_mttkrp_seq, "priv": lib().oracle_mttkrp_priv,
          "atomic": lib().oracle_mttkrp_atomic}[strategy]
    _check(fn(a.N, a.dims.ctypes.data, a.M, a.inds.ctypes.data, v.ctypes.data, a.ptrs, a.R, a.ldf, int(mode),
              out.ctypes.data))
    return out


def cp_sample(dims, inds, factors) -> np.ndarray:
    """mhat_m = sum_r prod_k U_k[i_k(m), r] in FP64."""
    a = _Args(dims, inds, factors)
    out = np.empty(a.M, dtype=np.float64)
    _check(lib().oracle_cp_sample(a.N, a.dims.ctypes.data, a.M, a.inds.ctypes.data, a.ptrs, a.R, a.ldf,
                                  out.ctypes.data))
    return out


def cp_loss(dims, inds, vals, factors):
    """(loss, resid): resid = mhat - x, loss = 1/2 sum resid^2, FP64."""
    a = _Args(dims, inds, factors)
    v = np.ascontiguousarray(np.asarray(vals), dtype=np.float64)
    resid = np.empty(a.M, dtype=np.float64)
    loss = np.zeros(1, dtype=np.float64)
    _check(lib().oracle_cp_loss(a.N, a.dims.ctypes.data, a.M, a.inds.ctypes.data, v.ctypes.data, a.ptrs, a.R,
                                a.ldf, resid.ctypes.data, loss.ctypes.data))
    return float(loss[0]), resid


def cp_grad(dims, inds, vals, factors, strategy: str = "seq"):
    """(loss, [dL/dU_n]) of the observed-entry least-squares CP loss, FP64."""
    loss, resid = cp_loss(dims, inds, vals, factors)
    grads = [mttkrp(dims, inds, resid, factors, n, strategy) for n in range(len(dims))]
    return loss, grads


def sort_perm(rows) -> np.ndarray:
    """Stable order of the nonzeros by their mode-n index (ties keep caller order)."""
    return np.argsort(np.asarray(rows), kind="stable").astype(np.uint32)


def mode_orders(inds):
    """The order of the nonzeros for every mode: mode n's order is lexicographic in
    (i_n, i_{n-1}, ..., i_0), then i_{N-1} (for n < N-1), then caller position (each
    mode's order is the stable sort by i_n of the previous mode's order, mode N-1's
    coming from the caller's order sorted stably by i_{N-1}). One stable ``np.lexsort``
    per mode on that key (its last key is the primary one; ties keep caller order)."""
    inds = np.asarray(inds)
    N = inds.shape[0]
    out = []
    for n in range(N):
        key = [inds[k] for k in range(n, -1, -1)] + ([inds[N - 1]] if n < N - 1 else [])
        out.append(np.lexsort(key[::-1]).astype(np.uint32))
    return out


def rowptr(sorted_rows, size: int) -> np.ndarray:
    """rowptr[i] = first position of row i in the sorted stream; rowptr[size] = nnz."""
    return np.searchsorted(np.asarray(sorted_rows), np.arange(size + 1), side="left").astype(np.uint32)


def bf16_round(a) -> np.ndarray:
    """float32 -> bfloat16 by round-to-nearest-even on the bit pattern, as float32 values."""
    u = np.ascontiguousarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    lsb = (u >> np.uint64(16)) & np.uint64(1)
    r = ((u + np.uint64(0x7FFF) + lsb) >> np.uint64(16)) << np.uint64(16)
    return r.astype(np.uint32).view(np.float32)


def bf16_bits(a) -> np.ndarray:
    """The uint16 bit patterns of ``bf16_round(a)``."""
    return (bf16_round(a).view(np.uint32) >> np.uint32(16)).astype(np.uint16)


def rel_fro(y, ystar) -> float:
    """||y - y*||_F / ||y*||_F; if ||y*|| = 0 the result is ||y|| (must be exactly 0)."""
    y = np.asarray(y, dtype=np.float64)
    ystar = np.asarray(ystar, dtype=np.float64)
    den = float(np.linalg.norm(ystar))
    num = float(np.linalg.norm(y - ystar))
    return num / den if den > 0 else float(np.linalg.norm(y))


def cp_als_update(dims, inds, vals, factors, n: int, strategy: str = "seq"):
    """One mode of a CP-ALS sweep in FP64 (alternating least squares for CPD, Section
    3.1.1): M = MTTKRP_n, V = Hadamard_{k!=n} U_k^T U_k, U_n = M V^{-1} (a library
    solve), then the columns of U_n scaled to unit 2-norm (zero columns stay zero).
    Returns (U_n, lambda = the column norms, M, the 2-norm condition number of V)."""
    U = [None if f is None else np.asarray(f, dtype=np.float64) for f in factors]
    M = mttkrp(dims, inds, vals, U, n, strategy)
    R = M.shape[1]
    V = np.ones((R, R))
    for k in range(len(dims)):
        if k != n:
            V *= U[k].T @ U[k]
    Un = np.linalg.solve(V, M.T).T
    lam = np.linalg.norm(Un, axis=0)
    return np.where(lam > 0, Un / np.where(lam > 0, lam, 1.0), 0.0), lam, M, float(np.linalg.cond(V))


def cp_fit(dims, inds, vals, factors, lam) -> float:
    """1 - ||X - [[lambda; U]]|| / ||X|| over the full tensor (X zero off the nonzeros),
    with ||[[lambda; U]]||^2 = lambda^T (Hadamard_k U_k^T U_k) lambda and the inner
    product taken at the nonzeros (the model's values there, from cp_sample), so the
    coordinates are taken to be distinct."""
    U = [np.asarray(f, dtype=np.float64) for f in factors]
    lam = np.asarray(lam, dtype=np.float64)
    x = np.asarray(vals, np.float64)
    x2 = float(x @ x)
    G = np.ones((lam.size, lam.size))
    for u in U:
        G *= u.T @ u
    model2 = float(lam @ G @ lam)
    inner = float(x @ cp_sample(dims, inds, [U[0] * lam[None, :]] + U[1:]))
    return 1.0 - np.sqrt(max(0.0, x2 + model2 - 2.0 * inner)) / np.sqrt(x2) if x2 > 0 else 0.0


def cp_als_sweep(dims, inds, vals, factors, strategy: str = "seq"):
    """One CP-ALS sweep in FP64: ``cp_als_update`` for modes 0 .. N-1 in turn, each
    with the factors updated so far. Returns (factors, lambda of the last mode, fit)
    with fit = 1 - ||X - [[lambda; U]]|| / ||X|| computed from the Gram matrices and
    the last MTTKRP (<X, model> = sum_r lambda_r <M[:, r], U_{N-1}[:, r]>); ||X||^2
    is the sum of the squared values, so the coordinates are taken to be distinct."""
    U = [np.array(f, dtype=np.float64) for f in factors]
    N = len(dims)
    lam, M = None, None
    for n in range(N):
        U[n], lam, M, _ = cp_als_update(dims, inds, vals, U, n, strategy)
    x2 = float(np.dot(np.asarray(vals, np.float64), np.asarray(vals, np.float64)))
    G = np.ones((U[0].shape[1],) * 2)
    for k in range(N):
        G *= U[k].T @ U[k]
    model2 = float(lam @ G @ lam)
    inner = float(np.sum(M * U[N - 1] * lam[None, :]))
    fit = 1.0 - np.sqrt(max(0.0, x2 + model2 - 2.0 * inner)) / np.sqrt(x2) if x2 > 0 else 0.0
    return U, lam, fit


def fiber_order(inds, mode: int) -> np.ndarray:
    """Order of the nonzeros in which every mode-``mode`` fiber is one contiguous run:
    lexicographic in the other modes' indices taken in mode order, then i_mode, then
    caller position (``np.lexsort`` is stable; its last key is the primary one)."""
    inds = np.asarray(inds)
    N = inds.shape[0]
    keys = [inds[mode]] + [inds[k] for k in reversed(range(N)) if k != mode]
    return np.lexsort(keys).astype(np.uint32)


def fibers(inds, mode: int):
    """(order, fptr, coords) of the mode-``mode`` fibers that hold nonzeros.

    order: ``fiber_order``; fptr[f]: position in that order of the first nonzero
    of fiber f, fptr[nfibs] = nnz; coords: [N-1, nfibs], the fixed indices of
    each fiber, modes in increasing order with ``mode`` left out."""
    inds = np.asarray(inds)
    N, M = inds.shape
    other = [k for k in range(N) if k != mode]
    o = fiber_order(inds, mode)
    s = inds[:, o]
    if M == 0:
        return o, np.zeros(1, np.uint32), np.zeros((N - 1, 0), np.uint32)
    new = np.ones(M, dtype=bool)
    new[1:] = np.any(s[other][:, 1:] != s[other][:, :-1], axis=0)
    starts = np.flatnonzero(new)
    fptr = np.append(starts, M).astype(np.uint32)
    return o, fptr, s[other][:, starts].astype(np.uint32)


def ttm(dims, inds, vals, U, mode: int):
    """Sparse TTM, Y = X x_n U with U of shape I_n x R (the paper's orientation,
    eq. ttm), FP64. Alg. 5: for every fiber f, Y[f, :] = sum over the nonzeros m
    of the fiber of x_m U[i_n(m), :]. Returns (fptr, coords, Y[nfibs, R])."""
    inds = np.asarray(inds)
    U = np.asarray(U, dtype=np.float64)
    if U.ndim != 2 or U.shape[0] != int(dims[mode]):
        raise ValueError("U must be [dims[mode], R]")
    if inds.size and int(inds[mode].max()) >= int(dims[mode]):
        raise ValueError("index out of range")
    o, fptr, coords = fibers(inds, mode)
    x = np.asarray(vals, dtype=np.float64)[o]
    contrib = x[:, None] * U[inds[mode][o].astype(np.int64)]
    nf = fptr.size - 1
    Y = np.add.reduceat(contrib, fptr[:-1].astype(np.int64), axis=0) if nf else np.zeros((0, U.shape[1]))
    return fptr, coords, Y


def ttv(dims, inds, vals, v, mode: int):
    """Sparse TTV, Y = X x_n v (Section 4.3), FP64. Alg. 4: for every fiber f,
    Y[f] = sum over the nonzeros m of the fiber of x_m v[i_n(m)].
    Returns (fptr, coords, Y[nfibs])."""
    v = np.asarray(v, dtype=np.float64)
    if v.ndim != 1:
        raise ValueError("v must be a vector")
    fptr, coords, Y = ttm(dims, inds, vals, v[:, None], mode)
    return fptr, coords, Y[:, 0]


_EW = {"add": lambda a, b: a + b, "sub": lambda a, b: a - b, "mul": lambda a, b: a * b, "div": lambda a, b: a / b}


def tew_eq(op: str, x, y) -> np.ndarray:
    """Element-wise operation of two tensors with the same nonzero pattern (Alg. 1 and its
    siblings, Section 4.1): z[m] = x[m] op y[m], FP64 (IEEE: x / 0 is +-inf or nan)."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    if x.shape != y.shape:
        raise ValueError("same pattern: the value arrays must match")
    with np.errstate(divide="ignore", invalid="ignore"):
        return _EW[op](x, y)


def ts(op: str, x, s: float) -> np.ndarray:
    """Tensor-scalar operation on every nonzero (Section 4.2, Alg. 3): y[m] = x[m] op s, FP64."""
    x = np.asarray(x, dtype=np.float64)
    with np.errstate(divide="ignore", invalid="ignore"):
        return _EW[op](x, np.float64(s))


def lex_order(inds) -> np.ndarray:
    """Stable lexicographic order of the nonzeros, mode 0 most significant (Section 5.2)."""
    inds = np.asarray(inds)
    return np.lexsort([inds[k] for k in reversed(range(inds.shape[0]))]).astype(np.uint32)


def tew(op: str, dims_x, inds_x, vals_x, dims_y, inds_y, vals_y):
    """General element-wise operation of two sparse tensors of the same order (Alg. 2):
    the output shape is the element-wise maximum of the two shapes; both inputs are
    sorted lexicographically and merged, every coordinate held by either input
    appearing once in lexicographic order. add: x + y (or the one present); sub:
    x - y (or x, or -y); mul: x * y where both hold the coordinate. Repeated
    coordinates within one input count as their sum. FP64.
    Returns (dims_z, inds_z [N, nnz_z] uint32, vals_z [nnz_z])."""
    code = {"add": 0, "sub": 1, "mul": 2}[op]
    inds_x = np.asarray(inds_x, dtype=np.uint32)
    inds_y = np.asarray(inds_y, dtype=np.uint32)
    N = inds_x.shape[0]
    if inds_y.shape[0] != N or len(dims_x) != N or len(dims_y) != N:
        raise ValueError("the two tensors need the same order")
    dims_z = tuple(max(int(a), int(b)) for a, b in zip(dims_x, dims_y))
    ox, oy = lex_order(inds_x), lex_order(inds_y)
    sx = np.ascontiguousarray(inds_x[:, ox])
    sy = np.ascontiguousarray(inds_y[:, oy])
    vx = np.ascontiguousarray(np.asarray(vals_x, np.float64)[ox])
    vy = np.ascontiguousarray(np.asarray(vals_y, np.float64)[oy])
    Mx, My = sx.shape[1], sy.shape[1]
    cap = Mx + My
    iz = np.empty((N, max(cap, 1)), dtype=np.uint32)
    vz = np.empty(max(cap, 1), dtype=np.float64)
    nz = lib().oracle_tew_merge(N, code, Mx, sx.ctypes.data, vx.ctypes.data, My, sy.ctypes.data, vy.ctypes.data,
                                max(cap, 1), iz.ctypes.data, vz.ctypes.data)
    if nz < 0:
        raise ValueError("oracle: bad argument")
    return dims_z, np.ascontiguousarray(iz[:, :nz]), vz[:nz].copy()
