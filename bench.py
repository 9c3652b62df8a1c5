#!/usr/bin/env python3
"""Benchmark of the MI355X COO MTTKRP path on one GPU.

The headline workload is the largest tensor that the measurements name: the
order-5 hypersparse 1M x 1M x 100K x 1K x 100 tensor with 200M nonzeros
(Zipf(1.1) indices on every mode, lognormal values), rank R = 64. One timed
step is one pass of the whole hot path over it:
  1. preprocessing (index check, stable sort per mode, row offsets);
  2. MTTKRP of every mode with fp32 factors, then with bf16 factors;
  3. one CP gradient step with fp32 factors (loss + residual-weighted MTTKRP
     of every factor + Adam), and the same step with bf16 factor copies of
     fp32 masters (Adam writes the bf16 copies in the same pass).
`value` is the fp32 MTTKRP throughput of step 2: nonzeros x modes / time, in
Gnnz/s (the suite sums its MTTKRP times over all modes). Inputs are resident
in GPU memory before timing starts. --config 2 or 3 puts the timed step on
the 50M-nonzero order-3 or the 100M-nonzero order-4 tensor instead.

Roofline. The MTTKRP main kernel is priced against the 8 TB/s HBM peak with
the compulsory bytes of a launch (every byte it must touch once: the
index/value stream, each other factor once, the output once), so `frac` is a
true fraction of a bound. The no-reuse byte counts (Table 2's MTTKRP memory
access, and the same with the output row written once per row) charge every
factor-row gather to HBM although most are served by the caches; they are
kept under `model_fractions` as request volumes, not HBM bounds. The kernel's
factor-row gathers are also compared with a measured ceiling of the vector
memory pipeline (`gather_pipeline`): a probe kernel making the same 16-byte
per lane row gathers from a cache-resident table. The kernel's duration comes
from HIP events recorded on its own stream around its launch. `traffic` is
its fabric bytes per launch as rocprofv3 measured them (FETCH_SIZE and
WRITE_SIZE, each scaled by what it reads for a plain device copy), read from
profiles/ while the kernel sources are the ones it was measured on.

Outside the timed steps the line also carries (unless --no-extra): the
50M-nonzero order-3 tensor (MTTKRP fp32 / bf16, CP step, CP-ALS sweep, fibers,
TTM, TTV, element-wise and tensor-scalar operations, general TEW, and its
whole-tensor errors against the FP64 oracle), the order-4 tensor (MTTKRP and
CP step), and the CP fit: 50 Adam steps of the fused CP gradient on the
planted-value 50M-nonzero tensor. Unless --no-cpu-baseline, the FP64 oracle is
timed on the host cores on a bounded sample of the headline tensor, and the
GPU results on that sample are compared with it.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline] [--no-extra]
"""
from __future__ import annotations

import argparse
import ctypes
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "MTTKRP Gnnz/s + % HBM peak; CP grad step ms, BF16 vs FP32 at stated error"
HBM_PEAK_GBPS = 8000.0
KERNEL_SOURCES = [os.path.join(ROOT, "paper_1902_03317_amd", "csrc", f)
                  for f in ("kernels_order.hip", "common.h")]
KERNEL_NAMES = {1: "mttkrp_seg_kernel", 2: "mttkrp_wave_kernel"}  # by the form the library reports
SHORT = {"zipf1.1-50Kx40Kx30K": "zipf50M", "zipf1.2-100Kx10Kx1Kx200": "zipf4d100M",
         "zipf1.1-1Mx1Mx100Kx1Kx100": "zipf5d200M"}


def traffic_file(kernel: str, workload: str, rank: int, dtype: str) -> str:
    """The committed FETCH_SIZE / WRITE_SIZE summary of a main MTTKRP kernel on a workload."""
    return os.path.join(ROOT, "profiles", f"{kernel.replace('_kernel', '')}_{SHORT.get(workload, workload)}"
                                          f"_r{rank}_{dtype}_traffic.json")


# --------------------------------------------------------------------------------------
# bytes models (Table 2 of the suite, generalised to order N and factor element size s_f)
# --------------------------------------------------------------------------------------
def bytes_paper(N: int, R: int, sf: int) -> int:
    """Table 2's MTTKRP memory access per nonzero: N indices, one value, N-1 gathered
    factor rows and one output-row update (16 + 12R at N = 3, fp32)."""
    return 4 * N + 4 + (N - 1) * R * sf + 4 * R


def bytes_alg_per_nnz(N: int, R: int, sf: int) -> int:
    """Bytes per nonzero with no factor-row reuse: the index and value stream plus
    N-1 gathered rows (the output row is written once per row)."""
    return 4 * N + 4 + (N - 1) * R * sf


def bytes_alg(N: int, R: int, sf: int, nnz: int, I_n: int) -> int:
    return nnz * bytes_alg_per_nnz(N, R, sf) + 4 * R * I_n


def bytes_ttm(R: int, sf: int, nnz: int, nfibs: int) -> int:
    """Sparse TTM over the fiber-ordered stream: fiber id, i_n and value per nonzero,
    one gathered R-row of U per nonzero (no reuse), one R-row written per fiber."""
    return nnz * (12 + R * sf) + 4 * R * nfibs


def bytes_ttv(nnz: int, nfibs: int) -> int:
    """Sparse TTV: fiber id, i_n, value and the gathered v entry per nonzero, one value per fiber."""
    return nnz * 16 + 4 * nfibs


def bytes_compulsory(dims, R: int, sf: int, nnz: int, n: int) -> int:
    """Every byte a mode-n launch must touch once: the stream, every other factor
    once, the output once (a lower bound on its HBM traffic with cold caches)."""
    N = len(dims)
    return nnz * (4 * N + 4) + sf * R * sum(d for k, d in enumerate(dims) if k != n) + 4 * R * dims[n]


def lanes_per_row(R: int, sf: int) -> int:
    """Lanes of a group in the contiguous kernel shapes: one 16-byte slice each, a power of two."""
    need = max(1, -(-R * sf // 16))
    L = 1
    while L < need:
        L *= 2
    return L


def kernel_hash() -> str:
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        h.update(open(p, "rb").read())
    return h.hexdigest()[:16]


def host_cpu() -> dict:
    """The host's CPU model (as lscpu names it) and the cores this process may use."""
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        nproc = len(os.sched_getaffinity(0))
    except AttributeError:
        nproc = os.cpu_count()
    return {"cpu_model": model, "nproc": nproc}


# --------------------------------------------------------------------------------------
# HIP events on the launch stream (the runtime torch already loaded)
# --------------------------------------------------------------------------------------
class Hip:
    def __init__(self):
        path = None
        for line in open("/proc/self/maps"):
            if "libamdhip64" in line:
                path = line.split()[-1]
                break
        self.lib = ctypes.CDLL(path or "libamdhip64.so")
        self.lib.hipEventCreate.argtypes = [ctypes.POINTER(ctypes.c_void_p)]
        self.lib.hipEventRecord.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
        self.lib.hipEventSynchronize.argtypes = [ctypes.c_void_p]
        self.lib.hipEventElapsedTime.argtypes = [ctypes.POINTER(ctypes.c_float), ctypes.c_void_p, ctypes.c_void_p]
        self.lib.hipEventDestroy.argtypes = [ctypes.c_void_p]

    def event(self):
        e = ctypes.c_void_p()
        assert self.lib.hipEventCreate(ctypes.byref(e)) == 0
        return e

    def record(self, e, stream):
        assert self.lib.hipEventRecord(e, stream) == 0

    def ms(self, a, b) -> float:
        assert self.lib.hipEventSynchronize(b) == 0
        t = ctypes.c_float()
        assert self.lib.hipEventElapsedTime(ctypes.byref(t), a, b) == 0
        return float(t.value)


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def median(xs):
    s = sorted(xs)
    return s[len(s) // 2]


class Ctx:
    """Device, stream, event helper and the library handles shared by the measurements."""

    def __init__(self, args):
        import torch
        from paper_1902_03317_amd import api
        from paper_1902_03317_amd._lib import lib
        self.torch, self.api, self.plib, self.args = torch, api, lib, args
        self.dev = torch.device("cuda:0")
        self.hip = Hip()
        self.stream = torch.cuda.current_stream().cuda_stream
        self.s_ptr = ctypes.c_void_p(self.stream)

    def timed(self, fn, reps: int, kernel: bool = False):
        """Median call time (and the armed main kernel's time) of ``fn`` over ``reps`` runs, after one warm-up."""
        fn()
        calls, kerns = [], []
        for _ in range(reps):
            c0, c1 = self.hip.event(), self.hip.event()
            if kernel:
                k0, k1 = self.hip.event(), self.hip.event()
                self.plib.pasta_arm_kernel_events(k0, k1)
            self.hip.record(c0, self.s_ptr)
            fn()
            self.hip.record(c1, self.s_ptr)
            calls.append(self.hip.ms(c0, c1))
            if kernel:
                kerns.append(self.hip.ms(k0, k1))
        return (median(calls), median(kerns)) if kernel else median(calls)

    def last_form(self) -> int:
        f = ctypes.c_int(0)
        self.plib.pasta_last_mttkrp_form(ctypes.byref(f))
        return f.value


class Workload:
    """One generated tensor on the GPU, preprocessed, with fp32 and bf16 factor copies."""

    def __init__(self, ctx: Ctx, cfg: int):
        import numpy as np
        from paper_1902_03317_amd import synth
        torch, api = ctx.torch, ctx.api
        self.ctx, self.cfg = ctx, cfg
        self.spec = spec = synth.CONFIGS[cfg]
        self.N, self.R = spec.order, spec.rank
        t0 = time.perf_counter()
        self.coo = coo = synth.load_or_make_coo(spec, ctx.args.cache)
        self.U = synth.make_factors(spec)
        log(f"generated {spec.name}: {coo.nnz} nonzeros in {time.perf_counter() - t0:.1f} s")
        dev = ctx.dev
        self.inds_d = torch.from_numpy(coo.inds.view(np.int32)).to(dev)
        self.vals_d = torch.from_numpy(coo.vals).to(dev)
        self.U32 = [torch.from_numpy(u).to(dev) for u in self.U]
        self.U16 = [api.cast_bf16(u) for u in self.U32]
        self.outs = [torch.empty((d, self.R), dtype=torch.float32, device=dev) for d in coo.dims]
        self.ws_coo = torch.empty(api.coo_workspace_bytes(coo.dims, coo.nnz), dtype=torch.uint8, device=dev)
        self.X = api.Coo(coo.dims, self.inds_d, self.vals_d, workspace=self.ws_coo)
        self.ws_m = torch.empty(max(api.mttkrp_workspace_bytes(self.X, n, self.R, dt) for n in range(self.N)
                                    for dt in (torch.float32, torch.bfloat16)), dtype=torch.uint8, device=dev)
        torch.cuda.synchronize()

    def factors(self, dtype: str):
        return self.U32 if dtype == "f32" else self.U16

    def mttkrp(self, n: int, dtype: str):
        self.ctx.api.mttkrp(self.X, self.factors(dtype), n, out=self.outs[n], workspace=self.ws_m)

    def mttkrp_modes(self, dtype: str, reps: int = 5):
        """Median call and main-kernel ms per mode, and the kernel each mode ran."""
        calls, kerns, forms = [], [], []
        for n in range(self.N):
            c, k = self.ctx.timed(lambda: self.mttkrp(n, dtype), reps, kernel=True)
            calls.append(c)
            kerns.append(k)
            forms.append(self.ctx.last_form())
        return calls, kerns, forms

    def fractions(self, dtype: str, kern_ms) -> dict:
        """The main kernel's rate under each bytes model, as fractions of the HBM peak."""
        N, R, M, dims = self.N, self.R, self.coo.nnz, self.coo.dims
        sf = 2 if dtype == "bf16" else 4
        t = sum(kern_ms) * 1e-3
        qmin = sum(bytes_compulsory(dims, R, sf, M, n) for n in range(N))
        alg = sum(bytes_alg(N, R, sf, M, dims[n]) for n in range(N))
        paper = N * M * bytes_paper(N, R, sf)
        return {"q_min": round(qmin / t / 1e9 / HBM_PEAK_GBPS, 4),
                "b_alg_no_reuse": round(alg / t / 1e9 / HBM_PEAK_GBPS, 4),
                "b_paper_no_reuse": round(paper / t / 1e9 / HBM_PEAK_GBPS, 4)}

    def gather_rate(self, dtype: str, kern_ms) -> float:
        """Bytes of factor rows the main kernel delivers to lanes per second (every
        gathered row counted, R * s_f bytes rounded up to whole 16-byte lane slices)."""
        sf = 2 if dtype == "bf16" else 4
        per_row = lanes_per_row(self.R, sf) * 16
        return self.N * self.coo.nnz * (self.N - 1) * per_row / (sum(kern_ms) * 1e-3)

    def cp_state(self, spec=None):
        """Fit state for CP gradient steps on this tensor's coordinates: fp32 masters
        (one copy per dtype) drawn from the init stream of ``spec`` (default: this
        tensor's), Adam moments, bf16 shadows, gradients, workspaces."""
        from paper_1902_03317_amd import synth
        torch, api = self.ctx.torch, self.ctx.api
        sc = synth.cp_planted_scale(self.R, self.N)
        init = synth.make_init(spec or self.spec, rank=self.R, scale=sc)
        st = {}
        for dt in ("f32", "bf16"):
            m = [torch.from_numpy(u).to(self.ctx.dev) for u in init]
            st[dt] = {"m": m, "sh": [api.cast_bf16(t) for t in m] if dt == "bf16" else None,
                      "mom": [(torch.zeros_like(t), torch.zeros_like(t)) for t in m],
                      "g": [torch.empty_like(t) for t in m],
                      "ws": torch.empty(api.cp_grad_workspace_bytes(
                          self.X, self.R, torch.bfloat16 if dt == "bf16" else torch.float32),
                          dtype=torch.uint8, device=self.ctx.dev), "step": 0}
        return st

    def cp_step(self, st, dt: str, X=None):
        from paper_1902_03317_amd.autograd import adam_step
        s = st[dt]
        s["step"] += 1
        fac = s["sh"] if dt == "bf16" else s["m"]
        loss, _ = self.ctx.api.cp_grad(X or self.X, fac, grads=s["g"], workspace=s["ws"])
        adam_step(s["m"], s["g"], [a for a, _ in s["mom"]], [b for _, b in s["mom"]], s["step"], shadows=s["sh"])
        return loss


def gather_ceiling(ctx: Ctx, L: int) -> dict:
    """Measured rate of 16-byte-per-lane row gathers (lanes per row = L): every
    group of an instruction on its own row (share 1) or the wave on one row, from
    a 2 MiB table (L2-resident) and a 16 KiB one (L1-resident), in bytes delivered
    to lanes per second and in load instructions per ns (one instruction moves
    64 x 16 bytes)."""
    torch = ctx.torch
    steps, blocks = 256, 8192
    out = torch.empty(blocks * 256 * 4, dtype=torch.int32, device=ctx.dev)
    res = {"lanes": L}
    for name, nbytes in (("l2", 2 << 20), ("l1", 16 << 10)):
        rows = nbytes // (L * 16)
        table = torch.randint(0, 1 << 30, (nbytes // 4,), dtype=torch.int32, device=ctx.dev)
        for share_name, share in (("distinct", 1), ("wave_shared", 64 // L)):
            def run():
                st = ctx.plib.pasta_probe_gather(table.data_ptr(), rows, L, share, 64 // L, steps, blocks,
                                                 out.data_ptr(), ctx.s_ptr)
                assert st == 0, st
            t = ctx.timed(run, 5)
            res[f"{name}_{share_name}_gbps"] = round(blocks * 256 * steps * 16 / (t * 1e-3) / 1e9, 1)
            res[f"{name}_{share_name}_instr_per_ns"] = round(blocks * 4 * steps / (t * 1e6), 2)
    return res


def copy_rate(ctx: Ctx) -> float:
    """Achievable streaming bandwidth: a plain 1 GiB device-to-device copy (GB/s, read + write)."""
    torch = ctx.torch
    a = torch.empty(1 << 28, dtype=torch.float32, device=ctx.dev)
    b = torch.empty_like(a)
    t = ctx.timed(lambda: b.copy_(a), 5)
    return 2 * a.numel() * 4 / (t * 1e-3) / 1e9


def measured_counters(w: Workload, kernel, dtype: str) -> dict:
    """rocprofv3 counters of the main kernel committed for these sources: fabric bytes per
    launch and vector memory read instructions per launch (empty if none match)."""
    if not isinstance(kernel, str):
        return {}
    p = traffic_file(kernel, w.spec.name, w.R, dtype)
    if not os.path.exists(p):
        return {}
    tr = json.load(open(p))
    if tr.get("kernel_hash") == kernel_hash() and tr.get("workload") == w.spec.name and \
            kernel in tr.get("kernel", "") and tr.get("factor_dtype") == dtype:
        return tr
    return {}


def kernel_label(forms):
    return KERNEL_NAMES.get(forms[0], "?") if len(set(forms)) == 1 else [KERNEL_NAMES.get(f, "?") for f in forms]


def cpu_baseline(coo, U, budget_s: float = 15.0):
    """The FP64 oracle (privatised OpenMP MTTKRP where the private buffers fit, else
    atomics; all modes) timed on the host cores: passes over a prefix of the
    nonzeros (a uniform sample: caller order is random) sized to about
    ``budget_s`` seconds, the whole tensor if one pass fits in it."""
    import numpy as np
    import oracle
    Uo = [u.astype(np.float64) for u in U]
    threads = oracle.max_threads()

    def run(m):
        inds = np.ascontiguousarray(coo.inds[:, :m])
        vals = coo.vals[:m].astype(np.float64)
        t0 = time.perf_counter()
        outs = [oracle.mttkrp(coo.dims, inds, vals, Uo, n, "auto") for n in range(coo.order)]
        return time.perf_counter() - t0, outs, inds, vals

    m = min(coo.nnz, 2_000_000)
    t, _, _, _ = run(m)  # also the first touch of the buffers and thread start-up
    t2, _, _, _ = run(2 * m) if 2 * m <= coo.nnz else (t * 2, None, None, None)
    # per-nonzero cost from the difference (the fixed cost per pass is the private buffers)
    per_nnz = max((t2 - t) / m, 1e-12)
    fixed = max(t - per_nnz * m, 0.0)
    m = coo.nnz if fixed + per_nnz * coo.nnz <= budget_s else max(m, int((budget_s - fixed) / per_nnz))
    reps, total = 0, 0.0
    while reps == 0 or total < budget_s:
        t, outs, inds, vals = run(m)
        total += t
        reps += 1
    what = "the whole tensor" if m == coo.nnz else f"the first {m} of {coo.nnz} nonzeros (a uniform sample)"
    return {"value": round(reps * coo.order * m / total / 1e9, 5), "unit": "Gnnz/s", "cores": threads,
            "kind": "oracle",
            "sample": f"{what}, all {coo.order} modes, {reps} passes, FP64 OpenMP MTTKRP "
                      f"(privatised where the per-thread buffers fit in 16 GB, else atomics), {total:.1f} s",
            **host_cpu()}, (m, inds, vals, outs)


def oracle_errors(ctx: Ctx, w: Workload, m, inds_s, vals_s, outs_o, with_cp: bool = True) -> dict:
    """Errors of the GPU MTTKRP (fp32 and bf16 factors) and CP gradient on the first m
    nonzeros against the FP64 oracle on the fp32 factors (bf16: end to end)."""
    import numpy as np
    import oracle
    from paper_1902_03317_amd import synth
    torch, api = ctx.torch, ctx.api
    N = w.N
    Xs = w.X if m == w.coo.nnz else api.Coo(w.coo.dims, torch.from_numpy(inds_s.view(np.int32)).to(ctx.dev),
                                            torch.from_numpy(vals_s.astype(np.float32)).to(ctx.dev))
    res = {"sample_nnz": int(m)}
    for dt in ("f32", "bf16"):
        res[f"mttkrp_{dt}_max_mode_rel_fro"] = max(
            oracle.rel_fro(api.mttkrp(Xs, w.factors(dt), n).cpu().numpy(), outs_o[n]) for n in range(N))
    if with_cp:
        init = synth.make_init(w.spec, rank=w.R, scale=synth.cp_planted_scale(w.R, N))
        I32 = [torch.from_numpy(u).to(ctx.dev) for u in init]
        _, go = oracle.cp_grad(w.coo.dims, inds_s, vals_s, [u.astype(np.float64) for u in init], "auto")
        for dt, fac in (("f32", I32), ("bf16", [api.cast_bf16(u) for u in I32])):
            _, gg = api.cp_grad(Xs, fac)
            res[f"cp_grad_{dt}_max_mode_rel_fro"] = max(
                oracle.rel_fro(gg[n].cpu().numpy(), go[n]) for n in range(N))
    return res


def side_row(ctx: Ctx, w: Workload, with_cp: bool = True) -> dict:
    """MTTKRP (fp32 and bf16, every mode) and CP step timings of one tensor, outside the timed steps."""
    row = {"workload": w.spec.name, "dims": list(w.coo.dims), "nnz": w.coo.nnz, "rank": w.R}
    for dt in ("f32", "bf16"):
        calls, kerns, forms = w.mttkrp_modes(dt)
        row[f"mttkrp_{dt}"] = {"gnnz_s": round(w.N * w.coo.nnz / (sum(calls) * 1e-3) / 1e9, 3),
                               "ms_per_mode": [round(c, 4) for c in calls],
                               "kernel_ms": [round(k, 4) for k in kerns], "kernel": kernel_label(forms),
                               "hbm_frac": w.fractions(dt, kerns),
                               "gather_gbps": round(w.gather_rate(dt, kerns) / 1e9, 1)}
    if with_cp:
        st = w.cp_state()
        cp = {dt: ctx.timed(lambda: w.cp_step(st, dt), 5) for dt in ("f32", "bf16")}
        row["cp_step_ms"] = {"f32": round(cp["f32"], 4), "bf16": round(cp["bf16"], 4),
                             "bf16_speedup": round(cp["f32"] / cp["bf16"], 3)}
    return row


def order3_extras(ctx: Ctx, w: Workload) -> dict:
    """CP-ALS sweep, fibers, TTM, TTV, TEW-eq, TS and general TEW on the order-3 tensor."""
    torch, api, plib = ctx.torch, ctx.api, ctx.plib
    X, N, R, M, dev = w.X, w.N, w.R, w.coo.nnz, ctx.dev
    out = {}
    Ua = [u.clone() for u in w.U32]
    lam = torch.empty(R, dtype=torch.float32, device=dev)
    nb = ctypes.c_size_t()
    plib.pasta_cp_als_workspace_bytes(X.handle, R, ctypes.byref(nb))
    ws_a = torch.empty(nb.value, dtype=torch.uint8, device=dev)
    api.cp_als_sweep(X, Ua, lam=lam, workspace=ws_a)
    out["cp_als_sweep_ms"] = round(ctx.timed(lambda: api.cp_als_sweep(X, Ua, lam=lam, workspace=ws_a), 5), 4)
    del Ua, ws_a
    fib = {"ttm": ([], []), "ttv": ([], [])}
    pre_f, nfibs = [], []
    for n in range(N):
        e0, e1 = ctx.hip.event(), ctx.hip.event()
        ctx.hip.record(e0, ctx.s_ptr)
        F = api.Fibers(X, n)
        ctx.hip.record(e1, ctx.s_ptr)
        pre_f.append(ctx.hip.ms(e0, e1))
        nfibs.append(F.nfibs)
        y = torch.empty((F.nfibs, R), dtype=torch.float32, device=dev)
        yv = torch.empty(F.nfibs, dtype=torch.float32, device=dev)
        ws_t = torch.empty(max(api.ttm_workspace_bytes(F, R), api.ttv_workspace_bytes(F)), dtype=torch.uint8,
                           device=dev)
        v = w.U32[n][:, 0].contiguous()
        Un = w.U32[n]
        for name, fn in (("ttm", lambda: api.ttm(F, Un, out=y, workspace=ws_t)),
                         ("ttv", lambda: api.ttv(F, v, out=yv, workspace=ws_t))):
            c, k = ctx.timed(fn, 10, kernel=True)
            fib[name][0].append(c)
            fib[name][1].append(k)
        del F, y, yv, ws_t
    for name in ("ttm", "ttv"):
        calls, kerns = fib[name]
        algb = [bytes_ttm(R, 4, M, nf) if name == "ttm" else bytes_ttv(M, nf) for nf in nfibs]
        out[name] = {"gnnz_s": round(N * M / (sum(calls) * 1e-3) / 1e9, 3),
                     "ms_per_mode": [round(c, 4) for c in calls], "kernel_ms": [round(k, 4) for k in kerns],
                     "no_reuse_frac": round(sum(algb) / (sum(kerns) * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4),
                     "bytes_no_reuse_per_mode": algb, "nfibs": nfibs}
    out["ttm"]["rank"] = R
    out["fibers_preprocess_ms"] = [round(t, 3) for t in pre_f]
    vals_d, inds_d = w.vals_d, w.inds_d
    y2 = (vals_d * 0.5 + 1.0).contiguous()
    zt = torch.empty_like(vals_d)
    t_eq = ctx.timed(lambda: api.tew_eq("add", vals_d, y2, out=zt), 10)
    t_ts = ctx.timed(lambda: api.ts("mul", vals_d, 0.5, out=zt), 10)
    ws_tew = torch.empty(api.tew_workspace_bytes(N, M, M), dtype=torch.uint8, device=dev)
    res = {}

    def general():
        res["z"] = api.tew("add", w.coo.dims, inds_d, vals_d, w.coo.dims, inds_d, vals_d, workspace=ws_tew)
    t_tew = ctx.timed(general, 3)
    for name, t, nbytes in (("tew_eq", t_eq, 12 * M), ("ts", t_ts, 8 * M)):
        out[name] = {"op": "add" if name == "tew_eq" else "mul", "ms": round(t, 4),
                     "gb_s": round(nbytes / (t * 1e-3) / 1e9, 1),
                     "hbm_frac": round(nbytes / (t * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4), "bytes": nbytes}
    out["tew"] = {"op": "add", "inputs": "the tensor with itself", "ms": round(t_tew, 3),
                  "gnnz_s": round(2 * M / (t_tew * 1e-3) / 1e9, 3), "nnz_out": int(res["z"][2].numel())}
    return out


def cp_fit(ctx: Ctx, w: Workload, steps: int) -> dict:
    """The CP fit on the planted tensor: the coordinates of the 50M-nonzero order-3
    tensor with planted rank-R values plus 1% Gaussian noise, fit from an
    independent start by `steps` Adam steps of the fused gradient (fp32 factors,
    and bf16 copies of fp32 masters). Fit = 1 - ||x - mhat|| / ||x|| over the nonzeros."""
    import numpy as np
    from paper_1902_03317_amd import synth
    torch, api = ctx.torch, ctx.api
    cspec = synth.CONFIGS[4]
    R, N = cspec.rank, cspec.order
    sc = synth.cp_planted_scale(R, N)
    A = [torch.from_numpy(a).to(ctx.dev) for a in synth.make_factors(cspec, rank=R, scale=sc)]
    x = api.cp_sample(w.X, A)
    rms = torch.sqrt(torch.mean(x.double() ** 2)).item()
    noise = torch.from_numpy(synth.make_noise(cspec, w.coo.nnz).astype(np.float32)).to(ctx.dev)
    xv = (x + np.float32(0.01 * rms) * noise).contiguous()
    del noise, x, A
    X4 = api.Coo(w.coo.dims, w.inds_d, xv)
    xnorm = torch.linalg.vector_norm(xv.double()).item()
    st = w.cp_state(cspec)
    out = {"workload": cspec.name, "steps": steps, "rank": R, "lr": 1e-2}
    for dt in ("f32", "bf16"):
        losses = []
        e0, e1 = ctx.hip.event(), ctx.hip.event()
        ctx.hip.record(e0, ctx.s_ptr)
        for _ in range(steps):
            losses.append(w.cp_step(st, dt, X=X4))
        ctx.hip.record(e1, ctx.s_ptr)
        ms = ctx.hip.ms(e0, e1) / steps
        first, last = losses[0].item(), losses[-1].item()
        out[dt] = {"ms_per_step": round(ms, 4), "loss_first": first, "loss_last": last,
                   "fit_first": round(1 - (2 * first) ** 0.5 / xnorm, 5),
                   "fit_last": round(1 - (2 * last) ** 0.5 / xnorm, 5)}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra", action="store_true", help="skip the order-3 / order-4 rows and the CP fit")
    ap.add_argument("--config", type=int, default=5, choices=[2, 3, 5],
                    help="timed workload: 5 (order 5, 200M nnz, the default), 3 (order 4) or 2 (order 3)")
    ap.add_argument("--mttkrp-only", action="store_true",
                    help="time only the all-mode MTTKRP of --factor-dtype (profiling runs)")
    ap.add_argument("--factor-dtype", choices=["f32", "bf16"], default="f32",
                    help="factor storage of a --mttkrp-only step (arithmetic is fp32 either way)")
    ap.add_argument("--cache", default=os.environ.get("PASTA_BENCH_CACHE", ""),
                    help="directory for cached generated tensors (reused between runs)")
    ap.add_argument("--mttkrp-form", choices=["auto", "run", "wave"], default="auto",
                    help="MTTKRP kernel form (auto: wave-run form for long rows)")
    ap.add_argument("--fit-steps", type=int, default=50)
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MiB",
                    help="run one plain device copy of this size (counter calibration) and exit")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}, WORLD_SIZE {world}); "
              "this build has no multi-GPU path.", file=sys.stderr)
        sys.exit(2)

    import torch

    so = os.path.join(ROOT, "paper_1902_03317_amd", "libpasta.so")
    if not os.path.exists(so):
        import __graft_entry__
        __graft_entry__.build()

    torch.cuda.set_device(0)
    if args.copy_calibration:
        n = args.copy_calibration << 20
        a = torch.ones(n // 4, dtype=torch.float32, device="cuda:0")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": n, "copy_bytes_written": n}))
        return

    ctx = Ctx(args)
    ctx.plib.pasta_set_mttkrp_form({"auto": 0, "run": 1, "wave": 2}[args.mttkrp_form])
    w = Workload(ctx, args.config)
    N, R, M = w.N, w.R, w.coo.nnz
    do_cp = not args.mttkrp_only
    dtypes = ("f32", "bf16") if do_cp else (args.factor_dtype,)
    st = w.cp_state() if do_cp else None
    hip, s_ptr = ctx.hip, ctx.s_ptr

    def one_step(rec):
        ev = {k: hip.event() for k in ("t0", "pre", "f32", "bf16", "cp_f32", "cp_bf16")}
        kev = {dt: [(hip.event(), hip.event()) for _ in range(N)] for dt in dtypes}
        cev = {dt: [(hip.event(), hip.event()) for _ in range(N)] for dt in dtypes}
        forms = {dt: [0] * N for dt in dtypes}
        hip.record(ev["t0"], s_ptr)
        if do_cp:
            w.X = ctx.api.Coo(w.coo.dims, w.inds_d, w.vals_d, workspace=w.ws_coo)  # preprocessing (waits once)
        hip.record(ev["pre"], s_ptr)
        for dt in dtypes:
            for n in range(N):
                ctx.plib.pasta_arm_kernel_events(kev[dt][n][0], kev[dt][n][1])
                hip.record(cev[dt][n][0], s_ptr)
                w.mttkrp(n, dt)
                hip.record(cev[dt][n][1], s_ptr)
                forms[dt][n] = ctx.last_form()
            hip.record(ev[dt], s_ptr)
        losses = {}
        if do_cp:
            for dt in ("f32", "bf16"):
                losses[dt] = w.cp_step(st, dt)
                hip.record(ev["cp_" + dt], s_ptr)
        rec.append((ev, kev, cev, forms, losses))

    log(f"warmup {args.warmup} steps")
    warm = []
    for _ in range(args.warmup):
        one_step(warm)
    torch.cuda.synchronize()
    log(f"timing {args.steps} steps")
    recs = []
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for _ in range(args.steps):
        one_step(recs)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    log(f"timed region {wall:.3f} s")

    K = len(recs)
    pre = sum(hip.ms(r[0]["t0"], r[0]["pre"]) for r in recs) / K
    call = {dt: [sum(hip.ms(*r[2][dt][n]) for r in recs) / K for n in range(N)] for dt in dtypes}
    kern = {dt: [sum(hip.ms(*r[1][dt][n]) for r in recs) / K for n in range(N)] for dt in dtypes}
    forms = recs[-1][3]
    head = dtypes[0]
    t_modes = sum(call[head])
    value = N * M / (t_modes * 1e-3) / 1e9
    kernel = kernel_label(forms[head])
    sf = 2 if head == "bf16" else 4
    qmin = [bytes_compulsory(w.coo.dims, R, sf, M, n) for n in range(N)]
    achieved = sum(qmin) / (sum(kern[head]) * 1e-3) / 1e9
    counters = measured_counters(w, kernel, head)
    traffic = counters.get("bytes_per_launch")
    vmem = counters.get("vmem_rd_instr_per_launch")
    mean_launch = sum(kern[head]) / N * 1e-3
    log("gather-pipeline probe and device copy")
    ceil = gather_ceiling(ctx, lanes_per_row(R, sf))
    copy_gbps = copy_rate(ctx)
    grate = w.gather_rate(head, kern[head]) / 1e9
    line = {
        "metric": METRIC,
        "value": round(value, 4),
        "unit": "Gnnz/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall * 1e3 / args.steps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": w.spec.name, "dims": list(w.coo.dims), "nnz": M, "rank": R, "order": N,
                   "factor_dtype": head, "distribution": f"Zipf{w.spec.zipf} over seeded permutations, distinct",
                   "values": w.spec.values, "seed": w.spec.seed},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBPS, 4), "traffic": traffic,
                     "bytes_model": "compulsory bytes per launch: nnz (4N + 4) + s_f R sum_{k != n} I_k + 4 R I_n",
                     "bytes_per_launch": qmin, "kernel": kernel, "launch_ms": [round(k, 4) for k in kern[head]],
                     "traffic_gbps": round(traffic / mean_launch / 1e9, 1) if traffic else None,
                     "traffic_frac": round(traffic / mean_launch / 1e9 / HBM_PEAK_GBPS, 4) if traffic else None,
                     "copy_gbps": round(copy_gbps, 1)},
        "gather_pipeline": {"nominal_gbps": round(grate, 1), **ceil,
                            "nominal_frac_of_l2_distinct": round(grate / ceil["l2_distinct_gbps"], 4),
                            # the kernel's load instructions (rocprofv3 SQ_INSTS_VMEM_RD per launch) per ns,
                            # against the probe's rate for L2-resident distinct rows
                            "kernel_vmem_instr_per_ns": round(vmem / (mean_launch * 1e9), 2) if vmem else None,
                            "instr_frac_of_l2_distinct": round(vmem / (mean_launch * 1e9) /
                                                               ceil["l2_distinct_instr_per_ns"], 4) if vmem else None,
                            "note": "the factor-row bytes the method reads per second (every row of every nonzero "
                                    "counted, also rows the kernel holds in registers or reads from LDS) vs the "
                                    "probe's rate for the same 16-byte-per-lane row gathers"},
        "model_fractions": {dt: w.fractions(dt, kern[dt]) for dt in dtypes},
        "breakdown_ms": {"preprocess": round(pre, 4),
                         **{f"mttkrp_all_modes_{dt}": round(sum(call[dt]), 4) for dt in dtypes},
                         **{f"mttkrp_per_mode_{dt}": [round(c, 4) for c in call[dt]] for dt in dtypes}},
    }
    if "bf16" in dtypes and head != "bf16":
        line["mttkrp_bf16_gnnz_s"] = round(N * M / (sum(call["bf16"]) * 1e-3) / 1e9, 4)
    if do_cp:
        # fp32 step: from the end of the MTTKRPs to its Adam update; bf16 step: the rest
        cp = {"f32": sum(hip.ms(r[0][dtypes[-1]], r[0]["cp_f32"]) for r in recs) / K,
              "bf16": sum(hip.ms(r[0]["cp_f32"], r[0]["cp_bf16"]) for r in recs) / K}
        line["cp_step_ms"] = {"f32": round(cp["f32"], 4), "bf16": round(cp["bf16"], 4),
                              "bf16_speedup": round(cp["f32"] / cp["bf16"], 3)}
        line["cp_loss_last"] = {dt: recs[-1][4][dt].item() for dt in ("f32", "bf16")}
    print(json.dumps({"partial": True, **line}), file=sys.stderr, flush=True)

    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        cb, (m, inds_s, vals_s, outs_o) = cpu_baseline(w.coo, w.U)
        line["cpu_baseline"] = cb
        import numpy as np
        import oracle
        ms_ = min(M, 2_000_000)
        i1 = np.ascontiguousarray(w.coo.inds[:, :ms_])
        v1 = w.coo.vals[:ms_].astype(np.float64)
        U64 = [u.astype(np.float64) for u in w.U]
        t1 = time.perf_counter()
        for n in range(N):
            oracle.mttkrp(w.coo.dims, i1, v1, U64, n, "seq")
        t1 = time.perf_counter() - t1
        line["cpu_baseline_1thread"] = {"value": round(N * ms_ / t1 / 1e9, 5), "unit": "Gnnz/s", "cores": 1,
                                        "kind": "oracle", "sample": f"the first {ms_} nonzeros, all {N} modes, "
                                        f"sequential FP64 MTTKRP, {t1:.1f} s"}
        log("errors against the oracle on the sample ...")
        line["error_vs_fp64_oracle"] = oracle_errors(ctx, w, m, inds_s, vals_s, outs_o, with_cp=do_cp)
        del outs_o, inds_s, vals_s

    if not args.no_extra and not args.mttkrp_only:
        extra = {}
        del st
        keep_cfg = args.config
        if keep_cfg == 2:
            line.update(order3_extras(ctx, w))
            log("CP fit on the planted tensor")
            line["cp_fit"] = cp_fit(ctx, w, args.fit_steps)
        del w
        torch.cuda.empty_cache()
        for cfg in (2, 3):
            if cfg == keep_cfg:
                continue
            log(f"side workload {cfg}")
            wx = Workload(ctx, cfg)
            row = side_row(ctx, wx)
            if cfg == 2:
                row.update(order3_extras(ctx, wx))
                log("CP fit on the planted tensor")
                row["cp_fit"] = cp_fit(ctx, wx, args.fit_steps)
                if not args.no_cpu_baseline:
                    import numpy as np
                    import oracle
                    log("whole-tensor errors of the order-3 tensor against the oracle ...")
                    Uo = [u.astype(np.float64) for u in wx.U]
                    outs_o = [oracle.mttkrp(wx.coo.dims, wx.coo.inds, wx.coo.vals.astype(np.float64), Uo, n, "auto")
                              for n in range(wx.N)]
                    row["error_vs_fp64_oracle"] = oracle_errors(ctx, wx, wx.coo.nnz, wx.coo.inds,
                                                                wx.coo.vals.astype(np.float64), outs_o)
            extra[wx.spec.name] = row
            del wx
            torch.cuda.empty_cache()
        line["other_workloads"] = extra
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
