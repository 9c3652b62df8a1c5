#!/usr/bin/env python3
"""Benchmark of the MI355X COO MTTKRP path on one GPU.

One step is one pass of the whole hot path over one synthetic tensor:
  1. preprocessing of the 50Kx40Kx30K, 50M-nonzero Zipf(1.1) tensor (index
     check, stable sort per mode, row offsets);
  2. MTTKRP of every mode, fp32 factors, R = 32;
  3. one CP gradient step in fp32 (loss + residual-weighted MTTKRP for every
     factor, Adam) on the same coordinates with planted rank-32 values;
  4. the same step with bf16 factor copies (fp32 masters, Adam writes the
     bf16 copies in the same pass).
`value` is the MTTKRP throughput of step 2, nonzeros x modes / time, in
Gnnz/s (the suite sums its MTTKRP times over all modes). Inputs are resident
in GPU memory before timing starts. With --config 3 or 5 the step runs on the
order-4 or order-5 workload (the CP step then on that tensor's own values).

Outside the timed steps the line also reports, on the headline tensor: a
CP-ALS sweep, fiber pre-processing, sparse TTM (R = 32) and TTV per mode,
same-pattern element-wise and tensor-scalar operations and the general
element-wise operation of the tensor with itself; the bandwidth of a plain
device copy (the achievable streaming rate beside the spec peak); and, unless
--no-cpu-baseline, the FP64 oracle timed on the host cores (all threads, and
one thread on a sample) with the GPU results' errors against it.

The roofline object prices the MTTKRP main kernel against the 8 TB/s HBM
peak under the algorithmic bytes model B = (4N + 4 + (N-1) R s_f) bytes per
nonzero + 4 R I_n per launch (Table 2's MTTKRP memory access for order N,
with the output row written once per row). The kernel's duration is taken
from HIP events recorded on its own stream around its launch. `traffic` is
that kernel's fabric bytes per launch as rocprofv3 measured them (FETCH_SIZE
and WRITE_SIZE, each scaled by what it reads for a plain device copy), taken
from profiles/ while the kernel sources are the ones it was measured on;
traffic_gbps and traffic_frac put it over the same launch time. The library
reports which MTTKRP kernel ran (the wave-run form on long rows, else the run
form); --mttkrp-form forces one.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import ctypes
import hashlib
import json
import math
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


def traffic_file(kernel: str) -> str:
    """The committed FETCH_SIZE / WRITE_SIZE summary of a main MTTKRP kernel on the headline tensor."""
    return os.path.join(ROOT, "profiles", kernel.replace("_kernel", "") + "_zipf50M_r32_traffic.json")


# --------------------------------------------------------------------------------------
# bytes model (Table 2 of the suite, generalised to order N and factor element size s_f)
# --------------------------------------------------------------------------------------
def bytes_paper(N: int, R: int, sf: int) -> int:
    """Table 2's MTTKRP memory access per nonzero: N indices, one value, N-1 gathered
    factor rows and one output-row update (16 + 12R at N = 3, fp32)."""
    return 4 * N + 4 + (N - 1) * R * sf + 4 * R


def bytes_alg_per_nnz(N: int, R: int, sf: int) -> int:
    """Bytes per nonzero the method must move with no factor-row reuse: the index
    and value stream plus N-1 gathered rows (the output row is written per row)."""
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
    """Every byte touched once: the stream, every other factor once, the output once."""
    N = len(dims)
    return nnz * (4 * N + 4) + sf * R * sum(d for k, d in enumerate(dims) if k != n) + 4 * R * dims[n]


def kernel_hash() -> str:
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        h.update(open(p, "rb").read())
    return h.hexdigest()[:16]


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


def cpu_baseline(coo, U, budget_s: float = 12.0):
    """The FP64 oracle (privatised OpenMP MTTKRP, all modes) timed on the host cores:
    whole-tensor passes repeated until about ``budget_s`` seconds, or a prefix of the
    nonzeros (a uniform sample: caller order is random) if one pass would take longer."""
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
    run(m)  # first touch of the buffers and thread start-up
    t, _, _, _ = run(m)
    per_nnz = t / m
    if per_nnz * coo.nnz > 2.5 * budget_s:
        m = max(m, int(budget_s / per_nnz))
    else:
        m = coo.nnz
    # passes until about budget_s seconds (the small first run overstates the per-nonzero cost)
    reps, total = 0, 0.0
    while reps == 0 or total < budget_s:
        t, outs, inds, vals = run(m)
        total += t
        reps += 1
    what = "the whole tensor" if m == coo.nnz else f"the first {m} of {coo.nnz} nonzeros (a uniform sample)"
    return {"value": round(reps * coo.order * m / total / 1e9, 5), "unit": "Gnnz/s", "cores": threads,
            "kind": "oracle",
            "sample": f"{what}, all {coo.order} modes, {reps} passes, FP64 privatised OpenMP MTTKRP, {total:.1f} s"}, \
        (m, inds, vals, outs)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--config", type=int, default=2, help="2 (headline), 3 or 5: MTTKRP workload")
    ap.add_argument("--mttkrp-only", action="store_true", help="time only the all-mode MTTKRP (profiling runs)")
    ap.add_argument("--factor-dtype", choices=["f32", "bf16"], default="f32",
                    help="factor storage of the MTTKRP step (arithmetic is fp32 either way)")
    ap.add_argument("--cache", default=os.environ.get("PASTA_BENCH_CACHE", ""),
                    help="directory for cached generated tensors (reused between runs)")
    ap.add_argument("--mttkrp-form", choices=["auto", "run", "wave"], default="auto",
                    help="MTTKRP kernel form (auto: wave-run form for long rows)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MiB",
                    help="run one plain device copy of this size (counter calibration) and exit")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}, WORLD_SIZE {world}); "
              "this build has no multi-GPU path.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    so = os.path.join(ROOT, "paper_1902_03317_amd", "libpasta.so")
    if not os.path.exists(so):
        import __graft_entry__
        __graft_entry__.build()
    from paper_1902_03317_amd import api, synth
    from paper_1902_03317_amd.autograd import adam_step

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.copy_calibration:
        n = args.copy_calibration << 20
        a = torch.ones(n // 4, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": n, "copy_bytes_written": n}))
        return

    hip = Hip()
    from paper_1902_03317_amd._lib import lib as _plib
    _plib.pasta_set_mttkrp_form({"auto": 0, "run": 1, "wave": 2}[args.mttkrp_form])
    spec = synth.CONFIGS[args.config]
    N, R = spec.order, spec.rank
    t0 = time.perf_counter()
    coo = synth.load_or_make_coo(spec, args.cache)
    U = synth.make_factors(spec)
    log(f"generated {spec.name}: {coo.nnz} nonzeros in {time.perf_counter() - t0:.1f} s")
    inds_d = torch.from_numpy(coo.inds.view(np.int32)).to(dev)
    vals_d = torch.from_numpy(coo.vals).to(dev)
    Ud = [torch.from_numpy(u).to(dev) for u in U]
    if args.factor_dtype == "bf16":
        Ud = [api.cast_bf16(u) for u in Ud]
    outs = [torch.empty((d, R), dtype=torch.float32, device=dev) for d in coo.dims]
    ws_coo = torch.empty(api.coo_workspace_bytes(coo.dims, coo.nnz), dtype=torch.uint8, device=dev)
    X = api.Coo(coo.dims, inds_d, vals_d, workspace=ws_coo)
    ws_m = torch.empty(max(api.mttkrp_workspace_bytes(X, n, R, Ud[0].dtype) for n in range(N)), dtype=torch.uint8,
                       device=dev)

    do_cp = not args.mttkrp_only
    do_extra = do_cp and args.config == 2  # CP-ALS, TTM/TTV and TEW/TS timings: headline tensor only
    if do_cp:
        sc = synth.cp_planted_scale(R, N)
        if args.config == 2:
            # the CP fit's tensor: same coordinates, planted rank-R values + 1% noise
            cspec = synth.CONFIGS[4]
            A = [torch.from_numpy(a).to(dev) for a in synth.make_factors(cspec, rank=R, scale=sc)]
            x = api.cp_sample(X, A)
            rms = torch.sqrt(torch.mean(x.double() ** 2)).item()
            noise = torch.from_numpy(synth.make_noise(cspec, coo.nnz).astype(np.float32)).to(dev)
            xv = (x + np.float32(0.01 * rms) * noise).contiguous()
            del noise, x, A
            X4 = api.Coo(coo.dims, inds_d, xv)
        else:  # the gradient step on the tensor's own values (its timing does not depend on them)
            cspec = spec
            X4 = X
        init = synth.make_init(cspec, rank=R, scale=sc)
        m32 = [torch.from_numpy(u).to(dev) for u in init]
        m16 = [t.clone() for t in m32]
        sh16 = [api.cast_bf16(t) for t in m16]
        st32 = [(torch.zeros_like(t), torch.zeros_like(t)) for t in m32]
        st16 = [(torch.zeros_like(t), torch.zeros_like(t)) for t in m16]
        g32 = [torch.empty_like(t) for t in m32]
        g16 = [torch.empty_like(t) for t in m16]
        ws_g = torch.empty(api.cp_grad_workspace_bytes(X4, R, torch.float32), dtype=torch.uint8, device=dev)
        ws_g16 = torch.empty(api.cp_grad_workspace_bytes(X4, R, torch.bfloat16), dtype=torch.uint8, device=dev)
        step_no = {"f32": 0, "bf16": 0}
    torch.cuda.synchronize()

    stream = torch.cuda.current_stream().cuda_stream
    s_ptr = ctypes.c_void_p(stream)
    from paper_1902_03317_amd._lib import lib as plib

    form = ctypes.c_int(0)
    forms = [0] * N  # which main kernel each mode's MTTKRP launched

    def one_step(rec):
        nonlocal X
        ev = [hip.event() for _ in range(6)]
        kev = [(hip.event(), hip.event()) for _ in range(N)]
        cev = [(hip.event(), hip.event()) for _ in range(N)]
        hip.record(ev[0], s_ptr)
        if not args.mttkrp_only:
            X = api.Coo(coo.dims, inds_d, vals_d, workspace=ws_coo)  # preprocessing (waits once)
        hip.record(ev[1], s_ptr)
        for n in range(N):
            plib.pasta_arm_kernel_events(kev[n][0], kev[n][1])
            hip.record(cev[n][0], s_ptr)
            api.mttkrp(X, Ud, n, out=outs[n], workspace=ws_m)
            hip.record(cev[n][1], s_ptr)
            plib.pasta_last_mttkrp_form(ctypes.byref(form))
            forms[n] = form.value
        hip.record(ev[2], s_ptr)
        losses = {}
        if do_cp:
            step_no["f32"] += 1
            l32, _ = api.cp_grad(X4, m32, grads=g32, workspace=ws_g)
            adam_step(m32, g32, [s[0] for s in st32], [s[1] for s in st32], step_no["f32"])
            hip.record(ev[3], s_ptr)
            step_no["bf16"] += 1
            l16, _ = api.cp_grad(X4, sh16, grads=g16, workspace=ws_g16)
            adam_step(m16, g16, [s[0] for s in st16], [s[1] for s in st16], step_no["bf16"], shadows=sh16)
            hip.record(ev[4], s_ptr)
            losses = {"f32": l32, "bf16": l16}
        else:
            hip.record(ev[3], s_ptr)
            hip.record(ev[4], s_ptr)
        rec.append((ev, kev, cev, losses))

    log(f"warmup {args.warmup} steps")
    warm = []
    for _ in range(args.warmup):
        one_step(warm)
    torch.cuda.synchronize()
    log(f"timing {args.steps} steps")
    recs = []
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for i in range(args.steps):
        one_step(recs)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    log(f"timed region {wall:.3f} s")

    pre, mtt, cp32, cp16, kern, call = [], [], [], [], [[] for _ in range(N)], [[] for _ in range(N)]
    loss_hist = []
    for ev, kev, cev, losses in recs:
        pre.append(hip.ms(ev[0], ev[1]))
        mtt.append(hip.ms(ev[1], ev[2]))
        cp32.append(hip.ms(ev[2], ev[3]))
        cp16.append(hip.ms(ev[3], ev[4]))
        for n in range(N):
            kern[n].append(hip.ms(kev[n][0], kev[n][1]))
            call[n].append(hip.ms(cev[n][0], cev[n][1]))
        if losses:
            loss_hist.append((losses["f32"].item(), losses["bf16"].item()))
    M = coo.nnz
    t_modes = sum(sum(c) for c in call) / len(recs)  # ms per all-mode MTTKRP
    value = N * M / (t_modes * 1e-3) / 1e9
    sf = 2 if args.factor_dtype == "bf16" else 4
    kern_ms = [sum(k) / len(k) for k in kern]
    alg_bytes = [bytes_alg(N, R, sf, M, coo.dims[n]) for n in range(N)]
    achieved = sum(alg_bytes) / (sum(kern_ms) * 1e-3) / 1e9  # GB/s over the launches of all modes
    kernel = KERNEL_NAMES.get(forms[0], "?") if len(set(forms)) == 1 else [KERNEL_NAMES.get(f, "?") for f in forms]
    traffic = None
    if isinstance(kernel, str) and os.path.exists(traffic_file(kernel)):
        tr = json.load(open(traffic_file(kernel)))
        if (tr.get("kernel_hash") == kernel_hash() and tr.get("workload") == spec.name
                and kernel in tr.get("kernel", "") and tr.get("factor_dtype") == args.factor_dtype):
            traffic = tr.get("bytes_per_launch")
    ms_step = wall * 1e3 / args.steps
    # achievable streaming bandwidth on this device: a plain 1 GiB device-to-device copy
    cbuf = torch.empty(1 << 28, dtype=torch.float32, device=dev)
    cdst = torch.empty_like(cbuf)
    cdst.copy_(cbuf)
    ctimes = []
    for _ in range(5):
        a0, a1 = hip.event(), hip.event()
        hip.record(a0, s_ptr)
        cdst.copy_(cbuf)
        hip.record(a1, s_ptr)
        ctimes.append(hip.ms(a0, a1))
    copy_gbps = 2 * cbuf.numel() * 4 / (sorted(ctimes)[2] * 1e-3) / 1e9
    del cbuf, cdst
    line = {
        "metric": METRIC,
        "value": round(value, 4),
        "unit": "Gnnz/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": spec.name, "dims": list(coo.dims), "nnz": M, "rank": R, "order": N,
                   "factor_dtype": args.factor_dtype, "distribution": f"Zipf{spec.zipf} over seeded permutations, distinct",
                   "values": spec.values, "seed": spec.seed},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBPS, 4), "traffic": traffic,
                     # the measured fabric bytes per launch over the same launch time
                     "traffic_gbps": round(traffic / (sum(kern_ms) / N * 1e-3) / 1e9, 1) if traffic else None,
                     "traffic_frac": round(traffic / (sum(kern_ms) / N * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4)
                     if traffic else None,
                     "copy_gbps": round(copy_gbps, 1),
                     "kernel": kernel, "bytes_per_nnz": bytes_alg_per_nnz(N, R, sf),
                     "launch_ms": [round(k, 4) for k in kern_ms]},
        "breakdown_ms": {"preprocess": round(sum(pre) / len(pre), 4), "mttkrp_all_modes": round(t_modes, 4),
                         "mttkrp_per_mode": [round(sum(c) / len(c), 4) for c in call],
                         "cp_step_f32": round(sum(cp32) / len(cp32), 4) if do_cp else None,
                         "cp_step_bf16": round(sum(cp16) / len(cp16), 4) if do_cp else None},
        "model_fractions": {
            "b_alg": round(achieved / HBM_PEAK_GBPS, 4),
            "b_paper": round(sum(M * bytes_paper(N, R, sf) for _ in range(N)) / (sum(kern_ms) * 1e-3) / 1e9
                             / HBM_PEAK_GBPS, 4),
            "q_min": round(sum(bytes_compulsory(coo.dims, R, sf, M, n) for n in range(N)) /
                           (sum(kern_ms) * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4)},
    }
    if do_cp:
        line["cp_step_ms"] = {"f32": line["breakdown_ms"]["cp_step_f32"], "bf16": line["breakdown_ms"]["cp_step_bf16"],
                              "bf16_speedup": round(line["breakdown_ms"]["cp_step_f32"] /
                                                    line["breakdown_ms"]["cp_step_bf16"], 3)}
        line["cp_loss_last"] = {"f32": loss_hist[-1][0], "bf16": loss_hist[-1][1]}
    if do_extra:
        # CP-ALS sweep (MTTKRP + normal equations + normalisation, every mode), timed apart
        Ua = [u.clone() for u in Ud] if args.factor_dtype == "f32" else [torch.from_numpy(u).to(dev) for u in U]
        lam = torch.empty(R, dtype=torch.float32, device=dev)
        import ctypes as _ct
        nb = _ct.c_size_t()
        plib.pasta_cp_als_workspace_bytes(X.handle, R, _ct.byref(nb))
        ws_a = torch.empty(nb.value, dtype=torch.uint8, device=dev)
        for _ in range(2):
            api.cp_als_sweep(X, Ua, lam=lam, workspace=ws_a)
        ts = []
        for _ in range(5):
            e0, e1 = hip.event(), hip.event()
            hip.record(e0, s_ptr)
            _, fit, _ = api.cp_als_sweep(X, Ua, lam=lam, workspace=ws_a)
            hip.record(e1, s_ptr)
            ts.append(hip.ms(e0, e1))
        line["cp_als_sweep_ms"] = round(sorted(ts)[len(ts) // 2], 4)
    if do_extra:
        # sparse TTM (rank R, fp32 U) and TTV along every mode (Algs. 5 and 4), timed apart:
        # fiber pre-processing once per mode, then call and main-kernel times (median of 10)
        Uf = [torch.from_numpy(u).to(dev) for u in U]
        fib = {"ttm": ([], []), "ttv": ([], [])}
        pre_f, nfibs = [], []
        for n in range(N):
            e0, e1 = hip.event(), hip.event()
            hip.record(e0, s_ptr)
            F = api.Fibers(X, n)
            hip.record(e1, s_ptr)
            pre_f.append(hip.ms(e0, e1))
            nfibs.append(F.nfibs)
            y = torch.empty((F.nfibs, R), dtype=torch.float32, device=dev)
            yv = torch.empty(F.nfibs, dtype=torch.float32, device=dev)
            ws_t = torch.empty(max(api.ttm_workspace_bytes(F, R), api.ttv_workspace_bytes(F)), dtype=torch.uint8,
                               device=dev)
            v = Uf[n][:, 0].contiguous()
            runs = {"ttm": lambda: api.ttm(F, Uf[n], out=y, workspace=ws_t),
                    "ttv": lambda: api.ttv(F, v, out=yv, workspace=ws_t)}
            for name, fn in runs.items():
                fn()
                fn()
                calls, kerns = [], []
                for _ in range(10):
                    k0, k1, c0, c1 = hip.event(), hip.event(), hip.event(), hip.event()
                    plib.pasta_arm_kernel_events(k0, k1)
                    hip.record(c0, s_ptr)
                    fn()
                    hip.record(c1, s_ptr)
                    calls.append(hip.ms(c0, c1))
                    kerns.append(hip.ms(k0, k1))
                fib[name][0].append(sorted(calls)[5])
                fib[name][1].append(sorted(kerns)[5])
            del F, y, yv, ws_t
        for name in ("ttm", "ttv"):
            calls, kerns = fib[name]
            algb = [bytes_ttm(R, 4, M, nf) if name == "ttm" else bytes_ttv(M, nf) for nf in nfibs]
            line[name] = {"gnnz_s": round(N * M / (sum(calls) * 1e-3) / 1e9, 3),
                          "ms_per_mode": [round(c, 4) for c in calls], "kernel_ms": [round(k, 4) for k in kerns],
                          "hbm_frac": round(sum(algb) / (sum(kerns) * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4),
                          "bytes_alg_per_mode": algb, "nfibs": nfibs}
        line["ttm"]["rank"] = R
        line["fibers_preprocess_ms"] = [round(t, 3) for t in pre_f]

        # same-pattern element-wise op, tensor-scalar op (pure streams) and the general
        # element-wise op of the tensor with itself (the paper's setup: sort + merge)
        def timed(fn, reps):
            fn()
            ts_ = []
            for _ in range(reps):
                a0, a1 = hip.event(), hip.event()
                hip.record(a0, s_ptr)
                fn()
                hip.record(a1, s_ptr)
                ts_.append(hip.ms(a0, a1))
            return sorted(ts_)[len(ts_) // 2]

        y2 = (vals_d * 0.5 + 1.0).contiguous()
        zt = torch.empty_like(vals_d)
        t_eq = timed(lambda: api.tew_eq("add", vals_d, y2, out=zt), 10)
        t_ts = timed(lambda: api.ts("mul", vals_d, 0.5, out=zt), 10)
        ws_tew = torch.empty(api.tew_workspace_bytes(N, M, M), dtype=torch.uint8, device=dev)
        res = {}

        def general():
            res["z"] = api.tew("add", coo.dims, inds_d, vals_d, coo.dims, inds_d, vals_d, workspace=ws_tew)
        t_tew = timed(general, 3)
        for name, t, nb in (("tew_eq", t_eq, 12 * M), ("ts", t_ts, 8 * M)):
            line[name] = {"op": "add" if name == "tew_eq" else "mul", "ms": round(t, 4),
                          "gb_s": round(nb / (t * 1e-3) / 1e9, 1),
                          "hbm_frac": round(nb / (t * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4), "bytes": nb}
        line["tew"] = {"op": "add", "inputs": "the tensor with itself", "ms": round(t_tew, 3),
                       "gnnz_s": round(2 * M / (t_tew * 1e-3) / 1e9, 3), "nnz_out": int(res["z"][2].numel())}
        del ws_tew, res, y2, zt
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        cb, (m, inds_s, vals_s, outs_o) = cpu_baseline(coo, U)
        line["cpu_baseline"] = cb
        # the single-thread sequential oracle (the suite's speedup reference), on the first 2M nonzeros
        import oracle
        ms = min(coo.nnz, 2_000_000)
        i1 = np.ascontiguousarray(coo.inds[:, :ms])
        v1 = coo.vals[:ms].astype(np.float64)
        U64 = [u.astype(np.float64) for u in U]
        t1 = time.perf_counter()
        for n in range(N):
            oracle.mttkrp(coo.dims, i1, v1, U64, n, "seq")
        t1 = time.perf_counter() - t1
        line["cpu_baseline_1thread"] = {"value": round(N * ms / t1 / 1e9, 5), "unit": "Gnnz/s", "cores": 1,
                                        "kind": "oracle", "sample": f"the first {ms} nonzeros, all {N} modes, "
                                        f"sequential FP64 MTTKRP, {t1:.1f} s"}
        # error of the GPU path on the same sample vs the FP64 oracle results just computed
        import oracle
        Xs = X if m == coo.nnz else api.Coo(coo.dims, torch.from_numpy(inds_s.view(np.int32)).to(dev),
                                            torch.from_numpy(vals_s.astype(np.float32)).to(dev))
        U32 = [torch.from_numpy(u).to(dev) for u in U]  # the fp32 factors, whatever the timed dtype
        e32 = max(oracle.rel_fro(api.mttkrp(Xs, U32, n).cpu().numpy(), outs_o[n]) for n in range(N))
        Ub = [api.cast_bf16(u) for u in U32]
        e16 = max(oracle.rel_fro(api.mttkrp(Xs, Ub, n).cpu().numpy(), outs_o[n]) for n in range(N))
        line["error_vs_fp64_oracle"] = {"mttkrp_f32_max_mode_rel_fro": e32, "mttkrp_bf16_max_mode_rel_fro": e16,
                                        "sample_nnz": m}
        if do_cp:
            # the CP gradient (loss + every factor's gradient) at the fit's starting point, fp32 and bf16
            # factors, against the FP64 oracle's gradient of the same sample
            init_s = synth.make_init(cspec, rank=R, scale=synth.cp_planted_scale(R, N))
            I32 = [torch.from_numpy(u).to(dev) for u in init_s]
            _, gg32 = api.cp_grad(Xs, I32)
            _, gg16 = api.cp_grad(Xs, [api.cast_bf16(u) for u in I32])
            _, go = oracle.cp_grad(coo.dims, inds_s, vals_s, [u.astype(np.float64) for u in init_s], "auto")
            line["error_vs_fp64_oracle"]["cp_grad_f32_max_mode_rel_fro"] = max(
                oracle.rel_fro(gg32[n].cpu().numpy(), go[n]) for n in range(N))
            line["error_vs_fp64_oracle"]["cp_grad_bf16_max_mode_rel_fro"] = max(
                oracle.rel_fro(gg16[n].cpu().numpy(), go[n]) for n in range(N))
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
