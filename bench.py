#!/usr/bin/env python3
"""Benchmark: delayed-update Cholesky on one MI355X.

Workload (one "step"): the binary64 Cholesky factorisation of
A = G G^T / n + I (G n x n i.i.d. N(0,1)), n = 16384, through chol_factor -- the
whole hot path: diagonal factorisations, panel solves and the trailing updates
S = R R^T subtracted from the remaining matrix (Sec. 2, Algorithm 1 of
arXiv 1812.02056).  The step size s is swept over {64, 118, 168, 256, 384, 512,
640, 768} (168 ~ n^0.5286 is the paper's step, 118 the configuration's listed
value); the reported value is the best s.  Metric: TFLOP/s counted as n^3/3 per
factorisation.  Inputs are resident in HBM (one fresh copy of A per timed step)
before the timed region starts.

Also reported on the same JSON line: the dominant trailing-update kernel of the
timed steps against its roofline (binary64 MFMA peak; its launches are timed
with HIP events on the stream they run on), the CPU oracle's rate on the same
matrix, the fixed-step schedule, the one-level Strassen update, LU without
pivoting (2n^3/3) with one and two Strassen levels, the binary32 and
bfloat16-operand factorisations with their update kernels, the triangular
solves, QR (Sec. 2, Algorithm 3) over its step sweep and at the paper's sizes,
the mixed-precision table (n in {16384, 32768}, lambda in {1, 1e-3, 1e-6}, 1 and
16 right-hand sides, every result's error stated) and the serving workload.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--quick]
    python bench.py --leg lowprec|trisolve|qr|solve     # one leg alone, for profiling
    python bench.py --copy-calibration                  # 1 GiB copies for HBM counter scaling
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

MI355X_HBM_GBS = 8000.0
MI355X_PEAK_TFLOPS = {"f64": 78.6, "f32": 157.3, "bf16": 2500.0}
# sources the update kernel is built from (the traffic record names their hash)
UPDATE_SRCS = [os.path.join(ROOT, "paper_1812_02056_amd", "csrc", f) for f in ("update.hip", "grid.hpp", "common.hpp")]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "update_wide_f64_n16384_traffic.json")
KERNEL_OF_SHAPE = {"64x64": "update_wide_kernel<double, 32, 2, ...>",
                   "128x128": "update_wide_kernel<double, 64, 2, ...>",
                   "256x128": "update_wide_kernel<double, 64, 4, ...>"}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=5)
    p.add_argument("--warmup", type=int, default=2)
    p.add_argument("--n", type=int, default=16384)
    p.add_argument("--s", type=str, default="64,118,168,256,384,512,640,768")
    p.add_argument("--quick", action="store_true", help="headline only: no LU / Strassen / mixed / CPU legs")
    p.add_argument("--no-cpu", action="store_true")
    p.add_argument("--no-extras", action="store_true")
    p.add_argument("--no-mixed", action="store_true", help="skip the mixed-precision table")
    p.add_argument("--mixed-only", action="store_true", help="only the mixed-precision table")
    p.add_argument("--leg", choices=("lowprec", "trisolve", "qr", "solve"), default=None,
                   help="only one leg, for profiling: the binary32 / bfloat16 factorisations, the triangular "
                        "solves, QR, or one mixed-precision cell (lambda = 1e-6, 1 and 16 right-hand sides)")
    p.add_argument("--qr-steps", type=str, default="64,96,112,128,142",
                   help="step sizes of the QR leg's sweep at n = 16384")
    p.add_argument("--serving-only", action="store_true", help="only the serving leg (many independent solves)")
    p.add_argument("--serving-requests", type=int, default=10000)
    p.add_argument("--copy-calibration", action="store_true",
                   help="only run a plain 1 GiB device copy 3 times (reference kernel for HBM counter scaling)")
    return p.parse_args()


def source_hash(paths):
    h = hashlib.sha256()
    for path in paths:
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: this library has no multi-GPU path "
              "(the sharding design is documented, not built); run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_1812_02056_amd as ff
    from paper_1812_02056_amd import workloads as wl  # noqa: F811

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    dev = torch.device("cuda:0")
    if args.copy_calibration:
        src = torch.ones(1 << 27, dtype=torch.float64, device=dev)     # 1 GiB
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log("[bench] copy calibration: 3 x 1 GiB read + 1 GiB written")
        return
    ff.load()
    if args.leg is not None:
        n = args.n
        if args.leg == "lowprec":
            A0 = wl.spd_scaled_device(n, seed=0, lam=1.0, device=dev)
            res = run_low_precision_factor(ff, torch, dev, n, A0)
        elif args.leg == "qr":
            res = run_qr(ff, torch, wl, dev, n=n, steps=tuple(int(v) for v in args.qr_steps.split(",")))
        elif args.leg == "solve":
            res = run_solve_cell(ff, torch, wl, dev, n)
        else:
            res = run_trisolve(ff, torch, dev, n)
        log(f"[bench] {args.leg}: {res}")
        print(json.dumps({args.leg: res}), flush=True)
        return
    if args.mixed_only:
        from paper_1812_02056_amd import workloads as wl
        res = run_mixed_table(ff, torch, wl, dev, oracle_refs=not args.no_cpu)
        print(json.dumps({"mixed_solve": res}), flush=True)
        return
    if args.serving_only:
        from paper_1812_02056_amd import workloads as wl
        res = run_serving(ff, torch, wl, dev, nreq=args.serving_requests)
        print(json.dumps({"serving": res}), flush=True)
        return
    n = args.n
    svals = [int(x) for x in args.s.split(",")]
    K, W = args.steps, args.warmup
    flops = n ** 3 / 3.0

    log(f"[bench] generating A = G G^T/n + I, n={n}")
    A0 = wl.spd_scaled_device(n, seed=0, lam=1.0, device=dev)          # symmetric: row-major == column-major
    torch.cuda.synchronize()

    sweep = {}
    best = None
    for s in svals:
        copies = [A0.clone() for _ in range(W + K)]
        info = torch.zeros(1, dtype=torch.int32, device=dev)
        for i in range(W):
            ff.chol_factor(copies[i].t(), s, dtype="f64", info=info)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(W, W + K):
            ff.chol_factor(copies[i].t(), s, dtype="f64", info=info)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / K
        ok = int(info.item()) == 0
        sweep[s] = {"ms": dt * 1e3, "tflops": flops / dt / 1e12, "info": int(info.item())}
        log(f"[bench] chol f64 n={n} s={s}: {dt*1e3:.2f} ms  {flops/dt/1e12:.2f} TFLOP/s  info={info.item()}")
        if ok and (best is None or dt < sweep[best]["ms"] / 1e3):
            best = s
        del copies
    if best is None:
        print("every factorisation reported a failure", file=sys.stderr)
        sys.exit(1)
    s = best
    # timed region proper: K steps of the best s, bracketed by synchronisation
    copies = [A0.clone() for _ in range(W + K)]
    info = torch.zeros(1, dtype=torch.int32, device=dev)
    for i in range(W):
        ff.chol_factor(copies[i].t(), s, dtype="f64", info=info)
    torch.cuda.synchronize()
    # The library brackets each trailing-update launch with HIP events on its own
    # stream while profiling is on; event records cost microseconds of host time
    # each, so the K steps are timed once without and once with them.
    t0 = time.perf_counter()
    for i in range(W, W + K):
        ff.chol_factor(copies[i].t(), s, dtype="f64", info=info)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / K
    for i in range(W, W + K):
        copies[i].copy_(A0)
    torch.cuda.synchronize()
    ff.update_profile_enable(True)
    for i in range(W, W + K):
        ff.chol_factor(copies[i].t(), s, dtype="f64", info=info)
    torch.cuda.synchronize()
    ff.update_profile_enable(False)
    prof = ff.update_profile_read()
    if int(info.item()) != 0:
        print(f"factorisation failed: info={int(info.item())}", file=sys.stderr)
        sys.exit(1)
    value = flops / dt / 1e12
    log(f"[bench] timed: s={s} {dt*1e3:.2f} ms/step  {value:.2f} TFLOP/s")

    # accuracy of the timed factor: backward error via a binary64 GEMM (torch, not this library)
    L = torch.tril(copies[-1].t())      # column-major buffer viewed as a matrix: element (i,j) = buffer[j, i]
    Am = A0.t()
    bwd = float(torch.linalg.norm(Am - L @ L.t()) / torch.linalg.norm(Am))
    del L, copies
    torch.cuda.empty_cache()

    # roofline of the dominant kernel: the trailing-update shape with the most time
    shape, pk = max(prof.items(), key=lambda kv: kv[1]["total_ms"])
    avg_ms = pk["total_ms"] / max(1, pk["launches"])
    avg_flops = pk["total_flops"] / max(1, pk["launches"])
    achieved = avg_flops / (avg_ms * 1e-3) / 1e12
    peak = MI355X_PEAK_TFLOPS["f64"]
    kname = KERNEL_OF_SHAPE[shape]
    traffic = None
    if os.path.exists(TRAFFIC_FILE):
        try:
            tr = json.load(open(TRAFFIC_FILE)).get(str(s), {})   # one record per step size
            if (tr.get("source_sha256_16") == source_hash(UPDATE_SRCS) and int(tr.get("s", -1)) == s
                    and tr.get("kernel") == kname):
                traffic = tr.get("bytes_per_launch")
        except Exception:
            traffic = None
    roofline = {"bound": "mfma", "achieved": round(achieved, 3), "peak": peak, "unit": "TFLOP/s",
                "frac": round(achieved / peak, 4), "traffic": traffic, "traffic_unit": "bytes/launch",
                "kernel": kname, "avg_launch_ms": round(avg_ms, 4), "launches": pk["launches"],
                "flops_per_launch": avg_flops,
                "algorithmic_bytes_per_launch": round(pk.get("total_bytes", 0.0) / max(1, pk["launches"])),
                "time_share_of_step": round(pk["total_ms"] / (K * dt * 1e3), 4),
                "other_update_shapes": {k: v for k, v in prof.items() if k != shape and v["launches"]}}
    log(f"[bench] dominant kernel {kname}: avg {avg_ms:.3f} ms/launch over {pk['launches']} launches, "
        f"{achieved:.2f} TFLOP/s ({achieved/peak*100:.1f}% of FP64 MFMA peak), "
        f"{pk['total_ms'] / (K * dt * 1e3) * 100:.1f}% of step time")

    # the same step with every block exactly s wide (Algorithm 1's schedule verbatim):
    # by default blocks at the start and over the last 6144 columns are 192 wide
    fixed = None
    if s > 192 and not args.quick and not args.no_extras:
        copies = [A0.clone() for _ in range(W + K)]
        for i in range(W):
            ff.chol_factor(copies[i].t(), s, dtype="f64", info=info, fixed_step=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(W, W + K):
            ff.chol_factor(copies[i].t(), s, dtype="f64", info=info, fixed_step=True)
        torch.cuda.synchronize()
        dtf = (time.perf_counter() - t0) / K
        fixed = {"s": s, "ms": round(dtf * 1e3, 3), "tflops": round(flops / dtf / 1e12, 3), "info": int(info.item())}
        log(f"[bench] fixed step s={s}: {dtf*1e3:.2f} ms  {flops/dtf/1e12:.2f} TFLOP/s")
        del copies
        torch.cuda.empty_cache()

    extras = {}
    if not args.quick and not args.no_extras:
        extras = run_extras(ff, torch, wl, dev, n, A0)
    A_host = A0.cpu().numpy() if (not args.quick and not args.no_cpu) else None
    del A0
    torch.cuda.empty_cache()

    cpu, L_oracle = None, None
    if A_host is not None:
        cpu, L_oracle = cpu_baseline(A_host)
        del A_host

    if not args.quick and not args.no_extras and not args.no_mixed:
        try:
            extras["mixed_solve"] = run_mixed_table(ff, torch, wl, dev, oracle_refs=not args.no_cpu,
                                                    oracle_L1=L_oracle)
        except Exception as e:
            extras["mixed_solve"] = {"error": str(e)}
    del L_oracle

    line = {
        "metric": "Cholesky TFLOP/s (n^3/3), FP64, n=16384",
        "value": round(value, 3),
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": round(dt * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"Cholesky FP64 A=GG^T/n+I n={n}, step size s={s} (best of sweep {svals})"
                               + ("; first block and last 6144 columns in 192-column blocks" if s > 192 else ""),
                   "n": n, "s": s, "parallelism": "single GPU"},
        "bwd_A": bwd,
        "s_sweep": {str(k): round(v["tflops"], 3) for k, v in sweep.items()},
        "fixed_step": fixed,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    line.update(extras)
    print(json.dumps(line), flush=True)


def run_extras(ff, torch, wl, dev, n, A0):
    out = {}
    # --- one Strassen level in the update, same workload, s = 512 and 256
    try:
        res = {}
        for s in (256, 512):
            for strassen in (False, True):
                Ac = A0.clone()
                info = torch.zeros(1, dtype=torch.int32, device=dev)
                ff.chol_factor(Ac.t(), s, dtype="f64", strassen=strassen, info=info)   # warm
                Ac.copy_(A0)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                ff.chol_factor(Ac.t(), s, dtype="f64", strassen=strassen, info=info)
                torch.cuda.synchronize()
                dt = time.perf_counter() - t0
                L = torch.tril(Ac.t())
                bwd = float(torch.linalg.norm(A0.t() - L @ L.t()) / torch.linalg.norm(A0))
                res[f"s{s}_{'strassen1' if strassen else 'classical'}"] = {
                    "ms": round(dt * 1e3, 3), "tflops_nominal": round(n ** 3 / 3 / dt / 1e12, 3), "bwd_A": bwd}
                del L, Ac
        out["strassen_vs_classical"] = res
        log(f"[bench] strassen: {res}")
    except Exception as e:  # report, never hide
        out["strassen_vs_classical"] = {"error": str(e)}
    torch.cuda.empty_cache()

    # --- LU without pivoting, diagonally dominant, n = 16384: step sizes swept, the
    #     best one timed over three factorisations and its backward error reported
    try:
        D = wl.diag_dominant_device(n, seed=0, device=dev)
        Dc = D.clone()
        info = torch.zeros(1, dtype=torch.int32, device=dev)
        sweep_lu = {}
        for s_lu in (168, 256, 512, 768):
            Dc.copy_(D)
            ff.lu_nopiv_factor(Dc.t(), s_lu, info=info)      # warm-up
            best_lu = 1e30
            for _ in range(3):
                Dc.copy_(D)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                ff.lu_nopiv_factor(Dc.t(), s_lu, info=info)
                torch.cuda.synchronize()
                best_lu = min(best_lu, time.perf_counter() - t0)
            sweep_lu[s_lu] = best_lu
        s_lu = min(sweep_lu, key=sweep_lu.get)
        Dc.copy_(D)
        ff.lu_nopiv_factor(Dc.t(), s_lu, info=info)
        torch.cuda.synchronize()
        dt = sweep_lu[s_lu]
        LU = Dc.t()
        Lm = torch.tril(LU, -1) + torch.eye(n, dtype=torch.float64, device=dev)
        Um = torch.triu(LU)
        bwd = float(torch.linalg.norm(D.t() - Lm @ Um) / torch.linalg.norm(D))
        out["lu_nopiv_f64_n16384"] = {"s": s_lu, "ms": round(dt * 1e3, 3),
                                      "tflops": round(2 * n ** 3 / 3 / dt / 1e12, 3),
                                      "info": int(info.item()), "bwd_A": bwd,
                                      "s_sweep_ms": {str(k): round(v * 1e3, 3) for k, v in sweep_lu.items()}}
        log(f"[bench] LU: {out['lu_nopiv_f64_n16384']}")
        del LU, Lm, Um
        # Strassen on the LU product: one level per super-tile, and two levels
        # (a matrix-level level over it), against the classical update
        lu_str = {}
        for levels in (1, 2):
            for s_lu in (512, 768):
                wsp = torch.empty(max(1, ff.load().ff_lu_workspace_size(n, s_lu, 0, 1 if levels == 1 else 32)),
                                  dtype=torch.uint8, device=dev)
                Dc.copy_(D)
                ff.lu_nopiv_factor(Dc.t(), s_lu, info=info, strassen=levels, ws=wsp)      # warm-up
                best_s = 1e30
                for _ in range(3):
                    Dc.copy_(D)
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    ff.lu_nopiv_factor(Dc.t(), s_lu, info=info, strassen=levels, ws=wsp)
                    torch.cuda.synchronize()
                    best_s = min(best_s, time.perf_counter() - t0)
                LU = Dc.t()
                bwd_s = float(torch.linalg.norm(D.t() - (torch.tril(LU, -1) + torch.eye(n, dtype=torch.float64,
                                                                                             device=dev))
                                                @ torch.triu(LU)) / torch.linalg.norm(D))
                lu_str[f"s{s_lu}_strassen{levels}"] = {"ms": round(best_s * 1e3, 3), "bwd_A": bwd_s,
                                                        "classical_ms": round(sweep_lu[s_lu] * 1e3, 3),
                                                        "info": int(info.item())}
                del wsp, LU
        out["lu_strassen_vs_classical"] = lu_str
        log(f"[bench] LU strassen: {lu_str}")
        del D, Dc
    except Exception as e:
        out["lu_nopiv_f64_n16384"] = {"error": str(e)}
    torch.cuda.empty_cache()

    # --- binary32 / bfloat16-operand factorisations on their own, with their update kernels
    try:
        out["low_precision_factor_n16384"] = run_low_precision_factor(ff, torch, dev, n, A0)
        log(f"[bench] low-precision factors: {out['low_precision_factor_n16384']}")
    except Exception as e:
        out["low_precision_factor_n16384"] = {"error": str(e)}
    torch.cuda.empty_cache()

    # --- triangular solves with a factor (forward + backward), per call
    try:
        out["trisolve_n16384"] = run_trisolve(ff, torch, dev, n)
        log(f"[bench] trisolve: {out['trisolve_n16384']}")
    except Exception as e:
        out["trisolve_n16384"] = {"error": str(e)}
    torch.cuda.empty_cache()

    # --- QR (Algorithm 3)
    try:
        out["qr_f64_n16384"] = run_qr(ff, torch, wl, dev, n=n)
        log(f"[bench] QR: {out['qr_f64_n16384']}")
    except Exception as e:
        out["qr_f64_n16384"] = {"error": str(e)}
    torch.cuda.empty_cache()

    # --- serving: continuous batching of many independent solves
    try:
        out["serving"] = run_serving(ff, torch, wl, dev)
    except Exception as e:
        out["serving"] = {"error": str(e)}
    torch.cuda.empty_cache()
    return out


def run_serving(ff, torch, wl, dev, nreq=10000, seed=0, window=128, rhos=(0.5, 0.8, 0.95), arena_gb=200,
                modes=("f64", "f32"), seq_requests=2000):
    """Continuous batching of many independent SPD solves (the serving workload):
    nreq requests, n = round(exp(U(ln 256, ln 8192))), nrhs ~ U{1..8}; with
    probability 0.3 a request repeats the matrix (and key) of one of the last 64
    distinct ones, served from its resident factor.  Every distinct matrix is
    A = G G^T / n + I from its own seed (10^6 + its index), generated just before
    its first submission on a producer stream, up to 8 requests ahead (the
    product in bfloat16 GEMM, rounded, then scaled and shifted in binary64 and
    mirrored; SPD since the rounding moves eigenvalues by about 2e-3 and
    lambda_min >= 1); its GPU time is reported separately.  A request is
    submitted, and its arrival stamped, once its A is resident.
    Per precision mode (binary64; binary32 factors with binary64 refinement): a
    closed loop (window of outstanding requests) gives the saturation rate X_max,
    open loops with exponential arrivals at rho * X_max give latency percentiles
    (device time from the submit stamp to the end of the solve, plus any lateness
    of the host loop behind the nominal arrival).  HBM budget: a 200 GB arena."""
    import collections
    import math
    import numpy as np
    rng = np.random.default_rng(seed)
    reqs, distinct = [], []
    for i in range(nreq):
        if distinct and rng.uniform() < 0.3:
            key, j, n = distinct[int(rng.integers(max(0, len(distinct) - 64), len(distinct)))]
        else:
            j = len(distinct)
            n = int(round(math.exp(rng.uniform(math.log(256), math.log(8192)))))
            key = j + 1
            distinct.append((key, j, n))
        reqs.append((key, j, n, int(rng.integers(1, 9))))
    prod = torch.cuda.Stream(device=dev)
    gen = {"matrices": 0, "gpu_ms": 0.0}
    cache = collections.OrderedDict()        # the last 64 distinct matrices (repeats only reach those)
    pending = collections.OrderedDict()      # matrices being generated: j -> (A, start, end event)
    LOOKAHEAD = 8

    def enqueue(j, n):
        # generate the matrix of distinct index j on the producer stream (no host wait)
        if j in cache or j in pending:
            return
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        with torch.cuda.stream(prod):
            e0.record(prod)
            g = torch.Generator(device=dev)
            g.manual_seed(10 ** 6 + j)
            G = torch.randn(n, n, dtype=torch.bfloat16, device=dev, generator=g)
            A = torch.mm(G, G.t().contiguous()).to(torch.float64)
            del G
            A.div_(float(n))
            A.diagonal().add_(1.0)
            A = torch.tril(A) + torch.tril(A, -1).t()
            e1.record(prod)
        pending[j] = (A, e0, e1)

    def matrix(j, n):
        A = cache.get(j)
        if A is not None:
            return A
        enqueue(j, n)
        A, e0, e1 = pending.pop(j)
        e1.synchronize()                 # resident before its request arrives
        gen["matrices"] += 1
        gen["gpu_ms"] += e0.elapsed_time(e1)
        cache[j] = A
        if len(cache) > 64:
            cache.popitem(last=False)
        return A

    def prefetch(rq, start):
        for key, j, n, nrhs in rq[start:start + LOOKAHEAD]:
            enqueue(j, n)

    def run(mode, rq, arrivals=None):
        arena = torch.empty(int(arena_gb * 1e9) // 8, dtype=torch.float64, device=dev)
        srv = ff.Server(arena, dtype=mode)
        flops = 0.0
        lat, hits, iters, conv, sizes = [], 0, [], 0, {}
        nominal = {}
        g0 = gen["gpu_ms"]
        t0 = time.perf_counter()
        nxt, done = 0, 0
        last_done, last_t, last_log = 0, 0.0, 0.0
        while done < len(rq):
            now = time.perf_counter() - t0
            if done != last_done:
                last_done, last_t = done, now
            elif now - last_t > 60.0 and nxt > done:
                raise RuntimeError(f"serving made no progress for 60 s ({done}/{len(rq)} done)")
            if now - last_log > 10.0:
                log(f"[bench] serving {mode}: {done}/{len(rq)} done after {now:.1f} s")
                last_log = now
            while nxt < len(rq) and (nxt - done) < window and (arrivals is None or arrivals[nxt] <= now):
                key, j, n, nrhs = rq[nxt]
                A = matrix(j, n).t()
                prefetch(rq, nxt + 1)
                B = torch.randn(nrhs, n, dtype=torch.float64, device=dev).t()
                X = torch.empty_like(B)
                rid = srv.submit(A, B, X, key=key)
                t_sub = time.perf_counter() - t0
                nominal[rid] = (t_sub - arrivals[nxt]) * 1e3 if arrivals is not None else 0.0
                sizes[rid] = n
                nxt += 1
            srv.step()
            for r in srv.poll():
                done += 1
                hits += r["cache_hit"]
                iters.append(r["iters"])
                conv += r["converged"]
                if r["info"] != 0:
                    raise RuntimeError(f"serving request failed: info={r['info']}")
                if not r["cache_hit"]:
                    flops += sizes[r["id"]] ** 3 / 3.0
                lat.append(r["latency_ms"] + nominal[r["id"]])
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        st = srv.stats()
        srv.close()
        del arena
        torch.cuda.empty_cache()
        lat = np.array(lat)
        out = {"requests": len(rq), "wall_s": round(wall, 3), "solves_per_s": round(len(rq) / wall, 1),
               "p50_ms": round(float(np.percentile(lat, 50)), 3), "p99_ms": round(float(np.percentile(lat, 99)), 3),
               "cache_hit_rate": round(hits / len(rq), 3), "factor_tflops": round(flops / wall / 1e12, 3),
               "generation_gpu_ms_in_run": round(gen["gpu_ms"] - g0, 1),
               "steps": st["steps"], "grouped_launches": st["grouped_launches"], "evictions": st["evictions"]}
        if mode != "f64":
            out["mean_refinement_iters"] = round(float(np.mean(iters)), 2)
            out["converged_fraction"] = round(conv / len(rq), 4)
        return out

    def sequential(rq):
        # the same requests one at a time through chol_factor + chol_trisolve
        # (binary64, resident factors reused for repeats)
        facs = {}
        for key, j, n, nrhs in rq:
            if key not in facs:
                matrix(j, n)                 # generated before the clock starts
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for key, j, n, nrhs in rq:
            if key not in facs:
                L = matrix(j, n).t().clone(memory_format=torch.preserve_format)
                ff.chol_factor(L, min(n, 192))
                facs[key] = L
                if len(facs) > 64:
                    facs.pop(next(iter(facs)))
            X = torch.randn(nrhs, n, dtype=torch.float64, device=dev).t()
            ff.chol_trisolve(facs[key], X)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        del facs
        torch.cuda.empty_cache()
        return {"requests": len(rq), "wall_s": round(wall, 3), "solves_per_s": round(len(rq) / wall, 1)}

    log(f"[bench] serving: {nreq} requests, {len(distinct)} distinct matrices")
    res = {"workload": f"{nreq} requests, n log-uniform [256, 8192], nrhs U{{1..8}}, 30% repeats of the last 64 "
                       f"distinct matrices, per-request seeds (A = G G^T/n + I generated on a producer stream), "
                       f"arena {arena_gb} GB, window {window} in closed loop"}
    for mode in modes:
        run(mode, reqs[:200])                                 # warm-up (kernels, allocator)
        closed = run(mode, reqs)
        log(f"[bench] serving {mode} closed loop: {closed}")
        xmax = closed["solves_per_s"]
        entry = {"closed_loop": closed}
        for rho in rhos:
            arr = np.cumsum(np.random.default_rng(seed + 1).exponential(1.0 / (rho * xmax), size=len(reqs)))
            entry[f"open_loop_rho{rho}"] = run(mode, reqs, arr)
            log(f"[bench] serving {mode} rho={rho}: {entry[f'open_loop_rho{rho}']}")
        res[mode] = entry
    if seq_requests:
        res["one_at_a_time_f64"] = sequential(reqs[:seq_requests])
        log(f"[bench] one request at a time: {res['one_at_a_time_f64']}")
    res["generation"] = {"matrices": gen["matrices"], "gpu_ms": round(gen["gpu_ms"], 1),
                         "note": "producer stream, bfloat16 GEMM, up to 8 requests ahead of submission; "
                                 "runs beside the server (its interference is part of every rate), "
                                 "never inside a latency (arrival is stamped once A is resident)"}
    cache.clear()
    pending.clear()
    torch.cuda.empty_cache()
    return res


MIXED_STEP = {16384: {"f64": 768, "f32": 512, "bf16": 512}, 32768: {"f64": 768, "f32": 768, "bf16": 768}}


def median_time(fn, reps, torch):
    """Median wall time of reps calls of fn() (each bracketed by synchronisation),
    after one untimed call; returns (seconds, last result)."""
    import statistics
    res = fn()
    ts = []
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = fn()
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t0)
    return statistics.median(ts), res


def run_low_precision_factor(ff, torch, dev, n, A0, reps=3):
    """chol_factor with binary32 storage (binary32 and bfloat16-operand updates) on
    the benchmark matrix: median time, n^3/3 rate against each precision's MFMA
    peak, and the update kernels' own rate from the library's event timing."""
    res = {}
    A32 = A0.to(torch.float32)
    for dtype in ("f32", "bf16"):
        W = A32.clone()
        info = torch.zeros(1, dtype=torch.int32, device=dev)
        # step sweep (factor only, median of reps), then the detailed run at the best step
        sweep = {}
        for s_try in (256, 384, 512, 640, 768, 1024):
            def fac_try():
                W.copy_(A32)
                ff.chol_factor(W.t(), s_try, dtype=dtype, info=info)
            sweep[s_try] = median_time(fac_try, reps, torch)[0]
        s = min(sweep, key=sweep.get)

        def fac():
            W.copy_(A32)
            ff.chol_factor(W.t(), s, dtype=dtype, info=info)
            return None
        dt, _ = median_time(fac, reps, torch)
        # the copy of A into W is inside the timed call; time it alone and take it out
        dtc, _ = median_time(lambda: W.copy_(A32), reps, torch)
        dt = max(dt - dtc, 1e-9)
        W.copy_(A32)
        torch.cuda.synchronize()
        ff.update_profile_enable(True)
        ff.chol_factor(W.t(), s, dtype=dtype, info=info)
        torch.cuda.synchronize()
        ff.update_profile_enable(False)
        prof = ff.update_profile_read()[dtype]
        upd_ms = prof["total_ms"]
        upd_tf = prof["total_flops"] / max(upd_ms, 1e-9) / 1e9
        peak = MI355X_PEAK_TFLOPS[dtype]
        entry = {"s": s, "s_sweep_ms_incl_copy": {str(k): round(v * 1e3, 3) for k, v in sweep.items()},
                 "ms": round(dt * 1e3, 3), "tflops": round(n ** 3 / 3 / dt / 1e12, 3),
                 "frac_of_peak": round(n ** 3 / 3 / dt / 1e12 / peak, 4), "info": int(info.item()),
                 "update_kernels": {"launches": prof["launches"], "total_ms": round(upd_ms, 3),
                                    "tflops": round(upd_tf, 3), "frac_of_mfma_peak": round(upd_tf / peak, 4),
                                    "algorithmic_GBps": round(prof["total_bytes"] / max(upd_ms, 1e-9) / 1e6, 1),
                                    "frac_of_hbm": round(prof["total_bytes"] / max(upd_ms, 1e-9) / 1e6
                                                         / MI355X_HBM_GBS, 4),
                                    "share_of_factor": round(upd_ms / (dt * 1e3), 3)}}
        res[dtype] = entry
        del W
    del A32
    return res


def run_qr(ff, torch, wl, dev, n=16384, steps=(64, 96, 112, 128, 142), reps=3, paper_sizes=((2000, 100), (4000, 200))):
    """qr_factor (Algorithm 3) on the benchmark family A = G G^T / n + I: median
    time per step, the rate at the conventional 4n^3/3 and at the algorithm's own
    count (projections 2 n^3, R = Q^T A's upper triangle n^2 (n + 1)), and
    orthogonality / residual by torch's binary64 GEMMs; the paper's two sizes
    (n = 2000, s = 100; n = 4000, s = 200, the block capped at ff.qr_step) for
    context."""
    res = {}
    A = wl.spd_scaled_device(n, seed=0, lam=1.0, device=dev).t()     # symmetric
    Q = ff.colmajor_empty(n, n, torch.float64, dev)
    R = ff.colmajor_empty(n, n, torch.float64, dev)
    info = torch.zeros(1, dtype=torch.int32, device=dev)
    sweep = {}
    for s in steps:
        ws = torch.empty(max(1, ff.qr_workspace_size(n, n, s)), dtype=torch.uint8, device=dev)

        def call():
            ff.qr_factor(A, s, Q=Q, R=R, ws=ws, info=info)
        dt, _ = median_time(call, reps, torch)
        sweep[s] = (dt, ff.qr_step(n, n, s), int(info.item()))
        log(f"[bench] qr n={n} s={s}: {dt * 1e3:.2f} ms")
        del ws
    s_best = min(sweep, key=lambda k: sweep[k][0])
    dt, blk, inf = sweep[s_best]
    ws = torch.empty(max(1, ff.qr_workspace_size(n, n, s_best)), dtype=torch.uint8, device=dev)
    ff.qr_factor(A, s_best, Q=Q, R=R, ws=ws, info=info)
    torch.cuda.synchronize()
    QtQ = torch.mm(Q.t(), Q)
    QtQ.diagonal().sub_(1.0)
    orth = float(QtQ.abs().max())
    del QtQ
    resid = float((torch.mm(Q, R) - A).abs().max() / A.abs().max())
    alg = 2.0 * n ** 3 + n * n * (n + 1.0)
    res[f"n{n}"] = {"s": s_best, "block": blk, "ms": round(dt * 1e3, 3), "info": inf,
                    "tflops_4n3_3": round(4 * n ** 3 / 3 / dt / 1e12, 3),
                    "tflops_algorithmic": round(alg / dt / 1e12, 3),
                    "frac_of_fp64_mfma_peak": round(alg / dt / 1e12 / MI355X_PEAK_TFLOPS["f64"], 4),
                    "orth_max": orth, "resid_max_rel": resid,
                    "s_sweep_ms": {str(k): round(v[0] * 1e3, 3) for k, v in sweep.items()}}
    del A, Q, R, ws
    torch.cuda.empty_cache()
    for m, s in paper_sizes:
        A = wl.spd_scaled_device(m, seed=1, lam=1.0, device=dev).t()
        Q = ff.colmajor_empty(m, m, torch.float64, dev)
        R = ff.colmajor_empty(m, m, torch.float64, dev)
        ws = torch.empty(max(1, ff.qr_workspace_size(m, m, s)), dtype=torch.uint8, device=dev)

        def call():
            ff.qr_factor(A, s, Q=Q, R=R, ws=ws, info=info)
        dt, _ = median_time(call, max(reps, 5), torch)
        res[f"n{m}_s{s}"] = {"block": ff.qr_step(m, m, s), "ms": round(dt * 1e3, 3), "info": int(info.item()),
                             "tflops_4n3_3": round(4 * m ** 3 / 3 / dt / 1e12, 3)}
        log(f"[bench] qr n={m} s={s}: {dt * 1e3:.2f} ms")
        del A, Q, R, ws
    return res


def run_solve_cell(ff, torch, wl, dev, n, lam=1e-6, reps=3):
    """One cell of the mixed-precision table, for profiling the solve path: binary64
    and binary32 + refinement (escalation allowed) at lambda = 1e-6 with 1 and 16
    right-hand sides, median of reps solves after one untimed solve."""
    A = wl.spd_scaled_device(n, seed=0, lam=lam, device=dev)          # symmetric
    res = {}
    for nrhs in (1, 16):
        B = wl.rhs_device(n, nrhs, seed=1000, device=dev).t()
        for dtype in ("f64", "f32"):
            s = MIXED_STEP.get(n, MIXED_STEP[16384])[dtype]
            W = ff.colmajor_empty(n, n, torch.float64 if dtype == "f64" else torch.float32, dev)
            ws = torch.empty(ff.solve_workspace_size(n, s, nrhs, dtype, escalate=dtype != "f64"), dtype=torch.uint8,
                             device=dev)
            X = ff.colmajor_empty(n, nrhs, torch.float64, dev)

            def solve():
                return ff.chol_solve(A.t(), B, s, dtype=dtype, W=W, X=X, ws=ws, tol=1e-12,
                                     max_iter=0 if dtype == "f64" else 50, escalate=dtype != "f64")[2]
            dt, info = median_time(solve, reps, torch)
            res[f"{dtype}_nrhs{nrhs}"] = {"ms": round(dt * 1e3, 3), "s": s, "iters": info["total_iters"],
                                          "info": info["info"], "backward_err": info["backward_err"]}
            del W, ws, X
    return res


def run_trisolve(ff, torch, dev, n, reps=5):
    """chol_trisolve (forward + backward sweep, including the per-factor inverse
    blocks) on a well-conditioned factor: median ms per call and the rate against
    the bytes of tril(L) read twice."""
    g = torch.Generator(device=dev).manual_seed(7)
    L64 = torch.tril(torch.randn(n, n, dtype=torch.float64, device=dev, generator=g) / n, -1)
    L64.diagonal().fill_(1.5)
    res = {}
    for dtype, st in (("f64", torch.float64), ("f32", torch.float32)):
        Lc = L64.t().contiguous().t().to(st)   # column-major storage of L
        ws = torch.zeros(ff.trisolve_workspace_size(n, dtype), dtype=torch.uint8, device=dev)
        for nrhs in (1, 4, 8, 16):
            B = torch.randn(nrhs, n, dtype=st, device=dev, generator=g).t()
            X = B.clone()

            def call():
                X.copy_(B)
                ff.chol_trisolve(Lc, X, dtype=dtype, ws=ws)
            dt, _ = median_time(call, reps, torch)
            err = int(ws[:4].view(torch.int32).item())
            gbytes = 2 * (n * (n + 1) / 2) * Lc.element_size() / 1e9
            res[f"{dtype}_nrhs{nrhs}"] = {"ms": round(dt * 1e3, 3), "GBps_tril_twice": round(gbytes / dt, 1),
                                          "frac_of_hbm": round(gbytes / dt / MI355X_HBM_GBS, 4), "error_word": err}
        del Lc, ws
    del L64
    return res


# (name, factor precision, GMRES-based refinement)
VARIANTS = (("f64", "f64", False), ("f32", "f32", False), ("bf16", "bf16", False),
            ("f32_gmres", "f32", True), ("bf16_gmres", "bf16", True))


def run_mixed_table(ff, torch, wl, dev, sizes=(16384, 32768), lams=(1.0, 1e-3, 1e-6), reps=3, oracle_refs=True,
                    oracle_L1=None):
    """Mixed-precision solves against the plain binary64 solve over the
    configuration's grid: n, lambda (A = G G^T / n + lambda I) and 1 or 16
    right-hand sides.  binary64: factor + one forward/backward solve.  binary32 and
    bfloat16: factor, refinement to ||dX|| <= 1e-12 ||X|| (or stagnation) with
    escalation to a higher precision when that fails; the *_gmres variants solve
    each correction equation by factor-preconditioned GMRES.  Every result's error is
    stated: backward error by torch's binary64 GEMM (independent of the library),
    forward error against the CPU oracle's solution at n = 16384 and against the
    binary64 GPU solve at larger n (labelled).  Accuracy criterion: backward error
    <= 1e-12 and, for lambda >= 1e-3 (where binary64 reaches the oracle to 1e-12),
    forward error <= 1e-12; a low-precision result beats binary64 when it meets
    the criterion in less time (median of reps)."""
    import numpy as np
    import oracle
    table = {}
    for n in sizes:
        for lam in lams:
            A = wl.spd_scaled_device(n, seed=0, lam=lam, device=dev)        # symmetric
            Ah = None
            Lo = oracle_L1 if (lam == 1.0 and n == 16384 and oracle_L1 is not None) else None
            if oracle_refs and n == 16384 and Lo is None:
                Ah = A.cpu().numpy()
                Lo, oinfo = oracle.chol(Ah)
                if oinfo != 0:
                    Lo = None
                del Ah
            anorm = float(A.abs().sum(dim=1).max())
            for nrhs in (1, 16):
                B = wl.rhs_device(n, nrhs, seed=1000, device=dev).t()       # n x nrhs column-major
                Xo = oracle.chol_solve(Lo, B.cpu().numpy()) if Lo is not None else None
                cell, xs = {}, {}
                for name, dtype, gm in VARIANTS:
                    s = MIXED_STEP.get(n, MIXED_STEP[16384])[dtype]
                    W = ff.colmajor_empty(n, n, torch.float64 if dtype == "f64" else torch.float32, dev)
                    ws = torch.empty(ff.solve_workspace_size(n, s, nrhs, dtype, escalate=dtype != "f64", gmres=gm),
                                     dtype=torch.uint8, device=dev)
                    X = ff.colmajor_empty(n, nrhs, torch.float64, dev)

                    def solve():
                        return ff.chol_solve(A.t(), B, s, dtype=dtype, W=W, X=X, ws=ws, tol=1e-12,
                                             max_iter=0 if dtype == "f64" else (20 if gm else 50),
                                             escalate=dtype != "f64", gmres=gm)[2]
                    dt, info = median_time(solve, reps, torch)
                    R = B - A @ X
                    bx = float((R.abs().amax(dim=0) / (anorm * X.abs().amax(dim=0) + B.abs().amax(dim=0))).max())
                    e = {"ms": round(dt * 1e3, 3), "s": s, "tflops_effective": round(n ** 3 / 3 / dt / 1e12, 3),
                         "dtype_used": ["f64", "f32", "bf16"][info["dtype_used"]], "escalations": info["escalations"],
                         "first_info": info["first_info"], "iters": info["total_iters"], "info": info["info"],
                         "bwd_x": bx}
                    if gm:
                        e["krylov_iters"] = info["krylov_iters"]
                    if Xo is not None:
                        e["fwd_x_vs_oracle"] = float(np.max(np.abs(X.cpu().numpy() - Xo)) / np.max(np.abs(Xo)))
                    xs[name] = X
                    cell[name] = e
                    del W, ws, R
                if Xo is None:
                    X64 = xs["f64"]
                    for name in cell:
                        cell[name]["fwd_x_vs_f64_gpu_solve"] = float((xs[name] - X64).abs().max() / X64.abs().max())
                fkey = "fwd_x_vs_oracle" if Xo is not None else "fwd_x_vs_f64_gpu_solve"
                for name, e in cell.items():
                    e["meets_1e-12"] = bool(e["info"] == 0 and e["bwd_x"] <= 1e-12
                                            and (lam < 1e-3 or e[fkey] <= 1e-12))
                    if name != "f64":
                        e["beats_f64"] = bool(e["meets_1e-12"] and e["ms"] < cell["f64"]["ms"])
                key = f"n{n}_lam{lam:g}_nrhs{nrhs}"
                table[key] = cell
                log(f"[bench] mixed {key}: " + ", ".join(
                    f"{d} {c['ms']} ms ({c['dtype_used']}, {c['iters']} it, bwd {c['bwd_x']:.1e}, "
                    f"fwd {c[fkey]:.1e}{', beats f64' if c.get('beats_f64') else ''})" for d, c in cell.items()))
                del xs, B, Xo
                torch.cuda.empty_cache()
            del A, Lo
            torch.cuda.empty_cache()
    table["criterion"] = ("backward error <= 1e-12 (torch binary64 GEMM) and, for lambda >= 1e-3, forward error "
                          "<= 1e-12 (vs the CPU oracle at n=16384, vs the binary64 GPU solve at n=32768); "
                          "times are medians of 3 solves (factor + solves + refinement)")
    return table


def cpu_baseline(A_host):
    """The oracle (textbook Cholesky, all host cores) on the benchmark matrix
    itself: one factorisation, timed.  Returns (record, L) -- L is reused as the
    reference solution's factor of the mixed-precision table."""
    import oracle
    n_cpu = A_host.shape[0]
    log(f"[bench] cpu oracle on the benchmark matrix, n={n_cpu}, {oracle.num_threads()} threads")
    t0 = time.perf_counter()
    L, info = oracle.chol(A_host)
    dt = time.perf_counter() - t0
    return ({"value": round(n_cpu ** 3 / 3 / dt / 1e12, 6), "unit": "TFLOP/s", "cores": oracle.num_threads(),
             "kind": "oracle", "sample": f"Cholesky of the timed matrix A=GG^T/n+I, n={n_cpu} (info={info}), "
                                         f"one run, {dt:.1f} s",
             "seconds": round(dt, 2)}, (L if info == 0 else None))


if __name__ == "__main__":
    main()
