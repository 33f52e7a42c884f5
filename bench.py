#!/usr/bin/env python3
"""Throughput of the entropic JKO hot path on one MI355X.

Workload (the 256x256 crowd-motion flow): 2D congestion energy
f = iota_[0,kappa] + <w, p> with 6 rectangular obstacles (kappa = 0 inside,
1.2/N outside), w = squared distance to the exit (0.9, 0.5), 8 Gaussian bumps
projected onto the capacity, gamma = 2e-4, tau = 2e-3; each JKO step iterates
until the marginal violation ||b * xi^T a - q||_1 <= 1e-6 (checked every 10
iterations, cap 2000).  A timed "step" is one JKO step of the flow; the flow
state carries over from step to step.

Prints ONE JSON line.  `value` is Sinkhorn iterations per second (iterations
whose result the step returns), with every input resident in HBM.  Extras:
JKO steps/s, the split-BF16 run, the 128^3 3D flow, the 512^2 porous-medium
flow (density-scaled), adjoint/forward time, and
the roofline of the dominant contraction kernel from HIP-event timings of its
launches on the library's stream.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import platform
import sys
import time

import numpy as np

PEAK_FP32_MFMA_TFLOPS = 157.3
PEAK_BF16_MFMA_TFLOPS = 2500.0
PEAK_HBM_GBPS = 8000.0


def _args():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--precision", default="fp32", choices=["fp32", "split_bf16"])
    ap.add_argument("--no-extra", action="store_true", help="skip the 3D, split and adjoint extras")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--pmc-probe", choices=["crowd256", "crowd128c", "porous512_scaled", "heat100"], default=None,
                    help="profiling probe: one fixed-count step of the workload, "
                         "then a 64 MiB device copy of known size (counter calibration)")
    ap.add_argument("--heat-leg", action="store_true",
                    help="run only the heat-kernel leg (heat100) and print its JSON record")
    ap.add_argument("--attraction-leg", action="store_true",
                    help="run only the attraction leg (crowd256_attraction, both precisions) and print its record")
    return ap.parse_args()


def _dev(a):
    import torch
    return None if a is None else torch.from_numpy(np.ascontiguousarray(np.asarray(a, np.float32))).cuda()


def _energy(wl):
    import paper_1502_06216_amd as jk
    return jk.EnergySpec(kind=wl.kind, w=_dev(wl.w), kappa=_dev(wl.kappa), kappa_scalar=wl.kappa_scalar,
                         coef=_dev(wl.coef), coef_scalar=wl.coef_scalar, m=wl.m,
                         density_scale=wl.density_scale, m_field=_dev(wl.m_field), target=_dev(wl.target))


def run_flow(wl, precision, steps, warmup, tol=None, max_iters=None, resident=True, **kw):
    """Run warmup + timed JKO steps of a workload; returns (iters, seconds, stats)."""
    import torch
    import paper_1502_06216_amd as jk
    en = _energy(wl)
    tol = wl.tol if tol is None else tol
    max_iters = wl.max_iters if max_iters is None else max_iters
    q = _dev(wl.p0)
    for _ in range(warmup):
        q, _ = jk.step(q, en, wl.gamma, wl.tau, max_iters=max_iters, tol=tol, check_every=wl.check_every,
                       precision=precision, resident=resident, **kw)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    iters = 0
    stats = []
    for _ in range(steps):
        q, st = jk.step(q, en, wl.gamma, wl.tau, max_iters=max_iters, tol=tol, check_every=wl.check_every,
                        precision=precision, resident=resident, **kw)
        iters += st["iters"]
        stats.append(st)
    torch.cuda.synchronize()
    return iters, time.perf_counter() - t0, stats, q


def band_halfwidth(n, gamma):
    """Largest |i - j| at which the float32 factor exp(-((i-j)/n)^2/gamma) is non-zero."""
    return min(int(math.floor(math.sqrt(152.0 * math.log(2.0) * gamma) * n)) + 1, n - 1)


def band32_sum(n, W):
    """Sum over the 32-wide output chunks of an axis of 32 x the length of
    the chunk's band of k, aligned to 32 (the k range the panel-form passes,
    the 3D plane pass and the axis-0 pass stage and multiply)."""
    tot = 0
    for i0 in range(0, n, 32):
        kb0 = max(0, i0 - W) & ~31
        kb1 = min(n, (i0 + 32 + W + 31) & ~31)
        tot += 32 * (kb1 - kb0)
    return tot


def fused_tile(n0, n1):
    """Output tile edge the library picks for a 2D grid: 16 while the grid
    has at most 256 such tiles, else 32."""
    return 16 if ((n0 + 15) // 16) * ((n1 + 15) // 16) <= 256 else 32


def fused2d_executed_flops(n0, n1, W0, W1, precision="fp32"):
    """MFMA flops one application of the 2D band kernel executes (FP32
    equivalent): per TT x TT tile, the first contraction over the halo rows
    and columns and the second over the halo rows, the halo extents padded
    to whole MFMA k-steps (16 for FP32, 32 for split-BF16)."""
    TT = fused_tile(n0, n1)
    rnd = 16 if precision == "fp32" else 32
    tot = 0
    for i0 in range(0, n0, TT):
        ib0 = max(0, i0 - W0) & ~3
        LIp = (min(n0, i0 + TT + W0) - ib0 + rnd - 1) // rnd * rnd
        for j0 in range(0, n1, TT):
            jb0 = max(0, j0 - W1) & ~3
            LJp = (min(n1, j0 + TT + W1) - jb0 + rnd - 1) // rnd * rnd
            tot += 2 * LIp * TT * LJp + 2 * TT * TT * LIp
    return tot


CSRC = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_1502_06216_amd", "csrc")
PROFILES = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles")
# counter summaries of the dominant launch per (workload, precision)
TRAFFIC_PROFILES = {("crowd256", "fp32"): "resident2d_congestion_crowd256_traffic.md",
                    ("crowd128c", "fp32"): "plane_pass_crowd128c_traffic.md",
                    ("porous512_scaled", "fp32"): "resident_pass_porous512_traffic.md"}


def resident_pass_shape(shape):
    """True when a 2D step of this shape runs on the resident pass kernel
    rather than the resident tile kernel (the library's rule for the bench's
    workloads: more than 256 tiles of 16 x 16, axes of a multiple of 32)."""
    n0, n1 = shape
    return -(-n0 // 16) * -(-n1 // 16) > 256 and n0 % 32 == 0 and n1 % 32 == 0


def kernel_source_hash(kernel_file):
    """sha256 of the sources one kernel is compiled from (its file and every
    header of the library it includes, directly or not); a stored counter
    reading is valid only for the sources it was taken on."""
    import hashlib
    import re
    files = []

    def visit(f):
        if f in files or not os.path.exists(os.path.join(CSRC, f)):
            return
        files.append(f)
        with open(os.path.join(CSRC, f)) as fh:
            for inc in re.findall(r'^#include "([^"]+)"', fh.read(), re.M):
                visit(inc)

    visit(kernel_file)
    h = hashlib.sha256()
    for f in sorted(files):
        with open(os.path.join(CSRC, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def stored_traffic(profile_name, kernel_file, launch):
    """Calibrated HBM bytes per dispatch from a committed counter summary
    (FETCH_SIZE and WRITE_SIZE passes), or None when the summary is missing,
    covers another launch, or the kernel's sources changed since it was
    taken."""
    import re
    path = os.path.join(PROFILES, profile_name)
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    m_h = re.search(r"^source_sha256:\s*([0-9a-f]{64})", txt, re.M)
    if not m_h or m_h.group(1) != kernel_source_hash(kernel_file):
        return None
    # one "launch:" line per measured launch, each followed by its figures
    for m in re.finditer(r"^launch:\s*(.+?)\s*$", txt, re.M):
        if m.group(1) != launch:
            continue
        m_b = re.compile(r"^traffic_bytes_per_dispatch:\s*([0-9.eE+]+)", re.M).search(txt, m.end())
        return float(m_b.group(1)) if m_b else None
    return None


def _field_bytes(wl):
    """Bytes per cell the prox epilogue reads for the energy's fields."""
    fields = 0
    if wl.kind == "congestion":
        fields += (wl.w is not None) + (wl.kappa is not None)
    elif wl.kind in ("entropy", "porous"):
        fields += wl.coef is not None
    return 4 * fields


def roofline(wl, precision, q, traffic_profile=None, resident=True):
    """Per-launch durations of the kernel launches of one iteration (HIP
    events on the library's stream) and the roofline of the slowest launch.

    Algorithmic work per launch:
      flops  the dense separable contraction, 2 n_k N per axis pass
             (2 (n0 + n1) N for a fused 2D application, 2 (n1 + n2) N for
             a 3D plane pass);
      bytes  each field read or written once: a pass without epilogue reads
             X and writes Y (8 B/cell); the b-update epilogue reads t's input,
             q and writes b (12 B/cell); the prox epilogue reads s's input and
             the energy's fields and writes a (8 B/cell + 4 per field).
    A resident 2D launch runs `wl.max_iters` iterations: twice the fused
    application's work per iteration, plus the b-update and prox bytes.
    The bound is the roof with the larger lower-bound time."""
    import paper_1502_06216_amd as jk
    en = _energy(wl)
    d = len(wl.shape)
    N = int(np.prod(wl.shape))
    fb = _field_bytes(wl)
    ms = jk.time_iteration(q, en, wl.gamma, wl.tau, precision=precision, reps=200, resident=False)
    if d == 2 and resident:
        msr = jk.time_iteration(q, en, wl.gamma, wl.tau, precision=precision, reps=5, iters=wl.max_iters)
        if len(msr) == 1:
            per_launch = ms
            ms = msr
    if len(ms) == 1:
        K = wl.max_iters
        flops = [K * 2 * 2.0 * (wl.shape[0] + wl.shape[1]) * N]
        nbytes = [K * (12.0 + 8.0 + fb) * N]
        W = [band_halfwidth(n, wl.gamma) for n in wl.shape]
        if resident_pass_shape(wl.shape):
            # four panel passes per iteration, each 32-wide output chunk over
            # its band of k rounded out to 32
            n0, n1 = wl.shape
            names = [f"resident pass kernel, {K} iterations"]
            kfile = "respass.hip"
            executed = [K * 2 * 2 * (n0 * band32_sum(n1, W[1]) + n1 * band32_sum(n0, W[0]))]
        else:
            names = [f"resident 2D kernel, {K} iterations"]
            kfile = "gibbs2d.hip"
            executed = [K * 2 * fused2d_executed_flops(wl.shape[0], wl.shape[1], W[0], W[1], precision)]
    elif len(ms) == 2 and d == 2:
        flops = [2.0 * (wl.shape[0] + wl.shape[1]) * N] * 2
        nbytes = [12.0 * N, (8.0 + fb) * N]
        names = ["fused 2D application, b-update epilogue", "fused 2D application, prox epilogue"]
        kfile = "gibbs2d.hip"
        W = [band_halfwidth(n, wl.gamma) for n in wl.shape]
        executed = [fused2d_executed_flops(wl.shape[0], wl.shape[1], W[0], W[1], precision)] * 2
    elif len(ms) == 4 and d == 3:
        # plane pass (axes 1 and 2, intermediate on chip), then the axis-0 pass with the epilogue
        fp, fs = 2.0 * (wl.shape[1] + wl.shape[2]) * N, 2.0 * wl.shape[0] * N
        flops = [fp, fs, fp, fs]
        nbytes = [8.0 * N, 12.0 * N, 8.0 * N, (8.0 + fb) * N]
        names = ["plane pass (axes 1, 2)", "axis-0 pass, b-update epilogue",
                 "plane pass (axes 1, 2)", "axis-0 pass, prox epilogue"]
        kfile = "contract.hip"
        n0, n1, n2 = wl.shape
        W = [band_halfwidth(n, wl.gamma) for n in wl.shape]
        ep = 2 * n0 * (n1 * band32_sum(n2, W[2]) + n2 * band32_sum(n1, W[1]))
        es = 2 * n1 * n2 * band32_sum(n0, W[0])
        executed = [ep, es, ep, es]
    else:
        order = list(range(d - 1, -1, -1)) * 2
        flops = [2.0 * wl.shape[ax] * N for ax in order]
        nbytes = [12.0 * N if i == d - 1 else (8.0 + fb) * N if i == 2 * d - 1 else 8.0 * N
                  for i in range(2 * d)]
        names = [f"axis-{ax} pass" + (", b-update epilogue" if i == d - 1 else ", prox epilogue" if i == 2 * d - 1 else "")
                 for i, ax in enumerate(order)]
        kfile = "contract.hip"
        # panel-form passes (axes of a multiple of 32) stage 32-aligned bands
        W = [band_halfwidth(n, wl.gamma) for n in wl.shape]
        executed = [2 * (N // wl.shape[ax]) * band32_sum(wl.shape[ax], W[ax]) if wl.shape[ax] % 32 == 0 else None
                    for ax in order]
    k = int(np.argmax(ms))
    sec = ms[k] * 1e-3
    peak_f = PEAK_FP32_MFMA_TFLOPS if precision == "fp32" else PEAK_BF16_MFMA_TFLOPS
    t_mfma = flops[k] / (peak_f * 1e12)
    t_hbm = nbytes[k] / (PEAK_HBM_GBPS * 1e9)
    mfma = {"achieved": round(flops[k] / sec / 1e12, 3), "peak": peak_f, "unit": "TFLOP/s",
            "frac": round(flops[k] / sec / 1e12 / peak_f, 4)}
    hbm = {"achieved": round(nbytes[k] / sec / 1e9, 1), "peak": PEAK_HBM_GBPS, "unit": "GB/s",
           "frac": round(nbytes[k] / sec / 1e9 / PEAK_HBM_GBPS, 4)}
    bound = "mfma" if t_mfma >= t_hbm else "hbm"
    main = mfma if bound == "mfma" else hbm
    traffic = stored_traffic(traffic_profile, kfile, names[k]) if traffic_profile else None
    out = {"bound": bound, **main, "traffic": traffic, "kernel": names[k],
           "flops_per_launch": flops[k], "algorithmic_bytes_per_launch": nbytes[k],
           "ms_per_launch": round(ms[k], 5), "ms_per_launch_all": [round(x, 5) for x in ms],
           "other_roof": hbm if bound == "mfma" else mfma}
    if executed is not None and executed[k] is not None:
        # executed MFMA work: the band-limited, tile-padded products the kernel
        # issues (split-BF16 issues three bfloat16 products per FP32 product)
        ex = executed[k] * (1 if precision == "fp32" else 3)
        out["executed_mfma_flops_per_launch"] = ex
        out["executed_mfma_frac"] = round(ex / sec / 1e12 / peak_f, 4)
    if len(ms) == 1:
        out["us_per_iteration"] = round(1e3 * ms[0] / wl.max_iters, 3)
        out["launch_per_application_ms"] = [round(x, 5) for x in per_launch]
    return out


def cpu_baseline(wl, seconds):
    """The FP64 oracle (numpy/BLAS, separable kernel) on the same workload:
    first JKO step, a fixed number of iterations sized to ~`seconds`."""
    import oracle as O
    en = O.Energy(kind=wl.kind, w=wl.w, kappa=wl.kappa, kappa_scalar=wl.kappa_scalar,
                  coef=wl.coef, coef_scalar=wl.coef_scalar, m=wl.m, density_scale=wl.density_scale)
    O.jko_step(wl.p0, en, wl.gamma, wl.tau, 5)   # warm-up (first-call costs)
    t0 = time.perf_counter()
    O.jko_step(wl.p0, en, wl.gamma, wl.tau, 30)
    per_it = (time.perf_counter() - t0) / 30
    n_it = int(max(10, min(50000, seconds / per_it)))
    t0 = time.perf_counter()
    O.jko_step(wl.p0, en, wl.gamma, wl.tau, n_it)
    el = time.perf_counter() - t0
    cores = len(os.sched_getaffinity(0))
    blas_desc = "unknown BLAS"
    try:   # threads the BLAS behind numpy actually runs
        from threadpoolctl import threadpool_info
        blas = [t for t in threadpool_info() if t.get("user_api") == "blas"]
        if blas:
            cores = min(cores, max(t["num_threads"] for t in blas))
            b = blas[0]
            blas_desc = f"{b.get('internal_api', '?')} {b.get('version', '?')} ({b.get('num_threads')} threads)"
    except Exception:
        pass
    return {
        "value": round(n_it / el, 3), "unit": "Sinkhorn iters/s", "cores": cores, "kind": "oracle",
        "cpu_model": _cpu_model(), "blas": blas_desc,
        "sample": f"FP64 oracle jko_step on {wl.name} {wl.shape} (separable numpy/BLAS kernel), "
                  f"first JKO step, {n_it} fixed iterations, {el:.1f} s",
    }


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or platform.machine()


def equal_accuracy_128(n_steps=20, iters=300, ref_iters=3000):
    """Split-BF16 against FP32 on the 128^3 crowd flow (20 JKO steps x 300
    iterations, absorption on max|log a| > 50) at equal final-density
    accuracy.  Accuracy is the rel-L1 distance of p_T to a reference flow
    whose steps run ten times longer (3000 iterations, FP32): at 300
    iterations each step is short of its limit by far more than either
    precision's rounding, so both precisions reach the same accuracy at the
    same iteration count, and the speedup at equal accuracy is the ratio of
    the flows' wall times."""
    import torch
    import paper_1502_06216_amd as jk
    from workloads import make_workload
    wl = make_workload("crowd128c")
    en = _energy(wl)
    p0 = _dev(wl.p0)

    def run(prec, k):
        jk.flow(p0, en, wl.gamma, wl.tau, 1, max_iters=10, precision=prec, with_stats=False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        pT, _, _ = jk.flow(p0, en, wl.gamma, wl.tau, n_steps, max_iters=k, precision=prec, with_stats=False,
                           absorb_threshold=50.0, absorb_on_a=True)
        torch.cuda.synchronize()
        return pT.double().cpu().numpy(), time.perf_counter() - t0

    ref, _ = run("fp32", ref_iters)
    out = {"flow": f"crowd128c {n_steps} JKO steps x {iters} iterations",
           "reference": f"the same flow at {ref_iters} iterations per step, FP32"}
    res = {}
    for prec in ("fp32", "split_bf16"):
        p, t = run(prec, iters)
        res[prec] = (p, t)
        out[prec] = {"rel_l1_to_reference": float(np.abs(p - ref).sum() / np.abs(ref).sum()), "flow_s": round(t, 4)}
    f, sp = res["fp32"][0], res["split_bf16"][0]
    out["rel_l1_split_vs_fp32"] = float(np.abs(sp - f).sum() / np.abs(f).sum())
    acc = [out[p]["rel_l1_to_reference"] for p in ("fp32", "split_bf16")]
    out["accuracy_ratio_split_over_fp32"] = round(acc[1] / acc[0], 4)
    out["speedup_split_over_fp32"] = round(res["fp32"][1] / res["split_bf16"][1], 4)
    return out


def adjoint_ratio(precision="fp32"):
    """Forward flow (20 steps x 300 iterations, checkpoints kept) vs backward
    (recompute + reverse sweep) on the 256x256 crowd workload."""
    import torch
    import paper_1502_06216_amd as jk
    from workloads import make_workload
    wl = make_workload("crowd256_fixed")
    en = _energy(wl)
    p0 = _dev(wl.p0)
    jk.flow(p0, en, wl.gamma, wl.tau, 1, max_iters=10, checkpoints=True, with_stats=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pT, _, ck = jk.flow(p0, en, wl.gamma, wl.tau, wl.n_steps, max_iters=wl.max_iters, checkpoints=True,
                        with_stats=False, precision=precision)
    torch.cuda.synchronize()
    t_fwd = time.perf_counter() - t0
    g = torch.ones_like(pT)
    t0 = time.perf_counter()
    jk.backward(ck, [wl.max_iters] * wl.n_steps, g, en, wl.gamma, wl.tau, precision=precision)
    torch.cuda.synchronize()
    t_bwd = time.perf_counter() - t0
    return {"forward_s": round(t_fwd, 4), "backward_s": round(t_bwd, 4), "ratio": round(t_bwd / t_fwd, 3),
            "workload": "crowd256_fixed 20 steps x 300 iterations"}


def pmc_probe(name, precision):
    """A fixed-count step of `name` (the workload's cap in 2D, where it is one
    resident launch; 50 iterations in 3D) followed by a plain 64 MiB device
    copy, for hardware-counter passes (FETCH_SIZE / WRITE_SIZE per dispatch).
    The copy's source is evicted from the caches first (a 512 MiB fill runs
    between writing it and copying it), so its counters read the copy's
    known byte counts and calibrate the ones of the step's kernels."""
    import torch
    import paper_1502_06216_amd as jk
    from workloads import make_workload
    wl = make_workload(name)
    en = _energy(wl)
    q = _dev(wl.p0)
    if name == "heat100":
        # the operator build, then 30 iterations (60 operator passes)
        import numpy as np
        mask = torch.from_numpy(np.ascontiguousarray(wl.mask.astype(np.uint8))).cuda()
        op = jk.HeatOperator(wl.shape, wl.gamma, wl.heat_L, mask=mask)
        iters = 30
        p, st = op.step(q, en, wl.tau, max_iters=iters)
    else:
        iters = wl.max_iters if len(wl.shape) == 2 else 50
        p, st = jk.step(q, en, wl.gamma, wl.tau, max_iters=iters, tol=0.0, precision=precision)
    torch.cuda.synchronize()
    src = torch.ones(16 * 1024 * 1024, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    evict = torch.empty(128 * 1024 * 1024, dtype=torch.float32, device="cuda")
    evict.fill_(2.0)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"probe": name, "iterations": iters, "precision": precision,
                      "copy_bytes_read": src.numel() * 4, "copy_bytes_written": dst.numel() * 4}), flush=True)


def heat_pass_traffic():
    """Calibrated HBM bytes of one operator pass (tile pass plus b-update
    finish) from the
    committed counter summary, or None when it is missing or the heat
    kernels' sources changed since it was taken."""
    import re
    path = os.path.join(PROFILES, "heat_pass_heat100.md")
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    m_h = re.search(r"^source_sha256:\s*([0-9a-f]{64})", txt, re.M)
    m_t = re.search(r"^traffic_bytes_per_pass:\s*([0-9]+)", txt, re.M)
    if not m_h or not m_t or m_h.group(1) != kernel_source_hash("heat.hip"):
        return None
    return int(m_t.group(1))


def heat_bench(wl):
    """The heat-kernel Gibbs operator on an obstacle room (Section 4.1):
    operator build time, then n_steps timed JKO steps (one warm-up step
    first).  Each iteration is two passes over the stored operator; the
    algorithmic bytes of a pass are its packed upper-triangular 128 x 128
    float32 tiles over the free cells, the tile partial sums written and
    read back, and three float32 fields of the epilogue per free cell."""
    import numpy as np
    import torch
    import paper_1502_06216_amd as jk
    mask = torch.from_numpy(np.ascontiguousarray(wl.mask.astype(np.uint8))).cuda()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    op = jk.HeatOperator(wl.shape, wl.gamma, wl.heat_L, mask=mask)
    torch.cuda.synchronize()
    build = time.perf_counter() - t0
    en = _energy(wl)
    q = _dev(wl.p0)
    op.flow(q, en, wl.tau, 1, max_iters=wl.max_iters)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, sts = op.flow(q, en, wl.tau, wl.n_steps, max_iters=wl.max_iters)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    iters = sum(s["iters"] for s in sts)
    nf = int(wl.mask.sum())
    nT = (nf + 127) // 128
    per_pass = nT * (nT + 1) // 2 * 128 * 128 * 4 + 2 * nT * nT * 128 * 4 + 3 * nf * 4
    achieved = 2 * per_pass * iters / el / 1e9
    return {"iters_per_s": round(iters / el, 2), "jko_steps_per_s": round(wl.n_steps / el, 3),
            "iters_per_step": wl.max_iters, "operator_build_s": round(build, 3),
            "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": 8000.0, "unit": "GB/s",
                         "frac": round(achieved / 8000.0, 4), "traffic": heat_pass_traffic(),
                         "algorithmic_bytes_per_pass": per_pass,
                         "note": "whole-step rate over the timed steps (two operator passes per iteration); "
                                 "memory-side bandwidth: the packed operator (187 MB) stays resident in the "
                                 "256 MB last-level cache between passes, so this is not an HBM fraction"}}


def heat_solve_bench(wl, steps=1, iters=100):
    """The heat-kernel operator applied the paper's way (L implicit solves
    per product, FP64 Chebyshev stencil sweeps) on a room beyond the stored
    operator's 2^16 cells.  Algorithmic bytes of one Chebyshev step: D, X, R
    read and X, R and the next D written once per cell (48 B; D's neighbours
    come from cache), of the start of a solve 24 B; a product is L starts
    and L K steps."""
    import numpy as np
    import torch
    import paper_1502_06216_amd as jk
    mask = torch.from_numpy(np.ascontiguousarray(wl.mask.astype(np.uint8))).cuda()
    op = jk.HeatOperator(wl.shape, wl.gamma, wl.heat_L, mask=mask)
    en = _energy(wl)
    q = _dev(wl.p0)
    op.flow(q, en, wl.tau, 1, max_iters=5)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, sts = op.flow(q, en, wl.tau, steps, max_iters=iters)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    it = sum(s["iters"] for s in sts)
    N = int(np.prod(wl.shape))
    nu = [wl.gamma * n * n / wl.heat_L for n in wl.shape]
    beta = 1.0 + 4.0 * sum(nu)
    c = (math.sqrt(beta) - 1.0) / (math.sqrt(beta) + 1.0)
    K = math.ceil(math.log(0.5e-13) / math.log(c))
    per_product = wl.heat_L * (24 + 48 * K) * N
    achieved = 2 * per_product * it / el / 1e9
    return {"iters_per_s": round(it / el, 2), "grid": list(wl.shape), "free_cells": int(wl.mask.sum()),
            "chebyshev_steps_per_solve": K,
            "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": 8000.0, "unit": "GB/s",
                         "frac": round(achieved / 8000.0, 4), "traffic": None,
                         "algorithmic_bytes_per_product": per_product,
                         "note": "whole-step rate on the per-sweep algorithmic bytes; the solves run "
                                 "eight sweeps per launch on tiles with an eight-cell halo"}}


def attraction_bench(wl, precision):
    """The Wasserstein attraction with congestion (Section 5.2) on its two
    stacked couplings: a 2D grid whose band is too wide for the fused kernel
    runs four rotating passes per iteration (t = xi^T a for both couplings,
    axis 1 then axis 0 with the b-update epilogue; s = xi b likewise, the
    last pass with the paired proximal epilogue).  The roofline is the
    whole-iteration rate against FP32 (or BF16) MFMA peak, on the dense
    per-axis flops (2 couplings x N cells x n per pass, two flops each) and
    on the flops the panel form executes (each 32-wide output chunk
    multiplies its band of k rounded out to 32)."""
    it, el, st, _ = run_flow(wl, precision, wl.n_steps, 1)
    n0, n1 = wl.shape
    N = n0 * n1
    dense = 2 * 2 * 2 * N * (n0 + n1)            # 2 applications x (axis 1 + axis 0), 2 couplings
    W0, W1 = band_halfwidth(n0, wl.gamma), band_halfwidth(n1, wl.gamma)
    executed = 2 * 2 * 2 * (n0 * band32_sum(n1, W1) + n1 * band32_sum(n0, W0))
    peak = 157.3 if precision == "fp32" else 2500.0
    rate = it / el
    achieved = dense * rate / 1e12
    return {"iters_per_s": round(rate, 2), "jko_steps_per_s": round(wl.n_steps / el, 3),
            "iters_per_step": wl.max_iters, "band": [W0, W1],
            "roofline": {"bound": "mfma", "achieved": round(achieved, 3), "peak": peak, "unit": "TFLOP/s",
                         "frac": round(achieved / peak, 4), "traffic": None,
                         "flops_per_iteration": dense, "executed_mfma_flops_per_iteration": executed,
                         "executed_mfma_frac": round(executed * rate / 1e12 / peak * (3 if precision != "fp32"
                                                                                        else 1), 4),
                         "note": "whole-iteration rate over four latency-bound passes of 128 blocks per "
                                 "iteration (split-BF16: three bf16 products per executed flop)"}}


def main():
    args = _args()
    if args.pmc_probe:
        pmc_probe(args.pmc_probe, args.precision)
        return
    if args.heat_leg:
        import paper_1502_06216_amd as jk
        from workloads import make_workload
        jk.load()
        print(json.dumps({"heat100_fp32": heat_bench(make_workload("heat100"))}), flush=True)
        return
    if args.attraction_leg:
        import paper_1502_06216_amd as jk
        from workloads import make_workload
        jk.load()
        wla = make_workload("crowd256_attraction")
        print(json.dumps({f"crowd256_attraction_{p}": attraction_bench(wla, p) for p in ("fp32", "split_bf16")}),
              flush=True)
        return
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (asked for --gpus {args.gpus}); "
              "a flow would shard by slabs along axis 0, which is not built", file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_1502_06216_amd as jk
    from workloads import make_workload
    jk.load()
    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(1)

    wl = make_workload("crowd256")
    iters, el, stats, q = run_flow(wl, args.precision, args.steps, args.warmup)
    value = iters / el
    line = {
        "metric": "Sinkhorn iters/s + JKO steps/s at 256^2 and 128^3, FP32 vs split-BF16; adjoint time",
        "value": round(value, 2),
        "unit": "Sinkhorn iters/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(1e3 * el / args.steps, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32" if args.precision == "fp32" else "bf16x3",
        "data": "synthetic",
        "config": {
            "workload": "crowd256: 2D crowd motion 256x256, 6 obstacles, 8 bumps (projected onto kappa), "
                        "gamma=2e-4, tau=2e-3, tol 1e-6 L1 (check every 10, cap 2000)",
            "grid": list(wl.shape), "gamma": wl.gamma, "tau": wl.tau, "tol": wl.tol,
            "cap": wl.max_iters, "check_every": wl.check_every, "precision": args.precision,
        },
        "jko_steps_per_s": round(args.steps / el, 3),
        "iters_per_step": [s["iters"] for s in stats],
        "marginal_l1": [s["marginal_l1"] for s in stats],
    }
    line["roofline"] = roofline(wl, args.precision, q, TRAFFIC_PROFILES.get(("crowd256", args.precision)))
    extra = {}
    if not args.no_extra:
        other = "split_bf16" if args.precision == "fp32" else "fp32"
        it2, el2, st2, _ = run_flow(wl, other, args.steps, args.warmup)
        extra[f"crowd256_{other}"] = {"iters_per_s": round(it2 / el2, 2), "jko_steps_per_s": round(args.steps / el2, 3),
                                      "iters_per_step": [s["iters"] for s in st2]}
        if args.precision == "fp32":
            it4, el4, st4, _ = run_flow(wl, "fp32", args.steps, args.warmup, resident=False)
            extra["crowd256_fp32_launch_per_application"] = {
                "iters_per_s": round(it4 / el4, 2), "jko_steps_per_s": round(args.steps / el4, 3),
                "iters_per_step": [s["iters"] for s in st4]}
        # the 128^3 crowd as its precision configuration states it: absorption
        # when max|log a| exceeds 50 (JKO_FLAG_ABSORB_ON_A; max|log a| stays
        # near 5 here, so the step stays in the plain domain), checks every 10
        wl3 = make_workload("crowd128c")
        for prec in ("fp32", "split_bf16"):
            it3, el3, st3, q3 = run_flow(wl3, prec, 2, 1, tol=0.0, max_iters=300, absorb_threshold=50.0,
                                         absorb_on_a=True)
            extra[f"crowd128c_{prec}"] = {"iters_per_s": round(it3 / el3, 2), "jko_steps_per_s": round(2 / el3, 3),
                                         "iters_per_step": 300, "absorb_threshold": 50.0, "absorb_on": "max|log a|",
                                         "absorptions": [s["absorptions"] for s in st3],
                                         "max_abs_log_a": [round(s["max_abs_log_a"], 3) for s in st3],
                                         "roofline": roofline(wl3, prec, q3, TRAFFIC_PROFILES.get(("crowd128c", prec)))}
        extra["crowd128c_equal_accuracy"] = equal_accuracy_128()
        # the non-convex binary constraint {0, kappa} on the same crowd
        # (300 iterations per step: the non-convex iteration has no tolerance to reach)
        wlb = make_workload("crowd256_binary")
        for prec in ("fp32", "split_bf16"):
            itb, elb, stb, _ = run_flow(wlb, prec, wlb.n_steps, 1)
            extra[f"crowd256_binary_{prec}"] = {"iters_per_s": round(itb / elb, 2),
                                                "jko_steps_per_s": round(wlb.n_steps / elb, 3),
                                                "iters_per_step": wlb.max_iters}
        # Wasserstein attraction with congestion (two couplings, Section 5.2)
        wla = make_workload("crowd256_attraction")
        for prec in ("fp32", "split_bf16"):
            extra[f"crowd256_attraction_{prec}"] = attraction_bench(wla, prec)
        # generalised entropies with exponents varying from 1 to 2 over the grid
        wlg = make_workload("gen512")
        for prec in ("fp32", "split_bf16"):
            itg, elg, stg, qg = run_flow(wlg, prec, wlg.n_steps, 1)
            extra[f"gen512_{prec}"] = {"iters_per_s": round(itg / elg, 2),
                                       "jko_steps_per_s": round(wlg.n_steps / elg, 3),
                                       "iters_per_step": wlg.max_iters,
                                       "roofline": roofline(wlg, prec, qg)}
        wl5 = make_workload("porous512_scaled")
        for prec in ("fp32", "split_bf16"):
            it5, el5, st5, q5 = run_flow(wl5, prec, 3, 1)
            extra[f"porous512_scaled_{prec}"] = {"iters_per_s": round(it5 / el5, 2),
                                                 "jko_steps_per_s": round(3 / el5, 3),
                                                 "iters_per_step": [s["iters"] for s in st5],
                                                 "roofline": roofline(wl5, prec, q5,
                                                                      TRAFFIC_PROFILES.get(("porous512_scaled", prec)))}
        # heat-kernel Gibbs operator (L = 10 implicit steps) on a 100x100 room with obstacles
        extra["heat100_fp32"] = heat_bench(make_workload("heat100"))
        # beyond the stored operator: a 300 x 300 room by per-product solves
        from workloads import heat_room
        extra["heat300_per_product_fp32"] = heat_solve_bench(heat_room(300, 300, seed=0))
        extra["adjoint_fp32"] = adjoint_ratio("fp32")
    line["extra"] = extra
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(make_workload("crowd256"), args.cpu_seconds)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
