"""Benchmark of the GNA hot path on one MI355X.

A step is one evaluation of the whole chain -- P_ee, flux x cross section,
Gauss-Legendre bin integration, smearing, Poisson chi^2 and its 5-component
gradient -- for the batched scan: 4096 parameter points on a 64 x 64 grid in
(dm2_31, sin^2 th13), 240 bins x 5 Gauss-Legendre nodes (1200 points), one
52.5 km baseline, in FP64.  `value` is chi^2+gradient evaluations per second
(parameter points per second), inputs resident in HBM.  Tiles of 16 points
with common (dm2_21, dm2_31) -- every tile of this grid, whose fast axis is
sin^2 th13 -- evaluate their phases once (the library's default); the roofline
states the fraction of the ALU peak both for that executed work and for the
per-point count of a kernel that shares nothing.

The same JSON line also carries, measured in this run:
  * mixed: the same scan in mixed precision (FP64 phases, FP32 elsewhere);
  * per_point_phases: the grid with phase sharing switched off, FP64 and mixed;
  * random_batch: 4096 points that share nothing (every parameter drawn
    around the reference point), FP64 and mixed;
  * mixed_vs_fp64: per output (prediction, chi^2, gradient) for the grid
    scan, the random batch, the 1200-point and the 8-baseline single-point
    chains; the uneven batch's is under fitset, P_ee's under pee_sweep;
  * pee: elementwise P_ee over N = 1e8 energies (52.5 km) in FP64 and mixed,
    evaluations/s and HBM bandwidth against 8 TB/s;
  * pee_sweep: the same over N in {1e6, 1e7, 1e8} and L in {1, 52.5, 1300} km,
    with the mixed-vs-FP64 error per baseline;
  * chain_1pt / chain_8L / fitset: the single-point chain (1200 points), the
    single-point chain with 8 baselines and 100 800 points, and the uneven
    batch of 1024 fits (evaluations/s, FP64 and mixed; the fitset as the
    autotuned shape and as one persistent launch); the single-point chains
    also replayed from a captured HIP graph;
  * transfer_pipeline: P_ee over N = 1e8 energies in host memory, copies in
    and out serialized against the library's pipelined transfers;
  * graph: the transformation graph of the config-0 chain read back after a
    change of dm2_31 (full recompute) or of the normalisation only (lazy:
    two nodes), beside the fused chain;
  * roofline of the dominant kernel, cpu_baseline of the oracle (all host
    threads and one thread, with the CPU model).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--quick]
"""
from __future__ import annotations

import argparse
import glob
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0
# Vector ALU peak with unpacked FP32/FP64 FMAs: 256 CUs x 4 SIMDs x 16 lanes
# x 2 flops x 2.4 GHz = 78.6 TFLOP/s (the kernels are built without packed FP32).
ALU_PEAK_TFLOPS = 78.6
# Flops of one (quadrature point, baseline, parameter point) evaluation of P_ee
# and its 4 tangents in the scan kernel, FMA counted as 2 (q = KL/E is a
# configuration-stage table there): 3 phases (3); per phase the reduction
# (7), x (1), sin kernel (13), cos kernel (15), sin^2 / cos^2 / sin cos (3),
# sin 2phi (1), i.e. 40 x 3; P (6); tangents (18); baseline weight (10);
# flux factor (10).
FLOPS_PER_PEE_GRAD_EVAL = 167
# The generic chain kernel computes the phase q = (K L) / E per (quadrature
# point, baseline) itself (a reciprocal-based quotient, counted as 2).
FLOPS_PER_CHAIN_ITEM = FLOPS_PER_PEE_GRAD_EVAL + 2
# A tile of 16 points with common (dm2_21, dm2_31) shares its phases: per
# (quadrature point, baseline) item the three phases' terms (3 x 40), the
# weights f w and f w q (2) and 10 weighted bin sums (19); per (parameter
# point, bin) nu from the smeared sums (9), the chi^2 term with its division
# and logarithm counted as one flop each (5) and the gradient projections
# (16).  The smearing GEMM of the sums runs on the matrix cores and is not
# counted here.
FLOPS_SHARED_PER_ITEM = 141
FLOPS_SHARED_PER_POINT_BIN = 30
SCAN_TILE = 16


def scan_flops(P, n_items, n_bins, share=True):
    """Algorithmic flops of one scan launch: shared tiles pay the per-item sums
    once plus the per-point combination; other tiles pay every evaluation."""
    P = np.asarray(P)
    flops = 0
    for t in range(0, P.shape[0], SCAN_TILE):
        blk = P[t:t + SCAN_TILE]
        if share and np.all(blk[:, 0] == blk[0, 0]) and np.all(blk[:, 1] == blk[0, 1]):
            flops += n_items * FLOPS_SHARED_PER_ITEM + \
                blk.shape[0] * n_bins * FLOPS_SHARED_PER_POINT_BIN
        else:
            flops += blk.shape[0] * n_items * FLOPS_PER_PEE_GRAD_EVAL
    return flops


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def source_hash():
    """Hash of the kernel sources with comments and blank space removed:
    counter readings are valid only for this code (a comment edit keeps them)."""
    h = hashlib.sha256()
    for f in sorted(glob.glob(os.path.join(ROOT, "paper_1804_07682_amd", "csrc", "*"))):
        if f.endswith((".hip", ".h")):
            text = open(f).read()
            text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
            text = re.sub(r"//[^\n]*", " ", text)
            h.update(" ".join(text.split()).encode())
    return h.hexdigest()[:16]


def measured_traffic(kernel_key):
    """HBM bytes per launch of `kernel_key` from profiles/traffic_pmc.txt (rocprofv3
    FETCH_SIZE / WRITE_SIZE runs, scaled by the same counters on the streaming
    copy of known size), or None if absent or taken on other kernel sources."""
    path = os.path.join(ROOT, "profiles", "traffic_pmc.txt")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m = re.search(r"source_hash\s+(\w+)", text)
    if not m or m.group(1) != source_hash():
        return None
    for line in text.splitlines():
        if line.startswith("kernel ") and f"key={kernel_key} " in line + " ":
            t = re.search(r"traffic_bytes=([0-9.eE+]+)", line)
            return float(t.group(1)) if t else None
    return None


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=400)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--quick", action="store_true", help="skip the secondary workloads")
    ap.add_argument("--only", default=None,
                    help="run one workload for profiling: scan|scan64|scan_pp|scan64_pp|pee|pee64|copy|"
                         "chain1|chain8|fitset|fitset1|fitsetq|graph")
    ap.add_argument("--no-tune", action="store_true",
                    help="keep the automatic launch shape (no autotuning), for counter runs")
    ap.add_argument("--prec", default="mixed", choices=["mixed", "fp64"])
    ap.add_argument("--opts", default=None,
                    help="with --only fitset* / chain1 / chain8: launch options as JSON, e.g. "
                         "'{\"split_tail\": 2, \"threads\": 128}' (no autotuning)")
    return ap.parse_args()


class Timer:
    """HIP events on the stream the library launches on (torch's current stream).

    run() times `steps` calls back to back, bracketed by a synchronize and a
    pair of events only (no per-step work on the host, which would otherwise
    show up as gaps between launches): the host wall time and the event span
    divided by `steps` (the launch period, which for a GPU-bound loop is the
    kernel's average duration plus the dispatch gap).  It then repeats `steps`
    calls with an event pair around each for the mean and median of single
    calls (those events add a few microseconds of their own per call)."""

    def __init__(self, torch):
        self.torch = torch

    def run(self, fn, steps, warmup):
        torch = self.torch
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        e0.record()
        for _ in range(steps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        self.period = e0.elapsed_time(e1) * 1e-3 / steps
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(steps)]
        for a, b in ev:
            a.record()
            fn()
            b.record()
        torch.cuda.synchronize()
        k = np.array([a.elapsed_time(b) for a, b in ev]) * 1e-3
        return wall, float(k.mean()), float(np.median(k))


TUNE = True
STREAM_WARMUP = 120


def scan_setup(gna, W, torch, prec, dev, share=True, params=None):
    model = W.model()
    pr = W.config0()
    # Pseudo-data: Poisson counts drawn from this library's own FP64 prediction.
    tmp = gna.Chain(pr, model, max_batch=1, prec="fp64", opts={"smear_mfma": 0}, device=dev)
    nu = tmp.eval(torch.tensor(W.THETA0, device=dev).reshape(1, 5), grad=False,
                  pred=True)["pred"].cpu().numpy()[0]
    pr["data"] = W.poisson_counts(nu, W.SEED)
    P = torch.tensor(W.config3_params() if params is None else params, dtype=torch.float64,
                     device=dev)
    plan = gna.Chain(pr, model, max_batch=P.shape[0], prec=prec, device=dev,
                     opts=None if share else {"no_shared_phases": 1})
    if TUNE:
        plan.autotune(P, reps=10)
    return pr, model, plan, P


def bench_scan(gna, W, torch, timer, prec, dev, steps, warmup, share=True, params=None):
    pr, model, plan, P = scan_setup(gna, W, torch, prec, dev, share, params)
    out = {"chi2": torch.empty(P.shape[0], dtype=torch.float64, device=dev),
           "grad": torch.empty((P.shape[0], 5), dtype=torch.float64, device=dev)}
    fn = lambda: plan.eval(P, grad=True, out=out)
    wall, kpair, kmed = timer.run(fn, steps, warmup)
    kmean = timer.period
    plan.status()
    flops = scan_flops(P.cpu().numpy(), 1200, 240, share)
    # The per-point count: every (quadrature point, parameter point) pays a
    # full P_ee + tangents evaluation, shared phases or not.
    pp_flops = P.shape[0] * 1200 * FLOPS_PER_PEE_GRAD_EVAL
    return {"plan": plan, "pr": pr, "P": P, "wall": wall, "kernel_s": kmean,
            "event_pair_s": kpair, "event_pair_med_s": kmed,
            "evals_per_s": P.shape[0] * steps / wall, "shape": plan.shape(),
            "flops": flops, "tflops": flops / kmean / 1e12,
            "pp_flops": pp_flops, "pp_tflops": pp_flops / kmean / 1e12}


def bench_pee(gna, W, torch, timer, dev, n, L, prec, steps):
    E = torch.from_numpy(W.config1_energies(n)).to(dev)
    odt = torch.float64 if prec == "fp64" else torch.float32
    out = torch.empty(n, dtype=odt, device=dev)
    fn = lambda: gna.gna_pee(E, L, W.THETA0, prec=prec, out=out)
    # Streaming rates ramp up over the first ~100 back-to-back launches on a
    # fresh allocation; the untimed warm-up covers that, so the figure is the
    # sustained one.
    wall, _, _ = timer.run(fn, steps, STREAM_WARMUP)
    kmean = timer.period
    nbytes = n * (8 + out.element_size())
    res = {"evals_per_s": n * steps / wall, "kernel_ms": kmean * 1e3,
           "GBps": nbytes / kmean / 1e9, "bytes_per_eval": 8 + out.element_size()}
    res["hbm_frac"] = res["GBps"] / HBM_PEAK_GBPS
    del E, out
    return res


def pee_sweep(gna, W, torch, timer, dev):
    """Elementwise P_ee over N in {1e6, 1e7, 1e8} energies and L in {1, 52.5,
    1300} km, FP64 and mixed: GB/s per case (only N = 1e8 exceeds the 256 MB
    Infinity Cache; 1e6 is launch-bound) and the largest relative error of
    mixed against FP64 per baseline (N = 1e6)."""
    out = {}
    for n in (10 ** 6, 10 ** 7, 10 ** 8):
        for L in (1.0, 52.5, 1300.0):
            key = f"N={n:.0e} L={L:g}"
            out[key] = {}
            for prec in ("fp64", "mixed"):
                r = bench_pee(gna, W, torch, timer, dev, n, L, prec, 20 if n == 10 ** 8 else 100)
                out[key][prec] = {"GBps": round(r["GBps"], 1), "hbm_frac": round(r["hbm_frac"], 4),
                                  "kernel_us": round(r["kernel_ms"] * 1e3, 2)}
    err = {}
    E = torch.from_numpy(W.config1_energies(10 ** 6)).to(dev)
    for L in (1.0, 52.5, 1300.0):
        a = gna.gna_pee(E, L, W.THETA0, prec="fp64").cpu().numpy()
        b = gna.gna_pee(E, L, W.THETA0, prec="mixed").double().cpu().numpy()
        err[f"L={L:g}"] = {"max_rel": float(np.max(np.abs(b - a) / np.abs(a))),
                           "max_abs": float(np.max(np.abs(b - a)))}
    out["mixed_vs_fp64"] = err
    return out


def copy_probe(gna, torch, timer, dev, n=10 ** 8, steps=20):
    """The library's streaming copy (16 B loads and stores, the P_ee grid shape)."""
    a = torch.empty(n, dtype=torch.float64, device=dev).fill_(1.0)
    b = torch.empty_like(a)
    timer.run(lambda: gna.gna_stream_copy(a, b), steps, STREAM_WARMUP)
    kmean = timer.period
    return {"GBps": 16 * n / kmean / 1e9, "bytes": 16 * n, "kernel_ms": kmean * 1e3}


def bench_chain_single(gna, W, torch, timer, dev, problem_fn, seed, steps, prec, opts=None):
    model = W.model()
    pr = problem_fn()
    tmp = gna.Chain(pr, model, max_batch=1, prec="fp64", opts={"smear_mfma": 0}, device=dev)
    nu = tmp.eval(torch.tensor(W.THETA0, device=dev).reshape(1, 5), grad=False,
                  pred=True)["pred"].cpu().numpy()[0]
    pr["data"] = W.poisson_counts(nu, seed)
    plan = gna.Chain(pr, model, max_batch=1, prec=prec, device=dev, opts=opts)
    P = torch.tensor(W.THETA0 * np.array([1.01, 0.99, 1.02, 0.97, 1.0]),
                     device=dev).reshape(1, 5)
    if opts is None:
        plan.autotune(P, reps=5)
    out = {"chi2": torch.empty(1, dtype=torch.float64, device=dev),
           "grad": torch.empty((1, 5), dtype=torch.float64, device=dev)}
    wall, kpair, _ = timer.run(lambda: plan.eval(P, grad=True, out=out), steps, 10)
    res = {"evals_per_s": steps / wall, "launch_period_us": timer.period * 1e6,
           "event_pair_us": kpair * 1e6, "shape": plan.shape()}
    # Point-pass work against the ALU peak (the smearing tail is not counted).
    items = (len(pr["edges"]) - 1) * int(pr["gl_order"]) * int(pr.get("n_sub", 1)) * len(pr["L"])
    flops = items * FLOPS_PER_CHAIN_ITEM
    res["alu"] = {"flops_per_eval": flops, "achieved_tflops": flops / timer.period / 1e12,
                  "frac": flops / timer.period / 1e12 / ALU_PEAK_TFLOPS,
                  "flop_model": f"{FLOPS_PER_CHAIN_ITEM} per (quadrature point, baseline)"}
    res["graph"] = graph_rate(torch, lambda: plan.eval(P, grad=True, out=out), steps)
    return res


def graph_rate(torch, fn, steps, per_graph=20):
    """Evaluations per second when `per_graph` evaluations are captured in one
    HIP graph and the graph is replayed (no per-launch host work)."""
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        fn()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        for _ in range(per_graph):
            fn()
    reps = max(1, steps // per_graph)
    for _ in range(3):
        g.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        g.replay()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    return {"evals_per_s": reps * per_graph / dt, "us_per_eval": dt / (reps * per_graph) * 1e6,
            "evals_per_graph": per_graph}


def bench_fitset(gna, W, torch, timer, dev, steps, prec, opts=None, tune=True):
    model = W.model()
    problems, params = W.config4()
    # Pseudo-data per fit from this library's FP64 prediction at THETA0.
    tmp = gna.FitSet(problems, model, prec="fp64", device=dev)
    th0 = torch.tensor(np.tile(W.THETA0, (len(problems), 1)), device=dev)
    nu = tmp.eval(th0, grad=False, pred=True)["pred"].cpu().numpy()
    del tmp
    off = 0
    for f, pb in enumerate(problems):
        nb = len(pb["edges"]) - 1
        pb["data"] = W.poisson_counts(nu[off:off + nb], W.config4_data_seed(f))
        off += nb
    plan = gna.FitSet(problems, model, prec=prec, device=dev, opts=opts)
    P = torch.tensor(params, device=dev)
    if TUNE and tune:
        plan.autotune(P, reps=3)
    wall, _, _ = timer.run(lambda: plan.eval(P, grad=True), steps, 3)
    kmean = timer.period
    shape = plan.shape()
    # A split tail is the point pass plus two tail launches; the fused and the
    # queued tails are one launch.
    return {"fits_per_s": len(problems) * steps / wall, "kernel_ms": kmean * 1e3,
            "launches": 3 if shape["split_tail"] == 1 else 1, "shape": shape,
            "problems": problems, "plan": plan, "P": P}


def table1_gpu(gna, W, torch, timer, dev):
    """GPU side of the Table-1 analogue (FP64 P_ee, 52.5 km): compute-only
    kernel time, and time with the host transfers of E (H2D) and P (D2H)
    through pinned buffers, per evaluation."""
    out = {}
    for n in (10 ** 4, 10 ** 6):
        E_host = torch.from_numpy(W.config1_energies(n)).pin_memory()
        P_host = torch.empty(n, dtype=torch.float64).pin_memory()
        E_dev = E_host.to(dev)
        P_dev = torch.empty(n, dtype=torch.float64, device=dev)
        _, kmean, _ = timer.run(lambda: gna.gna_pee(E_dev, 52.5, W.THETA0, out=P_dev), 200, 10)

        def with_transfers():
            E_dev.copy_(E_host, non_blocking=True)
            gna.gna_pee(E_dev, 52.5, W.THETA0, out=P_dev)
            P_host.copy_(P_dev, non_blocking=True)
            torch.cuda.current_stream().synchronize()

        for _ in range(10):
            with_transfers()
        reps = 200
        t0 = time.perf_counter()
        for _ in range(reps):
            with_transfers()
        serial = (time.perf_counter() - t0) / reps
        chunk = min(1 << 18, n + (n & 1))
        piped = lambda: gna.gna_pee_host(E_host, 52.5, W.THETA0, out=P_host, chunk=chunk,
                                         n_streams=3)
        for _ in range(10):
            piped()
        t0 = time.perf_counter()
        for _ in range(reps):
            piped()
        out[str(n)] = {"gpu_compute_s": kmean, "gpu_with_transfers_s": serial,
                       "gpu_with_transfers_pipelined_s": (time.perf_counter() - t0) / reps}
    return out


def transfer_pipeline(gna, W, torch, dev, n=10 ** 8):
    """P_ee for N = 1e8 energies in pinned host memory, results back to host:
    serialized (copy in, kernel, copy out) against the library's pipelined
    transfers (chunks of 2^22 on 3 streams).  GB/s counts the 16 B per element
    that cross the host link."""
    E_host = torch.from_numpy(W.config1_energies(n)).pin_memory()
    P_host = torch.empty(n, dtype=torch.float64).pin_memory()
    E_dev = torch.empty(n, dtype=torch.float64, device=dev)
    P_dev = torch.empty(n, dtype=torch.float64, device=dev)

    def serial():
        E_dev.copy_(E_host, non_blocking=True)
        gna.gna_pee(E_dev, 52.5, W.THETA0, out=P_dev)
        P_host.copy_(P_dev, non_blocking=True)
        torch.cuda.current_stream().synchronize()

    ws = None
    res = {"n": n, "bytes_over_link": 16 * n}
    for tag, fn in (("serial", serial),
                    ("pipelined", lambda: gna.gna_pee_host(E_host, 52.5, W.THETA0, out=P_host,
                                                           chunk=1 << 22, n_streams=3))):
        fn()
        reps = 5
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        dt = (time.perf_counter() - t0) / reps
        res[tag] = {"s": dt, "GBps": 16 * n / dt / 1e9}
    res["speedup"] = res["serial"]["s"] / res["pipelined"]["s"]
    del E_host, P_host, E_dev, P_dev
    return res


def _median_us(fn, reps):
    """Median host wall time of fn(i), i < reps, in microseconds (robust to the
    occasional host-side stall that would dominate a mean)."""
    t = []
    for i in range(reps):
        t0 = time.perf_counter()
        fn(i)
        t.append(time.perf_counter() - t0)
    return float(np.median(t)) * 1e6


def graph_lazy(gna, W, torch, dev, reps=200):
    """Transformation graph of the config-0 chain (points -> P_ee -> flux product
    -> bin sums -> smearing -> norm -> chi^2), read back after changing dm2_31
    (every node after the points recomputed) or only the normalisation (two
    nodes recomputed), against the fused chain for the same evaluation, and
    the graph's fused chain node (chi^2 and gradient) read back."""
    model = W.model()
    pr = W.config0()
    tmp = gna.Chain(pr, model, max_batch=1, prec="fp64", opts={"smear_mfma": 0}, device=dev)
    nu = tmp.eval(torch.tensor(W.THETA0, device=dev).reshape(1, 5), grad=False,
                  pred=True)["pred"].cpu().numpy()[0]
    pr["data"] = W.poisson_counts(nu, W.SEED)
    g = gna.Graph(dev)
    v = [g.variable(nm, W.THETA0[i]) for i, nm in enumerate(("dm21", "dm31", "s12", "s13", "norm"))]
    pts = g.points(pr, model)
    osc = g.oscprob(pts, 52.5, v[0], v[1], v[2], v[3])
    chi2 = g.chi2(g.scale(g.smear(g.integrate(g.product(g.flux(pts), osc), pts), pts), v[4]), pts)
    g.bind()
    res = {}
    for tag, var, base in (("dm31_changed", v[1], W.THETA0[1]), ("norm_changed", v[4], 1.0)):
        for i in range(10):  # untimed warm-up of this change pattern
            g.set(var, base * (1.0 + 1e-6 * (i % 2 + 1)))
            g.read(chi2)
        res[f"{tag}_us"] = _median_us(
            lambda i: (g.set(var, base * (1.0 + 1e-6 * (i % 2 + 1))), g.read(chi2)), reps)
    plan = gna.Chain(pr, model, max_batch=1, device=dev, opts={"smear_mfma": 0})
    P = torch.tensor(W.THETA0, device=dev).reshape(1, 5)
    out = {"chi2": torch.empty(1, dtype=torch.float64, device=dev)}
    host = torch.empty(1, dtype=torch.float64).pin_memory()
    def fused():
        plan.eval(P, grad=False, out=out)
        host.copy_(out["chi2"], non_blocking=True)
        torch.cuda.current_stream().synchronize()
    fused()
    res["fused_chain_us"] = _median_us(lambda i: fused(), reps)
    out6 = torch.empty(6, dtype=torch.float64, device=dev)
    host6 = torch.empty(6, dtype=torch.float64).pin_memory()
    outg = {"chi2": out6[:1], "grad": out6[1:].view(1, 5)}
    def fused_grad():
        plan.eval(P, grad=True, out=outg)
        host6.copy_(out6, non_blocking=True)
        torch.cuda.current_stream().synchronize()
    fused_grad()
    res["fused_chain_grad_us"] = _median_us(lambda i: fused_grad(), reps)
    g.close()
    # The same evaluation as one fused chain node of a graph (chi^2 and its
    # gradient in one launch), after a dm2_31 change and with nothing changed
    # (the read returns the host mirror; no launch, no copy).
    g = gna.Graph(dev)
    v = [g.variable(nm, W.THETA0[i]) for i, nm in enumerate(("dm21", "dm31", "s12", "s13", "norm"))]
    pts = g.points(pr, model)
    node = g.chain(pts, v, "fp64")
    g.bind()
    for i in range(10):  # untimed warm-up
        g.set(v[1], W.THETA0[1] * (1.0 + 1e-6 * (i % 2 + 1)))
        g.read(node)
    res["chain_node_dm31_changed_us"] = _median_us(
        lambda i: (g.set(v[1], W.THETA0[1] * (1.0 + 1e-6 * (i % 2 + 1))), g.read(node)), reps)
    res["chain_node_unchanged_us"] = _median_us(lambda i: g.read(node), reps)
    res["note"] = ("host wall time per evaluation, median of the repetitions; chi^2 read "
                   "back to the host each time (one synchronising copy per evaluation); the "
                   "chain node also returns the gradient")
    g.close()
    return res


def table1_cpu(W, threads):
    import oracle
    res = {}
    for n in (10 ** 4, 10 ** 6):
        E = W.config1_energies(n)
        for nt, tag in ((1, "cpu_1core_s"), (threads, "cpu_all_cores_s")):
            oracle.pee(E, 52.5, W.THETA0, n_threads=nt)
            reps = max(1, int(2e6 // n))
            t0 = time.perf_counter()
            for _ in range(reps):
                oracle.pee(E, 52.5, W.THETA0, n_threads=nt)
            res.setdefault(str(n), {})[tag] = (time.perf_counter() - t0) / reps
    return res


GRAD_ERR_DEF = ("max over points and components of |theta_c (g_mixed - g_fp64)| / "
                "max(|theta_c g_fp64|, chi2_fp64, 1)")


def output_errors(a, b, th):
    """Largest error of mixed-precision outputs `a` against FP64 outputs `b` per
    output: the prediction nu (relative), chi^2 (relative and absolute) and the
    gradient (scaled: it is ~0 near a minimum, see GRAD_ERR_DEF)."""
    res = {"pred_max_rel": float(np.max(np.abs(a["pred"] - b["pred"]) / np.abs(b["pred"]))),
           "chi2_max_rel": float(np.max(np.abs(a["chi2"] - b["chi2"]) / np.abs(b["chi2"]))),
           "chi2_max_abs": float(np.max(np.abs(a["chi2"] - b["chi2"])))}
    th = np.atleast_2d(th)
    scale = np.maximum(np.maximum(np.abs(th * b["grad"]), b["chi2"][:, None]), 1.0)
    res["grad_max_scaled"] = float(np.max(np.abs(th * (a["grad"] - b["grad"])) / scale))
    res["meets_1e-6"] = bool(max(res["pred_max_rel"], res["chi2_max_rel"],
                                 res["grad_max_scaled"]) <= 1e-6)
    return res


def mixed_errors(gna, W, torch, dev, pr, P):
    """Mixed against FP64 on a chain plan of B points (the same launch shape rules)."""
    model = W.model()
    outs = {}
    for prec in ("fp64", "mixed"):
        plan = gna.Chain(pr, model, max_batch=P.shape[0], prec=prec, device=dev)
        outs[prec] = {k: v.cpu().numpy() for k, v in plan.eval(P, grad=True, pred=True).items()}
        plan.close()
    return output_errors(outs["mixed"], outs["fp64"], P.cpu().numpy())


def single_point_problem(gna, W, torch, dev, problem_fn, seed):
    """A single-point geometry with Poisson pseudo-data from this library's
    FP64 prediction at THETA0."""
    model = W.model()
    pr = problem_fn()
    tmp = gna.Chain(pr, model, max_batch=1, prec="fp64", opts={"smear_mfma": 0}, device=dev)
    nu = tmp.eval(torch.tensor(W.THETA0, device=dev).reshape(1, 5), grad=False,
                  pred=True)["pred"].cpu().numpy()[0]
    tmp.close()
    pr["data"] = W.poisson_counts(nu, seed)
    return pr


def fitset_errors(gna, W, torch, dev, problems, P):
    model = W.model()
    outs = {}
    for prec in ("fp64", "mixed"):
        plan = gna.FitSet(problems, model, prec=prec, device=dev)
        outs[prec] = {k: v.cpu().numpy() for k, v in plan.eval(P, grad=True, pred=True).items()}
        plan.close()
    return output_errors(outs["mixed"], outs["fp64"], P.cpu().numpy())


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_threads():
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return max(1, min(threads, os.cpu_count() or 1))


def cpu_baseline(W, pr_gpu):
    """The oracle, as it stands, on the scan workload (its own pseudo-data): all
    host threads over the parameter points, then one thread on a 256-point
    slice of the same scan."""
    import oracle
    model = W.model()
    pr = W.config0()
    pr["data"] = W.poisson_counts(oracle.prediction(pr, model, W.THETA0), W.SEED)
    P = W.config3_params()
    threads = cpu_threads()
    oracle.chain(pr, model, P[:64], grad=True, n_threads=threads)  # warm-up
    t0 = time.perf_counter()
    reps = 0
    while True:
        oracle.chain(pr, model, P, grad=True, n_threads=threads)
        reps += 1
        if time.perf_counter() - t0 > 10.0 or reps >= 500:
            break
    dt = time.perf_counter() - t0
    t0 = time.perf_counter()
    reps1 = 0
    while True:
        oracle.chain(pr, model, P[:256], grad=True, n_threads=1)
        reps1 += 1
        if time.perf_counter() - t0 > 5.0:
            break
    dt1 = time.perf_counter() - t0
    return {"value": P.shape[0] * reps / dt, "unit": "chi2+grad evals/s", "cores": threads,
            "kind": "oracle",
            "sample": f"{reps} x the full 4096-point scan (1200 points, 240 bins, FP64), "
                      f"{dt:.1f} s, OpenMP over parameter points",
            "cpu_model": cpu_model(), "host_threads": os.cpu_count(),
            "single_thread": {"value": 256 * reps1 / dt1, "unit": "chi2+grad evals/s",
                              "cores": 1,
                              "sample": f"{reps1} x the first 256 points of the scan, "
                                        f"{dt1:.1f} s"}}


def main():
    args = parse()
    global TUNE
    TUNE = not args.no_tune
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: the library has no multi-GPU path "
              "(the design notes describe how the scan would shard).", file=sys.stderr)
        sys.exit(2)
    import torch

    import paper_1804_07682_amd as gna
    import workloads as W
    gna.load()
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    timer = Timer(torch)

    if args.only:
        o = args.only
        if o in ("scan", "scan64", "scan_pp", "scan64_pp", "scan_rnd", "scan64_rnd"):
            r = bench_scan(gna, W, torch, timer, "fp64" if o.startswith("scan64") else "mixed",
                           dev, args.steps, args.warmup, share=not o.endswith("_pp"),
                           params=W.config3_random_params() if o.endswith("_rnd") else None)
            log(f"{o}: {r['evals_per_s']:.4g} evals/s kernel {r['kernel_s'] * 1e6:.1f} us "
                f"shape {r['shape']}")
        elif o in ("pee", "pee64"):
            r = bench_pee(gna, W, torch, timer, dev, 10 ** 8, 52.5,
                          "fp64" if o == "pee64" else "mixed", args.steps)
            log(f"{o}: {r}")
        elif o == "graph":
            log(f"graph: {graph_lazy(gna, W, torch, dev)}")
        elif o == "copy":
            log(f"copy probe: {copy_probe(gna, torch, timer, dev, steps=args.steps)}")
        elif o == "chain1":
            log(str(bench_chain_single(gna, W, torch, timer, dev, W.config0, W.SEED, args.steps,
                                       args.prec, json.loads(args.opts) if args.opts else None)))
        elif o == "chain8":
            log(str(bench_chain_single(gna, W, torch, timer, dev, W.config2, W.SEED + 2,
                                       args.steps, args.prec,
                                       json.loads(args.opts) if args.opts else None)))
        elif o in ("fitset", "fitset1", "fitsetq"):
            opts = {"fitset1": {"split_tail": 1, "persistent": 1},
                    "fitsetq": {"split_tail": 3, "persistent": 1}}.get(o)
            if args.opts:
                opts = dict(opts or {}, **json.loads(args.opts))
            r = bench_fitset(gna, W, torch, timer, dev, args.steps, args.prec, opts=opts,
                             tune=o == "fitset" and not args.opts)
            for k in ("problems", "P", "plan"):
                r.pop(k)
            log(f"{o}: {r}")
        return

    log("scan (fp64) ...")
    torch.cuda.synchronize()
    main_r = bench_scan(gna, W, torch, timer, "fp64", dev, args.steps, args.warmup)
    B = main_r["P"].shape[0]
    v64 = main_r["shape"]["smear_mfma"] + 1
    line = {
        "metric": "P_ee evals/s and chi2+grad evals/s, mixed-prec vs FP64 at <=1e-6 rel err",
        "value": main_r["evals_per_s"],
        "unit": "chi2+grad evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": main_r["wall"] / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "batched scan in FP64: 4096 points (64x64 grid in dm2_31 x "
                               "sin2th13), 240 bins x 5-point Gauss-Legendre (1200 points), "
                               "L=52.5 km, chi2 + 5-parameter adjoint gradient per point",
                   "points": B, "bins": 240, "quadrature_points": 1200, "baselines": 1,
                   "precision": "FP64 throughout",
                   "shape": main_r["shape"]},
        "pee_evals_per_s_per_chi2_eval": 1200,
        "roofline": {"bound": "alu",
                     "kernel": f"scan_kernel<double,true,512,{v64},true> (FP64, tiles of 16 "
                               "points with common dm2 share their phases)",
                     "achieved": main_r["tflops"], "peak": ALU_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": main_r["tflops"] / ALU_PEAK_TFLOPS,
                     "traffic": measured_traffic(f"scan_kernel<double,true,512,{v64},true>"),
                     "kernel_us": main_r["kernel_s"] * 1e6,
                     "kernel_time": "launch period of the timed back-to-back loop (HIP events "
                                    "around all steps / steps)",
                     "event_pair_us": main_r["event_pair_s"] * 1e6,
                     "flops_per_launch": main_r["flops"],
                     "flop_model": f"executed work: shared tiles {FLOPS_SHARED_PER_ITEM} per "
                                   f"(quadrature point, baseline) + {FLOPS_SHARED_PER_POINT_BIN} "
                                   f"per (point, bin); other tiles {FLOPS_PER_PEE_GRAD_EVAL} per "
                                   f"(quadrature point, baseline, point)",
                     "per_point_count": {
                         "flops_per_launch": main_r["pp_flops"],
                         "achieved": main_r["pp_tflops"],
                         "frac": main_r["pp_tflops"] / ALU_PEAK_TFLOPS,
                         "model": f"4096 x 1200 = 4.9e6 P_ee + tangent evaluations x "
                                  f"{FLOPS_PER_PEE_GRAD_EVAL} flops, the work of a kernel "
                                  f"that shares nothing (above 1 is impossible for such a "
                                  f"kernel: the shared tiles skip that work)"}},
    }
    log("scan (mixed) ...")
    rmx = bench_scan(gna, W, torch, timer, "mixed", dev, args.steps, args.warmup)
    vmx = rmx["shape"]["smear_mfma"] + 1
    line["mixed"] = {"value": rmx["evals_per_s"], "kernel_us": rmx["kernel_s"] * 1e6,
                     "speedup_over_fp64": rmx["evals_per_s"] / main_r["evals_per_s"],
                     "kernel": f"scan_kernel<float,true,512,{vmx},true>",
                     "achieved_tflops": rmx["tflops"], "frac": rmx["tflops"] / ALU_PEAK_TFLOPS,
                     "traffic": measured_traffic(f"scan_kernel<float,true,512,{vmx},true>"),
                     "shape": rmx["shape"]}
    if not args.quick:
        log("scan with per-point phases, and a batch of unrelated points ...")
        pp = {}
        for prec in ("fp64", "mixed"):
            r = bench_scan(gna, W, torch, timer, prec, dev, args.steps, args.warmup, share=False)
            pp[prec] = {"value": r["evals_per_s"], "kernel_us": r["kernel_s"] * 1e6,
                        "achieved_tflops": r["tflops"], "frac": r["tflops"] / ALU_PEAK_TFLOPS,
                        "shape": r["shape"]}
        pp["note"] = "the grid with phase sharing switched off (no_shared_phases=1)"
        line["per_point_phases"] = pp
        rnd = {}
        rparams = W.config3_random_params()
        for prec in ("fp64", "mixed"):
            r = bench_scan(gna, W, torch, timer, prec, dev, args.steps, args.warmup,
                           params=rparams)
            rnd[prec] = {"value": r["evals_per_s"], "kernel_us": r["kernel_s"] * 1e6,
                         "achieved_tflops": r["tflops"], "frac": r["tflops"] / ALU_PEAK_TFLOPS,
                         "shape": r["shape"]}
        rnd["note"] = ("4096 points drawn as THETA0 x U(0.8, 1.2) per parameter: no two "
                       "points share (dm2_21, dm2_31), so no tile shares its phases")
        line["random_batch"] = rnd
        log("mixed vs fp64 errors per output ...")
        errs = {"definition": {"pred": "max |nu_mixed - nu_fp64| / nu_fp64",
                               "chi2": "max relative and absolute difference",
                               "grad": GRAD_ERR_DEF}}
        errs["scan_grid"] = mixed_errors(gna, W, torch, dev, main_r["pr"], main_r["P"])
        errs["scan_random"] = mixed_errors(gna, W, torch, dev, main_r["pr"],
                                           torch.tensor(rparams, device=dev))
        th1 = torch.tensor(W.THETA0 * np.array([1.01, 0.99, 1.02, 0.97, 1.0]),
                           device=dev).reshape(1, 5)
        errs["chain_1pt"] = mixed_errors(
            gna, W, torch, dev, single_point_problem(gna, W, torch, dev, W.config0, W.SEED), th1)
        errs["chain_8L"] = mixed_errors(
            gna, W, torch, dev, single_point_problem(gna, W, torch, dev, W.config2, W.SEED + 2),
            th1)
        line["mixed_vs_fp64"] = errs
        log("pee N=1e8 ...")
        pee = {}
        for prec in ("fp64", "mixed"):
            pee[prec] = bench_pee(gna, W, torch, timer, dev, 10 ** 8, 52.5, prec, 20)
        pee["copy_probe"] = copy_probe(gna, torch, timer, dev)
        for prec, key in (("fp64", "pee_kernel<double,true,true>"),
                          ("mixed", "pee_kernel<float,true,false>")):
            pee[prec]["copy_frac"] = pee[prec]["GBps"] / pee["copy_probe"]["GBps"]
            pee[prec]["traffic"] = measured_traffic(key)
            pee[prec]["meets_70pct_hbm"] = bool(pee[prec]["hbm_frac"] >= 0.70)
        pee["workload"] = "N=1e8 energies uniform in [1.8, 12] MeV, L=52.5 km, one parameter point"
        line["pee"] = pee
        log("P_ee sweep over N and L ...")
        line["pee_sweep"] = pee_sweep(gna, W, torch, timer, dev)
        log("single-point chains ...")
        line["chain_1pt"] = {p: bench_chain_single(gna, W, torch, timer, dev, W.config0, W.SEED,
                                                   400, p) for p in ("fp64", "mixed")}
        line["chain_8L"] = {p: bench_chain_single(gna, W, torch, timer, dev, W.config2,
                                                  W.SEED + 2, 200, p) for p in ("fp64", "mixed")}
        log("fitset ...")
        fs = {}
        for p in ("fp64", "mixed"):
            r = bench_fitset(gna, W, torch, timer, dev, 50, p)
            problems, P4 = r.pop("problems"), r.pop("P")
            r.pop("plan").close()
            fs[p] = r
            for tag, sp in (("one_launch_queued_tail", 3), ("one_launch_fused_tail", 1)):
                f1 = bench_fitset(gna, W, torch, timer, dev, 50, p, opts={"split_tail": sp})
                f1.pop("problems"), f1.pop("P"), f1.pop("plan").close()
                fs[p][tag] = f1
        fs["mixed_vs_fp64"] = fitset_errors(gna, W, torch, dev, problems, P4)
        fs["note"] = ("the autotuned shape (split_tail 1: the point pass plus two tail "
                      "launches; 2: the queued tail in one persistent launch), and the "
                      "autotuned one-launch forms: the queued tail (one tail item per fit "
                      "in the persistent queue, after the fit's tiles) and the fused tail "
                      "(each fit's tail in the work-group of its last tile)")
        line["fitset"] = fs
        log("table-1 analogue (GPU side) ...")
        t1_gpu = table1_gpu(gna, W, torch, timer, dev)
        log("transformation graph, lazy evaluation ...")
        line["graph"] = graph_lazy(gna, W, torch, dev)
        log("host-memory P_ee, N = 1e8, serialized vs pipelined transfers ...")
        line["transfer_pipeline"] = transfer_pipeline(gna, W, torch, dev)
    log("cpu baseline (oracle) ...")
    line["cpu_baseline"] = cpu_baseline(W, main_r["pr"])
    if not args.quick:
        # Context only: the paper's Table 1 ratios (FP64 OscProb, i7-6700HQ vs GTX
        # 970M) were 0.017 / 1.39 with transfers and 20.90 / 26.46 compute-only.
        t1 = table1_cpu(W, cpu_threads())
        for n, g in t1_gpu.items():
            t1[n].update(g)
            for tag in ("cpu_1core_s", "cpu_all_cores_s"):
                t1[n][f"ratio_{tag[:-2]}_over_gpu_with_transfers"] = t1[n][tag] / g["gpu_with_transfers_s"]
                t1[n][f"ratio_{tag[:-2]}_over_gpu_compute"] = t1[n][tag] / g["gpu_compute_s"]
                t1[n][f"ratio_{tag[:-2]}_over_gpu_with_pipelined_transfers"] = \
                    t1[n][tag] / g["gpu_with_transfers_pipelined_s"]
        line["cpu_baseline"]["table1_analogue"] = t1
    print(json.dumps(line, default=lambda o: o if not isinstance(o, np.generic) else o.item()),
          flush=True)


if __name__ == "__main__":
    main()
