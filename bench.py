"""Throughput benchmark: evaluations/s at D = 100, N = 2^18 on one MI355X.

One step evaluates the population of N = 2^18 candidate vectors (uniform in [-100, 100]^100,
resident in HBM) on the eight rotated/unrotated formulas {sphere, elliptic, Griewank,
shifted Rastrigin, rotated Rastrigin, Rosenbrock, rotated Schwefel, Ackley} through
func_evaluatef (default split-BF16 mode).  The FP64 path (func_evaluate) is timed on the same
points for comparison.  Kernel durations come from HIP events recorded on the library stream
around every launch of the timed region; the roofline figure uses the algorithmic bytes of
the dominant kernel (D*4 bytes read + 4 bytes written per row).

Secondary workloads (reported under "secondary", not in "value"): the D = 1000, N = 2^18 form
of the same eight formulas; a hybrid and a composition at D = 1000, N = 16384; 64 batched
populations in one persistent launch (graph replay, direct launch, one call per population);
50-row calls and DE generations; the host-pointer entry points with their PCIe transfers.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline] [--no-secondary]
                    [--copy-probe]
    python bench.py --pmc-summary FETCH_DIR WRITE_DIR   (writes profiles/traffic_d100_n262144.*)

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import csv
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

DIM = 100
N = 1 << 18
FIDS = [0, 2, 9, 10, 11, 14, 16, 19]
NAMES = {0: "sphere", 2: "elliptic", 9: "griewank", 10: "rastrigin_u", 11: "rastrigin", 14: "rosenbrock",
         16: "schwefel", 19: "ackley"}
# resident kernel instance (path, formula family, rotated) each formula runs at D = 100 in the
# default split mode: path 0 = three BF16 products, 3 = six; the sphere skips its rotation
RESIDENT_KERNEL = {0: (0, 0, 0), 2: (0, 0, 1), 9: (0, 5, 1), 10: (0, 6, 0), 11: (0, 6, 1), 14: (0, 9, 1),
                   16: (3, 10, 1), 19: (0, 13, 1)}
HBM_PEAK_GBS = 8000.0
# The paper's own figures (Sec. 2, Tab. 2 single precision and Tab. 3 double precision): speedup of
# its CUDA implementation over the CPU-based CEC'14 code, 50 concurrent evaluations x 1000 runs,
# at its largest dimension (96).  Quoted as context only: other hardware, other baseline.
PAPER_CONTEXT = {
    "hardware": "Intel Core i5-2310 CPU + NVIDIA GeForce GTX 560 Ti, Windows 7 SP1 x64, CUDA 5.5",
    "workload": "50 evaluations per call x 1000 runs, uniform random data, D in {10, 32, 64, 96}",
    "baseline": "CPU CEC'14 benchmark code (not available here)",
    "speedup_d96_fp32": {"griewank": 11.13, "rastrigin_u": 1.82, "rastrigin": 9.98, "rosenbrock": 8.75,
                         "schwefel": 14.38, "ackley": 11.32},
    "speedup_d96_fp64": {"griewank": 9.72, "rastrigin_u": 1.78, "rastrigin": 9.62, "rosenbrock": 7.87,
                         "schwefel": 11.91, "ackley": 9.75},
    "note": "no absolute rates are published; these ratios do not compare with this library's numbers",
}
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_d100_n262144.json")
KERNEL_SOURCES = ["eval_resident.h", "formulas.h", "devprob.h", "kernels.h"]
COPY_PROBE_BYTES = N * DIM * 4  # the probe reads the FP32 population once and writes it once


def progress(msg: str) -> None:
    """A progress line on stderr (stdout carries only the result line)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1407_7737_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def resident_key(fid: int) -> str:
    p, k, r = RESIDENT_KERNEL[fid]
    return f"k_eval_resident<{p},{k},{r},{1 if DIM % 4 == 0 else 0}>"


def measured_traffic(fid: int):
    """HBM bytes per launch of the formula's kernel from the committed rocprofv3 counter
    summary, or None when the kernel sources changed since the counters were taken."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_source_hash") != kernel_source_hash():
        return None
    k = t.get("kernels", {}).get(resident_key(fid))
    return None if k is None else k.get("hbm_bytes_per_launch")


def host_cpu() -> dict:
    """CPU model and logical CPU count of the host (lscpu's model name, nproc)."""
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.lower().startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"model_name": model, "nproc": os.cpu_count(),
            "affinity": len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else None}


def cpu_single_thread(x32: np.ndarray, budget_s: float = 4.0) -> dict:
    """The oracle on one thread (the plain, slow figure), on consecutive 512-row chunks."""
    import oracle
    probs = {fid: oracle.basic(fid, DIM, 0) for fid in FIDS}
    rows, t, start = 0, 0.0, 0
    while t < budget_s:
        sample = x32[start:start + 512].astype(np.float64)
        t0 = time.perf_counter()
        for fid in FIDS:
            probs[fid](sample, threads=1)
        t += time.perf_counter() - t0
        rows += 512
        start = (start + 512) % (N - 512)
    return {"value": rows * len(FIDS) / t, "unit": "evals/s", "cores": 1,
            "sample": f"{rows} rows x {len(FIDS)} formulas in {t:.1f} s"}


def cpu_baseline(x32: np.ndarray, gpu: dict, budget_s: float = 12.0):
    """The oracle as it stands, on the host cores, on a bounded sample of the same rows: chunks
    of the population (wrapping around) on all measured formulas until about budget_s seconds
    of CPU work have been timed.  Threads: the CPU share of one GPU on the box (16; OpenMP's
    default there), or fewer where the host has fewer."""
    import oracle
    threads = max(1, min(os.cpu_count() or 1, oracle.threads_available(), 16))
    probs = {fid: oracle.basic(fid, DIM, 0) for fid in FIDS}
    chunk = 4096
    total_rows, t_total, start = 0, 0.0, 0
    errors = {}
    while t_total < budget_s:
        idx = (start + np.arange(chunk)) % N
        sample = x32[idx].astype(np.float64)
        t0 = time.perf_counter()
        ref = {fid: probs[fid](sample, threads=threads) for fid in FIDS}
        t_total += time.perf_counter() - t0
        if not errors:
            # the first chunk also checks the timed GPU outputs of the same rows (FP32 inputs
            # widened exactly, so both paths see the oracle's points): |f - f_oracle| / max(1, |f_oracle|)
            for fid in FIDS:
                split, fp64 = gpu[fid]
                scale = np.maximum(1.0, np.abs(ref[fid]))
                es = np.abs(split[idx].astype(np.float64) - ref[fid]) / scale
                e64 = np.abs(fp64[idx] - ref[fid]) / scale
                errors[NAMES[fid]] = {"split_max_rel_err": float(es.max()), "split_rows_over_1e-4": int((es > 1e-4).sum()),
                                      "fp64_max_rel_err": float(e64.max()), "fp64_rows_over_1e-10": int((e64 > 1e-10).sum()),
                                      "rows": int(idx.size)}
        total_rows += chunk * len(FIDS)
        start = (start + chunk) % N
        chunk = min(chunk * 2, 1 << 16)
    return {
        "value": total_rows / t_total,
        "unit": "evals/s",
        "cores": threads,
        "kind": "oracle",
        "sample": f"{total_rows // len(FIDS)} rows of the D={DIM} population (consecutive chunks, wrapping) on "
                  f"each of the {len(FIDS)} formulas, {total_rows} evaluations in {t_total:.1f} s; FP64 "
                  f"dense-rotation oracle, OpenMP over rows",
        "errors_vs_oracle": errors,
        "single_thread": cpu_single_thread(x32),
        "host": host_cpu(),
    }


def event_time_ms(torch, fn, reps: int, warmup: int = 2) -> float:
    """Mean time of fn() on the current stream from HIP events around the repeated launches."""
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        fn()
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / reps


MFMA_BF16_PEAK_TFLOPS = 2500.0  # dense BF16 matrix peak (split paths)
MFMA_FP32_PEAK_TFLOPS = 157.3   # FP32 matrix/vector peak (the plain FP32 mode's 16x16x4 FP32 MFMA)
# formulas the default split mode evaluates with six BF16 products (at n variables)
SIX = {3, 7, 8, 12, 13, 16, 17}


def products(base: int, n: int) -> int:
    return 6 if base in SIX or (base in (4, 14) and n < 10) or (base == 2 and n < 50) else 3


def rotation_work(c, pid: int, comp: int = -1):
    """(sum of n_k^2 over the rotation blocks, BF16 products per term) of a basic or hybrid
    problem in the default split mode, from the library's exported structure."""
    st = c.get_structure(pid, comp)
    sizes = [int(v) for v in st["sizes"]]
    nsq = sum(v * v for v in sizes)
    if st["type"] == "hybrid":
        prods = 6 if any(products(int(b), int(n)) == 6 for b, n in zip(st["bases"], sizes)) else 3
    else:
        prods = products(int(st["bases"][0]), len(st["o"]))
    return nsq, prods


def mfma_frac(flops_per_row: float, rows: int, ms: float, peak_tflops: float) -> float:
    return flops_per_row * rows / (ms * 1e-3) / (peak_tflops * 1e12)


def secondary(torch, c, reps: int = 10) -> dict:
    """The other workload shapes, timed briefly (kernel time from HIP events).  Rotation work is
    algorithmic: 2 x sum n_k^2 multiply-adds per row over the nonzero blocks (no padding), times
    the BF16 products per term (3 or 6) on the split path, once on the plain FP32 path."""
    from paper_1407_7737_amd.inputs import batch_params, composition_params, hybrid_params, population
    out = {}
    dev = torch.device("cuda:0")
    # D = 1000, N = 2^18: the same eight formulas on the tiled path, default split mode and the
    # plain FP32 mode
    d, n = 1000, 1 << 18
    progress("secondary: D=1000, N=2^18")
    c.initialize(d, n, 0)
    try:
        x = torch.from_numpy(population(n, d, seed=0, dtype=np.float32)).to(dev)
        o = torch.empty(n, dtype=torch.float32, device=dev)
        per, per32, frac, frac32 = {}, {}, {}, {}
        # one pass over every formula first: the device sat idle while the population was drawn,
        # and the first function timed would otherwise carry the ramp back to full clocks
        for fid in FIDS:
            c.func_evaluatef(fid, x, out=o)
        for fid in FIDS:
            per[NAMES[fid]] = event_time_ms(torch, lambda: c.func_evaluatef(fid, x, out=o), reps)
        c.set_mode(c.MODE_FP32)
        for fid in FIDS:
            per32[NAMES[fid]] = event_time_ms(torch, lambda: c.func_evaluatef(fid, x, out=o), reps)
        c.set_mode(c.MODE_SPLIT)
        for fid in FIDS:
            nsq, prods = rotation_work(c, fid)
            if nsq == 0:
                continue  # unrotated: no matrix work, bound by HBM
            frac[NAMES[fid]] = {"products": prods, "flops_per_row": 2 * nsq * prods,
                                "mfma_frac": mfma_frac(2 * nsq * prods, n, per[NAMES[fid]], MFMA_BF16_PEAK_TFLOPS)}
            frac32[NAMES[fid]] = mfma_frac(2 * nsq, n, per32[NAMES[fid]], MFMA_FP32_PEAK_TFLOPS)
        tot = sum(per.values())
        out["d1000_n262144"] = {"evals_per_s": n * len(FIDS) / (tot * 1e-3), "ms_per_function": per,
                                "hbm_frac_per_function": {k: n * (d * 4 + 4) / (v * 1e-3) / 1e9 / HBM_PEAK_GBS
                                                          for k, v in per.items()},
                                "mfma_bf16_frac_per_function": frac,
                                "fp32_mode_ms_per_function": per32,
                                "fp32_mode_evals_per_s": n * len(FIDS) / (sum(per32.values()) * 1e-3),
                                "fp32_mode_frac_of_157tf_per_function": frac32,
                                "sum_nk2": rotation_work(c, 11)[0]}
        del x
        # hybrid and composition at D = 1000, N = 16384
        progress("secondary: hybrid and composition, D=1000, N=16384")
        m = 16384
        xh = torch.from_numpy(population(m, d, seed=1, dtype=np.float32)).to(dev)
        oh = torch.empty(m, dtype=torch.float32, device=dev)
        bases, props = hybrid_params(d, seed=0)
        c.define_hybrid(100, bases, props)
        cb, sig, lam, bias = composition_params(seed=0)
        c.define_composition(101, cb, sig, lam, bias)
        th = event_time_ms(torch, lambda: c.func_evaluatef(100, xh, out=oh), reps)
        tc = event_time_ms(torch, lambda: c.func_evaluatef(101, xh, out=oh), reps)
        hn, hp = rotation_work(c, 100)
        cflops = 0
        for i in range(len(cb)):
            cn, cp = rotation_work(c, 101, i)
            cflops += 2 * cn * cp
        out["hybrid_d1000_n16384"] = {"evals_per_s": m / (th * 1e-3), "ms": th, "groups": len(bases),
                                      "bases": bases, "flops_per_row": 2 * hn * hp, "products": hp,
                                      "mfma_frac": mfma_frac(2 * hn * hp, m, th, MFMA_BF16_PEAK_TFLOPS),
                                      "hbm_frac": m * (d * 4 + 4) / (th * 1e-3) / 1e9 / HBM_PEAK_GBS}
        out["composition_d1000_n16384"] = {"evals_per_s": m / (tc * 1e-3), "ms": tc, "components": len(cb),
                                           "flops_per_row": cflops,
                                           "mfma_frac": mfma_frac(cflops, m, tc, MFMA_BF16_PEAK_TFLOPS),
                                           "hbm_frac": m * (d * 4 + 4) / (tc * 1e-3) / 1e9 / HBM_PEAK_GBS}
    finally:
        c.dispose()
    # 64 batched populations
    progress("secondary: 64 batched populations")
    c.initialize(10, 2048, 0)
    try:
        fids, dims, counts = batch_params(64, seed=0)
        b = c.Batch(fids, dims, counts, seed=0)
        xs = [torch.from_numpy(population(int(k), int(dd), seed=i, dtype=np.float32)).to(dev)
              for i, (dd, k) in enumerate(zip(dims, counts))]
        outs = [torch.empty(int(k), dtype=torch.float32, device=dev) for k in counts]
        b.bind(xs, outs)
        default_shape = b.shape()
        t_default = event_time_ms(torch, b.run, 50)
        tuned = b.tune(reps=20)
        t_graph = event_time_ms(torch, b.run, 50)
        t_direct = event_time_ms(torch, b.run_direct, 50)
        # 16 persistent launches captured in one graph (e.g. 16 consecutive batches of an
        # optimiser), replayed: the per-launch cost against 16 direct launches back to back
        g16 = torch.cuda.CUDAGraph()
        s16 = torch.cuda.Stream()
        s16.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s16):
            with torch.cuda.graph(g16, stream=s16):
                for _ in range(16):
                    b.run_direct()
        torch.cuda.current_stream().wait_stream(s16)
        c.set_stream(torch.cuda.current_stream())
        t_g16 = event_time_ms(torch, g16.replay, 20) / 16
        t_d16 = event_time_ms(torch, lambda: [b.run_direct() for _ in range(16)], 20) / 16
        del g16
        b.close()
        rows = int(sum(counts))
        out["batch_64"] = {"rows": rows, "graph_ms": t_graph, "direct_ms": t_direct, "untuned_graph_ms": t_default,
                           "graph16_ms_per_launch": t_g16, "direct16_ms_per_launch": t_d16,
                           "evals_per_s": rows / (t_graph * 1e-3),
                           "evals_per_s_graph16": rows / (t_g16 * 1e-3), "tuned_shape": tuned,
                           "default_shape": default_shape}
    finally:
        c.dispose()
    # one call per population for comparison (the same populations as 64 single evaluations)
    per_call = 0.0
    for dd in sorted(set(dims)):
        idx = [i for i in range(len(dims)) if dims[i] == dd]
        c.initialize(int(dd), 2048, 0)
        try:
            for i in idx:
                per_call += event_time_ms(torch, lambda: c.func_evaluatef(int(fids[i]), xs[i], out=outs[i]), 20)
        finally:
            c.dispose()
    out["batch_64"]["one_call_per_population_ms"] = per_call
    progress("secondary: 50-row latency and DE generations")
    out["latency_n50"] = latency_small(torch, c)
    out["de_n50"] = de_generations(torch, c)
    progress("secondary: host entry points (PCIe included)")
    out["host_entry_d100_n262144"] = host_entry(torch, c)
    return out


def host_entry(torch, c, reps: int = 5) -> dict:
    """The host-pointer entry points (h_func_evaluatef, h_func_evaluate) at D = 100, N = 2^18 on
    rotated Rastrigin: copy to the device, evaluate, copy back and wait, so the rate includes
    both PCIe transfers.  Inputs in pageable (numpy) and in pinned host memory.  A figure for
    callers that hold their population on the host, never the headline value."""
    import time
    from paper_1407_7737_amd.inputs import population
    d, n = 100, 1 << 18
    res = {}
    c.initialize(d, n, 0)
    try:
        x32 = population(n, d, seed=0, dtype=np.float32)
        pinned = torch.empty((n, d), dtype=torch.float32, pin_memory=True)
        pinned.copy_(torch.from_numpy(x32))
        x64 = population(n, d, seed=0)
        for name, arr, fn in (("fp32_pageable", x32, c.h_func_evaluatef),
                              ("fp32_pinned", pinned.numpy(), c.h_func_evaluatef),
                              ("fp64_pageable", x64, c.h_func_evaluate)):
            fn(11, arr)
            t0 = time.perf_counter()
            for _ in range(reps):
                fn(11, arr)
            dt = (time.perf_counter() - t0) / reps
            res[name] = {"ms": dt * 1e3, "evals_per_s": n / dt, "input_gb_per_s": arr.nbytes / dt / 1e9}
    finally:
        c.dispose()
    return res


def de_generations(torch, c, gens: int = 100) -> dict:
    """An optimiser in the loop, the paper's own setting (50 candidates per evaluation call):
    DE/rand/1/bin generations (trial vectors, evaluation, selection) on rotated Rastrigin,
    captured 100 at a time in one graph; time per generation of the replayed graph."""
    from paper_1407_7737_amd.inputs import population
    res = {}
    for d in (10, 32, 64, 96):
        c.initialize(d, 64, 0)
        try:
            row = {}
            for fp64 in (False, True):
                dt = np.float64 if fp64 else np.float32
                de = c.DE(11, torch.from_numpy(population(50, d, seed=d).astype(dt)).cuda(), seed=1, fp64=fp64)
                de.capture(gens)
                de.replay()
                torch.cuda.synchronize()
                ms = event_time_ms(torch, de.replay, 5, warmup=1)
                row["fp64_us_per_generation" if fp64 else "fp32_us_per_generation"] = ms * 1e3 / gens
                row["fp64_best" if fp64 else "fp32_best"] = float(de.fit.min().item())
                del de
            res[f"d{d}"] = row
        finally:
            torch.cuda.synchronize()
            c.set_stream(None)
            c.dispose()
    return res


def latency_small(torch, c, calls: int = 100) -> dict:
    """The paper's own regime: many calls on 50 candidates (rotated Rastrigin, split path).
    Per call: wall-clock of back-to-back eager calls (Python and launch included), the same
    calls replayed from one captured graph, and the kernel alone (HIP events)."""
    from paper_1407_7737_amd.inputs import population
    res = {}
    for d in (10, 32, 64, 96):
        c.initialize(d, 64, 0)
        try:
            x = torch.from_numpy(population(50, d, seed=d, dtype=np.float32)).cuda()
            o = torch.empty(50, device="cuda")
            for _ in range(10):
                c.func_evaluatef(11, x, out=o)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(calls):
                c.func_evaluatef(11, x, out=o)
            torch.cuda.synchronize()
            eager = (time.perf_counter() - t0) / calls
            g = torch.cuda.CUDAGraph()
            s = torch.cuda.Stream()
            s.wait_stream(torch.cuda.current_stream())
            with torch.cuda.stream(s):
                with torch.cuda.graph(g, stream=s):
                    for _ in range(calls):
                        c.func_evaluatef(11, x, out=o)
            torch.cuda.current_stream().wait_stream(s)
            g.replay()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(5):
                g.replay()
            torch.cuda.synchronize()
            graph = (time.perf_counter() - t0) / (5 * calls)
            kern = event_time_ms(torch, lambda: c.func_evaluatef(11, x, out=o), 50) * 1e-3
            res[f"d{d}"] = {"eager_us": eager * 1e6, "graph_us": graph * 1e6, "kernel_us": kern * 1e6,
                            "evals_per_s_graph": 50 / graph}
            del g
        finally:
            torch.cuda.synchronize()
            c.set_stream(None)
            c.dispose()
    return res


def pmc_summary(fetch_dir: str, write_dir: str) -> None:
    """Per-kernel FETCH_SIZE / WRITE_SIZE (KiB per dispatch) from two rocprofv3 --pmc runs of
    this script with --copy-probe, scaled by what the counters read for the copy of a known
    number of bytes; writes profiles/traffic_d100_n262144.{json,txt}."""
    def load(d, counter):
        vals = {}
        for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
            for row in csv.DictReader(open(f)):
                if row["Counter_Name"] != counter:
                    continue
                vals.setdefault(row["Kernel_Name"], []).append(float(row["Counter_Value"]))
        return vals

    def short(name):
        m = (re.search(r"k_eval_residentILi(\d+)ELi(\d+)ELi(\d+)ELi(\d+)E", name)
             or re.search(r"k_eval_resident<(\d+), (\d+), (\d+), (\d+)>", name))
        if m:
            return "k_eval_resident<{},{},{},{}>".format(*m.groups())
        return None

    fetch, write = load(fetch_dir, "FETCH_SIZE"), load(write_dir, "WRITE_SIZE")
    copy_f = [v for k, vs in fetch.items() if "neg" in k.lower() for v in vs]
    copy_w = [v for k, vs in write.items() if "neg" in k.lower() for v in vs]
    cf = COPY_PROBE_BYTES / (float(np.median(copy_f)) * 1024.0)
    cw = COPY_PROBE_BYTES / (float(np.median(copy_w)) * 1024.0)
    kernels = {}
    for name in set(fetch) | set(write):
        key = short(name)
        if key is None:
            continue
        f = fetch.get(name, [])
        w = write.get(name, [])
        fk = float(np.median(f)) if f else 0.0
        wk = float(np.median(w)) if w else 0.0
        kernels[key] = {"fetch_kib": fk, "write_kib": wk, "hbm_bytes_per_launch": fk * 1024 * cf + wk * 1024 * cw}
    algo = N * (DIM * 4 + 4)
    res = {"kernel_source_hash": kernel_source_hash(), "copy_probe_bytes": COPY_PROBE_BYTES,
           "fetch_scale": cf, "write_scale": cw, "algorithmic_bytes_fp32": algo, "kernels": kernels}
    os.makedirs(os.path.join(ROOT, "profiles"), exist_ok=True)
    with open(TRAFFIC_FILE, "w") as f:
        json.dump(res, f, indent=1, sort_keys=True)
    lines = ["HBM traffic per launch, D=100, N=2^18 (rocprofv3 --pmc, one counter per run)", "",
             "commands (from the repository root):",
             "  rocprofv3 --pmc FETCH_SIZE --output-format csv -d <FETCH_DIR> -- python bench.py --steps 2 --warmup 1"
             " --no-cpu-baseline --no-secondary --copy-probe",
             "  rocprofv3 --pmc WRITE_SIZE --output-format csv -d <WRITE_DIR> -- python bench.py --steps 2 --warmup 1"
             " --no-cpu-baseline --no-secondary --copy-probe",
             "  python bench.py --pmc-summary <FETCH_DIR> <WRITE_DIR>", "",
             f"copy probe: {COPY_PROBE_BYTES} bytes read and written; counter scale fetch {cf:.4f}, write {cw:.4f}",
             f"algorithmic bytes per FP32 launch: {algo}", "",
             f"{'kernel':34s} {'FETCH KiB':>12s} {'WRITE KiB':>12s} {'HBM bytes':>14s} {'/ algorithmic':>14s}"]
    for k in sorted(kernels):
        v = kernels[k]
        lines.append(f"{k:34s} {v['fetch_kib']:12.0f} {v['write_kib']:12.0f} {v['hbm_bytes_per_launch']:14.0f} "
                     f"{v['hbm_bytes_per_launch'] / algo:14.3f}")
    with open(TRAFFIC_FILE.replace(".json", ".txt"), "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines))


FAMILY = {0: "wsphere", 5: "griewank", 6: "rastrigin", 9: "rosenbrock", 10: "schwefel", 13: "ackley"}
PATH_NAME = {0: "x3 split", 1: "FP32", 2: "FP64", 3: "x6 split"}


def trace_summary(kind: str, headline_dir: str, secondary_dir: str, steps: int = 5) -> None:
    """Per-kernel launch durations from two rocprofv3 --kernel-trace --stats runs of this script
    (the headline step, then the run with the secondary workloads); writes
    profiles/resident_d100_n262144_kernel_trace.txt and profiles/secondary_kernel_trace.txt.
    The headline table averages the last 2 * steps dispatches of each kernel (the timed steps
    back to back, then the event-bracketed ones), read from the per-dispatch trace: the
    autotuner's trial launches of the same kernels come first."""
    def dispatches(d):
        files = glob.glob(os.path.join(d, "**", "*kernel_trace.csv"), recursive=True)
        rows = []
        for f in files:
            rows.extend(csv.DictReader(open(f)))
        rows.sort(key=lambda r: int(r["Start_Timestamp"]))
        return rows

    def stats(d):
        f = os.path.join(d, "run_kernel_stats.csv")
        return list(csv.DictReader(open(f)))

    def short(name):
        m = re.search(r"(k_\w+)<([^>]*)>", name)
        if m:
            return m.group(1) + "<" + m.group(2).replace(" ", "") + ">"
        m = re.search(r"(k_\w+)", name)
        return m.group(1) if m else None

    cmd_head = ("rocprofv3 --kernel-trace --stats --output-format csv -d <OUT> -o run -- python -u bench.py "
                f"--steps {steps} --warmup 1 --no-cpu-baseline --no-secondary")
    cmd_sec = ("rocprofv3 --kernel-trace --stats --output-format csv -d <OUT2> -o run -- python -u bench.py "
               "--steps 2 --warmup 1 --no-cpu-baseline")
    summ = f"python bench.py --trace-summary <OUT> <OUT2>{'' if steps == 5 else f' --trace-steps {steps}'}"
    lines = ["Kernel durations, D=100, N=2^18 (bench step: 8 formulas, split path then FP64 path)", "",
             "commands (repository root):", "  " + cmd_head, "  " + summ,
             f"source: <OUT>/run_kernel_trace.csv: per kernel the last {2 * steps} dispatches ({steps} timed steps back",
             f"to back, then {steps} steps with each launch between two HIP events, as bench.py times them); the",
             "autotuner's trial launches and the warmup come before them and are not counted.",
             "k_eval_resident<path, family, rotated, vec>: path 0 = split BF16x3, 3 = split BF16x6, 2 = FP64;",
             "families 0 weighted sphere, 5 Griewank, 6 Rastrigin, 9 Rosenbrock, 10 Schwefel, 13 Ackley.", "",
             f"{'kernel':28s} {'path':9s} {'family':11s} {'rot':>3s} {'calls':>5s} {'avg us':>8s} {'min us':>8s} {'max us':>8s}"]
    per = {}
    for r in dispatches(headline_dir):
        k = short(r["Kernel_Name"])
        if k and k.startswith("k_eval_resident<"):
            per.setdefault(k, []).append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
    rows = []
    for k, durs in per.items():
        d = durs[-2 * steps:]
        pth, fam, rot, _ = (int(v) for v in k[len("k_eval_resident<"):-1].split(","))
        rows.append((float(np.mean(d)), k, pth, fam, rot, len(d), min(d), max(d)))
    for avg, k, pth, fam, rot, calls, mn, mx in sorted(rows, reverse=True):
        lines.append(f"{k:28s} {PATH_NAME[pth]:9s} {FAMILY.get(fam, str(fam)):11s} {rot:3d} {calls:5d} "
                     f"{avg:8.2f} {mn:8.2f} {mx:8.2f}")
    with open(os.path.join(ROOT, "profiles", "resident_d100_n262144_kernel_trace.txt"), "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines))
    lines = ["Kernel durations of the secondary workloads (bench.py --steps 2): D=1000 N=2^18 eight formulas,",
             "hybrid and composition at D=1000 N=16384, the 64-population batch (tuning included), 50-row",
             "latency calls, DE generations; the D=100 resident kernels of the headline step as well.", "",
             "commands (repository root):", "  " + cmd_sec, "  " + summ,
             "source: <OUT2>/run_kernel_stats.csv; every launch of the run is counted (calls include warmups and tuning).",
             "", f"{'kernel':60s} {'calls':>7s} {'avg us':>9s} {'total ms':>9s}"]
    agg = {}
    for r in stats(secondary_dir):
        k = short(r["Name"]) or r["Name"][:60]
        a = agg.setdefault(k, [0, 0.0])
        a[0] += int(r["Calls"])
        a[1] += float(r["TotalDurationNs"])
    for k, (calls, tot) in sorted(agg.items(), key=lambda kv: -kv[1][1]):
        lines.append(f"{k[:60]:60s} {calls:7d} {tot / calls / 1e3:9.2f} {tot / 1e6:9.3f}")
    with open(os.path.join(ROOT, "profiles", "secondary_kernel_trace.txt"), "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines[:12]))


def sq_summary(p1_dir: str, p2_dir: str) -> None:
    """Per-kernel SQ instruction and busy counters of the D=100 resident kernels from two
    rocprofv3 --pmc runs of the headline step; writes profiles/counters_d100_n262144.txt."""
    vals = {}
    for d in (p1_dir, p2_dir):
        for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
            for row in csv.DictReader(open(f)):
                m = (re.search(r"k_eval_resident<(\d+), (\d+), (\d+), (\d+)>", row["Kernel_Name"])
                     or re.search(r"k_eval_residentILi(\d+)ELi(\d+)ELi(\d+)ELi(\d+)E", row["Kernel_Name"]))
                if not m:
                    continue
                key = "k_eval_resident<{},{},{},{}>".format(*m.groups())
                vals.setdefault(key, {}).setdefault(row["Counter_Name"], []).append(float(row["Counter_Value"]))
    simds, xcds = 1024, 8
    groups = N // 16  # 16-row groups per launch
    lines = ["SQ counters of the D=100 resident kernels, N=2^18 (rocprofv3 --pmc, two runs of the headline step)", "",
             "commands (repository root):",
             "  rocprofv3 --pmc SQ_WAVES SQ_BUSY_CYCLES SQ_WAVE_CYCLES SQ_INSTS_VALU SQ_ACTIVE_INST_VALU SQ_INSTS_LDS "
             "SQ_INSTS_SALU SQ_LDS_BANK_CONFLICT GRBM_GUI_ACTIVE --output-format csv -d <P1> -- python -u bench.py "
             "--steps 2 --warmup 1 --no-cpu-baseline --no-secondary",
             "  rocprofv3 --pmc SQ_INSTS_MFMA SQ_VALU_MFMA_BUSY_CYCLES SQ_WAIT_ANY SQ_ACTIVE_INST_ANY SQ_INSTS_VMEM_RD "
             "SQ_WAIT_INST_LDS SQ_INSTS_VALU_TRANS_F32 GRBM_GUI_ACTIVE --output-format csv -d <P2> -- python -u bench.py "
             "--steps 2 --warmup 1 --no-cpu-baseline --no-secondary",
             "  python bench.py --sq-summary <P1> <P2>", "",
             "Per 16-row group (one wave iteration): wave-level instruction counts.  cycles: GRBM_GUI_ACTIVE / 8",
             "XCDs (the launch under the profiler).  MFMA%: SQ_VALU_MFMA_BUSY_CYCLES / (1024 SIMDs x cycles).",
             "VALU%: issue time of the VALU instructions at 2 cycles each plus 14 more per transcendental, per",
             "SIMD, over cycles (a floor: dependent issue is slower).  LDS conflict: SQ_LDS_BANK_CONFLICT / 256 CUs",
             "over cycles.  wait%: SQ_WAIT_ANY / SQ_WAVE_CYCLES (both quad-cycles).", "",
             f"{'kernel':28s} {'VALU':>6s} {'trans':>6s} {'SALU':>6s} {'LDS':>5s} {'MFMA':>5s} {'cycles':>8s} "
             f"{'MFMA%':>6s} {'VALU%':>6s} {'LDScf%':>6s} {'wait%':>6s}"]
    for key in sorted(vals):
        v = {c: float(np.median(x[1:] if len(x) > 1 else x)) for c, x in vals[key].items()}
        cyc = v.get("GRBM_GUI_ACTIVE", 0.0) / xcds
        if cyc <= 0:
            continue
        per = lambda c: v.get(c, 0.0) / groups
        valu_cyc = (2.0 * v.get("SQ_INSTS_VALU", 0.0) + 14.0 * v.get("SQ_INSTS_VALU_TRANS_F32", 0.0)) / simds
        lines.append(f"{key:28s} {per('SQ_INSTS_VALU'):6.0f} {per('SQ_INSTS_VALU_TRANS_F32'):6.1f} "
                     f"{per('SQ_INSTS_SALU'):6.0f} {per('SQ_INSTS_LDS'):5.0f} {per('SQ_INSTS_MFMA'):5.0f} {cyc:8.0f} "
                     f"{100 * v.get('SQ_VALU_MFMA_BUSY_CYCLES', 0.0) / (simds * cyc):6.1f} {100 * valu_cyc / cyc:6.1f} "
                     f"{100 * v.get('SQ_LDS_BANK_CONFLICT', 0.0) / 256 / cyc:6.1f} "
                     f"{100 * v.get('SQ_WAIT_ANY', 0.0) / max(v.get('SQ_WAVE_CYCLES', 1.0), 1.0):6.1f}")
    with open(os.path.join(ROOT, "profiles", "counters_d100_n262144.txt"), "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines))


PROFILE_ROWS = 1 << 16  # one pass of the tiled path


PROFILE_PHASES = ["formulas", "hybrid", "composition", "fp32 mode", "copy probe"]


def profile_d1000(torch, c, reps: int = 3) -> None:
    """The D = 1000 workloads alone, for rocprofv3 runs: the eight formulas on one 65536-row
    pass (default split mode), the hybrid and the composition at N = 16384, rotated Rastrigin
    and Rosenbrock in the FP32-MFMA mode (the tiled kernels), `reps` launches each, then the copy
    probe (torch.neg over the 65536-row population) that scales the byte counters.  A one-element
    torch.abs marks the end of each phase in the dispatch sequence."""
    from paper_1407_7737_amd.inputs import composition_params, hybrid_params, population
    d, n, m = 1000, PROFILE_ROWS, 16384
    c.initialize(d, n, 0)
    marker = torch.zeros(1, device="cuda")
    try:
        x = torch.from_numpy(population(n, d, seed=0, dtype=np.float32)).cuda()
        o = torch.empty(n, dtype=torch.float32, device="cuda")
        for fid in FIDS:
            for _ in range(reps):
                c.func_evaluatef(fid, x, out=o)
        torch.abs(marker)
        bases, props = hybrid_params(d, seed=0)
        c.define_hybrid(100, bases, props)
        cb, sig, lam, bias = composition_params(seed=0)
        c.define_composition(101, cb, sig, lam, bias)
        for pid in (100, 101):
            for _ in range(reps):
                c.func_evaluatef(pid, x[:m], out=o[:m])
            torch.abs(marker)
        c.set_mode(c.MODE_FP32)
        for fid in (11, 14):
            for _ in range(reps):
                c.func_evaluatef(fid, x, out=o)
        c.set_mode(c.MODE_SPLIT)
        torch.abs(marker)
        torch.cuda.synchronize()
        buf = torch.empty_like(x)
        for _ in range(reps):
            torch.neg(x, out=buf)
        torch.cuda.synchronize()
    finally:
        c.dispose()
    print(json.dumps({"profiled": "d1000", "rows": n, "reps": reps}), flush=True)


def tiled_summary(trace_dir: str, fetch_dir: str, write_dir: str, sq1_dir: str, sq2_dir: str) -> None:
    """Per-kernel durations, HBM traffic and SQ counters of the D = 1000 workloads from five
    rocprofv3 runs of `bench.py --profile-d1000`; writes profiles/tiled_d1000_kernels.txt.  The
    dispatches of each run are taken in order and labelled by workload (the eight formulas,
    three launches each, then the hybrid, then the composition, then the copy probe), so the
    component launches of the composition are not mixed with the formulas' launches."""
    def short(name):
        m = re.search(r"(k_\w+)<([^>]*)>", name)
        if m:
            return m.group(1) + "<" + m.group(2).replace(" ", "") + ">"
        m = re.search(r"(k_\w+)ILi(-?\d+)ELi(-?\d+)E", name) or re.search(r"(k_\w+)ILi(-?\d+)E", name)
        if m:
            return m.group(1) + "<" + ",".join(m.groups()[1:]) + ">"
        m = re.search(r"(k_\w+)", name)
        if m:
            return m.group(1)
        low = name.lower()
        return "neg" if "neg" in low else ("marker" if "abs" in low else None)

    def label(seq):
        """Workload label per dispatch: phases end at the torch.abs markers profile_d1000 puts
        between them; in the first phase each formula has its three launches, in FIDS order."""
        out, phase, k = [], 0, 0
        for name in seq:
            if name == "marker":
                out.append(None)
                phase += 1
                continue
            if phase == 0:
                out.append(NAMES[FIDS[min(k // 3, len(FIDS) - 1)]])
                k += 1
            else:
                out.append(PROFILE_PHASES[min(phase, len(PROFILE_PHASES) - 1)])
        return out

    def dispatches(d, with_counters):
        rows = {}
        pat = "*counter_collection.csv" if with_counters else "*kernel_trace.csv"
        for f in glob.glob(os.path.join(d, "**", pat), recursive=True):
            for r in csv.DictReader(open(f)):
                k = short(r["Kernel_Name"])
                if not k:
                    continue
                e = rows.setdefault(int(r["Dispatch_Id"]), {"kernel": k})
                if with_counters:
                    e[r["Counter_Name"]] = e.get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
                else:
                    e["us"] = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3
        seq = [rows[i] for i in sorted(rows)]
        for e, lab in zip(seq, label([e["kernel"] for e in seq])):
            e["workload"] = lab
        return [e for e in seq if e["workload"] is not None]

    groups = {}
    for d, wc in ((trace_dir, False), (fetch_dir, True), (write_dir, True), (sq1_dir, True), (sq2_dir, True)):
        for e in dispatches(d, wc):
            g = groups.setdefault((e["workload"], e["kernel"]), {})
            for cn, v in e.items():
                if cn not in ("kernel", "workload"):
                    g.setdefault(cn, []).append(v)
    med = {k: {cn: float(np.median(v)) for cn, v in cs.items()} for k, cs in groups.items()}
    probe = PROFILE_ROWS * 1000 * 4
    neg = med[("copy probe", "neg")]
    cf = probe / (neg["FETCH_SIZE"] * 1024.0)
    cw = probe / (neg["WRITE_SIZE"] * 1024.0)
    simds, xcds = 1024, 8
    lines = ["D=1000 workloads: per-kernel duration, HBM traffic and SQ counters (rocprofv3, five runs)", "",
             "commands (repository root):",
             "  rocprofv3 --kernel-trace --stats --output-format csv -d <T> -o run -- python -u bench.py --profile-d1000",
             "  rocprofv3 --pmc FETCH_SIZE --output-format csv -d <F> -- python -u bench.py --profile-d1000",
             "  rocprofv3 --pmc WRITE_SIZE --output-format csv -d <W> -- python -u bench.py --profile-d1000",
             "  rocprofv3 --pmc SQ_WAVES SQ_BUSY_CYCLES SQ_WAVE_CYCLES SQ_INSTS_VALU SQ_INSTS_LDS SQ_INSTS_SALU "
             "SQ_LDS_BANK_CONFLICT GRBM_GUI_ACTIVE --output-format csv -d <S1> -- python -u bench.py --profile-d1000",
             "  rocprofv3 --pmc SQ_INSTS_MFMA SQ_VALU_MFMA_BUSY_CYCLES SQ_WAIT_ANY SQ_ACTIVE_INST_ANY SQ_INSTS_VMEM_RD "
             "SQ_WAIT_INST_LDS GRBM_GUI_ACTIVE --output-format csv -d <S2> -- python -u bench.py --profile-d1000",
             "  python bench.py --tiled-summary <T> <F> <W> <S1> <S2>", "",
             "Workload: the eight formulas on one 65536-row pass at D=1000 (default split mode), 3 launches each;",
             "the hybrid and the composition (one launch per component plus the blend) at N=16384, 3 calls each;",
             "rotated Rastrigin and Rosenbrock in the FP32-MFMA mode (pack, tiled GEMM, finalize), 3 calls each.",
             f"Bytes: FETCH_SIZE/WRITE_SIZE (KiB per dispatch, summed over dies) scaled by the copy probe (torch.neg",
             f"of {probe} bytes read and written): fetch x{cf:.3f}, write x{cw:.3f}.  Algorithmic bytes per",
             "65536-row pass: X read once, 262.1 MB, plus 0.26 MB written (N=16384: 65.5 MB).  A read below the",
             "algorithmic figure is X partly served from the MALL (the three launches read the same rows).",
             "MFMA%: SQ_VALU_MFMA_BUSY_CYCLES / (1024 SIMDs x GRBM_GUI_ACTIVE/8).  Per-wave counts: per launch.", "",
             f"{'workload':12s} {'kernel':18s} {'n':>3s} {'avg us':>8s} {'read MB':>8s} {'write MB':>8s} {'MFMA%':>6s} "
             f"{'VALU/wave':>9s} {'LDS/wave':>8s} {'LDScf%':>6s} {'wait%':>6s}"]
    order = {n: i for i, n in enumerate([NAMES[f] for f in FIDS] + PROFILE_PHASES[1:])}
    for (wl, k) in sorted(med, key=lambda t: (order.get(t[0], 99), t[1])):
        v = med[(wl, k)]
        n = len(groups[(wl, k)].get("us", []))
        cyc = v.get("GRBM_GUI_ACTIVE", 0.0) / xcds
        waves = max(v.get("SQ_WAVES", 1.0), 1.0)
        rd = v.get("FETCH_SIZE", float("nan")) * 1024 * cf / 1e6
        wr = v.get("WRITE_SIZE", float("nan")) * 1024 * cw / 1e6
        mf = 100 * v.get("SQ_VALU_MFMA_BUSY_CYCLES", 0.0) / (simds * cyc) if cyc > 0 else float("nan")
        lc = 100 * v.get("SQ_LDS_BANK_CONFLICT", 0.0) / 256 / cyc if cyc > 0 else float("nan")
        wt = 100 * v.get("SQ_WAIT_ANY", 0.0) / max(v.get("SQ_WAVE_CYCLES", 1.0), 1.0)
        lines.append(f"{wl[:12]:12s} {k[:18]:18s} {n:3d} {v.get('us', float('nan')):8.2f} {rd:8.1f} {wr:8.1f} {mf:6.1f} "
                     f"{v.get('SQ_INSTS_VALU', 0.0) / waves:9.0f} {v.get('SQ_INSTS_LDS', 0.0) / waves:8.0f} "
                     f"{lc:6.1f} {wt:6.1f}")
    with open(os.path.join(ROOT, "profiles", "tiled_d1000_kernels.txt"), "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-secondary", action="store_true")
    ap.add_argument("--copy-probe", action="store_true")
    ap.add_argument("--no-tune", action="store_true", help="keep the built-in launch-shape heuristic")
    ap.add_argument("--pmc-summary", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"))
    ap.add_argument("--trace-summary", nargs=2, metavar=("HEADLINE_DIR", "SECONDARY_DIR"))
    ap.add_argument("--trace-steps", type=int, default=5, help="--steps of the profiled headline run")
    ap.add_argument("--sq-summary", nargs=2, metavar=("P1_DIR", "P2_DIR"))
    ap.add_argument("--profile-d1000", action="store_true", help="run only the D=1000 workloads (for rocprofv3)")
    ap.add_argument("--tiled-summary", nargs=5, metavar=("TRACE", "FETCH", "WRITE", "SQ1", "SQ2"))
    args = ap.parse_args()
    if args.tiled_summary:
        tiled_summary(*args.tiled_summary)
        return
    if args.pmc_summary:
        pmc_summary(*args.pmc_summary)
        return
    if args.trace_summary:
        trace_summary("all", *args.trace_summary, steps=args.trace_steps)
        return
    if args.sq_summary:
        sq_summary(*args.sq_summary)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only: the population shards by rows "
                                   "with no exchange, so N GPUs would each run this same single-GPU workload"}))
        sys.exit(2)

    import torch

    import paper_1407_7737_amd as c
    from paper_1407_7737_amd.inputs import population

    assert torch.cuda.is_available(), "bench needs a GPU"
    if args.profile_d1000:
        profile_d1000(torch, c)
        return
    dev = torch.device("cuda:0")
    x32h = population(N, DIM, seed=0, dtype=np.float32)
    x32 = torch.from_numpy(x32h).to(dev)
    x64 = x32.double()
    outs32 = {fid: torch.empty(N, dtype=torch.float32, device=dev) for fid in FIDS}
    outs64 = {fid: torch.empty(N, dtype=torch.float64, device=dev) for fid in FIDS}
    c.initialize(DIM, N, 0)
    stream = torch.cuda.current_stream()
    # launch shapes from the autotuner (every candidate timed on the bench's own buffers; the
    # search log goes into the result line)
    tuning = {}
    if not args.no_tune:
        progress("autotuning the launch shapes")
        for fid in FIDS:
            t = c.tune(fid, x32, fp64=False, reps=5)
            t64 = c.tune(fid, x64, fp64=True, reps=3)
            tuning[NAMES[fid]] = {"split": t, "fp64": t64}

    def step(fp64: bool, events=None):
        for fid in FIDS:
            if events is not None:
                events[fid][0].record(stream)
            if fp64:
                c.func_evaluate(fid, x64, out=outs64[fid])
            else:
                c.func_evaluatef(fid, x32, out=outs32[fid])
            if events is not None:
                events[fid][1].record(stream)

    def timed(fp64: bool):
        for _ in range(args.warmup):
            step(fp64)
        torch.cuda.synchronize()
        # the timed steps: the eight launches back to back, nothing else on the stream
        t0 = time.perf_counter()
        for _ in range(args.steps):
            step(fp64)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        # per-launch durations: the same steps again, each launch between two HIP events on the
        # stream it runs on (an event pair serialises the launches around it, so these are the
        # isolated kernel times a kernel trace reports, slightly above their share of the step)
        ev = {fid: [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
                    for _ in range(args.steps)] for fid in FIDS}
        torch.cuda.synchronize()
        for k in range(args.steps):
            step(fp64, {fid: ev[fid][k] for fid in FIDS})
        torch.cuda.synchronize()
        per = {fid: float(np.mean([a.elapsed_time(b) for a, b in ev[fid]])) for fid in FIDS}
        return wall, per

    progress("timing the split path")
    wall32, per32 = timed(False)
    progress("timing the FP64 path")
    wall64, per64 = timed(True)
    # the plain FP32 mode (FP32 matrix products) on the same points, per formula
    c.set_mode(c.MODE_FP32)
    plain32 = {fid: event_time_ms(torch, lambda: c.func_evaluatef(fid, x32, out=outs32[fid]), 10) for fid in FIDS}
    c.set_mode(c.MODE_SPLIT)
    torch.cuda.synchronize()
    # measured peaks beside the nominal ones: streaming reads of the FP32 population, and the
    # dense BF16 matrix-core rate
    meas = {"hbm_read_gbs": c.probe_read_gbs(x32), "mfma_bf16_tflops": c.probe_mfma_bf16_tflops(),
            "how": "curob_probe_read over the 104.9 MB FP32 population (read only), curob_probe_mfma_bf16 "
                   "(four 16x16x32 chains per wave, four waves per SIMD); fastest of the timed launches"}
    c.dispose()
    if args.copy_probe:
        # a plain streaming kernel of known traffic (reads and writes the FP32 population once),
        # for scaling the HBM byte counters; negation gives it a name found nowhere else
        buf = torch.empty_like(x32)
        for _ in range(3):
            torch.neg(x32, out=buf)
        torch.cuda.synchronize()
        del buf

    ms32 = wall32 / args.steps * 1e3
    ms64 = wall64 / args.steps * 1e3
    evals = N * len(FIDS)
    value = evals * args.steps / wall32
    bytes32 = N * (DIM * 4 + 4)
    bytes64 = N * (DIM * 8 + 8)
    dom = max(FIDS, key=lambda f: per32[f])
    ach = bytes32 / (per32[dom] * 1e-3) / 1e9
    traffic = measured_traffic(dom)
    per_fn = {NAMES[f]: {"split_ms": round(per32[f], 5), "fp64_ms": round(per64[f], 5),
                         "fp32_plain_ms": round(plain32[f], 5),
                         "split_evals_per_s": N / (per32[f] * 1e-3), "fp64_evals_per_s": N / (per64[f] * 1e-3),
                         "fp32_plain_evals_per_s": N / (plain32[f] * 1e-3),
                         "split_hbm_frac": bytes32 / (per32[f] * 1e-3) / 1e9 / HBM_PEAK_GBS,
                         "fp64_hbm_frac": bytes64 / (per64[f] * 1e-3) / 1e9 / HBM_PEAK_GBS,
                         "fp32_plain_hbm_frac": bytes32 / (plain32[f] * 1e-3) / 1e9 / HBM_PEAK_GBS,
                         "kernel": resident_key(f)} for f in FIDS}
    res = {
        "metric": "evals/sec at D=100,N=2^18: split-BF16 MFMA vs FP64 path; % of roofline",
        "value": value,
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms32,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "D=100, N=2^18 rows uniform in [-100,100]^D, 8 formulas "
                               "(sphere, elliptic, Griewank, Rastrigin_U, Rastrigin, Rosenbrock, Schwefel, Ackley), "
                               "func_evaluatef default split-BF16 mode",
                   "dim": DIM, "rows": N, "functions": len(FIDS)},
        "roofline": {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": ach / HBM_PEAK_GBS, "traffic": traffic, "kernel": resident_key(dom),
                     "function": NAMES[dom], "algorithmic_bytes_per_launch": bytes32,
                     "avg_launch_ms": per32[dom], "measured_peak": meas,
                     "frac_of_measured_read": ach / meas["hbm_read_gbs"]},
        "fp64_path": {"value": evals * args.steps / wall64, "unit": "evals/s", "ms_per_step": ms64,
                      "split_over_fp64": (evals * args.steps / wall32) / (evals * args.steps / wall64)},
        "per_function": per_fn,
        "autotune": tuning,
        "paper_context": PAPER_CONTEXT,
    }
    if not args.no_secondary:
        progress("secondary workloads")
        res["secondary"] = secondary(torch, c)
    if not args.no_cpu_baseline:
        gpu = {fid: (outs32[fid].cpu().numpy(), outs64[fid].cpu().numpy()) for fid in FIDS}
        progress("CPU oracle baseline")
        res["cpu_baseline"] = cpu_baseline(x32h, gpu)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
