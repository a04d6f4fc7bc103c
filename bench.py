"""Throughput benchmark: evaluations/s at D = 100, N = 2^18 on one MI355X.

One step evaluates the population of N = 2^18 candidate vectors (uniform in [-100, 100]^100,
resident in HBM) on the eight rotated/unrotated formulas {sphere, elliptic, Griewank,
shifted Rastrigin, rotated Rastrigin, Rosenbrock, rotated Schwefel, Ackley} through
func_evaluatef (default split-BF16 mode).  The FP64 path (func_evaluate) is timed on the same
points for comparison.  Kernel durations come from HIP events recorded on the library stream
around every launch of the timed region; the roofline figure uses the algorithmic bytes of
the dominant kernel (D*4 bytes read + 4 bytes written per row).

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
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
HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_d100_n262144.json")
KERNEL_SOURCES = ["eval_resident.h", "formulas.h", "devprob.h", "kernels.h"]


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1407_7737_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel_name: str, launch_bytes: float):
    """HBM bytes per launch from the committed rocprofv3 counter summary, or None when the
    kernel sources changed since the counters were taken."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_source_hash") != kernel_source_hash():
        return None
    k = t.get("kernels", {}).get(kernel_name)
    return None if k is None else k.get("hbm_bytes_per_launch")


def cpu_baseline(x32: np.ndarray, budget_s: float = 12.0):
    """The oracle as it stands, on the host cores, on a bounded sample of the same rows: chunks
    of the population (wrapping around) on all measured formulas until about budget_s seconds
    of CPU work have been timed."""
    import oracle
    threads = max(1, min(os.cpu_count() or 1, oracle.threads_available(), 16))
    probs = {fid: oracle.basic(fid, DIM, 0) for fid in FIDS}
    chunk = 4096
    total_rows, t_total, start = 0, 0.0, 0
    while t_total < budget_s:
        idx = (start + np.arange(chunk)) % N
        sample = x32[idx].astype(np.float64)
        t0 = time.perf_counter()
        for fid in FIDS:
            probs[fid](sample, threads=threads)
        t_total += time.perf_counter() - t0
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
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only: the population shards by rows "
                                   "with no exchange, so N GPUs would each run this same single-GPU workload"}))
        sys.exit(2)

    import torch

    import paper_1407_7737_amd as c
    from paper_1407_7737_amd.inputs import population

    assert torch.cuda.is_available(), "bench needs a GPU"
    dev = torch.device("cuda:0")
    x32h = population(N, DIM, seed=0, dtype=np.float32)
    x32 = torch.from_numpy(x32h).to(dev)
    x64 = x32.double()
    outs32 = {fid: torch.empty(N, dtype=torch.float32, device=dev) for fid in FIDS}
    outs64 = {fid: torch.empty(N, dtype=torch.float64, device=dev) for fid in FIDS}
    c.initialize(DIM, N, 0)
    stream = torch.cuda.current_stream()

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
        ev = {fid: [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
                    for _ in range(args.steps)] for fid in FIDS}
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(args.steps):
            step(fp64, {fid: ev[fid][k] for fid in FIDS})
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        per = {fid: float(np.mean([a.elapsed_time(b) for a, b in ev[fid]])) for fid in FIDS}
        return wall, per

    wall32, per32 = timed(False)
    wall64, per64 = timed(True)
    c.dispose()

    ms32 = wall32 / args.steps * 1e3
    ms64 = wall64 / args.steps * 1e3
    evals = N * len(FIDS)
    value = evals * args.steps / wall32
    bytes32 = N * (DIM * 4 + 4)
    bytes64 = N * (DIM * 8 + 8)
    dom = max(FIDS, key=lambda f: per32[f])
    ach = bytes32 / (per32[dom] * 1e-3) / 1e9
    kname = f"split:{NAMES[dom]}"
    traffic = measured_traffic(kname, bytes32)
    per_fn = {NAMES[f]: {"split_ms": round(per32[f], 5), "fp64_ms": round(per64[f], 5),
                         "split_evals_per_s": N / (per32[f] * 1e-3), "fp64_evals_per_s": N / (per64[f] * 1e-3),
                         "split_hbm_frac": bytes32 / (per32[f] * 1e-3) / 1e9 / HBM_PEAK_GBS,
                         "fp64_hbm_frac": bytes64 / (per64[f] * 1e-3) / 1e9 / HBM_PEAK_GBS} for f in FIDS}
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
                     "frac": ach / HBM_PEAK_GBS, "traffic": traffic, "kernel": kname},
        "fp64_path": {"value": evals * args.steps / wall64, "unit": "evals/s", "ms_per_step": ms64,
                      "split_over_fp64": (evals * args.steps / wall32) / (evals * args.steps / wall64)},
        "per_function": per_fn,
    }
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline(x32h)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
