"""Benchmark of the batched HMM micro-problem solve on one MI355X.

Workload (default): 1024 micro boxes of 64x64 points, one per node of a 32x32
macro grid, eps = 1/200, mu = mu' = 3 eps, eta = eps^2, alpha = 0.1 (RK4P,
517 steps), a = 1 + 0.5 sin(2 pi x1/eps) sin(2 pi x2/eps), Q_[4] initial data
from a seeded Gaussian random macro field, averaged field.  One "step" is one
llhmm_micro_batch + llhmm_upscale over the whole batch (all boxes, all time
steps); inputs are resident in HBM before timing.

Printed: one JSON line.  `value` is FP32 micro cell-steps/s (cell-step = one
grid point advanced one full time step); the FP64 path is timed on the same
batch and reported beside it, with p50/p99 batch latency, the roofline of the
dominant kernel and the oracle timed on the host cores.
"""
from __future__ import annotations

import argparse
import json
import os
import statistics
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32 = 157.3e12   # MI355X vector FP32 (packed), published
PEAK_FP64 = 78.6e12    # MI355X vector FP64, published

# Sources that define the time-stepping kernel: HBM traffic measured with PMC
# counters is reported only while these are unchanged since the measurement.
KERNEL_SOURCES = ["paper_2108_09463_amd/csrc/llhmm_micro_impl.h",
                  "paper_2108_09463_amd/csrc/llhmm_internal.h",
                  "paper_2108_09463_amd/csrc/llhmm_tiles.h",
                  "paper_2108_09463_amd/csrc/llhmm_tiles_f32_2d.hip",
                  "paper_2108_09463_amd/csrc/llhmm_tiles_f64_2d.hip",
                  "paper_2108_09463_amd/build.py"]
TRAFFIC_FILES = {"fp32": "profiles/k_micro_f32_two_d_batch_traffic.txt",
                 "fp64": "profiles/k_micro_f64_two_d_batch_traffic.txt"}


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(name):
    """HBM bytes per launch of the time-stepping kernel from the committed PMC
    summary, or None when absent or taken on other kernel sources."""
    path = os.path.join(ROOT, TRAFFIC_FILES[name])
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if ":" in line and not line.startswith(" "):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    if kv.get("kernel_sources_sha256_16") != kernel_source_hash():
        return None
    try:
        return float(kv["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def copy_calibration(nbytes=1 << 30, reps=3):
    """A plain device-to-device copy of known size, for scaling the PMC
    FETCH_SIZE / WRITE_SIZE counters to bytes (run under rocprofv3 --pmc)."""
    import torch
    src = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    src.fill_(1)
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes": nbytes, "reps": reps}), flush=True)


def flops_per_cell_step(dim, order, integ):
    """Algorithmic flops per cell-step (FMA = 2): per stage the field
    3(4d-1) (order 2) or 3(10d-1) (order 4) and the right-hand side 24; HeunP adds
    stage input, combination, projection and averaging (2H + 77), RK4P (4H + 149)."""
    h = 3 * (4 * dim - 1) if order == 2 else 3 * (10 * dim - 1)
    return 2 * h + 77 if integ == 1 else 4 * h + 149


def time_batch(prep, steps, warmup):
    """Times `steps` whole steps (set-up + time stepping + upscale) with torch
    events on the launch stream; separately, the library's own HIP events on the
    same stream give the set-up and time-stepping kernels' durations per step."""
    import torch
    from paper_2108_09463_amd import llhmm as L
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        prep.launch()
    torch.cuda.synchronize()
    prep.batch.set_timing(True)
    lat = []
    t0 = time.perf_counter()
    start_all = torch.cuda.Event(enable_timing=True)
    end_all = torch.cuda.Event(enable_timing=True)
    start_all.record(stream)
    for _ in range(steps):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(stream)
        prep.launch()
        b.record(stream)
        lat.append((a, b))
    end_all.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kept = min(steps, L.TIMING_SLOTS)
    phases = [prep.batch.timing(k) for k in range(kept)]
    prep.batch.set_timing(False)
    per = [x.elapsed_time(y) for x, y in lat]          # ms, micro solve + upscale
    total_ms = start_all.elapsed_time(end_all)
    return dict(ms_per_step=total_ms / steps, lat_ms=per, wall_s=wall,
                setup_ms=float(np.mean([p[0] for p in phases])),
                kernel_ms=float(np.mean([p[1] for p in phases])))


def pct(v, p):
    v = sorted(v)
    k = (len(v) - 1) * p / 100.0
    lo = int(np.floor(k))
    hi = min(lo + 1, len(v) - 1)
    return v[lo] + (v[hi] - v[lo]) * (k - lo)


def cpu_baseline(wl, sample, gpu_H=None):
    """The FP64 oracle on a bounded sample of the same boxes, threads = host cores."""
    from concurrent.futures import ThreadPoolExecutor
    from oracle import micro
    micro.build()
    # the host's share of cores (OMP_NUM_THREADS is set to it on the GPU hosts)
    cores = min(os.cpu_count() or 1, int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1)))
    idx = list(np.linspace(0, len(wl.boxes) - 1, sample).astype(int))

    def one(i):
        b = wl.boxes[i]
        return micro.solve_box(b, wl.coefs[b["coef_index"]], init_fn=wl.init_of(i), macro=wl.macro,
                               kernel=wl.kernel)

    t0 = time.perf_counter()
    with ThreadPoolExecutor(cores) as ex:
        res = list(ex.map(one, idx))
    dt = time.perf_counter() - t0
    cs = sum(r["M"] * wl.boxes[i]["n"] ** wl.boxes[i]["dim"] for r, i in zip(res, idx))
    out = dict(value=cs / dt, unit="cell-steps/s", cores=cores, kind="oracle",
               sample="%d of %d boxes (evenly spaced), FP64 C oracle, %d threads, %.1f s"
                      % (len(idx), len(wl.boxes), cores, dt))
    errs = {}
    if gpu_H is not None:
        Ho = np.stack([r["out"] for r in res])
        for k, H in gpu_H.items():
            Hg = H[idx, :Ho.shape[1]]
            e = np.linalg.norm(Hg - Ho, axis=1) / np.linalg.norm(Ho, axis=1)
            errs[k] = float(e.max())
    return out, errs


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle baseline")
    ap.add_argument("--cpu-sample", type=int, default=512)
    ap.add_argument("--precision", choices=["both", "fp32", "fp64"], default="both")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy (PMC counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the micro boxes shard across GPUs without "
              "communication, and multi-GPU runs are not part of this build", file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration()
        return

    import torch
    from paper_2108_09463_amd import inputs
    from paper_2108_09463_amd.runner import Prepared

    wl = inputs.two_d_batch()
    b0 = wl.boxes[0]
    res = {}
    gpu_H = {}
    precs = {"fp32": inputs.FP32, "fp64": inputs.FP64}
    if args.precision != "both":
        precs = {args.precision: precs[args.precision]}
    for name, prec in precs.items():
        prep = Prepared(wl, precision=prec)
        cs = prep.cell_steps()
        t = time_batch(prep, args.steps, args.warmup)
        torch.cuda.synchronize()
        gpu_H[name] = prep.H.cpu().numpy()
        integ = 2 if b0["alpha"] <= 0.2 else 1
        F = flops_per_cell_step(2, b0["order"], integ)
        rate = cs / (t["ms_per_step"] * 1e-3)
        # roofline of the time-stepping kernel: algorithmic flops per launch
        # (F x cell-steps of the batch) over its own event-timed duration
        achieved = F * cs / (t["kernel_ms"] * 1e-3)
        peak = PEAK_FP32 if prec == inputs.FP32 else PEAK_FP64
        res[name] = dict(cell_steps=cs, ms_per_step=t["ms_per_step"], rate=rate,
                         p50_ms=pct(t["lat_ms"], 50), p99_ms=pct(t["lat_ms"], 99),
                         setup_ms=t["setup_ms"], kernel_ms=t["kernel_ms"],
                         roofline=dict(bound="alu", achieved=achieved / 1e12, peak=peak / 1e12,
                                       unit="TFLOP/s", frac=achieved / peak,
                                       traffic=measured_traffic(name),
                                       kernel="k_micro (time stepping)",
                                       kernel_ms=t["kernel_ms"], flops_per_cell_step=F,
                                       flops_per_launch=F * cs))
        del prep
    cpu = None
    errs = {}
    if not args.no_cpu:
        cpu, errs = cpu_baseline(wl, args.cpu_sample, gpu_H)
    head = "fp32" if "fp32" in res else "fp64"
    r = res[head]
    line = {
        "metric": "micro cell-steps/s FP32 vs FP64 at stated error; p50/p99 micro-batch latency",
        "value": r["rate"],
        "unit": "cell-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if head == "fp32" else "f64",
        "data": "synthetic",
        "config": {"workload": "two_d_batch: 1024 boxes of 64x64 (32x32 macro grid), eps=1/200, "
                               "mu=mu'=3eps, eta=eps^2, alpha=0.1 RK4P (517 steps), order-2 stencil, "
                               "Q4 macro init, field average",
                   "boxes": len(wl.boxes), "cell_steps_per_step": r["cell_steps"]},
        "roofline": r["roofline"],
        "latency_ms": {"p50": r["p50_ms"], "p99": r["p99_ms"]},
        "phase_ms": {"setup": r["setup_ms"], "time_stepping": r["kernel_ms"]},
        "cpu_baseline": cpu,
        "max_rel_err_vs_oracle": errs,
    }
    if "fp64" in res and head == "fp32":
        f = res["fp64"]
        line["fp64"] = {"value": f["rate"], "ms_per_step": f["ms_per_step"],
                        "latency_ms": {"p50": f["p50_ms"], "p99": f["p99_ms"]},
                        "phase_ms": {"setup": f["setup_ms"], "time_stepping": f["kernel_ms"]},
                        "roofline": f["roofline"]}
        line["speedup_fp32_vs_fp64"] = r["rate"] / f["rate"]
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
