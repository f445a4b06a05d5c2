"""Benchmark of the batched HMM micro-problem solve on one MI355X.

Headline workload (default): 1024 micro boxes of 64x64 points, one per node of
a 32x32 macro grid, eps = 1/200, mu = mu' = 3 eps, eta = eps^2, alpha = 0.1
(RK4P, 517 steps), a = 1 + 0.5 sin(2 pi x1/eps) sin(2 pi x2/eps), Q_[4]
initial data from a seeded Gaussian random macro field, averaged field.  One
"step" is one llhmm_micro_batch + llhmm_upscale over the whole batch (all
boxes, all time steps); inputs are resident in HBM before timing.

Printed: one JSON line.  `value` is FP32 micro cell-steps/s (cell-step = one
grid point advanced one full time step); the FP64 path is timed on the same
batch and reported beside it, with p50/p99 batch latency, the roofline of the
time-stepping kernel (from the library's HIP events on the launch stream), the
oracle timed on the host cores, and the 4096-box uneven FP32 batch (sizes 32
to 128, large boxes in slab mode) as a nested record.
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
PEAK_HBM = 8.0e12      # MI355X HBM3E bandwidth, published (bytes/s)

# Sources that define the time-stepping kernel: HBM traffic measured with PMC
# counters is reported only while these are unchanged since the measurement.
KERNEL_SOURCES = ["paper_2108_09463_amd/csrc/llhmm_micro_impl.h",
                  "paper_2108_09463_amd/csrc/llhmm_internal.h",
                  "paper_2108_09463_amd/csrc/llhmm_tiles.h",
                  "paper_2108_09463_amd/csrc/llhmm_tiles_f32_2d.hip",
                  "paper_2108_09463_amd/csrc/llhmm_tiles_f64_2d.hip",
                  "paper_2108_09463_amd/build.py"]
KERNEL_SOURCES_3D = ["paper_2108_09463_amd/csrc/llhmm_micro3d.hip",
                     "paper_2108_09463_amd/csrc/llhmm_micro3d.h",
                     "paper_2108_09463_amd/csrc/llhmm_internal.h",
                     "paper_2108_09463_amd/build.py"]
TRAFFIC_FILES = {"fp32": "profiles/k_micro_f32_two_d_batch_traffic.txt",
                 "fp64": "profiles/k_micro_f64_two_d_batch_traffic.txt",
                 "3d": "profiles/k_micro3d_three_d_batch_traffic.txt"}


def kernel_source_hash(sources=None):
    import hashlib
    h = hashlib.sha256()
    for f in sources or KERNEL_SOURCES:
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
    sources = KERNEL_SOURCES_3D if name == "3d" else KERNEL_SOURCES
    if kv.get("kernel_sources_sha256_16") != kernel_source_hash(sources):
        return None
    try:
        return float(kv["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


COUNTER_FILES = {"fp32": "profiles/k_micro_f32_two_d_batch_counters.txt",
                 "fp64": "profiles/k_micro_f64_two_d_batch_counters.txt"}


def measured_counters(name):
    """VALU issue rate (wave64 instructions per CU per clock) and LDS
    bank-conflict rate of the time-stepping kernel from the committed PMC
    summary, or None when absent or taken on other kernel sources."""
    path = os.path.join(ROOT, COUNTER_FILES[name])
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if ":" in line and not line.startswith(" "):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip().split()[0] if v.strip() else ""
    if kv.get("kernel_sources_sha256_16") != kernel_source_hash(KERNEL_SOURCES):
        return None
    try:
        return {"valu_issue_rate": float(kv["valu_issue_rate"]),
                "valu_busy": float(kv["valu_busy"]),
                "lds_bank_conflict_rate": float(kv["lds_bank_conflict_rate"]),
                "hardware_over_algorithmic_flops": float(kv["hardware_over_algorithmic"]),
                "source": COUNTER_FILES[name]}
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


def time_batch(prep, steps, warmup, graph=False):
    """Times `steps` whole steps (set-up + time stepping + upscale) with torch
    events on the launch stream; separately, the library's own HIP events on the
    same stream give the set-up and time-stepping kernels' durations per step."""
    import torch
    from paper_2108_09463_amd import llhmm as L
    stream = torch.cuda.current_stream()
    launch = prep.launch_graph if graph else prep.launch
    for _ in range(warmup):
        launch()
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
        launch()
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
    r1 = one(idx[0])                      # one box alone: the single-thread rate
    dt1 = time.perf_counter() - t0
    t0 = time.perf_counter()
    with ThreadPoolExecutor(cores) as ex:
        res = list(ex.map(one, idx))
    dt = time.perf_counter() - t0
    cs = sum(r["M"] * wl.boxes[i]["n"] ** wl.boxes[i]["dim"] for r, i in zip(res, idx))
    cs1 = r1["M"] * wl.boxes[idx[0]]["n"] ** wl.boxes[idx[0]]["dim"]
    out = dict(value=cs / dt, unit="cell-steps/s", cores=cores, kind="oracle",
               sample="%d of %d boxes (evenly spaced), FP64 C oracle, %d threads, %.1f s"
                      % (len(idx), len(wl.boxes), cores, dt),
               single_thread_value=cs1 / dt1)
    errs = {}
    if gpu_H is not None:
        Ho = np.stack([r["out"] for r in res])
        den = np.linalg.norm(Ho, axis=1)
        den = np.maximum(den, 1e-3 * np.median(den))     # per-box relative error (floor for tiny boxes)
        for k, H in gpu_H.items():
            Hg = H[idx, :Ho.shape[1]]
            errs[k] = float((np.linalg.norm(Hg - Ho, axis=1) / den).max())
    return out, errs


def algorithmic_flops(boxes):
    """Sum over boxes of F x M x n^d (algorithmic flops of one step of the whole batch)."""
    from paper_2108_09463_amd import llhmm as L
    M, _, integ = L.llhmm_plan(boxes)
    tot = 0
    for b, m, ig in zip(boxes, M, integ):
        tot += flops_per_cell_step(b["dim"], b["order"], int(ig)) * int(m) * b["n"] ** b["dim"]
    return float(tot)


def measure(wl, precision, steps, warmup, tune=False, graph=False):
    """Times one workload at one precision; returns rates, latencies and the
    roofline of the time-stepping phase.  tune: run the slab-mode autotuner
    first; graph: launch the whole solve as one captured HIP graph (the
    library's events then time the whole call as time stepping)."""
    import torch
    from paper_2108_09463_amd import inputs
    from paper_2108_09463_amd.runner import Prepared
    prep = Prepared(wl, precision=precision)
    cs = prep.cell_steps()
    flops = algorithmic_flops(prep.boxes)
    slabs = None
    if tune:
        sp, spe = prep.tune(reps=1)
        slabs = {int(b["n"]): dict(slabs=int(k), steps_per_exchange=int(e))
                 for b, k, e in zip(prep.boxes, sp, spe) if k}
    t = time_batch(prep, steps, warmup, graph=graph)
    torch.cuda.synchronize()
    H = prep.H.cpu().numpy()
    st = prep.status.cpu().numpy()
    del prep
    rate = cs / (t["ms_per_step"] * 1e-3)
    # roofline of the time-stepping phase: algorithmic flops of the batch over the
    # event-timed duration of its time-stepping launches
    achieved = flops / (t["kernel_ms"] * 1e-3)
    peak = PEAK_FP32 if precision == inputs.FP32 else PEAK_FP64
    name = "fp32" if precision == inputs.FP32 else "fp64"
    return dict(cell_steps=cs, ms_per_step=t["ms_per_step"], rate=rate, slabs=slabs,
                p50_ms=pct(t["lat_ms"], 50), p99_ms=pct(t["lat_ms"], 99),
                setup_ms=t["setup_ms"], kernel_ms=t["kernel_ms"], H=H, status_ok=bool((st == 0).all()),
                roofline=dict(bound="alu", achieved=achieved / 1e12, peak=peak / 1e12,
                              unit="TFLOP/s", frac=achieved / peak,
                              traffic=measured_traffic(name) if wl.name == "two_d_batch" else None,
                              counters=measured_counters(name) if wl.name == "two_d_batch" else None,
                              kernel="time-stepping kernels", kernel_ms=t["kernel_ms"],
                              flops_per_cell_step=flops / cs, flops_per_launch=flops))


def _served_mode(stages, arrival, gap_mean_s=0.0):
    """`stages` macro stages of the served run with one arrival mode; per-stage
    request-latency percentiles and the stage records' summary."""
    import torch
    from paper_2108_09463_amd.serve import ServedRun
    # bit 4 (unresolved final state) is counted, not fatal: the eps = 1/100 boxes
    # reach 3.84 dX from their node, where Q_[4] extrapolates, and as the macro
    # field evolves a few of them start from unresolved data
    run = ServedRun(n_macro=128, max_inflight=4, max_batch_boxes=2048, device_bytes=24 << 30, allow_status=4)
    recs = []
    k = 0
    step = 0
    while len(recs) < stages:
        stage = 0
        while len(recs) < stages:
            rec = run.stage(run.Y, k, arrival, gap_mean_s)
            k += 1
            stage = run.macro_stage(step, stage, rec)
            recs.append(rec)
            if stage == 0:
                break
        step += 1
    torch.cuda.synchronize()
    cell_steps = run.cell_steps
    run.close()
    st = np.array([r["stage_s"] for r in recs])
    p50 = [pct(list(r["latency_us"] * 1e-3), 50) for r in recs]
    p99 = [pct(list(r["latency_us"] * 1e-3), 99) for r in recs]
    bl = np.concatenate([np.array(r["burst_s"]) for r in recs]) * 1e3
    nb = np.array([len(r["bursts"]) for r in recs])
    return recs, {
        "arrival": arrival, "stages": len(recs), "value": cell_steps * len(recs) / st.sum(),
        "unit": "cell-steps/s",
        "request_latency_ms_per_stage": {"p50": p50, "p99": p99},
        "request_latency_ms": {"p50_median_over_stages": float(np.median(p50)),
                               "p99_max_over_stages": float(np.max(p99))},
        "burst_latency_ms": {"p50": pct(list(bl), 50), "p99": pct(list(bl), 99)},
        "stage_latency_ms": {"p50": pct(list(st * 1e3), 50), "p99": pct(list(st * 1e3), 99)},
        "burst_service_ms": float((st / nb).mean() * 1e3),
        "unresolved_requests_per_stage": [int(((r["status"] & 4) != 0).sum()) for r in recs],
        "status_ok": all(bool(((r["status"] & ~4) == 0).all()) for r in recs)}, cell_steps


def served(stages, with_cpu=False):
    """The served HMM run on a 128x128 macro grid: each macro stage issues
    16384 micro requests (n in {32..128}, eps in {1/100, 1/200, 1/400},
    alpha_micro = 1.2, HeunP, Q_[4] data), released in shuffled bursts of
    256-4096 into the request loop, in three arrival modes: saturating (back to
    back), open loop (exponential gaps of mean 0.8 x the saturating run's
    service time per burst) and closed loop (next burst after the previous
    one has completed, at most 4 stages).  The macro stage reads the averages
    where the micro-batches left them on the device."""
    recs, sat, cell_steps = _served_mode(stages, "saturating")
    gap = 0.8 * sat["burst_service_ms"] * 1e-3
    _, opn, _ = _served_mode(stages, "open", gap)
    opn["gap_mean_ms"] = gap * 1e3
    _, clo, _ = _served_mode(min(stages, 4), "closed")
    extra = {}
    if with_cpu:
        # first stage: requests at the initial macro field; oracle on a sample of them
        from paper_2108_09463_amd import inputs
        boxes, coefs = inputs.served_boxes(128)
        wl = inputs.Workload("served", 2, boxes, coefs, precision=inputs.FP32,
                             macro=dict(n=128, dX=1.0 / 128, x0=(0.0, 0.0), M=inputs.served_macro(128)))
        extra["cpu_baseline"], extra["max_rel_err_vs_oracle"] = cpu_baseline(wl, 32, {"fp32": recs[0]["H"]})
    return {"workload": "served: 128x128 macro grid (EX2 macro data), 16384 requests per macro stage, "
                        "n in {32,48,64,96,128}, eps in {1/100,1/200,1/400}, mu=mu'=3eps, eta=eps^2, "
                        "alpha_micro=1.2 HeunP, Q4 init, FP32; bursts of 256-4096; "
                        "4 micro-batch slots of up to 2048 requests; H_avg kept on the device",
            "stages": sat["stages"], "value": sat["value"], "unit": "cell-steps/s",
            "cell_steps_per_stage": cell_steps,
            "request_latency_ms": sat["request_latency_ms"],
            "stage_latency_ms": sat["stage_latency_ms"],
            "modes": {"saturating": sat, "open": opn, "closed": clo},
            "status_ok": sat["status_ok"] and opn["status_ok"] and clo["status_ok"], **extra}


WORKLOADS = {
    "two_d_batch": ("two_d_batch: 1024 boxes of 64x64 (32x32 macro grid), eps=1/200, mu=mu'=3eps, "
                    "eta=eps^2, alpha=0.1 RK4P (517 steps), order-2 stencil, Q4 macro init, field average"),
    "two_d_batch_o4": ("two_d_batch_o4: the 1024 boxes of 64x64 of two_d_batch with the fourth-order "
                       "conservative stencil (RK4P), field average"),
    "uneven_batch": ("uneven_batch: 4096 2-D boxes, n uniform over {32,48,64,96,128}, quasi-periodic a, "
                     "alpha ~ U[0.01,0.2] (RK4P), mu=mu'=3eps, eps=1/200, eta=eps^2, EX2 initial data, "
                     "field average"),
    "one_d_batch": ("one_d_batch: 16384 1-D boxes of 256 points, mu=mu'=4eps, eps=0.01, alpha=0.01 RK4P, "
                    "eta=eps^2, seeded phases, flux average"),
    "three_d_batch": ("three_d_batch: 512 3-D boxes of 32^3, eps=1/200, mu=mu'=3eps, eta=eps^2, "
                      "alpha=0.1 RK4P, periodic m - m_init, a = 1 + 0.5 sin sin sin, FP64, field average"),
    "three_d_batch_o4": ("three_d_batch_o4: the 512 3-D boxes of 32^3 of three_d_batch with the "
                         "fourth-order conservative stencil, FP64, field average"),
}
THREE_D = ("three_d_batch", "three_d_batch_o4")

# d = 3 kernel: bytes streamed through HBM per cell and stage (FP64): stage input
# read 24, face coefficients 24 (three unique faces per cell), state m read 24,
# Runge-Kutta sum read and written 48, next stage input written 24
# Boxes of the cpu_baseline sample per workload, sized for about 10-30 s on 16
# host threads (all 512 boxes of the d = 3 batch take about 41 s, all 1024 of
# the 2-D batch about 14 s).
DEFAULT_CPU_SAMPLE = {"three_d_batch": 256, "three_d_batch_o4": 128}

# Bytes per cell that one stage of the d = 3 time loop must move through HBM:
# read the stage input, the state and the running sum, write the running sum
# (the state at the last stage) and the next stage input, 24 bytes each; the
# first stage of a step has no running sum to read.
BYTES_PER_CELL_STAGE_3D = 120.0
BYTES_FIRST_STAGE_SAVING_3D = 24.0
# The fourth-order kernel also reads the three stored faces of each cell (24 bytes).
BYTES_FACES_3D_O4 = 24.0


def hbm_roofline_3d(boxes, kernel_ms):
    """Roofline of k_micro3d: streamed bytes per launch over its duration."""
    from paper_2108_09463_amd import llhmm as L
    M, _, integ = L.llhmm_plan(boxes)
    nbytes = 0.0
    for b, m, ig in zip(boxes, M, integ):
        stages = 4 if int(ig) == 2 else 2
        per_stage = BYTES_PER_CELL_STAGE_3D + (BYTES_FACES_3D_O4 if b["order"] == 4 else 0.0)
        nbytes += int(m) * b["n"] ** 3 * (stages * per_stage - BYTES_FIRST_STAGE_SAVING_3D)
    o4 = all(b["order"] == 4 for b in boxes)
    achieved = nbytes / (kernel_ms * 1e-3)
    return {"bound": "hbm", "achieved": achieved / 1e9, "peak": PEAK_HBM / 1e9, "unit": "GB/s",
            "frac": achieved / PEAK_HBM, "traffic": None if o4 else measured_traffic("3d"),
            "kernel": "k_micro3d_o4" if o4 else "k_micro3d",
            "kernel_ms": kernel_ms,
            "bytes_per_cell_stage": BYTES_PER_CELL_STAGE_3D + (BYTES_FACES_3D_O4 if o4 else 0.0),
            "bytes_per_launch": nbytes}


def three_d_roofline(r, boxes):
    """d = 3: the VALU roofline (algorithmic flops over the FP64 peak) is the
    primary figure; the bytes the kernel streams through HBM are the design's
    own choice, not the method's, and are reported beside it."""
    hbm = hbm_roofline_3d(boxes, r["kernel_ms"])
    roof = dict(r["roofline"])
    roof["kernel"] = hbm["kernel"]
    roof["traffic"] = None
    roof["streamed_hbm"] = hbm
    return roof


def three_d_record(steps, warmup, with_cpu):
    """The d = 3 batch in FP64 with its VALU roofline (and the streamed-HBM figure)."""
    from paper_2108_09463_amd import inputs
    w3 = inputs.three_d_batch()
    r = measure(w3, inputs.FP64, steps, warmup)
    rec = {"workload": WORKLOADS["three_d_batch"], "dtype": "f64", "value": r["rate"],
           "unit": "cell-steps/s", "ms_per_step": r["ms_per_step"], "cell_steps_per_step": r["cell_steps"],
           "latency_ms": {"p50": r["p50_ms"], "p99": r["p99_ms"]},
           "phase_ms": {"setup": r["setup_ms"], "time_stepping": r["kernel_ms"]},
           "roofline": three_d_roofline(r, w3.boxes),
           "status_ok": r["status_ok"]}
    if with_cpu:
        rec["cpu_baseline"], rec["max_rel_err_vs_oracle"] = cpu_baseline(w3, 16, {"fp64": r["H"]})
    return rec


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle baseline")
    ap.add_argument("--cpu-sample", type=int, default=None,
                    help="boxes the oracle solves for cpu_baseline (default: about 10-30 s of host work)")
    ap.add_argument("--precision", choices=["both", "fp32", "fp64"], default="both")
    ap.add_argument("--workload", choices=sorted(WORKLOADS), default="two_d_batch")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the uneven-batch and served measurements added to the default line")
    ap.add_argument("--served-stages", type=int, default=10,
                    help="macro stages of the served 128x128 run in the default line")
    ap.add_argument("--served-only", action="store_true",
                    help="only the served run (--served-stages stages per arrival mode), as its own JSON line")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy (PMC counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU (--gpus 1): the boxes of a batch are independent, so "
              "N GPUs would each solve 1/N of them with no communication; this script does not "
              "launch several", file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration()
        return
    if args.served_only:
        print(json.dumps({"served": served(args.served_stages, with_cpu=not args.no_cpu)}), flush=True)
        return

    from paper_2108_09463_amd import inputs

    wl = getattr(inputs, args.workload)()
    precs = {"fp32": inputs.FP32, "fp64": inputs.FP64}
    if args.precision != "both":
        precs = {args.precision: precs[args.precision]}
    if args.workload in THREE_D:
        precs = {"fp64": inputs.FP64}          # d = 3 boxes are built in FP64
    res = {name: measure(wl, prec, args.steps, args.warmup) for name, prec in precs.items()}
    if args.workload in THREE_D:
        res["fp64"]["roofline"] = three_d_roofline(res["fp64"], wl.boxes)
    gpu_H = {k: v["H"] for k, v in res.items()}
    cpu = None
    errs = {}
    if not args.no_cpu:
        sample = args.cpu_sample or DEFAULT_CPU_SAMPLE.get(args.workload, 1024)
        cpu, errs = cpu_baseline(wl, min(sample, len(wl.boxes)), gpu_H)
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
        "config": {"workload": WORKLOADS[args.workload],
                   "boxes": len(wl.boxes), "cell_steps_per_step": r["cell_steps"]},
        "roofline": r["roofline"],
        "latency_ms": {"p50": r["p50_ms"], "p99": r["p99_ms"]},
        "phase_ms": {"setup": r["setup_ms"], "time_stepping": r["kernel_ms"]},
        "cpu_baseline": cpu,
        "max_rel_err_vs_oracle": errs,
        "status_ok": r["status_ok"],
    }
    if "fp64" in res and head == "fp32":
        f = res["fp64"]
        line["fp64"] = {"value": f["rate"], "ms_per_step": f["ms_per_step"],
                        "latency_ms": {"p50": f["p50_ms"], "p99": f["p99_ms"]},
                        "phase_ms": {"setup": f["setup_ms"], "time_stepping": f["kernel_ms"]},
                        "roofline": f["roofline"]}
        line["speedup_fp32_vs_fp64"] = r["rate"] / f["rate"]
    if args.workload == "two_d_batch" and not args.no_extra:
        w1 = inputs.one_d_batch()
        o32 = measure(w1, inputs.FP32, 5, 1)
        o64 = measure(w1, inputs.FP64, 5, 1)
        rec = {"workload": WORKLOADS["one_d_batch"], "dtype": "f32", "value": o32["rate"],
               "unit": "cell-steps/s", "ms_per_step": o32["ms_per_step"],
               "latency_ms": {"p50": o32["p50_ms"], "p99": o32["p99_ms"]},
               "roofline": o32["roofline"], "fp64_value": o64["rate"],
               "speedup_fp32_vs_fp64": o32["rate"] / o64["rate"],
               "status_ok": o32["status_ok"] and o64["status_ok"]}
        if not args.no_cpu:
            rec["cpu_baseline"], rec["max_rel_err_vs_oracle"] = cpu_baseline(
                w1, 256, {"fp32": o32["H"], "fp64": o64["H"]})
        line["one_d_batch"] = rec
        # the headline batch with the fourth-order stencil, both precisions
        w4 = inputs.two_d_batch_o4()
        f4 = measure(w4, inputs.FP32, 5, 1)
        d4 = measure(w4, inputs.FP64, 5, 1)
        rec4 = {"workload": WORKLOADS["two_d_batch_o4"], "dtype": "f32", "value": f4["rate"],
                "unit": "cell-steps/s", "ms_per_step": f4["ms_per_step"],
                "latency_ms": {"p50": f4["p50_ms"], "p99": f4["p99_ms"]},
                "roofline": f4["roofline"],
                "fp64": {"value": d4["rate"], "ms_per_step": d4["ms_per_step"], "roofline": d4["roofline"]},
                "speedup_fp32_vs_fp64": f4["rate"] / d4["rate"],
                "status_ok": f4["status_ok"] and d4["status_ok"]}
        if not args.no_cpu:
            rec4["cpu_baseline"], rec4["max_rel_err_vs_oracle"] = cpu_baseline(
                w4, 64, {"fp32": f4["H"], "fp64": d4["H"]})
        line["two_d_batch_o4"] = rec4
        # the single plain FP64 1-D box (box 0 of the 1-D batch): latency of one whole solve
        w0 = inputs.one_d_batch(nboxes=1)
        s0 = measure(w0, inputs.FP64, 50, 5)
        line["single_box"] = {"workload": "single_box: one 1-D FP64 box of 256 points, mu=mu'=4eps, eps=0.01, "
                                          "alpha=0.01 RK4P, eta=eps^2, flux average (box 0 of one_d_batch)",
                              "dtype": "f64", "value": s0["rate"], "unit": "cell-steps/s",
                              "solves": 50, "latency_ms": {"p50": s0["p50_ms"], "p99": s0["p99_ms"]},
                              "phase_ms": {"setup": s0["setup_ms"], "time_stepping": s0["kernel_ms"]},
                              "status_ok": s0["status_ok"]}
        wu = inputs.uneven_batch()
        u = measure(wu, inputs.FP32, 3, 1, tune=True, graph=True)
        line["uneven_batch"] = {"workload": WORKLOADS["uneven_batch"] + "; slab variant and exchange "
                                "interval tuned, whole solve launched as one HIP graph", "dtype": "f32",
                                "value": u["rate"], "unit": "cell-steps/s",
                                "ms_per_step": u["ms_per_step"], "cell_steps_per_step": u["cell_steps"],
                                "latency_ms": {"p50": u["p50_ms"], "p99": u["p99_ms"]},
                                "slabs_by_n": u["slabs"],
                                "roofline": u["roofline"], "status_ok": u["status_ok"]}
        if not args.no_cpu:
            (line["uneven_batch"]["cpu_baseline"],
             line["uneven_batch"]["max_rel_err_vs_oracle"]) = cpu_baseline(wu, 64, {"fp32": u["H"]})
        if args.served_stages > 0:
            line["served"] = served(args.served_stages, with_cpu=not args.no_cpu)
        line["three_d_batch"] = three_d_record(3, 1, not args.no_cpu)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
