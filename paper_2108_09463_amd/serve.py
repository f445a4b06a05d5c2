"""Served HMM run: the macro loop of eq. (macro_disc) whose micro problems go
through the library's continuous-batching request loop (llhmm_server_*).

Each macro stage issues one micro request per macro point at the current
stage input Y (Q_[4] initial data from Y), shuffled and released in bursts;
results are collected as their micro-batches finish, then one
llhmm_macro_step stage advances the macro state (HeunP start-up steps, then
MPEA).  The micro-batches also leave their averages in a device array, which
the macro stage reads in place (no host round trip).  Latencies are host
times from submit to the poll that returns them.

Arrival of the bursts:
  saturating  all bursts released back to back;
  closed      each burst released when the previous one has completed;
  open        bursts released at exponential gaps of a given mean (seeded),
              whatever has completed.
"""
from __future__ import annotations

import time

import numpy as np

from . import inputs
from . import llhmm as L


class ServeFailed(RuntimeError):
    """Requests of a macro stage came back with a nonzero status."""


def check_stage(rec, allow=0):
    """Raises ServeFailed unless every request of the stage record succeeded:
    a failed request leaves no average, and the macro stage must not advance on
    a missing field.  `allow`: status bits accepted (e.g. 4, an unresolved final
    state, for a run that only times the request loop)."""
    st = np.asarray(rec["status"])
    bad = np.nonzero((st != 0) & ((st < 0) | ((st & ~allow) != 0)))[0]
    if len(bad):
        raise ServeFailed("%d of %d requests failed (first: id %d, status %d)"
                          % (len(bad), len(st), int(bad[0]), int(st[bad[0]])))


class ServedRun:
    def __init__(self, n_macro=128, precision=inputs.FP32, ctx=None, max_inflight=4,
                 max_batch_boxes=1024, device_bytes=16 << 30, seed=5, sizes=inputs.UNEVEN_SIZES,
                 alpha_macro=0.01, dt_macro=None, boxes=None, coefs=None, M0=None, allow_status=0):
        import torch
        self.torch = torch
        self.dev = torch.device("cuda", 0)
        self.ctx = ctx or L.llhmm_create(0)
        if boxes is None:
            boxes, coefs = inputs.served_boxes(n_macro, seed, sizes)
        self.boxes = boxes
        self.n = n_macro
        self.npts = n_macro * n_macro
        self.macro = dict(dim=2, n=n_macro, dX=1.0 / n_macro, x0=(0.0, 0.0))
        M0 = inputs.served_macro(n_macro) if M0 is None else M0
        self.M = torch.from_numpy(np.ascontiguousarray(M0, dtype=np.float64).reshape(3, -1)).to(self.dev)
        self.Y = self.M.clone()
        self.work = torch.zeros(7 * 3 * self.npts, dtype=torch.float64, device=self.dev)
        self.server = L.Server(self.ctx, [L.to_coef(c) for c in coefs], precision,
                               max_inflight=max_inflight, max_batch_boxes=max_batch_boxes,
                               device_bytes=device_bytes)
        # the field averages of a stage, written by the micro-batches (request id = macro point)
        self.Hd = torch.zeros((self.npts, 3), dtype=torch.float64, device=self.dev)
        self.server.set_output(self.Hd, 3, self.npts)
        self.alpha = alpha_macro
        # macro dt: half the MPEA stability limit of about 0.1 dX^2 on these fields
        self.dt = dt_macro if dt_macro is not None else 0.05 / n_macro ** 2
        self.allow_status = allow_status
        self.seed = seed
        self.cell_steps = int(sum(int(m) * b["n"] ** 2 for m, b in zip(L.llhmm_plan(boxes)[0], boxes)))

    def stage(self, Y, stage_index=0, arrival="saturating", gap_mean_s=0.0):
        """One macro stage: a request per macro point at state Y (device [3][npts]),
        bursts released as `arrival` says (gap_mean_s: mean gap of "open").
        Returns H [npts, 3], statuses, per-request latencies (us), per-burst
        latencies (s), the stage latency (s) and the burst sizes."""
        rng = np.random.default_rng(self.seed * 1000 + stage_index)
        order = rng.permutation(self.npts)
        bursts = inputs.burst_sizes(self.npts, self.seed * 1000 + stage_index)
        if arrival == "open":
            gaps = rng.exponential(gap_mean_s, len(bursts))
        elif arrival in ("saturating", "closed"):
            gaps = np.zeros(len(bursts))
        else:
            raise ValueError("arrival: saturating, closed or open")
        H = np.full((self.npts, 3), np.nan)
        lat = np.zeros(self.npts)
        status = np.zeros(self.npts, np.int32)
        burst_of = np.zeros(self.npts, np.int64)
        t_burst = []
        got = 0
        t0 = time.perf_counter()
        t_next = t0
        pos = 0
        for bi, bsz in enumerate(bursts):
            if arrival == "closed":
                while got < pos:      # the previous bursts have completed
                    got += self._collect(H, lat, status, wait=True)
            elif arrival == "open":
                t_next += gaps[bi] if bi > 0 else 0.0
                while time.perf_counter() < t_next:
                    got += self._collect(H, lat, status, wait=False)
                    time.sleep(2e-4)
            ids = order[pos:pos + bsz]
            pos += bsz
            burst_of[ids] = bi
            t_burst.append(time.perf_counter())
            self.server.submit([self.boxes[i] for i in ids], ids, macro=self.macro, M_macro=Y)
            got += self._collect(H, lat, status, wait=False)
        while got < self.npts:
            got += self._collect(H, lat, status, wait=True)
        t_stage = time.perf_counter() - t0
        # burst latency: release of the burst to the completion of its last request
        t_end = np.array(t_burst)[burst_of] + lat * 1e-6
        burst_lat = [float(t_end[burst_of == b].max() - t_burst[b]) for b in range(len(bursts))]
        return dict(H=H, latency_us=lat, status=status, burst_s=burst_lat, stage_s=t_stage, bursts=bursts)

    def _collect(self, H, lat, status, wait):
        ids, Hk, st, lk = self.server.poll(wait=wait)
        H[ids] = Hk[:, :3]
        lat[ids] = lk
        status[ids] = st
        return len(ids)

    def macro_stage(self, step, stage, rec):
        """Advances the macro stepper by one stage with the H_avg the stage's
        micro-batches left on the device; refuses a stage with failed requests."""
        check_stage(rec, self.allow_status)
        scheme = L.MACRO_HEUNP if step < 2 else L.MACRO_MPEA
        nxt = L.llhmm_macro_step(self.ctx, self.npts, scheme, step, stage, self.dt, self.alpha,
                                 self.M, self.Hd, self.Y, self.work)
        self.torch.cuda.synchronize()
        return nxt

    def run(self, steps, arrival="saturating", gap_mean_s=0.0):
        """`steps` macro steps; returns the per-stage records."""
        out = []
        k = 0
        for step in range(steps):
            stage = 0
            while True:
                rec = self.stage(self.Y, k, arrival, gap_mean_s)
                k += 1
                stage = self.macro_stage(step, stage, rec)
                rec.update(step=step)
                out.append(rec)
                if stage == 0:
                    break
        return out

    def close(self):
        self.server.close()
