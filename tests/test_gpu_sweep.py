"""Micro-problem parameter sweep on the GPU (Section 4.4, Section 4.5).

Every point of the full sweep in tests/micro_sweep.py (176 boxes: mu, mu',
eta, alpha, eps and the tab:e1 setups; Dirichlet boxes with mu < mu') runs as
one batch, in FP64 and in FP32.

* FP64 parity per box (relative, as in test_gpu_parity):
  max(1e-12, 8 x the oracle's own FMA / no-FMA spread on that box).  The sweep
  boxes are large and many are badly conditioned: with weak damping in a
  16 eps box at 4 points per eps the average cancels about seven digits, and
  the oracle's self-spread reaches 3e-9.  The spread is one sample of the
  rounding noise per box; over 176 boxes the largest ratio of the GPU's
  deviation to it is larger than over the few boxes of the other parity
  tests (6.5 here, against at most 3 there), hence 8 rather than 4.
* FP32: the sweep measures E_avg, so the FP32 run must resolve it: per box
  |H_fp32 - H_oracle| <= max(0.05 E_avg, 1e-5 |H_oracle|), i.e. E_avg to 5%
  or, where E_avg is below FP32 resolution, the usual FP32 bar.  On badly
  conditioned boxes the FP32 error relative to |H| exceeds the 1e-5 of
  well-conditioned batches (up to 7e-5 here), while it stays 1e4-1e6 times
  the FP64 oracle's own spread, as on every other workload.
* The E_avg values (FP64 run) show the trends of fig:err_mu, fig:err_outer
  and fig:err_eta; the FP32 run shows the same.
"""
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import micro_sweep as S
from oracle import micro
from paper_2108_09463_amd import inputs
from paper_2108_09463_amd import llhmm as L
from test_gpu_parity import rel_err

pytestmark = pytest.mark.gpu


def oracle_sweep(pts, variant):
    with ThreadPoolExecutor(min(16, os.cpu_count() or 1)) as ex:
        return np.stack(list(ex.map(
            lambda p: micro.solve_box(p[1], p[2], init_fn=inputs.InitEX2(), variant=variant)["out"],
            pts)))


def test_full_sweep_parity_and_trends():
    import torch
    assert torch.cuda.is_available()
    pts = S.sweeps()
    print(f"sweep: {len(pts)} boxes", flush=True)
    ctx = L.llhmm_create(0)
    _, H64 = S.run_gpu(pts, precision=inputs.FP64, ctx=ctx)
    _, H32 = S.run_gpu(pts, precision=inputs.FP32, ctx=ctx)
    Ho = oracle_sweep(pts, "plain")
    spread = rel_err(oracle_sweep(pts, "fma")[:, :3], Ho[:, :3])
    e64 = rel_err(H64[:, :3], Ho[:, :3])
    print("FP64 max rel err", e64.max(), "max spread", spread.max(), flush=True)
    assert np.all(e64 <= np.maximum(1e-12, 8.0 * spread))
    eavg = np.array([S.e_avg(lab, h) for (lab, _, _), h in zip(pts, Ho)])
    d32 = np.linalg.norm(H32[:, :3] - Ho[:, :3], axis=1)
    nH = np.linalg.norm(Ho[:, :3], axis=1)
    print("FP32 max |dH| / max(E_avg, 2e-4 |H|)", (d32 / np.maximum(eavg, 2e-4 * nH)).max(),
          "max rel err", rel_err(H32[:, :3], Ho[:, :3]).max(), flush=True)
    assert np.all(d32 <= np.maximum(0.05 * eavg, 1e-5 * nH))
    assert len(S.check_trends([dict(lab, E_avg=S.e_avg(lab, h))
                               for (lab, _, _), h in zip(pts, H32)])) >= 15
    rows = [dict(lab, E_avg=S.e_avg(lab, h)) for (lab, _, _), h in zip(pts, H64)]
    assert len(S.check_trends(rows)) >= 15
    e1 = {ex: sorted(S.by(rows, "tab_e1", example=ex), reverse=True) for ex in ("EX2", "EX3")}
    print("tab:e1 setups, E_avg by dX:", e1)
    for ex, c in e1.items():
        # each row of tab:e1 targets a smaller dX and lowers E_avg
        assert all(a[1] > b[1] for a, b in zip(c, c[1:])), (ex, c)
