"""Micro-problem parameter sweep on the GPU (Section 4.4, Section 4.5).

Every point of the full sweep in tests/micro_sweep.py (176 boxes: mu, mu',
eta, alpha, eps and the tab:e1 setups; Dirichlet boxes with mu < mu') runs as
one FP32 batch.  Each box matches the FP64 oracle within the FP32 bar of
1e-5 (relative, as in test_gpu_parity), and the GPU's E_avg values show the
trends of fig:err_mu, fig:err_outer and fig:err_eta."""
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


def test_full_sweep_parity_and_trends():
    import torch
    assert torch.cuda.is_available()
    pts = S.sweeps()
    print(f"sweep: {len(pts)} boxes", flush=True)
    _, Hg = S.run_gpu(pts, ctx=L.llhmm_create(0))
    with ThreadPoolExecutor(min(16, os.cpu_count() or 1)) as ex:
        Ho = np.stack(list(ex.map(
            lambda p: micro.solve_box(p[1], p[2], init_fn=inputs.InitEX2())["out"], pts)))
    err = rel_err(Hg[:, :3], Ho)
    print("max rel err", err.max(), flush=True)
    assert err.max() <= 1e-5
    rows = [dict(lab, E_avg=S.e_avg(lab, h)) for (lab, _, _), h in zip(pts, Hg)]
    assert len(S.check_trends(rows)) >= 15
    e1 = {ex: sorted(S.by(rows, "tab_e1", example=ex), reverse=True) for ex in ("EX2", "EX3")}
    print("tab:e1 setups, E_avg by dX:", e1)
    for ex, c in e1.items():
        # each row of tab:e1 targets a smaller dX and lowers E_avg
        assert all(a[1] > b[1] for a, b in zip(c, c[1:])), (ex, c)
