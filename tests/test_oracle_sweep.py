"""Section 4.4 trends of the averaging error E_avg on the FP64 oracle (the
quick sweep of tests/micro_sweep.py): fall with mu to a plateau from about
3.5 eps, lower error with high damping, fall with mu' to a plateau that needs
larger boxes for longer eta, monotone fall with eta for alpha = 1, and the
E_eps plateau scaling like eps^2."""
from concurrent.futures import ThreadPoolExecutor
import os

import micro_sweep as S
from oracle import micro
from paper_2108_09463_amd import inputs


def test_quick_sweep_trends_on_oracle():
    pts = S.sweeps(quick=True)
    with ThreadPoolExecutor(min(8, os.cpu_count() or 1)) as ex:
        H = list(ex.map(lambda p: micro.solve_box(p[1], p[2], init_fn=inputs.InitEX2())["out"],
                        pts))
    rows = [dict(lab, E_avg=S.e_avg(lab, h)) for (lab, _, _), h in zip(pts, H)]
    done = S.check_trends(rows)
    assert len(done) >= 6
