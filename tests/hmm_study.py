"""HMM loop error study (Section 4.5, fig:hmm_err_ex3): L2 error at T of the
GPU HMM loop against the homogenized reference M0, per micro setup and macro
grid, beside the E_avg = 0 loop and the naive average coefficient.

  python tests/hmm_study.py --setups s1 s2 --dX 12 24 --out hmm.json
"""
import argparse
import json
import os
import sys
import time

import numpy as np

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))

import hmm_reference as R  # noqa: E402
from paper_2108_09463_amd import inputs  # noqa: E402
from paper_2108_09463_amd import llhmm as L  # noqa: E402
from paper_2108_09463_amd.hmm import HmmLoop  # noqa: E402


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--setups", nargs="+", default=list(inputs.HMM_SETUPS))
    ap.add_argument("--dX", nargs="+", type=int, default=[12, 24, 48])
    ap.add_argument("--T", type=float, default=0.1)
    ap.add_argument("--precision", default="fp32", choices=["fp32", "fp64"])
    ap.add_argument("--out", default=None)
    ap.add_argument("--no-ideal", action="store_true")
    ap.add_argument("--tune", action="store_true")
    args = ap.parse_args()
    prec = inputs.FP32 if args.precision == "fp32" else inputs.FP64
    ctx = L.llhmm_create(0)
    rows = []
    ideal_done = {}
    for setup in args.setups:
        ppe = inputs.HMM_SETUPS[setup][0]
        ref = R.M0(ppe, args.T)
        for n in args.dX:
            steps, dt = R.steps_for(n, args.T)
            tmpl = inputs.hmm_micro(setup)
            loop = HmmLoop(n, inputs.ex2_macro(n), inputs.coef_ex2(tmpl["eps"]), tmpl, R.ALPHA,
                           dt, precision=prec, ctx=ctx, tune=args.tune)
            t0 = time.perf_counter()
            loop.run(steps, progress=lambda k: print(
                f"  {setup} n={n} step {k}/{steps} {time.perf_counter() - t0:.1f}s", flush=True),
                every=max(1, steps // 8))
            wall = time.perf_counter() - t0
            M = loop.state()
            cs = loop.cell_steps_per_stage() * loop.stages
            loop.close()
            row = dict(setup=setup, n_macro=n, steps=steps, dt=dt, err=R.l2_err(M, ref),
                       wall_s=wall, cell_steps=cs, cell_steps_per_s=cs / wall)
            if not args.no_ideal and (ppe, n) not in ideal_done:
                ideal_done[ppe, n] = R.l2_err(R.ideal_loop(n, ppe, args.T), ref)
            row["ideal_err"] = ideal_done.get((ppe, n))
            rows.append(row)
            print(json.dumps(row), flush=True)
    naive = R.l2_err(R.M0(6, args.T, A_key=tuple((R.a_avg() * np.eye(2)).ravel())),
                     R.M0(6, args.T))
    out = dict(T=args.T, precision=args.precision, a_avg_err=naive, rows=rows)
    print(json.dumps(dict(a_avg_err=naive)))
    if args.out:
        with open(args.out, "w") as f:
            json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
