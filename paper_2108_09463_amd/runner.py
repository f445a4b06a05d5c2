"""Runs an inputs.Workload through the HIP path (libllhmm) on one GPU.

Device memory and the stream come from PyTorch; every computation of the
method happens in the library's kernels.
"""
from __future__ import annotations

import copy

import numpy as np

from . import llhmm as L


class Prepared:
    """A workload planned and uploaded once; `solve()` can be called repeatedly."""

    def __init__(self, wl, precision=None, ctx=None, device=0, boxes=None, K=None, coef_samples=None):
        """coef_samples: optional FP64 face values of a sampled coefficient, packed
        as llhmm_micro_batch's coef_dev (each box's block at its coef_offset);
        the workload's coefficients are then passed as sampled."""
        import torch
        self.torch = torch
        self.wl = wl
        self.dev = torch.device("cuda", device)
        self.ctx = ctx or L.llhmm_create(device)
        boxes = copy.deepcopy(boxes if boxes is not None else wl.boxes)
        self.m_init = None
        if any(b["init_mode"] == 0 for b in boxes):
            host, offs = L.pack_explicit_init(boxes, wl.init_of)
            for b, o in zip(boxes, offs):
                b["init_offset"] = o
            self.m_init = torch.from_numpy(host).to(self.dev)
        self.boxes = boxes
        self.macro = self.M_macro = None
        if any(b["init_mode"] == 1 for b in boxes):
            self.macro = L.macro_dict(wl.macro, dim=boxes[0]["dim"])
            self.M_macro = torch.from_numpy(np.ascontiguousarray(wl.macro["M"], dtype=np.float64)
                                            .reshape(3, -1)).to(self.dev)
        sampled = coef_samples is not None
        coefs = [L.to_coef(c, sampled=sampled) for c in wl.coefs]
        self.coef_dev = (torch.from_numpy(np.ascontiguousarray(coef_samples, dtype=np.float64)).to(self.dev)
                         if sampled else None)
        prec = wl.precision if precision is None else precision
        self.precision = prec
        self.batch = L.llhmm_batch_create(self.ctx, boxes, coefs, prec,
                                          K or L.kernel(*wl.kernel))
        self.ld = self.batch.nq_max
        self.H = torch.zeros((len(boxes), self.ld), dtype=torch.float64, device=self.dev)
        self.status = torch.zeros(len(boxes), dtype=torch.int32, device=self.dev)

    def launch(self, m_final=None, stream=None):
        L.llhmm_micro_batch(self.ctx, self.batch, self.m_init, self.macro, self.M_macro, self.coef_dev,
                            m_final, stream)
        L.llhmm_upscale(self.ctx, self.batch, self.H, self.ld, self.status, False, stream)

    def launch_graph(self, stream=None):
        """The same solve + upscale as one captured HIP graph (replayed while the
        arguments stay the same)."""
        L.llhmm_batch_run_graph(self.ctx, self.batch, self.H, self.ld, self.status, self.m_init,
                                self.macro, self.M_macro, self.coef_dev, None, stream)

    def tune(self, reps=2):
        L.llhmm_batch_tune(self.ctx, self.batch, self.m_init, self.macro, self.M_macro, self.coef_dev, reps)
        return L.llhmm_batch_slabs(self.batch)

    def solve(self, want_state=False):
        torch = self.torch
        mf = None
        if want_state:
            d = self.batch.dim_max
            mf = torch.zeros(len(self.boxes) * 3 * self.batch.n_max ** d, dtype=torch.float64,
                             device=self.dev)
        self.launch(mf)
        torch.cuda.synchronize(self.dev)
        out = dict(H=self.H.cpu().numpy().copy(), status=self.status.cpu().numpy().copy())
        if want_state:
            out["m_final"] = mf.cpu().numpy()
        return out

    def eval_field(self):
        torch = self.torch
        d = self.batch.dim_max
        Hf = torch.zeros(len(self.boxes) * 3 * self.batch.n_max ** d, dtype=torch.float64,
                         device=self.dev)
        L.llhmm_eval_field(self.ctx, self.batch, Hf, self.m_init, self.macro, self.M_macro, self.coef_dev)
        torch.cuda.synchronize(self.dev)
        return Hf.cpu().numpy()

    def cell_steps(self):
        return self.batch.cell_steps()


def box_state(flat, i, box, n_max, dim_max):
    """Slice box i's [3][n^d] block out of a packed m_final / H array."""
    stride = 3 * n_max ** dim_max
    n, d = box["n"], box["dim"]
    return flat[i * stride: i * stride + 3 * n ** d].reshape((3,) + (n,) * d)
