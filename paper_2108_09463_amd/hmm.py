"""The HMM macro loop on the GPU (Section 2.2, Section 3.1).

One micro problem per macro node and stage: every stage of a macro step solves
the whole batch at the stage input Y (micro initial data Q_[4] from Y, Section
4.1), averages it (eq. (upscaling)) and hands the average to the macro step.
Three macro models (Section 2.2):

* field, eq. (macro_disc): H_avg at the nodes; llhmm_macro_step (HeunP
  start-up steps, then MPEA, eqs. (h_mpea), (mpe_update));
* flux, eq. (macro_flux): the averaged flux of micro problems centred at the
  staggered points x_i + dX/2 e_j (one batch of d * npts problems), its
  divergence by llhmm_flux_divergence, then the field model's step;
* torque, eq. (macro_torque): T_avg at the nodes; llhmm_macro_step_torque
  (HeunP or RK4P with normalization; MPEA needs the cross-product form).

The macro grid is periodic with nodes x_i = i dX (the unit interval, square
or cube; d = 3 micro problems are FP64, field or torque); the macro state stays
on the device and every stage is queued on one
stream, the micro batch as a replayed HIP graph.
"""
from __future__ import annotations

import copy

import numpy as np

from . import inputs
from . import llhmm as L


class HmmLoop:
    """Runs eq. (macro_disc) with H_avg from the library's micro batches.

    n_macro    macro nodes per axis (dX = 1 / n_macro)
    M_init     macro initial data, [3] + [n_macro] * d, d = 1, 2, 3
    coef       the material coefficient a^eps (an inputs.SinSum)
    micro      box fields shared by every micro problem (n, eps, mu, mu_box, eta,
               alpha, bc, order, a_max, integrator, n_steps, quantity = field)
    alpha, dt  macro damping and time step
    tune       run the slab-mode autotuner once on the initial state
    model      "field", "flux" or "torque" (see the module docstring)
    flux_order order of the staggered divergence of the flux model (2 or 4)
    startup    macro scheme of the start-up steps (field, flux) or of every step
               (torque): llhmm.MACRO_HEUNP or llhmm.MACRO_RK4P
    """

    def __init__(self, n_macro, M_init, coef, micro, alpha, dt, precision=inputs.FP32,
                 K=None, ctx=None, graph=True, startup=None, tune=False, model="field",
                 flux_order=4):
        import torch
        self.torch = torch
        self.dev = torch.device("cuda", 0)
        self.ctx = ctx or L.llhmm_create(0)
        M_init = np.asarray(M_init, dtype=np.float64)
        self.dim = M_init.ndim - 1
        if self.dim not in (1, 2, 3) or any(s != n_macro for s in M_init.shape[1:]):
            raise ValueError("M_init must be [3] + [n_macro] * d, d = 1, 2 or 3")
        if model not in ("field", "flux", "torque"):
            raise ValueError("model must be field, flux or torque")
        self.model = model
        self.flux_order = flux_order
        self.n = n_macro
        self.npts = n_macro ** self.dim
        self.alpha, self.dt = float(alpha), float(dt)
        if startup is None:
            startup = L.MACRO_RK4P if model == "torque" else L.MACRO_HEUNP
        self.startup = startup
        dX = 1.0 / n_macro
        quantity = {"field": inputs.Q_FIELD, "flux": inputs.Q_FLUX, "torque": inputs.Q_TORQUE}[model]
        # flux model: one block of boxes per axis j, centred at x_p + dX/2 e_j
        shifts = [tuple(0.5 * (a == j) for a in range(3)) for j in range(self.dim)] \
            if model == "flux" else [(0.0, 0.0, 0.0)]
        boxes = []
        for sh in shifts:
            for p in range(self.npts):
                # node index p: the last coordinate runs fastest
                idx = [0, 0, 0]
                r = p
                for a in range(self.dim - 1, -1, -1):
                    idx[a] = r % n_macro
                    r //= n_macro
                b = inputs.make_box(**copy.deepcopy(micro))
                b.update(dim=self.dim, quantity=quantity, init_mode=inputs.INIT_MACRO_Q,
                         coef_index=0,
                         center=tuple((idx[a] + sh[a]) * dX if a < self.dim else 0.0
                                      for a in range(3)),
                         macro_index=tuple(idx))
                boxes.append(b)
        self.boxes = boxes
        self.macro = dict(dim=self.dim, n=n_macro, dX=dX, x0=(0.0, 0.0, 0.0))
        self.batch = L.llhmm_batch_create(self.ctx, boxes, [L.to_coef(coef)], precision,
                                          K or L.kernel())
        self.graph = graph
        f64 = dict(dtype=torch.float64, device=self.dev)
        self.M = torch.from_numpy(np.ascontiguousarray(M_init.reshape(3, -1))).to(self.dev)
        self.Y = self.M.clone()
        self.ld = 3 * self.dim if model == "flux" else 3
        self.Q = torch.zeros((len(boxes), self.ld), **f64)     # micro averages
        self.H = self.Q if model != "flux" else torch.zeros((self.npts, 3), **f64)
        self.work = torch.zeros(7 * 3 * self.npts, **f64)
        self.status = torch.zeros(len(boxes), dtype=torch.int32, device=self.dev)
        self.bad = torch.zeros(len(boxes), dtype=torch.int32, device=self.dev)
        self.step_index = 0
        self.stages = 0
        if tune:
            # slab boxes: pick the tile variant and exchange interval on this batch
            L.llhmm_batch_tune(self.ctx, self.batch, None, self.macro, self.Y, None, 1)

    def cell_steps_per_stage(self):
        return self.batch.cell_steps()

    def _micro(self):
        if self.graph:
            L.llhmm_batch_run_graph(self.ctx, self.batch, self.Q, self.ld, self.status, None,
                                    self.macro, self.Y)
        else:
            L.llhmm_micro_batch(self.ctx, self.batch, None, self.macro, self.Y)
            L.llhmm_upscale(self.ctx, self.batch, self.Q, self.ld, self.status, False)
        self.bad |= self.status
        if self.model == "flux":
            L.llhmm_flux_divergence(self.ctx, self.macro, self.flux_order, self.Q, self.ld, self.H)

    def step(self):
        """One macro step: as many micro batches and macro stages as the scheme has."""
        stage = 0
        while True:
            self._micro()
            if self.model == "torque":
                stage = L.llhmm_macro_step_torque(self.ctx, self.npts, self.startup, stage, self.dt,
                                                  self.alpha, self.M, self.H, self.Y, self.work)
            else:
                scheme = self.startup if self.step_index < 2 else L.MACRO_MPEA
                stage = L.llhmm_macro_step(self.ctx, self.npts, scheme, self.step_index, stage,
                                           self.dt, self.alpha, self.M, self.H, self.Y, self.work)
            self.stages += 1
            if stage == 0:
                break
        self.step_index += 1

    def run(self, steps, progress=None, every=100):
        """`steps` macro steps; progress(step_index) is called every `every` steps
        after the device has caught up (and checked for non-finite boxes)."""
        for k in range(steps):
            self.step()
            if progress is not None and (self.step_index % every == 0 or k == steps - 1):
                self.check()
                progress(self.step_index)
        self.check()

    def check(self):
        self.torch.cuda.synchronize(self.dev)
        nbad = int((self.bad != 0).sum().item())
        if nbad:
            raise L.LlhmmError(L.E_UNSTABLE, f"{nbad} micro problems reported non-finite values")

    def state(self):
        """M as a host array shaped like M_init."""
        self.torch.cuda.synchronize(self.dev)
        shape = (3,) + (self.n,) * self.dim
        return self.M.cpu().numpy().reshape(shape).copy()

    def close(self):
        self.batch.close()
