"""Oracle for the macro time step (Section 3.1 and Section 3.3).

Macro model eq. (macro_disc): dM_i/dt = -M_i x H_avg - alpha M_i x (M_i x H_avg).

* h(M) = H_avg + alpha M x H_avg                                  eq. (h_term)
* MPEA: hbar = 23/12 h^j - 16/12 h^{j-1} + 5/12 h^{j-2}           eq. (h_mpea)
  and (M^{j+1} - M^j)/dt = -(M^j + M^{j+1})/2 x hbar              eq. (mpe_update)
  Reading: eq. (imp_sys) writes the inverse factor with the opposite sign of
  eq. (imp_update); this oracle follows the difference equation
  eq. (mpe_update), i.e. (I - s[h]x) M^{j+1} = (I + s[h]x) M^j with s = dt/2.
  The 3x3 system per point is solved by Gaussian elimination (numpy.linalg.solve).
* Start-up steps (j = 0, 1) with HeunP or RK4P on the macro equation
  (Section 3.1: "values for m^1 (and m^2) ... using HeunP or RK4P"), each
  stage needing its own H_avg.

* Torque model eq. (macro_torque): dM/dt = -T_avg - alpha M x T_avg.  It has no
  cross product in its first term, so MPEA (built on the rotation structure)
  does not apply; every step uses the start-up scheme (HeunP or RK4P) followed
  by normalization (the projection of Section 3.1).
* Flux model eq. (macro_flux): the field model with H_avg replaced by the
  divergence of the averaged flux (see oracle.homogenized.staggered_divergence).

State layout: component-major arrays [3, npts].
"""
from __future__ import annotations

import numpy as np


def h_of(M, Havg, alpha):
    return Havg + alpha * np.cross(M, Havg, axis=0)


def skew(h):
    """[h]x such that [h]x v = h x v, for one 3-vector h."""
    return np.array([[0.0, -h[2], h[1]], [h[2], 0.0, -h[0]], [-h[1], h[0], 0.0]])


def implicit_midpoint_solve(M, hbar, dt):
    """Solve (I - s[hbar]x) M' = (I + s[hbar]x) M pointwise, s = dt/2 (one 3 x 3
    Gaussian elimination per point, all points in one stacked numpy.linalg.solve)."""
    s = 0.5 * dt
    S = np.stack([skew(hbar[:, i]) for i in range(M.shape[1])])      # [npts, 3, 3]
    I = np.eye(3)[None]
    rhs = np.einsum("pij,jp->pi", I + s * S, M)
    return np.ascontiguousarray(np.linalg.solve(I - s * S, rhs[:, :, None])[:, :, 0].T)


def mpea_hbar(h_j, h_jm1, h_jm2):
    return (23.0 * h_j - 16.0 * h_jm1 + 5.0 * h_jm2) / 12.0


def rhs(M, Havg, alpha):
    c = np.cross(M, Havg, axis=0)
    return -c - alpha * np.cross(M, c, axis=0)


def rhs_torque(M, T, alpha):
    return -T - alpha * np.cross(M, T, axis=0)


def normalize(M):
    return M / np.sqrt(np.sum(M * M, axis=0, keepdims=True))


class MacroStepper:
    """Drives one macro time step as a sequence of stages.  The caller supplies
    H_avg evaluated at ``self.Y`` for each stage."""

    def __init__(self, M0, alpha, dt, startup="heunp", model="field"):
        if model not in ("field", "torque"):
            raise ValueError(model)
        self.model = model
        self.M = np.array(M0, dtype=np.float64)
        self.Y = self.M.copy()
        self.alpha, self.dt = alpha, dt
        self.startup = startup
        self.hist = []          # h^j, h^{j-1}, h^{j-2}, newest first
        self.step = 0
        self.stage = 0
        self.k = []

    def scheme(self):
        if self.model == "torque":
            return self.startup
        if self.step >= 2:
            return "mpea"
        return self.startup

    def advance(self, Havg):
        a, dt = self.alpha, self.dt
        sch = self.scheme()
        if self.stage == 0 and self.model == "field":
            self.hist = [h_of(self.M, Havg, a)] + self.hist[:2]
        if sch == "mpea":
            hb = mpea_hbar(*self.hist)
            self.M = implicit_midpoint_solve(self.M, hb, dt)
            self._end_step()
            return
        k = rhs(self.Y, Havg, a) if self.model == "field" else rhs_torque(self.Y, Havg, a)
        self.k.append(k)
        if sch == "heunp":
            if self.stage == 0:
                self.Y = self.M + dt * k
                self.stage = 1
                return
            self.M = normalize(self.M + 0.5 * dt * (self.k[0] + self.k[1]))
            self._end_step()
            return
        # rk4p
        if self.stage < 3:
            c = 0.5 if self.stage < 2 else 1.0
            self.Y = self.M + c * dt * k
            self.stage += 1
            return
        k1, k2, k3, k4 = self.k
        self.M = normalize(self.M + dt / 6.0 * (k1 + 2 * k2 + 2 * k3 + k4))
        self._end_step()

    def _end_step(self):
        self.step += 1
        self.stage = 0
        self.k = []
        self.Y = self.M.copy()
