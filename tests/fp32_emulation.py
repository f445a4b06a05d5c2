"""CPU emulation of the FP32 arithmetic of the 2-D second-order kernels.

The FP32 path steps the micro problem of eq. (micro) in the reference +
perturbation form m = r + u (r = fl32(m_init), H(r) formed in FP64 and
stored rounded), with the HeunP/RK4P stages and projection of Section 3.1 and
a re-reference every 8 steps.  This module runs that scheme in numpy with
every result computed in FP64 and, per component, rounded to FP32 where the
kernel rounds it:

  faces    the scaled face coefficients a / dx^2
  ref      the reference r (and every re-referenced r')
  state    the perturbation u kept between steps
  h0       the stored H(r) and |r|^2 - 1 tables
  stencil  each operation of the field D(y) of a stage input
  f        m = r + y, h = H(r) + D(y) and the right-hand side -m x h - alpha m x (m x h)
  stage    stage inputs and the Runge-Kutta running sum
  proj     the projection in perturbation form

With no component rounded it is an FP64 implementation of the same scheme
(it agrees with the oracle to about 1e-10 on the boxes used here).  It is a
model of the kernel's rounding, used to find which boxes FP32 can solve within
the 1e-5 bar; it is not the oracle and not the product path.
"""
from __future__ import annotations

import numpy as np

from oracle import micro

COMPONENTS = ("faces", "ref", "state", "h0", "stencil", "f", "stage", "proj")
REREF_STEPS = 8


def _q(x, on):
    return x.astype(np.float32).astype(np.float64) if on else x


def _cross(a, b):
    return np.stack([a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0]])


def _field(y, ax, ay, bc, rnd):
    """D(y) of the perturbation: zero ghosts (Dirichlet) or periodic wrap."""
    if bc == 1:
        yp = np.zeros((3, y.shape[1] + 2, y.shape[2] + 2))
        yp[:, 1:-1, 1:-1] = y
    else:
        yp = np.pad(y, ((0, 0), (1, 1), (1, 1)), mode="wrap")
    gx = _q(yp[:, 1:-1, 1:] - yp[:, 1:-1, :-1], rnd)
    gy = _q(yp[:, 1:, 1:-1] - yp[:, :-1, 1:-1], rnd)
    fx = _q(ax[None] * gx, rnd)
    fy = _q(ay[None] * gy, rnd)
    return _q(_q(fx[:, :, 1:] - fx[:, :, :-1], rnd) + _q(fy[:, 1:, :] - fy[:, :-1, :], rnd), rnd)


def _field_ext(ext, ax, ay, G, n):
    yp = ext[:, G - 1:G + n + 1, G - 1:G + n + 1]
    fx = ax[None] * (yp[:, 1:-1, 1:] - yp[:, 1:-1, :-1])
    fy = ay[None] * (yp[:, 1:, 1:-1] - yp[:, :-1, 1:-1])
    return (fx[:, :, 1:] - fx[:, :, :-1]) + (fy[:, 1:, :] - fy[:, :-1, :])


def solve(box, coef, init_fn, rounded=COMPONENTS, kernel=(3, 7, 3, 7), reref_steps=REREF_STEPS,
          adjoint_average=False, series_projection=False):
    """Field average of one 2-D order-2 box with the given components rounded
    to FP32.  Returns (H_avg [3], M).  adjoint_average: form the step's
    spatial average sum_j w_j D(u)_j as sum_j (D^T w)_j u_j in FP64 (D is
    linear), so the average does not see the rounding of the FP32 field.
    series_projection: the projection as u = t + t s with t = ut - r q,
    q = sqrt(1 + e) - 1 and s = 1/sqrt(1 + e) - 1 from their series in e to
    second order, so every rounded quantity is perturbation-sized."""
    assert box["dim"] == 2 and box["order"] == 2 and box["quantity"] == 0
    P = {k: (k in rounded) for k in COMPONENTS}
    n, bc, G = box["n"], box["bc"], micro.GW
    A, dx = micro.face_coefficients(box, coef)
    mi = micro.initial_data(box, init_fn).reshape(3, n + 2 * G, n + 2 * G)
    integ, M, dt = micro.plan(box)
    w, _, wt = micro.weights(box, kernel, M)
    ax64 = A[0][G:G + n, G - 1:G + n] / dx ** 2
    ay64 = A[1][G - 1:G + n, G:G + n] / dx ** 2
    ax, ay = _q(ax64, P["faces"]), _q(ay64, P["faces"])
    mint = mi[:, G:G + n, G:G + n]
    r = _q(mint, P["ref"])
    U = _q(mint - r, P["state"])
    if bc == 1:
        ext = mi.copy()
        ext[:, G:G + n, G:G + n] = r
    else:
        ext = mi + np.pad(r - mint, ((0, 0), (G, G), (G, G)), mode="wrap")
    H0 = _q(_field_ext(ext, ax64, ay64, G, n), P["h0"])
    dm = _q(np.sum(r ** 2, axis=0) - 1.0, P["h0"])
    W = np.outer(w, w)
    const = np.einsum("ij,cij->c", W, _field_ext(ext, ax64, ay64, G, n)) * wt.sum()
    tails = np.cumsum(wt[::-1])[::-1]
    b = [1 / 6, 1 / 3, 1 / 3, 1 / 6] if integ == 2 else [0.5, 0.5]
    c = [0.5, 0.5, 1.0] if integ == 2 else [1.0]
    acc64 = np.zeros(3)
    alpha = box["alpha"]
    if adjoint_average:
        # D^T w with the kernel's faces: D is symmetric for these ghosts (zero or periodic)
        WT = _field(np.broadcast_to(W, (3,) + W.shape).copy(), ax, ay, bc, False)[0]
    for step in range(M):
        if step > 0 and step % reref_steps == 0:
            sv = _q(r + U, P["ref"])
            z = sv - r
            U = U - z
            r = sv
            dm = _q(np.sum(r ** 2, axis=0) - 1.0, P["h0"])
            Dz = _field(z, ax, ay, bc, P["stencil"])
            H0 = _q(H0 + Dz, P["h0"])
            const += tails[step] * np.einsum("ij,cij->c", W, Dz)
        y = U
        acc = None
        for s in range(len(b)):
            H = _field(y, ax, ay, bc, P["stencil"])
            if s == 0:
                if adjoint_average:
                    acc64 += wt[step] * np.einsum("ij,cij->c", WT, y)
                else:
                    acc64 += wt[step] * np.einsum("ij,cij->c", W, H)
            m = _q(r + y, P["f"])
            h = _q(H0 + H, P["f"])
            mh = _q(_cross(m, h), P["f"])
            f = _q(-(mh + alpha * _q(_cross(m, mh), P["f"])), P["f"])
            if s == 0:
                acc = _q(b[0] * f, P["stage"])
            elif s < len(b) - 1:
                acc = _q(acc + b[s] * f, P["stage"])
            if s < len(b) - 1:
                y = _q(U + dt * c[s] * f, P["stage"])
            else:
                ut = _q(U + dt * _q(b[s] * f + acc, P["stage"]), P["proj"])
                e = _q(2 * np.sum(r * ut, axis=0) + np.sum(ut * ut, axis=0) + dm, P["proj"])
                if series_projection:
                    qq = _q(e * _q(0.5 - 0.125 * e, P["proj"]), P["proj"])
                    ss = _q(e * _q(-0.5 + 0.375 * e, P["proj"]), P["proj"])
                    t = _q(ut - r * qq, P["proj"])
                    U = _q(t + t * ss, P["state"])
                else:
                    inv = _q(1.0 / np.sqrt(1.0 + e), P["proj"])
                    qq = _q(e / (1.0 + (1.0 + e) * inv), P["proj"])
                    U = _q((ut - r * qq) * inv, P["state"])
    return acc64 + const, M
