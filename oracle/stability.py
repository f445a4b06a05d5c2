"""Time-step rule for the micro problem (Section 3.2, eq. (f_alfa) and (Cstab)).

The paper shows that, for smooth data, the Jacobian eigenvalues of the
semi-discrete LL right-hand side lie on the rays omega (+-i - alpha) with omega in
[0, rho(-D)], rho(-D) = O(dx^-2), so an explicit method is stable when
dt * omega (-alpha + i) stays inside the method's stability region, and that the
stability constant scales with 1/max a.  It gives no formula for the constant.

Reading used here:
* omega_max = sigma * d * a_max / dx^2 with sigma = 4 (second-order stencil) or
  sigma = (7/3)^2 (fourth-order staggered stencil); these are the largest
  eigenvalues of the unit-coefficient operators per axis, times the bound a_max
  of assumption (A1);
* r*(alpha, R) = the largest r such that |R(s(-alpha + i))| <= 1 for all s in
  [0, r], with R the stability polynomial of Heun (RK2) or RK4, found by a scan
  with step 1e-3 followed by 80 bisection steps;
* M = ceil(eta / (0.9 r* / omega_max)), dt = eta / M, so the final time eta is hit
  exactly.
"""
from __future__ import annotations

import math

HEUNP, RK4P = 1, 2
SAFETY = 0.9
SCAN_STEP = 1e-3
SCAN_MAX = 20.0


def _growth(s, alpha, integ):
    """|R(z)|^2 - 1 at z = s(-alpha + i), R the stability polynomial."""
    z = complex(-alpha * s, s)
    if integ == HEUNP:
        r = 1 + z + z * z / 2
    else:
        r = 1 + z + z * z / 2 + z ** 3 / 6 + z ** 4 / 24
    return (r.real * r.real + r.imag * r.imag) - 1.0


def r_star(alpha, integ):
    if alpha <= 0.0:
        raise ValueError("alpha must be positive (assumption A2)")
    k = 1
    while True:
        s = k * SCAN_STEP
        if _growth(s, alpha, integ) > 0.0:
            break
        k += 1
        if s > SCAN_MAX:
            raise ValueError("no stability limit found")
    lo, hi = (k - 1) * SCAN_STEP, s
    for _ in range(80):
        mid = 0.5 * (lo + hi)
        if _growth(mid, alpha, integ) > 0.0:
            hi = mid
        else:
            lo = mid
    return lo


def resolve_integrator(integ, alpha):
    """AUTO reading: HeunP for alpha > 0.2 (end of Section 3), RK4P otherwise
    (Section 3.2: for alpha < 0.1 RK4 is cheaper than HeunP)."""
    if integ in (HEUNP, RK4P):
        return integ
    return HEUNP if alpha > 0.2 else RK4P


def sigma(order):
    return 4.0 if order == 2 else (7.0 / 3.0) ** 2


def plan_steps(eta, alpha, integ, order, dim, a_max, dx):
    omega = sigma(order) * dim * a_max / (dx * dx)
    dt_max = SAFETY * r_star(alpha, integ) / omega
    M = int(math.ceil(eta / dt_max))
    return M, eta / M
