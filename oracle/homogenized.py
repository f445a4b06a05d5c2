"""Oracle for the homogenized problem and the macro-level error split.

TEST INFRASTRUCTURE ONLY (see the package docstring): only tests, the smoke
check and the CPU baseline may use it.

* eq. (hom): dM0/dt = -M0 x F - alpha M0 x (M0 x F), F = div(grad M0 A^H), on the
  periodic unit interval / square, A^H a constant symmetric d x d matrix.
  Space: Fourier spectral second derivatives on an N^d grid (x_i = i / N);
  the mixed derivative is the product of two first derivatives, whose Nyquist
  mode is dropped.  Time: classical RK4 followed by normalization of every
  point, i.e. RK4P of Section 3.1 applied to eq. (hom).
* Closed form used to pin it: a precessing, damped plane wave
  m = (sin th cos phi, sin th sin phi, cos th), phi = k.x + phi(t), th = th(t),
  for which F = -(k^T A k)(m - cos th e3).  With c = cos th and
  lam = alpha k^T A k:  dc/dt = lam c (1 - c^2) and dphi/dt = k^T A k c, hence
  c(t) = v / sqrt(1 + v^2), v = exp(lam t) / tan th0, and
  phi(t) = phi0 + (asinh v(t) - asinh v(0)) / alpha.
* E_disc of eq. (E_approx) / eq. (E_interpol): the field
  div(grad m_init(0) A^H) at every macro node when m_init is the normalized
  interpolant Q_[4] = P_[4] / |P_[4]| of Section 4.1 (tensor-product Lagrange
  interpolation on the nodes -2..2 around the node, x1 then x2).  Its
  derivatives at the node follow from the Lagrange basis derivatives at 0 and
  the quotient rule for P / |P|.  A macro loop driven by this field is the HMM
  loop with E_avg = 0: its error against M0 is the discretization error alone.
* Flux model eq. (macro_flux): the E_avg = 0 flux column j of grad Q A at the
  staggered points x_i + dX/2 e_j (Q the interpolant around node i, evaluated
  half a cell off the node) and its fourth-order staggered divergence.  The
  paper asks for staggered flux locations but gives no divergence stencil;
  fourth order matches the order of Q_[4].  Torque model eq. (macro_torque):
  Q x div(grad Q A) at the nodes.
* run_loop: the macro loop of eq. (macro_disc), time stepped by
  oracle.macro.MacroStepper (HeunP start-up, then MPEA), with the field of each
  stage supplied by a callable (the exact-interpolant field above, or H_avg
  from micro problems).

Reading: the paper does not say how it computes its reference M0.  Any
sufficiently accurate solver of eq. (hom) serves; the spectral/RK4P one here
is pinned by the closed form and by the energy law below.
* Energy: E = 1/2 int grad M0 A^H . grad M0 satisfies dE/dt = -alpha int |M0 x F|^2,
  so E is constant for alpha = 0 and decreasing for alpha > 0.
"""
from __future__ import annotations

import numpy as np

from . import macro as macro_mod


# ----------------------------------------------------------------- spectral field
def _wavenumbers(N):
    """(k for even derivatives, k for odd derivatives with the Nyquist mode dropped)."""
    k = 2.0 * np.pi * np.fft.fftfreq(N, d=1.0 / N)
    ko = k.copy()
    if N % 2 == 0:
        ko[N // 2] = 0.0
    return k, ko


def hom_field(M, A):
    """F = div(grad M A) for M [3, N] (1-D) or [3, N, N] (2-D, M[:, i1, i2] at
    (i1/N, i2/N)); A is a scalar (1-D) or a symmetric 2 x 2 matrix."""
    M = np.asarray(M, dtype=np.float64)
    d = M.ndim - 1
    N = M.shape[1]
    k, ko = _wavenumbers(N)
    if d == 1:
        a = float(np.asarray(A).reshape(-1)[0])
        Mh = np.fft.fft(M, axis=1)
        return a * np.real(np.fft.ifft(-(k * k)[None, :] * Mh, axis=1))
    A = np.asarray(A, dtype=np.float64).reshape(2, 2)
    Mh = np.fft.fft2(M, axes=(1, 2))
    K1 = k[:, None]
    K2 = k[None, :]
    O1 = ko[:, None]
    O2 = ko[None, :]
    symbol = (A[0, 0] * (-K1 * K1) + A[1, 1] * (-K2 * K2)
              + (A[0, 1] + A[1, 0]) * ((1j * O1) * (1j * O2)))
    return np.real(np.fft.ifft2(symbol[None] * Mh, axes=(1, 2)))


def gradients(M):
    """First derivatives [d][3, ...] by the spectral rule (Nyquist dropped)."""
    M = np.asarray(M, dtype=np.float64)
    d = M.ndim - 1
    N = M.shape[1]
    _, ko = _wavenumbers(N)
    if d == 1:
        return [np.real(np.fft.ifft(1j * ko[None, :] * np.fft.fft(M, axis=1), axis=1))]
    Mh = np.fft.fft2(M, axes=(1, 2))
    g1 = np.real(np.fft.ifft2(1j * ko[None, :, None] * Mh, axes=(1, 2)))
    g2 = np.real(np.fft.ifft2(1j * ko[None, None, :] * Mh, axes=(1, 2)))
    return [g1, g2]


def energy(M, A):
    """E = 1/2 int sum_jk A_jk (d_j M . d_k M) over the unit interval / square."""
    g = gradients(M)
    A = np.asarray(A, dtype=np.float64).reshape(len(g), len(g))
    e = 0.0
    for j in range(len(g)):
        for kk in range(len(g)):
            e += A[j, kk] * np.mean(np.sum(g[j] * g[kk], axis=0))
    return 0.5 * e


def ll_rhs(M, F, alpha):
    """-M x F - alpha M x (M x F), component axis 0."""
    c = np.cross(M, F, axis=0)
    return -c - alpha * np.cross(M, c, axis=0)


def normalize(M):
    return M / np.sqrt(np.sum(M * M, axis=0, keepdims=True))


def solve_hom(M_init, A, alpha, T, steps):
    """M0(T) of eq. (hom) by RK4P with `steps` equal steps."""
    M = np.array(M_init, dtype=np.float64)
    dt = T / steps

    def f(Y):
        return ll_rhs(Y, hom_field(Y, A), alpha)

    for _ in range(steps):
        k1 = f(M)
        k2 = f(M + 0.5 * dt * k1)
        k3 = f(M + 0.5 * dt * k2)
        k4 = f(M + dt * k3)
        M = normalize(M + dt / 6.0 * (k1 + 2.0 * k2 + 2.0 * k3 + k4))
    return M


def stable_steps(A, N, alpha, T, dim, safety=0.5):
    """Step count for solve_hom: dt * omega_max <= safety * 2 sqrt(2) (RK4 on the
    imaginary axis), omega_max = k_max^2 * (sum of |A_jk|)."""
    kmax = np.pi * N
    omega = kmax * kmax * float(np.sum(np.abs(np.asarray(A, dtype=np.float64))))
    dt = safety * 2.0 * np.sqrt(2.0) / omega
    return int(np.ceil(T / dt))


def plane_wave(xs, kvec, A, alpha, theta0, phi0, t):
    """Closed-form solution of eq. (hom) (see the module docstring).

    xs: tuple of coordinate arrays (one per axis); kvec: wave vector (2 pi times
    integers for periodicity); 0 < theta0 < pi/2."""
    kv = np.asarray(kvec, dtype=np.float64)
    A = np.asarray(A, dtype=np.float64).reshape(len(kv), len(kv))
    aeff = float(kv @ A @ kv)
    lam = alpha * aeff
    tan0 = np.tan(theta0)
    if alpha > 0.0:
        v0 = 1.0 / tan0
        v = np.exp(lam * t) / tan0
        c = v / np.sqrt(1.0 + v * v)
        dphi = (np.arcsinh(v) - np.arcsinh(v0)) / alpha
    else:
        c = np.cos(theta0)
        dphi = aeff * c * t
    s = np.sqrt(1.0 - c * c)
    phase = sum(ki * x for ki, x in zip(kv, xs)) + phi0 + dphi
    return np.stack([s * np.cos(phase), s * np.sin(phase), c * np.ones_like(phase)])


# ----------------------------------------------------------------- E_disc field
def _lagrange_basis_derivs(s=0.0):
    """D[p][l] = p-th derivative at s of the Lagrange basis polynomial L_l on
    the nodes -2..2 (l = 0..4 for the nodes -2..2), p = 0, 1, 2."""
    nodes = np.arange(-2, 3, dtype=np.float64)
    D = np.zeros((3, 5))
    for l in range(5):
        others = np.delete(nodes, l)
        poly = np.polynomial.Polynomial.fromroots(others) / np.prod(nodes[l] - others)
        for p in range(3):
            D[p, l] = poly.deriv(p)(s) if p else poly(s)
    return D


def q4_node_derivatives(M, dX):
    """P = P_[4] and its derivatives at every macro node.

    M: [3, n] or [3, n, n] on a periodic grid of spacing dX.  Returns (P, dP, ddP):
    dP[j] = d_j P, ddP[j][k] = d_j d_k P, arrays shaped like M."""
    M = np.asarray(M, dtype=np.float64)
    d = M.ndim - 1
    D = _lagrange_basis_derivs()
    if d == 1:
        def comb(p):
            out = np.zeros_like(M)
            for l in range(5):
                out += D[p, l] * np.roll(M, -(l - 2), axis=1)
            return out / dX ** p
        return comb(0), [comb(1)], [[comb(2)]]

    def comb(p, q):
        # sum_a sum_b L_a^(p)(0) L_b^(q)(0) M[i + a, j + b]
        out = np.zeros_like(M)
        for a in range(5):
            for b in range(5):
                w = D[p, a] * D[q, b]
                if w != 0.0:
                    out += w * np.roll(np.roll(M, -(a - 2), axis=1), -(b - 2), axis=2)
        return out / dX ** (p + q)

    P = comb(0, 0)
    dP = [comb(1, 0), comb(0, 1)]
    ddP = [[comb(2, 0), comb(1, 1)], [comb(1, 1), comb(0, 2)]]
    return P, dP, ddP


def q4_node_field(M, A, dX):
    """div(grad Q A) at every macro node, Q = P / |P| (the E_avg = 0 upscaled field)."""
    P, dP, ddP = q4_node_derivatives(M, dX)
    d = len(dP)
    A = np.asarray(A, dtype=np.float64).reshape(d, d)
    r = np.sqrt(np.sum(P * P, axis=0))
    dr = [np.sum(P * dP[j], axis=0) / r for j in range(d)]
    F = np.zeros_like(P)
    for j in range(d):
        for k in range(d):
            if A[j, k] == 0.0:
                continue
            Pj = np.sum(P * dP[j], axis=0)
            Pk = np.sum(P * dP[k], axis=0)
            ddr = (np.sum(dP[k] * dP[j], axis=0) + np.sum(P * ddP[j][k], axis=0)) / r \
                - Pj * Pk / r ** 3
            ddQ = (ddP[j][k] / r - dP[j] * dr[k] / r ** 2 - dP[k] * dr[j] / r ** 2
                   - P * ddr / r ** 2 + 2.0 * P * dr[j] * dr[k] / r ** 3)
            F += A[j, k] * ddQ
    return F


# ----------------------------------------------------------------- flux and torque models
def q4_stagger_flux(M, A, dX, axis):
    """E_avg = 0 flux of the flux model eq. (macro_flux): column `axis` of
    grad Q A at the staggered points x_i + dX/2 e_axis, Q = P / |P| the
    interpolant around node i (Section 4.1) evaluated half a cell off the node.
    Returns F [3, n(, n)], F[..., i] belonging to x_i + dX/2 e_axis."""
    M = np.asarray(M, dtype=np.float64)
    d = M.ndim - 1
    A = np.asarray(A, dtype=np.float64).reshape(d, d)
    Dh = _lagrange_basis_derivs(0.5)      # along `axis`
    D0 = _lagrange_basis_derivs(0.0)      # along the other axis
    if d == 1:
        def comb(p):
            out = np.zeros_like(M)
            for l in range(5):
                out += Dh[p, l] * np.roll(M, -(l - 2), axis=1)
            return out / dX ** p
        P, dP = comb(0), [comb(1)]
    else:
        def comb(p0, p1):
            B0 = Dh if axis == 0 else D0
            B1 = Dh if axis == 1 else D0
            out = np.zeros_like(M)
            for a in range(5):
                for b in range(5):
                    w = B0[p0, a] * B1[p1, b]
                    if w != 0.0:
                        out += w * np.roll(np.roll(M, -(a - 2), axis=1), -(b - 2), axis=2)
            return out / dX ** (p0 + p1)
        P, dP = comb(0, 0), [comb(1, 0), comb(0, 1)]
    r = np.sqrt(np.sum(P * P, axis=0))
    F = np.zeros_like(P)
    for k in range(d):
        dQ = dP[k] / r - P * np.sum(P * dP[k], axis=0) / r ** 3
        F += A[k, axis] * dQ
    return F


def staggered_divergence(F, dX, order=4):
    """sum_j D_j F_j at the nodes from F_j at x_i + dX/2 e_j (F: list over axes of
    [3, n(, n)]).  order 4: (27 (F_{i+1/2} - F_{i-1/2}) - (F_{i+3/2} - F_{i-3/2}))
    / (24 dX); order 2: (F_{i+1/2} - F_{i-1/2}) / dX."""
    out = np.zeros_like(F[0])
    for j, Fj in enumerate(F):
        ax = j + 1

        def sh(k):           # F at staggered index i + k
            return np.roll(Fj, -k, axis=ax)
        if order == 4:
            out += (27.0 * (sh(0) - sh(-1)) - (sh(1) - sh(-2))) / (24.0 * dX)
        else:
            out += (sh(0) - sh(-1)) / dX
    return out


def q4_flux_field(M, A, dX, order=4):
    """The flux model's E_avg = 0 replacement for H_avg at the nodes."""
    d = np.asarray(M).ndim - 1
    return staggered_divergence([q4_stagger_flux(M, A, dX, j) for j in range(d)], dX, order)


def q4_node_torque(M, A, dX):
    """E_avg = 0 torque of eq. (macro_torque): Q x div(grad Q A) at the nodes."""
    M = np.asarray(M, dtype=np.float64)
    Q = M / np.sqrt(np.sum(M * M, axis=0, keepdims=True))
    return np.cross(Q, q4_node_field(M, A, dX), axis=0)


# ----------------------------------------------------------------- macro loop
def run_loop(M_init, field_fn, alpha, dt, steps, startup="heunp", model="field"):
    """`steps` macro steps of eq. (macro_disc) (model "field"; the flux model
    passes its divergence as the field) or eq. (macro_torque) (model "torque");
    field_fn(Y) returns the averaged quantity [3, npts] at the stage input
    Y [3, npts].  Returns M [3, npts]."""
    M0 = np.asarray(M_init, dtype=np.float64)
    st = macro_mod.MacroStepper(M0.reshape(3, -1), alpha, dt, startup, model)
    while st.step < steps:
        st.advance(field_fn(st.Y))
    return st.M
