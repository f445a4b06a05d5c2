"""Seeded synthetic inputs for the batched HMM micro-problem solve.

This module is the only code shared by the FP64 CPU oracle and the HIP
path.  It defines *inputs*: closed-form material coefficients a^eps,
closed-form initial magnetisations, seeded random macro fields and the box
lists of the five workloads.  It holds none of the method's arithmetic:
no grids, face positions, stencils, kernels, interpolation or time stepping.
Each side samples the closed forms at positions it computes itself.

Workload recipes (stand-ins for the paper's examples; the paper uses no
external data set):

* ``one_d_single``   1-D box, N=256, mu=mu'=4 eps, eps=0.01,
  a = 1 + 0.5 sin(2 pi x / eps), alpha=0.01, eta=eps^2, averaged flux,
  m(x) = normalize(0.5+0.2 cos 2pi(x+phi), 0.3 sin 2pi(x+phi), 1) with a
  seeded phase phi (seed 1); the coefficient is the EX1 coefficient
  (Section 2.3), the initial data mimics EX1's smooth profile.
* ``two_d_batch``    1024 boxes of 64x64 on a 32x32 macro grid, mu=mu'=3 eps,
  eps=1/200, a = 1 + 0.5 sin(2pi x1/eps) sin(2pi x2/eps), alpha=0.1,
  macro field = normalized seeded Gaussian random field (correlation
  length 0.2), fourth-order normalized interpolation init, averaged field.
* ``one_d_batch``    16384 copies of the 1-D box with seeded phases.
* ``uneven_batch``   4096 2-D boxes, N in {32,48,64,96,128}, quasi-periodic
  a = 1 + 0.4 sin(2pi x1/eps) + 0.25 sin(2pi x2/(sqrt2 eps)),
  alpha ~ U[0.01, 0.2], centres ~ U[0,1)^2, explicit init = EX2 initial data.
* ``served``         128x128 macro grid, EX2 macro initial data, per point
  N in {32..128}, eps in {1/100,1/200,1/400}, alpha_micro = 1.2.
* ``three_d_batch``  512 boxes of 32^3 (d = 3), mu = mu' = 3 eps, eps = 1/200,
  a = 1 + 0.5 sin(2pi x1/eps) sin(2pi x2/eps) sin(2pi x3/eps), alpha = 0.1,
  eta = eps^2, smooth 3-D initial data at seeded centres, FP64.
* ``three_d_batch_o4``  the same boxes with the fourth-order stencil.
* HMM loop setups (Section 4.5, fig:hmm_err_ex3): EX2 on the periodic unit
  square, alpha = 0.01, T = 0.1, alpha_micro = 1.2, mu = 3.9 eps, Dirichlet
  micro boxes, averaging kernels p = 3, q = 7.  eps = 1/384 (the paper: 1/400)
  so that every macro node x = i dX, dX in {1/12, 1/24, 1/48, 1/96}, is a
  multiple of eps, and dx = eps / P with an integer P, so all micro grids sit at
  the same phase of a^eps.  s1-s4 take the paper's eta / eps^2 and the box
  size mu' nearest the paper's that a supported N gives; s5 is an extra setup
  with a smaller averaging error.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# Enumerations mirrored from include/llhmm.h (kept as plain ints here).
FP64, FP32 = 0, 1
INTEG_AUTO, HEUNP, RK4P = 0, 1, 2
BC_PERIODIC_PERT, BC_DIRICHLET = 0, 1
Q_FIELD, Q_FLUX, Q_TORQUE = 0, 1, 2
INIT_EXPLICIT, INIT_MACRO_Q = 0, 1

TWO_PI = 2.0 * math.pi


# --------------------------------------------------------------------------
# Material coefficients: a(x) = c0 + sum_t amp_t prod_axis s_{t,axis}(x_axis)
# with s(x) = 1 when its frequency is 0, else sin(2 pi f x + phase).
# --------------------------------------------------------------------------
@dataclass
class SinSum:
    dim: int
    c0: float
    terms: list = field(default_factory=list)   # [(amp, [(freq, phase)]*dim)]
    a_min: float = 0.0                          # (A1) bounds, stated by hand
    a_max: float = 0.0

    def __call__(self, *xs):
        xs = [np.asarray(x, dtype=np.float64) for x in xs]
        out = np.full(np.broadcast(*xs).shape, self.c0, dtype=np.float64)
        for amp, axes in self.terms:
            prod = np.full(out.shape, amp, dtype=np.float64)
            for (f, ph), x in zip(axes, xs):
                if f != 0.0:
                    prod = prod * np.sin(TWO_PI * f * x + ph)
            out = out + prod
        return out


def coef_ex1(eps, dim=1):
    """EX1 / config-1 coefficient a = 1 + 0.5 sin(2 pi x1 / eps)."""
    axes = [(1.0 / eps, 0.0)] + [(0.0, 0.0)] * (dim - 1)
    return SinSum(dim, 1.0, [(0.5, axes)], a_min=0.5, a_max=1.5)


def coef_product(eps):
    """Config-2 coefficient a = 1 + 0.5 sin(2pi x1/eps) sin(2pi x2/eps)."""
    return SinSum(2, 1.0, [(0.5, [(1.0 / eps, 0.0), (1.0 / eps, 0.0)])],
                  a_min=0.5, a_max=1.5)


def coef_quasi(eps):
    """Config-4/5 quasi-periodic a = 1 + 0.4 sin(2pi x1/eps) + 0.25 sin(2pi x2/(sqrt2 eps))."""
    return SinSum(2, 1.0, [(0.4, [(1.0 / eps, 0.0), (0.0, 0.0)]),
                           (0.25, [(0.0, 0.0), (1.0 / (math.sqrt(2.0) * eps), 0.0)])],
                  a_min=0.35, a_max=1.65)


def coef_ex3(eps):
    """EX3 a = (1.1 + 0.5 sin 2pi x1/eps)(1.1 + 0.5 sin 2pi x2/eps), expanded."""
    f = 1.0 / eps
    return SinSum(2, 1.21, [(0.55, [(f, 0.0), (0.0, 0.0)]),
                            (0.55, [(0.0, 0.0), (f, 0.0)]),
                            (0.25, [(f, 0.0), (f, 0.0)])],
                  a_min=0.36, a_max=2.56)


def coef_ex2(eps):
    """EX2 a = 0.5 + (0.5+0.25 s1)(0.5+0.25 s2) + 0.25 (cos 2pi(y1-y2) + s1), y = x/eps.

    Expanded with cos(u-v) = cos u cos v + sin u sin v and cos u = sin(u + pi/2).
    """
    f = 1.0 / eps
    h = 0.5 * math.pi
    return SinSum(2, 0.75, [(0.125 + 0.25, [(f, 0.0), (0.0, 0.0)]),
                            (0.125, [(0.0, 0.0), (f, 0.0)]),
                            (0.0625 + 0.25, [(f, 0.0), (f, 0.0)]),
                            (0.25, [(f, h), (f, h)])],
                  a_min=0.2, a_max=1.6)


def coef_layered3(eps):
    """3-D laminate a = 1 + 0.5 sin(2 pi x1 / eps): its homogenized matrix is
    diag(harmonic mean, mean, mean) = diag(sqrt(0.75), 1, 1)."""
    f = 1.0 / eps
    return SinSum(3, 1.0, [(0.5, [(f, 0.0), (0.0, 0.0), (0.0, 0.0)])], a_min=0.5, a_max=1.5)


def coef_product3(eps):
    """a = 1 + 0.5 sin(2 pi x1/eps) sin(2 pi x2/eps) sin(2 pi x3/eps)."""
    f = 1.0 / eps
    return SinSum(3, 1.0, [(0.5, [(f, 0.0), (f, 0.0), (f, 0.0)])], a_min=0.5, a_max=1.5)


def coef_const(c, dim):
    return SinSum(dim, float(c), [], a_min=float(c), a_max=float(c))


def coef_smooth_periodic(dim, period):
    """A smooth coefficient that is periodic with the given period on every axis
    (used for energy and manufactured-solution checks)."""
    f = 1.0 / period
    if dim == 1:
        return SinSum(1, 1.0, [(0.3, [(f, 0.4)])], a_min=0.7, a_max=1.3)
    return SinSum(2, 1.0, [(0.3, [(f, 0.4), (0.0, 0.0)]),
                           (0.2, [(0.0, 0.0), (f, 1.1)]),
                           (0.1, [(f, 0.2), (f, 0.7)])], a_min=0.4, a_max=1.6)


# --------------------------------------------------------------------------
# Closed-form initial magnetisations (normalized by definition of the input).
# --------------------------------------------------------------------------
def _normalize(v):
    return v / np.sqrt(np.sum(v * v, axis=0, keepdims=True))


@dataclass
class InitCfg1:
    """m(x) = normalize(0.5+0.2 cos 2pi(x+phi), 0.3 sin 2pi(x+phi), 1)."""
    phi: float = 0.0

    def __call__(self, x1, *unused):
        t = TWO_PI * (np.asarray(x1, dtype=np.float64) + self.phi)
        v = np.stack([0.5 + 0.2 * np.cos(t), 0.3 * np.sin(t), np.ones_like(t)])
        return _normalize(v)


@dataclass
class InitEX1:
    def __call__(self, x1, *unused):
        x = np.asarray(x1, dtype=np.float64)
        v = np.stack([0.5 + np.exp(-0.1 * np.cos(TWO_PI * (x - 0.32))),
                      0.5 + np.exp(-0.2 * np.cos(TWO_PI * x)),
                      0.5 + np.exp(-0.1 * np.cos(TWO_PI * (x - 0.75)))])
        return _normalize(v)


@dataclass
class InitEX2:
    """EX2/EX3 initial data (Section 2.3)."""
    def __call__(self, x1, x2):
        x1 = np.asarray(x1, dtype=np.float64)
        x2 = np.asarray(x2, dtype=np.float64)
        c = np.cos
        v = np.stack([
            0.6 + np.exp(-0.3 * (c(TWO_PI * (x1 - 0.25)) + c(TWO_PI * (x2 - 0.12)))),
            0.5 + np.exp(-0.4 * (c(TWO_PI * x1) + c(TWO_PI * (x2 - 0.4)))),
            0.4 + np.exp(-0.2 * (c(TWO_PI * (x1 - 0.81)) + c(TWO_PI * (x2 - 0.73)))),
        ])
        return _normalize(v)


@dataclass
class InitSmooth3D:
    """A smooth normalized 3-D field built like the EX2 data (Section 2.3)."""
    def __call__(self, x1, x2, x3):
        x1, x2, x3 = (np.asarray(v, dtype=np.float64) for v in (x1, x2, x3))
        c = np.cos
        v = np.stack([
            0.6 + np.exp(-0.3 * (c(TWO_PI * (x1 - 0.25)) + c(TWO_PI * (x2 - 0.12)) + c(TWO_PI * x3))),
            0.5 + np.exp(-0.4 * (c(TWO_PI * x1) + c(TWO_PI * (x2 - 0.4)) + c(TWO_PI * (x3 - 0.3)))),
            0.4 + np.exp(-0.2 * (c(TWO_PI * (x1 - 0.81)) + c(TWO_PI * (x2 - 0.73)) + c(TWO_PI * (x3 - 0.6)))),
        ])
        return _normalize(v)


@dataclass
class InitSmoothPeriodic:
    """A normalized initial field that is periodic with the given period."""
    period: float
    dim: int = 1

    def __call__(self, x1, x2=None):
        f = TWO_PI / self.period
        x1 = np.asarray(x1, dtype=np.float64)
        x2 = np.zeros_like(x1) if x2 is None else np.asarray(x2, dtype=np.float64)
        v = np.stack([0.6 + 0.3 * np.cos(f * x1 + 0.2) + 0.1 * np.sin(f * x2),
                      0.4 + 0.3 * np.sin(f * x1 + 0.5 * np.cos(f * x2)),
                      0.8 + 0.2 * np.cos(f * (x1 + x2))])
        return _normalize(v)


# --------------------------------------------------------------------------
# Seeded Gaussian random field on the unit torus (config 2's macro field).
# --------------------------------------------------------------------------
def gaussian_random_field(seed, n_macro, corr=0.2, kmax=6, refine=4, min_norm=0.25):
    """Normalized 3-vector field sampled at x_i = i/n_macro, i in [0,n_macro)^2.

    Each component is an independent zero-mean unit-variance Fourier sum with
    Gaussian covariance exp(-r^2 / (2 corr^2)); the draw is rejected and
    re-seeded (seed+1, ...) when the raw vector length falls below min_norm on
    a grid refined by `refine`.
    """
    k = np.arange(-kmax, kmax + 1)
    k1, k2 = np.meshgrid(k, k, indexing="ij")
    spec = np.exp(-2.0 * math.pi ** 2 * corr ** 2 * (k1 ** 2 + k2 ** 2))
    amp = np.sqrt(spec / spec.sum())
    s = seed
    while True:
        rng = np.random.default_rng(s)
        xi = rng.standard_normal((3,) + k1.shape)
        zeta = rng.standard_normal((3,) + k1.shape)

        def sample(n):
            x = np.arange(n) / n
            X1, X2 = np.meshgrid(x, x, indexing="ij")
            ph = TWO_PI * (k1[..., None, None] * X1 + k2[..., None, None] * X2)
            c, sn = np.cos(ph), np.sin(ph)
            out = np.einsum("kl,cklij->cij", amp, xi[:, :, :, None, None] * c
                            + zeta[:, :, :, None, None] * sn)
            return out

        fine = sample(n_macro * refine)
        if np.sqrt((fine ** 2).sum(axis=0)).min() >= min_norm:
            raw = sample(n_macro)
            return _normalize(raw), s
        s += 1


# --------------------------------------------------------------------------
# Box lists.  A box is a dict with the llhmm_box fields (see include/llhmm.h).
# --------------------------------------------------------------------------
def make_box(**kw):
    box = dict(dim=1, n=64, order=2, integrator=INTEG_AUTO, bc=BC_PERIODIC_PERT,
               quantity=Q_FIELD, init_mode=INIT_EXPLICIT, n_steps=0, coef_index=0,
               eps=0.01, alpha=0.1, mu=0.03, mu_box=0.03, eta=1e-4, a_max=1.5,
               center=(0.0, 0.0), macro_index=(0, 0))
    box.update(kw)
    return box


@dataclass
class Workload:
    name: str
    dim: int
    boxes: list
    coefs: list
    init: object = None          # closed-form callable for INIT_EXPLICIT
    inits: list = None           # per-box callables (overrides init)
    macro: dict = None           # {'n': n, 'dX': dX, 'x0': (..), 'M': array[3,n,n]}
    precision: int = FP64
    kernel: tuple = (3, 7, 3, 7)  # p_x, q_x, p_t, q_t

    def init_of(self, i):
        return self.inits[i] if self.inits is not None else self.init


def one_d_single(seed=1, precision=FP64, order=2, n=256):
    eps = 0.01
    phi = float(np.random.default_rng(seed).random())
    box = make_box(dim=1, n=n, order=order, quantity=Q_FLUX, eps=eps, alpha=0.01,
                   mu=4 * eps, mu_box=4 * eps, eta=eps ** 2, a_max=1.5, center=(0.0, 0.0))
    return Workload("one_d_single", 1, [box], [coef_ex1(eps)], init=InitCfg1(phi),
                    precision=precision)


def one_d_batch(nboxes=16384, seed=1, precision=FP32, order=2, n=256):
    eps = 0.01
    phis = np.random.default_rng(seed).random(nboxes)
    boxes = [make_box(dim=1, n=n, order=order, quantity=Q_FLUX, eps=eps, alpha=0.01,
                      mu=4 * eps, mu_box=4 * eps, eta=eps ** 2, a_max=1.5)
             for _ in range(nboxes)]
    return Workload("one_d_batch", 1, boxes, [coef_ex1(eps)],
                    inits=[InitCfg1(float(p)) for p in phis], precision=precision)


def two_d_batch(n_macro=32, seed=2, precision=FP64, order=2, n=64, integrator=INTEG_AUTO):
    eps = 1.0 / 200.0
    M, used_seed = gaussian_random_field(seed, n_macro)
    boxes = []
    for i in range(n_macro):
        for j in range(n_macro):
            boxes.append(make_box(dim=2, n=n, order=order, integrator=integrator,
                                  quantity=Q_FIELD, init_mode=INIT_MACRO_Q, eps=eps,
                                  alpha=0.1, mu=3 * eps, mu_box=3 * eps, eta=eps ** 2,
                                  a_max=1.5, center=(i / n_macro, j / n_macro),
                                  macro_index=(i, j)))
    macro = dict(n=n_macro, dX=1.0 / n_macro, x0=(0.0, 0.0), M=M, seed=used_seed)
    return Workload("two_d_batch" if order == 2 else "two_d_batch_o4", 2, boxes, [coef_product(eps)],
                    macro=macro, precision=precision)


def two_d_batch_o4(n_macro=32, seed=2, precision=FP64):
    """two_d_batch with the fourth-order conservative stencil."""
    return two_d_batch(n_macro, seed, precision, order=4)


def three_d_batch(nboxes=512, seed=6, n=32, precision=FP64, order=2):
    """512 boxes of 32^3 (d = 3): eps = 1/200, mu = mu' = 3 eps, eta = eps^2,
    alpha = 0.1 (RK4P), periodic m - m_init, a = 1 + 0.5 prod_k sin(2 pi x_k / eps),
    explicit smooth 3-D initial data at seeded centres; field average."""
    eps = 1.0 / 200.0
    centres = np.random.default_rng(seed).random((nboxes, 3))
    boxes = [make_box(dim=3, n=n, order=order, quantity=Q_FIELD, eps=eps, alpha=0.1, mu=3 * eps,
                      mu_box=3 * eps, eta=eps ** 2, a_max=1.5,
                      center=tuple(float(v) for v in centres[b]), macro_index=(0, 0, 0))
             for b in range(nboxes)]
    return Workload("three_d_batch", 3, boxes, [coef_product3(eps)], init=InitSmooth3D(),
                    precision=precision)


def three_d_batch_o4(nboxes=512, seed=6, n=32, precision=FP64):
    """The d = 3 batch above with the fourth-order conservative stencil."""
    wl = three_d_batch(nboxes, seed, n, precision, order=4)
    wl.name = "three_d_batch_o4"
    return wl


UNEVEN_SIZES = (32, 48, 64, 96, 128)


def uneven_batch(nboxes=4096, seed=4, precision=FP32, sizes=UNEVEN_SIZES, order=2):
    eps = 1.0 / 200.0
    rng = np.random.default_rng(seed)
    ns = rng.choice(np.array(sizes), size=nboxes)
    alphas = rng.uniform(0.01, 0.2, size=nboxes)
    centres = rng.random((nboxes, 2))
    boxes = [make_box(dim=2, n=int(ns[b]), order=order, quantity=Q_FIELD,
                      init_mode=INIT_EXPLICIT, eps=eps, alpha=float(alphas[b]),
                      mu=3 * eps, mu_box=3 * eps, eta=eps ** 2, a_max=1.65,
                      center=(float(centres[b, 0]), float(centres[b, 1])))
             for b in range(nboxes)]
    return Workload("uneven_batch", 2, boxes, [coef_quasi(eps)], init=InitEX2(),
                    precision=precision)


SERVED_EPS = (1.0 / 100.0, 1.0 / 200.0, 1.0 / 400.0)

HMM_EPS = 1.0 / 384.0
# name: (points per eps P, micro N, eta / eps^2); mu' = N / (2 P) eps.
HMM_SETUPS = {
    "s1": (6, 48, 0.15),     # mu' = 4 eps     (paper: 4)
    "s2": (6, 64, 0.45),     # mu' = 5.33 eps  (paper: 5.5)
    "s3": (6, 96, 0.7),      # mu' = 8 eps     (paper: 7.5)
    "s4": (6, 128, 1.0),     # mu' = 10.67 eps (paper: 10)
    "s5": (5, 128, 2.0),     # mu' = 12.8 eps
}


def hmm_micro(setup, eps=HMM_EPS, alpha=1.2, mu_over_eps=3.9):
    """Box fields shared by every micro problem of an HMM loop setup."""
    ppe, n, eta = HMM_SETUPS[setup]
    return dict(n=n, order=2, integrator=INTEG_AUTO, bc=BC_DIRICHLET, eps=eps, alpha=alpha,
                mu=mu_over_eps * eps, mu_box=0.5 * n / ppe * eps, eta=eta * eps * eps,
                a_max=1.6)


def ex2_macro(n_macro):
    """EX2 initial data at the macro nodes x = (i, j) / n_macro, [3, n, n]."""
    x = np.arange(n_macro) / n_macro
    X1, X2 = np.meshgrid(x, x, indexing="ij")
    return InitEX2()(X1, X2)


def served_points(n_macro=128, seed=5, sizes=UNEVEN_SIZES):
    """Per macro point (fixed across stages): micro N, eps index."""
    rng = np.random.default_rng(seed)
    ns = rng.choice(np.array(sizes), size=n_macro * n_macro)
    ei = rng.integers(0, len(SERVED_EPS), size=n_macro * n_macro)
    return ns, ei


def served_boxes(n_macro=128, seed=5, sizes=UNEVEN_SIZES, order=2):
    ns, ei = served_points(n_macro, seed, sizes)
    coefs = [coef_quasi(e) for e in SERVED_EPS]
    boxes = []
    for i in range(n_macro):
        for j in range(n_macro):
            p = i * n_macro + j
            eps = SERVED_EPS[ei[p]]
            boxes.append(make_box(dim=2, n=int(ns[p]), order=order, integrator=INTEG_AUTO,
                                  quantity=Q_FIELD, init_mode=INIT_MACRO_Q,
                                  coef_index=int(ei[p]), eps=eps, alpha=1.2,
                                  mu=3 * eps, mu_box=3 * eps, eta=eps ** 2, a_max=1.65,
                                  center=(i / n_macro, j / n_macro), macro_index=(i, j)))
    return boxes, coefs


def served_macro(n_macro=128):
    x = np.arange(n_macro) / n_macro
    X1, X2 = np.meshgrid(x, x, indexing="ij")
    return InitEX2()(X1, X2)


def burst_sizes(total, seed, lo=256, hi=4096):
    rng = np.random.default_rng(seed)
    out, left = [], total
    while left > 0:
        b = int(min(left, rng.integers(lo, hi + 1)))
        out.append(b)
        left -= b
    return out
