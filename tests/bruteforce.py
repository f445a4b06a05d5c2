"""Independent brute-force reference for tiny micro problems (pins the oracle).

Written separately from oracle/: dense linear operators on an extended grid,
numpy cross products, a generic explicit Butcher-tableau loop, kernels fitted by
Gauss-Legendre quadrature, and an explicit double sum for the average.  Only
the closed-form inputs (paper_2108_09463_amd.inputs) are shared.
"""
from __future__ import annotations

import numpy as np

G = 3


def kernel_poly(p, q, one_sided):
    """Coefficients of K (or K0) from the moment conditions, by quadrature."""
    x, w = np.polynomial.legendre.leggauss(80)
    if one_sided:
        t = 0.5 * (x + 1.0)
        wt = 0.5 * w
        base = t ** (q + 1) * (1 - t) ** (q + 1)
    else:
        t, wt = x, w
        base = (1 - t * t) ** (q + 1)
    A = np.array([[np.sum(wt * base * t ** (r + i)) for i in range(p + 1)] for r in range(p + 1)])
    rhs = np.zeros(p + 1)
    rhs[0] = 1.0
    return np.linalg.solve(A, rhs)


def kernel_eval(c, q, x, one_sided):
    x = np.asarray(x, dtype=float)
    poly = sum(ci * x ** i for i, ci in enumerate(c))
    if one_sided:
        v = x ** (q + 1) * (1 - x) ** (q + 1) * poly
        return np.where((x > 0) & (x < 1), v, 0.0)
    v = (1 - x * x) ** (q + 1) * poly
    return np.where(np.abs(x) < 1, v, 0.0)


class Problem:
    """One micro box as dense operators on the flattened interior state."""

    def __init__(self, box, coef, init_fn=None, minit_ext=None):
        self.d, self.n = box["dim"], box["n"]
        self.order, self.bc = box["order"], box["bc"]
        n, d = self.n, self.d
        self.h = 2.0 * box["mu_box"] / n
        self.E = n + 2 * G
        j = np.arange(-G, n + G)
        self.xi = -box["mu_box"] + self.h * j
        c = box["center"]
        if minit_ext is None:
            if d == 1:
                minit_ext = init_fn(c[0] + self.xi)
            elif d == 2:
                X, Y = np.meshgrid(c[0] + self.xi, c[1] + self.xi, indexing="xy")
                minit_ext = init_fn(X, Y)
            else:
                # storage [i2][i1][i0]: the last meshgrid axis runs fastest
                Z, Y, X = np.meshgrid(c[2] + self.xi, c[1] + self.xi, c[0] + self.xi, indexing="ij")
                minit_ext = init_fn(X, Y, Z)
        self.mext0 = np.asarray(minit_ext, float).reshape(3, -1)
        ncell = n ** d
        next_ = self.E ** d
        # extension map: m_ext = P m + q  (per component, q depends on component)
        P = np.zeros((next_, ncell))
        qv = np.zeros((3, next_))
        for e in range(next_):
            idx = self._unravel(e, self.E)
            idx = [k - G for k in idx]             # (i0, i1, ...) interior coordinates
            inside = all(0 <= k < n for k in idx)
            if inside:
                P[e, self._cell(idx)] = 1.0
                continue
            n_out = sum(not (0 <= k < n) for k in idx)
            if n_out > 1:
                continue                           # corner ghosts: never used
            wrapped = [k % n for k in idx]
            ew = self._ext(wrapped)
            if self.bc == 0:
                P[e, self._cell(wrapped)] = 1.0
                qv[:, e] = self.mext0[:, e] - self.mext0[:, ew]
            else:
                qv[:, e] = self.mext0[:, e]
        self.P, self.q = P, qv
        # face gradient and divergence on the extended grid, per axis
        self.div = np.zeros((ncell, next_))
        self.faceflux = []                          # per axis: matrix ext -> east-face flux of cells
        for ax in range(d):
            s = self.E ** ax
            A = np.zeros(next_)
            for e in range(next_):
                idx = self._unravel(e, self.E)
                pos = [c[k] + self.xi[idx[k]] for k in range(d)]
                pos[ax] += 0.5 * self.h
                A[e] = coef(*pos)
            Gm = np.zeros((next_, next_))          # gradient on face e (between e and e+s)
            for e in range(next_):
                if self.order == 2:
                    pts = {e + s: 1.0, e: -1.0}
                    scale = 1.0 / self.h
                else:
                    pts = {e + s: 27.0, e: -27.0, e + 2 * s: -1.0, e - s: 1.0}
                    scale = 1.0 / (24.0 * self.h)
                if all(0 <= p < next_ for p in pts):
                    for p, v in pts.items():
                        Gm[e, p] += v * scale
            F = A[:, None] * Gm                      # flux on faces
            cells = [self._ext(list(self._unravel(ci, n))) for ci in range(ncell)]
            for ci, e in enumerate(cells):
                if self.order == 2:
                    self.div[ci] += (F[e] - F[e - s]) / self.h
                else:
                    self.div[ci] += (27.0 * (F[e] - F[e - s]) - (F[e + s] - F[e - 2 * s])) / (24.0 * self.h)
            self.faceflux.append(np.array([F[e] for e in cells]))

    def _unravel(self, e, size):
        """(i0, i1, ...) of flat index e, axis 0 fastest."""
        return tuple(int(v) for v in np.unravel_index(e, (size,) * self.d)[::-1])

    def _cell(self, idx):
        return sum(int(idx[k]) * self.n ** k for k in range(self.d))

    def _ext(self, idx):
        return sum((int(idx[k]) + G) * self.E ** k for k in range(self.d))

    def field(self, m):
        """H for interior state m [3, ncell]."""
        return np.stack([self.div @ (self.P @ m[c] + self.q[c]) for c in range(3)])

    def fluxes(self, m):
        return [np.stack([F @ (self.P @ m[c] + self.q[c]) for c in range(3)]) for F in self.faceflux]

    def interior0(self):
        n, d = self.n, self.d
        return np.stack([np.array([self.mext0[c, self._ext(list(self._unravel(ci, n)))]
                                   for ci in range(n ** d)]) for c in range(3)])


TABLEAUS = {
    1: (np.array([[0.0, 0.0], [1.0, 0.0]]), np.array([0.5, 0.5])),
    2: (np.array([[0, 0, 0, 0], [0.5, 0, 0, 0], [0, 0.5, 0, 0], [0, 0, 1.0, 0]]),
        np.array([1, 2, 2, 1]) / 6.0),
}


def solve(box, coef, init_fn=None, minit_ext=None, M=None, integ=None, kernel=(3, 7, 3, 7)):
    prob = Problem(box, coef, init_fn, minit_ext)
    alpha = box["alpha"]
    A, b = TABLEAUS[integ]
    dt = box["eta"] / M
    cx = kernel_poly(kernel[0], kernel[1], False)
    ct = kernel_poly(kernel[2], kernel[3], True)
    n, d = prob.n, prob.d
    xs = -box["mu_box"] + prob.h * np.arange(n)
    w1 = kernel_eval(cx, kernel[1], xs / box["mu"], False) * prob.h / box["mu"]
    wf1 = kernel_eval(cx, kernel[1], (xs + 0.5 * prob.h) / box["mu"], False) * prob.h / box["mu"]
    def prod(ws):
        """Product weight over the cells, flat in storage order (axis 0 fastest);
        ws[a] is the weight vector along axis a."""
        out = ws[0]
        for a in range(1, d):
            out = np.multiply.outer(ws[a], out)
        return out.reshape(-1)

    wcell = prod([w1] * d)
    wflux = [prod([wf1 if a == ax else w1 for a in range(d)]) for ax in range(d)]
    wt = kernel_eval(ct, kernel[3], np.arange(M + 1) / M, True) / M

    def f(m):
        H = prob.field(m)
        return -np.cross(m, H, axis=0) - alpha * np.cross(m, np.cross(m, H, axis=0), axis=0)

    m = prob.interior0()
    q = box["quantity"]
    out = np.zeros(3 * d if q == 1 else 3)
    for step in range(M + 1):
        H = prob.field(m)
        if q == 0:
            Q = [H]
        elif q == 2:
            Q = [np.cross(m, H, axis=0)]
        else:
            Q = prob.fluxes(m)
        for ax, Qa in enumerate(Q):
            W = wcell if q != 1 else wflux[ax]
            for c in range(3):
                for jj in range(W.size):          # the explicit double sum
                    out[3 * ax + c] += wt[step] * W[jj] * Qa[c, jj]
        if step == M:
            break
        ks = []
        for s in range(len(b)):
            y = m + dt * sum(A[s, r] * ks[r] for r in range(s))
            ks.append(f(y))
        m = m + dt * sum(b[s] * ks[s] for s in range(len(b)))
        m = m / np.linalg.norm(m, axis=0)
    return out, m
