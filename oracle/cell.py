"""Homogenized coefficient A^H (eq. (AH) and eq. (cell_problem), Section 2.1).

Used only to pin the micro solver against homogenization theory (Theorem 2:
H_avg approaches div(grad m_init(0) A^H) up to the averaging errors).

* 1-D: A^H = (int_0^1 1/a)^-1 (the harmonic mean; EX1 prints ~0.866).
* 2-D: second-order finite-volume discretization of div(a grad chi_k) = -d_k a
  on an n x n periodic unit cell, solved with a sparse direct solver (one value
  pinned to remove the constant null space); A^H_jk is the cell average of the
  j-th component of the flux a (e_k + grad chi_k) on the j-faces.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def harmonic_mean_1d(a_fun, n=200000):
    y = (np.arange(n) + 0.5) / n
    return 1.0 / np.mean(1.0 / a_fun(y))


def homogenized_2d(a_fun, n=128):
    h = 1.0 / n
    y = np.arange(n) * h
    Y0, Y1 = np.meshgrid(y, y, indexing="ij")          # [i0][i1]
    a_face = [a_fun(Y0 + 0.5 * h, Y1), a_fun(Y0, Y1 + 0.5 * h)]  # face between i and i+e_ax

    def idx(i0, i1):
        return (i0 % n) * n + (i1 % n)

    rows, cols, vals = [], [], []
    I0, I1 = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    I0, I1 = I0.ravel(), I1.ravel()
    me = idx(I0, I1)
    for ax in range(2):
        af = a_face[ax].ravel()
        am = np.roll(a_face[ax], 1, axis=ax).ravel()   # face between i-e and i
        nb_p = idx(I0 + (ax == 0), I1 + (ax == 1))
        nb_m = idx(I0 - (ax == 0), I1 - (ax == 1))
        rows += [me, me, me, me]
        cols += [nb_p, me, nb_m, me]
        vals += [af / h ** 2, -af / h ** 2, am / h ** 2, -am / h ** 2]
    L = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(n * n, n * n)).tolil()
    L[0, :] = 0.0
    L[0, 0] = 1.0
    L = L.tocsc()
    AH = np.zeros((2, 2))
    for k in range(2):
        af = a_face[k]
        am = np.roll(a_face[k], 1, axis=k)
        rhs = -((af - am) / h).ravel()
        rhs[0] = 0.0
        chi = spla.spsolve(L, rhs).reshape(n, n)
        for j in range(2):
            grad = (np.roll(chi, -1, axis=j) - chi) / h
            flux = a_face[j] * ((1.0 if j == k else 0.0) + grad)
            AH[j, k] = flux.mean()
    return AH
