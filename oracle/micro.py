"""Oracle set-up of one micro problem and the call into the FP64 C loop (micro.c).

Steps (paper passages in brackets):
  O1 grid    xi_j = -mu' + j dx, dx = 2 mu' / N, j in [0, N), with 3 ghost
             layers per side; absolute position x = x_c + xi [eq. (micro),
             Section 2.3: the micro domain [-mu', mu']^d around x_i].
             Reading: the N grid points start at -mu'; the point +mu' is the
             periodic image of -mu' (periodic m - m_init) or the first ghost
             (Dirichlet).  The box centre is the grid point j = N/2.
  O2 faces   a^eps at face midpoints, absolute coordinates [eq. (prob)].
  O3 init    explicit closed form, or the normalized interpolant
             Q_[4] = P_[4] / |P_[4]| of the macro values around x_k: 1-D
             Lagrange interpolation on the 5 macro nodes x_k + l dX,
             l = -2..2, applied along x1 then x2 [Section 4.1, eq. (Q_k)],
             at the absolute positions x_c + xi (the centre x_c may lie
             between nodes, e.g. the staggered points of the flux model).
             Macro indices wrap periodically (the macro domain is periodic).
  O8 plan    oracle.stability.plan_steps, or a forced number of steps.
  O9/O10     oracle.kernels weights.
  O4-O7, O11, O12 in micro.c.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

from . import kernels, stability

GW = 3
_HERE = os.path.dirname(os.path.abspath(__file__))
_LIBS = {}
_BUILD_LOCK = threading.Lock()   # threads of one process share the build

# Build variants of the same C source.  "plain": no FMA contraction (the
# oracle).  "fma": identical algorithm with a*b+c contracted to fused
# multiply-adds; the spread between the two measures the FP64 rounding floor
# of a result, which bounds how closely any other correct FP64 implementation
# can be expected to agree with the oracle.
_VARIANTS = {"plain": ["-ffp-contract=off"], "fma": ["-ffp-contract=fast", "-mfma"],
             "ld": ["-ffp-contract=off", "-DORACLE_LONG_DOUBLE"],
             "quad": ["-ffp-contract=off", "-DORACLE_QUAD"]}
# "ld" (x87 extended precision) and "quad" (binary128, libquadmath): the same
# algorithm in higher precision on the same FP64 inputs, the answers against
# which FP64 results are measured.  "ld" is the one the parity tests use (about
# three times the FP64 cost); "quad" (about 150 times) pins it on small boxes.


def lib_path(variant="plain"):
    name = "liboracle.so" if variant == "plain" else "liboracle_%s.so" % variant
    return os.path.join(_HERE, "_build", name)


def build(force=False, variant="plain"):
    """Compile micro.c with gcc (-O2, no fast-math)."""
    out = lib_path(variant)
    src = os.path.join(_HERE, "micro.c")
    if not force and os.path.exists(out) and os.path.getmtime(out) >= os.path.getmtime(src):
        return out
    os.makedirs(os.path.dirname(out), exist_ok=True)
    tmp = out + ".tmp%d_%d" % (os.getpid(), threading.get_ident())
    libs = ["-lquadmath", "-lm"] if variant == "quad" else ["-lm"]
    subprocess.check_call(["gcc", "-O2", "-std=gnu99", "-fPIC", "-shared"] + _VARIANTS[variant] +
                          ["-o", tmp, src] + libs)
    os.replace(tmp, out)
    return out


def _lib(variant="plain"):
    with _BUILD_LOCK:
        return _lib_locked(variant)


def _lib_locked(variant):
    if variant not in _LIBS:
        L = ctypes.CDLL(build(variant=variant))
        dp = ctypes.POINTER(ctypes.c_double)
        L.oracle_solve_box.argtypes = [ctypes.c_int] * 7 + [ctypes.c_double] * 3 + [ctypes.c_int] + [dp] * 9
        L.oracle_solve_box.restype = ctypes.c_int
        L.oracle_eval_field.argtypes = [ctypes.c_int] * 4 + [ctypes.c_double] + [dp] * 4
        L.oracle_eval_field.restype = ctypes.c_int
        _LIBS[variant] = L
    return _LIBS[variant]


def _ptr(a):
    if a is None:
        return ctypes.POINTER(ctypes.c_double)()
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


# ---------------------------------------------------------------- O1, O2, O3
def grid_positions(n, mu_box):
    """xi_j for j = -GW .. n+GW-1 and the spacing dx."""
    dx = 2.0 * mu_box / n
    j = np.arange(-GW, n + GW, dtype=np.float64)
    return -mu_box + j * dx, dx


def face_coefficients(box, coef):
    """A[ax] on the extended grid: a^eps on the face between cell idx and idx + e_ax."""
    d, n = box["dim"], box["n"]
    xi, dx = grid_positions(n, box["mu_box"])
    c = box["center"]
    if d == 1:
        return np.ascontiguousarray(coef(c[0] + xi + 0.5 * dx)[None, :]), dx
    if d == 2:
        X0, X1 = np.meshgrid(c[0] + xi, c[1] + xi, indexing="xy")   # [i1][i0]
        a0 = coef(X0 + 0.5 * dx, X1)
        a1 = coef(X0, X1 + 0.5 * dx)
        return np.ascontiguousarray(np.stack([a0, a1])), dx
    X0, X1, X2 = grid3(c, xi)                                       # [i2][i1][i0]
    a = [coef(X0 + 0.5 * dx, X1, X2), coef(X0, X1 + 0.5 * dx, X2), coef(X0, X1, X2 + 0.5 * dx)]
    return np.ascontiguousarray(np.stack(a)), dx


def grid3(c, xi):
    """Absolute coordinates of the 3-D extended grid, each shaped [i2][i1][i0]."""
    X2, X1, X0 = np.meshgrid(c[2] + xi, c[1] + xi, c[0] + xi, indexing="ij")
    return X0, X1, X2


def lagrange5(s):
    """Basis L_l(s), l = -2..2, on the nodes -2..2; shape (5,) + s.shape."""
    s = np.asarray(s, dtype=np.float64)
    nodes = [-2, -1, 0, 1, 2]
    out = []
    for l in nodes:
        v = np.ones_like(s)
        for mm in nodes:
            if mm != l:
                v = v * (s - mm) / (l - mm)
        out.append(v)
    return np.stack(out)


def q4_interpolant(macro, k, xi_axes):
    """Q_[4] at the tensor grid xi_axes (tuple of 1-D arrays) around macro node k.

    macro: dict(n, dX, M[3, n(, n(, n))]).  Returns [3] + grid shape with axis 0
    fastest: [3, len(xi1), len(xi0)] in 2-D, [3, len(xi2), len(xi1), len(xi0)] in 3-D.
    """
    n, dX, M = macro["n"], macro["dX"], np.asarray(macro["M"], dtype=np.float64)
    if len(xi_axes) == 3:
        Ls = [lagrange5(x / dX) for x in xi_axes]            # [5, n_a] per axis
        ids = [[(k[a] + l) % n for l in range(-2, 3)] for a in range(3)]
        vals = M[:, ids[0]][:, :, ids[1]][:, :, :, ids[2]]   # [3, l0, l1, l2]
        # along x1, then x2, then x3
        t0 = np.einsum("cabe,ai->cibe", vals, Ls[0])          # [3, n0, l1, l2]
        t1 = np.einsum("cibe,bj->cije", t0, Ls[1])            # [3, n0, n1, l2]
        P = np.einsum("cije,ek->ckji", t1, Ls[2])             # [3, n2, n1, n0]
        return P / np.sqrt(np.sum(P * P, axis=0, keepdims=True))
    if len(xi_axes) == 1:
        L0 = lagrange5(xi_axes[0] / dX)                   # [5, n0]
        idx = [(k[0] + l) % n for l in range(-2, 3)]
        vals = M[:, idx]                                  # [3, 5]
        P = np.einsum("cl,lj->cj", vals, L0)
    else:
        L0 = lagrange5(xi_axes[0] / dX)                   # [5, n0] along x1
        L1 = lagrange5(xi_axes[1] / dX)                   # [5, n1] along x2
        i0 = [(k[0] + l) % n for l in range(-2, 3)]
        i1 = [(k[1] + l) % n for l in range(-2, 3)]
        vals = M[:, i0][:, :, i1]                         # [3, l0, l1]
        # interpolate along x1 first, then along x2
        along_x1 = np.einsum("cab,aj->cjb", vals, L0)     # [3, n0, l1]
        P = np.einsum("cjb,bi->cij", along_x1, L1)        # [3, n1, n0]
    return P / np.sqrt(np.sum(P * P, axis=0, keepdims=True))


def node_offsets(box, macro):
    """Position of the box centre relative to its macro node x_k = x0 + k dX, per
    axis.  The interpolant of Section 4.1 is evaluated at absolute positions, so a
    centre between nodes (the staggered flux points of the flux model) shifts
    the Lagrange arguments.  Offsets within 1e-9 dX of zero count as zero, so a
    centre given as i / n and the node 0 + i dX are the same point."""
    dX = macro["dX"]
    x0 = macro.get("x0", (0.0, 0.0, 0.0))
    out = []
    for a in range(box["dim"]):
        o = box["center"][a] - (x0[a] + box["macro_index"][a] * dX)
        out.append(0.0 if abs(o) <= 1e-9 * dX else o)
    return out


def initial_data(box, init_fn=None, macro=None):
    """m_init on the extended grid, [3][E^d] (2-D storage: [3][i1][i0], 3-D:
    [3][i2][i1][i0])."""
    d, n = box["dim"], box["n"]
    xi, dx = grid_positions(n, box["mu_box"])
    c = box["center"]
    if box["init_mode"] == 1:
        k = box["macro_index"]
        off = node_offsets(box, macro)
        axes = tuple(xi + off[a] for a in range(d))
        mi = q4_interpolant(macro, k, axes)
    elif d == 1:
        mi = init_fn(c[0] + xi)
    elif d == 2:
        X0, X1 = np.meshgrid(c[0] + xi, c[1] + xi, indexing="xy")
        mi = init_fn(X0, X1)
    else:
        mi = init_fn(*grid3(c, xi))
    return np.ascontiguousarray(mi.reshape(3, -1), dtype=np.float64)


def plan(box):
    d, n = box["dim"], box["n"]
    dx = 2.0 * box["mu_box"] / n
    integ = stability.resolve_integrator(box["integrator"], box["alpha"])
    if box["n_steps"] > 0:
        M = int(box["n_steps"])
        return integ, M, box["eta"] / M
    M, dt = stability.plan_steps(box["eta"], box["alpha"], integ, box["order"], d,
                                 box["a_max"], dx)
    return integ, M, dt


def weights(box, kernel, M):
    p_x, q_x, p_t, q_t = kernel
    n = box["n"]
    xi, dx = grid_positions(n, box["mu_box"])
    cells = xi[GW:GW + n]
    w = kernels.space_weights(cells, box["mu"], dx, p_x, q_x)
    wf = kernels.space_weights(cells + 0.5 * dx, box["mu"], dx, p_x, q_x)
    wt = kernels.time_weights(M, p_t, q_t)
    return (np.ascontiguousarray(w), np.ascontiguousarray(wf), np.ascontiguousarray(wt))


# ---------------------------------------------------------------- solving a box
def solve_box(box, coef, init_fn=None, macro=None, kernel=(3, 7, 3, 7), project=True,
              want_state=False, want_trace=False, variant="plain"):
    d, n = box["dim"], box["n"]
    A, dx = face_coefficients(box, coef)
    mi = initial_data(box, init_fn, macro)
    integ, M, dt = plan(box)
    w, wf, wt = weights(box, kernel, M)
    nq = 3 * d if box["quantity"] == 1 else 3
    out = np.zeros(nq)
    mfinal = np.zeros(3 * n ** d) if want_state else None
    en = np.zeros(M + 1) if want_trace else None
    nd = np.zeros(M + 1) if want_trace else None
    rc = _lib(variant).oracle_solve_box(d, n, box["order"], integ, box["bc"], box["quantity"],
                                 1 if project else 0, dx, box["alpha"], dt, M,
                                 _ptr(A), _ptr(mi), _ptr(w), _ptr(wf),
                                 _ptr(wt), _ptr(out), _ptr(mfinal), _ptr(en), _ptr(nd))
    res = dict(out=out, M=M, dt=dt, integrator=integ, dx=dx, finite=(rc == 0))
    if want_state:
        res["mfinal"] = mfinal.reshape((3,) + (n,) * d)
    if want_trace:
        res["energy"], res["normdev"] = en, nd
    return res


def eval_field(box, coef, y_ext, init_fn=None, macro=None):
    """H(y) once (ghosts from the box's BC and m_init).  y_ext: [3][E^d]."""
    d, n = box["dim"], box["n"]
    A, dx = face_coefficients(box, coef)
    mi = initial_data(box, init_fn, macro)
    y = np.ascontiguousarray(y_ext, dtype=np.float64).reshape(3, -1)
    H = np.zeros(3 * n ** d)
    _lib().oracle_eval_field(d, n, box["order"], box["bc"], dx, _ptr(A), _ptr(mi), _ptr(y), _ptr(H))
    return H.reshape((3,) + (n,) * d)


def solve_workload_boxes(wl, indices, kernel=None, threads=1):
    """Oracle H_avg for selected boxes of an inputs.Workload (optionally threaded:
    the C loop releases the GIL)."""
    kernel = kernel or wl.kernel

    def one(i):
        b = wl.boxes[i]
        return solve_box(b, wl.coefs[b["coef_index"]], init_fn=wl.init_of(i),
                         macro=wl.macro, kernel=kernel)["out"]

    if threads <= 1:
        return [one(i) for i in indices]
    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(threads) as ex:
        return list(ex.map(one, indices))
