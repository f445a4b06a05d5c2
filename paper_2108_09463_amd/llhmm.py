"""Thin Python binding of libllhmm (include/llhmm.h): the same entry points,
argument marshalling only.  Every step of the micro solve runs in the gfx950
kernels of libllhmm.so; there is no Python or CPU fallback.  PyTorch is used
for device memory and streams only.
"""
from __future__ import annotations

import ctypes
import math
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libllhmm.so")
GHOST = 3
TIMING_SLOTS = 64          # LLHMM_TIMING_SLOTS
MAX_TERMS = 8

OK, E_INVALID, E_NOMEM, E_BUDGET, E_UNSTABLE, E_HIP, E_NOTSUP = 0, -1, -2, -3, -4, -5, -6
FP64, FP32 = 0, 1
MACRO_MPEA, MACRO_HEUNP, MACRO_RK4P = 0, 1, 2


class LlhmmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("llhmm error %d: %s" % (code, msg))
        self.code = code


class Kernel(ctypes.Structure):
    _fields_ = [("p_x", ctypes.c_int32), ("q_x", ctypes.c_int32),
                ("p_t", ctypes.c_int32), ("q_t", ctypes.c_int32)]


class Coef(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("n_terms", ctypes.c_int32),
                ("sampled", ctypes.c_int32), ("pad_", ctypes.c_int32),
                ("c0", ctypes.c_double), ("amp", ctypes.c_double * MAX_TERMS),
                ("freq", (ctypes.c_double * 3) * MAX_TERMS),
                ("phase", (ctypes.c_double * 3) * MAX_TERMS)]


class Box(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("n", ctypes.c_int32), ("order", ctypes.c_int32),
                ("integrator", ctypes.c_int32), ("bc", ctypes.c_int32),
                ("quantity", ctypes.c_int32), ("init_mode", ctypes.c_int32),
                ("n_steps", ctypes.c_int32), ("coef_index", ctypes.c_int32),
                ("macro_index", ctypes.c_int32 * 3),
                ("eps", ctypes.c_double), ("alpha", ctypes.c_double), ("mu", ctypes.c_double),
                ("mu_box", ctypes.c_double), ("eta", ctypes.c_double), ("a_max", ctypes.c_double),
                ("center", ctypes.c_double * 3), ("init_offset", ctypes.c_int64),
                ("coef_offset", ctypes.c_int64)]


class Macro(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("n", ctypes.c_int32), ("dX", ctypes.c_double),
                ("x0", ctypes.c_double * 3)]


class ServerCfg(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("max_inflight", ctypes.c_int32),
                ("max_batch_boxes", ctypes.c_int32), ("pad_", ctypes.c_int32),
                ("device_bytes", ctypes.c_int64), ("K", Kernel)]


_lib = None
_SYMBOLS = {
    "llhmm_abi_version": (ctypes.c_int32, []),
    "llhmm_last_error": (ctypes.c_char_p, []),
    "llhmm_create": (ctypes.c_int, [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int32]),
    "llhmm_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "llhmm_plan": (ctypes.c_int, [ctypes.POINTER(Box), ctypes.c_int32, ctypes.c_void_p,
                                  ctypes.c_void_p, ctypes.c_void_p]),
    "llhmm_check_boxes": (ctypes.c_int, [ctypes.POINTER(Box), ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                         ctypes.POINTER(ctypes.c_int32)]),
    "llhmm_kernel_coeffs": (ctypes.c_int, [ctypes.POINTER(Kernel), ctypes.c_void_p, ctypes.c_void_p]),
    "llhmm_batch_create": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Box), ctypes.c_int32,
                                          ctypes.POINTER(Kernel), ctypes.POINTER(Coef),
                                          ctypes.c_int32, ctypes.c_int32,
                                          ctypes.POINTER(ctypes.c_void_p)]),
    "llhmm_batch_destroy": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "llhmm_batch_cell_steps": (ctypes.c_int64, [ctypes.c_void_p]),
    "llhmm_batch_set_timing": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32]),
    "llhmm_batch_timing": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32,
                                          ctypes.POINTER(ctypes.c_float),
                                          ctypes.POINTER(ctypes.c_float)]),
    "llhmm_micro_batch": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                         ctypes.POINTER(Macro), ctypes.c_void_p, ctypes.c_void_p,
                                         ctypes.c_void_p, ctypes.c_void_p]),
    "llhmm_upscale": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                     ctypes.c_int32, ctypes.c_void_p, ctypes.c_int32,
                                     ctypes.c_void_p]),
    "llhmm_eval_field": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                        ctypes.POINTER(Macro), ctypes.c_void_p, ctypes.c_void_p,
                                        ctypes.c_void_p, ctypes.c_void_p]),
    "llhmm_batch_run_graph": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                             ctypes.POINTER(Macro), ctypes.c_void_p, ctypes.c_void_p,
                                             ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                                             ctypes.c_void_p, ctypes.c_void_p]),
    "llhmm_noalloc_bytes": (ctypes.c_int64, []),
    "llhmm_solve_noalloc": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Box), ctypes.c_int32,
                                           ctypes.POINTER(Kernel), ctypes.POINTER(Coef), ctypes.c_int32,
                                           ctypes.c_int32, ctypes.c_void_p, ctypes.POINTER(Macro),
                                           ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                           ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p]),
    "llhmm_batch_tune": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                        ctypes.POINTER(Macro), ctypes.c_void_p, ctypes.c_void_p,
                                        ctypes.c_int32, ctypes.c_void_p]),
    "llhmm_batch_slabs": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "llhmm_tune_save": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_char_p]),
    "llhmm_tune_load": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_char_p]),
    "llhmm_server_create": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ServerCfg), ctypes.POINTER(Coef),
                                           ctypes.c_int32, ctypes.POINTER(ctypes.c_void_p)]),
    "llhmm_server_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "llhmm_server_submit": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Box), ctypes.c_int32,
                                           ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(Macro),
                                           ctypes.c_void_p]),
    "llhmm_server_poll": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p,
                                         ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                         ctypes.POINTER(ctypes.c_int32)]),
    "llhmm_server_stats": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                          ctypes.c_void_p, ctypes.c_void_p]),
    "llhmm_server_set_output": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                                               ctypes.c_int64]),
    "llhmm_macro_step": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32,
                                        ctypes.c_int32, ctypes.c_int32, ctypes.c_double,
                                        ctypes.c_double, ctypes.c_void_p, ctypes.c_void_p,
                                        ctypes.c_void_p, ctypes.c_void_p,
                                        ctypes.POINTER(ctypes.c_int32), ctypes.c_void_p]),
    "llhmm_macro_step_torque": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32,
                                               ctypes.c_int32, ctypes.c_double, ctypes.c_double,
                                               ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                               ctypes.c_void_p, ctypes.POINTER(ctypes.c_int32),
                                               ctypes.c_void_p]),
    "llhmm_flux_divergence": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Macro), ctypes.c_int32,
                                             ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
                                             ctypes.c_void_p]),
}


def lib():
    """Loads libllhmm.so; raises if it has not been built (no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libllhmm.so is missing: run `python -m paper_2108_09463_amd.build` "
                               "(the HIP library is required; there is no CPU path)")
        # PyTorch carries its own HIP runtime (same soname as the system one);
        # loading it first makes libllhmm bind to that single runtime, so the
        # device pointers and streams PyTorch hands over belong to it.
        import torch  # noqa: F401
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SYMBOLS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(code):
    if code != OK:
        raise LlhmmError(code, lib().llhmm_last_error().decode())


# ---------------------------------------------------------------- marshalling
def to_box(d):
    b = Box()
    for k in ("dim", "n", "order", "integrator", "bc", "quantity", "init_mode", "n_steps",
              "coef_index", "eps", "alpha", "mu", "mu_box", "eta", "a_max"):
        setattr(b, k, d[k])
    mi = tuple(d.get("macro_index", (0, 0))) + (0, 0, 0)
    ce = tuple(d.get("center", (0.0, 0.0))) + (0.0, 0.0, 0.0)
    b.macro_index[0], b.macro_index[1], b.macro_index[2] = mi[:3]
    b.center[0], b.center[1], b.center[2] = ce[:3]
    b.init_offset = int(d.get("init_offset", 0))
    b.coef_offset = int(d.get("coef_offset", 0))
    return b


def box_array(dicts):
    arr = (Box * len(dicts))()
    for i, d in enumerate(dicts):
        arr[i] = to_box(d)
    return arr


def to_coef(c, sampled=False):
    """inputs.SinSum -> llhmm_coef."""
    out = Coef()
    out.dim = c.dim
    out.n_terms = len(c.terms)
    out.sampled = 1 if sampled else 0
    out.c0 = c.c0
    if len(c.terms) > MAX_TERMS:
        raise ValueError("too many coefficient terms")
    for t, (amp, axes) in enumerate(c.terms):
        out.amp[t] = amp
        for ax, (f, ph) in enumerate(axes):
            out.freq[t][ax] = f
            out.phase[t][ax] = ph
    return out


def kernel(p_x=3, q_x=7, p_t=3, q_t=7):
    return Kernel(p_x, q_x, p_t, q_t)


# ---------------------------------------------------------------- entry points
def llhmm_abi_version():
    return lib().llhmm_abi_version()


def llhmm_plan(boxes):
    arr = box_array(boxes)
    n = len(boxes)
    M = np.zeros(n, np.int32)
    dt = np.zeros(n, np.float64)
    integ = np.zeros(n, np.int32)
    _check(lib().llhmm_plan(arr, n, M.ctypes.data, dt.ctypes.data, integ.ctypes.data))
    return M, dt, integ


FP32_MAX_WIDTH_EPS = 6.0      # LLHMM_FP32_MAX_WIDTH_EPS
FP32_MIN_ALPHA_WIDE = 0.5      # LLHMM_FP32_MIN_ALPHA_WIDE
FP32_MIN_MU_EPS = 2.0          # LLHMM_FP32_MIN_MU_EPS
FP32_MIN_PPE_O4 = 8.0          # LLHMM_FP32_MIN_PPE_O4


def llhmm_check_boxes(boxes, precision, ncoefs=1 << 30):
    """(status, first failing box index or -1, message); host only."""
    arr = box_array(boxes)
    bad = ctypes.c_int32(-1)
    st = lib().llhmm_check_boxes(arr, len(boxes), ncoefs, precision, ctypes.byref(bad))
    return st, bad.value, ("" if st == OK else lib().llhmm_last_error().decode())


def llhmm_kernel_coeffs(p_x=3, q_x=7, p_t=3, q_t=7):
    c = np.zeros(p_x + 1)
    d = np.zeros(p_t + 1)
    K = kernel(p_x, q_x, p_t, q_t)
    _check(lib().llhmm_kernel_coeffs(ctypes.byref(K), c.ctypes.data, d.ctypes.data))
    return c, d


def _stream(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    return int(stream)


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


class Context:
    def __init__(self, device=0):
        h = ctypes.c_void_p()
        _check(lib().llhmm_create(ctypes.byref(h), device))
        self.h = h
        self.device = device

    def close(self):
        if self.h:
            lib().llhmm_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def llhmm_create(device=0):
    return Context(device)


class Batch:
    def __init__(self, ctx, boxes, coefs, precision, K=None):
        self.ctx = ctx
        self.boxes = boxes
        self.arr = box_array(boxes)
        self.coefs = (Coef * len(coefs))(*coefs)
        self.K = K or kernel()
        h = ctypes.c_void_p()
        _check(lib().llhmm_batch_create(ctx.h, self.arr, len(boxes), ctypes.byref(self.K),
                                        self.coefs, len(coefs), precision, ctypes.byref(h)))
        self.h = h
        self.n = len(boxes)
        self.nq_max = max(3 * b["dim"] if b["quantity"] == 1 else 3 for b in boxes)
        self.dim_max = max(b["dim"] for b in boxes)
        self.n_max = max(b["n"] for b in boxes)

    def cell_steps(self):
        return int(lib().llhmm_batch_cell_steps(self.h))

    def set_timing(self, enable=True):
        _check(lib().llhmm_batch_set_timing(self.h, 1 if enable else 0))

    def timing(self, back=0):
        """(set-up ms, time-stepping ms) of the timed call `back` calls before the
        last one (waits for it)."""
        s, t = ctypes.c_float(), ctypes.c_float()
        _check(lib().llhmm_batch_timing(self.h, back, ctypes.byref(s), ctypes.byref(t)))
        return float(s.value), float(t.value)

    def close(self):
        if self.h:
            lib().llhmm_batch_destroy(self.ctx.h, self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def llhmm_batch_create(ctx, boxes, coefs, precision, K=None):
    return Batch(ctx, boxes, coefs, precision, K)


def _macro_struct(macro):
    if macro is None:
        return None
    m = Macro()
    m.dim = macro["dim"]
    m.n = macro["n"]
    m.dX = macro["dX"]
    x0 = (tuple(macro.get("x0", (0.0, 0.0))) + (0.0, 0.0, 0.0))[:3]
    m.x0[0], m.x0[1], m.x0[2] = x0
    return ctypes.byref(m), m


def llhmm_micro_batch(ctx, batch, m_init=None, macro=None, M_macro=None, coef=None, m_final=None,
                      stream=None):
    ms = _macro_struct(macro)
    _check(lib().llhmm_micro_batch(ctx.h, batch.h, _ptr(m_init), ms[0] if ms else None,
                                   _ptr(M_macro), _ptr(coef), _ptr(m_final), _stream(stream)))


def llhmm_upscale(ctx, batch, H_avg, ld, status=None, check=False, stream=None):
    _check(lib().llhmm_upscale(ctx.h, batch.h, _ptr(H_avg), ld, _ptr(status), 1 if check else 0,
                               _stream(stream)))


def llhmm_batch_run_graph(ctx, batch, H_avg, ld, status=None, m_init=None, macro=None, M_macro=None,
                          coef=None, m_final=None, stream=None):
    ms = _macro_struct(macro)
    _check(lib().llhmm_batch_run_graph(ctx.h, batch.h, _ptr(m_init), ms[0] if ms else None,
                                       _ptr(M_macro), _ptr(coef), _ptr(m_final), _ptr(H_avg), ld,
                                       _ptr(status), _stream(stream)))


def llhmm_noalloc_bytes():
    return int(lib().llhmm_noalloc_bytes())


def llhmm_solve_noalloc(ctx, boxes, coefs, precision, H_avg, ld, status=None, m_init=None, macro=None,
                        M_macro=None, coef=None, K=None, stream=None):
    """Create + solve + upscale in the library's static scratch array (no device
    allocation).  coefs: llhmm_coef structs (see to_coef)."""
    arr = box_array(boxes)
    carr = (Coef * len(coefs))(*coefs)
    Kp = K or kernel()
    ms = _macro_struct(macro)
    _check(lib().llhmm_solve_noalloc(ctx.h, arr, len(boxes), ctypes.byref(Kp), carr, len(coefs), precision,
                                     _ptr(m_init), ms[0] if ms else None, _ptr(M_macro), _ptr(coef),
                                     _ptr(H_avg), ld, _ptr(status), _stream(stream)))


def llhmm_batch_tune(ctx, batch, m_init=None, macro=None, M_macro=None, coef=None, reps=2,
                     stream=None):
    ms = _macro_struct(macro)
    _check(lib().llhmm_batch_tune(ctx.h, batch.h, _ptr(m_init), ms[0] if ms else None,
                                  _ptr(M_macro), _ptr(coef), reps, _stream(stream)))


def llhmm_batch_slabs(batch):
    """(slabs per box, steps between slab exchanges per box); 0 for boxes
    solved whole by one workgroup."""
    out = np.zeros(batch.n, np.int32)
    spe = np.zeros(batch.n, np.int32)
    _check(lib().llhmm_batch_slabs(batch.h, out.ctypes.data, spe.ctypes.data))
    return out, spe


def llhmm_tune_save(ctx, path):
    _check(lib().llhmm_tune_save(ctx.h, path.encode()))


def llhmm_tune_load(ctx, path):
    _check(lib().llhmm_tune_load(ctx.h, path.encode()))


def llhmm_eval_field(ctx, batch, H, m_init=None, macro=None, M_macro=None, coef=None, stream=None):
    ms = _macro_struct(macro)
    _check(lib().llhmm_eval_field(ctx.h, batch.h, _ptr(m_init), ms[0] if ms else None,
                                  _ptr(M_macro), _ptr(coef), _ptr(H), _stream(stream)))


def llhmm_macro_step(ctx, npts, scheme, step_index, stage, dt, alpha, M, H_avg, Y, work,
                     stream=None):
    nxt = ctypes.c_int32()
    _check(lib().llhmm_macro_step(ctx.h, npts, scheme, step_index, stage, dt, alpha, _ptr(M),
                                  _ptr(H_avg), _ptr(Y), _ptr(work), ctypes.byref(nxt),
                                  _stream(stream)))
    return nxt.value


def llhmm_macro_step_torque(ctx, npts, scheme, stage, dt, alpha, M, T_avg, Y, work, stream=None):
    nxt = ctypes.c_int32()
    _check(lib().llhmm_macro_step_torque(ctx.h, npts, scheme, stage, dt, alpha, _ptr(M), _ptr(T_avg),
                                         _ptr(Y), _ptr(work), ctypes.byref(nxt), _stream(stream)))
    return nxt.value


def llhmm_flux_divergence(ctx, macro, order, F, ld, H, stream=None):
    ms = _macro_struct(macro)
    _check(lib().llhmm_flux_divergence(ctx.h, ms[0] if ms else None, order, _ptr(F), ld, _ptr(H),
                                       _stream(stream)))


# ---------------------------------------------------------------- input packing
def extended_positions(n, mu_box):
    """xi_j = -mu' + j dx for j = -GHOST .. n+GHOST-1 (the documented grid contract)."""
    dx = 2.0 * mu_box / n
    return -mu_box + np.arange(-GHOST, n + GHOST, dtype=np.float64) * dx


def pack_explicit_init(boxes, init_of):
    """Samples each box's closed-form initial data on its extended grid and
    returns (packed FP64 host array, offsets); init_of(i) returns the callable."""
    chunks, offs, off = [], [], 0
    for i, b in enumerate(boxes):
        xi = extended_positions(b["n"], b["mu_box"])
        cx, cy, cz = (tuple(b.get("center", (0.0, 0.0))) + (0.0, 0.0, 0.0))[:3]
        f = init_of(i)
        if b["dim"] == 1:
            v = f(cx + xi)
        elif b["dim"] == 2:
            X0, X1 = np.meshgrid(cx + xi, cy + xi, indexing="xy")
            v = f(X0, X1)
        else:
            # storage [i2][i1][i0], axis 0 fastest
            X2, X1, X0 = np.meshgrid(cz + xi, cy + xi, cx + xi, indexing="ij")
            v = f(X0, X1, X2)
        v = np.ascontiguousarray(v, dtype=np.float64).reshape(-1)
        chunks.append(v)
        offs.append(off)
        off += v.size
    return (np.concatenate(chunks) if chunks else np.zeros(0)), offs


def macro_dict(macro, dim=2):
    return dict(dim=dim, n=macro["n"], dX=macro["dX"], x0=macro.get("x0", (0.0, 0.0, 0.0)))


# ---------------------------------------------------------------- serving
class Server:
    """Continuous-batching request loop of the library (llhmm_server_*)."""

    def __init__(self, ctx, coefs, precision, max_inflight=4, max_batch_boxes=1024,
                 device_bytes=8 << 30, K=None):
        self.ctx = ctx
        cfg = ServerCfg()
        cfg.precision = precision
        cfg.max_inflight = max_inflight
        cfg.max_batch_boxes = max_batch_boxes
        cfg.device_bytes = int(device_bytes)
        cfg.K = K or kernel()
        self.coefs = (Coef * len(coefs))(*coefs)
        h = ctypes.c_void_p()
        _check(lib().llhmm_server_create(ctx.h, ctypes.byref(cfg), self.coefs, len(coefs), ctypes.byref(h)))
        self.h = h
        self.max_batch = max_batch_boxes
        self._keep = []   # host structs of pending submits

    def submit(self, boxes, ids, m_init=None, macro=None, M_macro=None):
        arr = box_array(boxes)
        idv = np.ascontiguousarray(ids, dtype=np.int64)
        ms = _macro_struct(macro)
        _check(lib().llhmm_server_submit(self.h, arr, len(boxes), idv.ctypes.data, _ptr(m_init),
                                         ms[0] if ms else None, _ptr(M_macro)))

    def poll(self, wait=False, max_results=4096):
        ids = np.zeros(max_results, np.int64)
        H = np.zeros((max_results, 6), np.float64)
        st = np.zeros(max_results, np.int32)
        lat = np.zeros(max_results, np.float64)
        n = ctypes.c_int32()
        _check(lib().llhmm_server_poll(self.h, 1 if wait else 0, max_results, ids.ctypes.data, H.ctypes.data,
                                       st.ctypes.data, lat.ctypes.data, ctypes.byref(n)))
        k = n.value
        return ids[:k], H[:k], st[:k], lat[:k]

    def set_output(self, H_dev, ld, nrows):
        """Results also into the device array H_dev[id * ld + q] (None: off)."""
        _check(lib().llhmm_server_set_output(self.h, _ptr(H_dev), int(ld) if H_dev is not None else 0,
                                             int(nrows) if H_dev is not None else 0))

    def stats(self):
        v = [ctypes.c_int64() for _ in range(4)]
        _check(lib().llhmm_server_stats(self.h, *[ctypes.byref(x) for x in v]))
        return dict(queued=v[0].value, inflight=v[1].value, bytes_in_use=v[2].value, bytes_total=v[3].value)

    def close(self):
        if self.h:
            lib().llhmm_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
