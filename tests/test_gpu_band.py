"""GPU parity of large 2-D boxes (n = 96, 128), which the library advances in
full-width row strips with halo rows ("band" mode), against the FP64 oracle.

The cases mix box sizes and damping values in one batch, so that strips of
boxes with different step counts share launches and band boxes share a batch
with boxes solved by the resident kernels.  Bars as in test_gpu_parity.
"""
import numpy as np
import pytest

from oracle import micro
from paper_2108_09463_amd import inputs
from paper_2108_09463_amd import llhmm as L

from test_gpu_parity import assert_parity, rel_err, run_gpu, run_oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return L.llhmm_create(0)


def band_batch(sizes, bc, qty, integrator=inputs.INTEG_AUTO, seed=21, eta_scale=0.1, order=2):
    """2-D boxes on the quasi-periodic coefficient with EX2 initial data; the
    first box of each size has alpha = 0.01, the others random alpha."""
    eps = 1.0 / 200.0
    rng = np.random.default_rng(seed)
    boxes = []
    for i, n in enumerate(sizes):
        alpha = 0.01 if i == 0 else float(rng.uniform(0.01, 0.2))
        boxes.append(inputs.make_box(dim=2, n=n, order=order, bc=bc, quantity=qty,
                                     integrator=integrator, eps=eps, alpha=alpha,
                                     mu=(3 if bc == 0 else 2) * eps, mu_box=3 * eps,
                                     eta=eta_scale * eps ** 2, a_max=1.65,
                                     center=(float(rng.random()), float(rng.random()))))
    return inputs.Workload("band", 2, boxes, [inputs.coef_quasi(eps)], init=inputs.InitEX2())


def check(ctx, wl, prec, want_state=False):
    _, out = run_gpu(ctx, wl, prec, want_state)
    ora = run_oracle(wl, want_state=want_state)
    print("band M", [r["M"] for r in ora])
    assert_parity(wl, prec, out["H"], ora, label="band")
    return out, ora


CASES = [(p, bc, q) for p in (inputs.FP32, inputs.FP64) for bc in (0, 1) for q in (0, 1)]


@pytest.mark.parametrize("prec,bc,qty", CASES)
def test_band_parity_rk4(ctx, prec, bc, qty):
    """n = 128 and 96 boxes (RK4P, one step per launch) beside a resident 64x64 box."""
    check(ctx, band_batch([128, 96, 128, 64, 96], bc, qty), prec)


@pytest.mark.parametrize("prec", [inputs.FP32, inputs.FP64])
def test_band_parity_heun_two_steps_per_launch(ctx, prec):
    """HeunP boxes: two time steps per launch within the same halo."""
    check(ctx, band_batch([128, 96, 128], 0, 0, integrator=inputs.HEUNP, seed=22), prec)


def test_band_torque(ctx):
    check(ctx, band_batch([128, 96], 0, 2, seed=23), inputs.FP32)


def test_band_final_state(ctx):
    from paper_2108_09463_amd.runner import box_state
    wl = band_batch([128, 96], 0, 0, seed=24, eta_scale=0.05)
    p, out = run_gpu(ctx, wl, inputs.FP64, want_state=True)
    ora = run_oracle(wl, want_state=True)
    for i, b in enumerate(wl.boxes):
        mg = box_state(out["m_final"], i, b, p.batch.n_max, p.batch.dim_max)
        d = np.abs(mg - ora[i]["mfinal"]).max()
        print("band final state max diff", i, d)
        assert d < 1e-13


@pytest.mark.parametrize("prec,bc", [(inputs.FP64, 0), (inputs.FP64, 1), (inputs.FP32, 0)])
def test_band_eval_field_elementwise(ctx, prec, bc):
    from paper_2108_09463_amd.runner import Prepared, box_state
    wl = band_batch([128, 96], bc, 0, seed=25)
    p = Prepared(wl, precision=prec, ctx=ctx)
    Hf = p.eval_field()
    for i, b in enumerate(wl.boxes):
        mi = micro.initial_data(b, wl.init, wl.macro)
        Ho = micro.eval_field(b, wl.coefs[0], mi, init_fn=wl.init, macro=wl.macro)
        Hg = box_state(Hf, i, b, p.batch.n_max, p.batch.dim_max)
        scale = np.abs(Ho).max()
        tol = 1e-13 if prec == inputs.FP64 else 3e-5
        d = np.abs(Hg - Ho).max() / scale
        print("band eval", i, d)
        assert d <= tol


def test_uneven_batch_sampled(ctx):
    """The 4096-box uneven FP32 batch (sizes 32..128, alpha ~ U[0.01, 0.2]) in
    full; one box of each size checked against the oracle."""
    wl = inputs.uneven_batch()
    ns = np.array([b["n"] for b in wl.boxes])
    idx = [int(np.nonzero(ns == n)[0][0]) for n in inputs.UNEVEN_SIZES]
    ora = run_oracle(wl, idx)
    Ho = np.stack([r["out"] for r in ora])
    _, out = run_gpu(ctx, wl, inputs.FP32)
    err = rel_err(out["H"][idx, :3], Ho)
    print("uneven sampled", dict(zip(inputs.UNEVEN_SIZES, err)))
    assert np.all(err <= 1e-5)
