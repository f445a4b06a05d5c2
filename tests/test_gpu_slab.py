"""GPU parity of large 2-D boxes (n = 96, 128), which the library cuts into
row slabs held by co-resident workgroups, each in a window of its own rows and
halo rows, that exchange their edge rows every few time steps (slab mode),
against the FP64 oracle.

The cases mix box sizes and damping values in one batch, so that slabs of
boxes with different step counts share one persistent launch and slab boxes
share a batch with boxes solved by the resident kernels.  Bars as in
test_gpu_parity.  Also: every slab tile variant and exchange interval, and the
bounded wait's give-up path forced from the host.
"""
import os

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


def slab_batch(sizes, bc, qty, integrator=inputs.INTEG_AUTO, seed=21, eta_scale=0.1, order=2):
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
    print("slab M", [r["M"] for r in ora])
    assert_parity(wl, prec, out["H"], ora, label="slab")
    return out, ora


CASES = [(p, bc, q) for p in (inputs.FP32, inputs.FP64) for bc in (0, 1) for q in (0, 1)]


@pytest.mark.parametrize("prec,bc,qty", CASES)
def test_slab_parity_rk4(ctx, prec, bc, qty):
    """n = 128 and 96 boxes (RK4P) beside a resident 64x64 box."""
    check(ctx, slab_batch([128, 96, 128, 64, 96], bc, qty), prec)


@pytest.mark.parametrize("prec", [inputs.FP32, inputs.FP64])
def test_slab_parity_heun(ctx, prec):
    """HeunP boxes (two stages per step)."""
    check(ctx, slab_batch([128, 96, 128], 0, 0, integrator=inputs.HEUNP, seed=22), prec)


@pytest.mark.parametrize("prec,bc,integ", [(inputs.FP64, 0, inputs.INTEG_AUTO), (inputs.FP64, 1, inputs.HEUNP),
                                            (inputs.FP32, 0, inputs.HEUNP), (inputs.FP32, 1, inputs.INTEG_AUTO)])
def test_slab_parity_order4(ctx, prec, bc, integ):
    """Fourth-order stencil on n = 128 and 96 boxes: three halo rows per stage,
    so 12 per RK4P step (8 slabs of 16 and 12 rows) and 6 per HeunP step."""
    wl = slab_batch([128, 96], bc, 0, integrator=integ, seed=29, eta_scale=0.05, order=4)
    p, out = run_gpu(ctx, wl, prec)
    slabs, spe = L.llhmm_batch_slabs(p.batch)
    print("order 4 slabs", slabs, "intervals", spe, flush=True)
    assert (slabs >= 2).all()
    assert_parity(wl, prec, out["H"], run_oracle(wl), label="slab order 4")


def test_slab_torque(ctx):
    check(ctx, slab_batch([128, 96], 0, 2, seed=23), inputs.FP32)


def test_slab_final_state(ctx):
    from paper_2108_09463_amd.runner import box_state
    wl = slab_batch([128, 96], 0, 0, seed=24, eta_scale=0.05)
    p, out = run_gpu(ctx, wl, inputs.FP64, want_state=True)
    ora = run_oracle(wl, want_state=True)
    for i, b in enumerate(wl.boxes):
        mg = box_state(out["m_final"], i, b, p.batch.n_max, p.batch.dim_max)
        d = np.abs(mg - ora[i]["mfinal"]).max()
        print("slab final state max diff", i, d)
        assert d < 1e-13


@pytest.mark.parametrize("prec,bc", [(inputs.FP64, 0), (inputs.FP64, 1), (inputs.FP32, 0)])
def test_slab_eval_field_elementwise(ctx, prec, bc):
    from paper_2108_09463_amd.runner import Prepared, box_state
    wl = slab_batch([128, 96], bc, 0, seed=25)
    p = Prepared(wl, precision=prec, ctx=ctx)
    Hf = p.eval_field()
    for i, b in enumerate(wl.boxes):
        mi = micro.initial_data(b, wl.init, wl.macro)
        Ho = micro.eval_field(b, wl.coefs[0], mi, init_fn=wl.init, macro=wl.macro)
        Hg = box_state(Hf, i, b, p.batch.n_max, p.batch.dim_max)
        scale = np.abs(Ho).max()
        tol = 1e-13 if prec == inputs.FP64 else 3e-5
        d = np.abs(Hg - Ho).max() / scale
        print("slab eval", i, d)
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


@pytest.mark.parametrize("prec,integ", [(inputs.FP32, inputs.INTEG_AUTO), (inputs.FP64, inputs.HEUNP)])
def test_slab_intervals_agree(ctx, prec, integ, tmp_path):
    """Every exchange interval the window allows (every stage, with no halo
    rows; 1, 2, 4 steps, with halos of up to 16 rows): each meets the parity
    bar; only the slab count, and with it the grouping of the partial sums,
    differs.  An interval the window cannot take falls back to the default."""
    from paper_2108_09463_amd.runner import Prepared
    wl = slab_batch([128, 96, 128], 1, 0, integrator=integ, seed=27)
    ora = run_oracle(wl)
    stages = 4 if integ == inputs.INTEG_AUTO else 2
    seen = set()
    for spe in (0, 1, 2, 4):
        path = str(tmp_path / "v.txt")
        with open(path, "w") as f:
            for n in (96, 128):
                f.write("%d %d 1 0 %d 0 %d\n" % (prec, n, stages, spe))
        c2 = L.llhmm_create(0)
        L.llhmm_tune_load(c2, path)
        p = Prepared(wl, precision=prec, ctx=c2)
        slabs, got = L.llhmm_batch_slabs(p.batch)
        print("interval", spe, "slabs", slabs, "intervals", got, flush=True)
        assert (slabs >= 2).all() and set(got) <= {0, 1, 2, 4, 8}
        seen |= set((int(a), int(b)) for a, b in zip(slabs, got))
        out = p.solve()
        assert (out["status"] == 0).all()
        assert_parity(wl, prec, out["H"], ora, label="slab interval %d" % spe)
    assert len({b for _, b in seen}) >= 2  # at least two intervals ran


def test_slab_wait_gives_up_when_forced(ctx):
    """A spin limit of zero polls (set from the host) makes the first wait that
    is not already satisfied give up: the launch still ends, the slab boxes
    report status 2, llhmm_upscale with check returns LLHMM_E_HIP, the
    resident box is unaffected, and the next solve with the normal limit is
    correct."""
    import torch
    from paper_2108_09463_amd.runner import Prepared
    wl = slab_batch([128, 64, 96], 0, 0, seed=28, eta_scale=0.05)
    p = Prepared(wl, precision=inputs.FP32, ctx=ctx)
    os.environ["LLHMM_SLAB_SPIN_MAX"] = "0"
    try:
        p.launch()
        torch.cuda.synchronize()
    finally:
        del os.environ["LLHMM_SLAB_SPIN_MAX"]
    st = p.status.cpu().numpy()
    print("forced give-up status", st, flush=True)
    assert st[1] == 0
    assert (st[[0, 2]] & 2).any()
    with pytest.raises(L.LlhmmError) as e:
        L.llhmm_upscale(ctx, p.batch, p.H, p.ld, p.status, check=True)
    assert e.value.code == L.E_HIP
    out = p.solve()
    assert (out["status"] == 0).all()
    assert_parity(wl, inputs.FP32, out["H"], run_oracle(wl), label="after give-up")
