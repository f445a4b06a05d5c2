"""Sampled coefficients (A2, sampled mode): the caller supplies a^eps on every
face of the extended grid instead of the closed form.  The samples given here
are the oracle's own face values (the ABI layout [dim][E^dim] with E = n + 6,
x1 fastest, is the one the oracle builds), so the GPU sees exactly the
oracle's faces: FP64 must match at rounding level, FP32 within its bar.
Resident and slab (128^2, FP32) boxes, both BCs, 1-D and 2-D."""
import numpy as np
import pytest

from oracle import micro
from paper_2108_09463_amd import inputs
from paper_2108_09463_amd.runner import Prepared
from test_gpu_parity import assert_fp64, assert_parity, fp64_truth, rel_err, run_oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_2108_09463_amd import llhmm as L
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return L.llhmm_create(0)


def sampled_workload(dim, sizes, seed):
    eps = 0.01
    rng = np.random.default_rng(seed)
    coef = inputs.coef_product(eps) if dim == 2 else inputs.coef_ex1(eps)
    init = inputs.InitEX2() if dim == 2 else inputs.InitEX1()
    boxes, blocks, off = [], [], 0
    for i, n in enumerate(sizes):
        b = inputs.make_box(dim=dim, n=n, order=2, bc=i % 2, quantity=inputs.Q_FIELD, integrator=2,
                            n_steps=0, eps=eps, alpha=float(rng.uniform(0.05, 0.5)),
                            mu=(2.5 if i % 2 else 3.0) * eps, mu_box=3 * eps, eta=0.1 * eps ** 2,
                            a_max=1.5, center=tuple(float(v) for v in rng.random(2)))
        A, _ = micro.face_coefficients(b, coef)
        b["coef_offset"] = off
        blocks.append(A.reshape(-1))
        off += A.size
        boxes.append(b)
    wl = inputs.Workload("sampled", dim, boxes, [coef], init=init, precision=inputs.FP64)
    return wl, np.concatenate(blocks)


@pytest.mark.parametrize("dim,sizes", [(1, (64, 256)), (2, (32, 64, 128))])
@pytest.mark.parametrize("prec", [inputs.FP64, inputs.FP32])
def test_sampled_coefficient_parity(ctx, dim, sizes, prec):
    print(f"sampled coefficient d={dim} sizes={sizes} prec={prec}", flush=True)
    wl, samples = sampled_workload(dim, sizes, seed=17 + dim)
    p = Prepared(wl, precision=prec, ctx=ctx, coef_samples=samples)
    if any(n >= 96 for n in sizes):
        p.tune()
    out = p.solve()
    assert (out["status"] == 0).all()
    ora = run_oracle(wl)
    assert_parity(wl, prec, out["H"], ora, label="sampled d=%d" % dim)
    p.batch.close()


def test_sampled_coefficient_3d(ctx):
    """d = 3 boxes with sampled faces (the time loop then reads the stored faces
    instead of forming them): second and fourth order, both BCs, field and
    flux, in one batch."""
    print("sampled coefficient d=3", flush=True)
    eps = 0.01
    coef = inputs.coef_product3(eps)
    rng = np.random.default_rng(5)
    boxes, blocks, off = [], [], 0
    for i, (n, order, q) in enumerate([(12, 2, inputs.Q_FIELD), (16, 2, inputs.Q_FLUX),
                                       (10, 4, inputs.Q_FIELD), (12, 4, inputs.Q_FLUX)]):
        b = inputs.make_box(dim=3, n=n, order=order, bc=i % 2, quantity=q, integrator=2, n_steps=0,
                            eps=eps, alpha=float(rng.uniform(0.05, 0.5)), mu=(2.5 if i % 2 else 3.0) * eps,
                            mu_box=3 * eps, eta=0.1 * eps ** 2, a_max=1.5,
                            center=tuple(float(v) for v in rng.random(3)), macro_index=(0, 0, 0))
        A, _ = micro.face_coefficients(b, coef)
        b["coef_offset"] = off
        blocks.append(A.reshape(-1))
        off += A.size
        boxes.append(b)
    wl = inputs.Workload("sampled3", 3, boxes, [coef], init=inputs.InitSmooth3D(), precision=inputs.FP64)
    p = Prepared(wl, precision=inputs.FP64, ctx=ctx, coef_samples=np.concatenate(blocks))
    out = p.solve()
    assert (out["status"] == 0).all()
    _, Ht, e_ref, _ = fp64_truth(wl)
    assert_fp64(out["H"], Ht, e_ref, "sampled 3-D")
    p.batch.close()
