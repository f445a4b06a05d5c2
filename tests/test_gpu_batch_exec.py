"""Batch execution on the GPU: tile classes spread over streams, the whole
solve captured as one HIP graph and replayed, and the autotuner of the
slab-mode variant and exchange interval.

Graph replays are interleaved with eager work and host synchronizations, and
every replay is compared with the eager result (bit for bit: the kernels and
their reduction order are the same).
"""
import numpy as np
import pytest

from paper_2108_09463_amd import inputs
from paper_2108_09463_amd import llhmm as L

from test_gpu_slab import slab_batch
from test_gpu_parity import rel_err, run_oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return L.llhmm_create(0)


def mixed(seed=31, integrator=inputs.INTEG_AUTO):
    return slab_batch([128, 96, 64, 48, 32, 128, 96], 0, 0, integrator=integrator, seed=seed)


@pytest.mark.parametrize("prec", [inputs.FP32, inputs.FP64])
def test_graph_replays_match_eager(ctx, prec):
    import torch
    from paper_2108_09463_amd.runner import Prepared
    wl = mixed()
    p = Prepared(wl, precision=prec, ctx=ctx)
    p.launch()
    torch.cuda.synchronize()
    He = p.H.cpu().numpy().copy()
    assert (p.status.cpu().numpy() == 0).all()
    for rep in range(3):
        p.H.zero_()                                   # eager work between replays
        junk = torch.randn(4096, device=p.dev).square().sum()
        torch.cuda.synchronize()
        p.launch_graph()
        torch.cuda.synchronize()
        assert float(junk) >= 0.0
        assert np.array_equal(p.H.cpu().numpy(), He), rep
        assert (p.status.cpu().numpy() == 0).all()
    # other output buffer: the graph is captured again
    H2 = torch.zeros_like(p.H)
    L.llhmm_batch_run_graph(ctx, p.batch, H2, p.ld, p.status, p.m_init, p.macro, p.M_macro)
    torch.cuda.synchronize()
    assert np.array_equal(H2.cpu().numpy(), He)
    # the eager path still works after graph use
    p.H.zero_()
    p.launch()
    torch.cuda.synchronize()
    assert np.array_equal(p.H.cpu().numpy(), He)


def test_graph_with_macro_init(ctx):
    """Q_[4] boxes read the macro field through the graph: a new field in the
    same buffer changes the result of the replay."""
    import torch
    from paper_2108_09463_amd.runner import Prepared
    from test_gpu_parity import small_2d
    wl = small_2d(32, 2, 0, 0, init_mode=1)
    p = Prepared(wl, precision=inputs.FP64, ctx=ctx)
    p.launch_graph()
    torch.cuda.synchronize()
    H1 = p.H.cpu().numpy().copy()
    M2 = np.roll(np.asarray(wl.macro["M"]), 1, axis=0)   # components permuted: still unit vectors
    p.M_macro.copy_(torch.from_numpy(np.ascontiguousarray(M2).reshape(3, -1)))
    p.launch_graph()
    torch.cuda.synchronize()
    H2 = p.H.cpu().numpy().copy()
    wl2 = small_2d(32, 2, 0, 0, init_mode=1)
    wl2.macro = dict(wl2.macro, M=M2)
    Ho = np.stack([r["out"] for r in run_oracle(wl2)])
    assert not np.array_equal(H1, H2)
    assert rel_err(H2, Ho).max() < 1e-10


def test_tuner_keeps_results_and_round_trips(ctx, tmp_path):
    import torch
    from paper_2108_09463_amd.runner import Prepared
    wl = mixed(seed=32)
    p = Prepared(wl, precision=inputs.FP32, ctx=ctx)
    before, spe0 = L.llhmm_batch_slabs(p.batch)
    ns = np.array([b["n"] for b in wl.boxes])
    assert ((before > 0) == (ns >= 96)).all() and (spe0[ns < 96] == 0).all()
    assert (before[ns >= 96] >= 2).all()
    out0 = p.solve()
    slabs, spe = p.tune(reps=1)
    assert ((slabs > 0) == (ns >= 96)).all()
    out1 = p.solve()
    assert (out1["status"] == 0).all()
    # another slab count: the same arithmetic per point, only the grouping of
    # the FP64 partial sums and the FP32 contraction of the stencil may change
    assert rel_err(out1["H"], out0["H"]).max() < 1e-5
    path = str(tmp_path / "tune.txt")
    L.llhmm_tune_save(ctx, path)
    ctx2 = L.llhmm_create(0)
    L.llhmm_tune_load(ctx2, path)
    p2 = Prepared(wl, precision=inputs.FP32, ctx=ctx2)
    s2, spe2 = L.llhmm_batch_slabs(p2.batch)
    assert np.array_equal(s2, slabs) and np.array_equal(spe2, spe)
    out2 = p2.solve()
    assert np.array_equal(out2["H"], out1["H"])   # same variants: same result
    torch.cuda.synchronize()


def test_tuned_heun_class(ctx):
    """HeunP slab boxes: after tuning the result still matches the oracle."""
    from paper_2108_09463_amd.runner import Prepared
    wl = slab_batch([128, 96], 0, 0, integrator=inputs.HEUNP, seed=33)
    p = Prepared(wl, precision=inputs.FP32, ctx=ctx)
    assert (L.llhmm_batch_slabs(p.batch)[0] >= 2).all()
    p.tune(reps=1)
    out = p.solve()
    Ho = np.stack([r["out"] for r in run_oracle(wl)])
    assert rel_err(out["H"][:, :3], Ho).max() <= 1e-5
