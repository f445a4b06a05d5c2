"""The allocation-free solve (llhmm_solve_noalloc) against the allocating path
(llhmm_batch_create + llhmm_micro_batch + llhmm_upscale) through the C-ABI.

Both run the same kernels on the same boxes, so the upscaled quantities must
agree bit for bit; the test asserts that, which is tighter than the parity bars
(FP64 1e-12, FP32 1e-5 relative).  Two calls in a row share the library's
scratch array, the second with a smaller batch: its results must not carry
anything over from the first.  A batch larger than the array is refused with
LLHMM_E_BUDGET before anything is enqueued.
"""
import numpy as np
import pytest

from paper_2108_09463_amd import inputs
from paper_2108_09463_amd import llhmm as L

pytestmark = pytest.mark.gpu


def _mixed(nsmall, nslab, seed, precision):
    """2-D boxes of several sizes (resident 32..64, row-strip 96/128), both BCs,
    explicit EX2 initial data at seeded centres."""
    eps = 1.0 / 200.0
    rng = np.random.default_rng(seed)
    boxes = []
    sizes = [32, 48, 64] * nsmall + [96, 128] * nslab
    sizes = sizes[:nsmall + nslab]
    for i, n in enumerate(sizes):
        boxes.append(inputs.make_box(dim=2, n=int(n), quantity=inputs.Q_FIELD, eps=eps,
                                     alpha=float(rng.uniform(0.05, 1.2)), mu=3 * eps,
                                     mu_box=3 * eps, eta=0.3 * eps ** 2, a_max=1.65,
                                     bc=inputs.BC_PERIODIC_PERT if i % 2 == 0 else inputs.BC_DIRICHLET,
                                     center=(float(rng.random()), float(rng.random()))))
    if nsmall + nslab > 1:
        boxes[1]["mu"] = 2 * eps   # Dirichlet box with mu < mu'
    return inputs.Workload("noalloc", 2, boxes, [inputs.coef_quasi(eps)], init=inputs.InitEX2(),
                           precision=precision)


def _noalloc(ctx, prep, stream=None):
    import torch
    H = torch.full((len(prep.boxes), prep.ld), float("nan"), dtype=torch.float64, device=prep.dev)
    st = torch.full((len(prep.boxes),), -7, dtype=torch.int32, device=prep.dev)
    coefs = [L.to_coef(c) for c in prep.wl.coefs]
    L.llhmm_solve_noalloc(ctx, prep.boxes, coefs, prep.precision, H, prep.ld, st, m_init=prep.m_init,
                          K=L.kernel(*prep.wl.kernel), stream=stream)
    return H, st


@pytest.mark.parametrize("precision", [inputs.FP32, inputs.FP64])
def test_noalloc_matches_allocating_path(precision):
    import torch
    from paper_2108_09463_amd.runner import Prepared
    assert torch.cuda.is_available()
    ctx = L.llhmm_create(0)
    big = Prepared(_mixed(24, 4, 31, precision), precision=precision, ctx=ctx)
    small = Prepared(_mixed(5, 1, 32, precision), precision=precision, ctx=ctx)
    ref_big = big.solve()
    ref_small = small.solve()
    print("noalloc", "fp32" if precision else "fp64", len(big.boxes), "then", len(small.boxes),
          "boxes", flush=True)
    # two calls in a row on one stream, the second smaller; both read back after
    s = torch.cuda.current_stream()
    Hb, sb = _noalloc(ctx, big, s.cuda_stream)
    Hs, ss = _noalloc(ctx, small, s.cuda_stream)
    torch.cuda.synchronize()
    for (H, st), ref in (((Hb, sb), ref_big), ((Hs, ss), ref_small)):
        H = H.cpu().numpy()
        assert (st.cpu().numpy() == 0).all()
        assert np.isfinite(H).all()
        assert np.array_equal(H, ref["H"]), np.abs(H - ref["H"]).max()


def test_noalloc_refuses_batch_beyond_scratch():
    import torch
    assert torch.cuda.is_available()
    ctx = L.llhmm_create(0)
    wl = inputs.two_d_batch(n_macro=32, precision=inputs.FP64)   # 1024 boxes of 64^2: ~0.5 GB of tables
    H = torch.zeros((len(wl.boxes), 3), dtype=torch.float64, device="cuda")
    M = torch.from_numpy(np.ascontiguousarray(wl.macro["M"]).reshape(3, -1)).cuda()
    with pytest.raises(L.LlhmmError) as e:
        L.llhmm_solve_noalloc(ctx, wl.boxes, [L.to_coef(c) for c in wl.coefs], inputs.FP64, H, 3,
                              macro=L.macro_dict(wl.macro), M_macro=M)
    assert e.value.code == L.E_BUDGET
    assert L.llhmm_noalloc_bytes() == 64 << 20
    # the refused call enqueued nothing: H is untouched
    torch.cuda.synchronize()
    assert float(H.abs().max()) == 0.0
