"""GPU parity of the 2-D box sizes between the configurations' ones: n = 16
(one wavefront per box), 80 and 112 (row slabs with five and seven points per
lane), second order, both precisions and boundary conditions, field and flux
averages, beside a 64x64 box in the same batch.  Bars as in test_gpu_parity;
the boxes lie inside the FP32 domain (mu' = 3 eps)."""
import numpy as np
import pytest

from paper_2108_09463_amd import inputs
from paper_2108_09463_amd import llhmm as L

from test_gpu_parity import assert_parity, run_gpu, run_oracle
from test_gpu_slab import slab_batch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return L.llhmm_create(0)


@pytest.mark.parametrize("prec,bc,qty", [(p, bc, q) for p in (inputs.FP32, inputs.FP64) for bc in (0, 1)
                                         for q in (0, 1)])
def test_more_sizes_parity(ctx, prec, bc, qty):
    wl = slab_batch([16, 80, 112, 64, 16], bc, qty, seed=41)
    p, out = run_gpu(ctx, wl, prec)
    slabs, _ = L.llhmm_batch_slabs(p.batch)
    ns = np.array([b["n"] for b in wl.boxes])
    print("sizes", ns, "slabs", slabs, flush=True)
    assert ((slabs >= 2) == (ns > 64)).all()
    assert_parity(wl, prec, out["H"], run_oracle(wl), label="sizes")
