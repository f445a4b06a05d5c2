"""Status bits 4 and 8 on the GPU: the boxes of health_cases (pinned against
the oracle in test_health_cpu) through the library.  With the planned steps
the status is 0; forced to half the steps (dt above the stability radius) the
run stays finite but its final state is grid-scale noise: bit 4, and
llhmm_upscale with check returns LLHMM_E_UNSTABLE."""
import numpy as np
import pytest

from health_cases import case
from paper_2108_09463_amd import inputs
from paper_2108_09463_amd import llhmm as L

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return L.llhmm_create(0)


def _run(ctx, dim, forced, prec):
    from paper_2108_09463_amd.runner import Prepared
    b, coef, init = case(dim, forced)
    wl = inputs.Workload("health", dim, [b], [coef], init=init, precision=prec)
    p = Prepared(wl, precision=prec, ctx=ctx)
    return p, p.solve()


@pytest.mark.parametrize("prec", [inputs.FP32, inputs.FP64])
@pytest.mark.parametrize("dim", [1, 2])
def test_status_flags_unresolved_final_state(ctx, dim, prec):
    _, ok = _run(ctx, dim, False, prec)
    assert ok["status"][0] == 0
    p, bad = _run(ctx, dim, True, prec)
    print("dim", dim, "prec", prec, "forced status", bad["status"], "H", bad["H"][0, :3], flush=True)
    assert bad["status"][0] & 4
    assert not bad["status"][0] & 8
    if bad["status"][0] == 4:          # finite: only the final-state check sees it
        assert np.isfinite(bad["H"]).all()
    with pytest.raises(L.LlhmmError) as e:
        L.llhmm_upscale(ctx, p.batch, p.H, p.ld, p.status, check=True)
    assert e.value.code == L.E_UNSTABLE
