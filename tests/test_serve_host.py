"""Host-side checks of the served HMM run (CPU): a macro stage whose requests
did not all succeed is refused before the macro stepper reads its field."""
import numpy as np
import pytest

from paper_2108_09463_amd import llhmm as L
from paper_2108_09463_amd import serve


def test_stage_with_failed_request_is_refused():
    st = np.zeros(64, np.int32)
    st[17] = L.E_BUDGET
    with pytest.raises(serve.ServeFailed, match="id 17"):
        serve.check_stage(dict(status=st))
    st[17] = 1          # non-finite average
    with pytest.raises(serve.ServeFailed):
        serve.check_stage(dict(status=st))


def test_stage_without_failures_passes():
    serve.check_stage(dict(status=np.zeros(64, np.int32)))


def test_allowed_bits_pass_and_others_still_fail():
    st = np.zeros(64, np.int32)
    st[3] = 4                      # unresolved final state: allowed when asked
    serve.check_stage(dict(status=st), allow=4)
    with pytest.raises(serve.ServeFailed):
        serve.check_stage(dict(status=st))
    st[5] = 4 | 1                  # non-finite as well: never allowed by allow=4
    with pytest.raises(serve.ServeFailed, match="id 5"):
        serve.check_stage(dict(status=st), allow=4)
    st[5] = 0
    st[7] = L.E_BUDGET             # a negative code never passes
    with pytest.raises(serve.ServeFailed, match="id 7"):
        serve.check_stage(dict(status=st), allow=4)


def test_unknown_arrival_mode_is_refused():
    run = serve.ServedRun.__new__(serve.ServedRun)   # no GPU: only the argument check runs
    run.seed, run.npts = 5, 16
    with pytest.raises(ValueError):
        run.stage(None, 0, arrival="sometimes")
