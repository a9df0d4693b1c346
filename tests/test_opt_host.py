"""Host-only parts of the optimisation layer (no GPU): the library's
continuation schedule against the oracle's for the settings of Secs. 3 and 6
and against its argument checks."""
import os

import pytest

from oracle import opt as O


def _lib():
    from paper_1909_13585_amd import _binding as B
    if not os.path.exists(B.LIB_PATH):
        pytest.skip("libmlb.so is not built (run __graft_entry__.build())")
    return B


def test_continuation_matches_oracle_schedules():
    _lib()
    from paper_1909_13585_amd.optimize import continuation
    for k in range(0, 760):
        assert continuation(k, 1.0, 0.25, 25, 6.0, 6.0) == O.sec3_schedule(k), k
        assert continuation(k, 3.0, 0.25, 25, 6.0, 1.0, 50, 32.0) == O.sec6_schedule(k), k
    # an uneven last increment and a beta cap below a power of two
    for k in range(0, 400, 7):
        assert continuation(k, 1.0, 0.3, 10, 2.0, 2.0, 20, 24.0) == O.continuation(k, 1.0, 0.3, 10, 2.0, 2.0, 20, 24.0)


def test_continuation_rejects_bad_arguments():
    B = _lib()
    from paper_1909_13585_amd.optimize import continuation
    for args in [(-1, 1.0, 0.25, 25, 6.0), (0, 1.0, 0.0, 25, 6.0), (0, 1.0, 0.25, 0, 6.0), (0, 7.0, 0.25, 25, 6.0),
                 (0, 1.0, 0.25, 25, 6.0, 0.0), (0, 1.0, 0.25, 25, 6.0, 4.0, 10, 2.0)]:
        with pytest.raises(B.MlbError):
            continuation(*args)
