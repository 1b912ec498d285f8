"""CPU checks of the test helpers themselves."""
from types import SimpleNamespace

import numpy as np

from conftest import ranks_agree


def _info(ranks, sig, deltas):
    return SimpleNamespace(ranks=ranks, sigmas=sig, deltas=deltas)


def test_ranks_agree_allows_only_numerically_zero_directions_to_go():
    sig = [np.array([1.0, 0.5, 3e-16, 1e-33]), np.array([2.0, 1e-3])]
    ref = _info([1, 4, 2, 1], sig, [0.0, 0.0])  # untruncated rounding
    assert ranks_agree([1, 4, 2, 1], ref)
    assert ranks_agree([1, 2, 2, 1], ref)      # the two rounding-level values dropped
    assert not ranks_agree([1, 1, 2, 1], ref)  # a real direction dropped
    assert not ranks_agree([1, 4, 1, 1], ref)  # 1e-3 is not zero
    assert not ranks_agree([1, 5, 2, 1], ref)  # never more than the oracle


def test_ranks_agree_noise_window_is_narrow():
    # 1e-13 relative lies above 64 u sqrt(4) = 1.4e-14: a real direction
    sig = [np.array([1.0, 0.5, 1e-13, 1e-33]), np.array([2.0, 1e-3])]
    ref = _info([1, 4, 2, 1], sig, [0.0, 0.0])
    assert ranks_agree([1, 3, 2, 1], ref)
    assert not ranks_agree([1, 2, 2, 1], ref)


def test_ranks_agree_is_exact_where_the_threshold_clears_the_noise():
    sig = [np.array([1.0, 0.5, 3e-16, 1e-33]), np.array([2.0, 1e-3])]
    ref = _info([1, 2, 2, 1], sig, [1e-10, 1e-10])  # the oracle truncated the noise itself
    assert ranks_agree([1, 2, 2, 1], ref)
    assert not ranks_agree([1, 1, 2, 1], ref)
    ref = _info([1, 3, 2, 1], [np.array([1.0, 0.5, 0.1, 1e-33]), sig[1]], [1e-10, 1e-10])
    assert not ranks_agree([1, 2, 2, 1], ref)
