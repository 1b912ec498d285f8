"""CPU checks of the test helpers themselves."""
import numpy as np

from conftest import ranks_agree


def test_ranks_agree_allows_only_numerically_zero_directions_to_go():
    sig = [np.array([1.0, 0.5, 3e-16, 1e-33]), np.array([2.0, 1e-3])]
    assert ranks_agree([1, 4, 2, 1], [1, 4, 2, 1], sig)
    assert ranks_agree([1, 2, 2, 1], [1, 4, 2, 1], sig)      # the two rounding-level values dropped
    assert not ranks_agree([1, 1, 2, 1], [1, 4, 2, 1], sig)  # a real direction dropped
    assert not ranks_agree([1, 4, 1, 1], [1, 4, 2, 1], sig)  # 1e-3 is not zero
    assert not ranks_agree([1, 5, 2, 1], [1, 4, 2, 1], sig)  # never more than the oracle
