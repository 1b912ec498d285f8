import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU test")


def ranks_agree(got_ranks, ref_ranks, ref_sigmas, zero_rel=1e-12):
    """Bond ranks of a GPU result against the oracle's: identical, except that
    the GPU may leave out directions whose oracle singular values lie at the
    rounding level of the path (at most zero_rel times the bond's largest).
    An untruncated rounding keeps every nonzero singular value, and on
    exactly rank-deficient inputs the null directions carry only rounding
    noise, which differs between LAPACK and the Jacobi SVD (whose rows that
    collapse below eps^2 of its largest input row are deflated to exact
    zeros and then dropped); ranks are compared where the margin exceeds
    that noise."""
    import numpy as np
    if len(got_ranks) != len(ref_ranks) or got_ranks[0] != ref_ranks[0] or got_ranks[-1] != ref_ranks[-1]:
        return False
    for b in range(1, len(ref_ranks) - 1):
        s = np.asarray(ref_sigmas[b - 1], dtype=float)
        nz = int(np.sum(s <= zero_rel * s[0])) if s.size and s[0] > 0 else 0
        if not (ref_ranks[b] - nz <= got_ranks[b] <= ref_ranks[b]):
            return False
    return True
