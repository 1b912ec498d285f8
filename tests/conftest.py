import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU test")


def ranks_agree(got_ranks, ref_info):
    """Bond ranks of a GPU result against the oracle's (ref_info: ranks,
    sigmas and per-bond truncation thresholds deltas).

    Identical ranks are required wherever the oracle's threshold at a bond
    is at least the combined size of the bond's noise-level singular values;
    the noise level is 64 u sqrt(p) s_1 for a bond with p singular values
    (both SVDs agree to about u sqrt(p) s_1 in every value).  Below that --
    in practice the untruncated tol = 0 roundings -- the oracle keeps values
    that are rounding noise of an exactly rank-deficient input, and the
    Jacobi SVD, which sets rows below 8 u sqrt(p) of its largest input row
    to exact zeros, may drop them: there the GPU rank may fall short of the oracle's
    by at most the number of noise-level values."""
    import numpy as np
    u = 2.0 ** -53
    if len(got_ranks) != len(ref_info.ranks) or got_ranks[0] != ref_info.ranks[0] \
            or got_ranks[-1] != ref_info.ranks[-1]:
        return False
    for b in range(1, len(ref_info.ranks) - 1):
        s = np.asarray(ref_info.sigmas[b - 1], dtype=float)
        want = ref_info.ranks[b]
        if s.size == 0 or s[0] <= 0:
            if got_ranks[b] != want:
                return False
            continue
        noise = 64.0 * u * np.sqrt(s.size) * s[0]
        nz = int(np.sum(s <= noise))
        if ref_info.deltas[b - 1] >= np.sqrt(max(nz, 1)) * noise:
            if got_ranks[b] != want:
                return False
        elif not (want - nz <= got_ranks[b] <= want):
            return False
    return True
