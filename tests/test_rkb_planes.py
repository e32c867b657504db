"""Host logic of the library's RKB small-component planes (CPU): the
library's qdcb_rkb_small_planes against the oracle's construction
(oracle/rkb.py, pinned in test_oracle_rkb.py), and its argument checks."""
import numpy as np
import pytest

import oracle.rkb as rkb


@pytest.fixture(scope="module")
def q():
    from paper_2606_04316_amd import qdcb
    return qdcb


def test_small_planes_match_oracle(q):
    rng = np.random.default_rng(3)
    for N, m, c in ((1, 1, 1.0), (5, 7, 2.5), (12, 3, rkb.SPEED_OF_LIGHT)):
        PS = rng.standard_normal((4, N, m))
        norms = rng.uniform(0.5, 3.0, 3 * N)
        got = q.rkb_small_planes(PS, norms, c)
        ref = rkb.small_component_planes(PS, norms, c)
        assert got.shape == (4, 3 * N, m)
        assert np.abs(got - ref).max() <= 1e-15 * np.abs(ref).max()


def test_small_planes_reject_bad_arguments(q):
    PS = np.ones((4, 2, 2))
    with pytest.raises(q.QdcbError):
        q.rkb_small_planes(PS, np.ones(6), 0.0)
    with pytest.raises(q.QdcbError):
        q.rkb_small_planes(PS, np.ones(6), float("nan"))
