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


def test_quaternion_small_components_are_the_kramers_pairs_spinor_planes(q):
    # the Kramers-restricted form: the two spinors of each quaternion
    # coefficient (columns of Q(C)) have exactly the oracle's RKB small
    # components, i.e. Q(-(n / 2c) e_K C) = (-i / 2c) n sigma_K Q(C)
    from paper_2606_04316_amd import workloads as wl
    rng = np.random.default_rng(4)
    for N, n, c in ((1, 1, 1.0), (4, 3, 2.5), (9, 5, rkb.SPEED_OF_LIGHT)):
        CS = rng.standard_normal((4, N, n))
        norms = rng.uniform(0.5, 3.0, 3 * N)
        Cq = q.rkb_small_quat(CS, norms, c)
        assert Cq.shape == (4, 3 * N, n)
        got = wl.quat_to_spinor_planes(Cq)
        ref = rkb.small_component_planes(wl.quat_to_spinor_planes(CS), norms, c)
        assert np.abs(got - ref).max() <= 1e-15 * np.abs(ref).max()
    with pytest.raises(q.QdcbError):
        q.rkb_small_quat(np.ones((4, 2, 2)), np.ones(6), -1.0)
