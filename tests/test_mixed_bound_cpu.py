"""CPU checks of the mixed-precision error bound used by the GPU tests
(tests/mixed_bound.py): its pieces reproduce the oracle's transform, and a
model of the reduced tiers (integral and density operands of the affected
contributions rounded to FP32 or BF16, products and sums exact) stays within
the bound element by element, for both tier rules."""
import numpy as np
import pytest

import oracle
from paper_2606_04316_amd import workloads as wl
from tests import mixed_bound as mb


def _f32(a):
    return a.astype(np.float32).astype(np.float64)


def _bf16(a):
    # round to nearest even on the upper 16 bits of the FP32 pattern
    x = a.astype(np.float32).view(np.uint32).astype(np.uint64)
    x = (x + 0x7FFF + ((x >> 16) & 1)) & 0xFFFF0000
    return x.astype(np.uint32).view(np.float32).astype(np.float64)


@pytest.mark.parametrize("ham", ["DC", "DCG"])
def test_bound_pieces_and_rounding_model(ham):
    s = wl.linear_chain(seed=60, n_atoms=5, spacing=3.0, nl_per_atom=3, ns_per_atom=4, n=4,
                        tau=1e-10, ham=ham, coefs="qr")
    Go, _ = oracle.transform_direct(s.L, s.S, s.CL, s.CS, ham, s.tau)
    G = mb.model(s, s.CL, s.CS, s.tau)
    gmax = np.abs(Go).max()
    assert np.abs(G - mb.upper_part(Go)).max() <= 1e-13 * gmax
    assert abs(_bf16(np.array([1.0 + 2.0 ** -9]))[0] - 1.0) == 0.0  # ties to even
    assert _bf16(np.array([1.0 + 3 * 2.0 ** -9]))[0] == 1.0 + 2.0 ** -7
    for rule, t32, t16 in (("g", 1e-2, 1e-4), ("screen", 1e-1, 1e-3), ("g", 1e300, 0.0),
                           ("screen", 1e300, 1e300)):
        Gr = mb.model(s, s.CL, s.CS, s.tau, rule, t32, t16, rounding=(_f32, _bf16))
        B = mb.bound(s, s.CL, s.CS, s.tau, rule, t32, t16)
        err = np.abs(Gr - G)
        assert err.max() > 0.0
        assert np.all(err <= B), (rule, t32, t16, float((err / B).max()))
