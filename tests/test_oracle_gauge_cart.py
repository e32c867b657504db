"""Pins of the oracle's gauge-kernel integrals over Cartesian functions.

[ab| r_K r_L / r^3 |cd] over p, d and f functions is evaluated in
McMurchie-Davidson form (Hermite expansion of each pair, derivatives of the
two-s-distribution kernel with the Leibniz rule for its X_K X_L factor).
Pinned by facts that form does not compute itself: the s quartet equals the
closed form of the s-type route; the trace over K = L equals the Coulomb
integral, which comes from the Obara-Saika recursion (sum_K r_K r_K / r^3 =
1 / r); a p primitive is (1/2a) d/dA_x of an s primitive, so integrals with a
p function equal centred finite differences of integrals with an s function
there, off-diagonal components included (likewise d from p); the nine
components transform as a tensor under a quarter turn about z, with the sign
each function picks up; the kernel is symmetric in K, L and in bra <-> ket.
"""
import numpy as np
import pytest

import oracle
from paper_2606_04316_amd import workloads as wl

POWERS = {0: (0, 0, 0), 1: (1, 0, 0), 2: (0, 1, 0), 3: (0, 0, 1), 4: (2, 0, 0), 5: (0, 2, 0),
          6: (0, 0, 2), 7: (1, 1, 0), 8: (1, 0, 1), 9: (0, 1, 1), 10: (3, 0, 0),
          11: (0, 3, 0), 12: (0, 0, 3), 13: (2, 1, 0), 14: (2, 0, 1), 15: (1, 2, 0),
          16: (0, 2, 1), 17: (1, 0, 2), 18: (0, 1, 2), 19: (1, 1, 1)}


def _g(ex, cen, cs):
    return oracle.prim_eri3_cart(ex[0], cen[0], cs[0], ex[1], cen[1], cs[1], ex[2], cen[2],
                                 cs[2], ex[3], cen[3], cs[3])


def _c(ex, cen, cs):
    return oracle.prim_eri_cart(ex[0], cen[0], cs[0], ex[1], cen[1], cs[1], ex[2], cen[2],
                                cs[2], ex[3], cen[3], cs[3])


def test_s_quartet_equals_closed_form():
    rng = np.random.default_rng(51)
    for trial in range(40):
        ex = rng.uniform(0.2, 3.0, 4)
        cen = rng.uniform(-1.5, 1.5, (4, 3))
        # single-primitive s functions; the s route (orc_eri3) normalizes each
        # primitive by (2a/pi)^{3/4}
        bases = [wl.Basis(cen[i:i + 1].copy(), np.ones(1, np.int32), ex[i:i + 1].copy(),
                          np.ones(1)) for i in range(4)]
        closed = oracle.eri3(bases[0], 0, bases[1], 0, bases[2], 0, bases[3], 0)
        nrm = np.prod((2.0 * ex / np.pi) ** 0.75)
        herm = nrm * _g(ex, cen, [0, 0, 0, 0])
        assert np.abs(herm - closed).max() <= 1e-13 * np.abs(closed).max()


def test_trace_is_the_coulomb_integral():
    rng = np.random.default_rng(52)
    worst = 0.0
    for trial in range(300):
        ex = rng.uniform(0.2, 3.0, 4)
        cen = rng.uniform(-1.5, 1.5, (4, 3))
        if trial % 4 == 0:
            cen[1] = cen[0]
        cs = [int(x) for x in rng.integers(0, 20, 4)]
        B = _g(ex, cen, cs)
        C = _c(ex, cen, cs)
        scale = max(abs(_c(ex, cen, [0, 0, 0, 0])), abs(C))
        worst = max(worst, abs(np.trace(B) - C) / scale)
    assert worst < 1e-12, worst


# code -> (lower code, derivative direction, multiple of the power-lowered
# term and its code): (r - A)_k^{l+1} M e = (1/2a) (d/dA_k [(r - A)_k^l M e]
# + l (r - A)_k^{l-1} M e)
def _lower(code):
    lf = POWERS[code]
    k = max(range(3), key=lambda i: lf[i])
    l1 = list(lf)
    l1[k] -= 1
    low = [c for c, p in POWERS.items() if p == tuple(l1)][0]
    if l1[k] == 0:
        return low, k, 0, None
    l2 = list(l1)
    l2[k] -= 1
    return low, k, l1[k], [c for c, p in POWERS.items() if p == tuple(l2)][0]


@pytest.mark.parametrize("top", [4, 10])
def test_components_are_centre_derivatives(top):
    # p from s (top 4: codes 1..3) and d from p (top 10: codes 4..9), every
    # component K, L
    rng = np.random.default_rng(53 + top)
    h = 1e-4
    worst = 0.0
    for trial in range(120):
        ex = list(rng.uniform(0.3, 2.5, 4))
        cen = [rng.uniform(-1.2, 1.2, 3) for _ in range(4)]
        cs = [int(x) for x in rng.integers(0, top, 4)]
        slot = int(rng.integers(0, 4))
        cs[slot] = int(rng.integers(1 if top == 4 else 4, top))
        low, k, l, low2 = _lower(cs[slot])
        lower = list(cs)
        lower[slot] = low

        def shifted(d):
            c2 = [x.copy() for x in cen]
            c2[slot][k] += d
            return _g(ex, c2, lower)

        fd = (shifted(h) - shifted(-h)) / (2 * h)
        if l:
            c3 = list(cs)
            c3[slot] = low2
            fd = fd + l * _g(ex, cen, c3)
        fd = fd / (2 * ex[slot])
        an = _g(ex, cen, cs)
        scale = max(np.abs(_g(ex, cen, [0, 0, 0, 0])).max(), np.abs(an).max())
        worst = max(worst, np.abs(fd - an).max() / scale)
    assert worst < 1e-6, worst


def test_tensor_covariance_under_rotation():
    R = np.array([[0.0, -1.0, 0.0], [1.0, 0.0, 0.0], [0.0, 0.0, 1.0]])
    code_of = {v: k for k, v in POWERS.items()}
    rng = np.random.default_rng(54)
    worst, flips = 0.0, 0
    for trial in range(150):
        ex = rng.uniform(0.3, 2.5, 4)
        cen = rng.uniform(-1.2, 1.2, (4, 3))
        cs = [int(x) for x in rng.integers(0, 20, 4)]
        img = [code_of[(POWERS[c][1], POWERS[c][0], POWERS[c][2])] for c in cs]
        sign = np.prod([(-1.0) ** POWERS[c][1] for c in cs])
        B = _g(ex, cen, cs)
        B2 = _g(ex, [R @ c for c in cen], img)
        want = sign * (R @ B @ R.T)
        scale = max(np.abs(_g(ex, cen, [0, 0, 0, 0])).max(), np.abs(B).max())
        worst = max(worst, np.abs(B2 - want).max() / scale)
        flips += sign < 0
    assert worst < 1e-12, worst
    assert flips > 20


def test_symmetries():
    rng = np.random.default_rng(55)
    for trial in range(60):
        ex = rng.uniform(0.3, 2.5, 4)
        cen = rng.uniform(-1.2, 1.2, (4, 3))
        cs = [int(x) for x in rng.integers(0, 20, 4)]
        B = _g(ex, cen, cs)
        scale = max(np.abs(_g(ex, cen, [0, 0, 0, 0])).max(), np.abs(B).max())
        assert np.abs(B - B.T).max() <= 1e-13 * scale
        sw = _g(ex[[2, 3, 0, 1]], cen[[2, 3, 0, 1]], [cs[2], cs[3], cs[0], cs[1]])
        assert np.abs(sw - B).max() <= 1e-12 * scale
