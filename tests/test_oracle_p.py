"""Pins of the oracle's p- and d-type (Cartesian l = 1, 2) integrals (CPU only).

The oracle evaluates integrals with p functions by the Obara-Saika
recursion.  These tests tie that recursion to facts it does not compute
itself:

* a p primitive is a derivative of an s primitive with respect to its centre,
  (x - A_x) exp(-a|r-A|^2) = (1/(2a)) d/dA_x exp(-a|r-A|^2), so every integral
  with a p function in one slot equals a centred finite difference of the
  same integral with an s function there (chained slot by slot from the
  closed-form s integral, every slot, every direction);
* the normalized contracted p function has unit self-overlap (Gauss-Hermite
  quadrature from numpy, not the oracle's overlap formula);
* the Coulomb operator is invariant under rotations: a quarter turn about z
  maps p_x to p_y and p_y to -p_x, so the MO integrals of the rotated system,
  with the coefficient rows of the p_y functions negated, are those of the
  original system (a wrong index or sign in the recursion breaks this);
* the Schwarz inequality holds for the contracted p-type integrals;
* d functions likewise: a d primitive is a centre derivative of a p primitive
  ((x-A_x)(y-A_y) e = (1/2a) d/dA_y [(x-A_x) e], and (x-A_x)^2 e adds the s
  term), unit self-overlap by quadrature, and rotation invariance of LL and DC
  transforms over s, p and d functions.

A dropped term of the recursion (the a_i/(2p) or c_i/(2(p+q)) terms, the
horizontal transfer) changes the value at the first order the finite
difference resolves.
"""
import math

import numpy as np
import pytest

import oracle
from paper_2606_04316_amd import workloads as wl


def _pe(ex, cen, cs):
    args = []
    for i in range(4):
        args += [ex[i], cen[i], cs[i]]
    return oracle.prim_eri_cart(*args)


def test_recursion_all_s_equals_closed_form():
    rng = np.random.default_rng(11)
    for _ in range(20):
        ex = rng.uniform(0.1, 5.0, 4)
        cen = [rng.uniform(-2, 2, 3) for _ in range(4)]
        # one-primitive normalized basis functions: the oracle's closed-form s route
        b = wl.Basis(np.array(cen), np.ones(4, np.int32), ex.copy(), np.ones(4))
        norm = (2 * ex / math.pi) ** 0.75
        ref = oracle.eri_tensor(b)[0, 1, 2, 3] / norm.prod()
        assert _pe(ex, cen, [0, 0, 0, 0]) == pytest.approx(ref, rel=1e-13, abs=0)


@pytest.mark.parametrize("geom", ["generic", "shared_centres", "one_centre"])
def test_p_integrals_are_centre_derivatives(geom):
    rng = np.random.default_rng({"generic": 1, "shared_centres": 2, "one_centre": 3}[geom])
    h = 1e-4
    worst = 0.0
    checked = 0
    for trial in range(300):
        ex = list(rng.uniform(0.2, 3.0, 4))
        if geom == "generic":
            cen = [rng.uniform(-1.5, 1.5, 3) for _ in range(4)]
        elif geom == "shared_centres":
            A, C = rng.uniform(-1.5, 1.5, 3), rng.uniform(-1.5, 1.5, 3)
            cen = [A, A.copy(), C, C.copy()]
        else:
            A = rng.uniform(-1, 1, 3)
            cen = [A.copy() for _ in range(4)]
        cs = [int(x) for x in rng.integers(0, 4, 4)]
        slot = int(rng.integers(0, 4))
        if cs[slot] == 0:
            cs[slot] = int(rng.integers(1, 4))
        comp = cs[slot] - 1
        lower = list(cs)
        lower[slot] = 0

        def shifted(d):
            c2 = [x.copy() for x in cen]
            c2[slot][comp] += d
            return _pe(ex, c2, lower)

        fd = (shifted(h) - shifted(-h)) / (2 * h) / (2 * ex[slot])
        an = _pe(ex, cen, cs)
        scale = max(abs(_pe(ex, cen, [0, 0, 0, 0])), abs(an))
        worst = max(worst, abs(fd - an) / scale)
        checked += 1
    assert checked > 200
    assert worst < 1e-6, worst


def test_p_normalization_by_quadrature():
    # numpy Gauss-Hermite nodes integrate x^2 exp(-s x^2) exactly:
    # int x^2 e^{-s x^2} dx = s^{-3/2} sum_k w_k t_k^2 with t = sqrt(s) x
    t, w = np.polynomial.hermite.hermgauss(20)
    rng = np.random.default_rng(5)
    b = wl.make_sp_basis(rng, np.zeros((1, 3)), 1, 2, (1, 4), 0.1, 10.0)
    nc = oracle.norm_coefs(b)
    off = b.offsets()
    for f in range(b.nfunc):
        e = b.exps[off[f]:off[f + 1]]
        c = nc[off[f]:off[f + 1]]
        tot = 0.0
        for i in range(len(e)):
            for j in range(len(e)):
                s = e[i] + e[j]
                one = (w.sum() / math.sqrt(s))            # int e^{-s y^2} dy
                two = (w * t * t).sum() / s ** 1.5        # int y^2 e^{-s y^2} dy
                tot += c[i] * c[j] * (two * one * one if b.cart[f] else one ** 3)
        assert tot == pytest.approx(1.0, rel=1e-13)


def _rotated(system):
    """Quarter turn about z: r -> (-y, x, z).  The rotated image of p_x on A
    is p_y on RA, of p_y is -p_x, of p_z is p_z."""
    R = np.array([[0.0, -1.0, 0.0], [1.0, 0.0, 0.0], [0.0, 0.0, 1.0]])
    newcart = np.array([0, 2, 1, 3], np.int32)
    sign = np.array([1.0, 1.0, -1.0, 1.0])

    def rot_basis(b, C):
        b2 = wl.Basis(np.ascontiguousarray(b.centers @ R.T), b.nprim.copy(), b.exps.copy(),
                      b.coefs.copy(), newcart[b.cart])
        return b2, np.ascontiguousarray(C * sign[b.cart][None, :, None])

    L2, CL2 = rot_basis(system.L, system.CL)
    if system.S is None:
        return L2, None, CL2, None
    S2, CS2 = rot_basis(system.S, system.CS)
    return L2, S2, CL2, CS2


@pytest.mark.parametrize("ham", ["LL", "DC", "DCG"])
def test_transform_invariant_under_rotation(ham):
    sy = wl.sp_cluster(seed=7, n_atoms=3, edge=4.0, nprim=(1, 2), n=4, ham=ham)
    G = oracle.transform_direct(sy.L, sy.S, sy.CL, sy.CS, ham=ham)[0]
    L2, S2, CL2, CS2 = _rotated(sy)
    G2 = oracle.transform_direct(L2, S2, CL2, CS2, ham=ham)[0]
    scale = np.abs(G).max()
    assert scale > 0
    assert np.abs(G2 - G).max() <= 1e-12 * scale
    # the p functions matter: dropping the sign flip breaks the invariance
    bad = oracle.transform_direct(L2, S2, sy.CL, sy.CS, ham=ham)[0]
    assert np.abs(bad - G).max() > 1e-3 * scale


def test_schwarz_inequality_with_p():
    sy = wl.sp_cluster(seed=8, n_atoms=2, edge=3.0, nprim=(1, 3), n=2, ham="LL")
    I = oracle.eri_tensor(sy.L)
    N = sy.L.nfunc
    diag = np.array([[I[m, n, m, n] for n in range(N)] for m in range(N)])
    assert (diag >= 0).all()
    Q = np.sqrt(diag)
    bound = Q[:, :, None, None] * Q[None, None, :, :]
    assert (np.abs(I) <= bound * (1 + 1e-12) + 1e-15).all()
    # permutational symmetry of real functions
    assert np.allclose(I, I.transpose(1, 0, 2, 3), rtol=0, atol=1e-14 * np.abs(I).max())
    assert np.allclose(I, I.transpose(2, 3, 0, 1), rtol=0, atol=1e-14 * np.abs(I).max())
    np.testing.assert_allclose(oracle.schwarz(sy.L), Q, rtol=1e-13, atol=0)


def test_gauge_hams_over_p_functions_two_routes():
    # the gauge integrals over p functions (pinned in test_oracle_gauge_cart.py)
    # through the unscreened definition route (literal four-spinor operators)
    # and the direct quaternion route agree
    sy = wl.sp_cluster(seed=9, n_atoms=2, edge=3.0, nprim=(1, 1), n=2, ham="DCB")
    Gd, _ = oracle.transform_def(sy.L, sy.S, sy.CL, sy.CS, ham="DCB")
    Go, so = oracle.transform_direct(sy.L, sy.S, sy.CL, sy.CS, ham="DCB")
    assert np.abs(Gd - Go).max() <= 1e-12 * np.abs(Go).max()


# --------------------------------------------------------------------------
# d functions (codes 4..9 = d_xx, d_yy, d_zz, d_xy, d_xz, d_yz)
# --------------------------------------------------------------------------

# d code -> (p code it comes from, derivative direction, adds the s term):
# (x-A_x)(y-A_y) e = (1/2a) d/dA_y [(x-A_x) e];
# (x-A_x)^2 e = (1/2a) (d/dA_x [(x-A_x) e] + e)
D_FROM_P = {4: (1, 0, True), 5: (2, 1, True), 6: (3, 2, True),
            7: (1, 1, False), 8: (1, 2, False), 9: (2, 2, False)}


@pytest.mark.parametrize("geom", ["generic", "shared_centres"])
def test_d_integrals_are_centre_derivatives_of_p(geom):
    rng = np.random.default_rng({"generic": 21, "shared_centres": 22}[geom])
    h = 1e-4
    worst = 0.0
    for trial in range(240):
        ex = list(rng.uniform(0.3, 2.5, 4))
        if geom == "generic":
            cen = [rng.uniform(-1.2, 1.2, 3) for _ in range(4)]
        else:
            A, C = rng.uniform(-1.2, 1.2, 3), rng.uniform(-1.2, 1.2, 3)
            cen = [A, A.copy(), C, C.copy()]
        cs = [int(x) for x in rng.integers(0, 10, 4)]
        slot = int(rng.integers(0, 4))
        if cs[slot] < 4:
            cs[slot] = int(rng.integers(4, 10))
        pcode, comp, add_s = D_FROM_P[cs[slot]]
        lower = list(cs)
        lower[slot] = pcode

        def shifted(d):
            c2 = [x.copy() for x in cen]
            c2[slot][comp] += d
            return _pe(ex, c2, lower)

        fd = (shifted(h) - shifted(-h)) / (2 * h)
        if add_s:
            s_codes = list(cs)
            s_codes[slot] = 0
            fd += _pe(ex, cen, s_codes)
        fd /= 2 * ex[slot]
        an = _pe(ex, cen, cs)
        scale = max(abs(_pe(ex, cen, [0, 0, 0, 0])), abs(an))
        worst = max(worst, abs(fd - an) / scale)
    assert worst < 1e-6, worst


def test_d_normalization_by_quadrature():
    t, w = np.polynomial.hermite.hermgauss(20)
    powers = {4: (2, 0, 0), 5: (0, 2, 0), 6: (0, 0, 2), 7: (1, 1, 0), 8: (1, 0, 1), 9: (0, 1, 1)}
    rng = np.random.default_rng(23)
    k = 3
    exps = np.tile(10.0 ** rng.uniform(-1, 1, k), 6)
    coefs = np.tile(rng.uniform(0.1, 1.0, k), 6)
    b = wl.Basis(np.zeros((6, 3)), np.full(6, k, np.int32), exps, coefs,
                 np.arange(4, 10, dtype=np.int32))
    nc = oracle.norm_coefs(b)
    off = b.offsets()
    for f in range(6):
        e, c = b.exps[off[f]:off[f + 1]], nc[off[f]:off[f + 1]]
        tot = 0.0
        for i in range(k):
            for j in range(k):
                s = e[i] + e[j]
                # int y^(2l) e^{-s y^2} dy = s^{-(2l+1)/2} sum_k w_k t_k^(2l)
                tot += c[i] * c[j] * np.prod([(w * t ** (2 * l)).sum() / s ** (l + 0.5)
                                              for l in powers[4 + f]])
        assert tot == pytest.approx(1.0, rel=1e-13)


# Cartesian powers of the codes (the library's and the oracle's table)
POWERS = {0: (0, 0, 0), 1: (1, 0, 0), 2: (0, 1, 0), 3: (0, 0, 1), 4: (2, 0, 0), 5: (0, 2, 0),
          6: (0, 0, 2), 7: (1, 1, 0), 8: (1, 0, 1), 9: (0, 1, 1), 10: (3, 0, 0),
          11: (0, 3, 0), 12: (0, 0, 3), 13: (2, 1, 0), 14: (2, 0, 1), 15: (1, 2, 0),
          16: (0, 2, 1), 17: (1, 0, 2), 18: (0, 1, 2), 19: (1, 1, 1)}


def _rotated_spd(L, C):
    """Quarter turn about z: the image of x^lx y^ly z^lz on A is
    (-1)^ly x^ly y^lx z^lz on RA."""
    R = np.array([[0.0, -1.0, 0.0], [1.0, 0.0, 0.0], [0.0, 0.0, 1.0]])
    pw = POWERS
    code_of = {v: k for k, v in pw.items()}
    new = np.array([code_of[(pw[c][1], pw[c][0], pw[c][2])] for c in L.cart], np.int32)
    sign = np.array([(-1.0) ** pw[c][1] for c in L.cart])
    L2 = wl.Basis(np.ascontiguousarray(L.centers @ R.T), L.nprim.copy(), L.exps.copy(),
                  L.coefs.copy(), new)
    return L2, np.ascontiguousarray(C * sign[None, :, None])


def _spd_basis(rng, atoms, nprim):
    cen, npr, ex, co, cart = [], [], [], [], []
    for a in atoms:
        for codes in ((0,), (1, 2, 3), (4, 5, 6, 7, 8, 9)):
            e = 10.0 ** rng.uniform(-1, 1, nprim)
            c = rng.uniform(0.1, 1.0, nprim)
            for code in codes:
                cen.append(a); npr.append(nprim); ex.append(e); co.append(c); cart.append(code)
    return wl.Basis(np.array(cen), np.array(npr, np.int32), np.concatenate(ex),
                    np.concatenate(co), np.array(cart, np.int32))


@pytest.mark.parametrize("ham", ["LL", "DC"])
def test_spd_transform_invariant_under_rotation(ham):
    rng = np.random.default_rng(24)
    atoms = rng.uniform(0, 3.0, (2, 3))
    L = _spd_basis(rng, atoms, 1)
    S = _spd_basis(rng, atoms, 1) if ham == "DC" else None
    NL, NS = L.nfunc, (S.nfunc if S is not None else 0)
    Q = wl.quat_qr_plus(rng.standard_normal((4, NL + NS, 3)))
    CL = np.ascontiguousarray(Q[:, :NL])
    CS = np.ascontiguousarray(Q[:, NL:]) if S is not None else None
    G = oracle.transform_direct(L, S, CL, CS, ham=ham)[0]
    L2, CL2 = _rotated_spd(L, CL)
    S2, CS2 = _rotated_spd(S, CS) if S is not None else (None, None)
    G2 = oracle.transform_direct(L2, S2, CL2, CS2, ham=ham)[0]
    scale = np.abs(G).max()
    assert np.abs(G2 - G).max() <= 1e-12 * scale
    bad = oracle.transform_direct(L2, S2, CL, CS, ham=ham)[0]
    assert np.abs(bad - G).max() > 1e-3 * scale


# --------------------------------------------------------------------------
# f functions (codes 10..19 = f_xxx, f_yyy, f_zzz, f_xxy, f_xxz, f_xyy, f_yyz,
# f_xzz, f_yzz, f_xyz)
# --------------------------------------------------------------------------

def _raise_source(code):
    """An f code as a raised d code: (d code, direction k, d power l_k) with
    (r-A)_k^{l+1} M e = (1/2a) (d/dA_k [(r-A)_k^l M e] + l (r-A)_k^{l-1} M e)."""
    lf = POWERS[code]
    for k in range(3):
        if lf[k] > 0:
            ld = list(lf)
            ld[k] -= 1
            dcode = [c for c, p in POWERS.items() if p == tuple(ld)][0]
            if 4 <= dcode <= 9:
                return dcode, k, ld[k]
    raise AssertionError(code)


@pytest.mark.parametrize("geom", ["generic", "shared_centres"])
def test_f_integrals_are_centre_derivatives_of_d(geom):
    rng = np.random.default_rng({"generic": 31, "shared_centres": 32}[geom])
    h = 1e-4
    worst = 0.0
    for trial in range(200):
        ex = list(rng.uniform(0.3, 2.5, 4))
        if geom == "generic":
            cen = [rng.uniform(-1.2, 1.2, 3) for _ in range(4)]
        else:
            A, C = rng.uniform(-1.2, 1.2, 3), rng.uniform(-1.2, 1.2, 3)
            cen = [A, A.copy(), C, C.copy()]
        cs = [int(x) for x in rng.integers(0, 20, 4)]
        slot = int(rng.integers(0, 4))
        if cs[slot] < 10:
            cs[slot] = int(rng.integers(10, 20))
        dcode, k, l = _raise_source(cs[slot])
        lower = list(cs)
        lower[slot] = dcode

        def shifted(d):
            c2 = [x.copy() for x in cen]
            c2[slot][k] += d
            return _pe(ex, c2, lower)

        fd = (shifted(h) - shifted(-h)) / (2 * h)
        if l > 0:  # the power-lowered term l (r-A)_k^{l-1} M e (a p function)
            lp = list(POWERS[dcode])
            lp[k] -= 1
            pcode = [c for c, p in POWERS.items() if p == tuple(lp)][0]
            p_codes = list(cs)
            p_codes[slot] = pcode
            fd += l * _pe(ex, cen, p_codes)
        fd /= 2 * ex[slot]
        an = _pe(ex, cen, cs)
        scale = max(abs(_pe(ex, cen, [0, 0, 0, 0])), abs(an))
        worst = max(worst, abs(fd - an) / scale)
    assert worst < 1e-6, worst


def test_f_normalization_by_quadrature():
    t, w = np.polynomial.hermite.hermgauss(20)
    rng = np.random.default_rng(33)
    k = 3
    exps = np.tile(10.0 ** rng.uniform(-1, 1, k), 10)
    coefs = np.tile(rng.uniform(0.1, 1.0, k), 10)
    b = wl.Basis(np.zeros((10, 3)), np.full(10, k, np.int32), exps, coefs,
                 np.arange(10, 20, dtype=np.int32))
    nc = oracle.norm_coefs(b)
    off = b.offsets()
    for f in range(10):
        e, c = b.exps[off[f]:off[f + 1]], nc[off[f]:off[f + 1]]
        tot = 0.0
        for i in range(k):
            for j in range(k):
                s = e[i] + e[j]
                tot += c[i] * c[j] * np.prod([(w * t ** (2 * l)).sum() / s ** (l + 0.5)
                                              for l in POWERS[10 + f]])
        assert tot == pytest.approx(1.0, rel=1e-13)


def test_f_integrals_invariant_under_rotation():
    # quarter turn about z: the image of x^lx y^ly z^lz on A is
    # (-1)^ly x^ly y^lx z^lz on RA, so every primitive integral over the
    # images equals the product of the four signs times the original
    R = np.array([[0.0, -1.0, 0.0], [1.0, 0.0, 0.0], [0.0, 0.0, 1.0]])
    code_of = {v: k for k, v in POWERS.items()}
    rng = np.random.default_rng(34)
    worst, flips = 0.0, 0
    for trial in range(300):
        ex = list(rng.uniform(0.3, 2.5, 4))
        cen = [rng.uniform(-1.2, 1.2, 3) for _ in range(4)]
        cs = [int(x) for x in rng.integers(0, 20, 4)]
        cs[int(rng.integers(0, 4))] = int(rng.integers(10, 20))
        img = [code_of[(POWERS[c][1], POWERS[c][0], POWERS[c][2])] for c in cs]
        sign = np.prod([(-1.0) ** POWERS[c][1] for c in cs])
        a = _pe(ex, cen, cs)
        b = _pe(ex, [R @ c for c in cen], img)
        scale = max(abs(_pe(ex, cen, [0, 0, 0, 0])), abs(a))
        worst = max(worst, abs(b - sign * a) / scale)
        flips += sign < 0 and abs(a) > 1e-6 * scale
    assert worst < 1e-13, worst
    assert flips > 20  # the signs matter


def test_invalid_cart_codes_are_refused():
    b = wl.Basis(np.zeros((1, 3)), np.ones(1, np.int32), np.ones(1), np.ones(1),
                 np.array([20], np.int32))
    with pytest.raises(ValueError):
        oracle.transform_direct(b, None, np.ones((4, 1, 1)), None, ham="LL")
