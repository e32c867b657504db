"""Pins of the oracle's RKB small components (oracle/rkb.py; CPU only).

The RKB construction (Eq. RKB) is tied to facts it does not compute itself:

* each gradient function is minus the centre derivative of its s function,
  d/dr_K chi(r; A) = -d/dA_K chi(r; A): its integrals equal centred finite
  differences of the s integrals (a wrong factor 2a, sign or norm fails);
* sigma . p sigma . p = p^2: a spinor whose small component comes from a real
  alpha-only RKB coefficient vector c has the small-component density
  |grad psi|^2 / 4c^2 (psi = sum c_mu chi_mu), so (aa|bb) against a
  large-component-only spinor b equals (1/4c^2) sum_K d^2/dh1 dh2 of the s
  integrals with the two bra functions' centres shifted along K;
* sigma . a sigma . b = a . b + i sigma . (a x b): between an alpha-only and a
  beta-only RKB small component (real psi, psi') the transition density is
  (1/4c^2) (X_y + i X_x), X = grad psi x grad psi' (the spin-orbit part; the
  cross-product integrals again from mixed centre finite differences);
* the small-component classes vanish as 1/c^2 (leading LL|SS and SS|LL);
* the integrals keep the symmetries (ab|cd) = (cd|ab) = conj((ba|dc)).
"""
import numpy as np
import pytest

import oracle
import oracle.rkb as rkb
from paper_2606_04316_amd import workloads as wl


def _basis(seed=1, n_atoms=2, nfunc=4, nprim=2):
    rng = np.random.default_rng(seed)
    atoms = rng.uniform(0.0, 2.5, (n_atoms, 3))
    return wl.make_basis(rng, atoms, nfunc, nprim, 0.3, 3.0)


def _shifted(L, K, h):
    c = L.centers.copy()
    c[:, K] += h
    return wl.Basis(c, L.nprim.copy(), L.exps.copy(), L.coefs.copy())


def test_gradient_functions_are_centre_derivatives():
    L = _basis()
    G, norms = rkb.gradient_basis(L)
    N = L.nfunc
    I = oracle.eri_tensor(G, L, L, L) * norms[:, None, None, None]
    h = 1e-4
    worst = 0.0
    for K in range(3):
        fd = np.empty((N, N, N, N))
        for mu in range(N):
            def one(d):
                c = L.centers.copy()
                c[mu, K] += d
                Lm = wl.Basis(c, L.nprim, L.exps, L.coefs)
                return oracle.eri_tensor(Lm, L, L, L)[mu]
            fd[mu] = -(one(h) - one(-h)) / (2 * h)
        worst = max(worst, np.abs(I[K::3] - fd).max() / np.abs(fd).max())
    assert worst < 1e-7, worst


@pytest.mark.parametrize("c", [1.0, 3.0])
def test_small_component_density_is_gradient_squared(c):
    L = _basis(seed=2, nfunc=4)
    N = L.nfunc
    rng = np.random.default_rng(3)
    cs = rng.uniform(-1, 1, N)   # real alpha-only RKB coefficients of spinor a
    dl = rng.uniform(-1, 1, N)   # large component of spinor b
    PL = np.zeros((4, N, 2))
    PS = np.zeros((4, N, 2))
    PS[0, :, 0] = cs
    PL[0, :, 1] = dl
    Grkb = rkb.transform_rkb(L, PL, PS, c=c)
    got = Grkb[0, 0, 1, 1]
    # (1/4c^2) sum_K d^2/dh1 dh2 sum cc dd (mu(h1) nu(h2) | ka la)
    h = 1e-3
    ref = 0.0
    for K in range(3):
        def F(h1, h2):
            T = oracle.eri_tensor(_shifted(L, K, h1), _shifted(L, K, h2), L, L)
            return np.einsum("m,n,mnkl,k,l->", cs, cs, T, dl, dl)
        ref += (F(h, h) - F(h, -h) - F(-h, h) + F(-h, -h)) / (4 * h * h)
    ref /= 4 * c * c
    assert abs(got.imag) <= 1e-14 * abs(got.real)
    assert got.real == pytest.approx(ref, rel=2e-6)


def test_small_component_transition_density_is_spin_orbit_cross_product():
    # four atoms off one plane: with two (or coplanar) centres the cross-product
    # integrals vanish by symmetry
    L = _basis(seed=8, n_atoms=4, nfunc=4)
    N, c = L.nfunc, 2.0
    rng = np.random.default_rng(9)
    ca = rng.uniform(-1, 1, N)   # alpha-only RKB coefficients of spinor 0
    cb = rng.uniform(-1, 1, N)   # beta-only RKB coefficients of spinor 1
    dl = rng.uniform(-1, 1, N)   # large component of spinor 2
    PL = np.zeros((4, N, 3))
    PS = np.zeros((4, N, 3))
    PS[0, :, 0] = ca
    PS[2, :, 1] = cb
    PL[0, :, 2] = dl
    got = rkb.transform_rkb(L, PL, PS, c=c)[0, 1, 2, 2]
    h = 1e-3

    def F(K, J):
        # sum ca cb dd (d_K mu d_J nu | ka la) = d^2/dh1 dh2 (mu(A + h1 e_K) nu(B + h2 e_J) | ..)
        def f(h1, h2):
            T = oracle.eri_tensor(_shifted(L, K, h1), _shifted(L, J, h2), L, L)
            return np.einsum("m,n,mnkl,k,l->", ca, cb, T, dl, dl)
        return (f(h, h) - f(h, -h) - f(-h, h) + f(-h, -h)) / (4 * h * h)

    Xx = F(1, 2) - F(2, 1)
    Xy = F(2, 0) - F(0, 2)
    ref = (Xy + 1j * Xx) / (4 * c * c)
    assert abs(ref) > 1e-4
    assert abs(got - ref) <= 2e-6 * abs(ref)


def test_small_component_classes_vanish_as_inverse_c_squared():
    L = _basis(seed=4, nfunc=4)
    N, m = L.nfunc, 3
    rng = np.random.default_rng(5)
    PL = rng.standard_normal((4, N, m))
    PS = rng.standard_normal((4, N, m))
    G_ll = oracle.transform_spinor(L, None, PL, None, "LL")[0]
    d1 = np.abs(rkb.transform_rkb(L, PL, PS, c=40.0) - G_ll).max()
    d2 = np.abs(rkb.transform_rkb(L, PL, PS, c=80.0) - G_ll).max()
    assert d1 > 0
    assert d1 / d2 == pytest.approx(4.0, rel=2e-3)


def test_rkb_integral_symmetries():
    L = _basis(seed=6, nfunc=4)
    N, m = L.nfunc, 3
    rng = np.random.default_rng(7)
    G = rkb.transform_rkb(L, rng.standard_normal((4, N, m)), rng.standard_normal((4, N, m)),
                          c=2.0)
    s = np.abs(G).max()
    assert np.abs(G - G.transpose(2, 3, 0, 1)).max() <= 1e-13 * s
    assert np.abs(G - G.transpose(1, 0, 3, 2).conj()).max() <= 1e-13 * s


def test_rkb_needs_s_functions():
    L = _basis()
    Lp = wl.Basis(L.centers, L.nprim, L.exps, L.coefs, np.ones(L.nfunc, np.int32))
    with pytest.raises(ValueError):
        rkb.gradient_basis(Lp)
