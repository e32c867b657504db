"""Pins of the FP64 CPU oracle against facts fixed by mathematics and the
paper, independent of the oracle's own formulas (CPU only).

Each test names what it pins and why a plausible mistake in the oracle
(dropped term, wrong sign or index, transposed operand) would fail it.
"""
import math

import numpy as np
import pytest
from scipy import integrate, special

import oracle
import oracle.brute as brute
from paper_2606_04316_amd import workloads as wl
from tests import qalg

# --------------------------------------------------------------------------
# Boys function
# --------------------------------------------------------------------------


@pytest.mark.parametrize("T", [0.0, 1e-14, 1e-9, 1e-4, 0.3, 1.0, 7.5, 29.0, 40.0, 120.0, 3e4])
def test_boys_against_library_and_quadrature(T):
    # F0(T) = 1F1(1/2; 3/2; -T) (library routine) = int_0^1 exp(-T u^2) du (quadrature)
    f = oracle.boys0(T)
    ref = special.hyp1f1(0.5, 1.5, -T)
    quad = integrate.quad(lambda u: math.exp(-T * u * u), 0.0, 1.0, epsabs=0, epsrel=1e-13)[0]
    assert f == pytest.approx(ref, rel=2e-14, abs=0)
    assert f == pytest.approx(quad, rel=1e-12, abs=0)
    if T == 0.0:
        assert f == 1.0
    if T >= 40:
        assert f == pytest.approx(0.5 * math.sqrt(math.pi / T), rel=1e-15)


@pytest.mark.parametrize("m", [0, 1, 2, 3])
@pytest.mark.parametrize("T", [0.0, 1e-9, 0.3, 2.0, 10.0, 29.9, 30.0, 45.0, 120.0])
def test_boys_fm_against_quadrature_and_library(m, T):
    # F_m(T) = int_0^1 u^{2m} exp(-T u^2) du = 1F1(m + 1/2; m + 3/2; -T) / (2m + 1)
    f = oracle.boys(m, T)
    quad = integrate.quad(lambda u: u ** (2 * m) * math.exp(-T * u * u), 0.0, 1.0, epsabs=0,
                          epsrel=1e-13, limit=200)[0]
    ref = special.hyp1f1(m + 0.5, m + 1.5, -T) / (2 * m + 1)
    assert f == pytest.approx(quad, rel=2e-13, abs=0)
    assert f == pytest.approx(ref, rel=1e-13, abs=0)
    if T == 0.0:
        assert f == 1.0 / (2 * m + 1)
    if m == 0:
        assert f == pytest.approx(oracle.boys0(T), rel=2e-15)


# --------------------------------------------------------------------------
# Basis normalization and AO integrals
# --------------------------------------------------------------------------


def _one_prim_basis(exps, centers):
    exps = np.asarray(exps, float)
    return wl.Basis(np.asarray(centers, float).reshape(-1, 3), np.ones(len(exps), np.int32),
                    exps, np.ones(len(exps)))


def test_contracted_functions_have_unit_norm_by_radial_quadrature():
    s = wl.config("ll24")
    nc = oracle.norm_coefs(s.L)
    off = s.L.offsets()
    for f in range(s.L.nfunc):
        a = s.L.exps[off[f]:off[f + 1]]
        c = nc[off[f]:off[f + 1]]
        chi = lambda r: float(np.sum(c * np.exp(-a * r * r)))
        val = integrate.quad(lambda r: 4 * math.pi * r * r * chi(r) ** 2, 0, np.inf,
                             epsrel=1e-13, limit=200)[0]
        assert val == pytest.approx(1.0, rel=1e-11)


@pytest.mark.parametrize("a,b", [(0.1, 0.1), (0.37, 2.9), (10.0, 0.2), (4.0, 4.0)])
def test_one_center_eri_closed_form(a, b):
    # (aa|bb) for normalized s primitives on one centre = 2 sqrt(2ab / (pi (a+b)))
    B = _one_prim_basis([a, b], [[0.3, -0.2, 1.1]] * 2)
    v = oracle.eri(B, 0, 0, B, 1, 1)
    assert v == pytest.approx(2 * math.sqrt(2 * a * b / (math.pi * (a + b))), rel=1e-14)


@pytest.mark.parametrize("a,b,R", [(0.1, 0.4, 0.5), (1.3, 0.7, 2.5), (5.0, 9.0, 6.0),
                                   (0.2, 0.2, 30.0)])
def test_two_center_eri_closed_form(a, b, R):
    # Coulomb energy of two normalized Gaussian densities (exponents 2a, 2b):
    # erf(sqrt(2ab/(a+b)) R) / R, tending to 1/R
    B = _one_prim_basis([a, b], [[0, 0, 0], [0, 0, R]])
    v = oracle.eri(B, 0, 0, B, 1, 1)
    assert v == pytest.approx(math.erf(math.sqrt(2 * a * b / (a + b)) * R) / R, rel=1e-14)


def test_four_center_eri_as_charge_distribution_energy():
    # Gaussian product theorem: chi_a chi_b = K_ab (2a/pi)^{3/4}(2b/pi)^{3/4} exp(-p|r-P|^2);
    # the Coulomb energy of two such s densities is E_a E_b erf(sqrt(pq/(p+q)) R)/R with
    # E = K (pi/p)^{3/2} n_a n_b -- an expression that never forms the Boys function.
    rng = np.random.default_rng(11)
    for _ in range(20):
        ex = 10 ** rng.uniform(-1, 1, 4)
        cen = rng.uniform(-2, 2, (4, 3))
        B = _one_prim_basis(ex, cen)
        v = oracle.eri(B, 0, 1, B, 2, 3)
        n = (2 * ex / math.pi) ** 0.75

        def dist(i, j):
            p = ex[i] + ex[j]
            P = (ex[i] * cen[i] + ex[j] * cen[j]) / p
            K = math.exp(-ex[i] * ex[j] / p * np.sum((cen[i] - cen[j]) ** 2))
            return p, P, K * n[i] * n[j] * (math.pi / p) ** 1.5

        p, P, Ep = dist(0, 1)
        q, Qc, Eq = dist(2, 3)
        R = float(np.linalg.norm(P - Qc))
        ref = Ep * Eq * math.erf(math.sqrt(p * q / (p + q)) * R) / R
        assert v == pytest.approx(ref, rel=1e-13)


def test_gauge_kernel_integrals_closed_form():
    # The r_K r_L / r^3 kernel of the gauge integrals, Eq. (gaugeInt), equals
    # delta_KL / r - d_K d_L r.  Between two s charge distributions (exponents
    # p, q, centres P, Q) the Gaussian-smeared |r| is, with rho = pq/(p+q),
    #   h(R) = exp(-rho R^2) / sqrt(pi rho) + (R + 1/(2 rho R)) erf(sqrt(rho) R)
    # and the smeared 1/r is erf(sqrt(rho) R) / R, both with the same charge
    # factor as the Coulomb integral.  So (mn|K L|kl) / (mn|kl) =
    # (delta_KL Phi - d_K d_L h) / Phi, the second derivatives taken
    # numerically at 40 digits -- an expression that never forms F1 or F2.
    import mpmath as mp
    mp.mp.dps = 40
    rng = np.random.default_rng(21)
    for it in range(8):
        ex = 10 ** rng.uniform(-1, 1, 4)
        cen = rng.uniform(-2, 2, (4, 3))
        if it == 7:
            cen[2:] += np.array([25.0, 0.0, 0.0])  # far apart: R_K R_L / R^3 times the charges
        B = _one_prim_basis(ex, cen)
        T3 = oracle.eri3(B, 0, B, 1, B, 2, B, 3)
        e = oracle.eri(B, 0, 1, B, 2, 3)
        p, q = ex[0] + ex[1], ex[2] + ex[3]
        R = (ex[0] * cen[0] + ex[1] * cen[1]) / p - (ex[2] * cen[2] + ex[3] * cen[3]) / q
        r = mp.mpf(p * q / (p + q))

        def h(x, y, z):
            RR = mp.sqrt(x * x + y * y + z * z)
            return (mp.exp(-r * RR ** 2) / mp.sqrt(mp.pi * r)
                    + (RR + 1 / (2 * r * RR)) * mp.erf(mp.sqrt(r) * RR))

        Rm = [mp.mpf(float(v)) for v in R]
        RR = mp.sqrt(sum(v * v for v in Rm))
        Phi = mp.erf(mp.sqrt(r) * RR) / RR
        for K in range(3):
            for L in range(3):
                o = [0, 0, 0]
                o[K] += 1
                o[L] += 1
                ref = float(((1 if K == L else 0) * Phi - mp.diff(h, Rm, tuple(o))) / Phi)
                assert T3[K, L] / e == pytest.approx(ref, rel=1e-12, abs=1e-14)
        # trace = the Coulomb integral; symmetric in K, L and under bra <-> ket
        assert np.trace(T3) == pytest.approx(e, rel=1e-14)
        assert np.abs(T3 - T3.T).max() <= 1e-15 * abs(e)
        assert np.abs(oracle.eri3(B, 2, B, 3, B, 0, B, 1) - T3).max() <= 1e-15 * abs(e)
        # positive charge distributions: |r_K r_L / r^3| <= 1/r bounds every element
        assert np.abs(T3).max() <= e * (1 + 1e-14)
        if it == 7:
            assert np.abs(T3 / e - np.outer(R, R) / R.dot(R)).max() < 5e-3


def test_eri_tensor_symmetry_schwarz_and_positive_definite():
    s = wl.config("ll24")
    E = oracle.eri_tensor(s.L)
    N = s.L.nfunc
    for perm in [(1, 0, 2, 3), (0, 1, 3, 2), (2, 3, 0, 1), (3, 2, 1, 0)]:
        assert np.allclose(E, E.transpose(perm), rtol=1e-14, atol=0)
    Q = oracle.schwarz(s.L)
    assert np.allclose(Q ** 2, np.einsum("ijij->ij", E), rtol=1e-14)
    bound = Q[:, :, None, None] * Q[None, None, :, :]
    assert np.all(np.abs(E) <= bound * (1 + 1e-13))
    # (mu nu|ka la) is the Gram matrix of the Coulomb metric over pair densities
    w = np.linalg.eigvalsh(E.reshape(N * N, N * N))
    assert w.min() > -1e-12 * w.max()
    # every ERI over positive-coefficient s functions is positive
    assert E.min() > 0


# --------------------------------------------------------------------------
# Generator
# --------------------------------------------------------------------------


@pytest.mark.parametrize("name", ["ll24"])
def test_generator_orthonormal_and_quaternion_structure(name):
    s = wl.config(name)
    Sm = wl.overlap_matrix(s.L, s.L)
    SC = np.einsum("mn,znp->zmp", Sm, s.CL)
    M = qalg.qmatmul(qalg.qconj(s.CL.transpose(0, 2, 1)), SC)
    I = np.zeros_like(M)
    I[0] = np.eye(s.n_mo)
    assert np.abs(M - I).max() < 1e-12
    # the positive-diagonal real QR keeps each 4x4 block a left-multiplication matrix
    rng = np.random.default_rng(3)
    Q = wl.quat_qr_plus(rng.standard_normal((4, 9, 4)))
    R = wl.quat_to_real(Q)
    assert np.abs(R.T @ R - np.eye(16)).max() < 1e-13
    for mu in range(9):
        for p in range(4):
            blk = R[4 * mu:4 * mu + 4, 4 * p:4 * p + 4]
            assert np.abs(blk - wl.quat_left_matrix(blk[:, 0])).max() < 1e-14


# --------------------------------------------------------------------------
# Full transform: three routes, identity, invariants, symmetries
# --------------------------------------------------------------------------


def _tiny(ham):
    if ham == "LL":
        return wl.small_ll(seed=7, n_atoms=2, nfunc=4, n=2)
    return wl.linear_chain(seed=7, n_atoms=2, nl_per_atom=2, ns_per_atom=2, n=2, tau=0.0)


@pytest.mark.parametrize("ham", ["LL", "DC", "DCG", "GAUNT", "GAUGE", "DCB"])
def test_brute_force_vs_definition_vs_direct(ham):
    s = _tiny(ham)
    Gb, sp = brute.transform(s.L, s.S, s.CL, s.CS, ham)
    Gd, im = oracle.transform_def(s.L, s.S, s.CL, s.CS, ham)
    Gr, st = oracle.transform_direct(s.L, s.S, s.CL, s.CS, ham, 0.0)
    scale = np.abs(Gb).max()
    assert np.abs(Gd - Gb).max() <= 1e-12 * scale
    assert np.abs(Gr - Gb).max() <= 1e-12 * scale
    assert im < 1e-14 * scale
    # the projection is lossless: the 16 reals rebuild every spinor integral
    E = [qalg.qrep(np.eye(4)[x]) for x in range(4)]
    n = s.n_mo
    rebuilt = np.einsum("pqrsxy,xab,ycd->paqbrcsd", Gb, np.array(E), np.array(E))
    assert np.abs(rebuilt.reshape(sp.shape) - sp).max() <= 1e-12 * np.abs(sp).max()


def test_definition_vs_direct_ll24():
    s = wl.config("ll24")
    # well-conditioned coefficients: the two routes agree to rounding of max|G|
    C = wl.quat_qr_plus(np.random.default_rng(5).standard_normal((4, 24, 12)))
    Gd, _ = oracle.transform_def(s.L, None, C, None, "LL")
    Gr, _ = oracle.transform_direct(s.L, None, C, None, "LL", 0.0)
    assert np.abs(Gd - Gr).max() <= 1e-13 * np.abs(Gd).max()
    # Loewdin coefficients of the config: agreement within the rounding scale
    Gd, _ = oracle.transform_def(s.L, None, s.CL, None, "LL")
    Gr, _ = oracle.transform_direct(s.L, None, s.CL, None, "LL", 0.0)
    scale = qalg.schwarz_scale([oracle.schwarz(s.L)], [s.CL])
    assert np.abs(Gd - Gr).max() <= 1e-13 * scale


def test_identity_round_trip():
    # C = 1 (n = N): G^{00}_{mu nu ka la} = (mu nu|ka la), every other component 0
    s = wl.small_ll(seed=4, n_atoms=3, nfunc=6, n=6)
    C = qalg.identity_coefficients(6)
    G, _ = oracle.transform_direct(s.L, None, C, None, "LL", 0.0)
    E = oracle.eri_tensor(s.L)
    assert np.abs(G[..., 0, 0] - E).max() < 1e-14
    G2 = G.copy()
    G2[..., 0, 0] = 0
    assert np.abs(G2).max() < 1e-15


def _random_symplectic(rng, n):
    return wl.quat_qr_plus(rng.standard_normal((4, n, n)))


@pytest.mark.parametrize("ham", ["LL", "DC"])
def test_unitary_invariance_of_occupied_J_and_K(ham):
    s = (wl.small_ll(seed=9, n_atoms=4, nfunc=8, n=4) if ham == "LL" else
         wl.linear_chain(seed=9, n_atoms=2, nl_per_atom=3, ns_per_atom=3, n=4, tau=0.0))
    n, occ = 4, 2
    rng = np.random.default_rng(21)
    U = np.zeros((4, n, n))
    U[:, :occ, :occ] = _random_symplectic(rng, occ)
    U[:, occ:, occ:] = _random_symplectic(rng, n - occ)

    def JK(CL, CS):
        G, _ = oracle.transform_direct(s.L, s.S, CL, CS, ham, 0.0)
        o = slice(0, occ)
        J = 4 * np.einsum("pprr->", G[o, o, o, o, 0, 0])
        Kx = G[..., 0, 0] - G[..., 1, 1] - G[..., 2, 2] - G[..., 3, 3]
        K = 2 * np.einsum("prrp->", Kx[o, o, o, o])
        return J, K, G

    J0, K0, G0 = JK(s.CL, s.CS)
    CL1 = qalg.qmatmul(s.CL, U)
    CS1 = qalg.qmatmul(s.CS, U) if s.CS is not None else None
    J1, K1, G1 = JK(CL1, CS1)
    assert J1 == pytest.approx(J0, rel=1e-12)
    assert K1 == pytest.approx(K0, rel=1e-12)
    # and the rotation does change individual integrals (the test is not vacuous)
    assert np.abs(G1 - G0).max() > 1e-3 * np.abs(G0).max()


@pytest.mark.parametrize("ham,sign", [("DC", 1.0), ("GAUNT", -1.0), ("GAUGE", -1.0)])
def test_mo_symmetries_kramers_and_hermiticity(ham, sign):
    s = wl.linear_chain(seed=5, n_atoms=2, nl_per_atom=2, ns_per_atom=3, n=3, tau=0.0)
    G, sp, _ = oracle.transform_def(s.L, s.S, s.CL, s.CS, ham, return_spinor=True)
    tol = 1e-12 * np.abs(sp).max()
    m = sp.shape[0]
    # hermiticity (ab|cd)* = (ba|dc)
    assert np.abs(sp.conj() - sp.transpose(1, 0, 3, 2)).max() < tol
    # bra-ket symmetry
    assert np.abs(sp - sp.transpose(2, 3, 0, 1)).max() < tol
    # time reversal T psi_2p = psi_2p+1, T psi_2p+1 = -psi_2p:
    # (Ta Tb|cd) = sign (ba|cd)   (Coulomb +, Gaunt -)
    T = np.zeros((m, m))
    for p in range(m // 2):
        T[2 * p + 1, 2 * p] = 1.0
        T[2 * p, 2 * p + 1] = -1.0
    lhs = np.einsum("ai,bj,ijcd->abcd", T, T, sp)  # (T a, T b | c d) with real T
    assert np.abs(lhs - sign * sp.transpose(1, 0, 2, 3)).max() < tol
    if sign > 0:
        for a in range(m):  # (a Ta | cd) = 0 for Coulomb
            ta = int(np.nonzero(T[:, a])[0][0])
            assert np.abs(sp[a, ta]).max() < tol
    # quaternion sign rules on G: p<->q gives sign*s_x, r<->s gives sign*s_y
    gt = 1e-12 * np.abs(G).max()
    sx = qalg.SIGNS[None, None, None, None, :, None]
    sy = qalg.SIGNS[None, None, None, None, None, :]
    assert np.abs(G.transpose(1, 0, 2, 3, 4, 5) - sign * sx * G).max() < gt
    assert np.abs(G.transpose(0, 1, 3, 2, 4, 5) - sign * sy * G).max() < gt
    assert np.abs(G.transpose(2, 3, 0, 1, 5, 4) - G).max() < gt


def test_gaunt_quaternion_formula_against_literal_alpha():
    # Reading: G^{xy}_Gaunt = + sum_K sum [D^{K,pq}_{mn}]_x (m^L n^S|k^L l^S) [D^{K,rs}_{kl}]_y,
    # D^{K,rt}_{mn} = conj(C^L_{m r}) e_K C^S_{n t} + conj(C^S_{n r}) e_K C^L_{m t},
    # e_x = k, e_y = j, e_z = i.  Compared with the brute-force -alpha.alpha sum.
    s = _tiny("GAUNT")
    Gb, _ = brute.transform(s.L, s.S, s.CL, s.CS, "GAUNT")
    E = oracle.eri_tensor(s.L, s.S, s.L, s.S)  # (m^L n^S | k^L l^S)
    NL, NS, n = s.L.nfunc, s.S.nfunc, s.n_mo
    unit = {0: np.array([0, 0, 0, 1.0]), 1: np.array([0, 0, 1.0, 0]), 2: np.array([0, 1.0, 0, 0])}
    G = np.zeros_like(Gb)
    for K in range(3):
        e = unit[K].reshape(4, 1, 1)
        D = np.zeros((4, NL, NS, n, n))
        for m_ in range(NL):
            for n_ in range(NS):
                a = qalg.qmul(qalg.qconj(s.CL[:, m_, :])[:, :, None] * np.ones((1, 1, n)),
                              e * np.ones((1, n, n)))
                t1 = qalg.qmul(a, s.CS[:, n_, :][:, None, :] * np.ones((1, n, 1)))
                b = qalg.qmul(qalg.qconj(s.CS[:, n_, :])[:, :, None] * np.ones((1, 1, n)),
                              e * np.ones((1, n, n)))
                t2 = qalg.qmul(b, s.CL[:, m_, :][:, None, :] * np.ones((1, n, 1)))
                D[:, m_, n_] = t1 + t2
        G += np.einsum("xmnpq,mnkl,ykl rs->pqrsxy".replace(" ", ""), D, E, D)
    assert np.abs(G - Gb).max() <= 1e-12 * np.abs(Gb).max()


# --------------------------------------------------------------------------
# Screening
# --------------------------------------------------------------------------


def test_screening_certificate_and_counts():
    # Every skipped directed contribution obeys |(mn|kl) D_y| <= Q Q Dmax < tau
    # (Eq. SchwarzDen), so |G_scr - G_full| is bounded by tau times the summed
    # bra weights of the skipped contributions.
    s = wl.small_ll(seed=13, n_atoms=6, nfunc=12, n=3, edge=14.0)
    C = wl.quat_qr_plus(np.random.default_rng(2).standard_normal((4, 12, 3)))
    N, n = 12, 3
    Qm = oracle.schwarz(s.L)
    Dm = oracle.dmax_coulomb(C)
    pairs = [(mu, nu) for nu in range(N) for mu in range(nu + 1)]
    Qp = np.array([Qm[a, b] for a, b in pairs])
    Dp = np.array([Dm[a, b] for a, b in pairs])
    bnd = np.outer(Qp, Qp * Dp)  # [bra, ket]
    tau = float(np.quantile(bnd, 0.4))
    skip = ~((Qp[:, None] * Qp[None, :]) * Dp[None, :] >= tau)
    assert 0.2 < skip.mean() < 0.6
    Gf, stf = oracle.transform_direct(s.L, None, C, None, "LL", 0.0)
    Gs, sts = oracle.transform_direct(s.L, None, C, None, "LL", tau)
    assert sts["total"][0] == len(pairs) ** 2
    assert sts["kept"][0] == int((~skip).sum())
    assert stf["kept"][0] == len(pairs) ** 2
    w = np.zeros((len(pairs), n, n, 4))
    for i, (a, b) in enumerate(pairs):
        w[i] = np.abs(qalg.pair_density(C, a, b)).transpose(1, 2, 0)
        if a != b:
            w[i] += np.abs(qalg.pair_density(C, b, a)).transpose(1, 2, 0)
    mult = np.array([1.0 if a == b else 2.0 for a, b in pairs])
    bound = tau * np.einsum("ij,ipqx,j->pqx", skip.astype(float), w, mult)
    diff = np.abs(Gs - Gf)
    slack = 1e-13 * np.abs(Gf).max()
    assert np.all(diff <= bound[:, :, None, None, :, None] + slack)
    assert diff.max() > 100 * slack  # screening did change the result


def _gaunt_pair_densities(s):
    """D^{K,pq}_{mn} = conj(C^L_mp) e_K C^S_nq + conj(C^S_np) e_K C^L_mq, [K][4][NL][NS][n][n]."""
    NL, NS, n = s.L.nfunc, s.S.nfunc, s.n_mo
    unit = {0: np.array([0, 0, 0, 1.0]), 1: np.array([0, 0, 1.0, 0]), 2: np.array([0, 1.0, 0, 0])}
    out = np.zeros((3, 4, NL, NS, n, n))
    for K in range(3):
        e = unit[K].reshape(4, 1, 1)
        for m_ in range(NL):
            for n_ in range(NS):
                a = qalg.qmul(qalg.qconj(s.CL[:, m_, :])[:, :, None] * np.ones((1, 1, n)),
                              e * np.ones((1, n, n)))
                t1 = qalg.qmul(a, s.CS[:, n_, :][:, None, :] * np.ones((1, n, 1)))
                b = qalg.qmul(qalg.qconj(s.CS[:, n_, :])[:, :, None] * np.ones((1, 1, n)),
                              e * np.ones((1, n, n)))
                t2 = qalg.qmul(b, s.CL[:, m_, :][:, None, :] * np.ones((1, n, 1)))
                out[K, :, m_, n_] = t1 + t2
    return out


def test_gauge_screening_certificate_and_counts():
    # The gauge classes take the Gaunt predicate Q_mn Q_kl Dmax_kl >= tau.  For
    # non-negative s pair distributions |B_KL| = |(T_KL - delta_KL / r)| / 2 is
    # at most (mn|kl) / 2 <= Q_mn Q_kl / 2, so a skipped contribution adds at
    # most (3/2) tau sum_K |[D^{K,pq}_mn]_x| to G^{xy}_{pqrs}.
    s = wl.linear_chain(seed=17, n_atoms=3, spacing=2.0, nl_per_atom=2, ns_per_atom=3, n=2,
                        tau=0.0, ham="GAUGE")
    NL, NS, n = s.L.nfunc, s.S.nfunc, s.n_mo
    Qp = oracle.schwarz(s.L, s.S).reshape(-1)
    Dp = oracle.dmax_gaunt(s.CL, s.CS).reshape(-1)
    bnd = np.outer(Qp, Qp * Dp)
    tau = float(np.quantile(bnd, 0.5))
    skip = ~((Qp[:, None] * Qp[None, :]) * Dp[None, :] >= tau)
    assert 0.3 < skip.mean() < 0.7
    Gf, stf = oracle.transform_direct(s.L, s.S, s.CL, s.CS, "GAUGE", 0.0)
    Gs, sts = oracle.transform_direct(s.L, s.S, s.CL, s.CS, "GAUGE", tau)
    assert sts["total_gaunt"] == (NL * NS) ** 2 and stf["kept_gaunt"] == (NL * NS) ** 2
    assert sts["kept_gaunt"] == int((~skip).sum())
    # the gauge route keeps exactly what the Gaunt route keeps
    assert oracle.transform_direct(s.L, s.S, s.CL, s.CS, "GAUNT", tau)[1]["kept_gaunt"] == \
        sts["kept_gaunt"]
    D = _gaunt_pair_densities(s)
    w = np.abs(D).sum(axis=0).reshape(4, NL * NS, n, n).transpose(1, 2, 3, 0)  # [pair][p][q][x]
    bound = 1.5 * tau * np.einsum("ij,ipqx->pqx", skip.astype(float), w)
    diff = np.abs(Gs - Gf)
    slack = 1e-13 * np.abs(Gf).max()
    assert np.all(diff <= bound[:, :, None, None, :, None] + slack)
    assert diff.max() > 100 * slack  # screening did change the result


def test_zero_threshold_keeps_everything_including_zeros():
    s = wl.small_ll(seed=4, n_atoms=3, nfunc=6, n=2)
    C = np.zeros((4, 6, 2))
    C[0, 0, 0] = 1.0
    C[2, 1, 1] = 1.0  # most pair densities vanish exactly
    G0, st0 = oracle.transform_direct(s.L, None, C, None, "LL", 0.0)
    assert st0["kept"][0] == st0["total"][0]
    G1, st1 = oracle.transform_direct(s.L, None, C, None, "LL", 1e-300)
    assert st1["kept"][0] < st1["total"][0]
    assert np.array_equal(G0, G1)


def test_gaunt_density_bound_matches_direct_route_screening():
    # orc_dmax_gaunt (quaternion products) against the direct route, whose Gaunt
    # bound is read off the sigma_K spinor densities: identical kept counts.
    s = wl.linear_chain(seed=17, n_atoms=4, spacing=3.0, nl_per_atom=2, ns_per_atom=2, n=3)
    QLS = oracle.schwarz(s.L, s.S)
    D = oracle.dmax_gaunt(s.CL, s.CS)
    q = QLS.reshape(-1)
    d = D.reshape(-1)
    b = np.outer(q, q * d)
    tau = float(np.quantile(b, 0.5))
    kept = int(((q[:, None] * q[None, :]) * d[None, :] >= tau).sum())
    _, st = oracle.transform_direct(s.L, s.S, s.CL, s.CS, "GAUNT", tau, second_half=False)
    assert st["tie_band"] == 0
    assert st["kept_gaunt"] == kept
    assert 0 < kept < q.size ** 2


@pytest.mark.parametrize("ham", ["DC", "DCG"])
def test_first_half_rows_reproduce_partial_G(ham):
    # The quaternion-component first-half rows (the comparison points of the
    # full-size GPU checks) carried through the quaternion second half written
    # here from the definitions, G^xy_pqrs = sum_mn [conj(C_mp) C_nq]_x V_mn^{rs}_y
    # (Coulomb, both orders of an unordered pair) + sum_K sum_LS [D^{K,pq}_mn]_x
    # V^{K,rs}_mn,y (Gaunt), must equal the direct route's G restricted to the
    # same bra pairs, which is computed in complex two-spinor arithmetic.
    s = wl.linear_chain(seed=71, n_atoms=4, spacing=3.0, nl_per_atom=2, ns_per_atom=3, n=3,
                        tau=1e-9, ham=ham)
    NL, NS, n = s.L.nfunc, s.S.nfunc, s.n_mo
    nLL, nSS = NL * (NL + 1) // 2, NS * (NS + 1) // 2
    P = oracle.num_bra_pairs(s.L, s.S, ham)
    rows = np.sort(np.random.default_rng(3).choice(P, size=min(P, 25), replace=False))
    if ham == "DCG":  # make sure some Gaunt rows are in
        rows = np.unique(np.concatenate([rows, [nLL + nSS, nLL + nSS + 7, P - 1]]))
    Vq = oracle.first_half_rows(s.L, s.S, s.CL, s.CS, ham, s.tau, rows)
    Gref, _ = oracle.transform_direct(s.L, s.S, s.CL, s.CS, ham, s.tau, rows=rows)
    npair = n * (n + 1) // 2
    iu = [(p, q) for p in range(n) for q in range(p, n)]
    G = np.zeros((n, n, n, n, 4, 4))
    units = [np.array([0, 0, 0, 1.0]), np.array([0, 0, 1.0, 0]), np.array([0, 1.0, 0, 0])]
    for r_i, row in enumerate(rows):
        if row < nLL + nSS:  # Coulomb pair (canonical index b(b+1)/2 + a)
            C = s.CL if row < nLL else s.CS
            k = row if row < nLL else row - nLL
            b = int((np.sqrt(8 * k + 1) - 1) // 2)
            a = k - b * (b + 1) // 2
            orders = [(a, b)] if a == b else [(a, b), (b, a)]
            for (m, nn) in orders:
                W = qalg.qmul(qalg.qconj(C[:, m, :])[:, :, None], C[:, nn, :][:, None, :])
                for c, (r, t) in enumerate(iu):
                    G[:, :, r, t] += np.einsum("xpq,y->pqxy", W, Vq[r_i, 4 * c:4 * c + 4])
        else:  # Gaunt pair mu in L, nu in S
            g = row - nLL - nSS
            m, nn = g // NS, g % NS
            for K in range(3):
                e = units[K][:, None, None]
                DK = (qalg.qmul(qalg.qmul(qalg.qconj(s.CL[:, m, :])[:, :, None], e),
                                s.CS[:, nn, :][:, None, :])
                      + qalg.qmul(qalg.qmul(qalg.qconj(s.CS[:, nn, :])[:, :, None], e),
                                  s.CL[:, m, :][:, None, :]))
                for c, (r, t) in enumerate(iu):
                    v = Vq[r_i, K * 4 * npair + 4 * c:K * 4 * npair + 4 * c + 4]
                    G[:, :, r, t] += np.einsum("xpq,y->pqxy", DK, v)
    sel = np.zeros((n, n), bool)
    for (r, t) in iu:
        sel[r, t] = True
    scale = np.abs(Gref).max()
    assert scale > 0
    assert np.abs(G[:, :, sel] - Gref[:, :, sel]).max() <= 1e-12 * scale


# --------------------------------------------------------------------------
# General (Kramers-unrestricted) two-spinor input
# --------------------------------------------------------------------------

def _tiny_general(ham, m=3):
    s = _tiny(ham)
    PL, PS, U = wl.general_spinors(s, m, seed=1)
    return s, PL, (PS if ham != "LL" else None), U


@pytest.mark.parametrize("ham", ["LL", "DC", "DCG", "GAUNT"])
def test_general_spinors_brute_force_vs_definition_vs_direct(ham):
    s, PL, PS, _ = _tiny_general(ham)
    spb = brute.spinor_integrals(s.L, s.S, PL, PS, ham, general=True)
    spd = oracle.transform_spinor_def(s.L, s.S, PL, PS, ham)
    spr, st = oracle.transform_spinor(s.L, s.S, PL, PS, ham, 0.0)
    scale = np.abs(spb).max()
    assert scale > 0
    assert np.abs(spd - spb).max() <= 1e-12 * scale
    assert np.abs(spr - spb).max() <= 1e-12 * scale
    # the spinors are not Kramers pairs: the result is not of quaternion form
    assert np.abs(spb[0::2, 0::2] - spb[1::2, 1::2].conj()).max() > 1e-3 * scale


@pytest.mark.parametrize("ham", ["DC", "DCG"])
def test_general_spinor_route_equals_unitary_mixing_of_kramers_route(ham):
    # (a'b'|c'd') = sum U*_{aa'} U_{bb'} U*_{cc'} U_{dd'} (ab|cd): the general
    # route on mixed spinors against the quaternion route's spinor integrals
    # well-conditioned (QR) coefficients: the four-index mixing of Loewdin
    # coefficients amplifies their rounding to the size of the bound itself
    s = wl.linear_chain(seed=9, n_atoms=3, spacing=2.8, nl_per_atom=2, ns_per_atom=3, n=3,
                        tau=0.0, ham=ham, coefs="qr")
    _, sp, _ = oracle.transform_def(s.L, s.S, s.CL, s.CS, ham, return_spinor=True)
    PL, PS, U = wl.general_spinors(s, 5, seed=2)
    mixed = np.einsum("aA,bB,cC,dD,abcd->ABCD", U.conj(), U, U.conj(), U, sp)
    spr, _ = oracle.transform_spinor(s.L, s.S, PL, PS, ham, 0.0)
    assert np.abs(spr - mixed).max() <= 1e-12 * np.abs(sp).max()


@pytest.mark.parametrize("ham", ["DC", "DCG"])
def test_general_spinor_integral_symmetries(ham):
    s = wl.linear_chain(seed=10, n_atoms=3, spacing=3.0, nl_per_atom=2, ns_per_atom=3, n=3,
                        tau=0.0, ham=ham)
    PL, PS, _ = wl.general_spinors(s, 6, seed=3)
    sp, _ = oracle.transform_spinor(s.L, s.S, PL, PS, ham, 0.0)
    scale = np.abs(sp).max()
    assert np.abs(sp - sp.transpose(2, 3, 0, 1)).max() <= 1e-12 * scale  # bra <-> ket
    assert np.abs(sp - sp.transpose(1, 0, 3, 2).conj()).max() <= 1e-12 * scale  # hermiticity


def _spinor_pair_density(P, a, b):
    # Pauli-scalar density sum_tau conj(c_{a tau}) c_{b tau} for all spinor pairs
    ca = P[0] + 1j * P[1]
    cb = P[2] + 1j * P[3]
    return np.outer(ca[a].conj(), ca[b]) + np.outer(cb[a].conj(), cb[b])


def test_general_spinor_screening_counts_and_certificate():
    s = wl.small_ll(seed=13, n_atoms=6, nfunc=12, n=3, edge=14.0)
    s.CL = wl.quat_qr_plus(np.random.default_rng(2).standard_normal((4, 12, 3)))
    PL, _, _ = wl.general_spinors(s, 5, seed=4)
    N, m = 12, 5
    Qm = oracle.schwarz(s.L)
    pairs = [(mu, nu) for nu in range(N) for mu in range(nu + 1)]
    # Dmax: largest |re| or |im| of the density of both orderings, all spinor pairs
    Dp = np.array([max(np.abs(_spinor_pair_density(PL, a, b).real).max(),
                       np.abs(_spinor_pair_density(PL, a, b).imag).max(),
                       np.abs(_spinor_pair_density(PL, b, a).real).max(),
                       np.abs(_spinor_pair_density(PL, b, a).imag).max()) for a, b in pairs])
    Qp = np.array([Qm[a, b] for a, b in pairs])
    bnd = np.outer(Qp, Qp * Dp)
    tau = float(np.quantile(bnd, 0.4))
    skip = ~((Qp[:, None] * Qp[None, :]) * Dp[None, :] >= tau)
    assert 0.2 < skip.mean() < 0.6
    spf, stf = oracle.transform_spinor(s.L, None, PL, None, "LL", 0.0)
    sps, sts = oracle.transform_spinor(s.L, None, PL, None, "LL", tau)
    assert stf["kept"][0] == len(pairs) ** 2
    assert sts["kept"][0] == int((~skip).sum())
    # |skipped (mn|kl) D~_kl| <= tau, carried into (ab|cd) by the bra weights
    w = np.zeros((len(pairs), m, m))
    for i, (a, b) in enumerate(pairs):
        w[i] = np.abs(_spinor_pair_density(PL, a, b))
        if a != b:
            w[i] += np.abs(_spinor_pair_density(PL, b, a))
    mult = np.array([1.0 if a == b else 2.0 for a, b in pairs])
    # each skipped ket contribution is at most tau in |re| and |im| per
    # ordering: sqrt(2) tau in modulus
    bound = np.sqrt(2) * tau * np.einsum("ij,iab,j->ab", skip.astype(float), w, mult)
    diff = np.abs(sps - spf)
    slack = 1e-13 * np.abs(spf).max()
    assert np.all(diff <= bound[:, :, None, None] + slack)
    assert diff.max() > 100 * slack


# --------------------------------------------------------------------------
# MO-driven variant (per-batch density bound)
# --------------------------------------------------------------------------

def test_mo_driven_reduces_to_ao_driven():
    # tau = 0 keeps everything in every batch; one batch of all MO pairs is
    # the AO-driven bound itself (kept counts equal the C route's)
    s = wl.linear_chain(seed=55, n_atoms=5, spacing=3.0, nl_per_atom=3, ns_per_atom=4, n=4,
                        tau=1e-9, ham="DCG")
    G0, _ = oracle.transform_direct(s.L, s.S, s.CL, s.CS, "DCG", 0.0)
    Gm0, _ = oracle.transform_direct_mo(s.L, s.S, s.CL, s.CS, "DCG", 0.0, 3)
    assert np.array_equal(Gm0, G0)
    tau = 1e-6
    Ga, sta = oracle.transform_direct(s.L, s.S, s.CL, s.CS, "DCG", tau)
    Gall, stall = oracle.transform_direct_mo(s.L, s.S, s.CL, s.CS, "DCG", tau, 10)
    assert np.array_equal(Gall, Ga)
    assert stall["kept"] == sta["kept"] and stall["kept_gaunt"] == sta["kept_gaunt"]


def test_mo_driven_batch_bounds_counts_and_certificate():
    s = wl.small_ll(seed=13, n_atoms=6, nfunc=12, n=3, edge=14.0)
    C = wl.quat_qr_plus(np.random.default_rng(2).standard_normal((4, 12, 3)))
    N, n, batch = 12, 3, 2
    Qm = oracle.schwarz(s.L)
    pairs = [(mu, nu) for nu in range(N) for mu in range(nu + 1)]
    mo = [(r, t) for r in range(n) for t in range(r, n)]
    Qp = np.array([Qm[a, b] for a, b in pairs])
    pd = {(a, b): np.abs(qalg.pair_density(C, a, b)) for a in range(N) for b in range(N)}
    Gf, _ = oracle.transform_direct(s.L, None, C, None, "LL", 0.0)
    tau = 3e-3
    Gm, stm = oracle.transform_direct_mo(s.L, None, C, None, "LL", tau, batch)
    Dall = np.array([max(pd[a, b].max(), pd[b, a].max()) for a, b in pairs])
    kept = 0
    w = np.zeros((len(pairs), n, n, 4))
    for i, (a, b) in enumerate(pairs):
        w[i] = pd[a, b].transpose(1, 2, 0) + (pd[b, a].transpose(1, 2, 0) if a != b else 0)
    mult = np.array([1.0 if a == b else 2.0 for a, b in pairs])
    slack = 1e-13 * np.abs(Gf).max()
    for b0 in range(0, len(mo), batch):
        bp = mo[b0:b0 + batch]
        Db = np.array([max(max(pd[a, b][:, r, t].max(), pd[b, a][:, r, t].max()) for r, t in bp)
                       for a, b in pairs])
        assert np.all(Db <= Dall)  # a batch bound never exceeds the all-pairs bound
        keep = (Qp[:, None] * Qp[None, :]) * Db[None, :] >= tau
        kept += int(keep.sum())
        bound = tau * np.einsum("ij,ipqx,j->pqx", (~keep).astype(float), w, mult)
        for r, t in bp:
            for a_, b_ in ((r, t), (t, r)):
                d = np.abs(Gm[:, :, a_, b_] - Gf[:, :, a_, b_])
                assert np.all(d <= bound[:, :, :, None] + slack)
    assert stm["kept"][0] == kept
    assert 0 < kept < len(pairs) ** 2 * (len(mo) + batch - 1) // batch
    assert np.abs(Gm - Gf).max() > 100 * slack  # screening changed the result


@pytest.mark.parametrize("ham", ["DC", "DCG", "DCB"])
def test_first_half_rows_for_a_column_subset(ham):
    # the column-subset form (used at full size, where all MO-pair columns
    # would not fit) equals the corresponding columns of the full rows, with
    # the density bound computed inside or given from the quaternion-route
    # bounds (the same predicate)
    s = wl.linear_chain(seed=70, n_atoms=5, spacing=3.0, nl_per_atom=3, ns_per_atom=4, n=5,
                        tau=1e-9, ham=ham, coefs="qr")
    P = oracle.num_bra_pairs(s.L, s.S, ham)
    rows = np.array([0, 5, P // 2, P - 1, P - 7])
    V = oracle.first_half_rows(s.L, s.S, s.CL, s.CS, ham, s.tau, rows)
    cols = np.array([14, 0, 3, 9])
    dm = oracle.pair_density_bounds(s.L, s.S, s.CL, s.CS, ham)
    nK, npair = (3 if ham != "DC" else 1), 15
    ref = np.concatenate([V[:, K * 4 * npair:(K + 1) * 4 * npair]
                          .reshape(len(rows), npair, 4)[:, cols].reshape(len(rows), -1)
                          for K in range(nK)], axis=1)
    for d in (None, dm):
        Vc = oracle.first_half_rows_cols(s.L, s.S, s.CL, s.CS, ham, s.tau, rows, cols, d)
        assert np.array_equal(Vc, ref)
    assert np.abs(ref).max() > 0
