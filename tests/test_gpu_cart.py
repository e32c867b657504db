"""GPU parity for bases with p functions (Cartesian s and p Gaussians).

The GPU evaluates integrals with p functions in McMurchie-Davidson form
(Hermite expansion of each pair, derivatives of the Boys kernel); the oracle
uses the Obara-Saika recursion (pinned in test_oracle_p.py).  Compared here:
Schwarz factors and single integrals (normwise 1e-13), kept contribution
counts (exact) and the MO integrals of LL, DC and DCG transforms
(max|G_gpu - G_oracle| <= 1e-12 max|G_oracle|), on systems whose pair spaces
span several 64-pair tiles with a ragged last tile, under both integral
schedules and with directed and unique tiles.  DCB plans with p functions
are refused (the gauge integrals take s functions only).
"""
import numpy as np
import pytest

import oracle
from paper_2606_04316_amd import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def q():
    from paper_2606_04316_amd import qdcb
    return qdcb


@pytest.fixture(scope="module")
def ctx(q):
    c = q.Context(0)
    yield c
    c.close()


def _sys(ham, tau, seed=41, n_atoms=7, n=5):
    # per atom one s function and one p shell in L and in S: N_L = N_S = 28,
    # 406 + 406 Coulomb pairs (12.7 tiles), 784 L-S pairs (12.25 tiles)
    return wl.sp_cluster(seed=seed, n_atoms=n_atoms, edge=5.0, nprim=(1, 2), n=n, ham=ham,
                         tau=tau)


def test_cart_schwarz_factors(q, ctx):
    s = _sys("DC", 0.0)
    for B in (s.L, s.S):
        Qg = q.Basis(ctx, B).schwarz()
        Qo = oracle.schwarz(B)
        assert np.abs(Qg - Qo).max() <= 1e-13 * np.abs(Qo).max()


def test_cart_eri_quartets(q, ctx):
    s = _sys("DC", 0.0, seed=42, n_atoms=3)
    A, B = q.Basis(ctx, s.L), q.Basis(ctx, s.S)
    rng = np.random.default_rng(1)
    NL, NS = s.L.nfunc, s.S.nfunc
    idx = np.stack([rng.integers(0, NL, 400), rng.integers(0, NL, 400),
                    rng.integers(0, NS, 400), rng.integers(0, NS, 400)], 1)
    idx[:40, 1] = idx[:40, 0]  # same-function and same-centre pairs
    got = q.eri_quartets(A, B, idx)
    ref = np.array([oracle.eri(s.L, a, b, s.S, c, d) for a, b, c, d in idx])
    scale = np.abs(ref).max()
    assert np.abs(got - ref).max() <= 1e-13 * scale
    # an s-only basis against one with p functions
    s2 = wl.small_ll(seed=3, n_atoms=3, nfunc=6, n=2)
    C = q.Basis(ctx, s2.L)
    idx2 = np.stack([rng.integers(0, NL, 100), rng.integers(0, NL, 100),
                     rng.integers(0, 6, 100), rng.integers(0, 6, 100)], 1)
    got2 = q.eri_quartets(A, C, idx2)
    ref2 = np.array([oracle.eri(s.L, a, b, s2.L, c, d) for a, b, c, d in idx2])
    assert np.abs(got2 - ref2).max() <= 1e-13 * np.abs(ref2).max()


def _check(q, ctx, s, tau, flags=0, tune=None):
    L = q.Basis(ctx, s.L)
    S = q.Basis(ctx, s.S) if s.S is not None else None
    plan = q.Plan(ctx, L, S, s.ham, s.n_mo, tau, flags=flags)
    if tune is not None:
        plan.tune = tune
    G, st = plan.transform(s.CL, s.CS)
    Go, sto = oracle.transform_direct(s.L, s.S, s.CL, s.CS, s.ham, tau)
    assert sto["tie_band"] == 0
    assert st["kept"] == sto["kept"]
    assert st["total"] == sto["total"]
    if s.ham == "DCG":
        assert st["kept_gaunt"] == sto["kept_gaunt"]
    err = np.abs(G - Go).max()
    scale = np.abs(Go).max()
    assert err <= 1e-12 * scale, (err, scale)
    return st, sto


@pytest.mark.parametrize("tau", [0.0, 1e-10])
@pytest.mark.parametrize("ham", ["LL", "DC", "DCG"])
def test_cart_transform(q, ctx, ham, tau):
    st, _ = _check(q, ctx, _sys(ham, tau), tau)
    if tau > 0:
        assert sum(st["kept"]) < sum(st["total"])


@pytest.mark.parametrize("eri_sched", [0, 1])
@pytest.mark.parametrize("flags", [0, 1])  # 1: directed tiles (no unique-pair mirroring)
def test_cart_schedules(q, ctx, eri_sched, flags):
    s = _sys("DC", 1e-10, seed=43)
    _check(q, ctx, s, 1e-10, flags=flags,
           tune={"eri_sched": eri_sched, "fh_order": 0, "sq_tile": 64})


def test_cart_p_in_one_basis_only(q, ctx):
    # s-only large component, s and p small component (pairs of an s-only
    # store carry no Cartesian data)
    s = _sys("DCG", 1e-10, seed=44)
    L = wl.small_ll(seed=45, n_atoms=7, nfunc=21, n=5).L
    rng = np.random.default_rng(46)
    Q = wl.quat_qr_plus(rng.standard_normal((4, L.nfunc + s.S.nfunc, s.n_mo)))
    s2 = wl.System("mixed", "DCG", L, s.S, np.ascontiguousarray(Q[:, :L.nfunc]),
                   np.ascontiguousarray(Q[:, L.nfunc:]), 1e-10, s.atoms)
    _check(q, ctx, s2, 1e-10)


def test_cart_refuses_gauge(q, ctx):
    s = _sys("DC", 0.0, n_atoms=2, n=2)
    L, S = q.Basis(ctx, s.L), q.Basis(ctx, s.S)
    with pytest.raises(q.QdcbError) as e:
        q.Plan(ctx, L, S, "DCB", 2, 0.0)
    assert e.value.status == -4
    with pytest.raises(q.QdcbError):
        q.Basis(ctx, wl.Basis(s.L.centers, s.L.nprim, s.L.exps, s.L.coefs,
                              np.full(s.L.nfunc, 4, np.int32)))
