"""GPU parity for bases with p functions (Cartesian s and p Gaussians).

The GPU evaluates integrals with p functions in McMurchie-Davidson form
(Hermite expansion of each pair, derivatives of the Boys kernel); the oracle
uses the Obara-Saika recursion (pinned in test_oracle_p.py).  Compared here:
Schwarz factors and single integrals (normwise 1e-13), kept contribution
counts (exact) and the MO integrals of LL, DC and DCG transforms
(max|G_gpu - G_oracle| <= 1e-12 max|G_oracle|), on systems whose pair spaces
span several 64-pair tiles with a ragged last tile, under both integral
schedules, with directed and unique tiles and in the primitive-band row order.  Codes beyond f
are refused (DCB plans over Cartesian bases: test_gpu_gauge_cart.py).
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
# 1: directed tiles (no unique-pair mirroring); 8: primitive-band row order
@pytest.mark.parametrize("flags", [0, 1, 8])
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


def test_cart_refuses_codes_beyond_f(q, ctx):
    s = _sys("DC", 0.0, n_atoms=2, n=2)
    with pytest.raises(q.QdcbError):
        q.Basis(ctx, wl.Basis(s.L.centers, s.L.nprim, s.L.exps, s.L.coefs,
                              np.full(s.L.nfunc, 20, np.int32)))


def test_cart_spinor_plan_matches_oracle(q, ctx):
    # general (Kramers-unrestricted) two-spinor plan over s and p functions
    s = _sys("DCG", 1e-10, seed=47, n_atoms=5, n=4)
    m = 6
    PL, PS, _ = wl.general_spinors(s, m, seed=12)
    L, S = q.Basis(ctx, s.L), q.Basis(ctx, s.S)
    plan = q.Plan(ctx, L, S, "DCG", m, 1e-10, flags=q.PLAN_SPINOR)
    G, st = plan.transform(PL, PS)
    Gc = G[..., 0] + 1j * G[..., 1]
    Go, so = oracle.transform_spinor(s.L, s.S, PL, PS, "DCG", 1e-10)
    assert so["tie_band"] == 0
    assert st["kept"] == so["kept"] and st["kept_gaunt"] == so["kept_gaunt"]
    assert np.abs(Gc - Go).max() <= 1e-12 * np.abs(Go).max()


def test_cart_mixed_and_mo_driven(q, ctx):
    s = _sys("DC", 1e-10, seed=48)
    L, S = q.Basis(ctx, s.L), q.Basis(ctx, s.S)
    ref = q.Plan(ctx, L, S, "DC", s.n_mo, 1e-10)
    G0, st0 = ref.transform(s.CL, s.CS)
    # every kept tile in the FP32 tier: FP32 operands, FP32 accumulation
    mp = q.Plan(ctx, L, S, "DC", s.n_mo, 1e-10, prec="mixed", tier_fp32=1e300, tier_bf16=0.0)
    G1, st1 = mp.transform(s.CL, s.CS)
    assert st1["tiles_tier"][1] == st1["tiles_kept"]
    err = np.abs(G1 - G0).max()
    assert 0.0 < err <= 2e-6 * np.abs(G0).max()
    # MO-driven variant: batches of MO pairs, same integrals and results
    mo = q.Plan(ctx, L, S, "DC", s.n_mo, 1e-10)
    mo.set_mo_batch(4)
    G2, st2 = mo.transform(s.CL, s.CS)
    Go, _ = oracle.transform_direct_mo(s.L, s.S, s.CL, s.CS, "DC", 1e-10, 4)
    assert np.abs(G2 - Go).max() <= 1e-12 * np.abs(Go).max()


def test_cart_graph_replays_equal_eager(q, ctx):
    import torch
    s = _sys("DCG", 1e-10, seed=49, n_atoms=5, n=6)
    L, S = q.Basis(ctx, s.L), q.Basis(ctx, s.S)
    plan = q.Plan(ctx, L, S, "DCG", s.n_mo, 1e-10)
    dev = torch.device("cuda:0")
    CL = torch.from_numpy(s.CL).to(dev)
    CS = torch.from_numpy(s.CS).to(dev)
    n = s.n_mo
    G = torch.empty((n, n, n, n, 4, 4), dtype=torch.float64, device=dev)
    stream = torch.cuda.Stream()
    plan.capture(CL, CS, G, stream)
    rng = np.random.default_rng(50)
    for k in range(3):
        cl = s.CL if k == 0 else s.CL + 1e-2 * rng.standard_normal(s.CL.shape)
        cs = s.CS if k == 0 else s.CS + 1e-2 * rng.standard_normal(s.CS.shape)
        CL.copy_(torch.from_numpy(cl))
        CS.copy_(torch.from_numpy(cs))
        torch.cuda.synchronize()
        st = plan.replay(stream)
        assert st["graph_replay"] or st["graph_fallback"]
        Gr = G.clone()
        Ge, ste = plan.transform(torch.from_numpy(cl).to(dev), torch.from_numpy(cs).to(dev))
        torch.cuda.synchronize()
        assert st["kept"] == ste["kept"]
        assert torch.equal(Gr, Ge)
