"""GPU parity for bases with Cartesian d functions (codes 4..9) and f
functions (codes 10..19).

A basis with a d or f function takes the general integral kernels: the pair
product in McMurchie-Davidson form with the Hermite coefficients of each
direction from their recursion and the Hermite integrals factorized by
direction (common.h), Boys orders to 12; the oracle uses the Obara-Saika
recursion (its d and f functions are pinned in test_oracle_p.py).  For f the
oracle's recursion carries up to 1.3e-13 relative rounding (measured against
the same integrals in extended precision), so single f integrals are compared
at 1e-12 of the largest; the f transform is LL over two atoms (the oracle's
recursion for (ff|ff) is slow).  Compared here:
Schwarz factors and single integrals (1e-13 of the largest), kept
contribution counts (exact) and the MO integrals of LL, DC and DCG transforms
(max|G_gpu - G_oracle| <= 1e-12 max|G_oracle| on QR coefficients), on pair
spaces of several 64-pair tiles with a ragged last tile, under both integral
schedules, with directed and unique tiles, in both row orders, with d
functions in one basis or in both; two-spinor plans, the FP32 tier, the
MO-driven variant and graph replays.  Codes beyond f are refused at basis
creation (DCB plans over Cartesian bases: test_gpu_gauge_cart.py).
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


def _sys(ham, tau, seed=61, n_atoms=4, n=4, d_s=0):
    # per atom s + p shell + d shell in L (N_L = 40: 820 pairs, 12.8 tiles),
    # s + p shell (+ d_s d shells) in S
    return wl.spd_cluster(seed=seed, n_atoms=n_atoms, edge=5.0, n=n, ham=ham, tau=tau, d_s=d_s)


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
    print(f"{s.name} tau {tau} flags {flags} tune {tune}: max|dG| {err:.3e}, max|G| {scale:.3e}")
    assert err <= 1e-12 * scale, (err, scale)
    return st, sto


def test_d_schwarz_factors(q, ctx):
    # compared as the integrals (mn|mn) = Q_mn^2: a Schwarz factor is the square
    # root of one, so a small Q carries the integral's rounding (cancellation
    # among the Hermite terms of distant d pairs, ~1e-14 absolute, in either
    # route) amplified by 1 / (2 Q)
    s = _sys("DC", 0.0, d_s=1)
    for B in (s.L, s.S):
        Qg = q.Basis(ctx, B).schwarz()
        Qo = oracle.schwarz(B)
        assert np.abs(Qg**2 - Qo**2).max() <= 1e-13 * (Qo**2).max()
        assert np.abs(Qg - Qo).max() <= 1e-12 * np.abs(Qo).max()


def test_d_eri_quartets(q, ctx):
    s = _sys("DC", 0.0, seed=62, n_atoms=3, d_s=1)
    A, B = q.Basis(ctx, s.L), q.Basis(ctx, s.S)
    rng = np.random.default_rng(2)
    NL, NS = s.L.nfunc, s.S.nfunc
    idx = np.stack([rng.integers(0, NL, 500), rng.integers(0, NL, 500),
                    rng.integers(0, NS, 500), rng.integers(0, NS, 500)], 1)
    idx[:50, 1] = idx[:50, 0]  # same-function and same-centre pairs
    got = q.eri_quartets(A, B, idx)
    ref = np.array([oracle.eri(s.L, a, b, s.S, c, d) for a, b, c, d in idx])
    assert np.abs(got - ref).max() <= 1e-13 * np.abs(ref).max()
    # (dd|dd) quartets of one atom's d shell, every component combination
    d0 = [f for f in range(NL) if s.L.cart[f] >= 4][:6]
    idx2 = np.array([(a, b, c, d) for a in d0 for b in d0 for c in d0[:3] for d in d0[3:]])
    got2 = q.eri_quartets(A, A, idx2)
    ref2 = np.array([oracle.eri(s.L, a, b, s.L, c, d) for a, b, c, d in idx2])
    assert np.abs(got2 - ref2).max() <= 1e-13 * np.abs(ref2).max()
    # an s-only basis against one with d functions
    s2 = wl.small_ll(seed=3, n_atoms=3, nfunc=6, n=2)
    C = q.Basis(ctx, s2.L)
    idx3 = np.stack([rng.integers(0, NL, 100), rng.integers(0, NL, 100),
                     rng.integers(0, 6, 100), rng.integers(0, 6, 100)], 1)
    got3 = q.eri_quartets(A, C, idx3)
    ref3 = np.array([oracle.eri(s.L, a, b, s2.L, c, d) for a, b, c, d in idx3])
    assert np.abs(got3 - ref3).max() <= 1e-13 * np.abs(ref3).max()


@pytest.mark.parametrize("tau", [0.0, 1e-10])
@pytest.mark.parametrize("ham", ["LL", "DC", "DCG"])
def test_d_transform(q, ctx, ham, tau):
    st, _ = _check(q, ctx, _sys(ham, tau), tau)
    if tau > 0:
        assert sum(st["kept"]) < sum(st["total"])


def test_d_in_both_bases(q, ctx):
    _check(q, ctx, _sys("DCG", 1e-10, seed=63, d_s=1), 1e-10)


@pytest.mark.parametrize("eri_sched", [0, 1])
# 1: directed tiles (no unique-pair mirroring); 0x10: plain Schwarz rows
@pytest.mark.parametrize("flags", [0, 1, 0x10])
def test_d_schedules(q, ctx, eri_sched, flags):
    s = _sys("DC", 1e-10, seed=64)
    _check(q, ctx, s, 1e-10, flags=flags,
           tune={"eri_sched": eri_sched, "fh_order": 0, "sq_tile": 64})


def test_d_refuses_codes_beyond_f(q, ctx):
    s = _sys("DC", 0.0, n_atoms=2, n=2)
    with pytest.raises(q.QdcbError):
        q.Basis(ctx, wl.Basis(s.L.centers, s.L.nprim, s.L.exps, s.L.coefs,
                              np.full(s.L.nfunc, 20, np.int32)))


def test_d_spinor_plan_matches_oracle(q, ctx):
    s = _sys("DCG", 1e-10, seed=65, n_atoms=3, n=3)
    m = 4
    PL, PS, _ = wl.general_spinors(s, m, seed=13)
    L, S = q.Basis(ctx, s.L), q.Basis(ctx, s.S)
    plan = q.Plan(ctx, L, S, "DCG", m, 1e-10, flags=q.PLAN_SPINOR)
    G, st = plan.transform(PL, PS)
    Gc = G[..., 0] + 1j * G[..., 1]
    Go, so = oracle.transform_spinor(s.L, s.S, PL, PS, "DCG", 1e-10)
    assert so["tie_band"] == 0
    assert st["kept"] == so["kept"] and st["kept_gaunt"] == so["kept_gaunt"]
    assert np.abs(Gc - Go).max() <= 1e-12 * np.abs(Go).max()


def test_d_mixed_and_mo_driven(q, ctx):
    s = _sys("DC", 1e-10, seed=66)
    L, S = q.Basis(ctx, s.L), q.Basis(ctx, s.S)
    ref = q.Plan(ctx, L, S, "DC", s.n_mo, 1e-10)
    G0, st0 = ref.transform(s.CL, s.CS)
    # every kept tile in the FP32 tier: FP32 operands, FP32 accumulation
    mp = q.Plan(ctx, L, S, "DC", s.n_mo, 1e-10, prec="mixed", tier_fp32=1e300, tier_bf16=0.0)
    G1, st1 = mp.transform(s.CL, s.CS)
    assert st1["tiles_tier"][1] == st1["tiles_kept"]
    err = np.abs(G1 - G0).max()
    assert 0.0 < err <= 2e-6 * np.abs(G0).max()
    mo = q.Plan(ctx, L, S, "DC", s.n_mo, 1e-10)
    mo.set_mo_batch(2)
    G2, st2 = mo.transform(s.CL, s.CS)
    Go, _ = oracle.transform_direct_mo(s.L, s.S, s.CL, s.CS, "DC", 1e-10, 2)
    assert np.abs(G2 - Go).max() <= 1e-12 * np.abs(Go).max()


def test_d_graph_replays_equal_eager(q, ctx):
    import torch
    s = _sys("DCG", 1e-10, seed=67, n_atoms=3, n=4)
    L, S = q.Basis(ctx, s.L), q.Basis(ctx, s.S)
    plan = q.Plan(ctx, L, S, "DCG", s.n_mo, 1e-10)
    dev = torch.device("cuda:0")
    CL = torch.from_numpy(s.CL).to(dev)
    CS = torch.from_numpy(s.CS).to(dev)
    n = s.n_mo
    G = torch.empty((n, n, n, n, 4, 4), dtype=torch.float64, device=dev)
    stream = torch.cuda.Stream()
    plan.capture(CL, CS, G, stream)
    rng = np.random.default_rng(68)
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


def _f_sys(ham="LL", tau=1e-10, seed=71):
    # two atoms, s + p shell + f shell in L (N_L = 28: 406 pairs, 6.3 tiles)
    return wl.spd_cluster(seed=seed, n_atoms=2, edge=5.0, n=3, ham=ham, tau=tau, d_l=0, f_l=1,
                          nprim=1, p_s=0)


def test_f_schwarz_factors(q, ctx):
    s = wl.spd_cluster(seed=72, n_atoms=2, edge=5.0, n=2, ham="LL", d_l=1, f_l=1)
    Qg = q.Basis(ctx, s.L).schwarz()
    Qo = oracle.schwarz(s.L)
    assert np.abs(Qg**2 - Qo**2).max() <= 1e-12 * (Qo**2).max()


def test_f_eri_quartets(q, ctx):
    s = wl.spd_cluster(seed=73, n_atoms=2, edge=4.0, n=2, ham="DC", d_l=1, f_l=1, d_s=1)
    A, B = q.Basis(ctx, s.L), q.Basis(ctx, s.S)
    rng = np.random.default_rng(4)
    NL, NS = s.L.nfunc, s.S.nfunc
    fl = np.array([f for f in range(NL) if s.L.cart[f] >= 10])
    idx = np.stack([rng.choice(fl, 300), rng.integers(0, NL, 300),
                    rng.integers(0, NS, 300), rng.integers(0, NS, 300)], 1)
    idx[:30, 1] = idx[:30, 0]
    got = q.eri_quartets(A, B, idx)
    ref = np.array([oracle.eri(s.L, a, b, s.S, c, d) for a, b, c, d in idx])
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()
    # (ff|ff) over one f shell and (ff|ds) across the two atoms
    idx2 = np.array([(a, b, c, d) for a in fl[:10:3] for b in fl[:10:2] for c in fl[10::3]
                     for d in fl[10::4]])
    got2 = q.eri_quartets(A, A, idx2)
    ref2 = np.array([oracle.eri(s.L, a, b, s.L, c, d) for a, b, c, d in idx2])
    assert np.abs(got2 - ref2).max() <= 1e-12 * np.abs(ref2).max()


def test_f_transform(q, ctx):
    s = _f_sys()
    _check(q, ctx, s, 1e-10)


@pytest.mark.parametrize("budget_mb", [40, 24])
def test_d_small_budgets(q, budget_mb):
    # small context budgets: several integral-panel batches, the general
    # kernels writing at slot offsets
    s = _sys("DCG", 1e-10, seed=69, n=6)
    c = q.Context(0, budget_bytes=budget_mb << 20)
    try:
        st, _ = _check(q, c, s, 1e-10, flags=q.PLAN_DIRECTED_TILES if budget_mb == 24 else 0)
        assert st["n_batches"] > 1, (st["n_chunks"], st["n_batches"])
    finally:
        c.close()
