"""GPU tests of the mixed-precision first half (FP64 / FP32 / BF16 tiers).

Tiles are assigned to a tier by their screening bound B = max Q (bra tile) x
max Q Dmax (ket tile).  Forcing every tile into one tier checks each kernel
path on its own: the FP64 tier run through the tier lists must equal the
FP64 plan bitwise (same tasks, same order), the FP32 and BF16 tiers must agree
with the FP64 result to their operand precision (relative rounding 2^-24 and
2^-9 of each operand, FP32 accumulation), measured against the Schwarz
magnitude bound of the sums (the same scale as the parity tests).  With the
default tiers the error is reported and must stay within the a-priori budget
of the low tiers.  The oracle pins the FP64 tier.
"""
import numpy as np
import pytest

import oracle
from paper_2606_04316_amd import workloads as wl
from tests import qalg

pytestmark = pytest.mark.gpu

HUGE = 1e300


@pytest.fixture(scope="module")
def q():
    from paper_2606_04316_amd import qdcb
    return qdcb


@pytest.fixture(scope="module")
def ctx(q):
    c = q.Context(0)
    yield c
    c.close()


def _run(q, ctx, s, prec="fp64", t32=1e-4, t16=1e-7, flags=0):
    L = q.Basis(ctx, s.L)
    S = q.Basis(ctx, s.S) if s.S is not None else None
    plan = q.Plan(ctx, L, S, s.ham, s.n_mo, s.tau, prec=prec, tier_fp32=t32, tier_bf16=t16,
                  flags=flags)
    G, st = plan.transform(s.CL, s.CS)
    plan.close()
    return G, st


def _scale(s):
    Qs, Cs = [oracle.schwarz(s.L)], [s.CL]
    if s.S is not None:
        Qs.append(oracle.schwarz(s.S))
        Cs.append(s.CS)
    sc = qalg.schwarz_scale(Qs, Cs)
    if s.ham == "DCG":
        nL = np.sqrt((s.CL ** 2).sum(0))
        nS = np.sqrt((s.CS ** 2).sum(0))
        a = nL.T @ oracle.schwarz(s.L, s.S) @ nS
        sc += 3 * float(np.max(a + a.T)) ** 2
    return sc


def _j_occ(G):
    # occupied-block Coulomb sum over the first n/2 Kramers pairs
    occ = range(G.shape[0] // 2)
    return 4.0 * sum(G[p, p, r, r, 0, 0] for p in occ for r in occ)


SYSTEMS = {
    "DC": lambda: wl.linear_chain(seed=60, n_atoms=8, spacing=3.0, nl_per_atom=3, ns_per_atom=6,
                                  n=6, tau=1e-10),
    "DCG": lambda: wl.linear_chain(seed=61, n_atoms=6, spacing=3.2, nl_per_atom=3,
                                   ns_per_atom=4, n=5, tau=1e-10, ham="DCG"),
}


@pytest.mark.parametrize("ham", ["DC", "DCG"])
def test_fp64_tier_equals_fp64_plan(q, ctx, ham):
    s = SYSTEMS[ham]()
    G0, st0 = _run(q, ctx, s)
    G1, st1 = _run(q, ctx, s, prec="mixed", t32=0.0, t16=0.0)
    assert st1["tiles_tier"][0] == st1["tiles_kept"] and st1["tiles_tier"][1:] == [0, 0]
    assert st1["kept"] == st0["kept"]
    assert np.array_equal(G0, G1)


@pytest.mark.parametrize("ham", ["DC", "DCG"])
@pytest.mark.parametrize("tier,tol", [(1, 2e-6), (2, 2e-2)])
def test_single_low_tier_within_operand_precision(q, ctx, ham, tier, tol):
    s = SYSTEMS[ham]()
    G0, _ = _run(q, ctx, s)
    t32, t16 = (HUGE, 0.0) if tier == 1 else (HUGE, HUGE)
    G1, st = _run(q, ctx, s, prec="mixed", t32=t32, t16=t16)
    assert st["tiles_tier"][tier] == st["tiles_kept"]
    err = np.abs(G1 - G0).max()
    scale = _scale(s)
    print(f"{ham} tier {tier}: max|dG| {err:.3e}, scale {scale:.3e}, rel {err / scale:.2e}")
    assert err <= tol * scale
    # not trivially equal: the reduced operands do change the result
    assert err > 0.0


@pytest.mark.parametrize("ham", ["DC", "DCG"])
@pytest.mark.parametrize("rule", ["screen", "g"])
def test_default_tiers_error(q, ctx, ham, rule):
    # Tiers 1e-4 / 1e-7.  The screening-bound rule ignores the bra-side
    # coefficients that carry a V error into G (|conj(C_mp) C_nq| up to the
    # bra pair's Dmax, large for Loewdin coefficients of a near-dependent basis);
    # the G rule includes them.  Reported, with the budgets: FP32 operands are
    # rounded to 2^-24 relative, BF16 to 2^-9, so with the G rule each low-tier
    # contribution moves G by at most ~1e-4 * 2^-23 or ~1e-7 * 2^-8.
    s = SYSTEMS[ham]()
    G0, st0 = _run(q, ctx, s)
    flags = q.PLAN_TIER_BY_G if rule == "g" else 0
    G1, st1 = _run(q, ctx, s, prec="mixed", flags=flags)
    Go, _ = oracle.transform_direct(s.L, s.S, s.CL, s.CS, ham, s.tau)
    assert st1["kept"] == st0["kept"]
    assert sum(st1["tiles_tier"]) == st1["tiles_kept"]
    err = np.abs(G1 - G0).max()
    derr = np.abs(G1 - Go).max()
    dj = abs(_j_occ(G1) - _j_occ(G0))
    print(f"{ham} rule {rule} tiers {st1['tiles_tier']}: max|dG| vs FP64 {err:.3e}, vs oracle "
          f"{derr:.3e}, |dJ_occ| {dj:.3e}, max|G| {np.abs(G0).max():.3e}")
    assert err <= 1e-6 * _scale(s)
    assert derr <= err + 1e-12 * _scale(s)


def test_mixed_graph_replay_equals_eager(q):
    import torch
    s = wl.linear_chain(seed=62, n_atoms=6, spacing=3.0, nl_per_atom=3, ns_per_atom=5, n=8,
                        tau=1e-10, ham="DCG")
    ctx = q.Context(0)
    L, S = q.Basis(ctx, s.L), q.Basis(ctx, s.S)
    plan = q.Plan(ctx, L, S, "DCG", s.n_mo, s.tau, prec="mixed", tier_fp32=1e-3, tier_bf16=1e-6)
    dev = torch.device("cuda:0")
    CL = torch.from_numpy(s.CL).to(dev)
    CS = torch.from_numpy(s.CS).to(dev)
    n = s.n_mo
    G = torch.empty((n, n, n, n, 4, 4), dtype=torch.float64, device=dev)
    stream = torch.cuda.Stream()
    plan.capture(CL, CS, G, stream)
    for k in range(3):
        cl, cs = (s.CL, s.CS) if k == 0 else wl.perturbed_coefficients(s, k)
        CL.copy_(torch.from_numpy(cl))
        CS.copy_(torch.from_numpy(cs))
        torch.cuda.synchronize()
        st = plan.replay(stream)
        assert st["graph_replay"] and not st["graph_fallback"]
        Gr = G.clone()
        Ge, ste = plan.transform(torch.from_numpy(cl).to(dev), torch.from_numpy(cs).to(dev))
        torch.cuda.synchronize()
        assert sum(ste["tiles_tier"][1:]) > 0
        assert torch.equal(Gr, Ge), k
    plan.close()
    ctx.close()
