"""GPU tests of the mixed-precision first half (FP64 / FP32 / BF16 tiers).

Tiles are assigned to a tier by their bound: the screening bound
B = max Q (bra tile pair) x max Q Dmax (ket tile), or with QDCB_PLAN_TIER_BY_G
the bound B_G = max Q Dmax (bra tile pair) x max Q Dmax (ket tile) of a
contribution's effect on G; the bra factor is taken over the pair of bra
tiles (2i, 2i + 1) that one first-half workgroup contracts.  The FP64 tier run through the tier lists must equal the FP64
plan bitwise (same tasks, same order).  The reduced tiers are checked element
by element against an a-priori bound (tests/mixed_bound.py): the contribution
bound decides the worst tier a contribution can land in, its rounding error is
at most eps_tier |I| |D~| (operand unit roundoff and FP32 accumulation), and
the second half carries it into G through the bra pair densities; the FP64
oracle is the reference, on well-conditioned (QR) coefficients where the FP64
part of the error is below 1e-12 of max|G|.  On the chain recipe with Loewdin
coefficients, the tiers the benchmark reports (G rule, 3e-6 / 1e-9) must keep
the reduced tiers' error (against the FP64 transform) below 1e-10 Eh, and on QR
coefficients max|G - G_oracle| <= 1e-10 Eh.
"""
import numpy as np
import pytest

import oracle
from paper_2606_04316_amd import workloads as wl
from tests import mixed_bound, qalg

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


QR_SYSTEMS = {
    "DC": lambda: wl.linear_chain(seed=60, n_atoms=8, spacing=3.0, nl_per_atom=3,
                                  ns_per_atom=6, n=6, tau=1e-10, coefs="qr"),
    "DCG": lambda: wl.linear_chain(seed=61, n_atoms=6, spacing=3.2, nl_per_atom=3,
                                   ns_per_atom=4, n=5, tau=1e-10, ham="DCG", coefs="qr"),
}


def _check_bound(s, G, st, rule, t32, t16, what):
    Go, so = oracle.transform_direct(s.L, s.S, s.CL, s.CS, s.ham, s.tau)
    assert st["kept"] == so["kept"] and st["kept_gaunt"] == so["kept_gaunt"]
    B = mixed_bound.bound(s, s.CL, s.CS, s.tau, rule, t32, t16)
    gmax = float(np.abs(Go).max())
    err = np.abs(mixed_bound.upper_part(G) - mixed_bound.upper_part(Go))
    ratio = float((err / (B + 1e-12 * gmax)).max())
    print(f"{what}: tiles {st['tiles_tier']}, max|dG| {err.max():.3e}, bound max "
          f"{B.max():.3e}, max|G| {gmax:.3e}, worst error / bound {ratio:.3f}")
    assert np.all(err <= B + 1e-12 * gmax), what
    return float(err.max()), float(B.max())


@pytest.mark.parametrize("ham", ["DC", "DCG"])
@pytest.mark.parametrize("tier", [1, 2])
def test_single_low_tier_within_a_priori_bound(q, ctx, ham, tier):
    s = QR_SYSTEMS[ham]()
    t32, t16 = (HUGE, 0.0) if tier == 1 else (HUGE, HUGE)
    G1, st = _run(q, ctx, s, prec="mixed", t32=t32, t16=t16)
    assert st["tiles_tier"][tier] == st["tiles_kept"]
    err, bmax = _check_bound(s, G1, st, "screen", t32, t16, f"{ham} all tiles in tier {tier}")
    # not trivially equal: the reduced operands do change the result
    assert err > 0.0


@pytest.mark.parametrize("ham", ["DC", "DCG"])
@pytest.mark.parametrize("rule", ["screen", "g"])
def test_specified_tiers_within_a_priori_bound(q, ctx, ham, rule):
    # the mixed configuration's tiers, 1e-4 (FP32) and 1e-7 (BF16)
    s = QR_SYSTEMS[ham]()
    flags = q.PLAN_TIER_BY_G if rule == "g" else 0
    G0, st0 = _run(q, ctx, s)
    G1, st1 = _run(q, ctx, s, prec="mixed", flags=flags)
    assert st1["kept"] == st0["kept"]
    assert sum(st1["tiles_tier"]) == st1["tiles_kept"]
    assert st1["tiles_tier"][1] > 0 and st1["tiles_tier"][2] > 0
    _check_bound(s, G1, st1, rule, 1e-4, 1e-7, f"{ham} rule {rule} tiers 1e-4 / 1e-7")
    dj = abs(_j_occ(G1) - _j_occ(G0))
    print(f"  |dJ_occ| vs FP64 {dj:.3e}")


@pytest.mark.parametrize("ham", ["DC", "DCG"])
@pytest.mark.parametrize("coefs", ["qr", "loewdin"])
def test_benchmark_tiers_meet_1e10_hartree(q, ctx, ham, coefs):
    # the tiers the benchmark reports: G rule, FP32 below 3e-6, BF16 below
    # 1e-9.  QR coefficients: max|G_mixed - G_oracle| <= 1e-10 Eh directly.
    # Loewdin coefficients (the benchmark's inputs, at test size): there the
    # FP64 path and the oracle already differ at the 1e-10 level (the MO
    # integrals are small differences of large terms, summed in different
    # orders), so the reduced tiers' part of the error is measured against
    # the FP64 GPU transform (identical except for the low-tier tiles), and
    # the FP64 transform is held to the oracle at the parity tolerance.
    s = (QR_SYSTEMS if coefs == "qr" else SYSTEMS)[ham]()
    G0, st0 = _run(q, ctx, s)
    G1, st1 = _run(q, ctx, s, prec="mixed", t32=3e-6, t16=1e-9, flags=q.PLAN_TIER_BY_G)
    Go, so = oracle.transform_direct(s.L, s.S, s.CL, s.CS, ham, s.tau)
    assert st1["kept"] == so["kept"] and st1["kept_gaunt"] == so["kept_gaunt"]
    assert st1["tiles_tier"][1] > 0
    err_o = float(np.abs(G1 - Go).max())
    err_64 = float(np.abs(G1 - G0).max())
    fp64_o = float(np.abs(G0 - Go).max())
    dj = abs(_j_occ(G1) - _j_occ(G0))
    print(f"{ham} {coefs} G rule 3e-6 / 1e-9: tiles {st1['tiles_tier']}, max|G - G_FP64| "
          f"{err_64:.3e} Eh, max|G - G_oracle| {err_o:.3e} Eh (FP64 vs oracle {fp64_o:.3e}), "
          f"|dJ_occ| {dj:.3e}, max|G| {np.abs(Go).max():.3e}")
    assert err_64 <= 1e-10
    if coefs == "qr":
        assert err_o <= 1e-10 and fp64_o <= 1e-12 * np.abs(Go).max()
    else:
        assert fp64_o <= 1e-12 * _schwarz_scale(s)


@pytest.mark.parametrize("budget_mb", [40, 24])
def test_tiers_in_chunks_and_batches_within_a_priori_bound(q, budget_mb):
    # small budgets: several MO-pair column chunks (each with its FP32 density
    # copy) and bra-tile batches of the integral panels, so tier sub-lists
    # start at odd bra tiles and the reduced-tier launches run per batch
    s = wl.linear_chain(seed=42, n_atoms=6, spacing=3.0, nl_per_atom=3, ns_per_atom=5, n=16,
                        tau=1e-10, ham="DCG", coefs="qr")
    small = q.Context(0, budget_bytes=budget_mb << 20)
    G1, st1 = _run(q, small, s, prec="mixed")
    small.close()
    print(f"budget {budget_mb} MB: chunks {st1['n_chunks']}, launches {st1['n_batches']}")
    assert st1["n_chunks"] > 1
    assert st1["tiles_tier"][1] > 0 and st1["tiles_tier"][2] > 0
    _check_bound(s, G1, st1, "screen", 1e-4, 1e-7, f"DCG {budget_mb} MB tiers 1e-4 / 1e-7")


def test_dcb_reduced_gaunt_tiers_match_fp64_within_operand_error(q, ctx):
    # DCB mixed plans: the Gaunt term in tiers, the gauge term in FP64 over the
    # same lists.  With every Gaunt tile in FP32 the result stays within the
    # FP32 operand error of the FP64 plan.
    s = wl.linear_chain(seed=63, n_atoms=5, spacing=3.0, nl_per_atom=3, ns_per_atom=4, n=5,
                        tau=1e-10, ham="DCB", coefs="qr")
    G0, st0 = _run(q, ctx, s)
    G1, st1 = _run(q, ctx, s, prec="mixed", t32=HUGE, t16=0.0)
    assert st1["tiles_tier"][1] == st1["tiles_kept"] > 0
    assert st1["kept"] == st0["kept"] and st1["kept_gaunt"] == st0["kept_gaunt"]
    err = float(np.abs(G1 - G0).max())
    gmax = float(np.abs(G0).max())
    print(f"DCB all Gaunt tiles FP32: max|G - G_FP64| {err:.3e}, max|G| {gmax:.3e}")
    assert 0.0 < err <= 1e-5 * gmax


def _schwarz_scale(s):
    # the Schwarz magnitude bound of the sums (the parity tolerance scale of
    # Loewdin-coefficient tests, see test_gpu_parity.py)
    Qs, Cs = [oracle.schwarz(s.L), oracle.schwarz(s.S)], [s.CL, s.CS]
    sc = qalg.schwarz_scale(Qs, Cs)
    if s.ham == "DCG":
        nL = np.sqrt((s.CL ** 2).sum(0))
        nS = np.sqrt((s.CS ** 2).sum(0))
        a = nL.T @ oracle.schwarz(s.L, s.S) @ nS
        sc += 3 * float(np.max(a + a.T)) ** 2
    return sc


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
