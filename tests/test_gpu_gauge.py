"""GPU parity of the gauge term of the Breit operator (QDCB_HAM_DCB) against
the oracle's DCB and gauge-only routes.

The gauge classes share the Gaunt classes' L-S pairs, screening predicate and
task lists; their integral tiles carry six components
B_KL = ((mn| r_K r_L / r^3 |kl) - delta_KL (mn|kl)) / 2 and their first half
couples K and L.  Tolerance: 1e-12 of the Schwarz magnitude bound of the sums
as in test_gpu_parity.py, with the L-S term's bound (max_mn,kl a)^2 scaled by
(1 + 3/2)^2: every |B_KL| is at most (mn|kl)/2 for the non-negative s pair
distributions, and V^K sums three of them.  Kept counts are exact.

FP64 plans contract the Gaunt and gauge terms together from fused Breit tiles
B_KL + delta_KL (mn|kl); a single class, or a mixed-precision plan (whose
Gaunt term has precision tiers), runs them apart.

Cases: quaternion and general-spinor plans, tau = 0 and tau > 0, every class
alone and summed, unique (resident) and directed-batch tiles, several column
chunks, both integral schedules, captured replays, the mixed-precision plan
with every tile in the FP64 tier, and the MO-driven variant.
"""
import numpy as np
import pytest

import oracle
from paper_2606_04316_amd import workloads as wl
from tests import qalg

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


def _ls_bound(s, CL, CS):
    nL = np.sqrt((CL ** 2).sum(0))
    nS = np.sqrt((CS ** 2).sum(0))
    a = nL.T @ oracle.schwarz(s.L, s.S) @ nS
    return float(np.max(a + a.T)) ** 2


def _scale(s, CL=None, CS=None, coulomb=True):
    CL = s.CL if CL is None else CL
    CS = s.CS if CS is None else CS
    sc = qalg.schwarz_scale([oracle.schwarz(s.L), oracle.schwarz(s.S)], [CL, CS]) if coulomb else 0.0
    return sc + 3 * 6.25 * _ls_bound(s, CL, CS)


def _chain(seed, n=4, tau=0.0, n_atoms=5, ns_per_atom=4):
    return wl.linear_chain(seed=seed, n_atoms=n_atoms, spacing=3.0, nl_per_atom=3,
                           ns_per_atom=ns_per_atom, n=n, tau=tau, ham="DCB")


@pytest.mark.parametrize("tau", [0.0, 1e-9])
def test_dcb_matches_oracle(q, ctx, tau):
    s = _chain(61, tau=tau)
    L, S = q.Basis(ctx, s.L), q.Basis(ctx, s.S)
    plan = q.Plan(ctx, L, S, "DCB", s.n_mo, tau)
    G, st = plan.transform(s.CL, s.CS)
    Go, so = oracle.transform_direct(s.L, s.S, s.CL, s.CS, "DCB", tau)
    assert so["tie_band"] == 0
    assert st["kept"] == so["kept"] and st["kept_gaunt"] == so["kept_gaunt"]
    assert st["classes"] == 7
    if tau > 0:
        assert st["kept_gaunt"] < st["total_gaunt"]
    scale = _scale(s)
    err = np.abs(G - Go).max()
    # the gauge term is not negligible next to the tolerance
    Gg, _ = oracle.transform_direct(s.L, s.S, s.CL, s.CS, "GAUGE", tau)
    print(f"DCB tau {tau}: max|dG| {err:.3e}, scale {scale:.3e}, max|G_gauge| "
          f"{np.abs(Gg).max():.3e}")
    assert err <= 1e-12 * scale
    assert np.abs(Gg).max() > 1e6 * max(err, 1e-16 * scale)
    # quaternion sign rules of the summed classes: bra-ket symmetry holds for
    # every class; the gauge part alone has the Gaunt signs under p <-> q
    assert np.abs(G.transpose(2, 3, 0, 1, 5, 4) - G).max() <= 1e-12 * scale


def test_classes_alone_and_summed(q, ctx):
    s = _chain(62, tau=1e-10)
    L, S = q.Basis(ctx, s.L), q.Basis(ctx, s.S)
    plan = q.Plan(ctx, L, S, "DCB", s.n_mo, s.tau)
    G, st = plan.transform(s.CL, s.CS)
    parts = {}
    for cls, ham in (("coulomb", "DC"), ("gaunt", "GAUNT"), ("gauge", "GAUGE")):
        Gc, stc = plan.transform(s.CL, s.CS, classes=cls)
        Go, so = oracle.transform_direct(s.L, s.S, s.CL, s.CS, ham, s.tau)
        assert stc["kept"] == so["kept"] and stc["kept_gaunt"] == so["kept_gaunt"], cls
        sc = _scale(s, coulomb=cls == "coulomb") if cls != "coulomb" else qalg.schwarz_scale(
            [oracle.schwarz(s.L), oracle.schwarz(s.S)], [s.CL, s.CS])
        err = np.abs(Gc - Go).max()
        print(f"class {cls}: max|dG| {err:.3e} (scale {sc:.3e})")
        assert err <= 1e-12 * sc, cls
        parts[cls] = Gc
    assert plan.transform(s.CL, s.CS, classes="gauge")[1]["classes"] == 4
    Gb, stb = plan.transform(s.CL, s.CS, classes="breit")
    assert stb["classes"] == 6
    scale = _scale(s)
    assert np.abs(parts["gaunt"] + parts["gauge"] - Gb).max() <= 1e-13 * scale
    assert np.abs(parts["coulomb"] + Gb - G).max() <= 1e-13 * scale
    # work accounting: the gauge first half has three times the Gaunt products
    stg = plan.transform(s.CL, s.CS, classes="gaunt")[1]
    stq = plan.transform(s.CL, s.CS, classes="gauge")[1]
    assert stq["flops_first_half"] == pytest.approx(3 * stg["flops_first_half"])
    assert stq["flops_mfma"] == pytest.approx(3 * stg["flops_mfma"])
    # DCG plans have no gauge class
    pg = q.Plan(ctx, L, S, "DCG", s.n_mo, s.tau)
    with pytest.raises(q.QdcbError):
        pg.transform(s.CL, s.CS, classes="gauge")
    # and their transform is the DCB plan's Coulomb + Gaunt classes
    Gdcg, _ = pg.transform(s.CL, s.CS)
    assert np.abs(Gdcg - parts["coulomb"] - parts["gaunt"]).max() <= 1e-13 * scale


@pytest.mark.parametrize("budget_mb,flags", [(0, 1), (24, 0)])
def test_directed_tiles_batches_and_chunks(q, budget_mb, flags):
    # flags = 1: QDCB_PLAN_DIRECTED_TILES (every directed tile computed, no
    # unique pairs); a small budget: several column chunks and panel batches
    s = _chain(63, n=12, tau=1e-10, n_atoms=6, ns_per_atom=5)
    ctx = q.Context(0, budget_bytes=budget_mb << 20)
    L, S = q.Basis(ctx, s.L), q.Basis(ctx, s.S)
    plan = q.Plan(ctx, L, S, "DCB", s.n_mo, s.tau, flags=flags)
    G, st = plan.transform(s.CL, s.CS)
    print(f"budget {budget_mb} MB flags {flags}: chunks {st['n_chunks']}, "
          f"batches {st['n_batches']}")
    if budget_mb:
        assert st["n_chunks"] > 1
    Go, so = oracle.transform_direct(s.L, s.S, s.CL, s.CS, "DCB", s.tau)
    assert st["kept"] == so["kept"] and st["kept_gaunt"] == so["kept_gaunt"]
    assert np.abs(G - Go).max() <= 1e-12 * _scale(s)
    plan.close()
    ctx.close()


def test_schedules_replay_and_mixed_fp64_tier(q, ctx):
    import torch
    s = _chain(64, n=6, tau=1e-10, n_atoms=6)
    L, S = q.Basis(ctx, s.L), q.Basis(ctx, s.S)
    res = []
    for e in (0, 1):
        plan = q.Plan(ctx, L, S, "DCB", s.n_mo, s.tau)
        plan.tune = {"eri_sched": e, "fh_order": 1 - e, "sq_tile": 64}
        res.append(plan.transform(s.CL, s.CS)[0])
        plan.close()
    assert np.array_equal(res[0], res[1])  # the schedule and order change no bit
    plan = q.Plan(ctx, L, S, "DCB", s.n_mo, s.tau)
    dev = torch.device("cuda:0")
    CL = torch.from_numpy(s.CL).to(dev)
    CS = torch.from_numpy(s.CS).to(dev)
    G = torch.empty(plan.g_shape(), dtype=torch.float64, device=dev)
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
        assert st["kept_gaunt"] == ste["kept_gaunt"]
        assert torch.equal(Gr, Ge), k
    # mixed precision with every tile in the FP64 tier is the FP64 plan to
    # rounding: the gauge term is contracted in FP64 in every precision mode,
    # apart from the Gaunt term's tiers (FP64 plans contract the two terms
    # together from the fused Breit tiles)
    pm = q.Plan(ctx, L, S, "DCB", s.n_mo, s.tau, prec="mixed", tier_fp32=0.0, tier_bf16=0.0)
    Gm, stm = pm.transform(s.CL, s.CS)
    Go, so = oracle.transform_direct(s.L, s.S, s.CL, s.CS, "DCB", s.tau)
    assert stm["kept_gaunt"] == so["kept_gaunt"]
    assert np.abs(Gm - res[0]).max() <= 1e-13 * _scale(s)
    assert np.abs(Gm - Go).max() <= 1e-12 * _scale(s)


def test_spinor_plan_dcb_matches_oracle(q, ctx):
    s = _chain(65, n=4, tau=1e-9)
    m = 7
    PL, PS, _ = wl.general_spinors(s, m, seed=14)
    L, S = q.Basis(ctx, s.L), q.Basis(ctx, s.S)
    plan = q.Plan(ctx, L, S, "DCB", m, s.tau, flags=q.PLAN_SPINOR)
    G, st = plan.transform(PL, PS)
    Gc = G[..., 0] + 1j * G[..., 1]
    Go, so = oracle.transform_spinor(s.L, s.S, PL, PS, "DCB", s.tau)
    assert so["tie_band"] == 0
    assert st["kept"] == so["kept"] and st["kept_gaunt"] == so["kept_gaunt"]
    scale = _scale(s, PL, PS)
    err = np.abs(Gc - Go).max()
    print(f"spinor DCB: max|dG| {err:.3e}, scale {scale:.3e}")
    assert err <= 1e-12 * scale
    assert np.abs(Gc - Gc.transpose(1, 0, 3, 2).conj()).max() <= 1e-12 * scale


def test_mo_driven_dcb_matches_oracle(q, ctx):
    s = _chain(66, n=5, tau=1e-9)
    L, S = q.Basis(ctx, s.L), q.Basis(ctx, s.S)
    plan = q.Plan(ctx, L, S, "DCB", s.n_mo, s.tau)
    plan.set_mo_batch(4)
    G, st = plan.transform(s.CL, s.CS)
    Go, so = oracle.transform_direct_mo(s.L, s.S, s.CL, s.CS, "DCB", s.tau, 4)
    assert st["kept"] == so["kept"] and st["kept_gaunt"] == so["kept_gaunt"]
    assert np.abs(G - Go).max() <= 1e-12 * _scale(s)


def test_degenerate_cases(q, ctx):
    # nothing kept: G is zero and no tile is made
    s = _chain(67, n=3, tau=1e30)
    L, S = q.Basis(ctx, s.L), q.Basis(ctx, s.S)
    G, st = q.Plan(ctx, L, S, "DCB", s.n_mo, 1e30).transform(s.CL, s.CS)
    assert not np.any(G) and st["kept_gaunt"] == 0 and st["tiles_kept"] == 0
    # one MO (a single MO pair, one column group) and a single-atom basis
    s1 = wl.linear_chain(seed=68, n_atoms=1, spacing=3.0, nl_per_atom=3, ns_per_atom=4, n=1,
                         tau=0.0, ham="DCB")
    L1, S1 = q.Basis(ctx, s1.L), q.Basis(ctx, s1.S)
    G1, st1 = q.Plan(ctx, L1, S1, "DCB", 1, 0.0).transform(s1.CL, s1.CS)
    Go, so = oracle.transform_direct(s1.L, s1.S, s1.CL, s1.CS, "DCB", 0.0)
    assert st1["kept_gaunt"] == so["kept_gaunt"] == (3 * 4) ** 2
    assert np.abs(G1 - Go).max() <= 1e-12 * _scale(s1)
