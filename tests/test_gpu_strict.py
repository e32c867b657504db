"""Strict GPU parity: every path of the HIP library on well-conditioned
coefficients, max|G_gpu - G_oracle| <= 1e-12 * max|G_oracle| (the normwise
reading of "1e-12 relative"), kept counts exact.

The other parity tests use Loewdin coefficients of numerically near-dependent
bases, where every MO integral is a small difference of large terms and two
equivalent FP64 routes of the oracle itself differ by up to ~1e-8 of max|G|;
they are held to 1e-12 of the Schwarz magnitude bound of the sums instead.
Here the coefficients are a random quaternion-orthonormal (N_L + N_S) x n
matrix (|C_mu p| <= 1, workloads.qr_coefficients), so the integrals are not
cancellations and max|G| is the scale.  Each test is the twin of a test that
runs the same path on Loewdin coefficients:

  DC and DCG chains, tau = 0 / screened         test_gpu_parity
  uneven contraction depth clusters (DC, DCG)    test_gpu_parity, test_gpu_tune
  unique vs directed integral tiles              test_gpu_parity
  column chunks and panel batches (24 / 40 MB)   test_gpu_parity
  every launch choice (schedule x order x tile)  test_gpu_tune
  DCB: all classes, each class alone, batches    test_gpu_gauge
  general two-spinor LL / DC / DCG / DCB plans   test_gpu_spinor, test_gpu_gauge
  MO-driven variant (DC, DCG, DCB)               test_gpu_mo_driven, test_gpu_gauge
  device pointers, blocked output                test_gpu_parity, test_gpu_blocks
  captured replays (vs the oracle, each replay)  test_gpu_replay_serving
"""
import numpy as np
import pytest

import oracle
from paper_2606_04316_amd import workloads as wl

pytestmark = pytest.mark.gpu

REL = 1e-12


@pytest.fixture(scope="module")
def q():
    from paper_2606_04316_amd import qdcb
    return qdcb


@pytest.fixture(scope="module")
def ctx(q):
    c = q.Context(0)
    yield c
    c.close()


def _strict(G, Go, what=""):
    gmax = float(np.abs(Go).max())
    err = float(np.abs(G - Go).max())
    print(f"{what}: max|dG| {err:.3e}, max|G| {gmax:.3e}, rel {err / max(gmax, 1e-300):.2e}",
          flush=True)
    assert gmax > 0.0, what
    assert err <= REL * gmax, (what, err / gmax)


def _chain(seed, n_atoms=6, spacing=3.0, nl=3, ns=4, n=5, tau=1e-10, ham="DC"):
    return wl.linear_chain(seed=seed, n_atoms=n_atoms, spacing=spacing, nl_per_atom=nl,
                           ns_per_atom=ns, n=n, tau=tau, ham=ham, coefs="qr")


def _bases(q, ctx, s):
    return q.Basis(ctx, s.L), (q.Basis(ctx, s.S) if s.S is not None else None)


def _run(q, ctx, s, ham=None, tau=None, flags=0, tune=None, classes=None, mo_batch=0):
    L, S = _bases(q, ctx, s)
    ham = s.ham if ham is None else ham
    tau = s.tau if tau is None else tau
    plan = q.Plan(ctx, L, S, ham, s.n_mo, tau, flags=flags)
    if tune is not None:
        plan.tune = tune
    if mo_batch:
        plan.set_mo_batch(mo_batch)
    G, st = plan.transform(s.CL, s.CS, classes=classes)
    plan.close()
    return G, st


def _same_counts(st, so):
    assert so["tie_band"] == 0
    assert st["kept"] == so["kept"], (st["kept"], so["kept"])
    assert st["kept_gaunt"] == so["kept_gaunt"]


@pytest.mark.parametrize("ham,tau", [("LL", 0.0), ("LL", 1e-9), ("DC", 0.0), ("DC", 1e-10),
                                     ("DC", 1e-5), ("DCG", 0.0), ("DCG", 1e-9)])
def test_chain_strict(q, ctx, ham, tau):
    # 8 atoms 4 bohr apart (DC: 24 L + 48 S functions, 1476 pairs = 23 tiles + 4 rows)
    if ham == "LL":
        s = wl.small_ll(seed=36, n_atoms=6, nfunc=30, n=7, edge=7.0, tau=tau, coefs="qr")
    elif ham == "DC":
        s = _chain(34, n_atoms=8, spacing=4.0, nl=3, ns=6, n=6, tau=tau)
    else:
        s = _chain(40, n_atoms=6, spacing=3.5, nl=3, ns=4, n=4, tau=tau, ham="DCG")
    G, st = _run(q, ctx, s)
    Go, so = oracle.transform_direct(s.L, s.S, s.CL, s.CS, ham, tau)
    _same_counts(st, so)
    if tau >= 1e-5:
        assert sum(st["kept"]) < 0.9 * sum(st["total"])
    _strict(G, Go, f"{ham} chain tau {tau}")


@pytest.mark.parametrize("ham", ["DC", "DCG"])
def test_uneven_depth_cluster_strict(q, ctx, ham):
    # contraction depth 1..6 per function: integral tiles of uneven primitive counts
    if ham == "DC":
        s = wl.cluster(seed=35, n_atoms=7, nl_per_atom=3, ns_per_atom=4, n=5, radius=6.0,
                       min_sep=1.5, tau=1e-9, ham="DC", coefs="qr")
    else:
        s = wl.cluster(seed=41, n_atoms=5, nl_per_atom=2, ns_per_atom=3, n=3, radius=5.0,
                       min_sep=1.5, tau=1e-10, ham="DCG", coefs="qr")
    Go, so = oracle.transform_direct(s.L, s.S, s.CL, s.CS, ham, s.tau)
    for flags in (0, q.PLAN_SCHWARZ_ROWS):  # primitive bands (default) and Schwarz rows
        G, st = _run(q, ctx, s, flags=flags)
        _same_counts(st, so)
        _strict(G, Go, f"{ham} cluster flags {flags}")


@pytest.mark.parametrize("ham,tau", [("DC", 0.0), ("DC", 1e-8), ("DCG", 1e-9)])
def test_unique_and_directed_tiles_strict(q, ctx, ham, tau):
    s = _chain(43, n_atoms=7, spacing=3.2, nl=3, ns=4, n=5, tau=tau, ham=ham)
    Go, so = oracle.transform_direct(s.L, s.S, s.CL, s.CS, ham, tau)
    Gu, stu = _run(q, ctx, s)
    Gd, std = _run(q, ctx, s, flags=q.PLAN_DIRECTED_TILES)
    assert stu["tiles_made"] < std["tiles_made"]
    for G, st, what in ((Gu, stu, "unique"), (Gd, std, "directed")):
        _same_counts(st, so)
        _strict(G, Go, f"{ham} {what} tiles tau {tau}")


@pytest.mark.parametrize("budget_mb,flags", [(40, 0), (24, 0), (24, 1)])
def test_chunks_and_batches_strict(q, budget_mb, flags):
    s = _chain(42, n_atoms=6, spacing=3.0, nl=3, ns=5, n=16, tau=1e-10, ham="DCG")
    small = q.Context(0, budget_bytes=budget_mb << 20)
    G, st = _run(q, small, s, flags=flags)
    print(f"budget {budget_mb} MB flags {flags}: chunks {st['n_chunks']}, "
          f"launches {st['n_batches']}")
    assert st["n_chunks"] > 1
    Go, so = oracle.transform_direct(s.L, s.S, s.CL, s.CS, "DCG", s.tau)
    _same_counts(st, so)
    _strict(G, Go, f"DCG {budget_mb} MB")
    small.close()


COMBOS = [(e, f, t) for e in (0, 1) for f in (0, 1) for t in (64, 128)]


@pytest.mark.parametrize("name", ["DC", "DCG", "DC34"])
def test_every_launch_choice_strict(q, ctx, name):
    if name == "DC":
        s = wl.cluster(seed=35, n_atoms=7, nl_per_atom=3, ns_per_atom=4, n=6, radius=6.0,
                       min_sep=1.5, tau=1e-9, ham="DC", coefs="qr")
    elif name == "DCG":
        s = wl.cluster(seed=41, n_atoms=5, nl_per_atom=2, ns_per_atom=3, n=4, radius=5.0,
                       min_sep=1.5, tau=1e-10, ham="DCG", coefs="qr")
    else:  # 4n = 136: ragged 128-wide second-quarter tiles in both dimensions
        s = _chain(44, n_atoms=4, spacing=3.0, nl=3, ns=6, n=34, tau=1e-10)
    Go, so = oracle.transform_direct(s.L, s.S, s.CL, s.CS, s.ham, s.tau)
    for e, f, t in COMBOS:
        tune = {"eri_sched": e, "fh_order": f, "sq_tile": t}
        G, st = _run(q, ctx, s, tune=tune)
        _same_counts(st, so)
        _strict(G, Go, f"{name} {tune}")


@pytest.mark.parametrize("tau", [0.0, 1e-9])
def test_dcb_all_classes_strict(q, ctx, tau):
    s = _chain(61, n_atoms=5, n=4, tau=tau, ham="DCB")
    L, S = _bases(q, ctx, s)
    plan = q.Plan(ctx, L, S, "DCB", s.n_mo, tau)
    G, st = plan.transform(s.CL, s.CS)
    Go, so = oracle.transform_direct(s.L, s.S, s.CL, s.CS, "DCB", tau)
    _same_counts(st, so)
    _strict(G, Go, f"DCB tau {tau}")
    # each class alone (FP64 plans fuse Gaunt and gauge tiles; a single class
    # runs its own kernels), and the Breit pair
    ref = {}
    for cls, ham in (("coulomb", "DC"), ("gaunt", "GAUNT"), ("gauge", "GAUGE")):
        Gc, stc = plan.transform(s.CL, s.CS, classes=cls)
        Gco, sco = oracle.transform_direct(s.L, s.S, s.CL, s.CS, ham, tau)
        _same_counts(stc, sco)
        _strict(Gc, Gco, f"DCB class {cls} tau {tau}")
        ref[cls] = Gco
    Gb, _ = plan.transform(s.CL, s.CS, classes="breit")
    _strict(Gb, ref["gaunt"] + ref["gauge"], f"DCB Breit classes tau {tau}")
    plan.close()


@pytest.mark.parametrize("budget_mb,flags", [(0, 1), (24, 0)])
def test_dcb_directed_tiles_batches_and_chunks_strict(q, budget_mb, flags):
    s = _chain(63, n_atoms=6, ns=5, n=12, tau=1e-10, ham="DCB")
    c = q.Context(0, budget_bytes=budget_mb << 20)
    G, st = _run(q, c, s, flags=flags)
    if budget_mb:
        assert st["n_chunks"] > 1
    Go, so = oracle.transform_direct(s.L, s.S, s.CL, s.CS, "DCB", s.tau)
    _same_counts(st, so)
    _strict(G, Go, f"DCB {budget_mb} MB flags {flags}")
    c.close()


def test_dcb_schedules_and_mixed_fp64_tier_strict(q, ctx):
    s = _chain(64, n_atoms=6, n=6, tau=1e-10, ham="DCB")
    Go, so = oracle.transform_direct(s.L, s.S, s.CL, s.CS, "DCB", s.tau)
    for e in (0, 1):
        G, st = _run(q, ctx, s, tune={"eri_sched": e, "fh_order": 1 - e, "sq_tile": 64})
        _same_counts(st, so)
        _strict(G, Go, f"DCB eri_sched {e}")
    L, S = _bases(q, ctx, s)
    pm = q.Plan(ctx, L, S, "DCB", s.n_mo, s.tau, prec="mixed", tier_fp32=0.0, tier_bf16=0.0)
    Gm, stm = pm.transform(s.CL, s.CS)
    _same_counts(stm, so)
    _strict(Gm, Go, "DCB mixed plan, every tile FP64")


SPINOR_CASES = [("LL", 5, 0.0), ("LL", 6, 1e-9), ("DC", 7, 0.0), ("DC", 8, 1e-10),
                ("DCG", 5, 0.0), ("DCG", 6, 1e-9), ("DCB", 7, 1e-9)]


@pytest.mark.parametrize("ham,m,tau", SPINOR_CASES)
def test_spinor_plans_strict(q, ctx, ham, m, tau):
    if ham == "LL":
        s = wl.small_ll(seed=51, n_atoms=5, nfunc=15, n=4, edge=8.0, coefs="qr")
    else:
        s = _chain(52 if ham != "DCB" else 65, n_atoms=5, n=4, tau=tau, ham=ham)
    PL, PS, _ = wl.general_spinors(s, m, seed=11)
    if ham == "LL":
        PS = None
    L, S = _bases(q, ctx, s)
    plan = q.Plan(ctx, L, S if ham != "LL" else None, ham, m, tau, flags=q.PLAN_SPINOR)
    G, st = plan.transform(PL, PS)
    Gc = G[..., 0] + 1j * G[..., 1]
    Go, so = oracle.transform_spinor(s.L, s.S if ham != "LL" else None, PL, PS, ham, tau)
    _same_counts(st, so)
    _strict(Gc, Go, f"spinor {ham} m {m} tau {tau}")
    plan.close()


@pytest.mark.parametrize("ham,batch,tau", [("DC", 3, 1e-8), ("DC", 7, 1e-10),
                                           ("DCG", 4, 1e-9), ("DCB", 4, 1e-9)])
def test_mo_driven_strict(q, ctx, ham, batch, tau):
    s = _chain(56 if ham != "DCB" else 66, n_atoms=6 if ham != "DCB" else 5, n=5, tau=tau,
               ham=ham)
    G, st = _run(q, ctx, s, mo_batch=batch)
    Go, so = oracle.transform_direct_mo(s.L, s.S, s.CL, s.CS, ham, tau, batch)
    assert st["kept"] == so["kept"] and st["kept_gaunt"] == so["kept_gaunt"]
    _strict(G, Go, f"MO-driven {ham} batch {batch} tau {tau}")


def test_device_pointers_and_blocks_strict(q, ctx):
    import torch
    s = _chain(38, n_atoms=5, nl=3, ns=4, n=7, tau=1e-10, ham="DCG")
    Go, so = oracle.transform_direct(s.L, s.S, s.CL, s.CS, "DCG", s.tau)
    L, S = _bases(q, ctx, s)
    plan = q.Plan(ctx, L, S, "DCG", s.n_mo, s.tau)
    dev = torch.device("cuda:0")
    Gd, std = plan.transform(torch.from_numpy(s.CL).to(dev), torch.from_numpy(s.CS).to(dev))
    torch.cuda.synchronize()
    _same_counts(std, so)
    _strict(Gd.cpu().numpy(), Go, "DCG device pointers")
    n = s.n_mo
    pairs = [(r, t) for r in range(n) for t in range(r, n)]
    Gb = np.full((n, n, n, n, 4, 4), np.nan)

    def take(i0, i1, B):
        for i in range(i0, i1):
            r, t = pairs[i]
            Gb[:, :, r, t] = B[i - i0, :, :, 0]
            Gb[:, :, t, r] = B[i - i0, :, :, 1]

    plan.transform_blocks(s.CL, s.CS, take)
    assert np.isfinite(Gb).all()
    _strict(Gb, Go, "DCG blocked output")
    plan.close()


def _qr_perturbed(s, k, eps=1e-2):
    # re-transform input k of a QR-coefficient system: QR+(C0 + eps G_k)
    C0 = np.concatenate([s.CL, s.CS], axis=1)
    g = np.random.default_rng(3000 + k).standard_normal(C0.shape)
    C = wl.quat_qr_plus(C0 + eps * g)
    NL = s.L.nfunc
    return np.ascontiguousarray(C[:, :NL]), np.ascontiguousarray(C[:, NL:])


@pytest.mark.parametrize("ham", ["DC", "DCG", "DCB"])
def test_graph_replays_strict(q, ham):
    import torch
    s = _chain(50, n_atoms=6, ns=5, n=8, tau=1e-10, ham=ham)
    c = q.Context(0)
    L, S = _bases(q, c, s)
    plan = q.Plan(c, L, S, ham, s.n_mo, s.tau)
    dev = torch.device("cuda:0")
    CL = torch.from_numpy(s.CL).to(dev)
    CS = torch.from_numpy(s.CS).to(dev)
    G = torch.empty(plan.g_shape(), dtype=torch.float64, device=dev)
    stream = torch.cuda.Stream()
    plan.capture(CL, CS, G, stream)
    for k in range(3):
        cl, cs = (s.CL, s.CS) if k == 0 else _qr_perturbed(s, k)
        CL.copy_(torch.from_numpy(cl))
        CS.copy_(torch.from_numpy(cs))
        torch.cuda.synchronize()
        st = plan.replay(stream)
        assert st["graph_replay"] and not st["graph_fallback"]
        Go, so = oracle.transform_direct(s.L, s.S, cl, cs, ham, s.tau)
        _same_counts(st, so)
        _strict(G.cpu().numpy(), Go, f"{ham} replay {k}")
    plan.close()
    c.close()


@pytest.mark.parametrize("case", ["DC", "DCG", "DCB", "mixed", "spinor"])
def test_intra_tile_row_order_on_and_off(q, ctx, case, monkeypatch):
    # the intra-tile row order (rows of each tile ranked by Q Dmax per
    # transform, masked 16-row steps skipped) against plans created with it
    # turned off: the same kept contributions, both at oracle parity, and no
    # more first-half MFMA work than without
    if case == "DCG":
        s = wl.cluster(seed=41, n_atoms=5, nl_per_atom=2, ns_per_atom=3, n=3, radius=5.0,
                       min_sep=1.5, tau=1e-10, ham="DCG", coefs="qr")
    elif case == "DCB":
        s = _chain(64, n_atoms=6, n=6, tau=1e-10, ham="DCB")
    else:
        s = _chain(34, n_atoms=8, spacing=4.0, nl=3, ns=6, n=6, tau=1e-10)
    L, S = _bases(q, ctx, s)
    kw = {}
    if case == "mixed":
        kw = dict(prec="mixed", tier_fp32=1e-3, tier_bf16=0.0)
    flags = q.PLAN_SPINOR if case == "spinor" else 0
    if case == "spinor":
        PL, PS, _ = wl.general_spinors(s, 7, seed=5)
        Go, so = oracle.transform_spinor(s.L, s.S, PL, PS, s.ham, s.tau)
        inputs, m = (PL, PS), 7
    else:
        Go, so = oracle.transform_direct(s.L, s.S, s.CL, s.CS, s.ham, s.tau)
        inputs, m = (s.CL, s.CS), s.n_mo
    res = {}
    for on in (True, False):
        if on:
            monkeypatch.delenv("QDCB_TILE_ORDER", raising=False)
        else:
            monkeypatch.setenv("QDCB_TILE_ORDER", "0")
        plan = q.Plan(ctx, L, S, s.ham, m, s.tau, flags=flags, **kw)
        G, st = plan.transform(*inputs)
        plan.close()
        if case == "spinor":
            G = G[..., 0] + 1j * G[..., 1]
        res[on] = (G, st)
    monkeypatch.delenv("QDCB_TILE_ORDER", raising=False)
    (G1, s1), (G0, s0) = res[True], res[False]
    assert s1["kept"] == s0["kept"] == so["kept"] and s1["kept_gaunt"] == s0["kept_gaunt"]
    assert s1["tiles_kept"] == s0["tiles_kept"]
    print(f"{case}: MFMA work with / without the order {s1['flops_mfma']:.4e} / "
          f"{s0['flops_mfma']:.4e}, fill {s1['flops_first_half'] / s1['flops_mfma']:.3f} / "
          f"{s0['flops_first_half'] / s0['flops_mfma']:.3f}")
    assert s1["flops_mfma"] <= s0["flops_mfma"]
    if case == "mixed":
        assert np.abs(G1 - G0).max() <= 1e-6 * np.abs(Go).max()
    else:
        _strict(G1, Go, f"{case} with the intra-tile order")
        _strict(G0, Go, f"{case} without")
