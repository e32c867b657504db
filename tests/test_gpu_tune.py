"""GPU tests of the plan's launch choices and of the autotuner.

Every combination of integral schedule (list order / persistent longest-first
queue), first-half workgroup order (XCD-aware / plain) and second-quarter tile
(64 / 128) is compared with the FP64 oracle at the parity tolerance (see
test_gpu_parity.py for the Schwarz magnitude scale).  The schedule and the
order change no bit of G (each integral tile and each V block is computed by
the same arithmetic whichever workgroup runs it, in the same order); the
second-quarter tile changes only that GEMM's summation order.  Kept counts,
which the integral kernels count tile by tile, are exact, so a tile that a
schedule skipped or computed twice would show.
"""
import os

import numpy as np
import pytest

import oracle
from paper_2606_04316_amd import workloads as wl
from tests import qalg

pytestmark = pytest.mark.gpu

COMBOS = [(e, f, t) for e in (0, 1) for f in (0, 1) for t in (64, 128)]


@pytest.fixture(scope="module")
def q():
    from paper_2606_04316_amd import qdcb
    return qdcb


@pytest.fixture(scope="module")
def ctx(q):
    c = q.Context(0)
    yield c
    c.close()


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


SYSTEMS = {
    # contraction depth 1..6 per function: tiles of uneven primitive counts
    "DC": lambda: wl.cluster(seed=35, n_atoms=7, nl_per_atom=3, ns_per_atom=4, n=6, radius=6.0,
                             min_sep=1.5, tau=1e-9, ham="DC"),
    "DCG": lambda: wl.cluster(seed=41, n_atoms=5, nl_per_atom=2, ns_per_atom=3, n=4,
                              radius=5.0, min_sep=1.5, tau=1e-10, ham="DCG"),
    # 4n = 136 and n = 34: ragged 128-wide second-quarter tiles in both dimensions
    "DC34": lambda: wl.linear_chain(seed=44, n_atoms=4, spacing=3.0, nl_per_atom=3,
                                    ns_per_atom=6, n=34, tau=1e-10),
}


def _plan(q, ctx, s, tune):
    L = q.Basis(ctx, s.L)
    S = q.Basis(ctx, s.S) if s.S is not None else None
    plan = q.Plan(ctx, L, S, s.ham, s.n_mo, s.tau)
    if tune is not None:
        plan.tune = tune
    return plan, (L, S)


@pytest.mark.parametrize("name", ["DC", "DCG", "DC34"])
def test_every_launch_choice_matches_the_oracle(q, ctx, name):
    s = SYSTEMS[name]()
    Go, sto = oracle.transform_direct(s.L, s.S, s.CL, s.CS, s.ham, s.tau)
    scale = _scale(s)
    res = {}
    for e, f, t in COMBOS:
        tune = {"eri_sched": e, "fh_order": f, "sq_tile": t}
        plan, keep = _plan(q, ctx, s, tune)
        assert plan.tune == tune
        G, st = plan.transform(s.CL, s.CS)
        plan.close()
        assert st["kept"] == sto["kept"], (tune, st["kept"], sto["kept"])
        assert st["kept_gaunt"] == sto["kept_gaunt"]
        assert st["tiles_made"] < st["tiles_kept"]  # unique tiles (both directions from one)
        err = np.abs(G - Go).max()
        assert err <= 1e-12 * scale, (tune, err / scale)
        res[(e, f, t)] = G
    for t in (64, 128):
        for e in (0, 1):
            for f in (0, 1):
                assert np.array_equal(res[(e, f, t)], res[(0, 0, t)]), (e, f, t)
    d = np.abs(res[(0, 0, 64)] - res[(0, 0, 128)]).max()
    print(f"{name}: sq_tile 64 vs 128 max|dG| {d:.3e} (scale {scale:.3e})")
    assert d <= 1e-13 * scale


def test_persistent_schedule_with_nothing_kept(q, ctx):
    s = wl.linear_chain(seed=45, n_atoms=4, spacing=3.0, nl_per_atom=3, ns_per_atom=5, n=4,
                        tau=1e30)
    plan, keep = _plan(q, ctx, s, {"eri_sched": 1, "fh_order": 1, "sq_tile": 128})
    G, st = plan.transform(s.CL, s.CS)
    assert sum(st["kept"]) == 0 and st["tiles_kept"] == 0 and st["tiles_made"] == 0
    assert not np.any(G)


def test_invalid_choices_are_rejected(q, ctx):
    s = wl.linear_chain(seed=46, n_atoms=3, spacing=3.0, nl_per_atom=2, ns_per_atom=3, n=5,
                        tau=1e-10)
    plan, keep = _plan(q, ctx, s, None)
    assert plan.tune["sq_tile"] == 64  # odd n: the 128 tile needs two columns per lane
    for bad in ({"sq_tile": 128}, {"sq_tile": 96}, {"eri_sched": 2}, {"fh_order": -1}):
        with pytest.raises(q.QdcbError):
            plan.tune = bad
    assert plan.tune == {"eri_sched": 1, "fh_order": 0, "sq_tile": 64}


def test_replays_with_persistent_schedule_equal_eager(q):
    import torch
    s = wl.linear_chain(seed=50, n_atoms=6, spacing=3.0, nl_per_atom=3, ns_per_atom=5, n=16,
                        tau=1e-10, ham="DCG")
    ctx = q.Context(0)
    plan, keep = _plan(q, ctx, s, {"eri_sched": 1, "fh_order": 1, "sq_tile": 128})
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
        junk = torch.randn(1 << 20, device=dev).sum()
        Ge, ste = plan.transform(torch.from_numpy(cl).to(dev), torch.from_numpy(cs).to(dev))
        torch.cuda.synchronize()
        assert torch.isfinite(junk)
        assert st["kept"] == ste["kept"] and st["kept_gaunt"] == ste["kept_gaunt"]
        assert torch.equal(Gr, Ge), k
    plan.close()
    ctx.close()


def test_autotune_times_every_choice_and_caches(q, ctx, tmp_path, monkeypatch):
    s = wl.linear_chain(seed=47, n_atoms=6, spacing=3.0, nl_per_atom=3, ns_per_atom=5, n=16,
                        tau=1e-10, ham="DCG")
    path = str(tmp_path / "tune.jsonl")
    plan, keep = _plan(q, ctx, s, None)
    rep = plan.autotune(s.CL, s.CS, cache=path)
    print("autotune report:", rep)
    assert rep["from_cache"] == 0 and rep["trials"] == 4
    for k in ("ms_eri", "ms_first_half", "ms_second_half"):
        assert all(np.isfinite(v) and v > 0 for v in rep[k]), (k, rep[k])
    assert plan.tune == rep["chosen"]
    assert q.tune_cache_lookup(path, plan.tune_key()) == rep["chosen"]
    # the tuned plan still transforms exactly
    G, st = plan.transform(s.CL, s.CS)
    Go, sto = oracle.transform_direct(s.L, s.S, s.CL, s.CS, s.ham, s.tau)
    assert st["kept"] == sto["kept"] and st["kept_gaunt"] == sto["kept_gaunt"]
    assert np.abs(G - Go).max() <= 1e-12 * _scale(s)
    # a plan of the same shape takes the cached choice without timing anything
    plan2, keep2 = _plan(q, ctx, s, {"eri_sched": 1 - rep["chosen"]["eri_sched"]})
    assert plan2.tune_key() == plan.tune_key()
    rep2 = plan2.autotune(s.CL, s.CS, cache=path)
    assert rep2["from_cache"] == 1 and rep2["chosen"] == rep["chosen"]
    assert plan2.tune == rep["chosen"]
    # the cache path may come from the environment
    env_path = str(tmp_path / "env_tune.jsonl")
    monkeypatch.setenv("QDCB_TUNE_CACHE", env_path)
    plan3, keep3 = _plan(q, ctx, s, None)
    rep3 = plan3.autotune(s.CL, s.CS)
    assert rep3["from_cache"] == 0
    assert os.path.exists(env_path)
    assert q.tune_cache_lookup(env_path, plan3.tune_key()) == rep3["chosen"]


@pytest.mark.parametrize("ham", ["DC", "DCB"])
def test_primitive_band_row_order_matches_the_oracle(q, ctx, ham):
    # the default row order regroups the Schwarz-ordered rows by primitive
    # count within bands of 512 rows (QDCB_PLAN_SCHWARZ_ROWS keeps the plain
    # order): the tiles change, the kept contributions and the integrals do
    # not (exact kept counts, parity tolerance); both flags at once are refused
    s = wl.cluster(seed=69, n_atoms=9, nl_per_atom=3, ns_per_atom=4, n=5, radius=7.0,
                   min_sep=1.5, tau=1e-10, ham=ham)
    assert (s.L.nfunc * (s.L.nfunc + 1) + s.S.nfunc * (s.S.nfunc + 1)) // 2 > 2 * 512
    Go, sto = oracle.transform_direct(s.L, s.S, s.CL, s.CS, ham, s.tau)
    L, S = q.Basis(ctx, s.L), q.Basis(ctx, s.S)
    res = {}
    with pytest.raises(q.QdcbError):
        q.Plan(ctx, L, S, ham, s.n_mo, s.tau, flags=q.PLAN_SCHWARZ_ROWS | q.PLAN_PRIM_BANDS)
    for flags in (q.PLAN_SCHWARZ_ROWS, 0, q.PLAN_PRIM_BANDS):
        plan = q.Plan(ctx, L, S, ham, s.n_mo, s.tau, flags=flags)
        G, st = plan.transform(s.CL, s.CS)
        plan.close()
        assert st["kept"] == sto["kept"] and st["kept_gaunt"] == sto["kept_gaunt"], flags
        sc = qalg.schwarz_scale([oracle.schwarz(s.L), oracle.schwarz(s.S)], [s.CL, s.CS])
        if ham == "DCB":  # the L-S term's bound, with the gauge factor (1 + 3/2)^2
            nL, nS = np.sqrt((s.CL ** 2).sum(0)), np.sqrt((s.CS ** 2).sum(0))
            a = nL.T @ oracle.schwarz(s.L, s.S) @ nS
            sc += 3 * 6.25 * float(np.max(a + a.T)) ** 2
        assert np.abs(G - Go).max() <= 1e-12 * sc, flags
        res[flags] = (G, st)
    (G0, st0), (G1, st1) = res[q.PLAN_SCHWARZ_ROWS], res[0]
    assert np.array_equal(res[q.PLAN_PRIM_BANDS][0], G1)  # the default, named
    print(f"{ham}: kept tiles {st0['tiles_kept']} (Schwarz order) vs {st1['tiles_kept']} (bands)")
    assert st0["tiles_kept"] != st1["tiles_kept"]  # the row order did change the tiles
