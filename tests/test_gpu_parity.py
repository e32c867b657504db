"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

Stage by stage (Schwarz factors, AO integrals, density bounds, kept
contribution counts) and end to end (the quaternion MO integrals G), on
seeded inputs that span several 64-pair tiles with a ragged last tile.

Tolerances.  Floating-point results are compared normwise,
max|G_gpu - G_oracle| <= 1e-12 * scale.  For well-conditioned coefficients
the scale is max|G|.  For Loewdin coefficients of a near-dependent basis the
MO integrals are small differences of large terms, and two exact-arithmetic
equivalent FP64 routes of the oracle itself already differ by ~3e-11 of
max|G| (see test_oracle_pins.test_definition_vs_direct_ll24); there the
scale is the Schwarz magnitude bound of the sums, (max_pq a_pq)^2 with
a_pq = sum |C_mp| Q_mn |C_nq|.  Integer outputs (kept counts) are exact.
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


def _gpu_transform(q, ctx, s, tau, C=None, flags=0):
    L = q.Basis(ctx, s.L)
    S = q.Basis(ctx, s.S) if s.S is not None else None
    CL = s.CL if C is None else C[0]
    CS = s.CS if C is None else C[1]
    plan = q.Plan(ctx, L, S, s.ham, CL.shape[2], tau, flags=flags)
    G, st = plan.transform(CL, CS)
    return G, st, plan, (L, S)


def _scale(s, CL, CS):
    Qs = [oracle.schwarz(s.L)]
    Cs = [CL]
    if s.S is not None:
        Qs.append(oracle.schwarz(s.S))
        Cs.append(CS)
    return qalg.schwarz_scale(Qs, Cs)


def _gaunt_scale(s):
    # Gaunt sums run over L-S products: |[D^K_pq]_x| <= |C^L_mp||C^S_nq| + |C^S_np||C^L_mq|,
    # three Pauli components K
    nL = np.sqrt((s.CL ** 2).sum(0))
    nS = np.sqrt((s.CS ** 2).sum(0))
    a = nL.T @ oracle.schwarz(s.L, s.S) @ nS
    return 3 * float(np.max(a + a.T)) ** 2


def test_schwarz_factors(q, ctx):
    for s in (wl.config("ll24"), wl.cluster(seed=31, n_atoms=5, nl_per_atom=3, ns_per_atom=2,
                                            n=2, radius=4.0, min_sep=1.0)):
        for B in (s.L,) + ((s.S,) if s.S is not None else ()):
            Qg = q.Basis(ctx, B).schwarz()
            Qo = oracle.schwarz(B)
            assert np.abs(Qg - Qo).max() <= 1e-14 * np.abs(Qo).max()
            assert np.all(np.abs(Qg - Qo) <= 1e-13 * Qo + 1e-300)


def test_eri_quartets(q, ctx):
    s = wl.cluster(seed=32, n_atoms=6, nl_per_atom=3, ns_per_atom=3, n=2, radius=5.0,
                   min_sep=1.0)
    A, B = q.Basis(ctx, s.L), q.Basis(ctx, s.S)
    rng = np.random.default_rng(0)
    idx = np.stack([rng.integers(0, s.L.nfunc, 300), rng.integers(0, s.L.nfunc, 300),
                    rng.integers(0, s.S.nfunc, 300), rng.integers(0, s.S.nfunc, 300)], 1)
    got = q.eri_quartets(A, B, idx)
    ref = np.array([oracle.eri(s.L, a, b, s.S, c, d) for a, b, c, d in idx])
    assert np.all(np.abs(got - ref) <= 1e-13 * np.abs(ref))


def test_density_bound_matches_oracle(q, ctx):
    s = wl.linear_chain(seed=33, n_atoms=4, nl_per_atom=3, ns_per_atom=5, n=5, tau=1e-10)
    G, st, plan, _ = _gpu_transform(q, ctx, s, s.tau)
    NL, NS = s.L.nfunc, s.S.nfunc
    P = NL * (NL + 1) // 2 + NS * (NS + 1) // 2
    dm = plan.fetch(q.FETCH_DMAX, P)
    ref = []
    for C, N in ((s.CL, NL), (s.CS, NS)):
        D = oracle.dmax_coulomb(C)
        ref += [D[mu, nu] for nu in range(N) for mu in range(nu + 1)]
    ref = np.array(ref)
    assert np.all(np.abs(dm - ref) <= 1e-14 * ref)


@pytest.mark.parametrize("tau", [0.0, 1e-12, 1e-6])
def test_transform_ll24(q, ctx, tau):
    s = wl.config("ll24")
    G, st, _, _ = _gpu_transform(q, ctx, s, tau)
    Go, sto = oracle.transform_direct(s.L, None, s.CL, None, "LL", tau)
    assert sto["tie_band"] == 0
    assert st["kept"] == sto["kept"]
    assert st["total"][0] == sto["total"][0]
    err = np.abs(G - Go).max()
    assert err <= 1e-12 * _scale(s, s.CL, None), (err, np.abs(Go).max())


def test_transform_ll24_well_conditioned_strict(q, ctx):
    s = wl.config("ll24")
    C = wl.quat_qr_plus(np.random.default_rng(5).standard_normal((4, 24, 12)))
    G, st, _, _ = _gpu_transform(q, ctx, s, 1e-12, C=(C, None))
    Go, sto = oracle.transform_direct(s.L, None, C, None, "LL", 1e-12)
    assert st["kept"] == sto["kept"]
    assert np.abs(G - Go).max() <= 1e-12 * np.abs(Go).max()


@pytest.mark.parametrize("tau", [0.0, 1e-10, 1e-5])
def test_transform_dc_chain(q, ctx, tau):
    # 8 atoms, 4 bohr apart: 24 L + 48 S functions, 1476 pairs = 23 tiles + 4 rows
    s = wl.linear_chain(seed=34, n_atoms=8, spacing=4.0, nl_per_atom=3, ns_per_atom=6, n=6,
                        tau=tau)
    G, st, _, _ = _gpu_transform(q, ctx, s, tau)
    Go, sto = oracle.transform_direct(s.L, s.S, s.CL, s.CS, "DC", tau)
    assert sto["tie_band"] == 0
    assert st["kept"] == sto["kept"]
    assert st["total"] == sto["total"]
    err = np.abs(G - Go).max()
    assert err <= 1e-12 * _scale(s, s.CL, s.CS), (err, np.abs(Go).max())
    if tau == 1e-5:
        assert sum(st["kept"]) < 0.9 * sum(st["total"])


def test_transform_mixed_contraction_depth_cluster(q, ctx):
    # contraction depth 1..6 per function (uneven tiles), odd n
    s = wl.cluster(seed=35, n_atoms=7, nl_per_atom=3, ns_per_atom=4, n=5, radius=6.0,
                   min_sep=1.5, tau=1e-9, ham="DC")
    G, st, _, _ = _gpu_transform(q, ctx, s, s.tau)
    Go, sto = oracle.transform_direct(s.L, s.S, s.CL, s.CS, "DC", s.tau)
    assert st["kept"] == sto["kept"]
    assert np.abs(G - Go).max() <= 1e-12 * _scale(s, s.CL, s.CS)


def test_degenerate_sizes(q, ctx):
    # one basis function, one MO
    s = wl.small_ll(seed=36, n_atoms=1, nfunc=1, n=1)
    G, st, _, _ = _gpu_transform(q, ctx, s, 0.0)
    Go, _ = oracle.transform_direct(s.L, None, s.CL, None, "LL", 0.0)
    assert np.abs(G - Go).max() <= 1e-14 * np.abs(Go).max()
    # threshold above every bound: nothing kept, G exactly zero
    s = wl.small_ll(seed=37, n_atoms=3, nfunc=9, n=3)
    G, st, _, _ = _gpu_transform(q, ctx, s, 1e30)
    assert sum(st["kept"]) == 0 and st["tiles_kept"] == 0
    assert not np.any(G)


def test_device_pointer_path_and_determinism(q, ctx):
    import torch
    s = wl.linear_chain(seed=38, n_atoms=5, spacing=3.0, nl_per_atom=3, ns_per_atom=4, n=7,
                        tau=1e-10)
    L, S = q.Basis(ctx, s.L), q.Basis(ctx, s.S)
    plan = q.Plan(ctx, L, S, "DC", 7, s.tau)
    Gh, st_h = plan.transform(s.CL, s.CS)
    CL = torch.from_numpy(s.CL).cuda()
    CS = torch.from_numpy(s.CS).cuda()
    Gd, st_d = plan.transform(CL, CS)
    torch.cuda.synchronize()
    Gd2, _ = plan.transform(CL, CS)
    torch.cuda.synchronize()
    assert np.array_equal(Gd.cpu().numpy(), Gh)
    assert torch.equal(Gd, Gd2)
    assert st_h["kept"] == st_d["kept"]


def test_invalid_arguments_fail_loudly(q, ctx):
    s = wl.small_ll(seed=39, n_atoms=2, nfunc=4, n=2)
    bad = wl.Basis(s.L.centers, s.L.nprim, -s.L.exps, s.L.coefs)
    with pytest.raises(q.QdcbError) as e:
        q.Basis(ctx, bad)
    assert e.value.status == -1
    L = q.Basis(ctx, s.L)
    with pytest.raises(q.QdcbError):
        q.Plan(ctx, L, None, "DC", 2, 0.0)  # DC needs an S basis
    plan = q.Plan(ctx, L, None, "LL", 2, 0.0)
    C = s.CL.copy()
    C[0, 0, 0] = np.nan
    with pytest.raises(q.QdcbError):
        plan.transform(C)


@pytest.mark.parametrize("tau", [0.0, 1e-9])
def test_transform_dcg_chain(q, ctx, tau):
    # Dirac-Coulomb + Gaunt: 18 L + 24 S functions, 756 ordered LS pairs (12 tiles)
    s = wl.linear_chain(seed=40, n_atoms=6, spacing=3.5, nl_per_atom=3, ns_per_atom=4, n=4,
                        tau=tau, ham="DCG")
    G, st, plan, _ = _gpu_transform(q, ctx, s, tau)
    Go, sto = oracle.transform_direct(s.L, s.S, s.CL, s.CS, "DCG", tau)
    assert sto["tie_band"] == 0
    assert st["kept"] == sto["kept"]
    assert st["kept_gaunt"] == sto["kept_gaunt"]
    assert st["total_gaunt"] == sto["total_gaunt"]
    scale = _scale(s, s.CL, s.CS) + _gaunt_scale(s)
    err = np.abs(G - Go).max()
    assert err <= 1e-12 * scale, (err, np.abs(Go).max())
    NL, NS = s.L.nfunc, s.S.nfunc
    dm = plan.fetch(q.FETCH_DMAX_GAUNT, NL * NS)
    ref = oracle.dmax_gaunt(s.CL, s.CS).reshape(-1)
    assert np.all(np.abs(dm - ref) <= 1e-14 * ref)


def test_dcg_cluster_mixed_depth(q, ctx):
    s = wl.cluster(seed=41, n_atoms=5, nl_per_atom=2, ns_per_atom=3, n=3, radius=5.0,
                   min_sep=1.5, tau=1e-10, ham="DCG")
    G, st, _, _ = _gpu_transform(q, ctx, s, s.tau)
    Go, sto = oracle.transform_direct(s.L, s.S, s.CL, s.CS, "DCG", s.tau)
    assert st["kept"] == sto["kept"] and st["kept_gaunt"] == sto["kept_gaunt"]
    scale = _scale(s, s.CL, s.CS) + _gaunt_scale(s)
    assert np.abs(G - Go).max() <= 1e-12 * scale


@pytest.mark.parametrize("budget_mb", [40, 24])
def test_column_chunks_and_panel_batches_are_exact(q, budget_mb):
    # A small device budget forces several MO-pair column chunks, narrow
    # second-half slices and (at 24 MB) several integral-panel batches whose
    # tiles are regenerated per chunk; every column is still accumulated in the
    # same order, so G is bitwise identical to the unconstrained run.  One
    # tile per directed task on both sides, so that the integral values are
    # the same bits.
    s = wl.linear_chain(seed=42, n_atoms=6, spacing=3.0, nl_per_atom=3, ns_per_atom=5, n=16,
                        tau=1e-10, ham="DCG")
    big = q.Context(0)
    f = q.PLAN_DIRECTED_TILES
    Gref, st_ref, _, _ = _gpu_transform(q, big, s, s.tau, flags=f)
    assert st_ref["n_chunks"] == 1
    small = q.Context(0, budget_bytes=budget_mb << 20)
    G, st, _, _ = _gpu_transform(q, small, s, s.tau, flags=f)
    print(f"budget {budget_mb} MB: chunks {st['n_chunks']}, launches {st['n_batches']}")
    assert st["n_chunks"] > 1
    assert st["kept"] == st_ref["kept"] and st["kept_gaunt"] == st_ref["kept_gaunt"]
    assert np.array_equal(G, Gref)


def test_unique_tiles_chunked_are_exact(q):
    # Unique tile pairs resident across several column chunks: the same tile
    # bits are read by every chunk, so G equals the one-chunk run bitwise.
    s = wl.linear_chain(seed=42, n_atoms=6, spacing=3.0, nl_per_atom=3, ns_per_atom=5, n=16,
                        tau=1e-10, ham="DCG")
    big = q.Context(0)
    Gref, st_ref, _, _ = _gpu_transform(q, big, s, s.tau)
    small = q.Context(0, budget_bytes=40 << 20)
    G, st, _, _ = _gpu_transform(q, small, s, s.tau)
    print(f"unique tiles: made {st['tiles_made']} of {st['tiles_kept']} directed, "
          f"chunks {st['n_chunks']}")
    assert st["n_chunks"] > 1
    assert st_ref["tiles_made"] < st_ref["tiles_kept"]
    assert st["tiles_made"] == st_ref["tiles_made"]
    assert np.array_equal(G, Gref)


@pytest.mark.parametrize("ham,tau", [("DC", 0.0), ("DC", 1e-8), ("DCG", 1e-9)])
def test_unique_tiles_match_directed_tiles_and_oracle(q, ctx, ham, tau):
    # One integral tile per unique pair (b >= k), read directly for (b, k) and
    # transposed for (k, b), against one tile per directed task: same kept
    # counts, G equal to rounding (the transposed integrals are summed over
    # primitives in the other order), both at oracle parity.
    s = wl.linear_chain(seed=43, n_atoms=7, spacing=3.2, nl_per_atom=3, ns_per_atom=4, n=5,
                        tau=tau, ham=ham)
    Gu, stu, _, _ = _gpu_transform(q, ctx, s, tau)
    Gd, std, _, _ = _gpu_transform(q, ctx, s, tau, flags=q.PLAN_DIRECTED_TILES)
    Go, sto = oracle.transform_direct(s.L, s.S, s.CL, s.CS, ham, tau)
    assert sto["tie_band"] == 0
    assert stu["kept"] == std["kept"] == sto["kept"]
    assert stu["kept_gaunt"] == std["kept_gaunt"] == sto["kept_gaunt"]
    assert stu["tiles_kept"] == std["tiles_kept"]
    assert std["tiles_made"] == std["tiles_kept"]
    assert stu["tiles_made"] < std["tiles_made"]
    scale = _scale(s, s.CL, s.CS) + (_gaunt_scale(s) if ham == "DCG" else 0.0)
    assert np.abs(Gu - Gd).max() <= 1e-13 * scale
    assert np.abs(Gu - Go).max() <= 1e-12 * scale
