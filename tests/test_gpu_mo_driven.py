"""GPU parity of the MO-driven variant (qdcb_plan_set_mo_batch) against the
oracle's MO-driven route: each batch of MO pairs is screened with the density
bound of its own pairs, so the kept contributions (exact counts, summed over
the batches) and G (parity tolerance of test_gpu_parity.py) follow the
oracle's batches.  At tau = 0 every batch keeps everything and the variant
equals the AO-driven transformation to rounding (same tiles and products;
each batch orders a tile's rows by its own bound).
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


def _scale(s):
    sc = qalg.schwarz_scale([oracle.schwarz(s.L), oracle.schwarz(s.S)], [s.CL, s.CS])
    if s.ham == "DCG":
        nL = np.sqrt((s.CL ** 2).sum(0))
        nS = np.sqrt((s.CS ** 2).sum(0))
        a = nL.T @ oracle.schwarz(s.L, s.S) @ nS
        sc += 3 * float(np.max(a + a.T)) ** 2
    return sc


@pytest.mark.parametrize("ham,batch,tau", [("DC", 3, 1e-8), ("DC", 7, 1e-10), ("DCG", 4, 1e-9)])
def test_mo_driven_matches_oracle(q, ctx, ham, batch, tau):
    s = wl.linear_chain(seed=56, n_atoms=6, spacing=3.0, nl_per_atom=3, ns_per_atom=4, n=5,
                        tau=tau, ham=ham)
    L, S = q.Basis(ctx, s.L), q.Basis(ctx, s.S)
    plan = q.Plan(ctx, L, S, ham, s.n_mo, tau)
    plan.set_mo_batch(batch)
    G, st = plan.transform(s.CL, s.CS)
    Go, so = oracle.transform_direct_mo(s.L, s.S, s.CL, s.CS, ham, tau, batch)
    assert st["kept"] == so["kept"] and st["kept_gaunt"] == so["kept_gaunt"]
    Ga, sa = q.Plan(ctx, L, S, ham, s.n_mo, tau).transform(s.CL, s.CS)
    scale = _scale(s)
    err = np.abs(G - Go).max()
    print(f"{ham} batch {batch} tau {tau}: max|dG| {err:.3e} (scale {scale:.3e}); kept "
          f"{sum(st['kept']) + st['kept_gaunt']} over the batches vs "
          f"{sum(sa['kept']) + sa['kept_gaunt']} AO-driven; max|G_mo - G_ao| "
          f"{np.abs(G - Ga).max():.3e}")
    assert err <= 1e-12 * scale


def test_mo_driven_at_zero_threshold_is_the_ao_transform(q, ctx):
    # at tau = 0 every batch keeps every contribution: the same integrals and
    # products as the AO-driven transform, summed in another order within a
    # tile (each batch ranks a tile's rows by its own bound), so equal to
    # rounding (well-conditioned coefficients: relative to max|G|)
    s = wl.linear_chain(seed=57, n_atoms=5, spacing=3.0, nl_per_atom=3, ns_per_atom=4, n=6,
                        tau=0.0, ham="DCG", coefs="qr")
    L, S = q.Basis(ctx, s.L), q.Basis(ctx, s.S)
    Ga, sa = q.Plan(ctx, L, S, "DCG", s.n_mo, 0.0).transform(s.CL, s.CS)
    plan = q.Plan(ctx, L, S, "DCG", s.n_mo, 0.0)
    plan.set_mo_batch(5)
    G, st = plan.transform(s.CL, s.CS)
    assert st["n_chunks"] > 1
    assert np.abs(G - Ga).max() <= 1e-13 * np.abs(Ga).max()
    # not offered: captures of the variant, spinor plans
    import torch
    dev = torch.device("cuda:0")
    CL, CS = torch.from_numpy(s.CL).to(dev), torch.from_numpy(s.CS).to(dev)
    Gd = torch.empty(plan.g_shape(), dtype=torch.float64, device=dev)
    with pytest.raises(q.QdcbError):
        plan.capture(CL, CS, Gd, torch.cuda.Stream())
    sp = q.Plan(ctx, L, S, "DCG", 4, 0.0, flags=q.PLAN_SPINOR)
    with pytest.raises(q.QdcbError):
        sp.set_mo_batch(2)
