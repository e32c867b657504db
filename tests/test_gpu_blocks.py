"""GPU tests of the class-selected and blocked outputs of the C ABI.

* QDCB_CLASS_COULOMB / QDCB_CLASS_GAUNT: each class alone against the oracle's
  Dirac-Coulomb and Gaunt-only transforms (parity tolerance, exact kept
  counts), and their sum equal to the DCG transform bitwise (the full
  transform adds the Gaunt part to the stored Coulomb part, one rounding).
* qdcb_transform_blocks: the blocks cover every MO pair (r <= s) once, in
  order, and reassemble G bitwise (both halves, G_pqrs and G_pqsr), on host and
  device pointers, also when the columns come in several chunks and slices.
* A block callback that stops the transformation, and a second call on the
  same plan from inside a callback (QDCB_E_BUSY); the plan stays usable.
"""
import ctypes

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


def _scale(s, gaunt=True):
    sc = qalg.schwarz_scale([oracle.schwarz(s.L), oracle.schwarz(s.S)], [s.CL, s.CS])
    if gaunt:
        nL = np.sqrt((s.CL ** 2).sum(0))
        nS = np.sqrt((s.CS ** 2).sum(0))
        a = nL.T @ oracle.schwarz(s.L, s.S) @ nS
        sc += 3 * float(np.max(a + a.T)) ** 2
    return sc


def _pairs(n):
    return [(r, t) for r in range(n) for t in range(r, n)]


def _assemble(n, blocks):
    G = np.full((n, n, n, n, 4, 4), np.nan)
    pairs = _pairs(n)
    nxt = 0
    for i0, i1, B in blocks:
        assert i0 == nxt and i1 > i0  # consecutive, each pair once
        nxt = i1
        for i in range(i0, i1):
            r, t = pairs[i]
            G[:, :, r, t] = B[i - i0, :, :, 0]
            G[:, :, t, r] = B[i - i0, :, :, 1]
    assert nxt == len(pairs)
    return G


def test_classes_alone_and_summed(q, ctx):
    s = wl.linear_chain(seed=48, n_atoms=6, spacing=3.1, nl_per_atom=3, ns_per_atom=4, n=5,
                        tau=1e-10, ham="DCG")
    L, S = q.Basis(ctx, s.L), q.Basis(ctx, s.S)
    plan = q.Plan(ctx, L, S, "DCG", s.n_mo, s.tau)
    G, st = plan.transform(s.CL, s.CS)
    Gc, stc = plan.transform(s.CL, s.CS, classes="coulomb")
    Gg, stg = plan.transform(s.CL, s.CS, classes="gaunt")
    assert st["classes"] == 3 and stc["classes"] == 1 and stg["classes"] == 2
    assert np.array_equal(Gc + Gg, G)
    Goc, soc = oracle.transform_direct(s.L, s.S, s.CL, s.CS, "DC", s.tau)
    Gog, sog = oracle.transform_direct(s.L, s.S, s.CL, s.CS, "GAUNT", s.tau)
    assert stc["kept"] == soc["kept"] and stc["kept_gaunt"] == 0
    assert stg["kept"] == [0, 0, 0, 0] and stg["kept_gaunt"] == sog["kept_gaunt"]
    assert st["kept"] == soc["kept"] and st["kept_gaunt"] == sog["kept_gaunt"]
    assert stc["flops_second_half"] + stg["flops_second_half"] == pytest.approx(
        st["flops_second_half"])
    sc = _scale(s)
    assert np.abs(Gc - Goc).max() <= 1e-12 * _scale(s, gaunt=False)
    assert np.abs(Gg - Gog).max() <= 1e-12 * sc
    # the Coulomb class of a DCG plan is the DC plan's transform
    pdc = q.Plan(ctx, L, S, "DC", s.n_mo, s.tau)
    Gdc, _ = pdc.transform(s.CL, s.CS)
    assert np.abs(Gdc - Gc).max() <= 1e-13 * _scale(s, gaunt=False)
    with pytest.raises(q.QdcbError):
        pdc.transform(s.CL, s.CS, classes="gaunt")  # no Gaunt class in a DC plan


@pytest.mark.parametrize("budget_mb,classes", [(0, None), (40, None), (40, "gaunt")])
def test_blocks_reassemble_g_host(q, budget_mb, classes):
    s = wl.linear_chain(seed=42, n_atoms=6, spacing=3.0, nl_per_atom=3, ns_per_atom=5, n=16,
                        tau=1e-10, ham="DCG")
    ctx = q.Context(0, budget_bytes=budget_mb << 20)
    L, S = q.Basis(ctx, s.L), q.Basis(ctx, s.S)
    plan = q.Plan(ctx, L, S, "DCG", s.n_mo, s.tau)
    G, st = plan.transform(s.CL, s.CS, classes=classes)
    blocks = []
    stb = plan.transform_blocks(s.CL, s.CS,
                                lambda i0, i1, B: blocks.append((i0, i1, B.copy())),
                                classes=classes)
    print(f"budget {budget_mb} MB: chunks {stb['n_chunks']}, blocks {len(blocks)}")
    if budget_mb:
        assert stb["n_chunks"] > 1 and len(blocks) > 1
    assert stb["kept"] == st["kept"] and stb["kept_gaunt"] == st["kept_gaunt"]
    Gb = _assemble(s.n_mo, blocks)
    assert np.array_equal(Gb, G)
    plan.close()
    ctx.close()


def _loaded_hip_runtime():
    # the HIP runtime this process already uses (torch's, shared by the
    # library), opened by its path so that no second copy is loaded
    with open("/proc/self/maps") as f:
        for line in f:
            if "libamdhip64" in line:
                return ctypes.CDLL(line.split()[-1])
    raise RuntimeError("no HIP runtime mapped")


def test_blocks_device_pointers(q, ctx):
    import torch
    hip = _loaded_hip_runtime()
    hip.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
    s = wl.linear_chain(seed=49, n_atoms=5, spacing=3.0, nl_per_atom=3, ns_per_atom=5, n=9,
                        tau=1e-10)
    L, S = q.Basis(ctx, s.L), q.Basis(ctx, s.S)
    plan = q.Plan(ctx, L, S, "DC", s.n_mo, s.tau)
    dev = torch.device("cuda:0")
    CL = torch.from_numpy(s.CL).to(dev)
    CS = torch.from_numpy(s.CS).to(dev)
    G, _ = plan.transform(CL, CS)
    n = s.n_mo
    blocks = []

    def take(i0, i1, ptr):
        assert ptr != 0
        B = torch.empty((i1 - i0, n, n, 2, 4, 4), dtype=torch.float64, device=dev)
        assert hip.hipMemcpy(B.data_ptr(), ptr, B.numel() * 8, 3) == 0  # device to device
        blocks.append((i0, i1, B.cpu().numpy()))

    plan.transform_blocks(CL, CS, take)
    torch.cuda.synchronize()
    assert np.array_equal(_assemble(n, blocks), G.cpu().numpy())


def test_block_callback_stop_and_busy_plan(q, ctx):
    s = wl.linear_chain(seed=42, n_atoms=6, spacing=3.0, nl_per_atom=3, ns_per_atom=5, n=16,
                        tau=1e-10)
    L, S = q.Basis(ctx, s.L), q.Basis(ctx, s.S)
    plan = q.Plan(ctx, L, S, "DC", s.n_mo, s.tau)
    seen, inner = [], []

    def cb(i0, i1, B):
        seen.append((i0, i1))
        try:
            plan.transform(s.CL, s.CS)  # same plan, inside its own call
        except q.QdcbError as e:
            inner.append(e.status)
        return True  # stop after the first block

    with pytest.raises(q.QdcbError) as ei:
        plan.transform_blocks(s.CL, s.CS, cb)
    assert ei.value.status == -6  # E_ABORTED
    assert len(seen) == 1 and inner == [-5]  # E_BUSY
    # the plan is free again and still exact
    G, st = plan.transform(s.CL, s.CS)
    Go, so = oracle.transform_direct(s.L, s.S, s.CL, s.CS, "DC", s.tau)
    assert st["kept"] == so["kept"]
    assert np.abs(G - Go).max() <= 1e-12 * _scale(s, gaunt=False)
    plan.close()
