"""GPU tests of the device allocator's cache: a destroyed plan's blocks go to
a per-device cache (after the plan's own stream events), and later plans take
them.  Plans created into reused blocks must give results bitwise equal to a
plan on fresh memory, whichever streams the plans ran on."""
import numpy as np
import pytest

from paper_2606_04316_amd import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def q():
    from paper_2606_04316_amd import qdcb
    return qdcb


def test_plans_in_reused_blocks_equal_fresh(q):
    import torch
    s = wl.linear_chain(seed=70, n_atoms=6, spacing=3.0, nl_per_atom=3, ns_per_atom=5, n=12,
                        tau=1e-10, ham="DCG")
    ctx = q.Context(0)
    L, S = q.Basis(ctx, s.L), q.Basis(ctx, s.S)
    ref = q.Plan(ctx, L, S, "DCG", s.n_mo, s.tau)
    Gref, _ = ref.transform(s.CL, s.CS)
    ref.close()
    dev = torch.device("cuda:0")
    CL = torch.from_numpy(s.CL).to(dev)
    CS = torch.from_numpy(s.CS).to(dev)
    n = s.n_mo
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    for k in range(6):
        st = streams[k % 2]
        plan = q.Plan(ctx, L, S, "DCG", n, s.tau)
        G = torch.empty((n, n, n, n, 4, 4), dtype=torch.float64, device=dev)
        plan.transform(CL, CS, G, stream=st.cuda_stream)
        # destroy first: the plan waits for its own work, then caches its blocks
        plan.close()
        # other device work, then a new plan of another size that takes blocks
        junk = torch.randn(1 << 20, device=dev).sum()
        other = q.Plan(ctx, L, S, "DC", n - 3, s.tau)
        Go, _ = other.transform(CL[:, :, :n - 3].contiguous(), CS[:, :, :n - 3].contiguous())
        other.close()
        st.synchronize()
        assert torch.isfinite(junk)
        assert np.array_equal(G.cpu().numpy(), Gref), k
    ctx.close()
