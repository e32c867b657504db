"""GPU tests of captured re-transforms (hipGraph replay) and of the request
loop (continuous batching): every replay equals the eager transform of the
same coefficients, and every served request equals the same request run
alone."""
import numpy as np
import pytest

from paper_2606_04316_amd import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def q():
    from paper_2606_04316_amd import qdcb
    return qdcb


@pytest.mark.parametrize("ham,budget_mb", [("DC", 0), ("DCG", 0), ("DCG", 24)])
def test_graph_replays_equal_eager(q, ham, budget_mb):
    import torch
    s = wl.linear_chain(seed=50, n_atoms=6, spacing=3.0, nl_per_atom=3, ns_per_atom=5, n=16,
                        tau=1e-10, ham=ham)
    ctx = q.Context(0, budget_bytes=budget_mb << 20)
    L, S = q.Basis(ctx, s.L), q.Basis(ctx, s.S)
    plan = q.Plan(ctx, L, S, ham, s.n_mo, s.tau)
    dev = torch.device("cuda:0")
    CL = torch.from_numpy(s.CL).to(dev)
    CS = torch.from_numpy(s.CS).to(dev)
    n = s.n_mo
    G = torch.empty((n, n, n, n, 4, 4), dtype=torch.float64, device=dev)
    stream = torch.cuda.Stream()
    plan.capture(CL, CS, G, stream)
    fallbacks = 0
    for k in range(4):
        cl, cs = (s.CL, s.CS) if k == 0 else wl.perturbed_coefficients(s, k)
        CL.copy_(torch.from_numpy(cl))
        CS.copy_(torch.from_numpy(cs))
        torch.cuda.synchronize()
        st = plan.replay(stream)
        fallbacks += st["graph_fallback"]
        assert st["graph_replay"] or st["graph_fallback"]
        Gr = G.clone()
        # eager transform of the same coefficients, with other device work around it
        junk = torch.randn(1 << 20, device=dev).sum()
        Ge, ste = plan.transform(torch.from_numpy(cl).to(dev), torch.from_numpy(cs).to(dev))
        torch.cuda.synchronize()
        assert torch.isfinite(junk)
        assert st["kept"] == ste["kept"] and st["kept_gaunt"] == ste["kept_gaunt"]
        assert torch.equal(Gr, Ge), (ham, budget_mb, k)
    if budget_mb:
        print(f"fallbacks at {budget_mb} MB: {fallbacks}")


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_served_requests_equal_alone(q, prec):
    from paper_2606_04316_amd import serving
    # arrivals 1 ms apart on average, far below a request's service time
    # (plan creation alone takes milliseconds), so requests must overlap
    reqs = serving.request_stream(12, seed=7, mean_gap_s=0.001, pool=4, atoms=(3, 6),
                                  nl=(6, 24), n_mo=(2, 6), radius_scale=8.0)
    # mixed: every tile in a reduced tier (FP32, BF16 below 1e-3), so that the
    # reduced-precision kernels run in the mix
    tiers = (1e300, 1e-3, 0)
    ex = serving.GpuExecutor(slots=3, prec=prec, tiers=tiers, keep_outputs=True)
    srv = serving.Server(ex, ex.reserve, slots=3, budget_bytes=8 << 30)
    out = srv.run(reqs)
    ex.drain()
    assert all(r.error is None for r in out), [r.error for r in out if r.error]
    summ = serving.summarize(out)
    assert summ["failed"] == 0 and summ["p99_ms"] >= summ["p50_ms"] > 0
    # continuous batching, not a queue: requests were admitted while others
    # ran, and their admission-to-result intervals overlap in time
    assert srv.max_concurrency > 1, srv.max_concurrency
    iv = sorted((r.t_admit, r.t_done) for r in out)
    overlaps = sum(1 for a, b in zip(iv, iv[1:]) if b[0] < a[1])
    print(f"max concurrency {srv.max_concurrency}, overlapping neighbours {overlaps}")
    assert overlaps > 0
    # the same requests one at a time, nothing else on the device: bitwise
    # equal G (same digest); a difference is reported with its size and the
    # two runs' launch statistics before the assertion fails
    alone_ex = serving.GpuExecutor(slots=1, prec=prec, tiers=tiers, keep_outputs=True)
    diffs = []
    for r in out[:8]:
        solo = serving.Request(rid=r.rid, system=r.system, arrival=0.0)
        solo.reserve = alone_ex.reserve(solo)
        res = alone_ex(solo, 0)
        if res["digest"] != r.result["digest"]:
            Ga, Gm = res["G"], r.result["G"]
            rel = float((Ga - Gm).abs().max() / Gm.abs().max())
            diffs.append((r.rid, rel, res["path"], r.result["path"]))
    alone_ex.drain()
    for d in diffs:
        print(f"request {d[0]}: max|G_alone - G_mix| / max|G| = {d[1]:.3e}, "
              f"alone {d[2]}, mix {d[3]}", flush=True)
    assert not diffs, [d[0] for d in diffs]
