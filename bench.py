"""Benchmark: quaternion Dirac-Coulomb AO->MO transformation on one MI355X.

Workload (the linear-chain benchmark system): 40 atoms 2.5 bohr apart,
N_L = 400 large-component and N_S = 800 small-component stand-in s
functions (3 primitives each), n = 64 quaternion MOs, Dirac-Coulomb classes
LL|LL + LL|SS + SS|LL + SS|SS, Schwarz threshold 1e-10, FP64.

One step = one full transformation (densities, screening, integral tiles,
first half, second half, output G in HBM) with inputs already resident on the
GPU.  value = quaternion MO integrals (pq|rs) per second, n^4 per step.

The JSON line also carries
  roofline      for the dominant kernel (the first-half FP64 MFMA contraction):
                algorithmic flops 2 * ncol * kept contributions over its
                average launch duration (HIP events on the transform's
                stream), against the FP64 MFMA peak; traffic from the
                committed rocprofv3 counter summary when it matches.
  cpu_baseline  the FP64 oracle on a seeded sample of bra pairs (first half
                only), scaled to the whole transformation.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64_MFMA = 78.6  # TFLOP/s, MI355X dense FP64 matrix
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "first_half_chain40_traffic.json")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="chain40", choices=["chain40", "ll24"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-rows", type=int, default=32)
    return ap.parse_args()


def cpu_baseline(sysm, n_rows, n):
    import numpy as np
    import oracle
    P = oracle.num_bra_pairs(sysm.L, sysm.S, sysm.ham)
    rows = np.sort(np.random.default_rng(0).choice(P, size=min(n_rows, P), replace=False))
    _, st = oracle.transform_direct(sysm.L, sysm.S, sysm.CL, sysm.CS, sysm.ham, sysm.tau,
                                    rows=rows, second_half=False)
    t_sample = st["seconds_first_half"]
    t_full = t_sample * P / len(rows)
    return {"value": n ** 4 / t_full, "unit": "quaternion MO integrals (pq|rs)/s",
            "cores": st["threads"], "kind": "oracle",
            "sample": (f"oracle first half (screened ERIs + density contraction, all "
                       f"{4 * n * n} spinor-pair columns) for {len(rows)} of {P} bra pairs "
                       f"drawn with seed 0, {t_sample:.2f} s, scaled by {P}/{len(rows)} to "
                       f"the whole transform; density set-up and the second half "
                       f"(a few percent in the paper) not included")}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    import numpy as np
    import torch
    from paper_2606_04316_amd import qdcb, workloads as wl

    sysm = wl.config(args.workload)
    n = sysm.n_mo
    dev = torch.device("cuda:0")
    ctx = qdcb.Context(0)
    L = qdcb.Basis(ctx, sysm.L)
    S = qdcb.Basis(ctx, sysm.S) if sysm.S is not None else None
    plan = qdcb.Plan(ctx, L, S, sysm.ham, n, sysm.tau)
    CL = torch.from_numpy(sysm.CL).to(dev)
    CS = torch.from_numpy(sysm.CS).to(dev) if sysm.CS is not None else None
    G = torch.empty((n, n, n, n, 4, 4), dtype=torch.float64, device=dev)
    for i in range(args.warmup):
        plan.transform(CL, CS, G)
        print(f"warmup {i + 1}/{args.warmup} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    stats = []
    t0 = time.perf_counter()
    for i in range(args.steps):
        _, st = plan.transform(CL, CS, G)
        stats.append(st)
        print(f"step {i + 1}/{args.steps}: {st['ms_total']:.1f} ms", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms = 1e3 * elapsed / args.steps
    value = n ** 4 * args.steps / elapsed

    fh_ms = sum(s["ms_first_half"] for s in stats)
    fh_launch = sum(s["n_batches"] for s in stats)
    fh_flops = sum(s["flops_first_half"] for s in stats)
    achieved = fh_flops / (fh_ms * 1e-3) / 1e12
    traffic = None
    if os.path.exists(TRAFFIC_FILE):
        with open(TRAFFIC_FILE) as f:
            tr = json.load(f)
        if tr.get("workload") == args.workload and tr.get("kernel_rev") == qdcb_kernel_rev():
            traffic = tr.get("bytes_per_launch")
    st0 = stats[-1]
    line = {
        "metric": "MO integrals/s (quaternion (pq|rs), FP64)",
        "value": value,
        "unit": "quaternion MO integrals (pq|rs)/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": sysm.name, "n_atoms": int(sysm.atoms.shape[0]),
                   "N_L": sysm.L.nfunc, "N_S": sysm.S.nfunc if sysm.S is not None else 0,
                   "n_mo": n, "ham": sysm.ham, "tau": sysm.tau},
        "spinor_integrals_per_s": (2 * n) ** 4 * args.steps / elapsed,
        "stages_ms": {k: st0[k] for k in ("ms_density", "ms_screen", "ms_eri", "ms_first_half",
                                          "ms_second_half", "ms_total")},
        "kept_fraction": sum(st0["kept"]) / max(1, sum(st0["total"])),
        "tile_fill": st0["flops_first_half"] / max(1.0, st0["flops_mfma"]),
        "roofline": {"kernel": "k_first_half", "bound": "mfma", "achieved": achieved,
                     "peak": PEAK_FP64_MFMA, "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_MFMA,
                     "traffic": traffic, "launches": fh_launch,
                     "avg_launch_ms": fh_ms / max(1, fh_launch)},
    }
    if not args.no_cpu_baseline:
        print("cpu baseline: oracle sample ...", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline(sysm, args.cpu_rows, n)
    print(json.dumps(line), flush=True)


def qdcb_kernel_rev():
    """Hash of the first-half kernel source, to tell whether committed
    counter data still describes the kernel being timed."""
    import hashlib
    p = os.path.join(ROOT, "paper_2606_04316_amd", "csrc", "k_gemm.hip")
    return hashlib.sha1(open(p, "rb").read()).hexdigest()[:12]


if __name__ == "__main__":
    main()
