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
  mfma_util     the first half's algorithmic FP64 flop rate over the MFMA peak.
  cluster       the compact-cluster configuration (60 atoms, N_L 600, N_S 1200,
                contraction depths 1..6, n 128, Dirac-Coulomb + Gaunt): FP64
                transforms with their own roofline, and the mixed-precision
                transform of the same inputs at the specified tiers (1e-4 /
                1e-7, screening bound) and at tiers that meet 1e-10 Eh
                (3e-6 / 1e-9, bound including the bra side): speedup, max
                |G_mixed - G_FP64 GPU| and the occupied Coulomb sum change.
  serving       the request stream (256 requests, 20 ms mean gap), p50/p99,
                with the size ranges it draws from.
The cluster and serving legs are skipped with --no-legs (profiling runs).
The headline value is the chain's: one cluster transform takes about 33 s,
so the 25 transforms of the default warm-up and timed steps do not fit the
run's time; the cluster leg times two.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64_MFMA = 78.6  # TFLOP/s, MI355X dense FP64 matrix
HEADLINE_METRIC = ("MO integrals/s & MFMA util, mixed vs FP64 at <=1e-10 Eh err; "
                   "serving p99 ms")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--mode", default="transform",
                    choices=["transform", "replay", "serving", "mixed"],
                    help="transform: the headline line; replay: captured re-transforms; "
                         "serving: the request loop; mixed: FP64/FP32/BF16 tiers vs FP64")
    ap.add_argument("--tiers", default="1e-4:1e-7:screen,1e-4:1e-7:g,3e-6:1e-9:g,1e-6:1e-9:g",
                    help="mixed: comma-separated tier_fp32:tier_bf16:rule settings "
                         "(rule screen = screening bound, g = bound including the bra side)")
    ap.add_argument("--workload", default=None,
                    help="transform: chain40 (default), cluster60, ll24, or <name>_spinor "
                         "(2 n general two-spinor MOs), <name>_rkb (RKB small components, "
                         "n general two-spinors), <name>_rkbq (RKB small components, n / 2 "
                         "Kramers pairs through a quaternion plan); replay: cluster24 "
                         "(default), chain40_dcg, chain40")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-legs", action="store_true",
                    help="transform: skip the mixed-precision and serving legs of the line")
    ap.add_argument("--cpu-rows", type=int, default=96)
    ap.add_argument("--cluster-steps", type=int, default=2,
                    help="transform: timed FP64 transforms of the cluster leg")
    ap.add_argument("--requests", type=int, default=256)
    ap.add_argument("--serving-prec", default="fp64,mixed",
                    help="serving: precisions to serve the stream in, one run each "
                         "(mixed: tiers 1e-6 / 1e-9 with the G-bound rule)")
    ap.add_argument("--slots", type=int, default=4)
    ap.add_argument("--serving-sizes", default="reduced", choices=["reduced", "full"],
                    help="serving: request sizes (reduced: 10-40 atoms, N_L 40-160, n 8-32, "
                         "the default leg; full: the recipe's 10-80 atoms, N_L 100-800, "
                         "n 16-128, where one GPU is saturated and a short stream is "
                         "measured with --requests)")
    ap.add_argument("--schwarz-rows", action="store_true",
                    help="transform: plans with QDCB_PLAN_SCHWARZ_ROWS (plain Schwarz row "
                         "order instead of the default primitive bands)")
    ap.add_argument("--serving-rows", default="bands", choices=["bands", "schwarz"],
                    help="serving: row order of the request plans (bands: the library "
                         "default; schwarz: QDCB_PLAN_SCHWARZ_ROWS)")
    ap.add_argument("--mo-batch", type=int, default=0,
                    help="transform: run the MO-driven variant with batches of this many MO "
                         "pairs, each screened with its own density bound (0: AO-driven)")
    ap.add_argument("--tune", default="auto", choices=["auto", "default"],
                    help="transform / replay: pick the plan's launch choices with the "
                         "autotuner before the untimed warm-up (auto), or keep the defaults")
    ap.add_argument("--tune-cache", default=None,
                    help="tuning cache file (JSON lines) for --tune auto")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="before the transform, run one elementwise copy kernel of this many "
                         "MiB (read and write), the reference for HBM byte counters")
    return ap.parse_args()


def cpu_model():
    """The host CPU's model name (Linux), for the baseline's record."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


# The paper's own timings (all on CPUs, none on GPUs), quoted as context with
# their hardware; none is on this build's synthetic workloads.
PAPER_TIMINGS = {
    "source": "arXiv 2606.04316, Sec. 3.3",
    "Au6_DCB": {"system": "planar Au6, dyall-ae2z, 1278 basis functions, 48 MO spinors, DCB",
                "wall_time_h": 14.0,
                "hardware": "2048 CPU cores (16 nodes x 128 AMD EPYC 7742)",
                "spinor_MO_integrals_per_s_derived": 48 ** 4 / (14.0 * 3600)},
    "Pu3_stage_s": {"system": "Pu3 chain, dyall-v2z (846 basis functions), 16 orbitals per "
                              "atom, tau 1e-12",
                    "columns": ["DC-SSSS", "DC", "Gaunt", "gauge"],
                    "AO_integrals": [9.13, 21.89, 18.68, 253.4],
                    "density": [61.49, 31.1, 61.88, 60.67],
                    "first_half": [2969.0, 804.8, 9215.0, 9556.0],
                    "second_half": [24.85, 17.48, 35.22, 34.91],
                    "hardware": "CPU cluster nodes (Hyak / Bridges-2), core count not stated"},
}


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
            "cores": st["threads"], "cpu_model": cpu_model(), "kind": "oracle",
            "sample": (f"oracle first half (screened ERIs + density contraction, all "
                       f"{4 * n * n} spinor-pair columns) for {len(rows)} of {P} bra pairs "
                       f"drawn with seed 0, {t_sample:.2f} s, scaled by {P}/{len(rows)} to "
                       f"the whole transform; density set-up and the second half "
                       f"(a few percent in the paper) not included")}


def autotune(args, plan, CL, CS, G):
    """Run the autotuner (untimed, before the warm-up) unless --tune default."""
    if args.tune != "auto":
        return {"chosen": plan.tune, "autotuned": False}
    t0 = time.perf_counter()
    rep = plan.autotune(CL, CS, G, cache=args.tune_cache)
    rep["autotuned"] = True
    rep["wall_s"] = time.perf_counter() - t0
    print(f"autotune: {rep['chosen']} (ERI ms {rep['ms_eri']}, first half ms "
          f"{rep['ms_first_half']}, second half ms {rep['ms_second_half']}, "
          f"{rep['wall_s']:.1f} s)", file=sys.stderr, flush=True)
    return rep


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    if args.mode == "replay":
        return main_replay(args)
    if args.mode == "serving":
        return main_serving(args)
    if args.mode == "mixed":
        return main_mixed(args)
    return main_transform(args)


def shell_kinds(sysm):
    """The angular momenta present in the system's bases ("s", "s, p", "s, p, d", ...)."""
    codes = [c for B in (sysm.L, sysm.S) if B is not None and getattr(B, "cart", None) is not None
             for c in B.cart]
    if not codes:
        return "s"
    top = max(codes)
    return "s, p, d, f" if top >= 10 else "s, p, d" if top >= 4 else "s, p"


def main_transform(args):
    import numpy as np
    import torch
    from paper_2606_04316_amd import qdcb, workloads as wl

    args.workload = args.workload or "chain40"
    # "<name>_spinor": the same basis with 2 n general two-spinor MOs (the
    # system's Kramers pairs mixed by a seeded unitary), a QDCB_PLAN_SPINOR plan.
    # "<name>_rkb": the system's L basis with RKB small components (its
    # gradient basis as S) and n general two-spinors, a QDCB_PLAN_SPINOR plan
    # "<name>_rkbq": the same RKB small components in Kramers-restricted form,
    # n_mo / 2 quaternion MOs (the same number of spinors as "<name>_rkb")
    # through a quaternion plan
    rkb = args.workload.endswith("_rkb")
    rkbq = args.workload.endswith("_rkbq")
    spinor = args.workload.endswith("_spinor") or rkb
    base = args.workload[:-len("_spinor")] if args.workload.endswith("_spinor") else \
        args.workload[:-len("_rkb")] if rkb else \
        args.workload[:-len("_rkbq")] if rkbq else args.workload
    sysm = wl.config(base)
    n = sysm.n_mo if rkb else 2 * sysm.n_mo if spinor else \
        sysm.n_mo // 2 if rkbq else sysm.n_mo
    dev = torch.device("cuda:0")
    # output and inputs first: the context's default budget is a share of
    # what is free when it is created
    if rkb:
        # n orthonormal general two-spinors over the L and RKB S coefficients
        # (QR of a Gaussian quaternion matrix, its Kramers pairs mixed)
        NLr = sysm.L.nfunc
        Q = wl.quat_qr_plus(wl.gaussian_quat(np.random.default_rng(8000), 2 * NLr, n // 2))
        U = wl.random_unitary(np.random.default_rng(8001), n, n)
        PL = wl.mix_spinors(wl.quat_to_spinor_planes(np.ascontiguousarray(Q[:, :NLr])), U)
        PS = wl.mix_spinors(wl.quat_to_spinor_planes(np.ascontiguousarray(Q[:, NLr:])), U)
        G = torch.empty((n, n, n, n, 2), dtype=torch.float64, device=dev)
    elif spinor:
        PL, PS, _ = wl.general_spinors(sysm, n, seed=0)
        G = torch.empty((n, n, n, n, 2), dtype=torch.float64, device=dev)
    elif rkbq:
        # n quaternion-orthonormal MOs over the L and RKB S coefficients
        NLr = sysm.L.nfunc
        Q = wl.quat_qr_plus(wl.gaussian_quat(np.random.default_rng(8000), 2 * NLr, n))
        PL, PS = np.ascontiguousarray(Q[:, :NLr]), np.ascontiguousarray(Q[:, NLr:])
        G = torch.empty((n, n, n, n, 4, 4), dtype=torch.float64, device=dev)
    else:
        PL, PS = sysm.CL, sysm.CS
        G = torch.empty((n, n, n, n, 4, 4), dtype=torch.float64, device=dev)
    CL = torch.from_numpy(PL).to(dev)
    CS = torch.from_numpy(PS).to(dev) if PS is not None else None
    ctx = qdcb.Context(0)
    L = qdcb.Basis(ctx, sysm.L)
    if rkb:
        S, norms = qdcb.rkb_basis(ctx, L)
        CS = torch.from_numpy(qdcb.rkb_small_planes(PS, norms, wl.SPEED_OF_LIGHT)).to(dev)
    elif rkbq:
        S, norms = qdcb.rkb_basis(ctx, L)
        CS = torch.from_numpy(qdcb.rkb_small_quat(PS, norms, wl.SPEED_OF_LIGHT)).to(dev)
    else:
        S = qdcb.Basis(ctx, sysm.S) if sysm.S is not None else None
    plan = qdcb.Plan(ctx, L, S, sysm.ham, n, sysm.tau,
                     flags=(qdcb.PLAN_SPINOR if spinor else 0) |
                     (qdcb.PLAN_SCHWARZ_ROWS if args.schwarz_rows else 0))
    if args.mo_batch:
        plan.set_mo_batch(args.mo_batch)
    if args.copy_calibration_mib:
        src = torch.ones(args.copy_calibration_mib << 17, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        torch.mul(src, 1.0, out=dst)
        torch.cuda.synchronize()
        print(f"copy calibration: {src.numel() * 8} bytes read and written", file=sys.stderr,
              flush=True)
        del src, dst
    tune = autotune(args, plan, CL, CS, G)
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
    traffic = committed_traffic(args.workload, plan.tune,
                                "Schwarz" if args.schwarz_rows else "primitive bands")
    st0 = stats[-1]
    kind = "complex spinor" if spinor else "quaternion"
    headline = (not spinor and not rkbq and not args.mo_batch and sysm.ham != "DCB"
                and getattr(sysm.L, "cart", None) is None)
    line = {
        "metric": HEADLINE_METRIC if headline else f"MO integrals/s ({kind} (pq|rs), FP64)",
        "value": value,
        "unit": f"{kind} MO integrals (pq|rs)/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": sysm.name + ("_rkb" if rkb else "_rkbq" if rkbq else
                                            "_spinor" if spinor else ""),
                   "n_atoms": int(sysm.atoms.shape[0]),
                   "N_L": sysm.L.nfunc,
                   "N_S": 3 * sysm.L.nfunc if rkb or rkbq else
                   sysm.S.nfunc if sysm.S is not None else 0,
                   "n_mo": n, "mo_kind": "general spinors" if spinor else "Kramers pairs",
                   "ham": sysm.ham, "tau": sysm.tau,
                   "algorithm": f"MO-driven, {args.mo_batch} MO pairs per batch"
                   if args.mo_batch else "AO-driven",
                   "row_order": "Schwarz" if args.schwarz_rows else "primitive bands",
                   "shells": shell_kinds(sysm),
                   "small_components": "RKB (gradient basis)" if rkb else
                   "RKB (gradient basis), Kramers-restricted" if rkbq else "stand-in basis"},
        "spinor_integrals_per_s": (n if spinor else 2 * n) ** 4 * args.steps / elapsed,
        "stages_ms": {k: st0[k] for k in ("ms_density", "ms_screen", "ms_eri", "ms_first_half",
                                          "ms_second_half", "ms_total")},
        "tune": tune,
        "kept_fraction": sum(st0["kept"]) / max(1, sum(st0["total"])),
        "tile_fill": st0["flops_first_half"] / max(1.0, st0["flops_mfma"]),
        "roofline": {"kernel": "k_first_half", "bound": "mfma", "achieved": achieved,
                     "peak": PEAK_FP64_MFMA, "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_MFMA,
                     "traffic": traffic, "launches": fh_launch,
                     "avg_launch_ms": fh_ms / max(1, fh_launch)},
    }
    line["mfma_util"] = {"first_half": achieved / PEAK_FP64_MFMA,
                         "basis": "algorithmic FP64 flops of k_first_half over its launch time, "
                                  "against the dense FP64 MFMA peak"}
    if headline and not args.no_legs:
        # the compact-cluster configuration (FP64 and mixed precision), after
        # this run's plan has released its memory
        plan.close()
        ctx.close()
        del G
        torch.cuda.empty_cache()
        line["cluster"] = cluster_leg(args)
        # the metric's mixed-precision part: the best mixed leg on the cluster
        # inputs that meets 1e-10 Eh (against the FP64 GPU transform)
        ok = [m for m in line["cluster"]["mixed_vs_fp64"] if m["meets_1e-10"]]
        best = max(ok, key=lambda m: m["speedup"]) if ok else None
        line["mixed_vs_fp64_at_1e-10_Eh"] = {
            "workload": line["cluster"]["workload"],
            "speedup": best["speedup"] if best else None,
            "tiers": [best["tier_fp32"], best["tier_bf16"], best["rule"]] if best else None,
            "max_abs_err_Eh": best["max_abs_err_vs_fp64_gpu_Eh"] if best else None}
    if not args.no_cpu_baseline and not spinor and not rkbq:
        print("cpu baseline: oracle sample ...", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline(sysm, args.cpu_rows, n)
    if headline and not args.no_legs:
        # the serving stream (FP64)
        line["serving"] = serving_run(args, "fp64")
    if headline:
        line["paper_timings"] = PAPER_TIMINGS
    print(json.dumps(line), flush=True)


def main_replay(args):
    """Re-transforms as captured-graph replays: the transformation is recorded
    once, then replayed for coefficients C_k (the system's orbitals perturbed
    by 1e-2 Gaussian noise, seed 3000 + k, re-orthonormalized) written into the
    same device buffers; eager transforms of C_0 and C_last are compared."""
    import torch
    from paper_2606_04316_amd import qdcb, workloads as wl

    name = args.workload or "cluster24"
    sysm = wl.config(name)
    print(f"workload {name} ready", file=sys.stderr, flush=True)
    n = sysm.n_mo
    dev = torch.device("cuda:0")
    CL = torch.from_numpy(sysm.CL).to(dev)
    CS = torch.from_numpy(sysm.CS).to(dev)
    G = torch.empty((n, n, n, n, 4, 4), dtype=torch.float64, device=dev)
    Geager_last = torch.empty_like(G)
    ctx = qdcb.Context(0)
    L, S = qdcb.Basis(ctx, sysm.L), qdcb.Basis(ctx, sysm.S)
    plan = qdcb.Plan(ctx, L, S, sysm.ham, n, sysm.tau)
    print("plan ready", file=sys.stderr, flush=True)
    tune = autotune(args, plan, CL, CS, G)
    stream = torch.cuda.Stream()
    nrep = max(1, args.steps)
    coefs = [(sysm.CL, sysm.CS)] + [wl.perturbed_coefficients(sysm, k) for k in range(1, nrep)]
    # eager reference timings
    eager_ms = []
    for cl, cs in (coefs[0], coefs[-1]):
        CL.copy_(torch.from_numpy(cl))
        CS.copy_(torch.from_numpy(cs))
        _, st = plan.transform(CL, CS, G)
        eager_ms.append(st["ms_total"])
        print(f"eager transform: {st['ms_total']:.1f} ms", file=sys.stderr, flush=True)
    Geager_last.copy_(G)
    plan.capture(CL, CS, G, stream)
    print("captured", file=sys.stderr, flush=True)
    rep_ms, fallbacks = [], 0
    t0 = time.perf_counter()
    for k, (cl, cs) in enumerate(coefs):
        CL.copy_(torch.from_numpy(cl))
        CS.copy_(torch.from_numpy(cs))
        torch.cuda.synchronize()
        st = plan.replay(stream)
        rep_ms.append(st["ms_total"])
        fallbacks += st["graph_fallback"]
        print(f"replay {k + 1}/{nrep}: {st['ms_total']:.1f} ms", file=sys.stderr, flush=True)
    wall = time.perf_counter() - t0
    same = bool(torch.equal(G, Geager_last))
    print(json.dumps({
        "metric": "re-transform time (captured-graph replays)", "mode": "replay",
        "value": sum(rep_ms) / len(rep_ms), "unit": "ms per re-transform",
        "higher_is_better": False, "replays": nrep, "fallbacks": fallbacks,
        "eager_ms": eager_ms, "replay_ms": rep_ms, "wall_s": wall,
        "last_replay_equals_eager": same, "tune": tune, "dtype": "f64", "data": "synthetic",
        "config": {"workload": sysm.name, "n_atoms": int(sysm.atoms.shape[0]),
                   "N_L": sysm.L.nfunc, "N_S": sysm.S.nfunc, "n_mo": n, "ham": sysm.ham,
                   "tau": sysm.tau}}), flush=True)


def main_mixed(args):
    """Mixed precision against the FP64 transform of the same inputs: for each
    tier setting, max |G_mixed - G_fp64|, the occupied-block Coulomb sum
    J_occ = 4 sum_{p,r < n/2} G^00_pprr, its change, the time and the speedup,
    with the tiles and first-half time per tier."""
    import torch
    from paper_2606_04316_amd import qdcb, workloads as wl

    name = args.workload or "cluster24"
    sysm = wl.config(name)
    n = sysm.n_mo
    dev = torch.device("cuda:0")
    CL = torch.from_numpy(sysm.CL).to(dev)
    CS = torch.from_numpy(sysm.CS).to(dev) if sysm.CS is not None else None
    G0 = torch.empty((n, n, n, n, 4, 4), dtype=torch.float64, device=dev)
    G1 = torch.empty_like(G0)
    ctx = qdcb.Context(0)
    L = qdcb.Basis(ctx, sysm.L)
    S = qdcb.Basis(ctx, sysm.S) if sysm.S is not None else None
    occ = torch.arange(n // 2, device=dev)

    def j_occ(G):
        # sum over p, r < n/2 of G^00_pprr, one p at a time (no large temporaries)
        return 4.0 * float(sum(G[p, p][occ, occ, 0, 0].sum() for p in range(n // 2)))

    def max_abs_diff(A, B):
        return max(float((A[p] - B[p]).abs().max()) for p in range(n))

    def timed(plan, G):
        for _ in range(max(1, args.warmup)):
            plan.transform(CL, CS, G)
        ms, st = [], None
        for _ in range(max(1, args.steps)):
            _, st = plan.transform(CL, CS, G)
            ms.append(st["ms_total"])
        return sorted(ms)[len(ms) // 2], st

    ref = qdcb.Plan(ctx, L, S, sysm.ham, n, sysm.tau)
    ms0, st0 = timed(ref, G0)
    ref.close()
    j0 = j_occ(G0)
    gmax = max(float(G0[p].abs().max()) for p in range(n))
    print(f"fp64: {ms0:.1f} ms", file=sys.stderr, flush=True)
    runs = []
    for spec in args.tiers.split(","):
        t32, t16, rule = spec.split(":")
        flags = qdcb.PLAN_TIER_BY_G if rule == "g" else 0
        plan = qdcb.Plan(ctx, L, S, sysm.ham, n, sysm.tau, prec="mixed", tier_fp32=float(t32),
                         tier_bf16=float(t16), flags=flags)
        ms, st = timed(plan, G1)
        plan.close()
        err = max_abs_diff(G1, G0)
        run = {"tier_fp32": float(t32), "tier_bf16": float(t16), "rule": rule, "ms": ms,
               "speedup": ms0 / ms, "max_abs_err": err, "abs_err_J_occ": abs(j_occ(G1) - j0),
               "meets_1e-10": err <= 1e-10, "tiles_tier": st["tiles_tier"],
               "ms_tier": st["ms_tier"], "ms_eri": st["ms_eri"],
               "ms_second_half": st["ms_second_half"]}
        runs.append(run)
        print(f"{spec}: {ms:.1f} ms, err {err:.2e}", file=sys.stderr, flush=True)
    ok = [r for r in runs if r["meets_1e-10"]]
    best = max(ok, key=lambda r: r["speedup"]) if ok else None
    print(json.dumps({
        "metric": "mixed vs FP64 speedup at max |dG| <= 1e-10 Eh", "mode": "mixed",
        "value": best["speedup"] if best else None, "unit": "x",
        "higher_is_better": True, "fp64_ms": ms0, "fp64_ms_tier": st0["ms_tier"],
        "fp64_ms_first_half": st0["ms_first_half"], "fp64_ms_eri": st0["ms_eri"],
        "max_abs_G": gmax, "J_occ": j0, "best": best, "runs": runs,
        "dtype": "f64+f32+bf16", "data": "synthetic",
        "config": {"workload": sysm.name, "n_atoms": int(sysm.atoms.shape[0]),
                   "N_L": sysm.L.nfunc, "N_S": sysm.S.nfunc if sysm.S is not None else 0,
                   "n_mo": n, "ham": sysm.ham, "tau": sysm.tau}}), flush=True)


SERVING_SIZES = {
    # the stream recipe's ranges, and the reduced ranges of the default leg
    "full": {"atoms": (10, 80), "nl": (100, 800), "n_mo": (16, 128)},
    "reduced": {"atoms": (10, 40), "nl": (40, 160), "n_mo": (8, 32)},
}


def serving_run(args, prec):
    """One run of the request stream (args.requests requests, mean gap 20 ms,
    the reduced or the full sizes) in one precision; eight requests re-run
    alone and compared bitwise."""
    import torch
    from paper_2606_04316_amd import qdcb, serving
    sz = SERVING_SIZES[args.serving_sizes]
    reqs = serving.request_stream(args.requests, seed=5, mean_gap_s=0.02, pool=12,
                                  atoms=sz["atoms"], nl=sz["nl"], n_mo=sz["n_mo"],
                                  radius_scale=20.0)
    pf = 0 if args.serving_rows == "bands" else qdcb.PLAN_SCHWARZ_ROWS
    # the eight requests re-run alone below (every len/8-th by arrival) are the
    # only ones hashed
    step = max(1, len(reqs) // 8)
    check_ids = [r.rid for r in sorted(reqs, key=lambda r: r.arrival)][::step][:8]
    # full sizes: G reaches tens of GB (n up to 128), so a request is served
    # when G is complete in device memory
    deliver = "device" if args.serving_sizes == "full" else "host"
    ex = serving.GpuExecutor(slots=args.slots, prec=prec, plan_flags=pf,
                             digest_ids=check_ids, deliver=deliver)
    budget = int(0.5 * torch.cuda.mem_get_info()[0])
    def done(r):  # progress of long streams: one line per served request
        if args.serving_sizes == "full":
            print(f"request {r.rid} served ({r.latency_ms:.0f} ms)", file=sys.stderr, flush=True)

    srv = serving.Server(ex, ex.reserve, slots=args.slots, budget_bytes=budget, on_done=done)
    out = srv.run(reqs)
    ex.drain()
    summ = serving.summarize(out)
    print(f"serving {prec}: {summ}", file=sys.stderr, flush=True)
    alone = serving.GpuExecutor(slots=1, prec=prec, plan_flags=pf, deliver=deliver)
    same = 0
    for r in [r for r in out if r.rid in set(check_ids)]:
        solo = serving.Request(rid=r.rid, system=r.system, arrival=0.0)
        solo.reserve = alone.reserve(solo)
        same += (r.error is None and
                 alone(solo, 0)["digest"] == r.result["digest"])
        if args.serving_sizes == "full":
            print(f"request {r.rid} re-run alone", file=sys.stderr, flush=True)
    alone.drain()
    summ.update({"stream": {"arrivals": "Poisson, mean gap 20 ms", "requests": len(reqs),
                            "atoms": list(sz["atoms"]), "N_L": list(sz["nl"]), "N_S": "2 N_L",
                            "n_mo": list(sz["n_mo"]), "contraction_depths": [1, 6],
                            "ham": "DC or DCG, 50/50", "tau": 1e-10, "pool": 12,
                            "note": ("the recipe's sizes" if args.serving_sizes == "full" else
                                     "reduced from 10-80 atoms, N_L 100-800, n_mo 16-128")},
                 "latency": ("arrival to G complete in device memory" if deliver == "device"
                             else "arrival to G in host memory"),
                 "slots": args.slots, "max_concurrency": srv.max_concurrency,
                 "row_order": "primitive bands" if args.serving_rows == "bands" else "Schwarz",
                 "peak_reserved_GB": srv.peak_in_use / 2 ** 30,
                 "alone_equals_mix": f"{same}/8"})
    if prec == "mixed":
        summ["tiers"] = {"tier_fp32": ex.tiers[0], "tier_bf16": ex.tiers[1], "rule": "g"}
    return summ


def main_serving(args):
    """The request loop on a seeded Poisson stream (mean gap 20 ms); each
    request is a cluster drawn from a pool, with its own active-space size and
    Hamiltonian (DC or DCG).  Sizes are reduced ranges of the stream recipe
    (10-40 atoms, N_L 40-160, n 8-32: at the recipe's full sizes one GPU is
    saturated and the latencies would measure the queue only); eight requests
    are re-run alone and compared bitwise."""
    runs = {prec: serving_run(args, prec) for prec in args.serving_prec.split(",")}
    first = runs[next(iter(runs))]
    line = {"metric": "serving p99 latency", "mode": "serving", "value": first["p99_ms"],
            "unit": "ms", "higher_is_better": False, "slots": args.slots,
            "requests": args.requests, "runs": runs, "data": "synthetic",
            "dtype": "f64" if "mixed" not in runs else "f64 / f64+f32+bf16"}
    if "fp64" in runs and "mixed" in runs:
        line["mixed_vs_fp64_throughput"] = (runs["mixed"]["mo_integrals_per_s"]
                                            / runs["fp64"]["mo_integrals_per_s"])
    print(json.dumps(line), flush=True)


def committed_traffic(workload, tune, row_order):
    """HBM bytes per first-half launch from the committed counter summary of
    this workload, when it was taken from the current kernel source in the
    same workgroup order and row order (else None)."""
    path = os.path.join(ROOT, "profiles", f"first_half_{workload}_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        tr = json.load(f)
    if (tr.get("kernel_rev") == qdcb_kernel_rev() and tr.get("fh_order") == tune["fh_order"]
            and tr.get("row_order") == row_order):
        return tr.get("bytes_per_launch")
    return None


def cluster_leg(args):
    """The compact-cluster configuration: 60 atoms in a 20 bohr ball, N_L 600,
    N_S 1200, contraction depths 1..6, n = 128, Dirac-Coulomb + Gaunt, tau
    1e-10, Loewdin coefficients.  FP64: autotuned launch choices (the tuner's
    warm-up sizes the integral panels), then args.cluster_steps timed
    transforms with the first half's roofline.  Mixed precision on the same
    inputs: the specified tiers (FP32 below 1e-4, BF16 below 1e-7, screening
    bound) and tiers that meet 1e-10 Eh here (3e-6 / 1e-9, bound including the
    bra side); each plan autotuned (its warm-up), one timed transform, its
    max |G_mixed - G_FP64| against the FP64 GPU result of the same inputs (the
    FP64 path is held to the oracle by the parity tests) and the change of the
    occupied-block Coulomb sum J_occ = 4 sum_{p,r < 64} G^00_pprr."""
    import torch
    from paper_2606_04316_amd import qdcb, workloads as wl

    t_start = time.perf_counter()
    sysm = wl.config("cluster60")
    n = sysm.n_mo
    dev = torch.device("cuda:0")
    G = torch.empty((n, n, n, n, 4, 4), dtype=torch.float64, device=dev)
    Gm = torch.empty_like(G)
    CL = torch.from_numpy(sysm.CL).to(dev)
    CS = torch.from_numpy(sysm.CS).to(dev)
    ctx = qdcb.Context(0)
    L, S = qdcb.Basis(ctx, sysm.L), qdcb.Basis(ctx, sysm.S)
    plan = qdcb.Plan(ctx, L, S, sysm.ham, n, sysm.tau)
    print(f"cluster leg: {sysm.name} ready", file=sys.stderr, flush=True)
    tune = autotune(args, plan, CL, CS, G)
    if not tune.get("autotuned") or tune.get("from_cache"):
        plan.transform(CL, CS, G)  # warm-up: sizes the integral panels
    torch.cuda.synchronize()
    stats = []
    t0 = time.perf_counter()
    for i in range(args.cluster_steps):
        _, st = plan.transform(CL, CS, G)
        stats.append(st)
        print(f"cluster step {i + 1}/{args.cluster_steps}: {st['ms_total']:.1f} ms",
              file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms = 1e3 * elapsed / args.cluster_steps
    fh_ms = sum(x["ms_first_half"] for x in stats)
    fh_launch = sum(x["n_batches"] for x in stats)
    achieved = sum(x["flops_first_half"] for x in stats) / (fh_ms * 1e-3) / 1e12
    sh_ms = sum(x["ms_second_half"] for x in stats)
    sh_rate = sum(x["flops_second_half"] for x in stats) / (sh_ms * 1e-3) / 1e12
    st0 = stats[-1]
    occ = torch.arange(n // 2, device=dev)

    def j_occ(X):
        return 4.0 * float(sum(X[p, p][occ, occ, 0, 0].sum() for p in range(n // 2)))

    j0 = j_occ(G)
    # the mixed plans below need the integral panels' memory
    plan.close()
    out = {
        "workload": sysm.name, "n_atoms": int(sysm.atoms.shape[0]), "N_L": sysm.L.nfunc,
        "N_S": sysm.S.nfunc, "n_mo": n, "ham": sysm.ham, "tau": sysm.tau,
        "contraction_depths": "1..6", "row_order": "primitive bands",
        "steps": args.cluster_steps, "ms_per_transform": ms,
        "value": n ** 4 / (ms * 1e-3), "unit": "quaternion MO integrals (pq|rs)/s",
        "spinor_integrals_per_s": (2 * n) ** 4 / (ms * 1e-3),
        "stages_ms": {k: st0[k] for k in ("ms_density", "ms_screen", "ms_eri", "ms_first_half",
                                          "ms_second_half", "ms_total")},
        "chunks": st0["n_chunks"], "tune": tune,
        "kept_fraction": (sum(st0["kept"]) + st0["kept_gaunt"])
        / max(1, sum(st0["total"]) + st0["total_gaunt"]),
        "tile_fill": st0["flops_first_half"] / max(1.0, st0["flops_mfma"]),
        "roofline": {"kernel": "k_first_half", "bound": "mfma", "achieved": achieved,
                     "peak": PEAK_FP64_MFMA, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP64_MFMA,
                     "traffic": committed_traffic("cluster60", tune["chosen"], "primitive bands"),
                     "launches": fh_launch, "avg_launch_ms": fh_ms / max(1, fh_launch)},
        "second_half": {"achieved": sh_rate, "frac": sh_rate / PEAK_FP64_MFMA,
                        "unit": "TFLOP/s"},
    }
    print(f"cluster leg fp64: {ms:.1f} ms per transform", file=sys.stderr, flush=True)
    mixed = []
    for t32, t16, rule in ((1e-4, 1e-7, "screen"), (3e-6, 1e-9, "g")):
        mp = qdcb.Plan(ctx, L, S, sysm.ham, n, sysm.tau, prec="mixed", tier_fp32=t32,
                       tier_bf16=t16, flags=qdcb.PLAN_TIER_BY_G if rule == "g" else 0)
        print(f"cluster leg mixed {t32}/{t16} {rule}: plan ready", file=sys.stderr, flush=True)
        mtune = autotune(args, mp, CL, CS, Gm)
        if not mtune.get("autotuned") or mtune.get("from_cache"):
            mp.transform(CL, CS, Gm)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        _, stm = mp.transform(CL, CS, Gm)
        torch.cuda.synchronize()
        ms_m = 1e3 * (time.perf_counter() - t1)
        err = max(float((Gm[p] - G[p]).abs().max()) for p in range(n))
        mixed.append({"tier_fp32": t32, "tier_bf16": t16,
                      "rule": "screening bound" if rule == "screen" else "G bound",
                      "ms_mixed": ms_m, "speedup": ms / ms_m,
                      "max_abs_err_vs_fp64_gpu_Eh": err, "meets_1e-10": err <= 1e-10,
                      "abs_err_J_occ_Eh": abs(j_occ(Gm) - j0),
                      "tiles_tier": stm["tiles_tier"], "ms_tier": stm["ms_tier"]})
        print(f"cluster leg mixed {t32}/{t16} {rule}: {ms_m:.1f} ms, max|dG| {err:.2e}",
              file=sys.stderr, flush=True)
        mp.close()
    out["mixed_vs_fp64"] = mixed
    out["J_occ"] = j0
    ctx.close()
    del G, Gm
    torch.cuda.empty_cache()
    out["wall_s"] = time.perf_counter() - t_start
    return out


def qdcb_kernel_rev():
    """Hash of the first-half kernel source, to tell whether committed
    counter data still describes the kernel being timed."""
    import hashlib
    p = os.path.join(ROOT, "paper_2606_04316_amd", "csrc", "k_gemm.hip")
    return hashlib.sha1(open(p, "rb").read()).hexdigest()[:12]


if __name__ == "__main__":
    main()
