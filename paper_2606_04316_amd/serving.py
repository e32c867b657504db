"""Request loop for transforms of different bases and active spaces.

Continuous batching on one GPU: requests arrive over time; each waits until a
worker slot is free and its device-memory reservation (the plan's footprint
estimate) fits what the running requests leave of the budget, and then runs
on that worker's own HIP stream, so the kernels of the admitted requests
overlap on the device.  AO pair data stays resident: bases are cached by the
content of their arrays and shared by every request that uses them.  Waiting
requests are admitted in arrival order, except that a request that fits may
pass a larger one at the head of the queue that does not (size-aware
admission).  Each transform's result depends only on its own inputs, so a
request gives the same output alone and in the mix.

The scheduler is independent of the GPU: ``Server(executor=...)`` accepts any
callable, which the CPU tests use to check admission and accounting.
"""
from __future__ import annotations

import dataclasses
import hashlib
import queue
import threading
import time
from typing import Callable, Dict, List, Optional

import numpy as np


@dataclasses.dataclass
class Request:
    rid: int
    system: object          # workloads.System
    arrival: float          # seconds after the stream start
    reserve: int = 0        # device bytes reserved while running
    # filled in by the server
    t_admit: float = 0.0
    t_done: float = 0.0
    result: object = None
    error: Optional[str] = None

    @property
    def latency_ms(self) -> float:
        return 1e3 * (self.t_done - self.arrival)


class Server:
    """``executor(request, slot) -> result`` runs one request; ``reserve(request)``
    gives its device-memory reservation in bytes."""

    def __init__(self, executor: Callable, reserve: Callable, slots: int, budget_bytes: int,
                 on_done: Optional[Callable] = None):
        if slots < 1:
            raise ValueError("need at least one slot")
        self.on_done = on_done  # called with each request once it is served
        self.executor = executor
        self.reserve = reserve
        self.slots = slots
        self.budget = int(budget_bytes)
        self._lock = threading.Condition()
        self._in_use = 0
        self._free_slots = list(range(slots))
        self._waiting: List[Request] = []
        self.peak_in_use = 0
        self.max_concurrency = 0
        self._running = 0

    def _release_memory(self, r: Request):
        with self._lock:
            self._in_use -= r.reserve
            self._lock.notify_all()

    def _try_admit(self) -> List[tuple]:
        """Admissions possible now (called with the lock held)."""
        out = []
        i = 0
        while i < len(self._waiting) and self._free_slots:
            r = self._waiting[i]
            if r.reserve > self.budget:
                # can never fit beside anything: run it alone with the whole budget
                if self._running == 0 and i == 0:
                    r.reserve = self.budget
                else:
                    i += 1
                    continue
            if self._in_use + r.reserve <= self.budget:
                self._waiting.pop(i)
                slot = self._free_slots.pop(0)
                self._in_use += r.reserve
                self._running += 1
                self.peak_in_use = max(self.peak_in_use, self._in_use)
                self.max_concurrency = max(self.max_concurrency, self._running)
                out.append((r, slot))
            else:
                i += 1
        return out

    def run(self, requests: List[Request], clock_scale: float = 1.0) -> List[Request]:
        """Replays the arrival times (seconds * clock_scale) and serves every
        request; returns them with timings filled in."""
        requests = sorted(requests, key=lambda r: r.arrival)
        for r in requests:
            r.reserve = int(self.reserve(r))
        t0 = time.perf_counter()
        threads = []

        # an executor that frees device memory after returning (deferred
        # release) reports each request's release through on_release; its
        # reservation stays counted until then
        deferred = bool(getattr(self.executor, "deferred_release", False))
        if deferred:
            self.executor.on_release = self._release_memory

        def work(r: Request, slot: int):
            try:
                r.result = self.executor(r, slot)
            except Exception as e:  # reported per request
                r.error = f"{type(e).__name__}: {e}"
            # the result is delivered when the executor says so (e.g. G on the
            # host), before any bookkeeping it does afterwards
            t_res = r.result.get("t_result") if isinstance(r.result, dict) else None
            r.t_done = (t_res if t_res is not None else time.perf_counter()) - t0
            with self._lock:
                if not deferred:
                    self._in_use -= r.reserve
                self._running -= 1
                self._free_slots.append(slot)
                self._free_slots.sort()
                self._lock.notify_all()
            if self.on_done is not None:
                self.on_done(r)

        def launch(batch):
            for r, slot in batch:
                r.t_admit = time.perf_counter() - t0
                th = threading.Thread(target=work, args=(r, slot), daemon=True)
                threads.append(th)
                th.start()

        pending = list(requests)
        while pending or self._waiting or self._running:
            now = time.perf_counter() - t0
            with self._lock:
                while pending and pending[0].arrival * clock_scale <= now:
                    r = pending.pop(0)
                    r.arrival *= clock_scale
                    self._waiting.append(r)
                batch = self._try_admit()
            if batch:
                launch(batch)
                continue
            with self._lock:
                if not (pending or self._waiting or self._running):
                    break
                wait = 0.05
                if pending:
                    wait = max(0.0, min(wait, pending[0].arrival * clock_scale - now))
                self._lock.wait(timeout=wait)
        for th in threads:
            th.join()
        return requests


# ---------------------------------------------------------------------------
# GPU executor
# ---------------------------------------------------------------------------

def basis_key(b) -> str:
    h = hashlib.sha1()
    for a in (b.centers, b.nprim, b.exps, b.coefs):
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()


class GpuExecutor:
    """Runs requests through the C ABI: a resident basis cache, one plan and
    one HIP stream (torch) per request, the plan created in a context whose
    budget is the request's reservation.  ``prec="mixed"`` runs every plan
    with the reduced-precision tiers (``tiers`` = tier_fp32, tier_bf16, plan
    flags); ``plan_flags`` are added to every plan's flags (for instance
    PLAN_SCHWARZ_ROWS for plain Schwarz row order).

    G comes to the host through a pinned staging buffer per slot (reused, so
    a result is delivered as the digest of that copy, or as the device tensor
    with keep_outputs; ``digest_ids`` limits the hashing to those requests).  Finished plans and their contexts are destroyed by a
    background thread: freeing device memory waits for the work of every
    stream on the device, which would otherwise hold the slot until the other
    slots' transforms finish.  ``drain()`` waits for those releases."""

    def __init__(self, slots: int, device: int = 0, keep_outputs: bool = False,
                 prec: str = "fp64", tiers=(1e-6, 1e-9, 0x2), plan_flags: int = 0,
                 digest_ids=None, deliver: str = "host"):
        import torch
        from paper_2606_04316_amd import qdcb
        self.torch = torch
        self.qdcb = qdcb
        self.device = device
        self.dev = torch.device(f"cuda:{device}")
        self.ctx = qdcb.Context(device)  # owns the resident bases
        self.streams = [torch.cuda.Stream(device=self.dev) for _ in range(slots)]
        self.bases: Dict[str, object] = {}
        self.block = threading.Lock()
        self.keep_outputs = keep_outputs
        self.prec = prec
        self.tiers = tiers
        self.plan_flags = int(plan_flags)
        # requests whose G is hashed for the alone-vs-mix comparison (None:
        # every request); the hash runs after delivery but holds the slot
        self.digest_ids = None if digest_ids is None else set(digest_ids)
        self.staging = [None] * slots  # pinned host buffers for G, per slot
        # "host": a request is served when G is in host memory; "device": when
        # G is complete in device memory (outputs of tens of GB at the largest
        # active spaces), its digest then taken from per-row integer sums of G's
        # bits on the device
        if deliver not in ("host", "device"):
            raise ValueError("deliver must be 'host' or 'device'")
        self.deliver = deliver
        self._retire: "queue.Queue" = queue.Queue()
        self._reaper = threading.Thread(target=self._reap, daemon=True)
        self._reaper.start()

    # the request loop counts a request's reservation until its plan is gone
    deferred_release = True
    on_release = None

    def _reap(self):
        while True:
            plan, ctx, r = self._retire.get()
            try:
                if plan is not None:
                    plan.close()
                if ctx is not None:
                    ctx.close()
            finally:
                if self.on_release is not None:
                    self.on_release(r)
                self._retire.task_done()

    def drain(self):
        """Wait until every finished plan has been destroyed."""
        self._retire.join()

    def _host_copy(self, G, slot: int, stream):
        torch = self.torch
        buf = self.staging[slot]
        if buf is None or buf.numel() < G.numel():
            buf = torch.empty(G.numel(), dtype=torch.float64, pin_memory=True)
            self.staging[slot] = buf
        h = buf[:G.numel()].view(G.shape)
        with torch.cuda.stream(stream):
            h.copy_(G, non_blocking=True)
        stream.synchronize()
        return h.numpy()

    def basis(self, b):
        k = basis_key(b)
        with self.block:
            if k not in self.bases:
                self.bases[k] = self.qdcb.Basis(self.ctx, b)
            return self.bases[k]

    def reserve(self, r: Request) -> int:
        s = r.system
        L = self.basis(s.L)
        S = self.basis(s.S) if s.S is not None else None
        return self.qdcb.Plan.estimate(L, S, s.ham, s.n_mo, s.tau, prec=self.prec)

    def __call__(self, r: Request, slot: int):
        held = {}  # the request's context and plan, destroyed by the reaper
        try:
            return self._run_request(r, slot, held)
        finally:
            self._retire.put((held.get("plan"), held.get("ctx"), r))

    def _run_request(self, r: Request, slot: int, held: dict):
        torch, qdcb = self.torch, self.qdcb
        s = r.system
        L = self.basis(s.L)
        S = self.basis(s.S) if s.S is not None else None
        t_start = time.perf_counter()
        ctx = held["ctx"] = qdcb.Context(self.device, budget_bytes=r.reserve)
        stream = self.streams[slot]
        with torch.cuda.stream(stream):
            if self.prec == "mixed":
                t32, t16, flags = self.tiers
                plan = qdcb.Plan(ctx, L, S, s.ham, s.n_mo, s.tau, prec="mixed",
                                 tier_fp32=t32, tier_bf16=t16, flags=flags | self.plan_flags)
            else:
                plan = qdcb.Plan(ctx, L, S, s.ham, s.n_mo, s.tau, flags=self.plan_flags)
            held["plan"] = plan
            t_plan = time.perf_counter()
            CL = torch.from_numpy(s.CL).to(self.dev, non_blocking=False)
            CS = torch.from_numpy(s.CS).to(self.dev) if s.CS is not None else None
            n = s.n_mo
            G = torch.empty((n, n, n, n, 4, 4), dtype=torch.float64, device=self.dev)
            G, st = plan.transform(CL, CS, G, stream=stream.cuda_stream)
        t_tr = time.perf_counter()
        want = self.digest_ids is None or r.rid in self.digest_ids
        digest = None
        if self.deliver == "device":
            stream.synchronize()
            t_result = time.perf_counter()  # G is complete on the device: served
            if want:
                with torch.cuda.stream(stream):
                    # integer sums wrap modulo 2^64 in any order: bitwise-equal G,
                    # equal sums
                    rows = G.view(n * n, -1).view(torch.int64).sum(dim=1).cpu().numpy()
                digest = hashlib.sha1(rows.tobytes()).hexdigest()
        else:
            Gh = self._host_copy(G, slot, stream)
            t_result = time.perf_counter()  # G is on the host: the request is served
            if want:
                digest = hashlib.sha1(Gh.tobytes()).hexdigest()
        out = {"digest": digest, "n": n, "ms_gpu": st["ms_total"], "t_result": t_result,
               "flops": st["flops_first_half"] + st["flops_second_half"],
               "ms_plan": 1e3 * (t_plan - t_start), "ms_transform_call": 1e3 * (t_tr - t_plan),
               "ms_copy": 1e3 * (t_result - t_tr),
               "ms_digest": 1e3 * (time.perf_counter() - t_result),
               "path": {k: st[k] for k in ("n_batches", "n_chunks", "tiles_made")}}
        if self.keep_outputs:
            out["G"] = G
        return out


def request_stream(count: int, seed: int = 5, mean_gap_s: float = 0.02, pool: int = 16,
                   atoms=(10, 80), nl=(100, 800), n_mo=(16, 128), radius_scale: float = 20.0):
    """Seeded Poisson request stream (exponential gaps).  Molecules come from a
    pool of ``pool`` random clusters (so bases repeat and stay resident); each
    request draws its active-space size and Hamiltonian (DC or DCG, 50/50)."""
    from paper_2606_04316_amd import workloads as wl
    rng = np.random.default_rng(seed)
    mols = []
    for m in range(pool):
        nat = int(rng.integers(atoms[0], atoms[1] + 1))
        nL = int(rng.integers(nl[0], nl[1] + 1))
        radius = radius_scale * (nat / 60.0) ** (1.0 / 3.0)
        mols.append((nat, nL, radius, 100 + m))
    reqs = []
    t = 0.0
    cache = {}
    for i in range(count):
        t += float(rng.exponential(mean_gap_s))
        nat, nL, radius, mseed = mols[int(rng.integers(0, pool))]
        n = int(rng.integers(n_mo[0], n_mo[1] + 1))
        ham = "DC" if rng.random() < 0.5 else "DCG"
        key = (mseed, n, ham)
        if key not in cache:
            per_atom_L = max(1, nL // nat)
            cache[key] = wl.cluster(seed=mseed, n_atoms=nat, radius=radius, min_sep=2.0,
                                    nl_per_atom=per_atom_L, ns_per_atom=2 * per_atom_L, n=n,
                                    nprim=(1, 6), tau=1e-10, ham=ham)
        reqs.append(Request(rid=i, system=cache[key], arrival=t))
    return reqs


def summarize(reqs: List[Request]) -> dict:
    errors = sorted({r.error for r in reqs if r.error is not None})[:3]
    lat = np.array([r.latency_ms for r in reqs if r.error is None])
    done = [r for r in reqs if r.error is None]
    span = max(r.t_done for r in reqs) - min(r.arrival for r in reqs) if reqs else 0.0
    mo = sum(r.system.n_mo ** 4 for r in done)
    wait = np.array([1e3 * (r.t_admit - r.arrival) for r in done])
    serve = np.array([1e3 * (r.t_done - r.t_admit) for r in done])
    gpu = np.array([r.result["ms_gpu"] for r in done
                    if isinstance(r.result, dict) and "ms_gpu" in r.result])

    def mean_of(k):
        v = [r.result[k] for r in done if isinstance(r.result, dict) and k in r.result]
        return float(np.mean(v)) if v else None
    return {"requests": len(reqs), "failed": sum(r.error is not None for r in reqs),
            "p50_ms": float(np.percentile(lat, 50)) if lat.size else None,
            "p99_ms": float(np.percentile(lat, 99)) if lat.size else None,
            "mean_ms": float(lat.mean()) if lat.size else None,
            "mean_wait_ms": float(wait.mean()) if wait.size else None,
            "mean_service_ms": float(serve.mean()) if serve.size else None,
            "mean_transform_ms": float(gpu.mean()) if gpu.size else None,
            "mean_parts_ms": {k: mean_of("ms_" + k) for k in ("plan", "transform_call", "copy",
                                                                 "digest")},
            "span_s": span, "mo_integrals_per_s": mo / span if span > 0 else None,
            "errors": errors}
