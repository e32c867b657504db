"""CPU tests of the request loop's admission and accounting (no GPU):
a fake executor stands in for the transform."""
import threading
import time

from paper_2606_04316_amd.serving import Request, Server


class FakeExec:
    def __init__(self, budget):
        self.lock = threading.Lock()
        self.in_use = 0
        self.peak = 0
        self.running = 0
        self.peak_running = 0
        self.budget = budget
        self.order = []

    def reserve(self, r):
        return r.system

    def __call__(self, r, slot):
        with self.lock:
            self.in_use += r.reserve
            self.running += 1
            self.peak = max(self.peak, self.in_use)
            self.peak_running = max(self.peak_running, self.running)
            self.order.append(r.rid)
        time.sleep(0.02 + 0.001 * (r.system % 7))
        with self.lock:
            self.in_use -= r.reserve
            self.running -= 1
        return {"digest": str(r.rid)}


def test_all_requests_served_within_budget_and_slots():
    fx = FakeExec(100)
    reqs = [Request(rid=i, system=10 + (i * 37) % 50, arrival=0.003 * i) for i in range(40)]
    srv = Server(fx, fx.reserve, slots=3, budget_bytes=100)
    out = srv.run(reqs)
    assert all(r.error is None and r.result["digest"] == str(r.rid) for r in out)
    assert fx.peak <= 100 and srv.peak_in_use <= 100
    assert fx.peak_running <= 3 and srv.max_concurrency >= 2
    assert all(r.t_done >= r.t_admit >= r.arrival for r in out)


def test_small_request_passes_a_large_one_that_does_not_fit():
    fx = FakeExec(100)
    reqs = [Request(rid=0, system=70, arrival=0.0),      # runs first
            Request(rid=1, system=60, arrival=0.001),    # must wait for rid 0
            Request(rid=2, system=20, arrival=0.002)]    # fits beside rid 0
    srv = Server(fx, fx.reserve, slots=3, budget_bytes=100)
    out = srv.run(reqs)
    assert fx.order.index(2) < fx.order.index(1)
    assert out[2].t_admit < out[1].t_admit


def test_request_larger_than_budget_runs_alone():
    fx = FakeExec(100)
    reqs = [Request(rid=0, system=30, arrival=0.0), Request(rid=1, system=500, arrival=0.001),
            Request(rid=2, system=30, arrival=0.002)]
    srv = Server(fx, fx.reserve, slots=2, budget_bytes=100)
    out = srv.run(reqs)
    assert all(r.error is None for r in out)
    assert out[1].reserve == 100  # clipped to the whole budget, run alone
    assert fx.peak <= 130


def test_executor_errors_are_reported_per_request():
    def bad(r, slot):
        if r.rid == 1:
            raise RuntimeError("boom")
        return {"digest": "ok"}

    reqs = [Request(rid=i, system=1, arrival=0.0) for i in range(3)]
    out = Server(bad, lambda r: 1, slots=2, budget_bytes=10).run(reqs)
    assert out[1].error and "boom" in out[1].error
    assert out[0].error is None and out[2].error is None


class DeferredExec(FakeExec):
    """Frees a request's memory some time after returning, from another thread,
    and reports it through on_release (as the GPU executor does)."""
    deferred_release = True
    on_release = None

    def __call__(self, r, slot):
        with self.lock:
            self.in_use += r.reserve
            self.running += 1
            self.peak = max(self.peak, self.in_use)
            self.peak_running = max(self.peak_running, self.running)
        time.sleep(0.01)
        with self.lock:
            self.running -= 1

        def later():
            time.sleep(0.03)
            with self.lock:
                self.in_use -= r.reserve
            self.on_release(r)

        threading.Thread(target=later, daemon=True).start()
        return {"digest": str(r.rid)}


def test_deferred_release_keeps_memory_counted_until_freed():
    fx = DeferredExec(100)
    reqs = [Request(rid=i, system=30 + (i * 13) % 40, arrival=0.002 * i) for i in range(30)]
    srv = Server(fx, fx.reserve, slots=4, budget_bytes=100)
    out = srv.run(reqs)
    assert all(r.error is None for r in out)
    # memory still being freed after a request returned counted against the budget
    assert fx.peak <= 100 and srv.peak_in_use <= 100
    time.sleep(0.1)
    assert fx.in_use == 0 and srv._in_use == 0
