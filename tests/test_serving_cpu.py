"""The continuous-batching scheduler on the CPU with a fake executor: request
splitting and reassembly, coalescing by k, workspace admission, overlap of
batches, latency accounting."""
import numpy as np
import pytest

from paper_1103_2635_amd.serving import Request, Scheduler, latency_stats, replay


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, s):
        self.t += max(s, 1e-6)


class FakeExecutor:
    """Batch latency = a + b * m; results are the query ids times k so the
    reassembly can be checked."""

    def __init__(self, clock, a=1e-3, b=1e-5, ws_per_query=1000):
        self.clock = clock
        self.a, self.b, self.ws = a, b, ws_per_query
        self.live = {}
        self.concurrent_peak = 0

    def workspace_bytes(self, m, k):
        return self.ws * m * k

    def launch(self, batch):
        ids = np.concatenate([np.arange(r.offset + s, r.offset + s + c) for (r, s, c) in batch.parts])
        res = (ids[:, None] * 10 + np.arange(batch.k)[None, :], ids[:, None] * 0.5 + np.zeros((1, batch.k)))
        h = (self.clock() + self.a + self.b * batch.m, res)
        self.live[id(batch)] = h
        self.concurrent_peak = max(self.concurrent_peak, len(self.live))
        return h

    def done(self, h):
        return self.clock() >= h[0]

    def results(self, batch):
        return self.live[id(batch)][1]

    def release(self, batch):
        del self.live[id(batch)]


def _trace(n, rate, seed, max_m=4096):
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1 / rate, n))
    sizes = np.clip(np.rint(np.exp(rng.normal(4, 1.5, n))), 1, max_m).astype(int)
    ks = np.where(rng.random(n) < 0.5, 1, 10)
    offs = rng.integers(0, 100000, n)
    return [Request(i, int(offs[i]), int(sizes[i]), int(ks[i]), float(t[i])) for i in range(n)]


def _check_results(reqs):
    for r in reqs:
        assert r.done_at is not None and r.done_at >= r.arrival
        got = sorted(r.results, key=lambda x: x[0])
        idx = np.concatenate([g[1] for g in got])
        assert idx.shape == (r.m, r.k)
        ids = np.arange(r.offset, r.offset + r.m)
        assert np.array_equal(idx, ids[:, None] * 10 + np.arange(r.k)[None, :])


def test_split_coalesce_and_reassembly():
    clk = FakeClock()
    ex = FakeExecutor(clk)
    s = Scheduler(ex, n_slots=3, mem_budget=10**12, max_batch=512)
    reqs = _trace(400, 2000.0, 1)
    done = replay(s, reqs, clk, clk.sleep)
    assert len(done) == 400
    _check_results(done)
    big = [r for r in reqs if r.m > 512]
    assert big, "the trace must contain requests larger than one batch"
    assert s.batches_launched < sum((r.m + 511) // 512 for r in reqs)  # some coalescing happened
    assert ex.concurrent_peak <= 3 and s.max_concurrent >= 2


def test_memory_admission_never_exceeds_budget():
    clk = FakeClock()
    ex = FakeExecutor(clk, ws_per_query=10)
    budget = 10 * 600 * 10  # about one full batch with k = 10
    s = Scheduler(ex, n_slots=8, mem_budget=budget, max_batch=600)
    reqs = _trace(300, 5000.0, 2)
    done = replay(s, reqs, clk, clk.sleep)
    _check_results(done)
    assert s.max_mem_used <= budget


def test_fifo_progress_and_latency_stats():
    clk = FakeClock()
    ex = FakeExecutor(clk, a=2e-3, b=0)
    s = Scheduler(ex, n_slots=1, mem_budget=10**12, max_batch=4096)
    reqs = [Request(i, i, 10, 1 + 9 * (i % 2), i * 1e-3) for i in range(50)]
    done = replay(s, reqs, clk, clk.sleep)
    st = latency_stats(done)
    assert st["requests"] == 50 and st["p99_ms"] >= st["p50_ms"] > 0
    # one slot, alternating k: batches cannot mix k, and no request waits forever
    assert max(r.done_at - r.arrival for r in done) < 0.2


def test_rejects_bad_configuration():
    with pytest.raises(ValueError):
        Scheduler(FakeExecutor(FakeClock()), 0, 1, 1)
