"""Host-side tests of the serving admission policy (no GPU)."""
import random

import pytest

from paper_2211_07260_amd import serving


def mk(n, seed=0):
    rng = random.Random(seed)
    out = []
    for i in range(n):
        kind = "conv_bf16" if rng.random() < 0.3 else "xcorr_f32"
        out.append(serving.Request(i, kind, rng.randint(16, 4096), rng.choice((3, 5, 9, 17)),
                                   32 if kind == "conv_bf16" else 1, i * 1e-3, i))
    return out


def test_footprint_values():
    assert serving.footprint("xcorr_f32", 4096, 17, 1) == 4 * (4112 ** 2 + 289 + 4096 ** 2)
    assert serving.footprint("conv_bf16", 128, 3, 32) == 2 * 128 * 128 * 32 + 2 * 32 * 9 * 32 + 4 * 128 * 128 * 32


@pytest.mark.parametrize("seed", range(5))
def test_admit_respects_budget_slots_and_order(seed):
    reqs = mk(200, seed)
    rng = random.Random(seed)
    for _ in range(50):
        mem = rng.randint(0, 4 << 30)
        slots = rng.randint(0, 40)
        n = serving.admit(reqs, mem, slots, max_batch=32)
        assert n <= min(slots, 32)
        assert sum(r.bytes for r in reqs[:n]) <= mem
        if n < min(slots, 32, len(reqs)):
            # stopped because the next request does not fit: no overtaking
            assert sum(r.bytes for r in reqs[:n + 1]) > mem


def test_admit_empty_and_zero():
    assert serving.admit([], 1 << 30, 10, 10) == 0
    assert serving.admit(mk(3), 0, 10, 10) == 0
    assert serving.admit(mk(3), 1 << 40, 0, 10) == 0


def test_latency_percentiles():
    class R:
        def __init__(self, a, d):
            self.t_arrive, self.t_done = a, d
    done = [R(0.0, k * 1e-3) for k in range(1, 101)]  # 1..100 ms
    s = serving.latency_stats(done)
    assert s["p50_ms"] == pytest.approx(50.0) and s["p99_ms"] == pytest.approx(99.0)


def test_energy_stats_counter_and_median():
    samples = [{"t_s": 10 + 0.01 * k, "power_w": 500.0 + (k % 3), "energy_t_s": float(k // 50),
                "energy_j": 1000.0 + 500.0 * (k // 50)} for k in range(300)]
    e = serving.energy_stats(samples, 10.0, 12.99, 100)
    assert e["p_median_w"] == 501.0
    assert e["j_per_request"] == pytest.approx(501.0 * 2.99 / 100)
    assert e["p_counter_w"] == pytest.approx(500.0)


class _FakeEvent:
    """Completes after being queried `delay` times."""
    def __init__(self, delay):
        self.left = delay

    def query(self):
        self.left -= 1
        return self.left < 0


def test_long_jobs_issue_in_order_and_retire_once(monkeypatch):
    # the long-request bookkeeping of the engine, without a GPU: parts are
    # issued in job order with at most parts_ahead queued, and every request
    # is retired exactly once, after its last part
    from paper_2211_07260_amd import serving
    issued = []
    monkeypatch.setattr(serving.gt, "conv2d_run_part",
                        lambda p, cfg, part, n, img, w, out, stream=None: issued.append((p, part, n)))

    class _Torch:
        class cuda:
            Event = staticmethod(lambda: _Ev())

    class _Ev:
        def record(self, stream):
            self.inner = _FakeEvent(delay=2)

        def query(self):
            return self.inner.query()

    eng = object.__new__(serving.Engine)
    eng.torch, eng.long_stream, eng.parts_ahead = _Torch, None, 2
    reqs = [serving.Request(k, "conv_bf16", 64, 3, 32, 0.0, k) for k in range(4)]
    jobs = []
    for k, r in enumerate(reqs):
        r.bufs, r.config = (None, None, None), (64, 1, 1, 1, 0, 0)
        jobs.append(serving.LongJob(r, "p%d" % k, k + 1))   # 1, 2, 3, 4 parts
    events = serving.collections.deque()
    retired = []
    for _ in range(200):
        retired += eng._retire_long(jobs, events)
        eng._issue_long(jobs, events)
        assert len(events) <= 2
        if not jobs:
            break
    assert retired == reqs and not events
    assert issued == [("p%d" % k, part, k + 1) for k in range(4) for part in range(k + 1)]


def test_long_job_that_cannot_be_split_runs_whole(monkeypatch):
    from paper_2211_07260_amd import serving
    calls = []

    def run_part(p, cfg, part, n, img, w, out, stream=None):
        if n > 1:
            raise serving.gt.GreentuneError(serving.gt.GT_E_UNSUPPORTED, "no parts for this shape")
        calls.append((part, n))
    monkeypatch.setattr(serving.gt, "conv2d_run_part", run_part)

    class _Ev:
        def record(self, stream):
            pass

        def query(self):
            return True

    class _Torch:
        class cuda:
            Event = staticmethod(lambda: _Ev())

    eng = object.__new__(serving.Engine)
    eng.torch, eng.long_stream, eng.parts_ahead = _Torch, None, 2
    r = serving.Request(0, "conv_bf16", 64, 11, 32, 0.0, 0)
    r.bufs, r.config = (None, None, None), (64, 1, 1, 1, 0, 0)
    jobs, events = [serving.LongJob(r, "p", 5)], serving.collections.deque()
    eng._issue_long(jobs, events)
    assert calls == [(0, 1)] and len(events) == 1 and jobs[0].n_parts == 1
    assert eng._retire_long(jobs, events) == [r] and not jobs
