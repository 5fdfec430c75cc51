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
