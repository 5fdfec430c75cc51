"""Continuous-batching serving loop for a mix of convolution requests.

Requests arrive over time (Poisson arrivals in the benchmark).  The loop
admits waiting requests first-come first-served while a slot is free and the
request's device footprint (input, filter, output) fits the memory budget;
each admitted group is launched at once -- single-channel requests as one
persistent batched launch per filter size, with the per-size autotuned
config, multi-channel BF16 requests on the MFMA kernel -- on alternating
compute streams, so new work is queued while earlier steps still run.  A
step's requests complete when its event has fired; their memory and slots are
then released and later arrivals are admitted.  Latency is completion minus
arrival; energy per request is the serving window's energy (median power times
window, and the energy counter) divided by the requests served.

Payloads are synthetic: a request's input and filter are views, at offsets
derived from its seed, into device-resident pools of uniform [0, 1) values
drawn once per device (FP32 and BF16), so serving spends no GPU time
generating data and a request's output can be recomputed alone for the
equality check.  The pools are larger than the device's last-level cache, so
requests that run together do not read each other's data from it.
"""
import collections
import math
import time

import paper_2211_07260_amd as gt
from paper_2211_07260_amd import autotune


# BF16 requests up to this output side (per filter size) share one
# persistent launch per step and filter size (batched global-load MFMA
# kernel, 280-400 TFLOP/s at C = 32); larger ones run the LDS-staged kernel
# alone, which reuses each input byte across the filter taps but costs a
# launch of 10-50 us however small the request.  From timing equal-size
# batches both ways on MI355X: batched ahead up to about these sides.
BF16_BATCH_SIDE = {3: 384, 5: 256, 9: 160, 17: 160}
BF16_BATCH_SIDE_OTHER = 160


class Request:
    __slots__ = ("rid", "kind", "side", "f", "c", "t_arrive", "seed", "t_admit", "t_done", "bufs", "config",
                 "bytes", "path")

    def __init__(self, rid, kind, side, f, c, t_arrive, seed):
        self.rid, self.kind, self.side, self.f, self.c = rid, kind, side, f, c
        self.t_arrive, self.seed = t_arrive, seed
        self.t_admit = self.t_done = None
        self.bufs = None
        self.config = None
        self.path = None  # "batched" (a persistent launch of its step), "single", or "parts"
        self.bytes = footprint(kind, side, f, c)

    def flops(self):
        if self.kind == "xcorr_f32":
            return 2.0 * self.side * self.side * self.f * self.f
        return 2.0 * self.side * self.side * self.c * self.c * self.f * self.f


def footprint(kind, side, f, c):
    """Device bytes of one request: input, filter and output."""
    if kind == "xcorr_f32":
        return 4 * ((side + f - 1) ** 2 + f * f + side * side)
    return 2 * side * side * c + 2 * c * f * f * c + 4 * side * side * c


def admit(waiting, mem_free, slots_free, max_batch):
    """First-come first-served admission: take requests from the head of the
    queue while a slot is free and the footprint fits; stop at the first that
    does not fit (no overtaking, so no request starves).  Returns the count."""
    n = 0
    for r in waiting:
        if n >= max_batch or slots_free <= 0 or r.bytes > mem_free:
            break
        mem_free -= r.bytes
        slots_free -= 1
        n += 1
    return n


POOL_F32_ELEMS = 1 << 28       # 1 GiB of FP32 values
POOL_BF16_ELEMS = 3 << 29      # 3 GiB of BF16 values
POOL_ALIGN = 64                # views start on 64-element boundaries (>= 128 bytes)
_pools = {}


def payload_pools(device):
    """The FP32 and BF16 value pools of a device (drawn on first use from a
    fixed seed, then kept for the life of the process)."""
    import torch
    key = str(torch.device(device))
    if key not in _pools:
        g = torch.Generator(device=device).manual_seed(20221114)
        f32 = torch.rand(POOL_F32_ELEMS, generator=g, device=device)
        bf16 = torch.rand(POOL_BF16_ELEMS, generator=g, device=device, dtype=torch.bfloat16)
        torch.cuda.synchronize(device)
        _pools[key] = (f32, bf16)
    return _pools[key]


def _pool_view(pool, n, seed, salt):
    """n contiguous pool values at an offset fixed by (seed, salt)."""
    slots = (pool.numel() - n) // POOL_ALIGN + 1
    h = (seed * 0x9E3779B1 + salt * 0x85EBCA77 + 0x27D4EB2F) & 0xFFFFFFFFFFFF
    off = (h % slots) * POOL_ALIGN
    return pool[off:off + n]


def make_payload(r, device):
    """(input, filter, output) of a request: pool views for the input and
    filter, a fresh output tensor."""
    import torch
    f32, bf16 = payload_pools(device)
    if r.kind == "xcorr_f32":
        ih = r.side + r.f - 1
        img = _pool_view(f32, ih * ih, r.seed, 0).view(ih, ih)
        w = _pool_view(f32, r.f * r.f, r.seed, 1).view(r.f, r.f)
        out = torch.empty(r.side, r.side, device=device)
    else:
        img = _pool_view(bf16, r.side * r.side * r.c, r.seed, 0).view(1, r.side, r.side, r.c)
        w = _pool_view(bf16, r.c * r.f * r.f * r.c, r.seed, 1).view(r.c, r.f, r.f, r.c)
        out = torch.empty(1, r.side, r.side, r.c, device=device)
    return img, w, out


class Step:
    __slots__ = ("reqs", "event", "batches")

    def __init__(self, reqs, event, batches):
        self.reqs, self.event, self.batches = reqs, event, batches


class LongJob:
    """A long BF16 request computed as n_parts launches (conv2d_run_part)."""
    __slots__ = ("req", "problem", "n_parts", "next_part")

    def __init__(self, req, problem, n_parts):
        self.req, self.problem, self.n_parts, self.next_part = req, problem, n_parts, 0


class Engine:
    """Continuous batching over streams.  Short requests are admitted in
    groups and launched as one step per group on the short streams in turn;
    a BF16 request of more than part_flops runs on its own stream in parts
    of about part_flops each, at most parts_ahead of them queued, so that
    short work issued meanwhile starts after the running part instead of
    after the whole request (part_flops=None: no parts).  objective: which
    per-size config of the autotuner's store the batched launches use
    ("time" or "energy").  BF16 requests of side at most bf16_batch_side
    (a {filter: side} dict, or one side for all filters) run as one
    persistent launch per (filter, channels) of their step (IgemmBatch);
    larger ones launch alone (0: never batched)."""

    def __init__(self, mem_budget=32 << 30, max_slots=512, max_batch=256, n_streams=2, store=None,
                 keep_outputs=False, device="cuda:0", streams=None, long_stream=None, part_flops=1.0e12,
                 parts_ahead=2, objective="time", bf16_batch_side=BF16_BATCH_SIDE):
        import torch
        if objective not in autotune.OBJECTIVES:
            raise ValueError("objective must be one of %s" % (autotune.OBJECTIVES,))
        self.objective = objective
        self.bf16_batch_side = bf16_batch_side
        self.torch = torch
        self.device = torch.device(device)
        self.mem_budget, self.max_slots, self.max_batch = mem_budget, max_slots, max_batch
        # torch's caching allocator keeps freed blocks per stream: engines
        # that share streams (streams=..., long_stream=...) reuse each
        # other's device buffers
        self.streams = list(streams) if streams else [torch.cuda.Stream(device=self.device) for _ in range(n_streams)]
        self.long_stream = long_stream if long_stream is not None else torch.cuda.Stream(device=self.device)
        self.part_flops, self.parts_ahead = part_flops, max(1, parts_ahead)
        self.store = store if store is not None else autotune.load()
        payload_pools(self.device)  # drawn once, before any request is timed
        self.keep_outputs = keep_outputs
        self.outputs = {}
        self.mem_used = 0
        self.peak_mem = 0
        self.slots_used = 0
        self.rejected = []

    def _bf16_side(self, f):
        b = self.bf16_batch_side
        return b.get(f, BF16_BATCH_SIDE_OTHER) if isinstance(b, dict) else b

    def is_long(self, r):
        return self.part_flops is not None and r.kind == "conv_bf16" and r.flops() > self.part_flops

    def _start_long(self, r):
        with self.torch.cuda.stream(self.long_stream):
            r.bufs = make_payload(r, self.device)
        r.config = (64, 1, 1, 1, 0, 0)
        r.path = "parts"
        p = gt.conv_problem(gt.IGEMM_BF16_MFMA, 1, r.side, r.side, r.c, r.c, r.f, r.f)
        return LongJob(r, p, max(1, int(math.ceil(r.flops() / self.part_flops))))

    def _retire_long(self, jobs, events):
        """Retire finished parts (in launch order: one stream); returns the
        requests whose last part has finished (their jobs leave `jobs`)."""
        finished = []
        while events and events[0][0].query():
            _, job, last = events.popleft()
            if last:
                finished.append(job.req)
                jobs.remove(job)
        return finished

    def _issue_long(self, jobs, events):
        """Keep up to parts_ahead parts queued on the long stream."""
        while len(events) < self.parts_ahead:
            job = next((j for j in jobs if j.next_part < j.n_parts), None)
            if job is None:
                break
            img, w, out = job.req.bufs
            try:
                gt.conv2d_run_part(job.problem, job.req.config, job.next_part, job.n_parts, img, w, out,
                                   stream=self.long_stream)
            except gt.GreentuneError as e:
                # a shape the tiled kernel does not cover cannot be split: run
                # it whole (nothing of it has been issued yet)
                if e.code != gt.GT_E_UNSUPPORTED or job.next_part != 0:
                    raise
                job.n_parts = 1
                gt.conv2d_run_part(job.problem, job.req.config, 0, 1, img, w, out, stream=self.long_stream)
            ev = self.torch.cuda.Event()
            ev.record(self.long_stream)
            job.next_part += 1
            events.append((ev, job, job.next_part == job.n_parts))

    def _launch(self, reqs, stream):
        torch = self.torch
        with torch.cuda.stream(stream):
            for r in reqs:
                r.bufs = make_payload(r, self.device)
            groups = collections.defaultdict(list)
            bf16_groups = collections.defaultdict(list)
            batches = []
            for r in reqs:
                if r.kind == "xcorr_f32":
                    groups[r.f].append(r)
                elif r.side <= self._bf16_side(r.f):
                    bf16_groups[(r.f, r.c)].append(r)
                else:
                    img, w, out = r.bufs
                    r.config = (64, 1, 1, 1, 0, 0)
                    r.path = "single"
                    p = gt.conv_problem(gt.IGEMM_BF16_MFMA, 1, r.side, r.side, r.c, r.c, r.f, r.f)
                    gt.conv2d_run(p, r.config, img, w, out, stream=stream)
            for (f, c), rs in bf16_groups.items():
                for r in rs:
                    r.config = (64, 1, 1, 1, 0, 0)
                    r.path = "batched"
                b = gt.IgemmBatch([(r.bufs[0][0], r.bufs[1], r.bufs[2][0], r.side, r.side) for r in rs], c, c, f,
                                  (f - 1) // 2)
                b.run(stream=stream)
                batches.append(b)
            for f, rs in groups.items():
                # config of the group's typical size (work-weighted mean side)
                side = math.sqrt(sum(r.side ** 2 for r in rs) / len(rs))
                cfg = autotune.lookup(self.store, f, side, self.objective)
                for r in rs:
                    r.config = cfg
                    r.path = "batched"
                b = gt.Batch([(r.bufs[0], r.bufs[1], r.bufs[2], r.side, r.side, f) for r in rs], cfg)
                b.run(stream=stream)
                batches.append(b)
            ev = torch.cuda.Event()
            ev.record(stream)
        return Step(reqs, ev, batches)

    def run(self, requests, realtime=True, poll_s=5e-5, progress=None):
        """Serve requests (sorted by t_arrive, seconds from the start).  With
        realtime=False every request is available at t = 0 (saturation)."""
        torch = self.torch
        pending = collections.deque(sorted(requests, key=lambda r: r.t_arrive))
        waiting = collections.deque()
        # launched steps per stream: a stream runs its steps in order, so only
        # the head of each queue needs polling
        inflight = [collections.deque() for _ in self.streams]
        long_jobs, long_events = [], collections.deque()
        done = []
        k = 0
        t0 = time.perf_counter()
        while pending or waiting or any(inflight) or long_jobs:
            now = time.perf_counter() - t0
            while pending and (not realtime or pending[0].t_arrive <= now):
                waiting.append(pending.popleft())
            # reap every finished step: steps on different streams finish out
            # of launch order, and a finished step must not wait for (or be
            # timed behind) a longer one launched before it on the other stream
            finished = []
            for q in inflight:
                while q and q[0].event.query():
                    finished.append(q.popleft())
            if long_jobs:
                done_long = self._retire_long(long_jobs, long_events)
                if done_long:
                    finished.append(Step(done_long, None, []))
                self._issue_long(long_jobs, long_events)
            for st in finished:
                t = time.perf_counter() - t0
                for r in st.reqs:
                    r.t_done = t
                    self.mem_used -= r.bytes
                    self.slots_used -= 1
                    if self.keep_outputs:
                        self.outputs[r.rid] = r.bufs[2]
                    r.bufs = None
                    done.append(r)
                if progress and len(done) // 500 != (len(done) - len(st.reqs)) // 500:
                    progress("served %d" % len(done))
            while waiting and waiting[0].bytes > self.mem_budget:  # can never fit: reject
                self.rejected.append(waiting.popleft())
            n = admit(waiting, self.mem_budget - self.mem_used, self.max_slots - self.slots_used, self.max_batch)
            if n:
                reqs = [waiting.popleft() for _ in range(n)]
                t = time.perf_counter() - t0
                for r in reqs:
                    r.t_admit = t
                    self.mem_used += r.bytes
                    self.slots_used += 1
                self.peak_mem = max(self.peak_mem, self.mem_used)
                short = [r for r in reqs if not self.is_long(r)]
                for r in reqs:
                    if self.is_long(r):
                        long_jobs.append(self._start_long(r))
                self._issue_long(long_jobs, long_events)
                if short:
                    si = k % len(self.streams)
                    inflight[si].append(self._launch(short, self.streams[si]))
                    k += 1
                continue
            if not any(inflight) and not long_jobs and not waiting and pending and realtime:
                time.sleep(max(0.0, min(pending[0].t_arrive - (time.perf_counter() - t0), 1e-3)))
            else:
                time.sleep(poll_s)
        torch.cuda.synchronize()
        return done


def requests_from_mix(mix, rate_scale=1.0, seed_base=1000):
    """Request objects from synthetic.serving_requests dicts; arrival times are
    multiplied by rate_scale (rate_scale < 1 compresses time)."""
    return [Request(i, m["kind"], m["side"], m["f"], m["c"], m["t_arrive"] * rate_scale, seed_base + i)
            for i, m in enumerate(mix)]


def latency_stats(done):
    lat = sorted((r.t_done - r.t_arrive) * 1e3 for r in done)
    if not lat:
        return {}

    def pct(p):
        return lat[min(len(lat) - 1, max(0, int(math.ceil(p / 100.0 * len(lat))) - 1))]
    return {"n": len(lat), "p50_ms": pct(50), "p99_ms": pct(99), "mean_ms": sum(lat) / len(lat),
            "max_ms": lat[-1]}


def energy_stats(samples, t_start, t_stop, n_req, discard_s=0.0):
    """Serving-window energy from sampler readings (host time t_s): the
    library's gt_energy_from_samples over the window [t_start, t_stop] with
    the stabilisation discard, taken as one run of n_req requests."""
    fin = [s for s in samples if s["power_w"] == s["power_w"]]
    try:
        e, med, n_used = gt.energy_from_samples([s["t_s"] for s in fin], [s["power_w"] for s in fin],
                                                t_start, t_stop, 1, discard_s)
    except gt.GreentuneError:
        return {}
    win = t_stop - t_start
    out = {"window_s": win, "discard_s": discard_s, "n_samples_used": n_used, "p_median_w": med,
           "j_per_request": e / n_req}
    kept = [s for s in samples if t_start + discard_s <= s["t_s"] <= t_stop]
    upd = [(s["energy_t_s"], s["energy_j"]) for i, s in enumerate(kept)
           if i > 0 and s["energy_t_s"] != kept[i - 1]["energy_t_s"]]
    if len(upd) >= 2 and upd[-1][0] > upd[0][0]:
        p_ctr = (upd[-1][1] - upd[0][1]) / (upd[-1][0] - upd[0][0])
        out["j_per_request_counter"] = p_ctr * win / n_req
        out["p_counter_w"] = p_ctr
    return out


def benchmark(n_req=8000, seed=0, util=0.7, mem_budget=64 << 30, discard_s=0.3, progress=print, **engine_kw):
    """The serving-mix benchmark: after one untimed pass that warms the
    device buffer pool, saturation throughput with every request queued at
    t = 0, then Poisson arrivals at util x that rate.  Energy per request is
    the median socket power over that run after a discard_s stabilisation
    prefix, times the run's length, over the requests served (section III.A-B:
    the run should last well over a second).  engine_kw go to every Engine
    (e.g. objective, bf16_batch_side).  Returns a report dict (latency
    percentiles, throughput, energy per request)."""
    import torch
    from synthetic import serving_requests
    mix = serving_requests(n_req, 1.0, seed=seed)
    # one pair of streams for every run, so the buffer pool warmed by the
    # first (untimed) pass serves the timed ones: a serving process keeps its
    # device buffers, and first-time device allocation is not request work
    streams = [torch.cuda.Stream() for _ in range(2)]
    long_stream = torch.cuda.Stream()
    Engine(mem_budget=mem_budget, streams=streams, long_stream=long_stream, **engine_kw).run(requests_from_mix(mix),
                                                                              realtime=False)
    # saturation
    eng = Engine(mem_budget=mem_budget, streams=streams, long_stream=long_stream, **engine_kw)
    reqs = requests_from_mix(mix)
    t0 = time.perf_counter()
    done = eng.run(reqs, realtime=False)
    t_sat = time.perf_counter() - t0
    if len(done) + len(eng.rejected) != len(reqs):
        raise RuntimeError("serving: %d of %d requests finished" % (len(done), len(reqs)))
    mu = len(done) / t_sat
    progress("saturation: %d requests in %.3f s (%.1f req/s)" % (len(done), t_sat, mu))
    lam = util * mu
    reqs = requests_from_mix(mix, rate_scale=1.0 / lam)
    eng = Engine(mem_budget=mem_budget, streams=streams, long_stream=long_stream, **engine_kw)
    gt.sampler_start(2.0)
    t_start = gt.sensor_read()["t_s"]
    t0 = time.perf_counter()
    done = eng.run(reqs, realtime=True)
    wall = time.perf_counter() - t0
    if len(done) + len(eng.rejected) != len(reqs):
        raise RuntimeError("serving: %d of %d requests finished" % (len(done), len(reqs)))
    t_stop = gt.sensor_read()["t_s"]
    samples = gt.sampler_stop()
    torch.cuda.synchronize()
    flops = sum(r.flops() for r in done)
    rep = {"requests": len(done), "arrival_rate_hz": lam, "saturation_rate_hz": mu, "util_target": util,
           "wall_s": wall, "throughput_rps": len(done) / wall, "tflops_delivered": flops / wall / 1e12,
           "peak_admitted_bytes": eng.peak_mem, "mem_budget_bytes": mem_budget,
           "mix": {"xcorr_f32": sum(r.kind == "xcorr_f32" for r in done),
                   "conv_bf16": sum(r.kind == "conv_bf16" for r in done)}}
    rep.update(latency=latency_stats(done),
               latency_by_kind={k: latency_stats([r for r in done if r.kind == k]) for k in ("xcorr_f32", "conv_bf16")},
               energy=energy_stats(samples, t_start, t_stop, len(done), discard_s=discard_s))
    return rep
