"""Per-size autotuner for batched convolutions.

For each (filter size, output-side bucket) the tuner times every candidate
config of the persistent batched kernel on a batch of equal-size synthetic
convolutions (the paper's search over a restricted space, section IV,
applied per problem size), then measures time and energy (median power
times time per launch, section III.A) of the fastest candidates over a
window and keeps both the time-optimal and the energy-optimal config (the
two objectives of section V.A).  Candidate timing replays a HIP graph of the
batched launch, so no host launch gap enters the comparison.  The result is
a small config store (JSON) that the serving engine consults; lookup picks
the bucket nearest in log-size and the config for the requested objective.
"""
import itertools
import json
import math
import os

import paper_2211_07260_amd as gt

BUCKETS = (128, 256, 512, 1024, 2048, 4096)
FILTERS = (3, 5, 9, 17)
STORE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuned", "batched_configs.json")
DEFAULT = (32, 8, 4, 2, 1, 0)
OBJECTIVES = ("time", "energy")


def candidates(f, lds_limit=163840):
    out = []
    for bx, by, tx, ty, pad in itertools.product((16, 32, 64), (4, 8, 16), (1, 2, 4, 8), (1, 2, 4, 8), (0, 1)):
        if bx * by > 1024:
            continue
        w = bx * tx + f - 1
        if 4 * ((w + 3) // 4 * 4 + 4 * pad) * (by * ty + f - 1) > lds_limit:
            continue
        out.append((bx, by, tx, ty, pad, 0))
    return out


def batch_count(side):
    """Convolutions per tuning batch: about 16 M output pixels in total."""
    return max(1, (4096 * 4096) // (side * side))


def time_batch(batch, reps=5, use_graph=True):
    """Seconds per launch of a packed batch: `reps` launches captured once in
    a HIP graph and the graph replayed (or the launches issued one by one)."""
    import torch
    stream = torch.cuda.Stream()
    torch.cuda.synchronize()  # the descriptor upload was queued on the current stream
    with torch.cuda.stream(stream):
        batch.run(stream=stream)
        graph = gt.Graph(lambda: [batch.run(stream=stream) for _ in range(reps)], stream) if use_graph else None
        try:
            if graph:
                graph.launch()
            stream.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            if graph:
                graph.launch()
            else:
                for _ in range(reps):
                    batch.run(stream=stream)
            e1.record(stream)
            stream.synchronize()
        finally:
            if graph:
                graph.close()
    return e0.elapsed_time(e1) * 1e-3 / reps


def pick(records, objective):
    """Index of the best of a list of measurement dicts for an objective:
    lower time (then energy), or lower energy (then time), then the earlier
    record (the order of section V.A's selection)."""
    if objective not in OBJECTIVES:
        raise ValueError("objective must be one of %s" % (OBJECTIVES,))
    a, b = ("t_run_s", "e_run_j") if objective == "time" else ("e_run_j", "t_run_s")
    return min(range(len(records)), key=lambda i: (records[i][a], records[i][b], i))


def tune(buckets=BUCKETS, filters=FILTERS, progress=print, energy_top=8, window_s=0.4, discard_s=0.1,
         cands=None):
    """Time every candidate per (filter, bucket), then measure time and energy
    of the energy_top fastest over a window; returns the store dict with the
    time-optimal config (by the windowed time) and the energy-optimal config
    of each bucket."""
    import torch
    dev = torch.device("cuda:0")
    store = {"kind": "xcorr_f32_batched", "objectives": list(OBJECTIVES), "buckets": list(buckets),
             "energy_top": energy_top, "window_s": window_s, "discard_s": discard_s, "configs": {}}
    for f in filters:
        store["configs"][str(f)] = {}
        for side in buckets:
            n = batch_count(side)
            ins = torch.rand(n, side + f - 1, side + f - 1, device=dev)
            w = torch.rand(f, f, device=dev)
            outs = torch.empty(n, side, side, device=dev)
            convs = [(ins[k], w, outs[k], side, side, f) for k in range(n)]
            timed = []
            for cfg in (cands(f) if cands else candidates(f)):
                timed.append((time_batch(gt.Batch(convs, cfg)), cfg))
            timed.sort(key=lambda tc: tc[0])
            leaders = [cfg for _, cfg in timed[:energy_top]]
            recs = []
            for cfg in leaders:
                b = gt.Batch(convs, cfg)
                torch.cuda.synchronize()
                recs.append(b.measure(window_s=window_s, discard_s=discard_s))
            flops = 2.0 * n * side * side * f * f
            entry = {"batch": n, "candidates": len(timed), "measured": len(leaders)}
            for obj in OBJECTIVES:
                i = pick(recs, obj)
                m = recs[i]
                entry[obj] = {"config": list(leaders[i]), "t_batch_s": m["t_run_s"], "e_batch_j": m["e_run_j"],
                              "p_median_w": m["p_median_w"], "tflops": flops / m["t_run_s"] / 1e12,
                              "gflops_per_w": m["gflops_per_w"]}
            entry["config"] = entry["time"]["config"]  # the time objective's config, as before
            store["configs"][str(f)][str(side)] = entry
            progress("autotune f=%d side=%d time %s %.1f TFLOP/s %.1f GFLOP/s/W; energy %s %.1f TFLOP/s %.1f "
                     "GFLOP/s/W" % (f, side, tuple(entry["time"]["config"]), entry["time"]["tflops"],
                                    entry["time"]["gflops_per_w"], tuple(entry["energy"]["config"]),
                                    entry["energy"]["tflops"], entry["energy"]["gflops_per_w"]))
            del ins, outs, convs
    return store


def save(store, path=STORE):
    with open(path, "w") as fh:
        json.dump(store, fh, indent=1)


def load(path=STORE):
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        return json.load(fh)


def lookup(store, f, side, objective="time"):
    """Config for filter f and output side: the bucket nearest in log-size,
    the config stored for the objective (a store tuned for time only has the
    time config, used for either)."""
    if objective not in OBJECTIVES:
        raise ValueError("objective must be one of %s" % (OBJECTIVES,))
    if not store or str(f) not in store["configs"]:
        return DEFAULT
    table = store["configs"][str(f)]
    b = min((int(k) for k in table), key=lambda k: (abs(math.log(k) - math.log(max(side, 1))), k))
    e = table[str(b)]
    if objective in e:
        return tuple(e[objective]["config"])
    return tuple(e["config"])


def time_bucket(f, side, reps=50, store=None, objective="time"):
    """Time the stored config of one (filter, side) bucket on its tuning batch
    (about 16 M output pixels of equal-size convolutions), as one persistent
    launch per repetition.  Returns a dict with the config, ms per launch and
    TFLOP/s."""
    import torch
    dev = torch.device("cuda:0")
    cfg = lookup(store if store is not None else load(), f, side, objective)
    n = batch_count(side)
    ins = torch.rand(n, side + f - 1, side + f - 1, device=dev)
    w = torch.rand(f, f, device=dev)
    outs = torch.empty(n, side, side, device=dev)
    b = gt.Batch([(ins[k], w, outs[k], side, side, f) for k in range(n)], cfg)
    t = time_batch(b, reps)
    flops = 2.0 * n * side * side * f * f
    return {"filter": f, "side": side, "batch": n, "config": list(cfg), "objective": objective, "ms": t * 1e3,
            "tflops": flops / t / 1e12}


def time_bf16_batch(f, side, c=32, reps=50):
    """Time one batched BF16 multi-channel launch (IgemmBatch) over a batch
    of equal-size requests of about 1 M output pixels in total (N = 1 each,
    c input and output channels, same padding), as one persistent launch per
    repetition.  Returns a dict with the batch size, ms per launch and
    TFLOP/s."""
    import torch
    dev = torch.device("cuda:0")
    n = max(1, (1024 * 1024) // (side * side))
    x = torch.randn(n, side, side, c, device=dev).to(torch.bfloat16)
    w = torch.randn(n, c, f, f, c, device=dev).to(torch.bfloat16)
    o = torch.empty(n, side, side, c, device=dev)
    b = gt.IgemmBatch([(x[k], w[k], o[k], side, side) for k in range(n)], c, c, f, (f - 1) // 2)
    t = time_batch(b, reps)
    return {"filter": f, "side": side, "c": c, "batch": n, "ms": t * 1e3, "tflops": b.flops() / t / 1e12}


if __name__ == "__main__":
    import argparse
    ap = argparse.ArgumentParser(description="per-size autotuner for the batched launch")
    ap.add_argument("--time", nargs=2, type=int, metavar=("FILTER", "SIDE"),
                    help="time the stored config of one bucket instead of tuning")
    ap.add_argument("--bf16-time", nargs=2, type=int, metavar=("FILTER", "SIDE"),
                    help="time a batched BF16 multi-channel launch (C=32) of equal-size requests instead")
    ap.add_argument("--objective", choices=OBJECTIVES, default="time")
    ap.add_argument("--reps", type=int, default=50)
    ap.add_argument("--filters", type=str, default=None, help="comma-separated subset of the filter sizes")
    ap.add_argument("--out", type=str, default=STORE)
    args = ap.parse_args()
    gt.init(0, 0)
    if args.bf16_time:
        print(json.dumps(time_bf16_batch(args.bf16_time[0], args.bf16_time[1], reps=args.reps)), flush=True)
    elif args.time:
        print(json.dumps(time_bucket(args.time[0], args.time[1], args.reps, objective=args.objective)), flush=True)
    else:
        filters = tuple(int(v) for v in args.filters.split(",")) if args.filters else FILTERS
        save(tune(filters=filters, progress=lambda m: print(m, flush=True)), args.out)
    gt.shutdown()
