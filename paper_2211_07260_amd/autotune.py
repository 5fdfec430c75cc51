"""Per-size autotuner for batched convolutions.

For each (filter size, output-side bucket) the tuner times every candidate
config of the persistent batched kernel on a batch of equal-size synthetic
convolutions and keeps the fastest (the paper's search over a restricted
space, section IV, applied per problem size).  The result is a small config
store (JSON) that the serving engine consults; lookup picks the bucket
nearest in log-size.
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


def time_batch(batch, reps=5):
    import torch
    batch.run()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        batch.run()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) * 1e-3 / reps


def tune(buckets=BUCKETS, filters=FILTERS, progress=print):
    """Time every candidate per (filter, bucket); returns the store dict."""
    import torch
    dev = torch.device("cuda:0")
    store = {"kind": "xcorr_f32_batched", "objective": "time", "buckets": list(buckets), "configs": {}}
    for f in filters:
        store["configs"][str(f)] = {}
        for side in buckets:
            n = batch_count(side)
            ins = torch.rand(n, side + f - 1, side + f - 1, device=dev)
            w = torch.rand(f, f, device=dev)
            outs = torch.empty(n, side, side, device=dev)
            convs = [(ins[k], w, outs[k], side, side, f) for k in range(n)]
            best = None
            for cfg in candidates(f):
                b = gt.Batch(convs, cfg)
                t = time_batch(b)
                if best is None or t < best[0]:
                    best = (t, cfg)
            flops = 2.0 * n * side * side * f * f
            store["configs"][str(f)][str(side)] = {"config": list(best[1]), "t_batch_s": best[0], "batch": n,
                                                   "tflops": flops / best[0] / 1e12}
            progress("autotune f=%d side=%d best %s %.1f TFLOP/s" % (f, side, best[1], flops / best[0] / 1e12))
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


def lookup(store, f, side):
    """Config for filter f and output side: the bucket nearest in log-size."""
    if not store or str(f) not in store["configs"]:
        return DEFAULT
    table = store["configs"][str(f)]
    b = min((int(k) for k in table), key=lambda k: (abs(math.log(k) - math.log(max(side, 1))), k))
    return tuple(table[str(b)]["config"])


def time_bucket(f, side, reps=50, store=None):
    """Time the stored config of one (filter, side) bucket on its tuning batch
    (about 16 M output pixels of equal-size convolutions), as one persistent
    launch per repetition.  Returns a dict with the config, ms per launch and
    TFLOP/s."""
    import torch
    dev = torch.device("cuda:0")
    cfg = lookup(store if store is not None else load(), f, side)
    n = batch_count(side)
    ins = torch.rand(n, side + f - 1, side + f - 1, device=dev)
    w = torch.rand(f, f, device=dev)
    outs = torch.empty(n, side, side, device=dev)
    b = gt.Batch([(ins[k], w, outs[k], side, side, f) for k in range(n)], cfg)
    t = time_batch(b, reps)
    flops = 2.0 * n * side * side * f * f
    return {"filter": f, "side": side, "batch": n, "config": list(cfg), "ms": t * 1e3, "tflops": flops / t / 1e12}


if __name__ == "__main__":
    import argparse
    ap = argparse.ArgumentParser(description="per-size autotuner for the batched launch")
    ap.add_argument("--time", nargs=2, type=int, metavar=("FILTER", "SIDE"),
                    help="time the stored config of one bucket instead of tuning")
    ap.add_argument("--reps", type=int, default=50)
    args = ap.parse_args()
    gt.init(0, 0)
    if args.time:
        print(json.dumps(time_bucket(args.time[0], args.time[1], args.reps)), flush=True)
    else:
        save(tune())
    gt.shutdown()
