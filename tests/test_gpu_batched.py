"""GPU tests of the persistent batched launch and graph replay: every
convolution of a mixed-size batch is bit-identical to its one-launch result
with the same config, and within 1e-5 of the FP64 oracle; a captured graph
replays to the same outputs."""
import random

import numpy as np
import pytest
import torch

import oracle
from synthetic import xcorr_inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gt():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2211_07260_amd as g
    g.init(0, 0)
    yield g
    g.shutdown()


def make_batch(f, n, seed, max_side=300):
    rng = random.Random(seed)
    dev = torch.device("cuda:0")
    convs, hosts = [], []
    for k in range(n):
        oh, ow = rng.randint(1, max_side), rng.randint(1, max_side)
        img, w = xcorr_inputs(oh, ow, f, f, seed=seed * 1000 + k)
        hosts.append((img, w))
        convs.append((img.to(dev), w.to(dev), torch.full((oh, ow), float("nan"), device=dev), oh, ow, f))
    return convs, hosts


@pytest.mark.parametrize("f,cfg", [(17, (32, 8, 4, 2, 1, 0)), (9, (16, 16, 2, 4, 0, 0)), (5, (64, 4, 8, 1, 0, 0)),
                                   (3, (32, 4, 1, 8, 1, 0))])
def test_batched_equals_single_launch(gt, f, cfg):
    convs, hosts = make_batch(f, 37, seed=f)
    print("case: batched f=%d cfg=%s" % (f, cfg), flush=True)
    b = gt.Batch(convs, cfg)
    b.run()
    torch.cuda.synchronize()
    for k, (di, dw, do, oh, ow, _) in enumerate(convs):
        single = torch.empty_like(do)
        gt.conv2d_run(gt.xcorr_problem(oh, ow, f, f), cfg, di, dw, single)
        torch.cuda.synchronize()
        assert torch.equal(do, single), k
        if k < 6:
            ref = oracle.xcorr2d(hosts[k][0].numpy(), hosts[k][1].numpy())
            assert oracle.max_rel_err(do.cpu().numpy(), ref) <= 1e-5


@pytest.mark.parametrize("grid", [7, 16, 24])
def test_batched_small_grid_strides(gt, grid):
    # a grid far smaller than the tile count: every workgroup walks many tiles
    # (7: one stride over the whole list; 16, 24: per-XCD contiguous eighths)
    convs, hosts = make_batch(17, 9, seed=3)
    cfg = (32, 4, 4, 4, 0, 0)
    b = gt.Batch(convs, cfg)
    print("case: batched grid=%d" % grid, flush=True)
    b.run(grid_blocks=grid)
    torch.cuda.synchronize()
    for k, (di, dw, do, oh, ow, f) in enumerate(convs):
        ref = oracle.xcorr2d(hosts[k][0].numpy(), hosts[k][1].numpy())
        assert oracle.max_rel_err(do.cpu().numpy(), ref) <= 1e-5


def test_graph_replay(gt):
    convs, _ = make_batch(5, 20, seed=11)
    cfg = (32, 8, 4, 4, 1, 0)
    b = gt.Batch(convs, cfg)
    b.run()
    torch.cuda.synchronize()
    eager = [c[2].clone() for c in convs]
    side = torch.cuda.Stream()
    g = gt.Graph(lambda: b.run(stream=side), side)
    try:
        for rep in range(3):
            for c in convs:
                c[2].zero_()           # eager work between replays
            torch.cuda.synchronize()
            g.launch()
            side.synchronize()
            for k, c in enumerate(convs):
                assert torch.equal(c[2], eager[k]), (rep, k)
    finally:
        g.close()


def test_batch_rejects_mixed_filters(gt):
    convs, _ = make_batch(5, 2, seed=1)
    convs2, _ = make_batch(3, 1, seed=2)
    with pytest.raises(gt.GreentuneError):
        gt.Batch(convs + convs2, (32, 8, 4, 4, 0, 0))
    with pytest.raises(gt.GreentuneError):
        gt.Batch(convs, (32, 8, 3, 4, 0, 0))  # tile 3 not instantiated for batching
