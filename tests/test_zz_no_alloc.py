"""The allocation-free batched launch (conv2d_run_batched_noalloc) against the
batched launch with a caller-owned descriptor blob (conv2d_run_batched): the
same kernel over the same tiles, so every output must be bit-identical.  Two
calls in a row on the library's one descriptor array, the second with fewer
and smaller convolutions, so that stale descriptors from the first call would
show."""
import ctypes
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


def make_convs(f, n, seed, max_side):
    rng = random.Random(seed)
    dev = torch.device("cuda:0")
    convs, hosts = [], []
    for k in range(n):
        oh, ow = rng.randint(1, max_side), rng.randint(1, max_side)
        img, w = xcorr_inputs(oh, ow, f, f, seed=seed * 1000 + k)
        hosts.append((img, w))
        convs.append((img.to(dev), w.to(dev), torch.full((oh, ow), float("nan"), device=dev), oh, ow, f))
    return convs, hosts


def with_outputs(convs):
    return [(di, dw, torch.full((oh, ow), float("nan"), device=di.device), oh, ow, f)
            for (di, dw, _, oh, ow, f) in convs]


# (filter, config, items, largest side): the first call spans several
# 64-descriptor upload chunks, the second is smaller in every respect
CALLS = [(5, (32, 8, 2, 2, 0, 0), 150, 260), (17, (32, 8, 4, 2, 1, 0), 37, 120)]


@pytest.mark.parametrize("grid", [0, 40])
def test_noalloc_matches_blob_launch_twice(gt, grid):
    for call, (f, cfg, n, side) in enumerate(CALLS):
        print("noalloc call %d: filter %d, %d items, side <= %d, config %s, grid %d" % (call, f, n, side, cfg, grid),
              flush=True)
        convs, hosts = make_convs(f, n, seed=11 + call, max_side=side)
        ref = with_outputs(convs)
        gt.Batch(ref, cfg).run(grid_blocks=grid)
        gt.conv2d_run_batched_noalloc(convs, cfg, grid_blocks=grid)
        torch.cuda.synchronize()
        for k, ((_, _, out, oh, ow, _), (_, _, r, _, _, _)) in enumerate(zip(convs, ref)):
            a, b = out.cpu().numpy(), r.cpu().numpy()
            assert np.array_equal(a.view(np.uint32), b.view(np.uint32)), (call, k, oh, ow)
        # and against the FP64 oracle on a few of them (bar 1e-5)
        for k in (0, n // 2, n - 1):
            img, w = hosts[k]
            err = oracle.max_rel_err(convs[k][2].cpu().numpy(), oracle.xcorr2d(img.numpy(), w.numpy()))
            assert err <= 1e-5, (call, k, err)


def test_noalloc_size_limit(gt):
    dev = torch.device("cuda:0")
    t = torch.zeros(64, device=dev)
    n = gt.BATCH_NOALLOC_MAX_ITEMS + 1
    items = (gt.BatchItem * n)()
    for k in range(n):
        items[k] = gt.BatchItem(t.data_ptr(), t.data_ptr(), t.data_ptr(), 1, 1, 3, 3)
    rc = gt.lib().conv2d_run_batched_noalloc(items, n, ctypes.byref(gt.as_config((16, 1, 1, 1, 0, 0))), 0, None)
    assert rc == gt.GT_E_INVAL
    assert "items" in gt.lib().gt_last_error().decode()


def test_noalloc_in_a_captured_graph(gt):
    """The entry point under HIP graph capture, its callers' case: the
    descriptors reach the device array through kernel arguments, so every
    replay rewrites them, also after an eager call in between has filled the
    array with another batch."""
    f, cfg = 9, (32, 8, 4, 4, 0, 0)
    convs, _ = make_convs(f, 70, seed=31, max_side=150)  # two upload chunks
    ref = with_outputs(convs)
    gt.Batch(ref, cfg).run()
    other, _ = make_convs(5, 20, seed=32, max_side=90)
    other_cfg = (32, 8, 2, 2, 0, 0)
    gt.conv2d_run_batched_noalloc(other, other_cfg)  # device address looked up before the capture
    torch.cuda.synchronize()
    side = torch.cuda.Stream()
    g = gt.Graph(lambda: gt.conv2d_run_batched_noalloc(convs, cfg, stream=side), side)
    try:
        for rep in range(3):
            print("noalloc graph replay %d" % rep, flush=True)
            for c in convs:
                c[2].fill_(float("nan"))                 # eager work between replays
            gt.conv2d_run_batched_noalloc(other, other_cfg)  # refills the descriptor array
            torch.cuda.synchronize()
            g.launch()
            side.synchronize()
            for k, (c, r) in enumerate(zip(convs, ref)):
                assert torch.equal(c[2], r[2]), (rep, k)
    finally:
        g.close()
