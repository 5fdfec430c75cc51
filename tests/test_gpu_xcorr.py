"""GPU parity of the FP32 cross-correlation kernels against the FP64 oracle,
through the C ABI.  Bar: normwise max relative error <= 1e-5; additionally
every configuration must produce bit-identical outputs (each output is one
FP32 FMA chain in the same order in every configuration)."""
import itertools
import sys

import numpy as np
import pytest
import torch

import oracle
from synthetic import xcorr_inputs

pytestmark = pytest.mark.gpu
TOL = 1e-5


@pytest.fixture(scope="module")
def gt():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2211_07260_amd as g
    g.init(0, 0)
    yield g
    g.shutdown()


def _run(gt, img, w, cfg, oh, ow, offset=0):
    fh, fw = w.shape
    dev = torch.device("cuda:0")
    if offset:
        buf = torch.empty(img.numel() + offset, dtype=torch.float32, device=dev)
        din = buf[offset:].view(img.shape)
        din.copy_(img)
    else:
        din = img.to(dev)
    dw = w.to(dev)
    out = torch.full((oh, ow), float("nan"), dtype=torch.float32, device=dev)
    gt.conv2d_run(gt.xcorr_problem(oh, ow, fh, fw), cfg, din, dw, out)
    torch.cuda.synchronize()
    return out.cpu()


def test_config0_workload(gt):
    # 256x256 output, 17x17 filter, uniform[0,1) from seed 0, one fixed config
    img, w = xcorr_inputs(256, 256, 17, 17, seed=0)
    print("case: config0 256x256 f17", flush=True)
    got = _run(gt, img, w, (32, 8, 2, 2, 1, 0), 256, 256)
    ref = oracle.xcorr2d(img.numpy(), w.numpy())
    assert oracle.max_rel_err(got.numpy(), ref) <= TOL


BLOCKS = [(16, 16), (32, 8), (64, 4), (128, 1), (16, 1), (64, 16), (32, 2), (128, 8)]


@pytest.mark.parametrize("f", [17, 9, 5, 3])
def test_all_tiles_both_paths_ragged(gt, f):
    # 61 x 67 output: several tiles and a ragged tail for every tile shape
    oh, ow = 61, 67
    img, w = xcorr_inputs(oh, ow, f, f, seed=f)
    ref = oracle.xcorr2d(img.numpy(), w.numpy())
    first = None
    k = 0
    for tx, ty in itertools.product(range(1, 9), range(1, 9)):
        for rp, pad in ((0, 0), (0, 1), (1, 0)):
            while True:  # next block shape whose LDS tile fits the device
                bx, by = BLOCKS[k % len(BLOCKS)]
                k += 1
                cfg = (bx, by, tx, ty, pad, rp)
                if gt.lds_bytes(gt.xcorr_problem(oh, ow, f, f), cfg) <= 163840:
                    break
            print("case: f=%d cfg=%s" % (f, cfg), flush=True)
            got = _run(gt, img, w, cfg, oh, ow).numpy()
            err = oracle.max_rel_err(got, ref)
            assert err <= TOL, (cfg, err)
            if first is None:
                first = got
            else:
                assert np.array_equal(got, first), cfg


@pytest.mark.parametrize("oh,ow,fh,fw", [(1, 1, 17, 17), (5, 3, 3, 3), (9, 130, 5, 17), (70, 8, 17, 3),
                                         (3, 200, 1, 9)])
def test_edge_shapes(gt, oh, ow, fh, fw):
    img, w = xcorr_inputs(oh, ow, fh, fw, seed=oh + ow)
    ref = oracle.xcorr2d(img.numpy(), w.numpy())
    for cfg in [(16, 1, 1, 1, 0, 0), (32, 8, 8, 8, 1, 0), (64, 2, 3, 5, 0, 0), (16, 4, 1, 1, 0, 1)]:
        print("case: edge %s cfg=%s" % ((oh, ow, fh, fw), cfg), flush=True)
        got = _run(gt, img, w, cfg, oh, ow).numpy()
        assert oracle.max_rel_err(got, ref) <= TOL, cfg


def test_direct_path_tile_larger_than_output_is_unsupported(gt):
    img, w = xcorr_inputs(3, 3, 3, 3)
    with pytest.raises(gt.GreentuneError) as e:
        _run(gt, img, w, (16, 1, 4, 1, 0, 1), 3, 3)
    assert e.value.code == gt.GT_E_UNSUPPORTED


def test_unsupported_filter_width_and_threads(gt):
    img, w = xcorr_inputs(8, 8, 4, 4)
    with pytest.raises(gt.GreentuneError) as e:
        _run(gt, img, w, (16, 1, 1, 1, 0, 0), 8, 8)
    assert e.value.code == gt.GT_E_UNSUPPORTED
    img, w = xcorr_inputs(8, 8, 3, 3)
    with pytest.raises(gt.GreentuneError) as e:
        _run(gt, img, w, (128, 16, 1, 1, 0, 0), 8, 8)
    assert e.value.code == gt.GT_E_UNSUPPORTED


def test_empty_problem_rejected(gt):
    t = torch.zeros(16, device="cuda:0")
    with pytest.raises(gt.GreentuneError) as e:
        gt.conv2d_run(gt.xcorr_problem(0, 4, 3, 3), (16, 1, 1, 1, 0, 0), t, t, t)
    assert e.value.code == gt.GT_E_INVAL


def test_unaligned_input_pointer(gt):
    # input offset by one float: the staging loads must fall back to 4-byte accesses
    img, w = xcorr_inputs(40, 44, 17, 17, seed=21)
    ref = oracle.xcorr2d(img.numpy(), w.numpy())
    for cfg in [(32, 4, 4, 2, 0, 0), (16, 8, 8, 1, 1, 0), (32, 2, 4, 4, 0, 1)]:
        got = _run(gt, img, w, cfg, 40, 44, offset=1).numpy()
        assert oracle.max_rel_err(got, ref) <= TOL, cfg


def test_large_lds_tile(gt):
    # > 64 KiB of LDS per workgroup (gfx950 allows 160 KiB)
    p = gt.xcorr_problem(300, 1100, 17, 17)
    cfg = (128, 4, 8, 4, 1, 0)
    assert 65536 < gt.lds_bytes(p, cfg) <= 163840
    img, w = xcorr_inputs(300, 1100, 17, 17, seed=22)
    ref = oracle.xcorr2d(img.numpy(), w.numpy())
    got = _run(gt, img, w, cfg, 300, 1100).numpy()
    assert oracle.max_rel_err(got, ref) <= TOL


def _tuned_configs():
    import json
    import os
    path = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2211_07260_amd",
                        "tuned", "xcorr_f32_4096x4096_f17.json")
    with open(path) as fh:
        t = json.load(fh)
    return [tuple(t["time_optimal"]["config"]), tuple(t["energy_optimal"]["config"])]


def test_full_size_4096(gt):
    # the benchmark workload: 4096x4096 output, 17x17 filter, whole output vs
    # the oracle, in the launch configurations the bench times (the stored
    # time- and energy-optimal configs) and a few others (looped rows, direct
    # read path)
    img, w = xcorr_inputs(4096, 4096, 17, 17, seed=0)
    ref = oracle.xcorr2d(img.numpy(), w.numpy())
    for cfg in _tuned_configs() + [(32, 8, 4, 8, 0, 0), (64, 4, 8, 4, 1, 0), (32, 8, 4, 8, 0, 1)]:
        print("case: 4096 cfg=%s" % (cfg,), flush=True)
        got = _run(gt, img, w, cfg, 4096, 4096).numpy()
        err = oracle.max_rel_err(got, ref)
        print("max rel err %.3e" % err, flush=True)
        assert err <= TOL, cfg
