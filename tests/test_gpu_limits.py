"""GPU parity at the largest sizes the kernels index with 32-bit element
offsets: an FP32 cross-correlation whose input holds just under 2^31
elements (8.5 GB), and a BF16 implicit GEMM whose input holds just under
2^31 elements (4.3 GB in, 8.6 GB out), each checked against the FP64 oracle
on sampled outputs (corners, last rows and columns, random points), and the
sizes one step past the limit refused by the library before any launch."""
import ctypes
import random

import numpy as np
import pytest
import torch

import oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gt():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2211_07260_amd as g
    g.init(0, 0)
    yield g
    g.shutdown()


def sample_points(h, w, n, seed):
    rng = random.Random(seed)
    pts = {(0, 0), (0, w - 1), (h - 1, 0), (h - 1, w - 1), (h - 1, w // 2), (h // 2, w - 1)}
    while len(pts) < n:
        pts.add((rng.randrange(h), rng.randrange(w)))
    return sorted(pts)


@pytest.mark.parametrize("cfg", [(32, 8, 4, 4, 0, 0), (64, 4, 4, 2, 0, 1)])
def test_xcorr_near_the_32bit_limit(gt, cfg):
    oh = ow = 46000
    f = 3
    ih, iw = oh + f - 1, ow + f - 1
    assert ih * iw < 1 << 31 < (46341 + f - 1) ** 2
    dev = torch.device("cuda:0")
    g = torch.Generator(device=dev).manual_seed(5)
    img = torch.rand(ih, iw, generator=g, device=dev)
    w = torch.rand(f, f, generator=g, device=dev)
    out = torch.full((oh, ow), float("nan"), device=dev)
    print("case: xcorr %dx%d f%d config %s" % (oh, ow, f, cfg), flush=True)
    gt.conv2d_run(gt.xcorr_problem(oh, ow, f, f), cfg, img, w, out)
    torch.cuda.synchronize()
    wh = w.cpu().numpy()
    for (y, x) in sample_points(oh, ow, 40, seed=1):
        win = img[y:y + f, x:x + f].cpu().numpy()
        ref = oracle.xcorr2d(win, wh)[0, 0]
        got = float(out[y, x].item())
        assert abs(got - ref) <= 1e-5 * abs(ref), (y, x, got, ref)
    del img, out
    torch.cuda.empty_cache()


def test_xcorr_past_the_limit_is_refused(gt):
    t = torch.zeros(16, device="cuda:0")
    p = gt.xcorr_problem(46341, 46341, 3, 3)
    cfg = gt.as_config((32, 8, 4, 4, 0, 0))
    rc = gt.lib().conv2d_run(ctypes.byref(p), ctypes.byref(cfg), gt.clock(), ctypes.c_void_p(t.data_ptr()),
                             ctypes.c_void_p(t.data_ptr()), ctypes.c_void_p(t.data_ptr()), None)
    assert rc == gt.GT_E_INVAL and "32-bit" in gt.lib().gt_last_error().decode()


def test_igemm_near_the_32bit_limit(gt):
    side, c, f = 5792, 64, 3
    assert side * side * c < 1 << 31 < (side + 1) * (side + 1) * c
    dev = torch.device("cuda:0")
    g = torch.Generator(device=dev).manual_seed(6)
    x = torch.randn(1, side, side, c, generator=g, device=dev).to(torch.bfloat16)
    wt = torch.randn(c, f, f, c, generator=g, device=dev).to(torch.bfloat16)
    out = torch.full((1, side, side, c), float("nan"), device=dev)
    print("case: igemm bf16 %dx%d C=%d f%d" % (side, side, c, f), flush=True)
    gt.conv2d_run(gt.Problem(gt.IGEMM_BF16_MFMA, 1, c, c, side, side, f, f, 1, 1), (64, 1, 1, 1, 0, 0), x, wt, out)
    torch.cuda.synchronize()
    wh = wt.float().cpu().numpy()
    for (y, xx) in sample_points(side, side, 24, seed=2):
        # the 3x3 input window of this output pixel, zero where it overhangs the image
        win = np.zeros((1, f, f, c), dtype=np.float32)
        y0, y1, x0, x1 = max(y - 1, 0), min(y + 2, side), max(xx - 1, 0), min(xx + 2, side)
        win[0, y0 - (y - 1):y1 - (y - 1), x0 - (xx - 1):x1 - (xx - 1)] = x[0, y0:y1, x0:x1].float().cpu().numpy()
        ref = oracle.conv_nhwc(win, wh, 0, 0)[0, 0, 0]
        got = out[0, y, xx].cpu().numpy()
        assert oracle.max_rel_err(got, ref) <= 2e-2, (y, xx)
    del x, out
    torch.cuda.empty_cache()


def test_igemm_past_the_limit_is_refused(gt):
    t = torch.zeros(16, device="cuda:0")
    side = 5793
    p = gt.Problem(gt.IGEMM_BF16_MFMA, 1, 64, 64, side, side, 3, 3, 1, 1)
    cfg = gt.as_config((64, 1, 1, 1, 0, 0))
    rc = gt.lib().conv2d_run(ctypes.byref(p), ctypes.byref(cfg), gt.clock(), ctypes.c_void_p(t.data_ptr()),
                             ctypes.c_void_p(t.data_ptr()), ctypes.c_void_p(t.data_ptr()), None)
    assert rc == gt.GT_E_INVAL and "32-bit" in gt.lib().gt_last_error().decode()
