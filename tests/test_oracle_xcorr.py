"""Pins for the convolution oracle (oracle/xcorr_oracle.c via oracle.xcorr2d,
oracle.conv_nhwc).  Each test checks the oracle against something other than
itself: brute force, closed forms, invariants, or a library routine."""
import numpy as np
import pytest
import torch

import oracle
from synthetic import integer_inputs, xcorr_inputs, conv_inputs


@pytest.mark.parametrize("oh,ow,fh,fw", [(1, 1, 1, 1), (3, 5, 2, 3), (5, 4, 3, 1), (8, 8, 5, 5),
                                         (2, 7, 1, 4), (6, 3, 4, 2)])
def test_bruteforce_exact_on_integers(oh, ow, fh, fw):
    img, w = integer_inputs(oh, ow, fh, fw, seed=oh * 100 + fw)
    ref = oracle.xcorr2d_loops(img.tolist(), w.tolist())
    got = oracle.xcorr2d(img.numpy(), w.numpy())
    assert got.shape == (oh, ow)
    assert np.array_equal(got, np.array(ref))  # integer data: exact


@pytest.mark.parametrize("a,b", [(0, 0), (0, 16), (16, 0), (7, 11), (16, 16)])
def test_delta_filter_shifts_image(a, b):
    img, _ = xcorr_inputs(37, 29, 17, 17, seed=3)
    w = np.zeros((17, 17), np.float32)
    w[a, b] = 1.0
    got = oracle.xcorr2d(img.numpy(), w)
    assert np.array_equal(got, img.numpy()[a:a + 37, b:b + 29].astype(np.float64))


def test_delta_filter_catches_flip_and_transpose():
    # an asymmetric delta: a flipped or transposed implementation shifts the wrong way
    img, _ = xcorr_inputs(9, 11, 3, 5, seed=4)
    w = np.zeros((3, 5), np.float32)
    w[0, 4] = 1.0
    got = oracle.xcorr2d(img.numpy(), w)
    assert np.array_equal(got, img.numpy()[0:9, 4:15].astype(np.float64))


def test_constant_image_gives_filter_sum():
    _, w = xcorr_inputs(4, 4, 17, 17, seed=5)
    c = 0.75
    img = np.full((20 + 16, 24 + 16), c, np.float32)
    got = oracle.xcorr2d(img, w.numpy())
    want = c * float(np.sum(w.numpy().astype(np.float64)))
    np.testing.assert_allclose(got, want, rtol=1e-13, atol=0)


def test_linearity_exact_on_integers():
    x, w = integer_inputs(13, 17, 4, 6, seed=6)
    y, _ = integer_inputs(13, 17, 4, 6, seed=7)
    a, b = 3.0, -2.0
    lhs = oracle.xcorr2d((a * x + b * y).numpy(), w.numpy())
    rhs = a * oracle.xcorr2d(x.numpy(), w.numpy()) + b * oracle.xcorr2d(y.numpy(), w.numpy())
    assert np.array_equal(lhs, rhs)


def test_small_closed_form():
    # 3x3 image 1..9, filter [[1,0],[0,-1]]: out[y][x] = in[y][x] - in[y+1][x+1] = -4
    img = np.arange(1, 10, dtype=np.float32).reshape(3, 3)
    w = np.array([[1, 0], [0, -1]], np.float32)
    assert np.array_equal(oracle.xcorr2d(img, w), np.full((2, 2), -4.0))


def test_matches_scipy_correlate2d():
    signal = pytest.importorskip("scipy.signal")
    img, w = xcorr_inputs(61, 67, 17, 17, seed=8)
    ref = signal.correlate2d(img.numpy().astype(np.float64), w.numpy().astype(np.float64),
                             mode="valid")
    got = oracle.xcorr2d(img.numpy(), w.numpy())
    np.testing.assert_allclose(got, ref, rtol=1e-13, atol=1e-11)


def test_fp64_accumulation_is_not_fp32():
    # A float32 accumulator would lose the 1 added to 2^24; FP64 keeps it.
    img = np.array([[2.0 ** 24, 1.0, -2.0 ** 24]], np.float32)
    w = np.ones((1, 3), np.float32)
    assert oracle.xcorr2d(img, w)[0, 0] == 1.0


def test_threads_do_not_change_result():
    img, w = xcorr_inputs(64, 48, 17, 17, seed=9)
    a = oracle.xcorr2d(img.numpy(), w.numpy(), nthreads=1)
    b = oracle.xcorr2d(img.numpy(), w.numpy(), nthreads=4)
    assert np.array_equal(a, b)


def test_bad_sizes_raise():
    with pytest.raises(ValueError):
        oracle.xcorr2d(np.zeros((3, 3), np.float32), np.zeros((4, 1), np.float32))


# ---- multi-channel ----

def test_multichannel_reduces_to_single_channel():
    img, w = xcorr_inputs(12, 10, 3, 5, seed=10)
    x = img.numpy()[None, :, :, None]
    wt = w.numpy()[None, :, :, None]
    got = oracle.conv_nhwc(x, wt, 0, 0)[0, :, :, 0]
    assert np.array_equal(got, oracle.xcorr2d(img.numpy(), w.numpy()))


def test_multichannel_is_sum_of_padded_single_channel():
    x, wt = conv_inputs(2, 9, 11, 3, 2, 3, 5, seed=11)
    xf, wf = x.float().numpy(), wt.float().numpy()
    got = oracle.conv_nhwc(xf, wf, 1, 2)
    for n in range(2):
        for co in range(2):
            acc = np.zeros((9, 11))
            for ci in range(3):
                padded = np.pad(xf[n, :, :, ci], ((1, 1), (2, 2)))
                acc += oracle.xcorr2d(padded, wf[co, :, :, ci])
            np.testing.assert_allclose(got[n, :, :, co], acc, rtol=1e-13, atol=1e-12)


@pytest.mark.parametrize("f", [3, 5])
def test_multichannel_matches_torch_conv2d_f64(f):
    x, wt = conv_inputs(2, 16, 12, 8, 6, f, f, seed=12)
    xf, wf = x.float(), wt.float()
    ref = torch.nn.functional.conv2d(xf.double().permute(0, 3, 1, 2), wf.double().permute(0, 3, 1, 2),
                                     padding=(f - 1) // 2).permute(0, 2, 3, 1).numpy()
    got = oracle.conv_nhwc(xf.numpy(), wf.numpy(), (f - 1) // 2, (f - 1) // 2)
    np.testing.assert_allclose(got, ref, rtol=1e-12, atol=1e-11)


def test_multichannel_delta_weight_selects_channel_and_shift():
    x, _ = conv_inputs(1, 8, 8, 4, 1, 3, 3, seed=13)
    xf = x.float().numpy()
    wt = np.zeros((2, 3, 3, 4), np.float32)
    wt[0, 0, 2, 1] = 1.0   # output 0 = channel 1 shifted by (-1, +1)
    wt[1, 1, 1, 3] = 1.0   # output 1 = channel 3 unshifted
    got = oracle.conv_nhwc(xf, wt, 1, 1)
    padded = np.pad(xf[0, :, :, 1], 1)
    assert np.array_equal(got[0, :, :, 0], padded[0:8, 2:10])
    assert np.array_equal(got[0, :, :, 1], xf[0, :, :, 3].astype(np.float64))


def test_multichannel_points_brute_force_integers():
    # integer data: the sampled-pixel oracle equals a pure-Python loop of the
    # definition exactly, at interior, edge and corner pixels
    g = np.random.default_rng(3)
    x = g.integers(-3, 4, (2, 6, 7, 3)).astype(np.float32)
    wt = g.integers(-3, 4, (4, 3, 5, 3)).astype(np.float32)
    ph, pw = 1, 2
    pts = [(0, 0, 0), (1, 5, 6), (0, 2, 3), (1, 0, 6), (0, 5, 0)]
    got = oracle.conv_nhwc_at(x, wt, ph, pw, pts)
    for k, (b, y, xo) in enumerate(pts):
        for co in range(4):
            s = 0.0
            for r in range(3):
                for q in range(5):
                    yi, xi = y + r - ph, xo + q - pw
                    if 0 <= yi < 6 and 0 <= xi < 7:
                        s += sum(float(x[b, yi, xi, c]) * float(wt[co, r, q, c]) for c in range(3))
            assert got[k, co] == s


def test_multichannel_points_equal_full_and_reject_outside():
    g = np.random.default_rng(4)
    x = g.standard_normal((2, 9, 8, 5)).astype(np.float32)
    wt = g.standard_normal((3, 5, 5, 5)).astype(np.float32)
    full = oracle.conv_nhwc(x, wt, 2, 2)
    pts = [(b, y, xo) for b in range(2) for y in range(9) for xo in range(8)]
    got = oracle.conv_nhwc_at(x, wt, 2, 2, pts)
    assert np.array_equal(got, full.reshape(-1, 3))
    with pytest.raises(ValueError):
        oracle.conv_nhwc_at(x, wt, 2, 2, [(0, 9, 0)])
