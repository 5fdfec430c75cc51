"""Property tests of the oracles over generated shapes and values
(Hypothesis): the cross-correlation against its brute-force definition and
its algebraic properties, the multi-channel convolution against the
single-channel one, and the power model's monotonicity and band."""
import numpy as np
from hypothesis import given, settings, strategies as st

import oracle
from oracle import power_model as opm

SETTINGS = settings(max_examples=40, deadline=None)


@st.composite
def xcorr_case(draw):
    fh = draw(st.integers(1, 6))
    fw = draw(st.integers(1, 6))
    oh = draw(st.integers(1, 9))
    ow = draw(st.integers(1, 9))
    seed = draw(st.integers(0, 2**31 - 1))
    rng = np.random.default_rng(seed)
    img = rng.integers(-8, 9, size=(oh + fh - 1, ow + fw - 1)).astype(np.float32)
    w = rng.integers(-8, 9, size=(fh, fw)).astype(np.float32)
    return img, w


@SETTINGS
@given(xcorr_case())
def test_xcorr_equals_its_definition(case):
    # integer data: every product and partial sum is exact in FP64
    img, w = case
    assert np.array_equal(oracle.xcorr2d(img, w), oracle.xcorr2d_loops(img, w))


@SETTINGS
@given(xcorr_case(), st.integers(-3, 3), st.integers(-3, 3))
def test_xcorr_is_bilinear(case, a, b):
    img, w = case
    rng = np.random.default_rng(int(abs(img).sum()))
    img2 = rng.integers(-8, 9, size=img.shape).astype(np.float32)
    w2 = rng.integers(-8, 9, size=w.shape).astype(np.float32)
    lhs = oracle.xcorr2d((a * img + b * img2).astype(np.float32), w)
    assert np.array_equal(lhs, a * oracle.xcorr2d(img, w) + b * oracle.xcorr2d(img2, w))
    lhs = oracle.xcorr2d(img, (a * w + b * w2).astype(np.float32))
    assert np.array_equal(lhs, a * oracle.xcorr2d(img, w) + b * oracle.xcorr2d(img, w2))


@SETTINGS
@given(xcorr_case())
def test_xcorr_delta_at_every_tap_shifts(case):
    img, w = case
    fh, fw = w.shape
    oh, ow = img.shape[0] - fh + 1, img.shape[1] - fw + 1
    for i in range(fh):
        for j in range(fw):
            d = np.zeros_like(w)
            d[i, j] = 1.0
            assert np.array_equal(oracle.xcorr2d(img, d), img[i:i + oh, j:j + ow].astype(np.float64))


@SETTINGS
@given(st.integers(1, 3), st.integers(1, 7), st.integers(1, 7), st.integers(1, 3), st.integers(1, 3),
       st.sampled_from([1, 3, 5]), st.integers(0, 2**31 - 1))
def test_conv_is_sum_of_single_channel_xcorrs(n, h, w_, ci, co, f, seed):
    rng = np.random.default_rng(seed)
    x = rng.integers(-4, 5, size=(n, h, w_, ci)).astype(np.float32)
    wt = rng.integers(-4, 5, size=(co, f, f, ci)).astype(np.float32)
    p = (f - 1) // 2
    got = oracle.conv_nhwc(x, wt, p, p)
    for b in range(n):
        for k in range(co):
            ref = sum(oracle.xcorr2d(np.pad(x[b, :, :, c], p), wt[k, :, :, c]) for c in range(ci))
            assert np.array_equal(got[b, :, :, k], ref)


@SETTINGS
@given(st.floats(0, 400), st.floats(0.01, 1.0), st.floats(0, 5e-3), st.floats(500, 2400), st.floats(300, 3000))
def test_power_model_nondecreasing_and_capped(p_idle, alpha, beta, tau, p_max):
    f = np.linspace(100.0, 3000.0, 400)
    p = opm.power(f, p_idle, alpha, beta, tau, p_max)
    assert np.all(np.diff(p) >= -1e-9 * p_max) and np.all(p <= p_max)


@SETTINGS
@given(st.floats(0, 400), st.floats(0.05, 1.0), st.floats(1e-4, 5e-3), st.floats(600, 2200),
       st.sampled_from([5.0, 25.0, 100.0]))
def test_band_brackets_the_optimum(p_idle, alpha, beta, tau, step):
    m = dict(p_idle=p_idle, alpha=alpha, beta=beta, tau=tau, p_max=1e9)
    settable = list(np.arange(500.0, 2400.0 + 1e-9, step))
    f_opt = opm.optimal_clock(settable, m)
    band = opm.clock_band(settable, f_opt, 0.1)
    assert f_opt in band and all(0.9 * f_opt - 1e-9 <= f <= 1.1 * f_opt + 1e-9 for f in band)
    e = [opm.energy_estimate(f, m) for f in settable]
    assert opm.energy_estimate(f_opt, m) <= min(e) * (1 + 1e-12)


@SETTINGS
@given(st.floats(50, 400), st.floats(0.05, 1.0), st.floats(0, 5e-3), st.floats(600, 2200),
       st.floats(500, 3000), st.sampled_from([5.0, 25.0, 100.0]))
def test_optimum_is_a_held_clock(p_idle, alpha, beta, tau, p_max, step):
    # f* never lies above the throttling clock while some settable clock does
    # not, and no held clock has a lower P*(f)/f
    m = dict(p_idle=p_idle, alpha=alpha, beta=beta, tau=tau, p_max=p_max)
    settable = list(np.arange(500.0, 2400.0 + 1e-9, step))
    f_thr = opm.throttle_clock(m)
    f_opt = opm.optimal_clock(settable, m)
    held = [f for f in settable if f <= f_thr]
    if not held:
        assert f_opt == settable[0]
        return
    assert f_opt in held
    e = lambda f: float(opm.power(f, p_idle, alpha, beta, tau, p_max)) / f  # noqa: E731
    assert all(e(f_opt) <= e(f) * (1 + 1e-12) for f in held)
