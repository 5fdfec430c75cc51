"""GPU parity of the multi-channel implicit-GEMM convolutions against the FP64
oracle, through the C ABI.  Inputs are BF16 values (N(0,1) rounded); the
FP32 VALU path consumes the same values widened to FP32.  Bars: normwise max
relative error <= 2e-2 for the BF16 MFMA path and <= 1e-5 for the FP32 path
(both accumulate in FP32 over exactly representable products, so both land
near 1e-7 in practice)."""
import numpy as np
import pytest
import torch

import oracle
from synthetic import conv_inputs

pytestmark = pytest.mark.gpu
TOL = {1: 2e-2, 2: 1e-5}


@pytest.fixture(scope="module")
def gt():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2211_07260_amd as g
    g.init(0, 0)
    yield g
    g.shutdown()


def run(gt, kind, x, wt, pad):
    n, h, w, ci = x.shape
    co, fh, fw, _ = wt.shape
    dev = torch.device("cuda:0")
    if kind == gt.IGEMM_BF16_MFMA:
        dx, dw = x.to(dev).contiguous(), wt.to(dev).contiguous()
    else:
        dx, dw = x.float().to(dev).contiguous(), wt.float().to(dev).contiguous()
    oh, ow = h + 2 * pad - fh + 1, w + 2 * pad - fw + 1
    out = torch.full((n, oh, ow, co), float("nan"), dtype=torch.float32, device=dev)
    p = gt.Problem(kind, n, ci, co, oh, ow, fh, fw, pad, pad)
    gt.conv2d_run(p, (64, 1, 1, 1, 0, 0), dx, dw, out)
    torch.cuda.synchronize()
    return out.cpu().numpy()


CASES = [  # n, h, w, c_in, c_out, f
    (2, 9, 13, 64, 64, 3), (1, 16, 16, 64, 64, 5), (3, 7, 11, 32, 32, 3), (2, 12, 10, 32, 64, 5),
    (1, 5, 37, 64, 32, 1), (1, 8, 9, 64, 128, 7), (1, 3, 3, 32, 32, 5), (2, 20, 17, 64, 64, 3),
    (1, 20, 23, 32, 32, 9), (1, 18, 19, 32, 32, 17), (1, 12, 40, 64, 64, 9), (2, 9, 9, 32, 64, 17),
    # three 32-channel blocks along c_out (c_out not a multiple of 64), and filter sizes without an
    # unrolled instance (the runtime-size kernels)
    (1, 20, 30, 64, 96, 3), (2, 13, 70, 32, 96, 5), (1, 11, 17, 32, 32, 11), (1, 9, 21, 64, 64, 13),
]


@pytest.mark.parametrize("kind", [1, 2])
@pytest.mark.parametrize("case", CASES)
def test_igemm_parity_ragged(gt, kind, case):
    n, h, w, ci, co, f = case
    if kind == 2 and co % 64:
        pytest.skip("FP32 VALU path: c_out % 64 == 0 only")
    x, wt = conv_inputs(n, h, w, ci, co, f, f, seed=sum(case))
    pad = (f - 1) // 2
    ref = oracle.conv_nhwc(x.float().numpy(), wt.float().numpy(), pad, pad)
    print("case:", kind, case, flush=True)
    got = run(gt, kind, x, wt, pad)
    err = oracle.max_rel_err(got, ref)
    print("max rel err %.3e" % err, flush=True)
    assert err <= TOL[kind]


def test_igemm_valid_padding_zero(gt):
    # pad 0: output shrinks by f-1 (both kinds)
    x, wt = conv_inputs(1, 12, 14, 64, 64, 3, 3, seed=5)
    ref = oracle.conv_nhwc(x.float().numpy(), wt.float().numpy(), 0, 0)
    for kind in (1, 2):
        got = run(gt, kind, x, wt, 0)
        assert got.shape == ref.shape
        assert oracle.max_rel_err(got, ref) <= TOL[kind]


@pytest.mark.parametrize("f", [3, 5])
def test_igemm_full_size(gt, f):
    # benchmark shape: N=16, C=64, K=64, 128x128, same padding; every output of
    # all 16 images, both paths
    x, wt = conv_inputs(16, 128, 128, 64, 64, f, f, seed=0)
    pad = (f - 1) // 2
    ref = oracle.conv_nhwc(x.float().numpy(), wt.float().numpy(), pad, pad)
    for kind in (1, 2):
        print("case: full f=%d kind=%d" % (f, kind), flush=True)
        got = run(gt, kind, x, wt, pad)
        assert np.isfinite(got).all()
        for b in range(16):
            err = oracle.max_rel_err(got[b:b + 1], ref[b:b + 1])
            assert err <= TOL[kind], (b, err)
        print("max rel err %.3e" % oracle.max_rel_err(got, ref), flush=True)


# Shapes with more tiles than the 256-CU device holds at once, so persistent
# workgroups run several tiles each, including runs that cross from one
# column strip (or image) to the next, ragged right and bottom tiles, each
# weight placement (all in LDS, one slab double-buffered, read from L2),
# both workgroup heights (four and eight output rows) and two channel groups
# per workgroup (3x3 with c_out = 64, both channel counts).
PERSISTENT_CASES = [  # n, h, w, c_in, c_out, f
    (4, 150, 250, 64, 64, 3), (3, 146, 190, 64, 64, 5), (3, 146, 190, 32, 64, 9), (3, 146, 190, 64, 64, 7),
    (3, 146, 190, 64, 64, 9), (3, 146, 190, 64, 32, 7), (3, 146, 190, 32, 64, 3), (2, 61, 200, 64, 128, 3),
]


@pytest.mark.parametrize("case", PERSISTENT_CASES)
def test_igemm_persistent_runs(gt, case):
    n, h, w, ci, co, f = case
    x, wt = conv_inputs(n, h, w, ci, co, f, f, seed=7 + f)
    pad = (f - 1) // 2
    ref = oracle.conv_nhwc(x.float().numpy(), wt.float().numpy(), pad, pad)
    print("case: persistent", case, flush=True)
    got = run(gt, gt.IGEMM_BF16_MFMA, x, wt, pad)
    err = oracle.max_rel_err(got, ref)
    print("max rel err %.3e" % err, flush=True)
    assert np.isfinite(got).all()
    assert err <= TOL[1]


def test_igemm_unaligned_output(gt):
    # an output that is not 16-byte aligned takes the global-load kernel (4-byte stores)
    x, wt = conv_inputs(1, 20, 30, 64, 64, 3, 3, seed=21)
    ref = oracle.conv_nhwc(x.float().numpy(), wt.float().numpy(), 1, 1)
    dev = torch.device("cuda:0")
    dx, dw = x.to(dev).contiguous(), wt.to(dev).contiguous()
    buf = torch.full((1 + 20 * 30 * 64,), float("nan"), dtype=torch.float32, device=dev)
    out = buf[1:].view(1, 20, 30, 64)
    assert out.data_ptr() % 16 != 0
    gt.conv2d_run(gt.Problem(gt.IGEMM_BF16_MFMA, 1, 64, 64, 20, 30, 3, 3, 1, 1), (64, 1, 1, 1, 0, 0), dx, dw, out)
    torch.cuda.synchronize()
    assert torch.isnan(buf[:1]).all()
    assert oracle.max_rel_err(out.cpu().numpy(), ref) <= TOL[1]


def test_igemm_unsupported(gt):
    x, wt = conv_inputs(1, 8, 8, 48, 64, 3, 3)
    with pytest.raises(gt.GreentuneError) as e:
        run(gt, 1, x, wt, 1)
    assert e.value.code == gt.GT_E_UNSUPPORTED
    x, wt = conv_inputs(1, 8, 8, 64, 32, 3, 3)
    with pytest.raises(gt.GreentuneError) as e:
        run(gt, 2, x, wt, 1)
    assert e.value.code == gt.GT_E_UNSUPPORTED


PART_CASES = [  # n, h, w, c_in, c_out, f: several tiles, ragged rows and strips
    (2, 40, 70, 64, 64, 3), (1, 33, 130, 32, 32, 17), (3, 20, 66, 64, 32, 5), (1, 8, 9, 64, 128, 7)]


@pytest.mark.parametrize("case", PART_CASES)
@pytest.mark.parametrize("n_parts", [1, 2, 3, 7, 1000])
def test_parts_equal_the_whole_run(gt, case, n_parts):
    # every part once, in reverse order: bit-identical to one conv2d_run, and
    # more parts than tiles leaves some parts empty
    n, h, w, ci, co, f = case
    x, wt = conv_inputs(n, h, w, ci, co, f, f, seed=sum(case) + n_parts)
    dev = torch.device("cuda:0")
    dx, dw = x.to(dev).contiguous(), wt.to(dev).contiguous()
    pad = (f - 1) // 2
    p = gt.conv_problem(gt.IGEMM_BF16_MFMA, n, h, w, ci, co, f, f)
    whole = torch.empty(n, h, w, co, dtype=torch.float32, device=dev)
    gt.conv2d_run(p, (64, 1, 1, 1, 0, 0), dx, dw, whole)
    parts = torch.full_like(whole, float("nan"))
    print("case:", case, "parts:", n_parts, flush=True)
    for k in reversed(range(n_parts)):
        gt.conv2d_run_part(p, (64, 1, 1, 1, 0, 0), k, n_parts, dx, dw, parts)
    torch.cuda.synchronize()
    assert torch.equal(parts, whole)
    ref = oracle.conv_nhwc(x.float().numpy(), wt.float().numpy(), pad, pad)
    assert oracle.max_rel_err(parts.cpu().numpy(), ref) <= TOL[1]


def test_parts_argument_errors(gt):
    x, wt = conv_inputs(1, 8, 8, 64, 64, 3, 3, seed=3)
    dev = torch.device("cuda:0")
    out = torch.empty(1, 8, 8, 64, dtype=torch.float32, device=dev)
    p = gt.conv_problem(gt.IGEMM_BF16_MFMA, 1, 8, 8, 64, 64, 3, 3)
    for part, n_parts in ((2, 2), (-1, 3), (0, 0)):
        with pytest.raises(gt.GreentuneError) as e:
            gt.conv2d_run_part(p, (64, 1, 1, 1, 0, 0), part, n_parts, x.to(dev), wt.to(dev), out)
        assert e.value.code == gt.GT_E_INVAL
    pf = gt.conv_problem(gt.IGEMM_F32_VALU, 1, 8, 8, 64, 64, 3, 3)
    with pytest.raises(gt.GreentuneError) as e:
        gt.conv2d_run_part(pf, (64, 1, 1, 1, 0, 0), 0, 2, x.float().to(dev), wt.float().to(dev), out)
    assert e.value.code == gt.GT_E_UNSUPPORTED


@pytest.mark.parametrize("f", [3, 5])
def test_parts_full_size(gt, f):
    # the benchmark's multi-channel workload (N=16, 128x128, C=64) in 7 parts on
    # two streams: bit-identical to the whole run
    x, wt = conv_inputs(16, 128, 128, 64, 64, f, f, seed=0)
    dev = torch.device("cuda:0")
    dx, dw = x.to(dev).contiguous(), wt.to(dev).contiguous()
    p = gt.conv_problem(gt.IGEMM_BF16_MFMA, 16, 128, 128, 64, 64, f, f)
    whole = torch.empty(16, 128, 128, 64, dtype=torch.float32, device=dev)
    gt.conv2d_run(p, (64, 1, 1, 1, 0, 0), dx, dw, whole)
    parts = torch.full_like(whole, float("nan"))
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    torch.cuda.synchronize()
    for k in range(7):
        gt.conv2d_run_part(p, (64, 1, 1, 1, 0, 0), k, 7, dx, dw, parts, stream=streams[k % 2])
    torch.cuda.synchronize()
    assert torch.equal(parts, whole)


@pytest.mark.parametrize("case", [(3, 146, 190, 64, 64, 3), (2, 61, 200, 64, 128, 3), (3, 146, 190, 64, 64, 5),
                                  (2, 40, 70, 64, 128, 5)])
def test_rows_per_tile_variants(gt, case):
    """tile_size_y = 4 or 8 picks the LDS-staged instance with that many
    output rows per tile (two 32-channel groups of four rows or one 64-channel
    group of eight for 3x3; 64 channels of four rows or 32 of eight for 5x5):
    both match the oracle and, accumulating in the same order, each other
    bit for bit; any other value is the default instance."""
    n, h, w, ci, co, f = case
    x, wt = conv_inputs(n, h, w, ci, co, f, f, seed=40 + f)
    pad = (f - 1) // 2
    ref = oracle.conv_nhwc(x.float().numpy(), wt.float().numpy(), pad, pad)
    dev = torch.device("cuda:0")
    dx, dw = x.to(dev).contiguous(), wt.to(dev).contiguous()
    p = gt.Problem(gt.IGEMM_BF16_MFMA, n, ci, co, h, w, f, f, pad, pad)
    outs = {}
    for rows in (4, 8, 1):
        print("case: rows", rows, case, flush=True)
        out = torch.full((n, h, w, co), float("nan"), dtype=torch.float32, device=dev)
        gt.conv2d_run(p, (64, 1, 1, rows, 0, 0), dx, dw, out)
        torch.cuda.synchronize()
        outs[rows] = out.cpu().numpy()
        assert oracle.max_rel_err(outs[rows], ref) <= TOL[1], rows
    assert np.array_equal(outs[4].view(np.uint32), outs[8].view(np.uint32))
    assert np.array_equal(outs[1].view(np.uint32), outs[4].view(np.uint32))
