"""GPU tests of the batched multi-channel BF16 launch (many convolutions of
one shape family in one persistent launch on the matrix cores): every
convolution of a mixed-size batch is bit-identical to the global-load MFMA
kernel run on it alone, and within the BF16 bar of the FP64 oracle; a
captured graph replays to the same outputs."""
import random

import numpy as np
import pytest
import torch

import oracle
from synthetic import conv_inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gt():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2211_07260_amd as g
    g.init(0, 0)
    yield g
    g.shutdown()


def unaligned_out(n_floats, dev):
    """A float tensor whose data pointer is 4 bytes past a 16-byte boundary:
    conv2d_run then takes the global-load MFMA kernel (the LDS-staged kernel
    needs 16-byte aligned output)."""
    base = torch.full((n_floats + 4,), float("nan"), device=dev)
    v = base[1:1 + n_floats]
    assert v.data_ptr() % 16 == 4
    return base, v


def make(c_in, c_out, f, n, seed, max_side):
    rng = random.Random(seed)
    dev = torch.device("cuda:0")
    convs, hosts = [], []
    for k in range(n):
        oh, ow = rng.randint(1, max_side), rng.randint(1, max_side)
        x, wt = conv_inputs(1, oh, ow, c_in, c_out, f, f, seed=seed * 1000 + k)
        hosts.append((x, wt, oh, ow))
        convs.append((x[0].to(dev).contiguous(), wt.to(dev).contiguous(),
                      torch.full((oh, ow, c_out), float("nan"), device=dev), oh, ow))
    return convs, hosts


@pytest.mark.parametrize("c_in,c_out,f,n,side", [(32, 32, 3, 40, 90), (32, 32, 5, 25, 70), (32, 32, 9, 12, 60),
                                                 (32, 32, 17, 6, 50), (64, 64, 3, 20, 80), (64, 64, 7, 8, 40),
                                                 (32, 64, 1, 30, 100)])
def test_batched_matches_single_global_kernel_and_oracle(gt, c_in, c_out, f, n, side):
    print("igemm batch: c_in %d c_out %d filter %d, %d items, side <= %d" % (c_in, c_out, f, n, side), flush=True)
    convs, hosts = make(c_in, c_out, f, n, seed=7 + f + c_in, max_side=side)
    pad = (f - 1) // 2
    b = gt.IgemmBatch(convs, c_in, c_out, f, pad)
    b.run()
    torch.cuda.synchronize()
    worst = 0.0
    for k, ((di, dw, do, oh, ow), (x, wt, _, _)) in enumerate(zip(convs, hosts)):
        p = gt.conv_problem(gt.IGEMM_BF16_MFMA, 1, oh, ow, c_in, c_out, f, f)
        base, single = unaligned_out(oh * ow * c_out, di.device)
        gt.conv2d_run(p, (64, 1, 1, 1, 0, 0), di, dw, single)
        torch.cuda.synchronize()
        a = do.cpu().numpy()
        s = single.cpu().numpy().reshape(oh, ow, c_out)
        assert np.array_equal(a.view(np.uint32), s.view(np.uint32)), (k, oh, ow)
        ref = oracle.conv_nhwc(x.float().numpy(), wt.float().numpy(), pad, pad)[0]
        err = oracle.max_rel_err(a, ref)
        worst = max(worst, err)
        assert err <= 2e-2, (k, err)
    print("worst normwise error vs FP64 oracle: %.3e" % worst, flush=True)


def test_batched_graph_replay(gt):
    print("igemm batch: graph replay, c 32 filter 5", flush=True)
    convs, hosts = make(32, 32, 5, 16, seed=99, max_side=64)
    b = gt.IgemmBatch(convs, 32, 32, 5, 2)
    b.run()
    torch.cuda.synchronize()
    eager = [do.clone() for (_, _, do, _, _) in convs]
    stream = torch.cuda.Stream()
    g = gt.Graph(lambda: b.run(stream=stream), stream)
    try:
        for rep in range(3):
            for (_, _, do, _, _) in convs:
                do.fill_(float("nan"))  # eager work between the replays
            torch.cuda.synchronize()
            g.launch()
            stream.synchronize()
            for k, (_, _, do, _, _) in enumerate(convs):
                assert torch.equal(do, eager[k]), (rep, k)
    finally:
        g.close()


def test_batch_pack_rejects(gt):
    dev = torch.device("cuda:0")
    # buffers large enough for every shape below: the library, not the
    # binding's extent check, is what refuses these shapes
    x = torch.zeros(8 * 8 * 64, dtype=torch.bfloat16, device=dev)
    w = torch.zeros(64 * 3 * 3 * 64, dtype=torch.bfloat16, device=dev)
    o = torch.zeros(8 * 8 * 64, device=dev)
    with pytest.raises(gt.GreentuneError) as e:
        gt.IgemmBatch([(x, w, o, 8, 8)], 48, 32, 3, 1)      # c_in not instantiated
    assert e.value.code == gt.GT_E_UNSUPPORTED
    with pytest.raises(gt.GreentuneError) as e:
        gt.IgemmBatch([(x, w, o, 8, 8)], 32, 40, 3, 1)      # c_out not a multiple of 32
    assert e.value.code == gt.GT_E_UNSUPPORTED
    with pytest.raises(gt.GreentuneError) as e:
        gt.IgemmBatch([(x, w, o, 1, 1)], 32, 32, 3, 2)      # padding larger than the input allows
    assert e.value.code == gt.GT_E_INVAL
