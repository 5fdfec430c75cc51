"""GPU tests of the continuous-batching serving loop: every request's result
is the same alone and in the mix (bit-identical with the config it ran with),
within tolerance of the FP64 oracle, and admission never exceeds the memory
budget."""
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


def small_mix(n, seed):
    from synthetic import serving_requests
    from paper_2211_07260_amd import serving
    mix = serving_requests(n, 2000.0, seed=seed, side_lo=16, side_hi=160)
    return serving, serving.requests_from_mix(mix)


def check_against_oracle(gt, serving, r, out, n_points=0, seed=0):
    """A served output against the FP64 oracle: every element, or for large
    multi-channel requests n_points random pixels (all channels each)."""
    img, w, _ = serving.make_payload(r, torch.device("cuda:0"))
    if r.kind == "xcorr_f32":
        ref = oracle.xcorr2d(img.cpu().numpy(), w.cpu().numpy())
        return oracle.max_rel_err(out.cpu().numpy(), ref), 1e-5
    pad = (r.f - 1) // 2
    x, wt = img.float().cpu().numpy(), w.float().cpu().numpy()
    got = out.cpu().numpy()
    if not n_points:
        return oracle.max_rel_err(got, oracle.conv_nhwc(x, wt, pad, pad)), 2e-2
    g = np.random.default_rng(seed)
    pts = [(0, 0, 0), (0, r.side - 1, r.side - 1), (0, 0, r.side - 1), (0, r.side - 1, 0)] + \
        [(0, int(y), int(xx)) for y, xx in g.integers(0, r.side, (n_points, 2))]
    ref = oracle.conv_nhwc_at(x, wt, pad, pad, pts)
    sub = np.stack([got[b, y, xx, :] for b, y, xx in pts])
    # normwise over the sampled pixels, scaled by the sample's largest |ref|
    return oracle.max_rel_err(sub, ref), 2e-2


@pytest.mark.parametrize("part_flops", [None, 2e8])
def test_alone_equals_mix(gt, part_flops):
    # part_flops=2e8 runs most BF16 requests of this mix in parts on the long
    # stream, interleaved with the short steps
    serving, reqs = small_mix(48, seed=7)
    eng = serving.Engine(mem_budget=1 << 30, max_batch=16, keep_outputs=True, part_flops=part_flops)
    n_long = sum(eng.is_long(r) for r in reqs)
    assert (n_long == 0) == (part_flops is None)
    done = eng.run(reqs, realtime=True)
    assert len(done) == len(reqs)
    dev = torch.device("cuda:0")
    paths = {r.path for r in done if r.kind == "conv_bf16"}
    # sides 16-160: every BF16 request is batched, unless it runs in parts
    assert paths == {"batched"} if part_flops is None else "parts" in paths
    for r in done:
        img, w, out = serving.make_payload(r, dev)
        if r.kind == "xcorr_f32":
            p = gt.xcorr_problem(r.side, r.side, r.f, r.f)
            gt.conv2d_run(p, r.config, img, w, out)
        elif r.path == "batched":  # alone: a batch of one, the same kernel
            gt.IgemmBatch([(img[0], w, out[0], r.side, r.side)], r.c, r.c, r.f, (r.f - 1) // 2).run()
        else:
            p = gt.conv_problem(gt.IGEMM_BF16_MFMA, 1, r.side, r.side, r.c, r.c, r.f, r.f)
            gt.conv2d_run(p, r.config, img, w, out)
        torch.cuda.synchronize()
        assert torch.equal(out, eng.outputs[r.rid]), (r.rid, r.kind, r.side, r.f)
        # every request of the mix against the oracle
        err, tol = check_against_oracle(gt, serving, r, eng.outputs[r.rid])
        assert err <= tol, (r.rid, r.kind, r.side, r.f, err)


def test_bench_size_mix_against_oracle(gt):
    # requests drawn as the benchmark draws them (side 128-4096, filters
    # {3,5,9,17}, 30 % BF16 C=32), served together; every single-channel
    # output is compared whole with the oracle, every BF16 one at 64 random
    # pixels plus the four corners (a 4096^2, 17x17 BF16 request is 9.9 TFLOP,
    # out of the CPU oracle's reach whole)
    from synthetic import serving_requests
    from paper_2211_07260_amd import serving
    mix = serving_requests(20, 5000.0, seed=11)
    reqs = serving.requests_from_mix(mix)
    assert max(r.side for r in reqs) > 1500 and any(r.kind == "conv_bf16" for r in reqs)
    eng = serving.Engine(mem_budget=48 << 30, keep_outputs=True)
    done = eng.run(reqs, realtime=False)
    assert len(done) == len(reqs)
    for r in done:
        print("case: serving rid=%d %s side=%d f=%d" % (r.rid, r.kind, r.side, r.f), flush=True)
        err, tol = check_against_oracle(gt, serving, r, eng.outputs[r.rid], n_points=64, seed=r.rid)
        assert err <= tol, (r.rid, r.kind, r.side, r.f, err)


def test_admission_budget_forces_queueing(gt):
    serving, reqs = small_mix(40, seed=9)
    budget = max(r.bytes for r in reqs) * 3
    eng = serving.Engine(mem_budget=budget, max_batch=64)
    done = eng.run(reqs, realtime=False)
    assert len(done) == len(reqs)
    assert eng.peak_mem <= budget
    assert all(r.t_done >= r.t_admit >= 0 for r in done)
