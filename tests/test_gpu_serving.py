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
    checked_oracle = 0
    for r in done:
        img, w, out = serving.make_payload(r, dev)
        if r.kind == "xcorr_f32":
            p = gt.xcorr_problem(r.side, r.side, r.f, r.f)
        else:
            p = gt.conv_problem(gt.IGEMM_BF16_MFMA, 1, r.side, r.side, r.c, r.c, r.f, r.f)
        gt.conv2d_run(p, r.config, img, w, out)
        torch.cuda.synchronize()
        assert torch.equal(out, eng.outputs[r.rid]), (r.rid, r.kind, r.side, r.f)
        if checked_oracle < 8 and r.side <= 64:
            if r.kind == "xcorr_f32":
                ref = oracle.xcorr2d(img.cpu().numpy(), w.cpu().numpy())
                tol = 1e-5
            else:
                pad = (r.f - 1) // 2
                ref = oracle.conv_nhwc(img.float().cpu().numpy(), w.float().cpu().numpy(), pad, pad)
                tol = 2e-2
            assert oracle.max_rel_err(out.cpu().numpy(), ref) <= tol
            checked_oracle += 1
    assert checked_oracle > 0


def test_admission_budget_forces_queueing(gt):
    serving, reqs = small_mix(40, seed=9)
    budget = max(r.bytes for r in reqs) * 3
    eng = serving.Engine(mem_budget=budget, max_batch=64)
    done = eng.run(reqs, realtime=False)
    assert len(done) == len(reqs)
    assert eng.peak_mem <= budget
    assert all(r.t_done >= r.t_admit >= 0 for r in done)
