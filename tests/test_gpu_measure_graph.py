"""Measurement of graph-replayed launches and of whole batches, and the
per-size autotuner's two objectives, on the GPU with the fake power sensor
(synthetic power from a known Eq. 2 model; real launches and HIP-event
timing): a measurement window of graph replays counts whole groups of
launches, leaves the output the kernel computes, and prices energy as the
model's power times the time per launch; a batch's measurement uses the
batch's flop count; the autotuner stores a time- and an energy-optimal
config that follow section V.A's selection over its measured leaders."""
import numpy as np
import pytest
import torch

import oracle
from synthetic import xcorr_inputs

pytestmark = pytest.mark.gpu

MODEL = dict(p_idle=240.0, alpha=0.35, beta=0.0012, tau=1250.0, p_max=5000.0)


@pytest.fixture(scope="module")
def gt():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2211_07260_amd as g
    g.init(0, g.INIT_FAKE_SENSOR | g.INIT_FAKE_DVFS)
    g.fake_sensor_model(g.power_model(MODEL["p_idle"], MODEL["alpha"], MODEL["beta"], MODEL["tau"], MODEL["p_max"]),
                        noise_w=0.0)
    yield g
    g.shutdown()


def _model_power(gt, f_mhz):
    m = gt.power_model(MODEL["p_idle"], MODEL["alpha"], MODEL["beta"], MODEL["tau"], MODEL["p_max"])
    return gt.power_model_eval(m, f_mhz)


@pytest.mark.parametrize("stream_kind", ["default", "side"])
def test_graph_window_small_problem(gt, stream_kind):
    # 256 x 256 output, 17 x 17 filter: a kernel of a few microseconds, where
    # host launch gaps matter
    print("graph window, 256x256 f17, stream %s" % stream_kind, flush=True)
    img, w = xcorr_inputs(256, 256, 17, 17, seed=0)
    dev = torch.device("cuda:0")
    di, dw = img.to(dev), w.to(dev)
    out = torch.full((256, 256), float("nan"), device=dev)
    prob = gt.xcorr_problem(256, 256, 17, 17)
    cfg = (32, 8, 2, 2, 1, 0)
    stream = torch.cuda.Stream() if stream_kind == "side" else None
    kw = dict(window_s=0.25, discard_s=0.05, stream=stream)
    plain = gt.measure_time_energy(prob, cfg, di, dw, out, **kw)
    graph = gt.measure_time_energy(prob, cfg, di, dw, out, use_graph=True, **kw)
    torch.cuda.synchronize()
    for r in (plain, graph):
        assert r["launches"] >= 10 and r["t_run_s"] > 0
        assert r["t_run_s"] == pytest.approx(r["window_s"] / r["launches"], rel=1e-12)
        assert r["gflops"] == pytest.approx(gt.problem_flops(prob) / r["t_run_s"] / 1e9, rel=1e-12)
        # fake sensor at the default clock (2400 MHz in the fake DVFS backend)
        assert r["p_median_w"] == pytest.approx(_model_power(gt, 2400.0), rel=1e-12)
        assert r["e_run_j"] == pytest.approx(r["p_median_w"] * r["t_run_s"], rel=1e-12)
    # a replayed group is at least as dense as launches one by one (allow noise)
    assert graph["t_run_s"] <= plain["t_run_s"] * 1.15
    err = oracle.max_rel_err(out.cpu().numpy(), oracle.xcorr2d(img.numpy(), w.numpy()))
    assert err <= 1e-5


def test_batch_measure(gt):
    print("batch measure, 40 convolutions f5", flush=True)
    rng = np.random.default_rng(5)
    dev = torch.device("cuda:0")
    convs, hosts = [], []
    for k in range(40):
        oh, ow = int(rng.integers(50, 300)), int(rng.integers(50, 300))
        img, w = xcorr_inputs(oh, ow, 5, 5, seed=500 + k)
        hosts.append((img, w))
        convs.append((img.to(dev), w.to(dev), torch.full((oh, ow), float("nan"), device=dev), oh, ow, 5))
    b = gt.Batch(convs, (32, 8, 4, 4, 0, 0))
    torch.cuda.synchronize()
    flops = sum(2.0 * oh * ow * 25 for (_, _, _, oh, ow, _) in convs)
    assert b.flops() == flops
    for use_graph in (False, True):
        r = b.measure(window_s=0.25, discard_s=0.05, use_graph=use_graph)
        assert r["gflops"] == pytest.approx(flops / r["t_run_s"] / 1e9, rel=1e-12)
        assert r["gflops_per_w"] == pytest.approx(flops / r["e_run_j"] / 1e9, rel=1e-12)
        assert r["p_median_w"] == pytest.approx(_model_power(gt, 2400.0), rel=1e-12)
    torch.cuda.synchronize()
    for k in (0, 17, 39):
        img, w = hosts[k]
        assert oracle.max_rel_err(convs[k][2].cpu().numpy(), oracle.xcorr2d(img.numpy(), w.numpy())) <= 1e-5


def test_autotune_two_objectives(gt):
    from paper_2211_07260_amd import autotune
    print("autotune: filter 3, bucket 128, 6 candidates", flush=True)
    cands = lambda f: autotune.candidates(f)[:6]
    st = autotune.tune(buckets=(128,), filters=(3,), progress=lambda m: print(m, flush=True), energy_top=3,
                       window_s=0.2, discard_s=0.05, cands=cands)
    e = st["configs"]["3"]["128"]
    assert e["candidates"] == 6 and e["measured"] == 3
    assert tuple(e["time"]["config"]) in cands(3) and tuple(e["energy"]["config"]) in cands(3)
    assert e["config"] == e["time"]["config"]
    # each objective's choice is the best of the measured leaders for it
    assert e["time"]["t_batch_s"] <= e["energy"]["t_batch_s"]
    assert e["energy"]["e_batch_j"] <= e["time"]["e_batch_j"]
    assert autotune.lookup(st, 3, 128, "energy") == tuple(e["energy"]["config"])
