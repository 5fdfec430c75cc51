"""A sweep's result log is append-only and resumable: a second run over the
same configs measures nothing new, and a run with other measurement
options (or another problem) does not reuse the logged rows.  Fake power
sensor; real launches and timing."""
import json

import pytest
import torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gt():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2211_07260_amd as g
    g.init(0, g.INIT_FAKE_SENSOR | g.INIT_FAKE_DVFS)
    g.fake_sensor_model(g.power_model(240.0, 0.35, 0.0012, 1250.0, 5000.0), noise_w=0.0)
    yield g
    g.shutdown()


def test_sweep_resume_and_context(gt, tmp_path):
    from paper_2211_07260_amd import tuner
    dev = torch.device("cuda:0")
    img = torch.rand(256 + 16, 256 + 16, device=dev)
    w = torch.rand(17, 17, device=dev)
    out = torch.empty(256, 256, device=dev)
    prob = gt.xcorr_problem(256, 256, 17, 17)
    cfgs = [(32, 8, 2, 2, 1, 0), (16, 16, 4, 2, 0, 0), (64, 4, 1, 4, 0, 1)]
    log = tmp_path / "sweep.jsonl"
    print("case: sweep of 3 configs, 256x256 f17, then resumed", flush=True)
    first = tuner.sweep(prob, cfgs, img, w, out, window_s=0.08, discard_s=0.02, log_path=str(log), progress_every=0)
    assert len(log.read_text().splitlines()) == 3
    again = tuner.sweep(prob, cfgs, img, w, out, window_s=0.08, discard_s=0.02, log_path=str(log), progress_every=0)
    # nothing re-measured: the same rows come back from the log
    assert [(r["config"], r["t_run_s"], r["e_run_j"]) for r in again] == \
        [(r["config"], r["t_run_s"], r["e_run_j"]) for r in first]
    assert len(log.read_text().splitlines()) == 3
    ctx = {json.loads(ln)["context"] for ln in log.read_text().splitlines()}
    assert len(ctx) == 1 and "0.08,0.02" in ctx.pop()
    # other options: measured anew and appended
    tuner.sweep(prob, cfgs[:2], img, w, out, window_s=0.1, discard_s=0.02, log_path=str(log), progress_every=0)
    assert len(log.read_text().splitlines()) == 5
    # another problem (same configs): measured anew
    img2 = torch.rand(128 + 16, 128 + 16, device=dev)
    out2 = torch.empty(128, 128, device=dev)
    tuner.sweep(gt.xcorr_problem(128, 128, 17, 17), cfgs[:1], img2, w, out2, window_s=0.08, discard_s=0.02,
                log_path=str(log), progress_every=0)
    assert len(log.read_text().splitlines()) == 6
