"""GPU check of the calibration-load choice on the real power sensor: the
power model is fitted to a synthetic load only if that load draws at least
the power of the workload being tuned at the default clock (section V.D
fits to a load that fully occupies the device); the FMA load's operands
change every trip, so it is not an idle-looking register loop."""
import pytest
import torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gt():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2211_07260_amd as g
    g.init(0, 0)
    yield g
    g.shutdown()


def test_calibration_load_at_least_the_workload(gt):
    from paper_2211_07260_amd import tuner
    from synthetic import xcorr_inputs
    dev = torch.device("cuda:0")
    img, w = xcorr_inputs(4096, 4096, 17, 17, seed=0)
    d_in, d_w = img.to(dev), w.to(dev)
    out = torch.empty(4096, 4096, device=dev)
    prob = gt.xcorr_problem(4096, 4096, 17, 17)
    buf = torch.empty(1 << 24, dtype=torch.float32, device=dev)
    kind, rep = tuner.choose_calibration(
        buf, lambda: gt.measure_time_energy(prob, (32, 8, 4, 4, 1, 0), d_in, d_w, out, window_s=0.8, discard_s=0.3),
        window_s=0.8, discard_s=0.3)
    print("calibration:", rep, flush=True)
    assert all(p > 100.0 for p in rep["load_power_w"].values())
    if kind is not None:
        assert rep["load_power_w"][kind] >= rep["workload_power_w"]
