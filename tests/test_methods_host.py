"""The five tuning methods of the paper's experiments (race-to-idle, lowest
energy at the top clock, the two two-step methods, and the global energy
optimum; section V.A) on a simulated device (CPU): each method's choice
must equal its definition evaluated by brute force over the full (config,
clock) table with the oracle's selection rule, every (config, clock) is
measured once, and the orderings the definitions imply hold."""
import numpy as np
import pytest

import paper_2211_07260_amd as gt
from paper_2211_07260_amd import tuner
from oracle import measure as om
from oracle import power_model as opm


@pytest.fixture(scope="module", autouse=True)
def host_only():
    gt.init(0, gt.INIT_HOST_ONLY)
    yield
    gt.shutdown()


def simulated(seed, cfgs, calls):
    """Run time scales as 1/f with a per-config constant; power follows Eq. 2/3
    with a per-config scale (configs differ in both speed and power draw)."""
    rng = np.random.default_rng(seed)
    model = dict(p_idle=rng.uniform(150, 350), alpha=rng.uniform(0.25, 0.45), beta=rng.uniform(8e-4, 2e-3),
                 tau=rng.uniform(1000, 1500))
    t0 = {c: rng.uniform(1.0e-4, 1.6e-4) for c in cfgs}
    scale = {c: rng.uniform(0.85, 1.15) for c in cfgs}

    def measure(c, f):
        calls.append((tuple(c), f))
        p = scale[tuple(c)] * float(opm.power(f, model["p_idle"], model["alpha"], model["beta"], model["tau"], 1e12))
        t = t0[tuple(c)] * 2400.0 / f
        return {"t_run_s": t, "p_median_w": p, "e_run_j": p * t}
    return measure


CFGS = [(16, 16, 4, 2, 1, 0), (32, 8, 4, 4, 0, 0), (16, 16, 8, 5, 0, 0), (64, 4, 2, 2, 1, 0), (32, 16, 8, 1, 0, 0)]
CLOCKS = [float(f) for f in range(600, 2401, 150)]


def brute(rows, objective, keep):
    sub = [r for r in rows if keep(r)]
    k = om.select([{"t_run": r["t_run_s"], "e_run": r["e_run_j"]} for r in sub], objective)
    return sub[k]


@pytest.mark.parametrize("seed", range(5))
@pytest.mark.parametrize("f_base", [None, 1500.0])
def test_methods_match_definitions(seed, f_base):
    calls = []
    rep = tuner.tuning_methods(simulated(seed, CFGS, calls), CFGS, CLOCKS, f_base=f_base)
    # the measured table, in (config, clock) enumeration order
    rows = sorted(({**r, "config": tuple(r["config"])} for r in rep["rows"]),
                  key=lambda r: (CFGS.index(r["config"]), r["clock_mhz"]))
    assert len(calls) == len(set(calls)) == len(CFGS) * len(CLOCKS)  # each point measured once
    f_max = max(CLOCKS)
    f_b = f_max if f_base is None else min(CLOCKS, key=lambda f: (abs(f - f_base), f))
    assert rep["base_clock_mhz"] == f_b

    def same(got, want):
        return tuple(got["config"]) == tuple(want["config"]) and got["clock_mhz"] == want["clock_mhz"]

    assert same(rep["race_to_idle"], brute(rows, "time", lambda r: True))
    assert same(rep["global_energy_to_solution"], brute(rows, "energy", lambda r: True))
    assert same(rep["energy_to_solution_maxclock"], brute(rows, "energy", lambda r: r["clock_mhz"] == f_max))
    c_t = brute(rows, "time", lambda r: r["clock_mhz"] == f_max)["config"]
    assert same(rep["race_to_idle_clocks"], brute(rows, "energy", lambda r: r["config"] == c_t))
    c_e = brute(rows, "energy", lambda r: r["clock_mhz"] == f_b)["config"]
    assert same(rep["energy_to_solution_clocks"], brute(rows, "energy", lambda r: r["config"] == c_e))

    e = {m: rep[m]["e_run_j"] for m in tuner.METHODS}
    assert all(e["global_energy_to_solution"] <= v for v in e.values())
    # run time ~ 1/f, so the fastest point sits at the top clock and the
    # two-step method can only lower its energy
    assert rep["race_to_idle"]["clock_mhz"] == f_max
    assert e["race_to_idle_clocks"] <= e["race_to_idle"]
    assert e["energy_to_solution_maxclock"] <= e["race_to_idle"]
    n, m = len(CFGS), len(CLOCKS)
    assert rep["race_to_idle"]["points"] == rep["global_energy_to_solution"]["points"] == n * m
    assert rep["energy_to_solution_maxclock"]["points"] == n
    assert rep["race_to_idle_clocks"]["points"] == rep["energy_to_solution_clocks"]["points"] == n + m - 1


def test_single_config_and_clock():
    calls = []
    rep = tuner.tuning_methods(simulated(0, CFGS[:1], calls), CFGS[:1], [2400.0])
    for m in tuner.METHODS:
        assert tuple(rep[m]["config"]) == CFGS[0] and rep[m]["clock_mhz"] == 2400.0
    assert len(calls) == 1
