"""Tuner drivers over the C ABI: sensor characterisation, exhaustive sweep of
the restricted tune space, objective selection, and the model-steered clock
search (sections III-V of the paper).

All measurement, fitting and selection arithmetic runs in the native library
(measure_time_energy, fit_power_model, gt_power_model_band, gt_select); this
module only loops, records and reports.
"""
import json
import math
import os
import time

import paper_2211_07260_amd as gt

CONV_SPACE = dict(block_size_x=[16, 32, 64, 128], block_size_y=[1, 2, 4, 8, 16],
                  tile_size_x=list(range(1, 9)), tile_size_y=list(range(1, 9)),
                  use_lds_padding=[0, 1], read_path=[0, 1])


def cfg_key(cfg):
    return ",".join(str(v) for v in gt.as_config(cfg).as_tuple())


# ---- sensor characterisation (the analog of the paper's Fig. 2 power trace) ----

def characterise_sensor(problem, cfg, d_in, d_w, d_out, idle_s=1.0, busy_s=2.5, batch=20):
    """Record sensor readings while idle, then while the kernel runs
    back-to-back.  Returns the trace and derived figures: refresh interval of
    the power reading, idle and loaded medians, and the stabilisation time
    (first time after the load starts from which the 50 ms rolling median stays
    within 3 % of the final loaded median)."""
    import torch
    trace = []
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < idle_s:
        s = gt.sensor_read()
        trace.append(("idle", time.perf_counter() - t0, s))
        time.sleep(0.0005)
    t_load = time.perf_counter() - t0
    k = 0
    while time.perf_counter() - t0 < idle_s + busy_s:
        for _ in range(batch):
            gt.conv2d_run(problem, cfg, d_in, d_w, d_out)
        k += 1
        if k % 8 == 0:
            torch.cuda.synchronize()
        s = gt.sensor_read()
        trace.append(("busy", time.perf_counter() - t0, s))
    torch.cuda.synchronize()
    pw = [(t, s["power_w"]) for ph, t, s in trace]
    changes = [pw[i][0] for i in range(1, len(pw)) if pw[i][1] != pw[i - 1][1]]
    dts = sorted(changes[i] - changes[i - 1] for i in range(1, len(changes)))
    busy = [(t, p) for (ph, t, s), (_, p) in zip(trace, pw) if ph == "busy"]
    idle = [p for (ph, t, s), (_, p) in zip(trace, pw) if ph == "idle"]
    final = sorted(p for t, p in busy if t > idle_s + busy_s - 0.5)
    p_final = final[len(final) // 2] if final else float("nan")
    # 50 ms rolling median of the loaded readings; stabilisation = first time
    # after which every rolling median stays within 3 % of the final median
    roll = []
    for i, (t, p) in enumerate(busy):
        w = sorted(q for u, q in busy[i:] if u - t < 0.05)
        roll.append((t, w[len(w) // 2]))
    stab = None
    for t, med in reversed(roll):
        if abs(med - p_final) > 0.03 * p_final:
            break
        stab = t - t_load
    return {
        "refresh_interval_s": dts[len(dts) // 2] if dts else None,
        "n_readings": len(trace), "n_changes": len(changes),
        "p_idle_median_w": sorted(idle)[len(idle) // 2] if idle else None,
        "p_load_median_w": p_final, "stabilisation_s": stab,
        "trace": [(ph, round(t, 5), s["power_w"], s["sclk_mhz"], s["temp_c"]) for ph, t, s in trace],
    }


# ---- exhaustive sweep ----

def sweep(problem, configs, d_in, d_w, d_out, clk=None, window_s=0.3, discard_s=0.1, log_path=None,
          resume=True, progress_every=50, time_only=False, repeats=20):
    """Measure every config (at one clock knob).  Rows are appended to a JSONL
    log when log_path is given; with resume, configs already in the log are
    skipped.  time_only: time with HIP events only (no sensor), for the
    performance landscape."""
    import torch
    clk_name = "default" if clk is None or clk.kind == gt.CLOCK_DEFAULT else "%d:%d" % (clk.kind, clk.value)
    # a logged row is reused only for the same device, problem and options
    ctx = "%s|%s|%s|%s" % (device_id(), ",".join(str(v) for v in problem_tuple(problem)),
                           "time_only" if time_only else "%g,%g" % (window_s, discard_s), clk_name)
    done = {}
    if log_path and resume and os.path.exists(log_path):
        with open(log_path) as fh:
            for ln in fh:
                r = json.loads(ln)
                if r.get("context", ctx) == ctx:
                    done[(r["config_key"], r.get("clock", "default"))] = r
    rows = []
    fh = open(log_path, "a") if log_path else None
    t0 = time.perf_counter()
    try:
        for i, cfg in enumerate(configs):
            key = cfg_key(cfg)
            if (key, clk_name) in done:
                rows.append(done[(key, clk_name)])
                continue
            row = {"config": list(gt.as_config(cfg).as_tuple()), "config_key": key, "clock": clk_name, "context": ctx}
            try:
                if time_only:
                    for _ in range(2):
                        gt.conv2d_run(problem, cfg, d_in, d_w, d_out, clk)
                    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                    e0.record()
                    for _ in range(repeats):
                        gt.conv2d_run(problem, cfg, d_in, d_w, d_out, clk)
                    e1.record()
                    torch.cuda.synchronize()
                    t = e0.elapsed_time(e1) * 1e-3 / repeats
                    row.update(t_run_s=t, gflops=gt.problem_flops(problem) / t * 1e-9)
                else:
                    m = gt.measure_time_energy(problem, cfg, d_in, d_w, d_out, clk, window_s=window_s,
                                               discard_s=discard_s)
                    row.update(m)
            except gt.GreentuneError as e:
                row["error"] = str(e)
                row["error_code"] = e.code
            rows.append(row)
            if fh:
                fh.write(json.dumps(row) + "\n")
                fh.flush()
            if progress_every and (i + 1) % progress_every == 0:
                ok = [r for r in rows if "error" not in r]
                best = min(ok, key=lambda r: r["t_run_s"]) if ok else None
                print("sweep %d/%d  %.0f s  best %s %.1f GFLOP/s" % (
                    i + 1, len(configs), time.perf_counter() - t0, best["config"] if best else None,
                    best["gflops"] if best else 0), flush=True)
    finally:
        if fh:
            fh.close()
    return rows


def device_id():
    """Identity of GPU 0 for result logs: its UUID where torch reports one,
    else its name and PCI bus id ("cpu" without a GPU)."""
    import torch
    if not torch.cuda.is_available():
        return "cpu"
    props = torch.cuda.get_device_properties(0)
    uuid = getattr(props, "uuid", None)
    if uuid:
        return str(uuid)
    return "%s@%s" % (props.name, getattr(props, "pci_bus_id", "?"))


def problem_tuple(problem):
    return (problem.kind, problem.n, problem.c_in, problem.c_out, problem.out_h, problem.out_w, problem.filt_h,
            problem.filt_w, problem.pad_h, problem.pad_w)


def optima(rows):
    """Time-optimal (race-to-idle) and energy-optimal rows, chosen by the
    library's gt_select (ties: the other objective, then index)."""
    ok = [r for r in rows if "error" not in r and "e_run_j" in r]
    if not ok:
        return None, None
    recs = [{"t_run_s": r["t_run_s"], "e_run_j": r["e_run_j"]} for r in ok]
    return ok[gt.select(recs, "time")], ok[gt.select(recs, "energy")]


def pareto(rows):
    """Non-dominated rows in (GFLOP/s, GFLOP/s/W) by the library's gt_pareto,
    fastest first."""
    ok = [r for r in rows if "error" not in r and "e_run_j" in r]
    front = [ok[k] for k in gt.pareto(ok)] if ok else []
    return sorted(front, key=lambda r: (r["t_run_s"], r["e_run_j"]))


# ---- model-steered clock search (section V.D) ----

def fit_clocks(settable, n=5):
    """n clocks spaced uniformly over the settable range, snapped to settable
    values (the paper samples the supported clocks uniformly)."""
    s = sorted(settable)
    lo, hi = s[0], s[-1]
    out = []
    for k in range(n):
        target = lo + (hi - lo) * k / max(n - 1, 1)
        snap = min(s, key=lambda f: (abs(f - target), f))
        if snap not in out:
            out.append(snap)
    return out


def fit_readings(measure_at, settable, p_max, n_fit=5):
    """<= n_fit power readings of one fully-loading workload and the fit of
    Eq. 2/3 to them (section V.D).  The model is fitted up to the highest
    clock before throttling, so the first reading is taken at the top clock:
    if the device throttles there, the remaining readings are spread uniformly
    below the clock it sustained instead of over the whole range.  Throttled
    readings are not fitted.  measure_at(clock_mhz) -> dict with p_median_w,
    sclk_act_mhz, throttled.  Returns (readings, PowerModel)."""
    s = sorted(settable)
    top = measure_at(s[-1])
    pts = [{"clock_mhz": s[-1], **top}]
    f_hi = s[-1]
    if top.get("throttled"):
        below = [f for f in s if f <= top.get("sclk_act_mhz", s[-1])]
        f_hi = below[-1] if below else s[0]
    for f in fit_clocks([f for f in s if f <= f_hi], n_fit - 1 if top.get("throttled") else n_fit):
        if f == s[-1]:
            continue
        pts.append({"clock_mhz": f, **measure_at(f)})
    use = [p for p in pts if not p.get("throttled")]
    model = gt.fit_power_model([p["clock_mhz"] for p in use], [p["p_median_w"] for p in use], p_max)
    return pts, model


def calibrate(kind, buf, settable, p_max, n_fit=5, window_s=1.0, discard_s=0.3):
    """Fit the power model once per GPU from <= n_fit readings of a synthetic
    full-load kernel (gt.LOAD_*), to be reused for every kernel tuned on that
    GPU (steered_search(..., model=...)): the paper's procedure of calibrating
    with a load that fully occupies the device.  buf: device scratch (>= 4 MiB)."""
    def measure_at(f):
        return gt.measure_load(kind, buf, gt.clock(gt.CLOCK_SCLK_MHZ, int(f)), window_s=window_s,
                               discard_s=discard_s)
    pts, model = fit_readings(measure_at, settable, p_max, n_fit)
    return {"kind": kind, "fit_points": pts, "model": model.as_dict()}


def pick_calibration(load_power_w, workload_power_w):
    """The synthetic load to calibrate the power model with: the paper fits
    to a load that fully occupies the device (section V.D), so a load drawing
    less power than the workload itself at the default clock cannot stand in
    for it.  Among the loads whose median power is at least the workload's,
    the one drawing the most; None when no load reaches it (calibrate with
    the workload instead).  load_power_w: {kind: watts}."""
    ok = {k: p for k, p in load_power_w.items() if p == p and p >= workload_power_w}
    if not ok:
        return None
    return max(sorted(ok), key=lambda k: ok[k])


def choose_calibration(buf, workload_measure, kinds=None, window_s=1.0, discard_s=0.3):
    """Measure the synthetic loads and the workload (workload_measure() ->
    dict with p_median_w) at the default clock, and pick the calibration load
    by pick_calibration.  Returns (kind or None, report)."""
    kinds = kinds if kinds is not None else (gt.LOAD_FP32_FMA, gt.LOAD_BF16_MFMA, gt.LOAD_COPY)
    powers = {k: gt.measure_load(k, buf, window_s=window_s, discard_s=discard_s)["p_median_w"] for k in kinds}
    p_work = workload_measure()["p_median_w"]
    kind = pick_calibration(powers, p_work)
    return kind, {"load_power_w": powers, "workload_power_w": p_work, "kind": kind}


def steered_search(measure, configs, settable, p_max, n_fit=5, rel_half=0.1, fit_config=None, model=None):
    """The paper's procedure (section V.D): fit Eq. 2/3 to <= n_fit power
    readings of one fully-loading config (fit_readings), take the clock
    minimising P*(f)/f, and measure the candidate configs only at the
    settable clocks within +-rel_half of it.  With `model` (a PowerModel or
    its as_dict(), e.g. from calibrate) no fit readings are taken.

    measure(config, clock_mhz) -> dict with t_run_s, e_run_j, p_median_w,
    sclk_act_mhz, throttled.  Returns a report dict."""
    s = sorted(settable)
    if model is None:
        fit_config = fit_config or configs[0]
        fit_pts, model = fit_readings(lambda f: measure(fit_config, f), s, p_max, n_fit)
    else:
        fit_pts = []
        if isinstance(model, dict):
            model = gt.power_model(model["p_idle"], model["alpha"], model["beta"], model["tau_mhz"], model["p_max"],
                                   literal=bool(model.get("literal_eq3", 0)))
    f_opt, band = gt.power_model_band(model, s, rel_half)
    rows = []
    for cfg in configs:
        for f in band:
            m = measure(cfg, f)
            rows.append({"config": list(gt.as_config(cfg).as_tuple()), "clock_mhz": f, **m})
    best = min(rows, key=lambda r: (r["e_run_j"], r["t_run_s"]))
    return {"fit_points": fit_pts, "model": model.as_dict(), "f_opt_mhz": f_opt, "band_mhz": band,
            "rows": rows, "best": best, "points_measured_band": len(rows),
            "points_measured_total": len(rows) + len(fit_pts)}


def exhaustive_clock_search(measure, configs, settable):
    rows = []
    for cfg in configs:
        for f in settable:
            m = measure(cfg, f)
            rows.append({"config": list(gt.as_config(cfg).as_tuple()), "clock_mhz": f, **m})
    best = min(rows, key=lambda r: (r["e_run_j"], r["t_run_s"]))
    return {"rows": rows, "best": best, "points_measured": len(rows)}


# ---- the tuning methods compared in the experiments (section V.A) ----

METHODS = ("race_to_idle", "energy_to_solution_maxclock", "race_to_idle_clocks", "energy_to_solution_clocks",
           "global_energy_to_solution")


def tuning_methods(measure, configs, settable, f_base=None):
    """The five ways of choosing a (config, clock) the paper compares:

    * race_to_idle: the fastest (config, clock) over the whole space;
    * energy_to_solution_maxclock: the lowest-energy config at the top clock;
    * race_to_idle_clocks: the fastest config at the top clock, then the
      lowest-energy clock for that config;
    * energy_to_solution_clocks: the lowest-energy config at the base clock
      f_base, then the lowest-energy clock for that config;
    * global_energy_to_solution: the lowest-energy (config, clock) overall.

    Ties go to the other objective, then to the earlier config and lower
    clock (the library's gt_select order).  Each (config, clock) is measured
    at most once and shared between methods; 'points' counts what a method
    needs on its own.  f_base defaults to the top clock (the device's default
    clock; MI355X publishes no separate base clock) and is snapped to the
    nearest settable clock.  measure(config, clock_mhz) -> dict with t_run_s
    and e_run_j.  Returns {method: {"config", "clock_mhz", "t_run_s",
    "e_run_j", ..., "points"}} plus the measured table under "rows"."""
    s = sorted(float(f) for f in settable)
    cfgs = [tuple(gt.as_config(c).as_tuple()) for c in configs]
    f_max = s[-1]
    f_b = f_max if f_base is None else min(s, key=lambda f: (abs(f - f_base), f))
    table = {}

    def get(c, f):
        key = (c, f)
        if key not in table:
            table[key] = {"config": list(c), "clock_mhz": f, **measure(c, f)}
        return table[key]

    def pick(rows, objective):
        recs = [{"t_run_s": r["t_run_s"], "e_run_j": r["e_run_j"]} for r in rows]
        return rows[gt.select(recs, objective)]

    everything = [get(c, f) for c in cfgs for f in s]
    at_max = [get(c, f_max) for c in cfgs]
    at_base = [get(c, f_b) for c in cfgs]
    c_t = tuple(pick(at_max, "time")["config"])
    c_e = tuple(pick(at_base, "energy")["config"])
    n_all, n_c, n_f = len(everything), len(cfgs), len(s)
    out = {
        "race_to_idle": dict(pick(everything, "time"), points=n_all),
        "energy_to_solution_maxclock": dict(pick(at_max, "energy"), points=n_c),
        "race_to_idle_clocks": dict(pick([get(c_t, f) for f in s], "energy"), points=n_c + n_f - 1),
        "energy_to_solution_clocks": dict(pick([get(c_e, f) for f in s], "energy"), points=n_c + n_f - 1),
        "global_energy_to_solution": dict(pick(everything, "energy"), points=n_all),
    }
    out["rows"] = list(table.values())
    out["base_clock_mhz"] = f_b
    return out


# ---- power capping versus clock tuning (section V.C) ----

def equidistant(lo, hi, n=7):
    """n equally spaced knob values from lo to hi, both included (the paper
    samples each knob's range at 7 points)."""
    if n < 2:
        return [float(hi)]
    return [lo + (hi - lo) * k / (n - 1) for k in range(n)]


def knob_search(measure, configs, knobs):
    """Every config at every knob value; the lowest-energy point (ties: time,
    then the earlier config, then the earlier knob, as gt_select orders).
    measure(config, knob) -> dict with t_run_s and e_run_j."""
    rows = []
    for cfg in configs:
        for k in knobs:
            rows.append({"config": list(gt.as_config(cfg).as_tuple()), "knob": k, **measure(cfg, k)})
    recs = [{"t_run_s": r["t_run_s"], "e_run_j": r["e_run_j"]} for r in rows]
    return {"rows": rows, "best": rows[gt.select(recs, "energy")], "points": len(rows)}


def cap_vs_clock(measure_clock, measure_cap, configs, clocks, caps):
    """Section V.C: the same configs searched once with the clock as the extra
    tunable and once with the power cap; the lowest energy each reaches.
    measure_clock(config, mhz), measure_cap(config, watts) -> dicts with
    t_run_s, e_run_j (and, for the power-versus-clock view, p_median_w and
    sclk_act_mhz)."""
    by_clock = knob_search(measure_clock, configs, clocks)
    by_cap = knob_search(measure_cap, configs, caps)
    e_clk, e_cap = by_clock["best"]["e_run_j"], by_cap["best"]["e_run_j"]
    return {"clock": by_clock, "cap": by_cap, "clocks_mhz": list(clocks), "caps_w": list(caps),
            "energy_cap_over_clock": e_cap / e_clk}


def load_power_views(kind, buf, clocks, caps, window_s=1.0, discard_s=0.3):
    """The power-versus-clock view of a synthetic full load under each knob
    (the paper's Fig. 6): for every clock limit and every power cap, the
    clock the device ran and the power it drew.  kind: gt.LOAD_*."""
    def one(clk):
        m = gt.measure_load(kind, buf, clk, window_s=window_s, discard_s=discard_s)
        return {"sclk_act_mhz": m["sclk_act_mhz"], "p_median_w": m["p_median_w"], "rate": m["gflops"]}
    return {"by_clock": [{"clock_mhz": f, **one(gt.clock(gt.CLOCK_SCLK_MHZ, int(f)))} for f in clocks],
            "by_cap": [{"cap_w": c, **one(gt.clock(gt.CLOCK_POWER_CAP_W, int(c)))} for c in caps]}


def hardware_measure(problem, d_in, d_w, d_out, window_s=1.0, discard_s=0.3):
    """measure(config, clock) over the real DVFS knob (needs privileges)."""
    def measure(cfg, f_mhz):
        return gt.measure_time_energy(problem, cfg, d_in, d_w, d_out, gt.clock(gt.CLOCK_SCLK_MHZ, f_mhz),
                                      window_s=window_s, discard_s=discard_s)
    return measure


def gain_pct(before, after):
    return (after / before - 1.0) * 100.0


def nan_to_none(obj):
    if isinstance(obj, float) and (math.isnan(obj) or math.isinf(obj)):
        return None
    if isinstance(obj, dict):
        return {k: nan_to_none(v) for k, v in obj.items()}
    if isinstance(obj, (list, tuple)):
        return [nan_to_none(v) for v in obj]
    return obj


# ---- summaries of a sweep (the tuned-config store) ----

SWEEP_CSV_FIELDS = ("block_size_x", "block_size_y", "tile_size_x", "tile_size_y", "use_lds_padding", "read_path",
                    "t_run_s", "p_median_w", "e_run_j", "e_run_counter_j", "gflops", "gflops_per_w", "sclk_act_mhz",
                    "temp_c")


def write_sweep_csv(rows, path):
    import csv
    with open(path, "w", newline="") as fh:
        w = csv.writer(fh)
        w.writerow(SWEEP_CSV_FIELDS)
        for r in rows:
            if "error" in r:
                continue
            w.writerow(list(r["config"]) + ["%.6g" % r[k] if isinstance(r[k], float) else r[k]
                                            for k in SWEEP_CSV_FIELDS[6:]])


def read_sweep_csv(path):
    import csv
    rows = []
    with open(path) as fh:
        for d in csv.DictReader(fh):
            cfg = [int(d[k]) for k in SWEEP_CSV_FIELDS[:6]]
            row = {k: float(d[k]) for k in SWEEP_CSV_FIELDS[6:]}
            row.update(config=cfg, config_key=",".join(map(str, cfg)))
            rows.append(row)
    return rows


def _pick(r):
    keys = ("t_run_s", "p_median_w", "e_run_j", "e_run_counter_j", "gflops", "gflops_per_w", "sclk_act_mhz",
            "temp_c", "window_s", "n_used")
    return {"config": r["config"], **{k: r[k] for k in keys if k in r}}


def summarize(sweep_rows, remeasure_rows=None, characterisation=None, workload=""):
    """Time- and energy-optimal configs of a sweep (objective selection by
    the library's gt_select), the same two re-measured with long windows when
    available, the energy/time trade-off, and the Pareto front."""
    t_opt, e_opt = optima(sweep_rows)
    out = {"workload": workload, "configs_measured": len([r for r in sweep_rows if "error" not in r]),
           "sweep_time_optimal": _pick(t_opt), "sweep_energy_optimal": _pick(e_opt)}
    final = remeasure_rows if remeasure_rows else [r for r in sweep_rows if "error" not in r]
    ft, fe = optima(final)
    out["time_optimal"], out["energy_optimal"] = _pick(ft), _pick(fe)
    out["efficiency_gain_energy_vs_time"] = fe["gflops_per_w"] / ft["gflops_per_w"]
    out["speed_change_energy_vs_time_pct"] = gain_pct(ft["gflops"], fe["gflops"])
    out["pareto_front"] = [{"config": r["config"], "gflops": r["gflops"], "gflops_per_w": r["gflops_per_w"]}
                           for r in pareto(sweep_rows)]
    if remeasure_rows:
        out["remeasured"] = len(remeasure_rows)
        ratios = [r["e_run_counter_j"] / r["e_run_j"] for r in remeasure_rows
                  if r.get("e_run_counter_j") == r.get("e_run_counter_j") and r.get("e_run_counter_j")]
        if ratios:
            out["energy_counter_vs_median_ratio"] = {"min": min(ratios), "max": max(ratios)}
    if characterisation:
        out["sensor"] = {k: v for k, v in characterisation.items() if k != "trace"}
    out["search_difficulty"] = search_difficulty(sweep_rows)
    return nan_to_none(out)


def search_difficulty(rows, p_values=(1.0, 1.02, 1.05, 1.1, 1.25, 1.5)):
    """Proportion of PageRank centrality of good local minima (section V.B) for
    the time and the energy objective over the measured space."""
    ok = [r for r in rows if "error" not in r and "e_run_j" in r]
    cfgs = [r["config"] for r in ok]
    out = {"p": list(p_values)}
    for name, key in (("time", "t_run_s"), ("energy", "e_run_j")):
        _, is_min, prop = gt.ffg_centrality(cfgs, [r[key] for r in ok], p_values)
        out[name] = {"local_minima": int(sum(is_min)), "proportion_of_centrality": prop}
    return out


def _main(argv=None):
    import argparse
    ap = argparse.ArgumentParser(description="summarise a sweep log into the tuned-config store")
    ap.add_argument("cmd", choices=["summarize"])
    ap.add_argument("--sweep", required=True, help="JSONL sweep log")
    ap.add_argument("--remeasure", default=None, help="JSON list of long-window re-measurements")
    ap.add_argument("--sensor", default=None, help="sensor characterisation JSON")
    ap.add_argument("--workload", default="")
    ap.add_argument("--out", required=True)
    ap.add_argument("--csv", default=None)
    a = ap.parse_args(argv)
    gt.init(0, gt.INIT_HOST_ONLY)
    rows = [json.loads(ln) for ln in open(a.sweep)]
    re = json.load(open(a.remeasure)) if a.remeasure else None
    ch = json.load(open(a.sensor)) if a.sensor else None
    s = summarize(rows, re, ch, a.workload)
    with open(a.out, "w") as fh:
        json.dump(s, fh, indent=1)
    if a.csv:
        write_sweep_csv(rows, a.csv)
    gt.shutdown()


if __name__ == "__main__":
    _main()
