"""Oracle for the measurement arithmetic and objective selection (test
infrastructure only).

Section III.A: energy over an interval is the integral of power; the paper
approximates it as a representative power times the elapsed time, taking the
median power reading.  Section III.B: the observer repeats the kernel for a
window (1 s by default) because the on-board sensor refreshes at about 10 Hz
and needs about 0.3 s to settle, so readings from the start of the window are
not representative and are discarded here.  Section III.C: compute
performance is GFLOP/s and energy efficiency is GFLOPs/W, the same as GFLOP/J.
Section V.A: race-to-idle picks the fastest configuration, energy tuning the
one with the least energy.
"""
import numpy as np


def median(values):
    """Median; mean of the two middle values for an even count."""
    v = sorted(float(x) for x in values)
    n = len(v)
    if n == 0:
        raise ValueError("no samples")
    m = n // 2
    return v[m] if n % 2 else 0.5 * (v[m - 1] + v[m])


def energy_per_run(sample_t, sample_p, t_start, t_stop, n_runs, discard_s):
    """Median power of the samples taken in [t_start + discard, t_stop],
    times the time per run (t_stop - t_start) / n_runs.  Returns
    (e_run_j, p_median_w, t_run_s, n_used)."""
    kept = [p for t, p in zip(sample_t, sample_p) if t_start + discard_s <= t <= t_stop]
    pm = median(kept)
    t_run = (t_stop - t_start) / n_runs
    return pm * t_run, pm, t_run, len(kept)


def flops_xcorr(out_h, out_w, fh, fw):
    """2 flops per filter tap per output (one multiply, one add)."""
    return 2.0 * out_h * out_w * fh * fw


def flops_conv(n, out_h, out_w, c_out, c_in, fh, fw):
    """2 flops per tap, padded taps included."""
    return 2.0 * n * out_h * out_w * c_out * c_in * fh * fw


def gflops(flops, t_run):
    return flops / t_run / 1e9


def gflops_per_watt(flops, e_run):
    """GFLOP/s per W == GFLOP per J."""
    return flops / e_run / 1e9


def select(rows, objective):
    """rows: sequence of dicts with 't_run', 'e_run'; index = position.
    objective 'time': min t_run, then min e_run, then lowest index.
    objective 'energy': min e_run, then min t_run, then lowest index."""
    if objective == "time":
        key = lambda k: (rows[k]["t_run"], rows[k]["e_run"], k)  # noqa: E731
    elif objective == "energy":
        key = lambda k: (rows[k]["e_run"], rows[k]["t_run"], k)  # noqa: E731
    else:
        raise ValueError(objective)
    return min(range(len(rows)), key=key)


def pareto_front(rows):
    """Indices of rows not dominated in (GFLOP/s, GFLOP/s/W), both maximised;
    that is, (t_run, e_run) both minimised.  Brute force, O(n^2)."""
    out = []
    for i, a in enumerate(rows):
        dominated = False
        for j, b in enumerate(rows):
            if j == i:
                continue
            if (b["t_run"] <= a["t_run"] and b["e_run"] <= a["e_run"]
                    and (b["t_run"] < a["t_run"] or b["e_run"] < a["e_run"])):
                dominated = True
                break
        if not dominated:
            out.append(i)
    return out


def relative_gain_pct(before, after):
    """Percentage change (after / before - 1) * 100, as Table 2 reports it."""
    return (after / before - 1.0) * 100.0


def mean_and_sample_std(values):
    """Mean and sample (n - 1) standard deviation, the form of the paper's
    "42.0 +- 24.1 %" summary of Table 2."""
    v = np.asarray(values, dtype=np.float64)
    return float(v.mean()), float(v.std(ddof=1))


def clock_space_reduction_pct(n_band, n_full):
    """Share of clock points the band removes from the full list (section V.E)."""
    return (1.0 - n_band / n_full) * 100.0
