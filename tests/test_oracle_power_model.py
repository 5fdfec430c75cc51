"""Pins for the power-model oracle (oracle/power_model.py): values of Eq. 2 /
Eq. 3 worked by hand, closed forms of the energy optimum, exact recovery of
known parameters, and a brute-force grid for the least-squares fit."""
import numpy as np
import pytest

from oracle import power_model as pm

M = dict(p_idle=100.0, alpha=0.2, beta=0.001, tau=1000.0, p_max=2000.0)


def P(f, **kw):
    m = dict(M, **kw)
    return float(pm.power(f, m["p_idle"], m["alpha"], m["beta"], m["tau"], m["p_max"]))


def test_eq2_eq3_hand_values():
    # below tau: v = 1 -> 100 + 0.2*800 = 260
    assert P(800.0) == pytest.approx(260.0, rel=1e-15)
    # at tau: v = 1 (continuous reading) -> 100 + 0.2*1000 = 300
    assert P(1000.0) == pytest.approx(300.0, rel=1e-15)
    # above: v = 1 + 0.001*500 = 1.5 -> 100 + 0.2*1500*2.25 = 775
    assert P(1500.0) == pytest.approx(775.0, rel=1e-15)
    # clipped: 100 + 0.2*2400*(2.4)^2 = 2864.8 -> P_max 2000
    assert P(2400.0) == pytest.approx(2000.0, rel=1e-15)


def test_literal_eq3_is_discontinuous_at_tau():
    v_lo = float(pm.voltage(999.999, 0.001, 1000.0, literal=True))
    v_at = float(pm.voltage(1000.0, 0.001, 1000.0, literal=True))
    assert v_lo == 1.0 and v_at == 0.0
    v_at_cont = float(pm.voltage(1000.0, 0.001, 1000.0))
    assert v_at_cont == 1.0


def test_beta_zero_gives_race_to_idle():
    # beta = 0: E*(f) = P_idle/f + alpha decreases -> f* = f_max
    m = dict(M, beta=0.0)
    settable = np.arange(500.0, 2401.0, 25.0)
    assert pm.optimal_clock(settable, m) == 2400.0


def test_optimum_at_or_above_tau():
    settable = np.arange(300.0, 2401.0, 5.0)
    f_opt = pm.optimal_clock(settable, M)
    assert f_opt >= M["tau"]


def test_interior_optimum_solves_stationarity():
    # For f > tau and unclipped: d/df (P_idle/f + alpha*v^2) = 0
    #   <=> P_idle / f^2 = 2 * alpha * beta * (1 + beta*(f - tau))
    from scipy.optimize import brentq
    m = dict(p_idle=2000.0, alpha=0.15, beta=0.002, tau=900.0, p_max=1e9)
    g = lambda f: m["p_idle"] / f ** 2 - 2 * m["alpha"] * m["beta"] * (1 + m["beta"] * (f - m["tau"]))  # noqa: E731
    assert g(m["tau"]) > 0  # the optimum lies strictly above tau
    root = brentq(g, m["tau"], 5000.0)
    settable = np.arange(500.0, 2500.0, 0.01)
    f_opt = pm.optimal_clock(settable, m)
    assert abs(f_opt - root) <= 0.011


def test_flat_tie_goes_to_highest_clock():
    # P_idle = 0: E* = alpha below tau (flat) and rises above -> highest flat clock = tau
    m = dict(p_idle=0.0, alpha=0.5, beta=0.01, tau=1200.0, p_max=1e9)
    settable = np.arange(500.0, 2001.0, 100.0)
    assert pm.optimal_clock(settable, m) == 1200.0


def test_throttle_clock_closed_form():
    # M: 100 + 0.2 f (1 + 0.001 (f - 1000))^2 = 2000 above tau.  With u = f/1000:
    # 0.2*1000 u (u)^2 = 1900 -> u^3 = 9.5 -> f = 1000 * 9.5^(1/3)
    f_thr = pm.throttle_clock(M)
    assert f_thr == pytest.approx(1000.0 * 9.5 ** (1.0 / 3.0), rel=1e-12)
    assert pm.throttle_clock(dict(M, beta=0.0, p_max=1e12)) == float("inf")


def test_clipping_region_energy_is_flat_at_throttle():
    # above the throttling clock the device runs at f_thr and P_max
    f_thr = pm.throttle_clock(M)
    e = pm.energy_estimate(np.array([2300.0, 2400.0, f_thr]), M)
    np.testing.assert_allclose(e, 2000.0 / f_thr, rtol=1e-12)


def test_optimum_never_above_throttle():
    # a cheap top clock under the clip must not look optimal: P_max / f would
    # decrease past f_thr if the clock were assumed to hold
    m = dict(p_idle=320.0, alpha=0.37, beta=0.00115, tau=1020.0, p_max=1400.0)
    settable = np.arange(500.0, 2401.0, 10.0)
    f_opt = pm.optimal_clock(settable, m)
    assert f_opt <= pm.throttle_clock(m)
    # and it is the interior stationary point found on a fine grid
    grid = np.arange(500.0, 2400.0, 0.5)
    e = pm.energy_estimate(grid, m)
    assert abs(f_opt - grid[np.argmin(e)]) <= 10.0


def test_beta_zero_with_throttling_picks_largest_held_clock():
    # beta = 0: E*(f) = P_idle/f + alpha falls with f, but the model reaches
    # P_max at f_thr = (P_max - P_idle)/alpha = 2200 MHz exactly; the device
    # cannot hold a clock above it, so f* is the largest settable clock <= 2200
    m = dict(p_idle=300.0, alpha=0.5, beta=0.0, tau=1000.0, p_max=1400.0)
    assert pm.throttle_clock(m) == pytest.approx(2200.0, rel=1e-12)
    assert pm.optimal_clock(np.arange(500.0, 2401.0, 25.0), m) == 2200.0
    settable = np.arange(500.0, 2401.0, 30.0)  # ... 2180, 2210, ...
    f_opt = pm.optimal_clock(settable, m)
    assert f_opt == 2180.0
    # the band is centred there: [1962, 2398]
    assert pm.clock_band(settable, f_opt) == [f for f in settable if 1962.0 <= f <= 2398.0]


def test_throttle_plateau_optimum_from_the_cubic():
    # P_idle 300, alpha 0.55, beta 5e-5, tau 1500, P_max 1400 (a full load at
    # the socket cap).  With v = a + beta f, a = 1 - beta tau, the throttling
    # clock is the real root of the cubic
    #   alpha beta^2 f^3 + 2 alpha a beta f^2 + alpha a^2 f + P_idle - P_max = 0
    m = dict(p_idle=300.0, alpha=0.55, beta=5e-5, tau=1500.0, p_max=1400.0)
    a = 1.0 - m["beta"] * m["tau"]
    roots = np.roots([m["alpha"] * m["beta"] ** 2, 2 * m["alpha"] * a * m["beta"], m["alpha"] * a * a,
                      m["p_idle"] - m["p_max"]])
    f_thr = max(r.real for r in roots if abs(r.imag) < 1e-9 and r.real > m["tau"])
    assert f_thr == pytest.approx(1918.8, abs=0.1)
    assert pm.throttle_clock(m) == pytest.approx(f_thr, rel=1e-9)
    # dE*/df = -P_idle/f^2 + 2 alpha beta v(f) is still negative at f_thr (its
    # zero lies near 2290 MHz), so E* falls all the way to the throttling clock
    assert -m["p_idle"] / f_thr ** 2 + 2 * m["alpha"] * m["beta"] * (a + m["beta"] * f_thr) < 0
    settable = np.arange(500.0, 2401.0, 25.0)
    f_opt = pm.optimal_clock(settable, m)
    assert f_opt == 1900.0 and f_opt <= f_thr
    assert pm.clock_band(settable, f_opt) == [f for f in settable if 1710.0 <= f <= 2090.0]


def test_all_clocks_throttle_gives_lowest_clock():
    # P_max below the power at the lowest settable clock: nothing can be held
    m = dict(p_idle=300.0, alpha=0.5, beta=0.0, tau=1000.0, p_max=400.0)  # f_thr = 200
    assert pm.optimal_clock(np.arange(500.0, 2401.0, 100.0), m) == 500.0


def test_band_closed_form():
    settable = np.arange(100.0, 2401.0, 100.0)
    assert pm.clock_band(settable, 1500.0) == [1400.0, 1500.0, 1600.0]
    # endpoints are inclusive: 0.9*1000 = 900, 1.1*1000 = 1100
    assert pm.clock_band(settable, 1000.0) == [900.0, 1000.0, 1100.0]
    # clamped to the settable range
    assert pm.clock_band(settable, 2400.0) == [2200.0, 2300.0, 2400.0]


def _synthetic(f, m):
    return pm.power(f, m["p_idle"], m["alpha"], m["beta"], m["tau"], m["p_max"])


@pytest.mark.parametrize("m", [
    dict(p_idle=180.0, alpha=0.12, beta=0.0012, tau=1350.0, p_max=5000.0),
    dict(p_idle=90.0, alpha=0.08, beta=0.0020, tau=1100.0, p_max=5000.0),
])
def test_fit_recovers_known_parameters_noise_free(m):
    f = np.linspace(500.0, 2400.0, 9)
    p = _synthetic(f, m)
    r = pm.fit(f, p, m["p_max"])
    for k in ("p_idle", "alpha", "beta"):
        assert r[k] == pytest.approx(m[k], rel=1e-6), k
    assert r["tau"] == pytest.approx(m["tau"], rel=1e-6)
    assert r["sse"] < 1e-12


def test_fit_five_points_recovers():
    m = dict(p_idle=150.0, alpha=0.1, beta=0.0015, tau=1000.0, p_max=5000.0)
    f = np.array([500.0, 975.0, 1450.0, 1925.0, 2400.0])
    p = _synthetic(f, m)
    r = pm.fit(f, p, m["p_max"])
    assert r["sse"] < 1e-10
    # identifiable: 2 points at or below tau fix (P_idle, alpha), 3 above fix (beta, tau)
    assert r["p_idle"] == pytest.approx(150.0, rel=1e-5)
    assert r["alpha"] == pytest.approx(0.1, rel=1e-5)


def test_fit_noisy_not_worse_than_bruteforce_grid():
    rng = np.random.default_rng(0)
    m = dict(p_idle=200.0, alpha=0.15, beta=0.0010, tau=1500.0, p_max=5000.0)
    f = np.linspace(600.0, 2400.0, 7)
    p = _synthetic(f, m) + rng.normal(0.0, 5.0, f.size)
    r = pm.fit(f, p, m["p_max"])
    # independent brute force: dense 4-D grid around the truth
    best = np.inf
    for pi in np.linspace(150, 250, 21):
        for al in np.linspace(0.10, 0.20, 21):
            for b in np.linspace(0.0, 0.002, 21):
                for t in np.linspace(1200, 1800, 25):
                    v = np.where(f >= t, 1 + b * (f - t), 1.0)
                    res = p - np.minimum(m["p_max"], pi + al * f * v * v)
                    best = min(best, float(res @ res))
    assert r["sse"] <= best * (1 + 1e-9)


def test_fit_with_measured_voltage_is_linear_least_squares():
    f = np.array([600.0, 1000.0, 1400.0, 1800.0, 2200.0])
    v = np.array([0.70, 0.70, 0.78, 0.90, 1.05])
    p = 120.0 + 0.3 * f * v * v
    r = pm.fit(f, p, 1e9, v=v)
    assert r["p_idle"] == pytest.approx(120.0, rel=1e-9)
    assert r["alpha"] == pytest.approx(0.3, rel=1e-9)


# ---- covariance of the fitted parameters ----

def test_covariance_measured_voltage_is_simple_regression():
    # with measured voltage Eq. 2 is P = P_idle + alpha * g, g = f v^2: the
    # covariance is that of simple linear regression, whose textbook scalar
    # forms are var(slope) = s^2 / Sxx, var(intercept) = s^2 (1/n + gbar^2 /
    # Sxx), cov = -gbar s^2 / Sxx, with Sxx = sum (g - gbar)^2
    rng = np.random.default_rng(3)
    f = np.array([600.0, 1000.0, 1400.0, 1800.0, 2200.0])
    v = np.array([0.70, 0.72, 0.80, 0.92, 1.05])
    p = 120.0 + 0.3 * f * v * v + rng.normal(0, 5.0, f.size)
    m = pm.fit(f, p, 1e9, v=v)
    c = pm.covariance(f, p, m, v=v)
    g = f * v * v
    n = f.size
    gbar = g.mean()
    sxx = float(((g - gbar) ** 2).sum())
    resid = p - (m["p_idle"] + m["alpha"] * g)
    s2 = float((resid ** 2).sum()) / (n - 2)
    assert c[1, 1] == pytest.approx(s2 / sxx, rel=1e-9)
    assert c[0, 0] == pytest.approx(s2 * (1.0 / n + gbar * gbar / sxx), rel=1e-9)
    assert c[0, 1] == pytest.approx(-gbar * s2 / sxx, rel=1e-9)
    assert c[1, 0] == c[0, 1]
    assert np.all(np.isnan(c[2:, :])) and np.all(np.isnan(c[:, 2:]))


@pytest.mark.parametrize("literal", [False, True])
def test_jacobian_matches_finite_differences(literal):
    # the analytic derivatives against central differences of Eq. 2/3 itself,
    # away from tau (where v has a kink) and from the P_max clip
    rng = np.random.default_rng(11 + literal)
    for _ in range(20):
        th = np.array([rng.uniform(50, 300), rng.uniform(0.05, 0.4), rng.uniform(2e-4, 2e-3),
                       rng.uniform(900, 1600)])
        f = np.array([600.0, 800.0, 1750.0, 2000.0, 2300.0])
        f = f[np.abs(f - th[3]) > 20.0]
        j = pm.jacobian(f, *th, 1e12, literal=literal)
        for q in range(4):
            h = 1e-6 * max(abs(th[q]), 1e-3)
            hi, lo = th.copy(), th.copy()
            hi[q] += h
            lo[q] -= h
            fd = (pm.power(f, *hi, 1e12, literal=literal) - pm.power(f, *lo, 1e12, literal=literal)) / (2 * h)
            assert np.allclose(j[:, q], fd, rtol=1e-6, atol=1e-9 * np.abs(fd).max() + 1e-12), (q, j[:, q], fd)


def test_jacobian_zero_where_clipped():
    f = np.array([500.0, 1500.0, 2400.0])
    j = pm.jacobian(f, 200.0, 0.5, 1e-3, 1000.0, 900.0)
    unclipped = 200.0 + 0.5 * f * pm.voltage(f, 1e-3, 1000.0) ** 2 < 900.0
    assert unclipped.tolist() == [True, False, False]
    assert np.all(j[~unclipped] == 0.0) and np.all(j[0, :2] != 0.0)


def test_covariance_undefined_cases():
    f = np.array([600.0, 1000.0, 1500.0, 2100.0])
    m = dict(p_idle=150.0, alpha=0.2, beta=1e-3, tau=1200.0, p_max=1e9)
    p = pm.power(f, m["p_idle"], m["alpha"], m["beta"], m["tau"], m["p_max"]) + np.array([1.0, -2.0, 0.5, 1.5])
    assert np.all(np.isnan(pm.covariance(f, p, m)))          # n = k = 4: no degrees of freedom
    f5 = np.append(f, 2400.0)
    p5 = np.append(p, 700.0)
    m0 = dict(m, beta=0.0)                                      # beta = 0: tau has no influence
    assert np.all(np.isnan(pm.covariance(f5, p5, m0)))
    c = pm.covariance(f5, p5, m)
    assert np.all(np.isfinite(c)) and np.all(np.diag(c) > 0) and np.allclose(c, c.T, rtol=1e-9)
