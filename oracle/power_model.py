"""Oracle for the paper's power-versus-clock model (test infrastructure only).

Section III.A writes dynamic power as P = P_static + N_c*C*f*V^2 (Eq. 1).
The "Model-steered frequency tuning" subsection turns this into

    Eq. 2   P*_load(f) = min(P_max, P*_idle + alpha * f * v(f)^2)

and, for GPUs without a voltage readout, estimates v from a threshold tau
above which voltage rises at rate beta (Eq. 3).  As printed, Eq. 3 gives
v = beta*(f - tau) above tau, which is zero at f = tau while v = 1 just below
it: power would drop at the ridge.  The reading taken here (``literal=False``,
the default) is the continuous one the text describes -- voltage stays at 1
below tau and grows with slope beta above it:

    v(f) = 1                       f <  tau
    v(f) = 1 + beta * (f - tau)    f >= tau

``literal=True`` evaluates the printed form instead.

Energy per run is estimated as E*(f) proportional to P*(f)/f (absolute
power divided by clock frequency, run time scaling as 1/f).  The paper takes
performance as linear in the clock, and fits and searches the clock range,
only up to the clock where throttling starts (Fig. 8 and the model-fitting
passage of section V.D); above the throttling clock f_thr, where the model
reaches P_max, the device cannot hold the requested clock.  So the
model-optimal clock is the argmin of P*(f)/f over the settable clocks at or
below f_thr (the lowest settable clock when none is), ties going to the
highest such clock (faster at equal energy); the tuning band is the settable
clocks within +-10 % of that optimum.

The fit is the non-linear least-squares problem the paper solves with
Levenberg-Marquardt.  The oracle solves it by exhaustive variable projection
(for fixed beta and tau the model is linear in P_idle and alpha) on a dense
grid, then polishes the best grid points with MINPACK's Levenberg-Marquardt
(``scipy.optimize.least_squares(method="lm")``) as a library step.  It is
pinned by exact recovery of known parameters and by a brute-force grid.
"""
import numpy as np

TIE_REL = 1e-12  # two energy estimates within this relative gap are a tie


def voltage(f, beta, tau, literal=False):
    """Eq. 3 (see module docstring for the reading)."""
    f = np.asarray(f, dtype=np.float64)
    above = f >= tau
    if literal:
        return np.where(above, beta * (f - tau), 1.0)
    return np.where(above, 1.0 + beta * (f - tau), 1.0)


def power(f, p_idle, alpha, beta, tau, p_max, v=None, literal=False):
    """Eq. 2.  ``v`` (measured voltage) replaces Eq. 3 when given."""
    f = np.asarray(f, dtype=np.float64)
    vv = voltage(f, beta, tau, literal) if v is None else np.asarray(v, dtype=np.float64)
    return np.minimum(p_max, p_idle + alpha * f * vv * vv)


def throttle_clock(model, f_hi=1e7):
    """Clock at which the unclipped model reaches P_max: above it the device
    cannot hold the clock (the clipped part of Eq. 2).  The unclipped curve
    P_idle + alpha f v(f)^2 is increasing, so the crossing is found by
    bisection; inf when it never reaches P_max below f_hi."""
    def g(f):
        v = float(voltage(f, model["beta"], model["tau"], model.get("literal", False)))
        return model["p_idle"] + model["alpha"] * f * v * v - model["p_max"]
    if g(f_hi) <= 0:
        return float("inf")
    lo, hi = 0.0, f_hi
    if g(lo) > 0:
        return 0.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if g(mid) <= 0:
            lo = mid
        else:
            hi = mid
    return lo


def energy_estimate(f, model, f_thr=None):
    """E*(f) proportional to P*(f)/f, with performance linear in the clock
    only up to the throttling clock f_thr (the paper's performance estimate,
    Fig. 8): above it the device runs at f_thr and P_max, so
    E*(f) = P*(min(f, f_thr)) / min(f, f_thr)."""
    f = np.asarray(f, dtype=np.float64)
    f_eff = np.minimum(f, throttle_clock(model) if f_thr is None else f_thr)
    return power(f_eff, model["p_idle"], model["alpha"], model["beta"], model["tau"],
                 model["p_max"], literal=model.get("literal", False)) / f_eff


def optimal_clock(settable, model):
    """argmin of E*(f) = P*(f)/f over the settable clocks f <= f_thr (the
    clocks the device can hold); ties -> the highest such clock.  When every
    settable clock lies above f_thr the lowest one is returned."""
    s = sorted(float(x) for x in settable)
    f_thr = throttle_clock(model)
    held = [f for f in s if f <= f_thr] or s[:1]
    best_f, best_e = None, None
    for f in held:
        e = float(power(f, model["p_idle"], model["alpha"], model["beta"], model["tau"], model["p_max"],
                        literal=model.get("literal", False))) / f
        if best_e is None or e <= best_e * (1.0 + TIE_REL):
            if best_e is None or e < best_e:
                best_e = e
            best_f = f
    return best_f


def clock_band(settable, f_opt, rel_half=0.1):
    """The settable clocks inside [(1-rel)*f_opt, (1+rel)*f_opt], ascending."""
    lo, hi = (1.0 - rel_half) * f_opt, (1.0 + rel_half) * f_opt
    return [float(f) for f in sorted(settable) if lo <= f <= hi]


def sse(params, f, p, p_max, literal=False):
    p_idle, alpha, beta, tau = params
    r = np.asarray(p, dtype=np.float64) - power(f, p_idle, alpha, beta, tau, p_max,
                                                literal=literal)
    return float(np.dot(r, r))


def _linear_given(f, p, p_max, beta, tau, literal):
    """For fixed (beta, tau): linear least squares for (P_idle, alpha) over all
    the points, treating the model as unclipped, then clamp to P_idle,
    alpha >= 0.  This only seeds the grid search and the Levenberg-Marquardt
    polish below, which minimise the clipped residual."""
    g = f * voltage(f, beta, tau, literal) ** 2
    a = np.stack([np.ones_like(f), g], axis=1)
    sol, *_ = np.linalg.lstsq(a, p, rcond=None)
    p_idle, alpha = max(sol[0], 0.0), max(sol[1], 0.0)
    return p_idle, alpha


def fit(f, p, p_max, v=None, literal=False, n_beta=161, n_tau=161):
    """Least-squares fit of Eq. 2 (+ Eq. 3 when ``v`` is None).

    Returns dict(p_idle, alpha, beta, tau, p_max, sse).  With measured voltage
    the model is linear in (P_idle, alpha) and solved directly (beta = tau = 0)."""
    from scipy.optimize import least_squares

    f = np.asarray(f, dtype=np.float64)
    p = np.asarray(p, dtype=np.float64)
    if v is not None:
        vv = np.asarray(v, dtype=np.float64)
        a = np.stack([np.ones_like(f), f * vv * vv], axis=1)
        sol, *_ = np.linalg.lstsq(a, p, rcond=None)
        r = p - np.minimum(p_max, sol[0] + sol[1] * f * vv * vv)
        return dict(p_idle=float(sol[0]), alpha=float(sol[1]), beta=0.0, tau=0.0,
                    p_max=float(p_max), sse=float(r @ r))
    fmin, fmax = float(f.min()), float(f.max())
    span = max(fmax - fmin, 1e-9)
    # beta grid: Eq. 3 bounds beta only below (beta >= 0), so the grid spans
    # voltage at f_max from 1x up to 21x of its floor value
    betas = np.concatenate([[0.0], np.geomspace(1e-4, 20.0, n_beta - 1)]) / span
    taus = np.linspace(fmin, fmax, n_tau)
    cands = []
    for b in betas:
        for t in taus:
            pi, al = _linear_given(f, p, p_max, b, t, literal)
            cands.append((sse((pi, al, b, t), f, p, p_max, literal), pi, al, b, t))
    cands.sort(key=lambda c: c[0])
    best = cands[0]
    scale = np.array([max(abs(best[1]), 1.0), max(abs(best[2]), 1e-12),
                      max(1.0 / span, 1e-12), span])

    def resid(z):
        pi, al, b, t = z * scale
        return p - power(f, pi, al, b, t, p_max, literal=literal)

    for c in cands[:8]:
        z0 = np.array(c[1:]) / scale
        try:
            res = least_squares(resid, z0, method="lm", xtol=1e-15, ftol=1e-15, gtol=1e-15,
                                max_nfev=20000)
        except Exception:  # noqa: BLE001 -- a failed polish keeps the grid point
            continue
        pi, al, b, t = res.x * scale
        if pi < 0 or al < 0 or b < 0 or t < fmin or t > fmax:
            continue
        s = sse((pi, al, b, t), f, p, p_max, literal)
        if s < best[0]:
            best = (s, pi, al, b, t)
    s, pi, al, b, t = best
    return dict(p_idle=float(pi), alpha=float(al), beta=float(b), tau=float(t),
                p_max=float(p_max), sse=float(s))


def jacobian(f, p_idle, alpha, beta, tau, p_max, v=None, literal=False):
    """Derivatives of Eq. 2 (with Eq. 3 unless measured voltage ``v`` is
    given) with respect to (P_idle, alpha, beta, tau) at the clocks f, one
    row per clock.  Where the model is clipped at P_max the row is zero (the
    clipped power does not depend on the parameters).  With v given, beta and
    tau have no influence (zero columns)."""
    f = np.asarray(f, dtype=np.float64)
    vv = voltage(f, beta, tau, literal) if v is None else np.asarray(v, dtype=np.float64)
    unclipped = p_idle + alpha * f * vv * vv < p_max
    above = (f >= tau) if v is None else np.zeros_like(f, dtype=bool)
    # P = P_idle + alpha f v^2; both forms of Eq. 3 have dv/dbeta = f - tau
    # and dv/dtau = -beta above tau (and v does not depend on them below)
    j = np.zeros((f.size, 4))
    j[:, 0] = 1.0
    j[:, 1] = f * vv * vv
    j[:, 2] = np.where(above, 2.0 * alpha * f * vv * (f - tau), 0.0)
    j[:, 3] = np.where(above, -2.0 * alpha * f * vv * beta, 0.0)
    j[~unclipped] = 0.0
    return j


def covariance(f, p, model, v=None):
    """Covariance of the fitted parameters (P_idle, alpha, beta, tau) of a
    least-squares fit: s^2 (J^T J)^-1 over the free parameters (all four, or
    P_idle and alpha with measured voltage) at the fitted model, with
    s^2 = SSE / (n - k) for n readings and k free parameters, the usual
    linearised estimate for non-linear least squares.  NaN (4 x 4) entries
    where undefined: parameters not fitted, n <= k, or J^T J singular."""
    f = np.asarray(f, dtype=np.float64)
    p = np.asarray(p, dtype=np.float64)
    k = 2 if v is not None else 4
    out = np.full((4, 4), np.nan)
    if f.size <= k:
        return out
    args = (model["p_idle"], model["alpha"], model["beta"], model["tau"], model["p_max"])
    j = jacobian(f, *args, v=v, literal=model.get("literal", False))[:, :k]
    a = j.T @ j
    # conditioning judged on the equilibrated matrix (unit diagonal), which
    # does not depend on the units of the parameters
    d = np.sqrt(np.diag(a))
    if not np.all(np.isfinite(a)) or not np.all(d > 0):
        return out
    ae = a / np.outer(d, d)
    if np.linalg.cond(ae) > 1e12:
        return out
    r = p - power(f, *args, v=v, literal=model.get("literal", False))
    s2 = float(r @ r) / (f.size - k)
    out[:k, :k] = s2 * np.linalg.inv(ae) / np.outer(d, d)
    return out
