// Power-versus-clock model of the paper (Eq. 2 with the voltage estimate of
// Eq. 3), its Levenberg-Marquardt least-squares fit, and the model-steered
// clock band (section V.D: tune within +-10 % of the clock where the energy
// estimate P*(f)/f is lowest).
//
// Reading of Eq. 3: as printed, v = beta*(f - tau) above tau is zero at tau
// while v = 1 below it.  The text says voltage is flat up to a threshold and
// then rises at rate beta, so the default is the continuous
//     v(f) = 1 + beta * max(0, f - tau);
// gt_power_model.literal_eq3 = 1 selects the printed form.
//
// Fit internals run in GHz for conditioning: x = f/1000, parameters
// (p_idle [W], a [W/GHz], b [1/GHz], t [GHz]); the public struct holds
// alpha = a/1000 [W/MHz], beta = b/1000 [1/MHz], tau = 1000 t [MHz].
#include <algorithm>
#include <cmath>
#include <vector>

#include "gt_internal.hpp"

namespace gt {
namespace {

struct Data {
    const double *x;   // GHz
    const double *p;   // W
    const double *v;   // measured voltage or null
    size_t n;
    double p_max;
    bool literal;
};

inline double volt(double x, double b, double t, bool literal) {
    if (x < t) return 1.0;
    return literal ? b * (x - t) : 1.0 + b * (x - t);
}

double sse_of(const Data &d, const double th[4]) {
    double s = 0.0;
    for (size_t i = 0; i < d.n; ++i) {
        const double vv = d.v ? d.v[i] : volt(d.x[i], th[2], th[3], d.literal);
        const double m = std::min(d.p_max, th[0] + th[1] * d.x[i] * vv * vv);
        const double r = d.p[i] - m;
        s += r * r;
    }
    return s;
}

// Solve the 4x4 (or k x k) system A z = g by Gaussian elimination with
// partial pivoting; returns false when singular.
bool solve(int k, double A[4][4], double g[4], double z[4]) {
    double M[4][5];
    for (int i = 0; i < k; ++i) {
        for (int j = 0; j < k; ++j) M[i][j] = A[i][j];
        M[i][k] = g[i];
    }
    for (int c = 0; c < k; ++c) {
        int piv = c;
        for (int r = c + 1; r < k; ++r)
            if (std::fabs(M[r][c]) > std::fabs(M[piv][c])) piv = r;
        if (!(std::fabs(M[piv][c]) > 1e-300)) return false;
        if (piv != c)
            for (int j = 0; j <= k; ++j) std::swap(M[c][j], M[piv][j]);
        for (int r = c + 1; r < k; ++r) {
            const double f = M[r][c] / M[c][c];
            for (int j = c; j <= k; ++j) M[r][j] -= f * M[c][j];
        }
    }
    for (int i = k - 1; i >= 0; --i) {
        double s = M[i][k];
        for (int j = i + 1; j < k; ++j) s -= M[i][j] * z[j];
        z[i] = s / M[i][i];
    }
    return true;
}

// Least squares for (p_idle, a) with (b, t) fixed, over the readings below
// P_max (a reading at the cap says nothing about the unclipped curve; all
// readings are used if fewer than two are below it), clamped to >= 0.
void linear_given(const Data &d, double b, double t, double th[4]) {
    size_t below = 0;
    for (size_t i = 0; i < d.n; ++i) below += d.p[i] < d.p_max * (1.0 - 1e-6);
    const bool use_all = below < 2;
    double s00 = 0, s01 = 0, s11 = 0, r0 = 0, r1 = 0;
    for (size_t i = 0; i < d.n; ++i) {
        if (!use_all && !(d.p[i] < d.p_max * (1.0 - 1e-6))) continue;
        const double vv = d.v ? d.v[i] : volt(d.x[i], b, t, d.literal);
        const double g = d.x[i] * vv * vv;
        s00 += 1;
        s01 += g;
        s11 += g * g;
        r0 += d.p[i];
        r1 += g * d.p[i];
    }
    const double det = s00 * s11 - s01 * s01;
    double pi = 0, a = 0;
    if (std::fabs(det) > 1e-300 * std::max(1.0, s00 * s11)) {
        pi = (s11 * r0 - s01 * r1) / det;
        a = (s00 * r1 - s01 * r0) / det;
    } else if (s11 > 0) {
        a = r1 / s11;
    }
    if (a < 0) {
        a = 0;
        pi = r0 / s00;
    }
    if (pi < 0) {
        pi = 0;
        a = s11 > 0 ? std::max(0.0, r1 / s11) : 0;
    }
    th[0] = pi;
    th[1] = a;
    th[2] = b;
    th[3] = t;
}

struct LmResult {
    double th[4];
    double sse;
    int iters;
    int status;
};

// Levenberg-Marquardt with Marquardt's diagonal scaling, projected onto the
// bounds p_idle, a, b >= 0 and t in [t_lo, t_hi].  k = number of free
// parameters (2 with measured voltage: p_idle and a only).
LmResult lm(const Data &d, const double th0[4], int k, double t_lo, double t_hi) {
    LmResult R;
    for (int i = 0; i < 4; ++i) R.th[i] = th0[i];
    R.sse = sse_of(d, R.th);
    R.iters = 0;
    R.status = 1;
    double lambda = 1e-3;
    std::vector<double> J(d.n * 4), r(d.n);
    for (int it = 0; it < 500; ++it) {
        R.iters = it + 1;
        const double pi = R.th[0], a = R.th[1], b = R.th[2], t = R.th[3];
        for (size_t i = 0; i < d.n; ++i) {
            const double x = d.x[i];
            const double vv = d.v ? d.v[i] : volt(x, b, t, d.literal);
            const double g = pi + a * x * vv * vv;
            double *Ji = &J[i * 4];
            if (g >= d.p_max) {
                Ji[0] = Ji[1] = Ji[2] = Ji[3] = 0.0;
                r[i] = d.p[i] - d.p_max;
                continue;
            }
            r[i] = d.p[i] - g;
            Ji[0] = 1.0;
            Ji[1] = x * vv * vv;
            const bool above = !d.v && x >= t;
            Ji[2] = above ? 2.0 * a * x * vv * (x - t) : 0.0;
            Ji[3] = above ? -2.0 * a * x * vv * b : 0.0;
        }
        double A[4][4] = {{0}}, gv[4] = {0};
        for (size_t i = 0; i < d.n; ++i)
            for (int p = 0; p < k; ++p) {
                gv[p] += J[i * 4 + p] * r[i];
                for (int q = 0; q < k; ++q) A[p][q] += J[i * 4 + p] * J[i * 4 + q];
            }
        double dmax = 0;
        for (int p = 0; p < k; ++p) dmax = std::max(dmax, A[p][p]);
        if (!(dmax > 0)) {
            R.status = 0;
            break;
        }
        bool improved = false;
        while (lambda < 1e20) {
            double B[4][4], z[4] = {0, 0, 0, 0};
            for (int p = 0; p < k; ++p)
                for (int q = 0; q < k; ++q)
                    B[p][q] = A[p][q] + (p == q ? lambda * std::max(A[p][p], 1e-12 * dmax) : 0.0);
            if (!solve(k, B, gv, z)) {
                lambda *= 10;
                continue;
            }
            double cand[4] = {R.th[0], R.th[1], R.th[2], R.th[3]};
            for (int p = 0; p < k; ++p) cand[p] += z[p];
            cand[0] = std::max(cand[0], 0.0);
            cand[1] = std::max(cand[1], 0.0);
            cand[2] = std::max(cand[2], 0.0);
            cand[3] = std::min(std::max(cand[3], t_lo), t_hi);
            const double s = sse_of(d, cand);
            if (s < R.sse) {
                double step = 0, norm = 0;
                for (int p = 0; p < 4; ++p) {
                    step += (cand[p] - R.th[p]) * (cand[p] - R.th[p]);
                    norm += R.th[p] * R.th[p];
                }
                const double rel_sse = (R.sse - s) / std::max(R.sse, 1e-300);
                for (int p = 0; p < 4; ++p) R.th[p] = cand[p];
                R.sse = s;
                lambda = std::max(lambda / 10, 1e-15);
                improved = true;
                if (step <= 1e-24 * std::max(norm, 1e-300) || rel_sse < 1e-15) R.status = 0;
                break;
            }
            lambda *= 10;
        }
        if (!improved) {
            R.status = 0;  // no descent step exists at this point: a (local) minimum
            break;
        }
        if (R.status == 0 || R.sse == 0.0) {
            R.status = 0;
            break;
        }
    }
    return R;
}

// Covariance of the fitted parameters: s^2 (J^T J)^-1 over the k free
// parameters at th (internal units), s^2 = sse / (n - k); written into
// cov[16] (public units, row-major (p_idle, alpha, beta, tau)), NaN where
// undefined.  Readings clipped at p_max have a zero Jacobian row, as in lm().
void covariance(const Data &d, const double th[4], int k, double sse, double cov[16]) {
    for (int i = 0; i < 16; ++i) cov[i] = NAN;
    if ((int)d.n <= k) return;
    double A[4][4] = {{0}};
    for (size_t i = 0; i < d.n; ++i) {
        const double x = d.x[i];
        const double vv = d.v ? d.v[i] : volt(x, th[2], th[3], d.literal);
        if (th[0] + th[1] * x * vv * vv >= d.p_max) continue;
        double Ji[4];
        Ji[0] = 1.0;
        Ji[1] = x * vv * vv;
        const bool above = !d.v && x >= th[3];
        Ji[2] = above ? 2.0 * th[1] * x * vv * (x - th[3]) : 0.0;  // dv/db = x - t in both forms of Eq. 3
        Ji[3] = above ? -2.0 * th[1] * x * vv * th[2] : 0.0;
        for (int p = 0; p < k; ++p)
            for (int q = 0; q < k; ++q) A[p][q] += Ji[p] * Ji[q];
    }
    // equilibrate (unit diagonal: the conditioning then does not depend on
    // the parameters' units), invert by solving A z = e_j, and leave NaN for
    // a singular or ill-conditioned matrix (max-abs norms of A and A^-1,
    // product beyond 1e12)
    double dg[4];
    for (int p = 0; p < k; ++p) {
        dg[p] = std::sqrt(A[p][p]);
        if (!(dg[p] > 0) || !std::isfinite(dg[p])) return;
    }
    for (int p = 0; p < k; ++p)
        for (int q = 0; q < k; ++q) A[p][q] /= dg[p] * dg[q];
    double inv[4][4];
    for (int j = 0; j < k; ++j) {
        double A2[4][4], e[4] = {0, 0, 0, 0}, z[4] = {0, 0, 0, 0};
        for (int p = 0; p < k; ++p)
            for (int q = 0; q < k; ++q) A2[p][q] = A[p][q];
        e[j] = 1.0;
        if (!solve(k, A2, e, z)) return;
        for (int p = 0; p < k; ++p) inv[p][j] = z[p];
    }
    double imax = 0, amax = 0;
    for (int p = 0; p < k; ++p)
        for (int q = 0; q < k; ++q) {
            imax = std::max(imax, std::fabs(inv[p][q]));
            amax = std::max(amax, std::fabs(A[p][q]));
        }
    if (!(amax * imax < 1e12)) return;
    for (int p = 0; p < k; ++p)
        for (int q = 0; q < k; ++q) inv[p][q] /= dg[p] * dg[q];
    const double s2 = sse / (double)((int)d.n - k);
    // internal -> public units: alpha = a / 1000, beta = b / 1000, tau = 1000 t
    const double scale[4] = {1.0, 1e-3, 1e-3, 1e3};
    for (int p = 0; p < k; ++p)
        for (int q = 0; q < k; ++q) cov[p * 4 + q] = s2 * inv[p][q] * scale[p] * scale[q];
}

}  // namespace
}  // namespace gt

using namespace gt;

extern "C" {

int fit_power_model(const double *f_mhz, const double *p_w, const double *v_or_null, size_t n,
                    double p_max_w, gt_power_model *out) {
    clear_error();
    if (!f_mhz || !p_w || !out) return set_error(GT_E_INVAL, "fit_power_model: null argument");
    if (!(p_max_w > 0)) return set_error(GT_E_INVAL, "fit_power_model: p_max must be positive");
    const bool literal = out->literal_eq3 != 0;
    const size_t need = v_or_null ? 2 : 4;
    if (n < need) return set_error(GT_E_INVAL, "fit_power_model: need at least %zu readings", need);
    std::vector<double> x(n);
    double xlo = INFINITY, xhi = -INFINITY;
    for (size_t i = 0; i < n; ++i) {
        if (!(f_mhz[i] > 0) || !std::isfinite(p_w[i]))
            return set_error(GT_E_INVAL, "fit_power_model: reading %zu is not valid", i);
        x[i] = f_mhz[i] / 1000.0;
        xlo = std::min(xlo, x[i]);
        xhi = std::max(xhi, x[i]);
    }
    Data d{x.data(), p_w, v_or_null, n, p_max_w, literal};
    LmResult best;
    best.sse = INFINITY;
    if (v_or_null) {
        double th[4];
        linear_given(d, 0, 0, th);
        best = lm(d, th, 2, 0, 0);
    } else {
        // Starting points by variable projection on a coarse (b, t) grid.
        const double span = std::max(xhi - xlo, 1e-9);
        struct Cand { double sse, th[4]; };
        std::vector<Cand> cands;
        const int nb = 24, nt = 25;
        for (int ib = 0; ib < nb; ++ib) {
            const double b = ib == 0 ? 0.0 : 1e-4 * std::pow(4.0 / 1e-4, (ib - 1) / double(nb - 2)) / span;
            for (int itau = 0; itau < nt + (int)n; ++itau) {
                const double t = itau < nt ? xlo + span * itau / (nt - 1) : x[itau - nt];
                Cand c;
                linear_given(d, b, t, c.th);
                c.sse = sse_of(d, c.th);
                cands.push_back(c);
            }
        }
        std::sort(cands.begin(), cands.end(), [](const Cand &a, const Cand &b) { return a.sse < b.sse; });
        const size_t nstart = std::min<size_t>(12, cands.size());
        for (size_t s = 0; s < nstart; ++s) {
            LmResult R = lm(d, cands[s].th, 4, xlo, xhi);
            if (R.sse < best.sse) best = R;
        }
    }
    out->p_idle = best.th[0];
    out->alpha = best.th[1] / 1000.0;
    out->beta = v_or_null ? 0.0 : best.th[2] / 1000.0;
    out->tau_mhz = v_or_null ? 0.0 : best.th[3] * 1000.0;
    out->p_max = p_max_w;
    out->rss = best.sse;
    out->v_measured = v_or_null ? 1 : 0;
    out->literal_eq3 = literal ? 1 : 0;
    out->iters = best.iters;
    out->status = best.status;
    covariance(d, best.th, v_or_null ? 2 : 4, best.sse, out->cov);
    return GT_OK;
}

double gt_power_model_eval(const gt_power_model *m, double f_mhz) {
    if (!m) return NAN;
    double v = 1.0;
    if (!m->v_measured && f_mhz >= m->tau_mhz)
        v = m->literal_eq3 ? m->beta * (f_mhz - m->tau_mhz) : 1.0 + m->beta * (f_mhz - m->tau_mhz);
    return std::min(m->p_max, m->p_idle + m->alpha * f_mhz * v * v);
}

double gt_power_model_throttle_clock(const gt_power_model *m) {
    if (!m) return NAN;
    // the unclipped curve p_idle + alpha f v(f)^2 is non-decreasing in f
    auto g = [m](double f) {
        double v = 1.0;
        if (!m->v_measured && f >= m->tau_mhz)
            v = m->literal_eq3 ? m->beta * (f - m->tau_mhz) : 1.0 + m->beta * (f - m->tau_mhz);
        return m->p_idle + m->alpha * f * v * v - m->p_max;
    };
    double lo = 0.0, hi = 1e7;
    if (g(hi) <= 0) return INFINITY;
    if (g(lo) > 0) return 0.0;
    for (int it = 0; it < 200; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (g(mid) <= 0)
            lo = mid;
        else
            hi = mid;
    }
    return lo;
}

int gt_power_model_band(const gt_power_model *m, const double *settable, size_t n, double rel_half,
                        double *f_opt, double *band, size_t cap, size_t *n_band) {
    clear_error();
    if (!m || !settable || !n || !f_opt || !n_band || (cap && !band) || !(rel_half >= 0))
        return set_error(GT_E_INVAL, "gt_power_model_band: bad argument");
    std::vector<double> s(settable, settable + n);
    std::sort(s.begin(), s.end());
    if (!(s[0] > 0)) return set_error(GT_E_INVAL, "gt_power_model_band: clocks must be positive");
    // energy estimate E*(f) = P*(f)/f over the clocks the device can hold:
    // the paper fits and searches only up to where throttling starts, and
    // above the throttling clock the requested clock is not reached.  When
    // every settable clock lies above it, the lowest one.  Ascending scan so
    // ties end on the highest held clock.
    const double f_thr = gt_power_model_throttle_clock(m);
    size_t n_held = 0;
    while (n_held < n && s[n_held] <= f_thr) ++n_held;
    if (n_held == 0) n_held = 1;
    auto energy = [&](double f) { return gt_power_model_eval(m, f) / f; };
    double best_f = s[0], best_e = energy(s[0]);
    for (size_t i = 1; i < n_held; ++i) {
        const double e = energy(s[i]);
        if (e <= best_e * (1.0 + 1e-12)) {
            if (e < best_e) best_e = e;
            best_f = s[i];
        }
    }
    *f_opt = best_f;
    const double lo = (1.0 - rel_half) * best_f, hi = (1.0 + rel_half) * best_f;
    size_t k = 0;
    for (size_t i = 0; i < n; ++i)
        if (s[i] >= lo && s[i] <= hi) {
            if (k < cap) band[k] = s[i];
            ++k;
        }
    *n_band = k;
    if (k > cap) return set_error(GT_E_CAPACITY, "gt_power_model_band: %zu clocks, capacity %zu", k, cap);
    return GT_OK;
}

}  // extern "C"
