// Terrain-weight estimate of Eq. (4) (Alg. 1, Step 3), host-only.
//
// minimise f(w) = ||Y - F w||^2 + gamma sum_i |w_i - p_i|  over the simplex
// {0 <= w_i <= 1, sum w_i = 1}, with Y = [Yv; Yw] and F = [Fv; Fw] stacked.
// Pairwise descent: a move w + t (e_i - e_j) keeps the simplex; along it the
// objective is a t^2 + beta t + gamma |w_i + t - p_i| + gamma |w_j - t - p_j|
// (a = Q_ii + Q_jj - 2 Q_ij, beta = g_i - g_j, g = 2 (Q w - c), Q = F^T F,
// c = F^T Y), a convex piecewise quadratic with at most two breakpoints whose
// minimum over the feasible interval is found exactly by checking each piece.
// The objective is convex and every feasible direction splits into pairwise
// moves of the same signs, so a point no pairwise move improves is optimal.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <string>
#include <vector>

#include "gpmppi.h"

namespace gpmppi {
gpmppi_status set_error(gpmppi_status st, const char *msg);
}

namespace {

double piece_value(double a, double beta, double gamma, double wi, double wj, double pi, double pj, double t) {
    return a * t * t + beta * t + gamma * (std::fabs(wi + t - pi) + std::fabs(wj - t - pj));
}

}  // namespace

extern "C" gpmppi_status gpmppi_terrain_weights(int32_t H, int32_t n, const double *Yv, const double *Yw,
                                                const double *Fv, const double *Fw, const double *w_prev,
                                                double gamma, double *w_out) {
    using gpmppi::set_error;
    if (!Yv || !Yw || !Fv || !Fw || !w_prev || !w_out) return set_error(GPMPPI_E_INVALID, "NULL argument");
    if (H < 1 || n < 1 || n > 8) return set_error(GPMPPI_E_INVALID, "need H >= 1 and 1 <= n <= 8");
    if (!std::isfinite(gamma) || gamma < 0) return set_error(GPMPPI_E_INVALID, "gamma must be finite and >= 0");
    for (long long i = 0; i < (long long)H * n; ++i)
        if (!std::isfinite(Fv[i]) || !std::isfinite(Fw[i])) return set_error(GPMPPI_E_NONFINITE, "non-finite F");
    for (int h = 0; h < H; ++h)
        if (!std::isfinite(Yv[h]) || !std::isfinite(Yw[h])) return set_error(GPMPPI_E_NONFINITE, "non-finite Y");
    for (int i = 0; i < n; ++i)
        if (!std::isfinite(w_prev[i])) return set_error(GPMPPI_E_NONFINITE, "non-finite w_prev");
    // Q = F^T F, c = F^T Y
    std::vector<double> Q(n * n, 0.0), c(n, 0.0);
    for (int h = 0; h < H; ++h)
        for (int s = 0; s < 2; ++s) {
            const double *F = (s ? Fw : Fv) + (size_t)h * n;
            const double y = s ? Yw[h] : Yv[h];
            for (int i = 0; i < n; ++i) {
                c[i] += F[i] * y;
                for (int j = 0; j < n; ++j) Q[i * n + j] += F[i] * F[j];
            }
        }
    // start from the previous weights if feasible, else uniform
    std::vector<double> w(w_prev, w_prev + n), p(w_prev, w_prev + n);
    double sum = 0.0;
    bool ok = true;
    for (int i = 0; i < n; ++i) {
        ok = ok && w[i] >= 0.0 && w[i] <= 1.0;
        sum += w[i];
    }
    if (!ok || std::fabs(sum - 1.0) > 1e-12) std::fill(w.begin(), w.end(), 1.0 / n);
    std::vector<double> g(n);
    auto refresh = [&]() {
        for (int i = 0; i < n; ++i) {
            double s = -c[i];
            for (int j = 0; j < n; ++j) s += Q[i * n + j] * w[j];
            g[i] = 2.0 * s;
        }
    };
    refresh();
    for (int sweep = 0; sweep < 20000; ++sweep) {
        double moved = 0.0;
        for (int i = 0; i < n; ++i)
            for (int j = i + 1; j < n; ++j) {
                const double a = Q[i * n + i] + Q[j * n + j] - 2.0 * Q[i * n + j];
                const double beta = g[i] - g[j];
                const double lo = std::max(-w[i], w[j] - 1.0), hi = std::min(1.0 - w[i], w[j]);
                if (hi - lo <= 0.0) continue;
                double cand[12];
                int nc = 0;
                double bp[2] = {p[i] - w[i], w[j] - p[j]};
                std::sort(bp, bp + 2);
                double edges[4] = {lo, std::clamp(bp[0], lo, hi), std::clamp(bp[1], lo, hi), hi};
                for (int e = 0; e < 4; ++e) cand[nc++] = edges[e];
                for (int e = 0; e < 3; ++e) {
                    const double l = edges[e], r = edges[e + 1];
                    if (r <= l) continue;
                    const double mid = 0.5 * (l + r);
                    const double si = (w[i] + mid - p[i]) >= 0 ? 1.0 : -1.0;
                    const double sj = (w[j] - mid - p[j]) >= 0 ? 1.0 : -1.0;
                    if (a > 0) cand[nc++] = std::clamp(-(beta + gamma * (si - sj)) / (2.0 * a), l, r);
                }
                double best_t = 0.0, best = piece_value(a, beta, gamma, w[i], w[j], p[i], p[j], 0.0);
                for (int e = 0; e < nc; ++e) {
                    const double v = piece_value(a, beta, gamma, w[i], w[j], p[i], p[j], cand[e]);
                    if (v < best) {
                        best = v;
                        best_t = cand[e];
                    }
                }
                if (best_t != 0.0) {
                    w[i] += best_t;
                    w[j] -= best_t;
                    for (int k = 0; k < n; ++k) g[k] += 2.0 * best_t * (Q[k * n + i] - Q[k * n + j]);
                    moved = std::max(moved, std::fabs(best_t));
                }
            }
        if (sweep % 64 == 63) refresh();   // limit drift of the incremental gradient
        if (moved < 1e-15) break;
    }
    double s = 0.0;
    for (int i = 0; i < n; ++i) {
        w[i] = std::clamp(w[i], 0.0, 1.0);
        s += w[i];
    }
    for (int i = 0; i < n; ++i) w_out[i] = w[i] / s;
    return GPMPPI_OK;
}
