// Pure-host parts of the library: the estimators that post-process measured
// series and spectra (Binder cumulant and its time-resolved form, mean and
// error with the integrated autocorrelation time, the dynamic exponent by
// curve collapse, the Lorentzian correlation length) and the thread's error
// message.  No HIP header: this file builds with a plain C++ compiler, which
// is how the sanitizer tests compile it.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/xyl.h"
#include "xyl_error.hpp"

namespace xyl {

thread_local std::string g_err;

double tau_int(const double* f, size_t n) {
    if (n < 2) return 0.5;
    double mean = 0.0;
    for (size_t i = 0; i < n; ++i) mean += f[i];
    mean /= (double)n;
    double c0 = 0.0;
    for (size_t i = 0; i < n; ++i) c0 += (f[i] - mean) * (f[i] - mean);
    c0 /= (double)n;
    if (!(c0 > 0.0)) return 0.5;
    double tau = 0.5;
    for (size_t M = 1; M < n; ++M) {
        double c = 0.0;
        for (size_t i = 0; i + M < n; ++i) c += (f[i] - mean) * (f[i + M] - mean);
        tau += c / (double)n / c0;
        if ((double)M >= 6.0 * tau) break;
    }
    return std::max(tau, 0.5);
}

// Least-squares fit of S(k) = A 2 xi / (1 + 4 pi^2 xi^2 (k/L)^2) over
// k_first..k_last: start from the straight line 1/S = a + b (k/L)^2, then
// Levenberg-Marquardt on (xi, A).
static void lorentzian_fit(const double* S, int L, int k0, int k1, double* xi_out, double* amp_out) {
    const double c = 4.0 * M_PI * M_PI;
    const int n = k1 - k0 + 1;
    double su = 0, sv = 0, suu = 0, suv = 0;
    for (int k = k0; k <= k1; ++k) {
        const double u = ((double)k / L) * ((double)k / L), v = 1.0 / S[k];
        su += u;
        sv += v;
        suu += u * u;
        suv += u * v;
    }
    const double det = n * suu - su * su;
    require(det > 0.0, XYL_EINVAL, "fit range needs two distinct k");
    const double b = (n * suv - su * sv) / det, a = (sv - b * su) / n;
    require(a > 0.0 && b > 0.0, XYL_ENUMERIC, "S(k) is not peaked at k = 0 over the fit range");
    double xi = std::sqrt(b / (a * c)), A = 1.0 / (2.0 * a * xi);
    auto sse = [&](double x, double amp) {
        double e = 0.0;
        for (int k = k0; k <= k1; ++k) {
            const double u = ((double)k / L) * ((double)k / L);
            const double r = S[k] - amp * 2.0 * x / (1.0 + c * x * x * u);
            e += r * r;
        }
        return e;
    };
    double E = sse(xi, A), lam = 1e-3;
    for (int it = 0; it < 200; ++it) {
        double jj[3] = {0, 0, 0}, jr[2] = {0, 0};
        for (int k = k0; k <= k1; ++k) {
            const double u = ((double)k / L) * ((double)k / L);
            const double D = 1.0 + c * xi * xi * u;
            const double f = A * 2.0 * xi / D;
            const double dA = 2.0 * xi / D;
            const double dx = 2.0 * A * (1.0 - c * xi * xi * u) / (D * D);
            const double r = S[k] - f;
            jj[0] += dx * dx;
            jj[1] += dx * dA;
            jj[2] += dA * dA;
            jr[0] += dx * r;
            jr[1] += dA * r;
        }
        bool accepted = false;
        for (int tries = 0; tries < 30 && !accepted; ++tries) {
            const double m00 = jj[0] * (1.0 + lam), m11 = jj[2] * (1.0 + lam), m01 = jj[1];
            const double d = m00 * m11 - m01 * m01;
            if (!(d > 0.0)) {
                lam *= 10.0;
                continue;
            }
            const double dxi = (m11 * jr[0] - m01 * jr[1]) / d, dA = (m00 * jr[1] - m01 * jr[0]) / d;
            const double E1 = sse(xi + dxi, A + dA);
            if (E1 <= E) {
                const bool small = std::fabs(dxi) <= 1e-13 * std::fabs(xi) && std::fabs(dA) <= 1e-13 * std::fabs(A);
                xi += dxi;
                A += dA;
                E = E1;
                lam = std::max(lam * 0.1, 1e-15);
                accepted = true;
                if (small) it = 200;
            } else {
                lam *= 10.0;
            }
        }
        if (!accepted) break;
    }
    require(std::isfinite(xi) && std::isfinite(A), XYL_ENUMERIC, "Lorentzian fit did not converge");
    *xi_out = std::fabs(xi);
    *amp_out = A;
}

}  // namespace xyl

using namespace xyl;

extern "C" {

int xyl_abi_version(void) { return XYL_ABI_VERSION; }

const char* xyl_last_error(void) { return g_err.c_str(); }

int xyl_lorentzian_xi(const double* S, int32_t L, int32_t k_first, int32_t k_last, double* xi, double* amplitude) {
    return guarded([&] {
        require(S != nullptr && xi != nullptr, XYL_EINVAL, "S/xi are NULL");
        require(L >= 2, XYL_EINVAL, "L must be >= 2");
        require(k_first >= 0 && k_last > k_first && k_last <= L / 2, XYL_EINVAL,
                "fit range must satisfy 0 <= k_first < k_last <= L/2");
        for (int k = k_first; k <= k_last; ++k)
            require(std::isfinite(S[k]) && S[k] > 0.0, XYL_EINVAL, "S(k) must be finite and > 0 over the fit range");
        double amp = 0.0;
        lorentzian_fit(S, L, k_first, k_last, xi, &amp);
        if (amplitude) *amplitude = amp;
    });
}

int xyl_xi_second_moment(const xyl_obs* s, uint64_t n, uint64_t discard, int32_t axis, int32_t L, double* xi) {
    return guarded([&] {
        require(s != nullptr && xi != nullptr, XYL_EINVAL, "NULL argument");
        require(discard < n, XYL_EINVAL, "discard must be < n");
        require(axis == 0 || axis == 1, XYL_EINVAL, "axis must be 0 (x) or 1 (y)");
        require(L >= 2, XYL_EINVAL, "L must be >= 2");
        double f0 = 0.0, fk = 0.0;
        for (uint64_t i = discard; i < n; ++i) {
            f0 += s[i].f0;
            fk += axis == 0 ? s[i].fkx : s[i].fky;
        }
        const double cnt = (double)(n - discard);
        f0 /= cnt;
        fk /= cnt;
        require(std::isfinite(f0) && std::isfinite(fk) && fk > 0.0, XYL_ENUMERIC,
                "<F(k_min)> must be positive and finite");
        const double r = f0 / fk - 1.0;
        *xi = r <= 0.0 ? 0.0 : std::sqrt(r) / (2.0 * std::sin(M_PI / (double)L));
    });
}

int xyl_binder(const double* m, uint64_t n, uint64_t discard, double* U, double* U_se) {
    return guarded([&] {
        require(m != nullptr && U != nullptr, XYL_EINVAL, "NULL argument");
        require(discard < n, XYL_EINVAL, "discard must be < n");
        const double* x = m + discard;
        const size_t cnt = n - discard;
        double m2 = 0.0, m4 = 0.0;
        for (size_t i = 0; i < cnt; ++i) {
            const double q = x[i] * x[i];
            m2 += q;
            m4 += q * q;
        }
        m2 /= (double)cnt;
        m4 /= (double)cnt;
        require(m2 > 0.0, XYL_ENUMERIC, "<m^2> is zero");
        *U = m4 / (m2 * m2);
        if (U_se) {
            // jackknife over blocks longer than twice the autocorrelation time of m^2
            std::vector<double> sq(cnt);
            for (size_t i = 0; i < cnt; ++i) sq[i] = x[i] * x[i];
            const double tau = tau_int(sq.data(), cnt);
            const size_t B = (size_t)std::ceil(2.0 * tau) + 1;
            const size_t nb = cnt / B;
            if (nb < 2) {
                *U_se = NAN;
            } else {
                std::vector<double> s2(nb, 0.0), s4(nb, 0.0);
                double t2 = 0.0, t4 = 0.0;
                for (size_t b = 0; b < nb; ++b) {
                    for (size_t i = b * B; i < (b + 1) * B; ++i) {
                        s2[b] += sq[i];
                        s4[b] += sq[i] * sq[i];
                    }
                    t2 += s2[b];
                    t4 += s4[b];
                }
                const double nn = (double)(nb - 1) * (double)B;
                double mean = 0.0;
                std::vector<double> ub(nb);
                for (size_t b = 0; b < nb; ++b) {
                    const double a2 = (t2 - s2[b]) / nn, a4 = (t4 - s4[b]) / nn;
                    ub[b] = a4 / (a2 * a2);
                    mean += ub[b];
                }
                mean /= (double)nb;
                double var = 0.0;
                for (size_t b = 0; b < nb; ++b) var += (ub[b] - mean) * (ub[b] - mean);
                *U_se = std::sqrt(var * (double)(nb - 1) / (double)nb);
            }
        }
    });
}

int xyl_binder_relaxation(const double* m, uint64_t nrep, uint64_t nt, uint64_t bin, double* U, double* U_se) {
    return guarded([&] {
        require(m != nullptr && U != nullptr, XYL_EINVAL, "NULL argument");
        require(nrep >= 1 && bin >= 1 && nt >= bin, XYL_EINVAL, "need nrep >= 1 and nt >= bin >= 1");
        const uint64_t nb = nt / bin;
        std::vector<double> s2(nrep), s4(nrep);
        for (uint64_t b = 0; b < nb; ++b) {
            // per-replica sums over the bin, then the pooled ratio of averages
            double t2 = 0.0, t4 = 0.0;
            for (uint64_t r = 0; r < nrep; ++r) {
                double a2 = 0.0, a4 = 0.0;
                for (uint64_t j = b * bin; j < (b + 1) * bin; ++j) {
                    const double q = m[r * nt + j] * m[r * nt + j];
                    a2 += q;
                    a4 += q * q;
                }
                s2[r] = a2;
                s4[r] = a4;
                t2 += a2;
                t4 += a4;
            }
            const double cnt = (double)nrep * (double)bin;
            require(t2 > 0.0, XYL_ENUMERIC, "<m^2> is zero in a bin");
            U[b] = (t4 / cnt) / ((t2 / cnt) * (t2 / cnt));
            if (U_se) {
                if (nrep < 2) {
                    U_se[b] = NAN;
                    continue;
                }
                // jackknife over replicas (independent realisations)
                const double c1 = (double)(nrep - 1) * (double)bin;
                double mean = 0.0;
                std::vector<double> uj(nrep);
                for (uint64_t r = 0; r < nrep; ++r) {
                    const double a2 = (t2 - s2[r]) / c1, a4 = (t4 - s4[r]) / c1;
                    uj[r] = a2 > 0.0 ? a4 / (a2 * a2) : NAN;
                    mean += uj[r];
                }
                mean /= (double)nrep;
                double var = 0.0;
                for (uint64_t r = 0; r < nrep; ++r) var += (uj[r] - mean) * (uj[r] - mean);
                U_se[b] = std::sqrt(var * (double)(nrep - 1) / (double)nrep);
            }
        }
    });
}

int xyl_z_collapse(const double* t1, const double* U1, uint64_t n1, double L1, const double* t2, const double* U2,
                   uint64_t n2, double L2, double z_lo, double z_hi, double z_step, double* z_best, double* cost) {
    return guarded([&] {
        require(t1 && U1 && t2 && U2 && z_best, XYL_EINVAL, "NULL argument");
        require(n1 >= 2 && n2 >= 2, XYL_EINVAL, "curves need >= 2 points");
        require(L1 > 0.0 && L2 > 0.0 && L1 != L2, XYL_EINVAL, "sizes must be positive and different");
        require(z_step > 0.0 && z_hi >= z_lo && std::isfinite(z_lo) && std::isfinite(z_hi), XYL_EINVAL,
                "bad z raster");
        for (uint64_t i = 1; i < n2; ++i) require(t2[i] > t2[i - 1], XYL_EINVAL, "t2 must increase");
        const double b = L1 / L2;
        const uint64_t nz = (uint64_t)std::floor((z_hi - z_lo) / z_step + 1e-9) + 1;
        double best = INFINITY, zb = NAN;
        for (uint64_t j = 0; j < nz; ++j) {
            const double z = z_lo + (double)j * z_step;
            const double scale = std::pow(b, -z);
            double e = 0.0;
            uint64_t cnt = 0;
            for (uint64_t i = 0; i < n1; ++i) {
                // U(t, L1) against U(b^-z t, L2), the latter interpolated linearly
                const double t = scale * t1[i];
                if (!(t >= t2[0] && t <= t2[n2 - 1])) continue;
                uint64_t hi = (uint64_t)(std::upper_bound(t2, t2 + n2, t) - t2);
                hi = std::min<uint64_t>(std::max<uint64_t>(hi, 1), n2 - 1);
                const uint64_t lo = hi - 1;
                const double w = (t - t2[lo]) / (t2[hi] - t2[lo]);
                const double u = U2[lo] + w * (U2[hi] - U2[lo]);
                e += (U1[i] - u) * (U1[i] - u);
                ++cnt;
            }
            if (cnt >= 3 && e / (double)cnt < best) {
                best = e / (double)cnt;
                zb = z;
            }
        }
        require(std::isfinite(best), XYL_EINVAL, "no z in the raster overlaps the curves in >= 3 points");
        *z_best = zb;
        if (cost) *cost = best;
    });
}

int xyl_mean_error(const double* f, uint64_t n, uint64_t discard, double* mean, double* se, double* tau) {
    return guarded([&] {
        require(f != nullptr, XYL_EINVAL, "NULL argument");
        require(discard < n, XYL_EINVAL, "discard must be < n");
        const double* x = f + discard;
        const size_t cnt = n - discard;
        double mu = 0.0;
        for (size_t i = 0; i < cnt; ++i) mu += x[i];
        mu /= (double)cnt;
        double var = 0.0;
        for (size_t i = 0; i < cnt; ++i) var += (x[i] - mu) * (x[i] - mu);
        var /= (double)cnt;
        const double t = tau_int(x, cnt);
        if (mean) *mean = mu;
        if (se) *se = std::sqrt(2.0 * t * var / (double)cnt);
        if (tau) *tau = t;
    });
}

}  // extern "C"
