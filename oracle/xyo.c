/*
 * xyo.c — plain FP64 CPU oracle (TEST INFRASTRUCTURE ONLY; see xyo.h).
 *
 * Everything here is the direct definition, written for a reader to check by
 * eye against the paper:
 *   - Hamiltonian: Sec. III.A, Eq. XY-Hamilton-Field (q = 1, p = 2; or the
 *     Si(001) mapping of Sec. III.C, q = 2 with real p) plus the kinetic term
 *     of Eq. XY-Hamilton-Kinetic with I = 1.
 *   - Equations of motion: Sec. III.D, Eq. Si-Langevin; noise <G G'> = delta.
 *   - Integrator: App. A.1, three stages (Eq. BBK-1, drift, Eq. BBK-2); the
 *     Gaussian draw n(t+dt) of the second half-kick of one step is the n(t) of
 *     the first half-kick of the next step.
 *   - Wrap after every step (Sec. III.D), to [-pi, pi) or, for the Si mapping,
 *     to [-pi/2, pi/2) (Sec. III.C).
 *   - Order parameter and Binder cumulant: Sec. IV.A, Eqs. Def-Binder-Cum and
 *     lattice-average (staggered when a coupling is antiferromagnetic; the
 *     site variable is cos th, or sin 2 th for the Si mapping).
 *   - Correlation function: App. C (rotor dot products, lattice average).
 *   - Linear quench: Sec. II.B, Eq. Linear-Quench, as a piecewise-linear T(k).
 * OpenMP parallelises the per-site loops only; every reduction is done per row
 * and then summed in row order, so results do not depend on the thread count.
 */
#include "xyo.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define PI64 3.14159265358979323846
#define TWO_PI64 (2.0 * PI64)

/* ------------------------------------------------------------------ Philox */
/* Philox4x32 with R = 10 rounds, as defined by Salmon et al. (SC'11):
 * each round multiplies words 0 and 2 by fixed 32-bit constants, takes the
 * 64-bit products apart into high and low halves and mixes them with the key;
 * the key is bumped by the Weyl constants between rounds. */
void xyo_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += W0;
            k1 += W1;
        }
        uint64_t p0 = (uint64_t)M0 * (uint64_t)c0;
        uint64_t p1 = (uint64_t)M1 * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

double xyo_uniform(uint32_t r) {
    return ((double)(r >> 9) + 0.5) * 0x1p-23;
}

static void philox_block(const xyo_model* m, uint64_t k, int64_t i, uint32_t out[4]) {
    uint32_t ctr[4] = {(uint32_t)(i >> 2), m->replica, (uint32_t)k, (uint32_t)(k >> 32)};
    uint32_t key[2] = {(uint32_t)m->seed, (uint32_t)(m->seed >> 32)};
    xyo_philox4x32_10(ctr, key, out);
}

/* Box-Muller: sites i with the same i>>2 share one Philox block; words
 * (2p, 2p+1) with p = (i&3)>>1 form one pair; even i takes the cosine branch,
 * odd i the sine branch. */
double xyo_normal(const xyo_model* m, uint64_t k, int64_t i) {
    uint32_t r[4];
    philox_block(m, k, i, r);
    int p = (int)((i & 3) >> 1);
    double u1 = xyo_uniform(r[2 * p]);
    double u2 = xyo_uniform(r[2 * p + 1]);
    double R = sqrt(-2.0 * log(u1));
    double phi = TWO_PI64 * u2;
    return (i & 1) ? R * sin(phi) : R * cos(phi);
}

void xyo_normals(const xyo_model* m, uint64_t k, double* n) {
    const int64_t N = (int64_t)m->Lx * m->Ly;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < N; ++i) n[i] = xyo_normal(m, k, i);
}

/* ---------------------------------------------------------------- schedule */
double xyo_temperature(const xyo_model* m, uint64_t k) {
    const int n = m->nknots;
    double T;
    if (k <= m->knot_step[0]) {
        T = m->knot_T[0];
    } else if (k >= m->knot_step[n - 1]) {
        T = m->knot_T[n - 1];
    } else {
        int j = 0;
        while (!(k >= m->knot_step[j] && k < m->knot_step[j + 1])) ++j;
        double ka = (double)m->knot_step[j], kb = (double)m->knot_step[j + 1];
        double frac = ((double)k - ka) / (kb - ka);
        int g = m->knot_gamma[j];
        double w = frac;
        if (g > 1) {
            for (int i = 1; i < g; ++i) w = w * frac;
        } else if (g < 0) {
            double r = 1.0 - frac;
            w = r;
            for (int i = 1; i < -g; ++i) w = w * r;
            w = 1.0 - w;
        }
        T = m->knot_T[j] + (m->knot_T[j + 1] - m->knot_T[j]) * w;
    }
    if (T < 0.0) T = 0.0;
    return T;
}

/* ------------------------------------------------------------------ lattice */
static int64_t site(const xyo_model* m, int64_t x, int64_t y) {
    x = ((x % m->Lx) + m->Lx) % m->Lx;
    y = ((y % m->Ly) + m->Ly) % m->Ly;
    return y * m->Lx + x;
}

int32_t xyo_stagger(const xyo_model* m, int64_t i) {
    int64_t x = i % m->Lx, y = i / m->Lx;
    int64_t e = (m->Jx > 0.0 ? x : 0) + (m->Jy > 0.0 ? y : 0);
    return (e & 1) ? -1 : 1;
}

/* Half-width W of the state space [-W, W): pi, or pi/2 for the Si mapping,
 * whose rotors are half circles (Sec. III.C). */
static double half_width(const xyo_model* m) {
    return m->model == XYO_MODEL_SI ? PI64 / 2.0 : PI64;
}

void xyo_init_random(const xyo_model* m, double* theta, double* omega) {
    const int64_t N = (int64_t)m->Lx * m->Ly;
    const uint64_t kinit = ~(uint64_t)0;
    const double W = half_width(m);
    for (int64_t i = 0; i < N; ++i) {
        uint32_t r[4];
        philox_block(m, kinit, i, r);
        double u = xyo_uniform(r[i & 3]);
        theta[i] = W * (2.0 * u - 1.0);
        omega[i] = 0.0;
    }
}

void xyo_init_ordered(const xyo_model* m, int32_t sign, double* theta, double* omega) {
    const int64_t N = (int64_t)m->Lx * m->Ly;
    /* Si mapping: -h cos(p th) with h < 0 has its minima at th = +-pi/p */
    const double th0 = (m->h < 0.0 && m->p > 2.0) ? PI64 / m->p : 0.0;
    for (int64_t i = 0; i < N; ++i) {
        int s = xyo_stagger(m, i) * (sign >= 0 ? 1 : -1);
        if (m->model == XYO_MODEL_SI)
            theta[i] = s > 0 ? th0 : -th0;
        else
            theta[i] = (s > 0) ? 0.0 : -PI64;
        omega[i] = 0.0;
    }
}

/* E_pot = sum over sites of the bond to the +x neighbour, the bond to the +y
 * neighbour and the on-site term; every bond is counted once. */
double xyo_energy_pot(const xyo_model* m, const double* theta) {
    const int Lx = m->Lx, Ly = m->Ly;
    const int si = m->model == XYO_MODEL_SI;
    double* row = (double*)calloc((size_t)Ly, sizeof(double));
#pragma omp parallel for schedule(static)
    for (int y = 0; y < Ly; ++y) {
        double s = 0.0;
        for (int x = 0; x < Lx; ++x) {
            double t = theta[site(m, x, y)];
            double e;
            if (si)
                e = m->Jx * cos(2.0 * (t - theta[site(m, x + 1, y)])) +
                    m->Jy * cos(2.0 * (t - theta[site(m, x, y + 1)])) - m->h * cos(m->p * t);
            else
                e = m->Jx * cos(t - theta[site(m, x + 1, y)]) +
                    m->Jy * cos(t - theta[site(m, x, y + 1)]) - m->h * cos(2.0 * t);
            s += e;
        }
        row[y] = s;
    }
    double E = 0.0;
    for (int y = 0; y < Ly; ++y) E += row[y];
    free(row);
    return E;
}

/* F_i = -dH/dth_i.  XY:
 *   F_i = Jx [sin(th_i - th_{i+x}) + sin(th_i - th_{i-x})]
 *       + Jy [sin(th_i - th_{i+y}) + sin(th_i - th_{i-y})] - 2 h sin(2 th_i);
 * Si mapping (q = 2):
 *   F_i = 2 Jx [sin(2 (th_i - th_{i+x})) + sin(2 (th_i - th_{i-x}))]
 *       + 2 Jy [sin(2 (th_i - th_{i+y})) + sin(2 (th_i - th_{i-y}))]
 *       - p h sin(p th_i). */
void xyo_force(const xyo_model* m, const double* theta, double* F) {
    const int Lx = m->Lx, Ly = m->Ly;
    const int si = m->model == XYO_MODEL_SI;
#pragma omp parallel for schedule(static)
    for (int y = 0; y < Ly; ++y) {
        for (int x = 0; x < Lx; ++x) {
            double t = theta[site(m, x, y)];
            if (si) {
                double fx = sin(2.0 * (t - theta[site(m, x + 1, y)])) + sin(2.0 * (t - theta[site(m, x - 1, y)]));
                double fy = sin(2.0 * (t - theta[site(m, x, y + 1)])) + sin(2.0 * (t - theta[site(m, x, y - 1)]));
                F[site(m, x, y)] = 2.0 * m->Jx * fx + 2.0 * m->Jy * fy - m->p * m->h * sin(m->p * t);
            } else {
                double fx = sin(t - theta[site(m, x + 1, y)]) + sin(t - theta[site(m, x - 1, y)]);
                double fy = sin(t - theta[site(m, x, y + 1)]) + sin(t - theta[site(m, x, y - 1)]);
                F[site(m, x, y)] = m->Jx * fx + m->Jy * fy - 2.0 * m->h * sin(2.0 * t);
            }
        }
    }
}

/* ------------------------------------------------------------------- BBK */
typedef struct {
    double a, c, hdt, dt;
} bbk_coef;

static bbk_coef coefficients(const xyo_model* m) {
    bbk_coef b;
    b.a = 1.0 - 0.5 * m->gamma * m->dt;
    b.c = 1.0 / (1.0 + 0.5 * m->gamma * m->dt);
    b.hdt = 0.5 * m->dt;
    b.dt = m->dt;
    return b;
}

/* Noise amplitude of one half-kick: (1/2) sqrt(2 gamma T_k dt). */
static double half_sigma(const xyo_model* m, uint64_t k) {
    return 0.5 * sqrt(2.0 * m->gamma * xyo_temperature(m, k) * m->dt);
}

/* Back into [-W, W) by one shift of 2W (Sec. III.D). */
static double wrap(double t, double W) {
    if (t >= W)
        t -= 2.0 * W;
    else if (t < -W)
        t += 2.0 * W;
    return t;
}

/* One BBK step of the whole lattice.  On entry F and n hold F(theta^k) and
 * n^k; on exit they hold F(theta^{k+1}) and n^{k+1}.  whalf receives
 * omega(t + dt/2) of every site. */
static int bbk_step(const xyo_model* m, const bbk_coef* b, uint64_t k, double* theta,
                    double* omega, double* F, double* n, double* whalf) {
    const int64_t N = (int64_t)m->Lx * m->Ly;
    const double hs0 = half_sigma(m, k);
    const double W = half_width(m);
    int fault = 0;
    /* Eq. BBK-1 (half-kick), then the drift and the wrap. */
#pragma omp parallel for schedule(static) reduction(| : fault)
    for (int64_t i = 0; i < N; ++i) {
        double t = b->hdt * F[i];
        t = fma(hs0, n[i], t);
        double w = fma(b->a, omega[i], t);
        whalf[i] = w;
        double th = wrap(fma(b->dt, w, theta[i]), W);
        if (!(fabs(th) <= 3.0 * W)) fault = 1;
        theta[i] = th;
    }
    /* Eq. BBK-2 (second half-kick) with the force at the new angles. */
    xyo_force(m, theta, F);
    xyo_normals(m, k + 1, n);
    const double hs1 = half_sigma(m, k + 1);
#pragma omp parallel for schedule(static) reduction(| : fault)
    for (int64_t i = 0; i < N; ++i) {
        double t = fma(b->hdt, F[i], whalf[i]);
        t = fma(hs1, n[i], t);
        double w = b->c * t;
        if (!isfinite(w)) fault = 1;
        omega[i] = w;
    }
    return fault ? -1 : 0;
}

int64_t xyo_run_measured(const xyo_model* m, double* theta, double* omega, uint64_t k0,
                         uint64_t nsteps, uint64_t every, double* out) {
    const int64_t N = (int64_t)m->Lx * m->Ly;
    double* F = (double*)malloc(sizeof(double) * (size_t)N);
    double* n = (double*)malloc(sizeof(double) * (size_t)N);
    double* wh = (double*)malloc(sizeof(double) * (size_t)N);
    if (!F || !n || !wh) {
        free(F); free(n); free(wh);
        return -1;
    }
    bbk_coef b = coefficients(m);
    xyo_force(m, theta, F);
    xyo_normals(m, k0, n);
    int64_t ns = 0;
    int rc = 0;
    for (uint64_t j = 0; j <= nsteps; ++j) {
        if (out && every > 0 && j % every == 0) {
            xyo_observables(m, theta, omega, out + ns * XYO_NOBS);
            ++ns;
        }
        if (j == nsteps) break;
        if (bbk_step(m, &b, k0 + j, theta, omega, F, n, wh) != 0) {
            rc = -1;
            break;
        }
    }
    free(F); free(n); free(wh);
    return rc ? -1 : ns;
}

int32_t xyo_run(const xyo_model* m, double* theta, double* omega, uint64_t k0, uint64_t nsteps) {
    return xyo_run_measured(m, theta, omega, k0, nsteps, 0, NULL) < 0 ? -1 : 0;
}

/* ------------------------------------------------------------ observables */
/* F(q) = (1/N) sum_{kappa} | sum_i eps_i s^kappa_i exp(-i q.r_i) |^2 over the
 * two rotor components (the lattice Fourier transform of App. C at one wave
 * vector).  XY: s^0 = cos th (the order-parameter component), s^1 = sin th;
 * Si mapping: s^0 = sin 2 th (Sec. IV.A), s^1 = cos 2 th. */
void xyo_observables(const xyo_model* m, const double* theta, const double* omega, double* out) {
    const int Lx = m->Lx, Ly = m->Ly;
    const double N = (double)Lx * (double)Ly;
    const int si = m->model == XYO_MODEL_SI;
    double epot = xyo_energy_pot(m, theta);
    double ekin = 0.0, ms = 0.0, a0s = 0.0;
    double kxr[2] = {0, 0}, kxi[2] = {0, 0}, kyr[2] = {0, 0}, kyi[2] = {0, 0};
    for (int y = 0; y < Ly; ++y) {
        for (int x = 0; x < Lx; ++x) {
            int64_t i = (int64_t)y * Lx + x;
            double e = (double)xyo_stagger(m, i);
            double s[2];
            if (si) {
                s[0] = e * sin(2.0 * theta[i]);
                s[1] = e * cos(2.0 * theta[i]);
            } else {
                s[0] = e * cos(theta[i]);
                s[1] = e * sin(theta[i]);
            }
            ekin += 0.5 * omega[i] * omega[i];
            ms += s[0];
            a0s += s[1];
            double qx = TWO_PI64 * (double)x / (double)Lx;
            double qy = TWO_PI64 * (double)y / (double)Ly;
            for (int kap = 0; kap < 2; ++kap) {
                kxr[kap] += s[kap] * cos(qx);
                kxi[kap] -= s[kap] * sin(qx);
                kyr[kap] += s[kap] * cos(qy);
                kyi[kap] -= s[kap] * sin(qy);
            }
        }
    }
    out[0] = epot / N;
    out[1] = ekin / N;
    out[2] = ms / N;
    out[3] = (ms * ms + a0s * a0s) / N;
    out[4] = (kxr[0] * kxr[0] + kxi[0] * kxi[0] + kxr[1] * kxr[1] + kxi[1] * kxi[1]) / N;
    out[5] = (kyr[0] * kyr[0] + kyi[0] * kyi[0] + kyr[1] * kyr[1] + kyi[1] * kyi[1]) / N;
}

/* C(r) = (1/N) sum_i eps_i eps_j cos(q (th_i - th_j)), j = i + r along the axis
 * (q = 1 for XY, 2 for the Si mapping: the dot product of the rotors). */
void xyo_correlation(const xyo_model* m, const double* theta, int32_t axis, int32_t rmax, double* C) {
    const int Lx = m->Lx, Ly = m->Ly;
    const double N = (double)Lx * (double)Ly;
    const double q = m->model == XYO_MODEL_SI ? 2.0 : 1.0;
    for (int r = 0; r <= rmax; ++r) {
        double s = 0.0;
        for (int y = 0; y < Ly; ++y)
            for (int x = 0; x < Lx; ++x) {
                int64_t i = site(m, x, y);
                int64_t j = axis == 0 ? site(m, x + r, y) : site(m, x, y + r);
                s += (double)(xyo_stagger(m, i) * xyo_stagger(m, j)) * cos(q * (theta[i] - theta[j]));
            }
        C[r] = s / N;
    }
}

/* ---------------------------------------------------------------- domains */
/* Spin sigma_i = eps_i * (|th_i| <= pi_p/2 ? +1 : -1) (XY) or
 * eps_i * (th_i >= 0 ? +1 : -1) (Si mapping).  Flood fill in order of
 * increasing linear index, so each cluster is labelled by its smallest index. */
int64_t xyo_domains(const xyo_model* m, const double* theta, int32_t precision_bits, int32_t* labels) {
    const int Lx = m->Lx, Ly = m->Ly;
    const int64_t N = (int64_t)Lx * Ly;
    const double pi_p = precision_bits == 32 ? (double)(float)PI64 : PI64;
    const double half = pi_p / 2.0;
    int8_t* spin = (int8_t*)malloc((size_t)N);
    int64_t* queue = (int64_t*)malloc(sizeof(int64_t) * (size_t)N);
    if (!spin || !queue) {
        free(spin); free(queue);
        return -1;
    }
    for (int64_t i = 0; i < N; ++i) {
        int up = m->model == XYO_MODEL_SI ? theta[i] >= 0.0 : fabs(theta[i]) <= half;
        spin[i] = (int8_t)(xyo_stagger(m, i) * (up ? 1 : -1));
        labels[i] = -1;
    }
    int64_t ndom = 0;
    for (int64_t s0 = 0; s0 < N; ++s0) {
        if (labels[s0] >= 0) continue;
        ++ndom;
        int64_t head = 0, tail = 0;
        queue[tail++] = s0;
        labels[s0] = (int32_t)s0;
        while (head < tail) {
            int64_t i = queue[head++];
            int64_t x = i % Lx, y = i / Lx;
            int64_t nb[4] = {site(m, x + 1, y), site(m, x - 1, y), site(m, x, y + 1), site(m, x, y - 1)};
            for (int d = 0; d < 4; ++d) {
                int64_t j = nb[d];
                if (labels[j] < 0 && spin[j] == spin[i]) {
                    labels[j] = (int32_t)s0;
                    queue[tail++] = j;
                }
            }
        }
    }
    free(spin);
    free(queue);
    return ndom;
}

/* ---------------------------------------------------------------- adjoint */
static double order_parameter(const xyo_model* m, const double* theta) {
    const int64_t N = (int64_t)m->Lx * m->Ly;
    double s = 0.0;
    for (int64_t i = 0; i < N; ++i) s += (double)xyo_stagger(m, i) * cos(theta[i]);
    return s / (double)N;
}

double xyo_loss(const xyo_model* m, const double* theta0, const double* omega0, uint64_t nsteps,
                uint64_t window) {
    const int64_t N = (int64_t)m->Lx * m->Ly;
    if (m->model != XYO_MODEL_XY) return NAN;
    double* th = (double*)malloc(sizeof(double) * (size_t)N);
    double* om = (double*)malloc(sizeof(double) * (size_t)N);
    double* out = (double*)malloc(sizeof(double) * XYO_NOBS * (size_t)(nsteps + 1));
    if (!th || !om || !out) {
        free(th); free(om); free(out);
        return NAN;
    }
    memcpy(th, theta0, sizeof(double) * (size_t)N);
    memcpy(om, omega0, sizeof(double) * (size_t)N);
    double L = NAN;
    if (xyo_run_measured(m, th, om, 0, nsteps, 1, out) >= 0) {
        L = 0.0;
        for (uint64_t k = nsteps - window + 1; k <= nsteps; ++k) {
            double ms = out[k * XYO_NOBS + 2];
            L += ms * ms;
        }
        L /= (double)window;
    }
    free(th); free(om); free(out);
    return L;
}

/* Reverse mode of the three BBK stages, step by step, with the stored
 * trajectory.  For one step s = (th, w) -> (th', w'):
 *     wh  = a w + hdt F(th) + hs_k n^k
 *     th' = wrap(th + dt wh)                      (wrap has derivative 1)
 *     w'  = c (wh + hdt F(th') + hs_{k+1} n^{k+1})
 * and dF/dth is the symmetric matrix
 *     (J v)_i = sum_d Jd sum_pm cos(th_i - th_{i pm d}) (v_i - v_{i pm d})
 *               - 4 h cos(2 th_i) v_i. */
static void jacobian_apply(const xyo_model* m, const double* th, const double* v, double* out) {
    const int Lx = m->Lx, Ly = m->Ly;
#pragma omp parallel for schedule(static)
    for (int y = 0; y < Ly; ++y)
        for (int x = 0; x < Lx; ++x) {
            int64_t i = site(m, x, y);
            int64_t nx[2] = {site(m, x + 1, y), site(m, x - 1, y)};
            int64_t ny[2] = {site(m, x, y + 1), site(m, x, y - 1)};
            double s = 0.0;
            for (int d = 0; d < 2; ++d) {
                s += m->Jx * cos(th[i] - th[nx[d]]) * (v[i] - v[nx[d]]);
                s += m->Jy * cos(th[i] - th[ny[d]]) * (v[i] - v[ny[d]]);
            }
            s -= 4.0 * m->h * cos(2.0 * th[i]) * v[i];
            out[i] = s;
        }
}

/* Accumulates sum_i v_i dF_i/d{Jx, Jy, h} into g[0..2]. */
static void force_param_grad(const xyo_model* m, const double* th, const double* v, double* g) {
    const int Lx = m->Lx, Ly = m->Ly;
    double gx = 0.0, gy = 0.0, gh = 0.0;
    for (int y = 0; y < Ly; ++y)
        for (int x = 0; x < Lx; ++x) {
            int64_t i = site(m, x, y);
            double dx = sin(th[i] - th[site(m, x + 1, y)]) + sin(th[i] - th[site(m, x - 1, y)]);
            double dy = sin(th[i] - th[site(m, x, y + 1)]) + sin(th[i] - th[site(m, x, y - 1)]);
            double dh = -2.0 * sin(2.0 * th[i]);
            gx += v[i] * dx;
            gy += v[i] * dy;
            gh += v[i] * dh;
        }
    g[0] += gx;
    g[1] += gy;
    g[2] += gh;
}

double xyo_adjoint(const xyo_model* m, const double* theta0, const double* omega0, uint64_t nsteps,
                   uint64_t window, double* grad, double* dtheta0, double* domega0) {
    const int64_t N = (int64_t)m->Lx * m->Ly;
    const size_t sz = sizeof(double) * (size_t)N;
    if (window == 0 || window > nsteps || m->model != XYO_MODEL_XY) return NAN;
    double* TH = (double*)malloc(sz * (size_t)(nsteps + 1));
    double* W = (double*)malloc(sz * (size_t)(nsteps + 1));
    double* WH = (double*)malloc(sz * (size_t)(nsteps + 1));
    double* F = (double*)malloc(sz);
    double* n = (double*)malloc(sz);
    double* lth = (double*)calloc((size_t)N, sizeof(double));
    double* lw = (double*)calloc((size_t)N, sizeof(double));
    double* lwh = (double*)malloc(sz);
    double* tmp = (double*)malloc(sz);
    double* jv = (double*)malloc(sz);
    double* nk = (double*)malloc(sz);
    double loss = NAN;
    if (!TH || !W || !WH || !F || !n || !lth || !lw || !lwh || !tmp || !jv || !nk) goto done;

    /* Forward sweep, storing every state and every omega(t + dt/2). */
    {
        bbk_coef b = coefficients(m);
        memcpy(TH, theta0, sz);
        memcpy(W, omega0, sz);
        xyo_force(m, TH, F);
        xyo_normals(m, 0, n);
        for (uint64_t k = 0; k < nsteps; ++k) {
            memcpy(TH + (k + 1) * N, TH + k * N, sz);
            memcpy(W + (k + 1) * N, W + k * N, sz);
            if (bbk_step(m, &b, k, TH + (k + 1) * N, W + (k + 1) * N, F, n, WH + k * N) != 0) goto done;
        }
        double msum = 0.0;
        for (uint64_t k = nsteps - window + 1; k <= nsteps; ++k) {
            double ms = order_parameter(m, TH + k * N);
            msum += ms * ms;
        }
        loss = msum / (double)window;

        /* Reverse sweep. */
        double ga = 0.0, gc = 0.0, ggam_hs = 0.0;
        double gp[3] = {0.0, 0.0, 0.0};
        for (uint64_t kk = nsteps + 1; kk-- > 0;) {
            /* Direct loss term at step kk: dL/dth_i = (2 m / W) (-eps_i sin th_i) / N. */
            if (kk >= nsteps - window + 1) {
                const double* th = TH + kk * N;
                double ms = order_parameter(m, th);
                for (int64_t i = 0; i < N; ++i)
                    lth[i] += (2.0 * ms / (double)window) * (-(double)xyo_stagger(m, i) * sin(th[i])) / (double)N;
            }
            if (kk == 0) break;
            const uint64_t k = kk - 1; /* undo step k: state k -> k+1 */
            const double* th0 = TH + k * N;
            const double* th1 = TH + kk * N;
            const double* w0 = W + k * N;
            const double* w1 = W + kk * N;
            const double* wh = WH + k * N;
            const double hs0 = half_sigma(m, k), hs1 = half_sigma(m, kk);
            /* w' = c B,  B = wh + hdt F(th') + hs1 n^{k+1} */
            (void)w1;
            xyo_normals(m, kk, nk);
            xyo_force(m, th1, F);
            for (int64_t i = 0; i < N; ++i) {
                double B = wh[i] + b.hdt * F[i] + hs1 * nk[i];
                gc += lw[i] * B;
                if (hs1 > 0.0) ggam_hs += b.c * lw[i] * nk[i] * hs1 / (2.0 * m->gamma);
                tmp[i] = b.c * lw[i]; /* dL/dB */
                lwh[i] = tmp[i];
            }
            /* through F(th') */
            for (int64_t i = 0; i < N; ++i) jv[i] = b.hdt * tmp[i];
            force_param_grad(m, th1, jv, gp);
            jacobian_apply(m, th1, jv, tmp);
            for (int64_t i = 0; i < N; ++i) lth[i] += tmp[i];
            /* th' = th + dt wh */
            for (int64_t i = 0; i < N; ++i) lwh[i] += b.dt * lth[i];
            /* wh = a w + hdt F(th) + hs0 n^k */
            xyo_normals(m, k, nk);
            for (int64_t i = 0; i < N; ++i) {
                ga += lwh[i] * w0[i];
                if (hs0 > 0.0) ggam_hs += lwh[i] * nk[i] * hs0 / (2.0 * m->gamma);
                jv[i] = b.hdt * lwh[i];
            }
            force_param_grad(m, th0, jv, gp);
            jacobian_apply(m, th0, jv, tmp);
            for (int64_t i = 0; i < N; ++i) {
                lth[i] += tmp[i]; /* lth now holds dL/dth^k (th' passed through with derivative 1) */
                lw[i] = b.a * lwh[i];
            }
        }
        if (grad) {
            grad[0] = gp[0];
            grad[1] = gp[1];
            grad[2] = gp[2];
            /* a = 1 - gamma dt/2, c = 1/(1 + gamma dt/2), hs = (1/2) sqrt(2 gamma T dt) */
            grad[3] = ga * (-0.5 * m->dt) + gc * (-0.5 * m->dt * b.c * b.c) + ggam_hs;
        }
        if (dtheta0) memcpy(dtheta0, lth, sz);
        if (domega0) memcpy(domega0, lw, sz);
    }
done:
    free(TH); free(W); free(WH); free(F); free(n); free(lth); free(lw);
    free(lwh); free(tmp); free(jv); free(nk);
    return loss;
}
