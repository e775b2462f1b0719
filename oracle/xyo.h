/*
 * xyo — plain FP64 CPU oracle for Langevin dynamics of the symmetry-broken XY
 * lattice (Weitzel, Schaller, Queisser, Schützhold, arXiv:2409.06412).
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists to check the HIP product path.
 * Only the tests, the smoke check and the CPU-baseline leg of the benchmark may
 * load it.  It shares no code, header, table or helper with the HIP library.
 *
 * Models (paper Sec. III.A, Eq. XY-Hamilton-Field, written with the sign
 * convention used by this project):
 *   XYO_MODEL_XY (q = 1, p = 2, angles in [-pi, pi)):
 *     H = sum_i [ Jx cos(th_i - th_{i+x}) + Jy cos(th_i - th_{i+y})
 *                 - h cos(2 th_i) + omega_i^2 / 2 ]
 *   XYO_MODEL_SI (the paper's Si(001) mapping of Sec. III.C: q = 2, real p,
 *   angles in [-pi/2, pi/2)):
 *     H = sum_i [ Jx cos(2 (th_i - th_{i+x})) + Jy cos(2 (th_i - th_{i+y}))
 *                 - h cos(p th_i) + omega_i^2 / 2 ]
 *   (the paper's J_par, J_perp, h are -Jx, -Jy, -h here).
 * on an Lx x Ly periodic lattice, site (x, y) at linear index i = y*Lx + x.
 * Dynamics: Langevin equations of Sec. III.D (Eq. Si-Langevin) with I = kB = 1,
 * integrated by the three-stage BBK scheme of App. A.1 (Eqs. BBK-1, BBK-2).
 * All arithmetic is IEEE binary64, round to nearest, no contraction.
 */
#ifndef XYO_H
#define XYO_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define XYO_MAX_KNOTS 16
#define XYO_NOBS 6
#define XYO_MODEL_XY 0
#define XYO_MODEL_SI 1

typedef struct {
    int32_t Lx, Ly;
    double Jx, Jy, h, gamma, dt;
    uint64_t seed;
    uint32_t replica;
    int32_t nknots;                      /* >= 1; one knot = constant T */
    uint64_t knot_step[XYO_MAX_KNOTS];   /* strictly increasing */
    double knot_T[XYO_MAX_KNOTS];        /* >= 0 */
    int32_t model;                       /* XYO_MODEL_XY or XYO_MODEL_SI */
    double p;                            /* field order of XYO_MODEL_SI (> 0) */
    int32_t knot_gamma[XYO_MAX_KNOTS];   /* shape of the segment from knot j: 0 or 1 linear,
                                            g > 1: w = f^g, g < 0: w = 1 - (1 - f)^|g| */
} xyo_model;

/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): one block. */
void xyo_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
/* Uniform in (0,1): ((r >> 9) + 1/2) * 2^-23. */
double xyo_uniform(uint32_t r);
/* Gaussian draw n_i^k of site i at step k (Box-Muller on the Philox block
 * with counter (i>>2, replica, k_lo, k_hi) and key (seed_lo, seed_hi)). */
double xyo_normal(const xyo_model* m, uint64_t k, int64_t i);
void xyo_normals(const xyo_model* m, uint64_t k, double* n);
/* Temperature T_k between knots a, b: T_a + (T_b - T_a) w with f = (k - k_a) /
 * (k_b - k_a) and w = f (linear, Sec. II.B Eq. Linear-Quench), w = f^g or
 * w = 1 - (1 - f)^|g| (the nonlinear protocols eps ~ t^g of Sec. V), powers
 * by repeated multiplication; held outside the knots. */
double xyo_temperature(const xyo_model* m, uint64_t k);

/* Initial states.  Random: th_i = W (2U - 1) from the reserved init stream
 * (step counter 2^64 - 1), omega = 0, with W = pi (XY) or pi/2 (SI).
 * Ordered: XY: staggered ground state th in {0, -pi}; SI: th_i = +-eps_i th0
 * with th0 = pi/p, the on-site minimum, when h < 0 and p > 2, else th0 = 0. */
void xyo_init_random(const xyo_model* m, double* theta, double* omega);
void xyo_init_ordered(const xyo_model* m, int32_t sign, double* theta, double* omega);
/* Staggering sign eps_i in {+1,-1}. */
int32_t xyo_stagger(const xyo_model* m, int64_t i);

/* Potential energy (total) and force F_i = -dH/dth_i. */
double xyo_energy_pot(const xyo_model* m, const double* theta);
void xyo_force(const xyo_model* m, const double* theta, double* F);

/* Advance (theta, omega) at step k0 by nsteps BBK steps.  Returns 0, or -1 on a
 * numeric fault (non-finite omega or |theta| > 3 pi after the wrap). */
int32_t xyo_run(const xyo_model* m, double* theta, double* omega, uint64_t k0, uint64_t nsteps);
/* Same, recording observables at k0 + j*every for j*every <= nsteps into
 * out[j*XYO_NOBS ...].  Returns the number of samples or -1. */
int64_t xyo_run_measured(const xyo_model* m, double* theta, double* omega, uint64_t k0,
                         uint64_t nsteps, uint64_t every, double* out);

/* Observables of a synchronized state, per site where noted:
 * out = {E_pot/N, E_kin/N, m_s, F(0), F(kx_min), F(ky_min)}.
 * The rotor of a site is (cos q th, sin q th); the order parameter m_s is the
 * staggered mean of cos th (XY) or of sin 2 th (SI, Sec. IV.A). */
void xyo_observables(const xyo_model* m, const double* theta, const double* omega, double* out);
/* Staggered rotor correlation C_axis(r), r = 0..rmax (axis 0 = x, 1 = y). */
void xyo_correlation(const xyo_model* m, const double* theta, int32_t axis, int32_t rmax, double* C);
/* Frozen domains: labels[i] = smallest linear index of the 4-connected periodic
 * cluster of equal staggered spin.  XY: the spin is +1 where |th| <= pi_p / 2
 * with pi_p the value of pi in the state precision (precision_bits 32 or 64);
 * SI: +1 where th >= 0 (the sign of sin 2 th).  Returns the number of domains. */
int64_t xyo_domains(const xyo_model* m, const double* theta, int32_t precision_bits, int32_t* labels);

/* Pathwise reverse-mode gradient of L = (1/W) sum_{k=N-W+1}^{N} m_s(theta^k)^2
 * with the Gaussian draws held fixed.  grad = dL/d{Jx, Jy, h, gamma};
 * dtheta0, domega0 = dL/d(initial state) (may be NULL).  Returns L, or NaN on a
 * numeric fault / allocation failure, and for XYO_MODEL_SI (whose on-site force
 * jumps at the wrap point, so the pathwise derivative does not exist). */
double xyo_adjoint(const xyo_model* m, const double* theta0, const double* omega0,
                   uint64_t nsteps, uint64_t window, double* grad, double* dtheta0, double* domega0);
/* The same loss by a plain forward run (for finite differences). */
double xyo_loss(const xyo_model* m, const double* theta0, const double* omega0,
                uint64_t nsteps, uint64_t window);

#ifdef __cplusplus
}
#endif
#endif
