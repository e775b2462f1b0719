/*
 * xyl.h — C-ABI of the MI355X (gfx950) Langevin-XY library.
 *
 * The library time-steps the underdamped Langevin equations of the angles
 * th_i and angular velocities w_i of a periodic Lx x Ly lattice under the
 * symmetry-broken XY Hamiltonian of Weitzel, Schaller, Queisser, Schützhold,
 * "Continuous Dimer Angles on the Silicon Surface" (arXiv:2409.06412),
 * Sec. III.A, Eq. XY-Hamilton-Field, taken at q = 1, p = 2 and written as
 *
 *     H = sum_i [ Jx cos(th_i - th_{i+x}) + Jy cos(th_i - th_{i+y})
 *                 - h cos(2 th_i) + w_i^2 / 2 ]                          (1)
 *
 * (kinetic term of Eq. XY-Hamilton-Kinetic with I = 1; every bond counted
 * once).  Jx > 0 favours antiparallel neighbours along x (the dimer rows).
 * The dynamics is Eq. Si-Langevin (Sec. III.D),
 *     d th/dt = w,   d w/dt = -gamma w - dH/dth + sqrt(2 gamma T(t)) G(t),
 * integrated with the three-stage Brünger-Brooks-Karplus scheme of App. A.1
 * (Eqs. BBK-1, BBK-2): half-kick, drift, half-kick, the Gaussian draw of a
 * step's second half-kick being the draw of the next step's first half-kick,
 * and the angle wrapped to [-pi_p, pi_p) after every step (Sec. III.D), pi_p
 * being pi rounded to the state precision.
 *
 * Noise.  The draw n_i^k of site i = y*Lx + x at step k comes from
 * Philox4x32-10 (Salmon et al., SC'11) with counter (i>>2, replica, k_lo,
 * k_hi) and key (seed_lo, seed_hi): words (2p, 2p+1), p = (i&3)>>1, give
 * U1, U2 with U(r) = ((r>>9) + 1/2) 2^-23, and n = sqrt(-2 ln U1) cos(2 pi U2)
 * for even i, sin(2 pi U2) for odd i.  Results are a pure function of
 * (parameters, schedule, seed, replica, step, lattice size, precision); they
 * do not depend on launch shape, batching or steps per launch.
 *
 * Layout.  Every per-site array is row-major, x fastest: element (x, y) at
 * y*Lx + x.  Host arrays passed to the library are float64 regardless of the
 * state precision; device states are float32 (XYL_F32) or float64 (XYL_F64).
 *
 * Errors.  Every call returns XYL_OK (0) or a negative status and records a
 * message for xyl_last_error().  No exception or abort crosses the ABI.
 * A numeric fault (non-finite angles, velocities or observables, e.g. from a
 * step size far too large) is reported as XYL_ENUMERIC by the calls that
 * bring results to the host (xyl_get_state, xyl_measure, xyl_step_measured),
 * after the values have been written.
 * Calls are asynchronous on the handle's stream unless they write host memory,
 * in which case they synchronise that stream first.  A handle is used by one
 * host thread at a time.
 */
#ifndef XYL_H
#define XYL_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define XYL_ABI_VERSION 5

enum {
    XYL_OK = 0,
    XYL_EINVAL = -1,       /* invalid argument */
    XYL_ENOMEM = -2,       /* device or host allocation failed */
    XYL_EDEVICE = -3,      /* HIP runtime error or no gfx950 device */
    XYL_ESTATE = -4,       /* call not valid in the handle's current state */
    XYL_EUNSUPPORTED = -5, /* shape or mode not supported */
    XYL_ENUMERIC = -6      /* non-finite value detected */
};

enum { XYL_F32 = 0, XYL_F64 = 1 };

#define XYL_MAX_KNOTS 16

/* One measurement at a synchronized step k (App. B; Sec. IV.A; App. C):
 *   e_pot = (1/N) sum of the potential terms of (1)
 *   e_kin = (1/N) sum w_i^2 / 2
 *   m_s   = (1/N) sum eps_i cos th_i         (staggered order parameter)
 *   f0, fkx, fky = F(q) = (1/N) sum_{kappa} |sum_i eps_i s^kappa_i e^{-i q.r_i}|^2
 *           at q = 0, (2 pi/Lx, 0), (0, 2 pi/Ly); s^0 = cos th, s^1 = sin th
 * with eps_i = (-1)^(x [Jx > 0] + y [Jy > 0]). */
typedef struct {
    double e_pot, e_kin, m_s, f0, fkx, fky;
} xyl_obs;

/* Models (Sec. III.A, Eq. XY-Hamilton-Field, with H = sum Jx cos(q dth_x)
 * + Jy cos(q dth_y) - h cos(p th) in this library's sign convention, so the
 * paper's J_par, J_perp and h are -Jx, -Jy and -h):
 *   XYL_MODEL_XY: q = 1, p = 2, angles in [-pi, pi); rotor (cos th, sin th),
 *                 order-parameter component cos th.  The default.
 *   XYL_MODEL_SI: the Si(001) dimer mapping of Sec. III.C: q = 2, real p
 *                 (the paper uses 2.5), angles in [-pi/2, pi/2) (a modulo after
 *                 every step, Sec. III.D); rotor (cos 2th, sin 2th),
 *                 order-parameter component sin 2th (Sec. IV.A, Eq.
 *                 lattice-average); domain spin eps_i * (th_i >= 0 ? +1 : -1).
 *                 The field's force jumps at +-pi/2, so the adjoint calls
 *                 refuse this model (XYL_EUNSUPPORTED). */
enum { XYL_MODEL_XY = 0, XYL_MODEL_SI = 1 };

typedef struct xyl_lattice xyl_lattice;
typedef struct xyl_ensemble xyl_ensemble;

/* ---------------------------------------------------------------- library */
int xyl_abi_version(void);
/* Message of the last failing call on this thread ("" if none).  Valid until
 * the next call on the same thread. */
const char* xyl_last_error(void);
/* Number of visible gfx950 devices (0 if none).  Never fails. */
int xyl_device_count(void);

/* ---------------------------------------------------------------- lattice */
/* Creates an Lx x Ly lattice on HIP device `device` with library-owned device
 * buffers (two angle buffers and one velocity buffer of the given precision).
 * Lx, Ly >= 2, Lx*Ly < 2^34.  Default parameters: Jx = 1, Jy = -0.1, h = 0.5,
 * gamma = 1, dt = 0.01, constant T = 0, seed 0, replica 0.  The state is
 * undefined until an init or set_state call (ESTATE before that). */
int xyl_create(xyl_lattice** out, int32_t Lx, int32_t Ly, int32_t dtype, int32_t device);
/* Same, on caller-owned device buffers of Lx*Ly elements of the given
 * precision (e.g. torch tensors): theta_a, theta_b, vel must be distinct, stay
 * alive and unaliased until xyl_destroy.  The current angles live in the
 * buffer reported by xyl_state_buffers. */
int xyl_create_wrapped(xyl_lattice** out, int32_t Lx, int32_t Ly, int32_t dtype, int32_t device,
                       void* theta_a, void* theta_b, void* vel);
int xyl_destroy(xyl_lattice* h); /* NULL is a no-op */
/* HIP stream (hipStream_t) for all later work; NULL = the null stream. */
int xyl_set_stream(xyl_lattice* h, void* stream);
/* Model and integrator parameters (Eq. (1), Eq. Si-Langevin, App. A.1).
 * dt > 0, gamma >= 0, all finite.  Takes effect at the next step. */
int xyl_set_params(xyl_lattice* h, double Jx, double Jy, double hfield, double gamma, double dt);
/* Selects the model (XYL_MODEL_*).  XYL_MODEL_XY needs p = 2; XYL_MODEL_SI
 * takes any finite 0 < p <= 16.  The state becomes undefined (ESTATE until the
 * next init or set_state call), because the two models' angle ranges differ. */
int xyl_set_model(xyl_lattice* h, int32_t model, double p);
/* Temperature schedule T(k), piecewise linear in the step index between knots
 * (k_j, T_j) and held outside them (Sec. II.B, Eq. Linear-Quench, with the
 * reduced temperature written as T).  1 <= n <= XYL_MAX_KNOTS, knot steps
 * strictly increasing, T_j >= 0 and finite. */
int xyl_set_schedule(xyl_lattice* h, const uint64_t* knot_step, const double* knot_T, int32_t n);
/* The same with a shape per segment (the nonlinear quench protocols
 * eps(t) ~ t^g of Sec. V): between knots j and j+1, with f the fraction of
 * the segment elapsed, T = T_j + (T_{j+1} - T_j) w where w = f for
 * knot_gamma[j] in {0, 1}, w = f^g for g > 1 (accelerating away from knot j)
 * and w = 1 - (1 - f)^|g| for g < 0 (decelerating into knot j+1).  Powers are
 * products of f in FP64, |g| <= 16.  A protocol through T_c with
 * eps = -sign(t) |t / tau|^g uses a segment of shape -g into the T_c knot and
 * one of shape g out of it. */
int xyl_set_schedule_shaped(xyl_lattice* h, const uint64_t* knot_step, const double* knot_T,
                            const int32_t* knot_gamma, int32_t n);
int xyl_set_seed(xyl_lattice* h, uint64_t seed, uint32_t replica);
/* th_i = W (2 U(w_{i&3}) - 1) from the Philox block of counter
 * (i>>2, replica, 2^32-1, 2^32-1) (the reserved step 2^64 - 1), with W = pi
 * (XY) or pi/2 (SI), computed in float64 and rounded to the state precision;
 * w = 0; step k = 0. */
int xyl_init_random(xyl_lattice* h);
/* Ordered state; w = 0; k = 0.  XY: th_i = 0 where sign*eps_i = +1, else
 * -pi_p (the staggered ground state).  SI: th_i = sign*eps_i*th0 with
 * th0 = pi/p (the field's minimum) when h < 0 and p > 2, else th0 = 0. */
int xyl_init_ordered(xyl_lattice* h, int32_t sign);
/* Copies a host state (float64, Lx*Ly each; converted to the state precision)
 * and sets the step index.  theta entries must be finite with |th| <= 3 pi
 * (XY) or, after rounding to the state precision, in [-pi_p/2, pi_p/2) (SI). */
int xyl_set_state(xyl_lattice* h, const double* theta, const double* omega, uint64_t step);
/* The same from caller-owned device buffers on the lattice's device: theta
 * and omega hold Lx*Ly elements of precision dtype (XYL_F32 or XYL_F64, e.g.
 * torch tensors), converted to the state precision on the device.  The
 * entries are checked where they lie (same rules as xyl_set_state; EINVAL and
 * the lattice unchanged if any fails); only the verdict crosses to the host.
 * The buffers must not overlap the lattice's own state buffers and must be
 * ready on its stream; the call returns once they have been read. */
int xyl_set_state_device(xyl_lattice* h, const void* theta, const void* omega, int32_t dtype, uint64_t step);
/* Copies the synchronized state (th^k, w^k) at the current step to host
 * float64 arrays (either may be NULL) and the step index (may be NULL). */
int xyl_get_state(xyl_lattice* h, double* theta, double* omega, uint64_t* step);
/* The integrator's own state (App. A.1): the angles th^k, the velocity buffer
 * u (w^{k-1/2}, the first half-kick's result, or w^k itself when *fresh is 1,
 * i.e. right after an init or set_state call) and the step index, as float64
 * host arrays (either may be NULL).  Restoring it with xyl_set_raw_state on a
 * lattice of the same configuration continues the run bit for bit: this is
 * the pair to checkpoint with.  (xyl_set_state with xyl_get_state's
 * synchronized w^k restarts from a fresh state, which agrees only to
 * rounding.)  The entries are checked as by xyl_set_state. */
int xyl_get_raw_state(xyl_lattice* h, double* theta, double* u, uint64_t* step, int32_t* fresh);
int xyl_set_raw_state(xyl_lattice* h, const double* theta, const double* u, uint64_t step, int32_t fresh);
/* Device pointers of the current angle buffer and of the velocity buffer and
 * whether the velocity buffer holds w^k ("fresh", 1) or w^{k-1/2} (0). */
int xyl_state_buffers(xyl_lattice* h, void** theta, void** vel, int32_t* fresh);
/* Advances nsteps BBK steps (stream-ordered, asynchronous). */
int xyl_step(xyl_lattice* h, uint64_t nsteps);
/* Advances nsteps steps and records observables at the current step k0 and at
 * k0 + j*every for j*every <= nsteps (every >= 1).  out has room for cap
 * samples; *nout receives the count (nsteps/every + 1; EINVAL if cap is
 * smaller).  Synchronises. */
int xyl_step_measured(xyl_lattice* h, uint64_t nsteps, uint64_t every, xyl_obs* out, uint64_t cap,
                      uint64_t* nout);
/* Observables at the current step.  Synchronises. */
int xyl_measure(xyl_lattice* h, xyl_obs* out);
/* Adaptive sampling (App. B: samples ds >~ 100 dt apart, ds ~ tau_C / 10,
 * adapted during the run).  Advances nsteps steps from the current step k0,
 * recording observables (and their steps) at k0 and then ds steps apart, ds
 * starting at ds0; the last sample is at k0 + nsteps.  Whenever `block`
 * samples (>= 4; the first block includes the one at k0) have been taken, the
 * integrated autocorrelation time tau of observable `which` (0..5, an xyl_obs
 * field index; automatic window, c = 6) over them, in samples, sets the
 * spacing of the following samples:
 * ds = clamp(floor(ds tau / 10 + 1/2), ds_min, ds_max), 1 <= ds_min <= ds0 <=
 * ds_max.  out and steps have room for cap >= nsteps / ds_min + 2 entries;
 * *nout receives the count.  Synchronises once per block. */
int xyl_step_adaptive(xyl_lattice* h, uint64_t nsteps, uint64_t ds0, uint64_t ds_min, uint64_t ds_max,
                      int32_t which, uint64_t block, xyl_obs* out, uint64_t* steps, uint64_t cap, uint64_t* nout);
/* Staggered rotor correlation along axis (0 = x, 1 = y) at the current step
 * (App. C, two-point function of the rotors, lattice average):
 * C(r) = (1/N) sum_i eps_i eps_j cos(q (th_i - th_j)), j = i + r along the axis,
 * r = 0..rmax, 0 <= rmax <= L_axis/2.  C has rmax+1 entries.  L_axis <= 4096
 * (XYL_EUNSUPPORTED otherwise).  Power-of-two L_axis: from the structure
 * factor, C(r) = (1/L) sum_k S(k) cos(2 pi k r / L) (equal to the pair sums up
 * to rounding; 16 bytes of device scratch per site); other lengths: the pair
 * sums themselves.  Synchronises. */
int xyl_correlation(xyl_lattice* h, int32_t axis, int32_t rmax, double* C);
/* Directional structure factor along axis (0 = x, 1 = y) at the current step
 * (App. C, Eqs. FT-Corr-delta and S-as-lattice-FT):
 * S(k) = sum_r C(r) exp(-2 pi i k r / L) = (1/N) sum over the lines along the
 * axis of sum_kappa |sum_r s^kappa_r exp(-2 pi i k r / L)|^2 with the staggered
 * rotor components s = eps (cos q th, sin q th), for k = 0..kmax,
 * 0 <= kmax <= L_axis/2 (S(L - k) = S(k)).  S has kmax+1 entries.  FP64,
 * summed over lines in a fixed order.  L_axis <= 4096 (XYL_EUNSUPPORTED
 * otherwise); power-of-two L_axis uses an FFT per line, other lengths a
 * direct sum.  Uses 16 bytes of device scratch per site (plus 16 per point
 * of the axis).  Synchronises. */
int xyl_structure_factor(xyl_lattice* h, int32_t axis, int32_t kmax, double* S);
/* Frozen domains of the current angles (Abstract; Figs. 1 and 6): spin
 * s_i = eps_i * (|th_i| <= pi_p/2 ? +1 : -1) (XY; eps_i * (th_i >= 0 ? +1 : -1)
 * for SI), clusters of equal spin under
 * 4-neighbour periodic connectivity.  labels (nullable, Lx*Ly) receives for
 * each site the smallest linear index of its cluster.  The size distribution
 * is returned as pairs (sizes[j], counts[j]) sorted by size, j < *n_sizes;
 * sizes/counts (nullable) have room for cap pairs (EINVAL if too few).
 * n_domains and max_size are nullable.  Synchronises. */
int xyl_domains(xyl_lattice* h, int32_t* labels, uint64_t* sizes, uint64_t* counts, uint64_t cap,
                uint64_t* n_sizes, uint64_t* n_domains, uint64_t* max_size);
/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): xyl_domains
 * with the same arguments and results, run without any device or host heap
 * allocation.  Its working memory is a static device array of the library,
 * one per device (about 48 MiB, held until the process ends), which limits
 * the lattice to at most 2^22 sites (e.g. 2048 x 2048; EINVAL beyond).  Calls
 * in one process are serialised by the library, since they all share the
 * device's array (each process has its own); a call synchronises the
 * handle's stream before it returns. */
int xyl_domains_noalloc(xyl_lattice* h, int32_t* labels, uint64_t* sizes, uint64_t* counts, uint64_t cap,
                        uint64_t* n_sizes, uint64_t* n_domains, uint64_t* max_size);
/* Blocks until all work issued on the handle's stream has finished. */
int xyl_sync(xyl_lattice* h);

/* ------------------------------------------------------ tuning and graphs */
/* Launch shape of the step kernels: rows per strip (>= 1) and waves per
 * workgroup (1, 2, 4 or 8); 0 keeps the current value.  Results do not
 * depend on it.  xyl_autotune times candidates on this lattice (as captured
 * graphs on scratch copies of the state, which it leaves untouched) and keeps
 * the fastest; for FP32 lattices that two steps per pass apply to, it also
 * times that pass at several strip heights and sets the steps per pass
 * (xyl_set_fusion) to whichever of 1 and 2 is faster per step; it also picks
 * the launch shape of the measurements that sampled runs take (results do
 * not depend on it either).  The choices are cached per (shape, precision)
 * for the process and applied to lattices created later. */
int xyl_set_launch(xyl_lattice* h, int32_t rows_per_strip, int32_t waves_per_block);
int xyl_get_launch(xyl_lattice* h, int32_t* rows_per_strip, int32_t* waves_per_block);
int xyl_autotune(xyl_lattice* h);
/* Steps per captured HIP graph used by xyl_step (0 or 1 disables graphs). */
int xyl_set_graph_steps(xyl_lattice* h, int32_t steps);
/* Steps per pass over the state for plain FP32 stepping (1 or 2; default 2).
 * With 2, runs of 4m steps without measurements advance two steps per pass
 * (one workgroup per strip of rows across the whole width, the second step
 * one row behind the first) where Ly >= 4 and Lx is at most 4096, uses at
 * least three quarters of the lanes of its waves (256 sites per wave) and at
 * least two lanes of the last.  Wider rows (Lx a multiple of 4) run as the
 * fewest column tiles that fit one workgroup with one quad of halo on each
 * side (at most 4096 sites) under the same lane rules, where such a split
 * exists.  Other shapes, FP64 and measurement steps use single steps.
 * Results are bitwise identical either way; two steps per pass read and write
 * the state once per two steps.  The library allocates a second velocity
 * buffer (4 Lx Ly bytes) on first use; the state returns to the lattice's own
 * buffers at the end of every call. */
int xyl_set_fusion(xyl_lattice* h, int32_t steps_per_pass);
/* The stepping mode in effect: *steps_per_pass = the value set by
 * xyl_set_fusion or chosen by xyl_autotune; *rows = rows per strip of the
 * two-step pass for this lattice on its device (xyl_autotune's choice, else a
 * rule from the CU count and the workgroups a CU holds), 0 where two steps
 * per pass do not apply (shape, FP64, or steps_per_pass 1).  Either pointer
 * may be NULL. */
int xyl_get_fusion(const xyl_lattice* h, int32_t* steps_per_pass, int32_t* rows);
/* Shape of the two-step pass (App. B's data-parallel sweep, two BBK steps of
 * App. A.1 per pass): rows per strip (2 to 64) and, for widths above 4096,
 * the most waves (of 256 sites) a column tile may span (2 to 16: narrower
 * tiles mean more of them, and up to eight workgroups per CU; below the
 * row's own waves it splits rows up to 4096 sites wide as well, into at least
 * two tiles); 0 keeps the current value.  A tile width no split fits falls
 * back to whole rows (up to 4096 sites) or the fewest tiles.
 * Results do not depend on it.  xyl_autotune sets both.  EINVAL outside the
 * ranges. */
int xyl_set_step2_shape(xyl_lattice* h, int32_t rows, int32_t tile_waves);
/* The shape in effect: rows per strip, most waves per tile and the number of
 * column tiles (whole rows: the row's waves and 1); zeros where two steps
 * per pass do not apply.  Any pointer may be NULL. */
int xyl_get_step2_shape(const xyl_lattice* h, int32_t* rows, int32_t* tile_waves, int32_t* tiles);

/* -------------------------------------------------------------- test hooks */
/* Raw Philox4x32-10 blocks computed on the device: for j < n, counter
 * ctr[4j..4j+3] and key (seed_lo, seed_hi) -> out[4j..4j+3]. */
int xyl_philox_blocks(int32_t device, uint64_t seed, const uint32_t* ctr, uint32_t* out, uint64_t n);
/* Measured streaming ceiling of the step's memory traffic shape on `device`:
 * best bandwidth (GB/s, 16 bytes per element) of a plain kernel that reads two
 * float arrays of n elements and writes two, ping-ponging between two pairs
 * like a lattice's state, over a few grid sizes and `reps` (>= 2) launches
 * each.  Allocates 16 n bytes while it runs.  A reference for the step
 * kernel's bandwidth besides the 8 TB/s peak. */
int xyl_stream_ceiling(int32_t device, uint64_t n, int32_t reps, double* gbs);
/* The Gaussian draws n_i^k of every site at step k as the step kernel of this
 * lattice computes them (in its precision), converted to float64. */
int xyl_noise(xyl_lattice* h, uint64_t k, double* out);

/* --------------------------------------------------------------- analysis */
/* Binder cumulant U = <m^4>/<m^2>^2 (Sec. IV.A, Eq. Def-Binder-Cum) of the
 * samples m[discard..n-1], and its standard error from blocks longer than
 * twice the integrated autocorrelation time (App. B); U_se may be NULL.
 * Pure host computation. */
int xyl_binder(const double* m, uint64_t n, uint64_t discard, double* U, double* U_se);
/* Integrated autocorrelation time (in samples; automatic window of Madras and
 * Sokal, c = 6) and standard error of the mean of f[discard..n-1] (App. B,
 * Eqs. Autocorrelation-Time and Time-Series-Var).  Pure host computation. */
int xyl_mean_error(const double* f, uint64_t n, uint64_t discard, double* mean, double* se, double* tau);
/* Time-resolved Binder cumulant (Sec. IV.B; App. B restricts the time
 * integral of Eq. ensemble-average-calculation to bins of width d sigma):
 * m holds nrep independent replicas' order-parameter series, replica-major
 * (m[r*nt + j], equally spaced samples).  For each bin b of `bin`
 * consecutive samples (nt/bin bins; a ragged tail is dropped),
 * U[b] = <m^4> / <m^2>^2 with both averages over all replicas and the bin's
 * samples; U_se[b] (nullable) is the jackknife error over replicas (NaN for
 * one replica).  Pure host computation. */
int xyl_binder_relaxation(const double* m, uint64_t nrep, uint64_t nt, uint64_t bin, double* U, double* U_se);
/* Dynamic exponent by curve collapse (Sec. IV.B): for z on the raster
 * z_lo, z_lo + z_step, ... <= z_hi, the mean squared deviation between
 * U1(t) of size L1 and U2(b^-z t) of size L2, b = L1/L2, with U2 linearly
 * interpolated in t (t2 strictly increasing) over the points of curve 1 that
 * fall inside curve 2's time range (at least 3); returns the minimising z and
 * its mean squared deviation (cost, nullable).  The paper rasterises z in
 * steps of 0.01.  Pure host computation. */
int xyl_z_collapse(const double* t1, const double* U1, uint64_t n1, double L1, const double* t2, const double* U2,
                   uint64_t n2, double L2, double z_lo, double z_hi, double z_step, double* z_best, double* cost);
/* Correlation length as the parameter of a least-squares fit of the
 * Lorentzian S(k) = A 2 xi / (1 + 4 pi^2 xi^2 (k/L)^2) (App. C, Eq.
 * Lorentzian-Peak, with the wave number read as k / L) to S[k_first..k_last],
 * 0 <= k_first < k_last <= L/2; k_first = 1 drops S(0), as the paper does below
 * T_c.  S(k) must be positive over the range.  Returns xi and the amplitude A
 * (nullable); XYL_ENUMERIC if S is not peaked at k = 0 over the range or the
 * fit does not converge.  Pure host computation. */
int xyl_lorentzian_xi(const double* S, int32_t L, int32_t k_first, int32_t k_last, double* xi, double* amplitude);

/* Second-moment correlation length along axis 0 (x) or 1 (y) from samples
 * s[discard..n-1] (as the measuring calls return them):
 *   xi = sqrt(<F(0)> / <F(k_min)> - 1) / (2 sin(pi / L)),
 * <.> the mean over the samples, F(0) = f0 and F(k_min) = fkx or fky, L the
 * side length along the axis; the means come before the ratio.  It is exact
 * for the lattice Lorentzian S(k) = S(0) / (1 + 4 xi^2 sin^2(pi k / L)),
 * which is the Lorentzian of App. C (Eq. Lorentzian-Peak, wave number k / L)
 * up to terms of relative order (k / L)^2, solved through k = 0 and k = 1
 * (the wave number 2 pi / L).  xi = 0
 * where <F(0)> <= <F(k_min)> (no correlation beyond the noise); XYL_ENUMERIC
 * if <F(k_min)> is not positive and finite.  Pure host computation. */
int xyl_xi_second_moment(const xyl_obs* s, uint64_t n, uint64_t discard, int32_t axis, int32_t L, double* xi);

/* --------------------------------------------------------------- ensemble */
/* One replica of a batched ensemble: its own lattice size, parameters,
 * schedule, noise key and number of steps to run. */
typedef struct {
    int32_t Lx, Ly;
    double Jx, Jy, h, gamma, dt;
    uint64_t seed;
    uint32_t replica;
    int32_t nknots;
    uint64_t knot_step[XYL_MAX_KNOTS];
    double knot_T[XYL_MAX_KNOTS];
    uint64_t nsteps;
    int32_t model;    /* XYL_MODEL_*; every replica of an ensemble has the same */
    double p;         /* field order, as for xyl_set_model */
    int32_t knot_gamma[XYL_MAX_KNOTS];   /* segment shapes as for xyl_set_schedule_shaped (0 = linear) */
} xyl_replica_desc;

/* Creates n >= 1 replicas on one device in one state allocation, indexed by a
 * per-replica offset table (App. B packs independent subsystems into one
 * simulation; here their sizes and parameters may differ).  Every replica
 * starts from xyl_init_random's state for its own (seed, replica). */
int xyl_ensemble_create(xyl_ensemble** out, const xyl_replica_desc* desc, int32_t n, int32_t dtype,
                        int32_t device);
int xyl_ensemble_destroy(xyl_ensemble* e); /* NULL is a no-op */
int xyl_ensemble_set_stream(xyl_ensemble* e, void* stream);
/* Advances every replica by up to nsteps steps without passing its own nsteps
 * (replicas that have finished stay where they are), in batched launches.
 * With every >= 1, replica r records observables at its steps that are
 * multiples of `every` (its step 0 included, at most one sample per step)
 * into out[r*cap + j], nout[r] receiving the running count (EINVAL on
 * overflow of cap).  every = 0 records nothing (out, nout may be NULL).
 * Synchronises when recording. */
int xyl_ensemble_step(xyl_ensemble* e, uint64_t nsteps, uint64_t every, xyl_obs* out, uint64_t cap,
                      uint64_t* nout);
/* Mode 0: all replicas in one launch per step (tiles of every replica in one
 * grid).  Mode 1: one launch per replica per step (the reference loop the
 * batched mode is measured against).  Default 0. */
int xyl_ensemble_set_mode(xyl_ensemble* e, int32_t mode);
/* Graph-captured chunks in the batched mode (App. B: many subsystems run
 * together).  The stepping of a chunk between samples (its two-step passes on
 * their class streams and its single tile-table steps) is captured as a graph
 * the second time a chunk of the same shape (first step, length) is met, and
 * replayed with the step index from a device counter after that; chunks of
 * fewer than 8 launches stay direct.  enable = 0: no graphs; 1 (the default):
 * graphs for chunks with at most one class of two-step passes (a replay
 * dispatches the parallel branches of several classes one after the other,
 * while direct launches, issued pass by pass across the classes, let them run
 * together); 2: graphs for every repeated chunk.  Graphs are dropped when the
 * task tables, the launch shape or the steps per pass change.  Results are
 * bitwise the same in every mode. */
int xyl_ensemble_set_graphs(xyl_ensemble* e, int32_t enable);
/* Steps per pass for the batched mode (1 or 2; default 2).  With 2 (FP32),
 * runs of 4m steps between samples advance the replicas on the tile path
 * whose width the two-step pass takes (as for xyl_set_fusion) two steps per
 * pass, in one launch
 * per pass for each class of replicas of the same number of waves per row;
 * the other tile-path replicas keep one batched tile launch per step.
 * Results are bitwise identical either way.  The library allocates a second
 * velocity buffer of the ensemble's size on first use. */
int xyl_ensemble_set_fusion(xyl_ensemble* e, int32_t steps_per_pass);
/* The steps per pass in effect (set, or chosen by xyl_ensemble_autotune). */
int xyl_ensemble_get_fusion(const xyl_ensemble* e, int32_t* steps_per_pass);
/* Launch shape (rows per strip, waves per workgroup) of the tile launches:
 * xyl_ensemble_autotune times candidates on scratch copies of the replicas'
 * state (the ensemble itself is not advanced) and keeps the fastest.  For
 * FP32 ensembles with replicas the two-step pass takes, it then times their
 * passes (with the other replicas' tile steps) against the best tile launch
 * for every step and sets the steps per pass (xyl_ensemble_set_fusion) to
 * whichever is faster.  Results do not depend on either. */
int xyl_ensemble_autotune(xyl_ensemble* e);
int xyl_ensemble_get_launch(xyl_ensemble* e, int32_t* rows, int32_t* wpb);
int xyl_ensemble_get_state(xyl_ensemble* e, int32_t r, double* theta, double* omega, uint64_t* step);
int xyl_ensemble_set_state(xyl_ensemble* e, int32_t r, const double* theta, const double* omega,
                           uint64_t step);
int xyl_ensemble_domains(xyl_ensemble* e, int32_t r, int32_t* labels, uint64_t* sizes, uint64_t* counts,
                         uint64_t cap, uint64_t* n_sizes, uint64_t* n_domains, uint64_t* max_size);
/* xyl_structure_factor of replica r. */
int xyl_ensemble_structure_factor(xyl_ensemble* e, int32_t r, int32_t axis, int32_t kmax, double* S);
int xyl_ensemble_sync(xyl_ensemble* e);

/* ---------------------------------------------------------------- adjoint */
/* Pathwise gradients with the Gaussian draws held fixed (a training-style
 * reverse mode of the discrete BBK map of App. A.1, Eqs. BBK-1 and BBK-2; the
 * wrap has derivative 1).  Loss L = (1/W) sum_{k=k0+N-W+1}^{k0+N} m_s(th^k)^2.
 * xyl_adjoint_forward runs N steps from the current state, keeping a
 * checkpoint every `ckpt_every` steps, returns L and (run, nullable) an
 * identifier of this run; the lattice advances.  1 <= W <= N.
 * XYL_MODEL_XY only.
 * xyl_adjoint_backward then returns dL/d(Jx, Jy, h, gamma) in grad[4] (gamma
 * must be > 0 when T > 0) and writes dL/d th^{k0} and dL/d w^{k0} as float64
 * host arrays (nullable).  `run` must name the lattice's latest forward run,
 * and the lattice must not have been stepped, re-initialised or given other
 * parameters, schedule, seed, model or launch shape since: otherwise
 * XYL_ESTATE (a second forward on the same lattice replaces the checkpoints
 * of the first, so the first run can no longer be differentiated).  A run
 * may be differentiated more than once.
 * xyl_adjoint_backward_device is the same with every output multiplied by
 * `scale` (e.g. an upstream derivative dF/dL), grad[4] on the host and the
 * state adjoints written into caller-owned device buffers of Lx*Ly elements
 * of precision dtype (XYL_F32 or XYL_F64; nullable) on the lattice's stream:
 * no per-site array passes through the host.  Returns after the stream has
 * finished (the buffers are then ready for any stream). */
int xyl_adjoint_forward(xyl_lattice* h, uint64_t nsteps, uint64_t ckpt_every, uint64_t window, double* loss,
                        uint64_t* run);
int xyl_adjoint_backward(xyl_lattice* h, uint64_t run, double* grad, double* dtheta0, double* domega0);
int xyl_adjoint_backward_device(xyl_lattice* h, uint64_t run, double scale, double* grad, void* dtheta0,
                                void* domega0, int32_t dtype);
/* Reverse steps per pass of xyl_adjoint_backward (App. A.1's step, run
 * backwards): 2 (the default) takes two reverse steps per pass over the state
 * where a strip of rows fits one workgroup (one site per lane, Lx at most
 * 1024, Ly >= 4, and (32 rows + 80) Lx bytes of FP32 state and draws, twice
 * that in FP64, within a CU's 160 KiB of LDS), and recomputes the checkpointed
 * segments two steps per pass too where the forward's two-step pass takes
 * the lattice; 1 keeps one step per pass for both.  rows: rows per strip of
 * the two-step reverse pass (1, 2 or 4; 0 keeps the current value,
 * initially 2: where that does not fit, single reverse steps unless 1 is
 * set).  dL/dth and dL/dw are bitwise
 * the same either way; the parameter gradients are sums taken in another
 * order.  EINVAL outside the ranges. */
int xyl_set_adjoint_fusion(xyl_lattice* h, int32_t steps_per_pass, int32_t rows);

#ifdef __cplusplus
}
#endif
#endif
