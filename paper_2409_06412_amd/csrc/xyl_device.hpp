// Device primitives of the Langevin-XY step: counter-based noise, the
// temperature schedule, precision traits and the per-lattice launch view.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "xyl_internal.hpp"

namespace xyl {

// ----------------------------------------------------------------- Philox
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two 32x32
// -> 64 bit products of words 0 and 2 with fixed multipliers, whose halves are
// mixed with words 1, 3 and the round key; the key advances by the Weyl
// constants between rounds.  The key is wave-uniform, so its schedule lives
// in scalar registers.
struct U32x4 {
    uint32_t v[4];
};

__device__ __forceinline__ U32x4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                               uint32_t k0, uint32_t k1) {
    constexpr uint32_t kMulA = 0xD2511F53u, kMulB = 0xCD9E8D57u;
    constexpr uint32_t kWeylA = 0x9E3779B9u, kWeylB = 0xBB67AE85u;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t pa = (uint64_t)kMulA * c0;
        const uint64_t pb = (uint64_t)kMulB * c2;
        const uint32_t ka = k0 + (uint32_t)r * kWeylA;
        const uint32_t kb = k1 + (uint32_t)r * kWeylB;
        // three-input XOR in one v_bitop3_b32 (truth table 0x96)
        const uint32_t n0 = __builtin_amdgcn_bitop3_b32((uint32_t)(pb >> 32), c1, ka, 0x96);
        const uint32_t n2 = __builtin_amdgcn_bitop3_b32((uint32_t)(pa >> 32), c3, kb, 0x96);
        c1 = (uint32_t)pb;
        c3 = (uint32_t)pa;
        c0 = n0;
        c2 = n2;
    }
    U32x4 o;
    o.v[0] = c0;
    o.v[1] = c1;
    o.v[2] = c2;
    o.v[3] = c3;
    return o;
}

// --------------------------------------------------------------- schedule
// T(k) between knots a, b: T_a + (T_b - T_a) w, f = (k - k_a) / (k_b - k_a),
// w = f (linear quench, Sec. II.B), f^g or 1 - (1 - f)^|g| (the power-law
// protocols of Sec. V; powers by repeated multiplication); held outside the
// knots.  FP64 with the operation order fixed so that every caller gets the
// same bits.
__host__ __device__ __forceinline__ double schedule_T(const Schedule& s, uint64_t k) {
    double T;
    if (k <= s.step[0]) {
        T = s.T[0];
    } else if (k >= s.step[s.n - 1]) {
        T = s.T[s.n - 1];
    } else {
        int j = 0;
        while (!(k >= s.step[j] && k < s.step[j + 1])) ++j;
        const double ka = (double)s.step[j], kb = (double)s.step[j + 1];
        const double frac = ((double)k - ka) / (kb - ka);
        const int g = s.g[j];
        double w = frac;
        if (g > 1) {
            for (int i = 1; i < g; ++i) w = w * frac;
        } else if (g < 0) {
            const double r = 1.0 - frac;
            w = r;
            for (int i = 1; i < -g; ++i) w = w * r;
            w = 1.0 - w;
        }
        T = s.T[j] + (s.T[j + 1] - s.T[j]) * w;
    }
    return T < 0.0 ? 0.0 : T;
}

// Noise amplitude of one half-kick, (1/2) sqrt(2 gamma T_k dt), in FP64.
__host__ __device__ __forceinline__ double half_sigma(const Schedule& s, double gamma, double dt, uint64_t k) {
    return 0.5 * sqrt(2.0 * gamma * schedule_T(s, k) * dt);
}

// -------------------------------------------------------- precision traits
template <typename R>
struct Prec;

template <>
struct Prec<float> {
    static constexpr float kPi = 3.14159274101257324e+00f;    // pi rounded to binary32
    static constexpr float kTwoPi = 6.28318548202514648e+00f;
    static constexpr float kHalfPi = 1.57079637050628662e+00f;
    // Native sine/cosine take revolutions; angles here lie in [-pi_p, pi_p].
    __device__ static __forceinline__ void sincos(float t, float& s, float& c) {
        const float x = t * 0.159154943091895336f;
        s = __builtin_amdgcn_sinf(x);
        c = __builtin_amdgcn_cosf(x);
    }
    // sin 2t, cos 2t: 2t / 2pi revolutions = t / pi
    __device__ static __forceinline__ void sincos2(float t, float& s, float& c) {
        const float x = t * 0.318309886183790672f;
        s = __builtin_amdgcn_sinf(x);
        c = __builtin_amdgcn_cosf(x);
    }
    // sin(p t) with f = p / 2pi (revolutions per radian)
    __device__ static __forceinline__ float sin_scaled(float t, float f) { return __builtin_amdgcn_sinf(t * f); }
    __device__ static __forceinline__ float fma(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
    // ((r >> 9) + 1/2) 2^-23, exactly: the top 23 bits under the exponent of
    // 1.0 (one v_alignbit: (0x7f << 23) | (r >> 9)) give 1 + (r >> 9) 2^-23 in
    // [1, 2); subtracting 1 - 2^-24 is exact.
    __device__ static __forceinline__ float uniform(uint32_t r) {
        return __uint_as_float(__builtin_amdgcn_alignbit(0x7fu, r, 9u)) - 0x1.fffffep-1f;
    }
    // One Box-Muller pair: radius sqrt(-2 ln u1) (ln via the native log2:
    // kk = -2 ln 2, or -2 ln 2 scale^2 to scale both draws by `scale` inside
    // the square root), angle 2 pi u2 (native sine/cosine in revolutions, no
    // multiplication).
    // The angle's uniform may be taken half a revolution on (c2 = 1/2 - 2^-24
    // instead of 1 - 2^-24 below, no extra instruction), which negates both
    // draws: cos(2 pi (u + 1/2)) = -cos(2 pi u), likewise the sine.
    static constexpr float kMinus2Ln2 = -1.38629436111989062f;
    static constexpr float kU2 = 0x1.fffffep-1f, kU2Half = 0x1.fffffcp-2f;
    __device__ static __forceinline__ void box_muller(uint32_t r1, uint32_t r2, float& nc, float& ns,
                                                      float kk = kMinus2Ln2, float c2 = kU2) {
        const float u1 = uniform(r1);
        const float u2 = __uint_as_float(__builtin_amdgcn_alignbit(0x7fu, r2, 9u)) - c2;
        const float rad = __builtin_amdgcn_sqrtf(kk * __builtin_amdgcn_logf(u1));
        nc = rad * __builtin_amdgcn_cosf(u2);
        ns = rad * __builtin_amdgcn_sinf(u2);
    }
};

template <>
struct Prec<double> {
    static constexpr double kPi = 3.14159265358979311600e+00;
    static constexpr double kTwoPi = 6.28318530717958623200e+00;
    static constexpr double kHalfPi = 1.57079632679489655800e+00;
    __device__ static __forceinline__ void sincos(double t, double& s, double& c) { ::sincos(t, &s, &c); }
    __device__ static __forceinline__ void sincos2(double t, double& s, double& c) { ::sincos(2.0 * t, &s, &c); }
    // sin(p t) with f = p
    __device__ static __forceinline__ double sin_scaled(double t, double f) { return sin(f * t); }
    __device__ static __forceinline__ double fma(double a, double b, double c) { return __builtin_fma(a, b, c); }
    __device__ static __forceinline__ double uniform(uint32_t r) { return ((double)(r >> 9) + 0.5) * 0x1p-23; }
    __device__ static __forceinline__ void box_muller(uint32_t r1, uint32_t r2, double& nc, double& ns) {
        const double u1 = uniform(r1), u2 = uniform(r2);
        const double rad = sqrt(-2.0 * log(u1));
        const double phi = kTwoPi * u2;
        nc = rad * cos(phi);
        ns = rad * sin(phi);
    }
};

// Wrap to [-W, W) with W = pi_p (XY) or pi_p / 2 (SI, whose rotors are half
// circles): exact by Sterbenz's lemma while |dt * u| < W.  Same result as
// "if t >= W: t -= 2W, else if t < -W: t += 2W" for every input.
// The shift is selected first and subtracted once: t - 2W, t + 2W (both exact)
// or t - (+0) = t, which keeps the sign of a zero.
// FP32 XY angles take the shift as 2W times the nearest integer to t / 2W
// (three operations instead of two compares, two selects and a subtraction):
// the same whenever t / 2W, rounded, is not exactly +-1/2, so only angles
// within an ulp or two of +-W may stay on the outer side of the boundary.
// The XY model's force and observables are 2 pi-periodic, so that changes
// nothing but the representative; the SI field is not, and keeps the exact
// rule, as does FP64.
template <typename R, int M>
__device__ __forceinline__ R wrap_angle(R t) {
    constexpr R W = M == kModelSI ? Prec<R>::kHalfPi : Prec<R>::kPi;
    constexpr R W2 = M == kModelSI ? Prec<R>::kPi : Prec<R>::kTwoPi;
    if constexpr (sizeof(R) == 4 && M == kModelXY) {
        const R r = __builtin_rintf(t * (R(1) / W2));
        return Prec<R>::fma(-W2, r, t);
    } else {
        const R shift = t >= W ? W2 : (t < -W ? -W2 : R(0));
        return t - shift;
    }
}

// Rotor of a site, (sin q t, cos q t): q = 1 (XY) or 2 (SI).
template <typename R, int M>
__device__ __forceinline__ void rotor(R t, R& s, R& c) {
    if constexpr (M == kModelSI) Prec<R>::sincos2(t, s, c);
    else Prec<R>::sincos(t, s, c);
}

// Four Gaussian draws of the sites 4q..4q+3 (q = i >> 2) at step k.
template <typename R>
__device__ __forceinline__ void noise4(uint32_t q, uint32_t replica, uint64_t k, uint32_t s0, uint32_t s1, R n[4]) {
    const U32x4 r = philox4x32_10(q, replica, (uint32_t)k, (uint32_t)(k >> 32), s0, s1);
    Prec<R>::box_muller(r.v[0], r.v[1], n[0], n[1]);
    Prec<R>::box_muller(r.v[2], r.v[3], n[2], n[3]);
}

// The noise coefficient of step k as noise4_kick and site_update take it:
// FP32 -2 ln 2 hs^2 (the draws' scale inside the Box-Muller square root, from
// the FP64 amplitude hs; for the factored kick F, divided by (hdt q Jx)^2 so
// that the draws come out divided by hdt q Jx); FP64 hs itself.
template <typename R, bool F = false>
__device__ __forceinline__ R noise_coeff(const Lat<R>& v, uint64_t k) {
    const double hs = half_sigma(v.sched, v.gamma, v.dtd, k);
    if constexpr (sizeof(R) == 4) {
        if constexpr (F) return (R)(-1.38629436111989062 * hs * hs * v.fnoise);
        else return (R)(-1.38629436111989062 * hs * hs);
    } else {
        return hs;
    }
}

// The draws as site_force takes them: FP32 scales them by the half-kick noise
// amplitude through the coefficient kk = noise_coeff (the same for every site
// of a step); FP64 returns the plain draws and site_update applies hs in the
// oracle's order.
// c2: the angle uniform's constant (Prec<float>::box_muller): kU2Half
// negates the draws, which the factored kick needs when hdt q Jx < 0 (its
// scale enters through the square root, which keeps the sign positive).
template <typename R>
__device__ __forceinline__ void noise4_kick(uint32_t q, uint32_t replica, uint64_t k, uint32_t s0, uint32_t s1, R kk,
                                            R n[4], R c2) {
    if constexpr (sizeof(R) == 4) {
        const U32x4 r = philox4x32_10(q, replica, (uint32_t)k, (uint32_t)(k >> 32), s0, s1);
        Prec<R>::box_muller(r.v[0], r.v[1], n[0], n[1], kk, c2);
        Prec<R>::box_muller(r.v[2], r.v[3], n[2], n[3], kk, c2);
    } else {
        (void)c2;
        noise4<R>(q, replica, k, s0, s1, n);
    }
}

// The draws' angle constant of a lattice's form of the FP32 kick.
template <typename R, bool F>
__device__ __forceinline__ R noise_u2(const Lat<R>& v) {
    if constexpr (sizeof(R) == 4 && F) return v.fu2;
    else if constexpr (sizeof(R) == 4) return Prec<float>::kU2;
    else return R(0);
}

// ------------------------------------------------------ per-site BBK math
// Shared by every kernel that advances sites, so that their states agree bit
// for bit.  F = -dH/dth from the rotors (s, c) = (sin q th, cos q th) of the
// site and its neighbours (x-1, x+1, y-1, y+1) and, for SI, the raw angle:
//   XY: F = Jx [s (cx+ + cx-) - c (sx+ + sx-)] + Jy [s (cy+ + cy-) - c (sy+ + sy-)] - 4 h s c
//   SI: F = 2Jx [s (cx+ + cx-) - c (sx+ + sx-)] + 2Jy [...] - p h sin(p th)
// (v.Jx, v.Jy hold q Jx, q Jy).  FP32 returns the whole kick g = hdt F + n
// (n the scaled draw), with hdt folded into the couplings so that the draw
// enters the last two fused multiply-adds; FP64 returns F in the oracle's
// order and site_update adds the rest.
// FP32 with F (the factored kick, where the lattice's `fact` is set): the
// kick divided by kx = hdt q Jx,
//   g / kx = s (Cx + r Cy - rh c) - c (Sx + r Sy) + n / kx    (XY)
//          = s (Cx + r Cy) - c (Sx + r Sy) - rph sin(p th) + n / kx   (SI)
// with r = Jy/Jx, rh = 4h/(q Jx), rph = p h/(q Jx) and the draw already
// divided by kx (noise_coeff<R, true>): the y sums enter through one fused
// multiply-add each and the scale kx moves into site_update's coefficients.
template <typename R, int M, bool F = false>
__device__ __forceinline__ R site_force(const Lat<R>& v, R s, R c, R sxm, R cxm, R sxp, R cxp, R sym, R cym, R syp,
                                        R cyp, R th, R n) {
    if constexpr (sizeof(R) == 4 && F) {
        const R X = Prec<R>::fma(v.fr, cyp + cym, cxp + cxm);
        const R Y = Prec<R>::fma(v.fr, syp + sym, sxp + sxm);
        const R cq = Prec<R>::fma(-c, Y, n);
        if constexpr (M == kModelSI) {
            const R sp = Prec<R>::sin_scaled(th, v.pf);
            return Prec<R>::fma(-v.fph, sp, Prec<R>::fma(s, X, cq));
        } else {
            return Prec<R>::fma(s, Prec<R>::fma(-v.fh, c, X), cq);
        }
    } else if constexpr (sizeof(R) == 4) {
        // couplings scaled by hdt on the host (kJx = hdt q Jx, ...)
        const R P0 = Prec<R>::fma(v.kJx, cxp + cxm, v.kJy * (cyp + cym));
        const R Q = Prec<R>::fma(v.kJx, sxp + sxm, v.kJy * (syp + sym));
        const R cq = Prec<R>::fma(-c, Q, n);
        if constexpr (M == kModelSI) {
            const R sp = Prec<R>::sin_scaled(th, v.pf);
            return Prec<R>::fma(-v.kph, sp, Prec<R>::fma(s, P0, cq));
        } else {
            // s (kJx Cx + kJy Cy - kh4 c) - c (kJx Sx + kJy Sy) + n
            const R P = Prec<R>::fma(-v.kh4, c, P0);
            return Prec<R>::fma(s, P, cq);
        }
    } else {
        (void)n;
        if constexpr (M == kModelSI) {
            const R sp = Prec<R>::sin_scaled(th, v.pf);
            const R fx = Prec<R>::fma(s, cxp + cxm, -(c * (sxp + sxm)));
            const R fy = Prec<R>::fma(s, cyp + cym, -(c * (syp + sym)));
            return Prec<R>::fma(-v.ph, sp, Prec<R>::fma(v.Jx, fx, v.Jy * fy));
        } else {
            const R fx = Prec<R>::fma(s, cxp + cxm, -(c * (sxp + sxm)));
            const R fy = Prec<R>::fma(s, cyp + cym, -(c * (syp + sym)));
            const R f = Prec<R>::fma(v.Jx, fx, v.Jy * fy);
            return Prec<R>::fma(-v.h4, s * c, f);
        }
    }
}

// cos of the field's angle for the energy: cos 2th = c^2 - s^2 from the rotor
// (XY); cos(p th) of the raw angle (SI), in the state's precision like the
// rotors: the native FP32 cosine for FP32 lattices (pf = p / 2pi revolutions
// per radian; an FP64 cosine here spilled the whole-in-LDS kernel's
// registers), FP64 cos for FP64 lattices.
template <typename R, int M>
__device__ __forceinline__ double onsite_cos(const Lat<R>& v, R th, double s, double c) {
    if constexpr (M == kModelSI) {
        if constexpr (sizeof(R) == 4) return (double)__builtin_amdgcn_cosf(th * v.pf);
        else return cos(v.pd * (double)th);
    } else {
        return c * c - s * s;
    }
}

// Completes the previous step's second half-kick (w^k; skipped at the fresh
// step, where u already holds w^k), then the next first half-kick, the drift
// and the wrap (App. A.1, Eqs. BBK-2 and BBK-1), with the fma order the
// oracle uses.
template <typename R, int M, bool F = false>
__device__ __forceinline__ void site_update(const Lat<R>& v, R f, R u, R th, R n, R hs, bool fresh, R& w, R& unew,
                                            R& thnew) {
    if constexpr (sizeof(R) == 4 && F) {
        // f = g / kx (the factored kick): u' = a w^k + g with w^k = c (u + g)
        // is ac u + kx (1 + ac) f on ordinary steps and a u + kx f on the
        // fresh one (w^k = u); w^k itself only where it is used
        (void)hs;
        (void)n;
        const R acf = fresh ? v.a : v.ac;
        const R c1 = fresh ? v.kJx : v.fc1;
        const R kf = fresh ? R(0) : v.kJx;
        const R cf = fresh ? R(1) : v.c;
        unew = Prec<R>::fma(acf, u, c1 * f);
        w = cf * Prec<R>::fma(kf, f, u);
    } else if constexpr (sizeof(R) == 4) {
        // FP32: f arrives as the kick g = hdt F + hs n (site_force), used by
        // both halves.  With sum = u + g (fma(1, g, u), exact rounding of the
        // sum) on ordinary steps and sum = u on the fresh step, w^k = c sum
        // and u' = a w^k + g; the kick takes u' = fma(a c, sum, g) with a c
        // rounded once, so w^k itself (one more product) is formed only where
        // it is used (measurements and the velocity read-out).
        (void)hs;
        (void)n;
        const R g = f;
        const R gf = fresh ? R(0) : R(1);
        const R cf = fresh ? R(1) : v.c;
        const R acf = fresh ? v.a : v.ac;
        const R sum = Prec<R>::fma(gf, g, u);
        w = cf * sum;
        unew = Prec<R>::fma(acf, sum, g);
    } else {
        R ww;
        if (fresh) {
            ww = u;
        } else {
            R t = Prec<R>::fma(v.hdt, f, u);
            t = Prec<R>::fma(hs, n, t);
            ww = v.c * t;
        }
        w = ww;
        R t2 = v.hdt * f;
        t2 = Prec<R>::fma(hs, n, t2);
        unew = Prec<R>::fma(v.a, ww, t2);
    }
    thnew = wrap_angle<R, M>(Prec<R>::fma(v.dt, unew, th));
}

// ---------------------------------------------------- lane exchange (DPP)
// wave_shr:1 moves a value to the next lane up, wave_shl:1 to the next lane
// down; lanes at the ends receive `old`.
__device__ __forceinline__ float from_lane_below(float v, float old = 0.0f) {
    return __int_as_float(
        __builtin_amdgcn_update_dpp(__float_as_int(old), __float_as_int(v), 0x138, 0xF, 0xF, false));
}
__device__ __forceinline__ float from_lane_above(float v, float old = 0.0f) {
    return __int_as_float(
        __builtin_amdgcn_update_dpp(__float_as_int(old), __float_as_int(v), 0x130, 0xF, 0xF, false));
}
__device__ __forceinline__ double from_lane_below(double v, double old = 0.0) {
    const int lo =
        __builtin_amdgcn_update_dpp((int)__double2loint(old), (int)__double2loint(v), 0x138, 0xF, 0xF, false);
    const int hi =
        __builtin_amdgcn_update_dpp((int)__double2hiint(old), (int)__double2hiint(v), 0x138, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double from_lane_above(double v, double old = 0.0) {
    const int lo =
        __builtin_amdgcn_update_dpp((int)__double2loint(old), (int)__double2loint(v), 0x130, 0xF, 0xF, false);
    const int hi =
        __builtin_amdgcn_update_dpp((int)__double2hiint(old), (int)__double2hiint(v), 0x130, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}

// A double moved between lanes by DPP (CTRL: the DPP control word; every
// source lane of the patterns used here is inside the wave).
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
    const int lo = __builtin_amdgcn_update_dpp(0, (int)__double2loint(v), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)__double2hiint(v), CTRL, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}
constexpr int kDppRowRor8 = 0x128;       // within rows of 16 lanes: lane i <- lane i ^ 8
constexpr int kDppRowHalfMirror = 0x141; // within groups of 8 lanes: lane i <- lane 7 - i
constexpr int kDppQuadXor2 = 0x4E;       // quad_perm [2, 3, 0, 1]
constexpr int kDppQuadXor1 = 0xB1;       // quad_perm [1, 0, 3, 2]

// The gfx950 lane-half swaps on a pair of doubles.  swap32: the upper 32
// lanes of x trade places with the lower 32 lanes of y.  swap16: the odd rows
// of 16 lanes of x (lanes 16-31, 48-63) with the even rows of y (0-15, 32-47).
// So with x, y = values j and j' of every lane, a lane in the lower half
// (even row) ends with its own and its partner's value j in (x, y), a lane in
// the upper half (odd row) with its partner's and its own value j'.
__device__ __forceinline__ void swap32_f64(double& x, double& y) {
    const auto lo = __builtin_amdgcn_permlane32_swap((unsigned)__double2loint(x), (unsigned)__double2loint(y), false,
                                                     false);
    const auto hi = __builtin_amdgcn_permlane32_swap((unsigned)__double2hiint(x), (unsigned)__double2hiint(y), false,
                                                     false);
    x = __hiloint2double((int)hi[0], (int)lo[0]);
    y = __hiloint2double((int)hi[1], (int)lo[1]);
}
__device__ __forceinline__ void swap16_f64(double& x, double& y) {
    const auto lo = __builtin_amdgcn_permlane16_swap((unsigned)__double2loint(x), (unsigned)__double2loint(y), false,
                                                     false);
    const auto hi = __builtin_amdgcn_permlane16_swap((unsigned)__double2hiint(x), (unsigned)__double2hiint(y), false,
                                                     false);
    x = __hiloint2double((int)hi[0], (int)lo[0]);
    y = __hiloint2double((int)hi[1], (int)lo[1]);
}

// Sums of eight FP64 values over the 64 lanes of a wave, in a fixed pattern:
// a reduce-scatter in which every exchange halves the values a lane carries
// (lanes with bit 5 set keep values 4..7 and send 0..3 to their partner, and
// so on for bits 4 and 3), then a butterfly over the last three bits.  The
// exchanges at bits 5 and 4 are lane-half swaps (no selects, no LDS), those
// at bit 3 and below DPP.  Lane L returns the total of value L >> 3; the
// eight lanes of a group return the same bits (each step adds the same two
// numbers on both lanes of a pair).  All 64 lanes must be active.
__device__ __forceinline__ double wave_sum8(const double a[8], int lane) {
    const bool b3 = (lane & 8) != 0;
    double k4[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        double x = a[j], y = a[j + 4];
        swap32_f64(x, y);
        k4[j] = x + y;
    }
    double k2[2];
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        double x = k4[j], y = k4[j + 2];
        swap16_f64(x, y);
        k2[j] = x + y;
    }
    double k1;
    {
        const double keep = b3 ? k2[1] : k2[0], send = b3 ? k2[0] : k2[1];
        k1 = keep + dpp_f64<kDppRowRor8>(send);
    }
    k1 += dpp_f64<kDppRowHalfMirror>(k1);
    k1 += dpp_f64<kDppQuadXor2>(k1);
    k1 += dpp_f64<kDppQuadXor1>(k1);
    return k1;
}

// The same for four FP64 values: lane L returns the total of value L >> 4.
__device__ __forceinline__ double wave_sum4(const double a[4], int lane) {
    const bool b5 = (lane & 32) != 0, b4 = (lane & 16) != 0;
    double k2[2];
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        const double keep = b5 ? a[j + 2] : a[j], send = b5 ? a[j] : a[j + 2];
        k2[j] = keep + __shfl_xor(send, 32, kWave);
    }
    double k1;
    {
        const double keep = b4 ? k2[1] : k2[0], send = b4 ? k2[0] : k2[1];
        k1 = keep + __shfl_xor(send, 16, kWave);
    }
#pragma unroll
    for (int off = 8; off >= 1; off >>= 1) k1 += __shfl_xor(k1, off, kWave);
    return k1;
}

template <typename R>
struct Vec4;
template <>
struct Vec4<float> {
    using T = float4;
};
template <>
struct Vec4<double> {
    using T = double4;
};

template <typename R>
__device__ __forceinline__ void load4(const R* p, R o[4]) {
    const typename Vec4<R>::T v = *reinterpret_cast<const typename Vec4<R>::T*>(p);
    o[0] = v.x;
    o[1] = v.y;
    o[2] = v.z;
    o[3] = v.w;
}
template <typename R>
__device__ __forceinline__ void store4(R* p, const R o[4]) {
    typename Vec4<R>::T v;
    v.x = o[0];
    v.y = o[1];
    v.z = o[2];
    v.w = o[3];
    *reinterpret_cast<typename Vec4<R>::T*>(p) = v;
}

// Element addresses as a wave-uniform base plus a lane's byte offset: the
// base (a row's start) stays in scalar registers and the offset in one 32-bit
// vector register, the operand form of global loads and stores with a scalar
// base, so no per-lane 64-bit address arithmetic is needed per row.
template <typename T>
__device__ __forceinline__ T* at_byte(T* base, uint32_t off) {
    return reinterpret_cast<T*>(reinterpret_cast<char*>(base) + off);
}
template <typename T>
__device__ __forceinline__ const T* at_byte(const T* base, uint32_t off) {
    return reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + off);
}
// Start of row y of an Lx-wide array (wave-uniform).
template <typename T>
__device__ __forceinline__ T* row_start(T* base, int y, int Lx) {
    return base + (size_t)((uint32_t)y * (uint32_t)Lx);
}

// Bijective remap of workgroup ids so that each of the eight XCDs (which
// receive workgroups round-robin) processes a contiguous range of logical
// workgroups: neighbouring strips, whose halo rows overlap, share one L2.
__device__ __forceinline__ int xcd_contiguous_block(int b, int nb) {
    constexpr int kXcd = 8;
    const int per = nb / kXcd, rem = nb % kXcd;
    const int xcd = b % kXcd, idx = b / kXcd;
    return xcd * per + (xcd < rem ? xcd : rem) + idx;
}

}  // namespace xyl
