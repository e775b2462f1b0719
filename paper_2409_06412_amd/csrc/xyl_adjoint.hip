// Discrete adjoint of the fused BBK step (reverse mode of the map that the
// step kernel applies, with the Gaussian draws held fixed and the wrap taken
// with derivative 1).
//
// Forward map of step k on the stored state (th, u), F = F(th^k):
//     w^k     = u^k                                   (at the fresh step)
//             = c (u^k + hdt F + hs_k n^k)            (otherwise; = c A)
//     u^{k+1} = a w^k + hdt F + hs_k n^k
//     th^{k+1} = wrap(th^k + dt u^{k+1})
// Reverse step, given lt' = dL/dth^{k+1} and lu' = dL/du^{k+1}:
//     g   = lu' + dt lt'           (total adjoint of u^{k+1})
//     lw  = a g,  lA = c lw        (lA only when not fresh)
//     lF  = hdt (g + lA)
//     lu  = lA (or lw at the fresh step)
//     lt  = lt' + J(th^k) lF + (direct loss term at k)
// with the symmetric force Jacobian
//     (J v)_i = sum_d Jd sum_pm cos(th_i - th_j)(v_i - v_j) - 4 h cos(2 th_i) v_i.
// Parameter adjoints (FP64 sums over sites and steps):
//     dL/dJd += lF_i dF_i/dJd,  dF_i/dJx = s_i (cx+ + cx-) - c_i (sx+ + sx-), ...
//     dL/dh  += lF_i (-4 s_i c_i)
//     dL/dgamma += g w (-dt/2) + lw A (-(dt/2) c^2) + (g + lA) n hs_k / (2 gamma)
// (a = 1 - gamma dt/2, c = 1/(1 + gamma dt/2), hs_k = sqrt(2 gamma T_k dt)/2).
// Every lF_j of a neighbour is recomputed from that neighbour's (lt', lu'),
// so one pass per step reads th, u, lt', lu' and writes lt, lu.
#include <mutex>
#include <set>

#include "xyl_device.hpp"

namespace xyl {

template <typename R>
struct AdjArgs {
    Lat<R> v;                 // model, noise key, schedule, shape (pointers unused)
    const R* th;              // th^k
    const R* u;               // u^k
    const R* lt_in;           // dL/dth^{k+1}
    const R* lu_in;           // dL/du^{k+1}
    R* lt_out;                // dL/dth^k
    R* lu_out;                // dL/du^k
    const double* cm;         // direct loss coefficient of step k at cm[k - cm_base]
    uint64_t cm_base;
    double* gacc;             // per-task parameter adjoints [ntasks][4], accumulated
};

// Coefficients of reverse step k (the same for every site).
template <typename R>
struct AdjStep {
    R kap;        // lF = kap (lu' + dt lt')
    R lu_fac;     // lu = lu_fac (lu' + dt lt')
    R cm;         // direct loss coefficient of step k
    R hs, ghs, ga, gc;
    bool fresh;
};

template <typename R>
__device__ __forceinline__ AdjStep<R> adj_step_coef(const AdjArgs<R>& A, uint64_t k) {
    const Lat<R>& v = A.v;
    AdjStep<R> K;
    const double hsd = half_sigma(v.sched, v.gamma, v.dtd, k);
    K.hs = (R)hsd;
    K.fresh = (k == v.fresh_k);
    const R ca = v.c * v.a;
    K.kap = K.fresh ? v.hdt : v.hdt * (R(1) + ca);
    K.lu_fac = K.fresh ? v.a : ca;
    K.cm = (R)A.cm[k - A.cm_base];
    K.ghs = v.gamma > 0.0 ? (R)(hsd / (2.0 * v.gamma)) : R(0);
    K.ga = (R)(-0.5 * v.dtd);
    K.gc = (R)(-0.5 * v.dtd * (double)v.c * (double)v.c);
    return K;
}

// The reverse step at one site.  In: (s, c) of its angle th^k, (sin, cos, lF)
// of its x- and y-neighbours (m = -1, p = +1), its own lF, lt', lu', u^k,
// draw n^k and staggering sign eps.  Out: lt, lu; its parameter adjoints are
// added to (rx, ry, rh, rg).
template <typename R>
__device__ __forceinline__ void adj_site(const Lat<R>& v, const AdjStep<R>& K, R s, R c, R sxm, R cxm, R fxm, R sxp,
                                         R cxp, R fxp, R sym, R cym, R fym, R syp, R cyp, R fyp, R lf, R lt, R lu, R u,
                                         R n, R eps, R& lto, R& luo, R& rx, R& ry, R& rh, R& rg) {
    // force and its parameter derivatives
    const R dFx = Prec<R>::fma(s, cxp + cxm, -(c * (sxp + sxm)));
    const R dFy = Prec<R>::fma(s, cyp + cym, -(c * (syp + sym)));
    const R dFh = R(-4) * s * c;
    const R F = Prec<R>::fma(v.Jx, dFx, Prec<R>::fma(v.Jy, dFy, (R)v.hd * dFh));
    // J lF with cos(th_i - th_j) = c c_j + s s_j
    const R jx = (c * cxp + s * sxp) * (lf - fxp) + (c * cxm + s * sxm) * (lf - fxm);
    const R jy = (c * cyp + s * syp) * (lf - fyp) + (c * cym + s * sym) * (lf - fym);
    const R jh = (c * c - s * s) * lf;
    const R Jl = Prec<R>::fma(v.Jx, jx, Prec<R>::fma(v.Jy, jy, -v.h4 * jh));
    const R g = Prec<R>::fma(v.dt, lt, lu);
    lto = lt + Jl + K.cm * (-eps * s);
    luo = K.lu_fac * g;
    // parameter adjoints
    rx = Prec<R>::fma(lf, dFx, rx);
    ry = Prec<R>::fma(lf, dFy, ry);
    rh = Prec<R>::fma(lf, dFh, rh);
    const R lw = v.a * g;
    if (K.fresh) {
        rg += K.ga * g * u + K.ghs * n * g;
    } else {
        const R Av = Prec<R>::fma(K.hs, n, Prec<R>::fma(v.hdt, F, u));
        const R w = v.c * Av;
        const R lA = v.c * lw;
        rg += K.ga * g * w + K.gc * lw * Av + K.ghs * n * (g + lA);
    }
}

template <typename R>
struct AdjRow {
    R th[4], lt[4], lu[4];
    R tL, tR, ltL, ltR, luL, luR;   // outer x-neighbours (edge lanes)
    R s[4], c[4], lF[4];
};

template <typename R>
__device__ __forceinline__ void adj_strip(const AdjArgs<R>& A, int task, int xw, int strip, int rows, uint64_t k,
                                          int lane) {
    const Lat<R>& v = A.v;
    const int Lx = v.Lx, Ly = v.Ly;
    const int y0 = strip * rows;
    if (y0 >= Ly) return;
    const int y1 = min(y0 + rows, Ly);
    const int x0 = xw * kWaveSites;
    const int nact = min(kWave, (Lx - x0) >> 2);
    const bool act = lane < nact;
    const bool edgeL = act && lane == 0;
    const bool edgeR = lane == nact - 1;
    const int x = x0 + kLaneSites * lane;
    const int xm = x == 0 ? Lx - 1 : x - 1;
    const int xp = x + 4 == Lx ? 0 : x + 4;
    const AdjStep<R> K = adj_step_coef(A, k);
    const R kap = K.kap;
    const uint32_t qrow = (uint32_t)(Lx >> 2);

    auto load_row = [&](AdjRow<R>& S, int y) {
        const uint32_t row = (uint32_t)y * (uint32_t)Lx;
        if (act) {
            load4(A.th + row + x, S.th);
            load4(A.lt_in + row + x, S.lt);
            load4(A.lu_in + row + x, S.lu);
        }
        if (edgeL) {
            S.tL = A.th[row + xm];
            S.ltL = A.lt_in[row + xm];
            S.luL = A.lu_in[row + xm];
        }
        if (edgeR) {
            S.tR = A.th[row + xp];
            S.ltR = A.lt_in[row + xp];
            S.luR = A.lu_in[row + xp];
        }
    };
    auto derive = [&](AdjRow<R>& S) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            Prec<R>::sincos(S.th[q], S.s[q], S.c[q]);
            S.lF[q] = kap * Prec<R>::fma(v.dt, S.lt[q], S.lu[q]);
        }
    };

    double gx = 0.0, gy = 0.0, gh = 0.0, gg = 0.0;

    auto do_row = [&](AdjRow<R>& P, AdjRow<R>& C, AdjRow<R>& N, int y) {
        const uint32_t row = (uint32_t)y * (uint32_t)Lx;
        derive(N);
        if (y + 2 <= y1) {
            int y2 = y + 2;
            if (y2 >= Ly) y2 -= Ly;
            load_row(P, y2);
        }
        R uc[4] = {R(0), R(0), R(0), R(0)};
        if (act) load4(A.u + row + x, uc);
        // x-neighbours (sin, cos, lF) of the lane's first and last site
        R sL = from_lane_below(C.s[3]), cL = from_lane_below(C.c[3]), fL = from_lane_below(C.lF[3]);
        R sR = from_lane_above(C.s[0]), cR = from_lane_above(C.c[0]), fR = from_lane_above(C.lF[0]);
        if (edgeL) {
            Prec<R>::sincos(C.tL, sL, cL);
            fL = kap * Prec<R>::fma(v.dt, C.ltL, C.luL);
        }
        if (edgeR) {
            Prec<R>::sincos(C.tR, sR, cR);
            fR = kap * Prec<R>::fma(v.dt, C.ltR, C.luR);
        }
        R n[4];
        noise4<R>((uint32_t)y * qrow + (uint32_t)(x >> 2), v.replica, k, v.seed_lo, v.seed_hi, n);

        R lto[4], luo[4];
        R rx = 0, ry = 0, rh = 0, rg = 0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const R sxm = q == 0 ? sL : C.s[q - 1], cxm = q == 0 ? cL : C.c[q - 1], fxm = q == 0 ? fL : C.lF[q - 1];
            const R sxp = q == 3 ? sR : C.s[q + 1], cxp = q == 3 ? cR : C.c[q + 1], fxp = q == 3 ? fR : C.lF[q + 1];
            const int xs = x + q;
            const R eps = (((xs * v.stag_x) + (y * v.stag_y)) & 1) ? R(-1) : R(1);
            adj_site(v, K, C.s[q], C.c[q], sxm, cxm, fxm, sxp, cxp, fxp, P.s[q], P.c[q], P.lF[q], N.s[q], N.c[q],
                     N.lF[q], C.lF[q], C.lt[q], C.lu[q], uc[q], n[q], eps, lto[q], luo[q], rx, ry, rh, rg);
        }
        if (act) {
            store4(A.lt_out + row + x, lto);
            store4(A.lu_out + row + x, luo);
            gx += (double)rx;
            gy += (double)ry;
            gh += (double)rh;
            gg += (double)rg;
        }
    };

    AdjRow<R> Ra, Rb, Rc;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        Ra.th[q] = Rb.th[q] = Rc.th[q] = R(0);
        Ra.lt[q] = Rb.lt[q] = Rc.lt[q] = R(0);
        Ra.lu[q] = Rb.lu[q] = Rc.lu[q] = R(0);
    }
    Ra.tL = Ra.tR = Ra.ltL = Ra.ltR = Ra.luL = Ra.luR = R(0);
    Rb.tL = Rb.tR = Rb.ltL = Rb.ltR = Rb.luL = Rb.luR = R(0);
    Rc.tL = Rc.tR = Rc.ltL = Rc.ltR = Rc.luL = Rc.luR = R(0);
    load_row(Ra, y0 == 0 ? Ly - 1 : y0 - 1);
    load_row(Rb, y0);
    load_row(Rc, y0 + 1 == Ly ? 0 : y0 + 1);
    derive(Ra);
    derive(Rb);
    int y = y0;
    for (; y + 3 <= y1; y += 3) {
        do_row(Ra, Rb, Rc, y);
        do_row(Rb, Rc, Ra, y + 1);
        do_row(Rc, Ra, Rb, y + 2);
    }
    if (y < y1) {
        do_row(Ra, Rb, Rc, y);
        if (y + 1 < y1) do_row(Rb, Rc, Ra, y + 1);
    }
    // wave sums in a fixed butterfly; the task's slot is owned by this wave
    double acc[4] = {gx, gy, gh, gg};
#pragma unroll
    for (int p = 0; p < 4; ++p)
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) acc[p] += __shfl_xor(acc[p], off, kWave);
    if (lane == 0) {
        double* dst = A.gacc + (size_t)task * 4;
#pragma unroll
        for (int p = 0; p < 4; ++p) dst[p] += acc[p];
    }
}

template <typename R>
__global__ __launch_bounds__(256) void k_adjoint(AdjArgs<R> A, const uint64_t* kdev, uint64_t koff, int rows,
                                                 int ntasks) {
    const int wpb = blockDim.x / kWave;
    const int b = xcd_contiguous_block(blockIdx.x, gridDim.x);
    const int t = b * wpb + __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave));   // wave-uniform
    if (t >= ntasks) return;
    const uint64_t k = koff + (kdev ? *kdev : 0);
    adj_strip<R>(A, t, t % A.v.nxw, t / A.v.nxw, rows, k, threadIdx.x & (kWave - 1));
}

// Two reverse steps per pass, k + 1 then k, for rows up to kAdj2MaxLx sites:
// one site per lane, a workgroup per strip of ROWS rows across the whole
// width, in three phases separated by two barriers.
//  1. The strip's rows and two on each side enter ring A: (sin, cos) of
//     th^{k+1} and lF of stage A (from the adjoint at k+2), per site.
//  2. Stage A, reverse step k+1, on the strip's rows and one on each side
//     (which the neighbouring strips compute with the same arithmetic), its
//     neighbours from ring A; lF of stage B from its results (lt, lu at k+1)
//     enters ring B with (sin, cos) of th^k.  The results themselves stay in
//     the lane's registers, which also hold the lane's own lt, lu at k+2:
//     a site's own adjoint is only ever read by its own lane.
//  3. Stage B, reverse step k, on the strip's rows from ring B, to memory.
// Every input is loaded up front, so the pass waits on one memory latency.
// Every site takes the arithmetic of adj_site with the same inputs as in two
// single reverse steps, so lt^k and lu^k are bitwise those; the parameter
// adjoints are summed in another order.
template <typename R>
struct Adj2Args {
    AdjArgs<R> a;       // th, u: th^k, u^k; lt_in, lu_in: step k+2; lt_out, lu_out: step k
    const R* th1;       // th^{k+1}
    const R* u1;        // u^{k+1}
};

constexpr int kAdj2MaxLx = 1024;

template <typename R, int ROWS>
__global__ __launch_bounds__(kAdj2MaxLx) void k_adjoint2(Adj2Args<R> A2, const uint64_t* kdev, uint64_t koff) {
    const AdjArgs<R>& A = A2.a;
    const Lat<R>& v = A.v;
    const int Lx = v.Lx, Ly = v.Ly;
    extern __shared__ unsigned char adj2_lds[];
    // ring A: rows y0-2 .. y0+ROWS+1, ring B: rows y0-1 .. y0+ROWS; per row
    // [s, c, lF][Lx]
    R* ringA = reinterpret_cast<R*>(adj2_lds);
    R* ringB = ringA + (size_t)(ROWS + 4) * 3 * Lx;
    // the draws of stage A's rows (step k+1) and stage B's (step k), [row][Lx]
    R* noiseA = ringB + (size_t)(ROWS + 2) * 3 * Lx;
    R* noiseB = noiseA + (size_t)(ROWS + 2) * Lx;
    const int strip = xcd_contiguous_block(blockIdx.x, gridDim.x);
    const int y0 = strip * ROWS;
    const int y1 = min(y0 + ROWS, Ly);
    auto rowA = [&](int r) { return ringA + (size_t)(r - (y0 - 2)) * 3 * Lx; };
    auto rowB = [&](int r) { return ringB + (size_t)(r - (y0 - 1)) * 3 * Lx; };
    const int x = threadIdx.x;
    const bool act = x < Lx;
    const int xa = act ? x : 0;
    const int xm = xa == 0 ? Lx - 1 : xa - 1, xp = xa + 1 == Lx ? 0 : xa + 1;
    auto wrap = [&](int r) { return r < 0 ? r + Ly : (r >= Ly ? r - Ly : r); };
    auto at = [&](int r) { return (size_t)wrap(r) * (size_t)Lx + (size_t)xa; };
    // the strip's inputs, in the order of the phases (rows past a ragged last
    // strip's end are loaded, wrapped, and not used)
    R th1[ROWS + 4], lt2[ROWS + 4], lu2[ROWS + 4], u1[ROWS + 2], th0[ROWS + 2], u0[ROWS];
#pragma unroll
    for (int i = 0; i < ROWS + 4; ++i) {
        th1[i] = A2.th1[at(y0 - 2 + i)];
        lt2[i] = A.lt_in[at(y0 - 2 + i)];
        lu2[i] = A.lu_in[at(y0 - 2 + i)];
    }
#pragma unroll
    for (int i = 0; i < ROWS + 2; ++i) {
        u1[i] = A2.u1[at(y0 - 1 + i)];
        th0[i] = A.th[at(y0 - 1 + i)];
    }
#pragma unroll
    for (int i = 0; i < ROWS; ++i) u0[i] = A.u[at(y0 + i)];
    const uint64_t k = koff + (kdev ? *kdev : 0);
    const AdjStep<R> KA = adj_step_coef(A, k + 1);
    const AdjStep<R> KB = adj_step_coef(A, k);
    // a stage's reverse step at row r, its rows r-1, r, r+1 at C - stride,
    // C, C + stride in its ring, the lane's own (lt', lu') and draw n, with
    // coefficients K; returns lt, lu and adds the parameter adjoints of the
    // strip's own rows to g
    auto stage = [&](const R* C, size_t stride, const AdjStep<R>& K, int r, R lt, R lu, R u, R n, R& lto, R& luo,
                     R g[4]) {
        const R* Pm = C - stride;
        const R* Np = C + stride;
        const int y = wrap(r);
        const R eps = (((xa * v.stag_x) + (y * v.stag_y)) & 1) ? R(-1) : R(1);
        R rx = 0, ry = 0, rh = 0, rg = 0;
        adj_site(v, K, C[xa], C[Lx + xa], C[xm], C[Lx + xm], C[2 * Lx + xm], C[xp], C[Lx + xp], C[2 * Lx + xp],
                 Pm[xa], Pm[Lx + xa], Pm[2 * Lx + xa], Np[xa], Np[Lx + xa], Np[2 * Lx + xa], C[2 * Lx + xa], lt, lu,
                 u, n, eps, lto, luo, rx, ry, rh, rg);
        if (r >= y0 && r < y1) {
            g[0] += rx;
            g[1] += ry;
            g[2] += rh;
            g[3] += rg;
        }
    };
    const size_t stride = (size_t)3 * Lx;
    // the lane's parameter adjoints, in the state precision (at most
    // 2 ROWS + 2 terms), then FP64 across the wave
    R g[4] = {R(0), R(0), R(0), R(0)};
    // the draws: one Philox block per (stage, row, quad), shared out over the
    // workgroup's lanes instead of computed by each of a quad's four lanes
    {
        const int nq = Lx >> 2;
        const int nbA = (ROWS + 2) * nq, nb = nbA + ROWS * nq;
        for (int b = x; b < nb; b += blockDim.x) {
            const bool a = b < nbA;
            const int i = a ? b / nq : (b - nbA) / nq;
            const int q = a ? b - i * nq : (b - nbA) - i * nq;
            const int y = wrap(a ? y0 - 1 + i : y0 + i);
            R n4[4];
            noise4<R>((uint32_t)y * (uint32_t)nq + (uint32_t)q, v.replica, a ? k + 1 : k, v.seed_lo, v.seed_hi, n4);
            store4((a ? noiseA : noiseB) + (size_t)i * Lx + 4 * q, n4);
        }
    }
    // 1. ring A
    if (act) {
#pragma unroll
        for (int i = 0; i < ROWS + 4; ++i) {
            R* w = ringA + (size_t)i * stride;
            R sn, cs;
            Prec<R>::sincos(th1[i], sn, cs);
            w[xa] = sn;
            w[Lx + xa] = cs;
            w[2 * Lx + xa] = KA.kap * Prec<R>::fma(v.dt, lt2[i], lu2[i]);
        }
    }
    __syncthreads();
    // 2. stage A (reverse step k+1) on rows y0-1 .. y1, into ring B; its
    // results (lt, lu at k+1) stay in registers for stage B
    R lt1[ROWS + 2], lu1[ROWS + 2];
#pragma unroll
    for (int i = 0; i < ROWS + 2; ++i) lt1[i] = lu1[i] = R(0);
    if (act) {
#pragma unroll
        for (int i = 0; i < ROWS + 2; ++i) {
            const int r = y0 - 1 + i;
            if (r > y1) break;
            stage(rowA(r), stride, KA, r, lt2[i + 1], lu2[i + 1], u1[i], noiseA[(size_t)i * Lx + xa], lt1[i],
                  lu1[i], g);
            R* w = rowB(r);
            R sn, cs;
            Prec<R>::sincos(th0[i], sn, cs);
            w[xa] = sn;
            w[Lx + xa] = cs;
            w[2 * Lx + xa] = KB.kap * Prec<R>::fma(v.dt, lt1[i], lu1[i]);
        }
    }
    __syncthreads();
    // 3. stage B (reverse step k) on rows y0 .. y1-1, to memory
    if (act) {
#pragma unroll
        for (int i = 0; i < ROWS; ++i) {
            const int r = y0 + i;
            if (r >= y1) break;
            R lto, luo;
            stage(rowB(r), stride, KB, r, lt1[i + 1], lu1[i + 1], u0[i], noiseB[(size_t)i * Lx + xa], lto, luo, g);
            A.lt_out[at(r)] = lto;
            A.lu_out[at(r)] = luo;
        }
    }
    // wave totals, lane 16p holding value p; one slot per wave
    const int lane = x & (kWave - 1);
    const double gd[4] = {(double)g[0], (double)g[1], (double)g[2], (double)g[3]};
    const double tot = wave_sum4(gd, lane);
    const size_t wave = (size_t)strip * (blockDim.x / kWave) + (size_t)(x / kWave);
    if ((lane & 15) == 0) A.gacc[wave * 4 + (lane >> 4)] += tot;
}

// Seed of the reverse sweep at the last step N: lt = direct loss term, lu = 0.
template <typename R>
__global__ void k_adj_seed(Lat<R> v, const R* th, R* lt, R* lu, double cmN) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t N = (size_t)v.Lx * v.Ly;
    if (i >= N) return;
    const int x = (int)(i % v.Lx), y = (int)(i / v.Lx);
    const R eps = (((x * v.stag_x) + (y * v.stag_y)) & 1) ? R(-1) : R(1);
    R s, c;
    Prec<R>::sincos(th[i], s, c);
    lt[i] = (R)cmN * (-eps * s);
    lu[i] = R(0);
}

template <typename R>
bool adjoint2_fits(const Lat<R>& v, int rows) {
    return (rows == 1 || rows == 2 || rows == 4) && v.Lx <= kAdj2MaxLx && v.Ly >= 4 &&
           adjoint2_lds<R>(v.Lx, rows) <= 160 * 1024;
}

template <typename R>
int adjoint_tasks(const Lat<R>& v, int rows, int rows2) {
    const int single = ((v.Ly + rows - 1) / rows) * v.nxw;
    if (!adjoint2_fits(v, rows2)) return single;
    const int fused = ((v.Ly + rows2 - 1) / rows2) * ((v.Lx + kWave - 1) / kWave);
    return std::max(single, fused);
}

template <typename R>
void launch_adjoint_step(const Lat<R>& v, const R* th, const R* u, const R* lt_in, const R* lu_in, R* lt_out,
                         R* lu_out, const double* cm, uint64_t cm_base, double* gacc, const uint64_t* kdev,
                         uint64_t koff, const Launch& l, hipStream_t s) {
    AdjArgs<R> A;
    A.v = v;
    A.th = th;
    A.u = u;
    A.lt_in = lt_in;
    A.lu_in = lu_in;
    A.lt_out = lt_out;
    A.lu_out = lu_out;
    A.cm = cm;
    A.cm_base = cm_base;
    A.gacc = gacc;
    const int wpb = std::min(l.wpb, 4);
    const int ntasks = ((v.Ly + l.rows - 1) / l.rows) * v.nxw;
    const int nblocks = (ntasks + wpb - 1) / wpb;
    k_adjoint<R><<<nblocks, wpb * kWave, 0, s>>>(A, kdev, koff, l.rows, ntasks);
    check_hip(hipGetLastError(), "adjoint kernel launch");
}

// the LDS above the default limit is allowed once per device and instance
template <typename R, int ROWS>
static void launch_adjoint2(const Adj2Args<R>& A2, int nstrips, int threads, size_t lds, const uint64_t* kdev,
                            uint64_t koff, hipStream_t s) {
    static std::mutex mu;
    static std::set<int> allowed;
    int dev = 0;
    check_hip(hipGetDevice(&dev), "hipGetDevice");
    {
        std::lock_guard<std::mutex> lk(mu);
        if (!allowed.count(dev)) {
            check_hip(hipFuncSetAttribute(reinterpret_cast<const void*>(k_adjoint2<R, ROWS>),
                                          hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024),
                      "hipFuncSetAttribute");
            allowed.insert(dev);
        }
    }
    k_adjoint2<R, ROWS><<<nstrips, threads, lds, s>>>(A2, kdev, koff);
    check_hip(hipGetLastError(), "two-step reverse kernel launch");
}

template <typename R>
void launch_adjoint_step2(const Lat<R>& v, const R* th0, const R* u0, const R* th1, const R* u1, const R* lt_in,
                          const R* lu_in, R* lt_out, R* lu_out, const double* cm, uint64_t cm_base, double* gacc,
                          const uint64_t* kdev, uint64_t koff, int rows, hipStream_t s) {
    if (!adjoint2_fits(v, rows)) throw Error(-5, "two-step reverse pass: shape not supported");
    Adj2Args<R> A2;
    A2.a.v = v;
    A2.a.th = th0;
    A2.a.u = u0;
    A2.a.lt_in = lt_in;
    A2.a.lu_in = lu_in;
    A2.a.lt_out = lt_out;
    A2.a.lu_out = lu_out;
    A2.a.cm = cm;
    A2.a.cm_base = cm_base;
    A2.a.gacc = gacc;
    A2.th1 = th1;
    A2.u1 = u1;
    const int nstrips = (v.Ly + rows - 1) / rows;
    const int threads = (v.Lx + kWave - 1) / kWave * kWave;
    const size_t lds = adjoint2_lds<R>(v.Lx, rows);
    switch (rows) {
        case 1: launch_adjoint2<R, 1>(A2, nstrips, threads, lds, kdev, koff, s); break;
        case 2: launch_adjoint2<R, 2>(A2, nstrips, threads, lds, kdev, koff, s); break;
        case 4: launch_adjoint2<R, 4>(A2, nstrips, threads, lds, kdev, koff, s); break;
        default: throw Error(-5, "two-step reverse pass: rows per strip must be 1, 2 or 4");
    }
}

template <typename R>
void launch_adjoint_seed(const Lat<R>& v, const R* th, R* lt, R* lu, double cmN, hipStream_t s) {
    const size_t N = (size_t)v.Lx * v.Ly;
    k_adj_seed<R><<<(unsigned)((N + 255) / 256), 256, 0, s>>>(v, th, lt, lu, cmN);
    check_hip(hipGetLastError(), "adjoint seed launch");
}

template bool adjoint2_fits<float>(const Lat<float>&, int);
template bool adjoint2_fits<double>(const Lat<double>&, int);
template int adjoint_tasks<float>(const Lat<float>&, int, int);
template int adjoint_tasks<double>(const Lat<double>&, int, int);
template void launch_adjoint_step2<float>(const Lat<float>&, const float*, const float*, const float*, const float*,
                                          const float*, const float*, float*, float*, const double*, uint64_t,
                                          double*, const uint64_t*, uint64_t, int, hipStream_t);
template void launch_adjoint_step2<double>(const Lat<double>&, const double*, const double*, const double*,
                                           const double*, const double*, const double*, double*, double*,
                                           const double*, uint64_t, double*, const uint64_t*, uint64_t, int,
                                           hipStream_t);
template void launch_adjoint_step<float>(const Lat<float>&, const float*, const float*, const float*, const float*,
                                         float*, float*, const double*, uint64_t, double*, const uint64_t*, uint64_t,
                                         const Launch&, hipStream_t);
template void launch_adjoint_step<double>(const Lat<double>&, const double*, const double*, const double*,
                                          const double*, double*, double*, const double*, uint64_t, double*,
                                          const uint64_t*, uint64_t, const Launch&, hipStream_t);
template void launch_adjoint_seed<float>(const Lat<float>&, const float*, float*, float*, double, hipStream_t);
template void launch_adjoint_seed<double>(const Lat<double>&, const double*, double*, double*, double, hipStream_t);

}  // namespace xyl
