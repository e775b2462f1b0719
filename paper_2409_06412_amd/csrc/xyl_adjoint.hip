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
    const double hsd = half_sigma(v.sched, v.gamma, v.dtd, k);
    const R hs = (R)hsd;
    const bool fresh = (k == v.fresh_k);
    const R ca = v.c * v.a;
    const R kap = fresh ? v.hdt : v.hdt * (R(1) + ca);    // lF = kap (lu' + dt lt')
    const R lu_fac = fresh ? v.a : ca;                    // lu = lu_fac (lu' + dt lt')
    const R cm = (R)A.cm[k - A.cm_base];
    const R ghs = v.gamma > 0.0 ? (R)(hsd / (2.0 * v.gamma)) : R(0);
    const R ga = (R)(-0.5 * v.dtd);
    const R gc = (R)(-0.5 * v.dtd * (double)v.c * (double)v.c);
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
            const R s = C.s[q], c = C.c[q];
            const R sxm = q == 0 ? sL : C.s[q - 1], cxm = q == 0 ? cL : C.c[q - 1], fxm = q == 0 ? fL : C.lF[q - 1];
            const R sxp = q == 3 ? sR : C.s[q + 1], cxp = q == 3 ? cR : C.c[q + 1], fxp = q == 3 ? fR : C.lF[q + 1];
            const R sym = P.s[q], cym = P.c[q], fym = P.lF[q];
            const R syp = N.s[q], cyp = N.c[q], fyp = N.lF[q];
            // force and its parameter derivatives
            const R dFx = Prec<R>::fma(s, cxp + cxm, -(c * (sxp + sxm)));
            const R dFy = Prec<R>::fma(s, cyp + cym, -(c * (syp + sym)));
            const R dFh = R(-4) * s * c;
            const R F = Prec<R>::fma(v.Jx, dFx, Prec<R>::fma(v.Jy, dFy, (R)v.hd * dFh));
            // J lF with cos(th_i - th_j) = c c_j + s s_j
            const R lf = C.lF[q];
            const R jx = (c * cxp + s * sxp) * (lf - fxp) + (c * cxm + s * sxm) * (lf - fxm);
            const R jy = (c * cyp + s * syp) * (lf - fyp) + (c * cym + s * sym) * (lf - fym);
            const R jh = (c * c - s * s) * lf;
            const R Jl = Prec<R>::fma(v.Jx, jx, Prec<R>::fma(v.Jy, jy, -v.h4 * jh));
            const R g = Prec<R>::fma(v.dt, C.lt[q], C.lu[q]);
            const int xs = x + q;
            const R eps = (((xs * v.stag_x) + (y * v.stag_y)) & 1) ? R(-1) : R(1);
            lto[q] = C.lt[q] + Jl + cm * (-eps * s);
            luo[q] = lu_fac * g;
            // parameter adjoints
            rx = Prec<R>::fma(lf, dFx, rx);
            ry = Prec<R>::fma(lf, dFy, ry);
            rh = Prec<R>::fma(lf, dFh, rh);
            const R lw = v.a * g;
            if (fresh) {
                const R w = uc[q];
                rg += ga * g * w + ghs * n[q] * g;
            } else {
                const R Av = Prec<R>::fma(hs, n[q], Prec<R>::fma(v.hdt, F, uc[q]));
                const R w = v.c * Av;
                const R lA = v.c * lw;
                rg += ga * g * w + gc * lw * Av + ghs * n[q] * (g + lA);
            }
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
int adjoint_tasks(const Lat<R>& v, int rows) {
    return ((v.Ly + rows - 1) / rows) * v.nxw;
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
    const int ntasks = adjoint_tasks(v, l.rows);
    const int nblocks = (ntasks + wpb - 1) / wpb;
    k_adjoint<R><<<nblocks, wpb * kWave, 0, s>>>(A, kdev, koff, l.rows, ntasks);
    check_hip(hipGetLastError(), "adjoint kernel launch");
}

template <typename R>
void launch_adjoint_seed(const Lat<R>& v, const R* th, R* lt, R* lu, double cmN, hipStream_t s) {
    const size_t N = (size_t)v.Lx * v.Ly;
    k_adj_seed<R><<<(unsigned)((N + 255) / 256), 256, 0, s>>>(v, th, lt, lu, cmN);
    check_hip(hipGetLastError(), "adjoint seed launch");
}

template int adjoint_tasks<float>(const Lat<float>&, int);
template int adjoint_tasks<double>(const Lat<double>&, int);
template void launch_adjoint_step<float>(const Lat<float>&, const float*, const float*, const float*, const float*,
                                         float*, float*, const double*, uint64_t, double*, const uint64_t*, uint64_t,
                                         const Launch&, hipStream_t);
template void launch_adjoint_step<double>(const Lat<double>&, const double*, const double*, const double*,
                                          const double*, double*, double*, const double*, uint64_t, double*,
                                          const uint64_t*, uint64_t, const Launch&, hipStream_t);
template void launch_adjoint_seed<float>(const Lat<float>&, const float*, float*, float*, double, hipStream_t);
template void launch_adjoint_seed<double>(const Lat<double>&, const double*, double*, double*, double, hipStream_t);

}  // namespace xyl
