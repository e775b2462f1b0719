// Fused Langevin step of the symmetry-broken XY lattice on gfx950.
//
// One pass per step does, for every site: stencil force at th^k, completion of
// the previous step's second half-kick (App. A.1, Eq. BBK-2) giving w^k, the
// next first half-kick (Eq. BBK-1) giving w^{k+1/2}, the drift and the wrap
// (Sec. III.D).  Both half-kicks around time k share the Gaussian draw n^k,
// generated in registers from Philox4x32-10 keyed on (seed, replica, k, site);
// no noise is stored.  State: two angle buffers (ping-pong, th^k in
// th[(k + p0) & 1]) and the velocity buffer u, which holds w^{k-1/2}, or w^k
// itself at the step `fresh_k` after an initialisation.
//
// Work decomposition: a wave owns 256 consecutive sites of a row (4 per lane,
// one Philox block per lane) and walks down a strip of rows, keeping the
// sine/cosine of rows y-1, y, y+1 in registers, so every angle is loaded once
// per strip and its sine/cosine evaluated once.  x-neighbours inside the wave
// come from the adjacent lanes through DPP; the two wave-edge lanes load their
// outer neighbour.  Bytes per site-update: read th and u, write th' and u'.
//
// FP32 plain stepping also has a two-steps-per-pass kernel (k_step2, below):
// a workgroup spans the row and runs the second step one row behind the
// first, so the state is read and written once per two site-updates.
#include "xyl_device.hpp"
#include <mutex>
#include <set>
#include <type_traits>

namespace xyl {

// Register window of one row: raw angles and the two outer x-neighbours
// (used by the wave's edge lanes), their sine/cosine and the velocities.
template <typename R>
struct RowSet {
    R th[4];
    R eL, eR;
    R s[4], c[4];
    R u[4];
};

template <typename R, int MODE, int M, bool FK>
__device__ __forceinline__ void run_strip(const Lat<R>& v, int xw, int strip, int rows, uint64_t j, int lane) {
    const int Lx = v.Lx, Ly = v.Ly;
    const uint64_t k = v.k_base + j;
    // a replica steps while k < k_end and can still be measured at k_end
    if ((MODE & kStore) ? k >= v.k_end : k > v.k_end) return;
    const int y0 = strip * rows;
    if (y0 >= Ly) return;
    const int y1 = min(y0 + rows, Ly);
    const int x0 = xw * kWaveSites;
    const int nact = min(kWave, (Lx - x0) >> 2);
    const bool act = lane < nact;
    const bool edgeL = act && lane == 0;
    const bool edgeR = lane == nact - 1;
    const int x = x0 + kLaneSites * lane;
    const int xm = x == 0 ? Lx - 1 : x - 1;          // outer neighbours of the lane's 4 sites
    const int xp = x + 4 == Lx ? 0 : x + 4;
    const int par = (int)((k + (uint64_t)v.cur) & 1);
    const R* __restrict__ thi = v.pingpong ? v.th[par] : v.th[0];
    R* __restrict__ tho = v.pingpong ? v.th[par ^ 1] : v.th[1];
    const R* uu = v.u;
    R* uw = v.u_out ? v.u_out : v.u;
    const R hs = noise_coeff<R, FK>(v, k);   // FP32: -2 ln 2 hs^2 (/ kx^2 if FK); FP64: hs
    const bool fresh = (k == v.fresh_k);
    const uint32_t qrow = (uint32_t)(Lx >> 2);
    // byte offsets of the lane's quad and of its two outer neighbours in a row
    const uint32_t xb = (uint32_t)x * (uint32_t)sizeof(R);
    const uint32_t xmb = (uint32_t)xm * (uint32_t)sizeof(R), xpb = (uint32_t)xp * (uint32_t)sizeof(R);
    // measurement: the phases e^{-2 pi i x / Lx} of the lane's four columns
    // (FP64, from the lattice's table; the same on every row, so read once
    // per strip), each times the column's staggered sign along x: x is a
    // multiple of 4, so column x + q has the parity of q and the sign of the
    // odd columns is sxo (the stag flags are 0 or 1).  mc = sign cos,
    // ms = -sign sin, so every x-mode term is one fma.
    double mc[4], ms[4];
    const double sxo = v.stag_x ? -1.0 : 1.0;
    if constexpr ((MODE & kMeasure) != 0) {
        const double2* ph = reinterpret_cast<const double2*>(v.xph) + x;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const double2 e = act ? ph[q] : make_double2(0.0, 0.0);
            const double sg = (q & 1) ? sxo : 1.0;
            mc[q] = sg * e.y;
            ms[q] = -(sg * e.x);
        }
    }

    auto load_theta = [&](RowSet<R>& S, int y) {
        const R* r = row_start(thi, y, Lx);
        if (act) load4(at_byte(r, xb), S.th);
        if (edgeL) S.eL = *at_byte(r, xmb);
        if (edgeR) S.eR = *at_byte(r, xpb);
    };
    auto trig = [&](RowSet<R>& S) {
#pragma unroll
        for (int q = 0; q < 4; ++q) rotor<R, M>(S.th[q], S.s[q], S.c[q]);
    };

    // One row y with the window P = y-1, C = y, N = y+1 and F = y+2.  At entry
    // N.th (loaded two rows ago) and C.u are in registers and F.th is in
    // flight.  The row issues the loads of row y+3 into P's raw-angle slots
    // (dead since row y-1 was stored; P's sin/cos, still needed here, are not
    // touched) and of the velocities of row y+2 into F.
    auto do_row = [&](RowSet<R>& P, RowSet<R>& C, RowSet<R>& N, RowSet<R>& F, int y) {
        trig(N);
        if (y + 3 <= y1) {   // row y+2 will be processed: it needs row y+3 and its velocities
            int y3 = y + 3;
            if (y3 >= Ly) y3 -= Ly;
            load_theta(P, y3);
            if (act) load4(at_byte(row_start(uu, y + 2, Lx), xb), F.u);
        }
        // x-neighbours of the lane's first and last site
        // (the wave's first lane takes its left neighbour, the last active lane
        // its right one, from the extra angle loaded with the row; a wave with
        // a single active lane needs both)
        // (lane 0 is the first lane of every wave: the shift leaves it its own
        // value; in a full wave the same holds for lane 63 and the right edge)
        R se, ce;
        rotor<R, M>(edgeL ? C.eL : C.eR, se, ce);
        const R sL = from_lane_below(C.s[3], se), cL = from_lane_below(C.c[3], ce);
        R sR, cR;
        if (nact == kWave) {
            sR = from_lane_above(C.s[0], se);
            cR = from_lane_above(C.c[0], ce);
        } else {
            sR = from_lane_above(C.s[0]);
            cR = from_lane_above(C.c[0]);
            sR = edgeR ? se : sR;
            cR = edgeR ? ce : cR;
            if (nact == 1) rotor<R, M>(C.eR, sR, cR);
        }

        R n[4];
        noise4_kick<R>((uint32_t)y * qrow + (uint32_t)(x >> 2), v.replica, k, v.seed_lo, v.seed_hi, hs, n,
                       noise_u2<R, FK>(v));

        R tho4[4], uo4[4], w[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const R sxm = q == 0 ? sL : C.s[q - 1], cxm = q == 0 ? cL : C.c[q - 1];
            const R sxp = q == 3 ? sR : C.s[q + 1], cxp = q == 3 ? cR : C.c[q + 1];
            const R f = site_force<R, M, FK>(v, C.s[q], C.c[q], sxm, cxm, sxp, cxp, P.s[q], P.c[q], N.s[q], N.c[q],
                                             C.th[q], n[q]);
            site_update<R, M, FK>(v, f, C.u[q], C.th[q], n[q], hs, fresh, w[q], uo4[q], tho4[q]);
        }
        if ((MODE & kStore) && act) {
            store4(at_byte(row_start(tho, y, Lx), xb), tho4);
            store4(at_byte(row_start(uw, y, Lx), xb), uo4);
        }
        if ((MODE & kOmega) && act) store4(at_byte(row_start(v.omega_out, y, Lx), xb), w);

        if (MODE & kMeasure) {
            // per lane: energy terms, the order parameter's two components
            // and their x modes; the y modes are the row's phase times the
            // row's totals of the two components
            // (value 1 is the sum of w^2: the finalize halves it, which is
            // exact, so the sums equal those of the halved terms bit for bit)
            // (values 2 to 7 carry the x part of the staggered sign here;
            // the row's y part, a sign flip of the totals, is exact)
            double acc[8];
#pragma unroll
            for (int p = 0; p < 8; ++p) acc[p] = 0.0;
            const bool odd_row = (y & v.stag_y & 1) != 0;
            if (act) {
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const double s = (double)C.s[q], c = (double)C.c[q];
                    const double sxp = (double)(q == 3 ? sR : C.s[q + 1]);
                    const double cxp = (double)(q == 3 ? cR : C.c[q + 1]);
                    const double syp = (double)N.s[q], cyp = (double)N.c[q];
                    // bonds cos(th - th') = c c' + s s', the field cos 2th = c^2 - s^2 (XY)
                    const double bx = fma(c, cxp, s * sxp), by = fma(c, cyp, s * syp);
                    const double fld = M == kModelSI ? onsite_cos<R, M>(v, C.th[q], s, c) : fma(c, c, -(s * s));
                    acc[0] += fma(-v.hd, fld, fma(v.Jxd, bx, v.Jyd * by));
                    const double wq = (double)w[q];
                    acc[1] = fma(wq, wq, acc[1]);
                    // order-parameter component first: cos th (XY), sin 2th (SI)
                    const double a = M == kModelSI ? s : c, b = M == kModelSI ? c : s;
                    acc[2] = (q & 1) ? fma(a, sxo, acc[2]) : acc[2] + a;
                    acc[3] = (q & 1) ? fma(b, sxo, acc[3]) : acc[3] + b;
                    acc[4] = fma(a, mc[q], acc[4]);
                    acc[5] = fma(a, ms[q], acc[5]);
                    acc[6] = fma(b, mc[q], acc[6]);
                    acc[7] = fma(b, ms[q], acc[7]);
                }
            }
            // lane 8p holds the wave's total of value p; the row's staggered
            // sign along y on values 2 to 7
            double tot = wave_sum8(acc, lane);
            if (odd_row && lane >= 16) tot = -tot;
            double* base = v.part + (v.part_stride ? (k - v.part_k0) * v.part_stride : 0);
            double* dst = base + ((size_t)y * v.nxw + xw) * kNPart;
            if ((lane & 7) == 0) dst[lane >> 3] = tot;
            if (lane == 16 || lane == 24) {
                // y modes of the row: e^{-2 pi i y / Ly} (the lattice's table)
                // times the totals of the components (values 2 and 3)
                const double2 e = reinterpret_cast<const double2*>(v.yph)[y];
                const int o = lane == 16 ? 8 : 10;
                dst[o] = tot * e.y;
                dst[o + 1] = -(tot * e.x);
            }
        }
    };

    RowSet<R> A, B, C, D;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        A.th[q] = B.th[q] = C.th[q] = D.th[q] = R(0);
        A.u[q] = B.u[q] = C.u[q] = D.u[q] = R(0);
    }
    A.eL = A.eR = B.eL = B.eR = C.eL = C.eR = D.eL = D.eR = R(0);
    // prologue: A = row y0-1, B = row y0 (with velocities), C = row y0+1
    // (with velocities), D = row y0+2 in flight
    load_theta(A, y0 == 0 ? Ly - 1 : y0 - 1);
    load_theta(B, y0);
    load_theta(C, y0 + 1 >= Ly ? y0 + 1 - Ly : y0 + 1);
    load_theta(D, y0 + 2 >= Ly ? y0 + 2 - Ly : y0 + 2);
    if (act) {
        load4(at_byte(row_start(uu, y0, Lx), xb), B.u);
        if (y0 + 1 < y1) load4(at_byte(row_start(uu, y0 + 1, Lx), xb), C.u);
    }
    trig(A);
    trig(B);

    int y = y0;
    for (; y + 4 <= y1; y += 4) {
        do_row(A, B, C, D, y);
        do_row(B, C, D, A, y + 1);
        do_row(C, D, A, B, y + 2);
        do_row(D, A, B, C, y + 3);
    }
    if (y < y1) {
        do_row(A, B, C, D, y);
        if (y + 1 < y1) {
            do_row(B, C, D, A, y + 1);
            if (y + 2 < y1) do_row(C, D, A, B, y + 2);
        }
    }
}

// The strip with the lattice's form of the FP32 kick (factored by the x
// coupling where its `fact` is set, which the two-step passes require, so the
// two agree bit for bit); FP64 has one form.
template <typename R, int MODE, int M>
__device__ __forceinline__ void run_strip_any(const Lat<R>& v, int xw, int strip, int rows, uint64_t j, int lane) {
    if constexpr (sizeof(R) == 4) {
        if (v.fact) run_strip<R, MODE, M, true>(v, xw, strip, rows, j, lane);
        else run_strip<R, MODE, M, false>(v, xw, strip, rows, j, lane);
    } else {
        run_strip<R, MODE, M, false>(v, xw, strip, rows, j, lane);
    }
}

template <typename R, int MODE, int M>
__global__ __launch_bounds__(512) void k_step(Lat<R> v, const uint64_t* kdev, uint64_t j0, int rows, int ntasks) {
    const int wpb = blockDim.x / kWave;
    const int b = xcd_contiguous_block(blockIdx.x, gridDim.x);
    // the wave's index is uniform: read it into a scalar register, so that the
    // strip, row and address arithmetic derived from it stays scalar
    const int t = b * wpb + __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave));
    if (t >= ntasks) return;
    const uint64_t j = j0 + (kdev ? *kdev : 0);
    run_strip_any<R, MODE, M>(v, t % v.nxw, t / v.nxw, rows, j, threadIdx.x & (kWave - 1));
}

template <typename R, int MODE, int M>
__global__ __launch_bounds__(512) void k_ensemble_step(const Lat<R>* __restrict__ reps, const Task* __restrict__ tasks,
                                                       const uint64_t* kdev, uint64_t j0, int rows, int ntasks) {
    const int wpb = blockDim.x / kWave;
    const int b = xcd_contiguous_block(blockIdx.x, gridDim.x);
    const int t = b * wpb + __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave));
    if (t >= ntasks) return;
    const Task task = tasks[t];
    const uint64_t j = j0 + (kdev ? *kdev : 0);
    run_strip_any<R, MODE, M>(reps[task.rep], task.xw, task.strip, rows, j, threadIdx.x & (kWave - 1));
}

template <typename R, int M>
static void dispatch_step(const Lat<R>& v, int mode, const Launch& l, const uint64_t* kdev, uint64_t j, hipStream_t s) {
    const int nstrips = (v.Ly + l.rows - 1) / l.rows;
    const int ntasks = nstrips * v.nxw;
    const int nblocks = (ntasks + l.wpb - 1) / l.wpb;
    const dim3 grid(nblocks), block(l.wpb * kWave);
    switch (mode) {
        case kStore: k_step<R, kStore, M><<<grid, block, 0, s>>>(v, kdev, j, l.rows, ntasks); break;
        case kStore | kMeasure:
            k_step<R, kStore | kMeasure, M><<<grid, block, 0, s>>>(v, kdev, j, l.rows, ntasks);
            break;
        case kMeasure: k_step<R, kMeasure, M><<<grid, block, 0, s>>>(v, kdev, j, l.rows, ntasks); break;
        case kOmega: k_step<R, kOmega, M><<<grid, block, 0, s>>>(v, kdev, j, l.rows, ntasks); break;
        default: throw Error(-5, "unsupported step mode");
    }
    check_hip(hipGetLastError(), "step kernel launch");
}

template <typename R>
void launch_step(const Lat<R>& v, int mode, const Launch& l, const uint64_t* kdev, uint64_t j, hipStream_t s) {
    if (v.model == kModelSI) dispatch_step<R, kModelSI>(v, mode, l, kdev, j, s);
    else dispatch_step<R, kModelXY>(v, mode, l, kdev, j, s);
}

template <typename R, int M>
static void dispatch_ensemble_step(const Lat<R>* reps, const Task* tasks, int ntasks, int mode, int rows, int wpb,
                                   const uint64_t* kdev, uint64_t j, hipStream_t s) {
    const int nblocks = (ntasks + wpb - 1) / wpb;
    const dim3 grid(nblocks), block(wpb * kWave);
    switch (mode) {
        case kStore: k_ensemble_step<R, kStore, M><<<grid, block, 0, s>>>(reps, tasks, kdev, j, rows, ntasks); break;
        case kStore | kMeasure:
            k_ensemble_step<R, kStore | kMeasure, M><<<grid, block, 0, s>>>(reps, tasks, kdev, j, rows, ntasks);
            break;
        case kMeasure:
            k_ensemble_step<R, kMeasure, M><<<grid, block, 0, s>>>(reps, tasks, kdev, j, rows, ntasks);
            break;
        case kOmega: k_ensemble_step<R, kOmega, M><<<grid, block, 0, s>>>(reps, tasks, kdev, j, rows, ntasks); break;
        default: throw Error(-5, "unsupported step mode");
    }
    check_hip(hipGetLastError(), "ensemble step kernel launch");
}

template <typename R>
void launch_ensemble_step(const Lat<R>* reps, const Task* tasks, int ntasks, int mode, int model, int rows, int wpb,
                          const uint64_t* kdev, uint64_t j, hipStream_t s) {
    if (model == kModelSI) dispatch_ensemble_step<R, kModelSI>(reps, tasks, ntasks, mode, rows, wpb, kdev, j, s);
    else dispatch_ensemble_step<R, kModelXY>(reps, tasks, ntasks, mode, rows, wpb, kdev, j, s);
}

// ------------------------------------------------ two steps per pass (FP32)
// Temporal blocking: one workgroup owns a strip of rows across the whole
// lattice width (Lx / 256 waves, Lx <= 4096) and advances it two steps per
// pass.  Stage A (step k) runs one row ahead of stage B (step k+1): after
// stage A has produced row y, stage B advances row y-1.  Stage A also covers
// one halo row on each side of the strip (recomputed by the neighbouring strip
// as well; same arithmetic, same values).  Stage A writes the rotors of its
// rows to an LDS ring of four rows (8 bytes per site per row), from which
// stage B takes all its neighbours; its angles and velocities stay in
// registers.  One barrier per row separates the stage-A writes from the
// stage-B reads; with four slots a wave that runs one row ahead writes a slot
// nobody still reads.  Register budget (1024 threads, 128 VGPRs, no spills, so
// no reload wait drains the prefetch): step-k angles and rotors of three rows,
// velocities and the outer-edge angle of two, stage-A outputs of two.  A row's
// angles are loaded one iteration before its rotors are needed, its velocities
// one iteration before its update.  Outputs go to the other angle buffer and a
// second velocity buffer, so no strip overwrites rows its neighbours still
// read.  Per-site arithmetic is the shared rotor / site_force / site_update /
// noise4_kick, so the states equal those of two single steps bit for bit.
// Bytes per two site-updates: read angle and velocity (plus the halo rows),
// write both.
struct Step2Buffers {
    const float* th_in;
    const float* u_in;
    float* th_out;
    float* u_out;
    float* th_mid = nullptr;   // with MID: the state after the first step
    float* u_mid = nullptr;
};

template <typename R>
struct TRow {          // step-k row: angles and rotors
    R th[4], s[4], c[4];
};
template <typename R>
struct URow {          // step-k row: velocities and the angle across the lane's outer edge
    R u[4];
    R e;
};
template <typename R>
struct BRow {          // step-(k+1) angles and velocities of one stage-A row
    R t[4], u[4];
};

// One strip of a two-step pass: rows [y0, y1) of the lattice v, swept in
// direction d (+1 top-down, -1 bottom-up), from step k.  rot is the LDS ring
// (4 slots x 2 x W floats).
//  * Whole rows (TILE false, xs = 0, W = Lx).  With PARTIAL the width need not
//    be a multiple of 256: lanes past the row's end work on its last quad
//    (every access in bounds) and store nothing, and the last active lane takes
//    its right neighbour across the row's end like a wave's last lane.  The
//    last wave has at least two active lanes (step2_width_ok), so no lane is
//    both the left and the right edge.
//  * A column tile of a wider row (TILE): the workgroup covers the W sites from
//    global column xs (wrapped; xs and W multiples of 4): the tile's own
//    columns and one quad on each side.  Stage A runs on all of them; stage B
//    stores all but the two outer quads, whose second step the neighbouring
//    tiles compute.  Every stored site so sees the same inputs as in single
//    steps.
//  * With MID (whole rows), stage A also stores the strip's own rows of the
//    state after the first step (th_mid, u_mid), as a single step would.
template <int M, bool PARTIAL, bool TILE = false, bool MID = false>
__device__ __forceinline__ void step2_strip(const Lat<float>& v, const Step2Buffers& B, int y0, int y1, int d,
                                            uint64_t k, float* rot, int xs = 0, int W = 0) {
    using R = float;
    const int Lx = v.Lx, Ly = v.Ly;
    const int Wd = TILE ? W : Lx;                    // sites the workgroup covers
    const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave));
    const int lane = threadIdx.x & (kWave - 1);
    const int xl = (wv << 8) + kLaneSites * lane;
    const bool valid = !(PARTIAL || TILE) || xl < Wd;
    const int x = valid ? xl : Wd - kLaneSites;      // local column of the lane's quad
    auto wrap_x = [&](int g) { return g < 0 ? g + Lx : (g >= Lx ? g - Lx : g); };
    const int gx = TILE ? wrap_x(xs + x) : x;        // its global column
    const bool edgeL = lane == 0;
    const bool edgeR = lane == kWave - 1 || ((PARTIAL || TILE) && xl + kLaneSites == Wd);
    // global column of the lane's outer neighbour (lane 0: left of the wave;
    // the right edge: right of it; other lanes: a site of their own, unused)
    const int xe = edgeL ? (TILE ? wrap_x(gx - 1) : (x == 0 ? Lx - 1 : x - 1))
                         : (edgeR ? (TILE ? wrap_x(gx + 4) : (x + 4 == Lx ? 0 : x + 4))
                                  : (TILE ? gx : min((wv << 8) + lane, Lx - 1)));
    // the same neighbour in the LDS ring (local columns; a tile's two outer
    // quads store no second step, so theirs is any column in range)
    const int xel = TILE ? (edgeL ? (x == 0 ? 0 : x - 1) : (edgeR ? (x + 4 == Wd ? Wd - 1 : x + 4) : x)) : xe;
    const bool store_b = valid && (!TILE || (x != 0 && x + kLaneSites != Wd));
    // right neighbour of the lane's last site: from the lane above, or the
    // edge value (DPP hands it to lane 63; a partial row's last lane selects it)
    auto right_of = [&](float v_above, float edge) {
        const float r = from_lane_above(v_above, edge);
        return (PARTIAL || TILE) ? (edgeR ? edge : r) : r;
    };
    // the two-step passes take lattices with the factored FP32 kick only
    const R hsA = noise_coeff<R, true>(v, k);
    const R hsB = noise_coeff<R, true>(v, k + 1);
    const bool freshA = (k == v.fresh_k), freshB = (k + 1 == v.fresh_k);
    const uint32_t qrow = (uint32_t)(Lx >> 2);
    auto wrap_y = [&](int y) { return y < 0 ? y + Ly : (y >= Ly ? y - Ly : y); };
    auto slot = [&](int it) { return rot + (size_t)(it & (kStep2Slots - 1)) * 2 * Wd; };

    // byte offsets of the lane's quad and of its outer neighbour in a row
    const uint32_t gxb = (uint32_t)gx * 4u, xeb = (uint32_t)xe * 4u;
    auto load_th = [&](TRow<R>& T, int y) { load4(at_byte(row_start(B.th_in, y, Lx), gxb), T.th); };
    auto load_u = [&](URow<R>& U, int y) {
        load4(at_byte(row_start(B.u_in, y, Lx), gxb), U.u);
        U.e = *at_byte(row_start(B.th_in, y, Lx), xeb);
    };
    auto trig = [&](TRow<R>& T) {
#pragma unroll
        for (int q = 0; q < 4; ++q) rotor<R, M>(T.th[q], T.s[q], T.c[q]);
    };
    // stage A on row y of iteration it: C = row y at step k, P and N its two
    // y-neighbours (the row before and the row after in the strip's direction);
    // rotors to LDS, angles and velocities to `out`
    auto stage_a = [&](const TRow<R>& P, const TRow<R>& C, const TRow<R>& N, const URow<R>& U, int y, int it,
                       BRow<R>& out) {
        R se, ce;
        rotor<R, M>(U.e, se, ce);
        const R sL = from_lane_below(C.s[3], se), cL = from_lane_below(C.c[3], ce);
        const R sR = right_of(C.s[0], se), cR = right_of(C.c[0], ce);
        R n[4];
        noise4_kick<R>((uint32_t)y * qrow + (uint32_t)(gx >> 2), v.replica, k, v.seed_lo, v.seed_hi, hsA, n,
                       noise_u2<R, true>(v));
        R s1[4], c1[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const R sxm = q == 0 ? sL : C.s[q - 1], cxm = q == 0 ? cL : C.c[q - 1];
            const R sxp = q == 3 ? sR : C.s[q + 1], cxp = q == 3 ? cR : C.c[q + 1];
            const R f = site_force<R, M, true>(v, C.s[q], C.c[q], sxm, cxm, sxp, cxp, P.s[q], P.c[q], N.s[q], N.c[q],
                                               C.th[q], n[q]);
            R w;
            site_update<R, M, true>(v, f, U.u[q], C.th[q], n[q], hsA, freshA, w, out.u[q], out.t[q]);
            rotor<R, M>(out.t[q], s1[q], c1[q]);
        }
        if (valid) {
            float* rs = slot(it);
            store4(rs + x, s1);
            store4(rs + Wd + x, c1);
        }
        if constexpr (MID) {
            // the first and last iterations are the strip's halo rows
            if (valid && it >= 1 && it <= (y1 - y0)) {
                store4(at_byte(row_start(B.th_mid, y, Lx), gxb), out.t);
                store4(at_byte(row_start(B.u_mid, y, Lx), gxb), out.u);
            }
        }
    };
    // stage B on row y (stage-A values C in registers; the rotors of row y
    // and of its two y-neighbours in the LDS slots of iterations it-1, it-2
    // and it)
    auto stage_b = [&](const BRow<R>& C, int y, int it) {
        const float* rp = slot(it - 2);
        const float* rc = slot(it - 1);
        const float* rn = slot(it);
        R sc[4], cc[4];
        load4(rc + x, sc);
        load4(rc + Wd + x, cc);
        const R se = rc[xel], ce = rc[Wd + xel];
        const R sL = from_lane_below(sc[3], se), cL = from_lane_below(cc[3], ce);
        const R sR = right_of(sc[0], se), cR = right_of(cc[0], ce);
        R sp[4], cp[4], sn[4], cn[4];
        load4(rp + x, sp);
        load4(rp + Wd + x, cp);
        load4(rn + x, sn);
        load4(rn + Wd + x, cn);
        R n[4];
        noise4_kick<R>((uint32_t)y * qrow + (uint32_t)(gx >> 2), v.replica, k + 1, v.seed_lo, v.seed_hi, hsB, n,
                       noise_u2<R, true>(v));
        R tho[4], uo[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const R sxm = q == 0 ? sL : sc[q - 1], cxm = q == 0 ? cL : cc[q - 1];
            const R sxp = q == 3 ? sR : sc[q + 1], cxp = q == 3 ? cR : cc[q + 1];
            const R f =
                site_force<R, M, true>(v, sc[q], cc[q], sxm, cxm, sxp, cxp, sp[q], cp[q], sn[q], cn[q], C.t[q], n[q]);
            R w;
            site_update<R, M, true>(v, f, C.u[q], C.t[q], n[q], hsB, freshB, w, uo[q], tho[q]);
        }
        if (store_b) {
            store4(at_byte(row_start(B.th_out, y, Lx), gxb), tho);
            store4(at_byte(row_start(B.u_out, y, Lx), gxb), uo);
        }
    };

    // Even strips run top-down, odd strips bottom-up (the force is symmetric in
    // the two y-neighbours, sums of the two, so the values do not depend on
    // the direction): the halo rows a strip shares with its neighbour are then
    // read by both at the same end of their passes, while the rows are in L2
    // (neighbouring strips run on one XCD).  With d = +1 or -1 and
    // r(i) = ys + d i (wrapped), iteration it (0 .. nit-1) runs stage A on row
    // r(it) and, from it = 2 on, stage B on row r(it-1).  On entry P holds the
    // rotors of row r(it-1), C the angles and rotors of r(it), N the angles of
    // r(it+1), UC the velocities of r(it); the iteration loads the angles of
    // r(it+2) into P and the velocities of r(it+1) into UN (the last iteration
    // reloads rows the one before loaded, so that every iteration loads and
    // nothing outside the strip's rows is fetched).
    const int nit = (y1 - y0) + 2;
    const int ys = d > 0 ? y0 - 1 : y1;
    auto rowof = [&](int i) { return wrap_y(ys + d * i); };
    TRow<R> T0, T1, T2;
    URow<R> U0, U1;
    BRow<R> B0, B1;
    load_th(T0, rowof(-1));
    load_th(T1, rowof(0));
    load_th(T2, rowof(1));
    load_u(U0, rowof(0));
    trig(T0);
    trig(T1);
    // Stage B runs in every iteration of the loop: the first two iterations
    // are peeled and end with a full wait, so that the compiler's counter
    // waits inside the loop need not cover a path without stores (which would
    // make the next row's wait also wait for the stores just issued).
    auto iterate = [&](auto with_b, TRow<R>& P, TRow<R>& C, TRow<R>& N, URow<R>& UC, URow<R>& UN, BRow<R>& Bn,
                       BRow<R>& Bp, int it) {
        trig(N);
        load_th(P, rowof(min(it + 2, nit)));
        load_u(UN, rowof(min(it + 1, nit - 1)));
        __builtin_amdgcn_sched_barrier(0);   // keep the loads ahead of stage A
        stage_a(P, C, N, UC, rowof(it), it, Bn);
        __syncthreads();
        if constexpr (decltype(with_b)::value) stage_b(Bp, rowof(it - 1), it);
    };
    const std::false_type first{};
    const std::true_type full{};
    iterate(first, T0, T1, T2, U0, U1, B0, B1, 0);
    iterate(first, T1, T2, T0, U1, U0, B1, B0, 1);
    __builtin_amdgcn_s_waitcnt(0);
    int it = 2;
    for (; it + 6 <= nit; it += 6) {
        iterate(full, T2, T0, T1, U0, U1, B0, B1, it);
        iterate(full, T0, T1, T2, U1, U0, B1, B0, it + 1);
        iterate(full, T1, T2, T0, U0, U1, B0, B1, it + 2);
        iterate(full, T2, T0, T1, U1, U0, B1, B0, it + 3);
        iterate(full, T0, T1, T2, U0, U1, B0, B1, it + 4);
        iterate(full, T1, T2, T0, U1, U0, B1, B0, it + 5);
    }
    if (it < nit) iterate(full, T2, T0, T1, U0, U1, B0, B1, it);
    if (it + 1 < nit) iterate(full, T0, T1, T2, U1, U0, B1, B0, it + 1);
    if (it + 2 < nit) iterate(full, T1, T2, T0, U0, U1, B0, B1, it + 2);
    if (it + 3 < nit) iterate(full, T2, T0, T1, U1, U0, B1, B0, it + 3);
    if (it + 4 < nit) iterate(full, T0, T1, T2, U0, U1, B0, B1, it + 4);
}

// The two-step pass of one lattice: strip b = rows [b rows, (b+1) rows), even
// strips top-down, odd strips bottom-up.
template <int M, bool PARTIAL, bool MID = false>
__global__ __launch_bounds__(1024) void k_step2(Lat<float> v, Step2Buffers B, const uint64_t* kdev, uint64_t j0,
                                                int rows) {
    extern __shared__ float rot[];   // [slot][s | c][Lx]
    const int strip = xcd_contiguous_block(blockIdx.x, gridDim.x);
    const int y0 = strip * rows;
    const int y1 = min(y0 + rows, v.Ly);
    const uint64_t k = v.k_base + j0 + (kdev ? *kdev : 0);
    step2_strip<M, PARTIAL, false, MID>(v, B, y0, y1, (strip & 1) ? -1 : 1, k, rot);
}

// The two-step pass of a lattice wider than 4096: each strip is split into ntx
// column tiles of w columns (the last takes the rest); workgroup b covers tile
// b % ntx of strip b / ntx and one quad on each side.
template <int M, int MAXW>
__global__ __launch_bounds__(MAXW * kWave, MAXW <= 8 ? 4 : 1) void k_step2_tiled(Lat<float> v, Step2Buffers B, const uint64_t* kdev,
                                                             uint64_t j0, int rows, int ntx, int w) {
    extern __shared__ float rot[];   // [slot][s | c][w + 8]
    const int b = xcd_contiguous_block(blockIdx.x, gridDim.x);
    const int strip = b / ntx, tx = b - strip * ntx;
    const int y0 = strip * rows;
    const int y1 = min(y0 + rows, v.Ly);
    const uint64_t k = v.k_base + j0 + (kdev ? *kdev : 0);
    const int wt = tx == ntx - 1 ? v.Lx - tx * w : w;
    step2_strip<M, true, true>(v, B, y0, y1, (strip & 1) ? -1 : 1, k, rot, tx * w - kLaneSites, wt + 2 * kLaneSites);
}

// The two-step pass of many replicas in one launch: one workgroup per task
// (replica, strip); every replica of the launch spans the same number of waves.
// The first pass of a pair (phase 0) reads the angles at step k from
// th[k & 1] and the velocities from u, and writes the other angle buffer and
// u2; the second (phase 1) goes back, so that a pair of passes leaves the
// state where the replica's step parity expects it.  u2 is the replica's
// velocities' place in a second array: u2_base + (v.u - u_base).
template <int M, bool PARTIAL>
__global__ __launch_bounds__(1024) void k_ensemble_step2(const Lat<float>* __restrict__ reps,
                                                         const Task2* __restrict__ tasks, int phase,
                                                         const float* u_base, float* u2_base, const uint64_t* kdev,
                                                         uint64_t j0) {
    extern __shared__ float rot[];
    const Task2 t = tasks[xcd_contiguous_block(blockIdx.x, gridDim.x)];
    const Lat<float>& v = reps[t.rep];
    const uint64_t k = v.k_base + j0 + (kdev ? *kdev : 0);
    float* u = v.u;
    float* u2 = u2_base + (u - u_base);
    float* tA = v.th[(int)((k + (uint64_t)v.cur + (uint64_t)phase) & 1)];
    float* tB = v.th[(int)((k + (uint64_t)v.cur + (uint64_t)phase + 1) & 1)];
    const Step2Buffers B{tA, phase ? u2 : u, tB, phase ? u : u2};
    step2_strip<M, PARTIAL>(v, B, t.y0, t.y1, t.dir, k, rot);
}

// the LDS ring of the widest rows (4096 sites: 128 KiB) is allowed once per
// device and kernel instance, not on every launch
template <typename F>
static void allow_step2_lds(F* kernel) {
    static std::mutex mu;
    static std::set<std::pair<int, const void*>> allowed;
    int dev = 0;
    check_hip(hipGetDevice(&dev), "hipGetDevice");
    std::lock_guard<std::mutex> lk(mu);
    if (allowed.count({dev, reinterpret_cast<const void*>(kernel)})) return;
    const int max_lds = (int)(sizeof(float) * 2 * kStep2Slots * 16 * kWaveSites);
    check_hip(hipFuncSetAttribute(reinterpret_cast<const void*>(kernel), hipFuncAttributeMaxDynamicSharedMemorySize,
                                  max_lds),
              "hipFuncSetAttribute");
    allowed.insert({dev, reinterpret_cast<const void*>(kernel)});
}

template <int M, bool PARTIAL, bool MID = false>
static void dispatch_step2(const Lat<float>& v, const Step2Buffers& b, int rows, const uint64_t* kdev, uint64_t j,
                           hipStream_t s) {
    allow_step2_lds(k_step2<M, PARTIAL, MID>);
    const int nstrips = (v.Ly + rows - 1) / rows;
    const size_t lds = sizeof(float) * 2 * (size_t)kStep2Slots * (size_t)v.Lx;
    const int waves = (v.Lx + kWaveSites - 1) / kWaveSites;
    k_step2<M, PARTIAL, MID><<<nstrips, waves * kWave, lds, s>>>(v, b, kdev, j, rows);
    check_hip(hipGetLastError(), "two-step kernel launch");
}

void launch_step2_mid(const Lat<float>& v, const float* th_in, const float* u_in, float* th_mid, float* u_mid,
                      float* th_out, float* u_out, int rows, const uint64_t* kdev, uint64_t j, hipStream_t s) {
    if (v.Ly < 4 || rows < 1 || !step2_width_ok(v.Lx) || v.model != kModelXY)
        throw Error(-5, "two-step pass with the middle state: XY lattices of whole-row widths only");
    Step2Buffers b{th_in, u_in, th_out, u_out};
    b.th_mid = th_mid;
    b.u_mid = u_mid;
    if (v.Lx % kWaveSites != 0) dispatch_step2<kModelXY, true, true>(v, b, rows, kdev, j, s);
    else dispatch_step2<kModelXY, false, true>(v, b, rows, kdev, j, s);
}

template <int M, int MAXW>
static void launch_step2_tiled(const Lat<float>& v, const Step2Buffers& b, int nwg, int waves, size_t lds, int rows,
                               const Step2Tiles& t, const uint64_t* kdev, uint64_t j, hipStream_t s) {
    allow_step2_lds(k_step2_tiled<M, MAXW>);
    k_step2_tiled<M, MAXW><<<nwg, waves * kWave, lds, s>>>(v, b, kdev, j, rows, t.ntx, t.w);
}

template <int M>
static void dispatch_step2_tiled(const Lat<float>& v, const Step2Buffers& b, int rows, const Step2Tiles& t,
                                 const uint64_t* kdev, uint64_t j, hipStream_t s) {
    const int nwg = ((v.Ly + rows - 1) / rows) * t.ntx;
    const int W = t.w + 2 * kLaneSites;
    const size_t lds = sizeof(float) * 2 * (size_t)kStep2Slots * (size_t)W;
    const int waves = (W + kWaveSites - 1) / kWaveSites;
    switch (step2_tile_bound(waves)) {
        case 4: launch_step2_tiled<M, 4>(v, b, nwg, waves, lds, rows, t, kdev, j, s); break;
        case 8: launch_step2_tiled<M, 8>(v, b, nwg, waves, lds, rows, t, kdev, j, s); break;
        case 11: launch_step2_tiled<M, 11>(v, b, nwg, waves, lds, rows, t, kdev, j, s); break;
        default: launch_step2_tiled<M, 16>(v, b, nwg, waves, lds, rows, t, kdev, j, s); break;
    }
    check_hip(hipGetLastError(), "tiled two-step kernel launch");
}

void launch_step2(const Lat<float>& v, const float* th_in, const float* u_in, float* th_out, float* u_out, int rows,
                  const uint64_t* kdev, uint64_t j, hipStream_t s, int tile_waves) {
    if (v.Ly < 4 || rows < 1) throw Error(-5, "two-step kernel needs Ly >= 4");
    const Step2Buffers b{th_in, u_in, th_out, u_out};
    Step2Tiles t;
    if ((tile_waves > 0 && step2_tiles(v.Lx, &t, tile_waves)) || step2_tiles(v.Lx, &t)) {
        if (v.model == kModelSI) dispatch_step2_tiled<kModelSI>(v, b, rows, t, kdev, j, s);
        else dispatch_step2_tiled<kModelXY>(v, b, rows, t, kdev, j, s);
        return;
    }
    if (!step2_width_ok(v.Lx))
        throw Error(-5, "two-step kernel: width must use 3/4 of its waves' lanes and two of the last, or exceed 4096");
    const bool partial = v.Lx % kWaveSites != 0;
    if (v.model == kModelSI) {
        if (partial) dispatch_step2<kModelSI, true>(v, b, rows, kdev, j, s);
        else dispatch_step2<kModelSI, false>(v, b, rows, kdev, j, s);
    } else {
        if (partial) dispatch_step2<kModelXY, true>(v, b, rows, kdev, j, s);
        else dispatch_step2<kModelXY, false>(v, b, rows, kdev, j, s);
    }
}

template <int M, bool PARTIAL>
static void dispatch_ensemble_step2(const Lat<float>* reps, const Task2* tasks, int ntasks, int waves, int max_lx,
                                    int phase, const float* u_base, float* u2_base, const uint64_t* kdev, uint64_t j,
                                    hipStream_t s) {
    allow_step2_lds(k_ensemble_step2<M, PARTIAL>);
    const size_t lds = sizeof(float) * 2 * (size_t)kStep2Slots * (size_t)max_lx;
    k_ensemble_step2<M, PARTIAL><<<ntasks, waves * kWave, lds, s>>>(reps, tasks, phase, u_base, u2_base, kdev, j);
    check_hip(hipGetLastError(), "ensemble two-step kernel launch");
}

void launch_ensemble_step2(const Lat<float>* reps, const Task2* tasks, int ntasks, int waves, bool partial,
                           int max_lx, int model, int phase, const float* u_base, float* u2_base,
                           const uint64_t* kdev, uint64_t j, hipStream_t s) {
    if (ntasks < 1 || waves < 1 || waves > 16 || max_lx > 16 * kWaveSites)
        throw Error(-5, "ensemble two-step launch: bad task count or width");
    if (model == kModelSI) {
        if (partial) dispatch_ensemble_step2<kModelSI, true>(reps, tasks, ntasks, waves, max_lx, phase, u_base, u2_base,
                                                             kdev, j, s);
        else dispatch_ensemble_step2<kModelSI, false>(reps, tasks, ntasks, waves, max_lx, phase, u_base, u2_base,
                                                      kdev, j, s);
    } else {
        if (partial) dispatch_ensemble_step2<kModelXY, true>(reps, tasks, ntasks, waves, max_lx, phase, u_base, u2_base,
                                                             kdev, j, s);
        else dispatch_ensemble_step2<kModelXY, false>(reps, tasks, ntasks, waves, max_lx, phase, u_base, u2_base,
                                                      kdev, j, s);
    }
}

// -------------------------------------------- whole replica in LDS (FP32)
// Small replicas of an ensemble: one workgroup holds the sine/cosine tables
// of a whole lattice in LDS (8 B per site, 128 KB at 128 x 128) and its
// angles and velocities in registers (up to 4 Philox blocks of 4 sites per
// thread), and advances it several steps per launch with two barriers per
// step and no HBM traffic between steps.  Per-site arithmetic is the shared
// site_force / site_update / noise4, so states equal those of the strip
// kernel bit for bit.
struct LdsJob {
    int32_t rep;        // replica index in the table
    int32_t measure;    // 1: record observables at the launch's first step
    int32_t nsteps;     // steps to advance (0: measure only)
    int32_t pad;
    double* obs;        // 6 doubles
};

template <int M, bool F>
__device__ __forceinline__ void lds_replica(const Lat<float>& v, const LdsJob& job, uint64_t j0, float* lds,
                                            double (*red)[kNPart]) {
    const int Lx = v.Lx, Ly = v.Ly;
    const int N = Lx * Ly, ng = N >> 2;
    float* S = lds;
    float* C = lds + N;
    const int tid = threadIdx.x, nt = blockDim.x;
    const uint64_t k0 = v.k_base + j0;
    float th[kLdsMaxGroups][4], u[kLdsMaxGroups][4];
    {
        const float* t0 = v.th[(int)((k0 + (uint64_t)v.cur) & 1)];
#pragma unroll
        for (int q = 0; q < kLdsMaxGroups; ++q) {
            const int g = tid + q * nt;
            if (g < ng) {
                load4(t0 + 4 * g, th[q]);
                load4(v.u + 4 * g, u[q]);
            } else {
#pragma unroll
                for (int e = 0; e < 4; ++e) th[q][e] = u[q][e] = 0.f;
            }
        }
    }
    auto tables = [&]() {
#pragma unroll
        for (int q = 0; q < kLdsMaxGroups; ++q) {
            const int g = tid + q * nt;
            if (g < ng) {
                float s4[4], c4[4];
#pragma unroll
                for (int e = 0; e < 4; ++e) rotor<float, M>(th[q][e], s4[e], c4[e]);
                store4(S + 4 * g, s4);
                store4(C + 4 * g, c4);
            }
        }
    };
    // neighbours of group g from the tables; returns the kick of its 4 sites
    // (site_force, with their scaled draws n)
    auto forces = [&](int g, const float t4[4], const float n[4], float f[4], float s4[4], float c4[4], float& sR,
                      float& cR, float sd[4], float cd[4]) {
        const int i0 = 4 * g;
        const int y = i0 / Lx, x = i0 - y * Lx;
        const int ym = y == 0 ? Ly - 1 : y - 1, yp = y + 1 == Ly ? 0 : y + 1;
        float su[4], cu[4];
        load4(S + i0, s4);
        load4(C + i0, c4);
        load4(S + ym * Lx + x, su);
        load4(C + ym * Lx + x, cu);
        load4(S + yp * Lx + x, sd);
        load4(C + yp * Lx + x, cd);
        const int il = y * Lx + (x == 0 ? Lx - 1 : x - 1);
        const int ir = y * Lx + (x + 4 == Lx ? 0 : x + 4);
        const float sL = S[il], cL = C[il];
        sR = S[ir];
        cR = C[ir];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const float sxm = e == 0 ? sL : s4[e - 1], cxm = e == 0 ? cL : c4[e - 1];
            const float sxp = e == 3 ? sR : s4[e + 1], cxp = e == 3 ? cR : c4[e + 1];
            f[e] = site_force<float, M, F>(v, s4[e], c4[e], sxm, cxm, sxp, cxp, su[e], cu[e], sd[e], cd[e], t4[e],
                                           n[e]);
        }
    };

    tables();
    __syncthreads();
    if (job.measure) {
        // observables of the synchronized state at k0 (same sums as the strip kernel)
        const float hs = noise_coeff<float, F>(v, k0);
        const bool fresh = (k0 == v.fresh_k);
        double acc[kNPart];
#pragma unroll
        for (int p = 0; p < kNPart; ++p) acc[p] = 0.0;
#pragma unroll
        for (int q = 0; q < kLdsMaxGroups; ++q) {
            const int g = tid + q * nt;
            if (g < ng) {
                float f[4], s4[4], c4[4], sd[4], cd[4], sR, cR, n[4];
                noise4_kick<float>((uint32_t)g, v.replica, k0, v.seed_lo, v.seed_hi, hs, n, noise_u2<float, F>(v));
                forces(g, th[q], n, f, s4, c4, sR, cR, sd, cd);
                const int i0 = 4 * g;
                const int y = i0 / Lx, x = i0 - y * Lx;
                const double2 ry = reinterpret_cast<const double2*>(v.yph)[y];
                const double rps = ry.x, rpc = ry.y;
                const bool odd_row = (y & v.stag_y & 1) != 0;
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    float w, un, tn;
                    site_update<float, M, F>(v, f[e], u[q][e], th[q][e], n[e], hs, fresh, w, un, tn);
                    const double sv = (double)s4[e], cv = (double)c4[e];
                    const double sxp = (double)(e == 3 ? sR : s4[e + 1]);
                    const double cxp = (double)(e == 3 ? cR : c4[e + 1]);
                    acc[0] += v.Jxd * (cv * cxp + sv * sxp) + v.Jyd * (cv * (double)cd[e] + sv * (double)sd[e]) -
                              v.hd * onsite_cos<float, M>(v, th[q][e], sv, cv);
                    acc[1] += (double)w * (double)w;   // halved below
                    const int xs = x + e;
                    // staggered sign (x is a multiple of 4, the stag flags 0 or 1)
                    const bool neg = ((e & 1) && v.stag_x) != odd_row;
                    const double a = M == kModelSI ? sv : cv, b = M == kModelSI ? cv : sv;
                    const double ec = neg ? -a : a, es = neg ? -b : b;
                    acc[2] += ec;
                    acc[3] += es;
                    const double2 px = reinterpret_cast<const double2*>(v.xph)[xs];
                    const double pxs = px.x, pxc = px.y;
                    acc[4] += ec * pxc;
                    acc[5] -= ec * pxs;
                    acc[6] += es * pxc;
                    acc[7] -= es * pxs;
                    acc[8] += ec * rpc;
                    acc[9] -= ec * rps;
                    acc[10] += es * rpc;
                    acc[11] -= es * rps;
                }
            }
        }
#pragma unroll
        for (int p = 0; p < kNPart; ++p)
#pragma unroll
            for (int off = 32; off >= 1; off >>= 1) acc[p] += __shfl_xor(acc[p], off, kWave);
        if ((tid & (kWave - 1)) == 0)
            for (int p = 0; p < kNPart; ++p) red[tid / kWave][p] = acc[p];
        __syncthreads();
        if (tid == 0) {
            double P[kNPart];
            for (int p = 0; p < kNPart; ++p) {
                P[p] = 0.0;
                for (int w = 0; w < nt / kWave; ++w) P[p] += red[w][p];
            }
            const double Nd = (double)N;
            job.obs[0] = P[0] / Nd;
            job.obs[1] = (0.5 * P[1]) / Nd;
            job.obs[2] = P[2] / Nd;
            job.obs[3] = (P[2] * P[2] + P[3] * P[3]) / Nd;
            job.obs[4] = (P[4] * P[4] + P[5] * P[5] + P[6] * P[6] + P[7] * P[7]) / Nd;
            job.obs[5] = (P[8] * P[8] + P[9] * P[9] + P[10] * P[10] + P[11] * P[11]) / Nd;
        }
    }
    int done = 0;
    for (int t = 0; t < job.nsteps; ++t) {
        const uint64_t k = k0 + (uint64_t)t;
        if (k >= v.k_end) break;
        if (t > 0) {
            tables();
            __syncthreads();
        }
        const float hs = noise_coeff<float, F>(v, k);
        const bool fresh = (k == v.fresh_k);
#pragma unroll
        for (int q = 0; q < kLdsMaxGroups; ++q) {
            const int g = tid + q * nt;
            if (g < ng) {
                float f[4], s4[4], c4[4], sd[4], cd[4], sR, cR, n[4];
                noise4_kick<float>((uint32_t)g, v.replica, k, v.seed_lo, v.seed_hi, hs, n, noise_u2<float, F>(v));
                forces(g, th[q], n, f, s4, c4, sR, cR, sd, cd);
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    float w;
                    site_update<float, M, F>(v, f[e], u[q][e], th[q][e], n[e], hs, fresh, w, u[q][e], th[q][e]);
                }
            }
        }
        ++done;
        __syncthreads();   // every table read of this step precedes the next step's writes
    }
    float* t1 = v.th[(int)((k0 + (uint64_t)done + (uint64_t)v.cur) & 1)];
#pragma unroll
    for (int q = 0; q < kLdsMaxGroups; ++q) {
        const int g = tid + q * nt;
        if (g < ng) {
            store4(t1 + 4 * g, th[q]);
            store4(v.u + 4 * g, u[q]);
        }
    }
}

// One launch takes replicas of one form of the FP32 kick (F: factored, the
// lattice's `fact`); the host launches each form's jobs separately.
template <int M, bool F>
__global__ __launch_bounds__(1024) void k_ensemble_lds(const Lat<float>* __restrict__ reps,
                                                       const LdsJob* __restrict__ jobs, uint64_t j0) {
    extern __shared__ float lds[];
    __shared__ double red[16][kNPart];
    const LdsJob job = jobs[blockIdx.x];
    lds_replica<M, F>(reps[job.rep], job, j0, lds, red);
}

int lds_threads(int N) {
    const int ng = N / 4;
    int t = (ng + kLdsMaxGroups - 1) / kLdsMaxGroups;
    t = (t + kWave - 1) / kWave * kWave;
    return t < kWave ? kWave : t;
}

template <int M, bool F>
static void dispatch_ensemble_lds(const Lat<float>* reps, const void* jobs, int njobs, int threads, size_t lds,
                                  uint64_t j0, hipStream_t s) {
    check_hip(hipFuncSetAttribute(reinterpret_cast<const void*>(k_ensemble_lds<M, F>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds),
              "hipFuncSetAttribute");
    k_ensemble_lds<M, F><<<njobs, threads, lds, s>>>(reps, reinterpret_cast<const LdsJob*>(jobs), j0);
    check_hip(hipGetLastError(), "LDS ensemble kernel launch");
}

void launch_ensemble_lds(const Lat<float>* reps, const void* jobs, int njobs, int threads, int max_sites, int model,
                         bool factored, uint64_t j0, hipStream_t s) {
    const size_t lds = 2 * sizeof(float) * (size_t)max_sites;
    if (model == kModelSI) {
        if (factored) dispatch_ensemble_lds<kModelSI, true>(reps, jobs, njobs, threads, lds, j0, s);
        else dispatch_ensemble_lds<kModelSI, false>(reps, jobs, njobs, threads, lds, j0, s);
    } else {
        if (factored) dispatch_ensemble_lds<kModelXY, true>(reps, jobs, njobs, threads, lds, j0, s);
        else dispatch_ensemble_lds<kModelXY, false>(reps, jobs, njobs, threads, lds, j0, s);
    }
}

// ------------------------------------------------------------------ init
template <typename R>
__global__ void k_init_random(Lat<R> v) {
    const size_t N = (size_t)v.Lx * v.Ly;
    const size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x;   // one Philox block per thread
    if (q * 4 >= N) return;
    const U32x4 r = philox4x32_10((uint32_t)q, v.replica, 0xFFFFFFFFu, 0xFFFFFFFFu, v.seed_lo, v.seed_hi);
    R* th = v.th[(int)((v.k_base + (uint64_t)v.cur) & 1)];
#pragma unroll
    for (int p = 0; p < 4; ++p) {
        const size_t i = q * 4 + p;
        if (i < N) {
            const double uni = ((double)(r.v[p] >> 9) + 0.5) * 0x1p-23;
            // W (2U - 1), W = pi or pi/2 (half-circle rotors of the Si mapping)
            const double W = v.model == kModelSI ? Prec<double>::kPi / 2.0 : Prec<double>::kPi;
            th[i] = (R)(W * (2.0 * uni - 1.0));
            v.u[i] = R(0);
        }
    }
}

template <typename R>
void launch_init_random(const Lat<R>& v, hipStream_t s) {
    const size_t nq = ((size_t)v.Lx * v.Ly + 3) / 4;
    k_init_random<R><<<(unsigned)((nq + 255) / 256), 256, 0, s>>>(v);
    check_hip(hipGetLastError(), "init kernel launch");
}

// ------------------------------------------------------------ test hooks
template <typename R>
__global__ void k_noise(Lat<R> v, uint64_t k, double* out) {
    const size_t N = (size_t)v.Lx * v.Ly;
    const size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q * 4 >= N) return;
    R n[4];
    noise4<R>((uint32_t)q, v.replica, k, v.seed_lo, v.seed_hi, n);
#pragma unroll
    for (int p = 0; p < 4; ++p)
        if (q * 4 + p < N) out[q * 4 + p] = (double)n[p];
}

template <typename R>
void launch_noise(const Lat<R>& v, uint64_t k, double* out, hipStream_t s) {
    const size_t nq = ((size_t)v.Lx * v.Ly + 3) / 4;
    k_noise<R><<<(unsigned)((nq + 255) / 256), 256, 0, s>>>(v, k, out);
    check_hip(hipGetLastError(), "noise kernel launch");
}

// Streaming ceiling for the step's traffic shape: per element read two float
// arrays and write two (16 B), float4 accesses, grid-stride.
__global__ __launch_bounds__(256) void k_stream_probe(const float4* __restrict__ a, const float4* __restrict__ b,
                                                      float4* __restrict__ c, float4* __restrict__ d, size_t n4) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += (size_t)gridDim.x * blockDim.x) {
        float4 x = a[i], y = b[i];
        x.x += 1.f;
        y.x += 1.f;
        c[i] = x;
        d[i] = y;
    }
}

void launch_stream_probe(const void* a, const void* b, void* c, void* d, size_t n4, int grid, hipStream_t s) {
    k_stream_probe<<<grid, 256, 0, s>>>(static_cast<const float4*>(a), static_cast<const float4*>(b),
                                        static_cast<float4*>(c), static_cast<float4*>(d), n4);
    check_hip(hipGetLastError(), "stream probe launch");
}

__global__ void k_philox_blocks(uint64_t seed, const uint32_t* ctr, uint32_t* out, uint64_t n) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const U32x4 r = philox4x32_10(ctr[4 * i], ctr[4 * i + 1], ctr[4 * i + 2], ctr[4 * i + 3], (uint32_t)seed,
                                  (uint32_t)(seed >> 32));
    for (int p = 0; p < 4; ++p) out[4 * i + p] = r.v[p];
}

void launch_philox_blocks(uint64_t seed, const uint32_t* ctr, uint32_t* out, uint64_t n, hipStream_t s) {
    k_philox_blocks<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(seed, ctr, out, n);
    check_hip(hipGetLastError(), "philox kernel launch");
}

// --------------------------------------------------- measurement finalize
// Sums the per-(row, wave chunk) partials in a fixed order (strided per
// thread, then a fixed tree), so a measurement is bit-reproducible for a
// given lattice shape whatever the strip height or workgroup size.
__device__ void finalize_block(const double* part, int nrp, double N, double* out) {
    __shared__ double red[256][kNPart];
    double acc[kNPart];
    for (int p = 0; p < kNPart; ++p) acc[p] = 0.0;
    for (int e = threadIdx.x; e < nrp; e += blockDim.x)
        for (int p = 0; p < kNPart; ++p) acc[p] += part[(size_t)e * kNPart + p];
    for (int p = 0; p < kNPart; ++p) red[threadIdx.x][p] = acc[p];
    __syncthreads();
    for (int w = 128; w >= 1; w >>= 1) {
        if ((int)threadIdx.x < w)
            for (int p = 0; p < kNPart; ++p) red[threadIdx.x][p] += red[threadIdx.x + w][p];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double* P = red[0];
        out[0] = P[0] / N;
        out[1] = (0.5 * P[1]) / N;   // value 1 is the sum of w^2
        out[2] = P[2] / N;
        out[3] = (P[2] * P[2] + P[3] * P[3]) / N;
        out[4] = (P[4] * P[4] + P[5] * P[5] + P[6] * P[6] + P[7] * P[7]) / N;
        out[5] = (P[8] * P[8] + P[9] * P[9] + P[10] * P[10] + P[11] * P[11]) / N;
    }
}

__global__ __launch_bounds__(256) void k_finalize_obs(const double* part, int nrp, double N, double* out) {
    finalize_block(part, nrp, N, out);
}

// First stage for large lattices: block b sums the contiguous range
// [b * chunk, (b + 1) * chunk) of partial rows (same fixed pattern), writing
// one partial row per block.
__global__ __launch_bounds__(256) void k_finalize_stage1(const double* part, int nrp, int chunk, double* out) {
    __shared__ double red[256][kNPart];
    const int b0 = blockIdx.x * chunk;
    const int b1 = min(b0 + chunk, nrp);
    double acc[kNPart];
    for (int p = 0; p < kNPart; ++p) acc[p] = 0.0;
    for (int e = b0 + (int)threadIdx.x; e < b1; e += blockDim.x)
        for (int p = 0; p < kNPart; ++p) acc[p] += part[(size_t)e * kNPart + p];
    for (int p = 0; p < kNPart; ++p) red[threadIdx.x][p] = acc[p];
    __syncthreads();
    for (int w = 128; w >= 1; w >>= 1) {
        if ((int)threadIdx.x < w)
            for (int p = 0; p < kNPart; ++p) red[threadIdx.x][p] += red[threadIdx.x + w][p];
        __syncthreads();
    }
    if (threadIdx.x < kNPart) out[(size_t)blockIdx.x * kNPart + threadIdx.x] = red[0][threadIdx.x];
}

void launch_finalize_obs(const double* part, int nrowparts, double N, double* out, hipStream_t s) {
    if (nrowparts > kFinalizeSplit) {
        // stage-1 output goes after the row partials (the buffer is sized for it)
        const int nb = kFinalizeBlocks;
        const int chunk = (nrowparts + nb - 1) / nb;
        double* tmp = const_cast<double*>(part) + (size_t)nrowparts * kNPart;
        k_finalize_stage1<<<nb, 256, 0, s>>>(part, nrowparts, chunk, tmp);
        check_hip(hipGetLastError(), "finalize stage-1 launch");
        k_finalize_obs<<<1, 256, 0, s>>>(tmp, nb, N, out);
    } else {
        k_finalize_obs<<<1, 256, 0, s>>>(part, nrowparts, N, out);
    }
    check_hip(hipGetLastError(), "finalize kernel launch");
}

// The phases of the lowest Fourier mode of one axis (App. C): sin and cos of
// 2 pi m / L, evaluated once per lattice shape instead of in every
// measurement.
__global__ __launch_bounds__(256) void k_phase_table(double* t, int L) {
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m < L) sincospi(2.0 * (double)m / (double)L, &t[2 * m], &t[2 * m + 1]);
}

void launch_phase_table(double* t, int L, hipStream_t s) {
    k_phase_table<<<(unsigned)((L + 255) / 256), 256, 0, s>>>(t, L);
    check_hip(hipGetLastError(), "phase table launch");
}

__global__ __launch_bounds__(256) void k_finalize_many(const double* part, int nrp, uint64_t stride, double N,
                                                       double* out) {
    finalize_block(part + (size_t)blockIdx.x * stride, nrp, N, out + 6 * (size_t)blockIdx.x);
}

void launch_finalize_many(const double* part, int nrowparts, uint64_t stride, double N, double* out, int count,
                          hipStream_t s) {
    if (count <= 0) return;
    k_finalize_many<<<count, 256, 0, s>>>(part, nrowparts, stride, N, out);
    check_hip(hipGetLastError(), "finalize-many launch");
}

struct FinalizeJob {
    const double* part;
    int nrp;
    double N;
    double* out;
};

__global__ __launch_bounds__(256) void k_finalize_obs_batched(const FinalizeJob* jobs) {
    const FinalizeJob jb = jobs[blockIdx.x];
    if (jb.out == nullptr) return;
    finalize_block(jb.part, jb.nrp, jb.N, jb.out);
}

void launch_finalize_jobs(const void* jobs, int njobs, hipStream_t s) {
    k_finalize_obs_batched<<<njobs, 256, 0, s>>>(reinterpret_cast<const FinalizeJob*>(jobs));
    check_hip(hipGetLastError(), "batched finalize kernel launch");
}

__global__ void k_counter(uint64_t* p, uint64_t add, uint64_t set, int mode) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *p = mode ? set : *p + add;
}

void launch_bump(uint64_t* kdev, uint64_t by, hipStream_t s) {
    k_counter<<<1, 64, 0, s>>>(kdev, by, 0, 0);
    check_hip(hipGetLastError(), "counter kernel launch");
}

void launch_set_counter(uint64_t* kdev, uint64_t value, hipStream_t s) {
    k_counter<<<1, 64, 0, s>>>(kdev, 0, value, 1);
    check_hip(hipGetLastError(), "counter kernel launch");
}

template void launch_step<float>(const Lat<float>&, int, const Launch&, const uint64_t*, uint64_t, hipStream_t);
template void launch_step<double>(const Lat<double>&, int, const Launch&, const uint64_t*, uint64_t, hipStream_t);
template void launch_ensemble_step<float>(const Lat<float>*, const Task*, int, int, int, int, int, const uint64_t*,
                                          uint64_t, hipStream_t);
template void launch_ensemble_step<double>(const Lat<double>*, const Task*, int, int, int, int, int, const uint64_t*,
                                           uint64_t, hipStream_t);
template void launch_init_random<float>(const Lat<float>&, hipStream_t);
template void launch_init_random<double>(const Lat<double>&, hipStream_t);
template void launch_noise<float>(const Lat<float>&, uint64_t, double*, hipStream_t);
template void launch_noise<double>(const Lat<double>&, uint64_t, double*, hipStream_t);

}  // namespace xyl
