// Internal declarations shared by the host runtime and the HIP kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include <stdexcept>
#include <string>

#include "xyl_error.hpp"

namespace xyl {

constexpr int kWave = 64;                  // CDNA wavefront width
constexpr int kLaneSites = 4;              // sites per lane = sites per Philox block
constexpr int kWaveSites = kWave * kLaneSites;
constexpr int kMaxKnots = 16;
constexpr int kNPart = 12;                 // measurement partial sums per (row, wave chunk)
constexpr uint64_t kInitStep = ~(uint64_t)0;  // reserved step counter of the init stream

// Piecewise schedule: segment j runs from knot j to knot j+1 with the shape
// g[j] (0 or 1: linear; g > 1: f^g; g < 0: 1 - (1 - f)^|g|).
struct Schedule {
    int32_t n;
    uint64_t step[kMaxKnots];
    double T[kMaxKnots];
    int32_t g[kMaxKnots];
};

// Everything a step kernel needs to know about one lattice (or one replica of
// an ensemble).  Buffers: two angle buffers (ping-pong) and one velocity
// buffer updated in place.
template <typename R>
struct Lat {
    R* th[2];
    R* u;
    int32_t cur;           // index of the angle buffer holding th^k at the view's base step
    int32_t Lx, Ly;
    int32_t nxw;           // wave chunks per row: ceil(Lx / 256)
    int32_t stag_x, stag_y;
    int32_t model;         // kModelXY or kModelSI (selects the kernel instance)
    // state-precision coefficients: force couplings q Jx, q Jy; 4h (XY field
    // force); p h and the field's angular factor (SI: p / 2pi revolutions in
    // FP32, p in FP64)
    R Jx, Jy, h4, ph, pf, a, c, hdt, dt;
    R kJx, kJy, kh4, kph;  // FP32 kick: hdt q Jx, hdt q Jy, hdt 4h, hdt p h
    R ac;                  // FP32 kick: a c, rounded once from FP64
    // FP32 kick factored by the x coupling (fact = 1; see site_force): the
    // ratios Jy/Jx, 4h/(q Jx) and p h/(q Jx), and c1 = hdt q Jx (1 + a c)
    int32_t fact;
    R fr, fh, fph, fc1;
    R fu2;                 // the draws' angle constant: negates them when hdt q Jx < 0
    double fnoise;         // 1 / (hdt q Jx)^2, the draws' extra scale
    double Jxd, Jyd, hd, pd;       // FP64 copies for the energy
    double gamma, dtd;             // FP64 for the noise amplitude
    Schedule sched;
    uint32_t seed_lo, seed_hi, replica;
    uint64_t k_base;       // step index at launch-step 0
    uint64_t fresh_k;      // step at which u holds w^k itself
    uint64_t k_end;        // steps while k < k_end; may be measured at k_end
    double* part;          // measurement partials [Ly][nxw][kNPart] (+ stage-1 room)
    // phases of the structure-factor modes: sin and cos of 2 pi m / Lx at
    // [2m], [2m + 1] (m < Lx), and of 2 pi m / Ly (m < Ly)
    const double* xph;
    const double* yph;
    R* omega_out;          // destination of w^k (omega mode)
    int32_t pingpong;      // 1: th[(k+cur)&1] -> th[(k+cur+1)&1]; 0: th[0] -> th[1]
    R* u_out;              // velocities written here instead of in place (or NULL)
    uint64_t part_k0;      // with part_stride > 0, step k writes its partials at
    uint64_t part_stride;  //   part + (k - part_k0) * part_stride
};

// Measurements of lattices with more than kFinalizeSplit partial rows are
// reduced in two stages (kFinalizeBlocks blocks, then one).
constexpr int kFinalizeSplit = 4096;
constexpr int kFinalizeBlocks = 256;
inline size_t part_elems(int nrowparts) {
    return ((size_t)nrowparts + (size_t)kFinalizeBlocks) * kNPart;
}

// Step-kernel modes (bit flags).
enum : int { kStore = 1, kMeasure = 2, kOmega = 4 };

// Models: the XY lattice with a two-fold field (q = 1, p = 2, angles in
// [-pi, pi)) and the Si(001) mapping (q = 2, real p, angles in [-pi/2, pi/2)).
enum : int { kModelXY = 0, kModelSI = 1 };

struct Launch {
    int rows = 16;     // rows per strip
    int wpb = 4;       // waves per workgroup
};

// One wave's work item inside a batched launch.
struct Task {
    int32_t rep, xw, strip, pad;
};

// One workgroup of a batched two-step pass: rows [y0, y1) of replica rep,
// swept top-down (dir = +1) or bottom-up (-1).
struct Task2 {
    int32_t rep, y0, y1, dir;
};

// Widths the two-step pass takes: up to 4096 sites (16 waves of 256), at
// least three quarters of the waves' lanes in use (lanes past the row's end
// idle), and at least two lanes in the last wave, whose first and last lanes
// take the row's two outer neighbours.
// A width wider than one workgroup's 16 waves is split into the fewest column
// tiles ntx of w columns (the last takes the rest), each workgroup covering
// its tile and one quad on each side (w + 8 sites, at most max_waves waves).
// A width that fits one workgroup is split as well when max_waves is below
// its waves (at least two tiles).  No tile may leave a single lane in its
// last wave.  Returns false if the width needs no tiles or none fit.
// Narrower tiles trade lanes left idle in a partial last wave, and the halo
// quads, for more workgroups per CU (each holds a 32 (w + 8) B LDS ring, and
// a barrier holds fewer waves); the kernel instance is chosen by the tile's
// waves (step2_tile_bound).
// Rows of sine/cosine in the two-step pass's LDS ring (8 B per site per row).
constexpr int kStep2Slots = 4;

struct Step2Tiles {
    int ntx = 0, w = 0;
};
inline bool step2_tiles(int Lx, Step2Tiles* t, int max_waves = 16) {
    if (Lx % 4 != 0 || max_waves < 2 || max_waves > 16) return false;
    if (Lx <= max_waves * kWaveSites && Lx <= 16 * kWaveSites) return false;
    const int kMax = max_waves * kWaveSites;
    auto lanes_ok = [](int W) { return W % kWaveSites == 0 || W % kWaveSites >= 2 * kLaneSites; };
    for (int ntx = std::max(2, (Lx + kMax - 9) / (kMax - 8)); ntx <= 64; ++ntx) {
        const int w = ((Lx + ntx - 1) / ntx + 3) / 4 * 4;
        const int wl = Lx - (ntx - 1) * w;
        if (w + 8 <= kMax && wl >= 4 && lanes_ok(w + 8) && lanes_ok(wl + 8)) {
            t->ntx = ntx;
            t->w = w;
            return true;
        }
    }
    return false;
}
// Waves of the kernel instance that runs tiles of `waves` waves: 4 and 8 (at
// most 128 VGPRs, so that 4 and 2 workgroups share a CU), 11 (one workgroup
// per CU with room for more registers) and 16.
inline int step2_tile_bound(int waves) { return waves <= 4 ? 4 : waves <= 8 ? 8 : waves <= 11 ? 11 : 16; }

inline bool step2_width_ok(int Lx) {
    if (Lx % 4 != 0 || Lx > 16 * kWaveSites) return false;
    const int waves = (Lx + kWaveSites - 1) / kWaveSites;
    const int last = Lx - (waves - 1) * kWaveSites;   // sites in the last wave
    return last >= 2 * kLaneSites && 4 * Lx >= 3 * waves * kWaveSites;
}

// ------------------------------------------------------------- launchers
template <typename R>
void launch_step(const Lat<R>& v, int mode, const Launch& l, const uint64_t* kdev, uint64_t j,
                 hipStream_t s);
template <typename R>
void launch_ensemble_step(const Lat<R>* reps, const Task* tasks, int ntasks, int mode, int model, int rows, int wpb,
                          const uint64_t* kdev, uint64_t j, hipStream_t s);
// Two steps per pass (FP32; Lx up to 4096 with step2_width_ok, Ly >= 4): angles
// and velocities at step k are read from th_in / u_in and those at k+2
// written to th_out / u_out (distinct buffers); k = v.k_base + j (+ *kdev).
// Widths above 4096 run as column tiles (step2_tiles) of at most tile_waves
// waves (0: 16, the fewest tiles; a value no tiling fits falls back to 16);
// rows per strip as given.
void launch_step2(const Lat<float>& v, const float* th_in, const float* u_in, float* th_out, float* u_out, int rows,
                  const uint64_t* kdev, uint64_t j, hipStream_t s, int tile_waves = 0);
// The same for XY lattices whose rows one workgroup takes whole, also storing
// the state after the first of the two steps into (th_mid, u_mid).
void launch_step2_mid(const Lat<float>& v, const float* th_in, const float* u_in, float* th_mid, float* u_mid,
                      float* th_out, float* u_out, int rows, const uint64_t* kdev, uint64_t j, hipStream_t s);
// Two steps per pass of many FP32 replicas (reps: the table of their views,
// k = k_base + j (+ *kdev)): one workgroup per task, every task's replica
// spanning `waves` waves (partial: some width not a multiple of 256), max_lx
// the widest.  phase 0 reads th[k & 1] and u and writes the other angle
// buffer and the velocities' place in u2_base; phase 1 the reverse.
void launch_ensemble_step2(const Lat<float>* reps, const Task2* tasks, int ntasks, int waves, bool partial,
                           int max_lx, int model, int phase, const float* u_base, float* u2_base,
                           const uint64_t* kdev, uint64_t j, hipStream_t s);
template <typename R>
void launch_init_random(const Lat<R>& v, hipStream_t s);
template <typename R>
void launch_noise(const Lat<R>& v, uint64_t k, double* out, hipStream_t s);
void launch_finalize_obs(const double* part, int nrowparts, double N, double* out, hipStream_t s);
// sin and cos of 2 pi m / L into t[2m], t[2m + 1] for m < L
void launch_phase_table(double* t, int L, hipStream_t s);
// count measurements whose partials lie stride apart: out[6 j ...] for j < count
void launch_finalize_many(const double* part, int nrowparts, uint64_t stride, double N, double* out, int count,
                          hipStream_t s);
void launch_set_counter(uint64_t* kdev, uint64_t value, hipStream_t s);
void launch_bump(uint64_t* kdev, uint64_t by, hipStream_t s);
void launch_stream_probe(const void* a, const void* b, void* c, void* d, size_t n4, int grid, hipStream_t s);
void launch_philox_blocks(uint64_t seed, const uint32_t* ctr, uint32_t* out, uint64_t n, hipStream_t s);
// C_delta(r), r = 0..rmax: part holds correlation_scratch() doubles
template <typename R>
void launch_correlation(const R* th, int Lx, int Ly, int sx, int sy, int model, int axis, int rmax, double* part,
                        double* out, hipStream_t s);
// S_delta(k), k = 0..kmax: zbuf holds 16 (Lx Ly + L) bytes, part nlines * (kmax + 1) doubles
template <typename R>
void launch_structure_factor(const R* th, int Lx, int Ly, int sx, int sy, int model, int axis, int kmax, void* zbuf,
                             double* part, double* out, hipStream_t s);
template <typename R>
void launch_domains(const R* th, int Lx, int Ly, int sx, int sy, int model, int32_t* parent, uint32_t* size,
                    uint32_t* hist, uint32_t* stats, hipStream_t s);

// Slots of parameter adjoints the reverse kernels use (rows per strip of
// the single and of the two-step reverse pass).
template <typename R>
int adjoint_tasks(const Lat<R>& v, int rows, int rows2);
// LDS of the two-step reverse pass with strips of `rows` rows: rows + 4 and
// rows + 2 rows of (sin, cos, lF) per site, and the draws of 2 rows + 2.
template <typename R>
constexpr size_t adjoint2_lds(int Lx, int rows) {
    return sizeof(R) * (3 * (size_t)(2 * rows + 6) + (size_t)(2 * rows + 2)) * (size_t)Lx;
}
// Whether the two-step reverse pass takes this lattice with strips of `rows`
// rows (1, 2 or 4; rows up to 1024 sites, Ly >= 4, its LDS within a CU's).
template <typename R>
bool adjoint2_fits(const Lat<R>& v, int rows);
// Reverse steps k+1 and k in one pass (k = koff + *kdev): th0, u0 the state at
// k, th1, u1 at k+1, (lt_in, lu_in) the adjoint at k+2, (lt_out, lu_out) at k.
template <typename R>
void launch_adjoint_step2(const Lat<R>& v, const R* th0, const R* u0, const R* th1, const R* u1, const R* lt_in,
                          const R* lu_in, R* lt_out, R* lu_out, const double* cm, uint64_t cm_base, double* gacc,
                          const uint64_t* kdev, uint64_t koff, int rows, hipStream_t s);
template <typename R>
void launch_adjoint_step(const Lat<R>& v, const R* th, const R* u, const R* lt_in, const R* lu_in, R* lt_out,
                         R* lu_out, const double* cm, uint64_t cm_base, double* gacc, const uint64_t* kdev,
                         uint64_t koff, const Launch& l, hipStream_t s);
template <typename R>
void launch_adjoint_seed(const Lat<R>& v, const R* th, R* lt, R* lu, double cmN, hipStream_t s);

// Whole-replica-in-LDS stepping of small FP32 replicas.
constexpr int kLdsMaxGroups = 4;      // Philox blocks (4 sites) per thread
constexpr int kLdsMaxSites = 16384;   // 128 x 128: 128 KB of sine/cosine tables
struct LdsJobHost {
    int32_t rep, measure, nsteps, pad;
    double* obs;
};
int lds_threads(int N);
// Every job of one launch is a replica whose `fact` equals `factored`.
void launch_ensemble_lds(const Lat<float>* reps, const void* jobs, int njobs, int threads, int max_sites, int model,
                         bool factored, uint64_t j0, hipStream_t s);

// State transfer between caller device buffers and a lattice (xyl_state.hip).
// launch_check_state ORs kStateBad* bits into *flag (which must start at 0)
// for offending elements of a caller's (theta, omega); launch_convert writes
// out[i] = in[i] (or in[i] * scale in FP64) rounded to the output precision;
// launch_fill_u32 sets n words (a kernel, so it may be captured in a graph).
enum : uint32_t { kStateBadTheta = 1u, kStateBadOmega = 2u, kStateBadHalfCircle = 4u };
void launch_check_state(const void* th, const void* om, int src_f64, size_t n, int half_circle, int state_f64,
                        uint32_t* flag, hipStream_t s);
void launch_convert(const void* in, int in_f64, void* out, int out_f64, size_t n, double scale, bool scaled,
                    hipStream_t s);
void launch_fill_u32(uint32_t* p, size_t n, uint32_t v, hipStream_t s);

void check_hip(hipError_t e, const char* what);

}  // namespace xyl
