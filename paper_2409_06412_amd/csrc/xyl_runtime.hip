// Host runtime behind the C-ABI of include/xyl.h.  Its sections, in order:
//   * devices, buffers (device memory and pinned host memory), parameters and
//     their validation, the launch rules;
//   * the lattice: creation (with its measurement phase tables), stepping
//     through captured graphs and two-step passes, sampled runs, observables,
//     correlation, structure factor, domains (and the allocation-free call),
//     the autotuner;
//   * the ensemble: replica tables, two-step classes on their own streams
//     (issued pass by pass), whole-in-LDS replicas on a side stream, chunk
//     graphs, samples through a finalize-job arena, its autotuner;
//   * the adjoint: the checkpointed forward run and the reverse sweep with
//     its recompute on a side stream.
// The host-only estimators (Binder cumulant, errors, fits) are in
// xyl_host.cpp.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <tuple>
#include <type_traits>
#include <vector>

#include "../../include/xyl.h"
#include "xyl_device.hpp"
#include "xyl_domains.hpp"
#include "xyl_internal.hpp"
#include "xyl_obs.hpp"

namespace xyl {

void launch_finalize_jobs(const void* jobs, int njobs, hipStream_t s);

struct FinalizeJobHost {
    const double* part;
    int nrp;
    double N;
    double* out;
};

void check_hip(hipError_t e, const char* what) {
    if (e != hipSuccess) throw Error(XYL_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

static void check_alloc(hipError_t e, const char* what) {
    if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation)
        throw Error(XYL_ENOMEM, std::string(what) + ": out of device memory");
    check_hip(e, what);
}

// ------------------------------------------------------------- devices
static bool is_gfx950(int dev) {
    hipDeviceProp_t p;
    if (hipGetDeviceProperties(&p, dev) != hipSuccess) return false;
    return std::strncmp(p.gcnArchName, "gfx950", 6) == 0;
}

static void select_device(int dev) {
    int n = 0;
    check_hip(hipGetDeviceCount(&n), "hipGetDeviceCount");
    require(dev >= 0 && dev < n, XYL_EINVAL, "device index out of range");
    require(is_gfx950(dev), XYL_EDEVICE, "device is not gfx950 (MI355X)");
    check_hip(hipSetDevice(dev), "hipSetDevice");
}

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev) {
        (void)hipGetDevice(&prev);
        check_hip(hipSetDevice(dev), "hipSetDevice");
    }
    ~DeviceGuard() {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

template <typename T>
struct DevBuf {
    T* p = nullptr;
    size_t n = 0;
    // owns its allocation: movable, not copyable
    DevBuf() = default;
    DevBuf(const DevBuf&) = delete;
    DevBuf& operator=(const DevBuf&) = delete;
    DevBuf(DevBuf&& o) noexcept : p(o.p), n(o.n) {
        o.p = nullptr;
        o.n = 0;
    }
    DevBuf& operator=(DevBuf&& o) noexcept {
        if (this != &o) {
            release();
            p = o.p;
            n = o.n;
            o.p = nullptr;
            o.n = 0;
        }
        return *this;
    }
    void reserve(size_t count) {
        if (count <= n && p) return;
        if (p) (void)hipFree(p);
        p = nullptr;
        n = 0;
        check_alloc(hipMalloc(reinterpret_cast<void**>(&p), sizeof(T) * std::max<size_t>(count, 1)), "hipMalloc");
        n = count;
    }
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        n = 0;
    }
    ~DevBuf() { release(); }
};

// Page-locked host memory (hipHostMalloc): device-to-host copies of samples
// land here directly instead of through the runtime's staging of pageable
// memory, then go to the caller's array with a plain memcpy.
template <typename T>
struct PinnedBuf {
    T* p = nullptr;
    size_t n = 0;
    PinnedBuf() = default;
    PinnedBuf(const PinnedBuf&) = delete;
    PinnedBuf& operator=(const PinnedBuf&) = delete;
    void reserve(size_t count) {
        if (count <= n && p) return;
        release();
        check_alloc(hipHostMalloc(reinterpret_cast<void**>(&p), sizeof(T) * std::max<size_t>(count, 1),
                                  hipHostMallocDefault),
                    "hipHostMalloc");
        n = count;
    }
    void release() {
        if (p) (void)hipHostFree(p);
        p = nullptr;
        n = 0;
    }
    ~PinnedBuf() { release(); }
};

// ------------------------------------------------------------ parameters
struct Params {
    double Jx = 1.0, Jy = -0.1, h = 0.5, gamma = 1.0, dt = 0.01;
    int model = kModelXY;   // XYL_MODEL_XY / XYL_MODEL_SI
    double p = 2.0;         // field order
};

static void validate_model(int model, double p) {
    require(model == XYL_MODEL_XY || model == XYL_MODEL_SI, XYL_EINVAL, "model must be XYL_MODEL_XY or XYL_MODEL_SI");
    if (model == XYL_MODEL_XY) require(p == 2.0, XYL_EINVAL, "the XY model has p = 2");
    else require(std::isfinite(p) && p > 0.0 && p <= 16.0, XYL_EINVAL, "p must be in (0, 16]");
}

static void validate_params(const Params& p) {
    require(std::isfinite(p.Jx) && std::isfinite(p.Jy) && std::isfinite(p.h) && std::isfinite(p.gamma) &&
                std::isfinite(p.dt),
            XYL_EINVAL, "parameters must be finite");
    require(p.dt > 0.0, XYL_EINVAL, "dt must be > 0");
    require(p.gamma >= 0.0, XYL_EINVAL, "gamma must be >= 0");
}

static Schedule make_schedule(const uint64_t* ks, const double* Ts, int32_t n, const int32_t* gs = nullptr) {
    require(n >= 1 && n <= kMaxKnots, XYL_EINVAL, "schedule needs 1..16 knots");
    require(ks != nullptr && Ts != nullptr, XYL_EINVAL, "schedule arrays are NULL");
    Schedule s{};
    s.n = n;
    for (int j = 0; j < n; ++j) {
        require(std::isfinite(Ts[j]) && Ts[j] >= 0.0, XYL_EINVAL, "schedule temperatures must be finite and >= 0");
        if (j > 0) require(ks[j] > ks[j - 1], XYL_EINVAL, "schedule steps must be strictly increasing");
        s.step[j] = ks[j];
        s.T[j] = Ts[j];
        const int g = gs ? gs[j] : 1;
        require(g >= -16 && g <= 16, XYL_EINVAL, "schedule shape exponents must lie in [-16, 16]");
        s.g[j] = g == 0 ? 1 : g;
    }
    return s;
}

// Whether the FP32 kick may be factored by the x coupling: it divides by
// hdt q Jx, so that and the ratios it creates must stay well inside binary32's
// range.  The two-step passes need it (their kernels are compiled for that
// form only); other lattices keep the unfactored kick in every kernel.
static bool kick_factored(const Params& p) {
    if (p.Jx == 0.0) return false;
    const double q = p.model == kModelSI ? 2.0 : 1.0;
    const double kjx = 0.5 * p.dt * q * p.Jx, big = 1048576.0;
    return std::fabs(p.Jy / p.Jx) <= big && std::fabs(4.0 * p.h / (q * p.Jx)) <= big &&
           std::fabs(p.p * p.h / (q * p.Jx)) <= big && std::fabs(kjx) >= 1e-12 && std::fabs(kjx) <= big;
}

template <typename R>
static void fill_lat(Lat<R>& v, int Lx, int Ly, const Params& p, const Schedule& s, uint64_t seed, uint32_t replica) {
    v.Lx = Lx;
    v.Ly = Ly;
    v.nxw = (Lx + kWaveSites - 1) / kWaveSites;
    v.stag_x = p.Jx > 0.0 ? 1 : 0;
    v.stag_y = p.Jy > 0.0 ? 1 : 0;
    v.model = p.model;
    const double q = p.model == kModelSI ? 2.0 : 1.0;
    v.Jx = (R)(q * p.Jx);
    v.Jy = (R)(q * p.Jy);
    v.h4 = (R)(4.0 * p.h);
    v.ph = (R)(p.p * p.h);
    // FP32 native sine takes revolutions: sin(p t) = sin_rev(t * p / 2pi)
    v.pf = sizeof(R) == 4 ? (R)(p.p / (2.0 * M_PI)) : (R)p.p;
    v.pd = p.p;
    v.a = (R)(1.0 - 0.5 * p.gamma * p.dt);
    v.c = (R)(1.0 / (1.0 + 0.5 * p.gamma * p.dt));
    const double acd = (1.0 - 0.5 * p.gamma * p.dt) / (1.0 + 0.5 * p.gamma * p.dt);
    v.ac = (R)acd;
    // the FP32 kick factored by the x coupling (site_force)
    v.fact = (sizeof(R) == 4 && kick_factored(p)) ? 1 : 0;
    const double kjx = 0.5 * p.dt * q * p.Jx;
    v.fr = v.fact ? (R)(p.Jy / p.Jx) : R(0);
    v.fh = v.fact ? (R)(4.0 * p.h / (q * p.Jx)) : R(0);
    v.fph = v.fact ? (R)(p.p * p.h / (q * p.Jx)) : R(0);
    v.fc1 = (R)(kjx * (1.0 + acd));
    v.fnoise = v.fact ? 1.0 / (kjx * kjx) : 1.0;
    // the draws divided by hdt q Jx: their scale goes through the Box-Muller
    // square root, so a negative divisor flips the angle by half a turn
    v.fu2 = (R)(v.fact && kjx < 0.0 ? 0.5 - 0x1p-24 : 1.0 - 0x1p-24);
    v.hdt = (R)(0.5 * p.dt);
    v.dt = (R)p.dt;
    v.kJx = (R)(0.5 * p.dt * q * p.Jx);
    v.kJy = (R)(0.5 * p.dt * q * p.Jy);
    v.kh4 = (R)(0.5 * p.dt * 4.0 * p.h);
    v.kph = (R)(0.5 * p.dt * p.p * p.h);
    v.Jxd = p.Jx;
    v.Jyd = p.Jy;
    v.hd = p.h;
    v.gamma = p.gamma;
    v.dtd = p.dt;
    v.sched = s;
    v.seed_lo = (uint32_t)seed;
    v.seed_hi = (uint32_t)(seed >> 32);
    v.replica = replica;
}

static void validate_shape(int Lx, int Ly) {
    require(Lx >= 2 && Ly >= 2, XYL_EINVAL, "Lx and Ly must be >= 2");
    require((double)Lx * (double)Ly < 17179869184.0, XYL_EINVAL, "Lx*Ly must be < 2^34");
    require(Lx % 4 == 0, XYL_EUNSUPPORTED, "Lx must be a multiple of 4 (one Philox block per 4 sites of a row)");
    require((double)Lx * (double)Ly < 2147483647.0, XYL_EUNSUPPORTED, "Lx*Ly must fit int32 labels");
}

static size_t elem_size(int dtype) { return dtype == XYL_F64 ? sizeof(double) : sizeof(float); }

// -------------------------------------------------------- launch tuning
static std::mutex g_tune_mu;
static std::map<std::tuple<int, int, int>, Launch> g_tuned;
// steps per pass, rows per strip and waves per column tile of the two-step
// pass, chosen by xyl_autotune
struct Tuned2 {
    int fusion, rows, tile_waves;
};
static std::map<std::tuple<int, int, int>, Tuned2> g_tuned2;
// launch shape of measurements without a step, chosen by xyl_autotune
static std::map<std::tuple<int, int, int>, Launch> g_tunedm;

// Launch shape before any autotuning: enough waves to occupy every SIMD of
// the 256 CUs (strips of up to 16 rows while there are >= 4096 wave-rows,
// down to single-row strips and one-wave workgroups for small lattices).
static Launch default_launch(int Lx, int Ly) {
    const long wave_rows = (long)Ly * ((Lx + kWaveSites - 1) / kWaveSites);
    Launch l;
    l.rows = (int)std::max<long>(1, std::min<long>(16, wave_rows / 4096));
    const long waves = wave_rows / l.rows;
    l.wpb = waves >= 8192 ? 4 : (waves >= 2048 ? 2 : 1);
    return l;
}

static void validate_launch(const Launch& l) {
    require(l.rows >= 1, XYL_EINVAL, "rows per strip must be >= 1");
    require(l.wpb == 1 || l.wpb == 2 || l.wpb == 4 || l.wpb == 8, XYL_EINVAL, "waves per block must be 1, 2, 4 or 8");
}


}  // namespace xyl

using namespace xyl;

// ===================================================================== lattice
struct xyl_lattice {
    int dtype = XYL_F32;
    int device = 0;
    int Lx = 0, Ly = 0;
    size_t N = 0;
    bool owns = true;
    void* th[2] = {nullptr, nullptr};
    void* u = nullptr;
    int cur = 0;                  // th^k lives in th[(k + cur) & 1]
    hipStream_t stream = nullptr;
    hipStream_t cap_stream = nullptr;
    Params p;
    Schedule sched{};
    uint64_t seed = 0;
    uint32_t replica = 0;
    uint64_t k = 0;
    uint64_t fresh_k = 0;
    bool initialized = false;
    Launch launch;
    // launch shape of measurements without a step (xyl_autotune's choice;
    // otherwise the stepping shape)
    Launch mlaunch;
    bool mlaunch_tuned = false;
    int graph_steps = 32;
    // captured step sequences, keyed by what their kernel arguments bake in
    struct GraphEntry {
        int mode = 0, S = 0;
        double* part = nullptr;
        uint64_t part_k0 = 0, part_stride = 0;
        uint64_t version = 0;
        hipGraphExec_t exec = nullptr;
    };
    std::vector<GraphEntry> graphs;
    uint64_t version = 0;
    bool counter_valid = false;
    int fusion = 2;                // steps per pass of plain FP32 stepping where the shape allows (1 or 2)
    int cus = 256;                 // compute units of the device
    int step2_rows_tuned = 0;      // rows per strip of the two-step pass from xyl_autotune (0: the size rule)
    int step2_tw_tuned = 0;        // most waves per column tile (widths above 4096) from xyl_autotune (0: the rule)
    int adj2_rows = 0;             // rows per strip of the two-step reverse pass (0: the rule)
    int adj_fusion = 2;            // reverse steps per pass of the adjoint sweep (1 or 2)
    DevBuf<char> u2;               // second velocity buffer of the two-step passes
    // device scratch
    DevBuf<uint64_t> kdev;
    DevBuf<double> part;
    DevBuf<double> obs;
    PinnedBuf<double> obs_host;   // host landing place of the samples' copy
    DevBuf<double> dscratch;
    DevBuf<char> omega_buf;
    DevBuf<int32_t> parent;
    DevBuf<uint32_t> usz;
    DevBuf<uint32_t> hist;
    DevBuf<uint32_t> stats;
    DevBuf<uint32_t> flag;        // validation result of xyl_set_state_device
    DevBuf<double> phases;        // measurement phases: the x table (2 Lx), then the y table (2 Ly)
    // adjoint state (see xyl_adjoint.hip)
    void* adj = nullptr;

    template <typename R>
    Lat<R> view() {
        Lat<R> v{};
        v.th[0] = static_cast<R*>(th[0]);
        v.th[1] = static_cast<R*>(th[1]);
        v.u = static_cast<R*>(u);
        v.cur = cur;
        fill_lat(v, Lx, Ly, p, sched, seed, replica);
        v.k_base = 0;
        v.fresh_k = fresh_k;
        v.k_end = ~(uint64_t)0;
        v.part = part.p;
        v.xph = phases.p;
        v.yph = phases.p + 2 * (size_t)Lx;
        v.omega_out = reinterpret_cast<R*>(omega_buf.p);
        v.pingpong = 1;
        v.u_out = nullptr;
        v.part_k0 = 0;
        v.part_stride = 0;
        return v;
    }
    void* cur_theta() { return th[(int)((k + (uint64_t)cur) & 1)]; }
    int nrowparts() const { return Ly * ((Lx + kWaveSites - 1) / kWaveSites); }
    void touch() { ++version; }
};

// State of a pathwise-gradient run between xyl_adjoint_forward and
// xyl_adjoint_backward: checkpoints every K steps, the loss samples and the
// device buffers of the reverse sweep.
struct AdjState {
    bool valid = false;          // a forward run completed and may be differentiated
    uint64_t run = 0;            // identifier of that run (process-wide, never reused)
    uint64_t version = 0;        // the lattice's configuration version when it ended
    uint64_t k0 = 0, N = 0, K = 0, W = 0;
    double loss = 0.0;
    std::vector<double> m;       // m_s at steps k0+N-W+1 .. k0+N
    DevBuf<char> ckpt, seg, lam;
    DevBuf<double> cm, gacc, obs, win;
    DevBuf<uint64_t> kseg;                 // step counters: [0] reverse (main stream), [1] recompute (side)
    // Backward sweep: segment buffers b = 0, 1 (K + 1 states each); the
    // recomputation of the next segment runs on a second stream into one
    // buffer while the reverse steps of the current one read the other.
    hipStream_t side = nullptr;
    hipEvent_t ev_rec[2] = {nullptr, nullptr}, ev_rev[2] = {nullptr, nullptr}, ev_start = nullptr;
    hipGraphExec_t rec_graph[2] = {nullptr, nullptr};        // K recompute steps into buffer b
    hipGraphExec_t rev_graph[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};   // [b][adjoint parity]
    // what the captured graphs bake in; they are rebuilt when it changes
    std::vector<uint64_t> graph_key;
    void drop_graphs() {
        for (auto& g : rec_graph) {
            if (g) (void)hipGraphExecDestroy(g);
            g = nullptr;
        }
        for (auto& r : rev_graph)
            for (auto& g : r) {
                if (g) (void)hipGraphExecDestroy(g);
                g = nullptr;
            }
    }
    ~AdjState() {
        drop_graphs();
        for (int b = 0; b < 2; ++b) {
            if (ev_rec[b]) (void)hipEventDestroy(ev_rec[b]);
            if (ev_rev[b]) (void)hipEventDestroy(ev_rev[b]);
        }
        if (ev_start) (void)hipEventDestroy(ev_start);
        if (side) (void)hipStreamDestroy(side);
    }
};

// Identifiers of adjoint forward runs: a backward call names the run it
// differentiates, and a later forward on the same lattice (which replaces the
// checkpoints) makes earlier identifiers stale.
static std::atomic<uint64_t> g_adj_runs{0};

static void adjoint_release(xyl_lattice* h) {
    delete static_cast<AdjState*>(h->adj);
    h->adj = nullptr;
}

static void destroy_graph(xyl_lattice* h) {
    for (auto& g : h->graphs)
        if (g.exec) (void)hipGraphExecDestroy(g.exec);
    h->graphs.clear();
}

template <typename R>
static void lattice_launch_one(xyl_lattice* h, int mode) {
    Lat<R> v = h->view<R>();
    const Launch& l = (mode == kMeasure && h->mlaunch_tuned) ? h->mlaunch : h->launch;
    launch_step<R>(v, mode, l, nullptr, h->k, h->stream);
}

// Captures S consecutive steps whose step index comes from the device counter
// (node j runs step *kdev + j), followed by a node that advances the counter.
template <typename R>
static hipGraphExec_t capture_steps(xyl_lattice* h, const Lat<R>& v, int mode, int S) {
    hipGraph_t g = nullptr;
    check_hip(hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
    try {
        for (int j = 0; j < S; ++j) launch_step<R>(v, mode, h->launch, h->kdev.p, (uint64_t)j, h->cap_stream);
        launch_bump(h->kdev.p, (uint64_t)S, h->cap_stream);
    } catch (...) {
        (void)hipStreamEndCapture(h->cap_stream, &g);
        if (g) (void)hipGraphDestroy(g);
        throw;
    }
    check_hip(hipStreamEndCapture(h->cap_stream, &g), "hipStreamEndCapture");
    hipGraphExec_t ex = nullptr;
    hipError_t e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    check_hip(e, "hipGraphInstantiate");
    return ex;
}

// Two steps per pass (FP32 plain stepping, width a multiple of 256 up to 4096).
static bool step2_shape(int Lx, int Ly) { return step2_width_ok(Lx) && Ly >= 4; }
// single lattices also take widths above 4096, as column tiles
static bool step2_lattice_shape(int Lx, int Ly) {
    Step2Tiles t;
    return Ly >= 4 && (step2_width_ok(Lx) || step2_tiles(Lx, &t));
}
static bool step2_eligible(const xyl_lattice* h) {
    return h->dtype == XYL_F32 && h->fusion == 2 && kick_factored(h->p) && step2_lattice_shape(h->Lx, h->Ly);
}

// Waves per column tile of the two-step pass when not tuned: rows up to 4096
// sites wide run whole (one workgroup per strip); wider ones as tiles of at
// most 4 waves, four workgroups per CU (8192^2: 9 tiles, 119 against 143 us
// per step with the fewest tiles, 3 of 11 waves; 6144^2, 12288 x 4096 and
// 16384 x 2048 gain 14-18% the same way), where such a tiling exists.
static int step2_tile_waves(int Lx) {
    Step2Tiles t;
    return Lx > 16 * kWaveSites && step2_tiles(Lx, &t, 4) ? 4 : 16;
}
static int step2_tile_waves(const xyl_lattice* h) {
    return h->step2_tw_tuned ? h->step2_tw_tuned : step2_tile_waves(h->Lx);
}

// Rows per strip of the two-step kernel.  A workgroup spans the row (Lx / 256
// waves of up to 128 VGPRs, 32 Lx bytes of LDS), so a CU holds
// per_cu = min(16 / waves, 160 KiB / LDS) of them.  The strip count aims at
// CUs x max(1, per_cu / 2): every CU busy, two or more workgroups per CU where
// they fit, and strips as tall as that allows (each strip recomputes two halo
// rows of the first step), 2 to 16 rows.  Measured best over 512^2 .. 4096^2,
// 4096 x 1024, 1024 x 4096 and 256 x 8192 (strip counts off a multiple of the
// CU count leave a partial last round of workgroups).
static int step2_rows(int Lx, int Ly, int cus, int tile_waves) {
    Step2Tiles t;
    if (step2_tiles(Lx, &t, tile_waves) || step2_tiles(Lx, &t)) {
        // column tiles.  Several workgroups per CU (tiles of at most 8 waves:
        // as many as 16 waves of 128 VGPRs and the 160 KiB of LDS allow):
        // 16-row strips, measured best at 8192^2, 6144^2 and 16384 x 2048
        // with 2- to 4-wave tiles (8-row strips 6-7% slower, 32-row 0-10%).
        const int W = t.w + 2 * kLaneSites;
        const int waves = (W + kWaveSites - 1) / kWaveSites;
        const int per_cu =
            waves > 8 ? 1 : std::max(1, std::min(16 / waves, (160 * 1024) / (int)(sizeof(float) * 2 * kStep2Slots * W)));
        if (per_cu >= 2) return 16;
        // One workgroup per CU: the last round of workgroups matters.  Score =
        // rows / (rows + 1) (the halo rows' share of the work) times the
        // fraction of the last round that is filled; strips of up to 32 rows.
        int best = 32;
        double best_score = -1.0;
        for (int rows = 32; rows >= 2; rows /= 2) {
            const long wgs = (long)((Ly + rows - 1) / rows) * t.ntx;
            const long rounds = (wgs + cus - 1) / cus;
            const double score = (double)rows / (rows + 1) * (double)wgs / (double)(rounds * cus);
            if (score > best_score + 1e-9) {
                best_score = score;
                best = rows;
            }
        }
        return best;
    }
    const int waves = (Lx + kWaveSites - 1) / kWaveSites;
    const int per_cu = std::max(1, std::min(16 / waves, (160 * 1024) / (32 * Lx)));
    const int strips = cus * std::max(1, per_cu / 2);
    return std::max(2, std::min(16, Ly / strips));
}
static int step2_rows(const xyl_lattice* h) {
    return h->step2_rows_tuned ? h->step2_rows_tuned : step2_rows(h->Lx, h->Ly, h->cus, step2_tile_waves(h));
}

// Launches for 4m steps from the current step: pairs of two-step passes,
// (A, u) -> (B, u2) -> (A, u), A the buffer holding the angles at step k, so
// that the state ends where it started.  With kdev the step index comes from
// the device counter (graph capture), else from j.
static void step2_launches(xyl_lattice* h, const Lat<float>& v, uint64_t nsteps, const uint64_t* kdev, uint64_t j,
                           int parity, hipStream_t s) {
    float* A = static_cast<float*>(h->th[parity]);
    float* Bb = static_cast<float*>(h->th[parity ^ 1]);
    float* u = static_cast<float*>(h->u);
    float* u2 = reinterpret_cast<float*>(h->u2.p);
    const int rows = step2_rows(h), tw = step2_tile_waves(h);
    for (uint64_t i = 0; i < nsteps; i += 4) {
        launch_step2(v, A, u, Bb, u2, rows, kdev, j + i, s, tw);
        launch_step2(v, Bb, u2, A, u, rows, kdev, j + i + 2, s, tw);
    }
}

// Captures S (a multiple of 4) steps as two-step passes, then the counter bump.
static hipGraphExec_t capture_steps2(xyl_lattice* h, const Lat<float>& v, int S, int parity) {
    hipGraph_t g = nullptr;
    check_hip(hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
    try {
        step2_launches(h, v, (uint64_t)S, h->kdev.p, 0, parity, h->cap_stream);
        launch_bump(h->kdev.p, (uint64_t)S, h->cap_stream);
    } catch (...) {
        (void)hipStreamEndCapture(h->cap_stream, &g);
        if (g) (void)hipGraphDestroy(g);
        throw;
    }
    check_hip(hipStreamEndCapture(h->cap_stream, &g), "hipStreamEndCapture");
    hipGraphExec_t ex = nullptr;
    hipError_t e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    check_hip(e, "hipGraphInstantiate");
    return ex;
}

// Advances n steps in the given mode.  With part_stride > 0 every step writes
// its measurement partials to part + (k - part_k0) * part_stride.
template <typename R>
static void lattice_steps_mode(xyl_lattice* h, uint64_t n, int mode, double* part, uint64_t part_k0,
                               uint64_t part_stride) {
    if constexpr (sizeof(R) == 4) {
        if (mode == kStore && part_stride == 0 && step2_eligible(h) && n >= 4) {
            h->u2.reserve(sizeof(float) * h->N);
            Lat<float> v2 = h->view<float>();
            v2.k_base = 0;
            const uint64_t n4 = n - n % 4;
            uint64_t done = 0;
            const int S = h->graph_steps - h->graph_steps % 4;
            while (done < n4) {
                const int parity = (int)((h->k + (uint64_t)h->cur) & 1);
                if (S >= 4 && n4 - done >= (uint64_t)S) {
                    const int key = kStore | (2 << 8) | (parity << 10);
                    xyl_lattice::GraphEntry* ge = nullptr;
                    for (auto& g : h->graphs)
                        if (g.mode == key && g.S == S) ge = &g;
                    if (ge && ge->version != h->version) {
                        (void)hipGraphExecDestroy(ge->exec);
                        ge->exec = nullptr;
                    }
                    if (!ge) {
                        if (h->graphs.size() >= 8) destroy_graph(h);
                        h->graphs.push_back(xyl_lattice::GraphEntry());
                        ge = &h->graphs.back();
                        ge->mode = key;
                        ge->S = S;
                    }
                    if (!ge->exec) {
                        ge->exec = capture_steps2(h, v2, S, parity);
                        ge->version = h->version;
                    }
                    if (!h->counter_valid) {
                        launch_set_counter(h->kdev.p, h->k, h->stream);
                        h->counter_valid = true;
                    }
                    check_hip(hipGraphLaunch(ge->exec, h->stream), "hipGraphLaunch");
                    h->k += (uint64_t)S;
                    done += (uint64_t)S;
                } else {
                    const uint64_t m = std::min<uint64_t>(n4 - done, 4);
                    step2_launches(h, v2, m, nullptr, h->k, parity, h->stream);
                    h->k += m;
                    done += m;
                    h->counter_valid = false;
                }
            }
            n -= n4;
        }
    }
    Lat<R> v = h->view<R>();
    if (part_stride) {
        v.part = part;
        v.part_k0 = part_k0;
        v.part_stride = part_stride;
    }
    while (n > 0) {
        const int S = h->graph_steps;
        if (S > 1 && n >= (uint64_t)S) {
            xyl_lattice::GraphEntry* ge = nullptr;
            for (auto& g : h->graphs)
                if (g.mode == mode && g.S == S && g.part == v.part && g.part_k0 == v.part_k0 &&
                    g.part_stride == v.part_stride)
                    ge = &g;
            if (ge && ge->version != h->version) {
                (void)hipGraphExecDestroy(ge->exec);
                ge->exec = nullptr;
            }
            if (!ge) {
                if (h->graphs.size() >= 8) destroy_graph(h);   // bound the cache
                h->graphs.push_back(xyl_lattice::GraphEntry());
                ge = &h->graphs.back();
                ge->mode = mode;
                ge->S = S;
                ge->part = v.part;
                ge->part_k0 = v.part_k0;
                ge->part_stride = v.part_stride;
            }
            if (!ge->exec) {
                ge->exec = capture_steps<R>(h, v, mode, S);
                ge->version = h->version;
            }
            if (!h->counter_valid) {
                launch_set_counter(h->kdev.p, h->k, h->stream);
                h->counter_valid = true;
            }
            check_hip(hipGraphLaunch(ge->exec, h->stream), "hipGraphLaunch");
            h->k += (uint64_t)S;
            n -= (uint64_t)S;
        } else {
            launch_step<R>(v, mode, h->launch, nullptr, h->k, h->stream);
            h->k += 1;
            h->counter_valid = false;
            n -= 1;
        }
    }
}

template <typename R>
static void lattice_steps(xyl_lattice* h, uint64_t n) {
    lattice_steps_mode<R>(h, n, kStore, nullptr, 0, 0);
}

template <typename R>
static void lattice_measure_into(xyl_lattice* h, bool advance, double* obs_dev) {
    lattice_launch_one<R>(h, advance ? (kStore | kMeasure) : kMeasure);
    launch_finalize_obs(h->part.p, h->nrowparts(), (double)h->N, obs_dev, h->stream);
    if (advance) {
        h->k += 1;
        h->counter_valid = false;
    }
}

// Observables of the current step into obs_dev, then `span` >= 1 steps.
// Where two steps per pass apply and the span holds at least one pair of
// passes, the sample is a measurement without a step (the same partial sums as
// a measured step) and every step of the span goes through the two-step
// passes; otherwise the measured step advances one step and the rest follow.
template <typename R>
static void lattice_sample_and_advance(xyl_lattice* h, uint64_t span, double* obs_dev) {
    if (span >= 4 && step2_eligible(h)) {
        lattice_measure_into<R>(h, false, obs_dev);
        lattice_steps<R>(h, span);
        return;
    }
    lattice_measure_into<R>(h, true, obs_dev);
    lattice_steps<R>(h, span - 1);
}

// A blown-up integration (dt far too large, say) shows up as non-finite
// values; calls that bring results to the host report it as XYL_ENUMERIC
// (the copied values are still written).
static void require_finite(const double* x, size_t n, const char* what) {
    for (size_t i = 0; i < n; ++i)
        if (!std::isfinite(x[i])) throw Error(XYL_ENUMERIC, std::string("non-finite ") + what + " (numeric fault)");
}

static void require_init(xyl_lattice* h) {
    require(h != nullptr, XYL_EINVAL, "NULL handle");
    require(h->initialized, XYL_ESTATE, "lattice state not initialised (call an init or set_state first)");
}

template <typename R>
static void to_host(const void* dev, double* host, size_t n, hipStream_t s) {
    std::vector<R> tmp(n);
    check_hip(hipMemcpyAsync(tmp.data(), dev, sizeof(R) * n, hipMemcpyDeviceToHost, s), "hipMemcpyAsync D2H");
    check_hip(hipStreamSynchronize(s), "hipStreamSynchronize");
    for (size_t i = 0; i < n; ++i) host[i] = (double)tmp[i];
}

template <typename R>
static void to_device(void* dev, const double* host, size_t n, hipStream_t s) {
    std::vector<R> tmp(n);
    for (size_t i = 0; i < n; ++i) tmp[i] = (R)host[i];
    check_hip(hipMemcpyAsync(dev, tmp.data(), sizeof(R) * n, hipMemcpyHostToDevice, s), "hipMemcpyAsync H2D");
    check_hip(hipStreamSynchronize(s), "hipStreamSynchronize");
}

template <typename R>
static void lattice_omega(xyl_lattice* h, double* omega) {
    if (h->k == h->fresh_k) {
        to_host<R>(h->u, omega, h->N, h->stream);
        return;
    }
    h->omega_buf.reserve(sizeof(R) * h->N);
    lattice_launch_one<R>(h, kOmega);
    to_host<R>(h->omega_buf.p, omega, h->N, h->stream);
}

template <typename R>
static void run_domains(const R* th, int Lx, int Ly, int sx, int sy, int model, DevBuf<int32_t>& parent,
                        DevBuf<uint32_t>& usz,
                        DevBuf<uint32_t>& hist, DevBuf<uint32_t>& stats, hipStream_t s, int32_t* labels,
                        uint64_t* sizes, uint64_t* counts, uint64_t cap, uint64_t* n_sizes, uint64_t* n_domains,
                        uint64_t* max_size) {
    const size_t N = (size_t)Lx * Ly;
    const uint32_t pcap = domain_size_cap(N);
    const size_t nst = kDomainPairs + 2 * (size_t)pcap;
    parent.reserve(N);
    usz.reserve(N);
    hist.reserve(N + 1);
    stats.reserve(nst);
    check_hip(hipMemsetAsync(hist.p, 0, sizeof(uint32_t) * (N + 1), s), "hipMemsetAsync");
    check_hip(hipMemsetAsync(stats.p, 0, sizeof(uint32_t) * kDomainPairs, s), "hipMemsetAsync");
    launch_domains<R>(th, Lx, Ly, sx, sy, model, parent.p, usz.p, hist.p, stats.p, s);
    // the (size, count) pairs were compacted on the device: only they come back
    std::vector<uint32_t> st(nst);
    check_hip(hipMemcpyAsync(st.data(), stats.p, sizeof(uint32_t) * nst, hipMemcpyDeviceToHost, s), "D2H");
    if (labels) check_hip(hipMemcpyAsync(labels, parent.p, sizeof(int32_t) * N, hipMemcpyDeviceToHost, s), "D2H");
    check_hip(hipStreamSynchronize(s), "hipStreamSynchronize");
    const uint64_t ns = st[0];
    require(ns >= 1 && ns <= pcap, XYL_EDEVICE, "domain size distribution overflowed its bound");
    std::vector<std::pair<uint32_t, uint32_t>> pairs(ns);
    for (uint64_t j = 0; j < ns; ++j) pairs[j] = {st[kDomainPairs + 2 * j], st[kDomainPairs + 2 * j + 1]};
    std::sort(pairs.begin(), pairs.end());
    if (sizes || counts) require(cap >= ns, XYL_EINVAL, "size-distribution capacity too small");
    uint64_t nd = 0, covered = 0;
    for (uint64_t j = 0; j < ns; ++j) {
        if (sizes) sizes[j] = pairs[j].first;
        if (counts) counts[j] = pairs[j].second;
        nd += pairs[j].second;
        covered += (uint64_t)pairs[j].first * pairs[j].second;
    }
    require(covered == N, XYL_EDEVICE, "domain sizes do not cover the lattice");
    if (n_sizes) *n_sizes = ns;
    if (n_domains) *n_domains = nd;
    if (max_size) *max_size = pairs[ns - 1].first;
}


#define DISPATCH(dt, FN, ...) ((dt) == XYL_F64 ? FN<double>(__VA_ARGS__) : FN<float>(__VA_ARGS__))

extern "C" {

int xyl_device_count(void) {
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess) return 0;
    int m = 0;
    for (int d = 0; d < n; ++d)
        if (is_gfx950(d)) ++m;
    return m;
}

static int create_impl(xyl_lattice** out, int32_t Lx, int32_t Ly, int32_t dtype, int32_t device, void* ta, void* tb,
                       void* vel) {
    return guarded([&] {
        require(out != nullptr, XYL_EINVAL, "out is NULL");
        *out = nullptr;
        require(dtype == XYL_F32 || dtype == XYL_F64, XYL_EINVAL, "dtype must be XYL_F32 or XYL_F64");
        validate_shape(Lx, Ly);
        select_device(device);
        std::unique_ptr<xyl_lattice> h(new xyl_lattice());
        h->dtype = dtype;
        h->device = device;
        check_hip(hipDeviceGetAttribute(&h->cus, hipDeviceAttributeMultiprocessorCount, device), "hipDeviceGetAttribute");
        h->Lx = Lx;
        h->Ly = Ly;
        h->N = (size_t)Lx * Ly;
        const uint64_t k0[1] = {0};
        const double T0[1] = {0.0};
        h->sched = make_schedule(k0, T0, 1);
        if (ta) {
            require(tb && vel && ta != tb && ta != vel && tb != vel, XYL_EINVAL, "wrapped buffers must be distinct");
            h->owns = false;
            h->th[0] = ta;
            h->th[1] = tb;
            h->u = vel;
        } else {
            const size_t bytes = elem_size(dtype) * h->N;
            for (int b = 0; b < 2; ++b) check_alloc(hipMalloc(&h->th[b], bytes), "hipMalloc theta");
            check_alloc(hipMalloc(&h->u, bytes), "hipMalloc velocity");
        }
        check_hip(hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking), "hipStreamCreate");
        h->kdev.reserve(1);
        h->part.reserve(part_elems(h->nrowparts()));
        h->phases.reserve(2 * ((size_t)Lx + Ly));
        launch_phase_table(h->phases.p, Lx, nullptr);
        launch_phase_table(h->phases.p + 2 * (size_t)Lx, Ly, nullptr);
        check_hip(hipStreamSynchronize(nullptr), "hipStreamSynchronize");
        h->obs.reserve(16 * 6);
        h->launch = default_launch(Lx, Ly);
        {
            std::lock_guard<std::mutex> lk(g_tune_mu);
            auto it = g_tuned.find({Lx, Ly, dtype});
            if (it != g_tuned.end()) h->launch = it->second;
            auto itm = g_tunedm.find({Lx, Ly, dtype});
            if (itm != g_tunedm.end()) {
                h->mlaunch = itm->second;
                h->mlaunch_tuned = true;
            }
            auto it2 = g_tuned2.find({Lx, Ly, dtype});
            if (it2 != g_tuned2.end()) {
                h->fusion = it2->second.fusion;
                h->step2_rows_tuned = it2->second.rows;
                h->step2_tw_tuned = it2->second.tile_waves;
            }
        }
        *out = h.release();
    });
}

int xyl_create(xyl_lattice** out, int32_t Lx, int32_t Ly, int32_t dtype, int32_t device) {
    return create_impl(out, Lx, Ly, dtype, device, nullptr, nullptr, nullptr);
}

int xyl_create_wrapped(xyl_lattice** out, int32_t Lx, int32_t Ly, int32_t dtype, int32_t device, void* theta_a,
                       void* theta_b, void* vel) {
    if (!theta_a || !theta_b || !vel) {
        g_err = "wrapped buffers must be non-NULL";
        return XYL_EINVAL;
    }
    return create_impl(out, Lx, Ly, dtype, device, theta_a, theta_b, vel);
}

int xyl_destroy(xyl_lattice* h) {
    if (!h) return XYL_OK;
    return guarded([&] {
        DeviceGuard g(h->device);
        (void)hipStreamSynchronize(h->stream);
        destroy_graph(h);
        adjoint_release(h);
        if (h->owns) {
            for (int b = 0; b < 2; ++b)
                if (h->th[b]) (void)hipFree(h->th[b]);
            if (h->u) (void)hipFree(h->u);
        }
        if (h->cap_stream) (void)hipStreamDestroy(h->cap_stream);
        delete h;
    });
}

int xyl_set_stream(xyl_lattice* h, void* stream) {
    return guarded([&] {
        require(h != nullptr, XYL_EINVAL, "NULL handle");
        h->stream = static_cast<hipStream_t>(stream);
    });
}

int xyl_set_params(xyl_lattice* h, double Jx, double Jy, double hf, double gamma, double dt) {
    return guarded([&] {
        require(h != nullptr, XYL_EINVAL, "NULL handle");
        Params p = h->p;
        p.Jx = Jx;
        p.Jy = Jy;
        p.h = hf;
        p.gamma = gamma;
        p.dt = dt;
        validate_params(p);
        h->p = p;
        h->touch();
    });
}

int xyl_set_model(xyl_lattice* h, int32_t model, double pfield) {
    return guarded([&] {
        require(h != nullptr, XYL_EINVAL, "NULL handle");
        validate_model(model, pfield);
        if (model != h->p.model) h->initialized = false;   // the angle ranges differ
        h->p.model = model;
        h->p.p = pfield;
        h->touch();
    });
}

int xyl_set_schedule(xyl_lattice* h, const uint64_t* ks, const double* Ts, int32_t n) {
    return guarded([&] {
        require(h != nullptr, XYL_EINVAL, "NULL handle");
        h->sched = make_schedule(ks, Ts, n);
        h->touch();
    });
}

int xyl_set_schedule_shaped(xyl_lattice* h, const uint64_t* ks, const double* Ts, const int32_t* gs, int32_t n) {
    return guarded([&] {
        require(h != nullptr, XYL_EINVAL, "NULL handle");
        require(gs != nullptr, XYL_EINVAL, "shape array is NULL");
        h->sched = make_schedule(ks, Ts, n, gs);
        h->touch();
    });
}

int xyl_set_seed(xyl_lattice* h, uint64_t seed, uint32_t replica) {
    return guarded([&] {
        require(h != nullptr, XYL_EINVAL, "NULL handle");
        h->seed = seed;
        h->replica = replica;
        h->touch();
    });
}

int xyl_init_random(xyl_lattice* h) {
    return guarded([&] {
        require(h != nullptr, XYL_EINVAL, "NULL handle");
        DeviceGuard g(h->device);
        h->k = 0;
        h->fresh_k = 0;
        h->cur = 0;
        h->counter_valid = false;
        h->touch();
        if (h->dtype == XYL_F64) launch_init_random<double>(h->view<double>(), h->stream);
        else launch_init_random<float>(h->view<float>(), h->stream);
        h->initialized = true;
    });
}

// Host values for the state precision: finite, |th| <= 3 pi, and for the half
// circle inside [-pi_p/2, pi_p/2) after rounding to the state precision.
static void validate_host_state(const xyl_lattice* h, const double* theta, const double* vel, const char* vname) {
    const bool si = h->p.model == kModelSI;
    const double wp = h->dtype == XYL_F64 ? Prec<double>::kHalfPi : (double)Prec<float>::kHalfPi;
    for (size_t i = 0; i < h->N; ++i) {
        require(std::isfinite(theta[i]) && std::fabs(theta[i]) <= 3.0 * M_PI, XYL_EINVAL,
                "theta entries must be finite with |theta| <= 3 pi");
        if (si) {
            const double t = h->dtype == XYL_F64 ? theta[i] : (double)(float)theta[i];
            require(t >= -wp && t < wp, XYL_EINVAL, "theta entries must lie in [-pi/2, pi/2) for the SI model");
        }
        require(std::isfinite(vel[i]), XYL_EINVAL, std::string(vname) + " entries must be finite");
    }
}

int xyl_set_state(xyl_lattice* h, const double* theta, const double* omega, uint64_t step) {
    return guarded([&] {
        require(h != nullptr, XYL_EINVAL, "NULL handle");
        require(theta != nullptr && omega != nullptr, XYL_EINVAL, "theta/omega are NULL");
        // SI: the field is evaluated on the raw angle, so the state must already
        // lie in the half circle [-pi_p/2, pi_p/2) of the state precision
        validate_host_state(h, theta, omega, "omega");
        DeviceGuard g(h->device);
        h->k = step;
        h->fresh_k = step;
        h->counter_valid = false;
        h->touch();
        if (h->dtype == XYL_F64) {
            to_device<double>(h->cur_theta(), theta, h->N, h->stream);
            to_device<double>(h->u, omega, h->N, h->stream);
        } else {
            to_device<float>(h->cur_theta(), theta, h->N, h->stream);
            to_device<float>(h->u, omega, h->N, h->stream);
        }
        h->initialized = true;
    });
}

int xyl_get_raw_state(xyl_lattice* h, double* theta, double* u, uint64_t* step, int32_t* fresh) {
    return guarded([&] {
        require_init(h);
        DeviceGuard g(h->device);
        if (theta) {
            if (h->dtype == XYL_F64) to_host<double>(h->cur_theta(), theta, h->N, h->stream);
            else to_host<float>(h->cur_theta(), theta, h->N, h->stream);
        }
        if (u) {
            if (h->dtype == XYL_F64) to_host<double>(h->u, u, h->N, h->stream);
            else to_host<float>(h->u, u, h->N, h->stream);
        }
        if (step) *step = h->k;
        if (fresh) *fresh = h->k == h->fresh_k ? 1 : 0;
        if (theta) require_finite(theta, h->N, "angles");
        if (u) require_finite(u, h->N, "velocities");
    });
}

int xyl_set_raw_state(xyl_lattice* h, const double* theta, const double* u, uint64_t step, int32_t fresh) {
    return guarded([&] {
        require(h != nullptr, XYL_EINVAL, "NULL handle");
        require(theta != nullptr && u != nullptr, XYL_EINVAL, "theta/u are NULL");
        require(fresh == 0 || fresh == 1, XYL_EINVAL, "fresh must be 0 or 1");
        validate_host_state(h, theta, u, "u");
        DeviceGuard g(h->device);
        h->k = step;
        // a stored half-step velocity is never the synchronized one again
        h->fresh_k = fresh ? step : ~(uint64_t)0;
        h->counter_valid = false;
        h->touch();
        if (h->dtype == XYL_F64) {
            to_device<double>(h->cur_theta(), theta, h->N, h->stream);
            to_device<double>(h->u, u, h->N, h->stream);
        } else {
            to_device<float>(h->cur_theta(), theta, h->N, h->stream);
            to_device<float>(h->u, u, h->N, h->stream);
        }
        h->initialized = true;
    });
}

int xyl_set_state_device(xyl_lattice* h, const void* theta, const void* omega, int32_t dtype, uint64_t step) {
    return guarded([&] {
        require(h != nullptr, XYL_EINVAL, "NULL handle");
        require(theta != nullptr && omega != nullptr, XYL_EINVAL, "theta/omega are NULL");
        require(dtype == XYL_F32 || dtype == XYL_F64, XYL_EINVAL, "dtype must be XYL_F32 or XYL_F64");
        DeviceGuard g(h->device);
        const int src64 = dtype == XYL_F64 ? 1 : 0, st64 = h->dtype == XYL_F64 ? 1 : 0;
        // validate where the state lies; only the verdict comes back
        h->flag.reserve(1);
        launch_fill_u32(h->flag.p, 1, 0u, h->stream);
        launch_check_state(theta, omega, src64, h->N, h->p.model == kModelSI ? 1 : 0, st64, h->flag.p, h->stream);
        uint32_t bad = 0;
        check_hip(hipMemcpyAsync(&bad, h->flag.p, sizeof(bad), hipMemcpyDeviceToHost, h->stream), "D2H");
        check_hip(hipStreamSynchronize(h->stream), "hipStreamSynchronize");
        require(!(bad & kStateBadTheta), XYL_EINVAL, "theta entries must be finite with |theta| <= 3 pi");
        require(!(bad & kStateBadOmega), XYL_EINVAL, "omega entries must be finite");
        require(!(bad & kStateBadHalfCircle), XYL_EINVAL, "theta entries must lie in [-pi/2, pi/2) for the SI model");
        h->k = step;
        h->fresh_k = step;
        h->counter_valid = false;
        h->touch();
        launch_convert(theta, src64, h->cur_theta(), st64, h->N, 1.0, false, h->stream);
        launch_convert(omega, src64, h->u, st64, h->N, 1.0, false, h->stream);
        // the caller may release or rewrite its buffers once this returns
        check_hip(hipStreamSynchronize(h->stream), "hipStreamSynchronize");
        h->initialized = true;
    });
}

int xyl_init_ordered(xyl_lattice* h, int32_t sign) {
    if (!h) {
        g_err = "NULL handle";
        return XYL_EINVAL;
    }
    std::vector<double> th(h->N), om(h->N, 0.0);
    const double pi_p = h->dtype == XYL_F64 ? Prec<double>::kPi : (double)Prec<float>::kPi;
    // SI: the field -h cos(p th) with h < 0 is lowest at th = +-pi/p
    const double th0 = (h->p.h < 0.0 && h->p.p > 2.0) ? M_PI / h->p.p : 0.0;
    const int sx = h->p.Jx > 0.0, sy = h->p.Jy > 0.0;
    for (int y = 0; y < h->Ly; ++y)
        for (int x = 0; x < h->Lx; ++x) {
            int e = ((x * sx + y * sy) & 1) ? -1 : 1;
            if (sign < 0) e = -e;
            if (h->p.model == kModelSI) th[(size_t)y * h->Lx + x] = e > 0 ? th0 : -th0;
            else th[(size_t)y * h->Lx + x] = e > 0 ? 0.0 : -pi_p;
        }
    return xyl_set_state(h, th.data(), om.data(), 0);
}

int xyl_get_state(xyl_lattice* h, double* theta, double* omega, uint64_t* step) {
    return guarded([&] {
        require_init(h);
        DeviceGuard g(h->device);
        if (theta) {
            if (h->dtype == XYL_F64) to_host<double>(h->cur_theta(), theta, h->N, h->stream);
            else to_host<float>(h->cur_theta(), theta, h->N, h->stream);
        }
        if (omega) {
            if (h->dtype == XYL_F64) lattice_omega<double>(h, omega);
            else lattice_omega<float>(h, omega);
        }
        if (step) *step = h->k;
        if (theta) require_finite(theta, h->N, "angles");
        if (omega) require_finite(omega, h->N, "velocities");
    });
}

int xyl_state_buffers(xyl_lattice* h, void** theta, void** vel, int32_t* fresh) {
    return guarded([&] {
        require_init(h);
        if (theta) *theta = h->cur_theta();
        if (vel) *vel = h->u;
        if (fresh) *fresh = h->k == h->fresh_k ? 1 : 0;
    });
}

int xyl_step(xyl_lattice* h, uint64_t nsteps) {
    return guarded([&] {
        require_init(h);
        DeviceGuard g(h->device);
        if (h->dtype == XYL_F64) lattice_steps<double>(h, nsteps);
        else lattice_steps<float>(h, nsteps);
    });
}

int xyl_step_measured(xyl_lattice* h, uint64_t nsteps, uint64_t every, xyl_obs* out, uint64_t cap, uint64_t* nout) {
    return guarded([&] {
        require_init(h);
        require(every >= 1, XYL_EINVAL, "every must be >= 1");
        require(out != nullptr, XYL_EINVAL, "out is NULL");
        const uint64_t ns = nsteps / every + 1;
        require(cap >= ns, XYL_EINVAL, "sample capacity too small");
        DeviceGuard g(h->device);
        h->obs.reserve(6 * ns);
        h->obs_host.reserve(6 * ns);
        for (uint64_t j = 0; j < ns; ++j) {
            double* o = h->obs.p + 6 * j;
            if (j * every == nsteps) {
                // a sample at the last step: measured without stepping
                if (h->dtype == XYL_F64) lattice_measure_into<double>(h, false, o);
                else lattice_measure_into<float>(h, false, o);
            } else {
                // up to the next sample, or to the end (nsteps not a multiple of every)
                const uint64_t span = std::min<uint64_t>(every, nsteps - j * every);
                if (h->dtype == XYL_F64) lattice_sample_and_advance<double>(h, span, o);
                else lattice_sample_and_advance<float>(h, span, o);
            }
        }
        check_hip(hipMemcpyAsync(h->obs_host.p, h->obs.p, sizeof(double) * 6 * ns, hipMemcpyDeviceToHost, h->stream),
                  "D2H");
        check_hip(hipStreamSynchronize(h->stream), "hipStreamSynchronize");
        std::memcpy(out, h->obs_host.p, sizeof(double) * 6 * ns);
        if (nout) *nout = ns;
        require_finite(reinterpret_cast<const double*>(out), 6 * ns, "observables");
    });
}

int xyl_step_adaptive(xyl_lattice* h, uint64_t nsteps, uint64_t ds0, uint64_t ds_min, uint64_t ds_max, int32_t which,
                      uint64_t block, xyl_obs* out, uint64_t* steps, uint64_t cap, uint64_t* nout) {
    return guarded([&] {
        require_init(h);
        require(out != nullptr && steps != nullptr, XYL_EINVAL, "out/steps are NULL");
        require(ds_min >= 1 && ds_min <= ds0 && ds0 <= ds_max, XYL_EINVAL, "need 1 <= ds_min <= ds0 <= ds_max");
        require(which >= 0 && which < 6, XYL_EINVAL, "which must index an observable (0..5)");
        require(block >= 4, XYL_EINVAL, "block must be >= 4 samples");
        require(cap >= nsteps / ds_min + 2, XYL_EINVAL, "cap must be >= nsteps / ds_min + 2");
        DeviceGuard g(h->device);
        h->obs.reserve(6 * block);
        const uint64_t kend = h->k + nsteps;
        uint64_t ds = ds0, n = 0;
        std::vector<double> vals;
        vals.reserve(block);
        // samples are measured into a device block and copied out when it is
        // full (the spacing decision needs them) or at the end
        uint64_t in_dev = 0;
        auto flush = [&]() {
            if (!in_dev) return;
            check_hip(hipMemcpyAsync(out + (n - in_dev), h->obs.p, sizeof(double) * 6 * in_dev,
                                     hipMemcpyDeviceToHost, h->stream),
                      "D2H");
            check_hip(hipStreamSynchronize(h->stream), "hipStreamSynchronize");
            in_dev = 0;
        };
        auto sample = [&](bool advance) {
            if (in_dev == block) flush();
            steps[n] = h->k;
            if (h->dtype == XYL_F64) lattice_measure_into<double>(h, advance, h->obs.p + 6 * in_dev);
            else lattice_measure_into<float>(h, advance, h->obs.p + 6 * in_dev);
            ++in_dev;
            ++n;
        };
        uint64_t blk = 0;   // samples in the current block (equal spacing)
        while (true) {
            const bool last = h->k == kend;
            sample(!last);   // measures at k and, unless last, advances one step
            ++blk;
            if (last) break;
            if (blk == block) {
                // the block's series of the chosen observable decides the
                // spacing from here on: ds' = ds tau / 10 with tau in samples
                // (App. B: ds ~ tau_C / 10)
                flush();
                vals.assign(block, 0.0);
                const xyl_obs* o = out + (n - block);
                for (uint64_t i = 0; i < block; ++i) vals[i] = reinterpret_cast<const double*>(o + i)[which];
                const double tau = tau_int(vals.data(), block);
                const double want = std::floor((double)ds * tau / 10.0 + 0.5);
                ds = (uint64_t)std::min<double>(std::max<double>(want, (double)ds_min), (double)ds_max);
                blk = 0;
            }
            const uint64_t adv = std::min<uint64_t>(ds, kend - (h->k - 1));
            if (adv > 1) {
                if (h->dtype == XYL_F64) lattice_steps<double>(h, adv - 1);
                else lattice_steps<float>(h, adv - 1);
            }
        }
        flush();
        if (nout) *nout = n;
        require_finite(reinterpret_cast<const double*>(out), 6 * n, "observables");
    });
}

int xyl_measure(xyl_lattice* h, xyl_obs* out) {
    return guarded([&] {
        require_init(h);
        require(out != nullptr, XYL_EINVAL, "out is NULL");
        DeviceGuard g(h->device);
        h->obs.reserve(6);
        h->obs_host.reserve(6);
        if (h->dtype == XYL_F64) lattice_measure_into<double>(h, false, h->obs.p);
        else lattice_measure_into<float>(h, false, h->obs.p);
        check_hip(hipMemcpyAsync(h->obs_host.p, h->obs.p, sizeof(double) * 6, hipMemcpyDeviceToHost, h->stream), "D2H");
        check_hip(hipStreamSynchronize(h->stream), "hipStreamSynchronize");
        std::memcpy(out, h->obs_host.p, sizeof(double) * 6);
        require_finite(reinterpret_cast<const double*>(out), 6, "observables");
    });
}

int xyl_correlation(xyl_lattice* h, int32_t axis, int32_t rmax, double* C) {
    return guarded([&] {
        require_init(h);
        require(axis == 0 || axis == 1, XYL_EINVAL, "axis must be 0 or 1");
        const int L = axis == 0 ? h->Lx : h->Ly;
        require(rmax >= 0 && rmax <= L / 2, XYL_EINVAL, "rmax must be in [0, L/2]");
        require(L <= 4096, XYL_EUNSUPPORTED, "correlation needs the axis length <= 4096");
        require(C != nullptr, XYL_EINVAL, "C is NULL");
        DeviceGuard g(h->device);
        const size_t nscr = correlation_scratch(h->Lx, h->Ly, axis, rmax);
        h->dscratch.reserve(nscr + (rmax + 1));
        double* part = h->dscratch.p;
        double* outd = h->dscratch.p + nscr;
        const int sx = h->p.Jx > 0.0, sy = h->p.Jy > 0.0;
        if (h->dtype == XYL_F64)
            launch_correlation<double>(static_cast<const double*>(h->cur_theta()), h->Lx, h->Ly, sx, sy, h->p.model,
                                       axis, rmax, part, outd, h->stream);
        else
            launch_correlation<float>(static_cast<const float*>(h->cur_theta()), h->Lx, h->Ly, sx, sy, h->p.model,
                                      axis, rmax, part, outd, h->stream);
        check_hip(hipMemcpyAsync(C, outd, sizeof(double) * (rmax + 1), hipMemcpyDeviceToHost, h->stream), "D2H");
        check_hip(hipStreamSynchronize(h->stream), "hipStreamSynchronize");
    });
}

}  // extern "C"

// S_delta(k) of one lattice's current angles into host S[0..kmax].
template <typename R>
static void structure_factor_into(const void* th, int Lx, int Ly, int sx, int sy, int model, int axis, int kmax,
                                  DevBuf<double>& scratch, hipStream_t s, double* S) {
    const int nlines = axis == 0 ? Ly : Lx;
    const int L = axis == 0 ? Lx : Ly;
    const size_t N = (size_t)Lx * Ly;
    // the lines (N complex), the twiddle table (L complex), the per-line
    // spectra and the sum
    scratch.reserve(2 * (N + (size_t)L) + (size_t)nlines * (kmax + 1) + (size_t)(kmax + 1));
    double* z = scratch.p;
    double* part = scratch.p + 2 * (N + (size_t)L);
    double* outd = part + (size_t)nlines * (kmax + 1);
    launch_structure_factor<R>(static_cast<const R*>(th), Lx, Ly, sx, sy, model, axis, kmax, z, part, outd, s);
    check_hip(hipMemcpyAsync(S, outd, sizeof(double) * (kmax + 1), hipMemcpyDeviceToHost, s), "D2H");
    check_hip(hipStreamSynchronize(s), "hipStreamSynchronize");
    require_finite(S, (size_t)kmax + 1, "structure factor");
}

static void validate_sf(int Lx, int Ly, int axis, int kmax, const double* S) {
    require(axis == 0 || axis == 1, XYL_EINVAL, "axis must be 0 or 1");
    const int L = axis == 0 ? Lx : Ly;
    require(kmax >= 0 && kmax <= L / 2, XYL_EINVAL, "kmax must be in [0, L/2]");
    require(L <= 4096, XYL_EUNSUPPORTED, "the structure factor needs the axis length <= 4096");
    require(S != nullptr, XYL_EINVAL, "S is NULL");
}


extern "C" {

int xyl_structure_factor(xyl_lattice* h, int32_t axis, int32_t kmax, double* S) {
    return guarded([&] {
        require_init(h);
        validate_sf(h->Lx, h->Ly, axis, kmax, S);
        DeviceGuard g(h->device);
        const int sx = h->p.Jx > 0.0, sy = h->p.Jy > 0.0;
        if (h->dtype == XYL_F64)
            structure_factor_into<double>(h->cur_theta(), h->Lx, h->Ly, sx, sy, h->p.model, axis, kmax, h->dscratch,
                                          h->stream, S);
        else
            structure_factor_into<float>(h->cur_theta(), h->Lx, h->Ly, sx, sy, h->p.model, axis, kmax, h->dscratch,
                                         h->stream, S);
    });
}


int xyl_domains(xyl_lattice* h, int32_t* labels, uint64_t* sizes, uint64_t* counts, uint64_t cap, uint64_t* n_sizes,
                uint64_t* n_domains, uint64_t* max_size) {
    return guarded([&] {
        require_init(h);
        DeviceGuard g(h->device);
        const int sx = h->p.Jx > 0.0, sy = h->p.Jy > 0.0;
        if (h->dtype == XYL_F64)
            run_domains<double>(static_cast<const double*>(h->cur_theta()), h->Lx, h->Ly, sx, sy, h->p.model,
                                h->parent, h->usz,
                                h->hist, h->stats, h->stream, labels, sizes, counts, cap, n_sizes, n_domains, max_size);
        else
            run_domains<float>(static_cast<const float*>(h->cur_theta()), h->Lx, h->Ly, sx, sy, h->p.model,
                               h->parent, h->usz,
                               h->hist, h->stats, h->stream, labels, sizes, counts, cap, n_sizes, n_domains, max_size);
    });
}

}  // extern "C"

// ----------------------------------------------- allocation-free domains
// Scratch of xyl_domains_noalloc, the domain labelling for callers that cannot
// allocate device memory: the union-find's parent, cluster-size and histogram
// arrays and its (size, count) pair list for lattices of up to
// kNoAllocMaxSites sites, 3 * 4 * 2^22 + 4 * (5 + 2 * 4096) bytes (about
// 48 MiB).  Each device the library runs on holds one copy until the process
// ends.  Host code never names the array itself (there it is a host-side
// stand-in): it uses the device address hipGetSymbolAddress returns, looked up
// once per device with that device current.
constexpr size_t kNoAllocMaxSites = size_t(1) << 22;
constexpr size_t kNoAllocMaxPairs = 4096;
constexpr size_t kNoAllocWords = 3 * kNoAllocMaxSites + 1 + kDomainPairs + 2 * kNoAllocMaxPairs;
static __device__ __align__(256) uint32_t scratch[kNoAllocWords];

constexpr int kNoAllocMaxDevices = 64;
static std::mutex g_scratch_mu;                         // one call at a time in this process
static uint32_t* g_scratch_dev[kNoAllocMaxDevices] = {};

// Device address of `scratch` on device dev (current); g_scratch_mu held.
static uint32_t* scratch_address(int dev) {
    require(dev >= 0 && dev < kNoAllocMaxDevices, XYL_EUNSUPPORTED, "device index beyond the scratch table");
    if (!g_scratch_dev[dev]) {
        uint32_t* ptr = nullptr;
        check_hip(hipGetSymbolAddress((void**)&ptr, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
        require(ptr != nullptr, XYL_EDEVICE, "hipGetSymbolAddress returned no address for the scratch array");
        g_scratch_dev[dev] = ptr;
    }
    return g_scratch_dev[dev];
}

// xyl_domains on the static scratch: zeroed by kernels (no memset), results
// read back into the caller's arrays and a fixed stack buffer (no heap).
template <typename R>
static void domains_noalloc(xyl_lattice* h, int32_t* labels, uint64_t* sizes, uint64_t* counts, uint64_t cap,
                            uint64_t* n_sizes, uint64_t* n_domains, uint64_t* max_size) {
    const size_t N = h->N;
    const uint32_t pcap = domain_size_cap(N);
    require(pcap <= kNoAllocMaxPairs, XYL_EDEVICE, "size-distribution bound exceeds the scratch");
    hipStream_t s = h->stream;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    uint32_t* base = scratch_address(h->device);
    int32_t* parent = reinterpret_cast<int32_t*>(base);
    uint32_t* usz = base + N;
    uint32_t* hist = base + 2 * N;
    uint32_t* stats = base + 3 * N + 1;
    // the previous call's contents stay in the array: clear what must start at 0
    launch_fill_u32(hist, N + 1, 0u, s);
    launch_fill_u32(stats, kDomainPairs, 0u, s);
    const int sx = h->p.Jx > 0.0, sy = h->p.Jy > 0.0;
    launch_domains<R>(static_cast<const R*>(h->cur_theta()), h->Lx, h->Ly, sx, sy, h->p.model, parent, usz, hist,
                      stats, s);
    uint32_t head[kDomainPairs];
    check_hip(hipMemcpyAsync(head, stats, sizeof(head), hipMemcpyDeviceToHost, s), "D2H");
    if (labels) check_hip(hipMemcpyAsync(labels, parent, sizeof(int32_t) * N, hipMemcpyDeviceToHost, s), "D2H");
    check_hip(hipStreamSynchronize(s), "hipStreamSynchronize");
    const uint64_t ns = head[0];
    require(ns >= 1 && ns <= pcap, XYL_EDEVICE, "domain size distribution overflowed its bound");
    if (sizes || counts) require(cap >= ns, XYL_EINVAL, "size-distribution capacity too small");
    // (size, count) pairs as two 32-bit words each; sorted by size as 64-bit
    // keys size << 32 | count (sizes are distinct)
    uint64_t pairs[kNoAllocMaxPairs];
    check_hip(hipMemcpyAsync(pairs, stats + kDomainPairs, sizeof(uint32_t) * 2 * ns, hipMemcpyDeviceToHost, s),
              "D2H");
    check_hip(hipStreamSynchronize(s), "hipStreamSynchronize");
    for (uint64_t j = 0; j < ns; ++j) {
        uint32_t w[2];
        std::memcpy(w, &pairs[j], sizeof(w));
        pairs[j] = ((uint64_t)w[0] << 32) | (uint64_t)w[1];
    }
    std::sort(pairs, pairs + ns);
    uint64_t nd = 0, covered = 0;
    for (uint64_t j = 0; j < ns; ++j) {
        const uint64_t sz = pairs[j] >> 32, ct = pairs[j] & 0xFFFFFFFFull;
        if (sizes) sizes[j] = sz;
        if (counts) counts[j] = ct;
        nd += ct;
        covered += sz * ct;
    }
    require(covered == N, XYL_EDEVICE, "domain sizes do not cover the lattice");
    if (n_sizes) *n_sizes = ns;
    if (n_domains) *n_domains = nd;
    if (max_size) *max_size = pairs[ns - 1] >> 32;
}

extern "C" {

int xyl_domains_noalloc(xyl_lattice* h, int32_t* labels, uint64_t* sizes, uint64_t* counts, uint64_t cap,
                        uint64_t* n_sizes, uint64_t* n_domains, uint64_t* max_size) {
    return guarded([&] {
        require_init(h);
        require(h->N <= kNoAllocMaxSites, XYL_EINVAL,
                "xyl_domains_noalloc takes lattices of at most 2^22 sites (its static scratch)");
        DeviceGuard g(h->device);
        if (h->dtype == XYL_F64) domains_noalloc<double>(h, labels, sizes, counts, cap, n_sizes, n_domains, max_size);
        else domains_noalloc<float>(h, labels, sizes, counts, cap, n_sizes, n_domains, max_size);
    });
}

int xyl_sync(xyl_lattice* h) {
    return guarded([&] {
        require(h != nullptr, XYL_EINVAL, "NULL handle");
        DeviceGuard g(h->device);
        check_hip(hipStreamSynchronize(h->stream), "hipStreamSynchronize");
    });
}

int xyl_set_launch(xyl_lattice* h, int32_t rows, int32_t wpb) {
    return guarded([&] {
        require(h != nullptr, XYL_EINVAL, "NULL handle");
        Launch l = h->launch;
        if (rows) l.rows = rows;
        if (wpb) l.wpb = wpb;
        validate_launch(l);
        h->launch = l;
        h->touch();
    });
}

int xyl_get_launch(xyl_lattice* h, int32_t* rows, int32_t* wpb) {
    return guarded([&] {
        require(h != nullptr, XYL_EINVAL, "NULL handle");
        if (rows) *rows = h->launch.rows;
        if (wpb) *wpb = h->launch.wpb;
    });
}

}  // extern "C"

// Times the single-step launch shapes and, for FP32 lattices of a shape the
// two-step pass takes, the two-step pass at several strip heights; returns
// the best single-step shape and sets *fusion (1 or 2, whichever is faster
// per step) and *rows2 (rows per strip of the best two-step pass, 0 if none).
template <typename R>
static Launch autotune_impl(xyl_lattice* h, int* fusion, int* rows2, int* tw2, Launch* mlaunch) {
    // time candidates on scratch copies so the lattice state is untouched;
    // each candidate runs as a captured graph of back-to-back steps, so the
    // host's launch overhead does not mask kernel time on small lattices
    const size_t bytes = sizeof(R) * h->N;
    DevBuf<char> tmp;
    tmp.reserve(4 * bytes);
    DevBuf<uint64_t> kc;
    kc.reserve(1);
    Lat<R> v = h->view<R>();
    v.th[0] = reinterpret_cast<R*>(tmp.p);
    v.th[1] = reinterpret_cast<R*>(tmp.p + bytes);
    v.u = reinterpret_cast<R*>(tmp.p + 2 * bytes);
    check_hip(hipMemcpyAsync(v.th[0], h->cur_theta(), bytes, hipMemcpyDeviceToDevice, h->stream), "D2D");
    check_hip(hipMemcpyAsync(v.th[1], h->cur_theta(), bytes, hipMemcpyDeviceToDevice, h->stream), "D2D");
    check_hip(hipMemcpyAsync(v.u, h->u, bytes, hipMemcpyDeviceToDevice, h->stream), "D2D");
    v.fresh_k = ~(uint64_t)0;
    launch_set_counter(kc.p, 0, h->stream);
    check_hip(hipStreamSynchronize(h->stream), "hipStreamSynchronize");
    hipEvent_t e0, e1;
    check_hip(hipEventCreate(&e0), "hipEventCreate");
    check_hip(hipEventCreate(&e1), "hipEventCreate");
    const int rows_c[] = {1, 2, 4, 8, 16, 32, 64};
    const int wpb_c[] = {1, 2, 4, 8};
    // about 2 ms of work per timing (at least 16 steps)
    const int reps = (int)std::max<double>(16.0, std::min<double>(512.0, 2.0e11 * 2e-3 / (double)h->N));
    auto time_graph = [&](const Launch& l, int repeats, int mode = kStore) {
        hipGraph_t g = nullptr;
        hipGraphExec_t ex = nullptr;
        check_hip(hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
        for (int i = 0; i < reps; ++i) launch_step<R>(v, mode, l, kc.p, (uint64_t)i, h->cap_stream);
        check_hip(hipStreamEndCapture(h->cap_stream, &g), "hipStreamEndCapture");
        hipError_t err = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        check_hip(err, "hipGraphInstantiate");
        check_hip(hipGraphLaunch(ex, h->stream), "hipGraphLaunch");   // warm-up
        float best_t = 1e30f;
        for (int rep = 0; rep < repeats; ++rep) {
            check_hip(hipEventRecord(e0, h->stream), "hipEventRecord");
            check_hip(hipGraphLaunch(ex, h->stream), "hipGraphLaunch");
            check_hip(hipEventRecord(e1, h->stream), "hipEventRecord");
            check_hip(hipEventSynchronize(e1), "hipEventSynchronize");
            float ms = 0.f;
            check_hip(hipEventElapsedTime(&ms, e0, e1), "hipEventElapsedTime");
            best_t = std::min(best_t, ms);
        }
        (void)hipGraphExecDestroy(ex);
        return best_t;
    };
    std::vector<std::pair<float, Launch>> scores;
    for (int r : rows_c) {
        if (r > h->Ly) continue;
        for (int w : wpb_c) {
            Launch l;
            l.rows = r;
            l.wpb = w;
            scores.push_back({time_graph(l, 1), l});
        }
    }
    // re-time the three fastest with repeats and keep the best minimum
    std::sort(scores.begin(), scores.end(), [](const auto& a, const auto& b) { return a.first < b.first; });
    Launch best = scores.front().second;
    float best_ms = 1e30f;
    for (size_t i = 0; i < std::min<size_t>(3, scores.size()); ++i) {
        const float t = time_graph(scores[i].second, 3);
        if (t < best_ms) {
            best_ms = t;
            best = scores[i].second;
        }
    }
    // measurements without a step (the samples of a run): the same timing
    // over the shapes, the partial sums written to the lattice's own buffer
    {
        std::vector<std::pair<float, Launch>> ms;
        for (int r : rows_c) {
            if (r > h->Ly) continue;
            for (int w : wpb_c) {
                Launch l;
                l.rows = r;
                l.wpb = w;
                ms.push_back({time_graph(l, 1, kMeasure), l});
            }
        }
        std::sort(ms.begin(), ms.end(), [](const auto& a, const auto& b) { return a.first < b.first; });
        *mlaunch = ms.front().second;
        float mbest = 1e30f;
        for (size_t i = 0; i < std::min<size_t>(3, ms.size()); ++i) {
            const float t = time_graph(ms[i].second, 3, kMeasure);
            if (t < mbest) {
                mbest = t;
                *mlaunch = ms[i].second;
            }
        }
    }
    // two steps per pass: the same timing over a multiple of 4 steps, per step
    *fusion = 1;
    *rows2 = 0;
    *tw2 = 0;
    if constexpr (std::is_same<R, float>::value) {
        if (step2_lattice_shape(h->Lx, h->Ly) && kick_factored(h->p)) {
            const int reps4 = (reps + 3) / 4 * 4;
            float* A = v.th[0];
            float* B = v.th[1];
            float* u = v.u;
            float* u2 = reinterpret_cast<float*>(tmp.p + 3 * bytes);
            check_hip(hipMemcpyAsync(u2, v.u, bytes, hipMemcpyDeviceToDevice, h->stream), "D2D");
            auto time_step2 = [&](int rows, int tw, int repeats) {
                hipGraph_t g = nullptr;
                hipGraphExec_t ex = nullptr;
                check_hip(hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal),
                          "hipStreamBeginCapture");
                for (int i = 0; i < reps4; i += 4) {
                    launch_step2(v, A, u, B, u2, rows, kc.p, (uint64_t)i, h->cap_stream, tw);
                    launch_step2(v, B, u2, A, u, rows, kc.p, (uint64_t)i + 2, h->cap_stream, tw);
                }
                check_hip(hipStreamEndCapture(h->cap_stream, &g), "hipStreamEndCapture");
                hipError_t err = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
                (void)hipGraphDestroy(g);
                check_hip(err, "hipGraphInstantiate");
                check_hip(hipGraphLaunch(ex, h->stream), "hipGraphLaunch");   // warm-up
                float best_t = 1e30f;
                for (int rep = 0; rep < repeats; ++rep) {
                    check_hip(hipEventRecord(e0, h->stream), "hipEventRecord");
                    check_hip(hipGraphLaunch(ex, h->stream), "hipGraphLaunch");
                    check_hip(hipEventRecord(e1, h->stream), "hipEventRecord");
                    check_hip(hipEventSynchronize(e1), "hipEventSynchronize");
                    float ms = 0.f;
                    check_hip(hipEventElapsedTime(&ms, e0, e1), "hipEventElapsedTime");
                    best_t = std::min(best_t, ms);
                }
                (void)hipGraphExecDestroy(ex);
                return best_t / (float)reps4;
            };
            // the tile width first (whole rows or the fewest tiles, and
            // narrower tiles; each at the rule's strip height for it), then
            // the strip height at the best width
            int tw = 16;
            {
                std::vector<std::pair<float, int>> st;
                std::vector<std::pair<int, int>> seen;   // (tiles, width) of the candidates timed
                for (int c : {16, 11, 8, 4, 3, 2}) {
                    Step2Tiles t;
                    if (!step2_tiles(h->Lx, &t, c)) {
                        if (c != 16) continue;
                        t.ntx = 1;             // whole rows
                        t.w = h->Lx;
                    }
                    if (std::find(seen.begin(), seen.end(), std::make_pair(t.ntx, t.w)) != seen.end()) continue;
                    seen.push_back({t.ntx, t.w});
                    st.push_back({time_step2(step2_rows(h->Lx, h->Ly, h->cus, c), c, 2), c});
                }
                std::sort(st.begin(), st.end());
                tw = st.front().second;
            }
            Step2Tiles t0;
            const bool tiled = step2_tiles(h->Lx, &t0, tw);
            std::vector<int> rows_c2 = {2, 4, 8, 16, step2_rows(h->Lx, h->Ly, h->cus, tw)};
            if (tiled) rows_c2.push_back(32);
            std::sort(rows_c2.begin(), rows_c2.end());
            rows_c2.erase(std::unique(rows_c2.begin(), rows_c2.end()), rows_c2.end());
            std::vector<std::pair<float, int>> s2;
            for (int r : rows_c2)
                if (r <= h->Ly) s2.push_back({time_step2(r, tw, 1), r});
            std::sort(s2.begin(), s2.end());
            float best2 = 1e30f;
            for (size_t i = 0; i < std::min<size_t>(2, s2.size()); ++i) {
                const float t = time_step2(s2[i].second, tw, 3);
                if (t < best2) {
                    best2 = t;
                    *rows2 = s2[i].second;
                }
            }
            *tw2 = tw;
            if (best2 < best_ms / (float)reps) *fusion = 2;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return best;
}

extern "C" {

int xyl_autotune(xyl_lattice* h) {
    return guarded([&] {
        require_init(h);
        DeviceGuard g(h->device);
        int fusion = 1, rows2 = 0, tw2 = 0;
        Launch lm;
        Launch l = h->dtype == XYL_F64 ? autotune_impl<double>(h, &fusion, &rows2, &tw2, &lm)
                                       : autotune_impl<float>(h, &fusion, &rows2, &tw2, &lm);
        h->launch = l;
        h->mlaunch = lm;
        h->mlaunch_tuned = true;
        if (h->dtype == XYL_F32) {
            h->fusion = fusion;
            h->step2_rows_tuned = rows2;
            h->step2_tw_tuned = tw2;
        }
        h->touch();
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tuned[{h->Lx, h->Ly, h->dtype}] = l;
        g_tunedm[{h->Lx, h->Ly, h->dtype}] = lm;
        if (h->dtype == XYL_F32) g_tuned2[{h->Lx, h->Ly, h->dtype}] = {fusion, rows2, tw2};
    });
}

int xyl_set_fusion(xyl_lattice* h, int32_t steps_per_pass) {
    return guarded([&] {
        require(h != nullptr, XYL_EINVAL, "NULL handle");
        require(steps_per_pass == 1 || steps_per_pass == 2, XYL_EINVAL, "steps_per_pass must be 1 or 2");
        h->fusion = steps_per_pass;
    });
}

int xyl_get_fusion(const xyl_lattice* h, int32_t* steps_per_pass, int32_t* rows) {
    return guarded([&] {
        require(h != nullptr, XYL_EINVAL, "NULL handle");
        if (steps_per_pass) *steps_per_pass = h->fusion;
        if (rows) *rows = step2_eligible(h) ? step2_rows(h) : 0;
    });
}

int xyl_set_step2_shape(xyl_lattice* h, int32_t rows, int32_t tile_waves) {
    return guarded([&] {
        require(h != nullptr, XYL_EINVAL, "NULL handle");
        require(rows == 0 || (rows >= 2 && rows <= 64), XYL_EINVAL, "rows per strip must be 0 or in [2, 64]");
        require(tile_waves == 0 || (tile_waves >= 2 && tile_waves <= 16), XYL_EINVAL,
                "waves per tile must be 0 or in [2, 16]");
        if (rows) h->step2_rows_tuned = rows;
        if (tile_waves) h->step2_tw_tuned = tile_waves;
        h->touch();
    });
}

int xyl_get_step2_shape(const xyl_lattice* h, int32_t* rows, int32_t* tile_waves, int32_t* tiles) {
    return guarded([&] {
        require(h != nullptr, XYL_EINVAL, "NULL handle");
        const bool on = step2_eligible(h);
        int tw = 0, ntx = 0;
        if (on) {
            Step2Tiles t;
            const int want = step2_tile_waves(h);
            if (step2_tiles(h->Lx, &t, want) || step2_tiles(h->Lx, &t)) {
                tw = want;
                ntx = t.ntx;
            } else {
                tw = (h->Lx + kWaveSites - 1) / kWaveSites;   // whole rows
                ntx = 1;
            }
        }
        if (rows) *rows = on ? step2_rows(h) : 0;
        if (tile_waves) *tile_waves = tw;
        if (tiles) *tiles = ntx;
    });
}

int xyl_set_graph_steps(xyl_lattice* h, int32_t steps) {
    return guarded([&] {
        require(h != nullptr, XYL_EINVAL, "NULL handle");
        require(steps >= 0 && steps <= 4096, XYL_EINVAL, "graph steps must be in [0, 4096]");
        h->graph_steps = steps;
        h->touch();
    });
}

int xyl_philox_blocks(int32_t device, uint64_t seed, const uint32_t* ctr, uint32_t* out, uint64_t n) {
    return guarded([&] {
        require(ctr != nullptr && out != nullptr, XYL_EINVAL, "NULL array");
        require(n >= 1 && n <= (1ull << 26), XYL_EINVAL, "n out of range");
        select_device(device);
        DevBuf<uint32_t> dc, dout;
        dc.reserve(4 * n);
        dout.reserve(4 * n);
        check_hip(hipMemcpy(dc.p, ctr, sizeof(uint32_t) * 4 * n, hipMemcpyHostToDevice), "H2D");
        launch_philox_blocks(seed, dc.p, dout.p, n, nullptr);
        check_hip(hipMemcpy(out, dout.p, sizeof(uint32_t) * 4 * n, hipMemcpyDeviceToHost), "D2H");
    });
}

int xyl_stream_ceiling(int32_t device, uint64_t n, int32_t reps, double* gbs) {
    return guarded([&] {
        require(gbs != nullptr, XYL_EINVAL, "gbs is NULL");
        require(n >= 4 && n % 4 == 0, XYL_EINVAL, "n must be a positive multiple of 4");
        require(reps >= 2, XYL_EINVAL, "reps must be >= 2");
        select_device(device);
        DevBuf<float> buf;
        buf.reserve(4 * n);
        check_hip(hipMemset(buf.p, 0, sizeof(float) * 4 * n), "hipMemset");
        float* A = buf.p;
        float* B = buf.p + n;
        float* C = buf.p + 2 * n;
        float* D = buf.p + 3 * n;
        hipEvent_t e0, e1;
        check_hip(hipEventCreate(&e0), "hipEventCreate");
        check_hip(hipEventCreate(&e1), "hipEventCreate");
        double best = 0.0;
        for (int grid : {1024, 2048, 4096, 8192, 16384, 65536}) {
            for (int w = 0; w < 4; ++w) launch_stream_probe(A, B, C, D, n / 4, grid, nullptr);
            check_hip(hipEventRecord(e0, nullptr), "hipEventRecord");
            for (int r = 0; r < reps; ++r) {
                // ping-pong between the two pairs, like a lattice's state
                if (r & 1) launch_stream_probe(C, D, A, B, n / 4, grid, nullptr);
                else launch_stream_probe(A, B, C, D, n / 4, grid, nullptr);
            }
            check_hip(hipEventRecord(e1, nullptr), "hipEventRecord");
            check_hip(hipEventSynchronize(e1), "hipEventSynchronize");
            float ms = 0.f;
            check_hip(hipEventElapsedTime(&ms, e0, e1), "hipEventElapsedTime");
            best = std::max(best, 16.0 * (double)n * reps / ((double)ms * 1e-3) / 1e9);
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        *gbs = best;
    });
}

int xyl_noise(xyl_lattice* h, uint64_t k, double* out) {
    return guarded([&] {
        require(h != nullptr && out != nullptr, XYL_EINVAL, "NULL argument");
        DeviceGuard g(h->device);
        h->dscratch.reserve(h->N);
        if (h->dtype == XYL_F64) launch_noise<double>(h->view<double>(), k, h->dscratch.p, h->stream);
        else launch_noise<float>(h->view<float>(), k, h->dscratch.p, h->stream);
        check_hip(hipMemcpyAsync(out, h->dscratch.p, sizeof(double) * h->N, hipMemcpyDeviceToHost, h->stream), "D2H");
        check_hip(hipStreamSynchronize(h->stream), "hipStreamSynchronize");
    });
}


}  // extern "C"

// ==================================================================== ensemble
struct xyl_ensemble {
    int dtype = XYL_F32;
    int device = 0;
    int n = 0;
    int mode = 0;
    hipStream_t stream = nullptr;
    std::vector<xyl_replica_desc> desc;
    std::vector<size_t> off;        // element offset of each replica
    std::vector<size_t> poff;       // partial-sum offset of each replica
    size_t total = 0, ptotal = 0;
    void* th[2] = {nullptr, nullptr};
    void* u = nullptr;
    std::vector<uint64_t> k;        // current step of each replica
    std::vector<uint64_t> fresh_k;
    std::vector<uint64_t> last_sample;  // step of the last recorded sample (+1), 0 = none
    uint64_t j = 0;                 // batched launches issued
    Launch launch;
    DevBuf<char> reps;              // Lat<R>[n]
    DevBuf<Task> tasks;
    int ntasks = 0;
    std::vector<int> task_active;   // replica ids the task list was built for
    DevBuf<double> part;
    DevBuf<double> phases;                  // measurement phase tables, one per side length
    std::map<int, size_t> phase_off;        // side length -> offset of its table in phases
    DevBuf<double> obs;
    DevBuf<FinalizeJobHost> jobs;
    PinnedBuf<FinalizeJobHost> jobs_host;   // the source of each flush's copy into `jobs`
    DevBuf<double> dscratch;
    DevBuf<char> omega_buf;
    DevBuf<int32_t> parent;
    DevBuf<uint32_t> usz, hist, stats;
    // small FP32 replicas stepped whole-in-LDS on a second stream
    std::vector<char> lds;          // per replica: 1 = LDS path
    int lds_max_sites = 0, lds_threads = 0;
    hipStream_t side = nullptr;
    hipEvent_t ev_main = nullptr, ev_side = nullptr;
    // the LDS launches' tables, double-buffered: a chunk writes table b while
    // the previous chunk's launch may still read table b ^ 1; ev_lds[b] marks
    // the end of the last launch that read table b (and of the copies into it)
    DevBuf<char> lds_reps[2];
    DevBuf<LdsJobHost> lds_jobs[2];
    // host sides of those tables in pinned memory: an asynchronous copy from
    // pageable memory waits for its stream to drain, which left the GPU idle
    // at every chunk boundary while the host waited
    PinnedBuf<LdsJobHost> lds_jobs_host[2];
    PinnedBuf<Lat<float>> lds_tab_host[2];
    hipEvent_t ev_lds[2] = {nullptr, nullptr};
    bool ev_lds_used[2] = {false, false};
    int lds_buf = 0;
    // two steps per pass for FP32 replicas on the tile path: one batched launch
    // per class of replicas spanning the same number of waves, per pass; the
    // other tile-path replicas keep one tile launch per step (tasks_rest)
    struct Step2Class {
        int waves = 0;
        bool partial = false;
        int max_lx = 0;
        int rows = 0;
        DevBuf<Task2> tasks;
        int ntasks = 0;
    };
    int fusion = 2;
    int cus = 256;
    int tables_fusion = 0;          // fusion setting the task tables were built for
    std::vector<Step2Class> s2cls;
    DevBuf<Task> tasks_rest;
    int ntasks_rest = 0;
    DevBuf<char> u2;                // second velocity buffer, allocated on first use
    // the classes hold different replicas: all but the first run on streams of
    // their own (default priority), forked from and joined to the ensemble's
    std::vector<hipStream_t> cls_streams;
    std::vector<hipEvent_t> cls_events;   // [0] fork, [1 + i] join of class i + 1
    // Chunks of steps captured as graphs (step index from the device counter
    // kc): keyed by (first step within the chunk, steps), captured the second
    // time a key is met and replayed after; all dropped when a table, the
    // launch shape or the steps per pass change (graph_version).
    // 0: no graphs; 1: graphs for chunks with at most one class of two-step
    // passes; 2: graphs for every repeated chunk.  A replayed graph dispatches
    // the parallel branches of several classes one after the other (one
    // class's whole chain before the next class's first pass), so the classes
    // barely overlap; issued directly, pass by pass across the classes, they
    // run together.
    int use_graphs = 1;
    hipStream_t cap_stream = nullptr;
    DevBuf<uint64_t> kc;
    uint64_t graph_version = 0, graphs_built_for = ~(uint64_t)0;
    struct ChunkGraph {
        int seen = 0;
        hipGraphExec_t exec = nullptr;
    };
    std::map<std::pair<uint64_t, uint64_t>, ChunkGraph> graphs;
    void drop_graphs() {
        for (auto& g : graphs)
            if (g.second.exec) (void)hipGraphExecDestroy(g.second.exec);
        graphs.clear();
    }
    void class_streams(size_t ncls) {
        while (cls_streams.size() + 1 < ncls) {
            hipStream_t st = nullptr;
            check_hip(hipStreamCreateWithFlags(&st, hipStreamNonBlocking), "hipStreamCreate");
            cls_streams.push_back(st);
        }
        // [0] fork, [1 + i] join of class i + 1, [ncls] end of a chunk's sample
        while (cls_events.size() < ncls + 1) {
            hipEvent_t ev = nullptr;
            check_hip(hipEventCreateWithFlags(&ev, hipEventDisableTiming), "hipEventCreate");
            cls_events.push_back(ev);
        }
    }

    template <typename R>
    Lat<R> view(int r, uint64_t jbase) {
        const xyl_replica_desc& d = desc[r];
        Lat<R> v{};
        R* t0 = static_cast<R*>(th[0]) + off[r];
        R* t1 = static_cast<R*>(th[1]) + off[r];
        v.th[0] = t0;
        v.th[1] = t1;
        v.u = static_cast<R*>(u) + off[r];
        v.cur = 0;
        Params p{d.Jx, d.Jy, d.h, d.gamma, d.dt, d.model, d.p};
        Schedule s{};
        s.n = d.nknots;
        for (int q = 0; q < d.nknots; ++q) {
            s.step[q] = d.knot_step[q];
            s.T[q] = d.knot_T[q];
            s.g[q] = d.knot_gamma[q] == 0 ? 1 : d.knot_gamma[q];
        }
        fill_lat(v, d.Lx, d.Ly, p, s, d.seed, d.replica);
        v.k_base = k[r] - jbase;   // k = k_base + j for the launches numbered from jbase
        v.fresh_k = fresh_k[r];
        v.k_end = d.nsteps;
        v.part = part.p + poff[r];
        v.xph = phases.p + phase_off.at(d.Lx);
        v.yph = phases.p + phase_off.at(d.Ly);
        v.omega_out = reinterpret_cast<R*>(omega_buf.p);
        v.pingpong = 1;
        v.u_out = nullptr;
        v.part_k0 = 0;
        v.part_stride = 0;
        return v;
    }
    void* cur_theta(int r) {
        const size_t es = elem_size(dtype);
        return static_cast<char*>(th[(int)(k[r] & 1)]) + es * off[r];
    }
    int nrp(int r) const { return desc[r].Ly * ((desc[r].Lx + kWaveSites - 1) / kWaveSites); }
    int model() const { return desc[0].model; }
};

template <typename R>
static void ens_upload_table(xyl_ensemble* e, uint64_t jbase, const std::vector<int>& active) {
    std::vector<Lat<R>> tab(e->n);
    for (int r = 0; r < e->n; ++r) tab[r] = e->view<R>(r, jbase);
    e->reps.reserve(sizeof(Lat<R>) * e->n);
    check_hip(hipMemcpyAsync(e->reps.p, tab.data(), sizeof(Lat<R>) * e->n, hipMemcpyHostToDevice, e->stream), "H2D");
    std::vector<Task> tk;
    for (int r : active) {
        const int nxw = (e->desc[r].Lx + kWaveSites - 1) / kWaveSites;
        const int nstrips = (e->desc[r].Ly + e->launch.rows - 1) / e->launch.rows;
        for (int s = 0; s < nstrips; ++s)
            for (int x = 0; x < nxw; ++x) tk.push_back(Task{r, x, s, 0});
    }
    e->ntasks = (int)tk.size();
    e->tasks.reserve(std::max<size_t>(tk.size(), 1));
    if (!tk.empty())
        check_hip(hipMemcpyAsync(e->tasks.p, tk.data(), sizeof(Task) * tk.size(), hipMemcpyHostToDevice, e->stream),
                  "H2D");
    // two-step classes (FP32): replicas whose width the two-step pass takes,
    // grouped by waves per row; the rest of the tile-path replicas
    std::vector<std::vector<Task2>> t2(17);
    std::vector<Task> rest;
    e->s2cls.clear();
    if (e->dtype == XYL_F32 && e->fusion == 2) {
        std::vector<std::vector<int>> byw(17);
        for (int r : active) {
            const xyl_replica_desc& d = e->desc[r];
            if (step2_shape(d.Lx, d.Ly) && kick_factored(Params{d.Jx, d.Jy, d.h, d.gamma, d.dt, d.model, d.p}))
                byw[(d.Lx + kWaveSites - 1) / kWaveSites].push_back(r);
            else
                for (const Task& t : tk)
                    if (t.rep == r) rest.push_back(t);
        }
        for (int w = 1; w <= 16; ++w) {
            if (byw[w].empty()) continue;
            xyl_ensemble::Step2Class cl;
            cl.waves = w;
            // strips as tall as keep at least two waves per SIMD busy (2 to 32
            // rows; 32 for the 60 x 2048^2 quench batch: 5.83 -> 5.98e11
            // site-updates/s against 16, 5.86e11 with 64).  Rows of more than
            // 8 waves hold one workgroup per CU and go to 64 (eight 4096^2
            // replicas: 6.05 -> 6.19e11)
            cl.rows = 2;
            for (int rows = w > 8 ? 64 : 32; rows >= 2; rows /= 2) {
                long strips = 0;
                for (int r : byw[w]) strips += (e->desc[r].Ly + rows - 1) / rows;
                if (strips * w >= 8L * e->cus) {
                    cl.rows = rows;
                    break;
                }
            }
            for (int r : byw[w]) {
                const xyl_replica_desc& d = e->desc[r];
                cl.partial = cl.partial || d.Lx % kWaveSites != 0;
                cl.max_lx = std::max(cl.max_lx, d.Lx);
                for (int s = 0; s * cl.rows < d.Ly; ++s)
                    t2[w].push_back(Task2{r, s * cl.rows, std::min(d.Ly, (s + 1) * cl.rows), (s & 1) ? -1 : 1});
            }
            cl.ntasks = (int)t2[w].size();
            cl.tasks.reserve(t2[w].size());
            check_hip(hipMemcpyAsync(cl.tasks.p, t2[w].data(), sizeof(Task2) * t2[w].size(), hipMemcpyHostToDevice,
                                     e->stream),
                      "H2D");
            e->s2cls.push_back(std::move(cl));
        }
        e->ntasks_rest = (int)rest.size();
        e->tasks_rest.reserve(std::max<size_t>(rest.size(), 1));
        if (!rest.empty())
            check_hip(hipMemcpyAsync(e->tasks_rest.p, rest.data(), sizeof(Task) * rest.size(), hipMemcpyHostToDevice,
                                     e->stream),
                      "H2D");
    }
    // the second velocity buffer and the class streams now, not in the first
    // chunk that steps through the classes
    if (!e->s2cls.empty()) {
        e->u2.reserve(sizeof(float) * e->total);
        e->class_streams(e->s2cls.size());
    }
    // the host vectors must outlive the copies
    check_hip(hipStreamSynchronize(e->stream), "hipStreamSynchronize");
    e->task_active = active;
    e->tables_fusion = e->fusion;
    e->graph_version += 1;
}

// Sample bookkeeping of one xyl_ensemble_step call: observables gathered in
// device memory (slots), copied out at the end.
struct EnsSamples {
    xyl_ensemble* e;
    uint64_t every, cap;
    std::vector<uint64_t> cnt;
    size_t nsamp = 0;
    std::vector<std::pair<size_t, size_t>> copies;   // (device slot, host index)
    // finalize jobs of this call: each flush takes the next slots of the
    // device arena, copied from the same slots of its pinned host mirror
    size_t njobs = 0;
    EnsSamples(xyl_ensemble* e_, uint64_t every_, uint64_t cap_, const uint64_t* nout)
        : e(e_), every(every_), cap(cap_), cnt(e_->n, 0) {
        if (every && nout)
            for (int r = 0; r < e->n; ++r) cnt[r] = nout[r];
    }
    EnsSamples(const EnsSamples&) = delete;
    EnsSamples& operator=(const EnsSamples&) = delete;
    // the pinned job slots are the sources of copies that may still be
    // queued; the next call writes them again
    ~EnsSamples() {
        if (njobs) (void)hipStreamSynchronize(e->stream);
    }
    bool wants(int r) const {
        return every && e->k[r] <= e->desc[r].nsteps && e->k[r] % every == 0 && e->last_sample[r] != e->k[r] + 1;
    }
    void reserve(size_t extra) {
        const size_t need = nsamp + extra;
        if (need * 6 <= e->obs.n) return;
        // the side stream may still be writing samples into the old buffer
        if (e->side) check_hip(hipStreamSynchronize(e->side), "hipStreamSynchronize");
        DevBuf<double> nb;
        nb.reserve(std::max(need * 6, e->obs.n * 2));
        if (e->obs.p && nsamp)
            check_hip(hipMemcpyAsync(nb.p, e->obs.p, sizeof(double) * 6 * nsamp, hipMemcpyDeviceToDevice, e->stream),
                      "D2D");
        check_hip(hipStreamSynchronize(e->stream), "hipStreamSynchronize");
        std::swap(e->obs.p, nb.p);
        std::swap(e->obs.n, nb.n);
    }
    double* take(int r) {   // device slot of replica r's next sample
        require(cnt[r] < cap, XYL_EINVAL, "ensemble sample capacity too small");
        const size_t slot = nsamp++;
        copies.push_back({slot, (size_t)r * cap + cnt[r]});
        cnt[r] += 1;
        e->last_sample[r] = e->k[r] + 1;
        return e->obs.p + 6 * slot;
    }
    void finish(xyl_obs* out, uint64_t* nout) {
        if (!every) return;
        std::vector<double> host(6 * nsamp);
        if (nsamp)
            check_hip(hipMemcpyAsync(host.data(), e->obs.p, sizeof(double) * 6 * nsamp, hipMemcpyDeviceToHost,
                                     e->stream),
                      "D2H");
        check_hip(hipStreamSynchronize(e->stream), "hipStreamSynchronize");
        for (auto& c : copies) std::memcpy(&out[c.second], &host[6 * c.first], sizeof(double) * 6);
        if (nout)
            for (int r = 0; r < e->n; ++r) nout[r] = cnt[r];
    }
};

// Reduces the measurement partials of `jobs` into their sample slots, on the
// ensemble's stream, without waiting for it: the job list moves into the
// call's store and takes the next slots of the device arena (a full arena is
// replaced, after the stream has drained, by one twice as large).
static void flush_finalize(xyl_ensemble* e, EnsSamples& smp, std::vector<FinalizeJobHost>& jobs) {
    if (jobs.empty()) return;
    if (smp.njobs + jobs.size() > e->jobs.n || !e->jobs.p || e->jobs_host.n < e->jobs.n) {
        check_hip(hipStreamSynchronize(e->stream), "hipStreamSynchronize");
        const size_t cap = std::max<size_t>(2 * e->jobs.n, std::max<size_t>(jobs.size(), 256));
        e->jobs.reserve(cap);
        e->jobs_host.reserve(e->jobs.n);
        smp.njobs = 0;
    }
    FinalizeJobHost* src = e->jobs_host.p + smp.njobs;
    std::memcpy(src, jobs.data(), sizeof(FinalizeJobHost) * jobs.size());
    FinalizeJobHost* dst = e->jobs.p + smp.njobs;
    check_hip(hipMemcpyAsync(dst, src, sizeof(FinalizeJobHost) * jobs.size(), hipMemcpyHostToDevice, e->stream),
              "H2D");
    launch_finalize_jobs(dst, (int)jobs.size(), e->stream);
    smp.njobs += jobs.size();
    jobs.clear();
}

// Reference loop: every replica launched on its own, one step at a time.
template <typename R>
static void ens_step_per_replica(xyl_ensemble* e, uint64_t nsteps, EnsSamples& smp) {
    std::vector<FinalizeJobHost> jobs;
    for (uint64_t it = 0; it <= nsteps; ++it) {
        std::vector<int> active, measuring;
        for (int r = 0; r < e->n; ++r) {
            if (smp.wants(r)) measuring.push_back(r);
            if (it < nsteps && e->k[r] < e->desc[r].nsteps) active.push_back(r);
        }
        if (active.empty() && measuring.empty()) break;
        smp.reserve(measuring.size());
        for (int r = 0; r < e->n; ++r) {
            const bool adv = std::find(active.begin(), active.end(), r) != active.end();
            const bool m = std::find(measuring.begin(), measuring.end(), r) != measuring.end();
            if (!adv && !m) continue;
            Lat<R> v = e->view<R>(r, e->j);
            launch_step<R>(v, (adv ? kStore : 0) | (m ? kMeasure : 0), e->launch, nullptr, e->j, e->stream);
            if (m)
                jobs.push_back(FinalizeJobHost{e->part.p + e->poff[r], e->nrp(r),
                                               (double)e->desc[r].Lx * (double)e->desc[r].Ly, smp.take(r)});
        }
        flush_finalize(e, smp, jobs);
        for (int r : active) e->k[r] += 1;
        if (!active.empty()) e->j += 1;
    }
}

// Batched loop: the steps every active replica takes before the next sample
// or end of any of them form a chunk; large replicas advance through one
// tile-table launch per step (after the chunk's first step, runs of 4m steps
// as batched two-step passes for the FP32 replicas whose width that pass
// takes), small FP32 replicas through one whole-in-LDS launch per chunk on a
// second stream.
template <typename R>
static void ens_step_batched(xyl_ensemble* e, uint64_t nsteps, EnsSamples& smp) {
    std::vector<FinalizeJobHost> jobs;
    const bool have_lds = std::any_of(e->lds.begin(), e->lds.end(), [](char c) { return c != 0; });
    if (have_lds) {
        check_hip(hipEventRecord(e->ev_main, e->stream), "hipEventRecord");
        check_hip(hipStreamWaitEvent(e->side, e->ev_main, 0), "hipStreamWaitEvent");
    }
    uint64_t it = 0;
    while (true) {
        std::vector<int> active_g, meas_g, only_meas_g, lds_set;
        std::vector<char> meas(e->n, 0), act(e->n, 0);
        bool any = false;
        for (int r = 0; r < e->n; ++r) {
            meas[r] = smp.wants(r);
            act[r] = it < nsteps && e->k[r] < e->desc[r].nsteps;
            if (!meas[r] && !act[r]) continue;
            any = true;
            if (e->lds[r]) {
                lds_set.push_back(r);
            } else if (act[r]) {
                active_g.push_back(r);
                if (meas[r]) meas_g.push_back(r);
            } else {
                only_meas_g.push_back(r);
            }
        }
        if (!any) break;
        uint64_t chunk = 0;
        bool any_active = false;
        for (int r = 0; r < e->n; ++r) {
            if (!act[r]) continue;
            uint64_t c = std::min<uint64_t>(nsteps - it, e->desc[r].nsteps - e->k[r]);
            if (smp.every) c = std::min<uint64_t>(c, smp.every - e->k[r] % smp.every);
            chunk = any_active ? std::min(chunk, c) : c;
            any_active = true;
        }
        size_t nmeas = 0;
        for (int r = 0; r < e->n; ++r) nmeas += meas[r];
        smp.reserve(nmeas);
        // small replicas: one launch for the whole chunk
        if (!lds_set.empty()) {
            // replicas with the factored FP32 kick first, then the others: one
            // launch per form of the kick
            const int b = e->lds_buf;
            e->lds_buf ^= 1;
            // table b was last read by the launch two chunks ago
            if (e->ev_lds_used[b]) check_hip(hipEventSynchronize(e->ev_lds[b]), "hipEventSynchronize");
            std::vector<LdsJobHost> jh;
            jh.reserve(lds_set.size());
            int nfact = 0;
            for (int pass = 0; pass < 2; ++pass)
                for (int r : lds_set) {
                    const xyl_replica_desc& d = e->desc[r];
                    const bool f = kick_factored(Params{d.Jx, d.Jy, d.h, d.gamma, d.dt, d.model, d.p});
                    if (f != (pass == 0)) continue;
                    nfact += f ? 1 : 0;
                    jh.push_back(LdsJobHost{r, meas[r] ? 1 : 0, act[r] ? (int32_t)chunk : 0, 0,
                                            meas[r] ? smp.take(r) : nullptr});
                }
            // (pinned table b's last copy went with that launch, so it is free)
            e->lds_jobs[b].reserve(jh.size());
            e->lds_jobs_host[b].reserve(jh.size());
            std::memcpy(e->lds_jobs_host[b].p, jh.data(), sizeof(LdsJobHost) * jh.size());
            check_hip(hipMemcpyAsync(e->lds_jobs[b].p, e->lds_jobs_host[b].p, sizeof(LdsJobHost) * jh.size(),
                                     hipMemcpyHostToDevice, e->side),
                      "H2D");
            e->lds_tab_host[b].reserve(e->n);
            Lat<float>* tab = e->lds_tab_host[b].p;
            for (int r = 0; r < e->n; ++r) tab[r] = e->view<float>(r, e->j);
            e->lds_reps[b].reserve(sizeof(Lat<float>) * e->n);
            check_hip(hipMemcpyAsync(e->lds_reps[b].p, tab, sizeof(Lat<float>) * e->n, hipMemcpyHostToDevice, e->side),
                      "H2D");
            const Lat<float>* lreps = reinterpret_cast<const Lat<float>*>(e->lds_reps[b].p);
            if (nfact)
                launch_ensemble_lds(lreps, e->lds_jobs[b].p, nfact, e->lds_threads, e->lds_max_sites, e->model(), true,
                                    e->j, e->side);
            if ((int)lds_set.size() > nfact)
                launch_ensemble_lds(lreps, e->lds_jobs[b].p + nfact, (int)lds_set.size() - nfact, e->lds_threads,
                                    e->lds_max_sites, e->model(), false, e->j, e->side);
            check_hip(hipEventRecord(e->ev_lds[b], e->side), "hipEventRecord");
            e->ev_lds_used[b] = true;
        }
        // large replicas
        if (!active_g.empty()) {
            if (active_g != e->task_active || e->tables_fusion != e->fusion) ens_upload_table<R>(e, e->j, active_g);
            const Lat<R>* reps = reinterpret_cast<const Lat<R>*>(e->reps.p);
            uint64_t c = 0;
            bool stepped = false;
            bool preforked = false;   // the later classes' first pass already issued (below)
            if (!meas_g.empty()) {
                // FP32 with two-step classes: the sample is a measurement
                // without a step, and the whole chunk runs in pairs of passes;
                // otherwise the chunk's first step carries the measurement
                bool passes = false;
                if constexpr (std::is_same<R, float>::value) passes = !e->s2cls.empty() && chunk >= 4;
                stepped = !passes;
                if constexpr (std::is_same<R, float>::value) {
                    // several classes issued directly: the classes after the
                    // first start their first pass beside the measurement (it
                    // reads the sampled state and writes the other buffers);
                    // their second pass, which overwrites that state, waits
                    // for the measurement's end
                    const size_t ncls = e->s2cls.size();
                    if (passes && ncls > 1 && e->use_graphs != 2) {
                        e->class_streams(ncls);
                        const float* ub = static_cast<const float*>(e->u);
                        float* u2b = reinterpret_cast<float*>(e->u2.p);
                        check_hip(hipEventRecord(e->cls_events[0], e->stream), "hipEventRecord");
                        for (size_t c2 = 1; c2 < ncls; ++c2) {
                            const auto& cl = e->s2cls[c2];
                            check_hip(hipStreamWaitEvent(e->cls_streams[c2 - 1], e->cls_events[0], 0),
                                      "hipStreamWaitEvent");
                            launch_ensemble_step2(reps, cl.tasks.p, cl.ntasks, cl.waves, cl.partial, cl.max_lx,
                                                  e->model(), 0, ub, u2b, nullptr, e->j, e->cls_streams[c2 - 1]);
                        }
                        preforked = true;
                    }
                }
                launch_ensemble_step<R>(reps, e->tasks.p, e->ntasks, passes ? kMeasure : (kStore | kMeasure),
                                        e->model(), e->launch.rows, e->launch.wpb, nullptr, e->j, e->stream);
                if (preforked)
                    check_hip(hipEventRecord(e->cls_events[e->s2cls.size()], e->stream), "hipEventRecord");
                for (int r : meas_g)
                    jobs.push_back(FinalizeJobHost{e->part.p + e->poff[r], e->nrp(r),
                                                   (double)e->desc[r].Lx * (double)e->desc[r].Ly, smp.take(r)});
                flush_finalize(e, smp, jobs);
                c = stepped ? 1 : 0;
            }
            // steps c0 .. c0 + n - 1 of the chunk, step offsets jb + c (with
            // kdev, jb = 0 and the device counter holds e->j)
            auto issue = [&](uint64_t c0, uint64_t n, const uint64_t* kdev, uint64_t jb, hipStream_t main) {
                uint64_t cc = c0;
                if constexpr (std::is_same<R, float>::value) {
                    const uint64_t n4 = n / 4 * 4;
                    if (n4 && !e->s2cls.empty()) {
                        e->u2.reserve(sizeof(float) * e->total);
                        const float* ub = static_cast<const float*>(e->u);
                        float* u2b = reinterpret_cast<float*>(e->u2.p);
                        const size_t ncls = e->s2cls.size();
                        e->class_streams(ncls);
                        // with `preforked` (a direct chunk of several classes,
                        // from its start), the later classes are forked and their
                        // first pass issued; their second waits for the sample
                        const bool pre = preforked && cc == 0 && kdev == nullptr;
                        if (ncls > 1 && !pre) {
                            check_hip(hipEventRecord(e->cls_events[0], main), "hipEventRecord");
                            for (size_t c2 = 1; c2 < ncls; ++c2)
                                check_hip(hipStreamWaitEvent(e->cls_streams[c2 - 1], e->cls_events[0], 0),
                                          "hipStreamWaitEvent");
                        }
                        // pass by pass across the classes: issued class by class, a
                        // class's first pass would wait for every pass of the
                        // classes before it to be issued (in a replayed graph,
                        // dispatched), and the classes would hardly overlap
                        for (uint64_t i = 0; i < n4; i += 4)
                            for (int ph = 0; ph < 2; ++ph)
                                for (size_t c2 = 0; c2 < ncls; ++c2) {
                                    const auto& cl = e->s2cls[c2];
                                    hipStream_t st = c2 == 0 ? main : e->cls_streams[c2 - 1];
                                    if (pre && c2 > 0 && i == 0) {
                                        if (ph == 0) continue;   // issued before the sample
                                        check_hip(hipStreamWaitEvent(st, e->cls_events[ncls], 0),
                                                  "hipStreamWaitEvent");
                                    }
                                    launch_ensemble_step2(reps, cl.tasks.p, cl.ntasks, cl.waves, cl.partial,
                                                          cl.max_lx, e->model(), ph, ub, u2b, kdev,
                                                          jb + cc + i + 2 * ph, st);
                                }
                        for (size_t c2 = 1; c2 < ncls; ++c2) {
                            check_hip(hipEventRecord(e->cls_events[c2], e->cls_streams[c2 - 1]), "hipEventRecord");
                            check_hip(hipStreamWaitEvent(main, e->cls_events[c2], 0), "hipStreamWaitEvent");
                        }
                        if (e->ntasks_rest)
                            for (uint64_t i = 0; i < n4; ++i)
                                launch_ensemble_step<R>(reps, e->tasks_rest.p, e->ntasks_rest, kStore, e->model(),
                                                        e->launch.rows, e->launch.wpb, kdev, jb + cc + i, main);
                        cc += n4;
                    }
                }
                for (; cc < c0 + n; ++cc)
                    launch_ensemble_step<R>(reps, e->tasks.p, e->ntasks, kStore, e->model(), e->launch.rows,
                                            e->launch.wpb, kdev, jb + cc, main);
            };
            const uint64_t n = chunk - c;
            // launches the chunk's stepping takes
            uint64_t nl = n;
            if constexpr (std::is_same<R, float>::value)
                if (!e->s2cls.empty()) nl = n / 4 * 2 * e->s2cls.size() + n % 4 + (e->ntasks_rest ? n / 4 * 4 : 0);
            xyl_ensemble::ChunkGraph* cg = nullptr;
            bool graphs = e->use_graphs == 2;
            if constexpr (std::is_same<R, float>::value)
                graphs = graphs || (e->use_graphs == 1 && e->s2cls.size() <= 1);
            else
                graphs = graphs || e->use_graphs == 1;
            if (graphs && nl >= 8) {
                if (e->graphs_built_for != e->graph_version) {
                    e->drop_graphs();
                    e->graphs_built_for = e->graph_version;
                }
                // at most kMaxChunkGraphs chunk shapes hold a graph at a time
                // (adaptive sampling can meet many)
                constexpr size_t kMaxChunkGraphs = 32;
                if (!e->graphs.count({c, n}) && e->graphs.size() >= 4 * kMaxChunkGraphs) e->drop_graphs();
                cg = &e->graphs[{c, n}];
                if (!cg->exec && cg->seen + 1 >= 2) {
                    size_t held = 0;
                    for (auto& g : e->graphs) held += g.second.exec != nullptr;
                    if (held >= kMaxChunkGraphs) {
                        e->drop_graphs();
                        cg = &e->graphs[{c, n}];
                        cg->seen = 1;
                    }
                }
                if (!cg->exec && ++cg->seen >= 2) {
                    // everything that allocates or creates happens before the capture
                    if (!e->cap_stream)
                        check_hip(hipStreamCreateWithFlags(&e->cap_stream, hipStreamNonBlocking), "hipStreamCreate");
                    e->kc.reserve(1);
                    if (!e->s2cls.empty()) {
                        e->u2.reserve(sizeof(float) * e->total);
                        e->class_streams(e->s2cls.size());
                    }
                    hipGraph_t gr = nullptr;
                    check_hip(hipStreamBeginCapture(e->cap_stream, hipStreamCaptureModeThreadLocal),
                              "hipStreamBeginCapture");
                    try {
                        issue(c, n, e->kc.p, 0, e->cap_stream);
                    } catch (...) {
                        (void)hipStreamEndCapture(e->cap_stream, &gr);
                        if (gr) (void)hipGraphDestroy(gr);
                        throw;
                    }
                    check_hip(hipStreamEndCapture(e->cap_stream, &gr), "hipStreamEndCapture");
                    hipError_t err = hipGraphInstantiate(&cg->exec, gr, nullptr, nullptr, 0);
                    (void)hipGraphDestroy(gr);
                    check_hip(err, "hipGraphInstantiate");
                }
            }
            if (cg && cg->exec) {
                launch_set_counter(e->kc.p, e->j, e->stream);
                check_hip(hipGraphLaunch(cg->exec, e->stream), "hipGraphLaunch");
            } else {
                issue(c, n, nullptr, e->j, e->stream);
            }
        }
        // replicas that only take a sample (a call ending on a sample step):
        // one batched measurement over the task table when they are the
        // replicas it was built for (the same strips and sums as one launch
        // per replica, which took about 1 ms for the 288-replica ensemble)
        const bool batched_only = !only_meas_g.empty() && only_meas_g == e->task_active && e->ntasks > 0;
        if (batched_only)
            launch_ensemble_step<R>(reinterpret_cast<const Lat<R>*>(e->reps.p), e->tasks.p, e->ntasks, kMeasure,
                                    e->model(), e->launch.rows, e->launch.wpb, nullptr, e->j, e->stream);
        for (int r : only_meas_g) {
            if (!batched_only) {
                Lat<R> v = e->view<R>(r, e->j);
                launch_step<R>(v, kMeasure, e->launch, nullptr, e->j, e->stream);
            }
            jobs.push_back(FinalizeJobHost{e->part.p + e->poff[r], e->nrp(r),
                                           (double)e->desc[r].Lx * (double)e->desc[r].Ly, smp.take(r)});
        }
        flush_finalize(e, smp, jobs);
        if (!any_active) break;
        for (int r = 0; r < e->n; ++r)
            if (act[r]) e->k[r] += chunk;
        e->j += chunk;
        it += chunk;
    }
    if (have_lds) {
        check_hip(hipEventRecord(e->ev_side, e->side), "hipEventRecord");
        check_hip(hipStreamWaitEvent(e->stream, e->ev_side, 0), "hipStreamWaitEvent");
    }
}

// Launch shape of the tile launches, timed on scratch copies of the state of
// the replicas that use the tile path (graph-captured steps, as for lattices).
template <typename R>
static Launch ensemble_autotune_impl(xyl_ensemble* e) {
    std::vector<int> reps;
    for (int r = 0; r < e->n; ++r)
        if (!e->lds[r]) reps.push_back(r);
    if (reps.empty()) return e->launch;
    const size_t bytes = sizeof(R) * e->total;
    DevBuf<char> tmp;
    tmp.reserve(4 * bytes);   // angles (2), velocities, second velocities of the two-step passes
    for (int b = 0; b < 2; ++b)
        check_hip(hipMemcpyAsync(tmp.p + b * bytes, e->th[b], bytes, hipMemcpyDeviceToDevice, e->stream), "D2D");
    check_hip(hipMemcpyAsync(tmp.p + 2 * bytes, e->u, bytes, hipMemcpyDeviceToDevice, e->stream), "D2D");
    check_hip(hipMemcpyAsync(tmp.p + 3 * bytes, e->u, bytes, hipMemcpyDeviceToDevice, e->stream), "D2D");
    std::vector<Lat<R>> tab(e->n);
    for (int r = 0; r < e->n; ++r) {
        tab[r] = e->view<R>(r, 0);
        tab[r].th[0] = reinterpret_cast<R*>(tmp.p) + e->off[r];
        tab[r].th[1] = reinterpret_cast<R*>(tmp.p + bytes) + e->off[r];
        tab[r].u = reinterpret_cast<R*>(tmp.p + 2 * bytes) + e->off[r];
        tab[r].fresh_k = ~(uint64_t)0;
        tab[r].k_end = ~(uint64_t)0;
    }
    DevBuf<char> dtab;
    dtab.reserve(sizeof(Lat<R>) * e->n);
    check_hip(hipMemcpyAsync(dtab.p, tab.data(), sizeof(Lat<R>) * e->n, hipMemcpyHostToDevice, e->stream), "H2D");
    DevBuf<uint64_t> kc;
    kc.reserve(1);
    launch_set_counter(kc.p, 0, e->stream);
    check_hip(hipStreamSynchronize(e->stream), "hipStreamSynchronize");
    size_t sites = 0;
    for (int r : reps) sites += (size_t)e->desc[r].Lx * e->desc[r].Ly;
    const int steps = (int)std::max<double>(4.0, std::min<double>(256.0, 2.0e11 * 2e-3 / (double)sites));
    hipStream_t cap = nullptr;
    check_hip(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking), "hipStreamCreate");
    hipEvent_t e0, e1;
    check_hip(hipEventCreate(&e0), "hipEventCreate");
    check_hip(hipEventCreate(&e1), "hipEventCreate");
    DevBuf<Task> dtasks;
    Launch best = e->launch;
    float best_ms = 1e30f;
    const int rows_c[] = {1, 2, 4, 8, 16, 32};
    const int wpb_c[] = {1, 2, 4, 8};
    for (int rows : rows_c) {
        std::vector<Task> tk;
        for (int r : reps) {
            const int nxw = (e->desc[r].Lx + kWaveSites - 1) / kWaveSites;
            const int nstrips = (e->desc[r].Ly + rows - 1) / rows;
            for (int st = 0; st < nstrips; ++st)
                for (int x = 0; x < nxw; ++x) tk.push_back(Task{r, x, st, 0});
        }
        dtasks.reserve(tk.size());
        check_hip(hipMemcpy(dtasks.p, tk.data(), sizeof(Task) * tk.size(), hipMemcpyHostToDevice), "H2D");
        for (int w : wpb_c) {
            hipGraph_t g = nullptr;
            hipGraphExec_t ex = nullptr;
            check_hip(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
            for (int i = 0; i < steps; ++i)
                launch_ensemble_step<R>(reinterpret_cast<const Lat<R>*>(dtab.p), dtasks.p, (int)tk.size(), kStore,
                                        e->model(), rows, w, kc.p, (uint64_t)i, cap);
            check_hip(hipStreamEndCapture(cap, &g), "hipStreamEndCapture");
            hipError_t err = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            check_hip(err, "hipGraphInstantiate");
            check_hip(hipGraphLaunch(ex, e->stream), "hipGraphLaunch");
            float t = 1e30f;
            for (int rep = 0; rep < 2; ++rep) {
                check_hip(hipEventRecord(e0, e->stream), "hipEventRecord");
                check_hip(hipGraphLaunch(ex, e->stream), "hipGraphLaunch");
                check_hip(hipEventRecord(e1, e->stream), "hipEventRecord");
                check_hip(hipEventSynchronize(e1), "hipEventSynchronize");
                float ms = 0.f;
                check_hip(hipEventElapsedTime(&ms, e0, e1), "hipEventElapsedTime");
                t = std::min(t, ms);
            }
            (void)hipGraphExecDestroy(ex);
            if (t < best_ms) {
                best_ms = t;
                best.rows = rows;
                best.wpb = w;
            }
        }
    }
    // Steps per pass (FP32): the two-step classes' passes plus the tile steps
    // of the replicas outside them, against the best tile launch for every
    // step, over the same steps.
    if constexpr (std::is_same<R, float>::value) {
        std::vector<int> active;
        for (int r : reps)
            if (e->k[r] < e->desc[r].nsteps) active.push_back(r);
        const int fusion0 = e->fusion;
        const Launch launch0 = e->launch;
        e->launch = best;
        e->fusion = 2;
        if (!active.empty()) ens_upload_table<R>(e, e->j, active);
        if (!active.empty() && !e->s2cls.empty()) {
            const int steps4 = (steps + 3) / 4 * 4;
            const Lat<float>* dreps = reinterpret_cast<const Lat<float>*>(dtab.p);
            const float* ub = reinterpret_cast<const float*>(tmp.p + 2 * bytes);
            float* u2b = reinterpret_cast<float*>(tmp.p + 3 * bytes);
            auto time_graph = [&](auto&& body, int nsteps) {
                hipGraph_t g = nullptr;
                hipGraphExec_t ex = nullptr;
                check_hip(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
                body();
                check_hip(hipStreamEndCapture(cap, &g), "hipStreamEndCapture");
                hipError_t err = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
                (void)hipGraphDestroy(g);
                check_hip(err, "hipGraphInstantiate");
                check_hip(hipGraphLaunch(ex, e->stream), "hipGraphLaunch");
                float t = 1e30f;
                for (int rep = 0; rep < 2; ++rep) {
                    check_hip(hipEventRecord(e0, e->stream), "hipEventRecord");
                    check_hip(hipGraphLaunch(ex, e->stream), "hipGraphLaunch");
                    check_hip(hipEventRecord(e1, e->stream), "hipEventRecord");
                    check_hip(hipEventSynchronize(e1), "hipEventSynchronize");
                    float ms = 0.f;
                    check_hip(hipEventElapsedTime(&ms, e0, e1), "hipEventElapsedTime");
                    t = std::min(t, ms);
                }
                (void)hipGraphExecDestroy(ex);
                return t / (float)nsteps;
            };
            // the classes' passes as the stepping issues them: on their own
            // streams, pass by pass across the classes, where a chunk with
            // several classes runs direct; one after the other in a graph
            // otherwise
            const size_t ncls = e->s2cls.size();
            auto classes = [&](hipStream_t main, bool fork) {
                if (fork) {
                    e->class_streams(ncls);
                    check_hip(hipEventRecord(e->cls_events[0], main), "hipEventRecord");
                    for (size_t c2 = 1; c2 < ncls; ++c2)
                        check_hip(hipStreamWaitEvent(e->cls_streams[c2 - 1], e->cls_events[0], 0),
                                  "hipStreamWaitEvent");
                }
                for (int i = 0; i < steps4; i += 4)
                    for (int ph = 0; ph < 2; ++ph)
                        for (size_t c2 = 0; c2 < ncls; ++c2) {
                            const auto& cl = e->s2cls[c2];
                            launch_ensemble_step2(dreps, cl.tasks.p, cl.ntasks, cl.waves, cl.partial, cl.max_lx,
                                                  e->model(), ph, ub, u2b, kc.p, (uint64_t)(i + 2 * ph),
                                                  fork && c2 > 0 ? e->cls_streams[c2 - 1] : main);
                        }
                if (fork)
                    for (size_t c2 = 1; c2 < ncls; ++c2) {
                        check_hip(hipEventRecord(e->cls_events[c2], e->cls_streams[c2 - 1]), "hipEventRecord");
                        check_hip(hipStreamWaitEvent(main, e->cls_events[c2], 0), "hipStreamWaitEvent");
                    }
                if (e->ntasks_rest)
                    for (int i = 0; i < steps4; ++i)
                        launch_ensemble_step<R>(reinterpret_cast<const Lat<R>*>(dtab.p), e->tasks_rest.p,
                                                e->ntasks_rest, kStore, e->model(), best.rows, best.wpb, kc.p,
                                                (uint64_t)i, main);
            };
            const bool direct = e->use_graphs == 0 || (ncls > 1 && e->use_graphs == 1);
            float t2 = 1e30f;
            if (direct) {
                classes(e->stream, ncls > 1);
                for (int rep = 0; rep < 2; ++rep) {
                    check_hip(hipEventRecord(e0, e->stream), "hipEventRecord");
                    classes(e->stream, ncls > 1);
                    check_hip(hipEventRecord(e1, e->stream), "hipEventRecord");
                    check_hip(hipEventSynchronize(e1), "hipEventSynchronize");
                    float ms = 0.f;
                    check_hip(hipEventElapsedTime(&ms, e0, e1), "hipEventElapsedTime");
                    t2 = std::min(t2, ms / (float)steps4);
                }
            } else {
                t2 = time_graph([&] { classes(cap, false); }, steps4);
            }
            const float t1 = time_graph(
                [&] {
                    for (int i = 0; i < steps4; ++i)
                        launch_ensemble_step<R>(reinterpret_cast<const Lat<R>*>(dtab.p), e->tasks.p, e->ntasks,
                                                kStore, e->model(), best.rows, best.wpb, kc.p, (uint64_t)i, cap);
                },
                steps4);
            e->fusion = t2 < t1 ? 2 : 1;
        } else {
            e->fusion = fusion0;
        }
        e->launch = launch0;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipStreamDestroy(cap);
    return best;
}

extern "C" {

int xyl_ensemble_autotune(xyl_ensemble* e) {
    return guarded([&] {
        require(e != nullptr, XYL_EINVAL, "NULL handle");
        DeviceGuard g(e->device);
        e->launch = e->dtype == XYL_F64 ? ensemble_autotune_impl<double>(e) : ensemble_autotune_impl<float>(e);
        e->task_active.clear();   // rebuild the tile table with the new strip height
    });
}

int xyl_ensemble_get_launch(xyl_ensemble* e, int32_t* rows, int32_t* wpb) {
    return guarded([&] {
        require(e != nullptr, XYL_EINVAL, "NULL handle");
        if (rows) *rows = e->launch.rows;
        if (wpb) *wpb = e->launch.wpb;
    });
}

int xyl_ensemble_create(xyl_ensemble** out, const xyl_replica_desc* desc, int32_t n, int32_t dtype, int32_t device) {
    return guarded([&] {
        require(out != nullptr && desc != nullptr, XYL_EINVAL, "NULL argument");
        *out = nullptr;
        require(n >= 1, XYL_EINVAL, "need at least one replica");
        require(dtype == XYL_F32 || dtype == XYL_F64, XYL_EINVAL, "dtype must be XYL_F32 or XYL_F64");
        select_device(device);
        std::unique_ptr<xyl_ensemble> e(new xyl_ensemble());
        e->dtype = dtype;
        e->device = device;
        check_hip(hipDeviceGetAttribute(&e->cus, hipDeviceAttributeMultiprocessorCount, device), "hipDeviceGetAttribute");
        e->n = n;
        e->desc.assign(desc, desc + n);
        for (int r = 0; r < n; ++r) {
            const xyl_replica_desc& d = desc[r];
            validate_shape(d.Lx, d.Ly);
            validate_params(Params{d.Jx, d.Jy, d.h, d.gamma, d.dt, d.model, d.p});
            validate_model(d.model, d.p);
            require(d.model == desc[0].model, XYL_EINVAL, "all replicas of an ensemble must use the same model");
            (void)make_schedule(d.knot_step, d.knot_T, d.nknots, d.knot_gamma);
            e->off.push_back(e->total);
            // keep every replica's base 256-byte aligned
            const size_t N = (size_t)d.Lx * d.Ly;
            e->total += (N + 63) / 64 * 64;
            e->poff.push_back(e->ptotal);
            e->ptotal += part_elems(e->nrp(r));
        }
        const size_t bytes = elem_size(dtype) * e->total;
        for (int b = 0; b < 2; ++b) check_alloc(hipMalloc(&e->th[b], bytes), "hipMalloc theta");
        check_alloc(hipMalloc(&e->u, bytes), "hipMalloc velocity");
        e->part.reserve(e->ptotal);
        {
            size_t nph = 0;
            for (int r = 0; r < n; ++r)
                for (int L : {desc[r].Lx, desc[r].Ly})
                    if (e->phase_off.emplace(L, nph).second) nph += 2 * (size_t)L;
            e->phases.reserve(nph);
            for (const auto& t : e->phase_off) launch_phase_table(e->phases.p + t.second, t.first, nullptr);
            check_hip(hipStreamSynchronize(nullptr), "hipStreamSynchronize");
        }
        e->lds.assign(n, 0);
        for (int r = 0; r < n; ++r) {
            const int N = desc[r].Lx * desc[r].Ly;
            if (dtype == XYL_F32 && N <= kLdsMaxSites) {
                e->lds[r] = 1;
                e->lds_max_sites = std::max(e->lds_max_sites, N);
            }
        }
        if (e->lds_max_sites) {
            e->lds_threads = lds_threads(e->lds_max_sites);
            check_hip(hipStreamCreateWithFlags(&e->side, hipStreamNonBlocking), "hipStreamCreate");
            check_hip(hipEventCreateWithFlags(&e->ev_main, hipEventDisableTiming), "hipEventCreate");
            check_hip(hipEventCreateWithFlags(&e->ev_side, hipEventDisableTiming), "hipEventCreate");
            for (int b = 0; b < 2; ++b)
                check_hip(hipEventCreateWithFlags(&e->ev_lds[b], hipEventDisableTiming), "hipEventCreate");
        }
        e->k.assign(n, 0);
        e->fresh_k.assign(n, 0);
        e->last_sample.assign(n, 0);
        for (int r = 0; r < n; ++r) {
            if (dtype == XYL_F64) launch_init_random<double>(e->view<double>(r, 0), e->stream);
            else launch_init_random<float>(e->view<float>(r, 0), e->stream);
        }
        check_hip(hipStreamSynchronize(e->stream), "hipStreamSynchronize");
        *out = e.release();
    });
}

int xyl_ensemble_destroy(xyl_ensemble* e) {
    if (!e) return XYL_OK;
    return guarded([&] {
        DeviceGuard g(e->device);
        (void)hipStreamSynchronize(e->stream);
        if (e->side) (void)hipStreamSynchronize(e->side);
        for (int b = 0; b < 2; ++b)
            if (e->th[b]) (void)hipFree(e->th[b]);
        if (e->u) (void)hipFree(e->u);
        for (hipStream_t st : e->cls_streams) (void)hipStreamSynchronize(st);
        if (e->side) (void)hipStreamDestroy(e->side);
        if (e->ev_main) (void)hipEventDestroy(e->ev_main);
        if (e->ev_side) (void)hipEventDestroy(e->ev_side);
        for (int b = 0; b < 2; ++b)
            if (e->ev_lds[b]) (void)hipEventDestroy(e->ev_lds[b]);
        for (hipStream_t st : e->cls_streams) (void)hipStreamDestroy(st);
        for (hipEvent_t ev : e->cls_events) (void)hipEventDestroy(ev);
        e->drop_graphs();
        if (e->cap_stream) (void)hipStreamDestroy(e->cap_stream);
        delete e;
    });
}

int xyl_ensemble_set_stream(xyl_ensemble* e, void* stream) {
    return guarded([&] {
        require(e != nullptr, XYL_EINVAL, "NULL handle");
        e->stream = static_cast<hipStream_t>(stream);
    });
}

int xyl_ensemble_set_graphs(xyl_ensemble* e, int32_t enable) {
    return guarded([&] {
        require(e != nullptr, XYL_EINVAL, "NULL handle");
        require(enable >= 0 && enable <= 2, XYL_EINVAL, "enable must be 0, 1 or 2");
        e->use_graphs = enable;
    });
}

int xyl_ensemble_get_fusion(const xyl_ensemble* e, int32_t* steps_per_pass) {
    return guarded([&] {
        require(e != nullptr && steps_per_pass != nullptr, XYL_EINVAL, "NULL argument");
        *steps_per_pass = e->fusion;
    });
}

int xyl_ensemble_set_fusion(xyl_ensemble* e, int32_t steps_per_pass) {
    return guarded([&] {
        require(e != nullptr, XYL_EINVAL, "NULL handle");
        require(steps_per_pass == 1 || steps_per_pass == 2, XYL_EINVAL, "steps_per_pass must be 1 or 2");
        e->fusion = steps_per_pass;
    });
}

int xyl_ensemble_set_mode(xyl_ensemble* e, int32_t mode) {
    return guarded([&] {
        require(e != nullptr, XYL_EINVAL, "NULL handle");
        require(mode == 0 || mode == 1, XYL_EINVAL, "mode must be 0 or 1");
        e->mode = mode;
    });
}

int xyl_ensemble_step(xyl_ensemble* e, uint64_t nsteps, uint64_t every, xyl_obs* out, uint64_t cap, uint64_t* nout) {
    return guarded([&] {
        require(e != nullptr, XYL_EINVAL, "NULL handle");
        if (every) require(out != nullptr && nout != nullptr, XYL_EINVAL, "out/nout are NULL");
        DeviceGuard g(e->device);
        EnsSamples smp(e, every, cap, nout);
        if (e->mode == 1) {
            if (e->dtype == XYL_F64) ens_step_per_replica<double>(e, nsteps, smp);
            else ens_step_per_replica<float>(e, nsteps, smp);
        } else {
            if (e->dtype == XYL_F64) ens_step_batched<double>(e, nsteps, smp);
            else ens_step_batched<float>(e, nsteps, smp);
        }
        smp.finish(out, nout);
    });
}

int xyl_ensemble_get_state(xyl_ensemble* e, int32_t r, double* theta, double* omega, uint64_t* step) {
    return guarded([&] {
        require(e != nullptr && r >= 0 && r < e->n, XYL_EINVAL, "bad handle or replica");
        DeviceGuard g(e->device);
        const size_t N = (size_t)e->desc[r].Lx * e->desc[r].Ly;
        if (theta) {
            if (e->dtype == XYL_F64) to_host<double>(e->cur_theta(r), theta, N, e->stream);
            else to_host<float>(e->cur_theta(r), theta, N, e->stream);
        }
        if (omega) {
            const size_t es = elem_size(e->dtype);
            if (e->k[r] == e->fresh_k[r]) {
                void* up = static_cast<char*>(e->u) + es * e->off[r];
                if (e->dtype == XYL_F64) to_host<double>(up, omega, N, e->stream);
                else to_host<float>(up, omega, N, e->stream);
            } else {
                e->omega_buf.reserve(es * N);
                if (e->dtype == XYL_F64) {
                    Lat<double> v = e->view<double>(r, 0);
                    v.k_end = ~(uint64_t)0;
                    launch_step<double>(v, kOmega, e->launch, nullptr, e->k[r] - v.k_base, e->stream);
                    to_host<double>(e->omega_buf.p, omega, N, e->stream);
                } else {
                    Lat<float> v = e->view<float>(r, 0);
                    v.k_end = ~(uint64_t)0;
                    launch_step<float>(v, kOmega, e->launch, nullptr, e->k[r] - v.k_base, e->stream);
                    to_host<float>(e->omega_buf.p, omega, N, e->stream);
                }
            }
        }
        if (step) *step = e->k[r];
    });
}

int xyl_ensemble_set_state(xyl_ensemble* e, int32_t r, const double* theta, const double* omega, uint64_t step) {
    return guarded([&] {
        require(e != nullptr && r >= 0 && r < e->n, XYL_EINVAL, "bad handle or replica");
        require(theta != nullptr && omega != nullptr, XYL_EINVAL, "theta/omega are NULL");
        const size_t N = (size_t)e->desc[r].Lx * e->desc[r].Ly;
        const bool si = e->model() == kModelSI;
        const double wp = e->dtype == XYL_F64 ? Prec<double>::kHalfPi : (double)Prec<float>::kHalfPi;
        for (size_t i = 0; i < N; ++i) {
            require(std::isfinite(theta[i]) && std::fabs(theta[i]) <= 3.0 * M_PI && std::isfinite(omega[i]), XYL_EINVAL,
                    "state entries must be finite with |theta| <= 3 pi");
            if (si) {
                const double t = e->dtype == XYL_F64 ? theta[i] : (double)(float)theta[i];
                require(t >= -wp && t < wp, XYL_EINVAL, "theta entries must lie in [-pi/2, pi/2) for the SI model");
            }
        }
        DeviceGuard g(e->device);
        e->k[r] = step;
        e->fresh_k[r] = step;
        e->last_sample[r] = 0;
        e->task_active.clear();   // force a table rebuild
        const size_t es = elem_size(e->dtype);
        void* up = static_cast<char*>(e->u) + es * e->off[r];
        if (e->dtype == XYL_F64) {
            to_device<double>(e->cur_theta(r), theta, N, e->stream);
            to_device<double>(up, omega, N, e->stream);
        } else {
            to_device<float>(e->cur_theta(r), theta, N, e->stream);
            to_device<float>(up, omega, N, e->stream);
        }
    });
}

int xyl_ensemble_domains(xyl_ensemble* e, int32_t r, int32_t* labels, uint64_t* sizes, uint64_t* counts, uint64_t cap,
                         uint64_t* n_sizes, uint64_t* n_domains, uint64_t* max_size) {
    return guarded([&] {
        require(e != nullptr && r >= 0 && r < e->n, XYL_EINVAL, "bad handle or replica");
        DeviceGuard g(e->device);
        const xyl_replica_desc& d = e->desc[r];
        const int sx = d.Jx > 0.0, sy = d.Jy > 0.0;
        if (e->dtype == XYL_F64)
            run_domains<double>(static_cast<const double*>(e->cur_theta(r)), d.Lx, d.Ly, sx, sy, d.model, e->parent,
                                e->usz,
                                e->hist, e->stats, e->stream, labels, sizes, counts, cap, n_sizes, n_domains, max_size);
        else
            run_domains<float>(static_cast<const float*>(e->cur_theta(r)), d.Lx, d.Ly, sx, sy, d.model, e->parent,
                               e->usz,
                               e->hist, e->stats, e->stream, labels, sizes, counts, cap, n_sizes, n_domains, max_size);
    });
}

int xyl_ensemble_structure_factor(xyl_ensemble* e, int32_t r, int32_t axis, int32_t kmax, double* S) {
    return guarded([&] {
        require(e != nullptr && r >= 0 && r < e->n, XYL_EINVAL, "bad handle or replica");
        const xyl_replica_desc& d = e->desc[r];
        validate_sf(d.Lx, d.Ly, axis, kmax, S);
        DeviceGuard g(e->device);
        check_hip(hipStreamSynchronize(e->side), "hipStreamSynchronize");
        const int sx = d.Jx > 0.0, sy = d.Jy > 0.0;
        if (e->dtype == XYL_F64)
            structure_factor_into<double>(e->cur_theta(r), d.Lx, d.Ly, sx, sy, d.model, axis, kmax, e->dscratch,
                                          e->stream, S);
        else
            structure_factor_into<float>(e->cur_theta(r), d.Lx, d.Ly, sx, sy, d.model, axis, kmax, e->dscratch,
                                         e->stream, S);
    });
}

int xyl_ensemble_sync(xyl_ensemble* e) {
    return guarded([&] {
        require(e != nullptr, XYL_EINVAL, "NULL handle");
        DeviceGuard g(e->device);
        check_hip(hipStreamSynchronize(e->stream), "hipStreamSynchronize");
    });
}

}  // extern "C"

// ===================================================================== adjoint
template <typename R>
static void adjoint_forward_impl(xyl_lattice* h, uint64_t N, uint64_t K, uint64_t W, double* loss, uint64_t* run) {
    // the state (buffers, streams, captured backward graphs) is kept from one
    // forward run to the next, so repeated gradient evaluations reuse it
    if (!h->adj) h->adj = new AdjState();
    AdjState* a = static_cast<AdjState*>(h->adj);
    a->valid = false;
    const size_t bytes = sizeof(R) * h->N;
    a->k0 = h->k;
    a->N = N;
    a->K = K;
    a->W = W;
    const uint64_t S = (N + K - 1) / K;
    a->ckpt.reserve(S * 2 * bytes);
    a->obs.reserve(6 * W);
    const uint64_t kw = a->k0 + N - W + 1;   // first step of the loss window
    // the window's measurement partials, one block per step, reduced together
    // at the end (falls back to one reduction per step for huge lattices)
    const uint64_t stride = (uint64_t)h->nrowparts() * kNPart;
    const bool batched = (double)W * (double)stride * 8.0 <= 1.0e9;
    if (batched) a->win.reserve(W * stride);
    for (uint64_t s = 0; s < S; ++s) {
        char* slot = a->ckpt.p + s * 2 * bytes;
        check_hip(hipMemcpyAsync(slot, h->cur_theta(), bytes, hipMemcpyDeviceToDevice, h->stream), "D2D");
        check_hip(hipMemcpyAsync(slot + bytes, h->u, bytes, hipMemcpyDeviceToDevice, h->stream), "D2D");
        const uint64_t kend = a->k0 + std::min<uint64_t>((s + 1) * K, N);
        while (h->k < kend) {
            if (h->k >= kw) {
                if (batched) {
                    lattice_steps_mode<R>(h, kend - h->k, kStore | kMeasure, a->win.p, kw, stride);
                } else {
                    lattice_measure_into<R>(h, true, a->obs.p + 6 * (h->k - kw));
                }
            } else {
                lattice_steps<R>(h, std::min(kend, kw) - h->k);
            }
        }
    }
    if (batched) {
        // the last sample (step k0 + N) is a measurement without a step
        Lat<R> v = h->view<R>();
        v.part = a->win.p;
        v.part_k0 = kw;
        v.part_stride = stride;
        launch_step<R>(v, kMeasure, h->launch, nullptr, h->k, h->stream);
        launch_finalize_many(a->win.p, h->nrowparts(), stride, (double)h->N, a->obs.p, (int)W, h->stream);
    } else {
        lattice_measure_into<R>(h, false, a->obs.p + 6 * (W - 1));
    }
    std::vector<double> o(6 * W);
    check_hip(hipMemcpyAsync(o.data(), a->obs.p, sizeof(double) * 6 * W, hipMemcpyDeviceToHost, h->stream), "D2H");
    check_hip(hipStreamSynchronize(h->stream), "hipStreamSynchronize");
    a->m.resize(W);
    double L = 0.0;
    for (uint64_t i = 0; i < W; ++i) {
        a->m[i] = o[6 * i + 2];
        L += a->m[i] * a->m[i];
    }
    a->loss = L / (double)W;
    if (loss) *loss = a->loss;
    a->run = ++g_adj_runs;
    a->version = h->version;
    a->valid = true;
    if (run) *run = a->run;
}

// Gradients of the lattice's adjoint run into grad[4] (host, times `scale`) and dL/dth^{k0},
// dL/dw^{k0}: host float64 arrays (dth0, dom0) or, with dev_out, caller
// device buffers of precision out_f64 (written on the lattice's stream, times
// `scale`).
// Rows per strip of the two-step reverse pass (1, 2 or 4): 2, where its LDS
// fits (512^2: 4.9 us per step, against 5.1 with 1-row strips and 7.8 with
// single reverse steps; 768^2 and 1024^2 within 2% of single reverse steps);
// where it does not (FP64 rows above 568 sites), single reverse steps.
static int adjoint2_rows(const xyl_lattice* h) { return h->adj2_rows ? h->adj2_rows : 2; }

template <typename R>
static void adjoint_backward_impl(xyl_lattice* h, double* grad, void* dth0, void* dom0, bool dev_out, int out_f64,
                                  double scale) {
    AdjState* a = static_cast<AdjState*>(h->adj);
    const size_t bytes = sizeof(R) * h->N;
    const uint64_t N = a->N, K = a->K, W = a->W, k0 = a->k0;
    const uint64_t S = (N + K - 1) / K;
    // direct loss coefficients dL/dm_k * dm_k/d(eps cos th) = (2 m_k / W) / Nsites
    std::vector<double> cmh(N + 1, 0.0);
    for (uint64_t i = 0; i < W; ++i) cmh[N - W + 1 + i] = 2.0 * a->m[i] / (double)W / (double)h->N;
    a->cm.reserve(N + 1);
    check_hip(hipMemcpyAsync(a->cm.p, cmh.data(), sizeof(double) * (N + 1), hipMemcpyHostToDevice, h->stream), "H2D");
    Launch l = h->launch;
    l.wpb = std::min(l.wpb, 4);
    Lat<R> v = h->view<R>();
    // two reverse steps per pass where the rows fit one workgroup's LDS rings
    const int rows2 = adjoint2_rows(h);
    const bool fuse = h->adj_fusion == 2 && adjoint2_fits<R>(v, rows2);
    const int ntasks = adjoint_tasks<R>(v, l.rows, fuse ? rows2 : 0);
    a->gacc.reserve((size_t)ntasks * 4);
    check_hip(hipMemsetAsync(a->gacc.p, 0, sizeof(double) * ntasks * 4, h->stream), "hipMemsetAsync");
    a->lam.reserve(4 * bytes);
    R* lt[2] = {reinterpret_cast<R*>(a->lam.p), reinterpret_cast<R*>(a->lam.p + bytes)};
    R* lu[2] = {reinterpret_cast<R*>(a->lam.p + 2 * bytes), reinterpret_cast<R*>(a->lam.p + 3 * bytes)};
    launch_adjoint_seed<R>(v, static_cast<const R*>(h->cur_theta()), lt[0], lu[0], cmh[N], h->stream);
    int li = 0;
    const size_t seg_bytes = (K + 1) * 2 * bytes;
    a->seg.reserve(2 * seg_bytes);
    auto slot_th = [&](int b, uint64_t j) { return reinterpret_cast<R*>(a->seg.p + b * seg_bytes + j * 2 * bytes); };
    auto slot_u = [&](int b, uint64_t j) {
        return reinterpret_cast<R*>(a->seg.p + b * seg_bytes + j * 2 * bytes + bytes);
    };
    a->kseg.reserve(2);
    if (!a->side) {
        check_hip(hipStreamCreateWithFlags(&a->side, hipStreamNonBlocking), "hipStreamCreate");
        for (int b = 0; b < 2; ++b) {
            check_hip(hipEventCreateWithFlags(&a->ev_rec[b], hipEventDisableTiming), "hipEventCreate");
            check_hip(hipEventCreateWithFlags(&a->ev_rev[b], hipEventDisableTiming), "hipEventCreate");
        }
        check_hip(hipEventCreateWithFlags(&a->ev_start, hipEventDisableTiming), "hipEventCreate");
    }
    auto recompute_node = [&](int b, uint64_t j, const uint64_t* kdev, uint64_t kj, hipStream_t st) {
        Lat<R> w = v;
        w.pingpong = 0;
        w.th[0] = slot_th(b, j);
        w.th[1] = slot_th(b, j + 1);
        w.u = slot_u(b, j);
        w.u_out = slot_u(b, j + 1);
        launch_step<R>(w, kStore, h->launch, kdev, kj, st);
    };
    // two recompute steps per pass (storing the state after each) where the
    // forward's two-step pass takes the lattice whole-row: the same states
    bool rec2 = false;
    if constexpr (std::is_same<R, float>::value)
        rec2 = h->adj_fusion == 2 && v.fact == 1 && v.model == kModelXY && step2_shape(h->Lx, h->Ly);
    const int rows_rec2 = rec2 ? step2_rows(h) : 0;
    auto recompute_run = [&](int b, uint64_t len, const uint64_t* kdev, uint64_t kbase, hipStream_t st) {
        uint64_t j = 0;
        if constexpr (std::is_same<R, float>::value) {
            if (rec2)
                for (; j + 2 <= len; j += 2)
                    launch_step2_mid(v, slot_th(b, j), slot_u(b, j), slot_th(b, j + 1), slot_u(b, j + 1),
                                     slot_th(b, j + 2), slot_u(b, j + 2), rows_rec2, kdev, kbase + j, st);
        }
        for (; j < len; ++j) recompute_node(b, j, kdev, kbase + j, st);
    };
    auto reverse_node = [&](int b, uint64_t j, int parity, const uint64_t* kdev, uint64_t kj, hipStream_t st) {
        launch_adjoint_step<R>(v, slot_th(b, j), slot_u(b, j), lt[parity], lu[parity], lt[parity ^ 1],
                               lu[parity ^ 1], a->cm.p, k0, a->gacc.p, kdev, kj, l, st);
    };
    // reverse steps j+1 and j of the segment in one pass
    auto reverse2_node = [&](int b, uint64_t j, int parity, const uint64_t* kdev, uint64_t kj, hipStream_t st) {
        launch_adjoint_step2<R>(v, slot_th(b, j), slot_u(b, j), slot_th(b, j + 1), slot_u(b, j + 1), lt[parity],
                                lu[parity], lt[parity ^ 1], lu[parity ^ 1], a->cm.p, k0, a->gacc.p, kdev, kj, rows2,
                                st);
    };
    // the reverse steps len-1 .. 0 of a segment from adjoint buffer `parity`
    // (an odd one first, then pairs); returns the buffer they end in
    auto reverse_segment = [&](int b, uint64_t len, int parity, const uint64_t* kdev, uint64_t kbase,
                               hipStream_t st) {
        uint64_t j = len;
        if (fuse) {
            if (j % 2 == 1) {
                --j;
                reverse_node(b, j, parity, kdev, kbase + j, st);
                parity ^= 1;
            }
            while (j >= 2) {
                j -= 2;
                reverse2_node(b, j, parity, kdev, kbase + j, st);
                parity ^= 1;
            }
        } else {
            while (j-- > 0) {
                reverse_node(b, j, parity, kdev, kbase + j, st);
                parity ^= 1;
            }
        }
        return parity;
    };
    // Full segments of even length replay captured graphs whose step indices
    // come from device counters set to the segment's first step: one graph
    // per buffer for the K recompute steps, one per (buffer, adjoint parity)
    // for the K reverse steps.
    const bool use_graph = h->graph_steps > 1 && K % 2 == 0 && K <= 4096;
    // key: every kernel argument the graphs capture (the lattice view by value,
    // the buffers, the step base and the launch shapes)
    std::vector<uint64_t> key = {K, (uint64_t)(uintptr_t)a->seg.p, (uint64_t)(uintptr_t)a->lam.p,
                                 (uint64_t)(uintptr_t)a->cm.p, (uint64_t)(uintptr_t)a->gacc.p,
                                 (uint64_t)(uintptr_t)a->kseg.p, (uint64_t)l.rows, (uint64_t)l.wpb, (uint64_t)rows2,
                                 (uint64_t)fuse, (uint64_t)rec2, (uint64_t)rows_rec2,
                                 (uint64_t)h->launch.rows, (uint64_t)h->launch.wpb, (uint64_t)ntasks, k0};
    {
        Lat<R> vz{};
        std::memcpy(&vz, &v, sizeof(vz));
        const size_t nw = (sizeof(vz) + 7) / 8;
        std::vector<uint64_t> words(nw, 0);
        std::memcpy(words.data(), &vz, sizeof(vz));
        key.insert(key.end(), words.begin(), words.end());
    }
    if (key != a->graph_key) {
        a->drop_graphs();
        a->graph_key = key;
    }
    auto capture = [&](auto&& body) {
        hipGraph_t gr = nullptr;
        hipGraphExec_t ex = nullptr;
        check_hip(hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
        try {
            body();
        } catch (...) {
            (void)hipStreamEndCapture(h->cap_stream, &gr);
            if (gr) (void)hipGraphDestroy(gr);
            throw;
        }
        check_hip(hipStreamEndCapture(h->cap_stream, &gr), "hipStreamEndCapture");
        hipError_t e = hipGraphInstantiate(&ex, gr, nullptr, nullptr, 0);
        (void)hipGraphDestroy(gr);
        check_hip(e, "hipGraphInstantiate");
        return ex;
    };
    // segment s occupies buffer (S - 1 - s) & 1
    auto recompute_segment = [&](uint64_t s) {
        const int b = (int)((S - 1 - s) & 1);
        const uint64_t ks = k0 + s * K;
        const uint64_t len = std::min<uint64_t>(K, k0 + N - ks);
        const char* ck = a->ckpt.p + s * 2 * bytes;
        check_hip(hipMemcpyAsync(slot_th(b, 0), ck, bytes, hipMemcpyDeviceToDevice, a->side), "D2D");
        check_hip(hipMemcpyAsync(slot_u(b, 0), ck + bytes, bytes, hipMemcpyDeviceToDevice, a->side), "D2D");
        if (use_graph && len == K) {
            if (!a->rec_graph[b])
                a->rec_graph[b] = capture([&] {
                    recompute_run(b, K, a->kseg.p + 1, 0, h->cap_stream);
                });
            launch_set_counter(a->kseg.p + 1, ks, a->side);
            check_hip(hipGraphLaunch(a->rec_graph[b], a->side), "hipGraphLaunch");
        } else {
            recompute_run(b, len, nullptr, ks, a->side);
        }
        check_hip(hipEventRecord(a->ev_rec[b], a->side), "hipEventRecord");
    };
    // the side stream starts after everything issued so far (checkpoints, seed)
    check_hip(hipEventRecord(a->ev_start, h->stream), "hipEventRecord");
    check_hip(hipStreamWaitEvent(a->side, a->ev_start, 0), "hipStreamWaitEvent");
    recompute_segment(S - 1);
    for (uint64_t s = S; s-- > 0;) {
        const int b = (int)((S - 1 - s) & 1);
        if (s > 0) {
            // the next segment's buffer is free once the reverse that used it ended
            if (S - 1 - s >= 1) check_hip(hipStreamWaitEvent(a->side, a->ev_rev[b ^ 1], 0), "hipStreamWaitEvent");
            recompute_segment(s - 1);
        }
        check_hip(hipStreamWaitEvent(h->stream, a->ev_rec[b], 0), "hipStreamWaitEvent");
        const uint64_t ks = k0 + s * K;
        const uint64_t len = std::min<uint64_t>(K, k0 + N - ks);
        if (use_graph && len == K) {
            int end = li;
            if (!a->rev_graph[b][li])
                a->rev_graph[b][li] = capture([&] { end = reverse_segment(b, K, li, a->kseg.p, 0, h->cap_stream); });
            else
                end = fuse ? li ^ (int)((K / 2) & 1) : li;   // K even
            launch_set_counter(a->kseg.p, ks, h->stream);
            check_hip(hipGraphLaunch(a->rev_graph[b][li], h->stream), "hipGraphLaunch");
            li = end;
        } else {
            li = reverse_segment(b, len, li, nullptr, ks, h->stream);
        }
        check_hip(hipEventRecord(a->ev_rev[b], h->stream), "hipEventRecord");
    }
    constexpr int kR64 = sizeof(R) == 8 ? 1 : 0;
    if (dev_out) {
        // the state adjoints stay on the device: converted (and scaled) into
        // the caller's buffers on the lattice's stream
        if (dth0) launch_convert(lt[li], kR64, dth0, out_f64, h->N, scale, true, h->stream);
        if (dom0) launch_convert(lu[li], kR64, dom0, out_f64, h->N, scale, true, h->stream);
    }
    std::vector<double> g((size_t)ntasks * 4);
    check_hip(hipMemcpyAsync(g.data(), a->gacc.p, sizeof(double) * ntasks * 4, hipMemcpyDeviceToHost, h->stream),
              "D2H");
    if (!dev_out && dth0) {
        std::vector<R> t(h->N);
        check_hip(hipMemcpyAsync(t.data(), lt[li], bytes, hipMemcpyDeviceToHost, h->stream), "D2H");
        check_hip(hipStreamSynchronize(h->stream), "hipStreamSynchronize");
        double* o = static_cast<double*>(dth0);
        for (size_t i = 0; i < h->N; ++i) o[i] = (double)t[i];
    }
    if (!dev_out && dom0) {
        std::vector<R> t(h->N);
        check_hip(hipMemcpyAsync(t.data(), lu[li], bytes, hipMemcpyDeviceToHost, h->stream), "D2H");
        check_hip(hipStreamSynchronize(h->stream), "hipStreamSynchronize");
        double* o = static_cast<double*>(dom0);
        for (size_t i = 0; i < h->N; ++i) o[i] = (double)t[i];
    }
    check_hip(hipStreamSynchronize(h->stream), "hipStreamSynchronize");
    if (grad) {
        for (int p = 0; p < 4; ++p) grad[p] = 0.0;
        for (int t = 0; t < ntasks; ++t)
            for (int p = 0; p < 4; ++p) grad[p] += g[(size_t)t * 4 + p];
        if (dev_out)
            for (int p = 0; p < 4; ++p) grad[p] *= scale;
    }
}

extern "C" {

int xyl_adjoint_forward(xyl_lattice* h, uint64_t nsteps, uint64_t ckpt_every, uint64_t window, double* loss,
                        uint64_t* run) {
    return guarded([&] {
        require_init(h);
        require(nsteps >= 1, XYL_EINVAL, "nsteps must be >= 1");
        require(window >= 1 && window <= nsteps, XYL_EINVAL, "window must be in [1, nsteps]");
        require(ckpt_every >= 1, XYL_EINVAL, "ckpt_every must be >= 1");
        require(h->p.model == kModelXY, XYL_EUNSUPPORTED,
                "the adjoint needs a smooth force: the SI model's field jumps at the wrap point");
        DeviceGuard g(h->device);
        if (h->dtype == XYL_F64) adjoint_forward_impl<double>(h, nsteps, ckpt_every, window, loss, run);
        else adjoint_forward_impl<float>(h, nsteps, ckpt_every, window, loss, run);
    });
}

// The forward run `run` may be differentiated: it is the lattice's latest,
// and neither the state nor any parameter changed since.
static void require_adjoint_run(xyl_lattice* h, uint64_t run) {
    require_init(h);
    AdjState* a = static_cast<AdjState*>(h->adj);
    require(a != nullptr && a->valid, XYL_ESTATE, "no adjoint forward run to differentiate");
    require(run == a->run, XYL_ESTATE,
            "stale adjoint run: another xyl_adjoint_forward replaced its checkpoints on this lattice");
    require(h->k == a->k0 + a->N && h->version == a->version, XYL_ESTATE,
            "lattice was stepped, reset or reconfigured after xyl_adjoint_forward");
    require(h->p.model == kModelXY, XYL_EUNSUPPORTED, "the adjoint supports the XY model only");
}

int xyl_set_adjoint_fusion(xyl_lattice* h, int32_t steps_per_pass, int32_t rows) {
    return guarded([&] {
        require(h != nullptr, XYL_EINVAL, "NULL handle");
        require(steps_per_pass == 1 || steps_per_pass == 2, XYL_EINVAL, "steps_per_pass must be 1 or 2");
        require(rows == 0 || rows == 1 || rows == 2 || rows == 4, XYL_EINVAL, "rows per strip must be 0, 1, 2 or 4");
        h->adj_fusion = steps_per_pass;
        if (rows) h->adj2_rows = rows;
    });
}

int xyl_adjoint_backward(xyl_lattice* h, uint64_t run, double* grad, double* dtheta0, double* domega0) {
    return guarded([&] {
        require_adjoint_run(h, run);
        DeviceGuard g(h->device);
        if (h->dtype == XYL_F64) adjoint_backward_impl<double>(h, grad, dtheta0, domega0, false, 1, 1.0);
        else adjoint_backward_impl<float>(h, grad, dtheta0, domega0, false, 1, 1.0);
    });
}

int xyl_adjoint_backward_device(xyl_lattice* h, uint64_t run, double scale, double* grad, void* dtheta0,
                                void* domega0, int32_t dtype) {
    return guarded([&] {
        require_adjoint_run(h, run);
        require(dtype == XYL_F32 || dtype == XYL_F64, XYL_EINVAL, "dtype must be XYL_F32 or XYL_F64");
        require(std::isfinite(scale), XYL_EINVAL, "scale must be finite");
        DeviceGuard g(h->device);
        const int of64 = dtype == XYL_F64 ? 1 : 0;
        if (h->dtype == XYL_F64) adjoint_backward_impl<double>(h, grad, dtheta0, domega0, true, of64, scale);
        else adjoint_backward_impl<float>(h, grad, dtheta0, domega0, true, of64, scale);
    });
}

}  // extern "C"
