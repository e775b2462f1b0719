// Device-side transfer of lattice states and gradients between caller-owned
// device buffers and the library's: validation of a caller's state where it
// lies, and element-wise conversion between binary32 and binary64 (with an
// optional FP64 scale factor, for gradients times an upstream derivative).
#include "xyl_device.hpp"

#include <algorithm>

namespace xyl {

// Each thread checks one site and ORs a bit into *flag for what it finds:
// angles must be finite with |th| <= 3 pi (a single 2 pi shift then brings a
// step's drift back into range), velocities finite, and, for the half-circle
// model, the angle rounded to the state precision inside [-pi_p/2, pi_p/2).
template <typename S>
__global__ void k_check_state(const S* __restrict__ th, const S* __restrict__ om, size_t n, int half_circle,
                              int state_f64, uint32_t* flag) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double t = (double)th[i], w = (double)om[i];
    uint32_t bad = 0u;
    if (!(isfinite(t) && fabs(t) <= 3.0 * Prec<double>::kPi)) bad |= kStateBadTheta;
    if (!isfinite(w)) bad |= kStateBadOmega;
    if (half_circle && !(bad & kStateBadTheta)) {
        const double r = state_f64 ? t : (double)(float)t;
        const double wp = state_f64 ? Prec<double>::kHalfPi : (double)Prec<float>::kHalfPi;
        if (!(r >= -wp && r < wp)) bad |= kStateBadHalfCircle;
    }
    if (bad) atomicOr(flag, bad);
}

// out[i] = in[i] rounded to D, or (in[i] * scale) in FP64 rounded to D.
template <typename S, typename D>
__global__ void k_convert(const S* __restrict__ in, D* __restrict__ out, size_t n, double scale, int scaled) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    out[i] = scaled ? (D)((double)in[i] * scale) : (D)in[i];
}

__global__ void k_fill_u32(uint32_t* p, size_t n, uint32_t v) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        p[i] = v;
}

static unsigned blocks_for(size_t n) { return (unsigned)((n + 255) / 256); }

void launch_check_state(const void* th, const void* om, int src_f64, size_t n, int half_circle, int state_f64,
                        uint32_t* flag, hipStream_t s) {
    if (n == 0) return;
    if (src_f64)
        k_check_state<double><<<blocks_for(n), 256, 0, s>>>(static_cast<const double*>(th),
                                                            static_cast<const double*>(om), n, half_circle,
                                                            state_f64, flag);
    else
        k_check_state<float><<<blocks_for(n), 256, 0, s>>>(static_cast<const float*>(th),
                                                           static_cast<const float*>(om), n, half_circle,
                                                           state_f64, flag);
    check_hip(hipGetLastError(), "state check launch");
}

void launch_convert(const void* in, int in_f64, void* out, int out_f64, size_t n, double scale, bool scaled,
                    hipStream_t s) {
    if (n == 0) return;
    const unsigned nb = blocks_for(n);
    const int sc = scaled ? 1 : 0;
    if (in_f64 && out_f64)
        k_convert<double, double><<<nb, 256, 0, s>>>(static_cast<const double*>(in), static_cast<double*>(out), n,
                                                     scale, sc);
    else if (in_f64)
        k_convert<double, float><<<nb, 256, 0, s>>>(static_cast<const double*>(in), static_cast<float*>(out), n,
                                                    scale, sc);
    else if (out_f64)
        k_convert<float, double><<<nb, 256, 0, s>>>(static_cast<const float*>(in), static_cast<double*>(out), n,
                                                    scale, sc);
    else
        k_convert<float, float><<<nb, 256, 0, s>>>(static_cast<const float*>(in), static_cast<float*>(out), n,
                                                   scale, sc);
    check_hip(hipGetLastError(), "convert launch");
}

void launch_fill_u32(uint32_t* p, size_t n, uint32_t v, hipStream_t s) {
    if (n == 0) return;
    const size_t nb = std::min<size_t>(blocks_for(n), 4096);
    k_fill_u32<<<(unsigned)nb, 256, 0, s>>>(p, n, v);
    check_hip(hipGetLastError(), "fill launch");
}

}  // namespace xyl
