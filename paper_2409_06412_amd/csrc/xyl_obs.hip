// Measurements outside the step: the staggered rotor correlation function and
// the frozen-domain labelling.
#include <algorithm>

#include "xyl_device.hpp"
#include "xyl_domains.hpp"
#include "xyl_obs.hpp"

namespace xyl {

// --------------------------------------------------------- correlation
// C(r) = (1/N) sum_i eps_i eps_j cos(q (th_i - th_j)), j = i + r along one
// axis (App. C, two-point function of the rotors averaged over the lattice;
// q = 1 for XY, 2 for the Si mapping).  One workgroup per line (row for axis
// 0, column for axis 1) stages the line's staggered rotors (eps cos q th,
// eps sin q th) in LDS in FP64; thread r sums the line's products in index
// order.  A second pass sums the lines in order.
template <typename R>
__global__ __launch_bounds__(256) void k_corr_lines(const R* __restrict__ th, int Lx, int Ly, int sx, int sy,
                                                    double q, int axis, int rmax, double* __restrict__ part) {
    extern __shared__ double lds[];
    const int line = blockIdx.x;
    const int L = axis == 0 ? Lx : Ly;
    double* cs = lds;
    double* sn = lds + L;
    for (int p = threadIdx.x; p < L; p += blockDim.x) {
        const int x = axis == 0 ? p : line;
        const int y = axis == 0 ? line : p;
        const double t = (double)th[(size_t)y * Lx + x];
        const double e = (((x * sx) + (y * sy)) & 1) ? -1.0 : 1.0;
        double s, c;
        sincos(q * t, &s, &c);
        cs[p] = e * c;
        sn[p] = e * s;
    }
    __syncthreads();
    for (int r = threadIdx.x; r <= rmax; r += blockDim.x) {
        double acc = 0.0;
        for (int p = 0; p < L; ++p) {
            int q = p + r;
            if (q >= L) q -= L;
            acc += cs[p] * cs[q] + sn[p] * sn[q];
        }
        part[(size_t)line * (rmax + 1) + r] = acc;
    }
}

// Sum of the per-line rows part[l][0..rmax] over the lines, in two passes of
// fixed order: chunks of kLineChunk lines are summed in parallel (thread r of
// chunk c writes its sum into column r of the chunk's first row, which only it
// touches), then the chunk sums are added in chunk order.
constexpr int kLineChunk = 64;

__global__ void k_line_sum_chunks(double* __restrict__ part, int nlines, int rmax) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r > rmax) return;
    const int l0 = blockIdx.y * kLineChunk;
    const int l1 = min(l0 + kLineChunk, nlines);
    double acc = 0.0;
    // unrolled so that the loads are in flight together; the sum keeps line order
#pragma unroll 16
    for (int l = l0; l < l1; ++l) acc += part[(size_t)l * (rmax + 1) + r];
    part[(size_t)l0 * (rmax + 1) + r] = acc;
}

__global__ void k_corr_sum(const double* __restrict__ part, int nlines, int rmax, double N, double* __restrict__ out) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r > rmax) return;
    double acc = 0.0;
#pragma unroll 16
    for (int l = 0; l < nlines; l += kLineChunk) acc += part[(size_t)l * (rmax + 1) + r];
    out[r] = acc / N;
}

static void launch_line_sum(double* part, int nlines, int rmax, double N, double* out, hipStream_t s) {
    const dim3 g1((rmax + 256) / 256, (nlines + kLineChunk - 1) / kLineChunk);
    k_line_sum_chunks<<<g1, 256, 0, s>>>(part, nlines, rmax);
    check_hip(hipGetLastError(), "line sum launch");
    k_corr_sum<<<(rmax + 256) / 256, 256, 0, s>>>(part, nlines, rmax, N, out);
    check_hip(hipGetLastError(), "line sum launch");
}

// C(r) from the structure factor of a power-of-two axis (App. C: C and S are
// a Fourier pair along the axis): C(r) = (1/L) sum_{k<L} S(k) cos(2 pi k r / L)
// with S(L - k) = S(k), i.e. (1/L) [S(0) + (-1)^r S(L/2) + 2 sum_{0<k<L/2}
// S(k) cos(2 pi k r / L)].  One workgroup per r sums in a fixed order (strided
// partial sums, then a fixed tree); cos from the twiddle table tw.
__global__ __launch_bounds__(256) void k_corr_from_sf(const double* __restrict__ S, const double2* __restrict__ tw,
                                                      int L, double* __restrict__ out) {
    __shared__ double red[256];
    const int r = blockIdx.x;
    const int h = L / 2;
    double acc = 0.0;
    for (int k = 1 + (int)threadIdx.x; k < h; k += blockDim.x) acc += S[k] * tw[(k * r) & (L - 1)].x;
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double last = L >= 2 ? ((r & 1) ? -S[h] : S[h]) : 0.0;
        out[r] = (S[0] + last + 2.0 * red[0]) / (double)L;
    }
}

template <typename R>
void launch_correlation(const R* th, int Lx, int Ly, int sx, int sy, int model, int axis, int rmax, double* part,
                        double* out, hipStream_t s) {
    const int nlines = axis == 0 ? Ly : Lx;
    const int L = axis == 0 ? Lx : Ly;
    if ((L & (L - 1)) == 0) {
        const size_t N = (size_t)Lx * Ly;
        double* z = part;
        double* spart = part + 2 * (N + (size_t)L);
        double* S = spart + (size_t)nlines * (L / 2 + 1);
        launch_structure_factor<R>(th, Lx, Ly, sx, sy, model, axis, L / 2, z, spart, S, s);
        k_corr_from_sf<<<rmax + 1, 256, 0, s>>>(S, reinterpret_cast<const double2*>(z) + N, L, out);
        check_hip(hipGetLastError(), "correlation kernel launch");
        return;
    }
    const size_t lds = 2 * sizeof(double) * (size_t)L;
    k_corr_lines<R><<<nlines, 256, lds, s>>>(th, Lx, Ly, sx, sy, model == kModelSI ? 2.0 : 1.0, axis, rmax, part);
    check_hip(hipGetLastError(), "correlation kernel launch");
    launch_line_sum(part, nlines, rmax, (double)Lx * (double)Ly, out, s);
}

// ------------------------------------------------- structure factor
// S_delta(k) = (1/N) sum over lines along delta of sum_kappa |s~^kappa_k|^2,
// s~^kappa_k = sum_r s^kappa_r exp(-2 pi i k r / L) (App. C, Eq.
// S-as-lattice-FT: the transform of C_delta(r), Eq. FT-Corr-delta).  Each
// line's two real rotor components are packed as one complex sequence
// z = eps (cos q th + i sin q th), whose transform Z gives
// sum_kappa |s~^kappa_k|^2 = (|Z_k|^2 + |Z_{L-k}|^2) / 2.
// Pass 1 writes z line-major (rows as they are; columns through a 32 x 32
// LDS transpose), pass 2 transforms one line per workgroup in LDS (Stockham
// passes of radix 16 for power-of-two L, a direct sum otherwise), pass 3
// sums the lines in a fixed order (launch_line_sum).  Power-of-two rows skip
// pass 1: the transform computes their rotors as it reads them.  zbuf holds
// N + L complex values: the lines, then the twiddle table.
template <typename R>
__global__ __launch_bounds__(256) void k_rotor_rows(const R* __restrict__ th, int Lx, int Ly, int sx, int sy,
                                                    double q, double2* __restrict__ z) {
    const size_t N = (size_t)Lx * Ly;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (size_t)gridDim.x * blockDim.x) {
        const int y = (int)(i / (size_t)Lx), x = (int)(i - (size_t)y * Lx);
        const double e = (((x * sx) + (y * sy)) & 1) ? -1.0 : 1.0;
        double sn, cs;
        sincos(q * (double)th[i], &sn, &cs);
        z[i] = make_double2(e * cs, e * sn);
    }
}

template <typename R>
__global__ __launch_bounds__(256) void k_rotor_cols(const R* __restrict__ th, int Lx, int Ly, int sx, int sy,
                                                    double q, double2* __restrict__ z) {
    __shared__ double2 tile[32][33];
    const int x0 = blockIdx.x * 32, y0 = blockIdx.y * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 32 x 8
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int x = x0 + tx, y = y0 + ty + 8 * j;
        if (x < Lx && y < Ly) {
            const double e = (((x * sx) + (y * sy)) & 1) ? -1.0 : 1.0;
            double sn, cs;
            sincos(q * (double)th[(size_t)y * Lx + x], &sn, &cs);
            tile[ty + 8 * j][tx] = make_double2(e * cs, e * sn);
        }
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int x = x0 + ty + 8 * j, y = y0 + tx;
        if (x < Lx && y < Ly) z[(size_t)x * Ly + y] = tile[tx][ty + 8 * j];
    }
}

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
    return make_double2(fma(a.x, b.x, -(a.y * b.y)), fma(a.x, b.y, a.y * b.x));
}
__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }

// tw[m] = exp(-2 pi i m / L), m < L: the twiddle table of one transform length
__global__ void k_sf_twiddles(double2* __restrict__ tw, int L) {
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m < L) {
        double sn, cs;
        sincospi(2.0 * (double)m / (double)L, &sn, &cs);
        tw[m] = make_double2(cs, -sn);
    }
}

// LDS slot of element i: one 16-B pad after every 16 elements, so that the
// strided stores of the early passes spread over the banks.
__device__ __forceinline__ int sf_slot(int i) { return i + (i >> 4); }

constexpr int bit_reverse_c(int q, int bits) {
    int r = 0;
    for (int b = 0; b < bits; ++b) r |= ((q >> b) & 1) << (bits - 1 - b);
    return r;
}
constexpr int log2_c(int n) { return n <= 1 ? 0 : 1 + log2_c(n / 2); }

// R-point DFT in registers, natural order in and out: radix-2 decimation in
// frequency (its result comes out bit-reversed and is read back through the
// bit reversal).  w_R^m = tw[m L / R].
template <int R>
__device__ __forceinline__ void dft_regs(double2 v[R], const double2* __restrict__ tw, int L) {
#pragma unroll
    for (int span = R / 2; span >= 1; span >>= 1) {
#pragma unroll
        for (int i0 = 0; i0 < R; i0 += 2 * span) {
#pragma unroll
            for (int j = 0; j < span; ++j) {
                const double2 a = v[i0 + j], b = v[i0 + j + span];
                v[i0 + j] = cadd(a, b);
                // w_{2 span}^j = exp(-2 pi i j / (2 span)) = tw[j L / (2 span)]
                v[i0 + j + span] = j == 0 ? csub(a, b) : cmul(csub(a, b), tw[j * (L / (2 * span))]);
            }
        }
    }
    double2 t[R];
#pragma unroll
    for (int q = 0; q < R; ++q) t[q] = v[bit_reverse_c(q, log2_c(R))];
#pragma unroll
    for (int q = 0; q < R; ++q) v[q] = t[q];
}

// One Stockham pass of radix R over a line of L points held in LDS (or, for
// the first pass, produced by `first`), with Ns the product of the radices of
// the passes before it: group j (of L / R) takes the points j + r L / R,
// multiplies point r by w^(r (j mod Ns)) with w = exp(-2 pi i / (Ns R)), takes
// their R-point DFT and stores output q at (j - j mod Ns) R + j mod Ns + q Ns.
// After the last pass the line holds its transform in natural order.  Every
// group of the pass is loaded before any is stored (L / R <= blockDim.x), so
// the pass runs in place.
template <int R, typename Src>
__device__ __forceinline__ void sf_pass(const Src& first, double2* buf, const double2* __restrict__ tw, int L,
                                        int Ns) {
    const int G = L / R;
    const int j = threadIdx.x;
    const bool act = j < G;
    double2 v[R];
    if (act) {
#pragma unroll
        for (int r = 0; r < R; ++r) v[r] = Ns == 1 ? first(j + r * G) : buf[sf_slot(j + r * G)];
        if (Ns > 1) {
            // w^r for r = 1 .. R-1 from one table load: w^2 = w w, w^3 = w^2 w, ...
            const double2 w1 = tw[(j & (Ns - 1)) * (L / (Ns * R))];
            double2 w = w1;
#pragma unroll
            for (int r = 1; r < R; ++r) {
                v[r] = cmul(v[r], w);
                w = cmul(w, w1);
            }
        }
        dft_regs<R>(v, tw, L);
    }
    __syncthreads();
    if (act) {
        const int k = j & (Ns - 1);
        const int base = (j - k) * R + k;
#pragma unroll
        for (int q = 0; q < R; ++q) buf[sf_slot(base + q * Ns)] = v[q];
    }
    __syncthreads();
}

// The transform of one line of L = 2^n points (2 .. 4096) by one workgroup of
// NT threads: Stockham passes of radix 16 with 256 threads, of radix 8 with
// 512 (half the registers per thread and twice the waves per CU for the
// 4096-point lines, whose 68 KiB of LDS allow two workgroups per CU), then
// one of 8, 4 or 2 for the rest of n; then sum_kappa |s~^kappa_k|^2 for
// k <= kmax into out.  Every pass has L / R <= NT groups.
template <int NT, typename Src>
__device__ __forceinline__ void sf_line(const Src& src, double2* sm, const double2* __restrict__ tw, int L, int kmax,
                                        double* __restrict__ out) {
    constexpr int RMAX = NT >= 512 ? 8 : 16;
    int Ns = 1;
    while (Ns < L) {
        const int left = L / Ns;
        if (left >= RMAX) {
            sf_pass<RMAX>(src, sm, tw, L, Ns);
            Ns *= RMAX;
        } else if (left == 8) {
            sf_pass<8>(src, sm, tw, L, Ns);
            Ns *= 8;
        } else if (left == 4) {
            sf_pass<4>(src, sm, tw, L, Ns);
            Ns *= 4;
        } else {
            sf_pass<2>(src, sm, tw, L, Ns);
            Ns *= 2;
        }
    }
    for (int k = threadIdx.x; k <= kmax; k += blockDim.x) {
        const double2 a = sm[sf_slot(k)], b = sm[sf_slot((L - k) & (L - 1))];
        out[k] = 0.5 * (a.x * a.x + a.y * a.y + b.x * b.x + b.y * b.y);
    }
}

// Points of a line: complex values written by the rotor pass, or the staggered
// rotors of one lattice row computed on the fly (the same arithmetic as
// k_rotor_rows).
struct ZLine {
    const double2* z;
    __device__ double2 operator()(int i) const { return z[i]; }
};
template <typename R>
struct RotorRow {
    const R* th;   // the row
    int y, sx, sy;
    double q;
    __device__ double2 operator()(int x) const {
        const double e = (((x * sx) + (y * sy)) & 1) ? -1.0 : 1.0;
        double sn, cs;
        sincos(q * (double)th[x], &sn, &cs);
        return make_double2(e * cs, e * sn);
    }
};

// Power-of-two lines, one per workgroup: columns from the transposed rotor
// field z, rows straight from the angles.
// (512 threads: at most 128 VGPRs, so that two workgroups share a CU)
template <int NT>
__global__ __launch_bounds__(NT, NT >= 512 ? 4 : 1) void k_sf_fft(const double2* __restrict__ z, const double2* __restrict__ tw, int L,
                                               int kmax, double* __restrict__ part) {
    extern __shared__ double2 sm[];
    sf_line<NT>(ZLine{z + (size_t)blockIdx.x * L}, sm, tw, L, kmax, part + (size_t)blockIdx.x * (kmax + 1));
}
template <typename R, int NT>
__global__ __launch_bounds__(NT, NT >= 512 ? 4 : 1) void k_sf_fft_rows(const R* __restrict__ th, int sx, int sy, double q,
                                                    const double2* __restrict__ tw, int L, int kmax,
                                                    double* __restrict__ part) {
    extern __shared__ double2 sm[];
    const int y = blockIdx.x;
    sf_line<NT>(RotorRow<R>{th + (size_t)y * L, y, sx, sy, q}, sm, tw, L, kmax, part + (size_t)y * (kmax + 1));
}

// Other lengths: the direct sum, one line per workgroup, with the full-circle
// twiddle table in LDS.
__global__ __launch_bounds__(256) void k_sf_direct(const double2* __restrict__ z, int L, int kmax,
                                                   double* __restrict__ part) {
    extern __shared__ double2 sm[];
    double2* buf = sm;
    double2* tw = sm + L;   // tw[m] = exp(-2 pi i m / L)
    const double2* zl = z + (size_t)blockIdx.x * L;
    for (int m = threadIdx.x; m < L; m += blockDim.x) {
        double sn, cs;
        sincospi(2.0 * (double)m / (double)L, &sn, &cs);
        tw[m] = make_double2(cs, -sn);
    }
    double* out = part + (size_t)blockIdx.x * (kmax + 1);
    for (int i = threadIdx.x; i < L; i += blockDim.x) buf[i] = zl[i];
    __syncthreads();
    for (int k = threadIdx.x; k <= kmax; k += blockDim.x) {
        // A = Z_k = sum z_x w^(k x), B = Z_{L-k} = sum z_x conj(w)^(k x)
        double ar = 0.0, ai = 0.0, br = 0.0, bi = 0.0;
        int m = 0;
        for (int x = 0; x < L; ++x) {
            const double2 w = tw[m], v = buf[x];
            ar += v.x * w.x - v.y * w.y;
            ai += v.x * w.y + v.y * w.x;
            br += v.x * w.x + v.y * w.y;
            bi += v.y * w.x - v.x * w.y;
            m += k;
            if (m >= L) m -= L;
        }
        out[k] = 0.5 * (ar * ar + ai * ai + br * br + bi * bi);
    }
}

template <typename R>
void launch_structure_factor(const R* th, int Lx, int Ly, int sx, int sy, int model, int axis, int kmax, void* zbuf,
                             double* part, double* out, hipStream_t s) {
    const double q = model == kModelSI ? 2.0 : 1.0;
    double2* z = static_cast<double2*>(zbuf);
    const int L = axis == 0 ? Lx : Ly;
    const int nlines = axis == 0 ? Ly : Lx;
    const bool pow2 = (L & (L - 1)) == 0;
    if (pow2) {
        // rows go straight from the angles into the transform; columns are
        // transposed into z first
        double2* tw = z + (size_t)Lx * Ly;     // zbuf holds N + L complex values
        k_sf_twiddles<<<(L + 255) / 256, 256, 0, s>>>(tw, L);
        check_hip(hipGetLastError(), "twiddle kernel launch");
        const size_t lds = sizeof(double2) * (size_t)(L + L / 16);
        // rows of 4096 points with 512 threads (radix 8): 0.195 -> 0.174 ms per
        // 4096^2 axis; columns, read from the transposed rotors, stay at 256
        // (radix 16; 512 measured 4% slower there)
        const bool wide = L >= 4096 && axis == 0;
        if (axis == 0) {
            const void* kf = wide ? reinterpret_cast<const void*>(k_sf_fft_rows<R, 512>)
                                  : reinterpret_cast<const void*>(k_sf_fft_rows<R, 256>);
            check_hip(hipFuncSetAttribute(kf, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds),
                      "hipFuncSetAttribute");
            if (wide) k_sf_fft_rows<R, 512><<<nlines, 512, lds, s>>>(th, sx, sy, q, tw, L, kmax, part);
            else k_sf_fft_rows<R, 256><<<nlines, 256, lds, s>>>(th, sx, sy, q, tw, L, kmax, part);
        } else {
            const dim3 grid((Lx + 31) / 32, (Ly + 31) / 32);
            k_rotor_cols<R><<<grid, 256, 0, s>>>(th, Lx, Ly, sx, sy, q, z);
            check_hip(hipGetLastError(), "rotor kernel launch");
            const void* kf = wide ? reinterpret_cast<const void*>(k_sf_fft<512>)
                                  : reinterpret_cast<const void*>(k_sf_fft<256>);
            check_hip(hipFuncSetAttribute(kf, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds),
                      "hipFuncSetAttribute");
            if (wide) k_sf_fft<512><<<nlines, 512, lds, s>>>(z, tw, L, kmax, part);
            else k_sf_fft<256><<<nlines, 256, lds, s>>>(z, tw, L, kmax, part);
        }
        check_hip(hipGetLastError(), "structure factor kernel launch");
    } else {
        if (axis == 0) {
            const size_t N = (size_t)Lx * Ly;
            const unsigned nb = (unsigned)std::min<size_t>((N + 255) / 256, 65536);
            k_rotor_rows<R><<<nb, 256, 0, s>>>(th, Lx, Ly, sx, sy, q, z);
        } else {
            const dim3 grid((Lx + 31) / 32, (Ly + 31) / 32);
            k_rotor_cols<R><<<grid, 256, 0, s>>>(th, Lx, Ly, sx, sy, q, z);
        }
        check_hip(hipGetLastError(), "rotor kernel launch");
        const size_t lds = sizeof(double2) * (size_t)(2 * L);
        check_hip(hipFuncSetAttribute(reinterpret_cast<const void*>(k_sf_direct),
                                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds),
                  "hipFuncSetAttribute");
        k_sf_direct<<<nlines, 256, lds, s>>>(z, L, kmax, part);
        check_hip(hipGetLastError(), "structure factor kernel launch");
    }
    launch_line_sum(part, nlines, kmax, (double)Lx * (double)Ly, out, s);
}

// -------------------------------------------------------------- domains
// Spin of site (x, y), decided in the state precision: eps * (|th| <= pi_p/2
// ? +1 : -1) (the sign of cos th, XY) or eps * (th >= 0 ? +1 : -1) (the sign
// of sin 2th on the half circle, SI).
template <typename R>
__device__ __forceinline__ int spin_of(const R* th, int Lx, int x, int y, int sx, int sy, int model) {
    const R t = th[(size_t)y * Lx + x];
    const bool up = model == kModelSI ? t >= R(0) : (t <= Prec<R>::kHalfPi && t >= -Prec<R>::kHalfPi);
    const int s = up ? 1 : -1;
    return (((x * sx) + (y * sy)) & 1) ? -s : s;
}

__device__ __forceinline__ int32_t uf_load(const int32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ int32_t uf_find(const int32_t* parent, int32_t a) {
    int32_t p = uf_load(parent + a);
    while (p != a) {
        a = p;
        p = uf_load(parent + a);
    }
    return a;
}

// Union with monotone links (the larger root is hooked under the smaller by
// atomicMin; parent[i] <= i always, so every find terminates).  If the hook
// finds that another thread re-parented that root first (to `old`), atomicMin
// may have replaced the link to `old` by the link to the other root, so the
// loop goes on uniting `old` with the other root: no connection is lost
// (Playne and Hawick, IEEE TPDS 2018).  The surviving root of a cluster is its
// smallest index.
__device__ __forceinline__ void uf_union(int32_t* parent, int32_t a, int32_t b) {
    while (true) {
        a = uf_find(parent, a);
        b = uf_find(parent, b);
        if (a == b) return;
        if (a < b) {
            const int32_t t = a;
            a = b;
            b = t;
        }
        // a > b: hook root a under b
        const int32_t old = atomicMin(parent + a, b);
        if (old == a) return;
        a = old;
    }
}

// The same find and union on a workgroup's LDS labels.
__device__ __forceinline__ int32_t uf_lds_load(const int32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ int32_t uf_lds_find(const int32_t* lab, int32_t a) {
    int32_t p = uf_lds_load(lab + a);
    while (p != a) {
        a = p;
        p = uf_lds_load(lab + a);
    }
    return a;
}
__device__ __forceinline__ void uf_lds_union(int32_t* lab, int32_t a, int32_t b) {
    while (true) {
        a = uf_lds_find(lab, a);
        b = uf_lds_find(lab, b);
        if (a == b) return;
        if (a < b) {
            const int32_t t = a;
            a = b;
            b = t;
        }
        const int32_t old = atomicMin(lab + a, b);
        if (old == a) return;
        a = old;
    }
}

// Labelling in two levels.  First every kUfTile x kUfTile tile is labelled in
// LDS with the bonds that lie inside it: a tile's sites in row-major order are
// in the lattice's index order, so the smallest local index of a piece is also
// its smallest lattice index, and parent[i] = that index keeps parent[i] <= i.
// Then only the bonds across a tile's right and bottom edges (the periodic
// wrap among them) are united in global memory, a few percent of all bonds
// (every bond on the global atomics before).
constexpr int kUfTile = 32;

template <typename R>
__global__ __launch_bounds__(256) void k_uf_local(const R* __restrict__ th, int Lx, int Ly, int sx, int sy,
                                                  int model, int ntx, int32_t* parent, uint32_t* size) {
    __shared__ int32_t lab[kUfTile * kUfTile];
    __shared__ int8_t spin[kUfTile * kUfTile];
    const int tx = (int)(blockIdx.x % (unsigned)ntx), ty = (int)(blockIdx.x / (unsigned)ntx);
    const int x0 = tx * kUfTile, y0 = ty * kUfTile;
    const int w = min(kUfTile, Lx - x0), h = min(kUfTile, Ly - y0);
    for (int l = threadIdx.x; l < kUfTile * kUfTile; l += blockDim.x) {
        const int ly = l / kUfTile, lx = l % kUfTile;
        lab[l] = l;
        spin[l] = (lx < w && ly < h) ? (int8_t)spin_of(th, Lx, x0 + lx, y0 + ly, sx, sy, model) : (int8_t)0;
    }
    __syncthreads();
    for (int l = threadIdx.x; l < kUfTile * kUfTile; l += blockDim.x) {
        const int ly = l / kUfTile, lx = l % kUfTile;
        if (lx >= w || ly >= h) continue;
        const int8_t s = spin[l];
        if (lx + 1 < w && spin[l + 1] == s) uf_lds_union(lab, l, l + 1);
        if (ly + 1 < h && spin[l + kUfTile] == s) uf_lds_union(lab, l, l + kUfTile);
    }
    __syncthreads();
    for (int l = threadIdx.x; l < kUfTile * kUfTile; l += blockDim.x) {
        const int ly = l / kUfTile, lx = l % kUfTile;
        if (lx >= w || ly >= h) continue;
        const int32_t r = uf_lds_find(lab, l);
        const size_t gi = (size_t)(y0 + ly) * Lx + (size_t)(x0 + lx);
        parent[gi] = (int32_t)((size_t)(y0 + r / kUfTile) * Lx + (size_t)(x0 + r % kUfTile));
        size[gi] = 0u;
    }
}

// Bonds across tile edges: thread t < ntx Ly takes the right edge of tile
// column t / Ly in row t % Ly (the last column's bond wraps to x = 0); the
// next nty Lx threads take the bottom edges of the tile rows (the last row's
// bond wraps to y = 0).
template <typename R>
__global__ void k_uf_boundary(const R* __restrict__ th, int Lx, int Ly, int sx, int sy, int model, int ntx, int nty,
                              int32_t* parent) {
    const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t nr = (size_t)ntx * Ly;
    int x, y, xn, yn;
    if (t < nr) {
        const int tx = (int)(t / (size_t)Ly);
        y = (int)(t % (size_t)Ly);
        x = min((tx + 1) * kUfTile, Lx) - 1;
        xn = x + 1 == Lx ? 0 : x + 1;
        yn = y;
    } else if (t < nr + (size_t)nty * Lx) {
        const size_t u = t - nr;
        const int ty = (int)(u / (size_t)Lx);
        x = (int)(u % (size_t)Lx);
        y = min((ty + 1) * kUfTile, Ly) - 1;
        xn = x;
        yn = y + 1 == Ly ? 0 : y + 1;
    } else {
        return;
    }
    if (spin_of(th, Lx, x, y, sx, sy, model) == spin_of(th, Lx, xn, yn, sx, sy, model))
        uf_union(parent, (int32_t)((size_t)y * Lx + x), (int32_t)((size_t)yn * Lx + xn));
}

// Labels and sizes per tile, after the edge merge.  Only roots had their
// parent changed by the merge, so a site's parent is its tile-local root or,
// for a local root, itself or the root it was hooked under.  In LDS each site
// points at its parent where that lies in the tile (an index no larger than
// its own); a chain ends at a root of the whole lattice or at a site whose
// parent lies outside the tile, which takes one find in global memory.  Every
// site's label is its chain end's, and each chain end adds its count of
// sites to its root's size once.  Concurrent finds from other tiles see a
// site's old parent or its root, both ancestors, so they still end at the
// root.
// Launched with 256 threads per tile (each thread keeps the chain ends of its
// TILE^2 / 256 sites in registers).
template <int TILE>
__global__ __launch_bounds__(256) void k_uf_flatten_tiles(int32_t* parent, uint32_t* size, int Lx, int Ly, int ntx) {
    static_assert(TILE * TILE % 256 == 0, "whole sites per thread");
    __shared__ int32_t nxt[TILE * TILE];
    __shared__ int32_t fin[TILE * TILE];
    __shared__ uint32_t cnt[TILE * TILE];
    const int tx = (int)(blockIdx.x % (unsigned)ntx), ty = (int)(blockIdx.x / (unsigned)ntx);
    const int x0 = tx * TILE, y0 = ty * TILE;
    const int w = min(TILE, Lx - x0), h = min(TILE, Ly - y0);
    for (int l = threadIdx.x; l < TILE * TILE; l += blockDim.x) {
        const int ly = l / TILE, lx = l % TILE;
        cnt[l] = 0u;
        nxt[l] = l;
        if (lx >= w || ly >= h) continue;
        const size_t gi = (size_t)(y0 + ly) * Lx + (size_t)(x0 + lx);
        const int32_t p = uf_load(parent + gi);
        const int py = (int)((size_t)p / (size_t)Lx), px = (int)((size_t)p % (size_t)Lx);
        if ((size_t)p == gi) {
            fin[l] = p;                                        // a root of the lattice
        } else if (py >= y0 && py < y0 + h && px >= x0 && px < x0 + w) {
            nxt[l] = (py - y0) * TILE + (px - x0);             // in the tile: at most l
        } else {
            nxt[l] = -1;                                       // leaves the tile
            fin[l] = uf_find(parent, p);
        }
    }
    __syncthreads();
    // the chain ends of the thread's sites (nxt is not written in this phase)
    constexpr int kPer = TILE * TILE / 256;
    int ends[kPer];
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
        const int l = (int)threadIdx.x + 256 * k;
        const int ly = l / TILE, lx = l % TILE;
        ends[k] = -1;
        if (lx >= w || ly >= h) continue;
        int e = l;
        while (nxt[e] >= 0 && nxt[e] != e) e = nxt[e];
        atomicAdd(&cnt[e], 1u);
        ends[k] = e;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
        const int l = (int)threadIdx.x + 256 * k;
        if (ends[k] < 0) continue;
        const int ly = l / TILE, lx = l % TILE;
        const size_t gi = (size_t)(y0 + ly) * Lx + (size_t)(x0 + lx);
        __hip_atomic_store(parent + gi, fin[ends[k]], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (cnt[l]) atomicAdd(size + fin[l], cnt[l]);
    }
}

// After the flatten pass every parent is a root: histogram the cluster sizes
// of the roots.  Each workgroup takes a contiguous chunk of sites and counts
// sizes below kHistLds in LDS, flushing each nonzero bin with one atomic;
// larger sizes (few, and spread over many bins) go to the histogram directly.
// This keeps the many small domains from queueing on a few global addresses.
constexpr int kHistLds = 1024;
__global__ __launch_bounds__(256) void k_uf_finish(const int32_t* __restrict__ parent,
                                                   const uint32_t* __restrict__ size, uint32_t* hist, size_t N) {
    __shared__ uint32_t h[kHistLds];
    for (int b = threadIdx.x; b < kHistLds; b += blockDim.x) h[b] = 0u;
    __syncthreads();
    const size_t chunk = (N + gridDim.x - 1) / gridDim.x;
    const size_t i0 = (size_t)blockIdx.x * chunk;
    const size_t i1 = i0 + chunk < N ? i0 + chunk : N;
    for (size_t i = i0 + threadIdx.x; i < i1; i += blockDim.x) {
        if (parent[i] == (int32_t)i) {
            const uint32_t sz = size[i];
            if (sz < (uint32_t)kHistLds) atomicAdd(&h[sz], 1u);
            else atomicAdd(hist + sz, 1u);
        }
    }
    __syncthreads();
    for (int b = threadIdx.x; b < kHistLds; b += blockDim.x)
        if (h[b]) atomicAdd(hist + b, h[b]);
}

// The size distribution as (size, count) pairs: every nonzero histogram entry
// hist[sz], sz = 1..N, appends one pair from stats[kDomainPairs] on (stats[0]
// counts them; the order is arbitrary).  Distinct sizes sum to at most N, so
// there are at most `cap` >= sqrt(2 N) of them.
__global__ void k_uf_sizes(const uint32_t* __restrict__ hist, uint32_t* stats, size_t N, uint32_t cap) {
    const size_t sz = (size_t)blockIdx.x * blockDim.x + threadIdx.x + 1;
    if (sz > N) return;
    const uint32_t c = hist[sz];
    if (c == 0u) return;
    const uint32_t j = atomicAdd(stats, 1u);
    if (j < cap) {
        stats[kDomainPairs + 2 * (size_t)j] = (uint32_t)sz;
        stats[kDomainPairs + 2 * (size_t)j + 1] = c;
    }
}

template <typename R>
void launch_domains(const R* th, int Lx, int Ly, int sx, int sy, int model, int32_t* parent, uint32_t* size,
                    uint32_t* hist,
                    uint32_t* stats, hipStream_t s) {
    const size_t N = (size_t)Lx * Ly;
    const unsigned nb = (unsigned)((N + 255) / 256);
    const int ntx = (Lx + kUfTile - 1) / kUfTile, nty = (Ly + kUfTile - 1) / kUfTile;
    k_uf_local<R><<<(unsigned)((size_t)ntx * nty), 256, 0, s>>>(th, Lx, Ly, sx, sy, model, ntx, parent, size);
    check_hip(hipGetLastError(), "uf local labelling launch");
    const size_t nbond = (size_t)ntx * Ly + (size_t)nty * Lx;
    k_uf_boundary<R><<<(unsigned)((nbond + 255) / 256), 256, 0, s>>>(th, Lx, Ly, sx, sy, model, ntx, nty, parent);
    check_hip(hipGetLastError(), "uf boundary merge launch");
    k_uf_flatten_tiles<kUfTile><<<(unsigned)((size_t)ntx * nty), 256, 0, s>>>(parent, size, Lx, Ly, ntx);
    check_hip(hipGetLastError(), "uf flatten launch");
    k_uf_finish<<<(unsigned)std::min<size_t>(nb, 1024), 256, 0, s>>>(parent, size, hist, N);
    check_hip(hipGetLastError(), "uf finish launch");
    k_uf_sizes<<<nb, 256, 0, s>>>(hist, stats, N, domain_size_cap(N));
    check_hip(hipGetLastError(), "uf sizes launch");
}

template void launch_correlation<float>(const float*, int, int, int, int, int, int, int, double*, double*,
                                        hipStream_t);
template void launch_correlation<double>(const double*, int, int, int, int, int, int, int, double*, double*,
                                         hipStream_t);
template void launch_structure_factor<float>(const float*, int, int, int, int, int, int, int, void*, double*,
                                             double*, hipStream_t);
template void launch_structure_factor<double>(const double*, int, int, int, int, int, int, int, void*, double*,
                                              double*, hipStream_t);
template void launch_domains<float>(const float*, int, int, int, int, int, int32_t*, uint32_t*, uint32_t*, uint32_t*,
                                    hipStream_t);
template void launch_domains<double>(const double*, int, int, int, int, int, int32_t*, uint32_t*, uint32_t*, uint32_t*,
                                     hipStream_t);

}  // namespace xyl
