// Scratch sizes of the observables' launchers, shared by the kernels and the
// host runtime.
#pragma once
#include <cstddef>

namespace xyl {

// Doubles of scratch launch_correlation needs.  Power-of-two axis lengths go
// through the structure factor (the complex lines and the twiddle table, the
// per-line spectra, S(k) for k <= L/2); other lengths keep the direct pair
// sums (one row of rmax + 1 per line).
inline size_t correlation_scratch(int Lx, int Ly, int axis, int rmax) {
    const size_t L = (size_t)(axis == 0 ? Lx : Ly), nlines = (size_t)(axis == 0 ? Ly : Lx);
    if ((L & (L - 1)) == 0) return 2 * ((size_t)Lx * Ly + L) + nlines * (L / 2 + 1) + (L / 2 + 1);
    return nlines * ((size_t)rmax + 1);
}

}  // namespace xyl
