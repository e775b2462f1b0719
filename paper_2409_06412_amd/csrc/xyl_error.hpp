// Error handling of the library's host code, free of any HIP header so that
// the pure-host parts build with a plain C++ compiler: inside the library a
// failure is an exception carrying an XYL_* status; `guarded` turns it into
// the C-ABI's return code and the thread's xyl_last_error() message.
#pragma once
#include <cstddef>
#include <new>
#include <stdexcept>
#include <string>

#include "../../include/xyl.h"

namespace xyl {

struct Error : std::runtime_error {
    int code;
    Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

extern thread_local std::string g_err;   // message of the thread's last failing call

inline void require(bool ok, int code, const std::string& msg) {
    if (!ok) throw Error(code, msg);
}

// Runs f; XYL_OK, or the status of what it threw (message in g_err).
template <typename F>
int guarded(F&& f) {
    try {
        g_err.clear();
        f();
        return XYL_OK;
    } catch (const Error& e) {
        g_err = e.what();
        return e.code;
    } catch (const std::bad_alloc&) {
        g_err = "host allocation failed";
        return XYL_ENOMEM;
    } catch (const std::exception& e) {
        g_err = e.what();
        return XYL_EDEVICE;
    } catch (...) {
        g_err = "unknown error";
        return XYL_EDEVICE;
    }
}

// Integrated autocorrelation time of f[0..n-1] in samples (automatic window
// of Madras and Sokal, c = 6; at least 1/2).  xyl_host.cpp.
double tau_int(const double* f, size_t n);

}  // namespace xyl
