"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (gcc,
CPU only): the FP64 oracle (oracle/xyo.c) and the library's pure-host
estimators (paper_2409_06412_amd/csrc/xyl_host.cpp), each linked into a small
driver that calls every function on small and degenerate inputs (the
smallest lattices, one sample, a single replica, fits and collapses that
must fail).  A sanitizer report, a leak or a wrong status fails the test."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
       "-ffp-contract=off"]

ORACLE_DRIVER = r"""
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include "xyo.h"

static int bad = 0;
#define CHECK(c) do { if (!(c)) { fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__); bad = 1; } } while (0)

static void finite_all(const double* x, size_t n) { for (size_t i = 0; i < n; ++i) CHECK(isfinite(x[i])); }

static void exercise(int Lx, int Ly, int model, double p, int shaped) {
    xyo_model m;
    memset(&m, 0, sizeof m);
    m.Lx = Lx; m.Ly = Ly;
    m.Jx = model ? -10.0 : 1.0; m.Jy = -0.1; m.h = model ? -1.0 : 0.5; m.gamma = 1.0; m.dt = 0.01;
    m.seed = 5; m.replica = 3; m.model = model; m.p = p;
    m.nknots = shaped ? 3 : 1;
    m.knot_step[0] = 0; m.knot_T[0] = 1.2; m.knot_gamma[0] = shaped ? 3 : 1;
    m.knot_step[1] = 20; m.knot_T[1] = 0.4; m.knot_gamma[1] = -2;
    m.knot_step[2] = 40; m.knot_T[2] = 0.0;
    const size_t N = (size_t)Lx * Ly;
    double* th = malloc(N * sizeof *th); double* om = malloc(N * sizeof *om);
    double* th0 = malloc(N * sizeof *th0); double* om0 = malloc(N * sizeof *om0);
    double* F = malloc(N * sizeof *F); double* n = malloc(N * sizeof *n);
    double* dth = malloc(N * sizeof *dth); double* dom = malloc(N * sizeof *dom);
    int32_t* lab = malloc(N * sizeof *lab);
    for (uint64_t k = 0; k < 50; k += 7) CHECK(xyo_temperature(&m, k) >= 0.0);
    uint32_t ctr[4] = {1, 2, 3, 4}, key[2] = {5, 6}, out[4];
    xyo_philox4x32_10(ctr, key, out);
    CHECK(xyo_uniform(0u) > 0.0 && xyo_uniform(0xFFFFFFFFu) < 1.0);
    xyo_normals(&m, 17, n);
    finite_all(n, N);
    CHECK(isfinite(xyo_normal(&m, 17, (int64_t)N - 1)));
    xyo_init_ordered(&m, -1, th, om);
    finite_all(th, N);
    xyo_init_random(&m, th, om);
    memcpy(th0, th, N * sizeof *th); memcpy(om0, om, N * sizeof *om);
    for (size_t i = 0; i < N; ++i) CHECK(abs(xyo_stagger(&m, (int64_t)i)) == 1);
    CHECK(isfinite(xyo_energy_pot(&m, th)));
    xyo_force(&m, th, F);
    finite_all(F, N);
    CHECK(xyo_run(&m, th, om, 0, 30) == 0);
    double obs[6 * 8];
    CHECK(xyo_run_measured(&m, th, om, 30, 25, 5, obs) == 6);
    finite_all(obs, 36);
    xyo_observables(&m, th, om, obs);
    finite_all(obs, 6);
    double C[64];
    xyo_correlation(&m, th, 0, Lx / 2, C);
    finite_all(C, (size_t)Lx / 2 + 1);
    xyo_correlation(&m, th, 1, Ly / 2, C);
    finite_all(C, (size_t)Ly / 2 + 1);
    const int64_t nd32 = xyo_domains(&m, th, 32, lab), nd64 = xyo_domains(&m, th, 64, lab);
    CHECK(nd32 >= 1 && nd64 >= 1 && nd64 <= (int64_t)N);
    for (size_t i = 0; i < N; ++i) CHECK(lab[i] >= 0 && (size_t)lab[i] <= i);
    double g[4] = {0, 0, 0, 0};
    const double L = xyo_adjoint(&m, th0, om0, 20, 5, g, dth, dom);
    if (model == XYO_MODEL_XY) {
        CHECK(isfinite(L));
        finite_all(g, 4); finite_all(dth, N); finite_all(dom, N);
        CHECK(fabs(xyo_loss(&m, th0, om0, 20, 5) - L) <= 1e-12 * fabs(L) + 1e-300);
        CHECK(isfinite(xyo_adjoint(&m, th0, om0, 1, 1, g, NULL, NULL)));
    } else {
        CHECK(isnan(L));
    }
    free(th); free(om); free(th0); free(om0); free(F); free(n); free(dth); free(dom); free(lab);
}

int main(void) {
    exercise(8, 6, XYO_MODEL_XY, 2.0, 0);
    exercise(4, 2, XYO_MODEL_XY, 2.0, 1);
    exercise(2, 2, XYO_MODEL_XY, 2.0, 0);
    exercise(8, 6, XYO_MODEL_SI, 2.5, 1);
    exercise(5, 3, XYO_MODEL_SI, 2.5, 0);
    if (bad) return 1;
    puts("ok");
    return 0;
}
"""

HOST_DRIVER = r"""
#include <cmath>
#include <cstdio>
#include <vector>
#include "xyl.h"

static int bad = 0;
#define CHECK(c) do { if (!(c)) { std::fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__); bad = 1; } } while (0)

int main() {
    CHECK(xyl_abi_version() == XYL_ABI_VERSION);
    std::vector<double> m(300);
    for (size_t i = 0; i < m.size(); ++i) m[i] = 0.3 + 0.2 * std::sin(0.37 * (double)i) + 0.05 * std::cos(1.3 * i);
    double U = 0, se = 0, mean = 0, err = 0, tau = 0;
    CHECK(xyl_binder(m.data(), m.size(), 60, &U, &se) == XYL_OK && std::isfinite(U) && std::isfinite(se));
    CHECK(xyl_binder(m.data(), 1, 0, &U, &se) == XYL_OK && U == 1.0 && std::isnan(se));
    CHECK(xyl_binder(m.data(), m.size(), 299, &U, nullptr) == XYL_OK);
    CHECK(xyl_binder(m.data(), m.size(), 300, &U, &se) == XYL_EINVAL);
    std::vector<double> z(10, 0.0);
    CHECK(xyl_binder(z.data(), z.size(), 0, &U, &se) == XYL_ENUMERIC && xyl_last_error()[0] != 0);
    CHECK(xyl_mean_error(m.data(), m.size(), 0, &mean, &err, &tau) == XYL_OK && tau >= 0.5);
    CHECK(xyl_mean_error(m.data(), 1, 0, &mean, &err, &tau) == XYL_OK && tau == 0.5);
    CHECK(xyl_mean_error(z.data(), z.size(), 3, &mean, &err, &tau) == XYL_OK && err == 0.0);
    const uint64_t nrep = 5, nt = 23;
    std::vector<double> mr(nrep * nt), Ub(nt), Ube(nt);
    for (size_t i = 0; i < mr.size(); ++i) mr[i] = 0.2 + 0.1 * std::sin(0.7 * (double)i);
    CHECK(xyl_binder_relaxation(mr.data(), nrep, nt, 4, Ub.data(), Ube.data()) == XYL_OK);
    CHECK(xyl_binder_relaxation(mr.data(), 1, nt, 4, Ub.data(), Ube.data()) == XYL_OK && std::isnan(Ube[0]));
    CHECK(xyl_binder_relaxation(mr.data(), nrep, nt, nt, Ub.data(), nullptr) == XYL_OK);
    CHECK(xyl_binder_relaxation(mr.data(), nrep, 3, 4, Ub.data(), nullptr) == XYL_EINVAL);
    std::vector<double> t1(40), u1(40), t2(30), u2(30);
    for (int i = 0; i < 40; ++i) { t1[i] = 2.0 * i; u1[i] = 1.0 + 2.0 * std::exp(-t1[i] / 20.0); }
    for (int i = 0; i < 30; ++i) { t2[i] = 3.0 * i; u2[i] = 1.0 + 2.0 * std::exp(-t2[i] / 20.0 * 1.5); }
    double zb = 0, cost = 0;
    CHECK(xyl_z_collapse(t1.data(), u1.data(), 40, 96, t2.data(), u2.data(), 30, 64, 0.5, 3.0, 0.01, &zb, &cost) == XYL_OK);
    CHECK(xyl_z_collapse(t1.data(), u1.data(), 40, 64, t2.data(), u2.data(), 30, 64, 0.5, 3.0, 0.01, &zb, &cost) == XYL_EINVAL);
    CHECK(xyl_z_collapse(t1.data(), u1.data(), 40, 96, t2.data(), u2.data(), 30, 64, -51.0, -50.0, 0.5, &zb, nullptr) == XYL_EINVAL);
    const int L = 256;
    std::vector<double> S(L / 2 + 1);
    for (int k = 0; k <= L / 2; ++k) {
        const double q = (double)k / L;
        S[k] = 0.7 * 2.0 * 6.0 / (1.0 + 4.0 * M_PI * M_PI * 36.0 * q * q);
    }
    double xi = 0, A = 0;
    CHECK(xyl_lorentzian_xi(S.data(), L, 0, 40, &xi, &A) == XYL_OK && std::fabs(xi - 6.0) < 1e-8);
    CHECK(xyl_lorentzian_xi(S.data(), L, 1, L / 2, &xi, nullptr) == XYL_OK);
    CHECK(xyl_lorentzian_xi(S.data(), L, 5, 5, &xi, &A) == XYL_EINVAL);
    std::vector<double> rising(L / 2 + 1);
    for (int k = 0; k <= L / 2; ++k) rising[k] = 1.0 + k;
    CHECK(xyl_lorentzian_xi(rising.data(), L, 0, 20, &xi, &A) == XYL_ENUMERIC);
    S[3] = -1.0;
    CHECK(xyl_lorentzian_xi(S.data(), L, 0, 20, &xi, &A) == XYL_EINVAL);
    std::vector<xyl_obs> smp(12);
    for (size_t i = 0; i < smp.size(); ++i) smp[i] = xyl_obs{-1.0, 0.5, 0.1, 2.0 + 0.01 * i, 0.5, 1.0};
    CHECK(xyl_xi_second_moment(smp.data(), smp.size(), 2, 0, 64, &xi) == XYL_OK && xi > 0.0);
    CHECK(xyl_xi_second_moment(smp.data(), smp.size(), 0, 1, 64, &xi) == XYL_OK && xi > 0.0);
    CHECK(xyl_xi_second_moment(smp.data(), smp.size(), 12, 0, 64, &xi) == XYL_EINVAL);
    CHECK(xyl_xi_second_moment(smp.data(), smp.size(), 0, 2, 64, &xi) == XYL_EINVAL);
    if (bad) return 1;
    std::puts("ok");
    return 0;
}
"""


def build_and_run(tmp_path, compiler, sources, driver_src, suffix, extra):
    drv = tmp_path / ("driver" + suffix)
    drv.write_text(driver_src)
    exe = tmp_path / "driver"
    cmd = [compiler, *SAN, *extra, *sources, str(drv), "-o", str(exe), "-lm"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    env = dict(os.environ, OMP_NUM_THREADS="2", ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=600)
    report = r.stdout + r.stderr
    assert r.returncode == 0 and r.stdout.strip().endswith("ok"), report
    assert "AddressSanitizer" not in report and "runtime error" not in report, report


def test_oracle_under_sanitizers(tmp_path):
    build_and_run(tmp_path, "gcc", [os.path.join(ROOT, "oracle", "xyo.c")], ORACLE_DRIVER, ".c",
                  ["-std=c11", "-fopenmp", "-I", os.path.join(ROOT, "oracle")])


def test_host_estimators_under_sanitizers(tmp_path):
    csrc = os.path.join(ROOT, "paper_2409_06412_amd", "csrc")
    build_and_run(tmp_path, "g++", [os.path.join(csrc, "xyl_host.cpp")], HOST_DRIVER, ".cpp",
                  ["-std=c++17", "-I", os.path.join(ROOT, "include"), "-I", csrc])
