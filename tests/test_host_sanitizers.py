"""The library's plain host C++ (the small dense eigen/Cholesky solvers of the
Rayleigh-Ritz problems and the element table builder) built with
AddressSanitizer and UndefinedBehaviorSanitizer by g++ and run on a driver
that exercises every routine over a range of sizes, elements and
dimensions.  Any invalid access or undefined operation aborts the driver."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_1909_13585_amd", "csrc")

DRIVER = r"""
#include <cmath>
#include <cstdio>
#include <random>
#include <vector>
#include "dense.h"
#include "tables.h"

int main() {
    std::mt19937_64 rng(7);
    std::normal_distribution<double> nd;
    int bad = 0;
    for (int n : {1, 2, 3, 5, 12, 24, 33, 64, 96}) {
        std::vector<double> M(n * n), A(n * n), B(n * n);
        for (auto& v : M) v = nd(rng);
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                double s = 0.0;
                for (int k = 0; k < n; ++k) s += M[i * n + k] * M[j * n + k];
                A[i * n + j] = 0.5 * (M[i * n + j] + M[j * n + i]);
                B[i * n + j] = s + (i == j ? n : 0.0);
            }
        // symmetric eigenproblem: A V = V diag(w)
        std::vector<double> w(n), V(n * n);
        if (!mlb::sym_eig(n, A.data(), w.data(), V.data())) ++bad;
        double r = 0.0;
        for (int i = 0; i < n; ++i)
            for (int q = 0; q < n; ++q) {
                double s = 0.0;
                for (int k = 0; k < n; ++k) s += A[i * n + k] * V[k * n + q];
                r = std::fmax(r, std::fabs(s - w[q] * V[i * n + q]));
            }
        if (!(r < 1e-9 * (1 + n))) ++bad;
        // symmetric-definite problem A y = mu B y (B SPD, the first argument)
        std::vector<double> mu(n), Y(n * n);
        if (!mlb::gen_eig(n, B.data(), A.data(), mu.data(), Y.data())) ++bad;
        double g = 0.0;
        for (int i = 0; i < n; ++i)
            for (int q = 0; q < n; ++q) {
                double s = 0.0, t = 0.0;
                for (int k = 0; k < n; ++k) s += A[i * n + k] * Y[k * n + q], t += B[i * n + k] * Y[k * n + q];
                g = std::fmax(g, std::fabs(s - mu[q] * t));
            }
        if (!(g < 1e-8 * (1 + n))) ++bad;
        // Cholesky of the SPD matrix
        std::vector<double> L(B);
        if (!mlb::cholesky(n, L.data())) ++bad;
        double e = 0.0;
        for (int i = 0; i < n; ++i)
            for (int j = 0; j <= i; ++j) {
                double s = 0.0;
                for (int k = 0; k <= j; ++k) s += L[i * n + k] * L[j * n + k];
                e = std::fmax(e, std::fabs(s - B[i * n + j]));
            }
        if (!(e < 1e-9 * n * n)) ++bad;
    }
    for (int dim : {2, 3})
        for (int element : {0, 1}) {
            mlb::Tables t;
            mlb::build_tables(dim, 0.3, element, &t);
            double asym = 0.0;
            for (int i = 0; i < t.nde; ++i)
                for (int j = 0; j < t.nde; ++j)
                    asym = std::fmax(asym, std::fabs(t.K0[i * t.nde + j] - t.K0[j * t.nde + i]));
            if (!(asym < 1e-12)) ++bad;
        }
    std::printf(bad ? "failures %d\n" : "ok\n", bad);
    return bad ? 1 : 0;
}
"""


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_host_code_under_address_and_undefined_sanitizers(tmp_path):
    src = tmp_path / "driver.cpp"
    src.write_text(DRIVER)
    exe = tmp_path / "driver"
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-static-libasan", "-I", CSRC, str(src), os.path.join(CSRC, "dense.cpp"),
           os.path.join(CSRC, "tables.cpp"), "-o", str(exe)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:verify_asan_link_order=0", UBSAN_OPTIONS="print_stacktrace=1")
    p = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=300)
    assert p.returncode == 0 and p.stdout.strip() == "ok", (p.stdout[-2000:], p.stderr[-4000:])
