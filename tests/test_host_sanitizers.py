"""The host-only C++ of the library (csrc/qp.cpp: the QP step and the evGW
update) built with g++ under AddressSanitizer and UndefinedBehaviorSanitizer
(host code only) and driven with seeded random valid and invalid inputs:
ragged sizes, Pade windows that keep few nodes, coincident frequencies,
non-finite values, duplicate and out-of-range states.  Any sanitizer report
fails the test; results are not checked here (the oracle tests do that)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

DRIVER = r"""
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>
#include "gw.h"
namespace gw {
void set_error(const std::string&) {}
void clear_error() {}
}
static uint64_t st = 0x9E3779B97F4A7C15ull;
static double u() { st = st * 6364136223846793005ull + 1442695040888963407ull; return (st >> 11) * 0x1.0p-53; }
int main() {
  int calls = 0;
  for (int it = 0; it < 400; ++it) {
    const int n_gw = 1 + (int)(u() * 6), n_tau = 1 + (int)(u() * 16), n_w = 1 + (int)(u() * 16);
    std::vector<double> so(n_gw * n_tau), sv(n_gw * n_tau), sx(n_gw), en(n_gw), vx(n_gw);
    std::vector<int32_t> occ(n_gw);
    std::vector<double> om(n_w), cw(n_w * n_tau), sw(n_w * n_tau), e(n_gw);
    std::vector<int32_t> status(n_gw);
    for (auto& x : so) x = -u();
    for (auto& x : sv) x = u();
    for (int n = 0; n < n_gw; ++n) { sx[n] = -u(); en[n] = u() - 0.5; vx[n] = 0.1 * u(); occ[n] = u() < 0.5; }
    double w = 0.0;
    for (int k = 0; k < n_w; ++k) { w += (u() < 0.1 ? 0.0 : 0.1 + u()); om[k] = w > 0 ? w : 0.05; }
    for (auto& x : cw) x = u() - 0.5;
    for (auto& x : sw) x = u() - 0.5;
    if (u() < 0.05) so[0] = NAN;
    gw_qp_opts o{u() < 0.5 ? 0.0 : u() * w, u() < 0.5 ? 0.0 : 1e-8, (int32_t)(u() * 50)};
    gw_continue_qp(n_gw, so.data(), sv.data(), sx.data(), en.data(), u() < 0.3 ? nullptr : vx.data(),
                   occ.data(), 0.0, n_tau, n_w, om.data(), cw.data(), sw.data(), u() < 0.3 ? nullptr : &o,
                   e.data(), status.data());
    ++calls;
    // evGW update
    const int n_mo = 2 + (int)(u() * 20), n_occ = 1 + (int)(u() * (n_mo - 1));
    std::vector<double> e0(n_mo), out(n_mo);
    for (int i = 0; i < n_mo; ++i) e0[i] = i - 0.5 * n_mo + 0.1 * u();
    const int m = 1 + (int)(u() * n_mo);
    std::vector<int32_t> states(m);
    std::vector<double> q(m);
    for (int i = 0; i < m; ++i) { states[i] = (int32_t)(u() * (n_mo + (u() < 0.1 ? 3 : 0))) - (u() < 0.05); q[i] = e0[states[i] >= 0 && states[i] < n_mo ? states[i] : 0] + (u() - 0.5); }
    if (u() < 0.05) q[0] = INFINITY;
    double mu = 0.0;
    gw_evgw_update(n_mo, n_occ, e0.data(), m, states.data(), q.data(), out.data(), u() < 0.2 ? nullptr : &mu);
    ++calls;
  }
  // argument errors
  gw_continue_qp(0, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, 0.0, 0, 0, nullptr, nullptr,
                 nullptr, nullptr, nullptr, nullptr);
  gw_evgw_update(1, 1, nullptr, 0, nullptr, nullptr, nullptr, nullptr);
  std::printf("calls %d\n", calls);
  return 0;
}
"""


def test_qp_host_code_under_asan_and_ubsan(tmp_path):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    drv = tmp_path / "driver.cpp"
    drv.write_text(DRIVER)
    exe = tmp_path / "driver"
    cmd = [gxx, "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-D__HIP_PLATFORM_AMD__",
           "-I" + os.path.join(ROOT, "include"), "-I/opt/rocm/include",
           os.path.join(ROOT, "paper_2104_09857_amd", "csrc", "qp.cpp"), str(drv), "-o", str(exe)]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=300)
    if r.returncode != 0 and "sanitizer" in (r.stderr or "").lower() and "cannot find" in r.stderr:
        pytest.skip("sanitizer runtime not available")
    assert r.returncode == 0, r.stderr[-3000:]
    env = dict(os.environ, ASAN_OPTIONS="abort_on_error=1:detect_leaks=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    run = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300, env=env)
    assert run.returncode == 0, (run.stdout[-2000:], run.stderr[-4000:])
    assert "runtime error" not in run.stderr and "AddressSanitizer" not in run.stderr
    assert "calls 800" in run.stdout
