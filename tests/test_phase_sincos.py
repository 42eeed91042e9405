"""Host check of the FP64 phase routine the 3D kernels use for exp(-i tau lam)
(`sincos_phase` in paper_1903_04946_amd/csrc/fft_core.hpp, a host/device
function): the same source text is compiled with g++ and compared with
long-double sin and cos over |x| <= 1e6, the routine's documented range."""
import os
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HDR = os.path.join(ROOT, "paper_1903_04946_amd", "csrc", "fft_core.hpp")

DRIVER = r"""
#include <cmath>
#include <cstdio>
#include <random>
#define __host__
#define __device__
#define __forceinline__ inline
namespace t {
#include "fn.inc"
}
int main() {
  std::mt19937_64 g(1903);
  double worst = 0.0;
  for (int dec = -2; dec <= 6; ++dec) {
    const double lim = std::pow(10.0, dec);
    std::uniform_real_distribution<double> d(-lim, lim);
    for (int i = 0; i < 200000; ++i) {
      const double x = d(g);
      double s, c;
      t::sincos_phase(x, &s, &c);
      const long double sl = sinl((long double)x), cl = cosl((long double)x);
      worst = std::fmax(worst, std::fabs((double)(s - sl)));
      worst = std::fmax(worst, std::fabs((double)(c - cl)));
    }
  }
  // multiples of pi/4 (quadrant boundaries) and signed zero
  for (int k = -40; k <= 40; ++k) {
    const double x = k * 0.78539816339744830962;
    double s, c;
    t::sincos_phase(x, &s, &c);
    worst = std::fmax(worst, std::fabs((double)(s - sinl((long double)x))));
    worst = std::fmax(worst, std::fabs((double)(c - cosl((long double)x))));
  }
  std::printf("%.6e\n", worst);
  return 0;
}
"""


def test_sincos_phase_matches_long_double():
    src = open(HDR).read()
    a = src.index("__host__ __device__ __forceinline__ void sincos_phase(")
    b = src.index("\n}\n", a) + 3
    with tempfile.TemporaryDirectory() as d:
        open(os.path.join(d, "fn.inc"), "w").write(src[a:b])
        open(os.path.join(d, "t.cpp"), "w").write(DRIVER)
        exe = os.path.join(d, "t")
        r = subprocess.run(["g++", "-O2", "-o", exe, os.path.join(d, "t.cpp"), "-lm"],
                           capture_output=True, text=True)
        if r.returncode != 0:
            pytest.fail(r.stderr)
        out = subprocess.run([exe], capture_output=True, text=True, check=True).stdout
    worst = float(out.strip())
    # within one unit in the last place of a result of modulus <= 1
    assert worst < 2.3e-16, worst
