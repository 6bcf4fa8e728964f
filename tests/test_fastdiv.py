"""Host check of the reciprocal division used for index arithmetic in the
FFT pass kernels (csrc/fastdiv.hpp compiles as plain C++): every divisor up
to 4100 and a spread of larger ones, numerators over [0, 2^31)."""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HDR = os.path.join(ROOT, "paper_2412_17445_amd", "csrc")

SRC = r"""
#include <cstdio>
#include <cstdint>
#include "fastdiv.hpp"
using namespace pff;
static uint64_t state = 0x12345678u;
static uint32_t next() { state = state * 6364136223846793005ull + 1442695040888963407ull; return uint32_t(state >> 33); }
int main() {
  long long bad = 0, checked = 0;
  auto check = [&](uint32_t d) {
    const FastDiv f = make_fastdiv(d);
    auto one = [&](uint32_t n) {
      ++checked;
      if (fdiv(n, f) != n / d || fmod_q(n, fdiv(n, f), f) != n % d) ++bad;
    };
    for (uint32_t n = 0; n < 70000; ++n) one(n);
    for (int k = 0; k < 2000; ++k) one(next() & 0x7fffffffu);
    for (uint32_t n = 0x7fffffffu - 3000; n < 0x7fffffffu; ++n) one(n);
    one(0x7fffffffu);
  };
  for (uint32_t d = 1; d <= 4100; ++d) check(d);
  for (uint32_t d = 4101; d < (1u << 30); d = d * 3 / 2 + 7) check(d);
  check((1u << 31) - 1);
  printf("%lld %lld\n", checked, bad);
  return bad != 0;
}
"""


@pytest.mark.skipif(shutil.which("g++") is None, reason="no host C++ compiler")
def test_fastdiv_matches_integer_division(tmp_path):
    src = tmp_path / "fd.cpp"
    exe = tmp_path / "fd"
    src.write_text(SRC)
    subprocess.run(["g++", "-O2", "-std=c++17", "-I", HDR, str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True)
    checked, bad = map(int, out.stdout.split())
    assert checked > 10 ** 8 // 4 and bad == 0, out.stdout
