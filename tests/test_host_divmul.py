"""The collide kernel splits its wave index with a multiply-high instead of a
division where the host hands it a multiplier (divmul.h).  This checks the
host rule against plain integer division on the CPU: exhaustively where the
range is small, and at every multiple of d (and its neighbours) plus random
samples up to the largest index the rule accepts.  No GPU."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2102_01305_amd", "csrc")

PROGRAM = r"""
#include <cstdio>
#include <cstdint>
#include <random>
#include "divmul.h"

static unsigned umulhi(unsigned a, unsigned b) { return (unsigned)(((uint64_t)a * b) >> 32); }

int main() {
  const unsigned long long ds[] = {2, 3, 4, 5, 6, 7, 9, 12, 64, 191, 192, 384, 1000, 4093, 65535, 65536, 1u << 20};
  std::mt19937_64 rng(7);
  long long bad = 0, checked = 0;
  for (unsigned long long d : ds) {
    // the largest range the rule accepts: n_end d < 2^32
    const unsigned long long n_end = ((1ULL << 32) - 1) / d;
    const unsigned m = ibmk::div_mul(d, n_end);
    if (m == 0) { std::printf("no multiplier for d=%llu\n", d); return 2; }
    if (ibmk::div_mul(d, n_end + 1) != 0) { std::printf("range not refused for d=%llu\n", d); return 3; }
    auto check = [&](unsigned long long n) {
      if (n >= n_end) return;
      ++checked;
      if (umulhi((unsigned)n, m) != n / d) {
        if (bad < 5) std::printf("d=%llu n=%llu: %u != %llu\n", d, n, umulhi((unsigned)n, m), n / d);
        ++bad;
      }
    };
    const unsigned long long dense = n_end < (1ULL << 22) ? n_end : (1ULL << 22);
    for (unsigned long long n = 0; n < dense; ++n) check(n);
    for (unsigned long long q = 0; q * d < n_end; q += 1 + q / 4096) {
      check(q * d); check(q * d + d - 1); check(q * d + 1);
    }
    for (int k = 0; k < 2000000; ++k) check(rng() % n_end);
    check(n_end - 1);
  }
  if (ibmk::div_mul(1, 10) != 0) { std::printf("d=1 must divide\n"); return 4; }
  std::printf("checked %lld bad %lld\n", checked, bad);
  return bad ? 1 : 0;
}
"""


def test_multiply_high_division_matches_integer_division(tmp_path):
    cxx = shutil.which("g++")
    if cxx is None:
        pytest.skip("no g++")
    src = tmp_path / "divmul_check.cpp"
    exe = tmp_path / "divmul_check"
    src.write_text(PROGRAM)
    subprocess.run([cxx, "-O2", "-std=c++17", "-I", CSRC, str(src), "-o", str(exe)], check=True)
    res = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300)
    print(res.stdout)
    assert res.returncode == 0, res.stdout + res.stderr
