"""The cell-index division the kernels use instead of the hardware-less
integer divide (constants of divisor_constants in csrc/vlb_internal.h, after
Granlund and Montgomery's division by invariant integers): compiled for the
host and checked against plain division for every divisor up to 2048 (edge
dividends, multiples and random ones) and random divisors below 2^31."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = r"""
#include <cstdio>
#include <cstdint>
#include <random>
#include "vlb_internal.h"
static uint32_t div_by(uint32_t n, uint32_t m, uint32_t sh)
{
    const uint32_t t = static_cast<uint32_t>((uint64_t(m) * n) >> 32);
    return (t + ((n - t) >> (sh & 0xffu))) >> (sh >> 8);
}
int main()
{
    std::mt19937_64 rng(7);
    unsigned long long bad = 0, checked = 0;
    auto check = [&](uint32_t d, uint32_t n) {
        uint32_t m, sh;
        vlb::divisor_constants(d, m, sh);
        ++checked;
        bad += div_by(n, m, sh) != n / d;
    };
    for (uint32_t d = 1; d <= 2048; ++d) {
        for (uint32_t n : {0u, 1u, d - 1, d, d + 1, 0xffffffffu, 0xfffffffeu, 0x80000000u})
            check(d, n);
        for (int k = 0; k < 500; ++k)
            check(d, static_cast<uint32_t>(rng()));
        for (uint32_t q = 1; q < 500; ++q) {
            check(d, q * d);
            check(d, q * d - 1);
        }
    }
    for (int k = 0; k < 100000; ++k) {
        const uint32_t d = 1 + static_cast<uint32_t>(rng() % 0x7fffffffu);
        const uint32_t q = static_cast<uint32_t>(rng() % (0xffffffffu / d + 1));
        check(d, static_cast<uint32_t>(rng()));
        check(d, q * d);
        if (q)
            check(d, q * d - 1);
    }
    std::printf("%llu %llu\n", checked, bad);
    return bad != 0;
}
"""


def test_invariant_divisor_constants_divide_exactly(tmp_path):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    src = tmp_path / "divcheck.cpp"
    src.write_text(SRC)
    exe = tmp_path / "divcheck"
    subprocess.run([hipcc, "-O2", "-std=c++17", "-I", os.path.join(ROOT, "paper_2009_12279_amd", "csrc"),
                    "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True, capture_output=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    checked, bad = (int(v) for v in out.stdout.split())
    assert checked > 3_000_000 and bad == 0 and out.returncode == 0
