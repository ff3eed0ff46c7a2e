"""Host-side check of the division by launch-fixed divisors that the kernels use for
node coordinates (FastDiv in csrc/internal.hpp: floor(n / d) = (n m) >> s with the
round-up magic number).  The header's own make_fastdiv / div are compiled into a small
host program and compared with integer division on every divisor up to 4096 (all n up
to 70,000 and the last 2,000 below 2^31), on the node counts of the benchmark meshes,
on powers of two, and on random divisors and dividends below 2^31."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

PROGRAM = r"""
#include "internal.hpp"
#include <cstdio>
#include <random>
using topo::FastDiv;
using topo::make_fastdiv;
static long check(unsigned d, unsigned n) {
    const FastDiv f = make_fastdiv(d);
    return f.div(n) != n / d ? 1 : 0;
}
int main() {
    long bad = 0, count = 0;
    for (unsigned d = 1; d <= 4096; ++d) {
        for (unsigned n = 0; n < 70000; ++n, ++count) bad += check(d, n);
        for (unsigned n = 0x7fffffffu - 2000; ; ++n) { bad += check(d, n); ++count; if (n == 0x7fffffffu) break; }
    }
    const unsigned mesh[] = {21, 61, 201, 601, 25, 49, 97, 193};  // ny1, nx1 of the workloads
    for (unsigned d : mesh)
        for (unsigned n = 0; n < 6000000; n += 7, ++count) bad += check(d, n);
    for (int l = 0; l < 31; ++l)
        for (unsigned n = 0; n < 100000; n += 3, ++count) bad += check(1u << l, n * 12345u & 0x7fffffffu);
    std::mt19937_64 rng(2024);
    for (int t = 0; t < 2000000; ++t, ++count) {
        const unsigned d = (unsigned)(rng() % 0x7fffffffu) + 1u, n = (unsigned)(rng() & 0x7fffffffu);
        bad += check(t & 1 ? d : (d % 100000u) + 1u, n);
    }
    std::printf("%ld %ld\n", bad, count);
    return 0;
}
"""


def _hipcc():
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    return None


def test_fastdiv_matches_integer_division(tmp_path):
    hipcc = _hipcc()
    if hipcc is None:
        pytest.skip("hipcc not available")
    src = tmp_path / "fastdiv_check.cpp"
    exe = tmp_path / "fastdiv_check"
    src.write_text(PROGRAM)
    cmd = [hipcc, "-x", "hip", "--offload-arch=gfx950", "-O2", "-std=c++17",
           "-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROOT, "paper_2004_05756_amd", "csrc"),
           str(src), "-o", str(exe)]
    res = subprocess.run(cmd, capture_output=True, text=True)
    assert res.returncode == 0, res.stderr[-2000:]
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stderr
    bad, count = map(int, out.stdout.split())
    assert count > 10_000_000 and bad == 0, (bad, count)
