"""Pins of the oracle's Philox4x32-10 generator.

The bijection is checked against the independent implementation in the rocRAND headers (a
library routine, compiled here for the host), and the derived uniforms against statistics.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

_PROBE = r"""
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>
struct Probe : rocrand_device::philox4x32_10_engine {
  uint4 bijection(uint4 c, uint2 k) { return ten_rounds(c, k); }
};
int main() {
  Probe e;
  unsigned c0, c1, c2, c3, k0, k1;
  while (scanf("%u %u %u %u %u %u", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
    uint4 r = e.bijection(uint4{c0, c1, c2, c3}, uint2{k0, k1});
    printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
  }
}
"""


@pytest.fixture(scope="module")
def rocrand_probe(tmp_path_factory):
    hdr = "/opt/rocm/include/rocrand/rocrand_philox4x32_10.h"
    if not os.path.exists(hdr) or shutil.which("g++") is None:
        pytest.skip("rocRAND headers or g++ not available")
    d = tmp_path_factory.mktemp("philox")
    src, exe = d / "probe.cpp", d / "probe"
    src.write_text(_PROBE)
    subprocess.run(["g++", "-O1", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", str(src), "-o",
                    str(exe)], check=True, capture_output=True)
    return str(exe)


def test_philox_matches_rocrand(orc, rocrand_probe):
    rng = np.random.default_rng(11)
    rows = rng.integers(0, 2**32, size=(500, 6), dtype=np.uint64)
    rows[:4] = [[0, 0, 0, 0, 0, 0], [2**32 - 1] * 6, [1, 2, 3, 4, 5, 6], [7, 0, 0, 0, 0, 1]]
    inp = "\n".join(" ".join(str(int(x)) for x in r) for r in rows) + "\n"
    out = subprocess.run([rocrand_probe], input=inp, capture_output=True, text=True, check=True)
    ref = [tuple(int(x) for x in line.split()) for line in out.stdout.strip().splitlines()]
    assert len(ref) == len(rows)
    for r, e in zip(rows, ref):
        assert orc.philox4x32_10(r[:4], r[4:]) == e


def test_u53_range_and_moments(orc):
    vals = np.array([orc.u53(*orc.draw(5, 0, it, p, 0, 0)[:2])
                     for it in range(40) for p in range(500)])
    assert vals.min() >= 0.0 and vals.max() < 1.0
    assert abs(vals.mean() - 0.5) < 0.01
    assert abs(vals.var() - 1 / 12) < 0.003
    hist = np.histogram(vals, bins=20, range=(0, 1))[0]
    chi2 = np.sum((hist - len(vals) / 20) ** 2 / (len(vals) / 20))
    assert chi2 < 45  # 19 dof, p ~ 1e-3


def test_u53_extremes(orc):
    assert orc.u53(0, 0) == 0.0
    assert orc.u53(0xFFFFFFFF, 0xFFFFFFFF) == 1.0 - 2.0**-53


def test_streams_distinct(orc):
    """Different purposes, dims, particles, iterations and swarms give different words."""
    base = orc.draw(0, 0, 0, 0, 0, 0)
    for args in [(0, 1, 0, 0, 0, 0), (0, 0, 1, 0, 0, 0), (0, 0, 0, 1, 0, 0), (0, 0, 0, 0, 1, 0),
                 (0, 0, 0, 0, 0, 1), (1, 0, 0, 0, 0, 0), (2**32, 0, 0, 0, 0, 0)]:
        assert orc.draw(*args) != base
