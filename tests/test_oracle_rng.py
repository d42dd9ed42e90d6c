"""Pins of the oracle's random numbers (the xi_i ~ N(0,1) of eq. euler).

Philox4x32-10 is checked bit for bit against an independent implementation,
PyTorch's header-only ``at::philox_engine`` (ATen/core/PhiloxRNGEngine.h),
compiled here into a tiny host program.  Its state maps onto ours as
key = seed (lo, hi), counter = (offset lo, offset hi, subsequence lo, hi),
and successive calls return the four output words in order.

The Box-Muller normals are checked against N(0,1) by moments, a
Kolmogorov-Smirnov test and independence checks.
"""
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest
from scipy import stats

SHIM = r"""
#include <ATen/core/PhiloxRNGEngine.h>
#include <cstdio>
#include <cinttypes>
int main() {
  unsigned c0, c1, c2, c3, k0, k1;
  while (std::scanf("%u %u %u %u %u %u", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
    uint64_t seed = (uint64_t)k0 | ((uint64_t)k1 << 32);
    uint64_t sub = (uint64_t)c2 | ((uint64_t)c3 << 32);
    uint64_t off = (uint64_t)c0 | ((uint64_t)c1 << 32);
    at::philox_engine e(seed, sub, off);
    unsigned a = e(), b = e(), c = e(), d = e();
    std::printf("%u %u %u %u\n", a, b, c, d);
  }
  return 0;
}
"""


def _torch_include():
    import torch.utils.cpp_extension as ce
    return ce.include_paths()


@pytest.fixture(scope="module")
def torch_philox():
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    inc = _torch_include()
    d = tempfile.mkdtemp()
    src = os.path.join(d, "shim.cpp")
    exe = os.path.join(d, "shim")
    with open(src, "w") as f:
        f.write(SHIM)
    cmd = ["g++", "-O1", "-std=c++17", src, "-o", exe] + [f"-I{p}" for p in inc]
    subprocess.run(cmd, check=True, capture_output=True)

    def run(rows):
        txt = "\n".join(" ".join(str(int(v)) for v in r) for r in rows) + "\n"
        out = subprocess.run([exe], input=txt, capture_output=True, text=True, check=True).stdout
        return np.array([[int(x) for x in line.split()] for line in out.strip().splitlines()],
                        dtype=np.uint64)

    yield run
    shutil.rmtree(d, ignore_errors=True)


def test_philox_matches_independent_engine(orc, torch_philox):
    rng = np.random.default_rng(7)
    rows = rng.integers(0, 2**32, size=(300, 6), dtype=np.uint64)
    rows[0] = 0
    rows[1] = 2**32 - 1
    rows[2, :4] = [5, 0, 9, 0]  # small counters as used by the path convention
    ref = torch_philox(rows)
    ours = np.array([orc.philox4x32_10(r[:4], r[4:]) for r in rows], dtype=np.uint64)
    assert np.array_equal(ours, ref)


def test_philox_key_and_counter_sensitivity(orc):
    base = orc.philox4x32_10([1, 2, 3, 4], [5, 6])
    for pos in range(4):
        c = [1, 2, 3, 4]
        c[pos] ^= 1
        assert not np.array_equal(orc.philox4x32_10(c, [5, 6]), base)
    assert not np.array_equal(orc.philox4x32_10([1, 2, 3, 4], [5, 7]), base)


def test_normals_reuse_one_block_per_two_steps(orc):
    # steps 2m and 2m+1 come from the same Philox block: words (w0,w1) and (w2,w3)
    z = orc.normals(11, np.arange(6), 3, 2)
    w = orc.philox4x32_10([1, 3, 2, 0], [11, 0])  # block of steps 2 and 3
    for step, (wa, wb) in ((2, (w[0], w[1])), (3, (w[2], w[3]))):
        ua = ((int(wa) >> 8) + 1) * 2.0**-24
        ub = (int(wb) >> 8) * 2.0**-24
        r = np.sqrt(-2 * np.log(ua))
        assert z[step, 0] == pytest.approx(r * np.cos(2 * np.pi * ub), abs=1e-15)
        assert z[step, 1] == pytest.approx(r * np.sin(2 * np.pi * ub), abs=1e-15)


def test_box_muller_is_standard_normal(orc):
    n = 400_000
    steps = np.arange(n, dtype=np.uint64) % 1000
    parts = (np.arange(n) // 1000).astype(np.uint32)
    z = orc.normals(2024, steps, parts, 5)
    for c in range(2):
        x = z[:, c]
        se = 1 / np.sqrt(n)
        assert abs(x.mean()) < 5 * se
        assert abs(x.var() - 1) < 5 * np.sqrt(2 / n)
        assert abs(stats.kurtosis(x, fisher=False) - 3) < 5 * np.sqrt(24 / n)
        assert stats.kstest(x, "norm").pvalue > 1e-4
    # the two components, and consecutive steps, are uncorrelated
    assert abs(np.corrcoef(z[:, 0], z[:, 1])[0, 1]) < 5 / np.sqrt(n)
    a = z[:-1, 0][steps[:-1] < 999]
    b = z[1:, 0][steps[:-1] < 999]
    assert abs(np.corrcoef(a, b)[0, 1]) < 5 / np.sqrt(a.size)
    # largest radius is bounded by sqrt(-2 ln 2^-24)
    assert np.max(np.hypot(z[:, 0], z[:, 1])) <= np.sqrt(-2 * np.log(2.0**-24)) + 1e-12


def test_distinct_particles_and_observations_get_distinct_streams(orc):
    a = orc.normals(3, np.arange(10), 0, 0)
    b = orc.normals(3, np.arange(10), 1, 0)
    c = orc.normals(3, np.arange(10), 0, 1)
    d = orc.normals(4, np.arange(10), 0, 0)
    for o in (b, c, d):
        assert not np.allclose(a, o)
