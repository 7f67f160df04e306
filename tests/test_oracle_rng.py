"""Oracle pins: the Philox stream and the uniform / integer maps built on it."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))


def _kat():
    rows = []
    with open(os.path.join(HERE, "golden", "philox4x32_10_kat.txt")) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            v = [int(t, 16) for t in line.split()]
            rows.append((v[0:4], v[4:6], v[6:10]))
    return rows


@pytest.mark.parametrize("ctr,key,expect", _kat())
def test_philox_known_answers(ctr, key, expect):
    assert [int(x) for x in oracle.philox(ctr, key)] == expect


ROCRAND_PROBE = r"""
#include <rocrand/rocrand_kernel.h>
#include <cstdio>
int main(){
  const unsigned long long seeds[3] = {0ULL, 0x0000000500000007ULL, 0xDEADBEEF12345678ULL};
  for (int s = 0; s < 3; ++s) {
    rocrand_state_philox4x32_10 st;
    rocrand_init(seeds[s], 0, 0, &st);
    for (int k = 0; k < 4; ++k) {
      uint4 a = rocrand4(&st);
      printf("%llu %d %u %u %u %u\n", seeds[s], k, a.x, a.y, a.z, a.w);
    }
  }
}
"""


@pytest.mark.skipif(shutil.which("hipcc") is None, reason="hipcc not installed")
def test_philox_matches_rocrand_host(tmp_path):
    """rocRAND's host-side Philox4x32-10 (counter word 0 = block index, key = seed)
    is an independent implementation of the same published generator."""
    src = tmp_path / "probe.cpp"
    src.write_text(ROCRAND_PROBE)
    exe = tmp_path / "probe"
    subprocess.run(["hipcc", "-O1", "-o", str(exe), str(src)], check=True,
                   capture_output=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    for line in out.strip().splitlines():
        seed, k, *words = (int(t) for t in line.split())
        key = (seed & 0xFFFFFFFF, seed >> 32)
        assert [int(x) for x in oracle.philox((k, 0, 0, 0), key)] == words


def test_u01_exact_in_single_precision_and_open_interval():
    L = oracle.lib()
    rs = [0, 1, 511, 512, 0x7FFFFFFF, 0xFFFFFE00, 0xFFFFFFFF, 123456789]
    for r in rs:
        u = L.orc_u01(r)
        assert 0.0 < u < 1.0
        assert float(np.float32(u)) == u
    assert L.orc_u01(0) == 2.0 ** -24
    assert L.orc_u01(0xFFFFFFFF) == 1.0 - 2.0 ** -24


def test_pick_range_and_uniformity():
    L = oracle.lib()
    key = (11, 22)
    n = 7
    counts = np.zeros(n)
    for k in range(20000):
        w = oracle.philox((k, 0, 0, 0), key)
        for r in w:
            v = L.orc_pick(int(r), n)
            assert 0 <= v < n
            counts[v] += 1
    exp = counts.sum() / n
    chi2 = ((counts - exp) ** 2 / exp).sum()
    assert chi2 < 22.5  # chi-square, 6 dof, p ~ 0.001
    assert L.orc_pick(0xFFFFFFFF, n) == n - 1
    assert L.orc_pick(0, n) == 0


def test_uniform_stream_ks():
    L = oracle.lib()
    key = (3, 9)
    us = []
    for k in range(25000):
        for r in oracle.philox((k, 1, 2, 3), key):
            us.append(L.orc_u01(int(r)))
    us = np.sort(np.array(us))
    n = len(us)
    d = np.max(np.maximum(np.arange(1, n + 1) / n - us, us - np.arange(n) / n))
    assert d * np.sqrt(n) < 1.95  # Kolmogorov-Smirnov, p ~ 0.001
