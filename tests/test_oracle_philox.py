"""Pins of the oracle's counter-based generator.

Philox4x32-10 is pinned against an independent implementation: rocRAND's
``philox4x32_10_engine`` (a library routine, compiled here as host code from its
header).  Seeding that engine with (seed = key, subsequence = counter words 2-3,
offset = 4 x counter words 0-1) makes its first output block the bare bijection.
Uniformity and independence are checked statistically.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle

HELPER = r"""
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>
int main() {
  unsigned long long c0, c1, c2, c3, k0, k1;
  while (scanf("%llu %llu %llu %llu %llu %llu", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
    rocrand_device::philox4x32_10_engine e(k0 | (k1 << 32), c2 | (c3 << 32), 4ull * (c0 | (c1 << 32)));
    uint4 r = e.next4();
    printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
  }
  return 0;
}
"""


@pytest.fixture(scope="module")
def rocrand_ref(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    hdr = "/opt/rocm/include/rocrand/rocrand_philox4x32_10.h"
    if not (os.path.exists(hipcc) and os.path.exists(hdr)):
        pytest.skip("rocRAND header or hipcc not available")
    d = tmp_path_factory.mktemp("rocrand")
    src, exe = d / "ref.cpp", d / "ref"
    src.write_text(HELPER)
    subprocess.check_call([hipcc, "-x", "c++", "-O1", "-I/opt/rocm/include", "-D__HIP_PLATFORM_AMD__",
                           str(src), "-o", str(exe)])

    def run(cases):
        txt = "\n".join(" ".join(str(int(v)) for v in c) for c in cases) + "\n"
        out = subprocess.run([str(exe)], input=txt, capture_output=True, text=True, check=True).stdout
        return np.array([[int(v) for v in line.split()] for line in out.strip().split("\n")], dtype=np.uint64)
    return run


def test_philox_bijection_matches_rocrand(rocrand_ref):
    rng = np.random.default_rng(7)
    m = 0xFFFFFFFF
    # the reference route passes counter words 0-1 as a 64-bit offset times 4, so word 1
    # stays below 2^30 here; words 2-3 and the key take any value
    c1max = (1 << 30) - 1
    cases = [(0, 0, 0, 0, 0, 0), (m, c1max, m, m, m, m), (1, 0, 0, 0, 0, 0), (0, 0, 0, 0, 1, 0),
             (0x243F6A88, 0x05A308D3, 0x13198A2E, 0x03707344, 0xA4093822, 0x299F31D0)]
    for _ in range(200):
        v = rng.integers(0, 2**32, 6)
        v[1] %= 1 << 30
        cases.append(tuple(int(x) for x in v))
    ref = rocrand_ref(cases)
    for c, r in zip(cases, ref):
        got = oracle.philox4x32_10(c[:4], c[4:])
        assert np.array_equal(got.astype(np.uint64), r), (c, got, r)


def test_uniform_layout_matches_rocrand(rocrand_ref):
    """uniform4(id, step, stream, seed): counter (step lo, step hi16 | stream<<16,
    seed lo, seed hi), key (id lo, id hi), u -> (u + 1/2) 2^-32."""
    pid, step, stream, seed = (1 << 40) + 12345, 70000, 2, 0xDEADBEEF12345
    r = oracle.uniform4(pid, step, stream, seed)
    c = (step & 0xFFFFFFFF, ((step >> 32) & 0xFFFF) | (stream << 16), seed & 0xFFFFFFFF, seed >> 32,
         pid & 0xFFFFFFFF, pid >> 32)
    u = rocrand_ref([c])[0].astype(np.float64)
    assert np.array_equal(r, (u + 0.5) / 2**32)


def test_uniform_statistics():
    n = 40000
    r = np.array([oracle.uniform4(i, 17, 1, 5) for i in range(n)])
    assert r.min() > 0 and r.max() < 1
    # each of the four outputs is uniform: chi^2 over 32 bins (4 sigma ~ 31 + 4*8)
    for k in range(4):
        h, _ = np.histogram(r[:, k], bins=32, range=(0, 1))
        chi2 = np.sum((h - n / 32) ** 2 / (n / 32))
        assert chi2 < 70, chi2
        assert abs(r[:, k].mean() - 0.5) < 4 * np.sqrt(1 / 12 / n)
    # outputs of one call and of neighbouring ids are uncorrelated
    c = np.corrcoef(r.T)
    assert np.max(np.abs(c - np.eye(4))) < 4 / np.sqrt(n)
    assert abs(np.corrcoef(r[:-1, 1], r[1:, 1])[0, 1]) < 4 / np.sqrt(n)


def test_streams_steps_seeds_are_distinct():
    a = oracle.uniform4(3, 10, 1, 1)
    assert not np.array_equal(a, oracle.uniform4(3, 10, 2, 1))
    assert not np.array_equal(a, oracle.uniform4(3, 11, 1, 1))
    assert not np.array_equal(a, oracle.uniform4(3, 10, 1, 2))
    assert not np.array_equal(a, oracle.uniform4(4, 10, 1, 1))
    assert np.array_equal(a, oracle.uniform4(3, 10, 1, 1))
