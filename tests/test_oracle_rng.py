"""Pins for the oracle's counter-based draws.

Philox4x32-10 (Salmon et al., SC'11) is checked against rocRAND's
independent implementation, run as a black box through its public API
(rocrand_init(seed, subsequence, offset) then rocrand4); the uniform,
bounded-integer and normal maps are checked statistically and against their
mathematical properties.
"""
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest
from scipy import stats

ROCRAND_PROG = r"""
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>
int main() {
  unsigned int k0, k1, c0, c1, c2, c3;
  while (scanf("%x %x %x %x %x %x", &k0, &k1, &c0, &c1, &c2, &c3) == 6) {
    rocrand_state_philox4x32_10 st;
    unsigned long long seed = ((unsigned long long)k1 << 32) | k0;
    unsigned long long sub = ((unsigned long long)c3 << 32) | c2;
    unsigned long long off = (((unsigned long long)c1 << 32) | c0) * 4ULL;
    rocrand_init(seed, sub, off, &st);
    uint4 r = rocrand4(&st);
    printf("%08x %08x %08x %08x\n", r.x, r.y, r.z, r.w);
  }
  return 0;
}
"""


def _rocrand_outputs(tuples):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available to build the rocRAND cross-check")
    with tempfile.TemporaryDirectory() as d:
        src = os.path.join(d, "p.cpp")
        exe = os.path.join(d, "p")
        open(src, "w").write(ROCRAND_PROG)
        subprocess.run([hipcc, "-x", "hip", "--offload-arch=gfx950", "-I/opt/rocm/include",
                        "-O1", src, "-o", exe], check=True, capture_output=True)
        inp = "\n".join(" ".join("%x" % v for v in t) for t in tuples) + "\n"
        out = subprocess.run([exe], input=inp, capture_output=True, text=True, check=True).stdout
    return [tuple(int(w, 16) for w in line.split()) for line in out.strip().splitlines()]


def test_philox_matches_rocrand(orc):
    g = np.random.default_rng(1)
    # rocRAND's offset counts 32-bit outputs, so offset = 4 (c0 + 2^32 c1) must
    # fit in 64 bits: counter word c1 is kept below 2^30
    tuples = [(0, 0, 0, 0, 0, 0), (0xffffffff, 0xffffffff, 0xffffffff, 2**30 - 1, 0xffffffff, 0xffffffff)]
    for _ in range(300):
        k0, k1, c0, c1, c2, c3 = (int(v) for v in g.integers(0, 2**32, 6, dtype=np.uint64))
        tuples.append((k0, k1, c0, c1 >> 2, c2, c3))
    tuples += [(int(a), int(b), int(c), 0, int(d), int(e)) for a, b, c, d, e in
               g.integers(0, 2**32, (50, 5), dtype=np.uint64)]
    ref = _rocrand_outputs(tuples)
    assert len(ref) == len(tuples)
    for t, r in zip(tuples, ref):
        k0, k1, c0, c1, c2, c3 = t
        assert orc.philox((c0, c1, c2, c3), (k0, k1)) == r, t


def test_philox_known_zero_vector(orc):
    # counter 0, key 0: the value rocRAND prints for seed 0, subsequence 0, offset 0
    assert orc.philox((0, 0, 0, 0), (0, 0)) == (0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8)


def test_u53_range_and_moments(orc):
    g = np.random.default_rng(2)
    w = g.integers(0, 2**32, (20000, 2), dtype=np.uint64)
    u = np.array([orc.u53(int(a), int(b)) for a, b in w])
    assert u.min() >= 0.0 and u.max() < 1.0
    assert orc.u53(0xffffffff, 0xffffffff) == 1.0 - 2.0**-53
    assert orc.u53(0, 0) == 0.0
    assert abs(u.mean() - 0.5) < 4 * np.sqrt(1 / 12 / u.size)
    assert stats.kstest(u, "uniform").pvalue > 1e-4


def test_normals_are_standard_normal(orc):
    z = np.concatenate([orc.island_normals(7, n, k, 1000) for n in range(5) for k in range(4)])
    assert abs(z.mean()) < 4 / np.sqrt(z.size)
    assert abs(z.var() - 1) < 4 * np.sqrt(2 / z.size)
    assert stats.kstest(z, "norm").pvalue > 1e-4
    # the pair (cos, sin) halves are uncorrelated
    assert abs(np.corrcoef(z[0::2], z[1::2])[0, 1]) < 4 / np.sqrt(z.size / 2)


def test_boxmuller_radius_and_angle(orc):
    # (z0, z1) = r (cos 2 pi v, sin 2 pi v) with r^2 = -2 log u1
    g = np.random.default_rng(3)
    for wa, wb in g.integers(0, 2**32, (500, 2), dtype=np.uint64):
        z0, z1 = orc.boxmuller(int(wa), int(wb))
        u1 = (int(wa) + 0.5) * 2.0**-32
        v = int(wb) * 2.0**-32
        assert np.isclose(z0 * z0 + z1 * z1, -2 * np.log(u1), rtol=1e-13)
        ang = np.arctan2(z1, z0) % (2 * np.pi)
        assert abs(((ang - 2 * np.pi * v + np.pi) % (2 * np.pi)) - np.pi) < 1e-12


def test_island_normals_layout(orc):
    # normal e of (n, k) comes from counter (e >> 2, k, n, NORMAL << 24), pairs (w0,w1), (w2,w3)
    z = orc.island_normals(99, 3, 5, 10)
    for e in range(10):
        w = orc.philox((e >> 2, 5, 3, orc.TAG_NORMAL << 24), (99, 0))
        pair = (e & 3) >> 1
        a, b = orc.boxmuller(w[2 * pair], w[2 * pair + 1])
        assert z[e] == (a if e % 2 == 0 else b)


@pytest.mark.parametrize("Q", [1, 2, 3, 7, 10, 1000])
def test_bounded_small_ranges_uniform(orc, Q):
    vals = np.array([orc.bounded(11, j, 2, 3, orc.TAG_SYS, Q) for j in range(6000)])
    assert vals.min() >= 0 and vals.max() < Q
    if Q == 1:
        assert (vals == 0).all()
        return
    bins = min(Q, 20)
    counts = np.bincount((vals * bins) // Q, minlength=bins)
    expect = np.array([len(range(b * Q // bins if b * Q % bins == 0 else b * Q // bins + 1,
                                     ((b + 1) * Q + bins - 1) // bins)) for b in range(bins)]) / Q * vals.size
    assert stats.chisquare(counts, expect).pvalue > 1e-4


def test_bounded_rejection_removes_bias(orc):
    # Q = 3 * 2^62: a plain multiply-shift of a uniform 64-bit word would give
    # the residues v mod 3 with probabilities 1/4, 1/2, 1/4 (it maps x -> floor(3x/4));
    # with rejection the outputs are uniform, so every residue has mass 1/3.
    Q = 3 << 62
    vals = [orc.bounded(5, j, 0, 0, orc.TAG_SYS, Q) for j in range(6000)]
    assert max(vals) < Q
    counts = np.bincount(np.array([v % 3 for v in vals]), minlength=3)
    assert stats.chisquare(counts).pvalue > 1e-4
