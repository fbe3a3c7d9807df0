"""Pins of the oracle's counter-based randomness.

Philox4x32-10 is checked against the known-answer vectors published with the
Random123 library (Salmon et al., SC'11) and against rocRAND's independent
host implementation; Bernoulli and coin rates against their binomial laws."""
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest

from oracle import oracle as O

# Random123 known-answer vectors for philox4x32_10: (counter, key, output)
KAT = [
    ((0, 0, 0, 0), (0, 0), (0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8)),
    ((0xFFFFFFFF,) * 4, (0xFFFFFFFF,) * 2, (0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD)),
    ((0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344), (0xA4093822, 0x299F31D0),
     (0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1)),
]


@pytest.mark.parametrize("ctr,key,out", KAT)
def test_philox_known_answers(ctr, key, out):
    assert tuple(int(v) for v in O.philox4x32_10(ctr, key)) == out


_ROCRAND_SRC = r"""
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>
#include <cstdlib>
int main(int argc, char** argv) {
  for (int i = 1; i + 5 < argc; i += 6) {
    unsigned long long k0 = strtoull(argv[i], 0, 0), k1 = strtoull(argv[i + 1], 0, 0);
    unsigned long long c0 = strtoull(argv[i + 2], 0, 0), c1 = strtoull(argv[i + 3], 0, 0);
    unsigned long long c2 = strtoull(argv[i + 4], 0, 0), c3 = strtoull(argv[i + 5], 0, 0);
    rocrand_device::philox4x32_10_engine eng(k0 | (k1 << 32), c2 | (c3 << 32),
                                             4ull * (c0 | (c1 << 32)));
    unsigned a = eng(), b = eng(), c = eng(), d = eng();
    printf("%u %u %u %u\n", a, b, c, d);
  }
}
"""


def test_philox_matches_rocrand_host_engine():
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc) or not os.path.exists(
            "/opt/rocm/include/rocrand/rocrand_philox4x32_10.h"):
        pytest.skip("rocRAND headers / hipcc not available")
    rng = np.random.default_rng(5)
    cases = []
    for _ in range(40):
        key = rng.integers(0, 2 ** 32, size=2, dtype=np.uint64)
        ctr = rng.integers(0, 2 ** 32, size=4, dtype=np.uint64)
        ctr[1] %= 2 ** 30  # the engine's offset argument is 4*(c0 | c1<<32)
        cases.append((key, ctr))
    with tempfile.TemporaryDirectory() as d:
        src = os.path.join(d, "kat.cpp")
        exe = os.path.join(d, "kat")
        with open(src, "w") as fh:
            fh.write(_ROCRAND_SRC)
        subprocess.check_call([hipcc, "-x", "hip", "--offload-host-only", "-O1", src, "-o",
                               exe], stderr=subprocess.DEVNULL)
        args = []
        for key, ctr in cases:
            args += [str(int(key[0])), str(int(key[1]))] + [str(int(c)) for c in ctr]
        out = subprocess.check_output([exe] + args, text=True).split("\n")
    for (key, ctr), line in zip(cases, out):
        want = [int(t) for t in line.split()]
        got = [int(v) for v in O.philox4x32_10(ctr.astype(np.uint32), key.astype(np.uint32))]
        assert got == want


def test_threshold_exact_values():
    assert O.threshold(0.0) == 0
    assert O.threshold(-1.0) == 0
    assert O.threshold(0.5) == 2 ** 31
    assert O.threshold(0.25) == 2 ** 30
    assert O.threshold(1.0) == 2 ** 32 - 1
    assert O.threshold(0.05) == int(np.floor(0.05 * 2.0 ** 32))
    assert O.threshold(2.0 ** -32) == 1


def test_uniform_is_word_of_block():
    # shot s reads word s mod 4 of the block at counter (site, cycle, s div 4, tag)
    seed = (7 << 32) | 3
    for shot in range(8):
        blk = O.philox4x32_10((11, 2, shot // 4, 1), (3, 7))
        assert O.uniform(seed, 11, 2, shot, 1) == int(blk[shot % 4])


def test_bernoulli_rate_within_binomial_bounds():
    o = O.Oracle(6)
    for p in (0.02, 0.05, 0.3):
        bits = np.zeros((64, o.n_edges), np.uint8)
        o.sample_noise(bits, 0, p, seed=1, cycle=3)
        n = bits.size
        th = O.threshold(p) / 2.0 ** 32
        sigma = np.sqrt(n * th * (1 - th))
        assert abs(bits.sum() - n * th) < 5 * sigma


def test_noise_xors_and_is_reproducible():
    o = O.Oracle(4)
    a = np.zeros((5, o.n_faces), np.uint8)
    o.sample_noise(a, 1, 0.2, seed=9, cycle=1, shot0=64)
    b = a.copy()
    o.sample_noise(b, 1, 0.2, seed=9, cycle=1, shot0=64)
    assert b.sum() == 0  # xor twice with the same draws cancels
    c = np.zeros((5, o.n_faces), np.uint8)
    o.sample_noise(c, 1, 0.2, seed=9, cycle=2, shot0=64)
    assert not np.array_equal(a, c)
    # shot k of a batch starting at shot0 equals shot shot0+k alone
    d = np.zeros((1, o.n_faces), np.uint8)
    o.sample_noise(d, 1, 0.2, seed=9, cycle=1, shot0=66)
    assert np.array_equal(d[0], a[2])


def test_uniform_chi_square():
    vals = np.array([O.uniform(1, i, 0, s, 0) for i in range(64) for s in range(64)],
                    dtype=np.uint64)
    hist = np.bincount((vals >> np.uint64(28)).astype(np.int64), minlength=16)
    exp = vals.size / 16
    chi2 = ((hist - exp) ** 2 / exp).sum()
    assert chi2 < 45  # 15 dof, p ~ 1e-4


def test_coin_rate_and_layout():
    coins = np.array([O.coin(1, e, 2, 0, s) for e in range(50) for s in range(128)])
    n = coins.size
    assert abs(coins.sum() - n / 2) < 5 * np.sqrt(n / 4)
    blk = O.philox4x32_10((5, 2, 1, 2 + 3), (1, 0))
    word = int(blk[0]) | (int(blk[1]) << 32)
    for s in range(64, 128):
        assert O.coin(1, 5, 2, 3, s) == (word >> (s - 64)) & 1
