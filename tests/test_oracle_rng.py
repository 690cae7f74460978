"""Pins of the oracle's random streams (CPU only).

* Philox4x32-10 against rocRAND's implementation of the same generator
  (Salmon et al., SC'11), compiled here for the host from its header, and
  against the known-answer vectors published with the generator's reference
  implementation (Random123) for 10 rounds;
* the uniform lattice (exact values);
* Box-Muller: the polar identities fix which word is the radius and which the
  angle; a path block's six normals read disjoint bits; the normals are
  N(0,1) by a KS test and uncorrelated across their positions in a block.
"""
import math
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest
from scipy import stats

import oracle

ROCRAND_HDR = "/opt/rocm/include/rocrand/rocrand_philox4x32_10.h"

_ROCRAND_PROG = r"""
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>
int main() {
    unsigned long long seed, subseq, offset;
    while (std::scanf("%llu %llu %llu", &seed, &subseq, &offset) == 3) {
        rocrand_state_philox4x32_10 s;
        rocrand_init(seed, subseq, offset, &s);
        uint4 r = rocrand4(&s);
        std::printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
    }
    return 0;
}
"""


@pytest.fixture(scope="module")
def rocrand_exe():
    if not os.path.exists(ROCRAND_HDR) or shutil.which("g++") is None:
        pytest.skip("rocRAND header or g++ not available")
    d = tempfile.mkdtemp(prefix="pps_rocrand_")
    src = os.path.join(d, "rr.cpp")
    exe = os.path.join(d, "rr")
    with open(src, "w") as f:
        f.write(_ROCRAND_PROG)
    subprocess.run(["g++", "-std=c++17", "-O1", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
                    src, "-o", exe], check=True)
    yield exe
    shutil.rmtree(d, ignore_errors=True)


def test_philox_matches_rocrand(rocrand_exe):
    """rocRAND keys Philox by the 64-bit seed and puts (offset/4) in counter
    words 0-1 and the subsequence in words 2-3; with offset = 4*(block +
    purpose*2^32) and subsequence = draw this is exactly the stream layout
    (block, purpose, lo32 draw, hi32 draw) keyed by (lo32 seed, hi32 seed)."""
    rng = np.random.default_rng(12345)
    cases = []
    for _ in range(3000):
        seed = int(rng.integers(0, 2**64, dtype=np.uint64))
        draw = int(rng.integers(0, 2**64, dtype=np.uint64))
        block = int(rng.integers(0, 2**32, dtype=np.uint64))
        purpose = int(rng.integers(0, 3))
        cases.append((seed, draw, block, purpose))
    cases += [(0, 0, 0, 0), (1, 0, 0, 1), (2**64 - 1, 2**64 - 1, 2**32 - 1, 1), (1, 12345, 249, 1)]
    lines = "".join(f"{s} {d} {4 * (b + (p << 32))}\n" for s, d, b, p in cases)
    res = subprocess.run([rocrand_exe], input=lines, capture_output=True, text=True, check=True)
    ref = np.array([[int(t) for t in ln.split()] for ln in res.stdout.strip().splitlines()],
                   dtype=np.uint64)
    assert ref.shape == (len(cases), 4)
    got = np.array([oracle.stream_block(s, d, b, p) for s, d, b, p in cases], dtype=np.uint64)
    np.testing.assert_array_equal(got, ref)


def test_philox_raw_interface_consistent():
    ctr = [7, 1, 0xDEADBEEF, 3]
    key = [0x12345678, 0x9ABCDEF0]
    a = oracle.philox(ctr, key)
    b = oracle.stream_block((key[1] << 32) | key[0], (3 << 32) | 0xDEADBEEF, 7, 1)
    np.testing.assert_array_equal(a, b)


def test_uniform_lattice_exact():
    assert oracle.uniform(0) == 2.0**-24
    assert oracle.uniform(0xFFFFFFFF) == 1.0 - 2.0**-24
    assert oracle.uniform(511) == 2.0**-24  # low 9 bits are dropped
    assert oracle.uniform(512) == 3 * 2.0**-24
    rng = np.random.default_rng(0)
    for w in rng.integers(0, 2**32, size=2000, dtype=np.uint64):
        u = oracle.uniform(int(w))
        k = u * 2**24
        assert k == int(k) and int(k) % 2 == 1 and 1 <= k <= 2**24 - 1
        assert float(np.float32(u)) == u  # exact in single precision
        assert int(k) == 2 * (int(w) >> 9) + 1


def test_box_muller_polar_identities():
    """z0 = r cos(2 pi u1), z1 = r sin(2 pi u1) with r^2 = -2 ln u0: the
    radius comes from the first word and the angle from the second."""
    rng = np.random.default_rng(1)
    for w0, w1 in rng.integers(0, 2**32, size=(2000, 2), dtype=np.uint64):
        z0, z1 = oracle.box_muller(int(w0), int(w1))
        u0, u1 = oracle.uniform(int(w0)), oracle.uniform(int(w1))
        assert math.isclose(z0 * z0 + z1 * z1, -2.0 * math.log(u0), rel_tol=1e-12, abs_tol=1e-300)
        ang = math.atan2(z1, z0) % (2 * math.pi)
        assert math.isclose(ang, 2 * math.pi * u1, rel_tol=1e-9, abs_tol=1e-9) or \
            math.isclose(abs(ang - 2 * math.pi * u1), 2 * math.pi, rel_tol=1e-9)


def test_path_normals_are_standard_normal():
    spec_seed = 99
    z = np.array([oracle.path_normal(spec_seed, d, n) for d in range(500) for n in range(200)])
    assert abs(z.mean()) < 4 / math.sqrt(len(z))
    assert abs(z.var() - 1) < 4 * math.sqrt(2 / len(z))
    assert stats.kstest(z, "norm").pvalue > 1e-4
    # |z| is bounded by the radius lattice: sqrt(-2 ln 2^-24) = 5.77
    assert np.abs(z).max() <= math.sqrt(-2 * math.log(2.0**-24)) + 1e-12
    # the six positions of a block (200 normals per draw = 33 whole blocks)
    blocks = z.reshape(500, 200)[:, :198].reshape(-1, 6)
    c = np.corrcoef(blocks.T)
    assert np.abs(c - np.eye(6)).max() < 5 / math.sqrt(len(blocks))


def test_path_normal_block_layout():
    """Normals 6b..6b+5 come from PATH block b: pair i takes its radius
    uniform from word i (top 23 bits) and its angle uniform from the low 9
    bits of word i followed by bits 22-10i..31-10i of word 3."""
    seed, draw = 5, 77
    for b in (0, 1, 166, 333):
        w = [int(v) for v in oracle.stream_block(seed, draw, b, 1)]
        z = [oracle.path_normal(seed, draw, 6 * b + j) for j in range(6)]
        for i in range(3):
            u0 = oracle.uniform(w[i])
            m = ((w[i] & 0x1FF) << 10) | ((w[3] >> (22 - 10 * i)) & 0x3FF)
            u1 = m / 2.0**19
            assert oracle.angle_uniform(w[i], w[3], i) == u1
            r = math.sqrt(-2.0 * math.log(u0))
            assert math.isclose(z[2 * i], r * math.cos(2 * math.pi * u1), rel_tol=1e-15, abs_tol=1e-15)
            assert math.isclose(z[2 * i + 1], r * math.sin(2 * math.pi * u1), rel_tol=1e-15, abs_tol=1e-15)


def test_path_normal_bits_are_disjoint():
    """The 19-bit angle indices of the three pairs and the three radius
    indices read disjoint bits of the block: flipping any one of the 126
    used bits changes exactly one of the six uniforms, and flipping one of
    the two unused bits (word 3, bits 0 and 1) changes none."""
    rng = np.random.default_rng(4)
    w = [int(v) for v in rng.integers(0, 2**32, size=4, dtype=np.uint64)]

    def uniforms(ws):
        return [oracle.uniform(ws[i]) for i in range(3)] + \
               [oracle.angle_uniform(ws[i], ws[3], i) for i in range(3)]

    base = uniforms(w)
    used = 0
    for word in range(4):
        for bit in range(32):
            ws = list(w)
            ws[word] ^= 1 << bit
            changed = sum(a != b for a, b in zip(base, uniforms(ws)))
            if word == 3 and bit < 2:
                assert changed == 0
            else:
                assert changed == 1, (word, bit)
                used += 1
    assert used == 126


# Known-answer vectors of Philox4x32 with 10 rounds (counter, key, output),
# as published with the generator's reference implementation (Random123).
PHILOX_KAT = [
    ((0x00000000, 0x00000000, 0x00000000, 0x00000000), (0x00000000, 0x00000000),
     (0x6627e8d5, 0xe169c58d, 0xbc57ac4c, 0x9b00dbd8)),
    ((0xffffffff, 0xffffffff, 0xffffffff, 0xffffffff), (0xffffffff, 0xffffffff),
     (0x408f276d, 0x41c83b0e, 0xa20bc7c6, 0x6d5451fd)),
    ((0x243f6a88, 0x85a308d3, 0x13198a2e, 0x03707344), (0xa4093822, 0x299f31d0),
     (0xd16cfe09, 0x94fdcceb, 0x5001e420, 0x24126ea1)),
]


@pytest.mark.parametrize("ctr,key,expect", PHILOX_KAT)
def test_philox_known_answers(ctr, key, expect):
    assert [int(v) for v in oracle.philox(ctr, key)] == list(expect)
    # the same block through the stream layout: counter (block, purpose,
    # lo32 draw, hi32 draw), key (lo32 seed, hi32 seed)
    seed = key[0] | (key[1] << 32)
    draw = ctr[2] | (ctr[3] << 32)
    assert [int(v) for v in oracle.stream_block(seed, draw, ctr[0], ctr[1])] == list(expect)

