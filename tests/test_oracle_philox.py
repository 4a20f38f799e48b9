"""Pins for the oracle's counter-based generator (Philox4x32-10, Salmon et al.,
SC'11) and for the FP32 control map.

The oracle's C Philox is checked against
  * a word-width-generic numpy Philox written here, whose 4x64 instantiation
    must reproduce numpy.random.Philox raw output (this pins the round
    structure: multiplier words, output permutation, key schedule), and
  * PyTorch's header-only Philox4x32-10 engine (an independent third-party
    implementation), compiled into a tiny host program at test time.
"""

import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest

import oracle

M32 = (1 << 32) - 1
M64 = (1 << 64) - 1
PHILOX_4x64 = dict(w=64, mult=(0xD2E7470EE14C6C93, 0xCA5A826395121157),
                   weyl=(0x9E3779B97F4A7C15, 0xBB67AE8584CAA73B))
PHILOX_4x32 = dict(w=32, mult=(0xD2511F53, 0xCD9E8D57), weyl=(0x9E3779B9, 0xBB67AE85))


def philox_generic(ctr, key, w, mult, weyl, rounds=10):
    mask = (1 << w) - 1
    c = [int(v) for v in ctr]
    k = [int(v) for v in key]
    for _ in range(rounds):
        p0 = mult[0] * c[0]
        p1 = mult[1] * c[2]
        hi0, lo0 = p0 >> w, p0 & mask
        hi1, lo1 = p1 >> w, p1 & mask
        c = [hi1 ^ c[1] ^ k[0], lo1, hi0 ^ c[3] ^ k[1], lo0]
        k = [(k[0] + weyl[0]) & mask, (k[1] + weyl[1]) & mask]
    return c


def test_generic_4x64_matches_numpy_philox():
    rng = np.random.default_rng(123)
    for _ in range(20):
        key = [int(x) for x in rng.integers(0, 2**63, size=2)]
        ctr = [int(x) for x in rng.integers(0, 2**63, size=4)]
        g = np.random.Philox(key=key, counter=ctr)
        raw = [int(x) for x in g.random_raw(4)]
        # numpy increments the 256-bit counter before each block
        c = ctr[:]
        c[0] = (c[0] + 1) & M64
        carry = c[0] == 0
        for i in range(1, 4):
            if not carry:
                break
            c[i] = (c[i] + 1) & M64
            carry = c[i] == 0
        assert philox_generic(c, key, **PHILOX_4x64) == raw


def test_oracle_philox_matches_generic_4x32():
    rng = np.random.default_rng(7)
    for _ in range(200):
        key = [int(x) for x in rng.integers(0, 2**32, size=2)]
        ctr = [int(x) for x in rng.integers(0, 2**32, size=4)]
        want = philox_generic(ctr, key, **PHILOX_4x32)
        got = [int(x) for x in oracle.philox4x32_10(ctr, key)]
        assert got == want


TORCH_PROG = r"""
#include <ATen/core/PhiloxRNGEngine.h>
#include <cstdio>
#include <cstdlib>
int main(int argc, char** argv) {
  // args: seed subseq offset  -> four words of the block at counter (offset, subseq)
  unsigned long long seed = strtoull(argv[1], 0, 10);
  unsigned long long sub = strtoull(argv[2], 0, 10);
  unsigned long long off = strtoull(argv[3], 0, 10);
  at::philox_engine e(seed, sub, off);
  for (int i = 0; i < 4; ++i) printf("%u\n", e());
  return 0;
}
"""


def _torch_include():
    try:
        import torch.utils.cpp_extension as ce
        for p in ce.include_paths():
            if os.path.exists(os.path.join(p, "ATen", "core", "PhiloxRNGEngine.h")):
                return p
    except Exception:
        return None
    return None


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_oracle_philox_matches_torch_engine():
    inc = _torch_include()
    if inc is None:
        pytest.skip("torch Philox header not found")
    d = tempfile.mkdtemp()
    src = os.path.join(d, "ph.cpp")
    exe = os.path.join(d, "ph")
    with open(src, "w") as f:
        f.write(TORCH_PROG)
    r = subprocess.run(["g++", "-std=c++17", "-O1", "-I", inc, src, "-o", exe],
                       capture_output=True, text=True)
    if r.returncode != 0:
        pytest.skip("could not compile the torch Philox engine: " + r.stderr[-300:])
    rng = np.random.default_rng(99)
    for _ in range(12):
        seed = int(rng.integers(0, 2**63))
        sub = int(rng.integers(0, 2**63))
        off = int(rng.integers(0, 2**40))
        out = subprocess.run([exe, str(seed), str(sub), str(off)], capture_output=True,
                             text=True, check=True).stdout.split()
        want = [int(x) for x in out]
        ctr = [off & M32, off >> 32, sub & M32, sub >> 32]
        key = [seed & M32, seed >> 32]
        got = [int(x) for x in oracle.philox4x32_10(ctr, key)]
        assert got == want


def test_philox_words_uniform_chi2():
    # 4 * 20000 words from consecutive counters, 16 buckets on the top nibble
    words = []
    for i in range(20000):
        words.extend(int(x) for x in oracle.philox4x32_10([i, 5, 0, 0], [17, 0]))
    top = np.array(words, np.uint64) >> np.uint64(28)
    counts = np.bincount(top.astype(np.int64), minlength=16)
    exp = len(words) / 16
    chi2 = float(((counts - exp) ** 2 / exp).sum())
    assert chi2 < 45.0  # 15 dof, p ~ 1e-4


def _fma_f32_exact(d, r, lo):
    # d (FP32) * r (24-bit fraction) is exact in FP64, and for the control
    # boxes used here d*r + lo is exact in FP64 as well, so one rounding to
    # FP32 gives the correctly rounded fused multiply-add.
    return np.float32(np.float64(d) * np.float64(r) + np.float64(lo))


@pytest.mark.parametrize("lo,hi", [(-1.0, 1.0), (0.0, 19.62), (-0.1, 0.1), (-10.0, 10.0)])
def test_control_map_fp32(lo, hi):
    lo32, hi32 = np.float32(lo), np.float32(hi)
    d = np.float32(hi32 - lo32)
    rng = np.random.default_rng(5)
    ws = list(rng.integers(0, 2**32, size=2000)) + [0, 255, 256, 2**32 - 1, 2**31]
    for w in ws:
        r = np.float32((int(w) >> 8) * 2.0**-24)
        want = _fma_f32_exact(d, r, lo32)
        got = oracle.control_map(int(w), lo32, hi32)
        assert got == want
        assert lo32 <= got <= hi32
