"""The FP64 -> bfloat16 rounding the BF16 paths use (csrc/bf16_round.h),
compiled for the host with g++ and checked against round-to-nearest-even
computed exactly with fractions: the nearest point of the bfloat16 grid
(8 significant bits, exponents down to -126, subnormal spacing 2^-133,
largest finite (2 - 2^-7) 2^127), ties to the even significand, and
overflow to infinity from (2 - 2^-8) 2^127 on.

The cases include the one where two roundings (FP64 -> FP32 -> BF16)
differ from one: 1 + 2^-8 + 2^-30.
"""

import math
import os
import struct
import subprocess
from fractions import Fraction

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER_DIR = os.path.join(ROOT, "paper_2307_00719_amd", "csrc")

DRIVER = r"""
#include <stdio.h>
#include <stdint.h>
#include <string.h>
#include "bf16_round.h"
int main() {
  unsigned long long u;
  while (scanf("%llx", &u) == 1) {
    double x;
    memcpy(&x, &u, 8);
    printf("%04x\n", (unsigned)bf16_bits_rne(x));
  }
  return 0;
}
"""


@pytest.fixture(scope="module")
def rounder(tmp_path_factory):
    d = tmp_path_factory.mktemp("bf16")
    src, exe = d / "drv.cpp", d / "drv"
    src.write_text(DRIVER)
    subprocess.run(["g++", "-O2", "-std=c++17", "-I", HEADER_DIR, str(src), "-o", str(exe)],
                   check=True)

    def run(xs):
        inp = "\n".join(format(struct.unpack("<Q", struct.pack("<d", float(x)))[0], "x")
                        for x in xs)
        out = subprocess.run([str(exe)], input=inp, capture_output=True, text=True,
                             check=True).stdout.split()
        return [int(h, 16) for h in out]

    return run


def bf16_value(bits):
    """The value a bfloat16 bit pattern stands for (upper half of binary32)."""
    return struct.unpack("<f", struct.pack("<I", bits << 16))[0]


def nearest_even(x):
    """Round-to-nearest-even onto the bfloat16 grid, as an exact Fraction
    (or +-inf), from the definition."""
    if x == 0:
        return Fraction(0)
    m, e = math.frexp(abs(x))                    # |x| = m 2^e, 1/2 <= m < 1
    q = max(e - 1 - 7, -133)                     # spacing exponent at |x|
    k = round(Fraction(abs(x)) / Fraction(2) ** q)   # Fraction round: ties to even
    v = k * Fraction(2) ** q
    if v >= Fraction(2) ** 128:
        return math.copysign(math.inf, x)
    return v if x > 0 else -v


def cases():
    one = 1.0
    xs = [0.0, -0.0, 1.0, -1.0, 0.5, 3.0, math.pi, -math.e, 1e-3, 123456.789,
          one + 2.0 ** -8 + 2.0 ** -30,            # two roundings give 1, one gives 1 + 2^-7
          -(one + 2.0 ** -8 + 2.0 ** -30),
          one + 2.0 ** -8,                         # exact tie, even -> 1
          one + 3 * 2.0 ** -8,                     # exact tie, odd -> up
          one + 2.0 ** -8 - 2.0 ** -52,            # just under the tie
          (2 - 2.0 ** -7) * 2.0 ** 127,            # largest finite
          (2 - 2.0 ** -8) * 2.0 ** 127,            # tie to the carry: infinity
          (2 - 2.0 ** -8 - 2.0 ** -40) * 2.0 ** 127,   # just under: largest finite
          1e300, -1e300, 2.0 ** -126, 2.0 ** -127, 2.0 ** -133, 3 * 2.0 ** -135,
          2.0 ** -134, 2.0 ** -134 + 2.0 ** -170,  # half the subnormal spacing: tie to 0, above
          (2.0 ** -126) * (1 - 2.0 ** -9),         # subnormal that rounds up into the normals
          1e-45, 5e-324, -5e-324, 1e-310]
    rng = np.random.default_rng(2307)
    xs += list(rng.standard_normal(300) * 10.0 ** rng.integers(-40, 40, 300))
    xs += list(np.ldexp(rng.random(200) + 1.0, rng.integers(-140, 129, 200)))
    xs += [float(np.float32(v)) for v in rng.standard_normal(200)]   # binary32-exact
    return xs


def test_bf16_rounding_is_nearest_even(rounder):
    xs = cases()
    got = rounder(xs)
    bad = []
    for x, b in zip(xs, got):
        want = nearest_even(x)
        v = bf16_value(b)
        ok = v == want
        if ok and v == 0:
            ok = math.copysign(1.0, v) == math.copysign(1.0, x)
        if not ok:
            bad.append((x, hex(b), v, float(want)))
    assert not bad, bad[:5]


def test_bf16_double_rounding_case(rounder):
    x = 1.0 + 2.0 ** -8 + 2.0 ** -30
    two_step = float(np.float32(x))
    assert two_step == 1.0 + 2.0 ** -8               # FP32 keeps the tie
    assert bf16_value(rounder([x])[0]) == 1.0 + 2.0 ** -7


def test_bf16_special_values(rounder):
    b = rounder([math.inf, -math.inf, math.nan])
    assert b[0] == 0x7F80 and b[1] == 0xFF80
    assert (b[2] & 0x7F80) == 0x7F80 and (b[2] & 0x7F) != 0
