"""The row formation divides by constants (the closed-form moment terms'
1/(m + k + 1), the radiation length 360.8 mm) and by the voxel spacing with
a reciprocal rounded to nearest and two residual corrections by FMA:
q = a * y; q += (a - b q) y; q += (a - b q) y.  By Markstein's theorem the
second correction of an estimate within one ulp, with a correctly rounded
reciprocal, gives the correctly rounded quotient, so the rows stay bit-exact
against the oracle's plain division.

This test checks that claim on the host, in C with the C library's
correctly rounded fma, against IEEE division: random operands across a
wide exponent range and operands next to exact multiples of the divisor
(the hard cases for rounding), for every divisor the kernels use.
"""
import os
import shutil
import subprocess

import pytest

SRC = r"""
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>
static uint64_t s = 88172645463325252ull;
static uint64_t nx(void) { s ^= s << 13; s ^= s >> 7; s ^= s << 17; return s; }
static double div_rn(double a, double b, double y)
{
    double q = a * y;
    double r = fma(-q, b, a);
    q = fma(r, y, q);
    r = fma(-q, b, a);
    return fma(r, y, q);
}
int main(void)
{
    const double divs[] = {3, 5, 6, 7, 360.8, 1.0, 2.0, 2.5, 0.8, 1.1, 0.5, 4.0};
    long bad = 0, tot = 0;
    for (int d = 0; d < (int)(sizeof(divs) / sizeof(divs[0])); d++) {
        const double b = divs[d], y = 1.0 / b;
        for (long i = 0; i < 2000000; i++) {
            uint64_t u = nx();
            double a;
            if (i & 1) {
                uint64_t e = 1023 - 300 + (u % 600), m = nx() & ((1ull << 52) - 1);
                uint64_t bits = (e << 52) | m | ((u >> 63) << 63);
                memcpy(&a, &bits, 8);
            } else {
                double k = (double)(int64_t)(u % 100000000);
                a = k * b;
                uint64_t bits;
                memcpy(&bits, &a, 8);
                bits += (uint64_t)((int64_t)(nx() % 7) - 3);
                memcpy(&a, &bits, 8);
            }
            double q1 = a / b, q2 = div_rn(a, b, y);
            tot++;
            if (memcmp(&q1, &q2, 8) != 0) bad++;
        }
    }
    printf("%ld %ld\n", tot, bad);
    return 0;
}
"""


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_two_corrections_give_the_ieee_quotient(tmp_path):
    c = os.path.join(tmp_path, "div.c")
    exe = os.path.join(tmp_path, "div")
    with open(c, "w") as fh:
        fh.write(SRC)
    subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-o", exe, c, "-lm"])
    tot, bad = map(int, subprocess.check_output([exe], text=True).split())
    assert tot == 24_000_000
    assert bad == 0
