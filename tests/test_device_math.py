"""The exponential the HIP kernels evaluate (2^t = 2^k 2^f, 2^f = exp(f ln 2)
by the polynomial kExpPoly of md_internal.h), checked on the host: the
coefficients as compiled (doubles parsed from the header), evaluated exactly,
against exp in 50-digit decimal arithmetic over the whole reduced interval."""
import os
import re
from decimal import Decimal as D, getcontext

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HDR = os.path.join(ROOT, "paper_1212_6332_amd", "csrc", "md_internal.h")


def coefficients():
    text = open(HDR).read()
    deg = int(re.search(r"constexpr int kExpDeg = (\d+);", text).group(1))
    body = re.search(r"kExpPoly\[kExpDeg \+ 1\] = \{(.*?)\};", text, re.S).group(1)
    c = [float(x) for x in body.replace("\n", " ").split(",") if x.strip()]
    assert len(c) == deg + 1
    return c


def test_exp_polynomial_error():
    getcontext().prec = 50
    c = coefficients()
    assert c[0] == 1.0
    h = D(2).ln() / 2          # |f ln 2| <= ln(2)/2 after rounding t to the nearest integer
    worst = D(0)
    for i in range(4001):
        x = -h + 2 * h * i / 4000
        p = D(0)
        for a in reversed(c):
            p = p * x + D(a)
        worst = max(worst, abs(p / x.exp() - 1))
    assert worst < D("3.5e-16"), worst
