"""The wall-function coefficient tables compiled into the library, read from
their header and evaluated on the host (no GPU) the way the device evaluates
them, against psi = 1 - 2 E_3 and psi'/2 = E_2 from mpmath (Sec. 3.1)."""
import os
import re

import mpmath
import numpy as np
import pytest

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                      "paper_1603_08221_amd", "csrc", "e1_table.h")


def _define(text, name):
    return int(re.search(rf"#define {name} \(?(-?\d+)\)?", text).group(1))


def _array(text, name):
    body = re.search(rf"LBSEP_TBL\({name}\)\[[^=]*=\s*\{{(.*?)\}};", text, re.S).group(1)
    return np.array([float(v.rstrip("f")) for v in re.findall(r"[-+0-9.eE]+f?", body)])


@pytest.fixture(scope="module")
def table():
    text = open(HEADER).read()
    lo, per, n, deg = (_define(text, k) for k in ("LBSEP_PW_F64_LO_OCT", "LBSEP_PW_F64_PER_OCT",
                                                    "LBSEP_PW_F64_N", "LBSEP_PW_F64_DEG"))
    c = _array(text, "lbsep_wall_pw_f64").reshape(n, 2, deg + 1)
    return lo, per, c


def _eval(a, lo, per, c):
    """Part index from the exponent and the top three mantissa bits, the local
    variable s = 2^(4-e) a - (17 + 2m), Horner with fused multiply-adds in
    exact arithmetic rounded once per step (as the device's v_fma_f64)."""
    m_, e = np.frexp(a)               # a = m_ 2^e, m_ in [0.5, 1)
    e = int(e) - 1                    # a = (1.f) 2^e
    m = int((a / 2.0 ** e - 1.0) * per)
    q = (e - lo) * per + m
    s = a * 2.0 ** (4 - e) - (17 + 2 * m)
    assert -1.0 <= s < 1.0
    out = []
    for which in (0, 1):
        p = mpmath.mpf(c[q, which, -1])
        for k in range(c.shape[2] - 2, -1, -1):
            p = mpmath.mpf(float(p * mpmath.mpf(s) + mpmath.mpf(c[q, which, k])))
        out.append(float(p))
    return out


def test_piecewise_table_layout(table):
    lo, per, c = table
    assert per == 8 and lo == -20 and c.shape[0] == (6 - lo) * per
    assert np.all(np.isfinite(c))


def test_piecewise_table_against_mpmath(table):
    lo, per, c = table
    mpmath.mp.dps = 40
    rng = np.random.default_rng(7)
    # every part: its two ends and a random point inside
    xs = []
    for q in range(c.shape[0]):
        e, m = lo + q // per, q % per
        a0, a1 = 2.0 ** e * (1 + m / per), 2.0 ** e * (1 + (m + 1) / per)
        xs += [a0, np.nextafter(a1, 0.0), a0 + (a1 - a0) * rng.random()]
    worst_psi = worst_h = 0.0
    for a in xs:
        psi, h = _eval(a, lo, per, c)
        ref_psi = 1 - 2 * mpmath.expint(3, mpmath.mpf(a))
        ref_h = mpmath.expint(2, mpmath.mpf(a))
        worst_psi = max(worst_psi, abs(float((psi - ref_psi) / ref_psi)))
        worst_h = max(worst_h, abs(float(h - ref_h)))
    assert worst_psi < 4e-16, worst_psi
    assert worst_h < 4e-16, worst_h
