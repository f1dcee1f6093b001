"""Generate the device tables for E1 used by the mean-free-path wall function.

Writes ``e1_table.h`` next to this script. Run: ``python gen_e1_table.py``.

Method (our own, from the mathematics; no vendor constants):
* 0 < a <= 1: from E1(a) = -gamma - ln a - sum_{k>=1} (-a)^k / (k k!)
  (Abramowitz & Stegun 5.1.11) the wall function and its half-derivative split
  into entire power series plus one logarithm:
    psi(a) = 1 + (a - 1) e^-a - a^2 E1(a) = A(a) + a^2 ln a,
    h(a)   = e^-a - a E1(a)              = B(a) + a ln a,
  A(a) = sum_n alpha_n a^n with alpha_0 = 0, alpha_1 = 2, alpha_2 = gamma - 3/2,
         alpha_n = (-1)^(n-1) (1/(n-1)! + 1/n!) + (-1)^n / ((n-2) (n-2)!) (n >= 3),
  B(a) = sum_n beta_n a^n with beta_0 = 1, beta_1 = gamma - 1,
         beta_n = (-1)^n / n! + (-1)^(n-1) / ((n-1) (n-1)!) (n >= 2).
  Neither needs an exponential, and psi ~ 2a carries no cancellation at small a.
  The table holds alpha_n and beta_n rounded to the target precision (checked
  here against mpmath).
* FP64, 1 < a < 2^NSEG: G(a) = a e^a E1(a) is smooth and bounded in (0.59, 1). On each
  octave [2^s, 2^(s+1)) it is replaced by a Chebyshev interpolant in
  t = (2a - 3 * 2^s) / 2^s, evaluated by Clenshaw's recurrence. Coefficients
  are computed here with mpmath at 50 digits from Chebyshev-node samples of
  the exact G (mpmath.e1), and truncated where the remaining terms are below
  the target tolerance (padded to one uniform degree per precision so the
  device loop has no divergent trip count).
* FP64, a >= 2^NSEG: the wall function is 1 to the target precision (its deficit is
  about 2 e^-a / a) and the device code does not evaluate E1 there.
* FP32 only, a > 1: one rational function replaces the octaves,
  G(a) ~ P(u) / Q(u) with u = 1/a in (0, 1], degrees (5, 5), Q(0) = 1. Fitted
  here by linearised least squares (Sanathanan-Koerner iteration: minimise
  |G Q - P| / Q_previous on Chebyshev-distributed samples of u), followed by
  Lawson reweighting towards the minimax error; checked against mpmath on
  [1, 10^4] with the coefficients rounded to float. With positive coefficients the FP32 Horner evaluation stays within
  a few ulp, and e^-a underflows to 0 long before the fit loses accuracy, so
  no cut-off branch is needed.
"""
import numpy as np
import os

import mpmath as mp

mp.mp.dps = 50

HERE = os.path.dirname(os.path.abspath(__file__))


def g_exact(a):
    a = mp.mpf(a)
    return a * mp.exp(a) * mp.e1(a)


def cheb_coeffs(lo, hi, n=80):
    """a_k of f(t) ~ sum_k a_k T_k(t) on [lo, hi] (Chebyshev interpolation, n nodes)."""
    lo, hi = mp.mpf(lo), mp.mpf(hi)
    nodes = [mp.cos(mp.pi * (j + mp.mpf(1) / 2) / n) for j in range(n)]
    vals = [g_exact((hi - lo) / 2 * t + (hi + lo) / 2) for t in nodes]
    out = []
    for k in range(n):
        c = 2 * mp.fsum(v * mp.cos(mp.pi * k * (j + mp.mpf(1) / 2) / n) for j, v in enumerate(vals)) / n
        out.append(c)
    out[0] /= 2
    return out


def alpha_coeffs(nterms):
    out = [mp.mpf(0), mp.mpf(2), mp.euler - mp.mpf(3) / 2]
    for n in range(3, nterms):
        out.append((-1) ** (n - 1) * (1 / mp.factorial(n - 1) + 1 / mp.factorial(n))
                   + (-1) ** n / ((n - 2) * mp.factorial(n - 2)))
    return out


def beta_coeffs(nterms):
    out = [mp.mpf(1), mp.euler - 1]
    for n in range(2, nterms):
        out.append((-1) ** n / mp.factorial(n) + (-1) ** (n - 1) / ((n - 1) * mp.factorial(n - 1)))
    return out


def check_small(nterms, tol):
    """A + a^2 ln a and B + a ln a against mpmath's psi and h on (0, 1]."""
    al, be = alpha_coeffs(nterms), beta_coeffs(nterms)
    worst = mp.mpf(0)
    for q in range(1, 101):
        a = mp.mpf(q) / 100
        psi = 1 + (a - 1) * mp.exp(-a) - a * a * mp.e1(a)
        h = mp.exp(-a) - a * mp.e1(a)
        A = mp.fsum(c * a ** n for n, c in enumerate(al))
        B = mp.fsum(c * a ** n for n, c in enumerate(be))
        worst = max(worst, abs(A + a * a * mp.log(a) - psi), abs(B + a * mp.log(a) - h))
    assert worst < tol, worst
    return worst


def build(nseg, tol):
    segs = []
    deg = 0
    for s in range(nseg):
        c = cheb_coeffs(2 ** s, 2 ** (s + 1))
        d = len(c) - 1
        while d > 0 and abs(c[d]) < tol:
            d -= 1
        deg = max(deg, d)
        segs.append(c)
    return [seg[:deg + 1] for seg in segs], deg


def clenshaw(coef, t):
    b1 = b2 = mp.mpf(0)
    for a in reversed(coef[1:]):
        b1, b2 = a + 2 * t * b1 - b2, b1
    return coef[0] + t * b1 - b2


def check(segs, nseg):
    worst = mp.mpf(0)
    for s in range(nseg):
        lo, hi = 2 ** s, 2 ** (s + 1)
        for q in range(97):
            a = mp.mpf(lo) + (hi - lo) * mp.mpf(q) / 96
            t = (2 * a - (hi + lo)) / (hi - lo)
            worst = max(worst, abs(clenshaw(segs[s], t) - g_exact(a)))
    return worst


def rational_fit(m=5, n=5, nsamp=4000, sk_iters=30, lawson_iters=60):
    """P (degree m) and Q (degree n, Q(0) = 1) with G(1/u) ~ P(u) / Q(u) on [0, 1]."""
    uu = 0.5 - 0.5 * np.cos(np.pi * (np.arange(nsamp) + 0.5) / nsamp)
    gg = np.array([float(g_exact(1 / mp.mpf(u))) for u in uu])
    vp = np.vander(uu, m + 1, increasing=True)
    vq = np.vander(uu, n + 1, increasing=True)[:, 1:]
    qprev = np.ones_like(uu)
    w = np.ones_like(uu)
    for it in range(sk_iters + lawson_iters):
        A = np.hstack([vp, -gg[:, None] * vq]) / qprev[:, None] * np.sqrt(w)[:, None]
        b = gg / qprev * np.sqrt(w)
        c = np.linalg.lstsq(A, b, rcond=None)[0]
        p, q = c[:m + 1], np.concatenate([[1.0], c[m + 1:]])
        qprev = np.polyval(q[::-1], uu)
        r = np.polyval(p[::-1], uu) / qprev - gg
        if it >= sk_iters:
            w = w * np.abs(r)
            w /= w.sum()
    return p, q


def check_rational(p, q, tol):
    """The rational in exact arithmetic (coefficients rounded to float) against G."""
    p32 = [mp.mpf(float(np.float32(c))) for c in p]
    q32 = [mp.mpf(float(np.float32(c))) for c in q]
    worst = mp.mpf(0)
    pts = [1 + mp.mpf(k) / 50 for k in range(951)] + [mp.mpf(20) * mp.mpf(500) ** (mp.mpf(k) / 100) for k in range(101)]
    for a in pts:
        u = 1 / a
        P = mp.fsum(c * u ** k for k, c in enumerate(p32))
        Q = mp.fsum(c * u ** k for k, c in enumerate(q32))
        worst = max(worst, abs(P / Q - g_exact(a)))
    assert worst < tol, worst
    assert all(c > 0 for c in p) and all(c > 0 for c in q)
    return worst


def psi_exact(a):
    return 1 + (a - 1) * mp.exp(-a) - a * a * mp.e1(a)


def h_exact(a):
    return mp.exp(-a) - a * mp.e1(a)


def pw_interval(q, lo_oct, per_oct):
    """[lo, hi) of interval q of the piecewise table: octave 2^e, e = lo_oct + q // per_oct,
    split into per_oct equal parts."""
    e, m = lo_oct + q // per_oct, q % per_oct
    base = mp.mpf(2) ** e
    return base * (1 + mp.mpf(m) / per_oct), base * (1 + mp.mpf(m + 1) / per_oct)


def cheb_to_monomial(c):
    """Monomial coefficients (ascending) of sum_k c_k T_k(s)."""
    n = len(c)
    out = [mp.mpf(0)] * n
    tkm1, tk = [mp.mpf(1)], [mp.mpf(0), mp.mpf(1)]
    for k, ck in enumerate(c):
        t = tkm1 if k == 0 else tk
        if k >= 2:
            nxt = [mp.mpf(0)] + [2 * v for v in tk]
            for i, v in enumerate(tkm1):
                nxt[i] -= v
            tkm1, tk = tk, nxt
            t = tk
        for i, v in enumerate(t):
            out[i] += ck * v
    return out


def pw_poly(f, lo, hi, deg, nodes=32):
    """Monomial coefficients in s = (2a - lo - hi) / (hi - lo) of the degree-deg
    truncation of f's Chebyshev interpolant on [lo, hi] (nodes points)."""
    mid, half = (lo + hi) / 2, (hi - lo) / 2
    th = [mp.pi * (j + mp.mpf(1) / 2) / nodes for j in range(nodes)]
    vals = [f(mid + half * mp.cos(t)) for t in th]
    c = [2 * mp.fsum(v * mp.cos(k * t) for v, t in zip(vals, th)) / nodes for k in range(deg + 1)]
    c[0] /= 2
    return cheb_to_monomial(c)


def build_pw(lo_oct, hi_oct, per_oct, deg):
    """psi and h on [2^lo_oct, 2^hi_oct): per interval the two monomial
    coefficient lists, and the worst errors of the double-rounded coefficients
    evaluated exactly (psi relative to psi, h absolute) on 33 points per interval."""
    rows, wpsi, wh = [], mp.mpf(0), mp.mpf(0)
    for q in range((hi_oct - lo_oct) * per_oct):
        lo, hi = pw_interval(q, lo_oct, per_oct)
        cp = [mp.mpf(float(v)) for v in pw_poly(psi_exact, lo, hi, deg)]
        ch = [mp.mpf(float(v)) for v in pw_poly(h_exact, lo, hi, deg)]
        rows.append((cp, ch))
        for k in range(33):
            s = -1 + mp.mpf(2 * k) / 32
            a = (lo + hi) / 2 + (hi - lo) / 2 * s
            P = mp.fsum(v * s ** i for i, v in enumerate(cp))
            H = mp.fsum(v * s ** i for i, v in enumerate(ch))
            wpsi = max(wpsi, abs(P / psi_exact(a) - 1))
            wh = max(wh, abs(H - h_exact(a)))
    return rows, wpsi, wh


def fmt(x, single):
    if single:
        return mp.nstr(x, 12, min_fixed=-1, max_fixed=-1) + "f"
    return mp.nstr(x, 20, min_fixed=-1, max_fixed=-1)


def main():
    cfg = {
        # precision: (number of octaves, Chebyshev tolerance, series terms)
        "double": (6, mp.mpf("2e-18"), 21),
        "float": (0, mp.mpf("1e-9"), 12),
    }
    lines = [
        "// Generated by gen_e1_table.py -- do not edit.",
        "// On (0, 1]: psi(a) = A(a) + a^2 ln a and psi'(a)/2 = B(a) + a ln a with",
        "// A, B entire power series (from A&S 5.1.11); coefficients alpha_n, beta_n.",
        "// G(a) = a e^a E1(a) on octaves [2^s, 2^(s+1)): Chebyshev coefficients in",
        "// t = (2a - 3*2^s) / 2^s, evaluated by Clenshaw's recurrence.",
        "#pragma once",
        "",
        "// Device code is compiled per translation unit, so every unit of the library",
        "// that evaluates the wall function defines its own copy of the tables;",
        "// LBSEP_TBL gives each unit's copy its own (external) name.",
        "#ifndef LBSEP_TBL",
        "#define LBSEP_TBL(name) name",
        "#endif",
        "",
        "#define LBSEP_EULER_GAMMA " + mp.nstr(mp.euler, 22),
    ]
    for name, (nseg, tol, nser) in cfg.items():
        single = name == "float"
        segs, deg = build(nseg, tol) if not single else ([], 0)
        worst = check(segs, nseg) if not single else mp.mpf(0)
        small = check_small(nser, mp.mpf("1e-18") if not single else mp.mpf("1e-9"))
        al, be = alpha_coeffs(nser), beta_coeffs(nser)
        tag = "F32" if single else "F64"
        lines.append("")
        if single:
            lines.append(f"// {name}: {nser}-term A, B series, max error {mp.nstr(small, 3)}")
        else:
            lines.append(f"// {name}: {nseg} octaves, degree {deg}, max |G error| = {mp.nstr(worst, 3)}; "
                         f"{nser}-term A, B series, max error {mp.nstr(small, 3)}")
        if not single:
            lines.append(f"#define LBSEP_E1_{tag}_NSEG {nseg}")
            lines.append(f"#define LBSEP_E1_{tag}_DEG {deg}")
        lines.append(f"#define LBSEP_E1_{tag}_NSER {nser}")
        lines.append(f"__constant__ {name} LBSEP_TBL(lbsep_psi_a_{tag.lower()})[{nser}] = {{")
        lines.append("    " + ", ".join(fmt(c, single) for c in al) + "};")
        lines.append(f"__constant__ {name} LBSEP_TBL(lbsep_psi_b_{tag.lower()})[{nser}] = {{")
        lines.append("    " + ", ".join(fmt(c, single) for c in be) + "};")
        if not single:  # FP32 uses the rational below for a > 1
            lines.append(f"__constant__ {name} LBSEP_TBL(lbsep_e1_cheb_{tag.lower()})[{nseg}][{deg + 1}] = {{")
            for seg in segs:
                lines.append("    {" + ", ".join(fmt(c, single) for c in seg) + "},")
            lines.append("};")
        print(name, "deg", deg, "worst", mp.nstr(worst, 3), "small-argument series", mp.nstr(small, 3))
    # FP64 piecewise polynomials of psi and h on [2^-20, 64)
    lo_oct, hi_oct, per_oct, deg = -20, 6, 8, 10
    rows, wpsi, wh = build_pw(lo_oct, hi_oct, per_oct, deg)
    assert wpsi < mp.mpf(2) ** -53 and wh < mp.mpf(2) ** -54, (wpsi, wh)
    lines.append("")
    lines.append(f"// double, 2^{lo_oct} <= a < 2^{hi_oct}: each octave [2^e, 2^(e+1)) in {per_oct} equal parts;")
    lines.append(f"// on part q = (e - ({lo_oct})) * {per_oct} + m the coefficients c_0..c_{deg} of psi and of h in")
    lines.append(f"// s = 2^(4-e) a - (17 + 2m) in [-1, 1) (monomials, ascending). Max relative psi error")
    lines.append(f"// {mp.nstr(wpsi, 3)}, max absolute h error {mp.nstr(wh, 3)} (coefficients as rounded, exact sums).")
    lines.append(f"#define LBSEP_PW_F64_LO_OCT ({lo_oct})")
    lines.append(f"#define LBSEP_PW_F64_HI_OCT {hi_oct}")
    lines.append(f"#define LBSEP_PW_F64_PER_OCT {per_oct}")
    lines.append(f"#define LBSEP_PW_F64_DEG {deg}")
    lines.append(f"#define LBSEP_PW_F64_N {len(rows)}")
    lines.append(f"__constant__ double LBSEP_TBL(lbsep_wall_pw_f64)[{len(rows)}][2][{deg + 1}] = {{")
    for cp, ch in rows:
        lines.append("    {{" + ", ".join(fmt(c, False) for c in cp) + "},")
        lines.append("     {" + ", ".join(fmt(c, False) for c in ch) + "}},")
    lines.append("};")
    print("double piecewise: psi rel", mp.nstr(wpsi, 3), "h abs", mp.nstr(wh, 3))
    p, q = rational_fit()
    worst = check_rational(p, q, mp.mpf("2e-8"))
    lines.append("")
    lines.append(f"// float, a > 1: G(a) ~ P(1/a) / Q(1/a), degrees (5, 5), max |G error| = {mp.nstr(worst, 3)}")
    lines.append("#define LBSEP_E1_F32_RAT_DEG 5")
    lines.append("constexpr float lbsep_e1_rat_p_f32[6] = {" + ", ".join(fmt(mp.mpf(float(c)), True) for c in p) + "};")
    lines.append("constexpr float lbsep_e1_rat_q_f32[6] = {" + ", ".join(fmt(mp.mpf(float(c)), True) for c in q) + "};")
    print("float rational worst", mp.nstr(worst, 3))
    with open(os.path.join(HERE, "e1_table.h"), "w") as fh:
        fh.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    main()
