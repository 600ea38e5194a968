"""Generate smoothing_coeffs.h: Taylor coefficients and far-field cutoffs
of the regularised kernel factors used by the HIP pair kernels.

The kernels need the even entire functions
    F1 = s1/rho, F2 = s2/rho^3, F3 = s3/rho^3, F4 = s4/rho^5
of the four smoothing functions of the paper (section "High-order
regularization of kernels on the surface"), and for position derivatives
    G_k = -F_k'(rho)/rho.
For small rho the closed forms cancel catastrophically, so the kernels sum a
truncated Taylor series in x = rho^2.  This script derives the series
exactly: it multiplies the power series of exp(-rho^2) by each printed
polynomial, subtracts the product from the power series of erf, and divides by
rho^p, all in rational arithmetic (the factor 2/sqrt(pi) is applied last, in
80-digit arithmetic).  The series are truncated where the next term falls
below the target precision at the branch point.

It also finds the far-field cutoff rho_cut beyond which every s_k used by
a kernel equals 1 to within half an ulp of the working precision, so that
the smoothing can be skipped there.

Run:  python gen_smoothing.py > smoothing_coeffs.h
"""
from fractions import Fraction as Fr
from math import factorial

import mpmath as mp

mp.mp.dps = 80
NTERMS = 40

# printed polynomials: s_k = erf(rho) - c * rho * P_k(rho^2) * e^{-rho^2},
# with c = 2/sqrt(pi); P_k as coefficients in x = rho^2 (low to high)
P = {
    1: [Fr(-5, 3), Fr(2, 3)],                               # -(1/3)(2x - 5) with sign folded below
    2: [Fr(-3, 3), Fr(2, 3)],
    3: [Fr(3, 3), Fr(-14, 3), Fr(4, 3)],
    4: [Fr(9, 9), Fr(6, 9), Fr(-36, 9), Fr(8, 9)],
}
# sign with which c*rho*P_k*E enters s_k (s2 has a plus sign)
SIGN = {1: -1, 2: +1, 3: -1, 4: -1}
POW = {1: 1, 2: 3, 3: 3, 4: 5}


def s_series(k):
    """Coefficients b_n of s_k / c = sum_n b_n rho^{2n+1} (exact)."""
    erf_c = [Fr((-1) ** n, factorial(n) * (2 * n + 1)) for n in range(NTERMS + 4)]
    exp_c = [Fr((-1) ** n, factorial(n)) for n in range(NTERMS + 4)]
    prod = [Fr(0)] * (NTERMS + 4)
    for i, p in enumerate(P[k]):
        for j, e in enumerate(exp_c):
            if i + j < len(prod):
                prod[i + j] += p * e
    return [erf_c[n] + SIGN[k] * prod[n] for n in range(NTERMS + 4)]


def F_series(k):
    """a_m with F_k / c = sum_m a_m x^m, x = rho^2."""
    b = s_series(k)
    shift = (POW[k] - 1) // 2  # rho^{2n+1} / rho^p = x^{n - shift}
    for n in range(shift):
        assert b[n] == 0, (k, n, b[n])
    return b[shift:shift + NTERMS]


def G_series(k):
    """a'_q with G_k / c = -F_k'/(rho c) = sum_q a'_q x^q."""
    a = F_series(k)
    return [-2 * (q + 1) * a[q + 1] for q in range(NTERMS - 1)]


def c_mp():
    return 2 / mp.sqrt(mp.pi)


def truncate(coef, rho_s, eps):
    x = Fr(rho_s) ** 2
    out = []
    for m, a in enumerate(coef):
        out.append(a)
        if m > 2 and abs(float(a) * float(x) ** (m + 1)) < eps * 1e-2:
            # next term negligible (terms alternate and decrease quickly)
            if abs(float(coef[m + 1]) * float(x) ** (m + 1)) < eps * abs(float(coef[0])):
                break
    return out


def s_mp(k, r):
    c = c_mp()
    r = mp.mpf(r)
    x = r * r
    poly = sum(mp.mpf(p.numerator) / p.denominator * x**i for i, p in enumerate(P[k]))
    return mp.erf(r) + SIGN[k] * c * r * poly * mp.e ** (-x)


def cutoff(ks, eps):
    """Smallest rho on a 0.01 grid beyond which |1 - s_k| < eps for all k in ks."""
    r = mp.mpf(12)
    while r > 0:
        if max(abs(1 - s_mp(k, r)) for k in ks) >= eps:
            return float(r + mp.mpf("0.01"))
        r -= mp.mpf("0.01")
    return 0.0


def erfcx_fit(lo, hi, p, deg, ctype):
    """Coefficients (low to high) of a polynomial g(t), t = 1/(1 + p rho), with
    g ~ erfc(rho) exp(rho^2) on [lo, hi]: interpolation at the Chebyshev
    points of the t interval in 60-digit arithmetic.  Returns (coefficients,
    max relative error of Horner's rule in the target precision on a grid)."""
    import numpy as np
    with mp.workdps(60):
        tlo, thi = 1 / (1 + p * mp.mpf(hi)), 1 / (1 + p * mp.mpf(lo))
        tm, th = (tlo + thi) / 2, (thi - tlo) / 2
        nodes = [tm + th * mp.cos(mp.pi * (k + mp.mpf(1) / 2) / (deg + 1)) for k in range(deg + 1)]
        vals = [mp.erfc((1 / t - 1) / p) * mp.exp(((1 / t - 1) / p) ** 2) for t in nodes]
        A = mp.matrix([[t ** j for j in range(deg + 1)] for t in nodes])
        c = mp.lu_solve(A, mp.matrix(vals))
        coef = [c[j] for j in range(deg + 1)]
        dt = np.float64 if ctype == "double" else np.float32
        cc = [dt(float(v)) for v in coef]
        worst = 0.0
        for r in np.linspace(lo, hi, 3001):
            r = dt(r)
            t = dt(1) / (dt(1) + dt(p) * r)
            a = cc[-1]
            for v in reversed(cc[:-1]):
                a = a * t + v
            ex = mp.erfc(mp.mpf(float(r))) * mp.exp(mp.mpf(float(r)) ** 2)
            worst = max(worst, abs(float((mp.mpf(float(a)) - ex) / ex)))
    return coef, worst


def emit_plain(name, vals, ctype, suffix):
    body = ",\n    ".join(mp.nstr(v, 25, min_fixed=-1, max_fixed=-1) + suffix for v in vals)
    return f"static constexpr int {name}_N = {len(vals)};\n" \
           f"__device__ static constexpr {ctype} {name}[{len(vals)}] = {{\n    {body}}};\n"


def emit(name, coef, ctype, suffix):
    c = c_mp()
    vals = [mp.mpf(a.numerator) / a.denominator * c for a in coef]
    body = ",\n    ".join(mp.nstr(v, 25, min_fixed=-1, max_fixed=-1) + suffix for v in vals)
    return f"static constexpr int {name}_N = {len(vals)};\n" \
           f"__device__ static constexpr {ctype} {name}[{len(vals)}] = {{\n    {body}}};\n"


def main():
    # series below rho_s; above it erf = 1 - exp(-rho^2) g(1/(1 + p rho)).
    # Float starts the fit at rho = 1, where every s_k >= 0.3, so the rounding
    # of t (amplified by 1/(1 - t) in g) stays near one ulp of s_k.
    rho_s64, rho_s32 = 0.5, 1.0
    eps64, eps32 = 2.0**-54, 2.0**-25
    out = ["// Generated by gen_smoothing.py; do not edit.",
           "// Taylor coefficients (in x = rho^2) of F1..F4 = s_k/rho^p and of",
           "// G2, G4 = -F'/rho, including the factor 2/sqrt(pi), and the far-field cutoffs.",
           "#pragma once", ""]
    out.append(f"#define SDBIE_RHO_SERIES_F64 {rho_s64}")
    out.append(f"#define SDBIE_RHO_SERIES_F32 {rho_s32}f")
    lap = cutoff([1, 2], 2.0**-53)
    sto = cutoff([1, 3, 4], 2.0**-53)
    lap32 = cutoff([1, 2], 2.0**-24)
    sto32 = cutoff([1, 3, 4], 2.0**-24)
    p_fit = 0.33
    g64, e64 = erfcx_fit(rho_s64 - 0.01, sto + 0.1, p_fit, 16, "double")
    g32, e32 = erfcx_fit(rho_s32 - 0.01, sto32 + 0.1, p_fit, 8, "float")
    assert e64 < 1.5e-15 and e32 < 4e-7, (e64, e32)
    # the adjoint's derivative factors also need s2 and s4 -> 1
    out.append(f"#define SDBIE_RHO_CUT_LAPLACE_F64 {lap}")
    out.append(f"#define SDBIE_RHO_CUT_STOKES_F64 {sto}")
    out.append(f"#define SDBIE_RHO_CUT_LAPLACE_F32 {lap32}f")
    out.append(f"#define SDBIE_RHO_CUT_STOKES_F32 {sto32}f")
    out.append("")
    for k in (1, 2, 3, 4):
        a = F_series(k)
        out.append(emit(f"kF{k}_F64", truncate(a, rho_s64, eps64), "double", ""))
        out.append(emit(f"kF{k}_F32", truncate(a, rho_s32, eps32), "float", "f"))
    out.append(f"// erfc(rho) exp(rho^2) ~ sum_j kERFCX_*[j] t^j, t = 1/(1 + SDBIE_ERFCX_P rho), on")
    out.append(f"// [{rho_s64 - 0.01}, {sto + 0.1}] (double, max rel. error {e64:.1e}) and "
               f"[{rho_s32 - 0.01}, {sto32 + 0.1}] (float, {e32:.1e})")
    out.append(f"#define SDBIE_ERFCX_P {p_fit}")
    out.append(emit_plain("kERFCX_F64", g64, "double", ""))
    out.append(emit_plain("kERFCX_F32", g32, "float", "f"))
    for k in (2, 4):
        g = G_series(k)
        out.append(emit(f"kG{k}_F64", truncate(g, rho_s64, eps64), "double", ""))
        out.append(emit(f"kG{k}_F32", truncate(g, rho_s32, eps32), "float", "f"))
    print("\n".join(out))


if __name__ == "__main__":
    main()
