"""Write gpoly.inc: FP32 coefficients for the short-range force shape.

Two polynomial forms are written.

(1) Q(v): exp(-u^2) Q(u) = g(u), used where exp(-u^2) is needed anyway (the
adjoint's Gaussian term).

(2) H(v): the forward force needs only g(u)/r^3.  g(u) - 1 holds only odd
powers of u from u^3 on (the u terms of erfc and of the Gaussian term
cancel), so g(u) = 1 + u^3 H(t) with t = u^2 and H entire, and
    g(u) / r^3 = r^-3 + H(t) / (2 x_s)^3 .
H is fitted in t on [0, 2.25^2] as a degree-9 polynomial in v = t - 3
(near-minimax in the absolute error of g), so the forward shape needs one
hardware rsqrt and one polynomial, with no exponential.

(3) H64(v): the same H for the FP64 path, degree 17 in v = t - 2.5, from
Chebyshev interpolation at 60 digits (mpmath) converted to the shifted
monomial basis at that precision and rounded to double; its derivative
(for the adjoint) comes from the same Horner pass.

The kernel shape of eq. p3m_gravity (section 2.1.3) is
    g(u) = erfc(u) + (2/sqrt(pi)) u exp(-u^2),   u = r / (2 x_s),
evaluated only for r < r_cut = 4.5 x_s, i.e. u in [0, 2.25).  Factor out the
Gaussian: g(u) = exp(-u^2) Q(u) with Q(u) = erfcx(u) + 2u/sqrt(pi), where
erfcx(u) = exp(u^2) erfc(u) is smooth and Q varies only from 1 to ~2.8.  The
GPU evaluates exp(-u^2) with the hardware base-2 exponential and Q with a
degree-9 polynomial in v = u - C0 (centering keeps FP32 Horner accurate).

The polynomial is a near-minimax fit of the relative error of g over
[0, 2.25] by Lawson's algorithm (iteratively reweighted least squares on a
Chebyshev basis), with Q evaluated in 40-digit mpmath.  Run:
    python gen_gpoly.py  > gpoly.inc
"""
import sys

import mpmath as mp
import numpy as np

U_MAX = 2.25
DEGREE = 9
C0 = 0.75


def fit(degree=DEGREE, c0=C0, n_grid=6001, iters=400):
    mp.mp.dps = 40
    us = np.linspace(0.0, U_MAX, n_grid)
    q = np.array([float(mp.erfc(u) * mp.exp(u * u) + 2 * u / mp.sqrt(mp.pi)) for u in us])
    w_rel = 1.0 / q                      # relative error of g per unit error of Q
    t = us / U_MAX * 2 - 1
    V = np.polynomial.chebyshev.chebvander(t, degree)
    wt = np.full(us.size, 1.0 / us.size)
    for _ in range(iters):
        W = np.sqrt(wt) * w_rel
        c, *_ = np.linalg.lstsq(V * W[:, None], q * W, rcond=None)
        err = np.abs(V @ c - q) * w_rel
        wt = wt * err
        wt /= wt.sum()
    mono_t = np.polynomial.Polynomial(np.polynomial.chebyshev.cheb2poly(c))
    in_u = mono_t(np.polynomial.Polynomial([-1.0, 2.0 / U_MAX]))
    in_v = in_u(np.polynomial.Polynomial([c0, 1.0]))
    coef = in_v.coef.astype(np.float32)
    # FP32 Horner error on the grid (relative error of g)
    v32 = (us - c0).astype(np.float32)
    acc = np.float32(coef[-1])
    for a in coef[-2::-1]:
        acc = np.float32(acc * v32 + a)
    fp32_err = float(np.max(np.abs(acc.astype(np.float64) - q) * w_rel))
    return coef, float(np.max(err)), fp32_err


H_DEGREE = 9
H_T0 = 3.0


def fit_h(degree=H_DEGREE, t0=H_T0, n_grid=8001, iters=400):
    """H(t) = (g(u) - 1) / u^3, t = u^2, near-minimax in |u^3 dH| (absolute error of g)."""
    mp.mp.dps = 40
    tmax = U_MAX * U_MAX
    ts = np.linspace(0.0, tmax, n_grid)

    def h_exact(t):
        if t == 0.0:
            return float(-4 / (3 * mp.sqrt(mp.pi)))
        u = mp.sqrt(mp.mpf(t))
        g = mp.erfc(u) + 2 * u / mp.sqrt(mp.pi) * mp.exp(-u * u)
        return float((g - 1) / u ** 3)

    h = np.array([h_exact(t) for t in ts])
    w = ts ** 1.5 + 1e-3
    x = ts / tmax * 2 - 1
    V = np.polynomial.chebyshev.chebvander(x, degree)
    wt = np.full(ts.size, 1.0 / ts.size)
    for _ in range(iters):
        W = np.sqrt(wt) * w
        c, *_ = np.linalg.lstsq(V * W[:, None], h * W, rcond=None)
        err = np.abs(V @ c - h) * w
        wt = wt * (err + 1e-300)
        wt /= wt.sum()
    in_t = np.polynomial.Polynomial(np.polynomial.chebyshev.cheb2poly(c))(
        np.polynomial.Polynomial([-1.0, 2.0 / tmax]))
    coef = in_t(np.polynomial.Polynomial([t0, 1.0])).coef.astype(np.float32)
    v32 = (ts - t0).astype(np.float32)
    acc = np.float32(coef[-1])
    for a in coef[-2::-1]:
        acc = np.float32(acc * v32 + a)
    g_err = float(np.max(np.abs(ts ** 1.5 * (acc.astype(np.float64) - h))))
    return coef, float(np.max(err)), g_err


H64_DEGREE = 17
H64_T0 = 2.5


def fit_h64(degree=H64_DEGREE, t0=H64_T0):
    """Chebyshev interpolant of H on [0, 2.25^2] in 60-digit arithmetic,
    returned as double coefficients of the polynomial in v = t - t0, with the
    largest absolute error of g = 1 + t^1.5 H over a check grid."""
    mp.mp.dps = 60
    tmax = mp.mpf(U_MAX) ** 2
    t0m = mp.mpf(t0)

    def h_exact(t):
        if t == 0:
            return -4 / (3 * mp.sqrt(mp.pi))
        u = mp.sqrt(t)
        return (mp.erfc(u) + 2 * u / mp.sqrt(mp.pi) * mp.exp(-u * u) - 1) / u ** 3

    n = degree + 1
    nodes = [tmax / 2 + tmax / 2 * mp.cos(mp.pi * (k + mp.mpf(1) / 2) / n) for k in range(n)]
    vals = [h_exact(x) for x in nodes]
    cheb = []
    for j in range(n):
        acc = sum(vals[k] * mp.cos(mp.pi * j * (k + mp.mpf(1) / 2) / n) for k in range(n))
        cheb.append(2 * acc / n)
    cheb[0] /= 2
    # Chebyshev basis in x = 2t/tmax - 1 -> monomials in x -> monomials in v
    tp = [[mp.mpf(1)], [mp.mpf(0), mp.mpf(1)]]
    for j in range(2, n):
        a = [mp.mpf(0)] + [2 * x for x in tp[-1]]
        b = tp[-2] + [mp.mpf(0)] * (len(a) - len(tp[-2]))
        tp.append([a[i] - b[i] for i in range(len(a))])
    px = [mp.mpf(0)] * n
    for j in range(n):
        for i, co in enumerate(tp[j]):
            px[i] += cheb[j] * co
    alpha, beta = 2 / tmax, 2 * t0m / tmax - 1
    res = [mp.mpf(0)] * n
    for i in range(n):
        for k in range(i + 1):
            res[k] += px[i] * mp.binomial(i, k) * alpha ** k * beta ** (i - k)
    coef = [float(x) for x in res]
    worst = mp.mpf(0)
    for m in range(0, 1001):
        t = tmax * m / 1000
        v = float(t - t0m)
        acc = coef[-1]
        for a_ in coef[-2::-1]:
            acc = acc * v + a_
        worst = max(worst, abs((mp.mpf(acc) - h_exact(t)) * t ** mp.mpf(1.5)))
    return coef, float(worst)


def main():
    coef, e_fit, e32 = fit()
    out = sys.stdout
    out.write("// Generated by gen_gpoly.py: Q(u) = erfcx(u) + 2u/sqrt(pi) on [0, 2.25],\n")
    out.write("// degree-%d polynomial in v = u - %.17g (near-minimax in the relative\n" % (DEGREE, C0))
    out.write("// error of g = exp(-u^2) Q).  Fit error %.2e, FP32 Horner error %.2e.\n"
              % (e_fit, e32))
    out.write("#define P3M_GPOLY_DEGREE %d\n" % DEGREE)
    out.write("#define P3M_GPOLY_C0 %sf\n" % float(np.float32(C0)).hex())
    out.write("static constexpr float kGpoly[P3M_GPOLY_DEGREE + 1] = {\n")
    for k, a in enumerate(coef):
        out.write("    %sf,%s\n" % (float(a).hex(), "  // v^%d" % k))
    out.write("};\n")
    hc, h_fit, h32 = fit_h()
    out.write("// H(t) = (g(u) - 1) / u^3, t = u^2 in [0, 2.25^2]: degree-%d polynomial in\n"
              "// v = t - %.17g, near-minimax in the absolute error of g.  Fit error %.2e,\n"
              "// FP32 Horner error %.2e (absolute, in units of g).\n" % (H_DEGREE, H_T0, h_fit, h32))
    out.write("#define P3M_HPOLY_DEGREE %d\n" % H_DEGREE)
    out.write("#define P3M_HPOLY_T0 %sf\n" % float(np.float32(H_T0)).hex())
    out.write("static constexpr float kHpoly[P3M_HPOLY_DEGREE + 1] = {\n")
    for k, a in enumerate(hc):
        out.write("    %sf,%s\n" % (float(a).hex(), "  // v^%d" % k))
    out.write("};\n")
    h64, e64 = fit_h64()
    out.write("// H(t) for the FP64 path: degree-%d polynomial in v = t - %.17g (Chebyshev\n"
              "// interpolant at 60 digits); FP64 Horner error %.2e (absolute, in units of g).\n"
              % (H64_DEGREE, H64_T0, e64))
    out.write("#define P3M_H64_DEGREE %d\n" % H64_DEGREE)
    out.write("#define P3M_H64_T0 %s\n" % float(H64_T0).hex())
    out.write("static constexpr double kH64[P3M_H64_DEGREE + 1] = {\n")
    for k, a in enumerate(h64):
        out.write("    %s,%s\n" % (float(a).hex(), "  // v^%d" % k))
    out.write("};\n")


if __name__ == "__main__":
    main()
