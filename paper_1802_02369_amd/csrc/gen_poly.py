"""Derives the polynomial coefficients of the device exp and log (lbm_device.hpp).

Both are Chebyshev interpolation fits computed here in 60-digit arithmetic
(mpmath.chebyfit), rounded to double, then checked on a dense grid:

  exp:  R(r) ~ (e^r - 1 - r) / r^2 on |r| <= 0.3466 (= ln 2 / 2 + margin), so
        e^r = 1 + r (1 + r R(r)), R of degree 9 (e^r to degree 11).
  log:  Q(w) ~ (2 atanh(z) - 2 z) / z^3 with w = z^2 on [0, 0.02944]
        (|z| <= (sqrt 2 - 1)/(sqrt 2 + 1)), so ln m = 2 z + z w Q(w).

Prints the C++ initialisers and the worst relative error of each
approximation with the double coefficients (evaluated exactly), which must
stay far below one ulp (1.1e-16).  Run: python3 gen_poly.py
"""
import mpmath as mp

mp.mp.dps = 60


def fit(f, a, b, deg):
    coef, _ = mp.chebyfit(f, [a, b], deg + 1, error=True)
    return [float(c) for c in coef]  # highest degree first


def horner(c, x):
    acc = mp.mpf(c[0])
    for k in c[1:]:
        acc = acc * x + mp.mpf(k)
    return acc


def worst(full, approx, a, b, n=20001):
    w = mp.mpf(0)
    for i in range(n):
        x = a + (b - a) * mp.mpf(i) / (n - 1)
        ref = full(x)
        w = max(w, abs(approx(x) - ref) / abs(ref))
    return w


def main():
    A = mp.mpf("0.3466")

    def R(r):
        return (mp.exp(r) - 1 - r) / r**2 if r != 0 else mp.mpf(1) / 2

    ce = fit(R, -A, A, 9)
    err_e = worst(mp.exp, lambda r: 1 + r * (1 + r * horner(ce, r)), -A, A)

    zmax = (mp.sqrt(2) - 1) / (mp.sqrt(2) + 1)
    W = zmax**2 * (1 + mp.mpf("1e-6"))

    def Q(w):
        if w == 0:
            return mp.mpf(2) / 3
        z = mp.sqrt(w)
        return (2 * mp.atanh(z) - 2 * z) / z**3

    cl = fit(Q, mp.mpf(0), W, 6)

    def ln_approx(z):
        w = z * z
        return 2 * z + z * w * horner(cl, w)

    err_l = worst(lambda z: 2 * mp.atanh(z), ln_approx, mp.mpf("1e-8"), zmax)

    print("// exp: R(r), degree 9, highest first; worst rel. error %.2e" % err_e)
    for c in ce:
        print("  %s," % float(c).hex())
    print("// log: Q(w), degree 6, highest first; worst rel. error %.2e" % err_l)
    for c in cl:
        print("  %s," % float(c).hex())


if __name__ == "__main__":
    main()
