"""Fits the FP64 Box-Muller polynomials of mg_kernels.hip (sincos_small and
log_unit) by the Remez exchange algorithm, in 60-digit arithmetic (mpmath),
and prints their coefficients, highest degree first, as the kernels hold
them.  A development tool: nothing imports it.

* sine on |r| <= pi/4: sin r = r + r^3 P(x), x = r^2, P of degree 5, minimax
  for the relative error of sin (weight x r / sin r on P's error);
* cosine: cos r = 1 - x/2 + x^2 C(x), C of degree 5, weight x^2 / cos r;
* logarithm: R(z) = 2 atanh(s)/s - 2 = z Q(z), z = s^2 <= ((sqrt 2 - 1) /
  (sqrt 2 + 1))^2, Q of degree 6, weight z/2 (R's share of log(1 + f)
  relative to log(1 + f) ~ 2 s).

The exchange runs on a dense Chebyshev grid: solve for the coefficients and
the levelled error E on n + 2 reference points, move the references to the
alternating extrema of the weighted error, repeat until the largest error
matches |E|.

    python minimax_fit.py
"""
import mpmath as mp

mp.mp.dps = 60


def remez(f, w, a, b, n, iters=40, grid=8000):
    xs = [a + (b - a) * (1 - mp.cos(mp.pi * i / (grid - 1))) / 2 for i in range(grid)]
    fx = [f(x) for x in xs]
    wx = [w(x) for x in xs]
    m = n + 2
    ref = [a + (b - a) * (1 - mp.cos(mp.pi * i / (m - 1))) / 2 for i in range(m)]
    coef, worst = None, None
    for _ in range(iters):
        A = mp.matrix(m, m)
        rhs = mp.matrix(m, 1)
        for i, x in enumerate(ref):
            for k in range(n + 1):
                A[i, k] = x ** k
            A[i, n + 1] = (-1) ** i / w(x)
            rhs[i] = f(x)
        sol = mp.lu_solve(A, rhs)
        coef, lev = [sol[k] for k in range(n + 1)], sol[n + 1]
        err = [wx[i] * (fx[i] - mp.polyval(coef[::-1], xs[i])) for i in range(grid)]
        worst = max(abs(e) for e in err)
        if abs(worst - abs(lev)) <= worst * mp.mpf("1e-8"):
            break
        ext = [i for i in range(grid)
               if i in (0, grid - 1) or (err[i] - err[i - 1]) * (err[i + 1] - err[i]) <= 0]
        alt = []
        for i in ext:
            if alt and mp.sign(err[i]) == mp.sign(err[alt[-1]]):
                if abs(err[i]) > abs(err[alt[-1]]):
                    alt[-1] = i
            else:
                alt.append(i)
        while len(alt) > m:
            alt.pop(0 if abs(err[alt[0]]) < abs(err[alt[-1]]) else -1)
        if len(alt) < m:
            break
        ref = [xs[i] for i in alt]
    return coef, worst


def main():
    tiny = mp.mpf("1e-40")
    X = (mp.pi / 4) ** 2
    Z = ((mp.sqrt(2) - 1) / (mp.sqrt(2) + 1)) ** 2
    fits = {
        "sine P": (lambda x: (mp.sin(mp.sqrt(x)) - mp.sqrt(x)) / (mp.sqrt(x) * x)
                   if x > 0 else mp.mpf(-1) / 6,
                   lambda x: x * mp.sqrt(x) / mp.sin(mp.sqrt(x)) if x > 0 else tiny, X, 5),
        "cosine C": (lambda x: (mp.cos(mp.sqrt(x)) - 1 + x / 2) / x ** 2
                     if x > 0 else mp.mpf(1) / 24,
                     lambda x: x ** 2 / mp.cos(mp.sqrt(x)) if x > 0 else tiny, X, 5),
        "logarithm Q": (lambda z: (2 * mp.atanh(mp.sqrt(z)) / mp.sqrt(z) - 2) / z
                        if z > 0 else mp.mpf(2) / 3,
                        lambda z: z / 2 if z > 0 else tiny, Z, 6),
    }
    for name, (f, w, b, n) in fits.items():
        coef, worst = remez(f, w, mp.mpf(0), b, n)
        print(f"{name}: weighted error {mp.nstr(worst, 4)} (2^{mp.nstr(mp.log(worst, 2), 4)})")
        for c in coef[::-1]:
            print(f"  {float(c)!r}")


if __name__ == "__main__":
    main()
