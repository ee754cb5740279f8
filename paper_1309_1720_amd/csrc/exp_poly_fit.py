"""Coefficients of the exponential's core polynomial in rd_device.h (exp_lean).

After the reduction x = n ln2 + r, |r| <= ln2/2, e^r is approximated as

    p(r) = 1 + r + r^2/2 + r^3 h(r),   h of degree 8,

with the low-order coefficients 1, 1, 1/2 held exact (so that they stay inline
operands of the multiply-adds) and h chosen to minimise the largest relative
error |p(r) - e^r| / e^r on the interval.  The fit is the Remez exchange
algorithm in 60-digit arithmetic: solve for the polynomial whose relative error
alternates in sign with equal size E on a reference of deg(h) + 2 points, move
the reference to the extrema of the new error curve, and repeat until the
extrema equal E.  Prints the coefficients as the kernel source writes them.

    python exp_poly_fit.py
"""
import mpmath as mp

mp.mp.dps = 60
A = mp.log(2) / 2
DEG = 8  # degree of h


def p_of(c, x):
    h = mp.mpf(0)
    for ck in reversed(c):
        h = h * x + ck
    return 1 + x + x * x / 2 + x ** 3 * h


def rel_err(c, x):
    return (p_of(c, x) - mp.exp(x)) / mp.exp(x)


def solve_reference(ref):
    """h's coefficients and E with p(x_i) - e^x_i = (-1)^i E e^x_i."""
    n = DEG + 2
    a, b = mp.matrix(n, n), mp.matrix(n, 1)
    for i, x in enumerate(ref):
        for k in range(DEG + 1):
            a[i, k] = x ** (3 + k)
        a[i, DEG + 1] = -((-1) ** i) * mp.exp(x)
        b[i] = mp.exp(x) - 1 - x - x * x / 2
    sol = mp.lu_solve(a, b)
    return [sol[k] for k in range(DEG + 1)], sol[DEG + 1]


def extrema(c, grid=4000):
    """One extremum of the relative error per run of equal sign."""
    xs = [-A + 2 * A * i / grid for i in range(grid + 1)]
    es = [rel_err(c, x) for x in xs]
    runs, start = [], 0
    for i in range(1, len(xs)):
        if es[i] != 0 and mp.sign(es[i]) != mp.sign(es[start]):
            runs.append((start, i - 1))
            start = i
    runs.append((start, len(xs) - 1))
    out = []
    g = (mp.sqrt(5) - 1) / 2
    for s0, s1 in runs:
        j = max(range(s0, s1 + 1), key=lambda i: abs(es[i]))
        if j in (0, len(xs) - 1):
            out.append(xs[j])  # an end point of the interval
            continue
        lo, hi = xs[j - 1], xs[j + 1]
        for _ in range(80):  # golden-section search for the largest |error|
            m1, m2 = hi - g * (hi - lo), lo + g * (hi - lo)
            if abs(rel_err(c, m1)) > abs(rel_err(c, m2)):
                hi = m2
            else:
                lo = m1
        out.append((lo + hi) / 2)
    return out


def fit():
    ref = [A * mp.cos(mp.pi * (DEG + 1 - i) / (DEG + 1)) for i in range(DEG + 2)]
    for _ in range(30):
        c, e = solve_reference(ref)
        ref = extrema(c)
        if len(ref) != DEG + 2:
            raise RuntimeError("the error curve lost its alternation")
        worst = max(abs(rel_err(c, x)) for x in ref)
        if abs(worst - abs(e)) <= 1e-6 * abs(e):
            return c, worst
    raise RuntimeError("Remez iteration did not settle")


if __name__ == "__main__":
    coeffs, worst = fit()
    print(f"// largest relative error of the exact polynomial: {mp.nstr(worst, 3)}")
    for k in reversed(range(DEG + 1)):
        print(f"r^{k + 3}: {float(coeffs[k])!r}")
