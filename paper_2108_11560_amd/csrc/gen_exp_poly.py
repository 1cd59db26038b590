"""Generate the polynomial coefficients of the device FP64 exponentials.

e^r on |r| <= ln(2)/(2 d) is approximated by a polynomial of the given degree
whose relative error is minimax (Remez exchange on the weight 1/e^r, in
50-digit mpmath), then rounded to double.  Prints the coefficients and the
error of the rounded polynomial; the values are pasted into bessel_device.hpp:
degree 10 with d = 1 for exp_f64 (3.0e-16), degree 3 with d = 256 for the
per-node exponential of the FP64 bins, whose reduction leaves |r| <= ln2/512
(1.8e-14, far below the 1e-12 the FP64 path is held to).

    python paper_2108_11560_amd/csrc/gen_exp_poly.py [degree [d]]
"""

import sys

import mpmath as mp

mp.mp.dps = 50


def remez(deg, a, iters=30):
    n = deg + 2
    # initial reference: Chebyshev extrema
    xs = [a * mp.cos(mp.pi * (n - 1 - i) / (n - 1)) for i in range(n)]
    coeffs = None
    for _ in range(iters):
        # solve sum c_j x^j + (-1)^i E e^x = e^x  (relative error alternation)
        M = mp.matrix(n, n)
        b = mp.matrix(n, 1)
        for i, xv in enumerate(xs):
            for j in range(deg + 1):
                M[i, j] = xv ** j
            M[i, deg + 1] = (-1) ** i * mp.e ** xv
            b[i] = mp.e ** xv
        sol = mp.lu_solve(M, b)
        coeffs = [sol[j] for j in range(deg + 1)]

        def err(xv):
            return (sum(c * xv ** j for j, c in enumerate(coeffs)) - mp.e ** xv) / mp.e ** xv

        # new reference: extrema of the error on a fine grid, one per sign run
        grid = [-a + 2 * a * k / 4000 for k in range(4001)]
        vals = [err(g) for g in grid]
        ext = []
        k = 0
        while k < len(grid):
            s = mp.sign(vals[k])
            best = k
            while k < len(grid) and mp.sign(vals[k]) == s:
                if abs(vals[k]) > abs(vals[best]):
                    best = k
                k += 1
            ext.append(grid[best])
        if len(ext) >= n:
            # keep the n largest-alternation points (trim from the ends)
            while len(ext) > n:
                if abs(err(ext[0])) < abs(err(ext[-1])):
                    ext.pop(0)
                else:
                    ext.pop()
            xs = ext
    return coeffs


def coefficients(deg: int, div: int = 1):
    """The rounded minimax coefficients c0..c_deg on |r| <= ln(2)/(2 div) and
    the maximum relative error of the rounded polynomial there."""
    a = mp.log(2) / (2 * div)
    cd = [float(v) for v in remez(deg, a)]
    worst = 0.0
    for k in range(20001):
        r = -a + 2 * a * k / 20000
        p = mp.mpf(0)
        for v in reversed(cd):
            p = p * r + mp.mpf(v)
        worst = max(worst, abs(float((p - mp.e ** r) / mp.e ** r)))
    return cd, worst


def main():
    deg = int(sys.argv[1]) if len(sys.argv) > 1 else 10
    div = int(sys.argv[2]) if len(sys.argv) > 2 else 1
    cd, worst = coefficients(deg, div)
    for j, v in enumerate(cd):
        print(f"c{j} = {v!r}")
    print(f"max relative error of the rounded polynomial on |r| <= ln2/{2 * div}: {worst:.3e}")


if __name__ == "__main__":
    main()
