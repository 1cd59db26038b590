"""Write domain_points.json: the oracle's log K_v(x), d/dv and d/dx at the
corners of the domain the GPU path is validated on (and a little beyond), and
large_order_points.json: the same and the second derivatives at orders
v = 1e4, 1e5, 1e6, beyond that domain.

    python tests/golden/make_domain_points.py

Calls only the oracle (oracle/, long-double adaptive quadrature of Eq. (1)-(2)
and Eq. (13)).  x = 1e10 is left out: the oracle's adaptive rule cannot meet
its tolerance there in reasonable time."""

import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import oracle  # noqa: E402

V = [0.0, 1e-10, 0.5, 10.0, 100.0, 1000.0]
X = [1e-35, 1e-30, 1e-20, 1e-12, 1e-6, 1e-3, 1.0, 1e3, 1e4, 1e5, 3e5, 1e6]
V_LARGE = [1e4, 1e5, 1e6]
X_LARGE = [1e-30, 1e-3, 1.0, 1e3, 1e4, 1e5, 1e6]


def write(name, vs, xs, second=False):
    vv, xx = (a.ravel() for a in np.meshgrid(vs, xs, indexing="ij"))
    lk, dv, dx = oracle.logk(vv, xx, deriv=True)
    points = [{"v": float(a), "x": float(b), "logk": float(c), "dv": float(d), "dx": float(e)}
              for a, b, c, d, e in zip(vv, xx, lk, dv, dx)]
    if second:
        h = oracle.logk_hess(vv, xx)
        for p, row in zip(points, h):
            p["d2v"], p["d2x"], p["dvx"] = (float(q) for q in row[3:])
    out = {"source": "oracle/oracle.c oracle_logk_batch (this script)", "points": points}
    with open(os.path.join(HERE, name), "w") as f:
        json.dump(out, f, indent=1)
    print(name, len(points), "points")


def main():
    write("domain_points.json", V, X)
    write("large_order_points.json", V_LARGE, X_LARGE, second=True)


if __name__ == "__main__":
    main()
