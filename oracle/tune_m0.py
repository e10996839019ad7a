"""Mass tuning for the synthetic workloads (workload preparation, oracle only).

The workloads ask for m0 such that the smallest singular value of D reaches a
target (1e-2 for 16^3x32, 3e-3 for 32^3x64, 1e-3 for 48^3x96), estimated by
100 inverse-iteration steps on D^dag D.  The oracle cannot afford that at the
full volumes, so the mass is tuned on a proxy lattice of the same link
roughness eps: the dense D(m0 = 0) is assembled once from the oracle's
operator (one column per unit vector); the mass only shifts its diagonal, so
every trial mass costs one LU factorisation of D(0) + m0 and 100 inverse
iterations y <- (D^dag D)^-1 y / |.|, sigma_min = |(D^dag D)^-1 y|^(-1/2).  The search starts on the heavy side (m0 = 0), steps
down by 0.05 while sigma_min decreases and stays above the target, then
narrows the bracket by golden-section search on the minimum (sigma_min is not
monotone past a zero crossing, so the search never goes beyond the first
minimum).  When the target is not reached, the mass at the minimum and the
sigma_min found there are recorded, and `reached` is false.

    python oracle/tune_m0.py C2 C3 C4        # writes workloads/m0_tuned.json
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from oracle.lattice import Lattice            # noqa: E402
from oracle.dirac import WilsonClover, clover_matrix  # noqa: E402
from workloads import su3_field               # noqa: E402
from workloads.configs import CONFIGS         # noqa: E402

PROXY_L = (4, 4, 4, 8)


def dense_operator(U, lat, m0, c_sw, A0):
    """D as a dense matrix, one oracle apply per unit vector."""
    A = A0 + (m0 * np.eye(12))[None]
    W = WilsonClover(U, lat, m0, c_sw, A=A)
    n = 12 * lat.V
    D = np.empty((n, n), dtype=np.complex128)
    e = np.zeros((lat.V, 4, 3), dtype=np.complex128)
    for k in range(n):
        e.reshape(-1)[k] = 1.0
        D[:, k] = W.apply(e).reshape(-1)
        e.reshape(-1)[k] = 0.0
    return D


def sigma_min(D0, m0, steps=100, seed=0):
    """Inverse iteration on D^dag D with D = D0 + m0 (LU of D, two solves per step)."""
    import scipy.linalg as sla
    n = D0.shape[0]
    lu = sla.lu_factor(D0 + m0 * np.eye(n))
    rng = np.random.default_rng(seed)
    y = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    y /= np.linalg.norm(y)
    nz = 1.0
    for _ in range(steps):
        z = sla.lu_solve(lu, y, trans=2)     # D^dag z = y
        z = sla.lu_solve(lu, z, trans=0)     # D w = z
        nz = np.linalg.norm(z)
        y = z / nz
    return float(nz ** -0.5)


def tune(name, log=print):
    cfg = CONFIGS[name]
    lat = Lattice(PROXY_L)
    U = su3_field(PROXY_L, cfg["eps"], cfg["gauge_seed"])
    A0 = clover_matrix(U, lat, 0.0, cfg["c_sw"])      # clover at m0 = 0; the mass shifts the diagonal
    D0 = dense_operator(U, lat, 0.0, cfg["c_sw"], A0)
    target = cfg["sigma_target"]
    cache = {}

    def s(m):
        if m not in cache:
            cache[m] = sigma_min(D0, m)
            log(f"{name}: m0={m:+.5f} sigma_min={cache[m]:.5e}", flush=True)
        return cache[m]

    m, step = 0.0, 0.05
    prev = s(m)
    while True:
        nxt = s(m - step)
        if nxt <= target:
            lo, hi = m - step, m          # bisection between heavy (hi) and light (lo)
            for _ in range(30):
                mid = 0.5 * (lo + hi)
                if s(mid) <= target:
                    lo = mid
                else:
                    hi = mid
                if abs(s(lo) / target - 1) <= 0.1 or hi - lo < 1e-4:
                    break
            return dict(m0=round(lo, 6), sigma_proxy=s(lo), target=target, reached=True, proxy_L=PROXY_L)
        if nxt > prev:
            break
        m, prev = m - step, nxt
    # minimum bracketed in [m - step, m + step]: golden-section search
    a, b = m - step, m + step
    gr = (np.sqrt(5) - 1) / 2
    c, d = b - gr * (b - a), a + gr * (b - a)
    while b - a > 2e-3:
        if s(c) < s(d):
            b = d
        else:
            a = c
        c, d = b - gr * (b - a), a + gr * (b - a)
    best = min(cache, key=cache.get)
    return dict(m0=round(best, 6), sigma_proxy=cache[best], target=target, reached=False, proxy_L=PROXY_L)


def main(names):
    path = os.path.join(ROOT, "workloads", "m0_tuned.json")
    out = {}
    if os.path.exists(path):
        with open(path) as f:
            out = json.load(f)
    for n in names:
        out[n] = tune(n)
        print(n, out[n], flush=True)
        with open(path, "w") as f:
            json.dump(out, f, indent=1, sort_keys=True)


if __name__ == "__main__":
    main(sys.argv[1:] or ["C2", "C3", "C4"])
