"""Bare mass for a target smallest singular value, on the full lattice.

Light-quark workloads are specified by sigma_min(D) rather than by m0.  This
tool finds m0 on the device: sigma_min from block inverse iteration through the
multigrid solver (spectrum.py), m0 bracketed from the heavy side (sigma_min(m0)
is not monotone past a near-zero crossing, and the solver slows down sharply
there) by secant steps towards the target, until sigma_min is within 10 % of
it or the trial budget is spent.  Each trial runs a fresh adaptive setup at its
mass.

    python -m paper_1811_00355_amd.tune_mass C3 --target 3e-3

writes {config: {m0, sigma_min, target, trials, ...}} into
workloads/m0_light.json (the benchmark's light-quark masses).
"""
import argparse
import json
import os
import sys
import time

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIGHT_PATH = os.path.join(_HERE, "..", "workloads", "m0_light.json")


def measure(ctx, cfg, links, m0, store, nvec, iters, tol, log):
    from . import binding as B
    from .spectrum import sigma_min
    g = B.Gauge(ctx, cfg["L"], cfg["block"], links, m0, cfg["c_sw"])
    try:
        p = B.default_params(block=cfg["block"], n_vec=cfg["n_vec"], setup_iters=cfg["setup_iters"],
                             inner_dtype=B.DD_F32, store_dtype=store, seed=cfg["tv_seed"])
        t0 = time.perf_counter()
        mg = B.MG(g, p)
        try:
            mg.dd_mg_set_graphs(1)
            ts = time.perf_counter() - t0
            sig, hist, its = sigma_min(mg, g.V, nvec=nvec, iters=iters, tol=tol, rtol=0.01, log=log)
        finally:
            mg.destroy()
    finally:
        g.destroy()
    return dict(m0=round(m0, 6), sigma_min=sig, history=[float(h) for h in hist],
                max_outer_iters=int(max(max(i) for i in its)), setup_s=round(ts, 2),
                s=round(time.perf_counter() - t0, 2))


def search(trial, target, m_start=0.0, step=0.05, max_trials=12):
    """The mass search, over a function trial(m0) -> sigma_min (inf where the
    solver gave up).  Approaches the critical mass from the heavy side, where
    sigma_min falls about linearly as m0 decreases: secant steps through the
    last two heavy points towards the target, bisection towards the heavy side
    whenever a trial lands below the target or past the crossing (sigma_min
    not below that of the last heavy point).  Returns [(m0, sigma_min)]."""
    seen = []

    def t(m):
        s = trial(m)
        seen.append((m, s))
        return s

    def close(sig):
        return abs(sig / target - 1) <= 0.1

    h1 = (m_start, t(m_start))
    h2 = (m_start - step, t(m_start - step))
    while not h2[1] < h1[1] and len(seen) < max_trials:     # not yet on the heavy side: move up
        h2 = h1
        h1 = (h1[0] + step, t(h1[0] + step))
    low = None          # lightest mass known to be below the target or past the crossing
    while len(seen) < max_trials and not close(h2[1]):
        if h2[1] > target:
            slope = (h1[1] - h2[1]) / (h1[0] - h2[0])
            m = max(h2[0] - (h2[1] - target) / slope, h2[0] - 2 * step)
        else:
            m = h2[0]
        if low is not None and m <= low:
            m = 0.5 * (h2[0] + low)
        s = t(m)
        if close(s):
            break
        if target < s < h2[1]:
            h1, h2 = h2, (m, s)
        else:
            low = m
    return seen


def tune(cfg, target, m_start=0.0, step=0.05, max_trials=12, store=None, nvec=4, iters=8, tol=1e-8, log=print):
    """search() with sigma_min measured on the device for the workload `cfg`."""
    from . import binding as B
    from workloads import su3_field
    store = B.DD_BF16 if store is None else store
    t0 = time.perf_counter()
    links = su3_field(cfg["L"], cfg["eps"], cfg["gauge_seed"])
    log(f"[tune] links {cfg['L']} eps {cfg['eps']} generated in {time.perf_counter() - t0:.1f} s")
    ctx = B.Context(0)
    trials = []

    def trial(m):
        try:
            r = measure(ctx, cfg, links, m, store, nvec, iters, tol, log)
        except B.DDError as e:
            if e.name != "DD_ENOCONV":
                raise
            # the solver's iteration cap was reached: past the crossing
            r = dict(m0=round(m, 6), sigma_min=float("inf"), history=[], max_outer_iters=None, setup_s=None,
                     s=None, note=str(e))
        trials.append(r)
        log(f"[tune] m0 {m:.6f}: sigma_min {r['sigma_min']:.4e} ({r['s']} s, outer iterations <= "
            f"{r['max_outer_iters']})")
        return r["sigma_min"]

    search(trial, target, m_start, step, max_trials)
    ctx.close()
    ok = [r for r in trials if np.isfinite(r["sigma_min"])]
    best = min(ok, key=lambda r: abs(np.log(r["sigma_min"] / target)))
    return dict(m0=best["m0"], sigma_min=best["sigma_min"], target=target,
                reached=bool(abs(best["sigma_min"] / target - 1) <= 0.1),
                estimator=dict(nvec=nvec, max_iters=iters, solve_tol=tol, store=int(store)), trials=trials)


def main(argv=None):
    from workloads import get_config
    ap = argparse.ArgumentParser(description="tune m0 to a target sigma_min on the full lattice")
    ap.add_argument("config")
    ap.add_argument("--target", type=float, default=None)
    ap.add_argument("--max-trials", type=int, default=12)
    ap.add_argument("--step", type=float, default=0.05)
    ap.add_argument("--start", type=float, default=0.0, help="heavy starting mass")
    ap.add_argument("--out", default=LIGHT_PATH)
    args = ap.parse_args(argv)
    log = lambda *a: print(*a, file=sys.stderr, flush=True)   # noqa: E731
    cfg = get_config(args.config)
    target = args.target or cfg["sigma_target"]
    res = tune(cfg, target, args.start, step=args.step, max_trials=args.max_trials, log=log)
    data = {}
    if os.path.exists(args.out):
        with open(args.out) as f:
            data = json.load(f)
    data[args.config] = res
    with open(args.out, "w") as f:
        json.dump(data, f, indent=1)
    print(json.dumps({k: v for k, v in res.items() if k != "trials"}), flush=True)


if __name__ == "__main__":
    main()
