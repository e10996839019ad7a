"""Workload shapes and seeds.

C1 is the small all-FP64 case (4^4, 2^4 aggregates, n = 8); C2..C4 are the
16^3x32, 32^3x64 and 48^3x96 lattices with 4^4 aggregates; C5 is the serving
mix.  The solver parameters not fixed by the workload descriptions take the
paper's DDalphaAMG settings (Sec. 4: 4^4 blocks, N_SAP = 4; Sec. 2: four
adaptive setup iterations, coarse tolerance 5e-2).  Masses marked "tuned" are
read from `m0_tuned.json`, written by the oracle-only tuning script in
`oracle/tune_m0.py`.
"""
import json
import os

_HERE = os.path.dirname(os.path.abspath(__file__))

CONFIGS = {
    "C1": dict(L=(4, 4, 4, 4), eps=0.3, c_sw=1.0, m0=-0.4, block=(2, 2, 2, 2), n_vec=8,
               setup_iters=4, nrhs=1, gauge_seed=1001, src_seed=2001, tv_seed=3001,
               sigma_target=None),
    "C2": dict(L=(16, 16, 16, 32), eps=0.25, c_sw=1.0, m0="tuned", block=(4, 4, 4, 4), n_vec=20,
               setup_iters=6, nrhs=1, gauge_seed=1002, src_seed=2002, tv_seed=3002,
               sigma_target=1e-2),
    "C3": dict(L=(32, 32, 32, 64), eps=0.2, c_sw=1.0, m0="tuned", block=(4, 4, 4, 4), n_vec=20,
               setup_iters=4, nrhs=12, gauge_seed=1003, src_seed=None, tv_seed=3003,
               sigma_target=3e-3),
    "C4": dict(L=(48, 48, 48, 96), eps=0.15, c_sw=1.0, m0="tuned", block=(4, 4, 4, 4), n_vec=24,
               setup_iters=4, nrhs=12, gauge_seed=1004, src_seed=None, tv_seed=3004,
               sigma_target=1e-3),
}

SERVING = dict(shapes=[(8, 8, 8, 8), (16, 16, 16, 32), (24, 24, 24, 48), (32, 32, 32, 64)],
               eps_range=(0.15, 0.3), c_sw=1.0, sigma_target=5e-3, n_vec=20,
               block=(4, 4, 4, 4), nrhs_range=(1, 12), reuse_prob=0.3,
               arrival_seed=5001, pool_seed_base=6000)


def tuned_masses():
    path = os.path.join(_HERE, "m0_tuned.json")
    if not os.path.exists(path):
        return {}
    with open(path) as f:
        return json.load(f)


def get_config(name):
    c = dict(CONFIGS[name])
    if c["m0"] == "tuned":
        t = tuned_masses().get(name)
        if t is None:
            raise KeyError(f"no tuned mass for {name}; run oracle/tune_m0.py")
        c["m0"] = float(t["m0"])
    return c
