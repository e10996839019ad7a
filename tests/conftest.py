import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the HIP library)")
    config.addinivalue_line("markers", "slow: CPU test that takes more than a few seconds")


@pytest.fixture(scope="session")
def c1():
    """The small all-FP64 case: 4^4, antiperiodic t, eps = 0.3, c_sw = 1,
    m0 = -0.4, 2^4 blocks, n = 8 (links, source and starting vectors seeded)."""
    from workloads import get_config, su3_field, gauss_spinor, gauss_vectors
    from oracle.lattice import Lattice
    from oracle.dirac import WilsonClover
    cfg = get_config("C1")
    lat = Lattice(cfg["L"], cfg["block"])
    U = su3_field(cfg["L"], cfg["eps"], cfg["gauge_seed"])
    W = WilsonClover(U, lat, cfg["m0"], cfg["c_sw"])
    b = gauss_spinor(cfg["L"], 1, cfg["src_seed"])[0]
    tv0 = gauss_vectors(cfg["n_vec"], lat.V, cfg["tv_seed"]).reshape(cfg["n_vec"], lat.V, 4, 3)
    return dict(cfg=cfg, lat=lat, U=U, W=W, b=b, tv0=tv0)


@pytest.fixture(scope="session")
def c1_mg(c1):
    """The C1 two-level method after the full adaptive setup."""
    from oracle import amg
    p = amg.MGParams(n_vec=c1["cfg"]["n_vec"], setup_iters=c1["cfg"]["setup_iters"])
    return amg.setup(c1["W"], p, c1["tv0"])


def rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    d = np.linalg.norm((a - b).ravel())
    n = np.linalg.norm(b.ravel())
    return d / n if n > 0 else d
