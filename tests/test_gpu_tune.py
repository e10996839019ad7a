"""Autotuner: every launch-shape choice gives the same bits; the tuner's choice
is stored in and read back from its JSON cache."""
import json

import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_1811_00355_amd import Context
    c = Context(0)
    yield c
    c.close()


def test_tuning_choices_bit_identical(ctx, tmp_path):
    import torch
    import _gpu
    from paper_1811_00355_amd import Gauge, MG, default_params
    from oracle.lattice import Lattice
    from workloads import su3_field, gauss_vectors, gauss_spinor
    L, blk, n = (8, 8, 8, 16), (4, 4, 4, 4), 20
    lat = Lattice(L, blk)
    g = Gauge(ctx, L, blk, su3_field(L, 0.2, 23), -0.1, 1.0)
    p = default_params(block=blk, n_vec=n, inner_dtype=1, store_dtype=1, init_sap_apps=2, setup_iters=1)
    mg = MG(g, p, tv_host=gauss_vectors(n, lat.V, 31).reshape(n, lat.V, 4, 3))
    nrhs = 3
    bd = _gpu.to_dev(gauss_spinor(L, nrhs, 65).reshape(nrhs, -1))
    ref = None
    for wpe, th, spw in [(2, 256, 4), (3, 64, 2), (2, 128, 8)]:
        g.dd_gauge_set_tuning(wpe, th, spw)
        x = torch.zeros_like(bd)
        info, _ = mg.dd_solve(nrhs, bd, x, 1e-10)
        torch.cuda.synchronize()
        if ref is None:
            ref = x.clone()
        same = torch.equal(x, ref)
        print(f"sap_wpe={wpe} dirac_threads={th} coarse_spw={spw}: iters {[i['outer_iters'] for i in info]} "
              f"bitwise {same}", flush=True)
        assert same
    with pytest.raises(Exception):
        g.dd_gauge_set_tuning(4, 256, 4)
    with pytest.raises(Exception):
        g.dd_gauge_set_tuning(2, 256, 4, coarse_half=2)
    cache = tmp_path / "tune.json"
    rep = mg.dd_autotune(nrhs, str(cache))
    print(rep, flush=True)
    with pytest.raises(Exception):
        g.dd_gauge_set_tuning(2, 256, 4, coarse_basis_half=2)
    with pytest.raises(Exception):
        g.dd_gauge_set_tuning(2, 256, 4, coarse_mfma_half=2)
    chosen = g.dd_gauge_get_tuning()
    numeric = ("coarse_half", "coarse_basis_half", "coarse_mfma_half")   # the caller's numerical choices
    assert all(chosen[k] == 0 for k in numeric)
    launch = {k: v for k, v in chosen.items() if k not in numeric}
    data = json.loads(cache.read_text())
    assert len(data) == 1 and list(data.values())[0] == launch
    # the cache holds launch shapes only: the caller's numerical choices survive a hit
    g.dd_gauge_set_tuning(3, 64, 2, coarse_basis_half=1, coarse_mfma_half=1)
    rep2 = mg.dd_autotune(nrhs, str(cache))
    assert "cache hit" in rep2 and g.dd_gauge_get_tuning() == dict(launch, coarse_half=0, coarse_basis_half=1,
                                                                   coarse_mfma_half=1)
    g.dd_gauge_set_tuning(**launch)
    x = torch.zeros_like(bd)
    mg.dd_solve(nrhs, bd, x, 1e-10)
    torch.cuda.synchronize()
    assert torch.equal(x, ref)
    mg.destroy()
    g.destroy()
