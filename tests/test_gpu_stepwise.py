"""Stepwise solve (dd_solve_begin / add / step / take / end): right-hand sides
that join a running batch at restart boundaries, into any slot, get the bits
and iteration counts they get from dd_solve alone; misuse is refused."""
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def setup():
    import torch
    from paper_1811_00355_amd import Context, Gauge, MG, default_params, DD_F32, DD_BF16
    from workloads import su3_field, gauss_spinor
    L, blk = (8, 8, 8, 16), (4, 4, 4, 4)
    ctx = Context(0)
    g = Gauge(ctx, L, blk, su3_field(L, 0.25, 6301), -0.25, 1.0)
    # a short restart length, so that every right-hand side takes several steps
    p = default_params(block=blk, n_vec=20, setup_iters=2, inner_dtype=DD_F32, store_dtype=DD_BF16, seed=9,
                       fgmres_restart=3)
    mg = MG(g, p)
    n = 6
    b = torch.from_numpy(gauss_spinor(L, n, 77).reshape(n, -1)).cuda()
    yield ctx, g, mg, b
    mg.destroy()
    g.destroy()
    ctx.close()


@pytest.mark.parametrize("graphs", [0, 1, 2])
def test_joins_match_dd_solve_alone(setup, graphs):
    import torch
    from paper_1811_00355_amd import binding as B
    ctx, g, mg, b = setup
    mg.dd_mg_set_graphs(graphs)
    n = b.shape[0]
    alone, iters = [], []
    for k in range(n):
        x = torch.zeros_like(b[k:k + 1])
        info, _ = mg.dd_solve(1, b[k:k + 1], x, 1e-10)
        torch.cuda.synchronize()
        alone.append(x[0].clone())
        iters.append(info[0]["outer_iters"])
    # capacity 3: rhs 0 and 1 start in slots 2 and 0, rhs 2 joins after one
    # step, the rest fill slots as they free up
    out, got_iters = {}, {}
    with mg.dd_solve_begin(3, 1e-10) as s:
        slot_of = {2: 0, 0: 1}
        s.add(2, b[0])
        s.add(0, b[1])
        nxt = 2
        states = s.step()
        assert states[2] == B.SLOT_RUNNING and states[0] == B.SLOT_RUNNING and states[1] == B.SLOT_FREE
        s.add(1, b[nxt])
        slot_of[1] = nxt
        nxt += 1
        steps = 1
        while slot_of:
            states = s.step()
            steps += 1
            assert steps < 200
            for slot, st in enumerate(states):
                if st == B.SLOT_DONE:
                    k = slot_of.pop(slot)
                    x = torch.empty_like(b[k])
                    info = s.take(slot, x)
                    out[k], got_iters[k] = x, info["outer_iters"]
                    assert info["converged"] and info["true_relres"] <= 1e-10
                    if nxt < n:
                        s.add(slot, b[nxt])
                        slot_of[slot] = nxt
                        nxt += 1
    torch.cuda.synchronize()
    for k in range(n):
        same = torch.equal(out[k], alone[k])
        print(f"graphs {graphs} rhs {k}: iters alone {iters[k]} joined {got_iters[k]} bitwise {same}", flush=True)
        assert same and got_iters[k] == iters[k]


def test_misuse_is_refused(setup):
    import torch
    from paper_1811_00355_amd import DDError
    ctx, g, mg, b = setup
    mg.dd_mg_set_graphs(1)
    s = mg.dd_solve_begin(2, 1e-10)
    try:
        s.add(0, b[0])
        with pytest.raises(DDError):
            s.add(0, b[1])                      # slot in use
        with pytest.raises(DDError):
            s.take(0, torch.empty_like(b[0]))   # still running
        with pytest.raises(DDError):
            s.add(2, b[1])                      # beyond the capacity
        with pytest.raises(DDError):
            mg.dd_solve_begin(1, 1e-10)         # one live state per multigrid
        x = torch.zeros_like(b[:1])
        with pytest.raises(DDError):
            mg.dd_solve(1, b[:1], x, 1e-10)     # the workspace is held
        bad = b[1].clone()
        bad[5] = float("nan")
        with pytest.raises(DDError):
            s.add(1, bad)
        states = s.step()
        assert states[1] == 0                   # the refused add left the slot free
        z = torch.zeros_like(b[0])
        s.add(1, z)                             # a zero source is done at once with x = 0
        assert s.step()[1] == 2
        x1 = torch.ones_like(b[0])
        info = s.take(1, x1)
        assert info["converged"] and not torch.any(x1 != 0)
    finally:
        s.end()
    x = torch.zeros_like(b[:1])
    info, _ = mg.dd_solve(1, b[:1], x, 1e-10)   # usable again after end
    assert info[0]["converged"]
