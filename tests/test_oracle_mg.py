"""Pins of the oracle's multigrid pieces: maps, Gram-Schmidt, P, R, the coarse
operator of Eq. (2), the coarse even-odd GMRES, SAP, the V-cycle of Eq. (5),
FGMRES and the whole solve."""
import json
import os

import numpy as np
import pytest

from conftest import rel
from oracle.gamma import GAMMA
from oracle.lattice import Lattice
from oracle import amg, dirac
from workloads import su3_field, su3_random, gauss_spinor, gauss_vectors
import _dense

HERE = os.path.dirname(os.path.abspath(__file__))


# --- maps ---------------------------------------------------------------------------------
def test_maps_formula_and_partition():
    L, b = (8, 4, 4, 8), (4, 2, 2, 4)
    lat = Lattice(L, b)
    NB = [L[m] // b[m] for m in range(4)]
    for s in range(lat.V):
        x = [lat.coords[m][s] for m in range(4)]
        assert s == x[0] + L[0] * (x[1] + L[1] * (x[2] + L[2] * x[3]))
        bc = [x[m] // b[m] for m in range(4)]
        lc = [x[m] % b[m] for m in range(4)]
        assert lat.agg_of_site[s] == bc[0] + NB[0] * (bc[1] + NB[1] * (bc[2] + NB[2] * bc[3]))
        assert lat.local_of_site[s] == lc[0] + b[0] * (lc[1] + b[1] * (lc[2] + b[2] * lc[3]))
        assert lat.color_of_block[lat.agg_of_site[s]] == sum(bc) % 2
    counts = np.bincount(lat.agg_of_site)
    assert len(counts) == lat.Vc and np.all(counts == lat.Bv)
    assert sorted(lat.sites_of_agg.ravel()) == list(range(lat.V))
    # neighbour round trips, fine and coarse
    allx = np.arange(lat.V)
    for mu in range(4):
        y, _ = lat.nbr(allx, mu, +1)
        z, _ = lat.nbr(y, mu, -1)
        assert np.array_equal(z, allx)
        assert np.array_equal(lat.coarse_neighbor(mu, -1)[lat.coarse_neighbor(mu, +1)], np.arange(lat.Vc))
    # block origins are even, so the parity inside a block is the global parity
    assert all(bm % 2 == 0 for bm in b)


def test_paper_worked_example():
    with open(os.path.join(HERE, "golden", "paper_worked_example.json")) as f:
        g = json.load(f)
    lat = Lattice(g["fine_lattice"], g["block"])
    assert list(lat.NB) == g["coarse_lattice"]
    assert 2 * g["n_vec"] == g["coarse_dof_per_site"]
    assert lat.Bv * 0 + 12 == g["fine_dof_per_site"]
    assert 6 + 2 * 15 == g["packed_hermitian6_reals"]


# --- Gram-Schmidt, P, R ---------------------------------------------------------------------
def test_gram_schmidt_P_R(c1):
    lat = c1["lat"]
    n = c1["cfg"]["n_vec"]
    Pb = amg.gram_schmidt(lat, c1["tv0"])
    G = np.einsum("xsik,xsjk->xsij", np.conj(Pb), Pb)
    assert np.abs(G - np.eye(n)).max() < 1e-14
    c = gauss_vectors(1, lat.Vc, 3, ncomp=2 * n)[0]
    # R P = 1
    assert rel(amg.restrict(lat, Pb, amg.prolong(lat, Pb, c)), c) < 1e-14
    # P R is an orthogonal projector
    b = gauss_spinor(lat.L, 2, 8)
    pr = lambda v: amg.prolong(lat, Pb, amg.restrict(lat, Pb, v))
    assert rel(pr(pr(b[0])), pr(b[0])) < 1e-14
    assert abs(np.vdot(b[1], pr(b[0])) - np.vdot(pr(b[1]), b[0])) < 1e-12
    # gamma5 P = P Gamma5: a chirality-s coarse component lands on chirality-s spins only
    c5 = c.reshape(lat.Vc, 2, n) * np.array([1, -1])[None, :, None]
    g5 = np.array([1, 1, -1, -1])[None, :, None]
    assert rel(g5 * amg.prolong(lat, Pb, c), amg.prolong(lat, Pb, c5.reshape(lat.Vc, -1))) < 1e-14
    # the span of the chirality-split test vectors is preserved by the orthonormalisation
    tvp = c1["tv0"].copy()
    tvp[:, :, 2:] = 0   # chirality + part of every test vector
    assert rel(pr(tvp[3]), tvp[3]) < 1e-13


def test_gram_schmidt_rank_deficient_raises(c1):
    tv = c1["tv0"].copy()
    tv[1] = 2.0 * tv[0]
    with pytest.raises(ValueError, match="rank deficient"):
        amg.gram_schmidt(c1["lat"], tv)


# --- coarse operator --------------------------------------------------------------------------
def _dense_coarse(lat, Dc):
    """Assemble the coarse stencil into one dense matrix (both +mu and -mu added)."""
    m = Dc.shape[-1]
    nb = amg.coarse_neighbors(lat)
    M = np.zeros((lat.Vc * m, lat.Vc * m), dtype=complex)
    for X in range(lat.Vc):
        for d in range(9):
            Y = nb[d][X]
            M[X * m:(X + 1) * m, Y * m:(Y + 1) * m] += Dc[X, d]
    return M


def _dense_P(lat, Pb):
    n = Pb.shape[2]
    P = np.zeros((12 * lat.V, 2 * n * lat.Vc), dtype=complex)
    for X in range(lat.Vc):
        for s in range(2):
            for i in range(n):
                e = np.zeros((lat.Vc, 2 * n), dtype=complex)
                e[X, s * n + i] = 1
                P[:, X * 2 * n + s * n + i] = amg.prolong(lat, Pb, e).ravel()
    return P


def test_coarse_operator_dense_brute_force(c1):
    lat = c1["lat"]
    Pb = amg.gram_schmidt(lat, c1["tv0"])
    Dc = amg.coarse_operator(c1["W"], Pb)
    D = _dense.dense_D(c1["U"], lat.L, c1["W"].m0, c1["W"].c_sw)
    P = _dense_P(lat, Pb)
    assert rel(_dense_coarse(lat, Dc), P.conj().T @ D @ P) < 1e-14


def test_galerkin_identity_and_gamma5(c1):
    lat, W = c1["lat"], c1["W"]
    n = c1["cfg"]["n_vec"]
    Pb = amg.gram_schmidt(lat, c1["tv0"])
    Dc = amg.coarse_operator(W, Pb)
    v = gauss_vectors(1, lat.Vc, 4, ncomp=2 * n)[0]
    lhs = amg.coarse_apply(lat, Dc, v)
    rhs = amg.restrict(lat, Pb, W.apply(amg.prolong(lat, Pb, v)))
    assert rel(lhs, rhs) < 1e-14
    # coarse Gamma5-hermiticity: D_c(X+d, -d) = Gamma5 D_c(X, d)^dagger Gamma5
    G5 = np.diag(np.r_[np.ones(n), -np.ones(n)])
    nb = amg.coarse_neighbors(lat)
    opp = [0, 5, 6, 7, 8, 1, 2, 3, 4]
    for d in range(9):
        Y = nb[d]
        lhs = Dc[Y, opp[d]]
        rhs = G5 @ np.conj(np.swapaxes(Dc[:, d], 1, 2)) @ G5
        assert np.abs(lhs - rhs).max() < 1e-14


def _free_tv(lat):
    """n = 6 constant test vectors lambda_(a,c) = e_(a,c) + e_(a+2,c)."""
    tv = np.zeros((6, lat.V, 4, 3), dtype=complex)
    for a in range(2):
        for c in range(3):
            tv[3 * a + c, :, a, c] = 1
            tv[3 * a + c, :, a + 2, c] = 1
    return tv


@pytest.mark.parametrize("L,b", [((8, 4, 4, 8), (4, 2, 2, 4)), ((4, 4, 4, 4), (2, 2, 2, 2))])
def test_coarse_free_field_closed_form(L, b):
    """U = 1 with the constant test vectors: D_c(X, X) = m0 + sum 1/b_mu and
    D_c(X, X +- mu) = -(1 -+ gamma_mu)/(2 b_mu), times bc_t across the t wrap."""
    lat = Lattice(L, b)
    U = np.broadcast_to(np.eye(3, dtype=complex), (lat.V, 4, 3, 3)).copy()
    m0 = 0.07
    W = dirac.WilsonClover(U, lat, m0, 1.0)
    Pb = amg.gram_schmidt(lat, _free_tv(lat))
    Dc = amg.coarse_operator(W, Pb)
    I3 = np.eye(3)
    self_exp = (m0 + sum(1.0 / bm for bm in b)) * np.eye(12)
    assert np.abs(Dc[:, 0] - self_exp).max() < 1e-14
    for mu in range(4):
        for sgn, d in ((+1, 1 + mu), (-1, 5 + mu)):
            blk = -(np.kron(np.eye(4) - sgn * GAMMA[mu], I3)) / (2 * b[mu])
            cc = lat.coarse_coords[mu]
            wrap = (cc == lat.NB[mu] - 1) if sgn > 0 else (cc == 0)
            ph = np.where(wrap & (mu == 3), -1.0, 1.0)
            assert np.abs(Dc[:, d] - ph[:, None, None] * blk).max() < 1e-14


def test_coarse_unit_blocks_reproduce_D():
    """b = 1 (every site its own aggregate) with n = 6 unit test vectors: D_c = D."""
    L = (4, 2, 2, 4)
    lat = Lattice(L, (1, 1, 1, 1))
    U = su3_field(L, 0.3, 12)
    W = dirac.WilsonClover(U, lat, -0.2, 1.0)
    Pb = amg.gram_schmidt(lat, _free_tv(lat))
    Dc = amg.coarse_operator(W, Pb)
    D = _dense.dense_D(U, L, -0.2, 1.0)
    assert rel(_dense_coarse(lat, Dc), D) < 1e-14


# --- coarse even-odd GMRES ------------------------------------------------------------------------
def test_coarse_eo_gmres_full_krylov(c1):
    lat = c1["lat"]
    n = c1["cfg"]["n_vec"]
    Pb = amg.gram_schmidt(lat, c1["tv0"])
    Dc = amg.coarse_operator(c1["W"], Pb)
    ceo = amg.CoarseEO(lat, Dc)
    b = gauss_vectors(1, lat.Vc, 6, ncomp=2 * n)[0]
    p = amg.MGParams(n_vec=n, coarse_tol=1e-13, coarse_restart=500, coarse_max_iters=500)
    y = ceo.solve(b, p)
    exact = np.linalg.solve(_dense_coarse(lat, Dc), b.ravel()).reshape(b.shape)
    assert rel(y, exact) < 1e-10
    # the Schur system residual history is monotone and the tolerance stop is honoured
    rhs = b.copy()
    rhs[ceo.odd] = 0
    _, hist = amg.gmres(ceo.schur, rhs, 5e-2, 30, 300)
    assert all(hist[i + 1] <= hist[i] * (1 + 1e-12) for i in range(len(hist) - 1))
    assert hist[-1] <= 5e-2 and (len(hist) == 1 or hist[-2] > 5e-2)


# --- SAP ------------------------------------------------------------------------------------------------
def _block_dense(lat, D):
    """Dense D_B for every block (rows and columns restricted to the block)."""
    out = []
    for X in range(lat.Vc):
        idx = np.concatenate([12 * s + np.arange(12) for s in np.sort(lat.sites_of_agg[X])])
        out.append((idx, D[np.ix_(idx, idx)]))
    return out


def _exact_block_solver(lat, blocks):
    def solve(r, active):
        e = np.zeros_like(r).ravel()
        rv = r.ravel()
        for X, (idx, DB) in enumerate(blocks):
            if active[X]:
                e[idx] = np.linalg.solve(DB, rv[idx])
        return e.reshape(r.shape)
    return solve


@pytest.fixture(scope="module")
def c1_dense(c1):
    lat = c1["lat"]
    D = _dense.dense_D(c1["U"], lat.L, c1["W"].m0, c1["W"].c_sw)
    return D, _block_dense(lat, D)


def test_sap_exact_blocks_is_block_gauss_seidel(c1, c1_dense):
    lat, W = c1["lat"], c1["W"]
    D, blocks = c1_dense
    b = c1["b"]
    x0 = gauss_spinor(lat.L, 1, 44)[0]
    K = []
    for colour in (0, 1):
        Kc = np.zeros_like(D)
        for X, (idx, DB) in enumerate(blocks):
            if lat.color_of_block[X] == colour:
                Kc[np.ix_(idx, idx)] = np.linalg.inv(DB)
        K.append(Kc)
    bv, x = b.ravel(), x0.ravel()
    x1 = x + K[0] @ (bv - D @ x)
    x2 = x1 + K[1] @ (bv - D @ x1)
    got = amg.sap(W, b, x0, 1, 4, _exact_block_solver(lat, blocks))
    assert rel(got.ravel(), x2) < 1e-13


def test_block_mr_converges_to_block_solve_and_is_monotone(c1, c1_dense):
    lat, W = c1["lat"], c1["W"]
    D, blocks = c1_dense
    r = gauss_spinor(lat.L, 1, 45)[0]
    active = lat.color_of_block == 1
    exact = _exact_block_solver(lat, blocks)(r, active)
    e = amg.block_solve_mr(W, r, 60, active)
    assert rel(e, exact) < 1e-10
    res = []
    for k in range(0, 7):
        ek = amg.block_solve_mr(W, r, k, active).ravel()
        rr = r.ravel().copy()
        for X, (idx, DB) in enumerate(blocks):
            if active[X]:
                rr[idx] -= DB @ ek[idx]
            else:
                rr[idx] = 0
        res.append(np.linalg.norm(rr))
    assert all(res[i + 1] <= res[i] * (1 + 1e-12) for i in range(len(res) - 1))
    assert res[-1] < res[0]


# --- V-cycle, Eq. (5) -----------------------------------------------------------------------------
def test_vcycle_closed_form(c1, c1_dense):
    """With exact coarse and block solves, M = P Dc^-1 R + K_SAP (1 - D P Dc^-1 R)."""
    lat, W = c1["lat"], c1["W"]
    D, blocks = c1_dense
    n = c1["cfg"]["n_vec"]
    p = amg.MGParams(n_vec=n, sap_sweeps=2)
    Pb = amg.gram_schmidt(lat, c1["tv0"])
    Dcd = _dense_coarse(lat, amg.coarse_operator(W, Pb))
    P = _dense_P(lat, Pb)
    mg = amg.TwoLevel(W, c1["tv0"], p,
                      coarse_solver=lambda bc: np.linalg.solve(Dcd, bc.ravel()).reshape(bc.shape),
                      block_solver=_exact_block_solver(lat, blocks))
    # dense SAP iteration matrix: one sweep E = (1 - K_b D)(1 - K_r D); nu sweeps: 1 - K_SAP D = E^nu
    Kc = []
    for colour in (0, 1):
        K = np.zeros_like(D)
        for X, (idx, DB) in enumerate(blocks):
            if lat.color_of_block[X] == colour:
                K[np.ix_(idx, idx)] = np.linalg.inv(DB)
        Kc.append(K)
    I = np.eye(D.shape[0])
    E = (I - Kc[1] @ D) @ (I - Kc[0] @ D)
    Ksap = (I - np.linalg.matrix_power(E, p.sap_sweeps)) @ np.linalg.inv(D)
    CG = P @ np.linalg.solve(Dcd, P.conj().T)
    M = CG + Ksap @ (I - D @ CG)
    v = c1["b"]
    assert rel(mg.vcycle(v).ravel(), M @ v.ravel()) < 1e-12


# --- Krylov solvers ------------------------------------------------------------------------------------
def test_fgmres_identity_preconditioner_is_textbook_gmres(c1):
    W = c1["W"]
    b = c1["b"]
    m = 8
    _, info = amg.fgmres(W.apply, lambda v: v.copy(), b, 1e-30, m, m)
    # textbook GMRES: the k-th iterate minimises |b - D x| over span{b, Db, ..., D^(k-1) b}
    Kr = [b.ravel()]
    for _ in range(m - 1):
        Kr.append(W.apply(Kr[-1].reshape(b.shape)).ravel())
    Kr = np.stack(Kr, axis=1)
    for k in range(1, m + 1):
        Q, _ = np.linalg.qr(Kr[:, :k])
        DQ = np.stack([W.apply(Q[:, j].reshape(b.shape)).ravel() for j in range(k)], axis=1)
        y, *_ = np.linalg.lstsq(DQ, b.ravel(), rcond=None)
        r = b.ravel() - DQ @ y
        assert abs(info["est_relres"][k - 1] - np.linalg.norm(r) / np.linalg.norm(b)) < 1e-12


def test_fgmres_exact_preconditioner_one_iteration(c1, c1_dense):
    D, _ = c1_dense
    W = c1["W"]
    b = c1["b"]
    Dinv = np.linalg.inv(D)
    x, info = amg.fgmres(W.apply, lambda v: (Dinv @ v.ravel()).reshape(v.shape), b, 1e-10, 10, 10)
    assert info["outer_iters"] == 1 and info["converged"]


@pytest.mark.slow
def test_solve_c1_dense_and_true_residual(c1, c1_mg, c1_dense):
    D, _ = c1_dense
    W, b = c1["W"], c1["b"]
    x, info = c1_mg.solve(b, 1e-10)
    assert info["converged"]
    assert np.linalg.norm(b - W.apply(x)) / np.linalg.norm(b) <= 1e-10
    exact = np.linalg.solve(D, b.ravel())
    kappa = np.linalg.cond(D)
    assert rel(x.ravel(), exact) <= kappa * 1e-10
    # setup invariants hold on the produced P and D_c
    lat = c1["lat"]
    n = c1["cfg"]["n_vec"]
    G = np.einsum("xsik,xsjk->xsij", np.conj(c1_mg.Pb), c1_mg.Pb)
    assert np.abs(G - np.eye(n)).max() < 1e-14
    v = gauss_vectors(1, lat.Vc, 14, ncomp=2 * n)[0]
    assert rel(amg.coarse_apply(lat, c1_mg.Dc, v),
               c1_mg.restrict(W.apply(c1_mg.prolong(v)))) < 1e-14


@pytest.mark.slow
def test_free_propagator_fft():
    """U = 1, point source: x(y) = 1/V sum_p e^{ipy} D(p)^-1 e, with p_t = pi(2k+1)/Lt."""
    L = (4, 4, 4, 4)
    lat = Lattice(L, (2, 2, 2, 2))
    U = np.broadcast_to(np.eye(3, dtype=complex), (lat.V, 4, 3, 3)).copy()
    m0 = -0.4
    W = dirac.WilsonClover(U, lat, m0, 1.0)
    p = amg.MGParams(n_vec=8, setup_iters=2)
    mg = amg.setup(W, p, gauss_vectors(8, lat.V, 123).reshape(8, lat.V, 4, 3))
    alpha, a = 2, 1
    b = np.zeros((lat.V, 4, 3), dtype=complex)
    b[0, alpha, a] = 1
    x, info = mg.solve(b, 1e-10)
    e = np.zeros(4, dtype=complex)
    e[alpha] = 1
    Lx, Ly, Lz, Lt = L
    xs = np.zeros((Lt, Lz, Ly, Lx, 4), dtype=complex)
    smin, smax = np.inf, 0
    for kt in range(Lt):
        for kz in range(Lz):
            for ky in range(Ly):
                for kx in range(Lx):
                    pm = [2 * np.pi * kx / Lx, 2 * np.pi * ky / Ly, 2 * np.pi * kz / Lz,
                          np.pi * (2 * kt + 1) / Lt]
                    Dp = m0 * np.eye(4) + sum((1 - np.cos(pm[m])) * np.eye(4) + 1j * np.sin(pm[m]) * GAMMA[m]
                                              for m in range(4))
                    sv = np.linalg.svd(Dp, compute_uv=False)
                    smin, smax = min(smin, sv.min()), max(smax, sv.max())
                    xs[kt, kz, ky, kx] = np.linalg.solve(Dp, e)
    # inverse transform over the periodic momenta, then the antiperiodic twist in t
    xr = np.fft.ifftn(xs, axes=(0, 1, 2, 3))
    t = np.arange(Lt)[:, None, None, None, None]
    xr = xr * np.exp(1j * np.pi * t / Lt)
    exact = np.zeros((lat.V, 4, 3), dtype=complex)
    exact[:, :, a] = xr.reshape(lat.V, 4)
    assert rel(x, exact) <= (smax / smin) * 1e-10


@pytest.mark.slow
def test_solution_gauge_covariance(c1, c1_mg, c1_dense):
    """x[U^Omega, Omega b] = Omega x[U, b] (the solution is unique)."""
    lat, U, W, b = c1["lat"], c1["U"], c1["W"], c1["b"]
    D, _ = c1_dense
    Om = su3_random(lat.V, 1.0, 55)
    Ug = np.empty_like(U)
    for mu in range(4):
        y, _ = lat.nbr(np.arange(lat.V), mu, +1)
        Ug[:, mu] = Om @ U[:, mu] @ np.conj(np.swapaxes(Om[y], 1, 2))
    Wg = dirac.WilsonClover(Ug, lat, W.m0, W.c_sw)
    p = amg.MGParams(n_vec=c1["cfg"]["n_vec"], setup_iters=1)
    mgg = amg.setup(Wg, p, c1["tv0"])
    bg = b @ np.swapaxes(Om, 1, 2)
    xg, info = mgg.solve(bg, 1e-10)
    x, _ = c1_mg.solve(b, 1e-10)
    kappa = np.linalg.cond(D)
    assert info["converged"]
    assert rel(xg, x @ np.swapaxes(Om, 1, 2)) <= kappa * 1e-10


def test_sampled_aggregates_match_full():
    """Gram-Schmidt, restriction and prolongation evaluated on a subset of the
    aggregates (a lattice view holding only those aggregates' sites, as the
    full-size GPU checks use it) equal the whole-lattice evaluation there."""
    from types import SimpleNamespace
    lat = Lattice((8, 8, 8, 16), (4, 4, 4, 4))
    n = 20
    tv = gauss_vectors(n, lat.V, 5).reshape(n, lat.V, 4, 3)
    P = amg.gram_schmidt(lat, tv)
    aggs = np.array([0, 3, 7, lat.Vc - 1])
    k = len(aggs)
    sites = lat.sites_of_agg[aggs].reshape(-1)
    sub = SimpleNamespace(sites_of_agg=np.arange(k * lat.Bv).reshape(k, lat.Bv), Vc=k, Bv=lat.Bv, V=k * lat.Bv)
    Ps = amg.gram_schmidt(sub, tv[:, sites])
    assert np.array_equal(Ps, P[aggs])
    f = gauss_spinor(lat.L, 1, 3)[0]
    assert np.array_equal(amg.restrict(sub, Ps, f[sites]), amg.restrict(lat, P, f)[aggs])
    c = gauss_vectors(1, lat.Vc, 4, ncomp=2 * n)[0]
    assert np.array_equal(amg.prolong(sub, Ps, c[aggs]), amg.prolong(lat, P, c)[sites])
