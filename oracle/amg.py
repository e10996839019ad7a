"""Two-level DD-alpha-AMG pieces in FP64 (paper Sec. 2).

  * aggregation with chirality split, Eq. (1): lambda_i(X, s) = (1 +- gamma5)/2 lambda_i
    on domain X, zero elsewhere; each (X, s) set is orthonormalised by a
    two-pass modified Gram-Schmidt (the paper's equations carry no
    orthonormalisation; it is the usual choice of the method and is adopted)
  * restriction, Eq. (3):  b_c(X, s, i) = <lambda_i(X, s) | b>
  * prolongation, Eq. (4): x = sum_{X,s,i} x_c(X, s, i) |lambda_i(X, s)>
  * coarse operator, Eq. (2): D_c(X,s,i; Y,t,j) = <lambda_i(X,s)| D |lambda_j(Y,t)>,
    stored per coarse site as 9 blocks of (2n)x(2n): self, +x,+y,+z,+t, -x,-y,-z,-t
  * coarse solver: even-odd preconditioned GMRES, stopped at a relative residual
    of 5e-2 (taken on the even-site Schur system); one classical Gram-Schmidt
    pass per Arnoldi step (the loose stop needs no re-orthogonalisation)
  * smoother: multiplicative SAP over red/black domains, each domain solved by a
    fixed number of site even-odd preconditioned minimal-residual iterations
  * preconditioner, Eq. (5): M = P D_c^-1 R + S (1 - D P D_c^-1 R), post-smoothing
    only; computed as x_c = P D_c^-1 R v, then SAP on D x = v started at x_c
  * outer solver: flexible GMRES, right-preconditioned by M
  * adaptive setup: approximate solves on random vectors, then repeated
    (build M from the current vectors, apply M to every vector)

Coarse vectors are complex128 [Vc][2n] with component index s*n + i.
Coarse parity = block colour (sum of block coordinates mod 2).
"""
from dataclasses import dataclass

import numpy as np

from .dirac import hop_one


@dataclass
class MGParams:
    n_vec: int = 8
    setup_iters: int = 4          # Sec. 2: four adaptive setup iterations
    init_sap_apps: int = 3        # approximate solves on the random vectors (reading)
    sap_sweeps: int = 4           # Sec. 4: N_SAP = 4
    sap_mr_iters: int = 4         # Sec. 2: fixed MR count (value is a reading)
    coarse_tol: float = 5e-2      # Sec. 2: coarse residual condition
    coarse_restart: int = 60
    coarse_max_iters: int = 300
    coarse_cgs_passes: int = 1    # classical Gram-Schmidt passes in the coarse GMRES (reading)
    coarse_fixed_iters: int = 0   # > 0: run exactly this many coarse iterations, no tolerance stop
    fgmres_restart: int = 10
    max_outer_iters: int = 200


# ---------------------------------------------------------------------------
# aggregation, Gram-Schmidt, P and R  (Eqs. (1), (3), (4))
# ---------------------------------------------------------------------------
def to_aggregates(lat, f):
    """Fine vector(s) [..., V, 4, 3] -> [..., Vc, 2, Bv*6]: per aggregate X and
    chirality s (spins 2s, 2s+1), the 6 components of every site of X in
    local-index order."""
    g = f[..., lat.sites_of_agg, :, :]                      # [..., Vc, Bv, 4, 3]
    g = g.reshape(g.shape[:-2] + (2, 6))                    # [..., Vc, Bv, 2, 6]
    g = np.moveaxis(g, -2, -3)                              # [..., Vc, 2, Bv, 6]
    return g.reshape(g.shape[:-2] + (lat.Bv * 6,))


def from_aggregates(lat, g):
    """Inverse of `to_aggregates`."""
    shp = g.shape[:-3]
    h = g.reshape(shp + (lat.Vc, 2, lat.Bv, 6))
    h = np.moveaxis(h, -3, -2).reshape(shp + (lat.Vc, lat.Bv, 4, 3))
    f = np.zeros(shp + (lat.V, 4, 3), dtype=np.complex128)
    f[..., lat.sites_of_agg, :, :] = h
    return f


def gram_schmidt(lat, tv, passes=2, rank_tol=1e-12):
    """Orthonormalise the chirality-split aggregates of the test vectors.

    tv: [n][V][4][3].  Returns Pb [Vc][2][n][Bv*6] with Pb[X,s,i] the
    orthonormalised lambda_i(X, s) restricted to X.  For every (X, s) the
    vectors are taken in order i = 0..n-1; each is orthogonalised against the
    previous ones by modified Gram-Schmidt, repeated `passes` times, and
    normalised (real positive norm).  A vector whose norm falls to rank_tol
    times its norm before the projections marks the set as rank deficient."""
    g = to_aggregates(lat, tv)                  # [n][Vc][2][K]
    g = np.moveaxis(g, 0, 2).copy()             # [Vc][2][n][K]
    return mgs_sets(g, passes, rank_tol)


def mgs_sets(g, passes=2, rank_tol=1e-12):
    """Modified Gram-Schmidt of every set g[X, s, :, :] (n vectors of length K),
    in place: vectors in order, `passes` projection sweeps, real positive norms."""
    n = g.shape[2]
    for i in range(n):
        v = g[:, :, i]
        nrm0 = np.sqrt(np.sum(np.abs(v) ** 2, axis=-1))
        for _ in range(passes):
            for j in range(i):
                q = g[:, :, j]
                d = np.sum(np.conj(q) * v, axis=-1)
                v -= d[..., None] * q
        nrm = np.sqrt(np.sum(np.abs(v) ** 2, axis=-1))
        if np.any(nrm <= rank_tol * nrm0):
            bad = np.argwhere(nrm <= rank_tol * nrm0)[0]
            raise ValueError(f"test vectors are rank deficient on aggregate {bad[0]} chirality {bad[1]}")
        v /= nrm[..., None]
    return g


def restrict(lat, Pb, b):
    """Eq. (3): b_c(X, s, i) = <lambda_i(X, s) | b>.  b: [V][4][3] -> [Vc][2n]."""
    bb = to_aggregates(lat, b)                  # [Vc][2][K]
    bc = np.einsum("xsik,xsk->xsi", np.conj(Pb), bb)
    return bc.reshape(lat.Vc, -1)


def prolong(lat, Pb, c):
    """Eq. (4): x = sum_{X,s,i} c(X, s, i) lambda_i(X, s).  c: [Vc][2n] -> [V][4][3]."""
    n = Pb.shape[2]
    cc = c.reshape(lat.Vc, 2, n)
    g = np.einsum("xsik,xsi->xsk", Pb, cc)
    return from_aggregates(lat, g)


# ---------------------------------------------------------------------------
# coarse operator (Eq. (2)) and its apply
# ---------------------------------------------------------------------------
COARSE_DIRS = [(0, 0)] + [(mu, +1) for mu in range(4)] + [(mu, -1) for mu in range(4)]


def coarse_operator(W, Pb):
    """D_c [Vc][9][2n][2n] from the plain definition of Eq. (2).

    Column (t, j) of every block is obtained from the fine vector
    phi = sum_Y lambda_j(Y, t): its image under D is split into the part that
    stays inside each domain (clover plus the hops between sites of the same
    domain; this is the self block D_c(X, X)) and, for each direction, the
    hops that cross a domain face (D_c(X, X+mu) from the forward hop of the
    sites on the +mu face of X, D_c(X, X-mu) from the backward hop on the
    -mu face).  Restricting each part with the lambda_i(X, s) gives the rows.
    +mu and -mu are kept apart even when X+mu and X-mu coincide."""
    lat = W.lat
    Vc, n = lat.Vc, Pb.shape[2]
    Dc = np.zeros((Vc, 9, 2 * n, 2 * n), dtype=np.complex128)
    for t in range(2):
        for j in range(n):
            c = np.zeros((Vc, 2, n), dtype=np.complex128)
            c[:, t, j] = 1.0
            phi = prolong(lat, Pb, c.reshape(Vc, -1))
            col = t * n + j
            Dc[:, 0, :, col] = restrict(lat, Pb, W.apply_block(phi))
            for d in range(1, 9):
                mu, sign = COARSE_DIRS[d]
                h = hop_one(W.U, lat, phi, mu, sign)
                inside = lat.inside_fwd[mu] if sign > 0 else lat.inside_bwd[mu]
                h *= (~inside)[:, None, None]
                Dc[:, d, :, col] = restrict(lat, Pb, h)
    return Dc


def coarse_neighbors(lat):
    """[9][Vc] neighbour index for each stored block direction."""
    nb = [np.arange(lat.Vc)]
    for d in range(1, 9):
        mu, sign = COARSE_DIRS[d]
        nb.append(lat.coarse_neighbor(mu, sign))
    return np.stack(nb)


def coarse_apply(lat, Dc, x, dirs=range(9)):
    """y(X) = sum over the stored directions d of D_c(X, d) x(X + d)."""
    nb = coarse_neighbors(lat)
    y = np.zeros_like(x)
    for d in dirs:
        y += np.einsum("xij,xj->xi", Dc[:, d], x[nb[d]])
    return y


class CoarseEO:
    """Even-odd (coarse parity) split of D_c: the Schur complement on even sites
    S = D_ee - D_eo D_oo^-1 D_oe, with D_oo the self blocks of the odd sites."""

    def __init__(self, lat, Dc):
        self.lat = lat
        self.Dc = Dc
        self.even = lat.color_of_block == 0
        self.odd = ~self.even
        self.Doo_inv = np.zeros_like(Dc[:, 0])
        self.Doo_inv[self.odd] = np.linalg.inv(Dc[self.odd, 0])

    def hop(self, x):
        return coarse_apply(self.lat, self.Dc, x, dirs=range(1, 9))

    def self_apply(self, x):
        return np.einsum("xij,xj->xi", self.Dc[:, 0], x)

    def oo_inv(self, x):
        y = np.einsum("xij,xj->xi", self.Doo_inv, x)
        y[self.even] = 0
        return y

    def schur(self, ye):
        """S y_e (vectors are full coarse vectors, zero on odd sites)."""
        t = self.oo_inv(self.hop(ye))
        out = self.self_apply(ye) - self.hop(t)
        out[self.odd] = 0
        return out

    def solve(self, b, p):
        """Approximate D_c^-1 b by GMRES on the Schur system, then odd reconstruction."""
        be = b.copy()
        be[self.odd] = 0
        bo = b.copy()
        bo[self.even] = 0
        rhs = be - self.hop(self.oo_inv(bo))
        rhs[self.odd] = 0
        fixed = p.coarse_fixed_iters
        ye, _ = gmres(self.schur, rhs, tol=0.0 if fixed else p.coarse_tol,
                      restart=p.coarse_restart,
                      max_iters=fixed if fixed else p.coarse_max_iters,
                      passes=p.coarse_cgs_passes)
        yo = self.oo_inv(bo - self.hop(ye))
        return ye + yo


# ---------------------------------------------------------------------------
# Krylov solvers
# ---------------------------------------------------------------------------
def _dot(a, b):
    return np.vdot(a.ravel(), b.ravel())


def _norm(a):
    return np.sqrt(np.real(_dot(a, a)))


def _cgs(Vb, w, passes=2):
    """Classical Gram-Schmidt of w against Vb, `passes` times (2: one
    re-orthogonalisation); returns the accumulated coefficients h."""
    h = np.zeros(len(Vb), dtype=np.complex128)
    for _ in range(passes):
        hp = np.array([_dot(v, w) for v in Vb])
        for i, v in enumerate(Vb):
            w -= hp[i] * v
        h += hp
    return h


def _givens(a, b):
    """c, s with [c s; -conj(s) c] [a; b] = [r; 0], c real."""
    if b == 0:
        return 1.0, 0.0
    if a == 0:
        return 0.0, np.conj(b) / abs(b)
    t = np.sqrt(abs(a) ** 2 + abs(b) ** 2)
    c = abs(a) / t
    s = (a / abs(a)) * np.conj(b) / t
    return c, s


def gmres(A, b, tol, restart, max_iters, x0=None, passes=2):
    """Restarted GMRES(m) with classical Gram-Schmidt Arnoldi (`passes` passes)
    and Givens rotations.  Stops when the residual estimate falls to tol*|b| or
    after max_iters iterations."""
    x = np.zeros_like(b) if x0 is None else x0.copy()
    bnorm = _norm(b)
    hist = []
    if bnorm == 0:
        return x, hist
    it = 0
    while it < max_iters:
        r = b - A(x) if it > 0 or x0 is not None else b.copy()
        beta = _norm(r)
        if beta <= tol * bnorm:
            break
        m = min(restart, max_iters - it)
        Vb = [r / beta]
        H = np.zeros((m + 1, m), dtype=np.complex128)
        cs = np.zeros(m)
        sn = np.zeros(m, dtype=np.complex128)
        g = np.zeros(m + 1, dtype=np.complex128)
        g[0] = beta
        k = 0
        for j in range(m):
            w = A(Vb[j])
            H[:j + 1, j] = _cgs(Vb, w, passes)
            H[j + 1, j] = _norm(w)
            for i in range(j):
                a, bb = H[i, j], H[i + 1, j]
                H[i, j] = cs[i] * a + sn[i] * bb
                H[i + 1, j] = -np.conj(sn[i]) * a + cs[i] * bb
            cs[j], sn[j] = _givens(H[j, j], H[j + 1, j])
            H[j, j] = cs[j] * H[j, j] + sn[j] * H[j + 1, j]
            g[j + 1] = -np.conj(sn[j]) * g[j]
            g[j] = cs[j] * g[j]
            k = j + 1
            it += 1
            hist.append(abs(g[j + 1]) / bnorm)
            hn = H[j + 1, j].real
            if abs(g[j + 1]) <= tol * bnorm or hn == 0:
                break
            if j + 1 < m:
                Vb.append(w / hn)
        y = np.linalg.solve(np.triu(H[:k, :k]), g[:k])
        for i in range(k):
            x += y[i] * Vb[i]
        if hist and hist[-1] <= tol:
            break
    return x, hist


def fgmres(apply_A, precond, b, tol, restart, max_outer, x0=None):
    """Flexible GMRES(m), right preconditioned: z_j = M v_j, w = A z_j, CGS2,
    Givens.  After each cycle the true residual b - A x is recomputed; the
    solve ends when |b - A x| <= tol |b| (true residual) or after max_outer
    outer iterations.  Returns x and a dict with the iteration history."""
    x = np.zeros_like(b) if x0 is None else x0.copy()
    bnorm = _norm(b)
    info = dict(outer_iters=0, restarts=0, true_relres=[], est_relres=[])
    r = b - apply_A(x) if x0 is not None else b.copy()
    beta = _norm(r)
    info["true_relres"].append(beta / bnorm)
    while beta > tol * bnorm and info["outer_iters"] < max_outer:
        m = min(restart, max_outer - info["outer_iters"])
        Vb = [r / beta]
        Z = []
        H = np.zeros((m + 1, m), dtype=np.complex128)
        cs = np.zeros(m)
        sn = np.zeros(m, dtype=np.complex128)
        g = np.zeros(m + 1, dtype=np.complex128)
        g[0] = beta
        k = 0
        for j in range(m):
            z = precond(Vb[j])
            Z.append(z)
            w = apply_A(z)
            H[:j + 1, j] = _cgs(Vb, w, 2)
            hn = _norm(w)
            H[j + 1, j] = hn
            for i in range(j):
                a, bb = H[i, j], H[i + 1, j]
                H[i, j] = cs[i] * a + sn[i] * bb
                H[i + 1, j] = -np.conj(sn[i]) * a + cs[i] * bb
            cs[j], sn[j] = _givens(H[j, j], H[j + 1, j])
            H[j, j] = cs[j] * H[j, j] + sn[j] * H[j + 1, j]
            g[j + 1] = -np.conj(sn[j]) * g[j]
            g[j] = cs[j] * g[j]
            k = j + 1
            info["outer_iters"] += 1
            info["est_relres"].append(abs(g[j + 1]) / bnorm)
            if abs(g[j + 1]) <= tol * bnorm or hn == 0:
                break
            Vb.append(w / hn)
        y = np.linalg.solve(np.triu(H[:k, :k]), g[:k])
        for i in range(k):
            x += y[i] * Z[i]
        r = b - apply_A(x)
        beta = _norm(r)
        info["restarts"] += 1
        info["true_relres"].append(beta / bnorm)
    info["converged"] = bool(beta <= tol * bnorm)
    return x, info


# ---------------------------------------------------------------------------
# SAP smoother
# ---------------------------------------------------------------------------
def _block_sum(lat, f):
    """Sum over the sites of every domain: [V, ...] -> [Vc]."""
    return f[lat.sites_of_agg].reshape(lat.Vc, -1).sum(axis=1)


def block_solve_mr(W, r, k, active):
    """Approximate D_B e = r on every active domain B (Dirichlet boundaries):
    even-site Schur complement S = A_ee - H_eo A_oo^-1 H_oe, minimal residual
    from e_e = 0 for exactly k iterations, then odd reconstruction
    e_o = A_oo^-1 (r_o - H_oe e_e).  H is the hopping term kept inside the domain."""
    lat = W.lat
    ev = (lat.parity == 0)[:, None, None]
    od = ~ev
    act = active[lat.agg_of_site][:, None, None]

    def schur(v):
        t = W.apply_Ainv(W.hop_block(v) * od) * od
        return (np.einsum("sij,sj->si", W.A, v.reshape(-1, 12)).reshape(v.shape) - W.hop_block(t)) * ev

    ro = r * od
    rho = (r - W.hop_block(W.apply_Ainv(ro) * od)) * ev * act
    e = np.zeros_like(r)
    for _ in range(k):
        p = schur(rho)
        pr = _block_sum(lat, np.conj(p) * rho)
        pp = _block_sum(lat, np.abs(p) ** 2).real
        alpha = np.where(active & (pp > 0), pr / np.where(pp > 0, pp, 1.0), 0.0)
        a = alpha[lat.agg_of_site][:, None, None]
        e += a * rho
        rho -= a * p
    eo = W.apply_Ainv((ro - W.hop_block(e)) * od) * od
    return (e + eo) * act


def sap(W, b, x0, sweeps, mr_iters, block_solver=None):
    """Multiplicative SAP: `sweeps` times, for the red then the black domains,
    r = b - D x, approximately solve D_B e = r_B on every domain of that
    colour (independently), x += e."""
    lat = W.lat
    x = x0.copy()
    for _ in range(sweeps):
        for colour in (0, 1):
            active = lat.color_of_block == colour
            r = b - W.apply(x)
            if block_solver is None:
                e = block_solve_mr(W, r, mr_iters, active)
            else:
                e = block_solver(r, active)
            x += e
    return x


# ---------------------------------------------------------------------------
# two-level preconditioner, solver and setup
# ---------------------------------------------------------------------------
class TwoLevel:
    """M of Eq. (5) for one set of test vectors."""

    def __init__(self, W, tv, params, coarse_solver=None, block_solver=None):
        """`coarse_solver` / `block_solver` replace the coarse GMRES and the
        domain MR solves (tests use exact dense solves to reach closed forms)."""
        self.W = W
        self.lat = W.lat
        self.p = params
        self.tv = tv
        self.Pb = gram_schmidt(self.lat, tv)
        self.Dc = coarse_operator(W, self.Pb)
        self.ceo = CoarseEO(self.lat, self.Dc)
        self.coarse_solver = coarse_solver
        self.block_solver = block_solver

    def restrict(self, b):
        return restrict(self.lat, self.Pb, b)

    def prolong(self, c):
        return prolong(self.lat, self.Pb, c)

    def coarse_solve(self, bc):
        if self.coarse_solver is not None:
            return self.coarse_solver(bc)
        return self.ceo.solve(bc, self.p)

    def vcycle(self, v):
        xc = self.prolong(self.coarse_solve(self.restrict(v)))
        return sap(self.W, v, xc, self.p.sap_sweeps, self.p.sap_mr_iters, self.block_solver)

    def solve(self, b, tol=1e-10):
        return fgmres(self.W.apply, self.vcycle, b, tol, self.p.fgmres_restart,
                      self.p.max_outer_iters)


def setup(W, params, tv0):
    """Adaptive setup (Sec. 2).  tv0: the random starting vectors [n][V][4][3].
    1. lambda_i <- SAP(D; b = lambda_i, x0 = 0), init_sap_apps times, normalised;
    2. build M from the lambda_i;
    3. setup_iters times: lambda_i <- M lambda_i (normalised), rebuild M."""
    tv = tv0.copy()
    zero = np.zeros_like(tv[0])
    for _ in range(params.init_sap_apps):
        for i in range(len(tv)):
            v = sap(W, tv[i], zero, params.sap_sweeps, params.sap_mr_iters)
            tv[i] = v / _norm(v)
    mg = TwoLevel(W, tv, params)
    for _ in range(params.setup_iters):
        for i in range(len(tv)):
            v = mg.vcycle(tv[i])
            tv[i] = v / _norm(v)
        mg = TwoLevel(W, tv, params)
    return mg
