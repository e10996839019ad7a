"""Three-level extension of the two-level method (test infrastructure only).

The paper runs two levels and notes that the coarse solver may itself be a
multigrid method (Sec. 1, Sec. 2).  This module applies the same construction
once more, to the coarse operator D_c of Eq. (2), written out plainly in FP64:

  * level-2 aggregates: blocks of 2^4 coarse sites, tiled from the origin of the
    coarse lattice; a level-3 site is red when the sum of its coordinates is even;
  * chirality split of a coarse vector: components s*n .. s*n + n - 1 (the
    coarse gamma5 is +1 on the first n components of a site, -1 on the last n);
  * P2 from n2 level-2 test vectors, each (aggregate, chirality) set
    orthonormalised by the same modified Gram-Schmidt as level 1;
  * R2 = P2^dag and the level-3 operator D3 = P2^dag D_c P2, stored as 9 blocks
    per level-3 site: block d of X collects P2(x)^dag D_c(x, dd) P2(x + dd) over
    the coarse sites x of X and the stored directions dd, with d = self when
    x + dd lies in the same block of 2^4 (local coordinate in range) and d = dd
    when it crosses the block face (+mu and -mu kept apart even when they reach
    the same level-3 site);
  * level-3 solve: the even-odd GMRES of the coarse level (amg.CoarseEO) on D3;
  * level-2 solve (replacing the coarse even-odd GMRES): one cycle of flexible
    GMRES on D_c, right preconditioned by M2 v = MR_k(D_c; v, x0 = P2 D3^-1 R2 v)
    (k steps of minimal residual started from the coarse correction), one
    classical Gram-Schmidt pass per step, stopped when its residual estimate
    reaches tol |b| or after max_iters steps.
None of this is printed in the paper: each point above is a reading of it.
"""
from dataclasses import dataclass
from types import SimpleNamespace

import numpy as np

from .amg import COARSE_DIRS, CoarseEO, coarse_apply, coarse_neighbors, _cgs, _dot, _givens, _norm, mgs_sets


@dataclass
class L3Params:
    n_vec2: int = 8            # level-2 test vectors
    block2: tuple = (2, 2, 2, 2)
    mr_steps: int = 4          # MR smoothing steps on D_c after the level-3 correction
    kcycle_tol: float = 5e-2   # level-2 solve: relative residual estimate (the coarse tolerance of level 1)
    kcycle_max_iters: int = 20
    kcycle_fixed: bool = False # parity mode: exactly kcycle_max_iters steps
    l3_tol: float = 5e-2       # level-3 even-odd GMRES
    l3_restart: int = 60
    l3_max_iters: int = 300
    l3_fixed_iters: int = 0


class Level2Lattice:
    """The coarse lattice of `lat` seen as sites of a second aggregation."""

    def __init__(self, lat, block2=(2, 2, 2, 2)):
        self.lat = lat
        self.b2 = tuple(int(b) for b in block2)
        for mu in range(4):
            if lat.NB[mu] % self.b2[mu]:
                raise ValueError("coarse extent not divisible by the level-2 block edge")
        NB, b2 = lat.NB, self.b2
        self.NB3 = tuple(NB[m] // b2[m] for m in range(4))
        self.Vc3 = int(np.prod(self.NB3))
        self.Bv2 = int(np.prod(b2))
        cc = lat.coarse_coords                                   # [4][Vc]
        bc = np.stack([cc[m] // b2[m] for m in range(4)])
        lc = np.stack([cc[m] % b2[m] for m in range(4)])
        N3 = self.NB3
        self.agg3 = bc[0] + N3[0] * (bc[1] + N3[1] * (bc[2] + N3[2] * bc[3]))
        self.local2 = lc[0] + b2[0] * (lc[1] + b2[1] * (lc[2] + b2[2] * lc[3]))
        self.lc = lc
        order = np.lexsort((self.local2, self.agg3))
        self.sites_of_agg3 = order.reshape(self.Vc3, self.Bv2)
        t, z, y, x = np.meshgrid(*[np.arange(N3[m]) for m in (3, 2, 1, 0)], indexing="ij")
        c3 = np.stack([x.ravel(), y.ravel(), z.ravel(), t.ravel()])

        def nb3(mu, sign):
            c = c3.copy()
            c[mu] = (c[mu] + sign) % N3[mu]
            return c[0] + N3[0] * (c[1] + N3[1] * (c[2] + N3[2] * c[3]))

        # the level-3 lattice in the form CoarseEO / coarse_apply take
        self.lat3 = SimpleNamespace(Vc=self.Vc3, color_of_block=c3.sum(axis=0) % 2, coarse_neighbor=nb3)

    def crossing(self, x, d):
        """Stored level-3 direction of the coarse hop (x, d): 0 inside the block, else d."""
        if d == 0:
            return 0
        mu, sign = COARSE_DIRS[d]
        v = self.lc[mu][x] + sign
        return 0 if 0 <= v < self.b2[mu] else d


def to_aggregates2(lev, n, f):
    """Coarse vector(s) [..., Vc, 2n] -> [..., Vc3, 2, Bv2*n]: per level-3 site X and
    chirality s, the n components of chirality s of every coarse site of X in
    local-index order."""
    g = f[..., lev.sites_of_agg3, :]                         # [..., Vc3, Bv2, 2n]
    g = g.reshape(g.shape[:-1] + (2, n))                     # [..., Vc3, Bv2, 2, n]
    g = np.moveaxis(g, -2, -3)                               # [..., Vc3, 2, Bv2, n]
    return g.reshape(g.shape[:-2] + (lev.Bv2 * n,))


def from_aggregates2(lev, n, g):
    shp = g.shape[:-3]
    h = g.reshape(shp + (lev.Vc3, 2, lev.Bv2, n))
    h = np.moveaxis(h, -3, -2).reshape(shp + (lev.Vc3, lev.Bv2, 2 * n))
    f = np.zeros(shp + (lev.lat.Vc, 2 * n), dtype=np.complex128)
    f[..., lev.sites_of_agg3, :] = h
    return f


def gram_schmidt2(lev, n, tv2, passes=2, rank_tol=1e-12):
    """P2 [Vc3][2][n2][Bv2*n]: the chirality-split level-2 aggregates of the
    test vectors tv2 [n2][Vc][2n], each set orthonormalised (amg.mgs_sets)."""
    g = to_aggregates2(lev, n, tv2)              # [n2][Vc3][2][K]
    g = np.moveaxis(g, 0, 2).copy()              # [Vc3][2][n2][K]
    return mgs_sets(g, passes, rank_tol)


def restrict2(lev, n, P2, v):
    """b3(X, s, i) = <P2_i(X, s) | v>.  v: [Vc][2n] -> [Vc3][2 n2]."""
    vv = to_aggregates2(lev, n, v)
    return np.einsum("xsik,xsk->xsi", np.conj(P2), vv).reshape(lev.Vc3, -1)


def prolong2(lev, n, P2, c):
    """v = sum_{X,s,i} c(X, s, i) P2_i(X, s).  c: [Vc3][2 n2] -> [Vc][2n]."""
    n2 = P2.shape[2]
    g = np.einsum("xsik,xsi->xsk", P2, c.reshape(lev.Vc3, 2, n2))
    return from_aggregates2(lev, n, g)


def site_basis2(lev, n, P2, x):
    """[2 n2][2n]: row (s, i) is P2_i(X, s) on the coarse site x (zero off chirality s)."""
    X, l = lev.agg3[x], lev.local2[x]
    n2 = P2.shape[2]
    B = np.zeros((2 * n2, 2 * n), dtype=np.complex128)
    for s in range(2):
        B[s * n2:(s + 1) * n2, s * n:(s + 1) * n] = P2[X, s, :, l * n:(l + 1) * n]
    return B


def galerkin3(lev, n, Dc, P2):
    """D3 [Vc3][9][2 n2][2 n2] from the definition written out (see the module text)."""
    lat = lev.lat
    nb = coarse_neighbors(lat)
    n2 = P2.shape[2]
    D3 = np.zeros((lev.Vc3, 9, 2 * n2, 2 * n2), dtype=np.complex128)
    B = [site_basis2(lev, n, P2, x) for x in range(lat.Vc)]
    for x in range(lat.Vc):
        X = lev.agg3[x]
        for d in range(9):
            y = nb[d][x]
            D3[X, lev.crossing(x, d)] += np.conj(B[x]) @ Dc[x, d] @ B[y].T
    return D3


def mr_smooth(A, b, x0, steps):
    """`steps` minimal-residual steps on A x = b from x0: alpha = <Ar, r> / <Ar, Ar>."""
    x = x0.copy()
    r = b - A(x)
    for _ in range(steps):
        ar = A(r)
        alpha = _dot(ar, r) / np.real(_dot(ar, ar))
        x += alpha * r
        r -= alpha * ar
    return x


class ThreeLevelCoarse:
    """Approximate solver for the coarse system D_c y = b_c by the two-level
    method one level down (the coarse_solver of amg.TwoLevel)."""

    def __init__(self, lat, n, Dc, tv2, p3, p1):
        self.lev = Level2Lattice(lat, p3.block2)
        self.n = n
        self.Dc = Dc
        self.p3 = p3
        self.P2 = gram_schmidt2(self.lev, n, tv2)
        self.D3 = galerkin3(self.lev, n, Dc, self.P2)
        self.ceo3 = CoarseEO(self.lev.lat3, self.D3)
        self.p_l3 = SimpleNamespace(coarse_tol=p3.l3_tol, coarse_restart=p3.l3_restart,
                                    coarse_max_iters=p3.l3_max_iters, coarse_fixed_iters=p3.l3_fixed_iters,
                                    coarse_cgs_passes=p1.coarse_cgs_passes)
        self.steps = []

    def apply_Dc(self, x):
        return coarse_apply(self.lev.lat, self.Dc, x)

    def precond(self, v):
        e3 = self.ceo3.solve(restrict2(self.lev, self.n, self.P2, v), self.p_l3)
        x0 = prolong2(self.lev, self.n, self.P2, e3)
        return mr_smooth(self.apply_Dc, v, x0, self.p3.mr_steps)

    def __call__(self, b):
        """One FGMRES cycle on D_c (one Gram-Schmidt pass per step)."""
        p = self.p3
        x = np.zeros_like(b)
        bnorm = _norm(b)
        if bnorm == 0:
            return x
        m = p.kcycle_max_iters
        tol = 0.0 if p.kcycle_fixed else p.kcycle_tol
        Vb = [b / bnorm]
        Z = []
        H = np.zeros((m + 1, m), dtype=np.complex128)
        cs = np.zeros(m)
        sn = np.zeros(m, dtype=np.complex128)
        g = np.zeros(m + 1, dtype=np.complex128)
        g[0] = bnorm
        k = 0
        for j in range(m):
            z = self.precond(Vb[j])
            Z.append(z)
            w = self.apply_Dc(z)
            H[:j + 1, j] = _cgs(Vb, w, 1)
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
            if abs(g[j + 1]) <= tol * bnorm or hn == 0:
                break
            Vb.append(w / hn)
        self.steps.append(k)
        y = np.linalg.solve(np.triu(H[:k, :k]), g[:k])
        for i in range(k):
            x += y[i] * Z[i]
        return x
